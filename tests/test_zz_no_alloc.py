"""The no-allocation structure factor (lam_structure_factor_static, scratch in a static device
array) against lam_structure_factor of a simulation holding the same field: the same kernels in
the same order, so the results must agree bit for bit.  Two calls in a row, the second on a
smaller lattice (the static array keeps the first call's contents), then a lattice too large for
the array, which must be refused before anything is launched."""
import ctypes as C

import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu


def _developed(lam, nx, ny, steps, seed):
    import torch
    p = S.model_params("paper_2d_tau5", nx=nx, ny=ny, xi=-1.0)
    g = lam.Sim(p).init_fields(torch.tensor(S.phi0((ny, nx), seed=seed, amplitude=0.01),
                                            dtype=torch.float32))
    g.step(steps)
    return g


def test_static_structure_factor_matches_workspace_version(gpu):
    for (nx, ny, nbins), seed in (((384, 256, 128), 3), ((136, 200, 68), 4)):
        g = _developed(gpu, nx, ny, 600, seed)
        ref = g.structure_factor(nbins)
        phi = g.fields()["phi"].contiguous()
        out = gpu.structure_factor_static(phi, nbins, stream=g.stream)
        print(nx, ny, "k_peak", ref["k_peak"], out["k_peak"])
        assert max(ref["S"]) > 0.0
        assert np.array_equal(np.array(out["S"]), np.array(ref["S"]))
        for k in ("k_peak", "S_peak", "k_mean"):
            assert out[k] == ref[k], k


def test_static_structure_factor_rejects_oversized_lattice(gpu):
    import torch
    phi = torch.zeros((1536, 1536), dtype=torch.float32, device="cuda:0")
    with pytest.raises(gpu.LamError) as ei:
        gpu.structure_factor_static(phi, 64)
    assert ei.value.code == gpu.LAM_ESIZE
    assert "LAM_SK_STATIC_BYTES" in str(ei.value)
