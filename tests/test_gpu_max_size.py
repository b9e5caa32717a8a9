"""Near-maximal lattices: a population plane just under 2^32 bytes (the limit of the 32-bit byte
offsets the step kernels address planes with).  One step of a 32768 x 32767 D2Q9 lattice and of a
1024 x 1024 x 1023 D3Q19 lattice, compared site by site with the FP64 oracle at sampled sites:
around each sample the oracle runs one step on a periodic box that contains every cell the
sample's outputs depend on (radius 3 n_phi + 1; the temperature is uniform there), with the same
n_phi as the full lattice.  Samples include the highest element offsets and the periodic wrap."""
import numpy as np
import pytest

import synthetic as S
from oracle import Oracle

pytestmark = pytest.mark.gpu

SEED = 17
BOX = 48     # oracle box edge (half-width 24 > 3 n_phi + 1 + CORE / 2 for n_phi <= 5)
CORE = 4     # compared cells per axis around each sample


def _check(gpu, name, over, samples):
    import torch
    torch.cuda.empty_cache()
    p = S.model_params(name, **over)
    dim = p["dim"]
    shape = (p["ny"], p["nx"]) if dim == 2 else (p["nz"], p["ny"], p["nx"])
    assert int(np.prod(shape)) * 4 < 2 ** 32
    sim = gpu.Sim(p).init_fields(torch.from_numpy(S.phi0_f32(shape, seed=SEED)))
    n_phi, _ = sim.substeps
    assert 3 * n_phi + 1 + CORE // 2 < BOX // 2
    sim.step(1)
    sim.stream.synchronize()
    sim._keep = None
    f = sim.fields()
    q = dict(p, walls=0, Tw=p["T0"], n_phi_sub=n_phi, allow_unstable=1)
    q.update(nx=BOX, ny=BOX, nz=BOX if dim == 3 else 1)
    got, want = {"phi": [], "u": [], "n": []}, {"phi": [], "u": [], "n": []}
    lo = BOX // 2 - CORE // 2
    core = tuple(slice(lo, lo + CORE) for _ in range(dim))
    for c in samples:
        origin = tuple(ci - BOX // 2 for ci in c)
        o = Oracle(q).init_fields(S.phi0_patch(shape, origin, (BOX,) * dim, seed=SEED)).step(1)
        fo = o.fields()
        idx = [torch.tensor([(origin[a] + lo + k) % shape[a] for k in range(CORE)],
                            device=f["phi"].device) for a in range(dim)]
        grid = torch.meshgrid(*idx, indexing="ij")
        for k in ("phi", "n"):
            got[k].append(f[k][grid].double().cpu().numpy().ravel())
            want[k].append(fo[k][core].ravel())
        got["u"].append(torch.stack([f["u"][a][grid] for a in range(dim)]).double().cpu().numpy().ravel())
        want["u"].append(np.stack([fo["u"][a][core] for a in range(dim)]).ravel())
    del f, sim
    torch.cuda.empty_cache()
    g = {k: np.concatenate(v) for k, v in got.items()}
    w = {k: np.concatenate(v) for k, v in want.items()}
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))  # noqa: E731
    print(f"{name} {shape}: n_phi {n_phi}, rel-L2 phi {rel(g['phi'], w['phi']):.2e}, "
          f"u {rel(g['u'], w['u']):.2e}, max |dn| {np.abs(g['n'] - w['n']).max():.2e}")
    assert rel(g["phi"], w["phi"]) <= 1e-6
    assert rel(g["u"], w["u"]) <= 1e-4
    assert np.abs(g["n"] - w["n"]).max() < 1e-6


def test_max_size_2d(gpu):
    ny, nx = 32767, 32768
    _check(gpu, "m1_4096sq", dict(nx=nx, ny=ny),
           [(ny // 2, 1000), (ny - 300, nx - 2), (300, 5)])


def test_max_size_3d(gpu):
    nz, ny, nx = 1023, 1024, 1024
    _check(gpu, "c3_256cube_xi0.1", dict(nx=nx, ny=ny, nz=nz),
           [(nz // 2, ny // 2, nx // 2), (nz - 300, ny - 1, nx - 1), (300, 0, 5)])
