"""FP16 storage of the population deviations (pop_storage = 1): FP32 arithmetic, FP16 round-to-
nearest storage between steps.

Tolerance.  Each stored deviation carries a relative rounding error of at most 2^-12; with
deviations of order 1e-2 near the interfaces that is ~2e-6 absolute per population and step, about
100x the FP32 rounding.  The FP32 path reaches rel-L2(phi) ~1e-5 after 1000 steps, so the FP16
bar is 1e-3 (FP32 bar x 100) against the FP64 oracle, and mass may drift by the accumulated
random rounding (bounded here by 1e-5 per site after 1000 steps)."""
import numpy as np
import pytest

import synthetic as S
from tests._helpers import gpu_fields, rel_l2, run_pair, workload

pytestmark = pytest.mark.gpu


def test_fp16_start_is_exact(gpu):
    p, phi0 = workload("c1_64sq", pop_storage=1)
    o, g = run_pair(gpu, p, phi0, 0)
    fo, fg = o.fields(), gpu_fields(g)
    assert np.abs(fg["u"] - fo["u"]).max() < 2e-5 * np.abs(fo["u"]).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_fp16_parity(gpu, dim):
    if dim == 2:
        p, phi0 = workload("c1_64sq", Tw=0.9, pop_storage=1)
        steps = 1000
    else:
        p = S.model_params("c3_256cube_xi0.1", nx=24, ny=16, nz=20, Tw=0.9, pop_storage=1)
        phi0 = S.phi0((20, 16, 24), seed=7)
        steps = 1000
    o, g = run_pair(gpu, p, phi0, 0)
    ob0 = g.observables()
    o.step(steps)
    g.step(steps)
    fo, fg = o.fields(), gpu_fields(g)
    err = rel_l2(fg["phi"], fo["phi"])
    print(f"fp16 dim={dim} steps={steps} rel-L2(phi)={err:.3e} rel-L2(u)={rel_l2(fg['u'], fo['u']):.3e}")
    assert err <= 1e-3
    ob = g.observables()
    N = phi0.size
    print(f"fp16 mass drift per site {abs(ob['mass_dev'] - ob0['mass_dev']) / N:.3e}")
    assert abs(ob["mass_dev"] - ob0["mass_dev"]) / N < 1e-5
    assert abs(ob["phi_sum"] - ob0["phi_sum"]) / N < 1e-6


def test_fp16_tiles_and_checkpoint_bitwise(gpu):
    import torch
    p, phi0 = workload("c1_64sq", Tw=0.9, pop_storage=1, nx=100, ny=70)
    t = torch.tensor(phi0, dtype=torch.float32)
    a = gpu.Sim(dict(p, tile_hint=16)).init_fields(t).step(30)
    b = gpu.Sim(dict(p, tile_hint=32)).init_fields(t).step(30)
    assert np.array_equal(gpu_fields(a)["phi"], gpu_fields(b)["phi"])
    c = gpu.Sim(dict(p, tile_hint=16)).init_fields(t).step(15)
    d = gpu.Sim(dict(p, tile_hint=16)).set_state(c.get_state()).step(15)
    assert np.array_equal(gpu_fields(a)["phi"], gpu_fields(d)["phi"])
    with pytest.raises(gpu.LamError):
        gpu.Sim(dict(p, pop_storage=0)).set_state(c.get_state())
