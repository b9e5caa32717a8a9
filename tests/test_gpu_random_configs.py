"""Seeded random configurations against the FP64 oracle: ragged lattice shapes, walls or periodic,
hydrodynamics on or off, both force forms, tau from near 1/2 to 3, Gamma = 0 (pure advection) or
positive, instantaneous quench / no diffusion / finite xi, FP32 or FP16 populations, every tile
height and extra phi sub-steps, in 2D and 3D.  30 steps each; rel-L2 of phi and u within the
bars of the fixed parity tests (1e-5 FP32, 1e-3 FP16), mass and sum(phi) drift below 1e-6 per
site.  The draws come from a SplitMix64 stream, so the cases are the same on every run."""
import numpy as np
import pytest

import synthetic as S
from oracle import Oracle
from tests._helpers import gpu_fields, rel_l2

pytestmark = pytest.mark.gpu

STEPS = 30


def draw_case(i):
    u = S.uniform01(4242, 16, offset=16 * i)
    dim = 3 if u[0] < 0.35 else 2
    pick = lambda x, opts: opts[min(int(x * len(opts)), len(opts) - 1)]  # noqa: E731
    if dim == 2:
        nx, ny, nz = 8 + int(u[1] * 150), 8 + int(u[2] * 110), 1
    else:
        nx, ny, nz = 8 + int(u[1] * 70), 8 + int(u[2] * 20), 8 + int(u[3] * 50)
    p = dict(dim=dim, nx=nx, ny=ny, nz=nz,
             walls=int(u[4] < 0.7), hydro=int(u[5] < 0.8),
             tau=pick(u[6], [0.52, 0.6, 0.8, 1.0, 1.5, 3.0]),
             Gamma=pick(u[7], [0.0, 0.05, 0.1]),
             b=0.1, kappa=pick(u[8], [-0.006, -0.03]), c=pick(u[9], [0.0375, 0.03]),
             Tc=1.0, T0=pick(u[10], [1.5, 1.05, 0.95]), Tw=pick(u[11], [0.9, 0.95, 1.2]),
             xi=pick(u[12], [-1.0, 0.0, 0.01, 0.3, 1.0]),
             force_form=int(u[13] < 0.3), pop_storage=int(u[14] < 0.3),
             tile_hint=pick(u[15], [0, 8, 16, 32, 64]))
    if u[3] < 0.25 and dim == 2:
        p["n_phi_sub"], p["allow_unstable"] = 3, 1
    return p


CASES = [draw_case(i) for i in range(14)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_random_config_against_oracle(gpu, case):
    import torch
    p = CASES[case]
    shape = S.shape_of(p)
    phi0 = S.phi0(shape, seed=300 + case, amplitude=0.1)
    o = Oracle(dict(p, pop_storage=0)).init_fields(phi0)
    a0 = o.observables()
    o.step(STEPS)
    g = gpu.Sim(p).init_fields(torch.tensor(phi0, dtype=torch.float32)).step(STEPS)
    fo, fg = o.fields(), gpu_fields(g)
    bar = 1e-3 if p["pop_storage"] else 1e-5
    e_phi = rel_l2(fg["phi"], fo["phi"])
    e_u = rel_l2(fg["u"], fo["u"]) if np.abs(fo["u"]).max() > 1e-12 else np.abs(fg["u"]).max()
    ob = g.observables()
    N = phi0.size
    print(f"case {case} {p}: phi {e_phi:.2e}, u {e_u:.2e}")
    assert not ob["nonfinite"]
    assert e_phi <= bar
    assert e_u <= (bar * 10 if p["hydro"] else 1e-12)
    assert abs(ob["phi_sum"] - a0["phi_sum"]) / N < 1e-6
    if p["walls"] or not p["hydro"]:
        assert abs(ob["mass_dev"] - a0["mass_dev"]) / N < (1e-5 if p["pop_storage"] else 1e-6)
