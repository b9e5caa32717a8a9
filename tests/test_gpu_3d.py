"""GPU parity of the D3Q19 path (z-marching kernels) against the FP64 oracle, through the C-ABI.
Same tolerances as the 2D tests (see test_gpu_parity.py)."""
import numpy as np
import pytest

import synthetic as S
from oracle import Oracle
from tests._helpers import gpu_fields, rel_l2, run_pair

pytestmark = pytest.mark.gpu


def params3(nx=24, ny=16, nz=20, **kw):
    return S.model_params("c3_256cube_xi0.1", nx=nx, ny=ny, nz=nz, **kw)


def test_force_and_velocity_at_start_3d(gpu):
    for ff in (0, 1):
        p = params3(force_form=ff)
        phi0 = S.phi0((20, 16, 24), seed=3)
        o, g = run_pair(gpu, p, phi0, 0)
        fo, fg = o.fields(), gpu_fields(g)
        scale = np.abs(fo["u"]).max()
        assert scale > 1e-6
        assert np.abs(fg["u"] - fo["u"]).max() < 2e-5 * scale, ff
        assert np.abs(fg["n"] - fo["n"]).max() < 1e-6


@pytest.mark.parametrize("shape,walls", [((20, 16, 24), 1), ((37, 12, 40), 1), ((16, 24, 8), 0),
                                         ((70, 8, 16), 1), ((33, 10, 20), 1)])
def test_parity_3d(gpu, shape, walls):
    """Several z chunks (16 slices for the step kernel; the phi kernel's chunk length is chosen
    from the lattice, 16 slices on lattices this small), ragged last chunks (one slice long at
    nz = 33) and ragged x/y tiles; walls on and fully periodic."""
    nz, ny, nx = shape
    p = params3(nx=nx, ny=ny, nz=nz, walls=walls, Tw=0.9, T0=1.5 if walls else 0.95)
    phi0 = S.phi0(shape, seed=7)
    o, g = run_pair(gpu, p, phi0, 40)
    fo, fg = o.fields(), gpu_fields(g)
    assert rel_l2(fg["phi"], fo["phi"]) <= 1e-5
    assert rel_l2(fg["u"], fo["u"]) <= 1e-4
    assert np.abs(fg["T"] - fo["T"]).max() < 1e-5


@pytest.mark.parametrize("shape", [(70, 12, 37), (40, 9, 70)])
def test_parity_3d_1000_steps(gpu, shape):
    """The spec bar in 3D with hydrodynamics: 1000 steps at 0.9 Tc walls, rel-L2(phi)
    <= 1e-5, mass and sum(phi) drift < 1e-6.  (70, 12, 37) spans five chunks of both kernels
    (16 slices, ragged last), with a ragged x tile;
    (40, 9, 70) spans two x tiles and two y tiles (the second one row high)."""
    nz, ny, nx = shape
    p = params3(nx=nx, ny=ny, nz=nz, Tw=0.9)
    phi0 = S.phi0(shape, seed=7)
    o, g = run_pair(gpu, p, phi0, 0)
    ob0 = g.observables()
    o.step(1000)
    g.step(1000)
    fo, fg = o.fields(), gpu_fields(g)
    assert np.abs(fo["phi"]).max() > 0.5
    err = rel_l2(fg["phi"], fo["phi"])
    print(f"3d {shape} 1000 steps: rel-L2(phi) {err:.3e} rel-L2(u) {rel_l2(fg['u'], fo['u']):.3e}")
    assert err <= 1e-5
    ob = g.observables()
    N = phi0.size
    assert abs(ob["mass_dev"] - ob0["mass_dev"]) / N < 1e-6
    assert abs(ob["phi_sum"] - ob0["phi_sum"]) / N < 1e-6


def test_parity_3d_without_hydrodynamics(gpu):
    """The paper's 3D runs solve phi and T only (Section 3, Fig. 3)."""
    p = S.model_params("paper_3d_nohydro", nx=16, ny=16, nz=48)
    phi0 = S.phi0((48, 16, 16), seed=2, amplitude=0.01)
    o, g = run_pair(gpu, p, phi0, 200)
    fo, fg = o.fields(), gpu_fields(g)
    assert rel_l2(fg["phi"], fo["phi"]) <= 1e-5
    assert np.abs(fg["u"]).max() == 0.0


def test_observables_and_conservation_3d(gpu):
    p = params3()
    phi0 = S.phi0((20, 16, 24), seed=4)
    o, g = run_pair(gpu, p, phi0, 0)
    a0 = g.observables()
    o.step(60)
    g.step(60)
    a, b = o.observables(), g.observables()
    N = phi0.size
    assert abs(a["mass_dev"] - b["mass_dev"]) / N < 1e-6
    assert abs(a["phi_sum"] - b["phi_sum"]) / N < 1e-6
    assert abs(b["phi_sum"] - a0["phi_sum"]) / N < 1e-6
    assert np.abs(np.array(a["mom"]) - np.array(b["mom"])).max() / N < 1e-7
    assert b["max_u"] == pytest.approx(a["max_u"], rel=1e-4)
    assert b["free_energy"] == pytest.approx(a["free_energy"], rel=1e-5)


def test_checkpoint_and_roll_3d(gpu):
    import torch
    p = params3()
    phi0 = S.phi0((20, 16, 24), seed=5)
    t = lambda a: torch.tensor(a, dtype=torch.float32)  # noqa: E731
    ref = gpu.Sim(p).init_fields(t(phi0)).step(21)
    a = gpu.Sim(p).init_fields(t(phi0)).step(10)
    b = gpu.Sim(p).set_state(a.get_state()).step(11)
    assert np.array_equal(gpu_fields(ref)["phi"], gpu_fields(b)["phi"])
    c = gpu.Sim(p).init_fields(t(np.roll(phi0, (3, 5), axis=(1, 2)))).step(21)
    assert np.array_equal(np.roll(gpu_fields(ref)["phi"], (3, 5), axis=(1, 2)), gpu_fields(c)["phi"])


def test_graph_replay_matches_direct_launches_3d(gpu):
    """As in 2D: graph-replayed step pairs and direct launches give bit-identical fields."""
    import torch
    p = params3(nx=24, ny=16, nz=40)
    t = torch.tensor(S.phi0((40, 16, 24), seed=6), dtype=torch.float32)
    a = gpu.Sim(p, stream=torch.cuda.Stream()).init_fields(t).step(27).step(6)
    assert a.launch_mode()["graphs"] in (0, 1)  # the first call measured both ways
    b = gpu.Sim(p, stream=torch.cuda.Stream()).init_fields(t).set_timing(True).step(33)
    fa, fb = gpu_fields(a), gpu_fields(b)
    for k in ("phi", "u", "n", "T"):
        assert np.array_equal(fa[k], fb[k]), k


def test_orientation_3d_parity(gpu):
    """The 3D orientation observable (angle of grad phi to the wall normal, Q = weighted second
    Legendre polynomial, Q per layer) of a developed field against the oracle's definition, on
    the same FP32 field.  A site whose angle lies within 1e-4 rad of a bin edge may land on either
    side in FP32: its weight may move to the neighbour bin."""
    import math
    import torch
    from oracle import spectra
    p = S.model_params("paper_3d_nohydro", nx=24, ny=20, nz=48, xi=1.0)
    g = gpu.Sim(p).init_fields(torch.tensor(S.phi0((48, 20, 24), seed=8, amplitude=0.01),
                                            dtype=torch.float32))
    g.step(600)
    phi = gpu_fields(g)["phi"]
    nb = 9
    ref = spectra.orientation(phi, nb, walls=True)
    got = g.orientation(nb)
    assert ref["total_weight"] > 0 and abs(ref["Q"]) > 0.05
    assert got["Q"] == pytest.approx(ref["Q"], abs=1e-5)
    np.testing.assert_allclose(got["Q_row"], ref["Q_row"], atol=1e-5)
    width = 0.5 * math.pi / nb
    th, w = ref["theta"].ravel(), ref["weight"].ravel() / ref["total_weight"]
    frac = th / width - np.floor(th / width)
    amb = (frac < 1e-4 / width) | (frac > 1 - 1e-4 / width)
    slack = np.zeros(nb)
    b = np.minimum((th / width).astype(int), nb - 1)
    for d in (-1, 0, 1):
        np.add.at(slack, np.clip(b[amb] + d, 0, nb - 1), w[amb])
    assert np.all(np.abs(np.array(got["hist"]) - ref["hist"]) <= slack + 1e-5)


def test_full_size_3d_one_step(gpu):
    """The 256^3 workload in the launch configuration of the benchmark line, one step, every
    site compared with the oracle."""
    p = S.model_params("c3_256cube_xi0.1")
    phi0 = S.initial_phi("c3_256cube_xi0.1")
    o, g = run_pair(gpu, p, phi0, 1)
    fo, fg = o.fields(), gpu_fields(g)
    assert rel_l2(fg["phi"], fo["phi"]) <= 1e-6
    assert rel_l2(fg["u"], fo["u"]) <= 1e-4
    assert np.abs(fg["n"] - fo["n"]).max() < 1e-6


@pytest.mark.parametrize("tau", [0.6, 1.7])
def test_shear_wave_3d(gpu, tau):
    """A transverse shear wave u_x(z) = 1e-3 sin(2 pi z / L) on a periodic lattice without an order
    parameter decays as in the oracle over 300 steps: rel-L2(u) <= 1e-5.  At tau < 1 (omega > 1)
    this holds the rounding of the collision: writing it as (1 - omega) g + omega geq, or summing
    the equilibrium in pieces, loses bits systematically and misses the bound."""
    L = 64
    p = S.model_params("c3_256cube_xi0.1", nx=8, ny=12, nz=L, walls=0, T0=1.5, Tw=1.5, tau=tau)
    z = np.arange(L)
    u0 = np.zeros((3, L, 12, 8))
    u0[0] = (1e-3 * np.sin(2 * np.pi * z / L))[:, None, None]
    o, g = run_pair(gpu, p, np.zeros((L, 12, 8)), 300, u0=u0)
    err = rel_l2(gpu_fields(g)["u"], o.fields()["u"])
    print(f"tau {tau}: rel-L2(u) after 300 steps {err:.3e}")
    assert err < 1e-5
