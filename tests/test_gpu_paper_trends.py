"""The paper's own workloads without hydrodynamics, in 2D (Fig. 1 parameters: 256^2,
b = 0.1, kappa = -c = -0.03, walls at 0.9 Tc): the lamellar orientation as a function of the
thermal conductivity xi.  The paper reports it qualitatively (Section 3): an instantaneous quench
leaves a disordered texture, intermediate xi orders the lamellae parallel to the thermal fronts
(that is, to the walls), and very small xi turns them perpendicular to the walls.  The figure of
merit is Q = sum(g_y^2 - g_x^2) / sum |grad phi|^2 (+1 parallel to the walls).

Each run with a finite xi stops at the same diffusive time xi t = 46 251, about 3.5 times the
time at which the middle row of the 256-row slab drops below Tc: every row has then been quenched
by the front from the nearer wall, slowly or fast according to xi.  The thresholds are loose: they
check the sign and the strength of the order, not the values of one seed.  The 3D counterparts
(Fig. 3) follow at the end of the file."""
import math

import numpy as np
import pytest
import torch

import synthetic as S

XI_T = 46251.0


def _run(gpu, xi, steps=None):
    p = S.model_params("paper_2d_nohydro", xi=xi)
    sim = gpu.Sim(p).init_fields(torch.tensor(S.initial_phi("paper_2d_nohydro"),
                                              dtype=torch.float32))
    n = steps if steps is not None else int(XI_T / xi)
    done = 0
    while done < n:
        k = min(100000, n - done)
        sim.step(k)
        done += k
    assert not sim.observables()["nonfinite"]
    o = sim.orientation(18)
    return o["Q"], np.array(o["Q_row"])


@pytest.mark.gpu
def test_instant_quench_is_disordered(gpu):
    q, _ = _run(gpu, -1.0, steps=1950)
    assert abs(q) < 0.15


@pytest.mark.gpu
def test_fast_front_orders_parallel_to_walls(gpu):
    q, rows = _run(gpu, 3.0)
    assert rows[16:48].mean() > 0.5 and rows[-48:-16].mean() > 0.5
    assert q > 0.5


@pytest.mark.gpu
def test_slow_front_orders_perpendicular_to_walls(gpu):
    q, rows = _run(gpu, 0.03)
    assert q < -0.9
    assert rows[:48].mean() < -0.9 and rows[-48:].mean() < -0.9


def test_stopping_time_quenches_every_row():
    """At xi t = XI_T the discrete per-row temperature (the same FTCS the solver runs, here on the
    host) is below Tc on every row, and it was not yet at a quarter of that time."""
    p = S.model_params("paper_2d_nohydro", xi=0.3)
    ny = 256
    T = np.full(ny, p["T0"])
    T[0] = T[-1] = p["Tw"]
    nT = math.ceil(p["xi"] / 0.45)
    r = p["xi"] / nT
    n = int(XI_T / p["xi"])
    for i in range(n * nT):
        T[1:-1] += r * (T[2:] - 2 * T[1:-1] + T[:-2])
        if i == (n * nT) // 4:
            assert T.max() > p["Tc"]
    assert T.max() < p["Tc"]


# ---------------------------------------------------------------------------------------------
# The paper's 3D runs without hydrodynamics (Section 3, Fig. 3: 32 x 32 x 256, walls normal to
# the long axis z): short-range order only for a fast front, stacks of lamellae parallel to the
# fronts for intermediate xi, and perpendicular order near the walls that is lost far from them
# for very small xi.  Q is the weighted second Legendre polynomial of the gradient direction
# relative to z: +1 parallel to the walls, -1/2 perpendicular, 0 isotropic.  The paper's printed
# times (110 - 7800 steps) are too short for any ordering at its coefficients (the fastest linear
# growth is about 0.005 per step), so as in 2D the runs stop at equal diffusive time (or, for the
# slowest front, once the near-wall layers have ordered).


def _run3(gpu, xi, steps):
    p = S.model_params("paper_3d_nohydro", xi=xi)
    sim = gpu.Sim(p).init_fields(torch.tensor(S.initial_phi("paper_3d_nohydro"),
                                              dtype=torch.float32))
    sim.step(steps)
    assert not sim.observables()["nonfinite"]
    o = sim.orientation(9)
    return o["Q"], np.array(o["Q_row"])


@pytest.mark.gpu
def test_3d_fast_front_is_disordered(gpu):
    q, _ = _run3(gpu, 100.0, 3000)
    assert abs(q) < 0.1


@pytest.mark.gpu
def test_3d_intermediate_front_stacks_parallel_to_walls(gpu):
    q, rows = _run3(gpu, 1.0, int(XI_T))
    assert q > 0.4
    assert rows[32:-32].mean() > 0.5


@pytest.mark.gpu
def test_3d_slow_front_perpendicular_near_walls(gpu):
    q, rows = _run3(gpu, 0.03, 50000)
    assert q < -0.25
    assert np.concatenate([rows[:8], rows[-8:]]).mean() < -0.3


@pytest.mark.gpu
def test_fig2c_hydrodynamic_quench_runs_its_21000_steps(gpu):
    """The paper's Fig. 2 run with an instantaneous quench and hydrodynamics (256^2, tau = 5, so
    eta = 1.5; xi = infinity) for its full 21 000 steps: finite throughout with Ma < 0.1
    (sampled every 1000 steps; Section 2 states Ma < 0.1 during the evolution), ending in a
    texture of differently oriented grains (no net orientation: |Q| < 0.3)."""
    p = S.model_params("paper_2d_tau5", xi=-1.0)
    sim = gpu.Sim(p).init_fields(torch.tensor(S.initial_phi("paper_2d_tau5"),
                                              dtype=torch.float32))
    mach = 0.0
    for _ in range(21):
        sim.step(1000)
        ob = sim.observables()
        assert not ob["nonfinite"]
        mach = max(mach, ob["mach"])
    assert 1e-3 < mach < 0.1
    assert abs(sim.orientation(18)["Q"]) < 0.3
