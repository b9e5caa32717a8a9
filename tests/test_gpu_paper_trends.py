"""The paper's own 2D workload without hydrodynamics (Section 3, Fig. 1 parameters: 256^2,
b = 0.1, kappa = -c = -0.03, walls at 0.9 Tc): the lamellar orientation as a function of the
thermal conductivity xi.  The paper reports it qualitatively (Section 3): an instantaneous quench
leaves a disordered texture, intermediate xi orders the lamellae parallel to the thermal fronts
(that is, to the walls), and very small xi turns them perpendicular to the walls.  The figure of
merit is Q = sum(g_y^2 - g_x^2) / sum |grad phi|^2 (+1 parallel to the walls).

Each run with a finite xi stops at the same diffusive time xi t = 46 251, about 3.5 times the
time at which the middle row of the 256-row slab drops below Tc: every row has then been quenched
by the front from the nearer wall, slowly or fast according to xi.  The thresholds are loose: they
check the sign and the strength of the order, not the values of one seed."""
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
