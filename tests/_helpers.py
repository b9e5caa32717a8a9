"""Shared helpers of the GPU parity tests: run the same seeded workload through the oracle and
through the C-ABI, and compare."""
import json
import os

import numpy as np

import synthetic as S
from oracle import Oracle


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_pair(lam, params, phi0, steps, u0=None, n0=None):
    """Advance the oracle and the GPU library by `steps` from the same initial fields."""
    import torch
    o = Oracle(params).init_fields(phi0, u0=u0, n0=n0)
    g = lam.Sim(params)
    tt = lambda a: None if a is None else torch.tensor(np.asarray(a, np.float32))  # noqa: E731
    g.init_fields(tt(phi0), tt(u0), tt(n0))
    if steps:
        o.step(steps)
        g.step(steps)
    return o, g


def gpu_fields(g):
    return {k: v.double().cpu().numpy() for k, v in g.fields().items()}


def workload(name, **over):
    """Model parameters of a named workload (with overrides) and its seeded initial phi."""
    p = S.model_params(name, **over)
    phi0 = S.initial_phi(name, **{k: v for k, v in over.items() if k in ("nx", "ny", "nz")})
    return p, phi0


def horizon_tol(case, steps, bar=1e-5):
    """The parity bar (rel-L2(phi) <= 1e-5 after 1000 steps) carried to a longer horizon by the
    scheme's own amplification of an error between step 1000 and `steps`: the ratio of the oracle's
    sensitivity to a 2^-24 perturbation of phi0 at the two times (tests/golden/sensitivity_floor.json,
    written from the oracle alone by tests/golden/make_sensitivity.py)."""
    if steps <= 1000:
        return bar
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sensitivity_floor.json")
    with open(path) as f:
        fl = json.load(f)[case]
    return bar * fl[str(steps)] / fl["1000"]
