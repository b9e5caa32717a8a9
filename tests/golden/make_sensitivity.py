"""Writes sensitivity_floor.json: how much the FP64 oracle itself amplifies a tiny perturbation of
the initial order parameter on the parity workloads.

For each case the oracle runs twice, from phi0 and from phi0 (1 + 2^-24 s) with s a random sign
per site, and records rel-L2(phi) between the two runs at the checkpoints.  The ratio between two
checkpoints is the scheme's own amplification of an error over that interval; the GPU parity tests
carry the 1e-5 bar at 1000 steps to longer horizons with it.  Calls only the oracle and the seeded
input generators.  Run: python tests/golden/make_sensitivity.py  (a few minutes on 8 cores).
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic as S  # noqa: E402
from oracle import Oracle  # noqa: E402

CASES = {
    "c1_64sq_Tw0.9": ("c1_64sq", dict(Tw=0.9), None, [1000, 2000]),
    "paper_2d_tau5_instant": ("paper_2d_tau5", dict(xi=-1.0), None, [1000, 2000]),
    "c3_37x12x70_Tw0.9": ("c3_256cube_xi0.1", dict(nx=37, ny=12, nz=70, Tw=0.9), 7, [1000]),
}


def floor(name, over, seed, checkpoints):
    p = S.model_params(name, **over)
    if seed is None:
        phi0 = S.initial_phi(name, **{k: v for k, v in over.items() if k in ("nx", "ny", "nz")})
    else:
        phi0 = S.phi0(S.shape_of(dict(S.WORKLOADS[name], **over)), seed=seed)
    sign = np.sign(S.phi0(phi0.shape, seed=99, amplitude=1.0))
    a = Oracle(p).init_fields(phi0)
    b = Oracle(p).init_fields(phi0 * (1.0 + sign * 2.0 ** -24))
    out, done = {}, 0
    for t in checkpoints:
        a.step(t - done)
        b.step(t - done)
        done = t
        fa, fb = a.fields()["phi"], b.fields()["phi"]
        out[str(t)] = float(np.linalg.norm(fa - fb) / np.linalg.norm(fa))
    return out


def main():
    res = {"note": "rel-L2(phi) between oracle runs from phi0 and from phi0 (1 + 2^-24 s), s a random "
                   "sign per site, at the given step counts; written by tests/golden/make_sensitivity.py"}
    for key, (name, over, seed, cps) in CASES.items():
        res[key] = floor(name, over, seed, cps)
        print(key, res[key], flush=True)
    with open(os.path.join(HERE, "sensitivity_floor.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
