"""Seeded synthetic inputs shared by the oracle-side and GPU-side tests and by the benchmark.

This module holds no arithmetic of the method itself: it only draws initial order-parameter
fields and names the workloads (lattice sizes and model parameters).

The paper starts every run from a disordered, symmetric state: the order parameter fluctuates
around zero in a small interval, the density is uniform and the fluid is at rest, and the
temperature is uniform above the critical value with cold walls (Section 3).  The workloads
here keep that structure with the amplitudes and parameters listed in ``WORKLOADS``.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used as a counter-based generator: the value for site ``i`` is the
``i``-th output of the stream whose state starts at ``seed``, so any site can be drawn alone.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, index: np.ndarray) -> np.ndarray:
    """The ``index``-th outputs (0-based) of the SplitMix64 stream started at state ``seed``."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (index.astype(np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """``n`` doubles in [0, 1) with 53 random bits each, sites ``offset .. offset+n-1``."""
    z = splitmix64(seed, np.arange(offset, offset + n, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def phi0(shape, seed: int = 1, amplitude: float = 0.05) -> np.ndarray:
    """Initial order parameter: iid uniform in [-amplitude, amplitude], rounded to float32.

    ``shape`` is (ny, nx) or (nz, ny, nx); site ``i = x + nx*(y + ny*z)`` takes draw ``i``.
    The values are returned as float64 holding exactly the float32 numbers, so the FP64 oracle
    and the FP32 GPU path start from bit-identical fields.
    """
    n = int(np.prod(shape))
    u = uniform01(seed, n)
    return (amplitude * (2.0 * u - 1.0)).astype(np.float32).astype(np.float64).reshape(shape)


def phi0_f32(shape, seed: int = 1, amplitude: float = 0.05, threads: int = 16,
             chunk: int = 1 << 23) -> np.ndarray:
    """The same field as ``phi0`` as a float32 array, generated in chunks on ``threads`` threads
    (for lattices of up to about 2^30 sites)."""
    from concurrent.futures import ThreadPoolExecutor
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.float32)

    def work(o):
        m = min(chunk, n - o)
        u = uniform01(seed, m, offset=o)
        out[o:o + m] = (amplitude * (2.0 * u - 1.0)).astype(np.float32)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, range(0, n, chunk)))
    return out.reshape(shape)


def phi0_patch(shape, origin, size, seed: int = 1, amplitude: float = 0.05) -> np.ndarray:
    """The values of ``phi0(shape, seed, amplitude)`` on a periodically wrapped box of ``size``
    cells per axis starting at ``origin`` (both in the axis order of ``shape``), without
    generating the whole field."""
    idx = np.zeros(size, dtype=np.int64)
    stride = 1
    for ax in range(len(shape) - 1, -1, -1):
        c = (origin[ax] + np.arange(size[ax])) % shape[ax]
        sh = [1] * len(shape)
        sh[ax] = size[ax]
        idx = idx + (c * stride).reshape(sh)
        stride *= shape[ax]
    z = splitmix64(seed, idx.reshape(-1).astype(np.uint64))
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return (amplitude * (2.0 * u - 1.0)).astype(np.float32).astype(np.float64).reshape(size)


# Model parameters of the workloads.  tau: BGK relaxation time; Gamma: mobility; b, kappa, c:
# Brazovskii free-energy coefficients; Tc, T0, Tw: critical, initial and wall temperatures;
# xi: thermal conductivity (a negative value stands for an infinitely fast quench).  _DEEP_QUENCH:
# the coefficients of the 64^2, 1024^2, 256^3 and ensemble workloads (walls at 0.7 Tc).
_DEEP_QUENCH = dict(Gamma=0.1, b=0.1, kappa=-0.006, c=0.0375, Tc=1.0, T0=1.5, Tw=0.7)

WORKLOADS = {
    # 64x64 D2Q9, periodic x, cold walls at y=0 and y=63: the parity workload.
    "c1_64sq": dict(dim=2, nx=64, ny=64, nz=1, walls=1, hydro=1, tau=1.0, xi=0.05, steps=2000,
                    seed=1, **_DEEP_QUENCH),
    # 1024x1024 D2Q9 at two viscosities: the throughput workload (S(k) and orientation every 1k).
    "c2_1024sq_tau0.6": dict(dim=2, nx=1024, ny=1024, nz=1, walls=1, hydro=1, tau=0.6, xi=0.01,
                             steps=50000, seed=1, **_DEEP_QUENCH),
    "c2_1024sq_tau2.0": dict(dim=2, nx=1024, ny=1024, nz=1, walls=1, hydro=1, tau=2.0, xi=0.01,
                             steps=50000, seed=1, **_DEEP_QUENCH),
    # 256^3 D3Q19, periodic x and y, cold walls at z=0 and z=255.
    "c3_256cube_xi0.001": dict(dim=3, nx=256, ny=256, nz=256, walls=1, hydro=1, tau=1.0,
                               xi=0.001, steps=20000, seed=1, **_DEEP_QUENCH),
    "c3_256cube_xi0.1": dict(dim=3, nx=256, ny=256, nz=256, walls=1, hydro=1, tau=1.0, xi=0.1,
                             steps=20000, seed=1, **_DEEP_QUENCH),
    # 4096x4096 D2Q9: a working set well above the last-level cache, for the HBM figure.
    "m1_4096sq": dict(dim=2, nx=4096, ny=4096, nz=1, walls=1, hydro=1, tau=0.6, xi=0.01,
                      steps=2000, seed=1, **_DEEP_QUENCH),
    # The paper's own parameter set (Section 3): 256x256, b=0.1, kappa=-c=-0.03, Tc=0.005,
    # Gamma=0.1, walls at 0.9 Tc, initial noise in [-0.01, 0.01]; tau=5 gives eta=1.5 (Fig. 2).
    "paper_2d_tau5": dict(dim=2, nx=256, ny=256, nz=1, walls=1, hydro=1, tau=5.0, xi=1e-3,
                          steps=20000, seed=1, Gamma=0.1, b=0.1, kappa=-0.03, c=0.03, Tc=0.005,
                          T0=0.0075, Tw=0.0045, amplitude=0.01),
    "paper_2d_nohydro": dict(dim=2, nx=256, ny=256, nz=1, walls=1, hydro=0, tau=1.0, xi=0.1,
                             steps=11700, seed=1, Gamma=0.1, b=0.1, kappa=-0.03, c=0.03,
                             Tc=0.005, T0=0.0075, Tw=0.0045, amplitude=0.01),
    "paper_3d_nohydro": dict(dim=3, nx=32, ny=32, nz=256, walls=1, hydro=0, tau=1.0, xi=1.0,
                             steps=1500, seed=1, Gamma=0.1, b=0.1, kappa=-0.03, c=0.03,
                             Tc=0.005, T0=0.0075, Tw=0.0045, amplitude=0.01),
}

MODEL_KEYS = ("dim", "nx", "ny", "nz", "walls", "hydro", "tau", "Gamma", "b", "kappa", "c",
              "Tc", "T0", "Tw", "xi")


def model_params(name_or_dict, **overrides) -> dict:
    """The model-parameter subset of a workload, with overrides applied."""
    w = dict(WORKLOADS[name_or_dict]) if isinstance(name_or_dict, str) else dict(name_or_dict)
    w.update(overrides)
    return {k: w[k] for k in MODEL_KEYS if k in w} | {
        k: w[k] for k in ("n_phi_sub", "n_T_sub", "force_form", "body_force", "pop_storage",
                          "allow_unstable", "tile_hint") if k in w}


def shape_of(p: dict):
    return (p["ny"], p["nx"]) if p["dim"] == 2 else (p["nz"], p["ny"], p["nx"])


def initial_phi(name_or_dict, seed=None, **overrides) -> np.ndarray:
    w = dict(WORKLOADS[name_or_dict]) if isinstance(name_or_dict, str) else dict(name_or_dict)
    w.update(overrides)
    return phi0(shape_of(w), seed=w.get("seed", 1) if seed is None else seed,
                amplitude=w.get("amplitude", 0.05))


def ensemble_members(seed: int = 1, count: int = 64, pop_storage: int = 1):
    """The batched-ensemble workload: `count` independent 2D runs with cold walls; side lengths
    log-uniform in [128, 512] (rounded), xi log-uniform in [1e-3, 1], tau uniform in
    [0.55, 3.0]; free-energy coefficients and temperatures as the 64^2 workload; populations
    stored in FP16 by default.  Draws come from three separate SplitMix64 streams of `seed`.
    Returns (parameter dicts, initial phi arrays)."""
    import math
    u_side = uniform01(seed, count, offset=1 << 40)
    u_xi = uniform01(seed, count, offset=2 << 40)
    u_tau = uniform01(seed, count, offset=3 << 40)
    members, phis = [], []
    for i in range(count):
        side = int(round(math.exp(math.log(128) + u_side[i] * (math.log(512) - math.log(128)))))
        xi = math.exp(math.log(1e-3) + u_xi[i] * (math.log(1.0) - math.log(1e-3)))
        tau = 0.55 + u_tau[i] * (3.0 - 0.55)
        p = dict(dim=2, nx=side, ny=side, nz=1, walls=1, hydro=1, tau=tau, xi=xi,
                 pop_storage=pop_storage, **_DEEP_QUENCH)
        members.append(p)
        phis.append(phi0((side, side), seed=seed * 1000 + i))
    return members, phis


def he_uniform(seed: int, shapes, head=None) -> np.ndarray:
    """Initial parameter vector of a stack of 3x3 convolutions: for each (C_in, C_out) in `shapes`
    the 9 C_out C_in weights are uniform in [-s, s], s = sqrt(6 / (9 C_in)) (He et al., 2015,
    uniform variant), followed by C_out zero biases; `head` = (C_in, C_out) of a final 1x1 layer,
    whose weights and biases start at zero.  Layer k draws from offset k << 32 of `seed`."""
    parts = []
    for k, (ci, co) in enumerate(shapes):
        s = np.sqrt(6.0 / (9 * ci))
        parts.append(s * (2.0 * uniform01(seed, 9 * ci * co, offset=k << 32) - 1.0))
        parts.append(np.zeros(co))
    if head is not None:
        parts.append(np.zeros(head[0] * head[1] + head[1]))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def surrogate_members(seed: int = 7, count: int = 8, side: int = 512, Tw: float = 0.95,
                      tau_range=(1.25, 2.0), instant: int = 0):
    """Training runs of the learned surrogate: `count` 2D runs on a side x side lattice with cold
    walls, xi log-uniform in [1e-3, 1] (the ensemble workload's distribution) and tau uniform in
    `tau_range`, free-energy coefficients of the 64^2 workload with the walls at Tw.  The default
    (walls at 0.95 Tc, tau in [1.25, 2]) is the part of the ensemble workload's range where the coupled
    scheme stays bounded over tens of thousands of steps at this size.  The last `instant` runs
    are quenched instantaneously (xi < 0: the whole lattice at Tw from the start).  Returns
    (parameter dicts, initial phi arrays)."""
    import math
    u_xi = uniform01(seed, count, offset=2 << 40)
    u_tau = uniform01(seed, count, offset=3 << 40)
    members, phis = [], []
    for i in range(count):
        xi = math.exp(math.log(1e-3) + u_xi[i] * (math.log(1.0) - math.log(1e-3)))
        if i >= count - instant:
            xi = -1.0
        tau = tau_range[0] + u_tau[i] * (tau_range[1] - tau_range[0])
        p = dict(dim=2, nx=side, ny=side, nz=1, walls=1, hydro=1, tau=tau, xi=xi,
                 **dict(_DEEP_QUENCH, Tw=Tw))
        members.append(p)
        phis.append(phi0((side, side), seed=seed * 1000 + i))
    return members, phis
