"""Pins of the oracle's finite-difference parts (order parameter and temperature) and of the
full coupled step against closed forms, exact discrete solutions and invariants.

Paper references: eq. (chem) for mu, eq. (massdiff) for phi, the temperature diffusion equation
and cold walls of Section 2, eq. (ff) for the force, the single-mode lamellar theory of Section 2.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

import synthetic as S
from oracle import Oracle


def par(dim=2, **kw):
    p = dict(dim=dim, nx=16, ny=16, nz=16 if dim == 3 else 1, walls=0, hydro=0, tau=1.0,
             Gamma=0.1, b=0.0, kappa=-0.006, c=0.0375, Tc=1.0, T0=1.3, Tw=1.3, xi=0.0)
    p.update(kw)
    return p


def grid(p):
    if p["dim"] == 2:
        y, x = np.mgrid[0:p["ny"], 0:p["nx"]]
        return x, y, None
    z, y, x = np.mgrid[0:p["nz"], 0:p["ny"], 0:p["nx"]]
    return x, y, z


def a_of(p):
    return (p["T0"] - p["Tc"]) / p["Tc"]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("walls", [0, 1])
def test_mu_linear_symbol(dim, walls):
    """mu = a phi - kappa lap phi + c lap^2 phi (eq. chem, b = 0) on a lattice eigenmode:
    lap -> -lambda, lap^2 -> lambda^2, lambda = sum_alpha 2(1 - cos k_alpha).  With walls the
    eigenmodes are cos(pi m (y + 1/2)/L_y) along the wall axis, which pins the even reflection
    about planes half a spacing outside the first and last layers."""
    p = par(dim, walls=walls, nx=12, ny=10, nz=8 if dim == 3 else 1)
    x, y, z = grid(p)
    rng = np.random.default_rng(11)
    for _ in range(4):
        m = rng.integers(0, 5, size=3)
        kx = 2 * np.pi * m[0] / p["nx"]
        if dim == 2:
            ky = (np.pi * m[1] / p["ny"]) if walls else 2 * np.pi * m[1] / p["ny"]
            fy = np.cos(ky * (y + 0.5)) if walls else np.cos(ky * y)
            phi = 1e-3 * np.cos(kx * x + 0.3) * fy
            lam = 2 * (1 - math.cos(kx)) + 2 * (1 - math.cos(ky))
        else:
            ky = 2 * np.pi * m[1] / p["ny"]
            kz = (np.pi * m[2] / p["nz"]) if walls else 2 * np.pi * m[2] / p["nz"]
            fz = np.cos(kz * (z + 0.5)) if walls else np.cos(kz * z)
            phi = 1e-3 * np.cos(kx * x + 0.3) * np.cos(ky * y - 0.2) * fz
            lam = sum(2 * (1 - math.cos(k)) for k in (kx, ky, kz))
        o = Oracle(p).init_fields(phi)
        mu = o.mu()
        sym = a_of(p) + p["kappa"] * lam + p["c"] * lam ** 2
        np.testing.assert_allclose(mu, sym * phi, atol=1e-13 * np.abs(phi).max())


def test_mu_cubic_term():
    """The b phi^3 term of eq. (chem): for a uniform field mu = a phi + b phi^3 exactly."""
    p = par(b=0.1, T0=0.7, Tw=0.7)
    phi = np.full((16, 16), 1.7)
    mu = Oracle(p).init_fields(phi).mu()
    np.testing.assert_allclose(mu, -0.3 * 1.7 + 0.1 * 1.7 ** 3, rtol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_force_total_vanishes_and_uniform_field(dim):
    """F = -div P telescopes: the total force vanishes on a periodic lattice with uniform a
    (momentum conservation), and vanishes pointwise for a uniform phi."""
    p = par(dim, hydro=1, b=0.1, T0=0.8, Tw=0.8, nx=10, ny=12, nz=6 if dim == 3 else 1)
    shp = (p["ny"], p["nx"]) if dim == 2 else (p["nz"], p["ny"], p["nx"])
    rng = np.random.default_rng(2)
    phi = rng.random(shp) - 0.5
    F = Oracle(p).init_fields(phi).force()
    for k in range(dim):
        assert abs(F[k].sum()) < 1e-13 * phi.size * np.abs(F).max()
    F0 = Oracle(p).init_fields(np.full(shp, 0.37)).force()
    assert np.abs(F0).max() < 1e-15


def test_force_tangential_total_vanishes_with_walls():
    """With walls the tangential total force still vanishes (P_xy is odd across the wall)."""
    p = par(hydro=1, walls=1, b=0.1, T0=0.8, Tw=0.8, nx=10, ny=12)
    phi = np.random.default_rng(4).random((12, 10)) - 0.5
    F = Oracle(p).init_fields(phi).force()
    assert abs(F[0].sum()) < 1e-13 * phi.size * np.abs(F).max()


def test_force_forms_agree_to_second_order():
    """-div P^phi equals -phi grad mu in the continuum for uniform a (the pressure tensor of
    Section 2 is built so that its divergence is phi grad mu); the two discrete forms must
    therefore differ by O(h^2): refining a fixed smooth pattern by 2 divides the gap by ~4."""
    gaps = []
    for L in (64, 128, 256):
        p = par(hydro=1, b=0.1, T0=0.8, Tw=0.8, nx=L, ny=L)
        x, y, _ = grid(p)
        phi = 0.8 * np.sin(2 * np.pi * 2 * x / L) + 0.5 * np.cos(2 * np.pi * 3 * y / L) * np.sin(
            2 * np.pi * x / L)
        F0 = Oracle(p).init_fields(phi).force()
        F1 = Oracle(dict(p, force_form=1)).init_fields(phi).force()
        gaps.append(np.abs(F0 - F1).max() / np.abs(F1).max())
    order = [math.log2(gaps[i] / gaps[i + 1]) for i in range(2)]
    assert min(order) > 1.9, (gaps, order)


@pytest.mark.parametrize("n_phi", [1, 2, 3])
@pytest.mark.parametrize("dim", [2, 3])
def test_linear_growth_factor(dim, n_phi):
    """Without flow and with b = 0 the phi update is linear and diagonal in Fourier space: one LB
    step of n_phi Euler sub-steps multiplies mode k by G = [1 - (Gamma/n_phi) lambda (a + kappa
    lambda + c lambda^2)]^n_phi (eqs massdiff and chem)."""
    p = par(dim, n_phi_sub=n_phi, T0=1.0002, Tw=1.0002, nx=12, ny=10, nz=8 if dim == 3 else 1)
    x, y, z = grid(p)
    a = a_of(p)
    for m in ((1, 0, 0), (2, 3, 1), (6, 5, 4), (3, 1, 2)):
        kx, ky = 2 * np.pi * m[0] / p["nx"], 2 * np.pi * m[1] / p["ny"]
        if dim == 2:
            phi = 1e-4 * np.cos(kx * x + ky * y + 0.1)
            lam = 2 * (1 - math.cos(kx)) + 2 * (1 - math.cos(ky))
        else:
            kz = 2 * np.pi * m[2] / p["nz"]
            phi = 1e-4 * np.cos(kx * x + ky * y + kz * z + 0.1)
            lam = sum(2 * (1 - math.cos(k)) for k in (kx, ky, kz))
        o = Oracle(p).init_fields(phi).step(1)
        G = (1 - p["Gamma"] / n_phi * lam * (a + p["kappa"] * lam + p["c"] * lam ** 2)) ** n_phi
        np.testing.assert_allclose(o.fields()["phi"], G * phi, atol=1e-12 * 1e-4)


def test_growth_rate_continuum_limit():
    """The discrete rate ln G converges to omega(k) = -Gamma k^2 (a + kappa k^2 + c k^4) as k -> 0,
    with the O(k^2) relative error of second-order differences."""
    p0 = par(T0=0.9, Tw=0.9, n_phi_sub=1)
    a = a_of(p0)
    errs = []
    for L in (64, 128, 256):
        p = dict(p0, nx=L, ny=4)
        x, _, _ = grid(p)
        k = 2 * np.pi * 4 / L
        phi = 1e-6 * np.cos(k * x)
        o = Oracle(p).init_fields(phi).step(1)
        G = o.fields()["phi"][0, 0] / phi[0, 0]
        om = -p["Gamma"] * k * k * (a + p["kappa"] * k * k + p["c"] * k ** 4)
        errs.append(abs(math.log(G) - om) / abs(om))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_lamellar_wavenumber_onset_1d():
    """k0^2 = -kappa/(2c) (Section 2).  Just below the onset a < kappa^2/(4c), on a 64-wide lattice
    only the mode closest to k0 grows: with kappa = -0.006, c = 0.0375 and a = 2.0e-4 that is m = 3
    (k = 0.2945, k0 = 0.2828); m = 2 and m = 4 decay."""
    p = par(nx=64, ny=4, T0=1.0002, Tw=1.0002, b=0.1, n_phi_sub=1)
    x, _, _ = grid(p)
    phi = 1e-8 * sum(np.cos(2 * np.pi * m * x / 64 + 0.7 * m) for m in range(1, 8))
    o = Oracle(p).init_fields(phi).step(400)
    f0 = np.abs(np.fft.fft(phi[0]))
    f1 = np.abs(np.fft.fft(o.fields()["phi"][0]))
    grows = {m for m in range(1, 8) if f1[m] > f0[m]}
    assert grows == {3}
    k0 = math.sqrt(-p["kappa"] / (2 * p["c"]))
    assert k0 == pytest.approx(0.28284, abs=1e-5)


def test_lamellar_onset_2d_set():
    """On 64x64 with a 2D random field the growing modes at a = 2.0e-4 are exactly those with
    a + kappa lambda + c lambda^2 < 0: (2,2), (3,0), (3,1), (2,1) and their images."""
    p = par(nx=64, ny=64, T0=1.0002, Tw=1.0002, b=0.1, n_phi_sub=1)
    phi = 1e-8 * (S.phi0((64, 64), seed=3) / 0.05)
    o = Oracle(p).init_fields(phi).step(300)
    f0 = np.abs(np.fft.fft2(phi))
    f1 = np.abs(np.fft.fft2(o.fields()["phi"]))
    grows = {(int(i), int(j)) for i, j in zip(*np.nonzero(f1 > f0))}
    canon = {tuple(sorted((min(i, 64 - i), min(j, 64 - j)))) for i, j in grows}
    assert canon == {(2, 2), (0, 3), (1, 3), (1, 2)}


def test_substep_rule():
    """Automatic sub-step counts: kappa = -0.006, c = 0.0375, a down to -0.3 need 2 phi sub-steps in 2D and 5 in 3D,
    the paper's coefficients 1 in 2D; n_T = ceil(xi / 0.45)."""
    assert Oracle(S.model_params("c1_64sq")).substeps == (2, 1)
    assert Oracle(S.model_params("c3_256cube_xi0.1", nx=8, ny=8, nz=8)).substeps == (5, 1)
    assert Oracle(S.model_params("paper_2d_tau5", nx=16, ny=16)).substeps == (1, 1)
    assert Oracle(S.model_params("c1_64sq", xi=1.0)).substeps[1] == 3


def test_stability_guard():
    """With kappa = -0.006, c = 0.0375 one Euler step per LB step is unstable at the checkerboard mode
    (G = -1.28 at a = 0.5), while the automatic count keeps the phi equation bounded."""
    p = S.model_params("c1_64sq", hydro=0)
    phi0 = S.initial_phi("c1_64sq")
    bad = Oracle(dict(p, n_phi_sub=1)).init_fields(phi0).step(300)
    ok = Oracle(p).init_fields(phi0).step(300)
    fb = bad.fields()["phi"]
    assert (not np.isfinite(fb).all()) or np.abs(fb).max() > 1e3
    assert np.abs(ok.fields()["phi"]).max() < 3.0


def dst_solution(L, T0, Tw, r, t):
    M = L - 1
    j = np.arange(1, M)
    e0 = np.full(M - 1, T0 - Tw)
    out = np.zeros(L)
    for m in range(1, M):
        s = np.sin(m * np.pi * j / M)
        cm = 2.0 / M * (e0 * s).sum()
        g = 1 - 4 * r * math.sin(m * np.pi / (2 * M)) ** 2
        out[1:M] += cm * g ** t * s
    return Tw + out


@pytest.mark.parametrize("xi", [0.05, 1.0])
def test_temperature_exact_discrete(xi):
    """FTCS with Dirichlet wall layers has the exact solution
    T_j - Tw = sum_m c_m [1 - 4 r sin^2(m pi / 2M)]^t sin(m pi j / M), M = L_y - 1."""
    L = 24
    p = par(nx=4, ny=L, walls=1, T0=1.5, Tw=0.7, xi=xi)
    o = Oracle(p).init_fields(np.zeros((L, 4)))
    nT = o.substeps[1]
    o.step(40)
    T = o.fields()["T"]
    exact = dst_solution(L, 1.5, 0.7, xi / nT, 40 * nT)
    np.testing.assert_allclose(T, np.repeat(exact[:, None], 4, 1), atol=1e-12)


def test_temperature_erfc_front():
    """Cold fronts from the two walls follow the diffusive profile
    Tw + (T0 - Tw)[erf(y / 2 sqrt(xi t)) + erf((L_y - 1 - y) / 2 sqrt(xi t)) - 1]."""
    L, xi = 64, 0.05
    p = par(nx=4, ny=L, walls=1, T0=1.5, Tw=0.7, xi=xi)
    o = Oracle(p).init_fields(np.zeros((L, 4)))
    y = np.arange(L)
    t = 0
    for tt in (200, 600, 2000):
        o.step(tt - t)
        t = tt
        T = o.fields()["T"][:, 0]
        s = 2 * math.sqrt(xi * t)
        cont = 0.7 + 0.8 * (erf(y / s) + erf((L - 1 - y) / s) - 1)
        assert np.abs(T - cont).max() < 5e-3 * 0.8


def test_conservation_full_model_walls():
    """Full coupled model with walls (C1 geometry, milder wall temperature so that the run stays
    bounded): total mass and total phi are conserved to round-off over 1000 steps."""
    p = S.model_params("c1_64sq", Tw=0.9)
    o = Oracle(p).init_fields(S.initial_phi("c1_64sq"))
    ob0 = o.observables()
    o.step(1000)
    ob = o.observables()
    N = 64 * 64
    assert not ob["nonfinite"]
    assert abs(ob["mass_dev"] - ob0["mass_dev"]) < 1e-12 * N
    assert abs(ob["phi_sum"] - ob0["phi_sum"]) < 1e-12 * N
    assert ob["max_u"] > 1e-3  # the flow is actually driven


def test_momentum_conservation_periodic():
    """Periodic lattice, uniform temperature: the pressure-tensor force telescopes, so the total
    momentum stays at its initial value (zero) to round-off."""
    p = S.model_params("c1_64sq", walls=0, T0=0.9, Tw=0.9)
    o = Oracle(p).init_fields(S.initial_phi("c1_64sq")).step(300)
    ob = o.observables()
    assert ob["max_u"] > 1e-4
    assert np.abs(ob["mom"]).max() < 1e-13 * 64 * 64


def test_conservation_3d_walls():
    p = S.model_params("c3_256cube_xi0.1", nx=12, ny=10, nz=14)
    phi0 = S.phi0((14, 10, 12), seed=2)
    o = Oracle(p).init_fields(phi0)
    ob0 = o.observables()
    o.step(60)
    ob = o.observables()
    assert abs(ob["mass_dev"] - ob0["mass_dev"]) < 1e-12 * phi0.size
    assert abs(ob["phi_sum"] - ob0["phi_sum"]) < 1e-12 * phi0.size


def test_hydro_off_leaves_fluid_at_rest():
    """Without hydrodynamics (Section 3, Figs 1 and 3) phi evolves by diffusion of mu only."""
    p = S.model_params("c1_64sq", hydro=0)
    o = Oracle(p).init_fields(S.initial_phi("c1_64sq")).step(20)
    f = o.fields()
    assert np.abs(f["u"]).max() == 0.0
    np.testing.assert_allclose(f["n"], 1.0, atol=1e-15)
