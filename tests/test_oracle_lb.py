"""Pins of the oracle's lattice-Boltzmann part against closed forms and independent computations.

Each test fixes a property that the paper's LB scheme (Section 2: eqs evoleqn, moment,
latticeforceterm, ff and the viscosity formula) implies, so that a plausible mistake (a wrong
weight, a transposed velocity, a dropped forcing term, a wrong half-step shift, a wrong wall
placement) fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import Oracle

# Velocity sets written out here, independently of the oracle's own tables.
D2Q9 = {(0, 0): 4 / 9, (1, 0): 1 / 9, (0, 1): 1 / 9, (-1, 0): 1 / 9, (0, -1): 1 / 9,
        (1, 1): 1 / 36, (-1, 1): 1 / 36, (-1, -1): 1 / 36, (1, -1): 1 / 36}
D3Q19 = {(0, 0, 0): 1 / 3}
for v in itertools.product((-1, 0, 1), repeat=3):
    m = sum(abs(c) for c in v)
    if m == 1:
        D3Q19[v] = 1 / 18
    elif m == 2:
        D3Q19[v] = 1 / 36


def base(dim=2, **kw):
    p = dict(dim=dim, nx=8, ny=8, nz=8 if dim == 3 else 1, walls=0, hydro=1, tau=1.0, Gamma=0.1,
             b=0.1, kappa=-0.006, c=0.0375, Tc=1.0, T0=1.0, Tw=1.0, xi=0.0)
    p.update(kw)
    return p


@pytest.mark.parametrize("dim", [2, 3])
def test_velocity_set_matches_standard(dim):
    e, w, opp = oracle.lattice(dim)
    ref = D2Q9 if dim == 2 else D3Q19
    got = {tuple(int(c) for c in e[q][:dim]): w[q] for q in range(len(w))}
    assert set(got) == set(ref)
    for k in ref:
        assert got[k] == pytest.approx(ref[k], rel=0, abs=1e-16)
    for q in range(len(w)):
        assert np.array_equal(e[opp[q]], -e[q])


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_and_forcing_moments(dim):
    """Moments fixed by Section 2: sum f^eq = n, sum f^eq e = n u, sum f^eq e e = n c_s^2 I + n u u;
    the forcing term has zero mass, momentum (1 - 1/2tau) F and second moment
    (1 - 1/2tau)(u F + F u)."""
    e, w, _ = oracle.lattice(dim)
    E = e[:, :dim].astype(float)
    rng = np.random.default_rng(3)
    for _ in range(5):
        n = 0.8 + 0.4 * rng.random()
        u = 0.1 * (rng.random(dim) - 0.5)
        F = 0.01 * (rng.random(dim) - 0.5)
        tau = 0.55 + 3 * rng.random()
        f = oracle.feq(dim, n, u)
        assert f.sum() == pytest.approx(n, abs=1e-14)
        np.testing.assert_allclose(E.T @ f, n * u, atol=1e-15)
        np.testing.assert_allclose(np.einsum("q,qa,qb->ab", f, E, E),
                                   n / 3 * np.eye(dim) + n * np.outer(u, u), atol=1e-15)
        g = oracle.guo(dim, tau, u, F)
        k = 1 - 0.5 / tau
        assert abs(g.sum()) < 1e-16
        np.testing.assert_allclose(E.T @ g, k * F, atol=1e-16)
        np.testing.assert_allclose(np.einsum("q,qa,qb->ab", g, E, E),
                                   k * (np.outer(u, F) + np.outer(F, u)), atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_body_force_momentum(dim):
    """Uniform acceleration g on a periodic fluid at rest: the momentum grows by exactly N n g per
    step, and the force-shifted velocity (eq. moment) is (t + 1/2) g at every site."""
    g = (1e-5, -2e-5, 3e-5)[:dim]
    p = base(dim, body_force=g, nx=6, ny=5, nz=4 if dim == 3 else 1)
    o = Oracle(p).init_fields(np.zeros(o_shape(p)))
    N = np.prod(o_shape(p))
    for t in (1, 7, 20):
        o.step(t - o.observables()["step"])
        ob = o.observables()
        np.testing.assert_allclose(ob["mom"], t * N * np.array(g), rtol=1e-12)
        u = o.fields()["u"].reshape(dim, -1)
        np.testing.assert_allclose(u, np.repeat((t + 0.5) * np.array(g)[:, None], N, 1), rtol=1e-11)


def o_shape(p):
    return (p["ny"], p["nx"]) if p["dim"] == 2 else (p["nz"], p["ny"], p["nx"])


def linear_lbe_shear_eigenvalue(vel, tau, k):
    """Slowest eigenvalue of the linearised BGK lattice Boltzmann operator for wavevector k,
    built here from the velocity set: streaming diag(exp(-i k.e)) times (I - (I - E)/tau),
    E = projector onto the linear equilibrium w (dn + 3 e.j)."""
    es = np.array(list(vel.keys()), float)
    ws = np.array(list(vel.values()))
    Q, d = es.shape
    Eq = np.zeros((Q, Q))
    for q in range(Q):
        Eq[q] = ws[q] * (1.0 + 3.0 * es @ es[q])
    A = np.diag(np.exp(-1j * es @ k)) @ (np.eye(Q) - (np.eye(Q) - Eq) / tau)
    lam = np.linalg.eigvals(A)
    # the transverse momentum mode: eigenvalue nearest the continuum decay exp(-nu k^2)
    nu = (tau - 0.5) / 3
    return lam[np.argmin(np.abs(lam - math.exp(-nu * (k @ k))))]


@pytest.mark.parametrize("dim,tau", [(2, 0.6), (2, 1.0), (2, 2.0), (3, 1.0)])
def test_shear_wave_decay(dim, tau):
    """Shear wave u_x = U0 sin(2 pi y / L) decays at the LBE eigenvalue (exact for the discrete
    scheme) and at nu k^2 with nu = (tau - 1/2)/3 (Section 2, viscosity formula) within the
    lattice error, which at L = 64 is below 1% for tau <= 2."""
    L, U0 = 64, 1e-4
    p = base(dim, nx=4, ny=L, nz=4 if dim == 3 else 1, tau=tau, Gamma=0.0, kappa=0.0, c=0.0)
    shp = o_shape(p)
    y = np.arange(L)
    prof = U0 * np.sin(2 * np.pi * y / L)
    u0 = np.zeros((dim,) + shp)
    if dim == 2:
        u0[0] = prof[:, None]
    else:
        u0[0] = prof[None, :, None]
    o = Oracle(p).init_fields(np.zeros(shp), u0=u0)

    def amp():
        ux = o.fields()["u"][0]
        ux = ux if dim == 2 else ux[0]
        return 2.0 / L * (ux[:, 0] * np.sin(2 * np.pi * y / L)).sum()

    o.step(200)
    a1 = amp()
    o.step(300)
    a2 = amp()
    k = np.zeros(dim)
    k[1] = 2 * np.pi / L
    vel = D2Q9 if dim == 2 else D3Q19
    lam = linear_lbe_shear_eigenvalue(vel, tau, k)
    assert a2 / a1 == pytest.approx(abs(lam) ** 300, rel=1e-6)
    rate = -math.log(a2 / a1) / 300
    nu = (tau - 0.5) / 3
    assert rate == pytest.approx(nu * k @ k, rel=1e-2)


def test_viscosity_of_paper_tau5():
    """Section 3 quotes eta = 1.5 for tau = 5 (Fig. 2); with n = 1, nu = eta.  Measured on a
    256-long shear wave, where the lattice error is well below 1%."""
    L, U0, tau = 256, 1e-4, 5.0
    p = base(2, nx=4, ny=L, tau=tau, Gamma=0.0, kappa=0.0, c=0.0)
    y = np.arange(L)
    u0 = np.zeros((2, L, 4))
    u0[0] = (U0 * np.sin(2 * np.pi * y / L))[:, None]
    o = Oracle(p).init_fields(np.zeros((L, 4)), u0=u0)

    def amp():
        return 2.0 / L * (o.fields()["u"][0][:, 0] * np.sin(2 * np.pi * y / L)).sum()

    o.step(100)
    a1 = amp()
    o.step(400)
    a2 = amp()
    nu = -math.log(a2 / a1) / 400 / (2 * np.pi / L) ** 2
    assert nu == pytest.approx(1.5, rel=1e-2)


def test_poiseuille_halfway_bounce_back():
    """Walls half a spacing outside the first and last fluid layers (Section 2 bounce-back):
    a body-force-driven channel reaches u(y) = g/(2 nu) (y + 1/2)(L_y - 1/2 - y); for BGK the
    bounce-back wall sits exactly there when tau = 1/2 + sqrt(3)/4, and for any tau the steady
    profile has second difference exactly -g/nu."""
    ny, g = 16, 1e-6
    y = np.arange(ny)
    for tau, tol in ((0.5 + math.sqrt(3) / 4, 1e-9), (1.0, 2e-3)):
        p = base(2, nx=4, ny=ny, walls=1, tau=tau, Gamma=0.0, kappa=0.0, c=0.0,
                 body_force=(g, 0.0))
        o = Oracle(p).init_fields(np.zeros((ny, 4)))
        o.step(20000)
        u = o.fields()["u"][0][:, 0]
        nu = (tau - 0.5) / 3
        exact = g / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
        assert np.abs(u - exact).max() <= tol * exact.max()
        np.testing.assert_allclose(np.diff(u, 2), -g / nu, rtol=1e-8)
        assert np.abs(o.fields()["u"][1]).max() < 1e-10 * exact.max()


@pytest.mark.parametrize("dim", [2, 3])
def test_bounce_back_conserves_mass(dim):
    """Bounce-back at the walls conserves mass exactly (Section 2): random initial density and
    velocity, walls on, 300 steps."""
    p = base(dim, nx=8, ny=10, nz=6 if dim == 3 else 1, walls=1, T0=1.5, Tw=0.9, xi=0.1)
    shp = o_shape(p)
    rng = np.random.default_rng(5)
    n0 = 1 + 0.01 * (rng.random(shp) - 0.5)
    u0 = 0.01 * (rng.random((dim,) + shp) - 0.5)
    phi0 = 0.05 * (rng.random(shp) - 0.5)
    o = Oracle(p).init_fields(phi0, u0=u0, n0=n0)
    m0 = o.observables()["mass_dev"]
    s0 = o.observables()["phi_sum"]
    o.step(300)
    ob = o.observables()
    N = np.prod(shp)
    assert abs(ob["mass_dev"] - m0) < 1e-13 * N
    assert abs(ob["phi_sum"] - s0) < 1e-13 * N * 0.05
