"""Pins of the oracle's observables, of its checkpoint and of symmetries of the scheme, and the
values the paper prints (tests/golden/paper_values.json)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synthetic as S
from oracle import Oracle, spectra

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def par(**kw):
    p = dict(dim=2, nx=64, ny=8, nz=1, walls=0, hydro=0, tau=1.0, Gamma=0.1, b=0.1,
             kappa=-0.006, c=0.0375, Tc=1.0, T0=0.8, Tw=0.8, xi=0.0)
    p.update(kw)
    return p


def fe_per_site(p, phi):
    o = Oracle(p).init_fields(phi)
    return o.observables()["free_energy"] / phi.size


def test_free_energy_single_mode_closed_form():
    """For phi = A sin(k x) on a lattice mode with 4k != 0 mod 2 pi the discrete free energy per
    site is (A^2/4)(a + kappa lambda + c lambda^2) + (3b/32) A^4, lambda = 2(1 - cos k)."""
    p = par()
    x = np.arange(64)[None, :].repeat(8, 0)
    a = (p["T0"] - p["Tc"]) / p["Tc"]
    for m, A in ((3, 0.7), (5, 1.9), (11, 0.2)):
        k = 2 * np.pi * m / 64
        lam = 2 * (1 - math.cos(k))
        got = fe_per_site(p, A * np.sin(k * x))
        want = A * A / 4 * (a + p["kappa"] * lam + p["c"] * lam ** 2) + 3 * p["b"] / 32 * A ** 4
        assert got == pytest.approx(want, rel=1e-13, abs=1e-16)


def test_free_energy_uniform_and_wall_gradient():
    """Uniform phi: a phi^2/2 + b phi^4/4 per site.  With walls, a profile varying only along the
    wall normal gets no gradient energy across the wall (even reflection)."""
    p = par(walls=1)
    v = 0.9
    assert fe_per_site(p, np.full((8, 64), v)) == pytest.approx(
        -0.2 * v * v / 2 + 0.1 * v ** 4 / 4, rel=1e-14)
    prof = np.linspace(-1, 1, 8)[:, None].repeat(64, 1)
    o = Oracle(dict(p, b=0.0, c=0.0, kappa=2.0, T0=1.0, Tw=1.0)).init_fields(prof)
    # only kappa/2 sum (phi(y+1) - phi(y))^2 over the 7 interior links remains
    want = 64 * 7 * (2.0 / 7) ** 2
    assert o.observables()["free_energy"] == pytest.approx(want, rel=1e-13)


def test_paper_single_mode_amplitude_and_transition():
    """The paper's single-mode theory (Section 2, printed in the golden file): at |a| = b the
    lamellar amplitude is A^2 = 4(1 + kappa^2/(4 c b))/3 with k0 = sqrt(-kappa/2c), and the
    lamellar phase becomes favourable below a = -1.11 kappa^2/c.  Checked on the oracle's
    free-energy observable with the paper's coefficients, on the lattice mode nearest k0."""
    g = GOLDEN["parameters_section3"]
    b, kap, c = g["b"], g["kappa"], g["c"]
    k0 = math.sqrt(-kap / (2 * c))
    L = 256
    m = round(k0 * L / (2 * math.pi))
    x = np.arange(L)[None, :].repeat(4, 0)
    k = 2 * math.pi * m / L

    def params(a):
        return dict(par(nx=L, ny=4, b=b, kappa=kap, c=c), Tc=1.0, T0=1.0 + a, Tw=1.0 + a)

    def lamellar_min(a):
        # f(A) = alpha A^2 + beta A^4 measured at two amplitudes, then minimised analytically
        f1 = fe_per_site(params(a), 0.5 * np.sin(k * x))
        f2 = fe_per_site(params(a), 1.0 * np.sin(k * x))
        beta = (f2 - 4 * f1) / (1.0 - 4 * 0.0625)
        alpha = (f2 - beta) / 1.0
        return alpha, beta

    alpha, beta = lamellar_min(-b)
    A2 = -alpha / (2 * beta)
    A2_paper = 4 * (1 + kap * kap / (4 * c * b)) / 3
    assert A2 == pytest.approx(A2_paper, rel=1e-2)

    def gap(a):
        al, be = lamellar_min(a)
        lam_f = -al * al / (4 * be)
        uni = fe_per_site(params(a), np.full((4, L), math.sqrt(-a / b)))
        return lam_f - uni

    lo, hi = -0.1, -0.001
    assert gap(lo) > 0 > gap(hi)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if gap(mid) > 0 else (lo, mid)
    a_t = 0.5 * (lo + hi)
    coef = GOLDEN["single_mode_theory"]["transition_coefficient"]
    assert a_t == pytest.approx(coef * kap * kap / c, rel=1.5e-2)


def test_checkpoint_resume_bitwise():
    p = S.model_params("c1_64sq", Tw=0.9)
    phi0 = S.initial_phi("c1_64sq")
    ref = Oracle(p).init_fields(phi0).step(120)
    a = Oracle(p).init_fields(phi0).step(60)
    blob = a.get_state()
    b = Oracle(p).set_state(blob).step(60)
    for k in ("phi", "u", "n", "T"):
        assert np.array_equal(ref.fields()[k], b.fields()[k])
    assert np.array_equal(ref.populations(), b.populations())
    assert b.observables()["step"] == 120
    with pytest.raises(ValueError):
        Oracle(S.model_params("c1_64sq", nx=32)).set_state(blob)


def test_x_roll_equivariance_bitwise():
    """Every operation is the same at every site, so rolling the initial field along the periodic
    axis rolls every later field bit for bit."""
    p = S.model_params("c1_64sq", Tw=0.9)
    phi0 = S.initial_phi("c1_64sq")
    a = Oracle(p).init_fields(phi0).step(40).fields()
    b = Oracle(p).init_fields(np.roll(phi0, 5, axis=1)).step(40).fields()
    assert np.array_equal(np.roll(a["phi"], 5, axis=1), b["phi"])
    assert np.array_equal(np.roll(a["u"], 5, axis=2), b["u"])


def test_wall_mirror_symmetry():
    """A field symmetric under y -> L_y - 1 - y stays symmetric (walls and fronts are symmetric);
    the normal velocity changes sign.  Round-off only, since sums over the velocity set are not
    mirror-ordered."""
    p = S.model_params("c1_64sq", Tw=0.9)
    phi0 = S.initial_phi("c1_64sq")
    phi0 = 0.5 * (phi0 + phi0[::-1])
    f = Oracle(p).init_fields(phi0).step(100).fields()
    assert np.abs(f["phi"] - f["phi"][::-1]).max() < 1e-13 * np.abs(f["phi"]).max()
    # velocities are differences of O(1) populations: round-off is absolute, about 1e-16 per step
    assert np.abs(f["u"][1] + f["u"][1][::-1]).max() < 1e-14


def test_shell_index_exact():
    for nx, ny in ((12, 20), (16, 16), (9, 7), (64, 48)):
        b = spectra.shell_index(nx, ny)
        for j in range(ny):
            for i in range(nx):
                mx = i if i < (nx + 1) // 2 else i - nx
                my = j if j < (ny + 1) // 2 else j - ny
                num = mx * mx * ny * ny + my * my * nx * nx
                q = num // (max(nx, ny) ** 2)
                assert b[j, i] == math.isqrt(q)


def test_structure_factor_single_mode_and_parseval():
    nx, ny, A = 48, 32, 0.3
    y, x = np.mgrid[0:ny, 0:nx]
    phi = 0.1 + A * np.cos(2 * np.pi * (5 * x / nx + 3 * y / ny))
    r = spectra.structure_factor(phi, 24)
    N = nx * ny
    kk = 2 * np.pi * math.hypot(5 / nx, 3 / ny)
    b = int(kk / r["dk"])
    assert r["S"][b] * r["counts"][b] == pytest.approx(2 * A * A * N / 4, rel=1e-12)
    assert np.count_nonzero(r["S"] > 1e-20) == 1
    assert r["k_mean"] == pytest.approx(kk, rel=1e-12)
    rng = np.random.default_rng(0)
    phi = rng.random((ny, nx))
    r = spectra.structure_factor(phi, 10 ** 6 // 1000)
    ph = np.fft.fft2(phi - phi.mean())
    tot = (np.abs(ph) ** 2).sum() / N
    assert tot == pytest.approx(((phi - phi.mean()) ** 2).sum(), rel=1e-12)


def test_orientation_of_stripes():
    nx, ny = 64, 32
    y, x = np.mgrid[0:ny, 0:nx]
    par_ = spectra.orientation(np.cos(2 * np.pi * 4 * (y + 0.5) / (2 * ny)), 18, walls=True)
    assert par_["Q"] == pytest.approx(1.0, abs=1e-12)
    assert par_["hist"][9] == pytest.approx(1.0, abs=1e-12)
    perp = spectra.orientation(np.cos(2 * np.pi * 4 * x / nx), 18, walls=True)
    assert perp["Q"] == pytest.approx(-1.0, abs=1e-12)
    assert perp["hist"][0] + perp["hist"][17] == pytest.approx(1.0, abs=1e-12)
    diag = spectra.orientation(np.cos(2 * np.pi * 4 * (x + y) / nx), 18, walls=False)
    assert diag["Q"] == pytest.approx(0.0, abs=1e-12)
    assert diag["hist"][4] == pytest.approx(1.0, abs=1e-12)


def test_orientation_3d_stripes_and_isotropy():
    """3D orientation: lamellae normal to z (parallel to the walls) give Q = +1 and all weight in
    the first angle bin; lamellae normal to x or y give Q = -1/2 and all weight in the last bin;
    a field whose gradients point along the three axes in equal measure gives Q = 0 (the second
    Legendre polynomial averages to zero over directions)."""
    nz, ny, nx = 24, 16, 20
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    par = np.cos(2 * np.pi * 3 * (z + 0.5) / (2 * nz))       # even across the wall planes
    r = spectra.orientation(par, 9, walls=True)
    assert r["Q"] == pytest.approx(1.0, abs=1e-12)
    assert r["hist"][0] == pytest.approx(1.0, abs=1e-12)
    np.testing.assert_allclose(r["Q_row"][r["weight"].sum(axis=(1, 2)) > 0], 1.0, atol=1e-12)
    for perp in (np.sin(2 * np.pi * 2 * x / nx) + 0 * z, np.cos(2 * np.pi * 3 * y / ny) + 0 * z):
        r = spectra.orientation(perp, 9, walls=True)
        assert r["Q"] == pytest.approx(-0.5, abs=1e-12)
        assert r["hist"][-1] == pytest.approx(1.0, abs=1e-12)
    z, y, x = np.mgrid[0:16, 0:16, 0:16]
    k = 2 * np.pi * 3 / 16
    iso = np.sin(k * x) + np.sin(k * y + 0.3) + np.sin(k * z + 0.7)
    r = spectra.orientation(iso, 9, walls=False)
    assert abs(r["Q"]) < 1e-12
