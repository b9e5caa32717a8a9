"""Pins of the surrogate oracle (U-Net forward and backward, FP64) against what mathematics fixes:
brute-force sums, adjoint identities, finite differences, translation equivariance, and the
bfloat16 rounding of a library routine."""
import itertools

import numpy as np
import pytest
import torch

import synthetic as S
from oracle import surrogate as U


def rng(seed):
    return np.random.default_rng(seed)


def test_conv3x3_brute_force():
    """Cross-correlation over the 3x3 taps, periodic in x and zero outside the walls, summed in
    plain Python loops."""
    H, W, ci, co = 4, 5, 2, 3
    r = rng(1)
    x = r.normal(size=(H, W, ci))
    Wt = r.normal(size=(9, co, ci))
    b = r.normal(size=co)
    got = U.conv3x3(x, Wt, b)
    for y, xx, o in itertools.product(range(H), range(W), range(co)):
        s = b[o]
        for dy, dx, c in itertools.product((-1, 0, 1), (-1, 0, 1), range(ci)):
            yy = y + dy
            if 0 <= yy < H:
                s += Wt[3 * (dy + 1) + dx + 1, o, c] * x[yy, (xx + dx) % W, c]
        assert got[y, xx, o] == pytest.approx(s, abs=1e-12)


def test_conv_adjoints():
    """<conv(x), g> = <x, input_grad(g)> = <W, weight_grad(x, g)>: the two gradients are the
    adjoints of the bilinear map, whatever the shapes."""
    r = rng(2)
    for H, W, ci, co in [(6, 7, 3, 4), (8, 8, 5, 2), (1, 3, 1, 1)]:
        x = r.normal(size=(H, W, ci))
        Wt = r.normal(size=(9, co, ci))
        g = r.normal(size=(H, W, co))
        lhs = np.sum(U.conv3x3(x, Wt, np.zeros(co)) * g)
        assert np.sum(x * U.conv3x3_input_grad(g, Wt)) == pytest.approx(lhs, rel=1e-12)
        dW, db = U.conv3x3_weight_grad(x, g)
        assert np.sum(Wt * dW) == pytest.approx(lhs, rel=1e-12)
        assert np.allclose(db, g.sum(axis=(0, 1)))


def test_pool_up_adjoint():
    r = rng(3)
    x = r.normal(size=(8, 6, 3))
    y = r.normal(size=(4, 3, 3))
    assert np.sum(U.pool(x) * y) == pytest.approx(np.sum(x * U.up(y) / 4.0), rel=1e-13)
    assert U.pool(U.up(y)) == pytest.approx(y, abs=1e-15)


def test_silu_derivative():
    z = np.linspace(-8, 8, 33)
    h = 1e-6
    fd = (U.silu(z + h) - U.silu(z - h)) / (2 * h)
    assert np.abs(fd - U.dsilu(z)).max() < 1e-9
    assert U.silu(np.array([0.0]))[0] == 0.0 and U.dsilu(np.array([0.0]))[0] == 0.5


def test_bf16_rounding_matches_torch():
    """Round to nearest even, as torch's float32 -> bfloat16 conversion does."""
    r = rng(4)
    x = np.concatenate([r.normal(size=1000) * 10.0 ** r.integers(-6, 6, size=1000),
                        [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8, 0.0]])
    x = x.astype(np.float32).astype(np.float64)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16(x), ref)
    assert U.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0            # tie -> even
    assert U.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def small_net(seed=5, widths=(4, 6, 8), H=8, W=12):
    shapes = [(ci, co) for _, ci, co in U.layers(widths)]
    theta = S.he_uniform(seed, shapes, head=(widths[0], U.OUT_CH))
    r = rng(seed)
    theta[-(U.OUT_CH * widths[0] + U.OUT_CH):] = r.normal(size=U.OUT_CH * widths[0] + U.OUT_CH)
    for name, (Wt, b) in U.split(theta, widths).items():
        b[...] = 0.1 * r.normal(size=b.shape)
    x = r.normal(size=(H, W, U.IN_CH))
    t = r.normal(size=(H, W, U.OUT_CH))
    return theta, x, t, widths


def test_parameter_layout():
    widths = (32, 64, 128, 256)
    assert U.param_count(widths) == 1947523
    th = np.arange(U.param_count(widths), dtype=np.float64)
    P = U.split(th, widths)
    assert P["e1a"][0].shape == (9, 32, 5) and P["d3a"][0].shape == (9, 128, 384)
    assert P["e1a"][0][0, 0, 0] == 0 and P["e1a"][1][0] == 9 * 32 * 5
    assert P["head"][1][-1] == th[-1]


def test_gradient_finite_differences():
    """Central differences of the loss against the analytic gradient, for a random sample of
    parameters of every layer and for input sites next to the walls and the x seam."""
    theta, x, t, widths = small_net()
    out, cache = U.forward(theta, x, widths)
    grad, gx = U.backward(theta, cache, out, t, widths)
    r = rng(6)
    h = 1e-6
    o = 0
    idx = []
    for name, ci, co in U.layers(widths):
        n = 9 * ci * co + co
        idx += list(o + r.choice(n, size=4, replace=False)) + [o + n - 1]
        o += n
    idx += list(range(o, theta.size))
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (U.loss(U.forward(tp, x, widths)[0], t) - U.loss(U.forward(tm, x, widths)[0], t)) / (2 * h)
        assert fd == pytest.approx(grad[i], rel=1e-5, abs=1e-9), i
    for (yy, xx, c) in [(0, 0, 0), (7, 11, 4), (0, 5, 2), (3, 0, 1), (7, 6, 3)]:
        xp = x.copy()
        xp[yy, xx, c] += h
        xm = x.copy()
        xm[yy, xx, c] -= h
        fd = (U.loss(U.forward(theta, xp, widths)[0], t) - U.loss(U.forward(theta, xm, widths)[0], t)) / (2 * h)
        assert fd == pytest.approx(gx[yy, xx, c], rel=1e-5, abs=1e-9)


def test_extra_output_gradient_finite_differences():
    """With g_extra = E the gradient is that of J = loss + sum(E * out): central differences of J
    for parameters of the first and last 3x3 layers and the head, and for input sites."""
    theta, x, t, widths = small_net(seed=8)
    E = rng(9).normal(size=t.shape)
    J = lambda th, xx: (lambda o: U.loss(o, t) + float(np.sum(E * o)))(U.forward(th, xx, widths)[0])  # noqa: E731
    out, cache = U.forward(theta, x, widths)
    grad, gx = U.backward(theta, cache, out, t, widths, g_extra=E)
    g0, gx0 = U.backward(theta, cache, out, t, widths)
    assert np.abs(grad - g0).max() > 1e-3  # the extra term is not negligible here
    h = 1e-6
    n_e1a = 9 * U.IN_CH * widths[0] + widths[0]
    lay = U.layers(widths)
    n_last = 9 * lay[-1][1] * lay[-1][2] + lay[-1][2]
    head0 = theta.size - (U.OUT_CH * widths[0] + U.OUT_CH)
    for i in [0, 17, n_e1a - 1, head0 - n_last, head0 - 1, head0, theta.size - 1]:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        assert (J(tp, x) - J(tm, x)) / (2 * h) == pytest.approx(grad[i], rel=1e-5, abs=1e-9), i
    for (yy, xx, c) in [(0, 3, 0), (7, 11, 4), (4, 0, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[yy, xx, c] += h
        xm[yy, xx, c] -= h
        assert (J(theta, xp) - J(theta, xm)) / (2 * h) == pytest.approx(gx[yy, xx, c], rel=1e-5, abs=1e-9)


def test_x_translation_equivariance():
    """The lattice is periodic in x; shifting the input by a multiple of 2^(L-1) columns (the
    pooling stride) shifts the output."""
    theta, x, t, widths = small_net(W=16)
    a = U.forward(theta, x, widths)[0]
    b = U.forward(theta, np.roll(x, 4, axis=1), widths)[0]
    assert np.allclose(np.roll(a, 4, axis=1), b, atol=1e-12)


def test_bf16_emulation_is_close():
    """q=True rounds at the device's storage points; the result stays within a few bf16 ulps of
    the FP64 network."""
    theta, x, t, widths = small_net()
    a = U.forward(theta, x, widths)[0]
    b = U.forward(theta, x, widths, q=True)[0]
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 3e-2
    ga = U.backward(theta, U.forward(theta, x, widths)[1], a, t, widths)[0]
    gb = U.backward(theta, U.forward(theta, x, widths, q=True)[1], b, t, widths, q=True)[0]
    assert np.linalg.norm(ga - gb) / np.linalg.norm(ga) < 5e-2


def test_adam_first_step():
    """After one step from zero moments, the bias-corrected update is lr g / (|g| + eps)."""
    r = rng(7)
    th = r.normal(size=50)
    g = r.normal(size=50)
    new, m, v = U.adam(th, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    assert np.allclose(th - new, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-10)


def test_he_uniform_bounds():
    th = S.he_uniform(3, [(5, 32), (32, 32)], head=(32, 3))
    assert th.size == 9 * 5 * 32 + 32 + 9 * 32 * 32 + 32 + 32 * 3 + 3
    w0 = th[:9 * 5 * 32]
    assert np.abs(w0).max() <= np.sqrt(6 / 45) and np.abs(w0).max() > 0.9 * np.sqrt(6 / 45)
    assert np.all(th[-(32 * 3 + 3):] == 0)


def test_gradient_finite_differences_other_channel_counts():
    """Six input and four output channels: the oracle's network takes its channel counts as
    parameters, and its gradient holds for counts other than the product's five and three."""
    widths = (4, 6)
    shapes = [(ci, co) for _, ci, co in U.layers(widths, in_ch=6)]
    r = rng(9)
    theta = S.he_uniform(8, shapes, head=(widths[0], 4))
    theta[-(4 * widths[0] + 4):] = r.normal(size=4 * widths[0] + 4)
    x = r.normal(size=(8, 8, 6))
    t = r.normal(size=(8, 8, 4))
    out, cache = U.forward(theta, x, widths, out_ch=4)
    assert out.shape == (8, 8, 4) and theta.size == U.param_count(widths, 6, 4)
    grad, gx = U.backward(theta, cache, out, t, widths)
    h = 1e-6
    for i in list(r.choice(theta.size, size=25, replace=False)) + [theta.size - 1]:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (U.loss(U.forward(tp, x, widths, out_ch=4)[0], t) -
              U.loss(U.forward(tm, x, widths, out_ch=4)[0], t)) / (2 * h)
        assert fd == pytest.approx(grad[i], rel=1e-5, abs=1e-9), i


def test_two_step_objective_finite_differences():
    """The two-step training gradient (tests/_two_step.py; what the training driver computes on
    the device) against central differences of L1 + L2, for parameters of the first and last
    layers and the head; the packing is an affine map with T entering two channels."""
    from tests._two_step import two_step
    theta, _, _, widths = small_net(seed=10)
    H, W = 8, 12
    r = rng(11)
    a = r.normal(size=(4, H, W))
    b = a + 0.3 * r.normal(size=a.shape)
    c = b + 0.3 * r.normal(size=a.shape)
    sc = (1.3, 0.7, 0.9, 1.1, 0.8)

    def pack(f):
        x = np.empty((H, W, 5))
        for k in range(4):
            x[..., k] = f[k] * sc[k]
        x[..., 4] = (f[3] - 1.0) * sc[4]
        return x

    def unpack(gx):
        g = np.stack([gx[..., k] * sc[k] for k in range(4)])
        g[3] += gx[..., 4] * sc[4]
        return g

    out_scale = (0.5, 0.2, 0.3)
    L1, L2, grad = two_step(theta, a, b, c, widths, pack, unpack, out_scale)
    h = 1e-6
    lay = U.layers(widths)
    n_last = 9 * lay[-1][1] * lay[-1][2] + lay[-1][2]
    head0 = theta.size - (U.OUT_CH * widths[0] + U.OUT_CH)
    for i in [3, 40, head0 - n_last + 5, head0 - 1, head0 + 2, theta.size - 2]:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (sum(two_step(tp, a, b, c, widths, pack, unpack, out_scale)[:2]) -
              sum(two_step(tm, a, b, c, widths, pack, unpack, out_scale)[:2])) / (2 * h)
        assert fd == pytest.approx(grad[i], rel=1e-5, abs=1e-9), i
