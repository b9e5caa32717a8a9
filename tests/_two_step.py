"""Reference of the two-step training objective of the surrogate (test helper), composed from the
oracle's forward and backward passes.

Step 1 maps fields a to the prediction x2 of the next snapshot b: x2 = a + s (y1 - mean y1) for
phi (and n: the shift keeps their sums), x2 = a + s y1 for the velocities, T of x2 is b's.  Step 2
predicts from x2 towards c.  L1 = loss(y1, (b - a) / s), L2 = loss(y2, (c - x2) / s); the
gradient of L1 + L2 with respect to the parameters follows x2's dependence on y1 through both the
input and the target of step 2."""
import numpy as np

from oracle import surrogate as U

PLANES = (0, 1, 2, 4)  # field plane of output channel 0, 1, 2, 3


def two_step(th, a, b, c, widths, pack, unpack_grad, out_scale, q=False):
    """a, b, c: fields [NF, H, W]; pack(f) -> packed input [H, W, C_in]; unpack_grad(gx) ->
    gradient with respect to the fields [NF, H, W].  Returns (L1, L2, gradient)."""
    nout = len(out_scale)
    s = np.asarray(out_scale, np.float64)
    pl = PLANES[:nout]
    y1, c1 = U.forward(th, pack(a), widths, q=q, out_ch=nout)
    t1 = np.stack([(b[p] - a[p]) / s[i] for i, p in enumerate(pl)], axis=2)
    x2 = a.copy()
    for i, p in enumerate(pl):
        inc = y1[..., i] - (y1[..., i].mean() if p in (0, 4) else 0.0)
        x2[p] = a[p] + s[i] * inc
    x2[3] = b[3]
    t2 = np.stack([(c[p] - x2[p]) / s[i] for i, p in enumerate(pl)], axis=2)
    y2, c2 = U.forward(th, pack(x2), widths, q=q, out_ch=nout)
    g2 = 2.0 * (y2 - t2) / y2.size
    gth2, gx2 = U.backward(th, c2, y2, t2, widths, q=q)
    fg2 = unpack_grad(gx2)
    og = np.stack([s[i] * fg2[p] + g2[..., i] for i, p in enumerate(pl)], axis=2)
    for i, p in enumerate(pl):
        if p in (0, 4):
            og[..., i] -= og[..., i].mean()
    gth1, _ = U.backward(th, c1, y1, t1, widths, q=q, g_extra=og)
    return U.loss(y1, t1), U.loss(y2, t2), gth1 + gth2
