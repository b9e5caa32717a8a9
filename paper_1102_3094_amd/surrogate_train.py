"""Training and evaluation driver of the learned surrogate.  It only sequences calls of the two
C-ABIs (solver runs and snapshots through lam.h; loss, gradients, Adam and rollouts through
lam_surrogate.h); torch holds the snapshot tensors on the device and does the elementwise glue of
the two-step gradient.

Workflow:
  1. snapshots(): plain solver runs; fields (phi, u_x, u_y, T)
     every `every` steps from t_start.
  2. normalisation(): input shifts/scales and output scales from the snapshot statistics.
  3. train(): Adam on random consecutive snapshot pairs (target = normalised increment), or on
     snapshot triples through two surrogate steps (two_step_backward).
  4. evaluate(): the same start state advanced by the plain solver and by the surrogate-
     accelerated rollout (and by the rollout with a zero network, i.e. the method without the
     learned part); S(k) peak position and height, its first moment <k>, phi error and
     wall-clock times.
"""
from __future__ import annotations

import math
import time

import numpy as np

import synthetic as S
from . import Ensemble, Sim
from .surrogate import Surrogate


def snapshots(members, phis, t_start, count, every=100, device="cuda:0"):
    """[M, count + 1, 4, H, W] FP32 device tensor of the fields (phi, u_x, u_y, T) at
    t_start + k * every."""
    import torch
    H, W = members[0]["ny"], members[0]["nx"]
    out = torch.empty((len(members), count + 1, 4, H, W), dtype=torch.float32, device=device)
    for m, (p, phi) in enumerate(zip(members, phis)):
        sim = Sim(p, device=device).init_fields(torch.tensor(phi, dtype=torch.float32))
        sim.step(t_start)
        for k in range(count + 1):
            if k:
                sim.step(every)
            sim.fields_into(out[m, k])
        sim.stream.synchronize()
        if sim.observables()["nonfinite"]:
            raise RuntimeError(f"training run {m} became non-finite")
    return out


def normalisation(snaps, Tc, u_ref=0.01, a_ref=0.25):
    """phi scaled to unit spread, velocities by a reference speed u_ref (a Mach-number scale:
    the spread of u is dominated by the few active runs), T - Tc and a by a reference reduced
    temperature a_ref (T may be uniform in every run); outputs scaled by the standard deviation
    of each increment over the pairs."""
    x = snaps[:, :-1]
    sd = lambda t: max(float(t.double().std()), 1e-12)  # noqa: E731
    in_scale = (1.0 / sd(x[:, :, 0]), 1.0 / u_ref, 1.0 / u_ref, 1.0 / (a_ref * Tc), 1.0 / a_ref)
    in_shift = (0.0, 0.0, 0.0, Tc, 0.0)
    out_scale = tuple(sd(snaps[:, 1:, c] - snaps[:, :-1, c]) for c in (0, 1, 2))
    return dict(Tc=Tc, in_shift=in_shift, in_scale=in_scale, out_scale=out_scale)


def mirror(f):
    """The lattice mirrored across its mid-plane between the walls: y -> H - 1 - y, u_y -> -u_y
    (a symmetry of the method with walls of equal temperature)."""
    g = f.flip(-2)
    g[2] = -g[2]
    return g


def two_step_backward(net: Surrogate, a, b, c, field_grad, want_loss=False):
    """Gradients of L1 + L2 added to the gradient buffer, where L1 is the one-step loss from
    snapshot a to b and L2 the loss of the second surrogate step, taken from the network's own
    prediction x2 of b (T of x2 is b's: T advances exactly between surrogate calls) towards c.
    The gradient of L2 flows back into the first step: through the input of the second pass
    (lsn_loss_backward_ex's field gradient) and through its target (c - x2) / s, then through
    x2 = a + s (y1 - conservation shift) to the first output.  field_grad: [NF, H, W] scratch.
    Returns (L1, L2) when want_loss."""
    x2 = net.advance(a.clone())
    x2[3] = b[3]
    t2 = net.make_target(x2, c)
    y2 = net.forward(x2)
    g2 = (2.0 / y2.numel()) * (y2 - t2)          # d L2 / d y2
    l2 = net.loss_backward(x2, t2, want_loss=want_loss, field_grad=field_grad)
    og = g2.clone()                               # s d L2 / d x2 = s (J^T g2 + g2 / s)
    for ch, plane in enumerate((0, 1, 2, 4)[:net.NOUT]):
        og[ch] += float(net.cfg.out_scale[ch]) * field_grad[plane]
    og[0] -= og[0].mean()                         # adjoint of the shift that keeps sum phi
    if net.NOUT > 3:
        og[3] -= og[3].mean()
    l1 = net.loss_backward(a, net.make_target(a, b), want_loss=want_loss, out_grad=og)
    return (l1, l2) if want_loss else None


def train(net: Surrogate, snaps, steps, batch=4, lr=1e-3, seed=1, log=None, augment=True,
          noise=0.0, pushforward=0.0, unroll=False):
    """Adam with a cosine learning-rate schedule; pairs drawn by SplitMix64 from `seed`; with
    `augment`, every other draw uses the mirrored pair.  With noise > 0 the input phi is
    perturbed by uniform noise of that amplitude (relative to the spread of phi in the pair) and
    the target is the step from the perturbed state to the true later state, so that the network
    learns to pull a drifted state back (the error it meets in a rollout).  With pushforward > 0
    that fraction of the draws starts from the network's own one-step prediction of a snapshot
    and targets the true state one step later (pushforward training, Brandstetter, Worrall &
    Welling, 2022: the rollout's own error distribution, without a gradient through the first
    step).  With `unroll` every draw is a snapshot triple trained through two surrogate steps
    (two_step_backward: the gradient of the second step's error reaches the first)."""
    import torch
    M, K = snaps.shape[0], snaps.shape[1] - 1
    if unroll and K < 2:
        raise ValueError("two-step training needs at least three snapshots per run")
    fg = torch.empty(snaps.shape[2:], dtype=torch.float32, device=snaps.device) if unroll else None
    draws = S.uniform01(seed, steps * batch)
    flips = S.uniform01(seed + 7919, steps * batch)
    pushes = S.uniform01(seed + 104729, steps * batch)
    losses = []
    for it in range(steps):
        net.zero_grad()
        tot = 0.0
        for b in range(batch):
            want = b == batch - 1 and (log is not None or it == steps - 1)
            if unroll:
                j = int(draws[it * batch + b] * M * (K - 1))
                m, k = j // (K - 1), j % (K - 1)
                trip = [snaps[m, k + i] for i in range(3)]
                if augment and flips[it * batch + b] < 0.5:
                    trip = [mirror(t) for t in trip]
                r = two_step_backward(net, *trip, fg, want_loss=want)
                tot = sum(r) if r is not None else tot
                continue
            push = pushforward > 0.0 and K > 1 and pushes[it * batch + b] < pushforward
            KK = K - 1 if push else K
            j = int(draws[it * batch + b] * M * KK)
            m, k = j // KK, j % KK
            a, c = snaps[m, k], snaps[m, k + (2 if push else 1)]
            if augment and flips[it * batch + b] < 0.5:
                a, c = mirror(a), mirror(c)
            if push:
                a = net.advance(a.clone())
            if noise > 0.0:
                a = a.clone()
                gen = torch.Generator(device=a.device).manual_seed(int(seed) * 1000003 + it * batch + b)
                r = torch.rand(a.shape[1:], generator=gen, device=a.device)
                a[0] += (noise * float(a[0].std())) * (2.0 * r - 1.0)
            tgt = net.make_target(a, c)
            r = net.loss_backward(a, tgt, want_loss=want)
            tot = r if r is not None else tot
        rate = lr * 0.5 * (1.0 + math.cos(math.pi * it / steps))
        net.adam(lr=rate, grad_scale=1.0 / batch)
        if want:
            losses.append(tot)
            if log is not None and (it % log == 0 or it == steps - 1):
                print(f"  train step {it}: loss {tot:.4e}", flush=True)
    return losses


def validation_loss(net: Surrogate, snaps, pairs=32, seed=2):
    """Mean loss over `pairs` consecutive snapshot pairs drawn from `seed` (no update: the
    gradient buffer is cleared before and after)."""
    M, K = snaps.shape[0], snaps.shape[1] - 1
    draws = S.uniform01(seed, pairs)
    tot = 0.0
    for d in draws:
        j = int(d * M * K)
        m, k = j // K, j % K
        net.zero_grad()
        tot += net.loss_backward(snaps[m, k], net.make_target(snaps[m, k], snaps[m, k + 1]))
    net.zero_grad()
    return tot / pairs


def evaluate(net: Surrogate, params, phi0, t0, cycles, calls=10, steps_per_call=100,
             anchor_steps=100, zero_net: Surrogate | None = None, device="cuda:0", limiter=1.05):
    """Plain solver against the surrogate-accelerated rollout from the same state at step t0
    (`limiter`: the rollout's order-parameter limiter factor, 0 for none)."""
    import torch
    total = cycles * (calls * steps_per_call + anchor_steps)
    start = Sim(params, device=device).init_fields(torch.tensor(phi0, dtype=torch.float32)).step(t0)
    state = start.get_state()
    res = dict(t0=t0, steps=total, cycles=cycles, calls=calls, steps_per_call=steps_per_call,
               anchor_steps=anchor_steps)

    def fresh():
        return Sim(params, device=device, stream=net.stream).set_state(state)

    # plain method: per-step launches, and the same run replayed from a HIP graph (one-member
    # ensemble); the faster of the two is the reference
    plain = fresh()
    plain.step(10)
    plain = fresh()
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain.step(total)
    plain.stream.synchronize()
    res["plain_s"] = time.perf_counter() - t
    ens = Ensemble([dict(params, pop_storage=0, tile_hint=32)], device=device)
    ens.sims[0].set_state(state)
    ens.step(2)                    # captures the graph of a step pair
    ens.sims[0].set_state(state)
    ens.synchronize()
    t = time.perf_counter()
    ens.step(total)
    ens.synchronize()
    res["plain_graph_s"] = time.perf_counter() - t
    res["plain_best_s"] = min(res["plain_s"], res["plain_graph_s"])
    sk = plain.structure_factor(params["nx"] // 2)
    res["plain_k_peak"], res["plain_S_peak"], res["plain_k_mean"] = sk["k_peak"], sk["S_peak"], sk["k_mean"]
    res["plain_S"] = sk["S"]
    phi_ref = plain.fields()["phi"].double()

    scratch = torch.empty((net.NF, params["ny"], params["nx"]), dtype=torch.float32, device=device)
    for name, n in (("surrogate", net), ("no_network", zero_net)):
        if n is None:
            continue
        n.set_limiter(limiter)
        s = fresh()
        n.rollout(s, scratch, 1, calls, steps_per_call, 0)   # warm-up of the launch path
        s = fresh()
        torch.cuda.synchronize()
        t = time.perf_counter()
        n.rollout(s, scratch, cycles, calls, steps_per_call, anchor_steps)
        s.stream.synchronize()
        res[f"{name}_s"] = time.perf_counter() - t
        finite = not s.observables()["nonfinite"]
        res[f"{name}_finite"] = finite
        if finite:
            sk = s.structure_factor(params["nx"] // 2)
            kp, sp = sk["k_peak"], sk["S_peak"]
            phi = s.fields()["phi"].double()
            res[f"{name}_k_peak"], res[f"{name}_S_peak"] = kp, sp
            res[f"{name}_S"] = sk["S"]
            res[f"{name}_k_mean_err"] = abs(sk["k_mean"] - res["plain_k_mean"]) / res["plain_k_mean"]
            res[f"{name}_k_peak_err"] = abs(kp - res["plain_k_peak"]) / res["plain_k_peak"]
            res[f"{name}_S_peak_err"] = abs(sp - res["plain_S_peak"]) / res["plain_S_peak"]
            res[f"{name}_phi_rel_l2"] = float((phi - phi_ref).norm() / phi_ref.norm())
        else:  # a run that blew up counts as a 100 % error
            res[f"{name}_k_peak"] = res[f"{name}_S_peak"] = res[f"{name}_S"] = None
            res[f"{name}_k_peak_err"] = res[f"{name}_S_peak_err"] = res[f"{name}_k_mean_err"] = 1.0
            res[f"{name}_phi_rel_l2"] = None
        res[f"{name}_speedup"] = res["plain_best_s"] / res[f"{name}_s"]
    return res
