"""Throughput benchmark of the fused hybrid LB/FD step on one MI355X.

Workload: the 1024 x 1024 D2Q9 lattice with cold walls at y = 0 and y = 1023, tau = 0.6,
xi = 0.01, free-energy coefficients b = 0.1, kappa = -0.006, c = 0.0375, Tc = 1, T0 = 1.5,
Tw = 0.7, Gamma = 0.1, phi0 uniform in [-0.05, 0.05] from seed 1 (synthetic, resident in device
memory before timing).  One benchmark step is one full time step of the method (force, stream,
collide, order-parameter sub-steps, temperature); the structure factor and the orientation
histogram are taken every 1000 steps inside the timed region.

Prints one JSON line: MLUPS (million lattice-site updates per second), the roofline of the
dominant kernel (fused force/stream/collide kernel; algorithmic bytes per site: populations read
and written, 2 x 9 x 4 B, plus phi read, 4 B = 76 B in 2D; 2 x 19 x 4 + 4 = 156 B in 3D), and the
FP64 CPU oracle's MLUPS on a bounded sample of the same workload (built with gcc -O3
-march=native on the host at run time; CPU model recorded).  The 1024^2 working set (about
100 MB) stays in the 256 MB Infinity Cache, so its bandwidth is a past-L2 figure; the line
therefore also carries "hbm_legs": the 4096^2 D2Q9 and 256^3 D3Q19 workloads (1.4 and 3.3 GB),
each with its MLUPS, dominant-kernel and whole-step roofline fractions and its own CPU
baseline.  --workload selects another named workload for the headline measurement.

The same line carries the learned-surrogate leg ("surrogate"): a U-Net (BF16 matrix-core kernels)
trained on the GPU on snapshots of plain 512^2 runs (one-step rounds, then two-step training),
then a surrogate-accelerated run (10 calls of 100 lattice steps each, then re-anchoring and
--surrogate-anchor-steps plain steps, 10 cycles) against the plain solver from the same state:
wall-clock speed-up, error of the S(k) peak position and height and of its first moment, and the
same for the run without the network (the method with the learned steps replaced by no change).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "c2_1024sq_tau0.6"
# working sets far above the 256 MB Infinity Cache: the HBM figures (steps timed per leg; the
# legs' 0.7 Tc coefficients leave the stable range after about 260 steps, so warm-up, the timed
# pass and the event-timed pass together stay below that and the fields are finite throughout)
HBM_LEGS = (("m1_4096sq", 100), ("c3_256cube_xi0.1", 60))
HBM_PEAK_GBS = 8000.0
OBS_EVERY = 1000


def byte_model(dim, pop_bytes=4):
    """Algorithmic bytes per site: (dominant kernel, whole step).  Dominant kernel: populations
    read and written plus phi read; whole step: populations and phi read and written."""
    q = 9 if dim == 2 else 19
    return 2 * pop_bytes * q + 4, 2 * (pop_bytes * q + 4)


def kernel_source_hash(dim):
    h = hashlib.sha256()
    name = "lam_2d.hip" if dim == 2 else "lam_3d.hip"
    with open(os.path.join(ROOT, "paper_1102_3094_amd", "csrc", name), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def copy_ceiling_gbps(nbytes, reps=20):
    """Bandwidth of a plain device-to-device copy of `nbytes` (read + write counted), timed with
    events on the current stream: the practical ceiling for streaming the population planes on
    this device, next to the nominal HBM peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def traffic_from_profiles(workload, dim):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary,
    or None when it is missing or was taken from another version of the kernel source."""
    kern = "lb2d" if dim == 2 else "lb3d"
    path = os.path.join(ROOT, "profiles", f"{kern}_{workload}_traffic.json")
    # only the FP32-storage kernel has committed counter summaries
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash(dim):
        return None
    return d.get("hbm_bytes_per_launch")


def host_cpu():
    """(CPU model name, threads this process may run on)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


_ORACLE_BUILD = []


def native_oracle():
    """Build the oracle with gcc -O3 -march=native for this host (once per process, into a
    temporary directory) and load it for the CPU baseline; falls back to the -O2 build."""
    if not _ORACLE_BUILD:
        import subprocess
        import tempfile
        import oracle
        from oracle.build import build_native
        try:
            d = tempfile.mkdtemp(prefix="lam_oracle_")
            oracle.use_library(build_native(os.path.join(d, "liblam_oracle_native.so")))
            _ORACLE_BUILD.append("gcc -O3 -march=native -fopenmp")
        except (OSError, subprocess.CalledProcessError, RuntimeError):
            _ORACLE_BUILD.append("gcc -O2 -fopenmp (native build failed)")
    return _ORACLE_BUILD[0]


def cpu_baseline(params, phi0, budget_s=12.0, single_s=4.0):
    """The FP64 oracle on the host: all OpenMP threads for about budget_s, then (unless single_s
    is None) one thread for about single_s; at least one step each, after one untimed step."""
    build = native_oracle()
    import oracle
    n = params["nx"] * params["ny"] * (params["nz"] if params["dim"] == 3 else 1)

    def rate(budget):
        o = oracle.Oracle(params).init_fields(phi0)
        o.step(1)  # first-touch of the arrays outside the timing
        t0 = time.perf_counter()
        steps = 0
        while (time.perf_counter() - t0 < budget or steps == 0) and steps < 2000:
            o.step(1)
            steps += 1
        dt = time.perf_counter() - t0
        del o
        return n * steps / dt / 1e6, steps, dt

    cores = oracle.threads()
    v, steps, dt = rate(budget_s)
    shape = "x".join(str(params[k]) for k in (("nx", "ny") if params["dim"] == 2 else ("nx", "ny", "nz")))
    sample = f"{steps} steps of the {shape} workload ({dt:.1f} s, FP64, OpenMP over sites)"
    out = {"value": v, "unit": "MLUPS", "cores": cores, "kind": "oracle", "sample": sample,
           "build": build}
    if single_s is not None:
        oracle.threads(1)
        v1, steps1, dt1 = rate(single_s)
        oracle.threads(cores)
        out["sample"] += f"; one thread: {steps1} steps in {dt1:.1f} s"
        out["single_thread_value"] = v1
    model, avail = host_cpu()
    out["cpu_model"] = model
    out["host_threads_available"] = avail
    return out


def bench_ensemble(args):
    """64 independent lattices (sides 128-512, xi and tau swept) in one persistent launch per
    kernel (work queues over the members' tiles), autotuned tile height and grid size, step pairs
    replayed from a HIP graph."""
    import torch
    import paper_1102_3094_amd as lam
    import synthetic as S
    members, phis = S.ensemble_members(seed=1, count=64, pop_storage=1)
    ens = lam.Ensemble(members)
    tile = ens.tune(40)
    ens.init_fields(phis)
    ens.step(args.warmup)
    ens.synchronize()
    t0 = time.perf_counter()
    ens.step(args.steps)
    ens.synchronize()
    dt = time.perf_counter() - t0
    sites = ens.sites
    mlups = sites * args.steps / dt / 1e6
    _, step_bytes = byte_model(2, 2)
    out = {"metric": "MLUPS (ensemble, all members)", "value": round(mlups, 1), "unit": "MLUPS",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 (populations stored f16)", "data": "synthetic",
           "config": {"workload": "64 D2Q9 lattices, sides log-uniform 128-512, xi log-uniform "
                                  "1e-3..1, tau uniform 0.55..3.0, cold walls, seed 1",
                      "sites": sites, "tile_height": tile,
                      "persistent_workgroups": ens.workgroups},
           "step_effective_roofline_frac": round(mlups * 1e6 * step_bytes / 8e12, 4)}
    print(json.dumps(out), flush=True)


def unet_shapes(in_ch, levels=4, base=32):
    """(C_in, C_out) of the 3x3 layers in parameter order."""
    widths = [base << l for l in range(levels)]
    shapes = [(in_ch, base), (base, base)]
    for l in range(1, levels):
        shapes += [(widths[l - 1], widths[l]), (widths[l], widths[l])]
    for l in range(levels - 2, -1, -1):
        shapes += [(widths[l + 1] + widths[l], widths[l]), (widths[l], widths[l])]
    return shapes


def bench_surrogate(members=16, train_steps=6000, anchor_steps=50, side=512, noise=0.0,
                    held_out=(99, 98, 97), unroll_steps=1000, curves=None):
    """Train the surrogate on plain runs and compare the accelerated run with the plain solver.
    `unroll_steps` Adam steps of two-step training follow the one-step rounds; `curves` (a path)
    receives the S(k) curves of the held-out runs as JSON."""
    import numpy as np
    import torch
    import synthetic as S
    from paper_1102_3094_amd import surrogate_train as ST
    from paper_1102_3094_amd.surrogate import Surrogate
    t_start, nsnap, every = 8000, 200, 100
    mem, phis = S.surrogate_members(seed=7, count=members + 1, side=side, instant=members + 1)
    t = time.perf_counter()
    snaps = ST.snapshots(mem, phis, t_start, nsnap, every)
    val, train = snaps[members:], snaps[:members]
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    print(f"surrogate: {members + 1} runs of {side}^2 snapshotted in {gen_s:.1f} s", file=sys.stderr,
          flush=True)
    norm = ST.normalisation(train, mem[0]["Tc"])
    shapes = unet_shapes(5)
    th = torch.tensor(S.he_uniform(5, shapes, head=(32, 3)), dtype=torch.float32, device="cuda:0")
    net = Surrogate(side, side, training=True, **norm).set_params(th)
    val0 = ST.validation_loss(net, val)
    stream = torch.cuda.Stream()  # a capturable stream: the rollout replays its step graph
    t = time.perf_counter()
    for rnd in range(4):
        ST.train(net, train, train_steps // 4, batch=4, lr=5e-4 * 0.5 ** rnd, seed=10 + rnd,
                 noise=noise)
        torch.cuda.synchronize()
        print(f"surrogate: training round {rnd + 1}/4 done ({time.perf_counter() - t:.1f} s)",
              file=sys.stderr, flush=True)
    if unroll_steps:
        ST.train(net, train, unroll_steps, batch=4, lr=1.25e-4, seed=20, unroll=True)
        torch.cuda.synchronize()
        print(f"surrogate: two-step training done ({time.perf_counter() - t:.1f} s)", file=sys.stderr,
              flush=True)
    train_s = time.perf_counter() - t
    val1 = ST.validation_loss(net, val)
    inf = Surrogate(side, side, stream=stream, **norm).set_params(net.params())
    inf.tune(train[0, 0], reps=5)
    zero = Surrogate(side, side, stream=stream, **norm).set_params(torch.zeros_like(th))
    f = train[0, 0].clone()
    inf.set_timing(True)
    ts = []
    for _ in range(20):
        inf.forward(f)
        ts.append(inf.forward_time_ms())
    inf.set_timing(False)
    fwd_ms = float(np.median(ts))
    flop = 0
    for lev, (ci, co) in zip([0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0], shapes):
        flop += 2 * 9 * ci * co * (side >> lev) ** 2
    p = dict(mem[0], tau=1.5)
    runs = [ST.evaluate(inf, p, S.phi0((side, side), seed=sd), t0=15000, cycles=10, calls=10,
                        steps_per_call=every, anchor_steps=anchor_steps, zero_net=zero)
            for sd in held_out]
    # wall-clock times summed over the held-out runs, errors averaged
    def mean(k):
        v = [q[k] for q in runs if q[k] is not None]
        return float(np.mean(v)) if v else None
    r = {k: mean(k) for k in runs[0] if isinstance(runs[0][k], (float, type(None)))}
    r.update({k: runs[0][k] for k in ("steps", "calls", "steps_per_call", "anchor_steps")})
    r["surrogate_finite"] = all(q["surrogate_finite"] for q in runs)
    r["surrogate_speedup"] = sum(q["plain_best_s"] for q in runs) / sum(q["surrogate_s"] for q in runs)
    def per(rs):
        return [{"seed": sd, "finite": bool(q["surrogate_finite"]),
                 "S_peak_position_err": round(q["surrogate_k_peak_err"], 4),
                 "S_peak_height_err": round(q["surrogate_S_peak_err"], 4),
                 "S_mean_k_err": round(q["surrogate_k_mean_err"], 4),
                 "no_network_S_peak_position_err": round(q["no_network_k_peak_err"], 4),
                 "no_network_S_peak_height_err": round(q["no_network_S_peak_err"], 4)}
                for sd, q in zip(held_out, rs)]
    per_run = per(runs)
    if curves:
        with open(curves, "w") as fh:
            json.dump([{"seed": sd, **{k: q[k] for k in ("plain_S", "surrogate_S", "no_network_S")}}
                       for sd, q in zip(held_out, runs)], fh)
    # the same runs re-anchored every 5 calls (25 plain steps), same simulated time
    runs5 = [ST.evaluate(inf, p, S.phi0((side, side), seed=sd), t0=15000, cycles=20, calls=5,
                         steps_per_call=every, anchor_steps=anchor_steps // 2)
             for sd in held_out]
    every5 = {"speedup_vs_plain": round(sum(q["plain_best_s"] for q in runs5) /
                                        sum(q["surrogate_s"] for q in runs5), 3),
              "S_peak_position_err": round(float(np.mean([q["surrogate_k_peak_err"] for q in runs5])), 4),
              "S_peak_height_err": round(float(np.mean([q["surrogate_S_peak_err"] for q in runs5])), 4),
              "finite_runs": sum(bool(q["surrogate_finite"]) for q in runs5),
              "per_run": [{"seed": sd, "finite": bool(q["surrogate_finite"]),
                           "S_peak_position_err": round(q["surrogate_k_peak_err"], 4),
                           "S_peak_height_err": round(q["surrogate_S_peak_err"], 4)}
                          for sd, q in zip(held_out, runs5)]}
    # the 10-call cadence without the order-parameter limiter
    runs0 = [ST.evaluate(inf, p, S.phi0((side, side), seed=sd), t0=15000, cycles=10, calls=10,
                         steps_per_call=every, anchor_steps=anchor_steps, limiter=0.0)
             for sd in held_out]
    no_lim = {"S_peak_position_err": round(float(np.mean([q["surrogate_k_peak_err"] for q in runs0])), 4),
              "S_peak_height_err": round(float(np.mean([q["surrogate_S_peak_err"] for q in runs0])), 4),
              "finite_runs": sum(bool(q["surrogate_finite"]) for q in runs0),
              "per_run": [{"seed": sd, "finite": bool(q["surrogate_finite"]),
                           "S_peak_position_err": round(q["surrogate_k_peak_err"], 4),
                           "S_peak_height_err": round(q["surrogate_S_peak_err"], 4)}
                          for sd, q in zip(held_out, runs0)]}
    tflops = flop / (fwd_ms * 1e-3) / 1e12
    return {
        "workload": f"D2Q9 {side}^2, walls at 0.95 Tc, instantaneous quench, tau in [1.25, 2]; "
                    f"{members} training runs + 1 validation run (seed 7), held-out runs seeds "
                    f"{', '.join(str(x) for x in held_out)}, tau 1.5, from step 15000 (errors are "
                    f"means over the held-out runs)",
        "speedup_vs_plain": round(r["surrogate_speedup"], 3),
        "plain_s": round(r["plain_best_s"], 5), "surrogate_s": round(r["surrogate_s"], 5),
        "lattice_steps": r["steps"], "calls_per_cycle": r["calls"],
        "steps_per_call": r["steps_per_call"], "anchor_steps": r["anchor_steps"],
        "S_peak_position_err": round(r["surrogate_k_peak_err"], 4),
        "S_peak_height_err": round(r["surrogate_S_peak_err"], 4),
        "S_mean_k_err": round(r["surrogate_k_mean_err"], 4),
        "phi_rel_l2_finite_runs": None if r["surrogate_phi_rel_l2"] is None else round(r["surrogate_phi_rel_l2"], 4),
        "no_network_S_peak_position_err": round(r["no_network_k_peak_err"], 4),
        "no_network_S_peak_height_err": round(r["no_network_S_peak_err"], 4),
        "no_network_phi_rel_l2": None if r["no_network_phi_rel_l2"] is None else round(r["no_network_phi_rel_l2"], 4),
        "finite": bool(r["surrogate_finite"]),
        "finite_runs": sum(bool(q["surrogate_finite"]) for q in runs), "held_out_runs": len(runs),
        "per_run": per_run, "input_noise": noise,
        "reanchor_every_5_calls": every5,
        "limiter_factor": 1.05, "without_limiter": no_lim,
        "validation_loss_untrained": round(val0, 4), "validation_loss_trained": round(val1, 4),
        "snapshot_s": round(gen_s, 2), "train_s": round(train_s, 2), "train_steps": train_steps,
        "two_step_train_steps": unroll_steps,
        "forward_ms": round(fwd_ms, 4),
        "roofline": {"bound": "mfma", "achieved": round(tflops, 1), "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(tflops / 2500.0, 4),
                     "kernel": "U-Net forward (14 conv3x3 implicit GEMMs, bf16)",
                     "flop_per_call": flop},
    }


def surrogate_profile_pass(side=512, calls=50):
    """For rocprofv3: the tuned 512^2 surrogate forward pass `calls` times (He-initialised
    weights, fields of a plain run at step 2000)."""
    import torch
    import synthetic as S
    import paper_1102_3094_amd as lam
    from paper_1102_3094_amd.surrogate import Surrogate
    from paper_1102_3094_amd import surrogate_train as ST
    mem, phis = S.surrogate_members(seed=7, count=1, side=side, instant=1)
    snaps = ST.snapshots(mem, phis, 2000, 1, 100)
    th = torch.tensor(S.he_uniform(5, unet_shapes(5), head=(32, 3)), dtype=torch.float32,
                      device="cuda:0")
    net = Surrogate(side, side, **ST.normalisation(snaps, 1.0)).set_params(th)
    codes = net.tune(snaps[0, 0])
    out = torch.empty((3, side, side), dtype=torch.float32, device="cuda:0")
    for _ in range(calls):
        net.forward(snaps[0, 0], out)
    torch.cuda.synchronize()
    print(json.dumps({"surrogate_profile_pass": True, "calls": calls, "shapes": codes}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pop-storage", type=int, default=0, choices=(0, 1),
                    help="population storage: 0 FP32 deviations, 1 FP16 deviations")
    ap.add_argument("--ensemble", action="store_true",
                    help="the batched ensemble instead: 64 uneven 2D lattices, FP16 populations")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="named workload of synthetic.WORKLOADS (default: the 1024^2 lattice)")
    ap.add_argument("--no-hbm-legs", action="store_true",
                    help="skip the 4096^2 and 256^3 legs (working sets above the last-level cache)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned-surrogate leg (training on the GPU, about a minute)")
    ap.add_argument("--surrogate-train-steps", type=int, default=6000)
    ap.add_argument("--surrogate-two-step", type=int, default=1000,
                    help="Adam steps of two-step (unrolled) training after the one-step rounds")
    ap.add_argument("--surrogate-anchor-steps", type=int, default=50,
                    help="plain steps after every 10 surrogate calls (re-anchoring)")
    ap.add_argument("--surrogate-curves", default=None,
                    help="file for the S(k) curves of the held-out surrogate runs (JSON)")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="only the learned-surrogate leg, printed as its own JSON line")
    ap.add_argument("--surrogate-profile-pass", action="store_true",
                    help="for rocprofv3: 50 tuned forward passes of the 512^2 surrogate")
    ap.add_argument("--profile-pass", action="store_true",
                    help="for rocprofv3 counter runs: a few steps of the workload, then one plain "
                         "device copy of 512 MiB whose counters calibrate the byte counts")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the method is built and "
              "measured on a single MI355X; multi-GPU slab decomposition is not part of it.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1102_3094_amd as lam
    import synthetic as S

    lam.load()
    if args.surrogate_profile_pass:
        return surrogate_profile_pass()
    if args.ensemble:
        return bench_ensemble(args)
    if args.surrogate_only:
        print(json.dumps({"surrogate": bench_surrogate(train_steps=args.surrogate_train_steps,
                                                       unroll_steps=args.surrogate_two_step,
                                                       curves=args.surrogate_curves,
                                                       anchor_steps=args.surrogate_anchor_steps)}),
              flush=True)
        return
    wl = args.workload
    if args.profile_pass:
        return profile_pass(lam, S, wl, args)
    head = measure(lam, S, wl, args.steps, args.warmup, args.pop_storage, OBS_EVERY)
    out = {
        "metric": "MLUPS + % HBM roofline; surrogate vs plain wall-time at equal S(k) peak error",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if not args.pop_storage else "f32 (populations stored f16)",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "step_effective_roofline_frac": head["step_effective_roofline_frac"],
        "kernel_avg_us": head["kernel_avg_us"],
        "state_finite_at_end": head["state_finite_at_end"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(head["params"], head["phi0"])
    del head
    torch.cuda.empty_cache()
    if not args.no_hbm_legs and wl == WORKLOAD:
        legs = []
        for name, steps in HBM_LEGS:
            leg = measure(lam, S, name, steps, 10, args.pop_storage, None)
            rec = {k: leg[k] for k in ("config", "roofline", "step_effective_roofline_frac",
                                        "kernel_avg_us", "state_finite_at_end", "ms_per_step")}
            rec["value"] = leg["mlups"]
            rec["unit"] = "MLUPS"
            rec["steps"] = steps
            if not args.no_cpu_baseline:
                rec["cpu_baseline"] = cpu_baseline(leg["params"], leg["phi0"], budget_s=6.0,
                                                   single_s=3.0 if leg["params"]["dim"] == 2 else None)
            legs.append(rec)
            del leg
            torch.cuda.empty_cache()
        out["hbm_legs"] = legs
    if not args.no_surrogate and wl == WORKLOAD:
        out["surrogate"] = bench_surrogate(train_steps=args.surrogate_train_steps,
                                           unroll_steps=args.surrogate_two_step,
                                           curves=args.surrogate_curves,
                                           anchor_steps=args.surrogate_anchor_steps)
    print(json.dumps(out), flush=True)


def profile_pass(lam, S, wl, args):
    """For rocprofv3 counter runs: warmup + steps steps of the workload, then one plain device
    copy of 512 MiB whose counters calibrate the byte counts."""
    import torch
    p = S.model_params(wl, pop_storage=args.pop_storage)
    sim = lam.Sim(p, device="cuda:0").init_fields(torch.tensor(S.initial_phi(wl), dtype=torch.float32))
    sim.step(args.warmup)
    sim.step(args.steps)
    src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_pass": True, "workload": wl, "steps": args.steps,
                      "copy_bytes": src.numel() * 4}))


def measure(lam, S, wl, steps, warmup, pop_storage, obs_every):
    """Time `steps` steps of workload `wl` (after `warmup`), then the same number again with HIP
    events on every kernel launch for the per-kernel durations.  With obs_every, the structure
    factor and the orientation histogram are taken every obs_every steps (2D) inside the timed
    region."""
    import torch
    p = S.model_params(wl, pop_storage=pop_storage)
    phi0 = S.initial_phi(wl)
    dim = p["dim"]
    n_sites = p["nx"] * p["ny"] * (p["nz"] if dim == 3 else 1)
    lb_bytes, step_bytes = byte_model(dim, 2 if pop_storage else 4)
    # a stream of its own: lam_step then replays captured pairs of steps from a HIP graph
    sim = lam.Sim(p, device="cuda:0", stream=torch.cuda.Stream(device="cuda:0"))
    sim.init_fields(torch.tensor(phi0, dtype=torch.float32))
    n_phi, n_T = sim.substeps
    sim_step = [0]

    def run(k):
        done = 0
        while done < k:
            chunk = k - done
            if obs_every:
                chunk = min(obs_every - (sim_step[0] % obs_every), chunk)
            sim.step(chunk)
            done += chunk
            sim_step[0] += chunk
            if obs_every and sim_step[0] % obs_every == 0 and dim == 2:
                sim.structure_factor(min(p["nx"], p["ny"]) // 2)
                sim.orientation(18)

    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mlups = n_sites * steps / dt / 1e6
    # second pass of the same length; every kernel launch carries HIP events (kernel timestamps)
    # on the library's stream
    sim.set_timing(True)
    run(steps)
    kt = sim.kernel_times()
    sim.set_timing(False)
    lb_ms, lb_n = kt["lb"]
    phi_ms, phi_n = kt["phi"]
    lb_avg_s = lb_ms / max(lb_n, 1) / 1e3
    achieved = lb_bytes * n_sites / lb_avg_s / 1e9
    q = 9 if dim == 2 else 19
    copy_gbps = copy_ceiling_gbps(q * n_sites * (2 if pop_storage else 4))
    ob = sim.observables()
    kname = "lb2d" if dim == 2 else "lb3d"
    shape = "x".join(str(p[k]) for k in (("nx", "ny") if dim == 2 else ("nx", "ny", "nz")))
    lattice = "D2Q9" if dim == 2 else "D3Q19"
    extras = f", S(k)+orientation every {obs_every} steps" if (obs_every and dim == 2) else ""
    ws = (2 * q * (2 if pop_storage else 4) + 4 * 4 + 4 * dim) * n_sites
    resident = ws < 256e6
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles(wl, dim),
            "kernel": f"{kname} (force + stream + collide)",
            "copy_ceiling": round(copy_gbps, 1),
            "frac_of_copy_ceiling": round(achieved / copy_gbps, 4),
            "bytes_per_site": lb_bytes, "avg_launch_us": lb_avg_s * 1e6, "launches": lb_n,
            "working_set_MB": round(ws / 1e6, 1),
            "level": ("past-L2: the working set fits the 256 MB Infinity Cache, so this is not an "
                      "HBM figure" if resident else "HBM: the working set exceeds the 256 MB "
                      "Infinity Cache")}
    return {
        "params": p, "phi0": phi0, "mlups": round(mlups, 1), "ms_per_step": dt / steps * 1e3,
        "config": {"workload": f"{lattice} {shape} cold walls, tau={p['tau']}, xi={p['xi']}, "
                               f"n_phi={n_phi}, n_T={n_T}{extras}",
                   "name": wl, "lattice": lattice, "shape": shape, "tau": p["tau"],
                   "pop_storage": "fp16" if pop_storage else "fp32",
                   "xi": p["xi"], "n_phi_sub": n_phi, "seed": 1},
        "roofline": roof,
        "step_effective_roofline_frac": round(mlups * 1e6 * step_bytes / 8e12, 4),
        "kernel_avg_us": {kname: lb_avg_s * 1e6,
                          ("phi2d" if dim == 2 else "phi3d"): phi_ms / max(phi_n, 1) * 1e3},
        "state_finite_at_end": not ob["nonfinite"],
    }


if __name__ == "__main__":
    main()
