#!/usr/bin/env python3
"""Throughput of the Strang-split fiber monodomain solver on one MI355X.

Workload (the batched plain Hodgkin-Huxley case): 1369 fibers with lengths
drawn uniformly from 1000..1500 nodes (h = 0.01 cm), each stimulated for
0.1 ms on three nodes in the central 10 % of the fiber at a seeded time in
[0, 5] ms, V_m noise N(0, 0.1 mV); dt_0D = dt_1D = dt_split = 1e-3 ms,
20 ms simulated (20000 split steps), FP32 on the GPU.

One bench step is the whole hot path over that batch: the initial state
(resting state plus noise, on the device), then fib_run over all 20000
split steps -- stimulus, R(dt/2) D(dt) R(dt/2), activation times and V_m
samples every 0.1 ms -- with inputs resident in HBM.

Prints one JSON line.  `value` = node-steps per second (one node advanced
through one split step), whole job.  `roofline` reports the fused kernel's
achieved VALU issue rate from its algorithmic op count against the chip's
FP32 VALU issue peak; `cpu_baseline` times the FP64 oracle on a bounded
subset of the same fibers on the host cores and doubles as a parity check
of those fibers.

`surrogate` (skipped with --no-surrogate) compares the plain FP32 method
with the learned surrogate step on the two surrogate workloads, each
network trained here on the GPU by the library's own kernels from plain
runs of a training realization and evaluated on an independent one:
  hh:   1369 x 1481 Hodgkin-Huxley nodes, dt_split 5e-3 ms (three Heun
        substeps of each half), 20 ms; network 5 -> 64 -> 64 -> 64 -> 4 SiLU;
  st57: 10000 x 2000 ST57 nodes (2e7), stimuli at 100 Hz from seeded onsets
        in [0, 10) ms, dt_split 5e-4 ms; network 57 -> 128 -> 128 -> 57
        ReLU; a bounded window of --st57-ms simulated ms is timed.
For each: node-steps/s of the plain path(s) and of the surrogate path over
the same run, the V_m / activation-time differences between them, the
rejected (fallback) share, and the FP64 oracle's V_m / activation-time
errors of the surrogate run on sampled fibers.

`adaptive` (skipped with --no-adaptive) compares the plain paths with the
adaptive computation of the subcellular model (relative tolerance
--adapt-tol) from an equilibrium start -- the scheme's premise: the same
fibers and stimuli without the initial noise --
  hh:   the 1369-fiber bundle above, 20 ms: plain fused vs adaptive in the
        fused kernel (states in LDS, solved nodes compacted per step) and in
        the split schedule;
  st57: 400 x 1481 ST57 nodes, stimuli in [0, 2] ms, 5 ms: plain split vs
        adaptive (split).
Reported: node-steps/s over all node-steps of the run, the share of
node-steps the adaptive run solved, and the FP64 oracle's V_m /
activation-time errors of the adaptive run on sampled fibers (against the
plain method).

`emg` (skipped with --no-emg) couples the static bidomain step to the fiber
solve: 37 x 37 fibers of 1481 nodes (the headline's stimulus recipe), a 3D
mesh of every 10th fiber node (37 x 37 x 149 nodes, 0.05 cm between fibers,
sigma_i 8.93, sigma_e 6.7 along / 3.35 across the fibers, mS/cm), and one
phi_e solve (CG to a relative residual of 1e-6, warm-started) every
--emg-every split steps (default 500: 0.5 ms, the 2 kHz sampling of an EMG
recording) over 20 ms: node-steps/s of the coupled run, the
share of time in the EMG solves, CG iterations and time per iteration, and
the FP64 residual of the last phi_e with the oracle's matrices.

`exp_approx` (skipped with --no-exp-approx) runs the headline workload with
the membrane whose exponentials are exp*(x) = (1 + x/1024)^1024 (the
thesis's approximation; on gfx950 the native exponential is one FMA and one
v_exp_f32, exp* an FMA and ten squarings): node-steps/s of the fused kernel,
its FP64-oracle parity against the exp* model, and how far that model lies
from the exact membrane, on sampled fibers.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "subcellular node-steps/sec at ≤0.5 mV Vm error: plain FP32 vs surrogate"

# Algorithmic cost of one node-step of the plain Hodgkin-Huxley path, in
# FP32 VALU issue slots (one slot = one lane-cycle of a 16-lane SIMD).  add,
# sub, mul, FMA, compare and select take one slot; v_exp_f32 and v_rcp_f32
# issue at half the FMA rate on gfx950 (measured), so they take two.  Counted
# from the formulas as the method is carried out in FP32 (states as offsets
# from rest, removable singularities guarded), not from the compiled code:
#   right-hand side G at absolute states, its V component scaled by Cm:
#     quotient arguments x_m, x_n/10 2; four exponentials (FMA argument +
#     exp) 12 and exp(x_n) as a constant multiple of exp(x_m) 1; two
#     quotients c x / (e^x - 1) with their guard (sub, rcp, mul, compare,
#     select of the limit c) 12; beta_h = 1/(c exp(x_m) + 1) 3; m^3 h and
#     n^4 5; I_ion as three driving-force FMAs and two FMAs 5; I - I_ion 1;
#     three gate rates 6  = 47
#   Heun step: offsets to absolute states 4 + 2 G + stage state 4 + sum 4
#     + update 4 (tau/2 and tau/Cm are per-launch constants) = 110
#   reaction: two half steps of one Heun substep each = 220
#   Crank-Nicolson: right-hand side 5, elimination 3, update 3 = 11
#   activation-time test: 2
# The counter-measured issue (rocprofv3 SQ_INSTS_VALU, transcendental
# instructions counted twice) agrees with this figure to a few percent.
SLOTS_PER_NODE_STEP = 233
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9
# EMG conjugate-gradient iteration, per mesh node (FP32 vectors): the
# stencil launch reads r, 1/diag, p_old and writes p, q (20 B); the update
# launch reads p, q, 1/diag, x, r and writes x, r (28 B)
EMG_BYTES_PER_NODE_ITERATION = 48


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--t-end", type=float, default=20.0, help="simulated ms per bench step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-fibers", type=int, default=0,
                    help="fibers in the oracle sample (default: 2 per host thread)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default workgroup shape instead of measuring candidates")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--sur-train-steps", type=int, default=20000)
    ap.add_argument("--sur-tol", type=float, default=1e-2)
    ap.add_argument("--no-sur-relu", action="store_true",
                    help="skip the Hodgkin-Huxley surrogate with a ReLU network")
    ap.add_argument("--no-adaptive", action="store_true")
    ap.add_argument("--no-exp-approx", action="store_true")
    ap.add_argument("--no-emg", action="store_true")
    ap.add_argument("--emg-every", type=int, default=500,
                    help="split steps between two EMG solves (500: a 2 kHz EMG sampling)")
    ap.add_argument("--adapt-tol", type=float, default=1e-6)
    ap.add_argument("--adapt-cases", default="hh,st57",
                    help="comma-separated adaptive cases to run (hh, st57)")
    ap.add_argument("--no-adapt-parity", action="store_true",
                    help="skip the oracle parity of the adaptive runs")
    ap.add_argument("--st57-ms", type=float, default=1.0,
                    help="simulated ms of the large ST57 bundle timed per path")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB before the timed "
                         "region, as the known-size reference for HBM byte counters")
    return ap.parse_args()


KERNEL_SOURCES = ("paper_2107_07104_amd/csrc/fib_kernels.hip",
                  "paper_2107_07104_amd/csrc/hh_model.h",
                  "paper_2107_07104_amd/csrc/fib_internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_run_hh.json")
SUR_SOURCES = ("paper_2107_07104_amd/csrc/surrogate_kernels.hip",
               "paper_2107_07104_amd/csrc/surrogate_internal.h",
               "paper_2107_07104_amd/csrc/st57_model.h",
               "paper_2107_07104_amd/csrc/hh_model.h",
               "paper_2107_07104_amd/csrc/fib_internal.h")
SUR_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_surrogate_st57.json")
# Algorithmic HBM bytes per node of one ST57 surrogate step: read and write
# the 57 FP32 states (456), the node's stimulus entry (4), the previous V_m
# for the activation test (read and write, 8) and the activation time (4).
SUR_ST57_BYTES_PER_NODE = 472
HBM_PEAK = 8.0e12
MFMA_BF16_PEAK = 2.5e15
# Matrix-core work per node of the ST57 network as the kernel runs it
# (inputs padded to 64, outputs to 64): 2 (64 x 128 + 128 x 128 + 128 x 64)
SUR_ST57_FLOP_PER_NODE = 65536


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(path=TRAFFIC_FILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    runs, or None if the kernel sources changed since they were taken."""
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash(sources):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(w, gpu_samples, gpu_tact, fibers):
    """Times the FP64 oracle on the first `fibers` fibers of the workload and
    compares them with the GPU run."""
    from oracle import oracle as O
    sub = w.subset(list(range(fibers)))
    cfg = O.Config(dt_0D=sub.dt_0D, dt_1D=sub.dt_1D, dt_split=sub.dt_split, v_th=sub.v_th)
    y0 = np.tile(O.rest_state()[:, None], (1, sub.n_total))
    y0[0] += sub.vm_noise.astype(np.float32)
    t0 = time.perf_counter()
    yo, so, to = O.run(cfg, sub.n_nodes, y0, sub.stims, sub.n_steps,
                       sample_every=sub.sample_every)
    dt = time.perf_counter() - t0
    n = sub.n_total
    vm_err = float(np.max(np.abs(gpu_samples[:, :n] - so)))
    tg = gpu_tact[:n].astype(np.float64)
    both = np.isfinite(tg) & np.isfinite(to)
    tact_err = float(np.max(np.abs(tg[both] - to[both]))) if both.any() else 0.0
    mismatch = int(np.sum(np.isfinite(tg) != np.isfinite(to)))
    return sub.node_steps() / dt, dict(fibers=fibers, nodes=n, seconds=dt, vm_max_err_mV=vm_err,
                                       tact_max_err_ms=tact_err, tact_mismatch=mismatch,
                                       activated=int(both.sum()))


def _log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def _timed_run(s, w, init, sample_every):
    """Initial state, then one fib_run over the whole workload with V_m
    samples; returns (seconds, samples [rows, n_total] on the device, t_act)."""
    import torch
    rows = w.n_steps // sample_every
    samples = torch.empty((rows, w.n_total), device="cuda")
    init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run(0, w.n_steps, sample_every, samples)
    s.sync()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, samples, s.tact()


def _compare(sa, ta, sb, tb, dt_split, t_end):
    """V_m and activation-time differences of run b against run a.  Nodes
    that activate in one run only are reported with the earliest activation
    time among them: within one split step of t_end, the other run would
    activate after the window."""
    dv = float((sa - sb).abs().max().item()) if sa.numel() else 0.0
    fa, fb = np.isfinite(ta), np.isfinite(tb)
    both = fa & fb
    one = fa != fb
    first = float(np.min(np.where(fa, ta, tb)[one])) if one.any() else None
    return dict(vm_max_diff_mV=dv,
                tact_max_diff_ms=float(np.max(np.abs(ta[both] - tb[both]))) if both.any() else 0.0,
                tact_mismatch=int(one.sum()), mismatch_earliest_tact_ms=first,
                t_end_ms=t_end, activated=int(both.sum()), dt_split_ms=dt_split)


def _oracle_parity(w, fibers, y0_cols, gpu_samples, gpu_tact, n_steps):
    """FP64 oracle on the listed fibers over the first n_steps split steps,
    against the GPU samples and activation times of the same nodes."""
    from oracle import oracle as O
    sub = w.subset(fibers).with_steps(n_steps)
    cfg = O.Config(model=sub.model, dt_0D=sub.dt_0D, dt_1D=sub.dt_1D, dt_split=sub.dt_split,
                   v_th=sub.v_th, Cm=sub.Cm, Am=sub.Am, sigma=sub.sigma, h=sub.h)
    t0 = time.perf_counter()
    yo, so, to = O.run(cfg, sub.n_nodes, y0_cols, sub.stims, n_steps, sample_every=w.sample_every)
    secs = time.perf_counter() - t0
    import torch
    off = w.offsets
    cols = np.concatenate([np.arange(off[f], off[f + 1]) for f in fibers])
    rows = n_steps // w.sample_every
    ci = torch.as_tensor(cols, device=gpu_samples.device)
    gs = gpu_samples[:rows].index_select(1, ci).cpu().numpy().astype(np.float64)
    tg = gpu_tact[cols].astype(np.float64)
    # activation times only count within the oracle's window
    tg = np.where(tg <= n_steps * w.dt_split, tg, np.inf)
    both = np.isfinite(tg) & np.isfinite(to)
    return dict(fibers=[int(f) for f in fibers], nodes=int(len(cols)), split_steps=int(n_steps),
                vm_max_err_mV=float(np.max(np.abs(gs - so))) if rows else 0.0,
                tact_max_err_ms=float(np.max(np.abs(tg[both] - to[both]))) if both.any() else 0.0,
                tact_mismatch=int(np.sum(np.isfinite(tg) != np.isfinite(to))),
                activated=int(both.sum()), oracle_seconds=secs)


def surrogate_hh(args):
    """Hodgkin-Huxley surrogate workload: train, then plain fused, plain
    split and surrogate runs of an independent realization."""
    from dataclasses import replace

    from paper_2107_07104_amd import fib as F
    from paper_2107_07104_amd import inputs as I
    from paper_2107_07104_amd import surrogate as SU
    wt = SU.hh_training_workload()
    snaps = [int(round(t / wt.dt_split)) for t in (1.0, 3.0, 5.0, 7.0, 10.0)]
    t0 = time.perf_counter()
    sur = SU.train_surrogate(I.MODEL_HH, wt, snaps, steps=args.sur_train_steps,
                             log=lambda m: _log("hh surrogate:" + m))
    train_s = time.perf_counter() - t0
    w = replace(I.batched_hh(n_min=1481, n_max=1481, dt=5e-3, realization=1), dt_0D=1e-3,
                name="hh_surrogate_eval_1369x1481")
    vm = w.vm_noise.astype(np.float32)
    res = {}
    runs = {}
    for path, sched in (("plain_fused", F.FIB_SCHED_FUSED), ("plain_split", F.FIB_SCHED_SPLIT),
                        ("surrogate", F.FIB_SCHED_SPLIT)):
        s = SU._solver(w, schedule=sched)
        s.set_stimulus(w.stims)
        net = None
        if path == "surrogate":
            net = sur.network()
            s.set_surrogate(net, sur.scales, args.sur_tol)
        _timed_run(s, w.with_steps(40), lambda: s.init_state(vm_noise=vm), w.sample_every)
        secs, smp, ta = _timed_run(s, w, lambda: s.init_state(vm_noise=vm), w.sample_every)
        runs[path] = (smp, ta)
        res[path] = dict(value=w.node_steps() / secs, seconds=secs)
        if net is not None:
            res[path]["fallbacks_last_step"] = int(s.last_fallbacks())
            net.close()
        s.close()
        _log(f"hh {path}: {res[path]['value']:.3e} node-steps/s")
    sp, tp = runs["plain_split"]
    ss, ts = runs["surrogate"]
    fibers = [0, 1, 2, 3]
    off = w.offsets
    from oracle import oracle as O
    cols = np.concatenate([np.arange(off[f], off[f + 1]) for f in fibers])
    y0 = np.tile(O.rest_state(I.MODEL_HH)[:, None], (1, len(cols)))
    y0[0] += vm[cols]
    parity = _oracle_parity(w, fibers, y0, ss, ts, w.n_steps)
    best_plain = max(res["plain_fused"]["value"], res["plain_split"]["value"])
    relu = None
    if not args.no_sur_relu:
        # the same network with ReLU: one packed integer max per two
        # activations instead of an exponential and a reciprocal each
        t0 = time.perf_counter()
        sr = SU.train_surrogate(I.MODEL_HH, wt, snaps, steps=args.sur_train_steps, act="relu",
                                log=lambda m: _log("hh relu surrogate:" + m))
        tr_s = time.perf_counter() - t0
        s = SU._solver(w, schedule=F.FIB_SCHED_SPLIT)
        s.set_stimulus(w.stims)
        net = sr.network()
        s.set_surrogate(net, sr.scales, args.sur_tol)
        _timed_run(s, w.with_steps(40), lambda: s.init_state(vm_noise=vm), w.sample_every)
        secs, sr_s, sr_t = _timed_run(s, w, lambda: s.init_state(vm_noise=vm), w.sample_every)
        fb = int(s.last_fallbacks())
        net.close()
        s.close()
        relu = dict(network="5-64-64-64-4 ReLU, BF16 MFMA", value=w.node_steps() / secs,
                    seconds=secs, fallbacks_last_step=fb,
                    train=dict(adam_steps=sr.info["steps"], final_loss=sr.info["losses"][-1][1],
                               seconds=tr_s),
                    over_best_plain=w.node_steps() / secs / best_plain,
                    vs_plain_split=_compare(sp, tp, sr_s, sr_t, w.dt_split,
                                            w.n_steps * w.dt_split),
                    vs_oracle=_oracle_parity(w, fibers, y0, sr_s, sr_t, w.n_steps))
        _log(f"hh relu surrogate: {relu['value']:.3e} node-steps/s, "
             f"{relu['over_best_plain']:.2f}x the best plain path")
    return dict(workload=w.name, fibers=int(len(w.n_nodes)), nodes=int(w.n_total),
                split_steps=int(w.n_steps), dt_split_ms=w.dt_split, dt_0D_ms=w.dt_0D,
                network="5-64-64-64-4 SiLU, BF16 MFMA", tol=args.sur_tol,
                train=dict(pairs=sur.info["pairs"], adam_steps=sur.info["steps"],
                           final_loss=sur.info["losses"][-1][1], seconds=train_s,
                           workload="realization 0 of the same bundle"),
                **res, surrogate_over_best_plain=res["surrogate"]["value"] / best_plain,
                surrogate_vs_plain_split=_compare(sp, tp, ss, ts, w.dt_split, w.n_steps * w.dt_split),
                surrogate_vs_oracle=parity, relu_variant=relu)


def surrogate_st57(args):
    """Large ST57 bundle: train on the 400 x 1481 bundle, then time the
    plain split path and the surrogate path on 10000 x 2000 nodes."""
    import torch

    from paper_2107_07104_amd import fib as F
    from paper_2107_07104_amd import inputs as I
    from paper_2107_07104_amd import surrogate as SU
    wt = I.st57_bundle(n_fibers=400, n_nodes=1481, t_end=5.0)
    snaps = [int(round(t / wt.dt_split)) for t in (0.5, 1.5, 2.5, 3.5, 4.5)]
    t0 = time.perf_counter()
    sur = SU.train_surrogate(I.MODEL_ST57, wt, snaps, steps=args.sur_train_steps,
                             log=lambda m: _log("st57 surrogate:" + m))
    train_s = time.perf_counter() - t0
    w = I.st57_bundle(n_fibers=10000, n_nodes=2000, t_end=args.st57_ms, onset_max=10.0,
                      period_ms=10.0, realization=2, host_noise=False)
    rel = I.device_rel_noise(w)
    res = {}
    runs = {}
    for path in ("plain_split", "surrogate"):
        s = SU._solver(w, schedule=F.FIB_SCHED_SPLIT)
        s.set_stimulus(w.stims)
        net = None
        if path == "surrogate":
            net = sur.network()
            s.set_surrogate(net, sur.scales, args.sur_tol)
        _timed_run(s, w.with_steps(20), lambda: s.init_state(rel_noise=rel), w.sample_every)
        secs, smp, ta = _timed_run(s, w, lambda: s.init_state(rel_noise=rel), w.sample_every)
        runs[path] = (smp, ta)
        res[path] = dict(value=w.node_steps() / secs, seconds=secs)
        if net is not None:
            res[path]["fallbacks_last_step"] = int(s.last_fallbacks())
            net.close()
        s.close()
        _log(f"st57 {path}: {res[path]['value']:.3e} node-steps/s")
    # the surrogate step kernel alone, timed with HIP events on the library's
    # stream (each step also launches the fallback kernel, a few percent)
    s = SU._solver(w, schedule=F.FIB_SCHED_SPLIT)
    s.set_stimulus(w.stims)
    net = sur.network()
    s.set_surrogate(net, sur.scales, args.sur_tol)
    s.init_state(rel_noise=rel)
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(10)]
    s.step_surrogate(0)
    for j, (e0, e1) in enumerate(evs):
        e0.record(stream)
        s.step_surrogate(1 + j)
        e1.record(stream)
    s.sync()
    torch.cuda.synchronize()
    step_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    net.close()
    s.close()
    achieved = SUR_ST57_BYTES_PER_NODE * w.n_total / (step_ms * 1e-3)
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": achieved / HBM_PEAK,
                "traffic": measured_traffic(SUR_TRAFFIC_FILE, SUR_SOURCES),
                "kernel": "k_surrogate<ST57> + k_fallback", "ms_per_step": step_ms,
                "bytes_per_node": SUR_ST57_BYTES_PER_NODE,
                "mfma_tflops": SUR_ST57_FLOP_PER_NODE * w.n_total / (step_ms * 1e-3) / 1e12,
                "mfma_frac": SUR_ST57_FLOP_PER_NODE * w.n_total / (step_ms * 1e-3) / MFMA_BF16_PEAK}
    _log(f"st57 surrogate step: {step_ms:.3f} ms, {achieved / 1e9:.0f} GB/s")
    sp, tp = runs["plain_split"]
    ss, ts = runs["surrogate"]
    cmp_plain = _compare(sp, tp, ss, ts, w.dt_split, w.n_steps * w.dt_split)
    # oracle on the fibers stimulated first (activity inside the window)
    onsets = np.array([st["step_on"] for st in w.stims])
    fibers = sorted(int(f) for f in np.argsort(onsets, kind="stable")[:8])
    off = w.offsets
    from oracle import oracle as O
    cols = np.concatenate([np.arange(off[f], off[f + 1]) for f in fibers])
    relc = rel[:, torch.as_tensor(cols, device="cuda")].cpu().numpy().astype(np.float64)
    y0 = O.rest_state(I.MODEL_ST57)[:, None] * (1.0 + relc)
    n_or = w.n_steps
    parity = _oracle_parity(w, fibers, y0, ss, ts, n_or)
    del rel, runs, sp, ss
    torch.cuda.empty_cache()
    return dict(workload=f"st57_10000x2000_100Hz_{args.st57_ms:g}ms", fibers=int(len(w.n_nodes)),
                nodes=int(w.n_total), split_steps=int(w.n_steps), dt_split_ms=w.dt_split,
                dt_0D_ms=w.dt_0D, network="57-128-128-57 ReLU, BF16 MFMA", tol=args.sur_tol,
                train=dict(pairs=sur.info["pairs"], adam_steps=sur.info["steps"],
                           final_loss=sur.info["losses"][-1][1], seconds=train_s,
                           workload="st57 400 x 1481 bundle, 5 ms"),
                **res, surrogate_over_plain=res["surrogate"]["value"] / res["plain_split"]["value"],
                surrogate_vs_plain_split=cmp_plain, surrogate_vs_oracle=parity,
                roofline=roofline)


def adaptive_bench(args):
    """Plain vs adaptive computation from an equilibrium start (see the
    module docstring)."""
    from dataclasses import replace

    from paper_2107_07104_amd import fib as F
    from paper_2107_07104_amd import inputs as I
    from oracle import oracle as O
    out = {}
    cases = (
        ("hh", replace(I.batched_hh(t_end=args.t_end), rel_noise=None),
         (("plain_fused", F.FIB_SCHED_FUSED, 0.0), ("adaptive", F.FIB_SCHED_FUSED, args.adapt_tol),
          ("adaptive_split", F.FIB_SCHED_SPLIT, args.adapt_tol)),
         [0, 1, 2, 3]),
        ("st57", I.st57_bundle(n_fibers=400, n_nodes=1481, t_end=5.0, host_noise=False),
         (("plain_split", F.FIB_SCHED_SPLIT, 0.0), ("adaptive", F.FIB_SCHED_SPLIT, args.adapt_tol)),
         [0, 1]),
    )
    wanted = set(args.adapt_cases.split(","))
    for name, w, paths, fibers in cases:
        if name not in wanted:
            continue
        w = replace(w, vm_noise=np.zeros_like(w.vm_noise))
        res = {}
        runs = {}
        for path, sched, tol in paths:
            s = F.Solver(w.n_nodes, model=w.model, schedule=sched, Cm=w.Cm, Am=w.Am,
                         sigma=w.sigma, h=w.h, dt_0D=w.dt_0D, dt_1D=w.dt_1D,
                         dt_split=w.dt_split, v_th=w.v_th)
            s.set_stimulus(w.stims)
            if sched == F.FIB_SCHED_FUSED:
                s.init_state()
                s.autotune(trial_steps=200, max_candidates=8)
            if tol > 0.0:
                s.set_adaptive(tol)
            _timed_run(s, w.with_steps(50), lambda: s.init_state(), w.sample_every)
            before = s.adaptive_solved() if tol > 0.0 else 0
            secs, smp, ta = _timed_run(s, w, lambda: s.init_state(), w.sample_every)
            runs[path] = (smp, ta)
            res[path] = dict(value=w.node_steps() / secs, seconds=secs, plan=s.plan())
            if tol > 0.0:
                res[path]["tol"] = tol
                res[path]["solved_share"] = (s.adaptive_solved() - before) / w.node_steps()
            s.close()
            _log(f"adaptive {name} {path}: {res[path]['value']:.3e} node-steps/s "
                 f"{res[path].get('solved_share', '')}")
        p0 = paths[0][0]
        sp, tp = runs[p0]
        sa, ta = runs["adaptive"]
        off = w.offsets
        cols = np.concatenate([np.arange(off[f], off[f + 1]) for f in fibers])
        y0 = np.tile(O.rest_state(w.model)[:, None], (1, len(cols)))
        parity = (None if args.no_adapt_parity
                  else _oracle_parity(w, fibers, y0, sa, ta, w.n_steps))
        out[name] = dict(workload=f"{w.name}, equilibrium start", fibers=int(len(w.n_nodes)),
                         nodes=int(w.n_total), split_steps=int(w.n_steps),
                         dt_split_ms=w.dt_split, **res,
                         adaptive_over_plain=res["adaptive"]["value"] / res[p0]["value"],
                         adaptive_vs_plain=_compare(sp, tp, sa, ta, w.dt_split,
                                                    w.n_steps * w.dt_split),
                         adaptive_vs_oracle_plain=parity)
    return out


def emg_bench(args):
    """The fiber solve coupled to the static bidomain step (module docstring)."""
    import torch

    from paper_2107_07104_amd import fib as F
    from paper_2107_07104_amd import inputs as I
    from oracle import emg as E
    nf, n, m, hxy = 37, 1481, 10, 0.05
    sig = dict(sigma_i=8.93, sigma_el=6.7, sigma_et=3.35)
    w = I.batched_hh(n_fibers=nf * nf, n_min=n, n_max=n, t_end=args.t_end)
    s = F.Solver(w.n_nodes, dt_0D=w.dt_0D, dt_1D=w.dt_1D, dt_split=w.dt_split)
    s.set_stimulus(w.stims)
    vm = torch.as_tensor(w.vm_noise.astype(np.float32), device="cuda")
    s.init_state(vm_noise=vm)
    s.autotune(trial_steps=200, max_candidates=8)
    emg = F.Emg(s, nf, nf, m, hxy, hxy, **sig)
    every = args.emg_every

    def run(timed):
        s.init_state(vm_noise=vm)
        its, t_emg = [], 0.0
        t0 = time.perf_counter()
        for c in range(0, w.n_steps, every):
            s.run(c, min(every, w.n_steps - c))
            if timed:
                s.sync()
                t1 = time.perf_counter()
            it, rel = emg.solve(tol=1e-6, max_iter=5000)
            if timed:
                t_emg += time.perf_counter() - t1
            its.append(it)
        s.sync()
        return time.perf_counter() - t0, its, t_emg

    run(False)                                   # warm-up (code objects, first solves)
    secs, its, _ = run(False)
    _, _, t_emg = run(True)                       # EMG share with a sync around each solve
    phi = emg.phi()
    V3 = E.prolongate(s.get_state()[0], nf, nf, n, m)
    g = E.Grid(nf, nf, (n - 1) // m + 1, hxy, hxy, m * w.h)
    Ki = E.stiffness_3d(g, (0.0, 0.0, sig["sigma_i"]))
    Kt = E.stiffness_3d(g, (sig["sigma_et"], sig["sigma_et"], sig["sigma_el"] + sig["sigma_i"]))
    b = -(Ki @ V3)
    b -= b.mean()
    res = float(np.linalg.norm(b - Kt @ phi) / np.linalg.norm(b))
    plan = s.plan()
    emg.close()
    s.close()
    n_solves = len(its)
    tot_it = int(sum(its))
    # CG iteration against HBM: algorithmic bytes per mesh node and iteration
    # (EMG_BYTES_PER_NODE_ITERATION) over the whole synchronized solve time,
    # so right-hand side, start, host checks and the final shift count too
    gbs = EMG_BYTES_PER_NODE_ITERATION * g.n * tot_it / t_emg / 1e9
    roof = dict(bound="hbm", achieved=gbs, peak=HBM_PEAK / 1e9, unit="GB/s",
                frac=gbs * 1e9 / HBM_PEAK, traffic=None, kernel="k_cg_q + k_cg_x",
                bytes_per_node_iteration=EMG_BYTES_PER_NODE_ITERATION,
                timing="whole EMG solves (host clock around synchronized solves)")
    out = dict(workload=f"hh_emg_{nf}x{nf}x{n}, 3D mesh {nf}x{nf}x{g.nz}, solve every {every} "
                        f"split steps", value=w.node_steps() / secs, seconds=secs, plan=plan,
               emg_solves=n_solves, cg_iterations_mean=tot_it / n_solves,
               cg_iterations_max=int(max(its)), emg_seconds=t_emg,
               emg_share=t_emg / secs, ms_per_cg_iteration=(t_emg / max(tot_it, 1)) * 1e3,
               last_phi_fp64_relative_residual=res, mesh_nodes=int(g.n), roofline=roof)
    _log(f"emg: {out['value']:.3e} node-steps/s, {n_solves} solves, {tot_it / n_solves:.1f} "
         f"CG iterations each, EMG share {out['emg_share']:.2f}, residual {res:.1e}")
    return out


def exp_approx_bench(args):
    """The headline workload with the exp* membrane (see the module docstring)."""
    from dataclasses import replace

    import torch

    from paper_2107_07104_amd import fib as F
    from paper_2107_07104_amd import inputs as I
    from oracle import oracle as O
    w = replace(I.batched_hh(t_end=args.t_end), model=F.FIB_MODEL_HH_APX_EXP)
    s = F.Solver(w.n_nodes, model=w.model, dt_0D=w.dt_0D, dt_1D=w.dt_1D, dt_split=w.dt_split)
    s.set_stimulus(w.stims)
    vm = torch.as_tensor(w.vm_noise.astype(np.float32), device="cuda")
    s.init_state(vm_noise=vm)
    s.autotune(trial_steps=200, max_candidates=8)
    _timed_run(s, w.with_steps(50), lambda: s.init_state(vm_noise=vm), w.sample_every)
    secs, smp, ta = _timed_run(s, w, lambda: s.init_state(vm_noise=vm), w.sample_every)
    plan = s.plan()
    s.close()
    _log(f"exp* membrane: {w.node_steps() / secs:.3e} node-steps/s")
    fibers = [0, 1, 2, 3]
    off = w.offsets
    cols = np.concatenate([np.arange(off[f], off[f + 1]) for f in fibers])
    out = dict(workload=f"{w.name}, exp* membrane", value=w.node_steps() / secs, seconds=secs,
               plan=plan)
    for model, key in ((F.FIB_MODEL_HH_APX_EXP, "vs_oracle_exp_star"),
                       (F.FIB_MODEL_HH, "vs_oracle_exact_membrane")):
        y0 = np.tile(O.rest_state(model)[:, None], (1, len(cols)))
        y0[0] += w.vm_noise[cols].astype(np.float32)
        out[key] = _oracle_parity(replace(w, model=model), fibers, y0, smp, ta, w.n_steps)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the fibers are "
              "independent, so a multi-GPU run would shard whole fibers with no "
              "communication -- not measured here.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2107_07104_amd import fib as F
    from paper_2107_07104_amd import inputs as I

    torch.cuda.set_device(0)
    w = I.batched_hh(t_end=args.t_end)
    stream = torch.cuda.current_stream()
    s = F.Solver(w.n_nodes, stream=stream.cuda_stream, dt_0D=w.dt_0D, dt_1D=w.dt_1D,
                 dt_split=w.dt_split)
    s.set_stimulus(w.stims)
    vm = torch.as_tensor(w.vm_noise.astype(np.float32), device="cuda")
    rows = w.n_steps // w.sample_every
    samples = torch.empty((rows, w.n_total), device="cuda")
    default_plan = s.plan()
    tuned = None
    if not args.no_autotune:
        # workgroup shape measured on the workload itself (outside the timed region)
        F.fib_init_state(s.ctx, vm.data_ptr(), 0)
        tuned = s.autotune(trial_steps=200, max_candidates=8)
    plan = s.plan()
    print(f"# workload {w.name}: {w.n_total} nodes, {w.n_steps} split steps; default plan "
          f"{default_plan}, plan {plan}", file=sys.stderr, flush=True)

    def step(ev=None):
        F.fib_init_state(s.ctx, vm.data_ptr(), 0)
        if ev is not None:
            ev[0].record(stream)
        s.run(0, w.n_steps, w.sample_every, samples)
        if ev is not None:
            ev[1].record(stream)

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(f"# calibration copy of {args.copy_calibration_mib} MiB done", file=sys.stderr,
              flush=True)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"# warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    s.sync()

    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s.sync()
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    print(f"# timed {args.steps} steps in {elapsed:.3f} s; fused kernel {kernel_ms:.2f} ms/launch",
          file=sys.stderr, flush=True)

    node_steps = w.node_steps()
    value = node_steps * args.steps / elapsed
    achieved = node_steps * SLOTS_PER_NODE_STEP / (kernel_ms * 1e-3)
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": VALU_PEAK_SLOTS / 1e12,
        "unit": "Tslot/s (FP32 VALU issue slots)",
        "frac": achieved / VALU_PEAK_SLOTS,
        "traffic": measured_traffic(),
        "kernel": "k_run_hh",
        "kernel_ms_per_launch": kernel_ms,
        "slots_per_node_step": SLOTS_PER_NODE_STEP,
    }

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        fibers = args.cpu_fibers or 2 * threads
        gs = samples.cpu().numpy().astype(np.float64)
        gt = s.tact()
        rate, parity = cpu_baseline(w, gs, gt, min(fibers, len(w.n_nodes)))
        cpu = {"value": rate, "unit": "node-steps/s", "cores": threads, "kind": "oracle",
               "sample": f"first {parity['fibers']} fibers ({parity['nodes']} nodes) of the "
                         f"same workload, all {w.n_steps} split steps, FP64, OpenMP over fibers"}
        print(f"# oracle: {rate:.3e} node-steps/s on {threads} threads; parity {parity}",
              file=sys.stderr, flush=True)

    sur = None
    adapt = None
    expx = None
    emg = None
    if (not args.no_surrogate or not args.no_adaptive or not args.no_exp_approx
            or not args.no_emg):
        s.close()
        s = None
    if not args.no_surrogate:
        sur = {"hh": surrogate_hh(args), "st57": surrogate_st57(args)}
    if not args.no_adaptive:
        adapt = adaptive_bench(args)
    if not args.no_emg:
        emg = emg_bench(args)
        emg["over_plain"] = emg["value"] / value
    if not args.no_exp_approx:
        expx = exp_approx_bench(args)
        expx["over_plain"] = expx["value"] / value

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "node-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "hh_batched_1369_fibers_1000-1500_nodes_20ms",
                   "fibers": int(len(w.n_nodes)), "nodes": int(w.n_total),
                   "split_steps": int(w.n_steps), "dt_split_ms": w.dt_split,
                   "schedule": "fused", "plan": plan, "default_plan": default_plan,
                   "autotune": tuned, "path": "plain"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "surrogate": sur,
        "adaptive": adapt,
        "exp_approx": expx,
        "emg": emg,
    }
    if s is not None:
        s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
