#!/usr/bin/env python3
"""Throughput of the Strang-split fiber monodomain solver on one MI355X:
subcellular node-steps per second at <= 0.5 mV V_m error, plain FP32
against the learned surrogate.

Headline workload (the large bundle, plain vs surrogate): 10000 fibers x
2000 nodes (2e7 nodes, h = 0.01 cm) of the 57-state ST57 model, every state
at rest times (1 + 0.01 N(0, 1)), each fiber stimulated for 0.1 ms every
10 ms (100 Hz) on three nodes in the central 10 % from a seeded onset in
[0, 10) ms; dt_0D = 1e-4 ms, dt_1D = dt_split = 5e-4 ms, 10 ms simulated
(20000 split steps), FP32 on the GPU, 4.6 GB of state resident in HBM.

One bench step is 1000 split steps (0.5 ms) of the whole hot path on that
bundle -- stimulus, the reaction halves (for the surrogate path: the
network's prediction, the implicit-midpoint corrector, the acceptance test
and the Heun fallback of rejected nodes), the Crank-Nicolson diffusion,
activation times and V_m samples every 0.1 ms -- so the default 20 steps
are the configured 10 ms from the initial state.  Warm-up steps run from
the same initial state before it is set again.

`value` is the node-steps/s (one node advanced through one split step) of
the surrogate path (network 57 -> 128 -> 128 -> 57, BF16 matrix cores,
trained on the GPU here by the library's own kernels from plain runs of
another bundle; acceptance tolerance 1e-3 of each state's range) when its
V_m and activation times stay within 0.5 mV and one split step of the FP64
oracle on the sampled fibers; otherwise the plain path's.  Beside it, over
the same K steps from the same state:
  plain:     the plain split schedule (streamed ST57 reaction kernel);
  predictor: the surrogate step with the network replaced by the explicit
             Euler increment (the method without the network);
each with its rejected share, its V_m / activation-time differences to the
plain run, and its FP64-oracle errors on the sampled fibers.  `roofline`
is the surrogate step kernel against HBM; `roofline_plain` the plain
reaction kernel against the FP32 vector issue rate; `ceilings` the
device's measured peaks.  `cpu_baseline` times the FP64 oracle on the host
cores on sampled fibers whose onsets span the window (in a background
process while the GPU runs) and at one thread.

Sections (each skippable):
  hh_batched:   the batched plain Hodgkin-Huxley workload (1369 fibers of
                1000..1500 nodes, dt 1e-3 ms, 20 ms) in the fused kernel,
                with its roofline and oracle baseline;
  st57_bundle:  400 x 1481 ST57 nodes with the 1 % perturbation, 5 ms,
                plain split, with its roofline and oracle parity;
  surrogate_hh: the Hodgkin-Huxley surrogate workload (1369 x 1481 nodes,
                dt_split 5e-3 ms, 20 ms; network 5 -> 64 -> 64 -> 64 -> 4
                SiLU) against the plain fused and split paths and the Euler
                predictor, tolerance 1e-3;
  adaptive, emg, exp_approx: adaptive computation of the subcellular
                model, the coupled static bidomain (EMG) step, and the
                thesis's exp* approximation.
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

# Cost model of the FP32 vector units (gfx950), in lane-operations at the
# published FP32 vector peak, 157.3 TFLOP/s = 256 CUs x 4 SIMDs x 32 lanes
# per clock x 2.4 GHz x 2 FLOP per FMA: an add, sub, mul, FMA, compare,
# select or max is one operation; v_exp_f32, v_log_f32 and v_rcp_f32 run at
# a quarter of that rate, so each counts four.  The probes of `ceilings`
# measure both on the device: two-operand (VOP2) adds, multiplies and
# accumulating FMAs reach 0.95-0.98 of 78.6 T/s, transcendentals 0.98 of
# 19.7 T/s, while three-operand (VOP3) encodings of the same FMA run at half
# rate -- an implementation cost, not part of the algorithmic count.
# Packed FP32 (two operations per lane) is not used.
VALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9
TRANS = 4

# Plain Hodgkin-Huxley path, operations per node-step, counted from the
# formulas as the method is carried out in FP32 (states as offsets from
# rest, removable singularities guarded), not from the compiled code:
#   right-hand side G at absolute states, its V component scaled by Cm:
#     quotient arguments x_m, x_n/10 2; four exponentials (FMA argument +
#     exp) 4 + 4 TRANS and exp(x_n) as a constant multiple of exp(x_m) 1;
#     two quotients c x / (e^x - 1) with their guard (sub, rcp, mul,
#     compare, select of the limit c) 8 + 2 TRANS; beta_h = 1/(c exp(x_m)
#     + 1) 1 + TRANS; m^3 h and n^4 5; I_ion as three driving-force FMAs and
#     two FMAs 5; I - I_ion 1; three gate rates 6  = 33 + 7 TRANS = 61
#   Heun step: 2 G + stage state 4 + sum 4 + update 4 (tau/2 and tau/Cm
#     are per-launch constants) = 134; the kernels' conversions between the
#     stored offsets from rest and absolute states (4 per step) are an
#     implementation cost of the FP32 representation, not counted
#   reaction: two half steps of one Heun substep each = 268
#   Crank-Nicolson: right-hand side 5, elimination 3, update 3 = 11
#   activation-time test: 2
HH_RHS_OPS = 33 + 7 * TRANS
OPS_PER_NODE_STEP = 2 * (12 + 2 * HH_RHS_OPS) + 13

# ST57 right-hand side at absolute states, operations per evaluation, by
# block (the same conventions; a negation folded into its use is free):
#   Na/K pump: Na^3 2, k1 = Na^3/(1000 + Na^3) 2 + TRANS,
#     k2 = 0.8 exp(0.3 V/kT) 2 + TRANS, K_t^2 1, k3 3 + TRANS, four fluxes
#     J = k y - b y' 8, four differences 4  = 22 + 3 TRANS
#   surface membrane: m^3 h 3, n^4 2, I_Na 2, I_K 2, I_L 1,
#     E_Cl = kT (log2 Cl_i - 7) ln 2 1 + TRANS, I_Cl 2, I_c 2, dV 7
#     = 22 + TRANS
#   Hodgkin-Huxley gates (each of the two sets): arguments 2, four
#     exponentials 4 + 4 TRANS, the shared one 1, two guarded quotients
#     8 + 2 TRANS, beta_h 1 + TRANS, three gate rates 6  = 22 + 7 TRANS,
#     twice
#   tubular membrane: five more logarithms 5 TRANS (log2 Cl_i is shared),
#     three Nernst potentials 6, I_Na,t 6, I_K,t 5, I_Cl,t 2, dV_t 6
#     = 25 + 5 TRANS
#   voltage-sensor chain: E = exp(V_t/25) 1 + TRANS, 1/E TRANS, eighteen
#     rates 18, nine net flows 18, eight differences 8  = 45 + 2 TRANS
#   Ca / Mg: f_load 3, J_rel 3, J_leak 1, J_up with c+ 5 + TRANS, J_tr 2,
#     seven binding rates with their free sites 28, dc_m 5, dc_s 2, dc_j 3,
#     dg_m 1  = 53 + TRANS
#   ion concentrations: I_p 1, six rates 4+4+3+3+3+2  = 20
#   thin-filament chain: theta 1, r_f 2, r_b 2 + TRANS, seven flows 14,
#     six differences 6  = 25 + TRANS
#   cross-bridge cycle and mechanics: a 1, detachment rate 5 + 2 TRANS,
#     eight fluxes 3+6+2, eight differences 8, F_n 3, dL_s 3, dgamma 2
#     = 33 + 2 TRANS
#   total  = 291 + 29 TRANS = 407
ST57_RHS_OPS = 291 + 29 * TRANS
ST57_S = 57
# Heun step on 57 states: 2 G + stage state 57 + sum 57 + update 57 (the
# offset-to-absolute conversions, 57 per step, are not counted, as above)
ST57_HEUN_OPS = 3 * ST57_S + 2 * ST57_RHS_OPS
# reaction launch of the split schedule: the second half of step n and the
# first half of step n+1, three Heun substeps each (dt_0D = 1e-4 ms over
# 2.5e-4 ms)
ST57_REACT_OPS = 6 * ST57_HEUN_OPS
# whole node-step: reaction + Crank-Nicolson 11 + activation test 2
ST57_OPS_PER_NODE_STEP = ST57_REACT_OPS + 13

# EMG conjugate-gradient iteration, per mesh node (FP32 vectors): the
# stencil launch reads r, 1/diag, p_old and writes p, q (20 B); the update
# launch reads p, q, 1/diag, x, r and writes x, r (28 B)
EMG_BYTES_PER_NODE_ITERATION = 48

HBM_PEAK = 8.0e12
MFMA_BF16_PEAK = 2.5e15
# Algorithmic HBM bytes per node of one ST57 surrogate step: read and write
# the 57 FP32 states (456), the node's stimulus entry (4), the previous V_m
# for the activation test (read and write, 8) and the activation time (4).
SUR_ST57_BYTES_PER_NODE = 472
# Matrix-core work per node of the ST57 network: 2 (57 x 128 + 128 x 128 +
# 128 x 57) FLOP; the kernel pads inputs and outputs to 64 (65536 FLOP)
SUR_ST57_FLOP_PER_NODE = 61952
SUR_ST57_FLOP_PER_NODE_PADDED = 65536

STEP_SPLIT_STEPS = 1000        # split steps per bench step of the headline
HEADLINE_T_END_MS = 10.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=20,
                    help="timed bench steps of 1000 split steps (20: the configured 10 ms)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-3,
                    help="acceptance tolerance of the surrogate step (fraction of each "
                         "state's range)")
    ap.add_argument("--train-steps", type=int, default=20000)
    ap.add_argument("--oracle-fibers", type=int, default=12,
                    help="fibers of the headline bundle the oracle runs (one host thread each)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-predictor", action="store_true",
                    help="skip the headline's Euler-predictor path")
    ap.add_argument("--sections", default="hh_batched,st57_bundle,surrogate_hh,adaptive,emg,"
                    "exp_approx", help="comma-separated sections to run after the headline")
    ap.add_argument("--t-end", type=float, default=20.0,
                    help="simulated ms of the Hodgkin-Huxley sections")
    ap.add_argument("--cpu-fibers", type=int, default=0,
                    help="fibers of the Hodgkin-Huxley oracle sample (default: 2 per host thread)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default workgroup shape instead of measuring candidates")
    ap.add_argument("--no-sur-relu", action="store_true",
                    help="skip the Hodgkin-Huxley surrogate with a ReLU network")
    ap.add_argument("--emg-every", type=int, default=500,
                    help="split steps between two EMG solves (500: a 2 kHz EMG sampling)")
    ap.add_argument("--adapt-tol", type=float, default=1e-6)
    ap.add_argument("--adapt-cases", default="hh,st57",
                    help="comma-separated adaptive cases to run (hh, st57)")
    ap.add_argument("--no-adapt-parity", action="store_true",
                    help="skip the oracle parity of the adaptive runs")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB before the timed "
                         "region, as the known-size reference for HBM byte counters")
    return ap.parse_args()


def _log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """Model name and usable threads of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    return model, threads


def measure_ceilings():
    """The device's measured peaks (fib_probe) and the transcendental weights
    they imply."""
    from paper_2107_07104_amd import fib as F
    fma = F.fib_probe(F.FIB_PROBE_FMA)
    fma3 = F.fib_probe(F.FIB_PROBE_FMA_VOP3)
    ex = F.fib_probe(F.FIB_PROBE_EXP)
    rcp = F.fib_probe(F.FIB_PROBE_RCP)
    pair = F.fib_probe(F.FIB_PROBE_LOG)
    # the LOG chain alternates exp and log: time per pair = 1/exp + 1/log
    lg = 1.0 / max(2.0 / pair - 1.0 / ex, 1e-30)
    copy = F.fib_probe(F.FIB_PROBE_COPY, 4 << 30)
    mfma = F.fib_probe(F.FIB_PROBE_MFMA_BF16)
    out = dict(fma_lane_ops_per_s=fma, exp_per_s=ex, rcp_per_s=rcp, log_per_s=lg,
               fma_vop3_lane_ops_per_s=fma3,
               ops_exp=VALU_PEAK_OPS / ex, ops_rcp=VALU_PEAK_OPS / rcp, ops_log=VALU_PEAK_OPS / lg,
               fma_over_peak=fma / VALU_PEAK_OPS, fma_vop3_over_peak=fma3 / VALU_PEAK_OPS,
               hbm_copy_bytes_per_s=copy, hbm_copy_over_peak=copy / HBM_PEAK,
               mfma_bf16_flop_per_s=mfma, mfma_over_peak=mfma / MFMA_BF16_PEAK,
               note="fib_probe kernels: eight independent chains per lane (VALU), a 4 GiB "
                    "device copy counted read + write (HBM), four accumulators per wave (MFMA)")
    _log("ceilings: FMA %.2f T/s (%.2f of the peak; VOP3 %.2f), exp %.1f ops, rcp %.1f, log %.1f; "
         "copy %.2f TB/s; MFMA bf16 %.2f PFLOP/s" % (fma / 1e12, out["fma_over_peak"],
                                                       out["fma_vop3_over_peak"], out["ops_exp"],
                                                       out["ops_rcp"], out["ops_log"],
                                                       copy / 1e12, mfma / 1e15))
    return out


def _oracle_job(job):
    """Runs in a background process: the FP64 oracle on a set of fibers
    (OpenMP over fibers), and optionally one fiber at one thread for the
    single-thread rate.  Returns samples, activation times and timings."""
    os.environ["OMP_NUM_THREADS"] = str(job["threads"])
    from oracle import oracle as O
    cfg = O.Config(**job["cfg"])
    res = {}
    if job.get("one_thread_steps"):
        nn1 = job["n_nodes"][:1]
        y1 = job["y0"][:, :int(nn1[0])]
        st1 = [s for s in job["stims"] if s["fiber"] == 0]
        t0 = time.perf_counter()
        O.run(cfg, nn1, y1, st1, job["one_thread_steps"])
        res["one_thread"] = dict(seconds=time.perf_counter() - t0,
                                 node_steps=int(nn1[0]) * job["one_thread_steps"])
    t0 = time.perf_counter()
    _, s, t = O.run(cfg, job["n_nodes"], job["y0"], job["stims"], job["n_steps"],
                    sample_every=job["sample_every"])
    res.update(samples=s, tact=t, seconds=time.perf_counter() - t0)
    return res


class Background:
    """One background process for oracle jobs (no GPU use in it)."""

    def __init__(self):
        import multiprocessing as mp
        self.pool = mp.get_context("spawn").Pool(1)
        self.jobs = {}

    def submit(self, name, job):
        self.jobs[name] = self.pool.apply_async(_oracle_job, (job,))

    def get(self, name, timeout=900):
        return self.jobs[name].get(timeout)

    def close(self):
        self.pool.close()
        self.pool.join()


def _cols(w, fibers):
    off = w.offsets
    return np.concatenate([np.arange(off[f], off[f + 1]) for f in fibers])


def _parity_cols(gs, tg, so, to, t_end):
    """V_m and activation-time errors of GPU columns against the oracle's."""
    gs = np.asarray(gs, dtype=np.float64)
    tg = np.asarray(tg, dtype=np.float64)
    tg = np.where(tg <= t_end, tg, np.inf)
    both = np.isfinite(tg) & np.isfinite(to)
    return dict(vm_max_err_mV=float(np.max(np.abs(gs - so))) if gs.size else 0.0,
                tact_max_err_ms=float(np.max(np.abs(tg[both] - to[both]))) if both.any() else 0.0,
                tact_mismatch=int(np.sum(np.isfinite(tg) != np.isfinite(to))),
                activated=int(both.sum()))


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




def _sample_fibers(w, n, window_ms):
    """n fibers whose first onsets lie nearest to n evenly spaced times of
    the window (so their activity spans it)."""
    onsets = np.array([st["step_on"] for st in w.stims]) * w.dt_split
    chosen = []
    for j in range(n):
        t = (j + 0.25) * window_ms / n
        order = np.argsort(np.abs(onsets - t), kind="stable")
        f = next(int(x) for x in order if int(x) not in chosen)
        chosen.append(f)
    return sorted(chosen)


def _run_timed(s, w, smp, steps, warmup, init, attach, label, step_split=STEP_SPLIT_STEPS):
    """Warm-up steps from the initial state, then the initial state again and
    `steps` timed bench steps of `step_split` split steps with V_m samples,
    under kernel timing; returns (seconds, per-step seconds)."""
    import torch
    per = step_split // w.sample_every

    def one(i, buf):
        s.run(i * step_split, step_split, w.sample_every, buf[i * per:(i + 1) * per])

    init()
    attach()
    for i in range(warmup):
        one(i, smp)
        torch.cuda.synchronize()
        _log(f"{label}: warm-up step {i + 1}/{warmup} done")
    init()
    attach()
    s.set_kernel_timing(True)
    s.sync()
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for i in range(steps):
        t1 = time.perf_counter()
        one(i, smp)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        if (i + 1) % 5 == 0 or i + 1 == steps:
            _log(f"{label}: step {i + 1}/{steps} done ({times[-1]:.3f} s)")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s.sync()
    return elapsed, times


def _ktimes(s):
    from paper_2107_07104_amd import fib as F
    out = {}
    for name, cls in (("fused", F.FIB_KT_FUSED), ("reaction", F.FIB_KT_REACTION),
                      ("diffusion", F.FIB_KT_DIFFUSION), ("surrogate", F.FIB_KT_SURROGATE),
                      ("fallback", F.FIB_KT_FALLBACK)):
        ms, n = s.kernel_time(cls)
        if n:
            out[name] = dict(ms_total=ms, launches=n, ms_per_launch=ms / n)
    return out


def headline(args, bg, ceil):
    """The large ST57 bundle: surrogate, plain and Euler-predictor paths
    (module docstring)."""
    import torch

    from oracle import oracle as O
    from paper_2107_07104_amd import fib as F
    from paper_2107_07104_amd import inputs as I
    from paper_2107_07104_amd import surrogate as SU

    K, W = args.steps, args.warmup
    n_steps = K * STEP_SPLIT_STEPS
    w = I.st57_bundle(n_fibers=10000, n_nodes=2000, t_end=HEADLINE_T_END_MS, onset_max=10.0,
                      period_ms=10.0, realization=2, host_noise=False).with_steps(n_steps)
    window = n_steps * w.dt_split
    rel = I.device_rel_noise(w)
    fibers = _sample_fibers(w, args.oracle_fibers, window)
    cols = _cols(w, fibers)
    ci = torch.as_tensor(cols, device="cuda")
    sub = w.subset(fibers)
    if not args.no_cpu_baseline:
        relc = rel[:, ci].cpu().numpy().astype(np.float64)
        y0 = O.rest_state(I.MODEL_ST57)[:, None] * (1.0 + relc)
        bg.submit("headline", dict(
            threads=len(fibers), one_thread_steps=500,
            cfg=dict(model=I.MODEL_ST57, Cm=w.Cm, Am=w.Am, sigma=w.sigma, h=w.h, dt_0D=w.dt_0D,
                     dt_1D=w.dt_1D, dt_split=w.dt_split, v_th=w.v_th),
            n_nodes=sub.n_nodes, y0=y0, stims=sub.stims, n_steps=n_steps,
            sample_every=w.sample_every))
        _log(f"oracle on fibers {fibers} started in the background")

    # training data: plain runs of another realization of the 400 x 1481
    # bundle over the same window as the headline run, so that the network
    # sees every time since a fiber's activation that the headline reaches
    # (trained on the first 5 ms only, it rejected 5e-3 of the node-steps,
    # rising to 2.5e-2 in the window's last quarter millisecond)
    wt = I.st57_bundle(n_fibers=400, n_nodes=1481, t_end=HEADLINE_T_END_MS)
    snap_ms = [0.0, 0.25] + [k + 0.5 for k in range(int(HEADLINE_T_END_MS))]
    snaps = [int(round(t / wt.dt_split)) for t in snap_ms]
    t0 = time.perf_counter()
    sur = SU.train_surrogate(I.MODEL_ST57, wt, snaps, steps=args.train_steps,
                             log=lambda m: _log("st57 surrogate:" + m))
    train_s = time.perf_counter() - t0

    rows = n_steps // w.sample_every
    runs, res = {}, {}
    paths = [("surrogate", W), ("plain", min(W, 1))]
    if not args.no_predictor:
        paths.append(("predictor", min(W, 1)))
    for path, warm in paths:
        s = SU._solver(w, schedule=F.FIB_SCHED_SPLIT)
        s.set_stimulus(w.stims)
        net = sur.network() if path == "surrogate" else None

        def attach(s=s, path=path, net=net):
            if path == "surrogate":
                s.set_surrogate(net, sur.scales, args.tol)
            elif path == "predictor":
                s.set_predictor(F.FIB_PRED_EULER, sur.scales["res_scale"], args.tol)

        smp = torch.empty((rows, w.n_total), device="cuda")
        secs, times = _run_timed(s, w, smp, K, warm, lambda s=s: s.init_state(rel_noise=rel),
                                 attach, f"st57 {path}")
        kt = _ktimes(s)
        r = dict(value=w.node_steps() / secs, seconds=secs, ms_per_step=secs / K * 1e3,
                 step_seconds_min=min(times), step_seconds_max=max(times), kernels=kt)
        if path != "plain":
            tot, nst = s.fallbacks()
            r["fallback_share"] = tot / max(1, nst * w.n_total)
            r["surrogate_steps"] = nst
        ta = s.tact()
        runs[path] = (smp, ta, smp.index_select(1, ci).cpu().numpy(), ta[cols])
        res[path] = r
        if net is not None:
            net.close()
        s.close()
        _log(f"st57 {path}: {r['value']:.3e} node-steps/s"
             + (f", rejected share {r['fallback_share']:.2e}" if "fallback_share" in r else ""))
        if path == "plain":
            sp, tp = runs["plain"][:2]
            ss, ts = runs["surrogate"][:2]
            res["surrogate"]["vs_plain"] = _compare(sp, tp, ss, ts, w.dt_split, window)
            runs["surrogate"] = (None, None) + runs["surrogate"][2:]
            del ss
            torch.cuda.empty_cache()
        if path == "predictor":
            sp, tp = runs["plain"][:2]
            res["predictor"]["vs_plain"] = _compare(sp, tp, smp, ta, w.dt_split, window)
            runs["predictor"] = (None, None) + runs["predictor"][2:]
        del smp
    runs["plain"] = (None, None) + runs["plain"][2:]
    del rel
    torch.cuda.empty_cache()

    # rooflines from the kernel times of the timed region
    ks = res["surrogate"]["kernels"]["surrogate"]["ms_per_launch"] * 1e-3
    achieved = SUR_ST57_BYTES_PER_NODE * w.n_total / ks
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": achieved / HBM_PEAK,
                "traffic": measured_traffic(SUR_TRAFFIC_FILE, SUR_SOURCES),
                "kernel": "k_surrogate<ST57>", "ms_per_launch": ks * 1e3,
                "launches": res["surrogate"]["kernels"]["surrogate"]["launches"],
                "bytes_per_node": SUR_ST57_BYTES_PER_NODE, "nodes_per_launch": int(w.n_total),
                "mfma_tflops": SUR_ST57_FLOP_PER_NODE * w.n_total / ks / 1e12,
                "mfma_frac": SUR_ST57_FLOP_PER_NODE * w.n_total / ks / MFMA_BF16_PEAK,
                "mfma_flop_per_node": SUR_ST57_FLOP_PER_NODE,
                "mfma_flop_per_node_padded": SUR_ST57_FLOP_PER_NODE_PADDED}
    kr = res["plain"]["kernels"]["reaction"]
    slots = ST57_REACT_OPS * w.n_total * n_steps / (kr["ms_total"] * 1e-3)
    roofline_plain = {"bound": "alu", "achieved": slots / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                      "unit": "T FP32 lane-ops/s (transcendental = 4)", "frac": slots / VALU_PEAK_OPS,
                      "kernel": "k_react_stream<ST57>",
                      "ms_per_launch": kr["ms_per_launch"], "launches": kr["launches"],
                      "ops_per_node_step": ST57_REACT_OPS,
                      "rhs_ops": ST57_RHS_OPS,
                      "whole_step_ops_per_node_step": ST57_OPS_PER_NODE_STEP,
                      "whole_step_frac": ST57_OPS_PER_NODE_STEP * res["plain"]["value"] /
                      VALU_PEAK_OPS}
    if "predictor" in res:
        kp = res["predictor"]["kernels"]["surrogate"]["ms_per_launch"] * 1e-3
        res["predictor"]["roofline"] = {
            "bound": "hbm", "achieved": SUR_ST57_BYTES_PER_NODE * w.n_total / kp / 1e9,
            "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": SUR_ST57_BYTES_PER_NODE * w.n_total / kp / HBM_PEAK,
            "kernel": "k_midpoint<ST57, Euler>", "ms_per_launch": kp * 1e3}

    cpu, parity = None, {}
    if not args.no_cpu_baseline:
        _log("waiting for the background oracle")
        o = bg.get("headline")
        so, to = o["samples"], o["tact"]
        for path in res:
            parity[path] = _parity_cols(runs[path][2], runs[path][3], so, to, window)
            parity[path].update(fibers=fibers, nodes=int(len(cols)), split_steps=n_steps)
        model, _ = host_cpu()
        node_steps = int(len(cols)) * n_steps
        one = o.get("one_thread")
        cpu = {"value": node_steps / o["seconds"], "unit": "node-steps/s",
               "cores": len(fibers), "kind": "oracle",
               "sample": f"{len(fibers)} fibers of the same bundle ({len(cols)} nodes) with "
                         f"onsets spread over the window, all {n_steps} split steps, FP64, "
                         f"OpenMP over fibers (one thread each), in a background process "
                         f"while the GPU ran",
               "seconds": o["seconds"], "cpu_model": model,
               "one_thread_value": one["node_steps"] / one["seconds"] if one else None,
               "one_thread_sample": "1 fiber (2000 nodes) x 500 split steps" if one else None}
        for path in res:
            res[path]["vs_oracle"] = parity[path]
        _log(f"oracle: {cpu['value']:.3e} node-steps/s on {len(fibers)} threads "
             f"({cpu['one_thread_value']:.3e} at one); parity {parity}")

    ok = lambda p: (p is not None and p["vm_max_err_mV"] <= 0.5 and
                    p["tact_max_err_ms"] <= w.dt_split and p["tact_mismatch"] == 0)
    sur_ok = ok(parity.get("surrogate")) if parity else None
    path = "surrogate" if (sur_ok or sur_ok is None) else "plain"
    out = dict(value=res[path]["value"], path=path, surrogate_within_budget=sur_ok,
               workload=w, fibers=fibers, roofline=roofline, roofline_plain=roofline_plain,
               cpu_baseline=cpu, paths=res, train=dict(
                   pairs=sur.info["pairs"], adam_steps=sur.info["steps"],
                   final_loss=sur.info["losses"][-1][1], seconds=train_s,
                   workload=f"st57 400 x 1481 bundle (realization 0), {HEADLINE_T_END_MS:g} ms, "
                            f"snapshots at {snap_ms} ms",
                   network="57-128-128-57 ReLU, BF16 MFMA"),
               surrogate_over_plain=res["surrogate"]["value"] / res["plain"]["value"])
    if "predictor" in res:
        out["surrogate_over_predictor"] = res["surrogate"]["value"] / res["predictor"]["value"]
    return out


def hh_batched(args):
    """The batched plain Hodgkin-Huxley workload in the fused kernel, with
    its VALU roofline and the FP64 oracle on a bounded subset of its fibers
    (module docstring)."""
    import torch

    from paper_2107_07104_amd import fib as F
    from paper_2107_07104_amd import inputs as I

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
        F.fib_init_state(s.ctx, vm.data_ptr(), 0)
        tuned = s.autotune(trial_steps=200, max_candidates=8)
    plan = s.plan()
    reps, warm = 5, 1
    for i in range(warm):
        F.fib_init_state(s.ctx, vm.data_ptr(), 0)
        s.run(0, w.n_steps, w.sample_every, samples)
        torch.cuda.synchronize()
    s.set_kernel_timing(True)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(reps):
        F.fib_init_state(s.ctx, vm.data_ptr(), 0)
        s.run(0, w.n_steps, w.sample_every, samples)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s.sync()
    kt = _ktimes(s)
    kernel_ms = kt["fused"]["ms_per_launch"]
    value = w.node_steps() * reps / elapsed
    achieved = w.node_steps() * OPS_PER_NODE_STEP / (kernel_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                "unit": "T FP32 lane-ops/s (transcendental = 4)", "frac": achieved / VALU_PEAK_OPS,
                "traffic": measured_traffic(), "kernel": "k_run_hh",
                "kernel_ms_per_launch": kernel_ms, "launches": kt["fused"]["launches"],
                "ops_per_node_step": OPS_PER_NODE_STEP}
    _log(f"hh batched: {value:.3e} node-steps/s, fused kernel {kernel_ms:.2f} ms, frac "
         f"{roofline['frac']:.3f}")
    cpu = parity = None
    if not args.no_cpu_baseline:
        model, threads = host_cpu()
        fibers = min(args.cpu_fibers or 2 * threads, len(w.n_nodes))
        gs = samples.cpu().numpy().astype(np.float64)
        rate, parity = cpu_baseline(w, gs, s.tact(), fibers)
        cpu = {"value": rate, "unit": "node-steps/s", "cores": threads, "kind": "oracle",
               "cpu_model": model,
               "sample": f"first {parity['fibers']} fibers ({parity['nodes']} nodes) of the "
                         f"same workload, all {w.n_steps} split steps, FP64, OpenMP over fibers"}
    s.close()
    return dict(workload="hh_batched_1369_fibers_1000-1500_nodes_20ms",
                fibers=int(len(w.n_nodes)), nodes=int(w.n_total), split_steps=int(w.n_steps),
                dt_split_ms=w.dt_split, schedule="fused", plan=plan, default_plan=default_plan,
                autotune=tuned, value=value, runs=reps, seconds=elapsed, roofline=roofline,
                cpu_baseline=cpu, parity_vs_oracle=parity)


def st57_bundle(args, bg):
    """400 x 1481 ST57 nodes with the 1 % perturbation, 5 ms, plain split
    schedule: throughput, the reaction kernel's VALU roofline, and the FP64
    oracle on two fibers (background); then the same bundle with the
    thesis's exp* and log* in the model (its speed, its oracle parity, and
    how far it lies from the exact model)."""
    from dataclasses import replace

    import torch

    from oracle import oracle as O
    from paper_2107_07104_amd import fib as F
    from paper_2107_07104_amd import inputs as I
    from paper_2107_07104_amd import surrogate as SU

    w0 = I.st57_bundle(n_fibers=400, n_nodes=1481, t_end=5.0)
    fibers = [0, 1]
    cols = _cols(w0, fibers)
    ci = torch.as_tensor(cols, device="cuda")
    rel = w0.rel_noise.astype(np.float32)
    relt = torch.as_tensor(rel, device="cuda")
    rows = w0.n_steps // w0.sample_every
    out, keep = {}, {}
    for key, model in (("exact", I.MODEL_ST57), ("exp_log_star", O.MODEL_ST57_APX)):
        w = replace(w0, model=model)
        if not args.no_cpu_baseline:
            sub = w.subset(fibers)
            y0 = O.rest_state(model)[:, None] * (1.0 + rel[:, cols].astype(np.float64))
            bg.submit(f"st57_bundle_{key}", dict(
                threads=2, cfg=dict(model=model, Cm=w.Cm, Am=w.Am, sigma=w.sigma, h=w.h,
                                    dt_0D=w.dt_0D, dt_1D=w.dt_1D, dt_split=w.dt_split,
                                    v_th=w.v_th),
                n_nodes=sub.n_nodes, y0=y0, stims=sub.stims, n_steps=w.n_steps,
                sample_every=w.sample_every))
        s = SU._solver(w, schedule=F.FIB_SCHED_SPLIT)
        s.set_stimulus(w.stims)
        smp = torch.empty((rows, w.n_total), device="cuda")
        secs, _ = _run_timed(s, w, smp, 1, 1, lambda s=s: s.init_state(rel_noise=relt),
                             lambda: None, f"st57 bundle {key}", step_split=w.n_steps)
        kt = _ktimes(s)
        r = dict(value=w.node_steps() / secs, seconds=secs, kernels=kt)
        if key == "exact":
            kr = kt["reaction"]
            ops = ST57_REACT_OPS * w.n_total * w.n_steps / (kr["ms_total"] * 1e-3)
            r["roofline"] = {"bound": "alu", "achieved": ops / 1e12,
                             "peak": VALU_PEAK_OPS / 1e12,
                             "unit": "T FP32 lane-ops/s (transcendental = 4)",
                             "frac": ops / VALU_PEAK_OPS, "kernel": "k_react_stream<ST57>",
                             "ops_per_node_step": ST57_REACT_OPS,
                             "whole_step_frac": ST57_OPS_PER_NODE_STEP * r["value"] /
                             VALU_PEAK_OPS}
        keep[key] = (smp, s.tact(), smp.index_select(1, ci).cpu().numpy())
        s.close()
        out[key] = r
        _log(f"st57 bundle {key}: {r['value']:.3e} node-steps/s")
    (sa, ta, _), (sb, tb, _) = keep["exact"], keep["exp_log_star"]
    out["exp_log_star"]["vs_exact"] = _compare(sa, ta, sb, tb, w0.dt_split,
                                               w0.n_steps * w0.dt_split)
    out["exp_log_star"]["over_exact"] = out["exp_log_star"]["value"] / out["exact"]["value"]
    if not args.no_cpu_baseline:
        for key in keep:
            o = bg.get(f"st57_bundle_{key}")
            out[key]["vs_oracle"] = _parity_cols(keep[key][2], keep[key][1][cols], o["samples"],
                                                 o["tact"], w0.n_steps * w0.dt_split)
            out[key]["vs_oracle"].update(fibers=fibers, oracle_seconds=o["seconds"])
    del keep, sa, sb
    torch.cuda.empty_cache()
    ex = out["exact"]
    return dict(workload="st57_400x1481_5ms, 1 % perturbation", fibers=400,
                nodes=int(w0.n_total), split_steps=int(w0.n_steps), dt_split_ms=w0.dt_split,
                value=ex["value"], seconds=ex["seconds"], kernels=ex["kernels"],
                roofline=ex["roofline"], vs_oracle=ex.get("vs_oracle"),
                exp_log_star=out["exp_log_star"])


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
    sur = SU.train_surrogate(I.MODEL_HH, wt, snaps, steps=args.train_steps,
                             log=lambda m: _log("hh surrogate:" + m))
    train_s = time.perf_counter() - t0
    w = replace(I.batched_hh(n_min=1481, n_max=1481, dt=5e-3, realization=1), dt_0D=1e-3,
                name="hh_surrogate_eval_1369x1481")
    vm = w.vm_noise.astype(np.float32)
    res = {}
    runs = {}
    for path, sched in (("plain_fused", F.FIB_SCHED_FUSED), ("plain_split", F.FIB_SCHED_SPLIT),
                        ("surrogate", F.FIB_SCHED_SPLIT), ("predictor", F.FIB_SCHED_SPLIT)):
        s = SU._solver(w, schedule=sched)
        s.set_stimulus(w.stims)
        net = None
        if path == "surrogate":
            net = sur.network()

        def attach(s=s, path=path, net=net):
            if path == "surrogate":
                s.set_surrogate(net, sur.scales, args.tol)
            elif path == "predictor":
                s.set_predictor(F.FIB_PRED_EULER, sur.scales["res_scale"], args.tol)

        attach()
        _timed_run(s, w.with_steps(40), lambda: s.init_state(vm_noise=vm), w.sample_every)
        attach()
        secs, smp, ta = _timed_run(s, w, lambda: s.init_state(vm_noise=vm), w.sample_every)
        runs[path] = (smp, ta)
        res[path] = dict(value=w.node_steps() / secs, seconds=secs)
        if path in ("surrogate", "predictor"):
            tot, nst = s.fallbacks()
            res[path]["fallback_share"] = tot / max(1, nst * w.n_total)
        if net is not None:
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
    spr, tpr = runs["predictor"]
    res["predictor"]["vs_plain_split"] = _compare(sp, tp, spr, tpr, w.dt_split,
                                                  w.n_steps * w.dt_split)
    res["predictor"]["vs_oracle"] = _oracle_parity(w, fibers, y0, spr, tpr, w.n_steps)
    best_plain = max(res["plain_fused"]["value"], res["plain_split"]["value"])
    relu = None
    if not args.no_sur_relu:
        # the same network with ReLU: one packed integer max per two
        # activations instead of an exponential and a reciprocal each
        t0 = time.perf_counter()
        sr = SU.train_surrogate(I.MODEL_HH, wt, snaps, steps=args.train_steps, act="relu",
                                log=lambda m: _log("hh relu surrogate:" + m))
        tr_s = time.perf_counter() - t0
        s = SU._solver(w, schedule=F.FIB_SCHED_SPLIT)
        s.set_stimulus(w.stims)
        net = sr.network()
        s.set_surrogate(net, sr.scales, args.tol)
        _timed_run(s, w.with_steps(40), lambda: s.init_state(vm_noise=vm), w.sample_every)
        s.set_surrogate(net, sr.scales, args.tol)
        secs, sr_s, sr_t = _timed_run(s, w, lambda: s.init_state(vm_noise=vm), w.sample_every)
        tot, nst = s.fallbacks()
        fb = tot / max(1, nst * w.n_total)
        net.close()
        s.close()
        relu = dict(network="5-64-64-64-4 ReLU, BF16 MFMA", value=w.node_steps() / secs,
                    seconds=secs, fallback_share=fb,
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
                network="5-64-64-64-4 SiLU, BF16 MFMA", tol=args.tol,
                train=dict(pairs=sur.info["pairs"], adam_steps=sur.info["steps"],
                           final_loss=sur.info["losses"][-1][1], seconds=train_s,
                           workload="realization 0 of the same bundle"),
                **res, surrogate_over_best_plain=res["surrogate"]["value"] / best_plain,
                surrogate_over_predictor=res["surrogate"]["value"] / res["predictor"]["value"],
                surrogate_vs_plain_split=_compare(sp, tp, ss, ts, w.dt_split, w.n_steps * w.dt_split),
                surrogate_vs_oracle=parity, relu_variant=relu)


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
    if "hh" in wanted:
        out["hh_as_specified"] = _adaptive_as_specified(args)
    return out


def _adaptive_as_specified(args):
    """Adaptive computation on the batched HH workload as specified, with its
    initial V_m noise: nodes freeze slightly off equilibrium, so the result
    is reported against the FP64 oracle's plain run with its budget flag."""
    import torch

    from paper_2107_07104_amd import fib as F
    from paper_2107_07104_amd import inputs as I
    from oracle import oracle as O
    w = I.batched_hh(t_end=args.t_end)
    vm = torch.as_tensor(w.vm_noise.astype(np.float32), device="cuda")
    res, runs = {}, {}
    for path, tol in (("plain_fused", 0.0), ("adaptive", args.adapt_tol)):
        s = F.Solver(w.n_nodes, schedule=F.FIB_SCHED_FUSED, dt_0D=w.dt_0D, dt_1D=w.dt_1D,
                     dt_split=w.dt_split, v_th=w.v_th)
        s.set_stimulus(w.stims)
        init = (lambda s=s: s.init_state(vm_noise=vm))
        init()
        s.autotune(trial_steps=200, max_candidates=8)
        if tol > 0.0:
            s.set_adaptive(tol)
        _timed_run(s, w.with_steps(50), init, w.sample_every)
        before = s.adaptive_solved() if tol > 0.0 else 0
        secs, smp, ta = _timed_run(s, w, init, w.sample_every)
        runs[path] = (smp, ta)
        res[path] = dict(value=w.node_steps() / secs, seconds=secs)
        if tol > 0.0:
            res[path].update(tol=tol, solved_share=(s.adaptive_solved() - before) / w.node_steps())
        s.close()
        _log(f"adaptive hh as specified {path}: {res[path]['value']:.3e} node-steps/s")
    fibers = [0, 1, 2, 3]
    off = w.offsets
    cols = np.concatenate([np.arange(off[f], off[f + 1]) for f in fibers])
    y0 = np.tile(O.rest_state()[:, None], (1, len(cols)))
    y0[0] += w.vm_noise.astype(np.float32)[cols].astype(np.float64)
    sa, ta = runs["adaptive"]
    parity = (None if args.no_adapt_parity
              else _oracle_parity(w, fibers, y0, sa, ta, w.n_steps))
    within = (None if parity is None else
              bool(parity["vm_max_err_mV"] <= 0.5 and parity["tact_max_err_ms"] <= w.dt_split
                   and parity["tact_mismatch"] == 0))
    sp, tp = runs["plain_fused"]
    return dict(workload=f"{w.name}, V_m noise as specified", **res,
                adaptive_over_plain=res["adaptive"]["value"] / res["plain_fused"]["value"],
                adaptive_vs_plain=_compare(sp, tp, sa, ta, w.dt_split, w.n_steps * w.dt_split),
                adaptive_vs_oracle_plain=parity, within_budget=within)


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
    # the last phi_e against the oracle's FP64 solution from the same V_m
    # (conjugate gradients to 1e-13: the mesh is too large for its direct solve)
    phi_o, _ = E.solve(g, V3, sig["sigma_i"], sig["sigma_el"], sig["sigma_et"], method="cg")
    phi_err = float(np.max(np.abs(phi - phi_o)) / np.max(np.abs(phi_o)))
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
               last_phi_fp64_relative_residual=res,
               last_phi_vs_oracle=dict(max_abs_err_over_max_phi=phi_err,
                                       max_phi_mV=float(np.max(np.abs(phi_o))),
                                       oracle="FP64 CG to a relative residual of 1e-13"),
               mesh_nodes=int(g.n), roofline=roof)
    _log(f"emg: {out['value']:.3e} node-steps/s, {n_solves} solves, {tot_it / n_solves:.1f} "
         f"CG iterations each, EMG share {out['emg_share']:.2f}, residual {res:.1e}, "
         f"phi vs oracle {phi_err:.1e}")
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


def trace_gaps(path, max_gap_us=500.0):
    """Idle time between consecutive kernels in a rocprofv3 kernel trace
    (csv): per kernel and grid size, launches, mean duration and the mean
    idle gap before it; overall, kernel time and the idle gaps below
    max_gap_us (gaps above it are host-side pauses between runs, not launch
    overhead)."""
    import csv
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"]
            short = name.split("(")[0]
            short = short.split("void ")[-1]
            if r.get("Grid_Size_X"):
                # the same kernel on workloads of different sizes apart
                short += f" [grid {r['Grid_Size_X']}]"
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short))
    rows.sort()
    per = {}
    busy = idle = 0.0
    for i, (t0, t1, k) in enumerate(rows):
        d = per.setdefault(k, dict(launches=0, kernel_us=0.0, gap_us=0.0, gaps=0))
        d["launches"] += 1
        d["kernel_us"] += (t1 - t0) / 1e3
        busy += (t1 - t0) / 1e3
        if i:
            g = (t0 - rows[i - 1][1]) / 1e3
            if 0.0 < g <= max_gap_us:
                d["gap_us"] += g
                d["gaps"] += 1
                idle += g
    table = {k: dict(launches=v["launches"], mean_us=v["kernel_us"] / v["launches"],
                     mean_gap_before_us=v["gap_us"] / max(1, v["gaps"]),
                     gap_share_of_own_time=v["gap_us"] / max(v["kernel_us"], 1e-9))
             for k, v in sorted(per.items(), key=lambda kv: -kv[1]["kernel_us"])}
    return dict(kernels=table, kernel_us=busy, idle_gap_us=idle,
                idle_share=idle / max(busy + idle, 1e-9), max_gap_us=max_gap_us)


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--trace-gaps":
        print(json.dumps(trace_gaps(sys.argv[2]), indent=1))
        return
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the fibers are "
              "independent, so a multi-GPU run would shard whole fibers with no "
              "communication -- not measured here.", file=sys.stderr)
        sys.exit(2)

    # the oracle's background process starts before anything touches the GPU
    bg = Background() if not args.no_cpu_baseline else None
    import torch

    torch.cuda.set_device(0)
    sections = [x for x in args.sections.split(",") if x]
    try:
        ceil = measure_ceilings()
        if args.copy_calibration_mib > 0:
            n = args.copy_calibration_mib * (1 << 20) // 4
            src = torch.ones(n, device="cuda")
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
            _log(f"calibration copy of {args.copy_calibration_mib} MiB done")
        head = headline(args, bg, ceil)
        extra = {}
        if "hh_batched" in sections:
            extra["hh_batched"] = hh_batched(args)
        if "st57_bundle" in sections:
            extra["st57_bundle"] = st57_bundle(args, bg)
        if "surrogate_hh" in sections:
            extra["surrogate_hh"] = surrogate_hh(args)
        if "adaptive" in sections:
            extra["adaptive"] = adaptive_bench(args)
        if "emg" in sections:
            extra["emg"] = emg_bench(args)
            if "hh_batched" in extra:
                extra["emg"]["over_plain"] = extra["emg"]["value"] / extra["hh_batched"]["value"]
        if "exp_approx" in sections:
            extra["exp_approx"] = exp_approx_bench(args)
            if "hh_batched" in extra:
                extra["exp_approx"]["over_plain"] = (extra["exp_approx"]["value"] /
                                                     extra["hh_batched"]["value"])
    finally:
        if bg is not None:
            bg.close()

    w = head["workload"]
    res = head["paths"]
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "node-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res[head["path"]]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "st57_10000x2000_100Hz_10ms", "fibers": int(len(w.n_nodes)),
                   "nodes": int(w.n_total), "split_steps_per_step": STEP_SPLIT_STEPS,
                   "split_steps": int(w.n_steps), "dt_split_ms": w.dt_split,
                   "dt_0D_ms": w.dt_0D, "schedule": "split", "path": head["path"],
                   "tol": args.tol, "network": head["train"]["network"]},
        "roofline": head["roofline"],
        "roofline_plain": head["roofline_plain"],
        "cpu_baseline": head["cpu_baseline"],
        "plain": res["plain"],
        "surrogate": res["surrogate"],
        "predictor": res.get("predictor"),
        "surrogate_over_plain": head["surrogate_over_plain"],
        "surrogate_over_predictor": head.get("surrogate_over_predictor"),
        "surrogate_within_budget": head["surrogate_within_budget"],
        "train": head["train"],
        "oracle_fibers": head["fibers"],
        "ceilings": ceil,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
