"""Training pipeline of the learned surrogate of the subcellular update.

The surrogate predicts the increment of every state over one split step dt,
i.e. the effect of the two reaction halves R(dt/2) R(dt/2) that meet
between consecutive diffusion steps (see fib_set_surrogate in
include/fib.h).  Everything numerical runs in libfib.so:

  1. states are collected from plain runs of a workload (fused or split
     schedule) at several times;
  2. the exact target for each state is the plain method's own update,
     two calls of fib_step_reaction over dt/2 with the stimulus off (and,
     for a share of the states, on everywhere);
  3. the network is trained on the GPU with fib_mlp_adam_step (BF16 matrix
     cores, FP32 masters) on normalized inputs and targets.

Torch only holds device buffers and shuffles sample indices.  The result is
a network plus the scalings fib_set_surrogate takes; save() / load() keep
them in a NumPy .npz file (no pickles).
"""
from __future__ import annotations

import argparse
import math
import os
import time
from dataclasses import dataclass

import numpy as np

from . import fib as F
from . import inputs as I

# Network of each model: layer widths and hidden activation.  The
# Hodgkin-Huxley network takes the four states and the stimulus flag, three
# hidden SiLU layers of 64; the ST57 network maps the 57 states through two
# hidden layers of 128 with ReLU, whose cost on the vector units is one
# packed integer max per two BF16 values (SiLU needs an exponential and a
# reciprocal per value, which at this width costs as much as the plain
# subcellular update the network replaces).
SHAPES = {I.MODEL_HH: [5, 64, 64, 64, 4], I.MODEL_ST57: [57, 128, 128, 57]}
ACTIVATION = {I.MODEL_HH: "silu", I.MODEL_ST57: "relu"}


@dataclass
class Surrogate:
    model: int
    sizes: list
    params: np.ndarray        # flat FP32 parameters
    scales: dict              # in_shift, in_scale, out_shift, out_scale, res_scale, flag_scale
    dt_split: float
    info: dict
    act: str = "silu"

    def network(self):
        net = F.Mlp(self.sizes, act=self.act)
        net.set_params(self.params)
        return net


def _solver(w: I.Workload, **kw) -> F.Solver:
    p = dict(model=w.model, Cm=w.Cm, Am=w.Am, sigma=w.sigma, h=w.h, dt_0D=w.dt_0D,
             dt_1D=w.dt_1D, dt_split=w.dt_split, v_th=w.v_th)
    p.update(kw)
    return F.Solver(w.n_nodes, **p)


def collect_states(w: I.Workload, snapshot_steps, log=print):
    """Offsets u = y - rest of every node at the given split steps of a plain
    run of `w` (device tensor [len(snapshots) * n_total, S], node-major, as
    fib_state_rows writes it)."""
    import torch
    s = _solver(w)
    s.set_stimulus(w.stims)
    s.init_state(vm_noise=w.vm_noise.astype(np.float32),
                 rel_noise=None if w.rel_noise is None else w.rel_noise.astype(np.float32))
    snaps = sorted(snapshot_steps)
    U = torch.empty((len(snaps) * s.n_total, s.S), dtype=torch.float32, device="cuda")
    done = 0
    for j, step in enumerate(snaps):
        if step > done:
            s.run(done, step - done)
            done = step
        F.fib_state_rows(s.ctx, U[j * s.n_total:].data_ptr())
        log(f"  snapshot at step {step} ({step * w.dt_split:.2f} ms)")
    s.sync()
    s.close()
    return U


def reaction_targets(w: I.Workload, U, amp: float):
    """Increment of the plain reaction pair R(dt/2) R(dt/2) from every row of
    U (offsets) with stimulus `amp` on every node (amp = 0: off), computed
    by fib_reaction_increments on a context of the workload's shape."""
    import torch
    s = _solver(w)
    if amp != 0.0:
        s.set_stimulus([dict(fiber=f, node=0, half_width=int(w.n_nodes[f]), step_on=0,
                             n_steps=1, period=0, amp=amp) for f in range(len(w.n_nodes))])
    U = U.contiguous()
    dU = torch.empty_like(U)
    F.fib_reaction_increments(s.ctx, U.data_ptr(), U.shape[0], 0, dU.data_ptr())
    s.sync()
    s.close()
    return dU


def fit_scales(U, dU, model: int):
    """Per-state normalisation of inputs and targets, and residual scales
    (the range of each state in the data), from the column statistics
    fib_column_stats computes on the device (FP64 sums, sample standard
    deviation)."""
    rows, S = U.shape
    u_mean, u_std, u_min, u_max = F.fib_column_stats(U.data_ptr(), rows, S)
    d_mean, d_std, _, _ = F.fib_column_stats(dU.data_ptr(), rows, S)
    u_min, u_max = u_min.astype(np.float64), u_max.astype(np.float64)
    floor_in = 1e-6 * np.maximum(np.abs(u_min), np.abs(u_max)) + 1e-8
    return dict(
        in_shift=u_mean.astype(np.float32),
        in_scale=(1.0 / np.maximum(u_std, floor_in)).astype(np.float32),
        out_shift=d_mean.astype(np.float32),
        out_scale=np.maximum(d_std, 1e-12).astype(np.float32),
        res_scale=np.maximum(u_max - u_min, 1e-9).astype(np.float32),
    )


def normalized_pairs(parts, scales, use_flag: bool):
    """Network inputs X = (u - in_shift) in_scale (and the stimulus flag of
    each part as the last input) and targets T = (du - out_shift) /
    out_scale, written by fib_normalize_rows; `parts` is a list of
    (U, dU, flag) with device tensors of shape [rows, S]."""
    import torch
    S = parts[0][0].shape[1]
    n = sum(p[0].shape[0] for p in parts)
    ldx = S + 1 if use_flag else S
    X = torch.empty((n, ldx), dtype=torch.float32, device="cuda")
    T = torch.empty((n, S), dtype=torch.float32, device="cuda")
    inv_out = (1.0 / scales["out_scale"].astype(np.float64)).astype(np.float32)
    r = 0
    for U, dU, flag in parts:
        m = U.shape[0]
        F.fib_normalize_rows(U.data_ptr(), m, S, scales["in_shift"], scales["in_scale"],
                             float(flag), X[r:].data_ptr(), ldx)
        F.fib_normalize_rows(dU.data_ptr(), m, S, scales["out_shift"], inv_out, 0.0,
                             T[r:].data_ptr(), S)
        r += m
    return X, T


def _init_params(sizes, seed):
    """Uniform initialisation scaled by 1/sqrt(fan_in) (seeded NumPy draw)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    flat = []
    for i in range(len(sizes) - 1):
        bound = math.sqrt(6.0 / sizes[i]) * 0.5
        flat.append(rng.uniform(-bound, bound, sizes[i + 1] * sizes[i]))
        flat.append(np.zeros(sizes[i + 1]))
    return np.concatenate(flat).astype(np.float32)


def train_surrogate(model: int, w: I.Workload, snapshot_steps, steps: int = 20000,
                    batch: int = 8192, lr: float = 2e-3, lr_end: float = 2e-5,
                    flag_share: float = 0.1, amp: float = I.AMP_SUPRA, seed: int = 7,
                    act=None, log=print) -> Surrogate:
    """Collects data from `w`, trains the network of SHAPES[model] with the
    library's Adam kernels and returns it with its scalings."""
    import torch
    sizes = SHAPES[model]
    act = ACTIVATION[model] if act is None else act
    t0 = time.time()
    U = collect_states(w, snapshot_steps, log=log)
    S = U.shape[1]
    use_flag = sizes[0] == S + 1
    dU0 = reaction_targets(w, U, 0.0)
    parts = [(U, dU0, 0.0)]
    if use_flag and flag_share > 0:
        g = torch.Generator(device="cpu").manual_seed(seed)
        k = max(1, int(flag_share * U.shape[0]))
        idx = torch.randperm(U.shape[0], generator=g)[:k].to(U.device)
        Uf = U[idx].contiguous()
        parts.append((Uf, reaction_targets(w, Uf, amp), 1.0))
    log(f"  {sum(p[0].shape[0] for p in parts)} training pairs collected in "
        f"{time.time() - t0:.1f} s")
    scales = fit_scales(U, dU0, model)
    scales["flag_scale"] = (1.0 / amp) if use_flag else 0.0
    X, T = normalized_pairs(parts, scales, use_flag)
    del parts
    net = F.Mlp(sizes, act=act)
    net.set_params(_init_params(sizes, seed))
    g = torch.Generator(device=U.device.type).manual_seed(seed)
    n = X.shape[0]
    loss = torch.empty(1, device=U.device)
    losses = []
    t1 = time.time()
    perm = torch.randperm(n, device=U.device, generator=g)
    pos = 0
    for it in range(steps):
        if pos + batch > n:
            perm = torch.randperm(n, device=U.device, generator=g)
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        xb = X[idx].contiguous()
        tb = T[idx].contiguous()
        frac = it / max(steps - 1, 1)
        lr_t = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * frac))
        net.adam_step(xb, tb, lr_t, loss)
        if it % max(steps // 10, 1) == 0 or it == steps - 1:
            losses.append((it, float(loss.item())))
            log(f"  step {it}: loss {losses[-1][1]:.3e} (lr {lr_t:.1e})")
    log(f"  trained {steps} steps in {time.time() - t1:.1f} s")
    params = net.get_params()
    net.close()
    info = dict(pairs=int(n), steps=steps, batch=batch, losses=losses,
                train_seconds=time.time() - t1, workload=w.name,
                snapshots=[int(s) for s in snapshot_steps])
    return Surrogate(model=model, sizes=sizes, params=params, scales=scales,
                     dt_split=w.dt_split, info=info, act=act)


def save(path: str, sur: Surrogate) -> None:
    np.savez(path, model=np.int32(sur.model), sizes=np.asarray(sur.sizes, dtype=np.int32),
             params=sur.params.astype(np.float32), dt_split=np.float64(sur.dt_split),
             flag_scale=np.float64(sur.scales["flag_scale"]),
             act=np.int32(F.ACTS[sur.act]),
             **{k: np.asarray(v, dtype=np.float32) for k, v in sur.scales.items()
                if k != "flag_scale"})


def load(path: str) -> Surrogate:
    z = np.load(path, allow_pickle=False)
    scales = {k: z[k] for k in ("in_shift", "in_scale", "out_shift", "out_scale", "res_scale")}
    scales["flag_scale"] = float(z["flag_scale"])
    act = {v: k for k, v in F.ACTS.items()}[int(z["act"])] if "act" in z else "silu"
    return Surrogate(model=int(z["model"]), sizes=[int(v) for v in z["sizes"]],
                     params=z["params"], scales=scales, dt_split=float(z["dt_split"]), info={},
                     act=act)


def hh_training_workload() -> I.Workload:
    """Hodgkin-Huxley bundle of the surrogate workload: 1369 fibers x 1481
    nodes, dt_split = 5e-3 ms (dt_0D = 1e-3 ms: three Heun substeps per
    half), seeded onsets in [0, 5] ms, 20 ms."""
    w = I.batched_hh(n_min=1481, n_max=1481, dt=5e-3)
    from dataclasses import replace
    return replace(w, name="hh_surrogate_1369x1481", dt_0D=1e-3)


def main():
    ap = argparse.ArgumentParser(description="train a surrogate with libfib.so")
    ap.add_argument("--model", choices=["hh", "st57"], default="hh")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.model == "hh":
        w = hh_training_workload()
        snaps = [int(round(t / w.dt_split)) for t in (1.0, 3.0, 5.0, 7.0, 10.0)]
        sur = train_surrogate(I.MODEL_HH, w, snaps, steps=args.steps)
    else:
        w = I.st57_bundle(n_fibers=400, n_nodes=1481, t_end=5.0)
        snaps = [int(round(t / w.dt_split)) for t in (0.5, 1.5, 2.5, 3.5, 4.5)]
        sur = train_surrogate(I.MODEL_ST57, w, snaps, steps=args.steps)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    save(args.out, sur)
    print(f"saved {args.out}: {sur.info['pairs']} pairs, final loss {sur.info['losses'][-1]}")


if __name__ == "__main__":
    main()
