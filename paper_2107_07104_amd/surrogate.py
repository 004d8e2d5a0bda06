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
    run of `w` (device tensor [len(snapshots) * n_total, S])."""
    import torch
    s = _solver(w)
    s.set_stimulus(w.stims)
    s.init_state(vm_noise=w.vm_noise.astype(np.float32),
                 rel_noise=None if w.rel_noise is None else w.rel_noise.astype(np.float32))
    out, done = [], 0
    for step in sorted(snapshot_steps):
        if step > done:
            s.run(done, step - done)
            done = step
        st, _ = s.state_tensor()
        out.append(st.t().contiguous().clone())
        log(f"  snapshot at step {step} ({step * w.dt_split:.2f} ms)")
    s.sync()
    s.close()
    return torch.cat(out, 0)


def reaction_targets(w: I.Workload, U, amp: float):
    """Increment of the plain reaction pair R(dt/2) R(dt/2) from every row of
    U (offsets) with stimulus `amp` on every node (amp = 0: off), computed
    by fib_step_reaction on a context of the workload's shape, one
    n_total-row chunk at a time."""
    import torch
    N, S = U.shape
    s = _solver(w)
    n = s.n_total
    if amp != 0.0:
        s.set_stimulus([dict(fiber=f, node=0, half_width=int(w.n_nodes[f]), step_on=0,
                             n_steps=1, period=0, amp=amp) for f in range(len(w.n_nodes))])
    s.init_state()
    st, _ = s.state_tensor()
    dU = torch.empty_like(U)
    for a in range(0, N, n):
        b = min(a + n, N)
        st.zero_()
        st[:, : b - a].copy_(U[a:b].t())
        s.step_reaction(0, 0.5 * w.dt_split)
        s.step_reaction(0, 0.5 * w.dt_split)
        torch.cuda.synchronize()
        dU[a:b] = st[:, : b - a].t() - U[a:b]
    s.sync()
    s.close()
    return dU


def fit_scales(U, dU, model: int):
    """Per-state normalisation of inputs and targets, and residual scales
    (the range of each state in the data)."""
    u = U.double()
    d = dU.double()
    in_shift = u.mean(0)
    in_std = u.std(0)
    out_shift = d.mean(0)
    out_std = d.std(0)
    rng = (u.max(0).values - u.min(0).values)
    floor_in = 1e-6 * u.abs().max(0).values + 1e-8
    scales = dict(
        in_shift=in_shift.float().cpu().numpy(),
        in_scale=(1.0 / torch_max(in_std, floor_in)).float().cpu().numpy(),
        out_shift=out_shift.float().cpu().numpy(),
        out_scale=torch_max(out_std, 1e-12 + 0 * out_std).float().cpu().numpy(),
        res_scale=torch_max(rng, 1e-9 + 0 * rng).float().cpu().numpy(),
    )
    return scales


def torch_max(a, b):
    import torch
    return torch.maximum(a, b)


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
    X_parts, T_parts, flags = [U], [dU0], [torch.zeros(U.shape[0], device=U.device)]
    if use_flag and flag_share > 0:
        g = torch.Generator(device="cpu").manual_seed(seed)
        k = max(1, int(flag_share * U.shape[0]))
        idx = torch.randperm(U.shape[0], generator=g)[:k].to(U.device)
        Uf = U[idx].contiguous()
        dUf = reaction_targets(w, Uf, amp)
        X_parts.append(Uf)
        T_parts.append(dUf)
        flags.append(torch.ones(k, device=U.device))
    Uall = torch.cat(X_parts, 0)
    dUall = torch.cat(T_parts, 0)
    fl = torch.cat(flags, 0)
    log(f"  {Uall.shape[0]} training pairs collected in {time.time() - t0:.1f} s")
    scales = fit_scales(U, dU0, model)
    scales["flag_scale"] = (1.0 / amp) if use_flag else 0.0
    ish = torch.as_tensor(scales["in_shift"], device=U.device)
    isc = torch.as_tensor(scales["in_scale"], device=U.device)
    osh = torch.as_tensor(scales["out_shift"], device=U.device)
    osc = torch.as_tensor(scales["out_scale"], device=U.device)
    X = (Uall - ish) * isc
    if use_flag:
        X = torch.cat([X, fl[:, None]], 1)
    T = (dUall - osh) / osc
    X = X.float().contiguous()
    T = T.float().contiguous()
    del Uall, dUall
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
