"""Shared helpers of the GPU parity tests: run a workload through the library
(HIP path) and through the oracle, on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

from oracle import oracle as O
from paper_2107_07104_amd import fib as F
from paper_2107_07104_amd import inputs as I


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_cfg(w: I.Workload, scheme=O.SCHEME_STRANG, theta=0.5) -> O.Config:
    return O.Config(model=w.model, scheme=scheme, Cm=w.Cm, Am=w.Am, sigma=w.sigma, h=w.h,
                    dt_0D=w.dt_0D, dt_1D=w.dt_1D, dt_split=w.dt_split, v_th=w.v_th,
                    theta=theta)


def oracle_init(w: I.Workload) -> np.ndarray:
    """Initial state per the input recipe: rest state, times (1 + relative
    noise) per state, plus the V_m noise."""
    rest = O.rest_state(w.model)
    y = np.tile(rest[:, None], (1, w.n_total))
    if w.rel_noise is not None:
        y = y * (1.0 + w.rel_noise.astype(np.float32).astype(np.float64))
    y[0] += w.vm_noise.astype(np.float32).astype(np.float64)
    return y


def oracle_run(w: I.Workload, n_steps=None, sample_every=None, y0=None, cfg=None):
    n_steps = w.n_steps if n_steps is None else n_steps
    se = w.sample_every if sample_every is None else sample_every
    y0 = oracle_init(w) if y0 is None else y0
    cfg = oracle_cfg(w) if cfg is None else cfg
    return O.run(cfg, w.n_nodes, y0, w.stims, n_steps, sample_every=se)


def gpu_solver(w: I.Workload, **kw) -> F.Solver:
    p = dict(model=w.model, Cm=w.Cm, Am=w.Am, sigma=w.sigma, h=w.h, dt_0D=w.dt_0D,
             dt_1D=w.dt_1D, dt_split=w.dt_split, v_th=w.v_th)
    p.update(kw)
    s = F.Solver(w.n_nodes, **p)
    s.set_stimulus(w.stims)
    s.init_state(vm_noise=w.vm_noise.astype(np.float32),
                 rel_noise=None if w.rel_noise is None else w.rel_noise.astype(np.float32))
    return s


def gpu_run(w: I.Workload, n_steps=None, sample_every=None, solver=None, **kw):
    import torch
    n_steps = w.n_steps if n_steps is None else n_steps
    se = w.sample_every if sample_every is None else sample_every
    s = solver or gpu_solver(w, **kw)
    rows = n_steps // se if se else 0
    samples = torch.full((max(rows, 1), w.n_total), float("nan"), device="cuda")
    s.run(0, n_steps, se, samples if rows else None)
    s.sync()
    y = s.get_state()
    ta = s.tact()
    out = samples[:rows].cpu().numpy().astype(np.float64) if rows else None
    return y, out, ta.astype(np.float64), s


def compare_runs(w, gpu, ora, vm_tol=0.5, tact_tol_steps=1.0):
    """Max |V_gpu - V_oracle| over all samples and the final state, and the
    activation-time agreement (finite in both or in neither; difference
    within tact_tol_steps split steps)."""
    yg, sg, tg, _ = gpu
    yo, so, to = ora
    err_final = float(np.max(np.abs(yg[0] - yo[0]))) if w.n_total else 0.0
    err_samples = float(np.max(np.abs(sg - so))) if sg is not None and sg.size else 0.0
    fin_g, fin_o = np.isfinite(tg), np.isfinite(to)
    both = fin_g & fin_o
    only = int(np.sum(fin_g != fin_o))
    dta = float(np.max(np.abs(tg[both] - to[both]))) if both.any() else 0.0
    return dict(vm_err=max(err_final, err_samples), tact_err=dta, tact_mismatch=only,
                activated=int(both.sum()))
