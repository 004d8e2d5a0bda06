"""Seeded synthetic workloads for the fiber monodomain solve.

This module only draws random numbers and lays out the inputs: fiber
lengths, per-node voltage noise, per-state relative noise and the stimulus
table.  It holds none of the method's arithmetic, so that the GPU library
and the CPU oracle can both be fed from it.

The fibers are straight and uniform, at the thesis's resolution of 100
elements per cm (h = 0.01 cm) and with 1481-node fibers as in its biceps
meshes; 1369 = 37 x 37 fibers as in its single-motor-unit scenario.  The
stimulus is a current on the three nodes around a neuromuscular junction
placed in the central 10 % of the fiber (section "Specification of
Stimulation Times Using Callback Functions").

Random streams are NumPy PCG64 generators, one per quantity, so a subset of
fibers of a large workload is bit-identical to the same fibers drawn alone.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

MODEL_HH = 0
MODEL_ST57 = 1

# Stimulus current densities (uA/cm^2).  40 is the value of the thesis's
# example settings; on a fiber with h = 0.01 cm it stays below threshold, so
# the activation-time observable is exercised with a supra-threshold pulse of
# roughly twice the threshold of a 0.1 ms pulse on three nodes.
AMP_AS_WRITTEN = 40.0
AMP_SUPRA = 1200.0

SEED_VM_NOISE = 1
SEED_LENGTHS = 2
SEED_STIM_NODE = 3
SEED_STIM_TIME = 4
SEED_REL_NOISE = 5


@dataclass
class Workload:
    name: str
    model: int
    n_nodes: np.ndarray          # int32, nodes per fiber
    vm_noise: np.ndarray         # float64, additive noise on V_m per node (mV)
    rel_noise: Optional[np.ndarray]  # float64 [S, N] multiplicative noise, or None
    stims: List[dict]            # one dict per stimulus entry
    n_steps: int                 # split steps
    sample_every: int            # split steps between V_m samples
    Cm: float = 1.0
    Am: float = 500.0
    sigma: float = 3.828
    h: float = 0.01
    dt_0D: float = 1e-3
    dt_1D: float = 1e-3
    dt_split: float = 1e-3
    v_th: float = -20.0
    extra: dict = field(default_factory=dict)

    @property
    def n_total(self) -> int:
        return int(self.n_nodes.sum())

    @property
    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.n_nodes, dtype=np.int64)])

    def node_steps(self) -> int:
        return self.n_total * self.n_steps

    def params(self) -> dict:
        return dict(model=self.model, Cm=self.Cm, Am=self.Am, sigma=self.sigma, h=self.h,
                    dt_0D=self.dt_0D, dt_1D=self.dt_1D, dt_split=self.dt_split,
                    v_th=self.v_th)

    def subset(self, fibers) -> "Workload":
        """The same workload restricted to the listed fibers (renumbered)."""
        fibers = [int(f) for f in fibers]
        off = self.offsets
        idx = np.concatenate([np.arange(off[f], off[f + 1]) for f in fibers]) if fibers \
            else np.zeros(0, dtype=np.int64)
        remap = {f: i for i, f in enumerate(fibers)}
        stims = []
        for s in self.stims:
            if s["fiber"] in remap:
                t = dict(s)
                t["fiber"] = remap[s["fiber"]]
                stims.append(t)
        rel = self.rel_noise[:, idx] if self.rel_noise is not None else None
        return replace(self, name=self.name + f"[{len(fibers)} fibers]",
                       n_nodes=self.n_nodes[fibers].astype(np.int32),
                       vm_noise=self.vm_noise[idx], rel_noise=rel, stims=stims)

    def with_steps(self, n_steps: int) -> "Workload":
        return replace(self, n_steps=int(n_steps))


def _normal(seed: int, n: int, scale: float) -> np.ndarray:
    return scale * np.random.Generator(np.random.PCG64(seed)).standard_normal(n)


def single_fiber(amp: float = AMP_AS_WRITTEN, n_nodes: int = 1000, t_end: float = 10.0,
                 dt: float = 1e-3) -> Workload:
    """One fiber of 1000 nodes, stimulus for 0.1 ms at the three centre nodes
    (int(N/2) - 1 .. int(N/2) + 1), V_m noise N(0, 0.1 mV), 10 ms."""
    n_steps = int(round(t_end / dt))
    return Workload(
        name=f"hh_single_fiber_{n_nodes}_amp{amp:g}", model=MODEL_HH,
        n_nodes=np.array([n_nodes], dtype=np.int32),
        vm_noise=_normal(SEED_VM_NOISE, n_nodes, 0.1), rel_noise=None,
        stims=[dict(fiber=0, node=n_nodes // 2, half_width=1, step_on=0,
                    n_steps=int(round(0.1 / dt)), period=0, amp=float(amp))],
        n_steps=n_steps, sample_every=int(round(0.1 / dt)),
        dt_0D=dt, dt_1D=dt, dt_split=dt)


def batched_hh(n_fibers: int = 1369, n_min: int = 1000, n_max: int = 1500,
               t_end: float = 20.0, amp: float = AMP_SUPRA, dt: float = 1e-3,
               onset_max: float = 5.0, realization: int = 0) -> Workload:
    """1369 fibers with lengths uniform in {1000..1500}; each fiber is
    stimulated for 0.1 ms on three nodes around a node drawn uniformly from
    the central 10 % of the fiber, at a time drawn uniformly from [0, 5] ms
    and snapped to a split step; V_m noise N(0, 0.1 mV); 20 ms.
    `realization` > 0 draws an independent set of stimulus nodes, onsets and
    noise (seeds shifted by 100 per realization) on the same fibers."""
    g_len = np.random.Generator(np.random.PCG64(SEED_LENGTHS))
    lengths = g_len.integers(n_min, n_max + 1, size=n_fibers).astype(np.int32)
    shift = 100 * int(realization)
    g_node = np.random.Generator(np.random.PCG64(SEED_STIM_NODE + shift))
    u_node = g_node.random(n_fibers)
    g_time = np.random.Generator(np.random.PCG64(SEED_STIM_TIME + shift))
    u_time = g_time.random(n_fibers)
    n_total = int(lengths.sum())
    noise = _normal(SEED_VM_NOISE + shift, n_total, 0.1)
    stims = []
    pulse = int(round(0.1 / dt))
    for f in range(n_fibers):
        N = int(lengths[f])
        lo, hi = int(np.floor(0.45 * N)), int(np.ceil(0.55 * N)) - 1
        node = lo + min(int(u_node[f] * (hi - lo + 1)), hi - lo)
        step_on = int(round(u_time[f] * onset_max / dt))
        stims.append(dict(fiber=f, node=node, half_width=1, step_on=step_on,
                          n_steps=pulse, period=0, amp=float(amp)))
    return Workload(
        name=f"hh_batched_{n_fibers}x{n_min}-{n_max}", model=MODEL_HH, n_nodes=lengths,
        vm_noise=noise, rel_noise=None, stims=stims, n_steps=int(round(t_end / dt)),
        sample_every=int(round(0.1 / dt)), dt_0D=dt, dt_1D=dt, dt_split=dt)


def st57_bundle(n_fibers: int = 400, n_nodes: int = 1481, t_end: float = 5.0,
                dt_0D: float = 1e-4, dt_split: float = 5e-4, amp: float = AMP_SUPRA,
                onset_max: float = 2.0, period_ms: float = 0.0,
                realization: int = 0, host_noise: bool = True) -> Workload:
    """ST57 fibers of equal length: every state starts at rest times
    (1 + 0.01 N(0, 1)) (seed 5); each fiber is stimulated for 0.1 ms on three
    nodes around a node drawn from the central 10 % (seed 3) at a time drawn
    from [0, onset_max] ms (seed 4), repeating every period_ms if > 0.
    dt_0D = 1e-4 ms, dt_1D = dt_split = 5e-4 ms.  `realization` > 0 shifts
    every seed by 100 per realization.  With host_noise False the
    perturbation is not drawn here (rel_noise None) but on the device by
    device_rel_noise(), for bundles too large for a host copy."""
    S = 57
    shift = 100 * int(realization)
    lengths = np.full(n_fibers, n_nodes, dtype=np.int32)
    n_total = int(lengths.sum())
    rel = (_normal(SEED_REL_NOISE + shift, S * n_total, 0.01).reshape(S, n_total)
           if host_noise else None)
    g_node = np.random.Generator(np.random.PCG64(SEED_STIM_NODE + shift))
    u_node = g_node.random(n_fibers)
    g_time = np.random.Generator(np.random.PCG64(SEED_STIM_TIME + shift))
    u_time = g_time.random(n_fibers)
    pulse = int(round(0.1 / dt_split))
    period = int(round(period_ms / dt_split)) if period_ms > 0 else 0
    stims = []
    lo, hi = int(np.floor(0.45 * n_nodes)), int(np.ceil(0.55 * n_nodes)) - 1
    for f in range(n_fibers):
        node = lo + min(int(u_node[f] * (hi - lo + 1)), hi - lo)
        step_on = int(round(u_time[f] * onset_max / dt_split))
        stims.append(dict(fiber=f, node=node, half_width=1, step_on=step_on, n_steps=pulse,
                          period=period, amp=float(amp)))
    return Workload(
        name=f"st57_{n_fibers}x{n_nodes}", model=MODEL_ST57, n_nodes=lengths,
        vm_noise=np.zeros(n_total), rel_noise=rel, stims=stims,
        n_steps=int(round(t_end / dt_split)), sample_every=int(round(0.1 / dt_split)),
        dt_0D=dt_0D, dt_1D=dt_split, dt_split=dt_split,
        extra=dict(rel_seed=SEED_REL_NOISE + shift))


def device_rel_noise(w: Workload, scale: float = 0.01):
    """Multiplicative perturbation N(0, scale) of every state of every node,
    drawn on the device (torch CUDA generator seeded from the workload) as a
    float32 tensor [S, n_total]; for fibers used in host-side checks, copy
    their columns back."""
    import torch
    S = 57 if w.model == MODEL_ST57 else 4
    g = torch.Generator(device="cuda")
    g.manual_seed(int(w.extra.get("rel_seed", SEED_REL_NOISE)))
    out = torch.empty((S, w.n_total), dtype=torch.float32, device="cuda")
    for k in range(S):
        out[k].normal_(0.0, scale, generator=g)
    return out


def stim_array(stims: List[dict]) -> np.ndarray:
    """Stimulus table as a packed record array matching the C struct layout
    (int32 fiber, node, half_width, pad; int64 step_on, n_steps, period;
    float64 amp)."""
    dt = np.dtype([("fiber", "<i4"), ("node", "<i4"), ("half_width", "<i4"), ("pad", "<i4"),
                   ("step_on", "<i8"), ("n_steps", "<i8"), ("period", "<i8"), ("amp", "<f8")])
    a = np.zeros(len(stims), dtype=dt)
    for i, s in enumerate(stims):
        a[i] = (s["fiber"], s["node"], s.get("half_width", 1), 0, s["step_on"], s["n_steps"],
                s.get("period", 0), s["amp"])
    return a
