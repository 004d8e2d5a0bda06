"""The large ST57 bundle at full size, in the launch configuration the
benchmark times: 10 000 fibers of 2000 nodes (2e7 nodes, 4.56 GB of FP32
state), the benchmark's realization with its device-drawn 1 % perturbation,
stimuli every 10 ms from onsets spread over [0, 10) ms, the split schedule
with the plan the library builds for it, the network surrogate at the
configured acceptance tolerance 1e-3, and the plain split schedule.  The
window is the first 2 ms of the benchmark's 10 ms (4000 split steps).

Checked:

* both runs against the FP64 oracle on sampled fibers that fire inside the
  window (fibers are independent: the per-fiber systems of eq.
  discretized_fibers_1 form a block-diagonal matrix, so the oracle's run of
  a fiber alone is its exact reference): V_m samples within 0.5 mV,
  activation times within one split step (and within a hundredth of one
  for the plain run, whose agreement is far closer), no node activated in
  one run and not the other;
* the surrogate against the plain run on all 2e7 nodes: V_m samples within
  0.5 mV, activation times within one split step where both activated, and
  a node activated in one run only just at the end of the window.

The network is trained by the library's kernels on the smaller bundle, with
fewer Adam steps than the benchmark.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2107_07104_amd import fib as F
from paper_2107_07104_amd import inputs as I
from paper_2107_07104_amd import surrogate as SU

from gpu_helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-3
WINDOW_MS = 2.0


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.lib()


def _sampled_fibers(w, window_ms):
    """The fiber with the earliest onset and the two nearest to a third and
    two thirds of the way to the window's last half millisecond."""
    onsets = np.array([st["step_on"] for st in w.stims]) * w.dt_split
    chosen = [int(np.argmin(onsets))]
    for t in ((window_ms - 0.5) / 3.0, 2.0 * (window_ms - 0.5) / 3.0):
        order = np.argsort(np.abs(onsets - t), kind="stable")
        chosen.append(next(int(x) for x in order if int(x) not in chosen))
    return sorted(chosen)


def _run(w, rel, cols, attach=None):
    s = SU._solver(w, schedule=F.FIB_SCHED_SPLIT)
    s.set_stimulus(w.stims)
    s.init_state(rel_noise=rel)
    if attach:
        attach(s)
    rows = w.n_steps // w.sample_every
    smp = torch.empty((rows, w.n_total), device="cuda")
    s.run(0, w.n_steps, w.sample_every, smp)
    s.sync()
    say(f"   plan {s.plan()}")
    ta = torch.as_tensor(s.tact(), device="cuda")
    rej = None
    if attach:
        tot, nst = s.fallbacks()
        rej = tot / max(1, nst * w.n_total)
    s.close()
    ci = torch.as_tensor(cols, device="cuda")
    return dict(smp=smp, ta=ta, smp_cols=smp.index_select(1, ci).cpu().numpy().astype(np.float64),
                ta_cols=ta[ci].cpu().numpy().astype(np.float64), rejected=rej)


def _vs_oracle(r, so, to):
    vm = float(np.max(np.abs(r["smp_cols"] - so)))
    tg = r["ta_cols"]
    both = np.isfinite(tg) & np.isfinite(to)
    dta = float(np.max(np.abs(tg[both] - to[both]))) if both.any() else 0.0
    return vm, dta, int(np.sum(np.isfinite(tg) != np.isfinite(to))), int(both.sum())


def test_headline_bundle_full_size_surrogate_and_plain():
    w = I.st57_bundle(n_fibers=10000, n_nodes=2000, t_end=10.0, onset_max=10.0, period_ms=10.0,
                      realization=2, host_noise=False)
    w = w.with_steps(int(round(WINDOW_MS / w.dt_split)))
    say(f"[headline full size] {w.name}: {w.n_total} nodes, {w.n_steps} steps")
    rel = I.device_rel_noise(w)
    fibers = _sampled_fibers(w, WINDOW_MS)
    off = w.offsets
    cols = np.concatenate([np.arange(off[f], off[f + 1]) for f in fibers])

    say("   training the network")
    wt = I.st57_bundle(n_fibers=400, n_nodes=1481, t_end=5.0)
    snaps = [int(round(t / wt.dt_split)) for t in (0.5, 1.5, 2.5, 3.5, 4.5)]
    sur = SU.train_surrogate(I.MODEL_ST57, wt, snaps, steps=4000, log=say)
    net = sur.network()
    say("   surrogate run")
    rs = _run(w, rel, cols, lambda s: s.set_surrogate(net, sur.scales, TOL))
    net.close()
    say(f"   rejected share {rs['rejected']:.2e}")
    say("   plain run")
    rp = _run(w, rel, cols)

    onsets = np.array([w.stims[f]["step_on"] for f in fibers]) * w.dt_split
    say(f"   oracle on fibers {fibers} (onsets {onsets} ms)")
    sub = w.subset(fibers)
    y0 = O.rest_state(I.MODEL_ST57)[:, None] * (
        1.0 + rel[:, torch.as_tensor(cols, device="cuda")].cpu().numpy().astype(np.float64))
    cfg = O.Config(model=sub.model, dt_0D=sub.dt_0D, dt_1D=sub.dt_1D, dt_split=sub.dt_split,
                   v_th=sub.v_th)
    _, so, to = O.run(cfg, sub.n_nodes, y0, sub.stims, sub.n_steps,
                      sample_every=sub.sample_every)
    for name, r, tight in (("surrogate", rs, False), ("plain", rp, True)):
        vm, dta, mism, act = _vs_oracle(r, so, to)
        say(f"   {name}: V_m {vm:.3e} mV, t_act {dta:.2e} ms, mismatch {mism}, "
            f"activated {act}")
        assert act > 100  # the fronts cross the sampled fibers' central nodes
        assert vm <= 0.5 and dta <= w.dt_split and mism == 0
        if tight:
            assert dta <= 0.01 * w.dt_split
    assert rs["rejected"] < 0.05

    # surrogate against plain on every node
    dv = float(torch.max(torch.abs(rs["smp"] - rp["smp"])))
    fs, fp = torch.isfinite(rs["ta"]), torch.isfinite(rp["ta"])
    both = fs & fp
    dt = float(torch.max(torch.abs(rs["ta"][both] - rp["ta"][both]))) if bool(both.any()) else 0.0
    only = fs ^ fp
    t_only = torch.where(fs, rs["ta"], rp["ta"])[only]
    earliest = float(t_only.min()) if bool(only.any()) else None
    say(f"   surrogate vs plain on {w.n_total} nodes: V_m {dv:.3e} mV, t_act {dt:.2e} ms "
        f"({int(both.sum())} activated in both), activated in one only {int(only.sum())}"
        + (f", earliest {earliest:.4f} ms" if earliest is not None else ""))
    assert int(both.sum()) > 10 ** 4
    assert dv <= 0.5 and dt <= w.dt_split
    if earliest is not None:
        assert earliest >= WINDOW_MS - 0.01
