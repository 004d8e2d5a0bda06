"""Adaptive computation on the GPU against the FP64 oracle's adaptive loop.

* a vanishing tolerance keeps every point active: the adaptive kernels
  reproduce the plain schedule bit for bit (fused and split) and count every
  node-step;
* an infinite tolerance solves exactly the stimulated points and their
  neighbours after the first step (solved counts equal the oracle's, an
  integer result, bit-exact), and freezes the state once the stimulus is off;
* fibers are untouched before their first stimulus;
* from an equilibrium start (the premise of the scheme: no initial noise),
  Hodgkin-Huxley batches under Strang and Godunov splitting and an ST57
  bundle stay within the method's budget (0.5 mV, one split step) of the
  oracle's adaptive run and of its plain run, and the solved node-steps
  agree with the oracle's to 2 % (the FP32 check may decide points near the
  threshold the other way);
* chunked runs, starting at odd and even steps, equal one run bit for bit;
* ST57 runs the list form (decisions, then the reaction parts over the list
  of solved nodes): at a vanishing tolerance it is the plain split run up
  to FP32 rounding under both splittings, it matches the oracle under Godunov
  splitting too, and chunked runs equal one run;
* the requests the library refuses.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_2107_07104_amd import fib as F
from paper_2107_07104_amd import inputs as I

from gpu_helpers import compare_runs, gpu_solver, oracle_cfg, oracle_init, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.lib()


def _quiet(w):
    """The workload from an equilibrium start: no V_m or state noise."""
    return replace(w, vm_noise=np.zeros_like(w.vm_noise), rel_noise=None)


def _run(s, w, n_steps, step0=0):
    rows = (step0 + n_steps) // w.sample_every - step0 // w.sample_every
    samples = torch.full((max(rows, 1), w.n_total), float("nan"), device="cuda")
    s.run(step0, n_steps, w.sample_every, samples if rows else None)
    s.sync()
    return (s.get_state(), samples[:rows].cpu().numpy().astype(np.float64), s.tact().astype(np.float64))


def _adaptive_gpu(w, tol, n_steps=None, schedule=F.FIB_SCHED_SPLIT, **kw):
    s = gpu_solver(w, schedule=schedule, **kw)
    s.set_adaptive(tol)
    out = _run(s, w, w.n_steps if n_steps is None else n_steps)
    return out + (s,)


def _at_zero(w):
    return replace(w, stims=[dict(st, step_on=0) for st in w.stims])


SCHEDULES = [F.FIB_SCHED_FUSED, F.FIB_SCHED_SPLIT]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("splitting", [F.FIB_SPLIT_STRANG, F.FIB_SPLIT_GODUNOV])
def test_vanishing_tolerance_is_the_plain_schedule(splitting, schedule):
    w = _at_zero(I.batched_hh(n_fibers=6, n_min=300, n_max=400, t_end=1.0))
    say(f"[adaptive tol->0] splitting={splitting} schedule={schedule}")
    plain = gpu_solver(w, schedule=schedule, splitting=splitting)
    yp, sp, tp = _run(plain, w, w.n_steps)
    plain.close()
    ya, sa, ta, s = _adaptive_gpu(w, 1e-30, schedule=schedule, splitting=splitting)
    np.testing.assert_array_equal(ya, yp)
    np.testing.assert_array_equal(sa, sp)
    np.testing.assert_array_equal(ta, tp)
    assert s.adaptive_solved() == w.n_total * w.n_steps
    assert np.all(s.adaptive_points() == 1)
    s.close()


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("splitting", [F.FIB_SPLIT_STRANG, F.FIB_SPLIT_GODUNOV])
def test_infinite_tolerance_counts_match_the_oracle(splitting, schedule):
    w = _quiet(I.batched_hh(n_fibers=5, n_min=40, n_max=90, t_end=0.3, onset_max=0.05))
    w.stims[1]["node"] = 0                      # clipped at the fiber's first node
    w.stims[2]["node"] = int(w.n_nodes[2]) - 1  # and at its last
    scheme = O.SCHEME_GODUNOV if splitting == F.FIB_SPLIT_GODUNOV else O.SCHEME_STRANG
    cfg = oracle_cfg(w, scheme=scheme)
    s = gpu_solver(w, schedule=schedule, splitting=splitting)
    s.set_adaptive(1e30)
    y = oracle_init(w)
    pt = None
    before = 0
    frozen = None
    for step in range(w.n_steps):
        y, _, _, pt, cnt = O.run_adaptive(cfg, w.n_nodes, y, w.stims, 1, step0=step,
                                          tol=np.inf, pt=pt)
        s.run(step, 1)
        got = s.adaptive_solved()
        assert got - before == cnt, f"step {step}: GPU {got - before}, oracle {cnt}"
        before = got
        np.testing.assert_array_equal(s.adaptive_points(), (pt == O.PT_ACTIVE).astype(np.uint8))
        if cnt == 0 and step > 150:
            if frozen is None:
                frozen = s.get_state()
            np.testing.assert_array_equal(s.get_state(), frozen)
    say(f"   solved node-steps {before}")
    assert frozen is not None
    s.close()


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_fibers_untouched_before_their_first_stimulus(schedule):
    w = I.batched_hh(n_fibers=6, n_min=200, n_max=300, t_end=1.0, onset_max=0.2)
    w.stims[2]["step_on"] = 600
    w.stims[4]["step_on"] = 10 ** 6
    s = gpu_solver(w, schedule=schedule)
    y0 = s.get_state()
    s.set_adaptive(1e-6)
    s.run(0, 600)
    s.sync()
    y = s.get_state()
    off = w.offsets
    for f in (2, 4):
        np.testing.assert_array_equal(y[:, off[f]:off[f + 1]], y0[:, off[f]:off[f + 1]])
    s.run(600, 1)
    y1 = s.get_state()
    assert np.any(y1[:, off[2]:off[3]] != y0[:, off[2]:off[3]])
    np.testing.assert_array_equal(y1[:, off[4]:off[5]], y0[:, off[4]:off[5]])
    s.close()


def _parity(w, tol, splitting=F.FIB_SPLIT_STRANG, schedule=F.FIB_SCHED_SPLIT):
    scheme = O.SCHEME_GODUNOV if splitting == F.FIB_SPLIT_GODUNOV else O.SCHEME_STRANG
    cfg = oracle_cfg(w, scheme=scheme)
    y0 = oracle_init(w)
    ya, sa, ta, pta, cnt = O.run_adaptive(cfg, w.n_nodes, y0, w.stims, w.n_steps,
                                          sample_every=w.sample_every, tol=tol)
    plain = O.run(cfg, w.n_nodes, y0, w.stims, w.n_steps, sample_every=w.sample_every)
    yg, sg, tg, s = _adaptive_gpu(w, tol, schedule=schedule, splitting=splitting)
    got = s.adaptive_solved()
    total = w.n_total * w.n_steps
    res_a = compare_runs(w, (yg, sg, tg, s), (ya, sa, ta))
    res_p = compare_runs(w, (yg, sg, tg, s), plain)
    say(f"   solved: GPU {got / total:.3f}, oracle {cnt / total:.3f} of the node-steps")
    say("   vs oracle adaptive", res_a)
    say("   vs oracle plain   ", res_p)
    for res in (res_a, res_p):
        assert res["vm_err"] <= 0.5
        assert res["tact_err"] <= w.dt_split
        assert res["tact_mismatch"] == 0
    assert abs(got - cnt) <= 0.02 * cnt
    s.close()
    return got / total


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("splitting", [F.FIB_SPLIT_STRANG, F.FIB_SPLIT_GODUNOV])
def test_hh_batch_matches_oracle(splitting, schedule):
    w = _quiet(I.batched_hh(n_fibers=24, t_end=7.0))
    say(f"[adaptive HH] splitting={splitting} schedule={schedule} steps={w.n_steps}")
    share = _parity(w, 1e-6, splitting, schedule)
    assert share < 0.6


def test_st57_bundle_matches_oracle():
    w = _quiet(I.st57_bundle(n_fibers=6, n_nodes=523, t_end=1.5, onset_max=0.5))
    say(f"[adaptive ST57] steps={w.n_steps}")
    share = _parity(w, 1e-6)
    assert share < 0.8


@pytest.mark.parametrize("splitting", [F.FIB_SPLIT_STRANG, F.FIB_SPLIT_GODUNOV])
def test_st57_vanishing_tolerance_is_the_plain_schedule(splitting):
    """ST57 takes the list form (decisions, then the reaction parts over the
    solved nodes): with every point active it is the plain split run up to
    FP32 rounding (the two kernels compile the same Heun steps with their
    multiply-adds contracted differently; a node solved twice or not at all
    would be millivolts off)."""
    w = _at_zero(I.st57_bundle(n_fibers=4, n_nodes=180, t_end=0.15, onset_max=0.0))
    say(f"[adaptive ST57 tol->0] splitting={splitting} nodes={w.n_total} steps={w.n_steps}")
    plain = gpu_solver(w, splitting=splitting)
    yp, sp, tp = _run(plain, w, w.n_steps)
    plain.close()
    ya, sa, ta, s = _adaptive_gpu(w, 1e-30, splitting=splitting)
    d = np.abs(ya - yp) / (1.0 + np.abs(yp))
    say(f"   max relative state difference {d.max():.2e}, "
        f"{np.count_nonzero(ya != yp)} of {ya.size} entries differ")
    assert d.max() < 1e-6
    np.testing.assert_allclose(sa, sp, rtol=0, atol=1e-4)
    assert np.array_equal(np.isfinite(ta), np.isfinite(tp)) and np.isfinite(tp).any()
    fin = np.isfinite(tp)
    assert np.max(np.abs(ta[fin] - tp[fin])) < 1e-6
    assert s.adaptive_solved() == w.n_total * w.n_steps
    s.close()


def test_st57_godunov_matches_oracle():
    w = _quiet(I.st57_bundle(n_fibers=4, n_nodes=301, t_end=1.0, onset_max=0.3))
    say(f"[adaptive ST57 Godunov] steps={w.n_steps}")
    share = _parity(w, 1e-6, F.FIB_SPLIT_GODUNOV)
    assert share < 0.8


@pytest.mark.parametrize("splitting", [F.FIB_SPLIT_STRANG, F.FIB_SPLIT_GODUNOV])
def test_st57_chunked_adaptive_runs_are_bitwise_identical(splitting):
    w = _quiet(I.st57_bundle(n_fibers=3, n_nodes=150, t_end=0.5, onset_max=0.1))
    ys, ss, ts, s = _adaptive_gpu(w, 1e-6, splitting=splitting)
    n1 = s.adaptive_solved()
    s.close()
    c = gpu_solver(w, splitting=splitting)
    c.set_adaptive(1e-6)
    for a, b in ((0, 171), (171, 500), (500, 733), (733, w.n_steps)):
        c.run(a, b - a)
    c.sync()
    np.testing.assert_array_equal(c.get_state(), ys)
    np.testing.assert_array_equal(c.tact(), ts)
    assert c.adaptive_solved() == n1 > 0
    c.close()


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_chunked_adaptive_runs_are_bitwise_identical(schedule):
    w = _quiet(I.batched_hh(n_fibers=5, n_min=200, n_max=300, t_end=2.0, onset_max=0.5))
    ys, ss, ts, s = _adaptive_gpu(w, 1e-6, schedule=schedule)
    n1 = s.adaptive_solved()
    s.close()
    c = gpu_solver(w, schedule=schedule)
    c.set_adaptive(1e-6)
    for a, b in ((0, 351), (351, 1000), (1000, 1433), (1433, 2000)):
        c.run(a, b - a)
    c.sync()
    np.testing.assert_array_equal(c.get_state(), ys)
    np.testing.assert_array_equal(c.tact(), ts)
    assert c.adaptive_solved() == n1
    c.close()


def test_fused_and_split_adaptive_agree():
    """The fused kernel (states in LDS, compacted solve list) and the split
    schedule take the same decisions: equal solved counts and states within
    FP32 rounding."""
    w = _quiet(I.batched_hh(n_fibers=12, n_min=600, n_max=900, t_end=3.0, onset_max=1.0))
    a = _adaptive_gpu(w, 1e-6, schedule=F.FIB_SCHED_FUSED)
    b = _adaptive_gpu(w, 1e-6, schedule=F.FIB_SCHED_SPLIT)
    na, nb = a[3].adaptive_solved(), b[3].adaptive_solved()
    say(f"   solved fused {na}, split {nb}; V diff {np.max(np.abs(a[0][0] - b[0][0])):.2e}")
    assert abs(na - nb) <= 0.01 * nb
    assert np.max(np.abs(a[1] - b[1])) < 0.05
    a[3].close()
    b[3].close()


def test_refused_requests():
    w = I.batched_hh(n_fibers=3, n_min=100, n_max=120, t_end=0.1)
    # ST57 states do not fit the fused kernel
    ws = I.st57_bundle(n_fibers=2, n_nodes=64, t_end=0.01)
    s = gpu_solver(ws, schedule=F.FIB_SCHED_FUSED)
    s.set_adaptive(1e-5)
    with pytest.raises(F.FibError) as e:
        s.run(0, 2)
    assert e.value.code == F.FIB_EUNSUPPORTED
    s.close()
    s = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(F.FibError) as e:
            s.set_adaptive(bad)
        assert e.value.code == F.FIB_EINVAL
    with pytest.raises(F.FibError) as e:
        s.adaptive_points()
    assert e.value.code == F.FIB_ESTATE
    s.set_adaptive(1e-5)
    s.set_adaptive(0.0)       # off again: the plain split schedule
    s.run(0, 10)
    s.sync()
    s.close()
