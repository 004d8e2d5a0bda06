"""Pins of the oracle's adaptive computation (section
sec:adaptive_computation_for_fiber_based, figure state_chart).

* tol = 0: a point becomes inactive only if a reaction part leaves its state
  bitwise unchanged, which no point near rest does in FP64, so with every
  fiber stimulated from step 0 the adaptive loop is the plain splitting loop
  bit for bit and solves every node in every step;
* tol = infinity: no point passes the equilibrium check, so after the first
  step exactly the stimulated points and their neighbours inside the fiber
  are solved while the stimulus is on (counted exactly, also for a stimulus
  clipped at a fiber end), and nothing once it is off; with nothing solved
  the diffusion is skipped too, so the state freezes;
* a fiber is left out until its first stimulus: its state is bitwise
  unchanged before that step and nothing of it is solved;
* from an equilibrium start (no V_m noise, the premise of the scheme) with a
  small tolerance the adaptive run stays within 0.01 mV of the plain run
  while solving a minority of the node-steps;
* the equilibrium check is relative to each state: at a tolerance just
  below or above the largest relative change of the step's last reaction
  part (from the reaction alone) a node is solved again or not.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_2107_07104_amd import inputs as I


def _cfg(w, scheme=O.SCHEME_STRANG):
    return O.Config(scheme=scheme, dt_0D=w.dt_0D, dt_1D=w.dt_1D, dt_split=w.dt_split)


def _rest(w):
    return np.tile(O.rest_state()[:, None], (1, w.n_total))


def _fibers(n_nodes, onsets, node=None, n_steps=20):
    stims = [dict(fiber=f, node=(n // 2 if node is None else node), half_width=1, step_on=s,
                  n_steps=n_steps, period=0, amp=I.AMP_SUPRA)
             for f, (n, s) in enumerate(zip(n_nodes, onsets))]
    return I.Workload(name="adaptive_pin", model=I.MODEL_HH,
                      n_nodes=np.array(n_nodes, dtype=np.int32),
                      vm_noise=np.zeros(sum(n_nodes)), rel_noise=None, stims=stims,
                      n_steps=300, sample_every=50, dt_0D=1e-3, dt_1D=1e-3, dt_split=1e-3)


@pytest.mark.parametrize("scheme", [O.SCHEME_STRANG, O.SCHEME_GODUNOV])
def test_zero_tolerance_is_the_plain_loop(scheme):
    w = _fibers([60, 33, 1, 2], [0, 0, 0, 0])
    y0 = _rest(w)
    y0[0] += 0.1 * np.random.default_rng(3).standard_normal(w.n_total)
    cfg = _cfg(w, scheme)
    yp, sp, tp = O.run(cfg, w.n_nodes, y0, w.stims, w.n_steps, sample_every=w.sample_every)
    ya, sa, ta, pt, cnt = O.run_adaptive(cfg, w.n_nodes, y0, w.stims, w.n_steps,
                                         sample_every=w.sample_every, tol=0.0)
    np.testing.assert_array_equal(ya, yp)
    np.testing.assert_array_equal(sa, sp)
    np.testing.assert_array_equal(ta, tp)
    assert cnt == w.n_total * w.n_steps
    assert np.all(pt == O.PT_ACTIVE)


@pytest.mark.parametrize("scheme", [O.SCHEME_STRANG, O.SCHEME_GODUNOV])
def test_infinite_tolerance_solves_the_stimulated_points_and_neighbours(scheme):
    dur = 20
    n = [50, 40]
    # fiber 0: centre stimulus (3 points + 2 neighbours); fiber 1: stimulus at
    # node 0, clipped to nodes 0 and 1 (+ neighbour 2)
    w = _fibers(n, [0, 0], n_steps=dur)
    w.stims[1]["node"] = 0
    cfg = _cfg(w, scheme)
    ya, _, _, pt, cnt = O.run_adaptive(cfg, w.n_nodes, _rest(w), w.stims, 1, tol=np.inf)
    assert cnt == sum(n)                       # step 0: every point starts active
    assert np.all(pt[[24, 26, 50 + 2]] == O.PT_INACTIVE)
    y = ya
    for step in range(1, dur):
        y, _, _, pt, cnt = O.run_adaptive(cfg, w.n_nodes, y, w.stims, 1, step0=step,
                                          tol=np.inf, pt=pt)
        assert cnt == 5 + 3
    y_off, _, _, pt, cnt = O.run_adaptive(cfg, w.n_nodes, y, w.stims, 1, step0=dur,
                                          tol=np.inf, pt=pt)
    assert cnt == 0 and np.all(pt == O.PT_INACTIVE)
    # nothing solved: no reaction and no diffusion, the state is frozen
    y_end, _, _, _, cnt = O.run_adaptive(cfg, w.n_nodes, y_off, w.stims, 50, step0=dur + 1,
                                         tol=np.inf, pt=pt)
    assert cnt == 0
    np.testing.assert_array_equal(y_end, y_off)


def test_fiber_left_out_until_its_first_stimulus():
    w = _fibers([40, 40, 40], [0, 100, 10 ** 6])
    y0 = _rest(w)
    y0[0] += 0.1 * np.random.default_rng(4).standard_normal(w.n_total)
    cfg = _cfg(w)
    y, _, _, pt, cnt = O.run_adaptive(cfg, w.n_nodes, y0, w.stims, 100, tol=1e-6)
    np.testing.assert_array_equal(y[:, 40:], y0[:, 40:])
    assert np.all(pt[40:] == O.PT_ACTIVE)       # untouched initial states
    y2, _, _, _, cnt2 = O.run_adaptive(cfg, w.n_nodes, y, w.stims, 1, step0=100, tol=1e-6,
                                       pt=pt)
    assert np.any(y2[:, 40:80] != y[:, 40:80])   # fiber 1 takes part from step 100
    np.testing.assert_array_equal(y2[:, 80:], y0[:, 80:])
    assert cnt2 >= 40                            # all its points start active


def test_equilibrium_start_stays_close_to_the_plain_run():
    w = I.batched_hh(n_fibers=4, n_min=300, n_max=400, t_end=6.0, onset_max=2.0)
    w = replace(w, vm_noise=np.zeros_like(w.vm_noise))
    y0 = _rest(w)
    cfg = _cfg(w)
    yp, sp, tp = O.run(cfg, w.n_nodes, y0, w.stims, w.n_steps, sample_every=w.sample_every)
    ya, sa, ta, pt, cnt = O.run_adaptive(cfg, w.n_nodes, y0, w.stims, w.n_steps,
                                         sample_every=w.sample_every, tol=1e-7)
    share = cnt / (w.n_total * w.n_steps)
    assert np.max(np.abs(sa - sp)) < 0.01 and np.max(np.abs(ya[0] - yp[0])) < 0.01
    fin = np.isfinite(tp)
    np.testing.assert_array_equal(np.isfinite(ta), fin)
    assert fin.sum() > 300
    assert np.max(np.abs(ta[fin] - tp[fin])) < 0.1 * w.dt_split
    assert share < 0.5


@pytest.mark.parametrize("scheme", [O.SCHEME_STRANG, O.SCHEME_GODUNOV])
def test_the_equilibrium_check_is_relative_to_each_state(scheme):
    """One node (no diffusion coupling), V_m 1 mV off rest, and a zero-
    current entry on in step 0 only (so the fiber takes part from step 0).
    The check compares the two ends of the step's last reaction part, which
    the pinned reaction alone gives: with the tolerance just below the
    largest relative change max_k |y+_k - y_k| / |y_k| the node is solved
    again in step 1, just above it it is not."""
    dt = 1e-3
    cfg = O.Config(scheme=scheme, dt_0D=dt, dt_1D=dt, dt_split=dt)
    y0 = O.rest_state()[:, None].copy()
    y0[0] += 1.0
    if scheme == O.SCHEME_STRANG:
        y1 = O.reaction(cfg, y0, 0.5 * dt)       # first half; one node: no diffusion
        y2 = O.reaction(cfg, y1, 0.5 * dt)
    else:
        y1, y2 = y0, O.reaction(cfg, y0, dt)
    rel = np.abs(y2[:, 0] - y1[:, 0]) / np.abs(y1[:, 0])
    # an absolute test |y+_k - y_k| > tol would keep the node active at both
    # tolerances: V_m changes by more than the larger one
    assert np.max(np.abs(y2[:, 0] - y1[:, 0])) > 1.01 * rel.max()
    stims = [dict(fiber=0, node=0, half_width=0, step_on=0, n_steps=1, period=0, amp=0.0)]
    for factor, solved in ((0.99, 2), (1.01, 1)):
        *_, cnt = O.run_adaptive(cfg, [1], y0, stims, 2, tol=factor * rel.max())
        assert cnt == solved, (factor, cnt)
