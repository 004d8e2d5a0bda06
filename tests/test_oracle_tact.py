"""Pins of the oracle's activation-time observable and of the conduction
velocity it measures.

The activation time of a node is the first upward crossing of v_th by V_m,
interpolated linearly between the ends of two consecutive split steps.  The
pins below do not restate that formula; they check what it must satisfy:

* consistency with the continuous problem: under joint refinement of all
  step widths the activation times of a travelling front converge at second
  order, like the Strang-split states they are read from (eq.
  monodomain_strang).  Attributing a crossing to the wrong split step, or
  interpolating from the wrong end of the step, leaves an error of order
  dt, which converges at first order and is about 0.9 dt in size;
* an exact case: with no diffusion, a one-step voltage prescription at a
  known step index k moves V_m from rest to just below the prescribed
  +40 mV (the outward current at +40 mV is between 0 and 100 uA/cm^2, so a
  step of 1e-3 ms lowers V_m by at most 0.1 mV); the crossing must then lie
  in step k, at the fraction (v_th - V_rest)/(V_end - V_rest) of it, with
  V_end only bracketed, not computed;
* only upward crossings count: a node that starts above v_th and falls
  through it keeps +inf, and a second upward crossing does not replace the
  first;
* the conduction velocity read from activation times converges under mesh
  refinement (second order in h); at h = 0.01 cm it is within 0.5 % of the
  finer mesh, the thesis's finding that 100 elements per cm resolve the
  propagation velocity (section "Effect of the Mesh Width on the Action
  Potential Propagation Velocity").
"""
import numpy as np

from oracle import oracle as O
from paper_2107_07104_amd import inputs as I


def _front_state():
    """A fiber of 200 nodes with an action potential under way (3 ms after a
    supra-threshold pulse at its centre)."""
    w = I.single_fiber(amp=I.AMP_SUPRA, n_nodes=200, t_end=3.0)
    y0 = np.tile(O.rest_state()[:, None], (1, w.n_total))
    y0[0] += w.vm_noise
    cfg = O.Config(dt_0D=w.dt_0D, dt_1D=w.dt_1D, dt_split=w.dt_split)
    y, _, _ = O.run(cfg, w.n_nodes, y0, w.stims, w.n_steps)
    return w, y


def test_activation_times_converge_at_second_order():
    w, ys = _front_state()
    T = 2.0

    def tact(dt):
        c = O.Config(dt_0D=dt, dt_1D=dt, dt_split=dt)
        return O.run(c, w.n_nodes, ys, [], int(round(T / dt)))[2]

    ref = tact(T / 16000)
    fin = np.isfinite(ref)
    assert fin.sum() > 50  # the front crosses many nodes inside the window
    dts = (4e-3, 2e-3, 1e-3)
    errs = []
    for dt in dts:
        ta = tact(dt)
        np.testing.assert_array_equal(np.isfinite(ta), fin)
        errs.append(np.max(np.abs(ta[fin] - ref[fin])))
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(np.abs(order - 2.0) < 0.2), order
    # a one-step offset would leave about 0.9 dt; the method leaves 0.006 dt
    assert errs[-1] < 0.02 * dts[-1], errs


def test_activation_time_of_a_prescribed_step():
    dt, k = 1e-3, 7
    n = 5
    cfg = O.Config(sigma=0.0, dt_0D=dt, dt_1D=dt, dt_split=dt)
    rest = O.rest_state()
    y0 = np.tile(rest[:, None], (1, n))
    stims = [dict(fiber=0, node=2, half_width=0, mode=1, step_on=k, n_steps=1, period=0,
                  amp=40.0)]
    y, _, ta = O.run(cfg, [n], y0, stims, 20)
    assert np.all(np.isinf(ta[[0, 1, 3, 4]]))
    vr = rest[0]
    # V_end in [39.9, 40]: bracket the interpolation fraction
    lo = k * dt + dt * (cfg.v_th - vr) / (40.0 - vr)
    hi = k * dt + dt * (cfg.v_th - vr) / (39.9 - vr)
    assert lo <= ta[2] <= hi, (ta[2], lo, hi)
    # the step that follows is where a one-step offset would put it, and the
    # reversed fraction lands at 0.52 of the step instead of 0.48
    assert ta[2] < (k + 0.5) * dt


def test_only_the_first_upward_crossing_counts():
    dt = 1e-3
    cfg = O.Config(sigma=0.0, dt_0D=dt, dt_1D=dt, dt_split=dt)
    rest = O.rest_state()
    y0 = np.tile(rest[:, None], (1, 3))
    # node 0 starts at +10 mV: it fires from there and repolarizes through
    # v_th downwards, which is no activation
    y0[0, 0] = 10.0
    # node 2 is prescribed above threshold twice, 6 ms apart
    stims = [dict(fiber=0, node=2, half_width=0, mode=1, step_on=3, n_steps=1, period=6000,
                  amp=40.0)]
    y, s, ta = O.run(cfg, [3], y0, stims, 12000, sample_every=100)
    assert s[:, 0].max() > 20.0 and s[-1, 0] < -60.0  # it did go up and come back down
    assert np.isinf(ta[0])
    assert np.isinf(ta[1])
    assert 3 * dt <= ta[2] < 4 * dt
    assert s[:, 2][(np.arange(1, 121) * 0.1) > 6.1].max() > 0.0  # the second pulse fired too


def test_conduction_velocity_converges_under_mesh_refinement():
    vel = []
    for h, n in ((0.02, 151), (0.01, 301), (0.005, 601)):
        c = n // 2
        hw = max(1, int(round(0.01 / h)))
        stims = [dict(fiber=0, node=c, half_width=hw, step_on=0, n_steps=100, period=0,
                      amp=I.AMP_SUPRA)]
        cfg = O.Config(h=h, dt_0D=1e-3, dt_1D=1e-3, dt_split=1e-3)
        y0 = np.tile(O.rest_state()[:, None], (1, n))
        _, _, ta = O.run(cfg, [n], y0, stims, 7500)
        a, b = c + int(round(0.5 / h)), c + int(round(1.2 / h))
        assert np.isfinite(ta[a]) and np.isfinite(ta[b])
        vel.append((b - a) * h / (ta[b] - ta[a]))
    v = np.array(vel)
    # a physiological HH velocity (cm/ms), rising to its limit under refinement
    assert 0.15 < v[-1] < 0.25 and v[0] < v[1] < v[2]
    order = np.log2((v[1] - v[0]) / (v[2] - v[1]))
    assert 1.7 < order < 2.3, order
    assert abs(v[1] - v[2]) < 0.005 * v[2]
