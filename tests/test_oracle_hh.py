"""Pins of the oracle's subcellular model and of its Heun step.

The Hodgkin-Huxley membrane is checked against values fixed outside the
oracle: the textbook resting values of Hodgkin & Huxley (1952), the limits of
the removable singularities of alpha_m and alpha_n, the resting potential and
action-potential shape stated in the thesis, and the exact amplification of
Heun's method on the linear gate equation (a 2-stage second-order
Runge-Kutta step multiplies the deviation from the fixed point of
y' = lambda (y_inf - y) by exactly 1 - z + z^2/2 with z = lambda tau).
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2107_07104_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hh_rest_textbook.json")


def test_rest_state_matches_textbook():
    g = json.load(open(GOLD))
    y = O.rest_state()
    assert abs(y[0] - g["rest_V_mV"]) < g["rest_V_tol_mV"]
    assert abs(y[1] - g["m0"]) < g["gate_tol"]
    assert abs(y[2] - g["h0"]) < g["gate_tol"]
    assert abs(y[3] - g["n0"]) < g["gate_tol"]


def test_rest_state_is_stationary():
    y = O.rest_state()
    G = O.hh_rhs(y, 0.0)
    assert np.max(np.abs(G)) < 1e-12


def test_removable_singularities():
    # alpha_m -> 1 at V = -50 mV, alpha_n -> 0.1 at V = -65 mV
    assert O.hh_gate_rates(-50.0)[0] == pytest.approx(1.0, abs=1e-15)
    assert O.hh_gate_rates(-65.0)[4] == pytest.approx(0.1, abs=1e-16)
    # continuity across the switch to the series (|x| = 1e-4 <=> |dV| = 1e-3 mV)
    for V0, k in ((-50.0, 0), (-65.0, 4)):
        vals = [O.hh_gate_rates(V0 + d)[k] for d in (-2e-3, -1.0001e-3, -0.9999e-3, 0.0,
                                                       0.9999e-3, 1.0001e-3, 2e-3)]
        assert np.all(np.diff(vals) > 0)  # alpha_m, alpha_n increase with V
        assert np.max(np.abs(np.diff(vals))) < 1e-4


def test_rates_against_limits_far_from_rest():
    # For strongly depolarized V the gates' linear alphas approach the
    # asymptote 0.1*(v-25) (alpha_m) and 0.01*(v-10) (alpha_n): x/(e^x-1) -> -x
    # for x -> -inf.  For strongly hyperpolarized V they vanish exponentially.
    V = 200.0
    v = V + 75.0
    ab = O.hh_gate_rates(V)
    assert ab[0] == pytest.approx(0.1 * (v - 25.0), rel=1e-9)
    assert ab[4] == pytest.approx(0.01 * (v - 10.0), rel=1e-4)
    ab = O.hh_gate_rates(-300.0)
    assert ab[0] < 1e-9 and ab[3] < 1e-10
    # beta_h is a logistic function with value 1/2 at v = 30
    assert O.hh_gate_rates(-45.0)[3] == pytest.approx(0.5, abs=1e-15)


def _frozen_cfg(dt):
    # A huge capacitance freezes V, so each gate obeys a linear ODE
    return O.Config(Cm=1e300, dt_0D=dt, dt_1D=dt, dt_split=dt)


@pytest.mark.parametrize("V", [-90.0, -75.0, -50.0, -20.0, 10.0, 40.0])
def test_heun_exact_amplification_on_frozen_voltage(V):
    tau = 0.05
    y0 = np.array([V, 0.3, 0.7, 0.1])
    y1 = O.reaction(_frozen_cfg(tau), y0[:, None], tau)[:, 0]
    ab = O.hh_gate_rates(V)
    assert y1[0] == V
    for k, (a, b) in enumerate(((ab[0], ab[1]), (ab[2], ab[3]), (ab[4], ab[5]))):
        lam = a + b
        yinf = a / lam
        z = lam * tau
        expect = yinf + (y0[k + 1] - yinf) * (1.0 - z + 0.5 * z * z)
        assert y1[k + 1] == pytest.approx(expect, rel=1e-13, abs=1e-15)


def test_heun_local_error_is_third_order():
    # Against the exact solution y_inf + (y0 - y_inf) exp(-lambda t)
    V = -40.0
    ab = O.hh_gate_rates(V)
    lam = ab[0] + ab[1]
    yinf = ab[0] / lam
    errs = []
    for tau in (0.08, 0.04, 0.02, 0.01):
        y1 = O.reaction(_frozen_cfg(tau), np.array([[V], [0.0], [0.5], [0.5]]), tau)[1, 0]
        errs.append(abs(y1 - (yinf - yinf * np.exp(-lam * tau))))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 7.0) and np.all(ratios < 9.0)


def test_substep_count_rule():
    assert O.n_substeps(5e-4, 1e-3) == 1
    assert O.n_substeps(1e-3, 1e-3) == 1
    assert O.n_substeps(2.5e-4, 1e-4) == 3
    assert O.n_substeps(2.5e-3, 1e-3) == 3
    assert O.n_substeps(3e-3, 1e-3) == 3


def test_reaction_substeps_split_span():
    # n_sub equal substeps: one call over 3 tau with dt_0D = tau equals three
    # calls over tau
    y0 = np.array([[-60.0], [0.2], [0.5], [0.4]])
    tau = 1e-3
    cfg = O.Config(dt_0D=tau)
    a = O.reaction(cfg, y0, 3 * tau)
    b = y0
    for _ in range(3):
        b = O.reaction(cfg, b, tau)
    np.testing.assert_array_equal(a, b)


def test_single_cell_action_potential_shape():
    g = json.load(open(GOLD))
    y = O.rest_state()[:, None].copy()
    dt = 1e-3
    cfg = O.Config(dt_0D=dt)
    V = []
    for step in range(40000):  # 40 ms
        I = np.array([40.0 if step < 500 else 0.0])
        y = O.reaction(cfg, y, dt, I)
        V.append(y[0, 0])
    V = np.array(V)
    assert abs(V.max() - g["ap_peak_mV"]) < g["ap_peak_tol_mV"]
    assert V.min() < g["rest_V_mV"] - 1.0  # after-hyperpolarization overshoot
    t = np.arange(1, V.size + 1) * dt
    assert np.all(np.abs(V[t > g["recovery_ms"] + 5.0] - g["rest_V_mV"]) < 1.5)


def test_gates_stay_in_unit_interval_during_ap():
    from paper_2107_07104_amd import inputs as I
    w = I.single_fiber(amp=I.AMP_SUPRA, n_nodes=200, t_end=6.0)
    cfg = O.Config(dt_0D=w.dt_0D, dt_1D=w.dt_1D, dt_split=w.dt_split)
    y0 = np.tile(O.rest_state()[:, None], (1, w.n_total))
    y0[0] += w.vm_noise
    y = y0
    for k in range(6):
        y, _, _ = O.run(cfg, w.n_nodes, y, w.stims, 1000, step0=1000 * k)
        assert np.all(y[1:] >= 0.0) and np.all(y[1:] <= 1.0)


# ---- Hodgkin-Huxley with the approximate exponential (eq. apx-e-function) ----

def _exp_star_closed(x, n=1024):
    """(1 + x/n)^n through log1p and exp: a route independent of the
    oracle's ten squarings."""
    return np.exp(n * np.log1p(x / n))


def test_exp_star_relative_error_bound_printed_in_the_thesis():
    # the thesis bounds the relative error at |x| = 12 by 0.07
    for x in (12.0, -12.0):
        e = O.exp_star(x)
        rel = abs(e - np.exp(x)) / np.exp(x)
        assert 0.06 < rel < 0.07
        assert e == pytest.approx(_exp_star_closed(x), rel=1e-12)
    assert O.exp_star(0.0) == 1.0
    # (1 + x/n)^n < e^x for x != 0, and it converges to e^x as x/n -> 0
    xs = np.linspace(-20.0, 20.0, 81)
    es = np.array([O.exp_star(x) for x in xs])
    assert np.all(es[xs != 0.0] < np.exp(xs[xs != 0.0]))
    np.testing.assert_allclose(es, _exp_star_closed(xs), rtol=1e-11)


@pytest.mark.parametrize("V", [-50.0 + d for d in (-1e-2, -1e-3, -2e-5, 0.0, 2e-5, 1e-3, 1e-2)]
                         + [-65.0 + d for d in (-1e-3, -2e-5, 0.0, 2e-5, 1e-3)])
def test_exp_star_rates_near_the_removable_singularities(V):
    """alpha_m and alpha_n with exp* against x / expm1(n log1p(x / n)), and
    the limit 1 (times the prefactor) at x = 0."""
    ab = O.hh_apx_rates(V)
    for k, shift, pre in ((0, 50.0, 1.0), (4, 65.0, 0.1)):
        x = -(V + shift) / 10.0
        want = pre * (1.0 if x == 0.0 else x / np.expm1(1024 * np.log1p(x / 1024)))
        assert ab[k] == pytest.approx(want, rel=1e-9)


def test_exp_star_rates_and_rest_state():
    V = np.linspace(-100.0, 40.0, 57)
    for v in V:
        ex, apx = O.hh_gate_rates(v), O.hh_apx_rates(v)
        # every rate moves by at most the exp* error at its largest argument
        # on this range (|x| <= 15: relative 0.1)
        np.testing.assert_allclose(apx, ex, rtol=0.11)
    y = O.rest_state(O.MODEL_HH_APX_EXP)
    y_exact = O.rest_state(O.MODEL_HH)
    assert np.max(np.abs(O.hh_apx_rhs(y))) < 1e-10
    assert 1e-6 < abs(y[0] - y_exact[0]) < 0.5


def test_exp_star_membrane_fires_and_propagates():
    w = I.single_fiber(amp=I.AMP_SUPRA, n_nodes=200, t_end=8.0)
    cfg = O.Config(model=O.MODEL_HH_APX_EXP, dt_0D=w.dt_0D, dt_1D=w.dt_1D, dt_split=w.dt_split)
    y0 = np.tile(O.rest_state(O.MODEL_HH_APX_EXP)[:, None], (1, w.n_total))
    y, s, ta = O.run(cfg, w.n_nodes, y0, w.stims, w.n_steps, sample_every=w.sample_every)
    assert np.all(np.isfinite(ta))
    assert np.nanmax(s) > 20.0


def test_capacitance_scales_only_the_voltage_equation():
    # eq. subcellular_model_helper3: Cm dV/dt = -I_ion + I_stim; the gates'
    # equations do not involve Cm
    y = np.array([-40.0, 0.3, 0.4, 0.5])
    for I in (0.0, 50.0):
        g1, g2 = O.hh_rhs(y, I, Cm=1.0), O.hh_rhs(y, I, Cm=2.5)
        assert g1[0] != 0.0
        np.testing.assert_allclose(g2[0], g1[0] / 2.5, rtol=1e-15)
        np.testing.assert_array_equal(g2[1:], g1[1:])
