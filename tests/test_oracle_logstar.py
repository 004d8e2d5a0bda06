"""Pins of the approximate logarithm log* and of the ST57 model with exp* and
log* (section "Evaluation of Code Generator Optimizations", figure apxlog,
eq. apx-e-function).

log*: the sixth-order Taylor polynomials of log around 1, 3 and 9 (pieces
split at 2 and 6), then one Newton step on exp*(y) = x with the derivative
taken as exp*(y), y <- y - (1 - x / exp*(y)), so that log* inverts exp*.

* the polynomials are exact at their expansion points and their relative
  error on [0.2, 20] is the thesis's: at most 0.105 except just below the
  break at 2, where the truncated series around 1 reaches 0.110 (reading:
  the thesis's bound is read from its plot); a fifth-order truncation or
  misplaced breaks exceed it;
* after the Newton step exp*(log*(x)) returns x within the step's quadratic
  remainder (5 % at the worst Taylor error), much closer near the expansion
  points, and six times closer than the Taylor value alone;
* outside [0.2, 20] an exact power-of-two scaling applies:
  log*(2x) - log*(x) = log 2 exactly when both lie outside;
* ST57 with exp* and log*: its resting state is a fixed point, Heun steps
  keep every linear invariant, the sensor chain relaxes to the Boltzmann
  distribution of its exp* rates, and it fires an action potential that
  departs from the exact model's by a few millivolts.
"""
import numpy as np
import pytest

from oracle import oracle as O


def _rel(approx, x):
    return np.abs(approx - np.log(x)) / np.abs(np.log(x))


def test_taylor_pieces_exact_at_expansion_points():
    for a in (1.0, 3.0, 9.0):
        assert O.log_star_taylor(a) == pytest.approx(np.log(a), abs=1e-15)
    assert O.log_star(1.0) == 0.0


def test_taylor_pieces_meet_only_at_the_breaks_2_and_6():
    # three polynomials, discontinuous exactly at x = 2 and x = 6: the value
    # jumps there and nowhere else on [0.2, 20)
    eps = 1e-9
    def jump(b):
        return abs(O.log_star_taylor(b) - O.log_star_taylor(b - eps))
    for b in (2.0, 6.0):
        assert jump(b) > 1e-4, b
    for b in np.linspace(0.25, 19.75, 157):
        if min(abs(b - 2.0), abs(b - 6.0)) > 1e-6:
            assert jump(b) < 1e-7, b


def test_taylor_error_bound_of_figure_apxlog():
    x = np.linspace(0.2, 20.0, 40001)
    x = x[np.abs(x - 1.0) > 1e-9]
    lt = np.array([O.log_star_taylor(v) for v in x])
    e = _rel(lt, x)
    near_break = (x > 1.97) & (x < 2.0)
    assert e[~near_break].max() <= 0.105
    assert 0.105 < e[near_break].max() <= 0.111
    # the pieces switch at 2 and 6: just above each break the next piece
    # is accurate to 1e-3
    for b in (2.0, 6.0):
        assert _rel(O.log_star_taylor(b), b) < 1e-3


def test_newton_step_makes_log_star_invert_exp_star():
    x = np.linspace(0.2, 20.0, 4001)
    ls = np.array([O.log_star(v) for v in x])
    res = np.array([O.exp_star(v) for v in ls]) / x - 1.0
    assert np.abs(res).max() < 0.05
    # the Taylor error enters squared (plus y/1024 of it from the derivative
    # taken as exp*(y)): near the expansion points the inverse holds to 1e-5
    for a in (1.0, 3.0, 9.0):
        for xx in (0.98 * a, 1.02 * a):
            assert abs(O.exp_star(O.log_star(xx)) / xx - 1.0) < 1e-5
    # without the step the residual is the Taylor error itself (6x larger)
    lt = np.array([O.log_star_taylor(v) for v in x])
    res_t = np.array([O.exp_star(v) for v in lt]) / x - 1.0
    assert np.abs(res_t).max() > 5 * np.abs(res).max()


def test_range_reduction_outside_the_design_interval():
    for x in (25.6, 40.0, 1e3, 0.0357, 0.15, 1e-3):
        lx, l2x = O.log_star(x), O.log_star(2.0 * x)
        if not (0.2 <= x < 20.0) and not (0.2 <= 2 * x < 20.0):
            assert l2x - lx == pytest.approx(np.log(2.0), abs=1e-14)
        assert abs(lx - np.log(x)) < 0.05
    assert np.isnan(O.log_star(0.0)) and np.isnan(O.log_star(-1.0))


@pytest.fixture(scope="module")
def rest_apx():
    return O.rest_state(O.MODEL_ST57_APX)


def test_st57_apx_rest_state_and_invariants(rest_apx):
    G = O.st57_apx_rhs(rest_apx)
    assert np.max(np.abs(G) / np.maximum(np.abs(rest_apx), 1.0)) < 1e-10
    np.testing.assert_allclose(O.st57_invariants(rest_apx), [1, 1, 1, 1, 2200, 1500], rtol=1e-13)
    exact = O.rest_state(O.MODEL_ST57)
    # a different fixed point, close to the exact model's
    assert 1e-4 < abs(rest_apx[0] - exact[0]) < 0.5
    rng = np.random.default_rng(3)
    y = rest_apx[:, None] * (1 + 0.05 * rng.standard_normal((57, 4)))
    y[0] += np.array([0, 30, 70, 110])
    inv0 = np.array([O.st57_invariants(y[:, i]) for i in range(4)])
    cfg = O.Config(model=O.MODEL_ST57_APX, dt_0D=1e-4)
    for _ in range(40):
        y = O.reaction(cfg, y, 5e-4, np.array([0.0, 0.0, 800.0, 0.0]))
    inv1 = np.array([O.st57_invariants(y[:, i]) for i in range(4)])
    np.testing.assert_allclose(inv1, inv0, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("Vt", [-80.0, -20.0, 30.0])
def test_st57_apx_sensor_chain_boltzmann(rest_apx, Vt):
    y = rest_apx.copy()
    y[4] = Vt
    y[8:18] = 0.1
    cfg = O.Config(model=O.MODEL_ST57_APX, Cm=1e300, dt_0D=2e-3)
    yy = y[:, None]
    for _ in range(60):
        yy = O.reaction(cfg, yy, 1.0)
    P = yy[8:18, 0]
    Vi = -70.0 + 7.5 * np.arange(9)
    ratio = np.array([O.exp_star((Vt - v) / 25.0) / O.exp_star(-(Vt - v) / 25.0) for v in Vi])
    w = np.concatenate([[1.0], np.cumprod(ratio)])
    np.testing.assert_allclose(P, w / w.sum(), rtol=1e-6, atol=1e-9)


def test_st57_apx_fires_close_to_the_exact_model():
    n = 120
    stims = [dict(fiber=0, node=60, half_width=1, step_on=0, n_steps=200, period=0, amp=1200.0)]
    out = {}
    for model in (O.MODEL_ST57, O.MODEL_ST57_APX):
        r = O.rest_state(model)
        cfg = O.Config(model=model, dt_0D=1e-4, dt_1D=5e-4, dt_split=5e-4)
        y, s, ta = O.run(cfg, [n], np.tile(r[:, None], (1, n)), stims, 3000, sample_every=100)
        assert 15.0 < np.nanmax(s) < 45.0 and np.all(np.isfinite(ta[45:76]))
        out[model] = (s, ta)
    dv = np.max(np.abs(out[O.MODEL_ST57][0] - out[O.MODEL_ST57_APX][0]))
    dta = np.max(np.abs(out[O.MODEL_ST57][1][45:76] - out[O.MODEL_ST57_APX][1][45:76]))
    # the approximations move the action potential by millivolts, not tens
    assert 0.01 < dv < 20.0 and dta < 0.2
