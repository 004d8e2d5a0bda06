"""GPU surrogate split step against the FP64 references.

* the network inside the step kernel (BF16 fragments in LDS, activations in
  registers) gives the same prediction as the FP64 network of
  oracle/mlp.py on the same normalized inputs, for both model shapes and a
  node count with a ragged last tile;
* with every node accepted, the corrected update is the FP64 fixed-point
  iteration du1 = dt G(y + du/2), du2 = dt G(y + du1/2) of the implicit
  midpoint rule started from the FP64 prediction, G from the oracle (two
  iterations for Hodgkin-Huxley, one for ST57);
* with every node rejected, a surrogate run is bitwise the plain split run
  (the fallback is the plain Heun pair);
* a network trained on the GPU from plain runs keeps a batched run within
  the V_m and activation-time tolerances of the FP64 oracle while it takes
  the step for most nodes (end-to-end, with the oracle on a subset).

The corrector's sensitivity to the prediction is (dt |dG/dy| / 2)^c after
c iterations (about 0.02^2 for Hodgkin-Huxley, 0.26 for ST57), so the
second check bounds the BF16 error of the prediction times that factor on
top of FP32 tolerances.
"""
import numpy as np
import pytest

from oracle import mlp as M
from oracle import oracle as O
from paper_2107_07104_amd import fib as F
from paper_2107_07104_amd import inputs as I
from paper_2107_07104_amd import surrogate as SU

from gpu_helpers import gpu_solver, say

ITERATIONS = {I.MODEL_HH: 2, I.MODEL_ST57: 1}

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.lib()


def _workload(model):
    """A few fibers (node count not a multiple of 64) with activity: plain
    runs to a state with upstrokes, plateaus and rest side by side."""
    if model == I.MODEL_HH:
        w = I.batched_hh(n_fibers=6, n_min=600, n_max=700, dt=5e-3, onset_max=1.0)
        w = w.subset([0, 1, 2, 3])
        from dataclasses import replace
        return replace(w, dt_0D=1e-3), 400      # 2 ms
    w = I.st57_bundle(n_fibers=3, n_nodes=523, t_end=1.0, onset_max=0.2)
    return w, 1000                             # 0.5 ms


def _active_state(model):
    w, steps = _workload(model)
    s = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
    s.run(0, steps)
    s.sync()
    y = s.get_state()
    return w, s, y, steps


def _random_net(model, seed):
    sizes = SU.SHAPES[model]
    params = M.init_params(sizes, seed)
    rng = np.random.default_rng(seed)
    params = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in params]
    net = F.Mlp(sizes)
    net.set_params(M.flatten(params).astype(np.float32))
    return sizes, params, net


def _scales(model, y, w, seed, out_mag):
    S = y.shape[0]
    rest = O.rest_state(model)
    u = y - rest[:, None]
    rng = np.random.default_rng(seed)
    sd = np.maximum(u.std(axis=1), 1e-3 * np.maximum(np.abs(rest), 1e-3))
    return dict(in_shift=(u.mean(axis=1) + 0.1 * sd * rng.standard_normal(S)).astype(np.float32),
                in_scale=(1.0 / sd).astype(np.float32),
                out_shift=(0.1 * out_mag * rng.standard_normal(S)).astype(np.float32),
                out_scale=out_mag.astype(np.float32),
                res_scale=np.ones(S, dtype=np.float32),
                flag_scale=1.0 / I.AMP_SUPRA)


def _reference_prediction(model, params, sc, y, I_stim, n_in):
    rest = O.rest_state(model)
    S = y.shape[0]
    u = (y - rest[:, None]).astype(np.float32).astype(np.float64)
    X = ((u.T - sc["in_shift"]) * sc["in_scale"])
    if n_in == S + 1:
        X = np.concatenate([X, (I_stim * sc["flag_scale"])[:, None]], axis=1)
    o, _ = M.forward(params, X)
    return o  # normalized outputs, (n_total, S)


def _rhs(model, y, I_stim, Cm):
    f = O.hh_rhs if model == I.MODEL_HH else O.st57_rhs
    return np.stack([f(y[:, j], float(I_stim[j]), Cm) for j in range(y.shape[1])], axis=1)


def _out_mag(model, w, y):
    """Typical increment of each state over one split step (per-state scale of
    the network's outputs in these tests)."""
    G = _rhs(model, y, np.zeros(y.shape[1]), w.Cm)
    return np.maximum(w.dt_split * np.abs(G).mean(axis=1), 1e-9)


@pytest.mark.parametrize("model", [I.MODEL_HH, I.MODEL_ST57])
def test_prediction_matches_reference_network(model):
    say(f"[surrogate predict] model {model}")
    w, s, y, steps = _active_state(model)
    sizes, params, net = _random_net(model, 11 + model)
    sc = _scales(model, y, w, 3, _out_mag(model, w, y))
    s.set_surrogate(net, sc, 1e-3)
    for step in (steps, 0):   # stimulus off / on for the stimulated nodes
        du = s.surrogate_predict(step).cpu().numpy().astype(np.float64)
        I_stim = O.stimulus_current(w.n_nodes, w.stims, step)
        o_ref = _reference_prediction(model, params, sc, y, I_stim, sizes[0])
        o_dev = ((du.T - sc["out_shift"]) / sc["out_scale"])
        err = np.max(np.abs(o_dev - o_ref)) / np.max(np.abs(o_ref))
        say(f"   step {step}: max |o| {np.max(np.abs(o_ref)):.3f}, rel err {err:.2e}, "
            f"stimulated nodes {int(np.sum(I_stim != 0))}")
        assert err < 3e-2
    # the prediction changes no state
    np.testing.assert_array_equal(s.get_state(), y)
    s.close()
    net.close()


@pytest.mark.parametrize("model", [I.MODEL_HH, I.MODEL_ST57])
def test_accepted_step_is_the_midpoint_iteration(model):
    say(f"[surrogate corrected step] model {model}")
    w, s, y, steps = _active_state(model)
    sizes, params, net = _random_net(model, 21 + model)
    sc = _scales(model, y, w, 4, _out_mag(model, w, y))
    s.set_surrogate(net, sc, 1e30)
    step = steps  # no stimulus in either half
    I_stim = O.stimulus_current(w.n_nodes, w.stims, step)
    assert not I_stim.any() and not O.stimulus_current(w.n_nodes, w.stims, step + 1).any()
    s.step_surrogate(step)
    s.sync()
    assert s.last_fallbacks() == 0
    y_dev = s.get_state()
    o = _reference_prediction(model, params, sc, y, I_stim, sizes[0])
    du = (sc["out_shift"] + sc["out_scale"] * o).T
    dt = w.dt_split
    duc = du
    for _ in range(ITERATIONS[model]):
        duc = dt * _rhs(model, y + 0.5 * duc, I_stim, w.Cm)
    y_ref = y + duc
    # FP32 rounding of the states and of G (relative 1e-5 of the state and
    # 2e-3 of the increment), and the BF16 error of the prediction (up to
    # 3e-2 of du) times the corrector's sensitivity: for one iteration its
    # effect is dt/2 dG/dy times that error, taken from the FP64 map
    eps = 3e-2 * np.abs(du).max(axis=1, keepdims=True)
    sens = np.zeros_like(duc)
    if ITERATIONS[model] == 1:
        sens = np.abs(dt * _rhs(model, y + 0.5 * (du + eps * np.sign(du)), I_stim, w.Cm) - duc)
    tol = (1e-5 * np.abs(y).max(axis=1, keepdims=True) + 2e-3 * np.abs(duc).max(axis=1, keepdims=True)
           + 2.0 * np.max(sens, axis=1, keepdims=True) + 1e-30)
    err = np.abs(y_dev - y_ref)
    worst = np.argmax((err / tol).max(axis=1))
    say(f"   max |du_c| V {np.abs(duc[0]).max():.3e}; worst state {worst}: err "
        f"{err[worst].max():.3e} vs tol {tol[worst, 0]:.3e}; V err {err[0].max():.3e}")
    assert np.all(err <= tol)
    s.close()
    net.close()


@pytest.mark.parametrize("model", [I.MODEL_HH, I.MODEL_ST57])
def test_all_rejected_is_bitwise_the_plain_split_run(model):
    say(f"[surrogate all rejected] model {model}")
    w, steps = _workload(model)
    n = min(steps, 300)
    a = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
    a.run(0, n)
    a.sync()
    ya, ta = a.get_state(), a.tact()
    a.close()
    b = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
    sizes, params, net = _random_net(model, 31)
    y0 = b.get_state()
    sc = _scales(model, y0, w, 5, np.full(y0.shape[0], 1e-3))
    b.set_surrogate(net, sc, 1e-30)
    b.run(0, n)
    b.sync()
    assert b.last_fallbacks() == w.n_total
    yb, tb = b.get_state(), b.tact()
    np.testing.assert_array_equal(yb, ya)
    np.testing.assert_array_equal(tb, ta)
    b.close()
    net.close()


def test_rejection_counts_of_consecutive_steps():
    """Each surrogate step counts its own rejections (the two alternating
    counters are cleared one step ahead), also across re-attachment."""
    say("[surrogate rejection counts]")
    w, s, y, steps = _active_state(I.MODEL_HH)
    sizes, params, net = _random_net(I.MODEL_HH, 41)
    sc = _scales(I.MODEL_HH, y, w, 6, _out_mag(I.MODEL_HH, w, y))
    s.set_surrogate(net, sc, 1e-30)          # every node rejected
    for j in range(5):
        s.step_surrogate(steps + j)
        s.sync()
        assert s.last_fallbacks() == w.n_total
    s.set_surrogate(net, sc, 1e30)           # every unstimulated node accepted
    for j in range(3):
        s.step_surrogate(steps + 5 + j)
        s.sync()
        assert s.last_fallbacks() == 0
    s.close()
    net.close()


@pytest.mark.parametrize("model", [I.MODEL_HH, I.MODEL_ST57])
@pytest.mark.parametrize("pred", [F.FIB_PRED_ZERO, F.FIB_PRED_EULER])
def test_closed_form_predictor_step(model, pred):
    """The step with a closed-form predictor and every node accepted is the
    fixed-point iteration of the implicit midpoint rule started from du = 0
    or from the explicit Euler increment du = dt G(y), with the oracle's
    right-hand sides; with every node rejected it is the plain split run
    bit for bit, and the running rejection count is the sum over steps."""
    say(f"[predictor step] model {model} predictor {pred}")
    w, s, y, steps = _active_state(model)
    S = y.shape[0]
    s.set_predictor(pred, np.ones(S, dtype=np.float32), 1e30)
    step = steps
    I_stim = O.stimulus_current(w.n_nodes, w.stims, step)
    assert not I_stim.any() and not O.stimulus_current(w.n_nodes, w.stims, step + 1).any()
    s.step_surrogate(step)
    s.sync()
    assert s.last_fallbacks() == 0 and s.fallbacks() == (0, 1)
    y_dev = s.get_state()
    dt = w.dt_split
    du = dt * _rhs(model, y, I_stim, w.Cm) if pred == F.FIB_PRED_EULER else np.zeros_like(y)
    for _ in range(ITERATIONS[model]):
        du = dt * _rhs(model, y + 0.5 * du, I_stim, w.Cm)
    # FP32 rounding of the states and of the right-hand sides
    tol = (1e-5 * np.abs(y).max(axis=1, keepdims=True) + 2e-3 * np.abs(du).max(axis=1, keepdims=True)
           + 1e-30)
    err = np.abs(y_dev - (y + du))
    say(f"   V err {err[0].max():.3e} (|du_V| up to {np.abs(du[0]).max():.3e}); worst ratio "
        f"{(err / tol).max():.2f}")
    assert np.all(err <= tol)
    with pytest.raises(F.FibError):
        s.surrogate_predict(step)      # no network attached
    s.close()

    n = min(steps, 200)
    a = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
    a.run(0, n)
    a.sync()
    ya, ta = a.get_state(), a.tact()
    a.close()
    b = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
    b.set_predictor(pred, np.ones(S, dtype=np.float32), 1e-30)
    b.run(0, n)
    b.sync()
    np.testing.assert_array_equal(b.get_state(), ya)
    np.testing.assert_array_equal(b.tact(), ta)
    total, k = b.fallbacks()
    # every step but the last of the call takes the surrogate path
    assert k == n - 1 and total == k * w.n_total
    b.close()
