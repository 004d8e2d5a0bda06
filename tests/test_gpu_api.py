"""Entry points of the C ABI not covered by the parity suites, on the GPU:

* fib_reset_observables sets every activation time back to +inf and leaves
  the state alone; crossings after it are recorded again, and only those;
* fib_state_device gives a zero-copy view of the FP32 state: the view plus
  the reference it reports is fib_get_state's FP64 state, and a write
  through the view is what the next run starts from;
* fib_clear_surrogate detaches the network: a run after it is bitwise the
  plain split run;
* fib_mlp_reset_optimizer clears the Adam moments and step count: the next
  step is the first-step closed form p - lr g / (|g| + eps) again.
"""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2107_07104_amd import fib as F
from paper_2107_07104_amd import inputs as I
from paper_2107_07104_amd import surrogate as SU

from gpu_helpers import gpu_solver, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.lib()


def _bundle():
    return I.batched_hh(n_fibers=3, n_min=200, n_max=260, t_end=3.0, onset_max=0.2)


def test_reset_observables():
    w = _bundle()
    w.stims[0]["step_on"] = 0
    w.stims[1]["step_on"] = 1200
    w.stims[2]["step_on"] = 10 ** 6
    s = gpu_solver(w)
    s.run(0, 1000)
    s.sync()
    t1 = s.tact()
    off = w.offsets
    f0, f1 = slice(off[0], off[1]), slice(off[1], off[2])
    before = np.isfinite(t1)
    assert before[f0].sum() > 10 and not before[f1].any()
    y = s.get_state()
    F.fib_reset_observables(s.ctx)
    assert np.all(np.isinf(s.tact()))
    np.testing.assert_array_equal(s.get_state(), y)
    s.run(1000, 1500)
    s.sync()
    t2 = s.tact()
    fin = np.isfinite(t2)
    say(f"[reset observables] {before.sum()} crossings before the reset, {fin.sum()} after")
    # only crossings after the reset: fiber 1's, and fiber 0's front further out
    assert np.all(t2[fin] >= 1000 * w.dt_split)
    assert fin[f1].sum() > 10
    assert not fin[before].any()
    s.close()


def test_state_device_view():
    w = _bundle()
    s = gpu_solver(w)
    s.run(0, 300)
    s.sync()
    view, ref = s.state_tensor()
    y = s.get_state()
    v = view.cpu().numpy().astype(np.float64).reshape(y.shape)
    np.testing.assert_array_equal(v + ref[:, None], y)
    # a prescribed V_m written through the view is the next run's start
    view.view(y.shape)[0, 5] += 30.0
    torch.cuda.synchronize()
    y2 = s.get_state()
    assert y2[0, 5] == pytest.approx(y[0, 5] + 30.0, abs=1e-4)
    a = gpu_solver(w)
    a.set_state(y2)
    for r in (s, a):
        r.run(300, 200)
        r.sync()
    np.testing.assert_array_equal(s.get_state(), a.get_state())
    s.close()
    a.close()


def test_clear_surrogate_restores_the_plain_run():
    from dataclasses import replace
    w = replace(I.batched_hh(n_fibers=3, n_min=200, n_max=260, dt=5e-3, onset_max=0.2),
                dt_0D=1e-3)
    sizes = SU.SHAPES[I.MODEL_HH]
    net = F.Mlp(sizes)
    net.set_params(M.flatten(M.init_params(sizes, 3)).astype(np.float32))
    S = 4
    sc = dict(in_shift=np.zeros(S, np.float32), in_scale=np.ones(S, np.float32),
              out_shift=np.zeros(S, np.float32), out_scale=np.full(S, 1e-3, np.float32),
              res_scale=np.ones(S, np.float32), flag_scale=1.0 / I.AMP_SUPRA)
    s = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
    s.set_surrogate(net, sc, 1e-2)
    s.run(0, 20)
    s.clear_surrogate()
    p = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
    p.set_state(s.get_state())
    for r in (s, p):
        r.run(20, 100)
        r.sync()
    np.testing.assert_array_equal(s.get_state(), p.get_state())
    s.close()
    p.close()
    net.close()


def test_reset_optimizer():
    sizes = [5, 64, 64, 64, 4]
    net = F.Mlp(sizes)
    net.set_params(M.flatten(M.init_params(sizes, 5)).astype(np.float32))
    rng = np.random.default_rng(6)
    X = torch.as_tensor(rng.standard_normal((2048, 5)), dtype=torch.float32, device="cuda")
    T = torch.as_tensor(rng.standard_normal((2048, 4)), dtype=torch.float32, device="cuda")
    for _ in range(5):
        net.adam_step(X, T, 1e-3)
    net.reset_optimizer()
    g, _ = net.gradient(X, T)
    g = g.cpu().numpy().astype(np.float64)
    p0 = net.get_params().astype(np.float64)
    net.adam_step(X, T, 1e-3)
    p1 = net.get_params().astype(np.float64)
    expect = p0 - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p1, expect, rtol=1e-5, atol=1e-7)
    net.close()
