"""Training data of the surrogate, computed in libfib.so.

* fib_column_stats: means and sample standard deviations (FP64 sums, two
  passes) against NumPy's FP64 statistics of the same FP32 data, exact
  minima and maxima; a large common offset must not cost accuracy (the
  second pass sums squared deviations from the mean);
* fib_normalize_rows: bitwise the FP32 (a - shift) * scale NumPy computes,
  the flag column, columns beyond it untouched;
* fib_state_rows: bitwise the transpose of the state;
* fib_reaction_increments: bitwise the increments of two fib_step_reaction
  calls over dt/2 on the same rows (several chunks of n_total rows, a
  ragged last chunk, stimulus off and on), and close to the oracle's FP64
  reaction pair from the same states.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_2107_07104_amd import fib as F
from paper_2107_07104_amd import inputs as I

from gpu_helpers import gpu_solver, oracle_cfg, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.lib()


@pytest.mark.parametrize("rows,cols,offset", [(1, 3, 0.0), (1000, 5, 0.0), (100003, 57, 0.0),
                                              (70001, 4, -80.0), (4097, 64, 1e4)])
def test_column_stats_match_numpy(rows, cols, offset):
    say(f"[column stats rows={rows} cols={cols} offset={offset}]")
    rng = np.random.default_rng(rows + cols)
    A = (offset + rng.standard_normal((rows, cols)) * np.linspace(1e-3, 10, cols)).astype(np.float32)
    mean, std, lo, hi = F.fib_column_stats(torch.from_numpy(A).cuda().data_ptr(), rows, cols)
    A64 = A.astype(np.float64)
    np.testing.assert_allclose(mean, A64.mean(0), rtol=1e-12, atol=1e-12 * (1 + abs(offset)))
    if rows > 1:
        np.testing.assert_allclose(std, A64.std(0, ddof=1), rtol=1e-10, atol=0)
    else:
        assert np.all(std == 0)
    np.testing.assert_array_equal(lo, A.min(0))
    np.testing.assert_array_equal(hi, A.max(0))


def test_column_stats_rejects_bad_shapes():
    x = torch.zeros(10, device="cuda")
    for rows, cols in ((0, 3), (5, 0), (1, 65)):
        with pytest.raises(F.FibError):
            F.fib_column_stats(x.data_ptr(), rows, cols)


@pytest.mark.parametrize("rows,cols,ldy", [(1, 4, 4), (3001, 57, 57), (3001, 4, 5),
                                           (777, 57, 60)])
def test_normalize_rows_is_bitwise_numpy(rows, cols, ldy):
    say(f"[normalize rows={rows} cols={cols} ldy={ldy}]")
    rng = np.random.default_rng(cols)
    A = rng.standard_normal((rows, cols)).astype(np.float32) * 30
    shift = rng.standard_normal(cols).astype(np.float32)
    scale = rng.uniform(0.01, 5, cols).astype(np.float32)
    Y = torch.full((rows, ldy), 7.25, device="cuda")
    F.fib_normalize_rows(torch.from_numpy(A).cuda().data_ptr(), rows, cols, shift, scale, 0.5,
                         Y.data_ptr(), ldy)
    y = Y.cpu().numpy()
    np.testing.assert_array_equal(y[:, :cols], (A - shift) * scale)
    if ldy > cols:
        assert np.all(y[:, cols] == 0.5)
        assert np.all(y[:, cols + 1:] == 7.25)


def _rows_pair(s, U, step, dt_split):
    """Increments by the step-by-step path: load n_total rows into the state,
    two fib_step_reaction calls over dt/2, subtract."""
    st, _ = s.state_tensor()
    n = s.n_total
    out = torch.empty_like(U)
    for a in range(0, U.shape[0], n):
        b = min(a + n, U.shape[0])
        st.zero_()
        st[:, : b - a].copy_(U[a:b].t())
        s.step_reaction(step, 0.5 * dt_split)
        s.step_reaction(step, 0.5 * dt_split)
        torch.cuda.synchronize()
        out[a:b] = st[:, : b - a].t() - U[a:b]
    return out


@pytest.mark.parametrize("model", [I.MODEL_HH, I.MODEL_ST57])
def test_state_rows_and_reaction_increments(model):
    if model == I.MODEL_HH:
        w = replace(I.batched_hh(n_fibers=3, n_min=200, n_max=300, dt=5e-3, onset_max=0.1),
                    dt_0D=1e-3)
    else:
        w = I.st57_bundle(n_fibers=2, n_nodes=300, t_end=0.2, onset_max=0.05)
    say(f"[training rows model={model}]")
    s = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
    s.run(0, 60)
    U1 = torch.empty((s.n_total, s.S), device="cuda")
    F.fib_state_rows(s.ctx, U1.data_ptr())
    st, _ = s.state_tensor()
    torch.cuda.synchronize()
    assert torch.equal(U1, st.t())
    # rows: 2.6 chunks of n_total, from the run's states and scaled copies
    n = s.n_total
    rng = torch.Generator(device="cpu").manual_seed(5)
    idx = torch.randint(0, n, (int(2.6 * n),), generator=rng).cuda()
    U = (U1[idx] * (1.0 + 0.1 * torch.rand(idx.shape[0], 1, generator=rng).cuda())).contiguous()
    for amp, stim in ((0.0, None), (I.AMP_SUPRA, "all")):
        s2 = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
        s3 = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
        stims = [dict(fiber=f, node=0, half_width=int(w.n_nodes[f]), step_on=0, n_steps=1,
                      period=0, amp=amp) for f in range(len(w.n_nodes))] if stim else []
        s2.set_stimulus(stims)
        s3.set_stimulus(stims)
        dU = torch.full_like(U, float("nan"))
        F.fib_reaction_increments(s2.ctx, U.data_ptr(), U.shape[0], 0, dU.data_ptr())
        ref = _rows_pair(s3, U, 0, w.dt_split)
        torch.cuda.synchronize()
        assert torch.equal(dU, ref), (amp, (dU - ref).abs().max().item())
        # against the oracle's FP64 reaction pair on a few rows, from the
        # same start (the library's FP32 reference state plus the row)
        _, ref0 = s2.state_tensor()
        pick = np.array([0, 1, n - 1, n, 2 * n + 3, U.shape[0] - 1])
        u = U[pick].double().cpu().numpy()
        y = np.asarray(ref0, np.float64)[:, None] + u.T
        cfg = oracle_cfg(w)
        Iv = np.full(len(pick), amp)
        y1 = O.reaction(cfg, O.reaction(cfg, y, 0.5 * w.dt_split, Iv), 0.5 * w.dt_split, Iv)
        want = (y1 - y).T
        got = dU[pick].double().cpu().numpy()
        tol = 4e-6 * np.maximum(np.abs(u), np.abs(ref0)[None, :]) + 2e-4 * np.abs(want) + 1e-9
        ratio = np.abs(got - want) / tol
        say(f"   amp {amp}: worst state {int(np.argmax(ratio.max(0)))} ratio {ratio.max():.3f}")
        assert ratio.max() <= 1.0
        s2.close()
        s3.close()
    s.close()
