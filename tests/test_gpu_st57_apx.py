"""ST57 with the thesis's exp* and log* (eq. apx-e-function, figure apxlog)
on the GPU against the FP64 oracle of the same model.

* reaction steps from perturbed, partly depolarized states: within the
  FP32 tolerance of the exact ST57 reaction test, doubled for the ten
  squarings of each exp* and the Taylor/Newton arithmetic of each log*;
* a whole run stays within the method's budget (0.5 mV over all samples and
  the final state, activation times within one split step) of the oracle's
  exp*/log* model, while that model departs from the exact ST57 by far more
  than the parity error, so the approximate functions are the ones computed;
* adaptive computation and the fused schedule refuse the model.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_2107_07104_amd import fib as F
from paper_2107_07104_amd import inputs as I

from gpu_helpers import compare_runs, gpu_run, oracle_cfg, oracle_init, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

APX = F.FIB_MODEL_ST57_APX


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.lib()


def test_st57_apx_reaction_matches_oracle():
    say("[st57 apx reaction]")
    rest = O.rest_state(O.MODEL_ST57_APX)
    rng = np.random.default_rng(31)
    n = [300, 5, 700]
    N = sum(n)
    y0 = rest[:, None] * (1 + 0.01 * rng.standard_normal((57, N)))
    y0[0] += rng.uniform(-5, 100, N)
    y0[4] += rng.uniform(-5, 60, N)
    stims = [dict(fiber=2, node=100, half_width=3, step_on=0, n_steps=4, period=0, amp=900.0)]
    s = F.Solver(n, model=APX, dt_0D=1e-4, dt_1D=5e-4, dt_split=5e-4)
    s.set_stimulus(stims)
    s.set_state(y0)
    y0f = s.get_state()
    cfg = O.Config(model=O.MODEL_ST57_APX, dt_0D=1e-4)
    yo = y0f
    for step in range(4):
        s.step_reaction(step, 2.5e-4)
        yo = O.reaction(cfg, yo, 2.5e-4, O.stimulus_current(n, stims, step))
    s.sync()
    yg = s.get_state()
    tol = (4e-6 * np.maximum(np.abs(y0f - rest[:, None]), np.abs(rest)[:, None])
           + 2e-4 * np.abs(yo - y0f) + 1e-9)
    ratio = np.abs(yg - yo) / tol
    say("   worst state", int(np.argmax(np.max(ratio, axis=1))), "ratio", float(ratio.max()),
        "V err", float(np.max(np.abs(yg[0] - yo[0]))))
    assert not (ratio > 1).any()
    s.close()


def test_st57_apx_run_matches_oracle_and_departs_from_exact():
    w = replace(I.st57_bundle(n_fibers=4, n_nodes=600, t_end=3.0, onset_max=0.5), model=APX)
    say(f"[st57 apx run] steps={w.n_steps}")
    ora = O.run(oracle_cfg(w), w.n_nodes, oracle_init(w), w.stims, w.n_steps,
                sample_every=w.sample_every)
    we = replace(w, model=O.MODEL_ST57)
    exact = O.run(oracle_cfg(we), we.n_nodes, oracle_init(we), we.stims, we.n_steps,
                  sample_every=we.sample_every)
    gpu = gpu_run(w)
    res = compare_runs(w, gpu, ora)
    gap = compare_runs(w, gpu, exact)
    say("   vs oracle exp*/log* ", res)
    say("   vs oracle exact     ", gap)
    assert res["vm_err"] <= 0.5 and res["tact_err"] <= w.dt_split and res["tact_mismatch"] == 0
    assert res["tact_err"] <= 0.01 * w.dt_split
    assert res["activated"] > 300
    assert gap["vm_err"] > 20 * res["vm_err"]
    gpu[3].close()


def test_st57_apx_refuses_adaptive_and_fused():
    s = F.Solver([50], model=APX, dt_0D=1e-4, dt_1D=5e-4, dt_split=5e-4)
    s.init_state()
    with pytest.raises(F.FibError):
        s.set_adaptive(1e-5)
    s.close()
    s = F.Solver([50], model=APX, schedule=F.FIB_SCHED_FUSED, dt_0D=1e-4, dt_1D=5e-4,
                 dt_split=5e-4)
    s.init_state()
    with pytest.raises(F.FibError):
        s.run(0, 2)
    s.close()
