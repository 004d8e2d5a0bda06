"""Graph replay of the split schedule against step-by-step launches.

fib_run captures one block of split steps per call and replays it; the
replays must give bitwise the results of the same kernels launched one by
one.  Each case runs two contexts on the same inputs, one with graphs off,
through several fib_run calls whose boundaries fall inside and between
blocks, with the program's own synchronizing work (a state read-back)
between the calls, and compares states, activation times and V_m samples
after every call; the graph path must actually have been replayed.
"""
from dataclasses import replace

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


def _attach(s, kind, model, net=None):
    S = 4 if model == I.MODEL_HH else 57
    if kind == "network":
        sc = dict(in_shift=np.zeros(S, np.float32), in_scale=np.ones(S, np.float32),
                  out_shift=np.zeros(S, np.float32), out_scale=np.full(S, 1e-3, np.float32),
                  res_scale=np.ones(S, np.float32), flag_scale=1.0 / I.AMP_SUPRA)
        # a moderate tolerance: some nodes are accepted, the rest fall back
        s.set_surrogate(net, sc, 2e-3)
    elif kind == "euler":
        s.set_predictor(F.FIB_PRED_EULER, np.ones(S, np.float32), 1e-3)


def _net(model):
    sizes = SU.SHAPES[model]
    params = [(W, 0.05 * b) for W, b in M.init_params(sizes, seed=3)]
    net = F.Mlp(sizes, act=SU.ACTIVATION[model])
    net.set_params(M.flatten(params).astype(np.float32))
    return net


def _case(w, kind, calls, sample_every):
    net = _net(w.model) if kind == "network" else None
    runs = {}
    for graphs in (False, True):
        s = gpu_solver(w, schedule=F.FIB_SCHED_SPLIT)
        s.set_graphs(graphs)
        _attach(s, kind, w.model, net)
        runs[graphs] = s
    step = 0
    rows_total = sum(calls) // sample_every if sample_every else 0
    smp = {g: torch.full((max(rows_total, 1), w.n_total), float("nan"), device="cuda")
           for g in (False, True)}
    row = 0
    for n in calls:
        rows = (step + n) // sample_every - step // sample_every if sample_every else 0
        for g, s in runs.items():
            s.run(step, n, sample_every, smp[g][row:row + rows] if rows else None)
        ys = {g: s.get_state() for g, s in runs.items()}
        np.testing.assert_array_equal(ys[True], ys[False])
        np.testing.assert_array_equal(runs[True].tact(), runs[False].tact())
        if kind != "plain":
            assert runs[True].fallbacks() == runs[False].fallbacks()
            assert runs[True].last_fallbacks() == runs[False].last_fallbacks()
        step += n
        row += rows
    if rows_total:
        np.testing.assert_array_equal(smp[True].cpu().numpy(), smp[False].cpu().numpy())
    replays = runs[True].graph_replays()
    assert runs[False].graph_replays() == 0
    for s in runs.values():
        s.close()
    if net is not None:
        net.close()
    return replays


@pytest.mark.parametrize("kind", ["plain", "network", "euler"])
def test_hh_graph_replay_is_bitwise_the_launch_sequence(kind):
    w = replace(I.batched_hh(n_fibers=12, n_min=300, n_max=500, dt=5e-3, onset_max=0.3),
                dt_0D=1e-3)
    say(f"[graph hh {kind}]")
    # sample interval 20 (0.1 ms): blocks of 40 steps; calls of uneven length
    reps = _case(w, kind, [133, 57, 200, 81, 40], 20)
    say(f"   graph replays {reps}")
    assert reps >= 8


def test_graph_replay_without_samples_and_odd_interval():
    w = replace(I.batched_hh(n_fibers=5, n_min=200, n_max=260, dt=5e-3, onset_max=0.2),
                dt_0D=1e-3)
    say("[graph hh no samples / odd interval]")
    assert _case(w, "plain", [150, 140, 64], 0) >= 3        # blocks of 64
    assert _case(w, "network", [100, 99], 7) >= 10          # blocks of 7


def test_st57_graph_replay_is_bitwise_the_launch_sequence():
    w = I.st57_bundle(n_fibers=3, n_nodes=500, t_end=0.5, onset_max=0.05)
    say("[graph st57]")
    for kind in ("plain", "euler"):
        assert _case(w, kind, [450, 330, 220], 200) >= 1
