"""Host-side checks of libfib.so that need no GPU: the library loads, it
exports every function include/fib.h declares, argument checking rejects bad
parameters, and the library's own resting-state search (Newton's method)
agrees with the oracle's (bisection), which is an independent
implementation."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2107_07104_amd import fib as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "fib.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fib_[a-z_0-9]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_function():
    L = F.lib()
    names = _declared()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    assert sorted(F.EXPORTS) == names


def test_n_states():
    assert F.fib_n_states(F.FIB_MODEL_HH) == 4
    assert F.lib().fib_n_states(99) == F.FIB_EINVAL
    assert "unknown model" in F.fib_last_error()


@pytest.mark.parametrize("field,value", [
    ("Cm", 0.0), ("Am", -1.0), ("h", float("nan")), ("sigma", -0.1), ("dt_0D", 0.0),
    ("dt_1D", float("inf")), ("dt_split", -1e-3), ("v_th", float("nan")),
    ("threads_per_group", 96), ("threads_per_group", 2048), ("nodes_per_thread", 1),
    ("nodes_per_thread", 15), ("groups", -1), ("model", 7), ("model", 4), ("schedule", 3),
    ("splitting", 2), ("time_1d", 2), ("time_1d", -1), ("tune", 2), ("tune", -1)])
def test_check_params_rejects(field, value):
    p = F.make_params()
    setattr(p, field, value)
    assert F.fib_check_params(p) == F.FIB_EINVAL
    assert F.fib_last_error() != ""


def test_check_params_accepts_defaults():
    assert F.fib_check_params(F.make_params()) == F.FIB_OK
    for split in (F.FIB_SPLIT_STRANG, F.FIB_SPLIT_GODUNOV):
        for t1 in (F.FIB_1D_CRANK_NICOLSON, F.FIB_1D_IMPLICIT_EULER):
            assert F.fib_check_params(F.make_params(splitting=split, time_1d=t1)) == F.FIB_OK
    assert F.fib_check_params(F.make_params(tune=1)) == F.FIB_OK


def test_implicit_euler_matrix_couples_more_strongly():
    """The implicit-Euler matrix I - dt L has twice the off-diagonal weight of
    the Crank-Nicolson matrix I - dt L / 2, so the reduced system keeps its
    couplings above 2^-40 over at least as many PCR levels."""
    n = [1000] * 8
    for dt in (1e-3, 0.05, 0.5):
        p = dict(dt_split=dt, dt_1D=dt, nodes_per_thread=2)
        cn = F.fib_plan_preview(F.make_params(**p), n, 8)
        ie = F.fib_plan_preview(F.make_params(time_1d=F.FIB_1D_IMPLICIT_EULER, **p), n, 8)
        assert ie["pcr_levels"] >= cn["pcr_levels"] > 0
    assert ie["pcr_levels"] > cn["pcr_levels"]   # dt = 0.5 ms: one more level


@pytest.mark.parametrize("threads,k,ok", [(768, 9, True), (960, 7, True), (512, 14, True),
                                          (1024, 9, False), (832, 10, False), (576, 12, False)])
def test_workgroup_shapes_follow_the_built_kernels(threads, k, ok):
    """Workgroup sizes are multiples of 64; 9-10 nodes per thread allow at most
    768 threads and 11-14 at most 512 (the kernels' register budgets)."""
    p = F.make_params(threads_per_group=threads, nodes_per_thread=k)
    assert (F.fib_check_params(p) == F.FIB_OK) == ok
    if ok:
        plan = F.fib_plan_preview(p, [threads * k // 2] * 3, 256)
        assert plan["threads"] == threads and plan["nodes_per_thread"] == k
    assert F.fib_check_params(F.make_params(threads_per_group=64, nodes_per_thread=8)) == F.FIB_OK


def test_rest_state_agrees_with_oracle():
    y_lib = F.fib_rest_state(F.make_params())
    y_or = O.rest_state()
    np.testing.assert_allclose(y_lib, y_or, rtol=0, atol=1e-10)
    # the membrane with exp* (eq. apx-e-function) has a rest state of its own
    y_apx = F.fib_rest_state(F.make_params(model=F.FIB_MODEL_HH_APX_EXP))
    np.testing.assert_allclose(y_apx, O.rest_state(O.MODEL_HH_APX_EXP), rtol=0, atol=1e-10)
    assert abs(y_apx[0] - y_lib[0]) > 1e-5
    # ST57 with exp* and log*: the library's Newton against the oracle's
    y57 = F.fib_rest_state(F.make_params(model=F.FIB_MODEL_ST57_APX))
    r57 = O.rest_state(O.MODEL_ST57_APX)
    np.testing.assert_allclose(y57, r57, rtol=1e-9, atol=1e-9)
    assert abs(y57[0] - O.rest_state(O.MODEL_ST57)[0]) > 1e-4


def test_create_rejects_bad_fibers_without_touching_the_gpu():
    out = F._vp()
    nn = np.array([5, 0, 3], dtype=np.int32)
    rc = F.lib().fib_create(F.C.byref(F.make_params()), 3, nn.ctypes.data_as(F._i32p), None,
                            F.C.byref(out))
    assert rc == F.FIB_EINVAL and out.value is None
    assert "fiber 1" in F.fib_last_error()


def test_plan_preview_packs_fibers_tightly():
    from paper_2107_07104_amd import inputs as I
    w = I.batched_hh()
    plan = F.fib_plan_preview(F.make_params(), w.n_nodes, 256)
    avg = w.n_total / 256
    assert plan["groups"] == 256
    assert plan["max_load"] <= avg + 10  # near-perfect multiway partition
    assert plan["threads"] * plan["nodes_per_thread"] >= plan["max_load"]
    assert plan["nodes_per_thread"] == 7 and plan["threads"] == 1024
    # one fiber: one bin, all threads of the bin busy
    one = F.fib_plan_preview(F.make_params(), [1000], 256)
    assert one["groups"] == 1 and one["threads"] * one["nodes_per_thread"] >= 1000
    # the longest fiber a workgroup holds (1024 threads x 8 nodes), and one more node
    big = F.fib_plan_preview(F.make_params(), [8192, 100], 256)
    assert big["threads"] * big["nodes_per_thread"] >= 8192
    for n in (8193, 9000):
        with pytest.raises(F.FibError) as e:
            F.fib_plan_preview(F.make_params(), [n], 256)
        assert e.value.code == F.FIB_EUNSUPPORTED
