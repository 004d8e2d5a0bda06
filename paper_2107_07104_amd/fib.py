"""ctypes binding of libfib.so (the C ABI in include/fib.h).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  Device arrays are passed as raw pointers, normally taken from
torch CUDA tensors (``tensor.data_ptr()``); the stream is a raw
``hipStream_t`` (``torch.cuda.current_stream().cuda_stream``).

The library is loaded on first use; if ``libfib.so`` has not been built the
loader raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfib.so")

FIB_OK = 0
FIB_EINVAL = -1
FIB_ENOMEM = -2
FIB_EHIP = -3
FIB_ENONFINITE = -4
FIB_ESTATE = -5
FIB_EUNSUPPORTED = -6

FIB_MODEL_HH = 0
FIB_MODEL_ST57 = 1
FIB_MODEL_HH_APX_EXP = 2
FIB_MODEL_ST57_APX = 3
FIB_ACT_SILU = 0
FIB_ACT_RELU = 1
ACTS = {"silu": FIB_ACT_SILU, "relu": FIB_ACT_RELU}
FIB_SCHED_AUTO = 0
FIB_SCHED_FUSED = 1
FIB_SCHED_SPLIT = 2
FIB_SPLIT_STRANG = 0
FIB_SPLIT_GODUNOV = 1
FIB_1D_CRANK_NICOLSON = 0
FIB_1D_IMPLICIT_EULER = 1
FIB_STIM_CURRENT = 0
FIB_STIM_VOLTAGE = 1
FIB_PRED_NETWORK = 0
FIB_PRED_ZERO = 1
FIB_PRED_EULER = 2
FIB_KT_FUSED = 0
FIB_KT_REACTION = 1
FIB_KT_DIFFUSION = 2
FIB_KT_SURROGATE = 3
FIB_KT_FALLBACK = 4
FIB_PROBE_FMA = 0
FIB_PROBE_EXP = 1
FIB_PROBE_RCP = 2
FIB_PROBE_LOG = 3
FIB_PROBE_COPY = 4
FIB_PROBE_MFMA_BF16 = 5
FIB_PROBE_FMA_VOP3 = 6

# Every function the header declares, for the export check.
EXPORTS = (
    "fib_n_states", "fib_rest_state", "fib_check_params", "fib_create", "fib_destroy",
    "fib_last_error", "fib_n_total", "fib_init_state", "fib_set_state", "fib_get_state",
    "fib_state_device", "fib_set_stimulus", "fib_step_reaction", "fib_step_diffusion",
    "fib_run", "fib_get_tact", "fib_reset_observables", "fib_sync", "fib_plan_info",
    "fib_plan_preview", "fib_mlp_create", "fib_mlp_destroy", "fib_mlp_n_params",
    "fib_mlp_set_params", "fib_mlp_get_params", "fib_mlp_forward", "fib_mlp_gradient",
    "fib_mlp_adam_step", "fib_mlp_reset_optimizer", "fib_mlp_gradient_noalloc",
    "fib_set_surrogate", "fib_clear_surrogate",
    "fib_surrogate_last_fallbacks", "fib_step_surrogate", "fib_surrogate_fallbacks",
    "fib_set_predictor", "fib_set_kernel_timing", "fib_kernel_time", "fib_probe",
    "fib_set_graphs", "fib_graph_replays", "fib_column_stats", "fib_normalize_rows",
    "fib_state_rows", "fib_reaction_increments",
    "fib_surrogate_predict", "fib_autotune", "fib_set_adaptive", "fib_adaptive_solved",
    "fib_adaptive_points", "fib_emg_create", "fib_emg_destroy", "fib_emg_dims",
    "fib_emg_solve", "fib_emg_get_phi", "fib_emg_get_rhs",
)


class fib_params(C.Structure):
    _fields_ = [("model", C.c_int32), ("schedule", C.c_int32), ("Cm", C.c_double),
                ("Am", C.c_double), ("sigma", C.c_double), ("h", C.c_double),
                ("dt_0D", C.c_double), ("dt_1D", C.c_double), ("dt_split", C.c_double),
                ("v_th", C.c_double), ("pcr_full", C.c_int32),
                ("threads_per_group", C.c_int32), ("nodes_per_thread", C.c_int32),
                ("groups", C.c_int32), ("splitting", C.c_int32), ("time_1d", C.c_int32),
                ("tune", C.c_int32)]


class fib_stim(C.Structure):
    _fields_ = [("fiber", C.c_int32), ("node", C.c_int32), ("half_width", C.c_int32),
                ("mode", C.c_int32), ("step_on", C.c_int64), ("n_steps", C.c_int64),
                ("period", C.c_int64), ("amp", C.c_double)]


class fib_emg_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("stride", C.c_int32),
                ("hx", C.c_double), ("hy", C.c_double), ("sigma_i", C.c_double),
                ("sigma_el", C.c_double), ("sigma_et", C.c_double)]


class FibError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libfib error {code}: {msg}")
        self.code = code


_lib = None
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_i32p = C.POINTER(C.c_int32)


def lib():
    """Loads libfib.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run "
                              "python -m paper_2107_07104_amd.csrc.build")
        L = C.CDLL(LIB_PATH)
        sig = {
            "fib_n_states": ([C.c_int32], C.c_int),
            "fib_rest_state": ([C.POINTER(fib_params), _dp], C.c_int),
            "fib_check_params": ([C.POINTER(fib_params)], C.c_int),
            "fib_create": ([C.POINTER(fib_params), C.c_int32, _i32p, _vp, C.POINTER(_vp)], C.c_int),
            "fib_destroy": ([_vp], None),
            "fib_last_error": ([], C.c_char_p),
            "fib_n_total": ([_vp], C.c_int64),
            "fib_init_state": ([_vp, _vp, _vp], C.c_int),
            "fib_set_state": ([_vp, _dp, C.c_int64], C.c_int),
            "fib_get_state": ([_vp, _dp, C.c_int64], C.c_int),
            "fib_state_device": ([_vp, C.POINTER(_vp), _dp], C.c_int),
            "fib_set_stimulus": ([_vp, C.POINTER(fib_stim), C.c_int32], C.c_int),
            "fib_step_reaction": ([_vp, C.c_int64, C.c_double], C.c_int),
            "fib_step_diffusion": ([_vp, C.c_double], C.c_int),
            "fib_run": ([_vp, C.c_int64, C.c_int64, C.c_int64, _vp, C.c_int64], C.c_int),
            "fib_get_tact": ([_vp, _fp, C.c_int64], C.c_int),
            "fib_reset_observables": ([_vp], C.c_int),
            "fib_sync": ([_vp], C.c_int),
            "fib_plan_info": ([_vp, _i32p, _i32p, _i32p, _i32p], C.c_int),
            "fib_autotune": ([_vp, C.c_int32, C.c_int32, C.POINTER(C.c_double)], C.c_int),
            "fib_plan_preview": ([C.POINTER(fib_params), C.c_int32, _i32p, C.c_int32, _i32p, _i32p,
                                  _i32p, _i32p, C.POINTER(C.c_int64)], C.c_int),
        }
        sig.update({
            "fib_mlp_create": ([C.c_int32, _i32p, C.c_int32, _vp, C.POINTER(_vp)], C.c_int),
            "fib_mlp_destroy": ([_vp], None),
            "fib_mlp_n_params": ([_vp], C.c_int64),
            "fib_mlp_set_params": ([_vp, _fp, C.c_int64], C.c_int),
            "fib_mlp_get_params": ([_vp, _fp, C.c_int64], C.c_int),
            "fib_mlp_forward": ([_vp, _vp, C.c_int64, _vp], C.c_int),
            "fib_mlp_gradient": ([_vp, _vp, _vp, C.c_int64, _vp, _vp], C.c_int),
            "fib_mlp_gradient_noalloc": ([_vp, _vp, _vp, C.c_int64, _vp, _vp], C.c_int),
            "fib_mlp_adam_step": ([_vp, _vp, _vp, C.c_int64, C.c_double, _vp], C.c_int),
            "fib_mlp_reset_optimizer": ([_vp], C.c_int),
            "fib_set_surrogate": ([_vp, _vp, _fp, _fp, _fp, _fp, _fp, C.c_double, C.c_double],
                                  C.c_int),
            "fib_clear_surrogate": ([_vp], C.c_int),
            "fib_step_surrogate": ([_vp, C.c_int64], C.c_int),
            "fib_surrogate_predict": ([_vp, C.c_int64, _vp], C.c_int),
            "fib_surrogate_last_fallbacks": ([_vp, C.POINTER(C.c_int64)], C.c_int),
            "fib_surrogate_fallbacks": ([_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
                                        C.c_int),
            "fib_set_predictor": ([_vp, C.c_int32, _fp, C.c_double], C.c_int),
            "fib_set_kernel_timing": ([_vp, C.c_int32], C.c_int),
            "fib_set_graphs": ([_vp, C.c_int32], C.c_int),
            "fib_column_stats": ([_vp, C.c_int64, C.c_int32, _vp, _dp, _dp, _fp, _fp], C.c_int),
            "fib_normalize_rows": ([_vp, C.c_int64, C.c_int32, _fp, _fp, C.c_double, _vp,
                                    C.c_int32, _vp], C.c_int),
            "fib_state_rows": ([_vp, _vp], C.c_int),
            "fib_reaction_increments": ([_vp, _vp, C.c_int64, C.c_int64, _vp], C.c_int),
            "fib_graph_replays": ([_vp, C.POINTER(C.c_int64)], C.c_int),
            "fib_kernel_time": ([_vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
                                C.c_int),
            "fib_probe": ([C.c_int32, C.c_int64, C.POINTER(C.c_double)], C.c_int),
            "fib_set_adaptive": ([_vp, C.c_double], C.c_int),
            "fib_adaptive_solved": ([_vp, C.POINTER(C.c_int64)], C.c_int),
            "fib_adaptive_points": ([_vp, _vp, C.c_int64], C.c_int),
            "fib_emg_create": ([_vp, C.POINTER(fib_emg_params), C.POINTER(_vp)], C.c_int),
            "fib_emg_destroy": ([_vp], None),
            "fib_emg_dims": ([_vp, _i32p, _i32p, _i32p], C.c_int),
            "fib_emg_solve": ([_vp, C.c_double, C.c_int32, _i32p, C.POINTER(C.c_double)],
                              C.c_int),
            "fib_emg_get_phi": ([_vp, _dp, C.c_int64], C.c_int),
            "fib_emg_get_rhs": ([_vp, _dp, C.c_int64], C.c_int),
        })
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != FIB_OK:
        raise FibError(rc, lib().fib_last_error().decode())
    return rc


def make_params(model=FIB_MODEL_HH, schedule=FIB_SCHED_AUTO, Cm=1.0, Am=500.0, sigma=3.828,
                h=0.01, dt_0D=1e-3, dt_1D=1e-3, dt_split=1e-3, v_th=-20.0, pcr_full=0,
                threads_per_group=0, nodes_per_thread=0, groups=0, splitting=0,
                time_1d=0, tune=0) -> fib_params:
    return fib_params(model, schedule, Cm, Am, sigma, h, dt_0D, dt_1D, dt_split, v_th,
                      pcr_full, threads_per_group, nodes_per_thread, groups, splitting,
                      time_1d, tune)


def _stim_array(stims):
    arr = (fib_stim * max(len(stims), 1))()
    for i, s in enumerate(stims):
        arr[i] = fib_stim(int(s["fiber"]), int(s["node"]), int(s.get("half_width", 1)),
                          int(s.get("mode", FIB_STIM_CURRENT)),
                          int(s["step_on"]), int(s["n_steps"]), int(s.get("period", 0)),
                          float(s["amp"]))
    return arr


# ---- functions with the C names ------------------------------------------------

def fib_n_states(model: int) -> int:
    rc = lib().fib_n_states(model)
    _check(min(rc, 0))
    return rc


def fib_rest_state(params: fib_params) -> np.ndarray:
    y = np.zeros(fib_n_states(params.model))
    _check(lib().fib_rest_state(C.byref(params), y.ctypes.data_as(_dp)))
    return y


def fib_check_params(params: fib_params) -> int:
    return lib().fib_check_params(C.byref(params))


def fib_create(params: fib_params, n_nodes, stream=None) -> int:
    nn = np.ascontiguousarray(n_nodes, dtype=np.int32)
    out = _vp()
    _check(lib().fib_create(C.byref(params), len(nn), nn.ctypes.data_as(_i32p),
                            _vp(stream) if stream else None, C.byref(out)))
    return out.value


def fib_destroy(ctx) -> None:
    lib().fib_destroy(_vp(ctx))


def fib_last_error() -> str:
    return lib().fib_last_error().decode()


def fib_n_total(ctx) -> int:
    return lib().fib_n_total(_vp(ctx))


def fib_init_state(ctx, vm_noise_ptr=0, rel_noise_ptr=0) -> None:
    _check(lib().fib_init_state(_vp(ctx), _vp(vm_noise_ptr or None), _vp(rel_noise_ptr or None)))


def fib_set_state(ctx, y: np.ndarray) -> None:
    y = np.ascontiguousarray(y, dtype=np.float64)
    _check(lib().fib_set_state(_vp(ctx), y.ctypes.data_as(_dp), y.size))


def fib_get_state(ctx, n_states: int) -> np.ndarray:
    n = fib_n_total(ctx)
    y = np.zeros((n_states, n))
    _check(lib().fib_get_state(_vp(ctx), y.ctypes.data_as(_dp), y.size))
    return y


def fib_state_device(ctx, n_states: int):
    """(device pointer of the FP32 state, ref); row k holds y_k - ref[k]."""
    p = _vp()
    ref = np.zeros(n_states)
    _check(lib().fib_state_device(_vp(ctx), C.byref(p), ref.ctypes.data_as(_dp)))
    return p.value, ref


def fib_set_stimulus(ctx, stims) -> None:
    arr = _stim_array(stims)
    _check(lib().fib_set_stimulus(_vp(ctx), arr, len(stims)))


def fib_step_reaction(ctx, step: int, span: float) -> None:
    _check(lib().fib_step_reaction(_vp(ctx), int(step), float(span)))


def fib_step_diffusion(ctx, span: float) -> None:
    _check(lib().fib_step_diffusion(_vp(ctx), float(span)))


def fib_run(ctx, step0: int, n_steps: int, sample_every: int = 0, samples_ptr=0,
            sample_rows: int = 0) -> None:
    _check(lib().fib_run(_vp(ctx), int(step0), int(n_steps), int(sample_every),
                         _vp(samples_ptr or None), int(sample_rows)))


def fib_get_tact(ctx) -> np.ndarray:
    n = fib_n_total(ctx)
    t = np.zeros(n, dtype=np.float32)
    _check(lib().fib_get_tact(_vp(ctx), t.ctypes.data_as(_fp), n))
    return t


def fib_set_adaptive(ctx, tol: float) -> None:
    _check(lib().fib_set_adaptive(_vp(ctx), float(tol)))


def fib_adaptive_solved(ctx) -> int:
    n = C.c_int64(0)
    _check(lib().fib_adaptive_solved(_vp(ctx), C.byref(n)))
    return int(n.value)


def fib_adaptive_points(ctx) -> np.ndarray:
    n = fib_n_total(ctx)
    a = np.zeros(max(n, 1), dtype=np.uint8)
    _check(lib().fib_adaptive_points(_vp(ctx), a.ctypes.data_as(_vp), n))
    return a[:n]


def fib_emg_create(ctx, nx, ny, stride, hx, hy, sigma_i, sigma_el, sigma_et):
    p = fib_emg_params(int(nx), int(ny), int(stride), float(hx), float(hy), float(sigma_i),
                       float(sigma_el), float(sigma_et))
    out = _vp()
    _check(lib().fib_emg_create(_vp(ctx), C.byref(p), C.byref(out)))
    return out


def fib_emg_destroy(emg) -> None:
    lib().fib_emg_destroy(emg)


def fib_emg_dims(emg):
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().fib_emg_dims(emg, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def fib_emg_solve(emg, tol: float, max_iter: int):
    it, rr = C.c_int32(0), C.c_double(0.0)
    _check(lib().fib_emg_solve(emg, float(tol), int(max_iter), C.byref(it), C.byref(rr)))
    return it.value, rr.value


def fib_emg_get_phi(emg, n: int) -> np.ndarray:
    out = np.zeros(n)
    _check(lib().fib_emg_get_phi(emg, out.ctypes.data_as(_dp), n))
    return out


def fib_emg_get_rhs(emg, n: int) -> np.ndarray:
    out = np.zeros(n)
    _check(lib().fib_emg_get_rhs(emg, out.ctypes.data_as(_dp), n))
    return out


class Emg:
    """Static bidomain (EMG) solve attached to a Solver's fiber bundle."""

    def __init__(self, solver, nx, ny, stride, hx, hy, sigma_i=8.93, sigma_el=6.7,
                 sigma_et=3.35):
        self.solver = solver
        self.h = fib_emg_create(solver.ctx, nx, ny, stride, hx, hy, sigma_i, sigma_el, sigma_et)
        self.dims = fib_emg_dims(self.h)
        self.n = self.dims[0] * self.dims[1] * self.dims[2]

    def solve(self, tol=1e-6, max_iter=2000):
        """Returns (iterations, relative residual)."""
        return fib_emg_solve(self.h, tol, max_iter)

    def phi(self):
        return fib_emg_get_phi(self.h, self.n)

    def rhs(self):
        return fib_emg_get_rhs(self.h, self.n)

    def close(self):
        if self.h:
            fib_emg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fib_reset_observables(ctx) -> None:
    _check(lib().fib_reset_observables(_vp(ctx)))


def fib_sync(ctx) -> None:
    _check(lib().fib_sync(_vp(ctx)))


def fib_plan_info(ctx):
    g, t, k, l = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().fib_plan_info(_vp(ctx), C.byref(g), C.byref(t), C.byref(k), C.byref(l)))
    return dict(groups=g.value, threads=t.value, nodes_per_thread=k.value, pcr_levels=l.value)


def fib_plan_preview(params: fib_params, n_nodes, compute_units: int = 256):
    nn = np.ascontiguousarray(n_nodes, dtype=np.int32)
    g, t, k, l = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    mx = C.c_int64()
    _check(lib().fib_plan_preview(C.byref(params), len(nn), nn.ctypes.data_as(_i32p),
                                  int(compute_units), C.byref(g), C.byref(t), C.byref(k),
                                  C.byref(l), C.byref(mx)))
    return dict(groups=g.value, threads=t.value, nodes_per_thread=k.value, pcr_levels=l.value,
                max_load=mx.value)


def fib_autotune(ctx, trial_steps: int = 100, max_candidates: int = 8) -> float:
    ms = C.c_double(0.0)
    _check(lib().fib_autotune(_vp(ctx), int(trial_steps), int(max_candidates), C.byref(ms)))
    return ms.value


def fib_mlp_create(sizes, stream=None, act: str = "silu") -> int:
    sz = np.ascontiguousarray(sizes, dtype=np.int32)
    out = _vp()
    _check(lib().fib_mlp_create(len(sz) - 1, sz.ctypes.data_as(_i32p), ACTS[act],
                                _vp(stream) if stream else None, C.byref(out)))
    return out.value


def fib_mlp_destroy(net) -> None:
    lib().fib_mlp_destroy(_vp(net))


def fib_mlp_n_params(net) -> int:
    return int(lib().fib_mlp_n_params(_vp(net)))


def fib_mlp_set_params(net, params: np.ndarray) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().fib_mlp_set_params(_vp(net), p.ctypes.data_as(_fp), p.size))


def fib_mlp_get_params(net) -> np.ndarray:
    p = np.zeros(fib_mlp_n_params(net), dtype=np.float32)
    _check(lib().fib_mlp_get_params(_vp(net), p.ctypes.data_as(_fp), p.size))
    return p


def fib_mlp_forward(net, X_ptr: int, B: int, O_ptr: int) -> None:
    _check(lib().fib_mlp_forward(_vp(net), _vp(X_ptr), int(B), _vp(O_ptr)))


def fib_mlp_gradient(net, X_ptr: int, T_ptr: int, B: int, grad_ptr: int = 0,
                     loss_ptr: int = 0) -> None:
    _check(lib().fib_mlp_gradient(_vp(net), _vp(X_ptr), _vp(T_ptr), int(B),
                                  _vp(grad_ptr or None), _vp(loss_ptr or None)))


def fib_mlp_gradient_noalloc(net, X_ptr: int, T_ptr: int, B: int, grad_ptr: int = 0,
                             loss_ptr: int = 0) -> None:
    _check(lib().fib_mlp_gradient_noalloc(_vp(net), _vp(X_ptr), _vp(T_ptr), int(B),
                                          _vp(grad_ptr or None), _vp(loss_ptr or None)))


def fib_mlp_adam_step(net, X_ptr: int, T_ptr: int, B: int, lr: float, loss_ptr: int = 0) -> None:
    _check(lib().fib_mlp_adam_step(_vp(net), _vp(X_ptr), _vp(T_ptr), int(B), float(lr),
                                   _vp(loss_ptr or None)))


def fib_mlp_reset_optimizer(net) -> None:
    _check(lib().fib_mlp_reset_optimizer(_vp(net)))


def fib_set_surrogate(ctx, net, in_shift, in_scale, out_shift, out_scale, res_scale,
                      flag_scale: float, tol: float) -> None:
    arrs = [np.ascontiguousarray(a, dtype=np.float32)
            for a in (in_shift, in_scale, out_shift, out_scale, res_scale)]
    _check(lib().fib_set_surrogate(_vp(ctx), _vp(net), *[a.ctypes.data_as(_fp) for a in arrs],
                                   float(flag_scale), float(tol)))


def fib_step_surrogate(ctx, step: int) -> None:
    _check(lib().fib_step_surrogate(_vp(ctx), int(step)))


def fib_surrogate_predict(ctx, step: int, du_ptr: int) -> None:
    _check(lib().fib_surrogate_predict(_vp(ctx), int(step), _vp(du_ptr)))


def fib_clear_surrogate(ctx) -> None:
    _check(lib().fib_clear_surrogate(_vp(ctx)))


def fib_surrogate_last_fallbacks(ctx) -> int:
    n = C.c_int64()
    _check(lib().fib_surrogate_last_fallbacks(_vp(ctx), C.byref(n)))
    return n.value


def fib_surrogate_fallbacks(ctx):
    """(rejected node-steps, surrogate steps) since the step was attached."""
    t, n = C.c_int64(), C.c_int64()
    _check(lib().fib_surrogate_fallbacks(_vp(ctx), C.byref(t), C.byref(n)))
    return t.value, n.value


def fib_column_stats(A_ptr: int, rows: int, cols: int, stream=None):
    """(mean, std, min, max) of the columns of a device array (host arrays)."""
    mean, std = np.zeros(cols), np.zeros(cols)
    lo, hi = np.zeros(cols, np.float32), np.zeros(cols, np.float32)
    _check(lib().fib_column_stats(_vp(A_ptr), int(rows), int(cols), _vp(stream),
                                  mean.ctypes.data_as(_dp), std.ctypes.data_as(_dp),
                                  lo.ctypes.data_as(_fp), hi.ctypes.data_as(_fp)))
    return mean, std, lo, hi


def fib_normalize_rows(A_ptr: int, rows: int, cols: int, shift, scale, extra: float, Y_ptr: int,
                       ldy: int, stream=None) -> None:
    sh = np.ascontiguousarray(shift, dtype=np.float32)
    sc = np.ascontiguousarray(scale, dtype=np.float32)
    _check(lib().fib_normalize_rows(_vp(A_ptr), int(rows), int(cols), sh.ctypes.data_as(_fp),
                                    sc.ctypes.data_as(_fp), float(extra), _vp(Y_ptr), int(ldy),
                                    _vp(stream)))


def fib_state_rows(ctx, U_ptr: int) -> None:
    _check(lib().fib_state_rows(_vp(ctx), _vp(U_ptr)))


def fib_reaction_increments(ctx, U_ptr: int, rows: int, step: int, dU_ptr: int) -> None:
    _check(lib().fib_reaction_increments(_vp(ctx), _vp(U_ptr), int(rows), int(step), _vp(dU_ptr)))


def fib_set_graphs(ctx, enable: bool) -> None:
    _check(lib().fib_set_graphs(_vp(ctx), 1 if enable else 0))


def fib_graph_replays(ctx) -> int:
    n = C.c_int64()
    _check(lib().fib_graph_replays(_vp(ctx), C.byref(n)))
    return n.value


def fib_set_kernel_timing(ctx, enable: bool) -> None:
    _check(lib().fib_set_kernel_timing(_vp(ctx), 1 if enable else 0))


def fib_kernel_time(ctx, cls: int):
    """(summed device ms, launches) of a kernel class since timing was turned on."""
    ms, n = C.c_double(), C.c_int64()
    _check(lib().fib_kernel_time(_vp(ctx), int(cls), C.byref(ms), C.byref(n)))
    return ms.value, n.value


def fib_probe(kind: int, nbytes: int = 0) -> float:
    """Measured ceiling of the current device (see fib.h)."""
    r = C.c_double()
    _check(lib().fib_probe(int(kind), int(nbytes), C.byref(r)))
    return r.value


def fib_set_predictor(ctx, predictor: int, res_scale, tol: float) -> None:
    r = np.ascontiguousarray(res_scale, dtype=np.float32)
    _check(lib().fib_set_predictor(_vp(ctx), int(predictor), r.ctypes.data_as(_fp), float(tol)))


class Mlp:
    """Owns one surrogate network; data arrays are torch CUDA tensors."""

    def __init__(self, sizes, stream=None, act: str = "silu"):
        import torch
        self.torch = torch
        self.sizes = list(sizes)
        self.act = act
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.net = fib_mlp_create(self.sizes, stream, act)

    def close(self):
        if self.net:
            fib_mlp_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_params(self):
        return fib_mlp_n_params(self.net)

    def set_params(self, flat):
        fib_mlp_set_params(self.net, flat)

    def get_params(self):
        return fib_mlp_get_params(self.net)

    def forward(self, X):
        t = self.torch
        X = X.contiguous().float()
        O = t.empty((X.shape[0], self.sizes[-1]), device=X.device)
        fib_mlp_forward(self.net, X.data_ptr(), X.shape[0], O.data_ptr())
        return O

    def gradient(self, X, T):
        t = self.torch
        g = t.empty(self.n_params, device=X.device)
        loss = t.empty(1, device=X.device)
        fib_mlp_gradient(self.net, X.contiguous().data_ptr(), T.contiguous().data_ptr(),
                         X.shape[0], g.data_ptr(), loss.data_ptr())
        return g, loss

    def reset_optimizer(self):
        fib_mlp_reset_optimizer(self.net)

    def adam_step(self, X, T, lr, loss=None):
        fib_mlp_adam_step(self.net, X.data_ptr(), T.data_ptr(), X.shape[0], lr,
                          loss.data_ptr() if loss is not None else 0)


# ---- convenience wrapper (still marshalling only) ---------------------------------

class Solver:
    """Owns one context; device buffers through torch (current CUDA device)."""

    def __init__(self, n_nodes, stream=None, **params):
        import torch
        self.torch = torch
        self.params = make_params(**params)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        self.ctx = fib_create(self.params, n_nodes, stream)
        self.n_total = fib_n_total(self.ctx)
        self.S = fib_n_states(self.params.model)

    def close(self):
        if self.ctx:
            fib_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_state(self, vm_noise=None, rel_noise=None):
        """Resting state times (1 + rel_noise) plus vm_noise on V_m; the noise
        arrays are host arrays or float32 CUDA tensors ([n_total], [S, n_total])."""
        t = self.torch

        def dev(a):
            if a is None:
                return None
            if isinstance(a, t.Tensor):
                return a.to(device="cuda", dtype=t.float32).contiguous()
            return t.as_tensor(np.asarray(a, dtype=np.float32), device="cuda")
        self._vm = dev(vm_noise)
        self._rel = dev(rel_noise)
        # the kernel reads n_total and S * n_total values: check before launching
        if self._vm is not None and self._vm.numel() != self.n_total:
            raise ValueError(f"vm_noise has {self._vm.numel()} values, expected {self.n_total}")
        if self._rel is not None and self._rel.numel() != self.S * self.n_total:
            raise ValueError(f"rel_noise has {self._rel.numel()} values, expected {self.S} x {self.n_total}")
        fib_init_state(self.ctx, self._vm.data_ptr() if self._vm is not None else 0,
                       self._rel.data_ptr() if self._rel is not None else 0)

    def set_state(self, y):
        fib_set_state(self.ctx, y)

    def get_state(self):
        return fib_get_state(self.ctx, self.S)

    def state_tensor(self):
        """Zero-copy torch view of the FP32 device state [S, n_total] and the
        reference state; row k of the view holds y_k - ref[k]."""
        ptr, ref = fib_state_device(self.ctx, self.S)
        n = self.S * self.n_total
        t = self.torch
        # wrap through the CUDA array interface without copying
        class _Arr:
            __cuda_array_interface__ = {"shape": (n,), "typestr": "<f4", "data": (ptr, False),
                                        "version": 2}
        return t.as_tensor(_Arr(), device="cuda").view(self.S, self.n_total), ref

    def set_stimulus(self, stims):
        fib_set_stimulus(self.ctx, stims)

    def step_reaction(self, step, span):
        fib_step_reaction(self.ctx, step, span)

    def step_diffusion(self, span):
        fib_step_diffusion(self.ctx, span)

    def run(self, step0, n_steps, sample_every=0, samples=None):
        rows = samples.shape[0] if samples is not None else 0
        fib_run(self.ctx, step0, n_steps, sample_every,
                samples.data_ptr() if samples is not None else 0, rows)

    def tact(self):
        return fib_get_tact(self.ctx)

    def sync(self):
        fib_sync(self.ctx)

    def plan(self):
        return fib_plan_info(self.ctx)

    def autotune(self, trial_steps=100, max_candidates=8):
        """Measures candidate workgroup shapes and keeps the fastest; returns
        the chosen plan with its trial time per split step (ms)."""
        ms = fib_autotune(self.ctx, trial_steps, max_candidates)
        out = dict(self.plan())
        out["trial_ms_per_step"] = ms
        return out

    def set_surrogate(self, net, scales: dict, tol: float):
        fib_set_surrogate(self.ctx, net.net, scales["in_shift"], scales["in_scale"],
                          scales["out_shift"], scales["out_scale"], scales["res_scale"],
                          scales.get("flag_scale", 0.0), tol)

    def step_surrogate(self, step):
        fib_step_surrogate(self.ctx, step)

    def surrogate_predict(self, step=0):
        """Predicted increments [S, n_total] (device tensor) for the current
        state; no state changes."""
        import torch
        du = torch.empty((self.S, self.n_total), dtype=torch.float32, device="cuda")
        fib_surrogate_predict(self.ctx, step, du.data_ptr())
        return du

    def clear_surrogate(self):
        fib_clear_surrogate(self.ctx)

    def last_fallbacks(self):
        return fib_surrogate_last_fallbacks(self.ctx)

    def fallbacks(self):
        """(rejected node-steps, surrogate steps) since the step was attached."""
        return fib_surrogate_fallbacks(self.ctx)

    def set_graphs(self, enable=True):
        fib_set_graphs(self.ctx, enable)

    def graph_replays(self):
        return fib_graph_replays(self.ctx)

    def set_kernel_timing(self, enable=True):
        fib_set_kernel_timing(self.ctx, enable)

    def kernel_time(self, cls):
        """(summed device ms, launches) of a kernel class (FIB_KT_*)."""
        return fib_kernel_time(self.ctx, cls)

    def set_predictor(self, predictor, res_scale, tol: float):
        """The surrogate step with a closed-form predictor (FIB_PRED_ZERO or
        FIB_PRED_EULER) in place of a network."""
        fib_set_predictor(self.ctx, predictor, res_scale, tol)

    def set_adaptive(self, tol):
        """Adaptive computation with relative tolerance tol (0: off)."""
        fib_set_adaptive(self.ctx, tol)

    def adaptive_solved(self):
        return fib_adaptive_solved(self.ctx)

    def adaptive_points(self):
        return fib_adaptive_points(self.ctx)
