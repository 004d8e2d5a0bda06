"""Python binding of the FP64 CPU oracle (``oracle/fib_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module; the GPU library
never does, and this module never imports the GPU library.

The oracle follows the thesis step by step (see the header of
``fib_oracle.c`` for the passage behind each function).  All arrays are
float64 NumPy arrays; states are structure-of-arrays ``y[k, i]`` with
``k = 0`` the membrane voltage (mV).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "fib_oracle.c"), os.path.join(_HERE, "st57_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

MODEL_HH = 0
MODEL_ST57 = 1
MODEL_HH_APX_EXP = 2   # Hodgkin-Huxley with exp* (eq. apx-e-function) in its rates
MODEL_ST57_APX = 3     # ST57 with exp* and log* (figure apxlog)
SCHEME_STRANG = 0
SCHEME_GODUNOV = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall",
               "-o", _LIB_PATH, *_SRCS, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


class Params(C.Structure):
    _fields_ = [("model", C.c_int32), ("scheme", C.c_int32),
                ("Cm", C.c_double), ("Am", C.c_double), ("sigma", C.c_double),
                ("h", C.c_double), ("dt_0D", C.c_double), ("dt_1D", C.c_double),
                ("dt_split", C.c_double), ("v_th", C.c_double), ("theta", C.c_double)]


class Stim(C.Structure):
    _fields_ = [("fiber", C.c_int32), ("node", C.c_int32), ("half_width", C.c_int32),
                ("mode", C.c_int32), ("step_on", C.c_int64), ("n_steps", C.c_int64),
                ("period", C.c_int64), ("amp", C.c_double)]


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        L.or_hh_gate_rates.argtypes = [C.c_double, _dp]
        L.or_hh_iion.argtypes = [_dp]
        L.or_hh_iion.restype = C.c_double
        L.or_hh_rhs.argtypes = [C.c_double, _dp, C.c_double, _dp]
        L.or_hh_rest.argtypes = [_dp]
        L.or_hh_apx_rest.argtypes = [_dp]
        L.or_hh_apx_gate_rates.argtypes = [C.c_double, _dp]
        L.or_hh_apx_rhs.argtypes = [C.c_double, _dp, C.c_double, _dp]
        L.or_exp_star.argtypes = [C.c_double]
        L.or_exp_star.restype = C.c_double
        L.or_log_star.argtypes = [C.c_double]
        L.or_log_star.restype = C.c_double
        L.or_log_star_taylor.argtypes = [C.c_double]
        L.or_log_star_taylor.restype = C.c_double
        L.or_st57_apx_rhs.argtypes = [C.c_double, _dp, C.c_double, _dp]
        L.or_st57_apx_rest.argtypes = [_dp, C.POINTER(C.c_int)]
        L.or_n_states.argtypes = [C.c_int]
        L.or_st57_rhs.argtypes = [C.c_double, _dp, C.c_double, _dp]
        L.or_st57_invariants.argtypes = [_dp, _dp]
        L.or_st57_rest.argtypes = [_dp, C.POINTER(C.c_int)]
        L.or_n_substeps.argtypes = [C.c_double, C.c_double]
        L.or_n_substeps.restype = C.c_int64
        L.or_thomas.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_reaction.argtypes = [C.POINTER(Params), C.c_int64, _dp, _dp, C.c_double]
        L.or_diffusion.argtypes = [C.POINTER(Params), C.c_int32, _ip, _dp, C.c_double]
        L.or_stimulus_current.argtypes = [C.c_int32, _ip, C.POINTER(Stim), C.c_int32,
                                          C.c_int64, _dp]
        L.or_run.argtypes = [C.POINTER(Params), C.c_int32, _ip, _dp, C.POINTER(Stim),
                             C.c_int32, C.c_int64, C.c_int64, C.c_int64, _dp, _dp]
        L.or_run_adaptive.argtypes = [C.POINTER(Params), C.c_int32, _ip, _dp, C.POINTER(Stim),
                                      C.c_int32, C.c_int64, C.c_int64, C.c_int64, _dp, _dp,
                                      C.c_double, _u8p, C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


@dataclass
class Config:
    """Physical and numerical parameters (units: cm, ms, mV, uA, uF, mS)."""
    model: int = MODEL_HH
    scheme: int = SCHEME_STRANG
    Cm: float = 1.0
    Am: float = 500.0
    sigma: float = 3.828
    h: float = 0.01
    dt_0D: float = 1e-3
    dt_1D: float = 1e-3
    dt_split: float = 1e-3
    v_th: float = -20.0
    theta: float = 0.5          # 1D time stepping: 0.5 Crank-Nicolson, 1 implicit Euler

    def c_params(self) -> Params:
        return Params(self.model, self.scheme, self.Cm, self.Am, self.sigma, self.h,
                      self.dt_0D, self.dt_1D, self.dt_split, self.v_th, self.theta)


def n_states(model: int = MODEL_HH) -> int:
    return int(lib().or_n_states(model))


def hh_gate_rates(V: float) -> np.ndarray:
    out = np.zeros(6)
    lib().or_hh_gate_rates(float(V), _d(out))
    return out


def hh_iion(y) -> float:
    y = _f64(y)
    return float(lib().or_hh_iion(_d(y)))


def hh_rhs(y, I_stim: float = 0.0, Cm: float = 1.0) -> np.ndarray:
    y = _f64(y)
    out = np.zeros(4)
    lib().or_hh_rhs(float(Cm), _d(y), float(I_stim), _d(out))
    return out


def rest_state(model: int = MODEL_HH) -> np.ndarray:
    y = np.zeros(n_states(model))
    if model == MODEL_HH:
        rc = lib().or_hh_rest(_d(y))
    elif model == MODEL_HH_APX_EXP:
        rc = lib().or_hh_apx_rest(_d(y))
    elif model == MODEL_ST57:
        it = C.c_int(0)
        rc = lib().or_st57_rest(_d(y), C.byref(it))
    elif model == MODEL_ST57_APX:
        it = C.c_int(0)
        rc = lib().or_st57_apx_rest(_d(y), C.byref(it))
    else:
        raise ValueError("unknown model")
    if rc != 0:
        raise RuntimeError("rest state search failed")
    return y


def exp_star(x: float) -> float:
    """exp*(x) = (1 + x/1024)^1024 (eq. apx-e-function)."""
    return lib().or_exp_star(float(x))


def log_star(x: float) -> float:
    """log*(x): piecewise sixth-order Taylor value refined by one Newton step
    on exp* (figure apxlog), with an exact power-of-two range reduction
    outside [0.2, 20]."""
    return lib().or_log_star(float(x))


def log_star_taylor(x: float) -> float:
    """The piecewise sixth-order Taylor polynomial of log alone."""
    return lib().or_log_star_taylor(float(x))


def hh_apx_rates(V: float) -> np.ndarray:
    ab = np.zeros(6)
    lib().or_hh_apx_gate_rates(float(V), _d(ab))
    return ab


def hh_apx_rhs(y, I_stim: float = 0.0, Cm: float = 1.0) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    d = np.zeros(4)
    lib().or_hh_apx_rhs(float(Cm), _d(y), float(I_stim), _d(d))
    return d


def st57_rhs(y, I_stim: float = 0.0, Cm: float = 1.0) -> np.ndarray:
    y = _f64(y)
    out = np.zeros(57)
    lib().or_st57_rhs(float(Cm), _d(y), float(I_stim), _d(out))
    return out


def st57_apx_rhs(y, I_stim: float = 0.0, Cm: float = 1.0) -> np.ndarray:
    y = _f64(y)
    out = np.zeros(57)
    lib().or_st57_apx_rhs(float(Cm), _d(y), float(I_stim), _d(out))
    return out


def st57_invariants(y) -> np.ndarray:
    """(sum P, sum Q, sum R, sum X, total Ca, total Mg) of one ST57 state."""
    y = _f64(y)
    out = np.zeros(6)
    lib().or_st57_invariants(_d(y), _d(out))
    return out


def n_substeps(span: float, dt: float) -> int:
    return int(lib().or_n_substeps(float(span), float(dt)))


def thomas(a, d, c, b) -> np.ndarray:
    a, d, c, b = (_f64(v) for v in (a, d, c, b))
    n = b.shape[0]
    x = np.zeros(n)
    work = np.zeros(max(n, 1))
    lib().or_thomas(n, _d(a), _d(d), _d(c), _d(b), _d(x), _d(work))
    return x


def _stims(stims):
    n = len(stims)
    arr = (Stim * max(n, 1))()
    for i, s in enumerate(stims):
        arr[i] = Stim(int(s["fiber"]), int(s["node"]), int(s.get("half_width", 1)),
                      int(s.get("mode", 0)),
                      int(s["step_on"]), int(s["n_steps"]), int(s.get("period", 0)),
                      float(s["amp"]))
    return arr, n


def stimulus_current(n_nodes, stims, step: int) -> np.ndarray:
    nn = np.ascontiguousarray(n_nodes, dtype=np.int32)
    arr, n = _stims(stims)
    out = np.zeros(int(nn.sum()))
    lib().or_stimulus_current(len(nn), nn.ctypes.data_as(_ip), arr, n, int(step), _d(out))
    return out


def reaction(cfg: Config, y: np.ndarray, span: float, I=None) -> np.ndarray:
    """Reaction part over `span` on every node; returns a new state array."""
    y = np.array(y, dtype=np.float64, order="C", copy=True)
    n_total = y.shape[1]
    Iv = _f64(I) if I is not None else None
    p = cfg.c_params()
    rc = lib().or_reaction(C.byref(p), n_total, _d(y), _d(Iv), float(span))
    if rc != 0:
        raise RuntimeError(f"or_reaction failed ({rc})")
    return y


def diffusion(cfg: Config, n_nodes, V: np.ndarray, span: float) -> np.ndarray:
    V = np.array(V, dtype=np.float64, copy=True)
    nn = np.ascontiguousarray(n_nodes, dtype=np.int32)
    p = cfg.c_params()
    rc = lib().or_diffusion(C.byref(p), len(nn), nn.ctypes.data_as(_ip), _d(V), float(span))
    if rc != 0:
        raise RuntimeError(f"or_diffusion failed ({rc})")
    return V


PT_ACTIVE, PT_INACTIVE, PT_NEIGHBOR = 0, 1, 2


def run_adaptive(cfg: Config, n_nodes, y0: np.ndarray, stims, n_steps: int, step0: int = 0,
                 sample_every: int = 0, t_act=None, tol: float = 1e-5, pt=None):
    """The splitting loop with adaptive computation (or_run_adaptive); returns
    (y, samples or None, t_act, point states, node-steps solved)."""
    nn = np.ascontiguousarray(n_nodes, dtype=np.int32)
    y = np.array(y0, dtype=np.float64, order="C", copy=True)
    n_total = int(nn.sum())
    assert y.shape[1] == n_total
    arr, n = _stims(stims)
    samples = None
    if sample_every > 0:
        first = step0 // sample_every
        last = (step0 + n_steps) // sample_every
        samples = np.full((max(last - first, 0), n_total), np.nan)
    ta = (np.full(n_total, np.inf) if t_act is None
          else np.array(t_act, dtype=np.float64, copy=True))
    pt = (np.full(n_total, PT_ACTIVE, dtype=np.uint8) if pt is None
          else np.array(pt, dtype=np.uint8, copy=True))
    cnt = C.c_int64(0)
    p = cfg.c_params()
    rc = lib().or_run_adaptive(C.byref(p), len(nn), nn.ctypes.data_as(_ip), _d(y), arr, n,
                               int(step0), int(n_steps), int(sample_every),
                               _d(samples) if samples is not None and samples.size else None,
                               _d(ta), float(tol), pt.ctypes.data_as(_u8p), C.byref(cnt))
    if rc != 0:
        raise RuntimeError(f"or_run_adaptive failed ({rc})")
    return y, samples, ta, pt, int(cnt.value)


def run(cfg: Config, n_nodes, y0: np.ndarray, stims, n_steps: int, step0: int = 0,
        sample_every: int = 0, t_act=None, want_samples: bool = True):
    """Runs the splitting loop; returns (y, samples or None, t_act)."""
    nn = np.ascontiguousarray(n_nodes, dtype=np.int32)
    y = np.array(y0, dtype=np.float64, order="C", copy=True)
    n_total = int(nn.sum())
    assert y.shape[1] == n_total
    arr, n = _stims(stims)
    samples = None
    if want_samples and sample_every > 0:
        first = step0 // sample_every
        last = (step0 + n_steps) // sample_every
        samples = np.full((max(last - first, 0), n_total), np.nan)
    ta = (np.full(n_total, np.inf) if t_act is None
          else np.array(t_act, dtype=np.float64, copy=True))
    p = cfg.c_params()
    rc = lib().or_run(C.byref(p), len(nn), nn.ctypes.data_as(_ip), _d(y), arr, n,
                      int(step0), int(n_steps), int(sample_every),
                      _d(samples) if samples is not None and samples.size else None, _d(ta))
    if rc != 0:
        raise RuntimeError(f"or_run failed ({rc})")
    return y, samples, ta
