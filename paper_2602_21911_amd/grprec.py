"""ctypes binding of libgrprec.so (the C ABI in include/grprec.h).

Functions carry the C names and only marshal arguments; every step of the
method runs in the library's HIP kernels.  PyTorch supplies device memory and
the stream.  ``Simulation`` bundles the buffers of one problem.

The library must be built (``python -m paper_2602_21911_amd.build``); loading
fails loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GRPREC_LIB", os.path.join(HERE, "libgrprec.so"))

GRPREC_OK = 0
GRPREC_E_INVALID = -1
GRPREC_E_UNSUPPORTED = -2
GRPREC_E_HIP = -3
GRPREC_E_NONPHYSICAL = -4
GRPREC_E_VACUUM = -5
GRPREC_E_NEWTON = -6
GRPREC_E_PREDICTOR = -7

GRPREC_ADVECTION, GRPREC_EULER = 0, 1
GRPREC_BC_PERIODIC, GRPREC_BC_TRANSMISSIVE = 0, 1
GRPREC_GUESS_PVRS, GRPREC_GUESS_MLP = 0, 1
GRPREC_SCHED_AUTO, GRPREC_SCHED_SEGMENT_TILES, GRPREC_SCHED_FLAT_TILES, GRPREC_SCHED_PACKED = 0, 1, 2, 3
GRPREC_SCHED_PER_DOMAIN = 4
GRPREC_RECON_LINEAR, GRPREC_RECON_NL = 0, 1
GRPREC_DATUM_EXACT, GRPREC_DATUM_TRRS = 0, 1
GRPREC_SOURCE_NONE, GRPREC_SOURCE_LINEAR = 0, 1
GRPREC_MLP_WEIGHTS = 1313
GRPREC_MLP_NPARAMS = 1325
GRPREC_MLP_NOALLOC_MAX = 65536

EXPORTED = [
    "grprec_workspace_bytes", "grprec_init", "grprec_step", "grprec_run", "grprec_state",
    "grprec_get_state",
    "grprec_segment_times", "grprec_set_state", "grprec_get_schedule", "grprec_set_schedule",
    "grprec_autotune", "grprec_enable_stats", "grprec_get_stats", "grprec_error_string",
    "grprec_destroy", "grprec_riemann_batch", "grprec_mlp_features", "grprec_mlp_forward",
    "grprec_mlp_work_bytes", "grprec_mlp_backward", "grprec_mlp_backward_noalloc",
    "grprec_mlp_loss_grad", "grprec_mlp_adam",
    "grprec_harvest",
]

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


class grprec_problem(ctypes.Structure):
    _fields_ = [("system", ctypes.c_int), ("order", ctypes.c_int), ("cfl", ctypes.c_double),
                ("lam", ctypes.c_double), ("gamma", ctypes.c_double), ("bc", ctypes.c_int),
                ("n_segments", ctypes.c_int), ("seg_cells", _i64p), ("seg_length", _dp),
                ("guess", ctypes.c_int), ("max_newton", ctypes.c_int),
                ("newton_tol", ctypes.c_double), ("max_picard", ctypes.c_int),
                ("picard_tol", ctypes.c_double), ("mlp_params", _vp),
                ("mlp_gate", ctypes.c_double), ("warm_start", ctypes.c_int),
                ("schedule", ctypes.c_int), ("block", ctypes.c_int), ("recon", ctypes.c_int),
                ("nl_lambda_c", ctypes.c_double), ("nl_eps", ctypes.c_double), ("datum", ctypes.c_int),
                ("source", ctypes.c_int), ("source_kappa", ctypes.c_double)]


class grprec_buffers(ctypes.Structure):
    _fields_ = [("q0", _vp), ("q1", _vp), ("v0", _vp), ("v1", _vp), ("work", _vp),
                ("work_bytes", ctypes.c_size_t)]


class grprec_stats(ctypes.Structure):
    _fields_ = [("rs_calls", ctypes.c_uint64), ("newton_iters", ctypes.c_uint64),
                ("picard_sweeps", ctypes.c_uint64), ("cells_predicted", ctypes.c_uint64),
                ("mlp_guesses", ctypes.c_uint64)]


class GrprecError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().grprec_error_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})")
        self.code = code


_lib = None


def lib():
    """Load libgrprec.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2602_21911_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        L.grprec_workspace_bytes.argtypes = [ctypes.POINTER(grprec_problem)]
        L.grprec_workspace_bytes.restype = ctypes.c_size_t
        L.grprec_init.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(grprec_problem),
                                  ctypes.POINTER(grprec_buffers), _vp]
        L.grprec_step.argtypes = [_vp, ctypes.c_double, _dp]
        L.grprec_run.argtypes = [_vp, ctypes.c_double, ctypes.c_int64, _i64p, _dp]
        L.grprec_state.argtypes = [_vp, ctypes.POINTER(ctypes.c_int), _dp, _dp, _i64p]
        L.grprec_get_state.argtypes = [_vp, _dp, _i64p]
        L.grprec_segment_times.argtypes = [_vp, _dp]
        L.grprec_set_state.argtypes = [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int64]
        L.grprec_get_schedule.argtypes = [_vp, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int)]
        L.grprec_set_schedule.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
        L.grprec_autotune.argtypes = [_vp, ctypes.c_int, _dp, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]
        L.grprec_enable_stats.argtypes = [_vp, ctypes.c_int]
        L.grprec_get_stats.argtypes = [_vp, ctypes.POINTER(grprec_stats)]
        L.grprec_error_string.argtypes = [ctypes.c_int]
        L.grprec_error_string.restype = ctypes.c_char_p
        L.grprec_destroy.argtypes = [_vp]
        L.grprec_destroy.restype = None
        L.grprec_riemann_batch.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                           _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           _vp, _vp, _vp]
        L.grprec_mlp_features.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_double, _vp, _vp,
                                          _vp]
        L.grprec_mlp_forward.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp]
        L.grprec_mlp_work_bytes.argtypes = [ctypes.c_int64]
        L.grprec_mlp_work_bytes.restype = ctypes.c_size_t
        L.grprec_mlp_backward.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp, _vp]
        L.grprec_mlp_backward_noalloc.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp]
        L.grprec_mlp_loss_grad.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp, _vp, _vp]
        L.grprec_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp]
        L.grprec_harvest.argtypes = [_vp, _vp, ctypes.c_int64, _vp]
        _lib = L
    return _lib


def _chk(rc: int, where: str):
    if rc != GRPREC_OK:
        raise GrprecError(rc, where)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# ------------------------------------------------------------------ thin wrappers
def grprec_workspace_bytes(p: grprec_problem) -> int:
    return lib().grprec_workspace_bytes(ctypes.byref(p))


def grprec_init(p: grprec_problem, b: grprec_buffers, stream=None) -> int:
    h = _vp()
    _chk(lib().grprec_init(ctypes.byref(h), ctypes.byref(p), ctypes.byref(b), _stream(stream)),
         "grprec_init")
    return h.value


def grprec_step(h: int, t_stop: float, want_dt: bool = False) -> Optional[float]:
    if want_dt:
        dt = ctypes.c_double(0.0)
        _chk(lib().grprec_step(h, t_stop, ctypes.byref(dt)), "grprec_step")
        return dt.value
    _chk(lib().grprec_step(h, t_stop, None), "grprec_step")
    return None


def grprec_run(h: int, t_end: float, max_steps: int = (1 << 62)):
    steps = ctypes.c_int64(0)
    t = ctypes.c_double(0.0)
    _chk(lib().grprec_run(h, t_end, max_steps, ctypes.byref(steps), ctypes.byref(t)), "grprec_run")
    return steps.value, t.value


def grprec_state(h: int):
    cur = ctypes.c_int(0)
    tmin, tmax = ctypes.c_double(0), ctypes.c_double(0)
    steps = ctypes.c_int64(0)
    _chk(lib().grprec_state(h, ctypes.byref(cur), ctypes.byref(tmin), ctypes.byref(tmax),
                            ctypes.byref(steps)), "grprec_state")
    return cur.value, tmin.value, tmax.value, steps.value


def grprec_get_state(h: int):
    """(time of the current state, steps since init)."""
    t = ctypes.c_double(0)
    steps = ctypes.c_int64(0)
    _chk(lib().grprec_get_state(h, ctypes.byref(t), ctypes.byref(steps)), "grprec_get_state")
    return t.value, steps.value


def grprec_segment_times(h: int, n_segments: int) -> np.ndarray:
    t = np.zeros(n_segments)
    _chk(lib().grprec_segment_times(h, t.ctypes.data_as(_dp)), "grprec_segment_times")
    return t


def grprec_set_state(h: int, current: int, t: float, steps: int):
    _chk(lib().grprec_set_state(h, current, t, steps), "grprec_set_state")


def grprec_get_schedule(h: int):
    s, b = ctypes.c_int(0), ctypes.c_int(0)
    _chk(lib().grprec_get_schedule(h, ctypes.byref(s), ctypes.byref(b)), "grprec_get_schedule")
    return s.value, b.value


def grprec_set_schedule(h: int, schedule: int, block: int):
    _chk(lib().grprec_set_schedule(h, schedule, block), "grprec_set_schedule")


def grprec_autotune(h: int, steps: int = 3):
    ms = np.zeros(9)
    n = ctypes.c_int(0)
    _chk(lib().grprec_autotune(h, steps, ms.ctypes.data_as(_dp), 9, ctypes.byref(n)),
         "grprec_autotune")
    return ms[: n.value]


def grprec_enable_stats(h: int, on: bool):
    _chk(lib().grprec_enable_stats(h, 1 if on else 0), "grprec_enable_stats")


def grprec_get_stats(h: int) -> dict:
    st = grprec_stats()
    _chk(lib().grprec_get_stats(h, ctypes.byref(st)), "grprec_get_stats")
    return {k: getattr(st, k) for k, _ in grprec_stats._fields_}


def grprec_error_string(code: int) -> str:
    return lib().grprec_error_string(code).decode()


def grprec_destroy(h: int):
    if h:
        lib().grprec_destroy(h)


def grprec_riemann_batch(wl, wr, gamma=1.4, guess=GRPREC_GUESS_PVRS, mlp_params=None, gate=-1.0,
                         tol=1e-12, max_iter=50, pstar=None, iters=None, stream=None):
    """wl, wr: device float64 [n,3] primitive states; returns (pstar, iters) tensors."""
    import torch
    n = wl.shape[0]
    if pstar is None:
        pstar = torch.empty(n, dtype=torch.float64, device=wl.device)
    if iters is None:
        iters = torch.empty(n, dtype=torch.int32, device=wl.device)
    _chk(lib().grprec_riemann_batch(_ptr(wl), _ptr(wr), n, gamma, guess, _ptr(mlp_params), gate, tol,
                                    max_iter, _ptr(pstar), _ptr(iters), _stream(stream)),
         "grprec_riemann_batch")
    return pstar, iters


def grprec_mlp_features(wl, wr, pstar=None, gamma=1.4, x=None, y=None, stream=None):
    import torch
    n = wl.shape[0]
    if x is None:
        x = torch.empty((n, 6), dtype=torch.float32, device=wl.device)
    if pstar is not None and y is None:
        y = torch.empty(n, dtype=torch.float32, device=wl.device)
    _chk(lib().grprec_mlp_features(_ptr(wl), _ptr(wr), _ptr(pstar), n, gamma, _ptr(x), _ptr(y),
                                   _stream(stream)), "grprec_mlp_features")
    return x, y


def grprec_mlp_forward(params, x, y=None, stream=None):
    import torch
    n = x.shape[0]
    if y is None:
        y = torch.empty(n, dtype=torch.float32, device=x.device)
    _chk(lib().grprec_mlp_forward(_ptr(params), _ptr(x), _ptr(y), n, _stream(stream)),
         "grprec_mlp_forward")
    return y


def grprec_mlp_work_bytes(n: int) -> int:
    return lib().grprec_mlp_work_bytes(n)


def grprec_mlp_backward(params, x, dy, grad, work, stream=None):
    _chk(lib().grprec_mlp_backward(_ptr(params), _ptr(x), _ptr(dy), _ptr(grad), x.shape[0], _ptr(work),
                                   _stream(stream)), "grprec_mlp_backward")


def grprec_mlp_backward_noalloc(params, x, dy, grad, stream=None):
    _chk(lib().grprec_mlp_backward_noalloc(_ptr(params), _ptr(x), _ptr(dy), _ptr(grad), x.shape[0],
                                           _stream(stream)), "grprec_mlp_backward_noalloc")


def grprec_mlp_loss_grad(params, x, y, grad, loss, work, stream=None):
    _chk(lib().grprec_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(y), x.shape[0], _ptr(grad),
                                    _ptr(loss), _ptr(work), _stream(stream)), "grprec_mlp_loss_grad")


def grprec_mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                    stream=None):
    _chk(lib().grprec_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1, beta2,
                               eps, _stream(stream)), "grprec_mlp_adam")


def grprec_harvest(h: int, ring=None, count=None):
    cap = 0 if ring is None else ring.shape[0]
    _chk(lib().grprec_harvest(h, _ptr(ring), cap, _ptr(count)), "grprec_harvest")


# ------------------------------------------------------------------ convenience
class Simulation:
    """Device buffers + handle for one problem (one or many independent domains).

    q_init: [nvar, total_cells]; v_left / v_right: [nvar, total_cells + S]
    one-sided limits of the initial condition at the interfaces.
    """

    def __init__(self, system: int, order: int, cells: Sequence[int], lengths: Sequence[float],
                 q_init: np.ndarray, v_left: np.ndarray, v_right: np.ndarray,
                 bc: int = GRPREC_BC_PERIODIC, cfl: float = 0.9, lam: float = 1.0,
                 gamma: float = 1.4, guess: int = GRPREC_GUESS_PVRS, mlp_params=None,
                 mlp_gate: float = 0.1, warm_start: int = 0, schedule: int = GRPREC_SCHED_AUTO,
                 block: int = 0, max_newton: int = 50, newton_tol: float = 1e-12,
                 max_picard: int = 64, picard_tol: float = 1e-13, recon: int = GRPREC_RECON_LINEAR,
                 nl_lambda_c: float = 1e9, nl_eps: float = 1e-14, datum: int = GRPREC_DATUM_EXACT,
                 source: int = GRPREC_SOURCE_NONE, kappa: float = 0.0, device: str = "cuda"):
        import torch
        self.torch = torch
        self.cells = np.ascontiguousarray(cells, dtype=np.int64)
        self.lengths = np.ascontiguousarray(lengths, dtype=np.float64)
        S = len(self.cells)
        self.S = S
        self.nvar = 1 if system == GRPREC_ADVECTION else 3
        tc = int(self.cells.sum())
        ti = tc + S
        self.tc, self.ti = tc, ti
        self.p = grprec_problem(system, order, cfl, lam, gamma, bc, S,
                                self.cells.ctypes.data_as(_i64p), self.lengths.ctypes.data_as(_dp),
                                guess, max_newton, newton_tol, max_picard, picard_tol,
                                None if mlp_params is None else mlp_params.data_ptr(), mlp_gate,
                                warm_start, schedule, block, recon, nl_lambda_c, nl_eps, datum,
                                source, kappa)
        self.mlp_params = mlp_params
        wb = grprec_workspace_bytes(self.p)
        if wb == 0:
            raise GrprecError(GRPREC_E_INVALID, "grprec_workspace_bytes")
        f64 = dict(dtype=torch.float64, device=device)
        q_init = np.asarray(q_init, dtype=np.float64).reshape(self.nvar, tc)
        self.q0 = torch.from_numpy(np.ascontiguousarray(q_init)).to(device)
        self.q1 = torch.zeros((self.nvar, tc), **f64)
        self.v0 = torch.from_numpy(np.ascontiguousarray(np.asarray(v_left, np.float64).reshape(self.nvar, ti))).to(device)
        self.v1 = torch.from_numpy(np.ascontiguousarray(np.asarray(v_right, np.float64).reshape(self.nvar, ti))).to(device)
        self.work = torch.zeros(wb, dtype=torch.uint8, device=device)
        self.b = grprec_buffers(self.q0.data_ptr(), self.q1.data_ptr(), self.v0.data_ptr(),
                                self.v1.data_ptr(), self.work.data_ptr(), wb)
        self.h = 0
        self.h = grprec_init(self.p, self.b)

    def step(self, t_stop: float, want_dt: bool = False):
        return grprec_step(self.h, t_stop, want_dt)

    def run(self, t_end: float, max_steps: int = (1 << 62)):
        return grprec_run(self.h, t_end, max_steps)

    def state(self):
        cur, tmin, tmax, steps = grprec_state(self.h)
        q = self.q1 if cur else self.q0
        v = self.v1 if cur else self.v0
        return q, v, cur, tmin, tmax, steps

    def numpy_state(self):
        q, v, cur, tmin, tmax, steps = self.state()
        return q.cpu().numpy(), v.cpu().numpy(), tmin, steps

    def times(self) -> np.ndarray:
        return grprec_segment_times(self.h, self.S)

    def close(self):
        if self.h:
            self.torch.cuda.synchronize()
            grprec_destroy(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
