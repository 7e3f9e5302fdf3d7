"""CPU oracle for the GRPrec finite-volume step (test infrastructure only).

The oracle is a plain serial C implementation (``grprec_oracle.c``) plus a
float64 numpy reference of the learned star-pressure network (``mlp.py``).
Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may use it.  It shares no code with the GPU library and imports nothing from
the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grprec_oracle.c")
# GRPREC_ORACLE_LIB names another build of the same source to load instead
# (the tests that plant mistakes in the oracle use it to run the pins against
# a mutated build); it is never rebuilt from here.
_LIB_ENV = os.environ.get("GRPREC_ORACLE_LIB")
_LIB = _LIB_ENV or os.path.join(_HERE, "libgrprec_oracle.so")
CFLAGS = ["-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
          "-shared"]

OK, E_INVALID, E_NONPHYSICAL, E_VACUUM, E_NEWTON, E_PREDICTOR = 0, -1, -4, -5, -6, -7
ADVECTION, EULER = 0, 1
PERIODIC, TRANSMISSIVE = 0, 1
LINEAR, NONLINEAR = 0, 1          # GRPrec (Sec. 3.1) or GRPrecNL (Sec. 3.3-3.4)
DATUM_EXACT, DATUM_TRRS = 0, 1    # Euler interface datum solver (Sec. 4.1)
# GRPrecNL weight of the centred polynomial, eq. (omega): the value Sec. 3.3
# prints, and the value with which the printed GRPrecNL advection results of
# Sec. 4.2.3 are reproduced (the reading of the two documented with the tests).
SOURCE_NONE, SOURCE_LINEAR = 0, 1  # S(Q) = 0 or -kappa Q
LAMBDA_C_PRINTED = 1e9
LAMBDA_C_TABLE = 10.0


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FMA contraction)."""
    if _LIB_ENV:
        return _LIB
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", *CFLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Cfg(ctypes.Structure):
    _fields_ = [("system", ctypes.c_int), ("m", ctypes.c_int), ("cfl", ctypes.c_double),
                ("lam", ctypes.c_double), ("gamma", ctypes.c_double),
                ("bc_left", ctypes.c_int), ("bc_right", ctypes.c_int),
                ("newton_tol", ctypes.c_double), ("newton_max", ctypes.c_int),
                ("picard_tol", ctypes.c_double), ("picard_max", ctypes.c_int),
                ("recon", ctypes.c_int), ("nl_lambda_c", ctypes.c_double),
                ("nl_eps", ctypes.c_double), ("nl_r", ctypes.c_double), ("datum", ctypes.c_int),
                ("source", ctypes.c_int), ("kappa", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("rs_calls", ctypes.c_int64), ("newton_iters", ctypes.c_int64),
                ("picard_iters", ctypes.c_int64), ("picard_max_seen", ctypes.c_int),
                ("newton_max_seen", ctypes.c_int)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, _D, _D]
        L.orc_recon_matrix.argtypes = [ctypes.c_int, _D]
        L.orc_pvrs_guess.argtypes = [ctypes.c_double, _D, _D]
        L.orc_pvrs_guess.restype = ctypes.c_double
        L.orc_riemann.argtypes = [ctypes.c_double, _D, _D, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, _D, _D, _D, ctypes.POINTER(ctypes.c_int)]
        L.orc_predictor_cell.argtypes = [ctypes.POINTER(Cfg), ctypes.c_double, _D, _D, _D, _D,
                                         ctypes.POINTER(ctypes.c_int)]
        L.orc_predictor_matrices.argtypes = [ctypes.c_int, _D, _D, _D, _D, _D]
        L.orc_smax.argtypes = [ctypes.POINTER(Cfg), ctypes.c_int, _D]
        L.orc_smax.restype = ctypes.c_double
        L.orc_segment_step.argtypes = [ctypes.POINTER(Cfg), ctypes.c_int, ctypes.c_double, _D, _D,
                                       ctypes.c_double, ctypes.c_double, _D, _D, _D, _D,
                                       ctypes.POINTER(Stats)]
        L.orc_init_interfaces.argtypes = [ctypes.POINTER(Cfg), ctypes.c_int, _D, _D, _D]
        L.orc_run_segment.argtypes = [ctypes.POINTER(Cfg), ctypes.c_int, ctypes.c_double, _D, _D,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int64, _D, _I64,
                                      ctypes.POINTER(Stats)]
        L.orc_trrs.argtypes = [ctypes.c_double, _D, _D, _D, _D, _D]
        L.orc_side_matrix.argtypes = [ctypes.c_int, ctypes.c_int, _D]
        L.orc_oi.argtypes = [ctypes.c_int, _D, ctypes.c_double]
        L.orc_oi.restype = ctypes.c_double
        L.orc_eigvec.argtypes = [ctypes.c_double, _D, _D]
        L.orc_recon_nl_cell.argtypes = [ctypes.POINTER(Cfg), ctypes.c_double, _D, _D, _D]
        L.orc_run_segments.argtypes = [ctypes.POINTER(Cfg), ctypes.c_int, _I64, _D, _D, _D, _D,
                                       ctypes.c_double, ctypes.c_int64, ctypes.POINTER(Stats)]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def cfg(system=ADVECTION, order=3, cfl=0.9, lam=1.0, gamma=1.4, bc=PERIODIC, newton_tol=1e-12,
        newton_max=50, picard_tol=1e-13, picard_max=64, recon=LINEAR,
        nl_lambda_c=LAMBDA_C_PRINTED, nl_eps=1e-14, nl_r=4.0, datum=DATUM_EXACT, source=SOURCE_NONE,
        kappa=0.0) -> Cfg:
    """GRPrecNL weights: r, eps and lambda_C = 1e9 as printed (Sec. 3.3).  With
    1e9 GRPrecNL coincides with GRPrec on smooth data; the paper's GRPrecNL
    results (Sec. 4.2.3 table, Sec. 4.2.2 square wave) are reproduced with
    lambda_C = 10 (pass nl_lambda_c=LAMBDA_C_TABLE).  source=SOURCE_LINEAR adds
    S(Q) = -kappa Q to eq. (eq_hyperbolic_system) (eqs. eq_finite_volume and
    source)."""
    return Cfg(system, order - 1, cfl, lam, gamma, bc, bc, newton_tol, newton_max, picard_tol,
               picard_max, recon, nl_lambda_c, nl_eps, nl_r, datum, source, kappa)


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle error {code} in {where}")
        self.code = code


def _chk(rc, where):
    if rc != OK:
        raise OracleError(rc, where)


# ---------------------------------------------------------------- pins / pieces
def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    _chk(lib().orc_gauss_legendre(n, _p(x), _p(w)), "gauss_legendre")
    return x, w


def recon_matrix(m: int) -> np.ndarray:
    """(m+1) x 5 matrix: monomial coefficients in xi in [-1/2,1/2] from
    (q_{i-1}, q_i, q_{i+1}, V_{i-1/2}, V_{i+1/2})."""
    R = np.zeros((m + 1, 5))
    _chk(lib().orc_recon_matrix(m, _p(R)), "recon_matrix")
    return R


def side_matrix(m: int, side: int) -> np.ndarray:
    """(m+1) x 7 matrix of GRPrecNL's left (side 0) or right (side 1)
    polynomial: monomial coefficients from (q_{i-1}, q_i, q_{i+1}, V_{i-1/2},
    V_{i+1/2}, V_{i-3/2}, V_{i+3/2})."""
    M = np.zeros((m + 1, 7))
    _chk(lib().orc_side_matrix(m, side, _p(M)), "side_matrix")
    return M


def oi(coef: np.ndarray, dx: float) -> float:
    """Oscillation indicator of a polynomial given by monomial coefficients in
    xi = (x - x_i)/dx."""
    c = np.ascontiguousarray(coef, dtype=np.float64)
    return lib().orc_oi(len(c) - 1, _p(c), dx)


def eigvec(gamma: float, Q) -> np.ndarray:
    """Right eigenvectors (columns) of the Euler flux Jacobian at conserved Q."""
    q = np.ascontiguousarray(Q, dtype=np.float64)
    R = np.zeros((3, 3))
    _chk(lib().orc_eigvec(gamma, _p(q), _p(R)), "eigvec")
    return R


def recon_nl_cell(c: Cfg, dx: float, d: np.ndarray):
    """GRPrecNL polynomial of one cell: d is [nv][7] data, returns
    (coefficients [nv][m+1], weights [nv][3])."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    nv = d.shape[0]
    coef = np.zeros((nv, c.m + 1))
    beta = np.zeros((nv, 3))
    _chk(lib().orc_recon_nl_cell(ctypes.byref(c), dx, _p(d), _p(coef), _p(beta)), "recon_nl_cell")
    return coef, beta


def predictor_matrices(m: int):
    n = m + 1
    g, w, kl0 = np.zeros(n), np.zeros(n), np.zeros(n)
    D, KW = np.zeros((n, n)), np.zeros((n, n))
    _chk(lib().orc_predictor_matrices(m, _p(g), _p(w), _p(D), _p(kl0), _p(KW)), "pred_mats")
    return g, w, D, kl0, KW


def predictor_cell(c: Cfg, nu: float, w: np.ndarray):
    """w: [nvar][m+1] nodal initial data -> (q[nvar][m+1][m+1], TL, TR [nvar][m+2], iters)."""
    n = c.m + 1
    nv = 1 if c.system == ADVECTION else 3
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(nv, n)
    q = np.zeros((nv, n, n))
    TL = np.zeros((nv, n + 1))
    TR = np.zeros((nv, n + 1))
    it = ctypes.c_int(0)
    _chk(lib().orc_predictor_cell(ctypes.byref(c), nu, _p(w), _p(q), _p(TL), _p(TR),
                                  ctypes.byref(it)), "predictor")
    return q, TL, TR, it.value


def riemann(gamma, WL, WR, guess=-1.0, tol=1e-12, maxit=50):
    """Exact Euler RS on primitive states -> (p*, u*, W(x/t=0), iterations)."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    W0 = np.zeros(3)
    ps, us = ctypes.c_double(0), ctypes.c_double(0)
    it = ctypes.c_int(0)
    rc = lib().orc_riemann(gamma, _p(WL), _p(WR), guess, tol, maxit, ctypes.byref(ps),
                           ctypes.byref(us), _p(W0), ctypes.byref(it))
    _chk(rc, "riemann")
    return ps.value, us.value, W0, it.value


def riemann_rc(gamma, WL, WR, guess=-1.0, tol=1e-12, maxit=50):
    """Like riemann() but returns (rc, p*, iterations) without raising."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    W0 = np.zeros(3)
    ps, us = ctypes.c_double(0), ctypes.c_double(0)
    it = ctypes.c_int(0)
    rc = lib().orc_riemann(gamma, _p(WL), _p(WR), guess, tol, maxit, ctypes.byref(ps),
                           ctypes.byref(us), _p(W0), ctypes.byref(it))
    return rc, ps.value, it.value


def trrs(gamma, WL, WR):
    """Two-rarefaction solver: (p*, u*, primitive state at x/t = 0)."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    ps, us, W0 = np.zeros(1), np.zeros(1), np.zeros(3)
    _chk(lib().orc_trrs(gamma, _p(WL), _p(WR), _p(ps), _p(us), _p(W0)), "trrs")
    return ps[0], us[0], W0


def pvrs_guess(gamma, WL, WR):
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    return lib().orc_pvrs_guess(gamma, _p(WL), _p(WR))


def smax(c: Cfg, q: np.ndarray) -> float:
    q = np.ascontiguousarray(q, dtype=np.float64)
    return lib().orc_smax(ctypes.byref(c), q.shape[-1], _p(q))


def init_interfaces(c: Cfg, vl: np.ndarray, vr: np.ndarray) -> np.ndarray:
    vl = np.ascontiguousarray(vl, dtype=np.float64)
    vr = np.ascontiguousarray(vr, dtype=np.float64)
    v = np.zeros_like(vl)
    _chk(lib().orc_init_interfaces(ctypes.byref(c), vl.shape[-1], _p(vl), _p(vr), _p(v)),
         "init_interfaces")
    return v


def step(c: Cfg, dx: float, q: np.ndarray, v: np.ndarray, t: float, t_end: float):
    """One step of one domain.  Returns (q_new, v_new, dt, t_new, stats)."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    qo, vo = np.zeros_like(q), np.zeros_like(v)
    dt, tn = ctypes.c_double(0), ctypes.c_double(0)
    st = Stats()
    n = q.shape[-1]
    _chk(lib().orc_segment_step(ctypes.byref(c), n, dx, _p(q), _p(v), t, t_end, _p(qo), _p(vo),
                                ctypes.byref(dt), ctypes.byref(tn), ctypes.byref(st)), "step")
    return qo, vo, dt.value, tn.value, st


def run(c: Cfg, dx: float, q: np.ndarray, v: np.ndarray, t0: float, t_end: float,
        max_steps: int = 1 << 62):
    """Advance one domain; returns (q, v, t, steps, stats).  Inputs are copied."""
    q = np.array(q, dtype=np.float64, order="C")
    v = np.array(v, dtype=np.float64, order="C")
    t = ctypes.c_double(0)
    k = ctypes.c_int64(0)
    st = Stats()
    _chk(lib().orc_run_segment(ctypes.byref(c), q.shape[-1], dx, _p(q), _p(v), t0, t_end, max_steps,
                               ctypes.byref(t), ctypes.byref(k), ctypes.byref(st)), "run")
    return q, v, t.value, k.value, st


def run_segments(c: Cfg, cell_off: np.ndarray, dx: np.ndarray, q: np.ndarray, v: np.ndarray,
                 t: np.ndarray, t_end: float, max_steps: int):
    """Advance back-to-back segments (flat SoA); returns copies (q, v, t, stats)."""
    cell_off = np.ascontiguousarray(cell_off, dtype=np.int64)
    dx = np.ascontiguousarray(dx, dtype=np.float64)
    q = np.array(q, dtype=np.float64, order="C")
    v = np.array(v, dtype=np.float64, order="C")
    t = np.array(t, dtype=np.float64, order="C")
    st = Stats()
    _chk(lib().orc_run_segments(ctypes.byref(c), len(dx), cell_off.ctypes.data_as(_I64), _p(dx),
                                _p(q), _p(v), _p(t), t_end, max_steps, ctypes.byref(st)),
         "run_segments")
    return q, v, t, st
