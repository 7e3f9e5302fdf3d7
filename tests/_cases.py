"""Shared test helpers: run one workload through the oracle and through the
GPU library from the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2602_21911_amd import inputs as I


def rel_linf(gpu: np.ndarray, ref: np.ndarray) -> float:
    """max over variables of max_i |gpu - ref| / max_i |ref|."""
    gpu = np.atleast_2d(gpu)
    ref = np.atleast_2d(ref)
    out = 0.0
    for g, r in zip(gpu, ref):
        scale = np.abs(r).max()
        out = max(out, np.abs(g - r).max() / (scale if scale > 0 else 1.0))
    return out


def oracle_cfg(system, order, bc, cfl=0.9, lam=1.0, gamma=1.4):
    return oracle.cfg(system, order, cfl=cfl, lam=lam, gamma=gamma, bc=bc)


def advection_case(kind: str, n: int):
    if kind == "sin2pi":
        return I.adv_sin2pi(n)
    if kind == "square":
        return I.adv_square(n)
    if kind == "sin4":
        return I.adv_sin4(n)
    raise ValueError(kind)


def acoustic_case(n: int, amp=0.2):
    """Smooth periodic data with varying rho, u and p (genuinely nonlinear)."""
    dx, xf = I.grid(n)
    gx, gw = np.polynomial.legendre.leggauss(8)
    xq = 0.5 * (xf[:-1, None] + xf[1:, None]) + 0.5 * dx * gx[None, :]
    prim = lambda x: (1.0 + amp * np.sin(2 * np.pi * x), 0.3 * np.sin(2 * np.pi * x + 0.4),
                      1.0 + 0.28 * np.cos(2 * np.pi * x))
    r, u, p = prim(xq)
    Q = I.prim_to_cons(r, u, p)
    q = (Q * (0.5 * gw)[None, None, :]).sum(axis=2)
    r, u, p = prim(xf)
    v = I.prim_to_cons(r, u, p)
    return dx, q, v, v.copy()


def network_case(n_seg: int, seed: int, nmax: int = 2000):
    return I.network(n_seg=n_seg, seed=seed, nmax=nmax)
