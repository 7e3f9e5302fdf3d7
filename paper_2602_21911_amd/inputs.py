"""Seeded synthetic inputs for the GRPrec step (shared by the GPU path and the
oracle; contains none of the method's arithmetic).

Every workload of the paper is an analytic initial condition, so the inputs are
exact cell averages of that condition plus the one-sided limits of the initial
condition at every interface (the library and the oracle each turn those into
the first-step interface data with their own Riemann solver).

Workloads
---------
* linear advection on periodic [x0, x0+L]: ``sin(2 pi x)``, ``sin^4(pi x)``
  (the paper's convergence test, Sec. 4.2.3) and the square wave (Sec. 4.2.2);
* Euler density wave rho = 1 + a sin(2 pi k x), constant u and p (Sec. 4.3.1);
* Euler shock tubes (Sod data of Sec. 4.3.2 and seeded random tubes);
* a network of independent Euler segments of uneven length (log-uniform cell
  counts, uniform lengths, per-segment wavenumber), all from one seed.

Layout: structure-of-arrays float64, ``q[var][cell]`` and ``v[var][iface]``.
A domain of n cells has n+1 interfaces, interface k at x0 + k dx.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_NETWORK = 20260221
SEED_TUBES_TRAIN = 20260222
SEED_TUBES_HELDOUT = 20260223
SEED_TUBE_NETWORK = 20260224
SEED_TUBES_GATE = 20260225


def grid(n: int, x0: float = 0.0, length: float = 1.0):
    dx = length / n
    xf = x0 + dx * np.arange(n + 1)
    return dx, xf


# ----------------------------------------------------------------- advection
def adv_sin2pi(n, x0=0.0, length=1.0, k=1):
    """u0 = sin(2 pi k x): exact cell averages, interface limits."""
    dx, xf = grid(n, x0, length)
    w = 2 * np.pi * k
    q = (np.cos(w * xf[:-1]) - np.cos(w * xf[1:])) / (w * dx)
    val = np.sin(w * xf)
    return dx, q[None, :].copy(), val[None, :].copy(), val[None, :].copy()


def adv_sin4(n, x0=-1.0, length=2.0):
    """u0 = sin^4(pi x) = 3/8 - cos(2 pi x)/2 + cos(4 pi x)/8 (Sec. 4.2.3)."""
    dx, xf = grid(n, x0, length)
    a, b = xf[:-1], xf[1:]
    q = (3.0 / 8.0 - 0.5 * (np.sin(2 * np.pi * b) - np.sin(2 * np.pi * a)) / (2 * np.pi * dx)
         + 0.125 * (np.sin(4 * np.pi * b) - np.sin(4 * np.pi * a)) / (4 * np.pi * dx))
    val = np.sin(np.pi * xf) ** 4
    return dx, q[None, :].copy(), val[None, :].copy(), val[None, :].copy()


def adv_sin4_exact_avg(n, t, lam=1.0, x0=-1.0, length=2.0):
    """Exact cell averages of sin^4(pi (x - lam t)) on the periodic grid."""
    dx, xf = grid(n, x0, length)
    a, b = xf[:-1] - lam * t, xf[1:] - lam * t
    return (3.0 / 8.0 - 0.5 * (np.sin(2 * np.pi * b) - np.sin(2 * np.pi * a)) / (2 * np.pi * dx)
            + 0.125 * (np.sin(4 * np.pi * b) - np.sin(4 * np.pi * a)) / (4 * np.pi * dx))


def adv_sin2pi_exact_avg(n, t, lam=1.0, x0=0.0, length=1.0, k=1):
    dx, xf = grid(n, x0, length)
    w = 2 * np.pi * k
    a, b = xf[:-1] - lam * t, xf[1:] - lam * t
    return (np.cos(w * a) - np.cos(w * b)) / (w * dx)


def adv_square(n, x0=0.0, length=1.0, lo=0.25, hi=0.75):
    """u0 = 1 on [lo, hi], else 0; jumps sit on interfaces when n*lo, n*hi are integers."""
    dx, xf = grid(n, x0, length)
    a, b = xf[:-1], xf[1:]
    q = np.clip(np.minimum(b, hi) - np.maximum(a, lo), 0.0, None) / dx
    left = ((xf > lo) & (xf <= hi)).astype(np.float64)   # limit from the left
    right = ((xf >= lo) & (xf < hi)).astype(np.float64)  # limit from the right
    return dx, q[None, :].copy(), left[None, :].copy(), right[None, :].copy()


def adv_polynomial(n, coeffs, x0=0.0, length=1.0):
    """u0 = sum_j coeffs[j] x^j (exact averages and point values)."""
    dx, xf = grid(n, x0, length)
    c = np.asarray(coeffs, dtype=np.float64)
    prim = np.concatenate([[0.0], c / np.arange(1, len(c) + 1)])  # antiderivative
    P = np.polynomial.polynomial.polyval(xf, prim)
    q = (P[1:] - P[:-1]) / dx
    val = np.polynomial.polynomial.polyval(xf, c)
    return dx, q[None, :].copy(), val[None, :].copy(), val[None, :].copy()


# ----------------------------------------------------------------- Euler
def prim_to_cons(rho, u, p, gamma=1.4):
    rho = np.asarray(rho, dtype=np.float64)
    return np.stack([rho, rho * u * np.ones_like(rho),
                     p / (gamma - 1.0) * np.ones_like(rho) + 0.5 * rho * u * u])


def euler_density_wave(n, amp=0.2, u=1.0, p=1.0, gamma=1.4, x0=0.0, length=1.0, k=1):
    """rho = 1 + amp sin(2 pi k x), u, p constant: conserved averages are exact
    because rho u and E are affine in rho."""
    dx, xf = grid(n, x0, length)
    w = 2 * np.pi * k
    rho_avg = 1.0 + amp * (np.cos(w * xf[:-1]) - np.cos(w * xf[1:])) / (w * dx)
    q = prim_to_cons(rho_avg, u, p, gamma)
    rho_f = 1.0 + amp * np.sin(w * xf)
    v = prim_to_cons(rho_f, u, p, gamma)
    return dx, q, v, v.copy()


def euler_density_wave_exact_rho(n, t, amp=0.2, u=1.0, x0=0.0, length=1.0, k=1):
    dx, xf = grid(n, x0, length)
    w = 2 * np.pi * k
    a, b = xf[:-1] - u * t, xf[1:] - u * t
    return 1.0 + amp * (np.cos(w * a) - np.cos(w * b)) / (w * dx)


def euler_shock_tube(n, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), xc=0.5, gamma=1.4,
                     x0=0.0, length=1.0):
    """Piecewise-constant Riemann data; xc should fall on an interface."""
    dx, xf = grid(n, x0, length)
    xm = 0.5 * (xf[:-1] + xf[1:])
    isl = xm < xc
    rho = np.where(isl, left[0], right[0])
    u = np.where(isl, left[1], right[1])
    p = np.where(isl, left[2], right[2])
    q = prim_to_cons(rho, u, p, gamma)
    lim_l = xf <= xc + 1e-12 * length  # left limit at interface takes the left state up to xc
    lim_r = xf < xc - 1e-12 * length
    vl = prim_to_cons(np.where(lim_l, left[0], right[0]), np.where(lim_l, left[1], right[1]),
                      np.where(lim_l, left[2], right[2]), gamma)
    vr = prim_to_cons(np.where(lim_r, left[0], right[0]), np.where(lim_r, left[1], right[1]),
                      np.where(lim_r, left[2], right[2]), gamma)
    return dx, q, vl, vr


def random_tube_states(seed: int, count: int):
    """Random Riemann data: rho log-uniform [0.01, 10], u uniform [-3, 3],
    p log-uniform [1e-3, 1e3] on each side.  Returns (WL, WR) [count, 3]."""
    rng = np.random.default_rng(seed)

    def side():
        rho = np.exp(rng.uniform(np.log(0.01), np.log(10.0), count))
        u = rng.uniform(-3.0, 3.0, count)
        p = np.exp(rng.uniform(np.log(1e-3), np.log(1e3), count))
        return np.stack([rho, u, p], axis=1)

    return side(), side()


# ----------------------------------------------------------------- networks
@dataclass
class Network:
    n_cells: np.ndarray   # [S] int64
    lengths: np.ndarray   # [S]
    wavenum: np.ndarray   # [S]
    cell_off: np.ndarray  # [S+1] int64
    dx: np.ndarray        # [S]
    q: np.ndarray         # [3][total]
    vl: np.ndarray        # [3][total + S]
    vr: np.ndarray        # [3][total + S]


def network(n_seg=10000, seed=SEED_NETWORK, nmin=3, nmax=2000, lmin=0.01, lmax=1.0, kmin=1.0,
            kmax=8.0, amp=0.1, u=0.5, p=1.0, gamma=1.4) -> Network:
    """Independent Euler segments: n_s = round(exp(U[ln nmin, ln nmax])), length
    U[lmin, lmax], rho = 1 + amp sin(k x_local) with k U[kmin, kmax] and x_local
    measured from the segment's left end, u and p constant."""
    rng = np.random.default_rng(seed)
    n_cells = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), n_seg))).astype(np.int64)
    lengths = rng.uniform(lmin, lmax, n_seg)
    wavenum = rng.uniform(kmin, kmax, n_seg)
    cell_off = np.zeros(n_seg + 1, dtype=np.int64)
    cell_off[1:] = np.cumsum(n_cells)
    total = int(cell_off[-1])
    dx = lengths / n_cells
    rho_c = np.empty(total)
    rho_f = np.empty(total + n_seg)
    for s in range(n_seg):
        n = int(n_cells[s])
        xf = dx[s] * np.arange(n + 1)
        k = wavenum[s]
        c0 = int(cell_off[s])
        rho_c[c0:c0 + n] = 1.0 + amp * (np.cos(k * xf[:-1]) - np.cos(k * xf[1:])) / (k * dx[s])
        rho_f[c0 + s:c0 + s + n + 1] = 1.0 + amp * np.sin(k * xf)
    q = prim_to_cons(rho_c, u, p, gamma)
    v = prim_to_cons(rho_f, u, p, gamma)
    return Network(n_cells, lengths, wavenum, cell_off, dx, q, v, v.copy())


def tube_network(n_seg=10000, seed=SEED_TUBE_NETWORK, nmin=20, nmax=200, ratio=2.0, du=0.1,
                 gamma=1.4) -> Network:
    """Independent shock tubes of unit length: n_s uniform integer in
    [nmin, nmax), the jump at interface n_s // 2; left state rho, p
    log-uniform [0.5, 2], right state rho and p the left ones times
    exp(U[-ln ratio, ln ratio]), u_L and u_R uniform [-du, du].  At the jump
    the left (right) interface limit is the left (right) state."""
    rng = np.random.default_rng(seed)
    n_cells = rng.integers(nmin, nmax, n_seg).astype(np.int64)
    lr = np.log(ratio)
    rl = np.exp(rng.uniform(np.log(0.5), np.log(2.0), n_seg))
    pl = np.exp(rng.uniform(np.log(0.5), np.log(2.0), n_seg))
    rr = rl * np.exp(rng.uniform(-lr, lr, n_seg))
    pr = pl * np.exp(rng.uniform(-lr, lr, n_seg))
    ul = rng.uniform(-du, du, n_seg)
    ur = rng.uniform(-du, du, n_seg)
    lengths = np.ones(n_seg)
    cell_off = np.zeros(n_seg + 1, dtype=np.int64)
    cell_off[1:] = np.cumsum(n_cells)
    total = int(cell_off[-1])
    dx = lengths / n_cells
    W = np.empty((3, total))
    WL = np.empty((3, total + n_seg))
    WR = np.empty((3, total + n_seg))
    for s in range(n_seg):
        n = int(n_cells[s])
        c0, i0, j = int(cell_off[s]), int(cell_off[s]) + s, n // 2
        left, right = (rl[s], ul[s], pl[s]), (rr[s], ur[s], pr[s])
        for v in range(3):
            W[v, c0:c0 + j] = left[v]
            W[v, c0 + j:c0 + n] = right[v]
            WL[v, i0:i0 + j + 1] = left[v]      # interfaces 0..j: left limit is the left state
            WL[v, i0 + j + 1:i0 + n + 1] = right[v]
            WR[v, i0:i0 + j] = left[v]          # interfaces 0..j-1: right limit is the left state
            WR[v, i0 + j:i0 + n + 1] = right[v]
    q = prim_to_cons(W[0], W[1], W[2], gamma)
    vl = prim_to_cons(WL[0], WL[1], WL[2], gamma)
    vr = prim_to_cons(WR[0], WR[1], WR[2], gamma)
    return Network(n_cells, lengths, np.zeros(n_seg), cell_off, dx, q, vl, vr)
