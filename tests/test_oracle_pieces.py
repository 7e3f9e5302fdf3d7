"""Pins of the oracle's building blocks against mathematics that does not go
through the oracle's own code: library quadrature, exact polynomial
integration, independent least-squares solves and the Galerkin weak form
evaluated with a separate quadrature."""
import numpy as np
import numpy.polynomial.legendre as npleg
import numpy.polynomial.polynomial as P
import pytest

import oracle

RNG = np.random.default_rng(1234)


# ------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_gauss_legendre_matches_numpy(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = npleg.leggauss(n)
    np.testing.assert_allclose(x, 0.5 * (xr + 1.0), atol=1e-15)
    np.testing.assert_allclose(w, 0.5 * wr, atol=1e-15)


# ------------------------------------------------------------- reconstruction
def _conditions(coef):
    """(mean_{i-1}, mean_i, mean_{i+1}, p(-1/2), p(1/2)) of a monomial polynomial in xi."""
    prim = P.polyint(coef)
    mean = lambda a, b: P.polyval(b, prim) - P.polyval(a, prim)
    return np.array([mean(-1.5, -0.5), mean(-0.5, 0.5), mean(0.5, 1.5),
                     P.polyval(-0.5, coef), P.polyval(0.5, coef)])


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_reconstruction_reproduces_polynomials(m):
    """Data sampled from any polynomial of degree <= m give that polynomial back
    (Sec. 3.1: every condition is then met exactly, so the least-squares
    residual is zero)."""
    R = oracle.recon_matrix(m)
    for _ in range(20):
        coef = RNG.normal(size=m + 1)
        got = R @ _conditions(coef)
        np.testing.assert_allclose(got, coef, atol=1e-13)


@pytest.mark.parametrize("m", [2, 4])
def test_reconstruction_exact_conditions(m):
    """Degrees 2 and 4 impose their conditions exactly (Sec. 3.1)."""
    R = oracle.recon_matrix(m)
    idx = [1, 3, 4] if m == 2 else [0, 1, 2, 3, 4]
    for _ in range(20):
        d = RNG.normal(size=5)
        c = R @ d
        np.testing.assert_allclose(_conditions(c)[idx], d[idx], atol=1e-13)


@pytest.mark.parametrize("m", [1, 3])
def test_reconstruction_least_squares_optimum(m):
    """Degrees 1 and 3: cell-i mean exact, unit-weight least squares on the rest
    (Sec. 3.1 functionals).  Checked by an independent solve: parametrise the
    constraint's null space and call numpy's lstsq."""
    R = oracle.recon_matrix(m)
    ls = [3, 4] if m == 1 else [0, 2, 3, 4]
    # condition rows as linear maps of the coefficients
    rows = np.array([_conditions(np.eye(m + 1)[j]) for j in range(m + 1)]).T  # 5 x (m+1)
    C = rows[1:2]
    A = rows[ls]
    _, _, Vt = np.linalg.svd(C)
    N = Vt[1:].T  # null space of C
    for _ in range(20):
        d = RNG.normal(size=5)
        c0 = np.linalg.lstsq(C, d[1:2], rcond=None)[0]  # particular solution
        z = np.linalg.lstsq(A @ N, d[ls] - A @ c0, rcond=None)[0]
        ref = c0 + N @ z
        np.testing.assert_allclose(R @ d, ref, atol=1e-13)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_reconstruction_uniqueness(m):
    """Sec. 3.2: the conditions determine a unique polynomial, i.e. the
    constraint block has full rank and the least-squares problem on its null
    space is non-degenerate."""
    rows = np.array([_conditions(np.eye(m + 1)[j]) for j in range(m + 1)]).T
    ex = {1: [1], 2: [1, 3, 4], 3: [1], 4: [0, 1, 2, 3, 4]}[m]
    assert np.linalg.matrix_rank(rows[ex]) == len(ex)
    assert np.linalg.matrix_rank(rows) == m + 1


def test_reconstruction_closed_forms():
    """Hand-derived closed forms in the zero-mean basis (derived separately from
    the paper's definitions): p = qbar + a1 xi + a2 (xi^2 - 1/12) + a3 xi^3 + a4 (xi^4 - 1/80)."""
    for _ in range(10):
        qm, q0, qp, vl, vr = RNG.normal(size=5)
        DI, SI, DC, SC = vr - vl, vl + vr - 2 * q0, qp - qm, qp + qm - 2 * q0
        forms = {
            1: [DI, 0, 0, 0],
            2: [DI, 3 * SI, 0, 0],
            3: [1.25 * DI - DC / 8, (3 * SI + 18 * SC) / 37, DC / 2 - DI, 0],
            4: [1.25 * DI - DC / 8, 3.75 * SI - SC / 8, DC / 2 - DI, 5 * SC / 12 - 2.5 * SI],
        }
        for m, (a1, a2, a3, a4) in forms.items():
            mono = np.array([q0 - a2 / 12 - a4 / 80, a1, a2, a3, a4])[: m + 1]
            got = oracle.recon_matrix(m) @ np.array([qm, q0, qp, vl, vr])
            np.testing.assert_allclose(got, mono, atol=1e-13)


# ------------------------------------------------------------- predictor
def _lagrange_basis(nodes):
    """Lagrange polynomials on nodes as numpy power-series coefficient arrays."""
    out = []
    for k in range(len(nodes)):
        others = np.delete(nodes, k)
        c = P.polyfromroots(others)
        out.append(c / P.polyval(nodes[k], c))
    return out


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_predictor_matrices_independent(m):
    """D[a][k] = l_k'(g_a); K^{-1} l(0) = 1; K^{-1} diag(w) from exactly
    integrated Lagrange polynomials (numpy polynomial arithmetic)."""
    g, w, D, kl0, KW = oracle.predictor_matrices(m)
    n = m + 1
    L = _lagrange_basis(g)
    Dref = np.array([[P.polyval(g[a], P.polyder(L[k])) for k in range(n)] for a in range(n)])
    np.testing.assert_allclose(D, Dref, atol=1e-11)
    K = np.zeros((n, n))
    for b in range(n):
        for l in range(n):
            integ = P.polyint(P.polymul(P.polyder(L[b]), L[l]))
            K[b, l] = P.polyval(1, L[b]) * P.polyval(1, L[l]) - (P.polyval(1, integ) - P.polyval(0, integ))
    np.testing.assert_allclose(kl0, np.ones(n), atol=1e-12)
    np.testing.assert_allclose(KW, np.linalg.solve(K, np.diag(w)), atol=1e-11)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_predictor_advection_is_exact_translation(m):
    """For q_t + lam q_x = 0 the space-time DG solution of polynomial data is
    the exact translation w(xi - nu t) (it lies in the trial space)."""
    c = oracle.cfg(oracle.ADVECTION, m + 1, lam=1.0)
    g, _, _, _, _ = oracle.predictor_matrices(m)
    for nu in (0.1, 0.55, 0.9, 1.0):
        coef = RNG.normal(size=m + 1)  # polynomial in xi in [0,1]
        w = P.polyval(g, coef)[None, :]
        q, TL, TR, it = oracle.predictor_cell(c, nu, w)
        assert it <= m + 1
        for a in range(m + 1):
            for b in range(m + 1):
                assert abs(q[0, a, b] - P.polyval(g[a] - nu * g[b], coef)) < 1e-12
        times = np.concatenate([g, [1.0]])
        np.testing.assert_allclose(TL[0], P.polyval(0.0 - nu * times, coef), atol=1e-12)
        np.testing.assert_allclose(TR[0], P.polyval(1.0 - nu * times, coef), atol=1e-12)


def _euler_flux(Q, gam=1.4):
    r, mo, E = Q
    u = mo / r
    p = (gam - 1) * (E - 0.5 * mo * u)
    return np.array([mo, mo * u + p, u * (E + p)])


@pytest.mark.parametrize("m", [1, 2, 3])
def test_predictor_euler_weak_form(m):
    """The converged Euler predictor satisfies the space-time Galerkin equations
    (time-upwind at t = 0, nodal flux interpolant), evaluated here with a
    separate 12-point quadrature and numpy Lagrange polynomials."""
    c = oracle.cfg(oracle.EULER, m + 1)
    g, _, _, _, _ = oracle.predictor_matrices(m)
    n = m + 1
    L = _lagrange_basis(g)
    xq, wq = npleg.leggauss(12)
    xq, wq = 0.5 * (xq + 1), 0.5 * wq
    Lx = np.array([P.polyval(xq, L[k]) for k in range(n)])            # [k][quad]
    dLx = np.array([P.polyval(xq, P.polyder(L[k])) for k in range(n)])
    L0 = np.array([P.polyval(0.0, L[k]) for k in range(n)])
    nu = 0.35
    # smooth, clearly non-trivial primitive data across the cell
    rho = 1.0 + 0.3 * np.sin(2.0 * g + 0.3)
    u = 0.4 + 0.5 * np.cos(1.7 * g)
    p = 1.0 + 0.4 * g
    w = np.stack([rho, rho * u, p / 0.4 + 0.5 * rho * u * u])
    q, _, _, it = oracle.predictor_cell(c, nu, w)
    F = np.zeros_like(q)
    for a in range(n):
        for b in range(n):
            F[:, a, b] = _euler_flux(q[:, a, b])
    # fields at quadrature points: [var][xi_q][t_q]
    qh = np.einsum("vab,ax,bt->vxt", q, Lx, Lx)
    dqdt = np.einsum("vab,ax,bt->vxt", q, Lx, dLx)
    dFdx = np.einsum("vab,ax,bt->vxt", F, dLx, Lx)
    q0 = np.einsum("vab,ax,b->vx", q, Lx, L0)       # q_h(xi, 0+)
    wx = np.einsum("va,ax->vx", w, Lx)              # initial data w(xi)
    for a in range(n):
        for b in range(n):
            th = np.outer(Lx[a], Lx[b])
            res = (np.einsum("vxt,xt,x,t->v", dqdt + nu * dFdx, th, wq, wq)
                   + np.einsum("vx,x,x->v", (q0 - wx) * L0[b], Lx[a], wq))
            assert np.all(np.abs(res) < 2e-12), (a, b, res)
    assert np.all(np.isfinite(qh))


def test_predictor_euler_constant_state():
    for m in (1, 2, 3, 4):
        c = oracle.cfg(oracle.EULER, m + 1)
        Q = np.array([0.7, -0.3, 2.1])
        w = np.repeat(Q[:, None], m + 1, axis=1)
        q, TL, TR, it = oracle.predictor_cell(c, 0.8, w)
        np.testing.assert_allclose(q, np.repeat(w[:, :, None], m + 1, axis=2), rtol=0, atol=1e-14)
        np.testing.assert_allclose(TL, np.repeat(Q[:, None], m + 2, axis=1), atol=1e-14)
