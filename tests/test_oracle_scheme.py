"""Pins of the oracle's whole step: exactness on polynomial data, exact shift at
Courant number 1, linear stability (the paper's Courant-1 claim, Sec. 4.1),
conservation, the printed advection convergence table (Sec. 4.2.3), the
observed Euler rates (Sec. 4.3.1), and reductions of Euler to advection."""
import os

import numpy as np
import pytest

import oracle
from paper_2602_21911_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
RNG = np.random.default_rng(99)


def _load_table(name):
    rows = np.loadtxt(os.path.join(HERE, "golden", name), comments="#")
    return {(int(r[0]), int(r[1])): r[2:] for r in rows}


# ------------------------------------------------------------- advection
@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_advection_polynomial_data_exact(order):
    """Reconstruction, evolution and GL flux integration are all exact for data
    from a polynomial of degree <= m, so one step reproduces the exact solution
    away from the periodic wrap (Sec. 3.1 + eq. eq_finite_volume)."""
    m = order - 1
    n = 24
    coef = RNG.normal(size=m + 1)
    dx, q, vl, vr = I.adv_polynomial(n, coef)
    c = oracle.cfg(oracle.ADVECTION, order, cfl=0.7)
    v = oracle.init_interfaces(c, vl, vr)
    qn, vn, dt, _, _ = oracle.step(c, dx, q, v, 0.0, 10.0)
    shifted = np.polynomial.polynomial.polyval(np.array([[0.0, -dt]]).T, 1)  # noqa: F841
    # exact translated data: u0(x - dt)
    c_sh = np.polynomial.polynomial.polycompanion  # noqa: F841
    xs = np.poly1d(coef[::-1])
    sh = np.poly1d([1.0, -dt])
    coef_t = xs(sh).c[::-1]
    _, qe, ve, _ = I.adv_polynomial(n, coef_t)
    sl = slice(4, n - 4)
    np.testing.assert_allclose(qn[0, sl], qe[0, sl], atol=1e-12)
    np.testing.assert_allclose(vn[0, 4:n - 3], ve[0, 4:n - 3], atol=1e-12)


@pytest.mark.parametrize("order", [3, 5])
def test_advection_courant_one_exact_shift(order):
    """At Courant number 1 degrees 2 and 4 shift the data by exactly one cell:
    they interpolate both interface values, so the polynomial's integral over
    the cell and its left-end value move one cell to the right."""
    n = 32
    c = oracle.cfg(oracle.ADVECTION, order, cfl=1.0)
    q = RNG.normal(size=(1, n))
    v = RNG.normal(size=(1, n + 1))
    v[0, n] = v[0, 0]
    qn, vn, dt, _, _ = oracle.step(c, 1.0 / n, q, v, 0.0, 10.0)
    np.testing.assert_allclose(qn[0], np.roll(q[0], 1), atol=1e-13)
    np.testing.assert_allclose(vn[0, 1:], v[0, :n], atol=1e-13)


def _step_matrix(order, cfl, n=16):
    """Matrix of one periodic advection step on the state (q_0..q_{n-1}, V_0..V_{n-1})."""
    c = oracle.cfg(oracle.ADVECTION, order, cfl=cfl)
    A = np.zeros((2 * n, 2 * n))
    for j in range(2 * n):
        q = np.zeros((1, n))
        v = np.zeros((1, n + 1))
        if j < n:
            q[0, j] = 1.0
        else:
            v[0, j - n] = 1.0
            if j == n:
                v[0, n] = 1.0
        qn, vn, _, _, _ = oracle.step(c, 1.0 / n, q, v, 0.0, 10.0)
        A[:n, j] = qn[0]
        A[n:, j] = vn[0, :n]
    return A


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_von_neumann_stability(order):
    """Sec. 4.1: FV + GRPrec is linearly stable up to Courant number 1 at every
    order; beyond it the spectral radius exceeds one."""
    for cfl in (0.1, 0.5, 0.9, 1.0):
        rho = np.abs(np.linalg.eigvals(_step_matrix(order, cfl))).max()
        # at Courant number 1 some unit-modulus eigenvalues are defective, which
        # perturbs computed eigenvalues by ~sqrt(machine epsilon)
        assert rho <= 1.0 + 1e-6, (cfl, rho)
    rho = np.abs(np.linalg.eigvals(_step_matrix(order, 1.05))).max()
    assert rho > 1.05, rho


@pytest.mark.parametrize("system", [oracle.ADVECTION, oracle.EULER])
def test_periodic_conservation(system):
    n = 50
    for order in (2, 3, 4):
        if system == oracle.ADVECTION:
            dx, q, vl, vr = I.adv_sin2pi(n)
            q = q + 0.1 * RNG.normal(size=q.shape)
        else:
            dx, q, vl, vr = I.euler_density_wave(n)
            q = q.copy()
            q[0] *= 1 + 0.05 * RNG.normal(size=n)
        c = oracle.cfg(system, order)
        v = oracle.init_interfaces(c, vl, vr)
        qn, vn, t, k, _ = oracle.run(c, dx, q, v, 0.0, 1.0, max_steps=20)
        tot0 = q.sum(axis=1)
        tot1 = qn.sum(axis=1)
        assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(q).sum(axis=1)), (tot0, tot1)


def test_paper_advection_table():
    """Sec. 4.2.3 table (FV + GRPrec, sin^4, t_out = 4).  First-step interface
    data are the exact point values of the initial condition (the paper does not
    say); errors are unnormalised sums dx |e|.  Order 2 agrees to 3 %, orders
    3-5 to 25 % at N = 256 (35 % at N = 128; the gap shrinks faster than the
    error itself), and the observed rates to 0.2 (0.4 at order 5)."""
    tab = _load_table("paper_advection_grprec.txt")
    for order in (2, 3, 4, 5):
        errs = {}
        for n in (64, 128, 256):
            dx, q, vl, vr = I.adv_sin4(n)
            c = oracle.cfg(oracle.ADVECTION, order)
            v = oracle.init_interfaces(c, vl, vr)
            qn, _, t, _, _ = oracle.run(c, dx, q, v, 0.0, 4.0)
            assert t == 4.0
            e = qn[0] - I.adv_sin4_exact_avg(n, 4.0)
            errs[n] = (np.abs(e).max(), (np.abs(e) * dx).sum())
        for n in (128, 256) if order > 2 else (64, 128, 256):
            tol = 0.03 if order == 2 else (0.25 if n == 256 else 0.35)
            for k in (0, 1):
                assert abs(errs[n][k] / tab[(order, n)][k] - 1) < tol, (order, n, k, errs[n][k])
        for n0, n1 in ((64, 128), (128, 256)):
            ours = np.log2(errs[n0][0] / errs[n1][0])
            paper = np.log2(tab[(order, n0)][0] / tab[(order, n1)][0])
            # order 5: the printed rates (5.3) exceed the design order; ours are 5.0
            assert abs(ours - paper) < (0.2 if order < 5 else 0.4), (order, n0, ours, paper)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_advection_convergence_order(order):
    """Config: u0 = sin(2 pi x) on [0,1], t_end = 1; order m+1 observed."""
    e = []
    for n in (32, 64):
        dx, q, vl, vr = I.adv_sin2pi(n)
        c = oracle.cfg(oracle.ADVECTION, order)
        v = oracle.init_interfaces(c, vl, vr)
        qn, _, _, _, _ = oracle.run(c, dx, q, v, 0.0, 1.0)
        e.append(np.abs(qn[0] - I.adv_sin2pi_exact_avg(n, 1.0)).max())
    assert np.log2(e[0] / e[1]) > order - 0.2


def test_square_wave_bounded():
    dx, q, vl, vr = I.adv_square(64)
    for order in (2, 3, 4, 5):
        c = oracle.cfg(oracle.ADVECTION, order)
        v = oracle.init_interfaces(c, vl, vr)
        qn, vn, t, _, _ = oracle.run(c, dx, q, v, 0.0, 1.0)
        assert np.all(np.isfinite(qn)) and np.abs(qn).max() < 2.0
        assert abs(qn.sum() - q.sum()) < 1e-12 * np.abs(q).sum()


# ------------------------------------------------------------- Euler
@pytest.mark.parametrize("bc", [oracle.PERIODIC, oracle.TRANSMISSIVE])
def test_euler_constant_state(bc):
    n = 20
    W = (0.8, 0.3, 1.7)
    Q = I.prim_to_cons(np.full(n, W[0]), W[1], W[2])
    for order in (2, 3, 4, 5):
        c = oracle.cfg(oracle.EULER, order, bc=bc)
        v = np.concatenate([Q, Q[:, :1]], axis=1)
        qn, vn, _, _, _ = oracle.run(c, 1.0 / n, Q, v, 0.0, 1.0, max_steps=5)
        # round-off only: rows of the differentiation matrix sum to ~1e-15, not 0
        np.testing.assert_allclose(qn, Q, rtol=1e-12)
        np.testing.assert_allclose(vn, v, rtol=1e-12)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_euler_density_wave_equals_advection(order):
    """With u and p constant, rho u and E are affine in rho, the interface
    problems are pure contacts and the flux is u Q + const, so the Euler scheme
    acting on rho is the advection scheme with lambda = u at the same dt."""
    n = 30
    dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=1.0)
    c = oracle.cfg(oracle.EULER, order)
    v = oracle.init_interfaces(c, vl, vr)
    S = oracle.smax(c, q)
    qe, ve, dte, _, _ = oracle.step(c, dx, q, v, 0.0, 10.0)
    ca = oracle.cfg(oracle.ADVECTION, order, cfl=0.9 * 1.0 / S, lam=1.0)
    qa, va, dta, _, _ = oracle.step(ca, dx, q[:1].copy(), v[:1].copy(), 0.0, 10.0)
    assert abs(dta - dte) < 1e-15
    np.testing.assert_allclose(qe[0], qa[0], atol=1e-12)
    np.testing.assert_allclose(ve[0], va[0], atol=1e-12)


def test_paper_euler_rates():
    """Sec. 4.3.1 table: the observed rates between N = 40, 80, 160 agree with
    the printed ones to 0.3 for orders 2-4 (magnitudes are not compared: the
    printed L1/Linf ratio does not fit the stated unit domain).  Order 5 is
    held to its design rate: the printed rates (5.96, 5.92) exceed it, ours
    are 4.99 and 5.00."""
    tab = _load_table("paper_euler_grprec.txt")
    for order in (2, 3, 4, 5):
        errs = {}
        for n in (40, 80, 160):
            dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=2.0)
            c = oracle.cfg(oracle.EULER, order)
            v = oracle.init_interfaces(c, vl, vr)
            qn, _, t, _, _ = oracle.run(c, dx, q, v, 0.0, 4.0)
            errs[n] = np.abs(qn[0] - I.euler_density_wave_exact_rho(n, 4.0)).max()
        for n0, n1 in ((40, 80), (80, 160)):
            ours = np.log2(errs[n0] / errs[n1])
            paper = np.log2(tab[(order, n0)][0] / tab[(order, n1)][0])
            if order < 5:
                assert abs(ours - paper) < 0.3, (order, n0, ours, paper)
            else:
                assert ours > 4.9 and paper > ours, (ours, paper)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_euler_nonlinear_smooth_self_convergence(order):
    """A smooth acoustic pulse (u and p vary, so the flux is genuinely
    nonlinear): differences between successive meshes fall at rate ~ m+1."""
    def run(n):
        dx, xf = I.grid(n)
        xs = []
        # cell averages by 8-point Gauss on each cell (smooth data)
        gx, gw = np.polynomial.legendre.leggauss(8)
        xq = 0.5 * (xf[:-1, None] + xf[1:, None]) + 0.5 * dx * gx[None, :]
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * xq)
        u = 0.3 * np.sin(2 * np.pi * xq)
        p = 1.0 + 0.28 * np.sin(2 * np.pi * xq)
        Q = I.prim_to_cons(rho, u, p)
        q = (Q * (0.5 * gw)[None, None, :]).sum(axis=2)
        rf = 1.0 + 0.2 * np.sin(2 * np.pi * xf)
        uf = 0.3 * np.sin(2 * np.pi * xf)
        pf = 1.0 + 0.28 * np.sin(2 * np.pi * xf)
        v = I.prim_to_cons(rf, uf, pf)
        c = oracle.cfg(oracle.EULER, order)
        qn, _, t, _, _ = oracle.run(c, dx, q, v, 0.0, 0.2)
        del xs
        return qn[0]
    r = [run(n) for n in (32, 64, 128)]
    coarsen = lambda a: 0.5 * (a[0::2] + a[1::2])
    d1 = np.abs(coarsen(r[1]) - r[0]).max()
    d2 = np.abs(coarsen(r[2]) - r[1]).max()
    assert np.log2(d1 / d2) > order - 0.4, (d1, d2)


def test_sod_with_linear_grprec_fails_at_first_step():
    """Reading: the paper runs shock tubes only with GRPrecNL.  Linear GRPrec
    (Godunov's theorem) puts a negative nodal pressure in the cell next to the
    Sod jump at the first step and the predictor does not converge."""
    for order in (2, 3, 4):
        dx, q, vl, vr = I.euler_shock_tube(100)
        c = oracle.cfg(oracle.EULER, order, bc=oracle.TRANSMISSIVE)
        v = oracle.init_interfaces(c, vl, vr)
        with pytest.raises(oracle.OracleError) as ei:
            oracle.step(c, dx, q, v, 0.0, 0.2)
        assert ei.value.code in (oracle.E_PREDICTOR, oracle.E_NONPHYSICAL)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_transmissive_ends_are_stable(order):
    """Reading of 'transmissive': a ghost cell holding the end cell's average as
    constant data.  Short domains stay physical and bounded for 1000 steps
    (extrapolating the end cell's own polynomial instead is unstable)."""
    for n in (3, 5, 12):
        dx, q, vl, vr = I.euler_density_wave(n, amp=0.1, u=0.5, p=1.0)
        c = oracle.cfg(oracle.EULER, order, bc=oracle.TRANSMISSIVE)
        v = oracle.init_interfaces(c, vl, vr)
        qn, _, _, k, _ = oracle.run(c, dx, q, v, 0.0, 1e9, 1000)
        assert k == 1000
        assert np.abs(qn[0] - 1.0).max() <= 0.1 + 1e-12
        assert np.abs(qn[1] / qn[0] - 0.5).max() < 1e-10


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_transmissive_outflow_advection(order):
    """A smooth bump carried out of a transmissive domain leaves it (nearly)
    empty; the inflow ghost keeps the upstream value."""
    n = 64
    dx, xf = I.grid(n)
    bump = lambda x: np.where(np.abs(x - 0.5) < 0.25, np.cos(2 * np.pi * (x - 0.5)) ** 4, 0.0)
    gx, gw = np.polynomial.legendre.leggauss(10)
    xq = 0.5 * (xf[:-1, None] + xf[1:, None]) + 0.5 * dx * gx[None, :]
    q = (bump(xq) * 0.5 * gw).sum(axis=1)[None, :]
    v = bump(xf)[None, :]
    c = oracle.cfg(oracle.ADVECTION, order, bc=oracle.TRANSMISSIVE)
    qn, _, _, _, _ = oracle.run(c, dx, q, v.copy(), 0.0, 1.0)
    assert np.abs(qn).max() < 1e-3


@pytest.mark.parametrize("order", [2, 3, 4])
def test_trrs_datum_on_contacts_equals_exact_datum(order):
    """A density wave has pure-contact interface problems, where the
    two-rarefaction datum is exact: the step is the same as with the exact
    datum."""
    n = 40
    dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=1.0)
    ce = oracle.cfg(oracle.EULER, order)
    ct = oracle.cfg(oracle.EULER, order, datum=oracle.DATUM_TRRS)
    v = oracle.init_interfaces(ce, vl, vr)
    qe, ve, _, _, _ = oracle.run(ce, dx, q, v, 0.0, 1.0, max_steps=5)
    qt, vt, _, _, _ = oracle.run(ct, dx, q, v, 0.0, 1.0, max_steps=5)
    np.testing.assert_allclose(qt, qe, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(vt, ve, rtol=1e-13, atol=1e-14)


def test_trrs_datum_shock_tube_runs_and_differs():
    """On a shock tube the datum changes the scheme (the datum at the shock is
    approximate) but the solution stays close to the exact-datum one."""
    dx, q, vl, vr = I.euler_shock_tube(100, left=(1.0, 0.0, 1.0), right=(0.5, 0.0, 0.5))
    ce = oracle.cfg(oracle.EULER, 3, bc=oracle.TRANSMISSIVE, recon=oracle.NONLINEAR,
                    nl_lambda_c=oracle.LAMBDA_C_TABLE)
    ct = oracle.cfg(oracle.EULER, 3, bc=oracle.TRANSMISSIVE, recon=oracle.NONLINEAR,
                    datum=oracle.DATUM_TRRS, nl_lambda_c=oracle.LAMBDA_C_TABLE)
    qe, _, _, _, _ = oracle.run(ce, dx, q, oracle.init_interfaces(ce, vl, vr), 0.0, 0.2)
    qt, _, _, _, _ = oracle.run(ct, dx, q, oracle.init_interfaces(ct, vl, vr), 0.0, 0.2)
    d = np.abs(qt - qe).max()
    assert 1e-8 < d < 2e-2, d
    assert abs(qt.sum() - qe.sum()) < 1e-12 * np.abs(q).sum()  # both conservative


def test_nonphysical_cell_is_reported_wherever_it_sits():
    """S_max is the largest |lambda_j(Q_i)| over the cells (Sec. 4.1); a cell
    with negative pressure has no real wave speeds, so the step reports a
    non-physical state whether or not valid cells follow it."""
    n = 30
    dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=1.0)
    c = oracle.cfg(oracle.EULER, 3)
    v = oracle.init_interfaces(c, vl, vr)
    for k in (0, 11, n - 1):
        qb = q.copy()
        qb[2, k] = 0.5 * qb[1, k] ** 2 / qb[0, k] - 0.1
        assert np.isnan(oracle.smax(c, qb))
        with pytest.raises(oracle.OracleError) as ei:
            oracle.step(c, dx, qb, v, 0.0, 1.0)
        assert ei.value.code == oracle.E_NONPHYSICAL


def _mixed_sign_states(rng, n):
    """Euler cell averages whose fastest wave runs left: velocities of both
    signs, the largest |u| + c at a cell with u < 0, and the largest |u| and
    the largest c in different cells (so max|u| + max c is not the answer)."""
    rho = rng.uniform(0.5, 2.0, n)
    u = rng.uniform(-0.5, 0.5, n)
    p = rng.uniform(0.5, 1.5, n)
    k = n // 3
    u[k], rho[k], p[k] = -2.5, 1.0, 1.0           # fastest: |u| + c = 2.5 + sqrt(1.4)
    u[k + 1], rho[k + 1], p[k + 1] = 2.0, 1.0, 1.0  # fastest rightward one is slower
    u[k + 2], rho[k + 2], p[k + 2] = 0.0, 0.5, 3.0  # largest c = sqrt(8.4), |u| = 0
    return rho, u, p


def test_smax_value_with_leftward_and_mixed_velocities():
    """Sec. 4.1: S_max = max_i max_j |lambda_j(Q_i)| = max_i (|u_i| + c_i).  The
    data put the maximum at a leftward-moving cell and the largest |u| and
    largest c in different cells, so max(u + c), max|u| + max c or a missing
    absolute value all give other numbers."""
    rng = np.random.default_rng(31)
    n = 40
    rho, u, p = _mixed_sign_states(rng, n)
    q = I.prim_to_cons(rho, u, p)
    c = oracle.cfg(oracle.EULER, 3)
    want = np.max(np.abs(u) + np.sqrt(1.4 * p / rho))
    got = oracle.smax(c, q)
    assert abs(got - want) <= 1e-15 * want
    assert want > np.max(u + np.sqrt(1.4 * p / rho)) + 0.1
    assert want < np.max(np.abs(u)) + np.max(np.sqrt(1.4 * p / rho)) - 0.1
    # whole-domain reversal u -> -u leaves S_max unchanged
    assert oracle.smax(c, I.prim_to_cons(rho, -u, p)) == got


def test_smax_per_segment_sets_each_segments_step():
    """Segments advance with their own dt = C_CFL dx_s / S_max,s (eq. dt-FV):
    after one unclipped step each segment's time is that dt, with S_max of its
    own cells only.  Smooth data whose velocity is mostly negative in every
    other segment, so the largest |u| + c sits at a leftward flow there."""
    sizes = [17, 9, 30, 12]
    lengths = [0.5, 0.2, 1.3, 0.7]
    qs, vs, want = [], [], []
    for s, n in enumerate(sizes):
        xm = (np.arange(n) + 0.5) / n
        xf = np.arange(n + 1) / n
        sgn = -1.0 if s % 2 else 1.0

        def prim(x):
            return (1.0 + 0.2 * np.sin(2 * np.pi * x), sgn * (1.0 + 0.5 * np.cos(2 * np.pi * x)) * (0.5 + s),
                    1.0 + 0.1 * np.cos(2 * np.pi * x))
        rho, u, p = prim(xm)
        qs.append(I.prim_to_cons(rho, u, p))      # point values stand in for averages
        vs.append(I.prim_to_cons(*prim(xf)))
        want.append(0.9 * (lengths[s] / n) / np.max(np.abs(u) + np.sqrt(1.4 * p / rho)))
    cell_off = np.concatenate([[0], np.cumsum(sizes)])
    c = oracle.cfg(oracle.EULER, 3, bc=oracle.TRANSMISSIVE)
    q = np.ascontiguousarray(np.concatenate(qs, axis=1))
    v = np.ascontiguousarray(np.concatenate(vs, axis=1))
    dx = np.array(lengths) / np.array(sizes)
    _, _, t, _ = oracle.run_segments(c, cell_off, dx, q, v, np.zeros(len(sizes)), 1e9, 1)
    np.testing.assert_allclose(t, want, rtol=1e-14)


def _mirror(q, v):
    """x -> -x: cells and interfaces in reverse order, momentum negated."""
    qm, vm = q[:, ::-1].copy(), v[:, ::-1].copy()
    qm[1] *= -1.0
    vm[1] *= -1.0
    return qm, vm


@pytest.mark.parametrize("order,recon", [(3, 0), (5, 0), (5, 1), (4, 1)])
def test_transmissive_step_is_mirror_symmetric(order, recon):
    """Both transmissive ends follow one rule (R9, R20: the ghost cell beyond
    an end holds the end average, also as the V_{i+-3/2} datum GRPrecNL reads
    at degree 4), so reversing the domain and the sign of the velocity
    commutes with a step.  The data make the end averages differ from the end
    interface values, so a rule applied at one end only breaks the symmetry."""
    n = 37
    dx = 1.0 / n
    xf = np.arange(n + 1) * dx
    xm = 0.5 * (xf[:-1] + xf[1:])

    def prim(x):
        return 1.0 + 0.3 * x * x + 0.1 * np.sin(7 * x), 0.4 * np.cos(3 * x) - 0.2, 1.0 + 0.5 * x ** 3

    q = I.prim_to_cons(*prim(xm))
    v = I.prim_to_cons(*prim(xf))
    c = oracle.cfg(oracle.EULER, order, bc=oracle.TRANSMISSIVE, recon=recon, nl_lambda_c=10.0)
    qa, va, dta, _, _ = oracle.step(c, dx, q, v, 0.0, 1.0)
    qmi, vmi = _mirror(q, v)
    qb, vb, dtb, _, _ = oracle.step(c, dx, qmi, vmi, 0.0, 1.0)
    qb, vb = _mirror(qb, vb)
    assert dta == dtb
    scale = np.abs(q).max()
    assert np.abs(qa - qb).max() <= 1e-13 * scale
    assert np.abs(va - vb).max() <= 1e-13 * scale
    # and the end data matter: the step moved the end cells
    assert np.abs(qa[:, [0, -1]] - q[:, [0, -1]]).max() > 1e-6


@pytest.mark.parametrize("lam", [1.0, -0.7])
def test_first_step_datum_is_the_upwind_limit_at_a_jump(lam):
    """R1: the first interface datum is the Riemann solution at x/t = 0
    between the two one-sided limits; for advection that is the upwind limit
    (the left one for lambda > 0, the right one for lambda < 0)."""
    n = 16
    dx, q, vl, vr = I.adv_square(n)
    c = oracle.cfg(oracle.ADVECTION, 3, lam=lam)
    v = oracle.init_interfaces(c, vl, vr)
    want = vl if lam > 0 else vr
    assert np.array_equal(v, want)
    assert not np.array_equal(vl, vr)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_first_step_datum_is_the_upwind_state_in_supersonic_flow(sign):
    """R1 for the Euler equations: where both one-sided states move faster than
    their sound speed in one direction, x/t = 0 lies outside the whole wave
    fan and the datum is the upwind state exactly."""
    WL = np.array([[1.0, 3.0 * sign, 1.0]])
    WR = np.array([[0.5, 3.2 * sign, 0.6]])
    QL, QR = I.prim_to_cons(*WL.T), I.prim_to_cons(*WR.T)
    c = oracle.cfg(oracle.EULER, 3, bc=oracle.TRANSMISSIVE)
    v = oracle.init_interfaces(c, QL, QR)
    want = QL if sign > 0 else QR
    np.testing.assert_allclose(v, want, rtol=1e-15, atol=0.0)
