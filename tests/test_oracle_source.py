"""Pins of the source term (eq. eq_finite_volume with S^n_i of eq. source) for
the linear relaxation S(Q) = -kappa Q, integrated over the space-time
polynomial of the locally implicit DET predictor (Sec. 2).

* Constant data have no flux gradient, so one step is the predictor's DG time
  evolution of q' = -kappa q followed by the source update; with z = kappa dt
  it multiplies the state by the (m, m+1) Pade approximant of exp(-z) (the
  stability function of degree-m DG time stepping), written out here from
  the textbook formula.
* With the relaxation source the exact solution is exp(-kappa t) times the
  solution without source (advection; and Euler, whose flux is homogeneous of
  degree one), so smooth runs converge at the design order to it.
* Stiff relaxation (kappa dt >> 1) of advection: one step brings the state to
  within O(1/(kappa dt)) of the equilibrium 0, as the locally implicit
  predictor allows; an explicit treatment would multiply by |1 - kappa dt|.
"""
from math import factorial

import numpy as np
import pytest

import oracle
from paper_2602_21911_amd import inputs as I


def pade_exp_minus(z, m):
    """(m, m+1) Pade approximant of exp(-z)."""
    j, k = m, m + 1
    num = sum(factorial(j + k - i) * factorial(j) / (factorial(j + k) * factorial(i) * factorial(j - i))
              * (-z) ** i for i in range(j + 1))
    den = sum(factorial(j + k - i) * factorial(k) / (factorial(j + k) * factorial(i) * factorial(k - i))
              * z ** i for i in range(k + 1))
    return num / den


def _src(system, order, kappa, **kw):
    return oracle.cfg(system, order, source=oracle.SOURCE_LINEAR, kappa=kappa, **kw)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
@pytest.mark.parametrize("bc", [oracle.PERIODIC, oracle.TRANSMISSIVE])
def test_constant_state_is_multiplied_by_the_pade_approximant(order, bc):
    n = 16
    dx = 1.0 / n
    for system in (oracle.ADVECTION, oracle.EULER):
        if system == oracle.ADVECTION:
            Q = np.full((1, n), 0.7)
            S = 1.0
        else:
            Q = I.prim_to_cons(np.full(n, 0.8), 0.3, 1.7)
            S = 0.3 + np.sqrt(1.4 * 1.7 / 0.8)
        V = np.concatenate([Q, Q[:, :1]], axis=1)
        dt = 0.9 * dx / S
        for z in (0.05, 1.0, 2.5, 40.0, 1e4):
            if system == oracle.EULER and z > 2.5:
                continue  # negative nodal densities: see test_euler_stiff_relaxation_is_reported
            c = _src(system, order, z / dt, bc=bc)
            qn, vn, dtn, _, _ = oracle.step(c, dx, Q, V, 0.0, 1.0)
            assert abs(dtn - dt) <= 1e-15 * dt
            R = pade_exp_minus(z, order - 1)
            np.testing.assert_allclose(qn, R * Q, rtol=1e-12, atol=1e-14 * np.abs(Q).max())
            np.testing.assert_allclose(vn, R * V, rtol=1e-12, atol=1e-14 * np.abs(V).max())


@pytest.mark.parametrize("system", [oracle.ADVECTION, oracle.EULER])
def test_zero_rate_is_the_scheme_without_source(system):
    n = 30
    if system == oracle.ADVECTION:
        dx, q, vl, vr = I.adv_sin2pi(n)
    else:
        dx, q, vl, vr = I.euler_density_wave(n)
    for bc in (oracle.PERIODIC, oracle.TRANSMISSIVE):
        c0 = oracle.cfg(system, 3, bc=bc)
        c1 = _src(system, 3, 0.0, bc=bc)
        v = oracle.init_interfaces(c0, vl, vr)
        a = oracle.run(c0, dx, q, v, 0.0, 1.0, max_steps=4)
        b = oracle.run(c1, dx, q, v, 0.0, 1.0, max_steps=4)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


def _rates(errs):
    return [np.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_advection_with_source_converges_to_the_damped_translation(order):
    kappa, t_end = 1.5, 0.5
    errs = []
    for n in (40, 80, 160):
        dx, q, vl, vr = I.adv_sin2pi(n)
        c = _src(oracle.ADVECTION, order, kappa)
        qn, _, t, _, _ = oracle.run(c, dx, q, oracle.init_interfaces(c, vl, vr), 0.0, t_end)
        assert t == t_end
        exact = np.exp(-kappa * t_end) * I.adv_sin2pi_exact_avg(n, t_end)
        errs.append(np.abs(qn[0] - exact).max())
    assert min(_rates(errs)) > order - 0.3, (errs, _rates(errs))


@pytest.mark.parametrize("order", [2, 3, 4])
def test_euler_density_wave_with_source_converges(order):
    """rho, rho u and E all relax at rate kappa; u is unchanged, so the density
    is exp(-kappa t) times the translated wave."""
    kappa, t_end = 1.0, 0.25
    errs = []
    for n in (40, 80, 160):
        dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=1.0)
        c = _src(oracle.EULER, order, kappa)
        qn, _, t, _, _ = oracle.run(c, dx, q, oracle.init_interfaces(c, vl, vr), 0.0, t_end)
        exact = np.exp(-kappa * t_end) * I.euler_density_wave_exact_rho(n, t_end, amp=0.2, u=1.0)
        errs.append(np.abs(qn[0] - exact).max())
    assert min(_rates(errs)) > order - 0.3, (errs, _rates(errs))


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_stiff_relaxation_reaches_equilibrium_in_one_step(order):
    n = 50
    dx, q, vl, vr = I.adv_sin2pi(n)
    q = q + 2.0  # away from the equilibrium everywhere
    vl, vr = vl + 2.0, vr + 2.0
    dt = 0.9 * dx
    for z in (1e3, 1e6):
        c = _src(oracle.ADVECTION, order, z / dt)
        v = oracle.init_interfaces(c, vl, vr)
        qn, vn, _, _, st = oracle.step(c, dx, q, v, 0.0, 1.0)
        assert np.abs(qn).max() <= 10.0 / z * np.abs(q).max()
        assert np.abs(vn).max() <= 10.0 / z * np.abs(v).max()
        assert st.picard_max_seen <= 2 * order + 2


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_euler_stiff_relaxation_is_reported(order):
    """For kappa dt >> 1 the degree-m DG time evolution of constant data
    oscillates about zero at the inner time nodes (its nodal values are
    (K + z diag(w))^{-1} l(0), with alternating signs for large z), so the
    Euler flux samples there see negative densities: the step reports a
    non-physical state instead of relaxing (advection has no such limit)."""
    n = 20
    dx, q, vl, vr = I.euler_density_wave(n)
    dt = 0.9 * dx / oracle.smax(oracle.cfg(oracle.EULER, order), q)
    c = _src(oracle.EULER, order, 40.0 / dt)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.step(c, dx, q, oracle.init_interfaces(c, vl, vr), 0.0, 1.0)
    assert ei.value.code == oracle.E_NONPHYSICAL
    c = _src(oracle.EULER, order, 2.0 / dt)  # moderate relaxation runs
    qn, _, _, _, _ = oracle.step(c, dx, q, oracle.init_interfaces(c, vl, vr), 0.0, 1.0)
    assert np.all(qn[0] > 0)


def test_invalid_source_is_rejected():
    dx, q, vl, vr = I.adv_sin2pi(10)
    for bad in (dict(source=2), dict(source=oracle.SOURCE_LINEAR, kappa=-1.0)):
        c = oracle.cfg(oracle.ADVECTION, 3, **bad)
        with pytest.raises(oracle.OracleError):
            oracle.step(c, dx, q, oracle.init_interfaces(c, vl, vr), 0.0, 1.0)
