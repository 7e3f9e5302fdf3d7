"""Pins of the oracle's exact Euler Riemann solver by properties of the exact
solution that do not use the pressure function: integral conservation of the
self-similar solution, the Rankine-Hugoniot conditions across shocks and the
isentrope and Riemann invariant across rarefactions, Galilean and scaling
invariance, symmetry, the two-rarefaction closed form, the vacuum condition
and guess independence."""
import numpy as np
import pytest

import oracle

G = 1.4


def _cons(W):
    r, u, p = W
    return np.array([r, r * u, p / (G - 1) + 0.5 * r * u * u])


def _flux(W):
    r, u, p = W
    E = p / (G - 1) + 0.5 * r * u * u
    return np.array([r * u, r * u * u + p, u * (E + p)])


def _sample(WL, WR, s):
    """Solution at x/t = s, via the same solver in the frame moving with speed s."""
    sl = np.array([WL[0], WL[1] - s, WL[2]])
    sr = np.array([WR[0], WR[1] - s, WR[2]])
    _, _, W0, _ = oracle.riemann(G, sl, sr)
    return np.array([W0[0], W0[1] + s, W0[2]])


CASES = [
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),         # Sod data (Sec. 4.3.2): rarefaction, contact, shock
    ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4)),          # 123-problem data (Sec. 4.3.2): two rarefactions
    ((1.0, 0.0, 800.0), (1.2, 0.0, 0.02)),        # strong shock
    ((6.0, 19.0, 450.0), (5.5, -6.5, 50.0)),      # colliding shocks
    ((1.0, 0.8, 1.0), (0.15, 0.0, 0.12)),         # transonic rarefaction
    ((0.3, -1.2, 0.02), (2.0, 0.4, 30.0)),
]


@pytest.mark.parametrize("WL,WR", CASES)
def test_integral_conservation(WL, WR):
    """For the self-similar solution W(x/t) of the Riemann problem,
    int_{-X}^{X} (Q(s) - Q0(s)) ds = F(W_L) - F(W_R) for X beyond all waves
    (the integral form of the conservation law at t = 1).  A wrong star pressure,
    velocity, shock density or fan profile breaks this identity."""
    WL, WR = np.array(WL), np.array(WR)
    cl, cr = np.sqrt(G * WL[2] / WL[0]), np.sqrt(G * WR[2] / WR[0])
    X = 2.0 * (abs(WL[1]) + abs(WR[1]) + 3 * cl + 3 * cr) + 5.0
    n = 100000
    s = -X + (np.arange(n) + 0.5) * (2 * X / n)
    Qs = np.array([_cons(_sample(WL, WR, si)) for si in s])
    Q0 = np.where((s < 0)[:, None], _cons(WL)[None, :], _cons(WR)[None, :])
    lhs = (Qs - Q0).sum(axis=0) * (2 * X / n)
    rhs = _flux(WL) - _flux(WR)
    scale = np.abs(_cons(WL)).max() + np.abs(_cons(WR)).max()
    # midpoint sampling puts an error of at most |jump| * ds / 2 at each of the
    # (at most three) discontinuities; a wrong star state is off by O(1)
    ds = 2 * X / n
    assert np.all(np.abs(lhs - rhs) < 1.5 * scale * ds), (lhs, rhs, ds)


@pytest.mark.parametrize("WL,WR", CASES)
def test_jump_relations_of_both_nonlinear_waves(WL, WR):
    """Star states sampled just beside the contact: across a shock (p* above
    the outer pressure) mass, momentum and energy fluxes jump consistently
    with one shock speed (Rankine-Hugoniot); across a rarefaction the
    entropy p/rho^g and the outgoing Riemann invariant u -/+ 2c/(g-1) are
    carried through."""
    ps, us, _, _ = oracle.riemann(G, WL, WR)
    d = 1e-9 * (1.0 + abs(us))
    for side, W, Ws in ((-1, np.array(WL), _sample(WL, WR, us - d)),
                        (1, np.array(WR), _sample(WL, WR, us + d))):
        assert abs(Ws[2] - ps) <= 1e-12 * ps and abs(Ws[1] - us) <= 1e-9 * (1 + abs(us))
        if ps > W[2]:  # shock
            q0, q1 = _cons(W), _cons(Ws)
            f0, f1 = _flux(W), _flux(Ws)
            S = (f1[0] - f0[0]) / (q1[0] - q0[0])  # shock speed from mass conservation
            for k in (1, 2):
                scale = abs(f0[k]) + abs(f1[k]) + abs(S) * (abs(q0[k]) + abs(q1[k]))
                assert abs((f1[k] - f0[k]) - S * (q1[k] - q0[k])) <= 1e-11 * scale, (k, S)
            assert side * (S - us) > 0  # the shock lies on its own side of the contact
        else:  # rarefaction
            c, cs = np.sqrt(G * W[2] / W[0]), np.sqrt(G * Ws[2] / Ws[0])
            assert abs(Ws[2] / Ws[0] ** G - W[2] / W[0] ** G) <= 1e-11 * W[2] / W[0] ** G
            inv = lambda u, cc: u - side * 2.0 * cc / (G - 1.0)
            assert abs(inv(Ws[1], cs) - inv(W[1], c)) <= 1e-11 * (abs(W[1]) + c)


@pytest.mark.parametrize("WL,WR", CASES)
def test_galilean_and_scaling_invariance(WL, WR):
    WL, WR = np.array(WL), np.array(WR)
    ps, us, _, _ = oracle.riemann(G, WL, WR)
    a = 0.37
    ps2, us2, _, _ = oracle.riemann(G, WL + [0, a, 0], WR + [0, a, 0])
    assert abs(ps2 - ps) < 1e-11 * ps and abs(us2 - (us + a)) < 1e-11 * (1 + abs(us))
    # (rho, u, p) -> (A rho, B u, A B^2 p) maps solutions to solutions
    A, B = 3.1, 0.6
    sc = np.array([A, B, A * B * B])
    ps3, us3, _, _ = oracle.riemann(G, WL * sc, WR * sc)
    assert abs(ps3 - A * B * B * ps) < 1e-11 * A * B * B * ps
    assert abs(us3 - B * us) < 1e-11 * (1 + abs(B * us))


def test_symmetric_data():
    for W in ([1.0, 1.0, 1.0], [0.5, -2.0, 0.3], [2.0, 0.7, 5.0]):
        WL = np.array(W)
        WR = np.array([W[0], -W[1], W[2]])
        ps, us, W0, _ = oracle.riemann(G, WL, WR)
        assert abs(us) < 1e-13


def test_identical_states_unchanged():
    for W in ([1.0, 0.0, 1.0], [0.3, 1.7, 0.02], [4.0, -0.9, 100.0]):
        W = np.array(W)
        ps, us, W0, it = oracle.riemann(G, W, W)
        assert ps == W[2] and us == W[1]
        np.testing.assert_array_equal(W0, W)


def test_two_rarefaction_closed_form():
    """When both waves are rarefactions the Riemann invariants give
    p* = [(cL + cR - (g-1)/2 (uR - uL)) / (cL pL^-z + cR pR^-z)]^(1/z), z = (g-1)/(2g)."""
    rng = np.random.default_rng(7)
    z = (G - 1) / (2 * G)
    n_checked = 0
    for _ in range(200):
        WL = np.array([rng.uniform(0.1, 3), rng.uniform(-3, 0), rng.uniform(0.1, 3)])
        WR = np.array([rng.uniform(0.1, 3), rng.uniform(0, 3), rng.uniform(0.1, 3)])
        cl, cr = np.sqrt(G * WL[2] / WL[0]), np.sqrt(G * WR[2] / WR[0])
        if 2 / (G - 1) * (cl + cr) <= WR[1] - WL[1]:
            continue
        pt = ((cl + cr - 0.5 * (G - 1) * (WR[1] - WL[1])) / (cl / WL[2] ** z + cr / WR[2] ** z)) ** (1 / z)
        if pt > min(WL[2], WR[2]):
            continue
        ps, _, _, _ = oracle.riemann(G, WL, WR)
        assert abs(ps - pt) < 1e-11 * pt
        n_checked += 1
    assert n_checked > 50


def test_vacuum_detected():
    rc, _, _ = oracle.riemann_rc(G, [1.0, -5.0, 0.4], [1.0, 5.0, 0.4])
    assert rc == oracle.E_VACUUM


def test_nonphysical_detected():
    rc, _, _ = oracle.riemann_rc(G, [1.0, 0.0, -0.4], [1.0, 0.0, 0.4])
    assert rc == oracle.E_NONPHYSICAL
    rc, _, _ = oracle.riemann_rc(G, [np.nan, 0.0, 0.4], [1.0, 0.0, 0.4])
    assert rc == oracle.E_NONPHYSICAL


def test_newton_cap_reported():
    rc, _, it = oracle.riemann_rc(G, [1.0, 0.0, 1000.0], [1.0, 0.0, 0.01], maxit=1)
    assert rc == oracle.E_NEWTON


@pytest.mark.parametrize("WL,WR", CASES)
def test_guess_independence(WL, WR):
    """f is increasing and concave, so Newton reaches the same root from any
    positive start."""
    ps0, _, _, _ = oracle.riemann(G, WL, WR)
    for guess in (1e-3 * ps0, 0.5 * ps0, 2 * ps0, 30 * ps0):
        ps, _, _, _ = oracle.riemann(G, WL, WR, guess=guess)
        assert abs(ps - ps0) < 1e-12 * ps0


# ------------------------------------------------- two-rarefaction datum (Sec. 4.1)
def _raref_f(g, p, r, u, pk):
    """Rarefaction-branch pressure function of one side (isentrope + Riemann
    invariant), written out directly."""
    c = np.sqrt(g * pk / r)
    return 2.0 * c / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def test_trrs_equals_exact_solver_for_two_rarefactions():
    """When the exact solution has two rarefactions (p* below both pressures)
    the approximation is exact: same p*, u* and state at x/t = 0."""
    rng = np.random.default_rng(31)
    seen = 0
    cases = [((1.0, -2.0, 0.4), (1.0, 2.0, 0.4))]  # the paper's 123 problem data
    for _ in range(400):
        WL = (np.exp(rng.uniform(-1, 1)), rng.uniform(-1, 0), np.exp(rng.uniform(-1, 1)))
        WR = (np.exp(rng.uniform(-1, 1)), rng.uniform(0, 1), np.exp(rng.uniform(-1, 1)))
        cases.append((WL, WR))
    for WL, WR in cases:
        rc, pe, _ = oracle.riemann_rc(1.4, WL, WR)
        if rc != oracle.OK or pe >= min(WL[2], WR[2]):
            continue
        seen += 1
        ps, us, W0 = oracle.trrs(1.4, WL, WR)
        pe, ue, We, _ = oracle.riemann(1.4, WL, WR)
        assert abs(ps - pe) <= 1e-11 * pe and abs(us - ue) <= 1e-11 * (1 + abs(ue))
        np.testing.assert_allclose(W0, We, rtol=1e-11, atol=1e-13)
    assert seen > 100


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0, 1.2])
def test_trrs_solves_the_two_rarefaction_pressure_equation(g):
    """p* is the root of f_L + f_R + u_R - u_L = 0 with both sides on the
    rarefaction branch (also for data whose exact solution has shocks), and
    u* = (u_L + u_R)/2 + (f_R - f_L)/2."""
    rng = np.random.default_rng(32)
    for _ in range(200):
        WL = (np.exp(rng.uniform(-2, 2)), rng.uniform(-1, 1), np.exp(rng.uniform(-2, 2)))
        WR = (np.exp(rng.uniform(-2, 2)), rng.uniform(-1, 1), np.exp(rng.uniform(-2, 2)))
        try:
            ps, us, _ = oracle.trrs(g, WL, WR)
        except oracle.OracleError:
            continue
        fl = _raref_f(g, ps, WL[0], WL[1], WL[2])
        fr = _raref_f(g, ps, WR[0], WR[1], WR[2])
        scale = np.sqrt(g * WL[2] / WL[0]) + np.sqrt(g * WR[2] / WR[0])
        assert abs(fl + fr + WR[1] - WL[1]) <= 1e-12 * scale
        assert abs(us - (0.5 * (WL[1] + WR[1]) + 0.5 * (fr - fl))) <= 1e-12 * scale


def test_trrs_mirror_symmetry_and_shock_bias():
    """Mirrored data (swap sides, negate velocities) give the same p* and the
    negated u*; where the exact solution has a shock, the rarefaction curve
    lies below the Hugoniot curve, so the approximate p* is not below the
    exact one (Sod: 0.3068 vs 0.3031)."""
    rng = np.random.default_rng(33)
    shocks = 0
    for _ in range(300):
        WL = (np.exp(rng.uniform(-2, 2)), rng.uniform(-1, 1), np.exp(rng.uniform(-2, 2)))
        WR = (np.exp(rng.uniform(-2, 2)), rng.uniform(-1, 1), np.exp(rng.uniform(-2, 2)))
        try:
            ps, us, W0 = oracle.trrs(1.4, WL, WR)
        except oracle.OracleError:
            continue
        pm, um, Wm = oracle.trrs(1.4, (WR[0], -WR[1], WR[2]), (WL[0], -WL[1], WL[2]))
        assert abs(pm - ps) <= 1e-13 * ps and abs(um + us) <= 1e-13 * (1 + abs(us))
        if abs(us) > 1e-12:
            np.testing.assert_allclose(Wm, [W0[0], -W0[1], W0[2]], rtol=1e-12, atol=1e-14)
        rc, pe, _ = oracle.riemann_rc(1.4, WL, WR)
        if rc == oracle.OK and pe > min(WL[2], WR[2]):
            shocks += 1
            assert ps >= pe * (1 - 1e-12)
    assert shocks > 50
    ps, _, _ = oracle.trrs(1.4, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    pe, _, _, _ = oracle.riemann(1.4, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert ps > pe


def test_trrs_weak_waves_and_vacuum():
    """Weak jumps: the approximation differs from the exact solution at third
    order in the jump (Hugoniot and isentrope agree to second order); vacuum
    is reported by the same criterion as the exact solver."""
    base = np.array([1.0, 0.2, 1.0])
    errs = []
    for eps in (1e-2, 5e-3):
        WR = base * np.array([1 + eps, 1.0, 1 + 2 * eps])  # compression: a weak shock
        ps, _, _ = oracle.trrs(1.4, base, WR)
        pe, _, _, _ = oracle.riemann(1.4, base, WR)
        errs.append(abs(ps - pe))
    assert errs[1] < errs[0] / 6.0  # ~ eps^3: ratio 8
    with pytest.raises(oracle.OracleError) as ei:
        oracle.trrs(1.4, (1.0, -6.0, 0.4), (1.0, 6.0, 0.4))
    assert ei.value.code == oracle.E_VACUUM
