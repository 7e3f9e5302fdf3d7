"""GPU parity of the relaxation source S(Q) = -kappa Q (eq. eq_finite_volume
with S^n_i of eq. source, the predictor locally implicit in the source,
Sec. 2) against the oracle: advection at every order, both signs of the
speed, periodic and transmissive ends, moderate and stiff rates; Euler at
every order on one domain and on a network of segments.  Bars: relative
L-infinity 1e-11 after one step, 1e-9 at the end of the run."""
import numpy as np
import pytest

import oracle
from paper_2602_21911_amd import inputs as I

from ._cases import acoustic_case, network_case, rel_linf

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ONE_STEP = 1e-11
T_END = 1e-9


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_21911_amd import grprec
    grprec.lib()
    return grprec


def _ocfg(system, order, bc, kappa, **kw):
    return oracle.cfg(system, order, bc=bc, source=oracle.SOURCE_LINEAR, kappa=kappa, **kw)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
@pytest.mark.parametrize("lam,bc", [(1.0, 0), (-0.7, 1), (0.6, 1)])
@pytest.mark.parametrize("kappa", [1.5, 3e5])
def test_advection_source_parity(G, order, lam, bc, kappa):
    """kappa = 3e5 makes kappa dt about 900 at 300 cells (stiff)."""
    n = 300
    dx, q, vl, vr = I.adv_sin2pi(n)
    q, vl, vr = q + 0.5, vl + 0.5, vr + 0.5
    obc = oracle.PERIODIC if bc == 0 else oracle.TRANSMISSIVE
    c = _ocfg(oracle.ADVECTION, order, obc, kappa, lam=lam)
    v = oracle.init_interfaces(c, vl, vr)
    sim = G.Simulation(G.GRPREC_ADVECTION, order, [n], [1.0], q, vl, vr, lam=lam,
                       bc=G.GRPREC_BC_PERIODIC if bc == 0 else G.GRPREC_BC_TRANSMISSIVE,
                       source=G.GRPREC_SOURCE_LINEAR, kappa=kappa)
    try:
        print(f"advection source order {order} lambda {lam} bc {bc} kappa {kappa}", flush=True)
        sim.step(1.0)
        qo, vo, _, _, _ = oracle.step(c, dx, q, v, 0.0, 1.0)
        qg, vg, _, _ = sim.numpy_state()
        assert rel_linf(qg, qo) <= ONE_STEP and rel_linf(vg, vo) <= ONE_STEP
        sim.run(0.05)
        qr, vr_, tr, kr, _ = oracle.run(c, dx, q, v, 0.0, 0.05)
        qg, vg, t, steps = sim.numpy_state()
        assert steps == kr and t == tr
        # a stiff run decays to round-off: compare against the initial scale
        scale = np.abs(q).max() if kappa > 1e3 else None
        if scale is None:
            assert rel_linf(qg, qr) <= T_END and rel_linf(vg, vr_) <= T_END
        else:
            assert np.abs(qg - qr).max() <= T_END * scale and np.abs(vg - vr_).max() <= T_END * scale
    finally:
        sim.close()


@pytest.mark.parametrize("order", [2, 3, 4, 5])
@pytest.mark.parametrize("bc,block", [(0, 64), (1, 256)])
def test_euler_source_parity(G, order, bc, block):
    n = 300
    dx, q, vl, vr = acoustic_case(n)
    obc = oracle.PERIODIC if bc == 0 else oracle.TRANSMISSIVE
    c = _ocfg(oracle.EULER, order, obc, 2.0)
    v = oracle.init_interfaces(c, vl, vr)
    sim = G.Simulation(G.GRPREC_EULER, order, [n], [1.0], q, vl, vr,
                       bc=G.GRPREC_BC_PERIODIC if bc == 0 else G.GRPREC_BC_TRANSMISSIVE,
                       schedule=G.GRPREC_SCHED_SEGMENT_TILES, block=block,
                       source=G.GRPREC_SOURCE_LINEAR, kappa=2.0)
    try:
        print(f"euler source order {order} bc {bc} block {block}", flush=True)
        dt = sim.step(1.0, want_dt=True)
        qo, vo, dto, _, _ = oracle.step(c, dx, q, v, 0.0, 1.0)
        assert abs(dt - dto) <= 1e-14 * dto
        qg, vg, _, _ = sim.numpy_state()
        assert rel_linf(qg, qo) <= ONE_STEP and rel_linf(vg, vo) <= ONE_STEP
        sim.run(0.1)
        qr, vr_, tr, kr, _ = oracle.run(c, dx, q, v, 0.0, 0.1)
        qg, vg, t, steps = sim.numpy_state()
        assert steps == kr and t == tr
        assert rel_linf(qg, qr) <= T_END and rel_linf(vg, vr_) <= T_END
    finally:
        sim.close()


@pytest.mark.parametrize("schedule,block", [(2, 64), (3, 128)])
def test_euler_source_network_parity(G, schedule, block):
    net = network_case(40, seed=9, nmax=400)
    S = len(net.n_cells)
    c = _ocfg(oracle.EULER, 3, oracle.TRANSMISSIVE, 1.0)
    v0 = oracle.init_interfaces(c, net.vl, net.vr)
    qr, vr_, tr, _ = oracle.run_segments(c, net.cell_off, net.dx, net.q, v0, np.zeros(S), 1e9, 6)
    sim = G.Simulation(G.GRPREC_EULER, 3, net.n_cells, net.lengths, net.q, net.vl, net.vr,
                       bc=G.GRPREC_BC_TRANSMISSIVE, schedule=schedule, block=block,
                       source=G.GRPREC_SOURCE_LINEAR, kappa=1.0)
    try:
        print(f"euler source network schedule {schedule} block {block}", flush=True)
        steps, _ = sim.run(1e9, 6)
        assert steps == 6
        qg, vg, _, _ = sim.numpy_state()
        np.testing.assert_allclose(sim.times(), tr, rtol=1e-14)
    finally:
        sim.close()
    for s in range(S):
        c0, c1 = net.cell_off[s], net.cell_off[s + 1]
        assert rel_linf(qg[:, c0:c1], qr[:, c0:c1]) <= 10 * ONE_STEP, s
        assert rel_linf(vg[:, c0 + s:c1 + s + 1], vr_[:, c0 + s:c1 + s + 1]) <= 10 * ONE_STEP, s


def test_euler_stiff_source_reported_like_the_oracle(G):
    """kappa dt = 40: the predictor's nodal densities turn negative (see the
    oracle pins); both sides report a non-physical state."""
    n = 20
    dx, q, vl, vr = I.euler_density_wave(n)
    dt = 0.9 * dx / oracle.smax(oracle.cfg(oracle.EULER, 3), q)
    kappa = 40.0 / dt
    c = _ocfg(oracle.EULER, 3, oracle.PERIODIC, kappa)
    with pytest.raises(oracle.OracleError):
        oracle.step(c, dx, q, oracle.init_interfaces(c, vl, vr), 0.0, 1.0)
    sim = G.Simulation(G.GRPREC_EULER, 3, [n], [1.0], q, vl, vr, schedule=G.GRPREC_SCHED_SEGMENT_TILES,
                       block=64, source=G.GRPREC_SOURCE_LINEAR, kappa=kappa)
    try:
        with pytest.raises(G.GrprecError) as ei:
            sim.step(1.0, want_dt=True)
        assert ei.value.code == G.GRPREC_E_NONPHYSICAL
    finally:
        sim.close()


def test_source_options_validated(G):
    dx, q, vl, vr = I.euler_density_wave(40)
    for kw, code in ((dict(source=7), G.GRPREC_E_INVALID),
                     (dict(source=G.GRPREC_SOURCE_LINEAR, kappa=-1.0), G.GRPREC_E_INVALID),
                     (dict(source=G.GRPREC_SOURCE_LINEAR, kappa=1.0, recon=G.GRPREC_RECON_NL),
                      G.GRPREC_E_UNSUPPORTED),
                     (dict(source=G.GRPREC_SOURCE_LINEAR, kappa=1.0, datum=G.GRPREC_DATUM_TRRS),
                      G.GRPREC_E_UNSUPPORTED)):
        with pytest.raises(G.GrprecError) as ei:
            G.Simulation(G.GRPREC_EULER, 3, [40], [1.0], q, vl, vr, **kw)
        assert ei.value.code == code, kw
