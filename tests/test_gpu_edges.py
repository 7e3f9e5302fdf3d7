"""Edge cases of the HIP path against the oracle: the smallest domains,
sizes on either side of the kernels' work-unit boundaries (63-cell wave
runs and 504-cell chunks of the advection kernel; 62/126/254-cell tiles of
the Euler kernel), a network with 2-cell segments, steps requested past
t_end, non-physical initial data, and advection at the 2^25 cells the
benchmark times."""
import numpy as np
import pytest

import oracle
from paper_2602_21911_amd import inputs as I

from ._cases import rel_linf

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


@pytest.mark.parametrize("n", [2, 3, 60, 61, 62, 63, 64, 121, 122, 123, 125, 126, 127, 487, 488, 489,
                               503, 504, 505, 975, 976, 977, 1009])
@pytest.mark.parametrize("lam,bc", [(1.0, 0), (-0.7, 1), (0.6, 1)])
def test_advection_sizes(G, n, lam, bc):
    """Run and chunk boundaries of the advection kernel (61 updated cells per
    wave, 488 per block chunk) and tiny domains, both signs of the speed."""
    order = 3 if n % 2 else 5
    dx, q, vl, vr = I.adv_sin2pi(n)
    obc = oracle.PERIODIC if bc == 0 else oracle.TRANSMISSIVE
    c = oracle.cfg(oracle.ADVECTION, order, lam=lam, bc=obc)
    v = oracle.init_interfaces(c, vl, vr)
    sim = G.Simulation(G.GRPREC_ADVECTION, order, [n], [1.0], q, vl, vr, lam=lam,
                       bc=G.GRPREC_BC_PERIODIC if bc == 0 else G.GRPREC_BC_TRANSMISSIVE)
    try:
        print(f"advection n={n} order {order} lambda {lam} bc {bc}", flush=True)
        sim.run(0.05)
        qr, vr_, tr, kr, _ = oracle.run(c, dx, q, v, 0.0, 0.05)
        qg, vg, t, steps = sim.numpy_state()
        assert steps == kr and t == tr
        assert rel_linf(qg, qr) <= T_END and rel_linf(vg, vr_) <= T_END
    finally:
        sim.close()


@pytest.mark.parametrize("n", [2, 3, 61, 62, 63, 126, 127, 253, 254, 255])
def test_euler_sizes(G, n):
    """Single periodic and transmissive Euler domains at tile boundaries for
    blocks of 64, 128 and 256 (62, 126, 254 useful cells per tile)."""
    dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=1.0)
    for bc, block in ((0, 64), (1, 128), (1, 256)):
        obc = oracle.PERIODIC if bc == 0 else oracle.TRANSMISSIVE
        c = oracle.cfg(oracle.EULER, 3, bc=obc)
        v = oracle.init_interfaces(c, vl, vr)
        sim = G.Simulation(G.GRPREC_EULER, 3, [n], [1.0], q, vl, vr,
                           bc=G.GRPREC_BC_PERIODIC if bc == 0 else G.GRPREC_BC_TRANSMISSIVE,
                           schedule=G.GRPREC_SCHED_SEGMENT_TILES, block=block)
        try:
            print(f"Euler n={n} bc {bc} block {block}", flush=True)
            sim.run(1e9, 5)
            qr, vr_, tr, kr, _ = oracle.run(c, dx, q, v, 0.0, 1e9, 5)
            qg, vg, t, steps = sim.numpy_state()
            assert steps == 5 and abs(t - tr) <= 1e-14 * tr
            assert rel_linf(qg, qr) <= T_END and rel_linf(vg, vr_) <= T_END
        finally:
            sim.close()


def test_network_with_two_cell_segments(G):
    """Segments of 2 and 3 cells (the smallest allowed) mixed with longer
    ones, every schedule."""
    rng = np.random.default_rng(12)
    cells = rng.choice([2, 3, 2, 5, 62, 63, 64, 200], size=40)
    S = len(cells)
    off = np.concatenate([[0], np.cumsum(cells)])
    lengths = rng.uniform(0.05, 1.0, S)
    dx = lengths / cells
    tc = int(off[-1])
    rho_c = np.empty(tc)
    rho_f = np.empty(tc + S)
    for s in range(S):
        xf = dx[s] * np.arange(cells[s] + 1)
        k = 3.0
        rho_c[off[s]:off[s + 1]] = 1.0 + 0.1 * (np.cos(k * xf[:-1]) - np.cos(k * xf[1:])) / (k * dx[s])
        rho_f[off[s] + s:off[s + 1] + s + 1] = 1.0 + 0.1 * np.sin(k * xf)
    q = I.prim_to_cons(rho_c, 0.4, 1.0)
    v = I.prim_to_cons(rho_f, 0.4, 1.0)
    c = oracle.cfg(oracle.EULER, 3, bc=oracle.TRANSMISSIVE)
    v0 = oracle.init_interfaces(c, v, v)
    qr, vr_, tr, _ = oracle.run_segments(c, off.astype(np.int64), dx, q, v0, np.zeros(S), 1e9, 4)
    for schedule, block in ((1, 64), (2, 128), (3, 256), (4, 64)):
        sim = G.Simulation(G.GRPREC_EULER, 3, cells, lengths, q, v, v, bc=G.GRPREC_BC_TRANSMISSIVE,
                           schedule=schedule, block=block)
        try:
            print(f"2-cell network schedule {schedule} block {block}", flush=True)
            steps, _ = sim.run(1e9, 4)
            assert steps == 4
            qg, vg, _, _ = sim.numpy_state()
            np.testing.assert_allclose(sim.times(), tr, rtol=1e-14)
        finally:
            sim.close()
        for s in range(S):
            c0, c1 = off[s], off[s + 1]
            assert rel_linf(qg[:, c0:c1], qr[:, c0:c1]) <= ONE_STEP * 10, (schedule, s)
            assert rel_linf(vg[:, c0 + s:c1 + s + 1], vr_[:, c0 + s:c1 + s + 1]) <= ONE_STEP * 10


def test_steps_past_t_end_leave_the_state(G):
    """Once every domain has reached t_end further steps change nothing."""
    n = 100
    dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=1.0)
    sim = G.Simulation(G.GRPREC_EULER, 3, [n], [1.0], q, vl, vr, bc=G.GRPREC_BC_PERIODIC)
    try:
        done, t = sim.run(0.01)
        assert t == 0.01
        q1, v1, _, _ = sim.numpy_state()
        for _ in range(3):
            sim.step(0.01)
        q2, v2, t2, _ = sim.numpy_state()
        assert t2 == 0.01
        np.testing.assert_array_equal(q1, q2)
        np.testing.assert_array_equal(v1, v2)
    finally:
        sim.close()


def test_nonphysical_initial_data_reported(G):
    """A negative initial pressure is reported as a non-physical state, by
    the oracle and through the C ABI."""
    n = 50
    dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=1.0)
    q = q.copy()
    q[2, 20] = 0.5 * q[1, 20] ** 2 / q[0, 20] - 0.1  # E below the kinetic energy: p < 0
    c = oracle.cfg(oracle.EULER, 3)
    v = oracle.init_interfaces(c, vl, vr)
    with pytest.raises(oracle.OracleError) as eo:
        oracle.step(c, dx, q, v, 0.0, 1.0)
    assert eo.value.code == oracle.E_NONPHYSICAL
    with pytest.raises(G.GrprecError) as eg:
        sim = G.Simulation(G.GRPREC_EULER, 3, [n], [1.0], q, vl, vr, bc=G.GRPREC_BC_PERIODIC,
                           schedule=G.GRPREC_SCHED_SEGMENT_TILES, block=64)
        try:
            sim.run(1.0, 3)
        finally:
            sim.close()
    assert eg.value.code == G.GRPREC_E_NONPHYSICAL


def test_advection_2e25_windows(G):
    """The benchmark's advection size: windows of the oracle with a margin
    reproduce the GPU state after 3 steps; the periodic total is conserved."""
    n = 1 << 25
    steps = 3
    dx, q, vl, vr = I.adv_sin2pi(n)
    sim = G.Simulation(G.GRPREC_ADVECTION, 3, [n], [1.0], q, vl, vr, bc=G.GRPREC_BC_PERIODIC)
    try:
        done, _ = sim.run(1e9, steps)
        assert done == steps
        qg, vg, t, _ = sim.numpy_state()
    finally:
        sim.close()
    c = oracle.cfg(oracle.ADVECTION, 3, bc=oracle.TRANSMISSIVE)
    cp = oracle.cfg(oracle.ADVECTION, 3, bc=oracle.PERIODIC)
    margin = 4 * steps + 4
    for start in (1000, n // 2 + 17, n - 1000 - 64):
        a, b = start - margin, start + 64 + margin
        v0 = oracle.init_interfaces(cp, vl[:, a:b + 1], vr[:, a:b + 1])
        qw, vw, tw, kw, _ = oracle.run(c, dx, q[:, a:b], v0, 0.0, 1e9, steps)
        sl = slice(margin, margin + 64)
        assert rel_linf(qg[:, a:b][:, sl], qw[:, sl]) <= 1e-11
        assert rel_linf(vg[:, a:b + 1][:, sl], vw[:, sl]) <= 1e-11
    assert abs(qg.sum() - q.sum()) <= 1e-12 * np.abs(q).sum()
