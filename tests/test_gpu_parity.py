"""GPU parity: the HIP path (through the C ABI) against the oracle on the same
seeded inputs.  Bar: relative L-infinity <= 1e-11 after one step and <= 1e-9
at t_end, per variable, for q and for the interface data."""
import numpy as np
import pytest

import oracle
from paper_2602_21911_amd import inputs as I

from ._cases import acoustic_case, advection_case, network_case, oracle_cfg, rel_linf

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


def _gpu_sim(G, system, order, cells, lengths, q, vl, vr, bc, **kw):
    return G.Simulation(system, order, cells, lengths, q, vl, vr, bc=bc, **kw)


# ------------------------------------------------------------- advection
@pytest.mark.parametrize("order", [2, 3, 4, 5])
@pytest.mark.parametrize("kind,n", [("sin2pi", 100), ("square", 64), ("sin2pi", 1027)])
def test_advection_parity(G, order, kind, n):
    dx, q, vl, vr = advection_case(kind, n)
    c = oracle_cfg(oracle.ADVECTION, order, oracle.PERIODIC)
    v = oracle.init_interfaces(c, vl, vr)
    sim = _gpu_sim(G, G.GRPREC_ADVECTION, order, [n], [1.0], q, vl, vr, G.GRPREC_BC_PERIODIC)
    try:
        dt = sim.step(1.0, want_dt=True)
        qo, vo, dto, _, _ = oracle.step(c, dx, q, v, 0.0, 1.0)
        assert abs(dt - dto) <= 1e-15 * dto
        qg, vg, t, steps = sim.numpy_state()
        assert rel_linf(qg, qo) <= ONE_STEP
        assert rel_linf(vg, vo) <= ONE_STEP
        steps, t = sim.run(1.0)
        qr, vr_, tr, kr, _ = oracle.run(c, dx, q, v, 0.0, 1.0)
        qg, vg, t, steps = sim.numpy_state()
        assert t == tr == 1.0 and steps == kr
        assert rel_linf(qg, qr) <= T_END
        assert rel_linf(vg, vr_) <= T_END
    finally:
        sim.close()


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_advection_negative_speed_transmissive(G, order):
    n = 80
    dx, q, vl, vr = advection_case("sin2pi", n)
    c = oracle_cfg(oracle.ADVECTION, order, oracle.TRANSMISSIVE, lam=-0.7)
    v = oracle.init_interfaces(c, vl, vr)
    sim = _gpu_sim(G, G.GRPREC_ADVECTION, order, [n], [1.0], q, vl, vr, G.GRPREC_BC_TRANSMISSIVE,
                   lam=-0.7)
    try:
        sim.run(0.3)
        qr, vr_, tr, kr, _ = oracle.run(c, dx, q, v, 0.0, 0.3)
        qg, vg, t, steps = sim.numpy_state()
        assert steps == kr
        assert rel_linf(qg, qr) <= T_END and rel_linf(vg, vr_) <= T_END
    finally:
        sim.close()


# ------------------------------------------------------------- Euler
@pytest.mark.parametrize("order", [2, 3, 4, 5])
@pytest.mark.parametrize("block", [64, 256])
def test_euler_density_wave_parity(G, order, block):
    n = 300  # several tiles and a ragged tail at every block size
    dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=1.0)
    c = oracle_cfg(oracle.EULER, order, oracle.PERIODIC)
    v = oracle.init_interfaces(c, vl, vr)
    sim = _gpu_sim(G, G.GRPREC_EULER, order, [n], [1.0], q, vl, vr, G.GRPREC_BC_PERIODIC,
                   schedule=G.GRPREC_SCHED_SEGMENT_TILES, block=block)
    try:
        dt = sim.step(2.0, want_dt=True)
        qo, vo, dto, _, _ = oracle.step(c, dx, q, v, 0.0, 2.0)
        assert abs(dt - dto) <= 1e-14 * dto
        qg, vg, _, _ = sim.numpy_state()
        assert rel_linf(qg, qo) <= ONE_STEP and rel_linf(vg, vo) <= ONE_STEP
        sim.run(0.25)
        qr, vr_, tr, kr, _ = oracle.run(c, dx, q, v, 0.0, 0.25)
        qg, vg, t, steps = sim.numpy_state()
        assert t == tr and steps == kr
        assert rel_linf(qg, qr) <= T_END and rel_linf(vg, vr_) <= T_END
    finally:
        sim.close()


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_euler_acoustic_parity(G, order):
    """Genuinely nonlinear smooth flow (rho, u, p all vary)."""
    n = 130
    dx, q, vl, vr = acoustic_case(n)
    c = oracle_cfg(oracle.EULER, order, oracle.PERIODIC)
    v = oracle.init_interfaces(c, vl, vr)
    sim = _gpu_sim(G, G.GRPREC_EULER, order, [n], [1.0], q, vl, vr, G.GRPREC_BC_PERIODIC,
                   schedule=G.GRPREC_SCHED_SEGMENT_TILES, block=128)
    try:
        sim.step(1.0)
        qo, vo, _, _, _ = oracle.step(c, dx, q, v, 0.0, 1.0)
        qg, vg, _, _ = sim.numpy_state()
        assert rel_linf(qg, qo) <= ONE_STEP and rel_linf(vg, vo) <= ONE_STEP
        sim.run(0.3)
        qr, vr_, tr, kr, _ = oracle.run(c, dx, q, v, 0.0, 0.3)
        qg, vg, t, steps = sim.numpy_state()
        assert steps == kr
        assert rel_linf(qg, qr) <= T_END and rel_linf(vg, vr_) <= T_END
    finally:
        sim.close()


@pytest.mark.parametrize("schedule", [1, 2, 3])
@pytest.mark.parametrize("block", [64, 128, 256])
def test_network_parity_every_schedule(G, schedule, block):
    """Independent transmissive segments of uneven length (3 .. 400 cells):
    every segment after one of its own steps equals the single-domain oracle
    within the one-step bar, and after 3 within 1e-10."""
    net = network_case(40, seed=5, nmax=400)
    S = len(net.n_cells)
    c = oracle_cfg(oracle.EULER, 3, oracle.TRANSMISSIVE)
    v0 = oracle.init_interfaces(c, net.vl, net.vr)
    q1, v1, _, _ = oracle.run_segments(c, net.cell_off, net.dx, net.q, v0, np.zeros(S), 1e9, 1)
    qr, vr_, tr, _ = oracle.run_segments(c, net.cell_off, net.dx, net.q, v0, np.zeros(S), 1e9, 3)
    sim = _gpu_sim(G, G.GRPREC_EULER, 3, net.n_cells, net.lengths, net.q, net.vl, net.vr,
                   G.GRPREC_BC_TRANSMISSIVE, schedule=schedule, block=block)
    try:
        steps, _ = sim.run(1e9, 1)
        assert steps == 1
        qg, vg, _, _ = sim.numpy_state()
        for s in range(S):
            c0, c1 = net.cell_off[s], net.cell_off[s + 1]
            assert rel_linf(qg[:, c0:c1], q1[:, c0:c1]) <= ONE_STEP, s
            assert rel_linf(vg[:, c0 + s:c1 + s + 1], v1[:, c0 + s:c1 + s + 1]) <= ONE_STEP, s
        steps, _ = sim.run(1e9, 2)
        assert steps == 2
        qg, vg, _, _ = sim.numpy_state()
        np.testing.assert_allclose(sim.times(), tr, rtol=1e-14)
        for s in range(S):
            c0, c1 = net.cell_off[s], net.cell_off[s + 1]
            assert rel_linf(qg[:, c0:c1], qr[:, c0:c1]) <= ONE_STEP * 10, s
            assert rel_linf(vg[:, c0 + s:c1 + s + 1], vr_[:, c0 + s:c1 + s + 1]) <= ONE_STEP * 10, s
    finally:
        sim.close()


def test_graph_replay_bitwise_equals_eager(G):
    """grprec_run (captured graphs of 30 steps) == the same steps launched one by one."""
    net = network_case(25, seed=11, nmax=300)
    outs = []
    for use_run in (True, False):
        sim = _gpu_sim(G, G.GRPREC_EULER, 3, net.n_cells, net.lengths, net.q, net.vl, net.vr,
                       G.GRPREC_BC_TRANSMISSIVE, schedule=G.GRPREC_SCHED_PACKED, block=128)
        try:
            if use_run:
                sim.run(1e9, 67)
            else:
                for _ in range(67):
                    sim.step(1e9)
            qg, vg, _, steps = sim.numpy_state()
            assert steps == 67
            outs.append((qg, vg))
        finally:
            sim.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


def test_sod_linear_grprec_reports_failure(G):
    """Both sides refuse the Sod tube with linear GRPrec at the first step."""
    n = 100
    dx, q, vl, vr = I.euler_shock_tube(n)
    c = oracle_cfg(oracle.EULER, 3, oracle.TRANSMISSIVE)
    v = oracle.init_interfaces(c, vl, vr)
    with pytest.raises(oracle.OracleError):
        oracle.step(c, dx, q, v, 0.0, 0.2)
    sim = _gpu_sim(G, G.GRPREC_EULER, 3, [n], [1.0], q, vl, vr, G.GRPREC_BC_TRANSMISSIVE)
    try:
        with pytest.raises(G.GrprecError) as ei:
            sim.step(0.2, want_dt=True)
        assert ei.value.code in (G.GRPREC_E_PREDICTOR, G.GRPREC_E_NONPHYSICAL)
    finally:
        sim.close()


# ------------------------------------------------------------- Riemann solver
def test_riemann_batch_matches_oracle(G):
    WL, WR = I.random_tube_states(20260223, 4000)
    wl = torch.from_numpy(WL).cuda()
    wr = torch.from_numpy(WR).cuda()
    ps, it = G.grprec_riemann_batch(wl, wr)
    ps = ps.cpu().numpy()
    it = it.cpu().numpy()
    n_ok = 0
    for k in range(len(WL)):
        rc, p_ref, it_ref = oracle.riemann_rc(1.4, WL[k], WR[k])
        if rc == oracle.OK:
            assert abs(ps[k] - p_ref) <= 1e-12 * p_ref, k
            assert abs(int(it[k]) - it_ref) <= 1, k
            n_ok += 1
        else:
            assert int(it[k]) == rc, (k, it[k], rc)
    assert n_ok > 1000


def test_riemann_batch_weak_waves(G):
    """Near-equal states (|p*/pK - 1| from 1e-12 to 1e-3) straddle the weak-wave
    threshold of the solver; p* agrees with the oracle's closed forms."""
    rng = np.random.default_rng(12)
    n = 3000
    base = np.stack([rng.uniform(0.3, 3, n), rng.uniform(-1, 1, n), rng.uniform(0.3, 3, n)], 1)
    eps = 10.0 ** rng.uniform(-12, -3, n)
    WL = base * (1 + eps[:, None] * rng.normal(size=(n, 3)))
    WR = base * (1 + eps[:, None] * rng.normal(size=(n, 3)))
    ps, it = G.grprec_riemann_batch(torch.from_numpy(WL).cuda(), torch.from_numpy(WR).cuda())
    ps = ps.cpu().numpy()
    for k in range(n):
        p_ref, _, _, _ = oracle.riemann(1.4, WL[k], WR[k])
        assert abs(ps[k] - p_ref) <= 1e-13 * p_ref, (k, eps[k])


@pytest.mark.parametrize("order", [2, 3])
def test_euler_weak_jumps_parity(G, order):
    """Smooth data with a tiny superposed perturbation: every interface problem
    is a weak wave; both sampling branches and the threshold are crossed."""
    n = 200
    dx, q, vl, vr = acoustic_case(n, amp=1e-4)
    c = oracle_cfg(oracle.EULER, order, oracle.PERIODIC)
    v = oracle.init_interfaces(c, vl, vr)
    sim = _gpu_sim(G, G.GRPREC_EULER, order, [n], [1.0], q, vl, vr, G.GRPREC_BC_PERIODIC,
                   schedule=G.GRPREC_SCHED_SEGMENT_TILES, block=64)
    try:
        sim.run(0.2)
        qr, vr_, tr, kr, _ = oracle.run(c, dx, q, v, 0.0, 0.2)
        qg, vg, t, steps = sim.numpy_state()
        assert steps == kr
        assert rel_linf(qg, qr) <= T_END and rel_linf(vg, vr_) <= T_END
    finally:
        sim.close()


@pytest.mark.parametrize("schedule,block", [(2, 64), (3, 128)])
def test_network_parity_order5(G, schedule, block):
    """Order 5 (degree 4) on the batched network: every segment after one of
    its own steps equals the single-domain oracle within the one-step bar,
    and after 3 within 1e-10."""
    net = network_case(30, seed=6, nmax=300)
    S = len(net.n_cells)
    c = oracle_cfg(oracle.EULER, 5, oracle.TRANSMISSIVE)
    v0 = oracle.init_interfaces(c, net.vl, net.vr)
    q1, v1, _, _ = oracle.run_segments(c, net.cell_off, net.dx, net.q, v0, np.zeros(S), 1e9, 1)
    qr, vr_, tr, _ = oracle.run_segments(c, net.cell_off, net.dx, net.q, v0, np.zeros(S), 1e9, 3)
    sim = _gpu_sim(G, G.GRPREC_EULER, 5, net.n_cells, net.lengths, net.q, net.vl, net.vr,
                   G.GRPREC_BC_TRANSMISSIVE, schedule=schedule, block=block)
    try:
        print(f"network order 5 schedule {schedule} block {block}", flush=True)
        steps, _ = sim.run(1e9, 1)
        assert steps == 1
        qg1, vg1, _, _ = sim.numpy_state()
        steps, _ = sim.run(1e9, 2)
        assert steps == 2
        qg, vg, _, _ = sim.numpy_state()
    finally:
        sim.close()
    for s in range(S):
        c0, c1 = net.cell_off[s], net.cell_off[s + 1]
        assert rel_linf(qg1[:, c0:c1], q1[:, c0:c1]) <= ONE_STEP, s
        assert rel_linf(vg1[:, c0 + s:c1 + s + 1], v1[:, c0 + s:c1 + s + 1]) <= ONE_STEP, s
    for s in range(S):
        c0, c1 = net.cell_off[s], net.cell_off[s + 1]
        assert rel_linf(qg[:, c0:c1], qr[:, c0:c1]) <= ONE_STEP * 10, s
        assert rel_linf(vg[:, c0 + s:c1 + s + 1], vr_[:, c0 + s:c1 + s + 1]) <= ONE_STEP * 10, s


# ------------------------------------------------------------- configured end times
@pytest.mark.parametrize("order", [2, 3, 4])
def test_euler_density_wave_to_configured_end_time(G, order):
    """The Euler density wave (rho = 1 + 0.2 sin 2 pi x, u = 1, p = 1,
    periodic) run to its configured end time t = 2 (about a thousand steps at
    200 cells): the t_end bar holds after the whole run, and the GPU took the
    oracle's number of steps and landed on t = 2."""
    n = 200
    dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=1.0)
    c = oracle_cfg(oracle.EULER, order, oracle.PERIODIC)
    v = oracle.init_interfaces(c, vl, vr)
    sim = _gpu_sim(G, G.GRPREC_EULER, order, [n], [1.0], q, vl, vr, G.GRPREC_BC_PERIODIC,
                   schedule=G.GRPREC_SCHED_SEGMENT_TILES, block=64)
    try:
        print(f"density wave to t = 2, order {order}", flush=True)
        sim.run(2.0)
        qr, vr_, tr, kr, _ = oracle.run(c, dx, q, v, 0.0, 2.0)
        qg, vg, t, steps = sim.numpy_state()
        assert t == tr == 2.0 and steps == kr and kr > 900
        assert rel_linf(qg, qr) <= T_END and rel_linf(vg, vr_) <= T_END
    finally:
        sim.close()


def test_network_parity_over_hundreds_of_steps(G):
    """A network of uneven transmissive segments (3 .. 300 cells) advanced 300
    of each segment's own steps: every segment within the t_end bar of the
    single-domain oracle."""
    net = network_case(24, seed=11, nmax=300)
    S = len(net.n_cells)
    c = oracle_cfg(oracle.EULER, 3, oracle.TRANSMISSIVE)
    v0 = oracle.init_interfaces(c, net.vl, net.vr)
    qr, vr_, tr, _ = oracle.run_segments(c, net.cell_off, net.dx, net.q, v0, np.zeros(S), 1e9, 300)
    sim = _gpu_sim(G, G.GRPREC_EULER, 3, net.n_cells, net.lengths, net.q, net.vl, net.vr,
                   G.GRPREC_BC_TRANSMISSIVE, schedule=G.GRPREC_SCHED_FLAT_TILES, block=64)
    try:
        print("network, 300 steps", flush=True)
        steps, _ = sim.run(1e9, 300)
        assert steps == 300
        qg, vg, _, _ = sim.numpy_state()
        np.testing.assert_allclose(sim.times(), tr, rtol=1e-12)
    finally:
        sim.close()
    for s in range(S):
        c0, c1 = net.cell_off[s], net.cell_off[s + 1]
        assert rel_linf(qg[:, c0:c1], qr[:, c0:c1]) <= T_END, s
        assert rel_linf(vg[:, c0 + s:c1 + s + 1], vr_[:, c0 + s:c1 + s + 1]) <= T_END, s


@pytest.mark.parametrize("schedule,block", [(1, 64), (2, 64), (3, 128)])
def test_network_segments_reach_t_end_at_their_own_steps(G, schedule, block):
    """Uneven transmissive segments advanced to a common t_end: each segment
    takes its own number of steps and then carries its state over while the
    others go on (including the interface value at its left end); every
    segment ends at t_end within the t_end bar of the oracle."""
    net = network_case(24, seed=13, nmax=120)
    S = len(net.n_cells)
    c = oracle_cfg(oracle.EULER, 3, oracle.TRANSMISSIVE)
    v0 = oracle.init_interfaces(c, net.vl, net.vr)
    t_end = 0.02
    qr, vr_, tr, _ = oracle.run_segments(c, net.cell_off, net.dx, net.q, v0, np.zeros(S), t_end, 100000)
    assert np.all(tr == t_end)
    sim = _gpu_sim(G, G.GRPREC_EULER, 3, net.n_cells, net.lengths, net.q, net.vl, net.vr,
                   G.GRPREC_BC_TRANSMISSIVE, schedule=schedule, block=block)
    try:
        print(f"network to t_end, schedule {schedule} block {block}", flush=True)
        steps, _ = sim.run(t_end)
        qg, vg, _, _ = sim.numpy_state()
        times = sim.times()
    finally:
        sim.close()
    np.testing.assert_array_equal(times, tr)
    for s in range(S):
        c0, c1 = net.cell_off[s], net.cell_off[s + 1]
        assert rel_linf(qg[:, c0:c1], qr[:, c0:c1]) <= T_END, s
        assert rel_linf(vg[:, c0 + s:c1 + s + 1], vr_[:, c0 + s:c1 + s + 1]) <= T_END, s


def test_results_do_not_depend_on_the_tiling(G):
    """Shock tubes (strong Riemann problems next to weak ones in the same
    waves) and a smooth network, 20 steps under every tile order and width:
    the states are bitwise equal, since each lane's solver choices and the
    order in which it takes its results do not depend on the other lanes."""
    tubes = I.tube_network(n_seg=300, seed=5)
    net = network_case(60, seed=3, nmax=400)
    for name, nw, recon, lam in (("tubes", tubes, 1, 10.0), ("network", net, 0, 1e9)):
        ref = None
        for schedule, block in ((1, 64), (2, 64), (2, 128), (3, 256), (1, 256)):
            sim = _gpu_sim(G, G.GRPREC_EULER, 3, nw.n_cells, nw.lengths, nw.q, nw.vl, nw.vr,
                           G.GRPREC_BC_TRANSMISSIVE, schedule=schedule, block=block, recon=recon,
                           nl_lambda_c=lam)
            try:
                print(f"{name} tiling {schedule}/{block}", flush=True)
                steps, _ = sim.run(1e9, 20)
                assert steps == 20
                qg, vg, _, _ = sim.numpy_state()
                t = sim.times()
            finally:
                sim.close()
            if ref is None:
                ref = (qg, vg, t)
            else:
                assert np.array_equal(qg, ref[0]) and np.array_equal(vg, ref[1]), (name, schedule, block)
                assert np.array_equal(t, ref[2])
