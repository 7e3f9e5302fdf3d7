"""GPU parity of the learned-guess kernels against the float64 reference, and
what the trained network gains over the PVRS start."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2602_21911_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_21911_amd import grprec
    grprec.lib()
    return grprec


def _params(seed=0):
    rng = np.random.default_rng(seed)
    P = rng.normal(scale=0.3, size=1325)
    P[1313:1319] = rng.normal(scale=0.1, size=6)
    P[1319:1325] = rng.uniform(0.5, 2.0, size=6)
    return P.astype(np.float32)


def test_features_match_reference(G):
    WL, WR = I.random_tube_states(5, 3000)
    x, _ = G.grprec_mlp_features(torch.from_numpy(WL).cuda(), torch.from_numpy(WR).cuda())
    xr, _ = mlp.features(WL, WR)
    np.testing.assert_allclose(x.cpu().numpy(), xr, rtol=2e-6, atol=2e-6)


def test_forward_matches_reference(G):
    P = _params()
    x = np.random.default_rng(1).normal(size=(5000, 6)).astype(np.float32)
    y = G.grprec_mlp_forward(torch.from_numpy(P).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
    yr = mlp.forward(P.astype(np.float64), x.astype(np.float64))
    assert np.abs(y - yr).max() <= 1e-5 * (1 + np.abs(yr).max())


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4096])
def test_loss_grad_matches_reference(G, n):
    P = _params(2)
    rng = np.random.default_rng(n)
    x = rng.normal(size=(n, 6)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    Pd = torch.from_numpy(P).cuda()
    grad = torch.zeros(G.GRPREC_MLP_WEIGHTS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    work = torch.zeros(G.grprec_mlp_work_bytes(n), dtype=torch.uint8, device="cuda")
    G.grprec_mlp_loss_grad(Pd, torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), grad, loss, work)
    gr = mlp.loss_grad(P.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    lr = mlp.loss(P.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    g = grad.cpu().numpy()
    assert abs(loss.item() - lr) <= 1e-4 * (1 + lr)
    assert np.abs(g - gr).max() <= 1e-4 * (1 + np.abs(gr).max())


def test_adam_matches_reference(G):
    P = _params(3)
    g = np.random.default_rng(4).normal(size=1313).astype(np.float32)
    Pd = torch.from_numpy(P.copy()).cuda()
    gd = torch.from_numpy(g).cuda()
    m = torch.zeros(1313, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    Pr, mr, vr = P.astype(np.float64), np.zeros(1313), np.zeros(1313)
    for step in (1, 2, 3):
        G.grprec_mlp_adam(Pd, gd, m, v, step, lr=1e-3)
        Pr, mr, vr = mlp.adam(Pr, g.astype(np.float64), mr, vr, step, lr=1e-3)
    np.testing.assert_allclose(Pd.cpu().numpy(), Pr, rtol=1e-5, atol=1e-6)


def test_training_gains_over_pvrs(G):
    """Trained on tube jumps + harvested states, the proposal needs fewer Newton
    iterations than PVRS on held-out random tubes, and Newton from it reaches
    the same star pressure (1e-11 relative)."""
    from paper_2602_21911_amd import learn
    ds = learn.build_dataset(200_000)
    P, hist = learn.train(ds, epochs=8)
    assert hist[-1] < hist[0]
    WL, WR = I.random_tube_states(I.SEED_TUBES_HELDOUT, 50_000)
    ev = learn.evaluate(P, torch.from_numpy(WL).cuda(), torch.from_numpy(WR).cuda())
    assert ev["mlp_mean"] < ev["pvrs_mean"], ev
    assert ev["max_rel_pstar_diff"] <= 1e-11, ev
    assert 0.0 <= ev["fallback_rate"] < 1e-3, ev
    # the gate chosen on a separate set: the library's solver, gated by the
    # device's own jump test, spends the Newton iterations the host's split
    # predicted, no more than either start alone
    GL, GR = I.random_tube_states(I.SEED_TUBES_GATE, 20_000)
    gate, cal = learn.calibrate_gate(P, GL, GR)
    _, it = G.grprec_riemann_batch(torch.from_numpy(GL).cuda(), torch.from_numpy(GR).cuda(),
                                   guess=G.GRPREC_GUESS_MLP, mlp_params=P, gate=gate)
    it = it.cpu().numpy()
    got = float(it[it > 0].sum())
    assert cal["problems"] == int((it > 0).sum())
    assert got == cal["newton_iters"], (got, cal)
    assert got <= min(cal["newton_iters_all_pvrs"], cal["newton_iters_all_learned"]), cal
    # the learned start leaves every star pressure at the oracle's value
    ps, it = G.grprec_riemann_batch(torch.from_numpy(WL[:500]).cuda(), torch.from_numpy(WR[:500]).cuda(),
                                    guess=G.GRPREC_GUESS_MLP, mlp_params=P)
    ps = ps.cpu().numpy()
    it = it.cpu().numpy()
    for k in range(500):
        rc, pr, _ = oracle.riemann_rc(1.4, WL[k], WR[k])
        if rc == oracle.OK:
            assert abs(ps[k] - pr) <= 1e-11 * pr
        else:
            assert it[k] == rc


def test_mlp_guess_step_parity(G):
    """A network run with the learned start equals the oracle (PVRS start)."""
    from ._cases import network_case, rel_linf
    net = network_case(30, seed=9, nmax=300)
    P = torch.from_numpy(_params(5)).cuda()
    c = oracle.cfg(oracle.EULER, 3, bc=oracle.TRANSMISSIVE)
    v0 = oracle.init_interfaces(c, net.vl, net.vr)
    S = len(net.n_cells)
    qr, vr_, tr, _ = oracle.run_segments(c, net.cell_off, net.dx, net.q, v0, np.zeros(S), 1e9, 4)
    sim = G.Simulation(G.GRPREC_EULER, 3, net.n_cells, net.lengths, net.q, net.vl, net.vr,
                       bc=G.GRPREC_BC_TRANSMISSIVE, guess=G.GRPREC_GUESS_MLP, mlp_params=P,
                       mlp_gate=-1.0, schedule=G.GRPREC_SCHED_PACKED, block=128)
    try:
        G.grprec_enable_stats(sim.h, True)
        sim.run(1e9, 4)
        st = G.grprec_get_stats(sim.h)
        qg, vg, _, _ = sim.numpy_state()
    finally:
        sim.close()
    assert st["mlp_guesses"] > 0
    assert rel_linf(qg, qr) <= 1e-10 and rel_linf(vg, vr_) <= 1e-10
