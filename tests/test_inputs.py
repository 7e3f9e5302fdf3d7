"""The seeded input generators: shapes, determinism and the structure each
workload is meant to have."""
import numpy as np

from paper_2602_21911_amd import inputs as I


def test_tube_network_structure():
    a = I.tube_network(n_seg=50)
    b = I.tube_network(n_seg=50)
    np.testing.assert_array_equal(a.q, b.q)
    S = len(a.n_cells)
    assert a.q.shape == (3, int(a.n_cells.sum()))
    assert a.vl.shape == a.vr.shape == (3, int(a.n_cells.sum()) + S)
    assert np.all((a.n_cells >= 20) & (a.n_cells < 200))
    for s in range(S):
        n, c0 = int(a.n_cells[s]), int(a.cell_off[s])
        i0, j = c0 + s, n // 2
        q = a.q[:, c0:c0 + n]
        # two constant states with the jump at interface j
        assert np.all(q[:, :j] == q[:, :1]) and np.all(q[:, j:] == q[:, -1:])
        vl, vr = a.vl[:, i0:i0 + n + 1], a.vr[:, i0:i0 + n + 1]
        np.testing.assert_array_equal(vl[:, j], q[:, 0])      # left limit at the jump
        np.testing.assert_array_equal(vr[:, j], q[:, -1])     # right limit at the jump
        np.testing.assert_array_equal(vl[:, :j], vr[:, :j])  # continuous elsewhere
        np.testing.assert_array_equal(vl[:, j + 1:], vr[:, j + 1:])
        rho = q[0]
        p = 0.4 * (q[2] - 0.5 * q[1] ** 2 / rho)
        assert 0.5 / 2.0 - 1e-12 <= rho.min() and rho.max() <= 2.0 * 2.0 + 1e-12
        assert p[-1] / p[0] <= 2.0 + 1e-12 and p[0] / p[-1] <= 2.0 + 1e-12
        assert np.abs(q[1] / rho).max() <= 0.1 + 1e-12


def test_network_structure():
    net = I.network(n_seg=200, seed=I.SEED_NETWORK)
    assert np.all((net.n_cells >= 3) & (net.n_cells <= 2000))
    assert net.cell_off[-1] == net.n_cells.sum()
    np.testing.assert_allclose(net.dx * net.n_cells, net.lengths, rtol=1e-15)
    np.testing.assert_array_equal(net.vl, net.vr)  # smooth data: equal one-sided limits
