"""bench.py's contract on a machine without a GPU: one GPU only (a request
for more exits with a message), the source digest that ties committed HBM
traffic figures to the kernel sources, and the all-cores oracle figure's
split of the network into segment groups (checked against one serial run)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle  # noqa: E402
from paper_2602_21911_amd import inputs as I  # noqa: E402


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_traffic_figures_follow_the_kernel_sources():
    d = bench.src_digest()
    assert len(d) == 16 and d == bench.src_digest()
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for kernel, r in rec.items():
        got = bench.traffic_from_profiles(kernel, 1.0)
        if r["source_digest"] == d:
            assert got == r["hbm_bytes_per_launch"] and got > 0
        else:
            assert got is None


def test_segment_groups_reproduce_the_serial_oracle():
    net = I.network(n_seg=37, seed=11)
    c = oracle.cfg(oracle.EULER, 3, bc=oracle.TRANSMISSIVE)
    v0 = oracle.init_interfaces(c, net.vl, net.vr)
    S = len(net.n_cells)
    qf, vf, tf, _ = oracle.run_segments(c, net.cell_off, net.dx, net.q, v0, np.zeros(S), 1e9, 2)
    bounds, jobs = bench.segment_groups(net, v0, 5)
    assert bounds[0] == 0 and bounds[-1] == S and len(jobs) == 5
    for (a, b), (off, dx, q, v) in zip(zip(bounds[:-1], bounds[1:]), jobs):
        c0, c1 = int(net.cell_off[a]), int(net.cell_off[b])
        qs, vs, ts, _ = oracle.run_segments(c, off, dx, q, v, np.zeros(b - a), 1e9, 2)
        assert np.array_equal(qs, qf[:, c0:c1])
        assert np.array_equal(vs, vf[:, c0 + a:c1 + b])
        assert np.array_equal(ts, tf[a:b])


def test_paper_cpu_table_matches_the_error_tables():
    """The CPU-seconds table covers exactly the runs of the two printed error
    tables (orders 2-5; advection N = 16..256, Euler N = 40..640), and the
    bench reads all three."""
    import bench
    cpu = bench._golden("paper_cpu_seconds.txt")
    assert cpu.shape == (40, 4) and np.all(cpu[:, 3] > 0)
    for sysid, name, cells in ((0, "paper_advection_grprec.txt", (16, 32, 64, 128, 256)),
                               (1, "paper_euler_grprec.txt", (40, 80, 160, 320, 640))):
        err = bench._golden(name)
        keys = {(int(r[0]), int(r[1])) for r in err}
        assert keys == {(o, n) for o in (2, 3, 4, 5) for n in cells}
        assert {(int(r[1]), int(r[2])) for r in cpu if int(r[0]) == sysid} == keys
