#!/usr/bin/env python3
"""Throughput of the GRPrec finite-volume step on one MI355X.

Workload (the headline): a network of 10,000 independent 1D Euler segments
(gamma 1.4, FP64, order 3), cell counts log-uniform in [3, 2000] from a seed,
lengths uniform in [0.01, 1], transmissive ends, smooth initial data
rho = 1 + 0.1 sin(k x), u = 0.5, p = 1 with per-segment k in [1, 8].
A step advances every segment by one of its own time steps.

Forms: "plain" (the single-domain kernel launched once per segment per step),
"batched" (one persistent launch per step over tiles of all segments, HIP
graphs, autotuned schedule) with the PVRS Newton start, and "batched + MLP"
(the learned star-pressure proposal, trained at start-up on the GPU).

Prints one JSON line (see the "roofline" and "cpu_baseline" objects).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 cell-updates/s (Euler, order 3) plain vs batched+MLP-guess; % HBM roofline"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6

# Algorithmic FP64 operations of the order-3 Euler step (add/mul = 1, fma = 2,
# div/sqrt/log2/exp2 = 1 each), counted from the method's arithmetic:
F_CELL = 289     # reconstruction 51, traces 198, flux sums 18, update + S_max 19, dt 3
F_SWEEP = 597    # one predictor sweep: 9 nodal fluxes 81, D.F 162, K^-1 W 162, update/check 192
F_RS = 78        # one Riemann problem without its Newton iterations
F_NEWTON = 32    # one Newton iteration on the star pressure
BYTES_EULER = 96  # read q and V, write q and V: 2 x 2 x 3 x 8 bytes per cell-update
BYTES_ADV = 32


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_digest() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2602_21911_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_record(kernel: str):
    """The committed rocprofv3 counter record of a kernel, if it was taken on
    the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel)
    except Exception:
        return None
    if not rec or rec.get("source_digest") != src_digest():
        return None
    return rec


def traffic_from_profiles(kernel: str, launch_units: float):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources; else None."""
    rec = profile_record(kernel)
    return rec.get("hbm_bytes_per_launch") if rec else None


def timed_run(sim, steps: int, torch):
    """grprec_run over exactly `steps` steps, timed with events on the stream
    the kernels run on."""
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    done, _ = sim.run(1e9, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert done == steps, (done, steps)
    return e0.elapsed_time(e1) / 1e3, wall


def make_network(G, net, guess, params, schedule, block=0, gate=0.1):
    return G.Simulation(G.GRPREC_EULER, 3, net.n_cells, net.lengths, net.q, net.vl, net.vr,
                        bc=G.GRPREC_BC_TRANSMISSIVE, guess=guess, mlp_params=params,
                        schedule=schedule, block=block, mlp_gate=gate)


def flops_per_launch(G, net, guess, params, schedule, block, gate=0.1):
    """Operation count of one step from the solver's own iteration counters
    (an untimed run with counters on)."""
    sim = make_network(G, net, guess, params, schedule, block, gate)
    try:
        G.grprec_enable_stats(sim.h, True)
        k = 3
        sim.run(1e9, k)
        st = G.grprec_get_stats(sim.h)
    finally:
        sim.close()
    cells = float(net.n_cells.sum())
    halo = st["cells_predicted"] / (k * cells)           # redundant halo predictions
    sweeps = st["picard_sweeps"] / k / halo
    rs = st["rs_calls"] / k
    newton = st["newton_iters"] / k
    flops = F_CELL * cells + F_SWEEP * sweeps + F_RS * rs + F_NEWTON * newton
    return flops, {"sweeps_per_cell": sweeps / cells, "rs_per_cell": rs / cells,
                   "newton_per_rs": newton / max(rs, 1.0), "halo_factor": halo,
                   "mlp_guesses_per_step": st["mlp_guesses"] / k}


def bench_network(args, G, torch, params, gate=0.1):
    from paper_2602_21911_amd import inputs as I
    net = I.network(n_seg=args.segments, seed=I.SEED_NETWORK)
    cells = int(net.n_cells.sum())
    out = {"cells": cells}
    # batched + learned guess (headline), autotuned schedule
    sim = make_network(G, net, G.GRPREC_GUESS_MLP if params is not None else G.GRPREC_GUESS_PVRS,
                       params, G.GRPREC_SCHED_AUTO, 0, gate)
    try:
        sched, block = G.grprec_get_schedule(sim.h)
        sim.run(1e9, args.warmup)
        sec, wall = timed_run(sim, args.steps, torch)
        out["batched_mlp"] = {"rate": cells * args.steps / sec, "ms_per_step": 1e3 * sec / args.steps,
                              "wall_s": wall, "schedule": sched, "block": block}
    finally:
        sim.close()
    # batched, PVRS start
    sim = make_network(G, net, G.GRPREC_GUESS_PVRS, None, sched, block)
    try:
        sim.run(1e9, args.warmup)
        sec, wall = timed_run(sim, args.steps, torch)
        out["batched_pvrs"] = {"rate": cells * args.steps / sec, "ms_per_step": 1e3 * sec / args.steps}
    finally:
        sim.close()
    # plain: one launch per segment per step
    sim = make_network(G, net, G.GRPREC_GUESS_PVRS, None, G.GRPREC_SCHED_PER_DOMAIN, 64)
    try:
        sim.run(1e9, 1)
        sec, wall = timed_run(sim, args.plain_steps, torch)
        out["plain"] = {"rate": cells * args.plain_steps / sec,
                        "ms_per_step": 1e3 * sec / args.plain_steps, "launches_per_step": args.segments}
    finally:
        sim.close()
    fl, it = flops_per_launch(G, net, G.GRPREC_GUESS_MLP if params is not None else G.GRPREC_GUESS_PVRS,
                              params, sched, block, gate)
    out["flops_per_step"] = fl
    out["iterations"] = it
    out["batched_mlp"]["learned_starts_per_step"] = it["mlp_guesses_per_step"]
    out["batched_mlp"]["learned_start_note"] = (
        "the learned start is taken only at interfaces whose first Riemann problem jumps by more than"
        " the gate (%.3g); on this smooth network that happens %g times per step, so this form runs the"
        " PVRS start's arithmetic; the tube network measures what the learned start gains"
        % (gate, it["mlp_guesses_per_step"]))
    out["net"] = net
    return out


LAMBDA_C_PRINTED = 1e9   # GRPrecNL lambda_C as Sec. 3.3 prints it
LAMBDA_C_TABLE = 10.0    # the value that reproduces the printed GRPrecNL advection table


def bench_advection(G, torch, n, order=3, steps=200, warmup=20, recon=0, nl_lambda_c=LAMBDA_C_PRINTED):
    from paper_2602_21911_amd import inputs as I
    dx, q, vl, vr = I.adv_sin2pi(n)
    sim = G.Simulation(G.GRPREC_ADVECTION, order, [n], [1.0], q, vl, vr, bc=G.GRPREC_BC_PERIODIC,
                       recon=recon, nl_lambda_c=nl_lambda_c)
    try:
        sim.run(1e9, warmup)
        sec, _ = timed_run(sim, steps, torch)
    finally:
        sim.close()
    per = sec / steps
    gbs = BYTES_ADV * n / per / 1e9
    key = "adv_step_order%d_2e25%s" % (order, "_nl" if recon else "")
    traffic = traffic_from_profiles(key, n) if n == 1 << 25 else None
    out = {"cells": n, "order": order, "recon": "GRPrecNL" if recon else "GRPrec", "rate": n / per,
           "ms_per_step": 1e3 * per, "hbm_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS, "bound": "hbm",
           "traffic": traffic}
    if recon:
        out["nl_lambda_c"] = nl_lambda_c
    return out


def advection_lines(G, torch):
    """Advection of sin 2 pi x (periodic, CFL 0.9): GRPrec orders 2-5 at 2^20,
    2^22 and 2^25 cells (the last beyond the 256 MB last-level cache), and
    GRPrecNL orders 3 and 5 at 2^25."""
    out = [bench_advection(G, torch, n, order=o) for o in (2, 3, 4, 5) for n in (1 << 20, 1 << 22, 1 << 25)]
    out += [bench_advection(G, torch, 1 << 25, order=o, recon=1) for o in (3, 5)]
    return out


def _golden(name):
    """Rows of a committed table of the paper's printed values."""
    return np.loadtxt(os.path.join(ROOT, "tests", "golden", name), comments="#", ndmin=2)


def bench_paper_tables(G, torch, I):
    """The runs of the paper's two FV+GRPrec convergence tables (Sec. 4.2.3:
    advection of sin^4(pi x) on periodic [-1,1], N = 16..256; Sec. 4.3.1:
    Euler density wave rho = 1 + 0.2 sin 2 pi x, u = 1, p = 2 on periodic
    [0,1], N = 40..640; orders 2-5, C_CFL 0.9, t_out 4) run whole on the GPU
    (graph-captured), with their errors against the exact cell averages, next
    to the errors and CPU seconds the paper prints (its hardware is not
    stated; its Euler magnitudes do not fit the stated unit domain, so only
    their rates are comparable)."""
    err = {0: {}, 1: {}}
    for sysid, name in ((0, "paper_advection_grprec.txt"), (1, "paper_euler_grprec.txt")):
        for r in _golden(name):
            err[sysid][(int(r[0]), int(r[1]))] = (float(r[2]), float(r[3]))
    out = {"advection": [], "euler": [],
           "note": "gpu_s: whole run on the GPU (grprec_run, HIP events); paper_cpu_s: the paper's"
                   " printed CPU seconds for the same run, hardware not stated"}
    for sysid, order, n, cpu_s in _golden("paper_cpu_seconds.txt"):
        sysid, order, n = int(sysid), int(order), int(n)
        if sysid == 0:
            dx, q, vl, vr = I.adv_sin4(n)
            sim = G.Simulation(G.GRPREC_ADVECTION, order, [n], [2.0], q, vl, vr, bc=G.GRPREC_BC_PERIODIC)
        else:
            dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=2.0)
            sim = G.Simulation(G.GRPREC_EULER, order, [n], [1.0], q, vl, vr, bc=G.GRPREC_BC_PERIODIC)
        try:
            stream = torch.cuda.current_stream()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            steps, _ = sim.run(4.0)
            e1.record(stream)
            torch.cuda.synchronize()
            gpu_s = e0.elapsed_time(e1) / 1e3
            qg, _, t, _ = sim.numpy_state()
        finally:
            sim.close()
        exact = I.adv_sin4_exact_avg(n, 4.0) if sysid == 0 else I.euler_density_wave_exact_rho(n, 4.0)
        e = np.abs(qg[0] - exact)
        pl, p1 = err[sysid][(order, n)]
        out["advection" if sysid == 0 else "euler"].append(
            {"order": order, "cells": n, "steps": int(steps), "t": t, "linf": float(e.max()),
             "l1": float(dx * e.sum()), "gpu_s": gpu_s, "paper_linf": pl, "paper_l1": p1,
             "paper_cpu_s": float(cpu_s)})
    return out


def bench_bulk_riemann(G, torch, I, P, gate, n=1_000_000, reps=10):
    """The bulk Riemann solver (one problem per lane) on n held-out random
    tube problems: PVRS start, learned start for every problem, learned start
    above the gate; time per call (HIP events, mean of reps) and the mean
    Newton iterations."""
    WL, WR = I.random_tube_states(I.SEED_TUBES_HELDOUT, n)
    wl = torch.from_numpy(WL).cuda()
    wr = torch.from_numpy(WR).cuda()
    ps = torch.empty(n, dtype=torch.float64, device="cuda")
    it = torch.empty(n, dtype=torch.int32, device="cuda")
    out = {"problems": n}
    for name, guess, g in (("pvrs", G.GRPREC_GUESS_PVRS, -1.0), ("learned_all", G.GRPREC_GUESS_MLP, -1.0),
                           ("learned_above_gate", G.GRPREC_GUESS_MLP, gate)):
        params = P if guess == G.GRPREC_GUESS_MLP else None
        for _ in range(2):
            G.grprec_riemann_batch(wl, wr, guess=guess, mlp_params=params, gate=g, pstar=ps, iters=it)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            G.grprec_riemann_batch(wl, wr, guess=guess, mlp_params=params, gate=g, pstar=ps, iters=it)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        k = it.cpu().numpy()
        out[name] = {"ms_per_call": ms, "problems_per_s": n / (ms / 1e3),
                     "newton_mean": float(k[k > 0].mean())}
    return out


def bench_small_case(G, torch, I, cfl=0.9):
    """Advection of sin 2 pi x on 100 periodic cells, order 3, to t = 1 (112
    steps): a latency-bound case, timed as whole runs through grprec_run
    (graph-captured chunks of steps) and as one grprec_step call per step
    (no host synchronisation between steps)."""
    import oracle
    n = 100
    dx, q, vl, vr = I.adv_sin2pi(n)
    out = {"workload": "advection sin 2 pi x, 100 periodic cells, order 3, CFL %g, t_end 1" % cfl}
    for form in ("graph", "eager"):
        best = None
        for _rep in range(5):
            sim = G.Simulation(G.GRPREC_ADVECTION, 3, [n], [1.0], q, vl, vr, bc=G.GRPREC_BC_PERIODIC,
                               cfl=cfl)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if form == "graph":
                    steps, _ = sim.run(1.0)
                else:
                    for _k in range(steps):
                        sim.step(1.0)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                assert sim.state()[3] == 1.0
            finally:
                sim.close()
            best = sec if best is None else min(best, sec)
        out[form] = {"steps": steps, "us_per_step": 1e6 * best / steps, "seconds": best}
    c = oracle.cfg(oracle.ADVECTION, 3, cfl=cfl)
    v = oracle.init_interfaces(c, vl, vr)
    t0 = time.perf_counter()
    _q, _v, _t, k, _st = oracle.run(c, dx, q, v, 0.0, 1.0)
    out["oracle_us_per_step"] = 1e6 * (time.perf_counter() - t0) / k
    return out


def _network_form(G, torch, net, guess, params, schedule, block, steps, warmup, recon, datum=0,
                  nl_lambda_c=LAMBDA_C_PRINTED, gate=0.1):
    """Rate of one batched form, and its solver counters over the same steps
    (counted in a second, untimed run)."""
    cells = int(net.n_cells.sum())
    kw = dict(bc=G.GRPREC_BC_TRANSMISSIVE, guess=guess, mlp_params=params, schedule=schedule,
              block=block, recon=recon, datum=datum, nl_lambda_c=nl_lambda_c, mlp_gate=gate)
    sim = G.Simulation(G.GRPREC_EULER, 3, net.n_cells, net.lengths, net.q, net.vl, net.vr, **kw)
    try:
        sched, blk = G.grprec_get_schedule(sim.h)
        sim.run(1e9, warmup)
        sec, _ = timed_run(sim, steps, torch)
    finally:
        sim.close()
    kw.update(schedule=sched, block=blk)
    sim = G.Simulation(G.GRPREC_EULER, 3, net.n_cells, net.lengths, net.q, net.vl, net.vr, **kw)
    try:
        G.grprec_enable_stats(sim.h, True)
        sim.run(1e9, warmup + steps)
        st = G.grprec_get_stats(sim.h)
    finally:
        sim.close()
    rs = max(1, st["rs_calls"])
    k = warmup + steps
    out = {"rate": cells * steps / sec, "ms_per_step": 1e3 * sec / steps, "schedule": sched,
           "block": blk, "newton_per_rs": st["newton_iters"] / rs,
           "mlp_starts_per_rs": st["mlp_guesses"] / rs,
           "newton_iters_per_step": st["newton_iters"] / k, "learned_starts_per_step": st["mlp_guesses"] / k,
           "sweeps_per_cell": st["picard_sweeps"] / max(1, st["cells_predicted"])}
    if recon:
        out["nl_lambda_c"] = nl_lambda_c
    return out


def bench_tube_network(G, torch, params, steps=100, warmup=10, gate=0.1):
    """10^4 shock tubes (GRPrecNL, order 3): the discontinuous workload on
    which the learned Newton start can matter; PVRS vs learned start, same
    schedule.  GRPrecNL runs with lambda_C = 10: the tube family was chosen as
    the strength GRPrecNL carries with it; with the printed 1e9 GRPrecNL is
    GRPrec on most cells and these tubes fail (non-physical states)."""
    from paper_2602_21911_amd import inputs as I
    net = I.tube_network(n_seg=10000, seed=I.SEED_TUBE_NETWORK)
    lam = LAMBDA_C_TABLE
    out = {"workload": "10000 shock tubes, GRPrecNL order 3 (lambda_C %g), cells uniform [20,200) (seed"
                       " %d), rho and p ratios up to 2, |u| <= 0.1, transmissive" % (lam, I.SEED_TUBE_NETWORK),
           "cells": int(net.n_cells.sum()), "nl_lambda_c": lam}
    first = G.GRPREC_GUESS_MLP if params is not None else G.GRPREC_GUESS_PVRS
    a = _network_form(G, torch, net, first, params, G.GRPREC_SCHED_AUTO, 0, steps, warmup, 1,
                      nl_lambda_c=lam, gate=gate)
    a["mlp_gate"] = gate
    out["batched_mlp" if params is not None else "batched_pvrs"] = a
    if params is not None:
        out["batched_pvrs"] = _network_form(G, torch, net, G.GRPREC_GUESS_PVRS, None, a["schedule"],
                                            a["block"], steps, warmup, 1, nl_lambda_c=lam)
    out["batched_pvrs_trrs_datum"] = _network_form(G, torch, net, G.GRPREC_GUESS_PVRS, None,
                                                   a["schedule"], a["block"], steps, warmup, 1,
                                                   G.GRPREC_DATUM_TRRS, nl_lambda_c=lam)
    if params is not None:
        # Newton iterations the learned start saves per step (same steps, same
        # schedule), and how many learned starts were taken
        out["newton_iters_saved_per_step"] = (out["batched_pvrs"]["newton_iters_per_step"]
                                              - a["newton_iters_per_step"])
        out["learned_starts_per_step"] = a["learned_starts_per_step"]
    return out


def bench_network_variants(G, torch, steps=100, warmup=10):
    """The headline network with GRPrecNL instead of GRPrec, and with the
    two-rarefaction datum instead of the exact one (PVRS start)."""
    from paper_2602_21911_amd import inputs as I
    net = I.network(n_seg=10000, seed=I.SEED_NETWORK)
    out = {"cells": int(net.n_cells.sum())}
    out["grprecnl"] = _network_form(G, torch, net, G.GRPREC_GUESS_PVRS, None, G.GRPREC_SCHED_AUTO, 0,
                                    steps, warmup, 1, nl_lambda_c=LAMBDA_C_PRINTED)
    out["grprecnl_lambda_c_10"] = _network_form(G, torch, net, G.GRPREC_GUESS_PVRS, None,
                                                G.GRPREC_SCHED_AUTO, 0, steps, warmup, 1,
                                                nl_lambda_c=LAMBDA_C_TABLE)
    out["trrs_datum"] = _network_form(G, torch, net, G.GRPREC_GUESS_PVRS, None, G.GRPREC_SCHED_AUTO, 0,
                                      steps, warmup, 0, G.GRPREC_DATUM_TRRS)
    return out


def bench_euler_single(G, torch, n, order=3, steps=50, warmup=5):
    from paper_2602_21911_amd import inputs as I
    dx, q, vl, vr = I.euler_density_wave(n, amp=0.2, u=1.0, p=1.0)
    sim = G.Simulation(G.GRPREC_EULER, order, [n], [1.0], q, vl, vr, bc=G.GRPREC_BC_PERIODIC,
                       schedule=G.GRPREC_SCHED_AUTO)
    try:
        sim.run(1e9, warmup)
        sec, _ = timed_run(sim, steps, torch)
    finally:
        sim.close()
    per = sec / steps
    gbs = BYTES_EULER * n / per / 1e9
    return {"cells": n, "order": order, "rate": n / per, "ms_per_step": 1e3 * per, "hbm_gbs": gbs,
            "hbm_frac": gbs / PEAK_HBM_GBS}


def cpu_baseline(net, steps: int):
    """The oracle (serial C, one core) on the same network for `steps` steps."""
    import oracle
    c = oracle.cfg(oracle.EULER, 3, bc=oracle.TRANSMISSIVE)
    v0 = oracle.init_interfaces(c, net.vl, net.vr)
    S = len(net.n_cells)
    t0 = time.perf_counter()
    oracle.run_segments(c, net.cell_off, net.dx, net.q, v0, np.zeros(S), 1e9, steps)
    sec = time.perf_counter() - t0
    cells = float(net.n_cells.sum())
    return {"value": cells * steps / sec, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"all {S} segments ({int(cells)} cells), {steps} steps each, serial C oracle",
            "seconds": sec}


def segment_groups(net, v, n_groups: int):
    """Contiguous groups of a network's segments as independent networks:
    (cell offsets from 0, dx, cell averages, interface values), the interface
    arrays holding one value more per segment than the cell arrays."""
    S = len(net.n_cells)
    bounds = np.linspace(0, S, n_groups + 1).astype(int)
    jobs = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        c0, c1 = int(net.cell_off[a]), int(net.cell_off[b])
        jobs.append((net.cell_off[a:b + 1] - c0, net.dx[a:b], net.q[:, c0:c1], v[:, c0 + a:c1 + b]))
    return bounds, jobs


def cpu_all_cores(net, steps: int):
    """Context figure: the same serial oracle run on contiguous groups of
    segments in host threads (the C call releases the interpreter lock)."""
    import concurrent.futures as cf
    import oracle
    c = oracle.cfg(oracle.EULER, 3, bc=oracle.TRANSMISSIVE)
    v0 = oracle.init_interfaces(c, net.vl, net.vr)
    S = len(net.n_cells)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    _, jobs = segment_groups(net, v0, 4 * threads)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda j: oracle.run_segments(c, j[0], j[1], j[2], j[3], np.zeros(len(j[1])), 1e9, steps), jobs))
    sec = time.perf_counter() - t0
    cells = float(net.n_cells.sum())
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": cells * steps / sec, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"all {S} segments, {steps} steps each, {len(jobs)} groups of segments over"
                      f" {threads} threads", "seconds": sec, "cpu_model": model,
            "visible_cpus": len(os.sched_getaffinity(0))}


def counters_run(G, torch, I):
    """Short fixed workload for rocprofv3 --pmc passes: 3 network steps (flat
    tiles, 64-wide blocks), 3 advection steps on 2^25 cells for GRPrec orders
    2-5 and GRPrecNL orders 3 and 5, and a 256 MiB device copy used to
    calibrate the byte counters."""
    net = I.network(n_seg=10000, seed=I.SEED_NETWORK)
    sim = make_network(G, net, G.GRPREC_GUESS_PVRS, None, G.GRPREC_SCHED_FLAT_TILES, 64)
    try:
        for _ in range(3):
            sim.step(1e9)
        torch.cuda.synchronize()
    finally:
        sim.close()
    dx, q, vl, vr = I.adv_sin2pi(1 << 25)
    for order, recon in ((2, 0), (3, 0), (4, 0), (5, 0), (3, 1), (5, 1)):
        sim = G.Simulation(G.GRPREC_ADVECTION, order, [1 << 25], [1.0], q, vl, vr,
                           bc=G.GRPREC_BC_PERIODIC, recon=recon)
        try:
            for _ in range(3):
                sim.step(1e9)
            torch.cuda.synchronize()
        finally:
            sim.close()
    a = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counters_run": "done", "network_cells": int(net.n_cells.sum()),
                      "advection_cells": 1 << 25, "copy_bytes": a.numel() * 8}), flush=True)


def trace_run(args, G, torch, I, learn):
    """The headline form (batched, learned start) on a fixed schedule: W warm-up
    and K timed steps, so a kernel trace's launches of the step kernel are
    exactly these steps."""
    ds = learn.build_dataset(args.train_n)
    P, _ = learn.train(ds, epochs=args.epochs, lr=args.lr, lr_final=1e-5)
    gate, _ = learn.calibrate_gate(P, *I.random_tube_states(I.SEED_TUBES_GATE, 100_000))
    net = I.network(n_seg=args.segments, seed=I.SEED_NETWORK)
    cells = int(net.n_cells.sum())
    sim = make_network(G, net, G.GRPREC_GUESS_MLP, P, args.schedule, args.block, gate)
    try:
        sim.run(1e9, args.warmup)
        sec, _ = timed_run(sim, args.steps, torch)
    finally:
        sim.close()
    print(json.dumps({"trace_run": "done", "cells": cells, "schedule": args.schedule, "block": args.block,
                      "warmup": args.warmup, "steps": args.steps, "ms_per_step": 1e3 * sec / args.steps,
                      "rate": cells * args.steps / sec}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--segments", type=int, default=10000)
    ap.add_argument("--train-n", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=3e-3, help="Adam step size, falling along a half"
                    " cosine to 1e-5 over the training run")
    ap.add_argument("--no-mlp", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=4,
                    help="network steps the oracle runs for cpu_baseline (about 11 s on one core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip advection / single-domain lines")
    ap.add_argument("--only", choices=["all", "advection", "counters", "trace", "paper"], default="all",
                    help="advection: only the advection lines; paper: only the runs of the paper's"
                         " convergence tables; counters: a short fixed run for"
                         " hardware-counter passes (network, advection 2^25, a 256 MB copy);"
                         " trace: the headline network form on a fixed schedule (--schedule,"
                         " --block; no autotuning), W + K steps, for a kernel trace whose every"
                         " launch of the step kernel is a warm-up or timed step")
    ap.add_argument("--schedule", type=int, default=2, help="tile schedule of --only trace")
    ap.add_argument("--block", type=int, default=64, help="workgroup size of --only trace")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(independent segments would shard across GPUs with no communication).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_21911_amd import grprec as G
    from paper_2602_21911_amd import inputs as I
    from paper_2602_21911_amd import learn
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    G.lib()
    if args.only == "advection":
        out = advection_lines(G, torch)
        print(json.dumps({"advection": out}), flush=True)
        return
    if args.only == "paper":
        print(json.dumps({"paper_tables": bench_paper_tables(G, torch, I)}), flush=True)
        return
    if args.only == "counters":
        counters_run(G, torch, I)
        return
    if args.only == "trace":
        trace_run(args, G, torch, I, learn)
        return

    params = None
    mlp = None
    gate = 0.1
    if not args.no_mlp:
        t0 = time.perf_counter()
        ds = learn.build_dataset(args.train_n)
        P, hist = learn.train(ds, epochs=args.epochs, lr=args.lr, lr_final=1e-5)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        WL, WR = I.random_tube_states(I.SEED_TUBES_HELDOUT, 100_000)
        ev = learn.evaluate(P, torch.from_numpy(WL).cuda(), torch.from_numpy(WR).cuda())
        # the step's gate: chosen on its own seeded set of random problems
        gate, cal = learn.calibrate_gate(P, *I.random_tube_states(I.SEED_TUBES_GATE, 100_000))
        params = P
        mlp = {"train_samples": int(ds.x.shape[0]), "vacuum_dropped": ds.n_vacuum,
               "epochs": args.epochs, "lr": args.lr, "lr_final": 1e-5, "final_loss": hist[-1],
               "train_s": t_train, "heldout": ev, "gate_calibration": cal}
        log(f"mlp trained in {t_train:.1f}s, loss {hist[-1]:.3e}, held-out {ev}, gate {cal}")

    res = bench_network(args, G, torch, params, gate)
    net = res.pop("net")
    cells = res["cells"]
    head = res["batched_mlp"]
    sec_per_step = head["ms_per_step"] / 1e3
    flops = res["flops_per_step"]
    bytes_step = BYTES_EULER * cells + 48.0 * len(net.n_cells)
    achieved_tf = flops / sec_per_step / 1e12
    traffic = traffic_from_profiles("euler_step_order3", cells)
    # FP64 flops the kernel executes (SQ_INSTS_VALU_FLOPS_FP64 of the committed
    # counter runs, same sources), over this run's launch time
    rec = profile_record("euler_step_order3") or {}
    counted = rec.get("fp64_flops_per_launch_counted")
    roofline = {
        "kernel": "euler_step<M=2> (fused reconstruct + predictor + Riemann + update)",
        "bound": "alu", "achieved": achieved_tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
        "frac": achieved_tf / PEAK_FP64_TFLOPS, "traffic": traffic,
        "flops_per_launch": flops, "launch_ms": head["ms_per_step"],
        "hbm_algorithmic_bytes_per_launch": bytes_step,
        "hbm_gbs": bytes_step / sec_per_step / 1e9,
        "hbm_frac": bytes_step / sec_per_step / 1e9 / PEAK_HBM_GBS,
        "iterations": res["iterations"],
        "counted_fp64_flops_per_launch": counted,
        "counted_tflops": counted / sec_per_step / 1e12 if counted else None,
        "counted_frac": counted / sec_per_step / 1e12 / PEAK_FP64_TFLOPS if counted else None,
    }
    line = {
        "metric": METRIC, "value": head["rate"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "network of %d independent Euler segments, order 3, cells log-uniform"
                               " [3,2000] (seed %d), transmissive, smooth data"
                               % (args.segments, I.SEED_NETWORK),
                   "segments": args.segments, "total_cells": cells, "order": 3, "gamma": 1.4,
                   "cfl": 0.9, "schedule": head["schedule"], "block": head["block"]},
        "forms": {"plain": res["plain"], "batched_pvrs": res["batched_pvrs"], "batched_mlp": head},
        "roofline": roofline,
    }
    if mlp is not None:
        line["mlp"] = mlp
    if not args.no_extras:
        line["advection"] = advection_lines(G, torch)
        line["euler_single_domain"] = [bench_euler_single(G, torch, n, order=o)
                                       for o in (2, 3, 4) for n in (1 << 20, 1 << 22)]
        line["network_variants"] = bench_network_variants(G, torch)
        line["tube_network"] = bench_tube_network(G, torch, params, gate=gate)
        line["small_case"] = bench_small_case(G, torch, I)
        line["paper_tables"] = bench_paper_tables(G, torch, I)
        if params is not None:
            line["mlp"]["bulk_riemann"] = bench_bulk_riemann(G, torch, I, params, gate)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(net, args.cpu_steps)
        line["cpu_all_cores"] = cpu_all_cores(net, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
