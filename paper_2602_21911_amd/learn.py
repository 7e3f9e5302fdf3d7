"""Learned star-pressure proposal: data, training and evaluation on the GPU.

Data are Riemann problems the method itself produces:
  * the first interface problems of seeded random shock tubes (left/right
    states rho log-uniform [0.01, 10], u uniform [-3, 3], p log-uniform
    [1e-3, 1e3]) -- the problem solved at the tube's jump;
  * interface problems recorded (``grprec_harvest``) while the library
    advances smooth Euler flows.
Labels are the exact star pressures from the library's own FP64 Newton solver
(``grprec_riemann_batch``, 1e-12 relative); vacuum cases are dropped.
Training runs the library's forward/backward/Adam kernels; torch only holds
the buffers, draws the seeded shuffles and computes the feature normaliser.
The step's gate (the data jump above which an interface's first problem
starts from the network) is then chosen on a separate seeded set of random
problems as the split that minimises their Newton iterations.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import grprec as G
from . import inputs as I


@dataclass
class Dataset:
    wl: "object"      # torch float64 [n,3] primitive left states (device)
    wr: "object"
    pstar: "object"   # torch float64 [n]
    x: "object"       # torch float32 [n,6] raw features
    y: "object"       # torch float32 [n] targets ln(p*/pbar)
    n_vacuum: int
    n_tubes: int
    n_harvested: int


def _harvest_smooth(n_target: int, device: str, seed: int):
    """Interface problems recorded while the method advances smooth flows
    (network segments and an acoustic wave)."""
    import torch
    rows = []
    got = 0
    net = I.network(n_seg=400, seed=seed)
    sim = G.Simulation(G.GRPREC_EULER, 3, net.n_cells, net.lengths, net.q, net.vl, net.vr,
                       bc=G.GRPREC_BC_TRANSMISSIVE, schedule=G.GRPREC_SCHED_PACKED, block=256)
    try:
        cap = max(1, n_target)
        ring = torch.zeros((cap, 7), dtype=torch.float64, device=device)
        count = torch.zeros(1, dtype=torch.int64, device=device)
        G.grprec_harvest(sim.h, ring, count)
        steps = max(1, math.ceil(n_target / max(1, int(net.n_cells.sum()))))
        sim.run(1e9, steps)
        G.grprec_harvest(sim.h, None, None)
        k = min(cap, int(count.item()))
        rows.append(ring[:k])
        got += k
    finally:
        sim.close()
    out = torch.cat(rows, dim=0) if rows else torch.zeros((0, 7), dtype=torch.float64, device=device)
    return out[:n_target]


def build_dataset(n_total: int = 1_000_000, seed: int = I.SEED_TUBES_TRAIN, tube_fraction: float = 0.8,
                  device: str = "cuda", gamma: float = 1.4) -> Dataset:
    import torch
    n_tubes = int(n_total * tube_fraction)
    WL, WR = I.random_tube_states(seed, n_tubes)
    wl = torch.from_numpy(WL).to(device)
    wr = torch.from_numpy(WR).to(device)
    hv = _harvest_smooth(n_total - n_tubes, device, seed)
    n_h = hv.shape[0]
    if n_h:
        wl = torch.cat([wl, hv[:, 0:3].contiguous()], dim=0)
        wr = torch.cat([wr, hv[:, 3:6].contiguous()], dim=0)
    ps, it = G.grprec_riemann_batch(wl, wr, gamma=gamma)
    ok = it > 0
    n_vac = int((it == G.GRPREC_E_VACUUM).sum().item())
    wl, wr, ps = wl[ok].contiguous(), wr[ok].contiguous(), ps[ok].contiguous()
    x, y = G.grprec_mlp_features(wl, wr, ps, gamma=gamma)
    return Dataset(wl, wr, ps, x, y, n_vac, n_tubes, n_h)


def init_params(x, seed: int = 0, device: str = "cuda"):
    """Uniform(+-1/sqrt(fan_in)) weights, zero biases, normaliser from x."""
    import torch
    g = torch.Generator().manual_seed(seed)
    def U(shape, fan):
        b = 1.0 / math.sqrt(fan)
        return (torch.rand(shape, generator=g, dtype=torch.float32) * 2 - 1) * b
    W1, b1 = U((32, 6), 6), torch.zeros(32)
    W2, b2 = U((32, 32), 32), torch.zeros(32)
    W3, b3 = U((32,), 32), torch.zeros(1)
    mean = x.mean(dim=0).float().cpu()
    std = x.std(dim=0).float().cpu().clamp_min(1e-6)
    P = torch.cat([W1.flatten(), b1, W2.flatten(), b2, W3, b3, mean, std]).to(device)
    assert P.numel() == G.GRPREC_MLP_NPARAMS
    return P.contiguous()


def train(ds: Dataset, epochs: int = 20, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          device: str = "cuda", log=None, lr_final: float | None = None):
    """Adam on the mean-squared error of ln(p*/pbar); returns (params, history).
    With lr_final the step size falls from lr to lr_final along a half cosine
    over the run."""
    import torch
    n = ds.x.shape[0]
    if n < batch:
        raise ValueError(f"training set has {n} problems, fewer than one batch of {batch}")
    P = init_params(ds.x, seed, device)
    grad = torch.zeros(G.GRPREC_MLP_WEIGHTS, dtype=torch.float32, device=device)
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    work = torch.zeros(G.grprec_mlp_work_bytes(batch), dtype=torch.uint8, device=device)
    gen = torch.Generator(device=device).manual_seed(seed + 1)
    hist = []
    step = 0
    t0 = time.time()
    total = epochs * max(1, (n - batch) // batch + 1)
    for ep in range(epochs):
        perm = torch.randperm(n, device=device, generator=gen)
        ep_loss = torch.zeros((), dtype=torch.float64, device=device)
        nb = 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            xb = ds.x[idx].contiguous()
            yb = ds.y[idx].contiguous()
            G.grprec_mlp_loss_grad(P, xb, yb, grad, loss, work)
            step += 1
            lr_s = lr
            if lr_final is not None:
                lr_s = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * (step - 1) / total))
            G.grprec_mlp_adam(P, grad, m, v, step, lr_s)
            ep_loss += loss[0].double()
            nb += 1
        hist.append(float(ep_loss.item() / max(1, nb)))
        if log:
            log(f"epoch {ep + 1}/{epochs} loss {hist[-1]:.3e} ({time.time() - t0:.1f}s)")
    return P, hist


def evaluate(P, wl, wr, gamma: float = 1.4, gate: float = -1.0):
    """Newton iterations from PVRS and from the learned start on the same
    problems, and the largest relative star-pressure difference."""
    import torch
    ps0, it0 = G.grprec_riemann_batch(wl, wr, gamma=gamma, guess=G.GRPREC_GUESS_PVRS)
    ps1, it1 = G.grprec_riemann_batch(wl, wr, gamma=gamma, guess=G.GRPREC_GUESS_MLP, mlp_params=P,
                                      gate=gate)
    ok = (it0 > 0) & (it1 > 0)
    a = it0[ok].double()
    b = it1[ok].double()
    # fallback: the solver takes PVRS when pbar exp(y) is not a positive finite
    # double, i.e. y non-finite or outside the range of exp in double precision
    x, _ = G.grprec_mlp_features(wl, wr, gamma=gamma)
    y = G.grprec_mlp_forward(P, x)
    fallback = (~torch.isfinite(y)) | (y > 709.0) | (y < -745.0)
    rel = ((ps1[ok] - ps0[ok]).abs() / ps0[ok]).max().item() if ok.any() else 0.0
    q = lambda t, f: float(torch.quantile(t, f).item())
    return {
        "n": int(ok.sum().item()),
        "failed": int((~ok).sum().item()),
        "pvrs_mean": float(a.mean().item()), "pvrs_p50": q(a, 0.5), "pvrs_p99": q(a, 0.99),
        "mlp_mean": float(b.mean().item()), "mlp_p50": q(b, 0.5), "mlp_p99": q(b, 0.99),
        "max_rel_pstar_diff": rel,
        "fallback_rate": float(fallback.double().mean().item()),
    }


def jump_size(wl, wr, gamma: float = 1.4):
    """The relative data jump the step's gate compares:
    |p_R - p_L| / pbar + |rho_R - rho_L| / rhobar + |u_R - u_L| / cbar with
    pbar, rhobar, cbar the means of the two sides (host float64 [n,3]
    primitive states in, [n] out)."""
    wl = np.asarray(wl, dtype=np.float64)
    wr = np.asarray(wr, dtype=np.float64)
    cl = np.sqrt(gamma * wl[:, 2] / wl[:, 0])
    cr = np.sqrt(gamma * wr[:, 2] / wr[:, 0])
    pbar = 0.5 * (wl[:, 2] + wr[:, 2])
    rbar = 0.5 * (wl[:, 0] + wr[:, 0])
    cbar = 0.5 * (cl + cr)
    return (np.abs(wr[:, 2] - wl[:, 2]) / pbar + np.abs(wr[:, 0] - wl[:, 0]) / rbar
            + np.abs(wr[:, 1] - wl[:, 1]) / cbar)


def best_split(jump, it_pvrs, it_learned):
    """Gate minimising the total Newton iterations when problems whose jump
    exceeds it start from the learned proposal and the others from PVRS.
    Returns (gate, total at that gate, total all PVRS, total all learned).
    The gate lies halfway between the largest jump left to PVRS and the
    smallest one given to the network (0 when every problem goes to the
    network, the largest jump when none does)."""
    j = np.asarray(jump, dtype=np.float64)
    order = np.argsort(j, kind="stable")
    js = j[order]
    a = np.asarray(it_pvrs, dtype=np.float64)[order]
    b = np.asarray(it_learned, dtype=np.float64)[order]
    # total(k): the k smallest jumps from PVRS, the rest from the network
    total = (np.concatenate([[0.0], np.cumsum(a)])
             + np.concatenate([np.cumsum(b[::-1])[::-1], [0.0]]))
    # a threshold cannot separate equal jumps
    cut = np.ones(len(js) + 1, dtype=bool)
    cut[1:-1] = js[1:] > js[:-1]
    k = int(np.argmin(np.where(cut, total, np.inf)))
    if k == 0:
        gate = 0.0
    elif k == len(js):
        gate = float(js[-1])
    else:
        gate = 0.5 * float(js[k - 1] + js[k])
    return gate, float(total[k]), float(total[-1]), float(total[0])


def calibrate_gate(P, wl, wr, gamma: float = 1.4):
    """The step's gate for the trained network P: Newton iterations from PVRS
    and from the learned start on the given problems (host float64 [n,3]
    primitive states; the library's batched solver), split by best_split.
    Returns (gate, summary)."""
    import torch
    dl = torch.from_numpy(np.ascontiguousarray(wl)).cuda()
    dr = torch.from_numpy(np.ascontiguousarray(wr)).cuda()
    _, it0 = G.grprec_riemann_batch(dl, dr, gamma=gamma, guess=G.GRPREC_GUESS_PVRS)
    _, it1 = G.grprec_riemann_batch(dl, dr, gamma=gamma, guess=G.GRPREC_GUESS_MLP, mlp_params=P, gate=-1.0)
    a = it0.cpu().numpy()
    b = it1.cpu().numpy()
    ok = (a > 0) & (b > 0)
    gate, tot, tot_pvrs, tot_learned = best_split(jump_size(wl, wr, gamma)[ok], a[ok], b[ok])
    return gate, {"problems": int(ok.sum()), "gate": gate, "newton_iters": tot,
                  "newton_iters_all_pvrs": tot_pvrs, "newton_iters_all_learned": tot_learned}


def main():
    import argparse
    import torch
    ap = argparse.ArgumentParser(description="train the learned star-pressure proposal")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    ds = build_dataset(a.n)
    print(f"dataset: {ds.x.shape[0]} problems ({ds.n_tubes} tube jumps, {ds.n_harvested} harvested,"
          f" {ds.n_vacuum} vacuum dropped)")
    P, hist = train(ds, epochs=a.epochs, log=print)
    WL, WR = I.random_tube_states(I.SEED_TUBES_HELDOUT, 100_000)
    ev = evaluate(P, torch.from_numpy(WL).cuda(), torch.from_numpy(WR).cuda())
    print(ev)
    if a.out:
        np.save(a.out, P.cpu().numpy())


if __name__ == "__main__":
    main()
