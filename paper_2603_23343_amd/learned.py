"""Learned-preconditioner workflow on top of the C ABI: generate (residual,
error) training pairs with the FP64 solver, train the network, and solve
with flexible CG. Orchestration only: every arithmetic step runs in the
library's kernels (snapshot solve, pair scaling, forward/backward, Adam).

Two sources of pairs, both from the solver itself:
  - generate_pairs: snapshots (r_k, x* - x_k) of FP64 Jacobi-PCG solves;
  - onpolicy_pairs: iterates x_k of the flexible solve with the current
    network, r_k = b - A x_k in FP64 and e_k = x* - x_k with x* from an
    FP64 solve -- the residuals the preconditioner meets inside the flexible
    solve, on which a network trained only on Jacobi-PCG residuals degrades.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _binding as B
from . import checkpoint


def snapshot_iterations(first: int, last: int, count: int) -> list[int]:
    """count distinct, geometrically spaced iterations in [first, last]."""
    its = sorted({int(round(v)) for v in np.geomspace(first, last, count)})
    k = last
    while len(its) < count and k > 0:
        if k not in its:
            its.append(k)
        k -= 1
    return sorted(its)[:count]


def generate_pairs(n: int, kcell: torch.Tensor, rhs_seeds, snaps_per_rhs: int = 16, rtol: float = 1e-12,
                   maxit: int = 20000, perm_seed: int = 0, stream=None):
    """Pairs from FP64 Jacobi-PCG on the variable-coefficient n^3 operator.

    For every seed, b ~ U[-1, 1] (FP64); one snapshot solve to rtol records
    (r_k, x_k) at geometrically spaced iterations k (up to ~60% of the
    iteration count of a probe solve); e_k = x* - x_k with x* the final
    iterate. Pairs are written to a random permutation of slots so that
    contiguous batches mix right-hand sides and snapshot depths.
    Returns (pairs BF16 [npairs * 2 * n^3], seconds).
    """
    import synthetic

    t0 = time.perf_counter()
    N = n ** 3
    ctx = B.pcg_create(n, n, n, torch.float64, stream=stream)
    B.pcg_set_coefficients(ctx, kcell)
    seeds = list(rhs_seeds)
    npairs = len(seeds) * snaps_per_rhs
    pairs = torch.empty(2 * npairs * N, dtype=torch.bfloat16, device="cuda")
    slots = np.random.default_rng(perm_seed).permutation(npairs)
    x = torch.empty(N, dtype=torch.float64, device="cuda")
    rs = torch.empty(snaps_per_rhs * N, dtype=torch.float64, device="cuda")
    xs = torch.empty_like(rs)
    probe = None
    for j, seed in enumerate(seeds):
        b = torch.from_numpy(synthetic.uniform(seed, N)).cuda()
        if probe is None:
            info = B.pcg_solve(ctx, b, x, rtol, maxit)
            probe = info["iters"]
        its = snapshot_iterations(1, max(snaps_per_rhs, int(0.6 * probe)), snaps_per_rhs)
        B.pcg_solve_snapshots(ctx, b, x, its, rs, xs, rtol=rtol, maxit=maxit)
        for s in range(snaps_per_rhs):
            slot = int(slots[j * snaps_per_rhs + s])
            B.pcg_make_pairs(ctx, 1, rs[s * N:(s + 1) * N], xs[s * N:(s + 1) * N], x,
                             pairs[2 * slot * N:2 * (slot + 1) * N])
    torch.cuda.synchronize()
    ctx.close()
    return pairs, time.perf_counter() - t0


def train(net, n: int, pairs: torch.Tensor, g: torch.Tensor, epochs: int, batch: int, lr: float,
          seed: int = 0, lr_decay: float = 1.0):
    """Adam over contiguous batches of pairs (visited in a random order each
    epoch) on the network's loss: the A-norm loss once cnn_set_operator has
    given it the operator, the relative MSE otherwise. Returns (per-epoch
    mean losses, seconds)."""
    N = n ** 3
    npairs = pairs.numel() // (2 * N)
    nb = npairs // batch
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        tot = 0.0
        for bi in rng.permutation(nb):
            chunk = pairs[2 * int(bi) * batch * N:2 * (int(bi) + 1) * batch * N]
            B.cnn_train_step(net, (n, n, n), chunk, g, batch, lr=lr, loss=loss)
            tot += loss.item()
        hist.append(tot / max(nb, 1))
        lr *= lr_decay
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def he_init(seed: int) -> np.ndarray:
    """He-normal initial weights of the 2 -> 16 -> 16 -> 16 -> 1 network (FP32)."""
    chans = [2, 16, 16, 16, 1]
    out = []
    for i in range(4):
        std = (2.0 / (27 * chans[i])) ** 0.5
        out.append(np.random.default_rng(seed + i).standard_normal(27 * chans[i] * chans[i + 1]) * std)
    return np.concatenate(out).astype(np.float32)


def onpolicy_pairs(net, n: int, kcell: torch.Tensor, g: torch.Tensor, rhs_seeds, snap_iters, rtol: float = 1e-12,
                   maxit: int = 20000, stream=None):
    """Pairs from flexible-CG trajectories with the current network.

    For each seed, b ~ U[-1, 1] (FP64); x* from FP64 Jacobi-PCG to rtol; for
    every k in snap_iters, x_k = the flexible solve's iterate after k
    iterations (FP32 vectors, FP64 x, b rounded to FP32), r_k = b - A x_k in
    FP64, and the pair (r_k, x* - x_k) scaled by rms(r_k).
    Returns (pairs BF16 [npairs * 2 * n^3], seconds).
    """
    import synthetic

    t0 = time.perf_counter()
    N = n ** 3
    ctx64 = B.pcg_create(n, n, n, torch.float64, stream=stream)
    B.pcg_set_coefficients(ctx64, kcell)
    ctx32 = B.pcg_create(n, n, n, torch.float32, stream=stream, x_dtype=torch.float64)
    B.pcg_set_coefficients(ctx32, kcell)
    seeds = list(rhs_seeds)
    its = list(snap_iters)
    pairs = torch.empty(2 * len(seeds) * len(its) * N, dtype=torch.bfloat16, device="cuda")
    xs = torch.empty(N, dtype=torch.float64, device="cuda")
    xk = torch.empty(N, dtype=torch.float64, device="cuda")
    ax = torch.empty(N, dtype=torch.float64, device="cuda")
    rk = torch.empty(N, dtype=torch.float64, device="cuda")
    slot = 0
    for seed in seeds:
        b64 = torch.from_numpy(synthetic.uniform(seed, N)).cuda()
        b32 = b64.float()
        B.pcg_solve(ctx64, b64, xs, rtol, maxit)
        for k in its:
            B.pcg_solve_flexible(ctx32, net, g, b32, xk, rtol=0.0, maxit=int(k), raise_on_error=False)
            B.stencil_apply(ctx64, xk, ax)
            B.axpy(ctx64, N, -1.0, ax, b64, rk)
            B.pcg_make_pairs(ctx64, 1, rk, xk, xs, pairs[2 * slot * N:2 * (slot + 1) * N])
            slot += 1
    torch.cuda.synchronize()
    ctx64.close()
    ctx32.close()
    return pairs, time.perf_counter() - t0


def train_onpolicy(net, n: int, kcell: torch.Tensor, g: torch.Tensor, train_seeds, rounds: int = 4,
                   epochs: int = 3, batch: int = 8, lr: float = 1e-3, snaps_per_rhs: int = 16,
                   onpolicy_seeds: int = 4, onpolicy_iters=None, seed: int = 0, stream=None,
                   checkpoint_path: str | None = None):
    """A-norm training (cnn_set_operator) of the Jacobi-plus-correction
    network: FP64 Jacobi-PCG snapshot pairs, then `rounds` rounds of
    `epochs` epochs, each followed by on-policy pairs from flexible-CG
    trajectories of `onpolicy_seeds` training right-hand sides (cycled).
    With checkpoint_path, the weights and Adam state are written there after
    every round (checkpoint.save; metadata: round, grid, loss, pairs).
    Returns a log dict (losses per round, pair counts, seconds)."""
    ctx = B.pcg_create(n, n, n, torch.float32, stream=stream)
    B.pcg_set_coefficients(ctx, kcell)
    B.cnn_set_operator(net, ctx)
    seeds = list(train_seeds)
    its = list(onpolicy_iters) if onpolicy_iters is not None else list(range(2, 25, 2))
    t0 = time.perf_counter()
    pairs, t_gen = generate_pairs(n, kcell, seeds, snaps_per_rhs=snaps_per_rhs, perm_seed=seed, stream=stream)
    log = {"losses": [], "pairs": [], "gen_s": t_gen, "train_s": 0.0, "onpolicy_s": 0.0}
    N = n ** 3
    for rnd in range(rounds):
        hist, tt = train(net, n, pairs, g, epochs, batch, lr, seed=seed + rnd)
        log["losses"].append(hist[-1])
        log["pairs"].append(pairs.numel() // (2 * N))
        log["train_s"] += tt
        if checkpoint_path:
            checkpoint.save(net, checkpoint_path, meta={"round": rnd + 1, "grid": n, "loss": hist[-1],
                                                        "pairs": log["pairs"][-1]})
        if rnd + 1 == rounds:
            break
        pick = [seeds[(rnd * onpolicy_seeds + j) % len(seeds)] for j in range(onpolicy_seeds)]
        extra, to = onpolicy_pairs(net, n, kcell, g, pick, its, stream=stream)
        log["onpolicy_s"] += to
        pairs = torch.cat([pairs, extra])
        # keep contiguous batches mixed: shuffle whole pairs
        npairs = pairs.numel() // (2 * N)
        perm = torch.from_numpy(np.random.default_rng(seed + 100 + rnd).permutation(npairs)).cuda()
        pairs = pairs.view(npairs, 2 * N)[perm].reshape(-1).contiguous()
    B.cnn_set_operator(net, None)
    ctx.close()
    log["total_s"] = time.perf_counter() - t0
    return log


def he_init_correction(seed: int) -> np.ndarray:
    """He-normal layers 1-3 and a zero last layer: the correction starts at 0,
    so the preconditioner D^-1 r + N starts as Jacobi."""
    w = he_init(seed)
    w[14688:] = 0.0
    return w
