"""Learned-preconditioner workflow on top of the C ABI: generate (residual,
error) training pairs with the FP64 solver, train the network, and solve
with flexible CG. Orchestration only: every arithmetic step runs in the
library's kernels (snapshot solve, pair scaling, forward/backward, Adam).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _binding as B


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
    """Adam on mean relative-MSE over contiguous batches (visited in a random
    order each epoch). Returns (per-epoch mean losses, seconds)."""
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
