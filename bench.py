"""Benchmark of the Jacobi-PCG hot path on one MI355X.

Step = one full FP32 Jacobi-PCG solve (x0 = 0, relative residual 1e-6 judged
in FP64, with restarts from the FP64 residual when the FP32 recursion drifts)
of the 256^3 seven-point Poisson system b = A x*, x* = lowest sine mode
+ 1e-3 U[-1,1] noise (seed 4). `value` = seconds per solve (lower is better).

Also reported on the same JSON line:
  multigrid     -- PCG with the geometric multigrid V-cycle preconditioner on
                   the same system (constant coefficients), beside Jacobi-PCG;
  refined       -- FP64 iterative refinement around BF16 / FP16 Jacobi-PCG on
                   the same system: seconds to FP64 true residual 1e-6 and
                   1e-10 (the FP32 solve's own true residual is in config);
  roofline      -- the dominant kernel (the PCG update kernel) measured with
                   HIP events on the library's stream in an event-timed solve
                   of the same workload, against 8 TB/s;
  learned       -- the learned preconditioner on the variable-coefficient
                   operator (k = exp(GRF), harmonic-mean faces): the
                   network's forward and training step at 128^3 (MFMA
                   TFLOP/s against the dense BF16 peak), and the whole
                   workflow (FP64 pair generation, on-policy rounds, A-norm
                   training, flexible CG on a held-out right-hand side)
                   against Jacobi-PCG and multigrid-preconditioned PCG at
                   each grid of --learned-n (64 and 128
                   by default);
  paper_grid    -- PCG time per iteration on the paper's 512 x 112 x 64
                   comparison grid (FP32 with two kernels or the
                   single-reduction form, and BF16 storage), beside the
                   paper's own per-iteration times (context, other hardware);
  small_grid    -- the 32^3 workload with both iteration forms;
  slab          -- one GPU's share of the 256^3 system split in z over 8
                   GPUs (256 x 256 x 32 planes): the iteration kernels on that
                   shape, the stencil over the slab with its two halo planes,
                   and the halo bytes an iteration would exchange;
  kernels_512   -- standalone stencil / axpy / dot at 512^3 (FP32 and BF16),
                   achieved GB/s of algorithmic bytes, beside torch's device
                   copy of the same size (the one-read-one-write reference);
  sell_spmv     -- general sparse SpMV (sliced ELLPACK) of the explicitly
                   stored seven-point matrix at 256^3 and on the paper's
                   comparison grid, beside the matrix-free stencil; Jacobi-PCG
                   on the stored matrix at 256^3 (the same b) and 32^3 beside
                   the matrix-free solves; a ragged random SPD matrix (1 M rows)
                   with and without sigma sorting;
  batched       -- 64 uneven problems (edges log-uniform in [16, 128], seed 5;
                   b_i ~ U[-1,1], seeds 1000 + i) in one persistent
                   hipGraph-captured launch: solves/s, per-problem latency,
                   against 64 sequential pcg_solve calls;
  cpu_baseline  -- the FP64 CPU oracle's Jacobi-PCG on the same system,
                   timed on a bounded number of iterations and scaled.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG seconds to 1e-6 rel resid @256³; stencil/dot/axpy achieved HBM GB/s"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per grid point of the two iteration kernels (FP32
# storage, FP64 x accumulator): direction reads r, p_old and writes p. The
# update advances x every second iteration: an odd iteration's update reads
# p, r and writes r (12); the next reads p, p_prev, r, x(FP64) and writes r,
# x(FP64) (32). The batched kernel does the same.
BYTES_DIRECTION = 12
BYTES_UPDATE_SKIP = 12
BYTES_UPDATE_PAIR = 32


def update_bytes(launches: int, es: int = 4, xs: int = 8) -> float:
    """Mean algorithmic bytes per point of `launches` consecutive update
    launches from the first iteration (odd ones skip x, even ones add two
    steps); es: storage bytes, xs: accumulator bytes."""
    skip, pair = 3 * es, 4 * es + 2 * xs
    n_pair = launches // 2
    return (skip * (launches - n_pair) + pair * n_pair) / max(launches, 1)


# Sources that define the PCG iteration kernels and their launch plans;
# counter-measured traffic in profiles/traffic.json is used only while these
# files are unchanged.
ITER_KERNEL_SOURCES = ["common.hpp", "zmarch.hpp", "ops.hpp", "zkernel.hpp", "pcg.hip", "internal.hpp", "runtime.hip"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_23343_amd", "csrc")
    for f in ITER_KERNEL_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """Counter-measured HBM bytes per launch from profiles/, if taken on the
    current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    ent = d.get(kernel)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def build_rhs(P, torch, n):
    """b = A x* on the GPU in FP64 (the library's FP64 stencil), then rounded to FP32."""
    import synthetic

    xs = torch.from_numpy(synthetic.smooth_plus_noise(n)).cuda()
    ctx64 = P.pcg_create(n, n, n, torch.float64)
    b64 = torch.empty_like(xs)
    P.stencil_apply(ctx64, xs, b64)
    torch.cuda.synchronize()
    P.pcg_destroy(ctx64)
    return b64.to(torch.float32), b64


def warm_up(torch, fn, seconds=0.05):
    """Launch fn until `seconds` of wall time have passed (at least 10
    launches): after seconds of host-side input generation the GPU needs tens
    of milliseconds of work to return to its working clocks."""
    t0 = time.perf_counter()
    k = 0
    while k < 10 or time.perf_counter() - t0 < seconds:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        k += 10


def time_kernels_512(P, torch, n, reps):
    """Standalone kernels at n^3: achieved GB/s of algorithmic bytes."""
    import synthetic

    out = {}
    N = n ** 3
    for name, dt, es in (("f32", torch.float32, 4), ("bf16", torch.bfloat16, 2)):
        x = torch.from_numpy(synthetic.uniform_f32(synthetic.SEED_C2_X, N)).cuda().to(dt)
        y = torch.from_numpy(synthetic.uniform_f32(synthetic.SEED_C2_Y, N)).cuda().to(dt)
        z = torch.empty_like(x)
        d = torch.zeros(1, dtype=torch.float32, device="cuda")
        ctx = P.pcg_create(n, n, n, dt)
        ops = {
            "stencil": (lambda: P.stencil_apply(ctx, x, z), 2 * es),
            "axpy": (lambda: P.axpy(ctx, N, 0.5, x, y, z), 3 * es),
            "dot": (lambda: P.dot(ctx, N, x, y, d), 2 * es),
            # reference, not this library's kernel: torch's device copy, the
            # same one-read-one-write stream pattern as the stencil
            "torch_copy": (lambda: z.copy_(x), 2 * es),
        }
        for op, (fn, bpp) in ops.items():
            warm_up(torch, fn)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = bpp * N / (ms * 1e-3) / 1e9
            out[f"{op}_{name}"] = {"us": round(ms * 1e3, 2), "GB/s": round(gbs, 1),
                                   "frac": round(gbs / HBM_PEAK_GBS, 4)}
        P.pcg_destroy(ctx)
        del x, y, z
        torch.cuda.empty_cache()
    return out


def bench_sell(P, torch, reps, grids=((256, 256, 256), None), b256=None, mf_solve_s=None):
    """General sparse SpMV in sliced ELLPACK (C = 64, sigma = 1) on the
    seven-point matrix stored explicitly, the form the paper's GPU comparison
    system uses, beside the matrix-free stencil on the same grid. Algorithmic
    bytes: 8 per stored entry (FP32 value, int32 column) + 4 per row for x
    and 4 for y; padding slots are reported apart."""
    import synthetic

    out = {}
    for dims in grids:
        nx, ny, nz = synthetic.PAPER_GRID if dims is None else dims
        N = nx * ny * nz
        rowptr, col, val = synthetic.poisson7_csr(nx, ny, nz)
        A = P.pcg_sell_create(rowptr, col, val, N, sigma=1)
        del rowptr, col, val
        x = torch.from_numpy(synthetic.uniform_f32(synthetic.SEED_C2_X, N)).cuda()
        y = torch.empty_like(x)
        ctx = P.pcg_create(nx, ny, nz, torch.float32)
        res = {"grid": [nx, ny, nz], "nnz": A.nnz, "slots": A.nslots}
        for name, fn, nbytes in (("sell_spmv", lambda: P.pcg_sell_spmv(A, x, y), 8 * A.nnz + 8 * N),
                                 ("matrix_free_stencil", lambda: P.stencil_apply(ctx, x, y), 8 * N)):
            warm_up(torch, fn)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            e1.synchronize()
            us = e0.elapsed_time(e1) / reps * 1e3
            gbs = nbytes / (us * 1e-6) / 1e9
            res[name] = {"us": round(us, 2), "bytes": nbytes, "GB/s": round(gbs, 1),
                         "frac": round(gbs / HBM_PEAK_GBS, 4)}
        if b256 is not None and (nx, ny, nz) == (256, 256, 256):
            # Jacobi-PCG on the stored matrix, the benchmark's b; per
            # iteration 8 B per entry + 52 B per row on average (q = A p: x
            # and q 8; update: q, r, r', D^-1 16, and every second one also
            # p, p_prev 8 and x 16; direction: r, D^-1, p_old, p 16).
            xs = torch.zeros(N, dtype=torch.float64, device="cuda")
            P.pcg_sell_solve(A, b256, xs, 1e-6, 5000, raise_on_error=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = P.pcg_sell_solve(A, b256, xs, 1e-6, 5000, raise_on_error=False)
            torch.cuda.synchronize()
            s = time.perf_counter() - t0
            it = max(info["iters"], 1)
            per_it = 8 * A.nnz + 52 * N
            res["pcg_solve"] = {"iters": info["iters"], "restarts": info["restarts"], "ms": round(s * 1e3, 2),
                                "status": P.STATUS_NAMES[info["status"]],
                                "us_per_iteration": round(s * 1e6 / it, 1),
                                "iteration_GB/s": round(per_it * it / s / 1e9, 1),
                                "true_relres": info["rel_res_true_fp64"],
                                "matrix_free_ms": None if mf_solve_s is None else round(mf_solve_s * 1e3, 2)}
            del xs
        out["x".join(str(v) for v in (nx, ny, nz))] = res
        P.pcg_destroy(ctx)
        A.close()
        del x, y
        torch.cuda.empty_cache()
    # Ragged rows: a random SPD matrix (1 M rows of 3..35 entries, seed 57)
    # in original order (sigma = 1) and sorted in windows of 4096 rows.
    rowptr, col, val = synthetic.random_spd_csr(1_000_000, seed=57)
    N = rowptr.size - 1
    x = torch.from_numpy(synthetic.uniform_f32(58, N)).cuda()
    y = torch.empty_like(x)
    ragged = {"rows": N, "nnz": int(rowptr[-1])}
    for sigma in (1, 4096):
        A = P.pcg_sell_create(rowptr, col, val, N, sigma=sigma)
        warm_up(torch, lambda: P.pcg_sell_spmv(A, x, y))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            P.pcg_sell_spmv(A, x, y)
        e1.record()
        e1.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        nbytes = 8 * A.nnz + 8 * N + (4 * N if sigma > 1 else 0)
        ragged[f"sigma_{sigma}"] = {"slots": A.nslots, "us": round(us, 2), "GB/s": round(nbytes / (us * 1e-6) / 1e9, 1)}
        A.close()
    out["random_spd_1M"] = ragged
    del rowptr, col, val, x, y
    # Latency-bound case: the 32^3 workload (b ~ U[-1, 1], seed 1) as a stored
    # matrix and matrix-free (two kernels per iteration).
    n1 = 32
    N = n1 ** 3
    A = P.pcg_sell_create(*synthetic.poisson7_csr(n1, n1, n1), N, sigma=1)
    b = torch.from_numpy(synthetic.uniform_f32(synthetic.SEED_C1_B, N)).cuda()
    xs = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx = P.pcg_create(n1, n1, n1, torch.float32, x_dtype=torch.float64, single_reduction=0)
    small = {}
    for name, fn in (("stored_matrix", lambda: P.pcg_sell_solve(A, b, xs, 1e-6, 500, raise_on_error=False)),
                     ("matrix_free", lambda: P.pcg_solve(ctx, b, xs, 1e-6, 500, raise_on_error=False))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            info = fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 5 * 1e3
        small[name] = {"iters": info["iters"], "ms": round(ms, 3),
                       "us_per_iteration": round(ms * 1e3 / max(info["iters"], 1), 2)}
    out["32x32x32_pcg"] = small
    P.pcg_destroy(ctx)
    A.close()
    return out


# The paper's per-iteration times on its comparison grid (its Table III):
# context only (other hardware), never the target.
PAPER_GRID_MS_PER_ITER = {"H100 FP32 (four separate kernels)": 0.28, "Wormhole BF16": 1.20, "Wormhole FP32": 2.45}


def bench_paper_grid(P, torch, steps):
    """PCG time per iteration on the paper's 512 x 112 x 64 comparison grid
    (b ~ U[-1, 1], to recursive 1e-6 for FP32 and 1e-3 for BF16). 3.67 M
    points: an iteration's vectors (73 MB FP32) sit in the last-level cache,
    so this measures latency and cache bandwidth rather than HBM."""
    import synthetic

    nx, ny, nz = synthetic.PAPER_GRID
    N = nx * ny * nz
    b32 = torch.from_numpy(synthetic.uniform_f32(synthetic.SEED_PAPER_GRID_B, N)).cuda()
    out = {"grid": [nx, ny, nz], "paper_ms_per_iteration": PAPER_GRID_MS_PER_ITER}
    for name, dt, xacc, xdt, tol, sr in (("f32", torch.float32, torch.float64, torch.float64, 1e-6, 0),
                                         ("f32_single_reduction", torch.float32, torch.float64, torch.float64, 1e-6, 1),
                                         ("bf16", torch.bfloat16, torch.float32, torch.float64, 1e-3, 0)):
        ctx = P.pcg_create(nx, ny, nz, dt, x_accum=xacc, x_dtype=xdt, single_reduction=sr)
        b = b32.to(dt)
        x = torch.empty(N, dtype=xdt, device="cuda")
        P.pcg_solve(ctx, b, x, tol, 5000, raise_on_error=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = P.pcg_solve(ctx, b, x, tol, 5000, raise_on_error=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        out[name] = {"rtol": tol, "iters": info["iters"], "ms_per_solve": round(ms, 3),
                     "ms_per_iteration": round(ms / max(info["iters"], 1), 5),
                     "true_relres": info["rel_res_true_fp64"]}
        P.pcg_destroy(ctx)
    return out


def bench_slab(P, torch, n=256, parts=8, iters=100):
    """One GPU's share of the n^3 system split into `parts` z-slabs: the two
    iteration kernels timed with HIP events on an n x n x n/parts grid (a
    fixed number of iterations), the standalone stencil over the slab with
    its two halo planes (n/parts + 2 planes), and the bytes one iteration
    would exchange with the two neighbours (one plane of r and of p_old each
    way: the direction kernel forms p on the fly from both)."""
    import synthetic

    nzs = n // parts
    N = n * n * nzs
    b = torch.from_numpy(synthetic.uniform_f32(synthetic.SEED_C1_B, N)).cuda()
    x = torch.empty(N, dtype=torch.float64, device="cuda")
    ctx = P.pcg_create(n, n, nzs, torch.float32, x_dtype=torch.float64, kernel_timing=1, max_restarts=0)
    P.pcg_solve(ctx, b, x, 1e-30, 20, raise_on_error=False)
    info = P.pcg_solve(ctx, b, x, 1e-30, iters, raise_on_error=False)
    k1 = info["k1_ms"] * 1e3 / max(info["k1_launches"], 1)
    k2 = info["k2_ms"] * 1e3 / max(info["k2_launches"], 1)
    P.pcg_destroy(ctx)
    sctx = P.pcg_create(n, n, nzs + 2, torch.float32)
    xs = torch.from_numpy(synthetic.uniform_f32(2, n * n * (nzs + 2))).cuda()
    ys = torch.empty_like(xs)
    warm_up(torch, lambda: P.stencil_apply(sctx, xs, ys))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(50):
        P.stencil_apply(sctx, xs, ys)
    e1.record()
    e1.synchronize()
    st_us = e0.elapsed_time(e1) * 1e3 / 50
    P.pcg_destroy(sctx)
    halo = 2 * 2 * n * n * 4  # r and p_old, one plane to each neighbour, FP32
    return {"slab": [n, n, nzs], "of": [n, n, n], "parts": parts, "iterations_timed": info["k2_launches"],
            "status": P.STATUS_NAMES[info["status"]],
            "direction_us": round(k1, 2), "update_us": round(k2, 2), "iteration_kernels_us": round(k1 + k2, 2),
            "iteration_GB/s": round((BYTES_DIRECTION + update_bytes(info["k2_launches"])) * N / ((k1 + k2) * 1e-6)
                                    / 1e9, 1),
            "stencil_with_halo_planes_us": round(st_us, 2),
            "halo_bytes_per_iteration_each_way": halo,
            "halo_note": "one plane of r and p_old to each z-neighbour per iteration (plus two scalar all-reduces); "
                         "not sent here: this build runs one GPU"}


def bench_multigrid(P, torch, b, n, steps, jacobi_s, nu=1, oracle_budget_s=0.0):
    """PCG with the geometric multigrid V-cycle preconditioner on the
    benchmark's n^3 system (constant coefficients): time to the FP64 true
    residual 1e-6 beside the Jacobi-PCG solve. Algorithmic bytes per
    iteration (FP32 vectors, FP64 x): the flexible iteration's direction (z,
    p_old, r read; p, q written: 20 B/pt) and update (p, q, r, x read; r, x
    written: 36 B/pt), plus the V-cycle: fine level 40 B/pt with one sweep
    per side (start sweep fused with the residual: g read, u and r written;
    restriction reads r; prolongation reads and writes u; the last sweep,
    which also does the flexible select step, reads u, g and q and writes z),
    coarser levels the same over 1/8 of the points each (8/7 in all)."""
    N = n ** 3
    ctx = P.pcg_create(n, n, n, torch.float32, x_dtype=torch.float64)
    t0 = time.perf_counter()
    P.pcg_set_multigrid(ctx, nu=nu)
    setup_s = time.perf_counter() - t0
    levels = P.pcg_mg_levels(ctx)
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    P.pcg_solve_mg(ctx, b, x, 1e-6, 200, raise_on_error=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = P.pcg_solve_mg(ctx, b, x, 1e-6, 200, raise_on_error=False)
    torch.cuda.synchronize()
    s = (time.perf_counter() - t0) / steps
    it = max(info["iters"], 1)
    vcycle = 40 if nu == 1 else 60
    per_it = (20 + 36 + vcycle * 8 / 7) * N
    out = {"grid": n, "nu": nu, "levels": [list(l) for l in levels], "setup_s": round(setup_s, 4),
           "iters": info["iters"], "ms": round(s * 1e3, 3), "us_per_iteration": round(s * 1e6 / it, 1),
           "true_relres": info["rel_res_true_fp64"], "status": P.STATUS_NAMES[info["status"]],
           "jacobi_pcg_ms": round(jacobi_s * 1e3, 3), "speedup_vs_jacobi_pcg": round(jacobi_s / s, 2),
           "iteration_GB/s_estimate": round(per_it / (s / it) / 1e9, 1)}
    ctx.close()
    if oracle_budget_s > 0:
        import oracle

        bh = b.double().cpu().numpy()
        t0 = time.perf_counter()
        ref = oracle.mg_pcg((n, n, n), bh, rtol=0.0, maxit=2)
        t2 = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(t2 / 2 * info["iters"], 2), "unit": "s", "cores": oracle.threads(),
                               "kind": "oracle", "sample": f"FP64 oracle MG-PCG on the same {n}^3 system: 2 "
                               f"iterations timed (set-up included), scaled to the GPU's {info['iters']}"}
    return out


def bench_small_grid(P, torch, steps, n=32):
    """The small workload (n^3, b ~ U[-1, 1] seed 1, FP32 to 1e-6): solve time
    with two kernels per iteration and with the single-reduction form (the
    default at this size). Latency-bound: a few microseconds of work per kernel."""
    import synthetic

    N = n ** 3
    b = torch.from_numpy(synthetic.uniform_f32(synthetic.SEED_C1_B, N)).cuda()
    out = {"grid": n}
    for name, sr in (("two_kernel", 0), ("single_reduction", 1)):
        ctx = P.pcg_create(n, n, n, torch.float32, x_dtype=torch.float64, single_reduction=sr)
        x = torch.empty(N, dtype=torch.float64, device="cuda")
        P.pcg_solve(ctx, b, x, 1e-6, 500, raise_on_error=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = P.pcg_solve(ctx, b, x, 1e-6, 500, raise_on_error=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        out[name] = {"iters": info["iters"], "ms_per_solve": round(ms, 4),
                     "us_per_iteration": round(ms * 1e3 / max(info["iters"], 1), 2),
                     "true_relres": info["rel_res_true_fp64"], "status": P.STATUS_NAMES[info["status"]]}
        P.pcg_destroy(ctx)
    return out


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo) and its logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name} ({os.cpu_count()} logical CPUs visible)"


def cpu_baseline(b64_host, n, gpu_iters, budget_s=15.0, single_budget_s=4.0):
    """The FP64 oracle's Jacobi-PCG on the same system: time a bounded number
    of iterations with all of the oracle's threads and scale to the iteration
    count of the solve; then the same at one thread on a shorter sample."""
    import oracle

    shape = (n, n, n)
    cores = oracle.threads()
    t0 = time.perf_counter()
    oracle.pcg(shape, b64_host, rtol=0.0, maxit=2)
    t2 = time.perf_counter() - t0
    per_iter = t2 / 2.0
    m = int(max(2, min(gpu_iters, budget_s / max(per_iter, 1e-9))))
    t0 = time.perf_counter()
    out = oracle.pcg(shape, b64_host, rtol=1e-6, maxit=m)
    tm = time.perf_counter() - t0
    its = out["iters"]
    full = out["status"] == oracle.OK
    per_iter = tm / max(its, 1)
    est = tm if full else per_iter * gpu_iters
    # one thread: a few iterations, scaled the same way
    oracle.set_threads(1)
    try:
        m1 = int(max(2, min(gpu_iters, single_budget_s / max(per_iter * cores, 1e-9))))
        t0 = time.perf_counter()
        o1 = oracle.pcg(shape, b64_host, rtol=0.0, maxit=m1)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    est1 = t1 / max(o1["iters"], 1) * gpu_iters
    return {"value": round(est, 3), "unit": "s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "single_thread": {"value": round(est1, 2), "unit": "s", "cores": 1,
                              "sample": f"first {o1['iters']} iterations at one thread ({t1:.1f} s), scaled to "
                                        f"the GPU's {gpu_iters} iterations"},
            "sample": (f"FP64 oracle Jacobi-PCG on the same {n}^3 system: "
                       + (f"full solve, {its} iterations" if full else
                          f"first {its} iterations timed ({tm:.1f} s), scaled to the GPU's {gpu_iters} iterations"))}


def cpu_baseline_sell(b32_host, n, gpu_iters, reps=3):
    """The oracle beside the stored-matrix rows: its compressed-row SpMV of
    the 256^3 seven-point matrix (FP64, `reps` products) and its Jacobi-PCG
    on the same b, 4 iterations timed and scaled to the GPU's count."""
    import oracle
    import synthetic

    rowptr, col, val = synthetic.poisson7_csr(n, n, n)
    x = synthetic.uniform_f32(synthetic.SEED_C2_X, n ** 3).astype("float64")
    oracle.csr_spmv(rowptr, col, val, x)
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.csr_spmv(rowptr, col, val, x)
    spmv_s = (time.perf_counter() - t0) / reps
    b64 = b32_host.astype("float64")
    t0 = time.perf_counter()
    out = oracle.csr_pcg(rowptr, col, val, b64, rtol=0.0, maxit=4)
    it_s = (time.perf_counter() - t0) / max(out["iters"], 1)
    return {"cores": oracle.threads(), "kind": "oracle", "spmv_ms": round(spmv_s * 1e3, 1),
            "pcg_s_estimate": round(it_s * gpu_iters, 2),
            "sample": (f"FP64 oracle on the stored {n}^3 seven-point matrix: {reps} products timed; "
                       f"Jacobi-PCG on the same b, 4 iterations timed (setup included) and scaled to the "
                       f"GPU's {gpu_iters} iterations")}


def bench_batched(P, torch, reps, oracle_budget_s=0.0):
    """The 64-problem batch: graph replays timed with torch events on the
    stream the batch was created on (the current stream)."""
    import synthetic

    sizes = synthetic.batch_sizes()
    dims = [(m, m, m) for m in sizes]
    t0 = time.perf_counter()
    bt = P.pcg_batch_create(dims)
    t_create = time.perf_counter() - t0
    b = torch.zeros(bt.total, dtype=torch.float32, device="cuda")
    for i, m in enumerate(sizes):
        bt.view(b, i).copy_(torch.from_numpy(synthetic.uniform_f32(synthetic.SEED_C4_B_BASE + i, m ** 3)))
    x = torch.zeros(bt.total, dtype=torch.float64, device="cuda")
    for _ in range(2):
        r = P.pcg_batch_solve(bt, b, x, rtol=1e-6, maxit=5000, raise_on_error=False)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        r = P.pcg_batch_solve(bt, b, x, rtol=1e-6, maxit=5000, raise_on_error=False)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    lat = sorted(r["latency_s"])
    # the batched kernel also advances x every second update (12 or 32 B/pt)
    traffic = sum((BYTES_DIRECTION + update_bytes(it)) * it * m ** 3 for m, it in zip(sizes, r["iters"]))
    # the same 64 problems one after another through pcg_solve
    ctxs = []
    for i, m in enumerate(sizes):
        ctx = P.pcg_create(m, m, m, torch.float32, x_dtype=torch.float64)
        ctxs.append((ctx, torch.empty(m ** 3, dtype=torch.float64, device="cuda")))
    for i, (ctx, xi) in enumerate(ctxs):
        P.pcg_solve(ctx, bt.view(b, i), xi, 1e-6, 5000, raise_on_error=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_iters = []
    for i, (ctx, xi) in enumerate(ctxs):
        seq_iters.append(P.pcg_solve(ctx, bt.view(b, i), xi, 1e-6, 5000, raise_on_error=False)["iters"])
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    for ctx, _ in ctxs:
        ctx.close()
    out = {"problems": len(sizes), "points": int(sum(m ** 3 for m in sizes)), "ms_per_batch": round(ms, 3),
           "solves_per_s": round(len(sizes) / (ms * 1e-3), 1),
           "latency_ms": {"min": round(lat[0] * 1e3, 3), "median": round(lat[len(lat) // 2] * 1e3, 3),
                          "max": round(lat[-1] * 1e3, 3)},
           "effective_GB/s": round(traffic / (ms * 1e-3) / 1e9, 1),
           "iters_total": int(sum(r["iters"])), "restarts_total": int(sum(r["restarts"])),
           "status": P.STATUS_NAMES[r["status"]],
           "max_true_relres": max(r["relres"]), "sequential_ms": round(seq * 1e3, 2),
           "speedup_vs_sequential": round(seq * 1e3 / ms, 3),
           "iters_equal_sequential": int(sum(1 for a, c in zip(r["iters"], seq_iters) if a == c)),
           "work_groups": bt.grid, "create_and_tune_s": round(t_create, 3),
           # per problem: edge, iterations, work-groups, latency (ms), in finishing order
           "per_problem": sorted(([m, int(it), int(bt.plans[i][2]), round(lt * 1e3, 2)]
                                  for i, (m, it, lt) in enumerate(zip(sizes, r["iters"], r["latency_s"]))),
                                 key=lambda e: e[3])}
    bt.close()
    if oracle_budget_s > 0:
        out["oracle"] = batched_oracle(sizes, r["iters"], oracle_budget_s)
    return out


def batched_oracle(sizes, gpu_iters, budget_s):
    """The FP64 oracle's Jacobi-PCG on the batch's problems, smallest first,
    until the budget is spent; scaled to all of them by point-iterations."""
    import oracle
    import synthetic

    order = sorted(range(len(sizes)), key=lambda i: sizes[i])
    t_done, work_done, solved = 0.0, 0.0, 0
    for i in order:
        m = sizes[i]
        b64 = synthetic.uniform_f32(synthetic.SEED_C4_B_BASE + i, m ** 3).astype("float64")
        t0 = time.perf_counter()
        ref = oracle.pcg((m, m, m), b64, rtol=1e-6, maxit=5000)
        t_done += time.perf_counter() - t0
        work_done += m ** 3 * ref["iters"]
        solved += 1
        if t_done > budget_s:
            break
    total = sum(m ** 3 * it for m, it in zip(sizes, gpu_iters))
    est = t_done * total / max(work_done, 1.0)
    return {"value": round(est, 3), "unit": "s", "cores": oracle.threads(), "kind": "oracle",
            "sample": (f"FP64 oracle Jacobi-PCG on the {solved} smallest of the {len(sizes)} problems "
                       f"({t_done:.1f} s), scaled to all by point-iterations"),
            "solves_per_s": round(len(sizes) / est, 3)}


BF16_PEAK_TFLOPS = 2500.0
# FLOP per voxel of one forward pass: 2 x 27 taps x (2*16 + 16*16 + 16*16 + 16*1)
CNN_FLOP_PER_VOXEL = 2 * 27 * (2 * 16 + 16 * 16 + 16 * 16 + 16)


def bench_learned(P, torch, n_works, rounds, n_kernel=128, oracle_cpu=False):
    import numpy as np

    import synthetic
    from paper_2603_23343_amd import learned as L

    out = {}
    # network kernels at n_kernel^3
    nk = n_kernel
    N = nk ** 3
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(L.he_init(7)).cuda())
    r = torch.from_numpy(synthetic.uniform_f32(1, N)).cuda()
    g = torch.from_numpy(synthetic.gaussian_random_field(nk).astype(np.float32)).cuda()
    z = torch.empty(N, device="cuda")
    warm_up(torch, lambda: P.cnn_forward(net, (nk, nk, nk), r, g, z))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(20):
        P.cnn_forward(net, (nk, nk, nk), r, g, z)
    ev1.record()
    torch.cuda.synchronize()
    fwd_ms = ev0.elapsed_time(ev1) / 20
    pairs = torch.from_numpy(synthetic.f32_to_bf16_bits(synthetic.uniform_f32(3, 2 * 4 * N)).view(np.int16)).view(
        torch.bfloat16).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.cnn_train_step(net, (nk, nk, nk), pairs, g, 4, lr=1e-5, loss=loss)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(3):
        P.cnn_train_step(net, (nk, nk, nk), pairs, g, 4, lr=1e-5, loss=loss)
    ev1.record()
    torch.cuda.synchronize()
    train_ms = ev0.elapsed_time(ev1) / 12
    fl = CNN_FLOP_PER_VOXEL * N
    out["network"] = {"grid": nk, "forward_ms": round(fwd_ms, 4),
                      "forward_TFLOP/s": round(fl / (fwd_ms * 1e-3) / 1e12, 1),
                      "forward_frac_of_bf16_peak": round(fl / (fwd_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4),
                      "train_ms_per_sample": round(train_ms, 3),
                      "train_TFLOP/s": round(3 * fl / (train_ms * 1e-3) / 1e12, 1)}
    net.close()
    out["workflow"] = [learned_workflow(P, torch, n, rounds, oracle_cpu) for n in n_works]
    return out


def learned_workflow(P, torch, n, rounds, oracle_cpu):
    """On-policy training of the correction network on one n^3 variable-coefficient
    problem, then Jacobi-PCG against flexible CG with the learned preconditioner on a
    held-out right-hand side (both judged by the FP64 true residual)."""
    import numpy as np

    import synthetic
    from paper_2603_23343_amd import learned as L

    N = n ** 3
    kd = torch.from_numpy(synthetic.coefficient_field(n)).cuda()
    gd = torch.from_numpy(synthetic.gaussian_random_field(n).astype(np.float32)).cuda()
    net = P.cnn_create()
    P.cnn_set_weights(net, torch.from_numpy(L.he_init_correction(7)).cuda())
    log = L.train_onpolicy(net, n, kd, gd, range(synthetic.SEED_C5_TRAIN_BASE, synthetic.SEED_C5_TRAIN_BASE + 8),
                           rounds=rounds, epochs=3)
    ctx = P.pcg_create(n, n, n, torch.float32, x_dtype=torch.float64)
    P.pcg_set_coefficients(ctx, kd)
    x = torch.empty(N, dtype=torch.float64, device="cuda")
    b = torch.from_numpy(synthetic.uniform_f32(synthetic.SEED_C5_HELDOUT_BASE, N)).cuda()
    P.pcg_solve(ctx, b, x, 1e-6, 20000, raise_on_error=False)
    jac = P.pcg_solve(ctx, b, x, 1e-6, 20000, raise_on_error=False)
    P.pcg_solve_flexible(ctx, net, gd, b, x, 1e-6, 20000, raise_on_error=False)
    fcg = P.pcg_solve_flexible(ctx, net, gd, b, x, 1e-6, 20000, raise_on_error=False)
    # the non-learned baseline: PCG with the geometric multigrid V-cycle
    P.pcg_set_multigrid(ctx)
    P.pcg_solve_mg(ctx, b, x, 1e-6, 500, raise_on_error=False)
    mgi = P.pcg_solve_mg(ctx, b, x, 1e-6, 500, raise_on_error=False)
    oracle_out = None
    if oracle_cpu:
        import oracle

        t0 = time.perf_counter()
        ref = oracle.pcg((n, n, n), b.double().cpu().numpy(), rtol=1e-6, maxit=20000,
                         kcell=kd.double().cpu().numpy())
        oracle_out = {"value": round(time.perf_counter() - t0, 3), "unit": "s", "cores": oracle.threads(),
                      "kind": "oracle", "iters": ref["iters"],
                      "sample": f"FP64 oracle Jacobi-PCG on the same {n}^3 variable-coefficient system, full solve"}
    out = {"grid": n, "rounds": rounds, "pairs": log["pairs"][-1], "jacobi_pcg_oracle": oracle_out,
           "final_loss": round(log["losses"][-1], 4), "pair_gen_s": round(log["gen_s"], 3),
           "onpolicy_s": round(log["onpolicy_s"], 3), "train_s": round(log["train_s"], 3),
           "jacobi_pcg": {"iters": jac["iters"], "ms": round(jac["seconds"] * 1e3, 3),
                          "true_relres": jac["rel_res_true_fp64"]},
           "flexible_cg_learned": {"iters": fcg["iters"], "ms": round(fcg["seconds"] * 1e3, 3),
                                   "fallback_used": fcg["fallback_used"],
                                   # iteration at which Jacobi-PCG took over (-1: never)
                                   "fallback_at": fcg["outer_iters"] if fcg["fallback_used"] == 1 else -1,
                                   "true_relres": fcg["rel_res_true_fp64"]},
           "multigrid_pcg": {"iters": mgi["iters"], "ms": round(mgi["seconds"] * 1e3, 3),
                             "true_relres": mgi["rel_res_true_fp64"], "status": P.STATUS_NAMES[mgi["status"]]},
           "iteration_ratio": round(fcg["iters"] / max(jac["iters"], 1), 3)}
    net.close()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--n-kernels", type=int, default=512)
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernels", action="store_true")
    ap.add_argument("--no-refined", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-paper-grid", action="store_true")
    ap.add_argument("--no-sell", action="store_true")
    ap.add_argument("--no-multigrid", action="store_true")
    ap.add_argument("--no-slab", action="store_true")
    ap.add_argument("--learned-n", default="64,128",
                    help="comma-separated grid sizes of the learned-preconditioner workflow")
    ap.add_argument("--learned-rounds", type=int, default=12)
    ap.add_argument("--batched-reps", type=int, default=10)
    ap.add_argument("--maxit", type=int, default=5000)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also copy a buffer of this many MiB 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver is single-GPU.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2603_23343_amd as P

    if args.copy_probe > 0:
        # A plain device copy of known size: its FETCH_SIZE / WRITE_SIZE
        # counters calibrate the counter bytes of the solver's kernels.
        src = torch.ones(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    n = args.n
    N = n ** 3
    b, b64 = build_rhs(P, torch, n)
    ctx = P.pcg_create(n, n, n, torch.float32, x_dtype=torch.float64)
    x = torch.empty(N, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        P.pcg_solve(ctx, b, x, 1e-6, args.maxit, raise_on_error=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(P.pcg_solve(ctx, b, x, 1e-6, args.maxit, raise_on_error=False))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    dt_solve = dt
    info = infos[-1]
    iters = info["iters"]
    print(f"# solve: {iters} iterations, {dt * 1e3:.2f} ms, recursive {info['rel_res_recursive']:.3e}, "
          f"true {info['rel_res_true_fp64']:.3e}", file=sys.stderr, flush=True)

    # Per-kernel durations: the same solve with HIP events around every
    # iteration kernel (eager launches on the same stream).
    tctx = P.pcg_create(n, n, n, torch.float32, x_dtype=torch.float64, kernel_timing=1)
    tinfo = P.pcg_solve(tctx, b, x, 1e-6, args.maxit, raise_on_error=False)
    k2_us = tinfo["k2_ms"] * 1e3 / max(tinfo["k2_launches"], 1)
    k1_us = tinfo["k1_ms"] * 1e3 / max(tinfo["k1_launches"], 1)
    # the dominant kernel: the update of even iterations (x += two steps)
    n_even = tinfo["k2_even_launches"]
    n_odd = tinfo["k2_launches"] - n_even
    k2e_us = tinfo["k2_even_ms"] * 1e3 / max(n_even, 1)
    k2o_us = (tinfo["k2_ms"] - tinfo["k2_even_ms"]) * 1e3 / max(n_odd, 1)
    achieved = BYTES_UPDATE_PAIR * N / (k2e_us * 1e-6) / 1e9
    bytes_upd = update_bytes(tinfo["k2_launches"])
    bytes_iter = BYTES_DIRECTION + update_bytes(iters)
    traffic = load_traffic("pcg_update_even")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "pcg_update, even iterations (k_pcg_update<..., OpUpdate<..., XM = 2>, FinAlpha>: finishes "
                          "p.Ap, then r -= alpha A p and x += alpha_prev p_prev + alpha p)",
                "bytes_per_launch": BYTES_UPDATE_PAIR * N, "avg_us": round(k2e_us, 2), "launches": n_even,
                "odd_update_avg_us": round(k2o_us, 2),
                "odd_update_GB/s": round(BYTES_UPDATE_SKIP * N / (k2o_us * 1e-6) / 1e9, 1),
                "update_mean_bytes_per_point": round(bytes_upd, 3),
                "update_mean_GB/s": round(bytes_upd * N / (k2_us * 1e-6) / 1e9, 1),
                "direction_kernel_avg_us": round(k1_us, 2),
                "direction_kernel_GB/s": round(BYTES_DIRECTION * N / (k1_us * 1e-6) / 1e9, 1),
                # both kernels' algorithmic bytes over the timed solve's time per iteration
                "iteration_GB/s": round(bytes_iter * N / (dt_solve / iters) / 1e9, 1),
                "iteration_frac": round(bytes_iter * N / (dt_solve / iters) / 1e9 / HBM_PEAK_GBS, 4),
                "event_timed_solve_ms": round(tinfo["seconds"] * 1e3, 2),
                # q = Ap is recomputed, never stored, and x advances every second
                # iteration: 34 B/pt per iteration here against 40 with x in every
                # update and 52 for the textbook fused iteration that stores q
                "bytes_convention": "design 12 + (12 or 32) = 34 B/pt per iteration on average (q never "
                                    "stored, x advanced every second iteration); 40 with x in every update; "
                                    "the textbook count with q stored is 52 B/pt",
                "iteration_frac_at_52B": round(52 * N / (dt_solve / iters) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic_note": "FETCH_SIZE counts L2 fills, last-level-cache hits included"}
    P.pcg_destroy(tctx)

    # Mixed-precision refinement on the same system: FP64 outer loop, BF16 /
    # FP16 inner Jacobi-PCG; time to FP64 true residual 1e-6 and 1e-10.
    refined = {}
    if not args.no_refined:
        for name, rdt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
            rctx = P.pcg_create(n, n, n, rdt, x_accum=torch.float32)
            x64 = torch.empty(N, dtype=torch.float64, device="cuda")
            P.pcg_solve_refined(rctx, b64, x64, rtol_outer=1e-10)
            torch.cuda.synchronize()
            r = P.pcg_solve_refined(rctx, b64, x64, rtol_outer=1e-10)
            refined[name] = {"t_1e6_s": round(r["t_1e6"], 5), "t_1e10_s": round(r["t_1e10"], 5),
                             "outer": r["outer_iters"], "inner_total": r["iters"],
                             "final_true_relres": r["rel_res_true_fp64"],
                             "speedup_vs_fp32_pcg_to_1e-6_recursive": round(dt_solve / max(r["t_1e6"], 1e-9), 3)}
            P.pcg_destroy(rctx)
            # per-kernel times of the inner iterations: the same refinement
            # with HIP events around every inner iteration kernel. Algorithmic
            # bytes per point with e-byte storage and the FP32 correction d:
            # direction reads r, p_old and writes p (3e); update reads p, r
            # and writes r (3e), and every second one also reads p_prev and
            # reads and writes d (4e + 8).
            tctx = P.pcg_create(n, n, n, rdt, x_accum=torch.float32, kernel_timing=1)
            tr = P.pcg_solve_refined(tctx, b64, x64, rtol_outer=1e-10)
            es = 2
            k1 = tr["k1_ms"] * 1e3 / max(tr["k1_launches"], 1)
            k2 = tr["k2_ms"] * 1e3 / max(tr["k2_launches"], 1)
            refined[name]["inner_kernels"] = {
                "direction_us": round(k1, 2), "direction_GB/s": round(3 * es * N / (k1 * 1e-6) / 1e9, 1),
                "update_us": round(k2, 2),
                "update_GB/s": round(update_bytes(tr["k2_launches"], es, 4) * N / (k2 * 1e-6) / 1e9, 1),
                "iteration_GB/s": round((3 * es + update_bytes(tr["k2_launches"], es, 4)) * N / ((k1 + k2) * 1e-6)
                                        / 1e9, 1),
                "launches": tr["k1_launches"]}
            P.pcg_destroy(tctx)
            del x64
        print(f"# refined: {refined}", file=sys.stderr, flush=True)

    slab = None
    if not args.no_slab:
        slab = bench_slab(P, torch)
        print(f"# slab: {slab}", file=sys.stderr, flush=True)

    multigrid = None
    if not args.no_multigrid:
        multigrid = bench_multigrid(P, torch, b, n, max(args.steps, 3), dt_solve,
                                    oracle_budget_s=0.0 if args.no_cpu_baseline else 1.0)
        print(f"# multigrid: {multigrid}", file=sys.stderr, flush=True)

    batched = None
    if not args.no_batched:
        batched = bench_batched(P, torch, args.batched_reps, 0.0 if args.no_cpu_baseline else 3.0)
        print(f"# batched: {batched}", file=sys.stderr, flush=True)

    paper_grid = small_grid = None
    if not args.no_paper_grid:
        paper_grid = bench_paper_grid(P, torch, max(args.steps, 3))
        print(f"# paper_grid: {paper_grid}", file=sys.stderr, flush=True)
        small_grid = bench_small_grid(P, torch, max(args.steps, 3) * 4)
        print(f"# small_grid: {small_grid}", file=sys.stderr, flush=True)

    learned = None
    if not args.no_learned:
        sizes = [int(v) for v in args.learned_n.split(",") if v.strip()]
        learned = bench_learned(P, torch, sizes, args.learned_rounds, oracle_cpu=not args.no_cpu_baseline)
        print(f"# learned: {learned}", file=sys.stderr, flush=True)

    sell = None
    if not args.no_sell:
        sell = bench_sell(P, torch, args.kernel_reps, b256=b if n == 256 else None, mf_solve_s=dt_solve)
        if not args.no_cpu_baseline and n == 256:
            g_it = sell["256x256x256"]["pcg_solve"]["iters"]
            sell["cpu_baseline"] = cpu_baseline_sell(b.cpu().numpy(), n, g_it)
        print(f"# sell: {sell}", file=sys.stderr, flush=True)

    kern = None
    if not args.no_kernels:
        del ctx
        torch.cuda.empty_cache()
        kern = time_kernels_512(P, torch, args.n_kernels, args.kernel_reps)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(b64.cpu().numpy(), n, iters)

    line = {
        "metric": METRIC, "value": round(dt, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{n}^3 seven-point Poisson, b = A x*, x* = sin*sin*sin + 1e-3 U[-1,1] "
                                "(seed 4); FP32 Jacobi-PCG from x0 = 0 to 1e-6, judged by the FP64 true residual "
                                "(restarts from r = b - A x when the recursion drifts), FP64 x accumulator"),
                   "grid": [n, n, n], "iters": iters, "rel_res_recursive": info["rel_res_recursive"],
                   "rel_res_true_fp64": info["rel_res_true_fp64"], "restarts": info["restarts"],
                   "status": P.STATUS_NAMES[info["status"]],
                   "per_iteration_us": round(dt * 1e6 / max(iters, 1), 2)},
        "roofline": roofline,
        "refined": refined or None,
        "multigrid": multigrid,
        "batched": batched,
        "paper_grid": paper_grid,
        "small_grid": small_grid,
        "slab": slab,
        "learned": learned,
        "kernels_512": kern,
        "sell_spmv": sell,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
