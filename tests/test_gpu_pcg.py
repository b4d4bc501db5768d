"""GPU parity of the fused Jacobi-PCG solver (paper Sec. VII) against the FP64
oracle, through the C ABI.

Bar: iteration counts within 2 of the oracle's FP64 Jacobi-PCG on random
right-hand sides; final FP64 true residual (recomputed on the CPU from the
returned x) <= 1e-6 for the FP32 solver with its FP64 x accumulator.
"""
import math

import numpy as np
import pytest
import torch

import synthetic
from gpu_helpers import check_status, host64, make_vec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2603_23343_amd as P

    return P


def _solve(P, shape, b, rtol=1e-6, maxit=500, x_dtype=None, **opts):
    nz, ny, nx = shape
    ctx = P.pcg_create(nx, ny, nz, b.dtype, **({"x_dtype": x_dtype} if x_dtype is not None else {}), **opts)
    x = torch.empty(b.numel(), dtype=x_dtype or b.dtype, device="cuda")
    info = P.pcg_solve(ctx, b, x, rtol, maxit, raise_on_error=False)
    hist = P.pcg_get_history(ctx)
    return ctx, x, info, hist


@pytest.mark.parametrize("x_dtype", [torch.float32, torch.float64])
def test_config1_32cubed(P, orc, x_dtype):
    """32^3, b ~ U[-1,1] (seed 1), x0 = 0, rtol 1e-6, maxit 500."""
    shape = (32, 32, 32)
    b, b64 = make_vec(synthetic.SEED_C1_B, 32 ** 3, torch.float32)
    ref = orc.pcg(shape, b64, rtol=1e-6, maxit=500, history=True)
    ctx, x, info, hist = _solve(P, shape, b, x_dtype=x_dtype)
    print(info, ref["iters"], flush=True)
    assert info["status"] == P.PCG_OK
    assert abs(info["iters"] - ref["iters"]) <= 2
    tr = orc.true_relres(shape, b64, host64(x))
    assert tr <= 1e-6
    assert abs(info["rel_res_true_fp64"] - tr) <= 1e-3 * tr
    # residual history follows the oracle's closely in the first iterations
    k = min(30, len(hist), len(ref["hist"]))
    assert np.all(np.abs(hist[:k] - ref["hist"][:k]) <= 1e-4 * ref["hist"][:k] + 1e-12)
    # solution agrees with the oracle's to what the tolerance allows
    xr = ref["x"]
    assert np.linalg.norm(host64(x) - xr) <= 1e-4 * np.linalg.norm(xr)


@pytest.mark.parametrize("shape", [(16, 16, 16), (23, 29, 37), (20, 12, 100), (64, 64, 64)])
def test_random_rhs_iterations(P, orc, shape):
    n = int(np.prod(shape))
    b, b64 = make_vec(21, n, torch.float32)
    ref = orc.pcg(shape, b64, rtol=1e-6, maxit=2000)
    _, x, info, _ = _solve(P, shape, b, maxit=2000, x_dtype=torch.float64)
    print(shape, info["iters"], ref["iters"], flush=True)
    assert info["status"] == P.PCG_OK
    assert abs(info["iters"] - ref["iters"]) <= 2
    assert orc.true_relres(shape, b64, host64(x)) <= 1e-6


def test_eigenvector_rhs(P):
    n = 16
    v = synthetic.sine_mode(n, n, n, 2, 1, 3).astype(np.float32)
    b = torch.from_numpy(v).cuda()
    _, x, info, hist = _solve(P, (n, n, n), b, rtol=1e-12, maxit=1, x_dtype=torch.float64)
    assert info["iters"] == 1 and info["status"] == P.PCG_E_NOCONV
    assert hist[1] <= 1e-4
    lam = 6 - 2 * (math.cos(2 * math.pi / 17) + math.cos(math.pi / 17) + math.cos(3 * math.pi / 17))
    assert np.max(np.abs(host64(x) - v / lam)) <= 1e-5 * np.max(np.abs(v / lam))


def test_zero_rhs(P):
    b = torch.zeros(4096, device="cuda")
    _, x, info, _ = _solve(P, (16, 16, 16), b)
    assert info["status"] == P.PCG_OK and info["iters"] == 0
    assert torch.count_nonzero(x).item() == 0


def test_nan_breakdown(P):
    b, _ = make_vec(3, 4096, torch.float32)
    b[100] = float("nan")
    _, _, info, _ = _solve(P, (16, 16, 16), b)
    assert info["status"] == P.PCG_E_BREAKDOWN


def test_maxit(P):
    b, _ = make_vec(3, 4096, torch.float32)
    _, _, info, hist = _solve(P, (16, 16, 16), b, rtol=1e-12, maxit=3)
    assert info["status"] == P.PCG_E_NOCONV and info["iters"] == 3 and len(hist) == 4
    with pytest.raises(P.PcgError):
        ctx = P.pcg_create(16, 16, 16)
        P.pcg_solve(ctx, b, torch.empty_like(b), 1e-12, 3)


@pytest.mark.parametrize("chunk", [2, 16, 64])
def test_graph_eager_timing_identical(P, chunk):
    """Captured graph chunks, eager launches and the event-timed mode run the
    same kernels in the same order: bit-identical results."""
    shape = (24, 40, 48)
    n = int(np.prod(shape))
    b, _ = make_vec(5, n, torch.float32)
    outs = []
    for opts in ({"use_graph": 1}, {"use_graph": 0}, {"kernel_timing": 1}, {"use_graph": 1}):
        _, x, info, _ = _solve(P, shape, b, x_dtype=torch.float64, chunk_iters=chunk, **opts)
        outs.append((info["iters"], host64(x).tobytes()))
        if opts.get("kernel_timing"):
            assert info["k1_ms"] > 0 and info["k2_ms"] > 0 and info["k1_launches"] >= info["iters"]
    assert all(o == outs[0] for o in outs)


@pytest.mark.parametrize("tile", [(64, 16), (128, 8), (256, 4), (64, 4), (64, 8)])
def test_tile_shapes_agree(P, orc, tile):
    shape = (30, 36, 72)
    n = int(np.prod(shape))
    b, b64 = make_vec(6, n, torch.float32)
    ref = orc.pcg(shape, b64, rtol=1e-6, maxit=1000)
    _, x, info, _ = _solve(P, shape, b, x_dtype=torch.float64, tile_x=tile[0], tile_y=tile[1], zchunk=5)
    assert abs(info["iters"] - ref["iters"]) <= 2
    assert orc.true_relres(shape, b64, host64(x)) <= 1e-6


def test_initial_guess(P, orc):
    shape = (20, 20, 20)
    b, b64 = make_vec(7, 8000, torch.float32)
    ref = orc.pcg(shape, b64, rtol=1e-9, maxit=1000)
    x0 = torch.from_numpy(ref["x"]).cuda()
    ctx = P.pcg_create(20, 20, 20, torch.float32, use_x0=1, x_dtype=torch.float64)
    info = P.pcg_solve(ctx, b, x0, 1e-6, 100)
    assert info["iters"] == 0
    # a half-way initial guess converges in fewer iterations than x0 = 0
    mid = orc.pcg(shape, b64, rtol=0.0, maxit=20)["x"]
    x1 = torch.from_numpy(mid).cuda()
    info = P.pcg_solve(ctx, b, x1, 1e-6, 1000)
    full = orc.pcg(shape, b64, rtol=1e-6, maxit=1000)["iters"]
    assert info["status"] == P.PCG_OK and info["iters"] < full
    assert orc.true_relres(shape, b64, host64(x1)) <= 1e-6


@pytest.mark.parametrize("dtype,floor", [(torch.bfloat16, 2e-2), (torch.float16, 2e-3)])
def test_low_precision_storage(P, orc, dtype, floor):
    """BF16/FP16 storage with FP32 arithmetic: the recursive residual reaches
    the reduced-precision regime; the FP64 true residual of the FP64
    accumulator is consistent with it."""
    shape = (32, 32, 32)
    b, b64 = make_vec(8, 32 ** 3, dtype)
    _, x, info, hist = _solve(P, shape, b, rtol=floor, maxit=500, x_dtype=torch.float64)
    check_status(P, info, floor)
    tr = orc.true_relres(shape, b64, host64(x))
    assert tr <= 20 * floor
    assert abs(info["rel_res_true_fp64"] - tr) <= 1e-6 + 1e-3 * tr


def test_deterministic_repeat(P):
    shape = (48, 48, 48)
    b, _ = make_vec(9, 48 ** 3, torch.float32)
    ctx = P.pcg_create(48, 48, 48, torch.float32)
    x1 = torch.empty_like(b)
    x2 = torch.empty_like(b)
    i1 = P.pcg_solve(ctx, b, x1, 1e-6, 1000, raise_on_error=False)
    i2 = P.pcg_solve(ctx, b, x2, 1e-6, 1000, raise_on_error=False)
    check_status(P, i1, 1e-6)
    assert i1["iters"] == i2["iters"] and torch.equal(x1, x2)


def test_fp64_residual_restart(P, orc):
    """rtol = 1e-7 is below what the FP32 recursion tracks faithfully at 40^3:
    with restarts from the FP64 residual the returned x has a true residual
    no worse than without them, and <= rtol unless all restarts were used."""
    shape = (40, 40, 40)
    n = 40 ** 3
    b, b64 = make_vec(23, n, torch.float32)
    _, x0, i0, _ = _solve(P, shape, b, rtol=1e-7, maxit=3000, x_dtype=torch.float64, max_restarts=0)
    _, x1, i1, _ = _solve(P, shape, b, rtol=1e-7, maxit=3000, x_dtype=torch.float64)
    t0 = orc.true_relres(shape, b64, host64(x0))
    t1 = orc.true_relres(shape, b64, host64(x1))
    print("no restart", i0["iters"], t0, "restarts", i1["restarts"], i1["iters"], t1, flush=True)
    assert i0["restarts"] == 0 and 0 <= i1["restarts"] <= 3
    check_status(P, i0, 1e-7)
    check_status(P, i1, 1e-7)
    assert t1 <= t0 * (1 + 1e-9)
    assert i1["restarts"] == 3 or t1 <= 1e-7
    assert abs(i1["rel_res_true_fp64"] - t1) <= 1e-6 * t1
    assert i1["iters"] >= i0["iters"]


def test_kernel_timing_counts_each_iteration_once(P, orc):
    """With a restart the per-kernel event sums still cover each iteration
    once: their total stays below the solve's wall time."""
    shape = (40, 40, 40)
    b, _ = make_vec(23, 40 ** 3, torch.float32)
    _, _, info, _ = _solve(P, shape, b, rtol=1e-7, maxit=3000, x_dtype=torch.float64, kernel_timing=1)
    assert info["k1_launches"] == info["iters"] == info["k2_launches"]
    assert info["k1_ms"] + info["k2_ms"] <= info["seconds"] * 1e3


@pytest.mark.parametrize("maxit", [7, 8, 2000])
@pytest.mark.parametrize("var", [False, True])
@pytest.mark.parametrize("use_graph", [1, 0])
def test_deferred_x_same_bits(P, orc, maxit, var, use_graph):
    """x advanced every second iteration (the default) against x advanced
    every iteration: the FP64 accumulator performs the same FP64 steps, so x
    is bit-identical, whether the run stops after an odd (7) or even (8)
    iteration count or at convergence (graph replays and eager launches)."""
    shape = (19, 24, 33)
    nz, ny, nx = shape
    n = nx * ny * nz
    b, b64 = make_vec(61, n, torch.float32)
    res = {}
    for defer in (1, 0):
        ctx = P.pcg_create(nx, ny, nz, torch.float32, x_dtype=torch.float64, x_defer=defer, use_graph=use_graph,
                           single_reduction=0)
        if var:
            k = torch.from_numpy(np.exp(synthetic.uniform_f32(62, n).astype(np.float64)).astype(np.float32)).cuda()
            P.pcg_set_coefficients(ctx, k)
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        info = P.pcg_solve(ctx, b, x, 1e-6, maxit, raise_on_error=False)
        res[defer] = (host64(x), info)
    (x1, i1), (x0, i0) = res[1], res[0]
    print(maxit, var, use_graph, i1["iters"], i0["iters"], i1["status"], flush=True)
    assert i1["iters"] == i0["iters"] and i1["status"] == i0["status"]
    assert np.array_equal(x1.view(np.uint64), x0.view(np.uint64))
    if maxit < 100:
        assert i1["iters"] == maxit and i1["status"] == P.PCG_E_NOCONV
    else:
        assert i1["status"] == P.PCG_OK
        if not var:
            assert orc.true_relres(shape, b64, x1) <= 1e-6


@pytest.mark.parametrize("storage", [torch.float32, torch.bfloat16])
def test_deferred_x_fp32_accumulator(P, orc, storage):
    """With an FP32 (or storage-type) accumulator the deferred form rounds x
    once per two steps instead of once per step: the recursion is unchanged
    (same iterations and residual history; no FP64 restarts, which read x)
    and x agrees to the accumulator's accuracy."""
    shape = (16, 20, 24)
    nz, ny, nx = shape
    n = nx * ny * nz
    b, b64 = make_vec(63, n, torch.float32)
    b = b.to(storage)
    out = {}
    for defer in (1, 0):
        ctx = P.pcg_create(nx, ny, nz, storage, x_accum=torch.float32, x_dtype=storage, x_defer=defer,
                           single_reduction=0, max_restarts=0)
        x = torch.empty(n, dtype=storage, device="cuda")
        info = P.pcg_solve(ctx, b, x, 1e-3, 500, raise_on_error=False)
        out[defer] = (x.double().cpu().numpy(), info, P.pcg_get_history(ctx))
    (x1, i1, h1), (x0, i0, h0) = out[1], out[0]
    assert i1["iters"] == i0["iters"]
    assert np.array_equal(h1, h0)
    tol = 2e-6 if storage == torch.float32 else 1e-2
    assert np.linalg.norm(x1 - x0) <= tol * np.linalg.norm(x0)
