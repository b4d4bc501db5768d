"""GPU parity of the single-reduction Jacobi-PCG (one fused kernel and one
grid reduction per iteration, Chronopoulos-Gear) against the FP64 oracle's
single-reduction form, through the C ABI.

Bars (as for the two-kernel form): iteration counts within 2 of the oracle;
FP64 true residual of the returned x <= 1e-6 for FP32 storage with the FP64
x accumulator; after a fixed small number of iterations the FP32 iterate
agrees with the FP64 oracle's to 1e-4 relative (FP32 rounding of the
vectors, amplified by at most a few steps); two solves are bit-identical.
"""
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


def _solve(P, shape, b, rtol=1e-6, maxit=500, x_dtype=torch.float64, **opts):
    nz, ny, nx = shape
    ctx = P.pcg_create(nx, ny, nz, b.dtype, x_dtype=x_dtype, single_reduction=1, **opts)
    x = torch.empty(b.numel(), dtype=x_dtype, device="cuda")
    info = P.pcg_solve(ctx, b, x, rtol, maxit, raise_on_error=False)
    hist = P.pcg_get_history(ctx)
    ctx.close()
    return x, info, hist


@pytest.mark.parametrize("shape", [(32, 32, 32), (11, 20, 37), (9, 13, 64), (64, 64, 64)])
def test_sr_iterations_and_residual(P, orc, shape):
    n = int(np.prod(shape))
    b, b64 = make_vec(synthetic.SEED_C1_B, n, torch.float32)
    print("sr", shape, flush=True)
    x, info, hist = _solve(P, shape, b, max_restarts=0)
    ref = orc.pcg_sr(shape, b64, rtol=1e-6, maxit=500, history=True)
    print(shape, "iters", info["iters"], "oracle", ref["iters"], flush=True)
    check_status(P, info, 1e-6)
    assert abs(info["iters"] - ref["iters"]) <= 2
    m = min(len(hist), len(ref["hist"]), 10)
    assert np.allclose(hist[:m], ref["hist"][:m], rtol=1e-4, atol=1e-7)
    x2, info2, _ = _solve(P, shape, b)
    tr = orc.true_relres(shape, b64, host64(x2))
    assert tr <= 1e-6
    assert abs(info2["rel_res_true_fp64"] - tr) <= 1e-6 * tr


@pytest.mark.parametrize("steps", [1, 2, 5])
def test_sr_fixed_steps_iterate(P, orc, steps):
    shape = (24, 20, 32)
    n = int(np.prod(shape))
    b, b64 = make_vec(7, n, torch.float32)
    x, info, _ = _solve(P, shape, b, rtol=0.0, maxit=steps, max_restarts=0)
    ref = orc.pcg_sr(shape, b64, rtol=0.0, maxit=steps)
    assert info["iters"] == steps == ref["iters"]
    got = host64(x)
    assert np.linalg.norm(got - ref["x"]) <= 1e-4 * np.linalg.norm(ref["x"])


def test_sr_agrees_with_two_kernel_form(P, orc):
    shape = (40, 36, 48)
    n = int(np.prod(shape))
    b, b64 = make_vec(3, n, torch.float32)
    x1, i1, _ = _solve(P, shape, b, max_restarts=0)
    nz, ny, nx = shape
    ctx = P.pcg_create(nx, ny, nz, torch.float32, x_dtype=torch.float64, single_reduction=0, max_restarts=0)
    x2 = torch.empty(n, dtype=torch.float64, device="cuda")
    i2 = P.pcg_solve(ctx, b, x2, 1e-6, 500)
    ctx.close()
    assert abs(i1["iters"] - i2["iters"]) <= 2
    assert torch.linalg.norm(x1 - x2).item() <= 1e-5 * torch.linalg.norm(x2).item()


def test_sr_deterministic_graph_and_eager(P):
    shape = (32, 32, 32)
    b, _ = make_vec(synthetic.SEED_C1_B, 32 ** 3, torch.float32)
    xa, ia, _ = _solve(P, shape, b)
    xb, ib, _ = _solve(P, shape, b)
    xc, ic, _ = _solve(P, shape, b, use_graph=0)
    xd, idd, _ = _solve(P, shape, b, kernel_timing=1)
    assert ia["iters"] == ib["iters"] == ic["iters"] == idd["iters"]
    assert torch.equal(xa, xb) and torch.equal(xa, xc) and torch.equal(xa, xd)
    assert idd["k1_launches"] == idd["iters"] and idd["k1_ms"] > 0.0


def test_sr_edge_cases(P, orc):
    shape = (16, 16, 16)
    n = 16 ** 3
    zero = torch.zeros(n, dtype=torch.float32, device="cuda")
    x, info, _ = _solve(P, shape, zero)
    assert info["status"] == P.PCG_OK and info["iters"] == 0 and not torch.any(x)
    b, b64 = make_vec(5, n, torch.float32)
    x, info, _ = _solve(P, shape, b, rtol=1e-12, maxit=3, max_restarts=0)
    assert info["status"] == P.PCG_E_NOCONV and info["iters"] == 3
    # one eigenvector: one step
    v = synthetic.sine_mode(16, 16, 16, 2, 1, 3)
    x, info, _ = _solve(P, shape, torch.from_numpy(v.astype(np.float32)).cuda(), rtol=1e-5, max_restarts=0)
    assert info["iters"] == 1
    # 1 x 1 x 1 and a single line
    for sh in ((1, 1, 1), (1, 1, 8), (5, 1, 1)):
        m = int(np.prod(sh))
        bb, bb64 = make_vec(2, m, torch.float32)
        x, info, _ = _solve(P, sh, bb, rtol=1e-6)
        assert orc.true_relres(sh, bb64, host64(x)) <= 1e-6


@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float16])
def test_sr_16bit_storage(P, orc, dt):
    shape = (32, 32, 32)
    n = 32 ** 3
    b, b64 = make_vec(synthetic.SEED_C1_B, n, dt)
    x, info, _ = _solve(P, shape, b, rtol=1e-3, x_accum=torch.float32, max_restarts=0)
    ref = orc.pcg_sr(shape, b64, rtol=1e-3, maxit=500)
    check_status(P, info, 1e-3)
    assert abs(info["iters"] - ref["iters"]) <= 2
    # drift of 16-bit r rounding (2^-9 BF16, 2^-12 FP16 per step), as for the two-kernel form
    assert orc.true_relres(shape, b64, host64(x)) <= 2e-2


def test_sr_refinement_reaches_1e10(P, orc):
    shape = (32, 32, 32)
    n = 32 ** 3
    b64 = synthetic.uniform(11, n)
    ctx = P.pcg_create(32, 32, 32, torch.bfloat16, x_accum=torch.float32, single_reduction=1)
    x64 = torch.empty(n, dtype=torch.float64, device="cuda")
    r = P.pcg_solve_refined(ctx, torch.from_numpy(b64).cuda(), x64, rtol_outer=1e-10)
    ctx.close()
    assert orc.true_relres(shape, b64, host64(x64)) <= 1e-10
    assert r["outer_iters"] >= 2


def test_sr_option_ignored_with_variable_coefficients(P, orc):
    """Variable coefficients keep the two-kernel form (the fused kernel is
    constant-coefficient only); the solve is still the oracle's."""
    n = 24
    shape = (n, n, n)
    k = np.exp(synthetic.gaussian_random_field(n)).astype(np.float32)
    kd = torch.from_numpy(k).cuda()
    b, b64 = make_vec(4, n ** 3, torch.float32)
    ctx = P.pcg_create(n, n, n, torch.float32, x_dtype=torch.float64, single_reduction=1, max_restarts=0)
    P.pcg_set_coefficients(ctx, kd)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = P.pcg_solve(ctx, b, x, 1e-6, 2000)
    ctx.close()
    ref = orc.pcg(shape, b64, rtol=1e-6, maxit=2000, kcell=k.astype(np.float64))
    assert abs(info["iters"] - ref["iters"]) <= 2


def test_sr_paper_comparison_grid(P, orc):
    nx, ny, nz = synthetic.PAPER_GRID
    shape = (nz, ny, nx)
    N = nx * ny * nz
    b32 = synthetic.uniform_f32(synthetic.SEED_PAPER_GRID_B, N)
    b = torch.from_numpy(b32).cuda()
    x, info, _ = _solve(P, shape, b, maxit=5000, max_restarts=0)
    ref = orc.pcg_sr(shape, b32.astype(np.float64), rtol=1e-6, maxit=5000)
    print("paper grid sr iters", info["iters"], "oracle", ref["iters"], flush=True)
    assert abs(info["iters"] - ref["iters"]) <= 2
