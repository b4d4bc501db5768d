"""GPU parity of the FP64 iterative refinement around the reduced-precision
Jacobi-PCG. Bar: final FP64 true residual <= 1e-10 (recomputed on the CPU by
the oracle from the returned x), outer-step count within 1 of the oracle's
emulation of the same storage precision (inner counts are reported only).
"""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2603_23343_amd as P

    return P


def _system(orc, n):
    shape = (n, n, n)
    xs = synthetic.smooth_plus_noise(n)
    b = orc.stencil(xs, shape)
    return shape, xs, b


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("dtype,fmt", [(torch.bfloat16, "bf16"), (torch.float16, "f16")])
@pytest.mark.parametrize("acc", ["f32", "lp"])
def test_refined_matches_emulation(P, orc, n, dtype, fmt, acc):
    """Inner correction accumulated in FP32 (default) or in the storage type."""
    shape, xs, b = _system(orc, n)
    ref = orc.ir_emulate(shape, b, fmt=fmt, rtol_outer=1e-10, rtol_in=P.REFINE_RTOL_INNER[dtype],
                         d_fmt="f32" if acc == "f32" else None)
    ctx = P.pcg_create(n, n, n, dtype, x_accum=torch.float32 if acc == "f32" else dtype)
    b64 = torch.from_numpy(b).cuda()
    x64 = torch.empty_like(b64)
    info = P.pcg_solve_refined(ctx, b64, x64, rtol_outer=1e-10)
    rel, inner = P.pcg_refine_history(ctx)
    print(n, fmt, "gpu outer", info["outer_iters"], list(inner), "oracle", ref["outer"], ref["inner"], flush=True)
    assert info["status"] == P.PCG_OK
    tr = orc.true_relres(shape, b, x64.cpu().numpy())
    assert tr <= 1e-10
    assert abs(info["rel_res_true_fp64"] - tr) <= 1e-3 * tr + 1e-15
    assert abs(info["outer_iters"] - ref["outer"]) <= 1
    assert 0 < info["t_1e6"] <= info["t_1e10"] <= info["seconds"]
    assert np.linalg.norm(x64.cpu().numpy() - xs) <= 1e-6 * np.linalg.norm(xs)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16, torch.float32])
def test_refined_fp64_accumulator(P, orc, dtype):
    """The inner solution accumulated in FP64 also reaches 1e-10."""
    n = 24
    shape, _, b = _system(orc, n)
    ctx = P.pcg_create(n, n, n, dtype, x_accum=torch.float64)
    b64 = torch.from_numpy(b).cuda()
    x64 = torch.empty_like(b64)
    info = P.pcg_solve_refined(ctx, b64, x64, rtol_outer=1e-10)
    assert info["status"] == P.PCG_OK
    assert orc.true_relres(shape, b, x64.cpu().numpy()) <= 1e-10


def test_refined_zero_rhs_and_limits(P):
    n = 8
    ctx = P.pcg_create(n, n, n, torch.bfloat16, x_accum=torch.float32)
    b64 = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    x64 = torch.ones_like(b64)
    info = P.pcg_solve_refined(ctx, b64, x64)
    assert info["status"] == P.PCG_OK and info["outer_iters"] == 0
    assert torch.count_nonzero(x64).item() == 0
    b64 = torch.from_numpy(synthetic.uniform(3, n ** 3)).cuda()
    info = P.pcg_solve_refined(ctx, b64, x64, rtol_outer=1e-14, max_outer=1, raise_on_error=False)
    assert info["status"] == P.PCG_E_NOCONV and info["outer_iters"] == 1
    c64 = P.pcg_create(n, n, n, torch.float64)
    with pytest.raises(P.PcgError) as e:
        P.pcg_solve_refined(c64, b64, x64)
    assert e.value.status == P.PCG_E_UNSUPPORTED


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_refined_256(P, orc, dtype):
    """Full size: 256^3, b = A x* (x* = sine mode + 1e-3 noise). Property at
    any size: the FP64 true residual of the returned x, recomputed on the CPU,
    is <= 1e-10; the solution error is at the level the residual implies."""
    n = 256
    shape, xs, b = _system(orc, n)
    ctx = P.pcg_create(n, n, n, dtype, x_accum=torch.float32)
    b64 = torch.from_numpy(b).cuda()
    x64 = torch.empty_like(b64)
    info = P.pcg_solve_refined(ctx, b64, x64, rtol_outer=1e-10)
    print(dtype, {k: info[k] for k in ("outer_iters", "iters", "t_1e6", "t_1e10", "seconds")}, flush=True)
    assert info["status"] == P.PCG_OK
    x = x64.cpu().numpy()
    assert orc.true_relres(shape, b, x) <= 1e-10
    assert np.linalg.norm(x - xs) <= 1e-5 * np.linalg.norm(xs)
