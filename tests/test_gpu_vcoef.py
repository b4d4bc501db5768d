"""GPU parity of the variable-coefficient operator -div(k grad u) (harmonic-mean
faces, boundary face k_f = k_p, zero Dirichlet ghosts) and of Jacobi-PCG on
it, against the FP64 oracle, through the C ABI.

Tolerances: FP32 apply within 2e-6 of sum_f k_f (|u_p| + |u_nb|) per point
(the harmonic mean adds three FP32 roundings per face to the stencil's);
FP64 within 1e-14 of the same sum; integer data with k = 1 or k = 4 exact;
PCG iterations within 2 of the oracle and FP64 true residual <= rtol.
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


def _kfield(n_or_shape, seed=6, grf=True):
    shape = n_or_shape if isinstance(n_or_shape, tuple) else (n_or_shape,) * 3
    if grf and shape[0] == shape[1] == shape[2]:
        return synthetic.coefficient_field(shape[0], seed)
    return np.exp(synthetic.uniform(seed, int(np.prod(shape)))).astype(np.float32)


def _abs_bound(orc, k64, u64, shape):
    au = np.abs(u64)
    return 2.0 * orc.vdiag(k64, shape) * au - orc.vstencil(k64, au, shape)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("shape", [(16, 16, 16), (23, 29, 37), (5, 33, 64), (64, 64, 64)])
def test_vstencil_random(P, orc, dtype, shape):
    nz, ny, nx = shape
    n = nx * ny * nz
    k32 = _kfield(shape, grf=shape[0] == shape[1] == shape[2])
    k64 = k32.astype(np.float64)
    ctx = P.pcg_create(nx, ny, nz, dtype)
    kd = torch.from_numpy(k32).cuda()
    P.pcg_set_coefficients(ctx, kd)
    x, x64 = make_vec(11, n, dtype)
    y = torch.empty_like(x)
    P.stencil_apply(ctx, x, y)
    ref = orc.vstencil(k64, x64, shape)
    tol = (2e-6 if dtype == torch.float32 else 1e-14) * _abs_bound(orc, k64, x64, shape)
    err = np.abs(host64(y) - ref)
    assert np.all(err <= tol), float(np.max(err - tol))


@pytest.mark.parametrize("kval", [1.0, 4.0])
def test_vstencil_constant_k_exact(P, orc, kval):
    shape = (17, 19, 44)
    nz, ny, nx = shape
    n = nx * ny * nz
    ctx = P.pcg_create(nx, ny, nz, torch.float32)
    kd = torch.full((n,), kval, dtype=torch.float32, device="cuda")
    P.pcg_set_coefficients(ctx, kd)
    x, x64 = make_vec(12, n, torch.float32, kind="int", lo=-1000, hi=1000)
    y = torch.empty_like(x)
    P.stencil_apply(ctx, x, y)
    assert np.array_equal(host64(y), kval * orc.stencil(x64, shape))
    P.pcg_set_coefficients(ctx, None)
    P.stencil_apply(ctx, x, y)
    assert np.array_equal(host64(y), orc.stencil(x64, shape))


def test_vcoef_unsupported_16bit(P):
    ctx = P.pcg_create(8, 8, 8, torch.bfloat16)
    kd = torch.ones(512, device="cuda")
    with pytest.raises(P.PcgError) as e:
        P.pcg_set_coefficients(ctx, kd)
    assert e.value.status == P.PCG_E_UNSUPPORTED


@pytest.mark.parametrize("n", [24, 48])
def test_vcoef_pcg_fp32(P, orc, n):
    shape = (n, n, n)
    k32 = _kfield(n)
    k64 = k32.astype(np.float64)
    b, b64 = make_vec(31, n ** 3, torch.float32)
    ref = orc.pcg(shape, b64, rtol=1e-6, maxit=3000, kcell=k64)
    ctx = P.pcg_create(n, n, n, torch.float32, x_dtype=torch.float64)
    kd = torch.from_numpy(k32).cuda()
    P.pcg_set_coefficients(ctx, kd)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = P.pcg_solve(ctx, b, x, 1e-6, 3000, raise_on_error=False)
    print(n, info["iters"], ref["iters"], flush=True)
    assert info["status"] == P.PCG_OK
    assert abs(info["iters"] - ref["iters"]) <= 2
    tr = orc.true_relres(shape, b64, x.cpu().numpy(), kcell=k64)
    assert tr <= 1e-6
    assert abs(info["rel_res_true_fp64"] - tr) <= 1e-3 * tr


def test_vcoef_pcg_fp64(P, orc):
    n = 32
    shape = (n, n, n)
    k32 = _kfield(n)
    k64 = k32.astype(np.float64)
    b, b64 = make_vec(32, n ** 3, torch.float64)
    ref = orc.pcg(shape, b64, rtol=1e-10, maxit=5000, kcell=k64)
    ctx = P.pcg_create(n, n, n, torch.float64)
    kd = torch.from_numpy(k32).cuda()
    P.pcg_set_coefficients(ctx, kd)
    x = torch.empty_like(b)
    info = P.pcg_solve(ctx, b, x, 1e-10, 5000, raise_on_error=False)
    check_status(P, info, 1e-10)
    assert abs(info["iters"] - ref["iters"]) <= 2
    assert orc.true_relres(shape, b64, x.cpu().numpy(), kcell=k64) <= 1.5e-10
    assert np.max(np.abs(x.cpu().numpy() - ref["x"])) <= 1e-8 * np.max(np.abs(ref["x"]))


def test_vcoef_unit_k_matches_constant_solver(P):
    """k = 1 everywhere: the variable-coefficient solver reproduces the
    constant-coefficient one (same iterations; iterates equal to rounding)."""
    n = 32
    b, _ = make_vec(33, n ** 3, torch.float32)
    c1 = P.pcg_create(n, n, n, torch.float32, x_dtype=torch.float64)
    c2 = P.pcg_create(n, n, n, torch.float32, x_dtype=torch.float64)
    kd = torch.ones(n ** 3, dtype=torch.float32, device="cuda")
    P.pcg_set_coefficients(c2, kd)
    x1 = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    x2 = torch.empty_like(x1)
    i1 = P.pcg_solve(c1, b, x1, 1e-6, 500)
    i2 = P.pcg_solve(c2, b, x2, 1e-6, 500)
    assert abs(i1["iters"] - i2["iters"]) <= 1
    assert torch.max(torch.abs(x1 - x2)).item() <= 1e-5 * torch.max(torch.abs(x1)).item()
