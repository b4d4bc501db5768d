"""GPU parity of the standalone kernels (stencil, axpy, dot) against the FP64
oracle, through the C ABI. Tolerances: FP32 stencil and axpy 1e-6 relative to
the absolute sum of the terms, FP32 dot 1e-5 relative to sum |x_i y_i|;
16-bit storage within one unit in the last place of the stored result (plus
the FP32 rounding bound); integer-valued data and axpy with alpha = 0.5 bit-exact.
"""
import math

import numpy as np
import pytest
import torch

import synthetic
from gpu_helpers import host64, make_vec, stencil_abs_bound, ulp

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.bfloat16, torch.float16, torch.float64]
SHAPES = [(8, 8, 8), (32, 32, 32), (17, 19, 96), (5, 33, 64), (23, 29, 37), (1, 1, 1), (3, 1, 130), (64, 40, 200)]


@pytest.fixture(scope="module")
def P():
    import paper_2603_23343_amd as P

    return P


def _tol_stencil(dtype, orc, x64, y_ref, shape):
    bound = stencil_abs_bound(orc, x64, shape)
    if dtype == torch.float64:
        return 1e-14 * bound
    base = 1e-6 * bound
    if dtype == torch.float32:
        return base
    return base + ulp(y_ref, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", SHAPES)
def test_stencil_random(P, orc, dtype, shape):
    nz, ny, nx = shape
    n = nx * ny * nz
    print(f"stencil {dtype} {shape}", flush=True)
    ctx = P.pcg_create(nx, ny, nz, dtype)
    x, x64 = make_vec(11, n, dtype)
    y = torch.empty_like(x)
    P.stencil_apply(ctx, x, y)
    torch.cuda.synchronize()
    ref = orc.stencil(x64, shape)
    err = np.abs(host64(y) - ref)
    tol = _tol_stencil(dtype, orc, x64, ref, shape)
    assert np.all(err <= tol), (float(err.max()), int(np.argmax(err - tol)))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("shape", [(16, 16, 16), (7, 9, 44), (23, 29, 37)])
def test_stencil_integers_exact(P, orc, dtype, shape):
    nz, ny, nx = shape
    n = nx * ny * nz
    lim = 16 if dtype in (torch.bfloat16, torch.float16) else 1 << 20
    ctx = P.pcg_create(nx, ny, nz, dtype)
    x, x64 = make_vec(12, n, dtype, kind="int", lo=-lim, hi=lim)
    y = torch.empty_like(x)
    P.stencil_apply(ctx, x, y)
    torch.cuda.synchronize()
    assert np.array_equal(host64(y), orc.stencil(x64, shape))


def test_stencil_sine_eigenvector(P):
    n = 64
    ctx = P.pcg_create(n, n, n, torch.float32)
    v = synthetic.sine_mode(n, n, n, 3, 5, 2)
    x = torch.from_numpy(v.astype(np.float32)).cuda()
    y = torch.empty_like(x)
    P.stencil_apply(ctx, x, y)
    lam = 6 - 2 * (math.cos(3 * math.pi / (n + 1)) + math.cos(5 * math.pi / (n + 1)) + math.cos(2 * math.pi / (n + 1)))
    got = host64(y)
    xs = host64(x)
    assert np.max(np.abs(got - lam * xs)) <= 1e-6 * 12 * np.max(np.abs(xs))


@pytest.mark.parametrize("tile", [(64, 16), (128, 8), (256, 4), (64, 4), (64, 8)])
@pytest.mark.parametrize("zchunk", [1, 3, 16])
def test_stencil_all_tile_shapes(P, orc, tile, zchunk):
    """Every compiled work-group shape and z-chunk length gives the exact
    result on integer data (ragged tiles in x, y and z)."""
    shape = (37, 45, 260)
    nz, ny, nx = shape
    n = nx * ny * nz
    ctx = P.pcg_create(nx, ny, nz, torch.float32, tile_x=tile[0], tile_y=tile[1], zchunk=zchunk)
    x, x64 = make_vec(13, n, torch.float32, kind="int", lo=-1000, hi=1000)
    y = torch.empty_like(x)
    P.stencil_apply(ctx, x, y)
    torch.cuda.synchronize()
    assert np.array_equal(host64(y), orc.stencil(x64, shape))


def test_stencil_rejects_aliasing(P):
    ctx = P.pcg_create(8, 8, 8, torch.float32)
    x = torch.zeros(512, device="cuda")
    with pytest.raises(P.PcgError) as e:
        P.stencil_apply(ctx, x, x)
    assert e.value.status == P.PCG_E_ARG
    with pytest.raises(P.PcgError):
        P.stencil_apply(ctx, x[4:], x[:508])


# ---------------------------------------------------------------- axpy

@pytest.mark.parametrize("n", [0, 1, 3, 4, 7, 8, 255, 32768, 1000003])
def test_axpy_half_exact_f32(P, orc, n):
    ctx = P.pcg_create(1, 1, 1, torch.float32)
    x, x64 = make_vec(2, n, torch.float32)
    y, y64 = make_vec(3, n, torch.float32)
    z = torch.empty_like(x)
    P.axpy(ctx, n, 0.5, x, y, z)
    torch.cuda.synchronize()
    ref = orc.axpy(0.5, x64, y64).astype(np.float32)
    assert np.array_equal(z.cpu().numpy(), ref)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_axpy_half_16bit(P, orc, dtype):
    """16-bit storage: FP32 arithmetic then one rounding to the storage type,
    which is exactly the oracle's FP64 -> FP32 -> 16-bit rounding of the exact
    result (0.5 x + y is exact in FP64 and rounded once to FP32)."""
    n = 100003
    ctx = P.pcg_create(1, 1, 1, dtype)
    x, x64 = make_vec(2, n, dtype)
    y, y64 = make_vec(3, n, dtype)
    z = torch.empty_like(x)
    P.axpy(ctx, n, 0.5, x, y, z)
    rnd = orc.round_bf16 if dtype == torch.bfloat16 else orc.round_f16
    assert np.array_equal(host64(z), rnd(orc.axpy(0.5, x64, y64)))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_axpy_general_alpha(P, orc, dtype):
    n = 123457
    ctx = P.pcg_create(1, 1, 1, dtype)
    x, x64 = make_vec(4, n, dtype)
    y, y64 = make_vec(5, n, dtype)
    z = torch.empty_like(x)
    alpha = -0.7310585786
    # alpha is rounded once to the arithmetic type: FP32 for FP32 storage,
    # unrounded for FP64 storage
    a_used = float(np.float32(alpha)) if dtype == torch.float32 else alpha
    P.axpy(ctx, n, alpha, x, y, z)
    ref = orc.axpy(a_used, x64, y64)
    tol = (1e-6 if dtype == torch.float32 else 1e-15) * (np.abs(a_used * x64) + np.abs(y64))
    assert np.all(np.abs(host64(z) - ref) <= tol)


def test_axpy_in_place(P, orc):
    n = 50001
    ctx = P.pcg_create(1, 1, 1, torch.float32)
    x, x64 = make_vec(6, n, torch.float32)
    y, y64 = make_vec(7, n, torch.float32)
    P.axpy(ctx, n, 0.5, x, y, y)  # y = 0.5 x + y
    ref = orc.axpy(0.5, x64, y64).astype(np.float32)
    assert np.array_equal(y.cpu().numpy(), ref)
    P.axpy(ctx, n, 0.5, x, y, x)  # x = 0.5 x + y
    assert np.array_equal(x.cpu().numpy(), orc.axpy(0.5, x64, ref.astype(np.float64)).astype(np.float32))
    with pytest.raises(P.PcgError):
        P.axpy(ctx, n - 4, 0.5, x, y, x[4:])


# ---------------------------------------------------------------- dot

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [0, 1, 5, 4096, 32768, 1048583])
def test_dot_random(P, orc, dtype, n):
    ctx = P.pcg_create(1, 1, 1, dtype)
    x, x64 = make_vec(2, n, dtype)
    y, y64 = make_vec(3, n, dtype)
    out = torch.zeros(1, dtype=torch.float32, device="cuda")
    out64 = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.dot(ctx, n, x, y, out)
    P.dot_f64(ctx, n, x, y, out64)
    ref = orc.dot(x64, y64)
    scale = float(np.sum(np.abs(x64 * y64)))
    tol = (1e-13 if dtype == torch.float64 else 1e-5) * scale
    assert abs(float(out64.item()) - ref) <= tol
    assert abs(float(out.item()) - ref) <= tol + abs(ref) * 2 ** -24


@pytest.mark.parametrize("n,density", [(32768, 1.0), (1 << 22, 1.0), ((1 << 24) + 13, 1 / 16)])
def test_dot_integers_exact(P, orc, n, density):
    ctx = P.pcg_create(1, 1, 1, torch.float32)
    x, x64 = make_vec(8, n, torch.float32, kind="int", lo=-2 if n < 1e5 else -1, hi=2 if n < 1e5 else 1,
                      density=density)
    y, y64 = make_vec(9, n, torch.float32, kind="int", lo=-2 if n < 1e5 else -1, hi=2 if n < 1e5 else 1)
    out64 = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.dot_f64(ctx, n, x, y, out64)
    assert float(out64.item()) == orc.dot(x64, y64)


def test_dot_deterministic(P):
    n = 3 * 10 ** 6 + 7
    ctx = P.pcg_create(1, 1, 1, torch.float32)
    x, _ = make_vec(10, n, torch.float32)
    y, _ = make_vec(11, n, torch.float32)
    outs = []
    for _ in range(5):
        o = torch.zeros(1, dtype=torch.float64, device="cuda")
        P.dot_f64(ctx, n, x, y, o)
        outs.append(o.item())
    assert len(set(outs)) == 1
