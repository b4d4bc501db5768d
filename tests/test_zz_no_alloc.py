"""The allocation-free dot product (dot_noalloc) against the context-based
dot / dot_f64 through the C ABI: the same kernels and summation order, so the
same bits, on two calls in a row (the second on a smaller input, so stale
partials of the first call would show), and within the dot tolerance of the
FP64 oracle (|d - d_ref| <= 1e-5 sum |x_i y_i|)."""
import numpy as np
import pytest
import torch

from gpu_helpers import make_vec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2603_23343_amd as P

    return P


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, torch.float64])
def test_noalloc_dot_matches_dot(P, orc, dtype):
    ctx = P.pcg_create(1, 1, 1, dtype)
    for n, seed in ((3_000_017, 41), (40_009, 43)):
        print("dot_noalloc", dtype, n, flush=True)
        x, x64 = make_vec(seed, n, dtype)
        y, y64 = make_vec(seed + 1, n, dtype)
        ref64 = torch.zeros(1, dtype=torch.float64, device="cuda")
        ref32 = torch.zeros(1, dtype=torch.float32, device="cuda")
        P.dot_f64(ctx, n, x, y, ref64)
        P.dot(ctx, n, x, y, ref32)
        got64 = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
        got32 = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
        P.dot_noalloc(n, x, y, got64)
        P.dot_noalloc(n, x, y, got32)
        torch.cuda.synchronize()
        assert got64.item() == ref64.item()
        assert got32.item() == ref32.item()
        exact = orc.dot(x64, y64)
        assert abs(got64.item() - exact) <= 1e-5 * float(np.sum(np.abs(x64 * y64)))
    ctx.close()


def test_noalloc_dot_empty_and_stream(P):
    """n = 0 gives 0; a side stream runs the call on that stream."""
    out = torch.full((1,), 3.0, dtype=torch.float64, device="cuda")
    x = torch.zeros(4, dtype=torch.float32, device="cuda")
    P.dot_noalloc(0, x, x, out)
    torch.cuda.synchronize()
    assert out.item() == 0.0
    n = 100_003
    a, a64 = make_vec(45, n, torch.float32)
    b, b64 = make_vec(46, n, torch.float32)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    P.dot_noalloc(n, a, b, out, stream=side)
    side.synchronize()
    ctx = P.pcg_create(1, 1, 1, torch.float32)
    ref = torch.zeros(1, dtype=torch.float64, device="cuda")
    P.dot_f64(ctx, n, a, b, ref)
    torch.cuda.synchronize()
    assert out.item() == ref.item()
    ctx.close()
