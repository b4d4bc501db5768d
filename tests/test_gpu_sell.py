"""GPU parity of the sliced-ELLPACK SpMV (pcg_sell_*) against the oracle's
compressed-row SpMV, through the C ABI.

Tolerance, per row of n entries: each of the n fused multiply-adds in FP32
rounds once, so |y - y_ref| <= gamma_n sum_j |a_ij x_j| with gamma_n =
n u / (1 - n u), u = 2^-24 (the oracle's FP64 sum is exact to far below that
on these FP32 inputs); the test uses 1.01 n u. Integer-valued matrices and
vectors whose partial sums stay below 2^24 are bit-exact.
"""
import numpy as np
import pytest
import torch

import synthetic
from gpu_helpers import check_status, dev, host64

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def P():
    import paper_2603_23343_amd as P

    return P


def _abs_bound(orc, rowptr, col, val, x64):
    return orc.csr_spmv(rowptr, col, np.abs(val.astype(np.float64)), np.abs(x64))


def _check(P, orc, rowptr, col, val, ncols, sigma, x32, exact=False):
    nrows = rowptr.size - 1
    A = P.pcg_sell_create(rowptr, col, val, ncols, sigma=sigma)
    x = dev(x32)
    y = torch.full((max(nrows, 1),), float("nan"), dtype=torch.float32, device="cuda")
    P.pcg_sell_spmv(A, x, y)
    torch.cuda.synchronize()
    x64 = x32.astype(np.float64)
    ref = orc.csr_spmv(rowptr, col, val, x64)
    got = host64(y)[:nrows]
    if exact:
        assert np.array_equal(got, ref)
    else:
        lens = np.maximum(np.diff(rowptr), 1).astype(np.float64)
        tol = 1.01 * lens * U32 * _abs_bound(orc, rowptr, col, val, x64)
        err = np.abs(got - ref)
        assert np.all(err <= tol), (float(err.max()), int(np.argmax(err - tol)))
    A.close()
    return got


@pytest.mark.parametrize("sigma", [1, 64, 512])
@pytest.mark.parametrize("dims", [(33, 17, 9), (32, 32, 32), (1, 1, 130), (7, 3, 1)])
def test_poisson_matrix(P, orc, dims, sigma):
    nx, ny, nz = dims
    print(f"sell poisson {dims} sigma {sigma}", flush=True)
    rowptr, col, val = synthetic.poisson7_csr(nx, ny, nz)
    n = nx * ny * nz
    _check(P, orc, rowptr, col, val, n, sigma, synthetic.uniform_f32(11, n))


@pytest.mark.parametrize("sigma", [1, 64, 1024])
@pytest.mark.parametrize("nrows,ncols,max_len,empty", [(10001, 7919, 40, 0.05), (4096, 20000, 3, 0.0),
                                                       (130, 130, 200, 0.5), (1, 5, 5, 0.0)])
def test_random_ragged_matrix(P, orc, nrows, ncols, max_len, empty, sigma):
    print(f"sell random {nrows}x{ncols} len<={max_len} empty {empty} sigma {sigma}", flush=True)
    rowptr, col, val = synthetic.random_csr(nrows, ncols, seed=41, max_len=max_len, empty_frac=empty)
    _check(P, orc, rowptr, col, val, ncols, sigma, synthetic.uniform_f32(12, ncols))


@pytest.mark.parametrize("sigma", [1, 256])
def test_integers_bit_exact(P, orc, sigma):
    print(f"sell integers sigma {sigma}", flush=True)
    rowptr, col, val = synthetic.random_csr(6007, 5003, seed=43, max_len=64, empty_frac=0.1, integer=True)
    x32 = synthetic.integers(13, 5003, -4, 4)
    _check(P, orc, rowptr, col, val, 5003, sigma, x32, exact=True)


def test_all_rows_empty_and_no_rows(P, orc):
    rowptr = np.zeros(101, dtype=np.int64)
    got = _check(P, orc, rowptr, np.zeros(0, np.int32), np.zeros(0, np.float32), 7, 64,
                 synthetic.uniform_f32(3, 7), exact=True)
    assert np.all(got == 0)
    A = P.pcg_sell_create(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 3)
    x = torch.ones(3, dtype=torch.float32, device="cuda")
    y = torch.ones(1, dtype=torch.float32, device="cuda")
    P.pcg_sell_spmv(A, x, y)  # no rows: nothing written
    torch.cuda.synchronize()
    assert float(y[0]) == 1.0
    A.close()


def test_overlap_rejected(P):
    rowptr, col, val = synthetic.poisson7_csr(8, 8, 8)
    A = P.pcg_sell_create(rowptr, col, val, 512)
    buf = torch.zeros(1024, dtype=torch.float32, device="cuda")
    with pytest.raises(P.PcgError):
        P.pcg_sell_spmv(A, buf[:512], buf[256:768])
    A.close()


@pytest.mark.parametrize("dims", [(256, 256, 256), synthetic.PAPER_GRID])
def test_poisson_full_size(P, orc, dims):
    """The seven-point matrix at the benchmark's sizes (256^3 and the paper's
    512 x 112 x 64 comparison grid), sigma = 1 as the benchmark times it,
    every row against the oracle."""
    nx, ny, nz = dims
    print(f"sell full size {dims}", flush=True)
    rowptr, col, val = synthetic.poisson7_csr(nx, ny, nz)
    n = nx * ny * nz
    _check(P, orc, rowptr, col, val, n, 1, synthetic.uniform_f32(synthetic.SEED_C2_X, n))


# ---------------------------------------------------------------------------
# Jacobi-PCG on the stored matrix (pcg_sell_solve) against the oracle's
# compressed-row Jacobi-PCG: iterations within 2 and the FP64 true residual
# at or below rtol (the reading for FP32 storage with an FP64 x accumulator).
# ---------------------------------------------------------------------------

def _solve_pair(P, orc, rowptr, col, val, b32, rtol, maxit, sigma, restarts=-1, with_oracle=True):
    """The GPU solve (FP64-residual restarts: -1 default, 0 none) and the
    oracle's compressed-row Jacobi-PCG of the same system."""
    n = rowptr.size - 1
    A = P.pcg_sell_create(rowptr, col, val, n, sigma=sigma)
    P.pcg_sell_set_restarts(A, restarts)
    b = dev(b32)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    got = P.pcg_sell_solve(A, b, x, rtol, maxit, raise_on_error=False)
    torch.cuda.synchronize()
    ref = orc.csr_pcg(rowptr, col, val, b32.astype(np.float64), rtol=rtol, maxit=maxit) if with_oracle else None
    xh = x.cpu().numpy()
    A.close()
    return got, ref, xh


def _parity_then_restarted(P, orc, rowptr, col, val, b32, rtol, maxit, sigma):
    """Iterations within 2 of the oracle's with restarts off (the oracle
    stops on its recursion too), then the default solve: PCG_OK and an FP64
    true residual <= rtol."""
    got0, ref, _ = _solve_pair(P, orc, rowptr, col, val, b32, rtol, maxit, sigma, restarts=0)
    assert ref["status"] == orc.OK
    assert got0["restarts"] == 0
    check_status(P, got0, rtol)
    assert abs(got0["iters"] - ref["iters"]) <= 2, (got0["iters"], ref["iters"])
    got, _, x = _solve_pair(P, orc, rowptr, col, val, b32, rtol, maxit, sigma, with_oracle=False)
    assert got["status"] == P.PCG_OK and got["rel_res_true_fp64"] <= rtol
    assert got["iters"] >= got0["iters"]
    return got, x


@pytest.mark.parametrize("sigma", [1, 64])
@pytest.mark.parametrize("dims", [(32, 32, 32), (33, 17, 9)])
def test_sell_pcg_poisson(P, orc, dims, sigma):
    nx, ny, nz = dims
    n = nx * ny * nz
    print(f"sell pcg poisson {dims} sigma {sigma}", flush=True)
    rowptr, col, val = synthetic.poisson7_csr(nx, ny, nz)
    b32 = synthetic.uniform_f32(synthetic.SEED_C1_B, n)
    got, x = _parity_then_restarted(P, orc, rowptr, col, val, b32, 1e-6, 500, sigma)
    r = b32.astype(np.float64) - orc.csr_spmv(rowptr, col, val, x)
    assert np.linalg.norm(r) <= 1e-6 * np.linalg.norm(b32.astype(np.float64)) * (1 + 1e-9)


@pytest.mark.parametrize("sigma", [1, 256])
@pytest.mark.parametrize("n,partners", [(10007, 12), (777, 40), (1, 1)])
def test_sell_pcg_random_spd(P, orc, n, partners, sigma):
    print(f"sell pcg random spd n {n} partners {partners} sigma {sigma}", flush=True)
    if n == 1:
        rowptr, col, val = np.array([0, 1], np.int64), np.array([0], np.int32), np.array([4.0], np.float32)
    else:
        rowptr, col, val = synthetic.random_spd_csr(n, seed=51, max_partners=partners)
    b32 = synthetic.uniform_f32(52, n)
    _parity_then_restarted(P, orc, rowptr, col, val, b32, 1e-6, 1000, sigma)


def test_sell_pcg_status_paths(P, orc):
    rowptr, col, val = synthetic.random_spd_csr(500, seed=53)
    # b = 0: x = 0 at once
    got, ref, x = _solve_pair(P, orc, rowptr, col, val, np.zeros(500, np.float32), 1e-6, 100, 1)
    assert got["status"] == P.PCG_OK and got["iters"] == 0 and np.all(x == 0)
    # maxit reached: the oracle's count exactly
    b32 = synthetic.uniform_f32(54, 500)
    got, ref, x = _solve_pair(P, orc, rowptr, col, val, b32, 1e-14, 3, 1)
    assert got["status"] == P.PCG_E_NOCONV and ref["status"] == orc.NOCONV and got["iters"] == ref["iters"] == 3
    # a matrix with a non-positive diagonal is rejected before any iteration
    A = P.pcg_sell_create(rowptr, col, -val, 500)
    with pytest.raises(P.PcgError):
        P.pcg_sell_solve(A, dev(b32), torch.zeros(500, dtype=torch.float64, device="cuda"))
    A.close()
    # indefinite matrix with a positive diagonal: breakdown (p.Ap <= 0)
    ind_val = val.copy()
    off = col != np.repeat(np.arange(500), np.diff(rowptr))
    ind_val[off] *= 50.0
    got, ref, x = _solve_pair(P, orc, rowptr, col, ind_val, b32, 1e-10, 500, 1)
    assert ref["status"] == orc.BREAKDOWN
    assert got["status"] == P.PCG_E_BREAKDOWN and abs(got["iters"] - ref["iters"]) <= 2


def test_sell_pcg_full_size(P, orc):
    """The stored seven-point matrix at 256^3 with the benchmark's b (b = A x*,
    x* = lowest sine mode + 1e-3 noise): the same iteration count as the
    matrix-free solve within 2 per segment, and the FP64 true residual at or
    below 1e-6 checked by the oracle's product."""
    n1 = 256
    n = n1 ** 3
    print("sell pcg full size 256^3", flush=True)
    rowptr, col, val = synthetic.poisson7_csr(n1, n1, n1)
    xs = synthetic.smooth_plus_noise(n1)
    b32 = orc.stencil(xs, (n1, n1, n1)).astype(np.float32)
    A = P.pcg_sell_create(rowptr, col, val, n)
    b = dev(b32)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    got = P.pcg_sell_solve(A, b, x, 1e-6, 5000)
    torch.cuda.synchronize()
    ctx = P.pcg_create(n1, n1, n1, torch.float32, x_dtype=torch.float64)
    x2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    mf = P.pcg_solve(ctx, b, x2, 1e-6, 5000)
    P.pcg_destroy(ctx)
    assert abs(got["iters"] - mf["iters"]) <= 2 * (1 + got["restarts"] + mf["restarts"]), (got["iters"], mf["iters"])
    r = b32.astype(np.float64) - orc.csr_spmv(rowptr, col, val, x.cpu().numpy())
    rel = np.linalg.norm(r) / np.linalg.norm(b32.astype(np.float64))
    assert rel <= 1e-6 and abs(rel - got["rel_res_true_fp64"]) <= 1e-9
    A.close()


def test_sell_pcg_graph_replay_matches_eager(P, orc):
    """Graph-replayed batches give the eager launches' bits: three solves
    each way on one handle, with other GPU work in between, and a second x
    buffer (recapture)."""
    rowptr, col, val = synthetic.random_spd_csr(20011, seed=55)
    n = rowptr.size - 1
    b = dev(synthetic.uniform_f32(56, n))
    A = P.pcg_sell_create(rowptr, col, val, n, sigma=64)
    xs = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(2)]
    P.pcg_sell_set_graph(A, False)
    ref = P.pcg_sell_solve(A, b, xs[0], 1e-6, 500)
    xe = xs[0].clone()
    P.pcg_sell_set_graph(A, True)
    for rep in range(3):
        for x in xs:
            x.fill_(float("nan"))
            got = P.pcg_sell_solve(A, b, x, 1e-6, 500)
            torch.cuda.synchronize()
            assert got["iters"] == ref["iters"] and got["restarts"] == ref["restarts"]
            assert torch.equal(x, xe), rep
            _ = (b * 2.0).sum().item()  # unrelated eager work between replays
    A.close()


@pytest.fixture(scope="module")
def large_spd():
    return synthetic.random_spd_csr(2_000_000, seed=57)


@pytest.mark.parametrize("sigma", [1, 4096])
def test_random_spd_large_ragged(P, orc, large_spd, sigma):
    """2 M rows of 3..35 entries (28 M entries): every row of the product
    against the oracle with sigma = 1 (1.7x padding) and sigma = 4096 (sorted
    windows, 1.5% padding), then Jacobi-PCG against the oracle's."""
    rowptr, col, val = large_spd
    n = rowptr.size - 1
    print(f"sell large ragged spd sigma {sigma}", flush=True)
    _check(P, orc, rowptr, col, val, n, sigma, synthetic.uniform_f32(58, n))
    b32 = synthetic.uniform_f32(59, n)
    _parity_then_restarted(P, orc, rowptr, col, val, b32, 1e-6, 500, sigma)


def test_sell_on_a_side_stream(P, orc):
    """A handle bound to its own stream runs the product and the solve there."""
    rowptr, col, val = synthetic.random_spd_csr(30011, seed=60)
    n = rowptr.size - 1
    x32 = synthetic.uniform_f32(61, n)
    b32 = synthetic.uniform_f32(62, n)
    x, b = dev(x32), dev(b32)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    xs = torch.zeros(n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    A = P.pcg_sell_create(rowptr, col, val, n, sigma=256, stream=side)
    P.pcg_sell_spmv(A, x, y)
    side.synchronize()
    ref = orc.csr_spmv(rowptr, col, val, x32.astype(np.float64))
    lens = np.maximum(np.diff(rowptr), 1).astype(np.float64)
    tol = 1.01 * lens * U32 * _abs_bound(orc, rowptr, col, val, x32.astype(np.float64))
    assert np.all(np.abs(host64(y) - ref) <= tol)
    P.pcg_sell_set_restarts(A, 0)
    got = P.pcg_sell_solve(A, b, xs, 1e-6, 500, raise_on_error=False)
    oref = orc.csr_pcg(rowptr, col, val, b32.astype(np.float64), rtol=1e-6, maxit=500)
    check_status(P, got, 1e-6)
    assert got["restarts"] == 0 and abs(got["iters"] - oref["iters"]) <= 2
    P.pcg_sell_set_restarts(A, -1)
    got = P.pcg_sell_solve(A, b, xs, 1e-6, 500)
    assert got["status"] == P.PCG_OK and got["rel_res_true_fp64"] <= 1e-6
    A.close()
