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
from gpu_helpers import dev, host64

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
