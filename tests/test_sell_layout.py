"""Host checks of the library's sliced-ELLPACK layout (pcg_sell_build makes
no GPU call): every row kept in storage order, the sorting inside sigma
windows, the chunk widths, and the product read back through the layout
against the oracle's compressed-row SpMV.
"""
import numpy as np
import pytest

import synthetic


@pytest.fixture(scope="module")
def P():
    import paper_2603_23343_amd as P

    return P


def _sell_rows(L, chunk, nrows):
    """Rebuild each original row's (columns, values) from the layout."""
    out = {}
    cp = L["chunk_ptr"]
    for s in range(nrows):
        c, l = divmod(s, chunk)
        w = (cp[c + 1] - cp[c]) // chunk
        slots = cp[c] + np.arange(w) * chunk + l
        cols, vals = L["col"][slots], L["val"][slots]
        n = int(np.sum(cols >= 0))
        assert np.all(cols[:n] >= 0) and np.all(cols[n:] == -1) and np.all(vals[n:] == 0)
        out[int(L["perm"][s])] = (cols[:n], vals[:n])
    return out


@pytest.mark.parametrize("chunk,sigma", [(4, 1), (4, 8), (8, 32), (64, 64), (1, 1)])
def test_sell_layout_keeps_every_row(P, chunk, sigma):
    nrows, ncols = 203, 150
    rowptr, col, val = synthetic.random_csr(nrows, ncols, seed=31, max_len=20, empty_frac=0.1)
    L = P.pcg_sell_build(rowptr, col, val, ncols, chunk=chunk, sigma=sigma)
    lens = np.diff(rowptr)
    perm = L["perm"]
    nch = (nrows + chunk - 1) // chunk
    assert L["chunk_ptr"].size == nch + 1 and L["chunk_ptr"][0] == 0
    # perm is a permutation of each sigma window, sorted by decreasing length, stable
    for w0 in range(0, nrows, sigma):
        win = perm[w0:w0 + sigma]
        assert sorted(win.tolist()) == list(range(w0, min(w0 + sigma, nrows)))
        key = [(-int(lens[r]), int(r)) for r in win]
        assert key == sorted(key)
    # chunk widths are the longest row of the chunk
    for c in range(nch):
        rows = perm[c * chunk:(c + 1) * chunk]
        w = (L["chunk_ptr"][c + 1] - L["chunk_ptr"][c]) // chunk
        assert w == (lens[rows].max() if rows.size else 0)
    rows = _sell_rows(L, chunk, nrows)
    assert sorted(rows) == list(range(nrows))
    for r in range(nrows):
        cols, vals = rows[r]
        assert np.array_equal(cols, col[rowptr[r]:rowptr[r + 1]])
        assert np.array_equal(vals, val[rowptr[r]:rowptr[r + 1]])


def test_sell_layout_product_matches_oracle(P, orc):
    """The product read back through the layout (FP64 on the host) equals the
    oracle's compressed-row product."""
    rowptr, col, val = synthetic.poisson7_csr(9, 5, 3)
    n = 9 * 5 * 3
    x = synthetic.uniform(6, n)
    L = P.pcg_sell_build(rowptr, col, val, n, chunk=16, sigma=32)
    y = np.zeros(n)
    for r, (cols, vals) in _sell_rows(L, 16, n).items():
        y[r] = float(np.dot(vals.astype(np.float64), x[cols]))
    assert np.max(np.abs(y - orc.csr_spmv(rowptr, col, val, x))) <= 1e-14


def test_sell_build_rejects_bad_input(P):
    rowptr = np.array([0, 2, 1], dtype=np.int64)
    with pytest.raises(P.PcgError):
        P.pcg_sell_build(rowptr, np.zeros(2, np.int32), np.zeros(2, np.float32), 4)
    with pytest.raises(P.PcgError):  # column out of range
        P.pcg_sell_build(np.array([0, 1], np.int64), np.array([4], np.int32), np.ones(1, np.float32), 4)
    with pytest.raises(P.PcgError):  # sigma not a multiple of the chunk
        P.pcg_sell_build(np.array([0, 1], np.int64), np.array([0], np.int32), np.ones(1, np.float32), 4,
                         chunk=4, sigma=6)
    L = P.pcg_sell_build(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 0)
    assert L["chunk_ptr"].tolist() == [0] and L["col"].size == 0
