"""Pins of oracle parts that no closed form of the operator covers:

* the reduced-precision inner Jacobi-PCG of the refinement emulation
  (iterative refinement: Wilkinson 1963, Moler 1967; the storage reading:
  every inner vector rounded to nearest even on each store, FP32 element
  arithmetic, FP64 scalars), pinned on a one-point grid by the same steps
  carried out in exact rational arithmetic with the roundings written from
  the IEEE 754 definition of the formats, and on larger grids by the
  representability of what it stores;
* axpy (paper Sec. IV's element-wise update) on values fixed by hand;
* the network's input scaling rms(r) and cnn_apply's output scale (the
  learned preconditioner z = rms(r) N(r / rms(r), g)), on a hand-computed
  fixture.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import synthetic


# ---------------------------------------------------------------------------
# Exact arithmetic with explicit roundings (independent of the oracle's
# numpy rounding code): round a rational to p significant bits, ties to even,
# never below the subnormal quantum 2^(emin - p + 1).
# ---------------------------------------------------------------------------

def _round(v: Fr, p: int, emin: int) -> Fr:
    if v == 0:
        return Fr(0)
    sign = -1 if v < 0 else 1
    a = abs(v)
    e = a.numerator.bit_length() - a.denominator.bit_length()  # 2^e <= a < 2^(e+2)
    if Fr(2) ** e > a:
        e -= 1
    if Fr(2) ** (e + 1) <= a:
        e += 1
    assert Fr(2) ** e <= a < Fr(2) ** (e + 1)
    e = max(e, emin)
    q = Fr(2) ** (e - p + 1)
    m = a / q
    n = m.numerator // m.denominator
    frac = m - n
    if frac > Fr(1, 2) or (frac == Fr(1, 2) and n % 2 == 1):
        n += 1
    return sign * n * q


def f64(v):
    return _round(v, 53, -1022)


def f32(v):
    return _round(v, 24, -126)


def bf16(v):
    return _round(f32(v), 8, -126)


def f16(v):
    return _round(f32(v), 11, -14)


def _one_point_inner(k, store, rhs=Fr(1), d_store=None):
    """k steps of Jacobi-PCG on the 1x1x1 grid (A = [6], D^-1 = 1/6) for the
    right-hand side rhs, every vector stored with `store` (the correction d
    with d_store, default `store`), element arithmetic
    rounded to FP32 after each operation, scalars in FP64. Returns the stored
    correction d after k steps (the loop ends early when r becomes 0 or the
    direction vanishes, p.Ap = 0)."""
    d_store = d_store or store
    dinv = f32(f64(Fr(1, 6)))
    r = store(rhs)
    d = Fr(0)
    p = Fr(0)
    rho = f64(dinv * r * r)
    beta = Fr(0)
    for _ in range(k):
        p = store(f32(f32(dinv * r) + f32(f32(beta) * p)))
        q = f32(6 * p)                       # the operator in FP32; no neighbours
        sigma = f64(p * q)
        if sigma <= 0:                       # breakdown ends the solve, d as it is
            break
        alpha = f32(f64(rho / sigma))
        d = d_store(f32(d + f32(alpha * p)))
        r = store(f32(r - f32(alpha * q)))
        if r == 0:
            break
        rho_new = f64(dinv * r * r)
        beta = f64(rho_new / rho)
        rho = rho_new
    return d, p, r


# right-hand sides of the one-point cases (exact in FP64; rounded to the
# storage format on the first store)
RHS = [Fr(1), Fr(3, 10), Fr(77, 100), Fr(19, 10), Fr(-5, 7)]


def test_round_helper_against_known_values():
    # 1/6 to BF16 by hand: 1/6 = 1.0101010101...b x 2^-3; 8 significant bits
    # 1.0101010|1010... round up to 1.0101011b x 2^-3 = 171/1024
    assert bf16(Fr(1, 6)) == Fr(171, 1024)
    # 1/6 to FP16: 11 bits 1.0101010101|0101... round down -> 1365/8192
    assert f16(Fr(1, 6)) == Fr(1365, 8192)
    # FP32 of 1/6: 24 bits, 1.01010101010101010101010|1010... round up
    assert f32(Fr(1, 6)) == Fr(11184811, 2 ** 26)
    # ties to even: 1 + 2^-8 is halfway between BF16 neighbours 1 and 1 + 2^-7
    assert bf16(1 + Fr(1, 2 ** 8)) == 1
    assert bf16(1 + Fr(3, 2 ** 8)) == 1 + Fr(1, 2 ** 6)


def test_one_point_first_direction_by_hand():
    """Step 1 by hand (BF16): p1 = bf16(fl32(1/6)) = 171/1024, q1 = 6 p1 =
    513/512 (exact), sigma = p1 q1 = 87723/2^19; the step then leaves a
    non-zero BF16 residual, which an unrounded FP64 step would not."""
    d, p, r = _one_point_inner(1, bf16)
    assert p == Fr(171, 1024)
    assert r != 0 and bf16(r) == r
    assert d == bf16(d) and abs(float(d) - 1.0 / 6.0) < 2 ** -8


@pytest.mark.parametrize("fmt,store", [("bf16", bf16), ("f16", f16)])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_inner_pcg_lp_one_point_exact(orc, fmt, store, k):
    """The oracle's emulated inner solve equals the exact-arithmetic
    derivation step by step (stagnation off, rtol 0 so only k or a zero
    residual ends it), for several right-hand sides."""
    for rhs in RHS:
        want, _, _ = _one_point_inner(k, store, Fr(float(rhs)))
        d, it = orc.inner_pcg_lp((1, 1, 1), np.array([float(rhs)]), fmt, rtol=0.0, maxit=k, stag_window=0)
        assert Fr(float(d[0])) == want, (k, float(rhs), float(d[0]), float(want))


@pytest.mark.parametrize("fmt,store", [("bf16", bf16), ("f16", f16)])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_inner_pcg_lp_one_point_f32_correction(orc, fmt, store, k):
    """The refinement's default reading: r and p in the 16-bit format, the
    correction d accumulated in FP32."""
    for rhs in RHS:
        want, _, _ = _one_point_inner(k, store, Fr(float(rhs)), d_store=f32)
        got, _ = orc.inner_pcg_lp((1, 1, 1), np.array([float(rhs)]), fmt, rtol=0.0, maxit=k, stag_window=0,
                                  d_fmt="f32")
        assert Fr(float(got[0])) == want, (k, float(rhs))


def _is_bf16(v):
    f = np.asarray(v, dtype=np.float64).astype(np.float32)
    return np.array_equal(f.astype(np.float64), v) and not np.any(f.view(np.uint32) & np.uint32(0xFFFF))


def test_inner_pcg_lp_stores_are_representable(orc):
    """On an 8 x 9 x 10 grid the stored correction is exactly representable
    in its storage format (BF16: an FP32 value whose low 16 bits are zero;
    FP16: unchanged by numpy's float16 cast), and the FP32 correction in FP32."""
    shape = (8, 9, 10)
    rhat = synthetic.uniform(71, 720)
    rhat = rhat / np.max(np.abs(rhat))
    d, it = orc.inner_pcg_lp(shape, rhat, "bf16", rtol=1e-2, maxit=60)
    assert it > 3 and _is_bf16(d)
    d, _ = orc.inner_pcg_lp(shape, rhat, "f16", rtol=1e-3, maxit=60)
    assert np.array_equal(d.astype(np.float16).astype(np.float64), d)
    d, _ = orc.inner_pcg_lp(shape, rhat, "bf16", rtol=1e-2, maxit=60, d_fmt="f32")
    assert np.array_equal(d.astype(np.float32).astype(np.float64), d) and not _is_bf16(d)


def test_inner_pcg_lp_f64_one_point_is_exact_solve(orc):
    """In FP64 storage the one-point system 6 d = 1 is solved in one step to
    rounding: d = 1/6."""
    d, it = orc.inner_pcg_lp((1, 1, 1), np.array([1.0]), "f64", rtol=1e-12, maxit=5, stag_window=0)
    assert it == 1 and abs(d[0] - 1.0 / 6.0) <= 2 ** -52


# ---------------------------------------------------------------------------
# axpy on values fixed by hand
# ---------------------------------------------------------------------------

def test_axpy_hand_values(orc):
    x = np.array([2.0, -4.0, 1.0, 0.0, 3.0, -1.5])
    y = np.array([1.0, 1.0, -0.5, 7.0, -1.5, 0.25])
    # 0.5 x + y, worked out by hand
    assert np.array_equal(orc.axpy(0.5, x, y), np.array([2.0, -1.0, 0.0, 7.0, 0.0, -0.5]))
    # alpha = -3: -3 x + y
    assert np.array_equal(orc.axpy(-3.0, x, y), np.array([-5.0, 13.0, -3.5, 7.0, -10.5, 4.75]))
    # alpha = 0 returns y; alpha = 1 with y = -x cancels exactly
    assert np.array_equal(orc.axpy(0.0, x, y), y)
    assert np.array_equal(orc.axpy(1.0, x, -x), np.zeros(6))
    # a ragged, odd length and an empty vector
    assert np.array_equal(orc.axpy(2.0, np.ones(7), np.arange(7.0)), np.arange(7.0) + 2.0)
    assert orc.axpy(2.0, np.zeros(0), np.zeros(0)).size == 0


# ---------------------------------------------------------------------------
# The network's input scaling and output scale
# ---------------------------------------------------------------------------

def test_precond_input_hand_rms(orc):
    """r = (3, -4, 0, 0) on a 4 x 1 x 1 grid: rms(r) = sqrt(25 / 4) = 2.5
    (mean |r| would be 1.75), so the residual channel is (1.2, -1.6, 0, 0)
    and the second channel is g unchanged."""
    shape = (1, 1, 4)
    r = np.array([3.0, -4.0, 0.0, 0.0])
    g = np.array([0.5, -1.0, 2.0, 0.0])
    inp, rho = orc.precond_input(r, g, shape)
    assert rho == 2.5
    assert inp.shape == (1, 1, 4, 2)
    assert np.allclose(inp[0, 0, :, 0], [1.2, -1.6, 0.0, 0.0], rtol=0, atol=1e-15)
    assert np.array_equal(inp[0, 0, :, 1], g)


def test_cnn_apply_output_scale_is_rms(orc):
    """A one-layer network whose only weight copies the g channel at the
    centre tap gives N = g, so z = rms(r) g: with g = 1 every output is
    rms(r) = 2.5 for the fixture above. A network reading only the residual
    channel gives z = r whatever the scale."""
    shape = (1, 1, 4)
    r = np.array([3.0, -4.0, 0.0, 0.0])
    w_g = np.zeros((27, 2, 1))
    w_g[13, 1, 0] = 1.0  # tap 13 = (dz, dy, dx) = (1, 1, 1): the centre
    z = orc.cnn_apply([w_g], r, np.ones(4), shape)
    assert np.allclose(z, 2.5, rtol=0, atol=1e-15)
    w_r = np.zeros((27, 2, 1))
    w_r[13, 0, 0] = 1.0
    z = orc.cnn_apply([w_r], r, np.ones(4), shape)
    assert np.allclose(z, r, rtol=0, atol=1e-14)
    # a uniform residual: rms = |c|
    z = orc.cnn_apply([w_g], np.full(4, -0.75), np.ones(4), shape)
    assert np.allclose(z, 0.75, rtol=0, atol=1e-15)
    assert math.isclose(orc.precond_input(np.full(4, -0.75), np.zeros(4), shape)[1], 0.75)
