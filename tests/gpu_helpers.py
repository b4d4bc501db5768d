"""Shared helpers of the GPU parity tests: seeded inputs to device tensors,
the widening of stored values to FP64 for the oracle, and tolerance bounds."""
import numpy as np
import torch

import synthetic


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def bf16_tensor(bits):
    return torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint16).view(np.int16)).view(torch.bfloat16)


def make_vec(seed, n, dtype, kind="uniform", lo=-2, hi=2, density=1.0):
    """(device tensor of `dtype`, the same values widened to FP64 on the host)."""
    if kind == "uniform":
        f32 = synthetic.uniform_f32(seed, n)
    else:
        f32 = synthetic.integers(seed, n, lo, hi, density)
    if dtype == torch.float32:
        return dev(f32), f32.astype(np.float64)
    if dtype == torch.float64:
        f64 = synthetic.uniform(seed, n) if kind == "uniform" else f32.astype(np.float64)
        return dev(f64), f64
    if dtype == torch.bfloat16:
        bits = synthetic.f32_to_bf16_bits(f32)
        return bf16_tensor(bits).to("cuda"), synthetic.bf16_bits_to_f32(bits).astype(np.float64)
    if dtype == torch.float16:
        h = f32.astype(np.float16)
        return dev(h), h.astype(np.float64)
    raise ValueError(dtype)


def check_status(P, info, rtol):
    """A solve that stopped on its recursion reports PCG_OK exactly when its
    FP64 true residual meets rtol, PCG_E_TRUE_RESIDUAL otherwise."""
    assert info["status"] in (P.PCG_OK, P.PCG_E_TRUE_RESIDUAL), info["status"]
    assert (info["status"] == P.PCG_OK) == (info["rel_res_true_fp64"] <= rtol), info


def host64(t):
    return t.detach().to("cpu").to(torch.float64).numpy().reshape(-1)


def ulp(v, dtype):
    """Unit in the last place of |v| in the given storage format."""
    p = {torch.float32: 24, torch.bfloat16: 8, torch.float16: 11, torch.float64: 53}[dtype]
    emin = {torch.float32: -126, torch.bfloat16: -126, torch.float16: -14, torch.float64: -1022}[dtype]
    _, e = np.frexp(np.abs(v))
    e = np.maximum(e - 1, emin)
    return np.ldexp(1.0, e - p + 1)


def stencil_abs_bound(orc, x64, shape):
    """6|x_c| + sum |x_nb| per point (A applied to |x| gives 6|x_c| - sum |x_nb|)."""
    ax = np.abs(x64)
    return 12.0 * ax - orc.stencil(ax, shape)
