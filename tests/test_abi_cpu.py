"""The C-ABI library loads and exports every entry point that include/*.h
declares; argument validation that needs no GPU behaves as documented."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_23343_amd", "libpcgmi.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             txt, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_2603_23343_amd.build as b

        b.build()
    return ctypes.CDLL(LIB)


def test_header_declares_core_entry_points():
    names = _declared()
    for n in ("pcg_create", "pcg_destroy", "stencil_apply", "axpy", "dot", "pcg_solve", "pcg_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_validation_without_gpu(lib):
    lib.pcg_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.pcg_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    assert lib.pcg_create(ctypes.byref(h), 0, 4, 4, 0, None, None) == 1  # PCG_E_ARG
    assert b"dims" in lib.pcg_last_error()
    assert lib.pcg_create(ctypes.byref(h), 4, 4, 4, 9, None, None) == 1
    assert lib.pcg_create(None, 4, 4, 4, 0, None, None) == 1
    assert lib.pcg_create(ctypes.byref(h), 1 << 12, 1 << 12, 1 << 12, 0, None, None) == 1
    vp = ctypes.c_void_p
    lib.stencil_apply.argtypes = [vp, vp, vp]
    assert lib.stencil_apply(None, None, None) == 1
    lib.axpy.argtypes = [vp, ctypes.c_int64, ctypes.c_double, vp, vp, vp]
    assert lib.axpy(None, 4, 1.0, None, None, None) == 1
    lib.dot.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
    assert lib.dot(None, 4, None, None, None) == 1
    lib.dot_noalloc.argtypes = [ctypes.c_int, ctypes.c_int64, vp, vp, vp, vp, vp]
    assert lib.dot_noalloc(0, -1, None, None, None, None, None) == 1  # negative length
    assert lib.dot_noalloc(9, 4, None, None, None, None, None) == 1  # unknown storage type
    assert lib.dot_noalloc(0, 4, 16, 32, None, None, None) == 1  # no output
    assert lib.dot_noalloc(0, 4, 20, 32, 64, None, None) == 1  # misaligned x
    assert lib.dot_noalloc(0, (1 << 40) + 1, 16, 32, 64, None, None) == 1  # above the maximum
    assert b"maximum" in lib.pcg_last_error()
    lib.pcg_solve.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int, vp]
    assert lib.pcg_solve(None, None, None, 1e-6, 10, None) == 1
    assert lib.pcg_destroy(None) == 0


def test_options_default(lib):
    import paper_2603_23343_amd as P

    o = P.pcg_options_default()
    assert o.chunk_iters == 16 and o.x_accum == -1 and o.use_graph == 1 and o.use_x0 == 0
    assert o.kernel_timing == 0 and o.x_dtype == -1 and o.stag_window == -1 and o.max_restarts == -1
    assert o.single_reduction == -1


def test_product_path_does_not_import_oracle():
    """The package and its sources never reference the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2603_23343_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if path.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
            txt = open(path).read()
            assert "import oracle" not in txt and "from oracle" not in txt, path
            assert "liboracle" not in txt, path


def test_batch_argument_validation_without_gpu(lib):
    vp, i = ctypes.c_void_p, ctypes.c_int
    lib.pcg_batch_create.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.c_char_p,
                                     i, vp]
    lib.pcg_last_error.restype = ctypes.c_char_p
    h = vp()
    dims = (i * 6)(16, 16, 16, 17, 8, 8)
    assert lib.pcg_batch_create(ctypes.byref(h), 0, dims, None, None, 0, None) == 1
    bad = (i * 3)(16, 0, 16)
    assert lib.pcg_batch_create(ctypes.byref(h), 1, bad, None, None, 0, None) == 1
    assert b"dimension" in lib.pcg_last_error()
    # tile shapes are 0, 1, 2 or 5
    assert lib.pcg_batch_create(ctypes.byref(h), 2, dims, (i * 2)(2, 3), None, 0, None) == 1
    assert b"tile shape 3" in lib.pcg_last_error()
    assert lib.pcg_batch_create(ctypes.byref(h), 2, dims, (i * 2)(-1, 0), None, 0, None) == 1
    lib.pcg_batch_solve.argtypes = [vp, vp, vp, ctypes.c_double, i, i, vp, vp, vp, vp, vp]
    assert lib.pcg_batch_solve(None, None, None, 1e-6, 10, 1, None, None, None, None, None) == 1
    lib.pcg_batch_destroy.argtypes = [vp]
    assert lib.pcg_batch_destroy(None) == 0


def test_sell_argument_validation_without_gpu(lib):
    """The stored-matrix entry points reject bad arguments before any GPU call."""
    vp, i, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.pcg_last_error.restype = ctypes.c_char_p
    lib.pcg_sell_create.argtypes = [ctypes.POINTER(vp), i64, i64, vp, vp, vp, i, vp]
    h = vp()
    rowptr = (i64 * 3)(0, 1, 3)
    col = (ctypes.c_int32 * 3)(0, 0, 2)  # column 2 is out of range for ncols = 2
    val = (ctypes.c_float * 3)(1.0, 1.0, 1.0)
    assert lib.pcg_sell_create(ctypes.byref(h), 2, 2, rowptr, col, val, 1, None) == 1
    assert b"out of range" in lib.pcg_last_error()
    assert lib.pcg_sell_create(ctypes.byref(h), 2, 3, rowptr, col, val, 3, None) == 1  # sigma not a multiple of 64
    assert lib.pcg_sell_create(None, 2, 3, rowptr, col, val, 1, None) == 1
    lib.pcg_sell_spmv.argtypes = [vp, vp, vp]
    assert lib.pcg_sell_spmv(None, None, None) == 1
    lib.pcg_sell_solve.argtypes = [vp, vp, vp, ctypes.c_double, i, vp]
    assert lib.pcg_sell_solve(None, None, None, 1e-6, 10, None) == 1
    lib.pcg_sell_info.argtypes = [vp, vp, vp, vp]
    assert lib.pcg_sell_info(None, None, None, None) == 1
    lib.pcg_sell_set_restarts.argtypes = [vp, i]
    assert lib.pcg_sell_set_restarts(None, 0) == 1
    lib.pcg_sell_destroy.argtypes = [vp]
    assert lib.pcg_sell_destroy(None) == 0
    lib.cnn_set_loss_norm.argtypes = [vp, i]
    assert lib.cnn_set_loss_norm(None, 0) == 1
    lib.cnn_get_adam.argtypes = [vp, vp, vp, vp]
    assert lib.cnn_get_adam(None, None, None, None) == 1
    lib.cnn_set_adam.argtypes = [vp, vp, vp, ctypes.c_int64]
    assert lib.cnn_set_adam(None, None, None, 0) == 1
