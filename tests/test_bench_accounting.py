"""The benchmark's algorithmic byte counts for the PCG iteration with x
advanced every second iteration (checked by hand from the streams each
kernel reads and writes)."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_update_bytes():
    b = _bench()
    # FP32 storage, FP64 x: odd updates read p, r and write r (12 B/pt); even
    # ones also read p_prev and read and write x (32 B/pt)
    assert b.BYTES_UPDATE_SKIP == 12 and b.BYTES_UPDATE_PAIR == 32
    assert b.update_bytes(1) == 12
    assert b.update_bytes(2) == 22
    assert b.update_bytes(3) == (12 + 32 + 12) / 3
    assert b.update_bytes(268) == 22
    # 16-bit storage with the FP32 correction: 6 and 16 B/pt
    assert b.update_bytes(2, es=2, xs=4) == 11
    assert b.update_bytes(0) == 0
    # an iteration of the 256^3 benchmark averages 12 + 22 = 34 B/pt
    assert b.BYTES_DIRECTION + b.update_bytes(268) == 34
