"""The network checkpoint file (JSON header line + raw little-endian FP32
payload): round trip, and refusal of truncated, edited or foreign files."""
import json

import numpy as np
import pytest

from paper_2603_23343_amd import checkpoint as C


def _arrays(seed):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(C.NUM_WEIGHTS).astype(np.float32)
    m = (rng.standard_normal(C.NUM_WEIGHTS) * 1e-3).astype(np.float32)
    v = (rng.random(C.NUM_WEIGHTS) * 1e-6).astype(np.float32)
    w[:4] = [np.float32(-0.0), np.float32(np.finfo(np.float32).tiny), np.float32(3.0e38), np.float32(1e-45)]
    return w, m, v


def test_round_trip_bits(tmp_path):
    w, m, v = _arrays(1)
    p = str(tmp_path / "net.ckpt")
    C.write_checkpoint(p, w, m, v, 1234, meta={"grid": [128, 128, 128], "pairs": 4096})
    ck = C.read_checkpoint(p)
    for name, a in zip(C.ARRAYS, (w, m, v)):
        assert ck[name].dtype == np.float32
        assert np.array_equal(ck[name].view(np.uint32), a.view(np.uint32))
    assert ck["step"] == 1234 and ck["meta"] == {"grid": [128, 128, 128], "pairs": 4096}
    # layout: one JSON line, then 3 x 15120 little-endian floats in header order
    data = open(p, "rb").read()
    nl = data.index(b"\n")
    header = json.loads(data[:nl])
    assert [e["name"] for e in header["arrays"]] == list(C.ARRAYS)
    assert len(data) - nl - 1 == 3 * 4 * C.NUM_WEIGHTS
    off = header["arrays"][2]["offset"]
    assert data[nl + 1 + off:nl + 1 + off + 4] == v[:1].astype("<f4").tobytes()


def _corrupt(tmp_path, mutate):
    w, m, v = _arrays(2)
    p = str(tmp_path / "net.ckpt")
    C.write_checkpoint(p, w, m, v, 7)
    data = bytearray(open(p, "rb").read())
    data = mutate(data)
    open(p, "wb").write(bytes(data))
    return p


def _header_edit(key, value):
    def f(data):
        nl = data.index(b"\n")
        h = json.loads(bytes(data[:nl]))
        h[key] = value
        return bytearray(json.dumps(h).encode()) + data[nl:]

    return f


@pytest.mark.parametrize("mutate,msg", [
    (lambda d: d[:-4], "payload"),                                # truncated
    (lambda d: d[:-1] + bytearray([d[-1] ^ 1]), "checksum"),      # one bit of the payload
    (lambda d: bytearray(b"garbage without a header"), "header"),
    (lambda d: bytearray(b"{not json\n") + d, "JSON"),
    (_header_edit("format", "something-else"), "not a"),
    (_header_edit("version", 2), "version"),
    (_header_edit("step", -1), "step"),
    (_header_edit("network", {"channels": [2, 8, 1]}), "network"),
    (_header_edit("arrays", []), "missing"),
])
def test_refuses_bad_files(tmp_path, mutate, msg):
    p = _corrupt(tmp_path, mutate)
    with pytest.raises(ValueError, match=msg):
        C.read_checkpoint(p)


def test_write_checks_sizes(tmp_path):
    w, m, v = _arrays(3)
    with pytest.raises(ValueError):
        C.write_checkpoint(str(tmp_path / "a"), w[:-1], m, v, 0)
    with pytest.raises(ValueError):
        C.write_checkpoint(str(tmp_path / "a"), w, m, v, 2**31)
    assert not (tmp_path / "a").exists()
