"""Training checkpoints of the learned preconditioner's network.

A checkpoint file holds everything training needs to resume exactly: the
15120 FP32 master weights and Adam's state (first and second moment
estimates, same length, and the step count that sets the bias correction).

File layout: one line of UTF-8 JSON (the header, ending in a newline), then
the raw payload, the arrays back to back as little-endian FP32. The header
names the format and version, the network's shape and weight packing, each
array's name, element count and byte offset in the payload, the step count,
the payload's SHA-256 and free-form metadata. Readers check all of these, so
a truncated, edited or foreign file is refused rather than loaded.

save() and load() move the state between a network and a file through the
library's C ABI (cnn_get_weights / cnn_get_adam, cnn_set_weights /
cnn_set_adam); write_checkpoint() and read_checkpoint() handle the file alone
and work on host arrays.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

FORMAT = "pcgmi-cnn-checkpoint"
VERSION = 1
NUM_WEIGHTS = 15120
ARRAYS = ("weights", "adam_m", "adam_v")
NETWORK = {
    "channels": [2, 16, 16, 16, 1],
    "kernel": [3, 3, 3],
    "packing": "W1[27][2][16] W2[27][16][16] W3[27][16][16] W4[27][16][1], tap = 9 dz + 3 dy + dx",
}


def write_checkpoint(path: str, weights, adam_m, adam_v, step: int, meta: dict | None = None) -> None:
    """Write a checkpoint from host arrays (each NUM_WEIGHTS values). The file
    appears complete or not at all (written beside it, then renamed)."""
    arrs = {}
    for name, a in zip(ARRAYS, (weights, adam_m, adam_v)):
        a = np.ascontiguousarray(np.asarray(a, dtype="<f4").reshape(-1))
        if a.size != NUM_WEIGHTS:
            raise ValueError(f"{name}: {a.size} values, expected {NUM_WEIGHTS}")
        arrs[name] = a
    step = int(step)
    if not 0 <= step < 2**31:
        raise ValueError(f"step {step} out of range")
    payload = b"".join(arrs[n].tobytes() for n in ARRAYS)
    entries, off = [], 0
    for n in ARRAYS:
        entries.append({"name": n, "dtype": "float32-le", "count": NUM_WEIGHTS, "offset": off})
        off += 4 * NUM_WEIGHTS
    header = {"format": FORMAT, "version": VERSION, "network": NETWORK, "arrays": entries, "step": step,
              "payload_bytes": len(payload), "sha256": hashlib.sha256(payload).hexdigest(), "meta": meta or {}}
    line = json.dumps(header, sort_keys=True).encode("utf-8")
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "wb") as f:
        f.write(line + b"\n")
        f.write(payload)
    os.replace(tmp, path)


def read_checkpoint(path: str) -> dict:
    """Read and check a checkpoint: returns {"weights", "adam_m", "adam_v"}
    (FP32 host arrays), "step" and "meta". ValueError if the file is not a
    complete checkpoint of this format."""
    with open(path, "rb") as f:
        data = f.read()
    nl = data.find(b"\n")
    if nl < 0:
        raise ValueError(f"{path}: no header line")
    try:
        header = json.loads(data[:nl].decode("utf-8"))
    except (UnicodeDecodeError, json.JSONDecodeError) as e:
        raise ValueError(f"{path}: header is not JSON ({e})") from None
    if not isinstance(header, dict) or header.get("format") != FORMAT:
        raise ValueError(f"{path}: not a {FORMAT} file")
    if header.get("version") != VERSION:
        raise ValueError(f"{path}: version {header.get('version')}, this reader knows {VERSION}")
    if header.get("network") != NETWORK:
        raise ValueError(f"{path}: network {header.get('network')} differs from {NETWORK}")
    payload = data[nl + 1:]
    if len(payload) != header.get("payload_bytes"):
        raise ValueError(f"{path}: payload is {len(payload)} bytes, header says {header.get('payload_bytes')}")
    if hashlib.sha256(payload).hexdigest() != header.get("sha256"):
        raise ValueError(f"{path}: payload checksum mismatch")
    step = header.get("step")
    if not isinstance(step, int) or not 0 <= step < 2**31:
        raise ValueError(f"{path}: bad step {step!r}")
    out = {"step": step, "meta": header.get("meta", {})}
    entries = {e.get("name"): e for e in header.get("arrays", [])}
    for n in ARRAYS:
        e = entries.get(n)
        if e is None or e.get("dtype") != "float32-le" or e.get("count") != NUM_WEIGHTS:
            raise ValueError(f"{path}: array {n} missing or malformed")
        off = e.get("offset")
        if not isinstance(off, int) or off < 0 or off + 4 * NUM_WEIGHTS > len(payload):
            raise ValueError(f"{path}: array {n} lies outside the payload")
        out[n] = np.frombuffer(payload, dtype="<f4", count=NUM_WEIGHTS, offset=off).astype(np.float32)
    return out


def save(net, path: str, meta: dict | None = None) -> None:
    """Checkpoint a network's weights and Adam state to path."""
    import torch

    from . import _binding as B

    w = B.cnn_get_weights(net)
    m, v, step = B.cnn_get_adam(net)
    torch.cuda.synchronize()
    write_checkpoint(path, w.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy(), step, meta)


def load(net, path: str) -> dict:
    """Restore a network's weights and Adam state from path; returns the
    checkpoint's metadata."""
    import torch

    from . import _binding as B

    ck = read_checkpoint(path)
    dev = {n: torch.from_numpy(ck[n]).cuda() for n in ARRAYS}
    torch.cuda.synchronize()  # the network's stream reads these next
    B.cnn_set_weights(net, dev["weights"])  # resets the moments; restored next
    B.cnn_set_adam(net, dev["adam_m"], dev["adam_v"], ck["step"])
    torch.cuda.synchronize()
    return ck["meta"]
