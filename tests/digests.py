"""Digests of clustering outputs, for whole-output parity at sizes where the
oracle takes minutes to hours.

The oracle's outputs for a workload are computed once, on the CPU, by
``tests/golden/make_oracle_digests.py`` (which calls only ``oracle/`` and the
seeded input generators) and stored as SHA-256 digests of canonical bytes in
``tests/golden/oracle_digests.json``.  A GPU test hashes the library's outputs
the same way and compares: equal digests mean equal arrays, bit for bit
(delta included: its float64 bit patterns are hashed).

Nothing here computes any part of the clustering.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DIGEST_FILE = os.path.join(HERE, "golden", "oracle_digests.json")

# canonical little-endian layout of every hashed array
_DTYPES = {"pts": "<i4", "rho": "<i4", "dep": "<i4", "delta": "<f8", "label": "<i4"}
OUT_KEYS = ("rho", "dep", "delta", "label")


def array_digest(kind: str, a) -> str:
    """SHA-256 (hex) of the array's canonical bytes, with its shape."""
    arr = np.ascontiguousarray(np.asarray(a).astype(_DTYPES[kind], copy=False))
    h = hashlib.sha256()
    h.update(f"{kind}:{arr.shape}".encode())
    h.update(arr.tobytes())
    return h.hexdigest()


def input_digest(job) -> str:
    """Digest of a job's points and thresholds (detects a changed generator)."""
    h = hashlib.sha256()
    h.update(array_digest("pts", job.pts).encode())
    h.update(repr((float(job.d_cut), int(job.rho_min), float(job.delta_min))).encode())
    return h.hexdigest()


def output_digests(out: dict, short: int = 64) -> dict:
    """Digests of rho, dep, delta and label, and ncenters, of one result."""
    rec = {k: array_digest(k, out[k])[:short] for k in OUT_KEYS}
    rec["ncenters"] = int(out["ncenters"])
    return rec


def load() -> dict:
    if not os.path.exists(DIGEST_FILE):
        return {}
    with open(DIGEST_FILE) as fh:
        return json.load(fh)


def save(data: dict) -> None:
    tmp = DIGEST_FILE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
        fh.write("\n")
    os.replace(tmp, DIGEST_FILE)
