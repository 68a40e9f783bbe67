"""Byte forms, digests and sample positions of the stored full-size oracle
results (shared by the script that writes them and the tests that read them;
no solver arithmetic).

* A CSR matrix is digested as SHA-256 over its row pointers as int64, its
  columns as int32 and its values as float64 (little endian), in that order.
* A C/F marker is digested as int8 (1 = C, -1 = F).
* Vectors are compared at a fixed set of positions: in every block segment of
  length N, ``PER_SEGMENT`` positions drawn without replacement by
  numpy's PCG64 from ``SAMPLE_SEED``, plus the segment's first and last entry,
  sorted ascending.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PER_SEGMENT = 512
SAMPLE_SEED = 20020458


def digest_csr(indptr, indices, data) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(indptr, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(indices, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(data, dtype="<f8").tobytes())
    return h.hexdigest()


def digest_cf(cf) -> str:
    return hashlib.sha256(np.ascontiguousarray(cf, dtype="i1").tobytes()).hexdigest()


def sample_positions(n_segments: int, N: int) -> np.ndarray:
    rng = np.random.default_rng(SAMPLE_SEED)
    out = []
    for s in range(n_segments):
        k = min(PER_SEGMENT, N)
        pos = rng.choice(N, size=k, replace=False)
        out.append(np.unique(np.concatenate([pos, [0, N - 1]])) + s * N)
    return np.concatenate(out).astype(np.int64)


def segment_norms(x: np.ndarray, n_segments: int):
    X = np.asarray(x).reshape(n_segments, -1)
    return np.linalg.norm(X, axis=1).tolist(), np.abs(X).max(axis=1).tolist()


def paths(workload: str):
    return (os.path.join(HERE, f"fullsize_{workload}.json"),
            os.path.join(HERE, f"fullsize_{workload}.npz"))
