"""Build and load the oracle's plain C loops (test infrastructure only).

The C sources next to this file are compiled with the host's gcc into a
shared object beside them, the first time they are needed or when the source
is newer than the built object.  -ffp-contract=off keeps every product and
sum separately rounded, as the oracle's arithmetic is specified.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "interp.c")
_LIB = os.path.join(_HERE, "_oracle_interp.so")
_CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off", "-fno-fast-math"]

_handle = None


def build(force: bool = False) -> str:
    """Compile the C loops if the shared object is missing or stale; returns its path."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    fd, tmp = tempfile.mkstemp(suffix=".so", dir=_HERE)
    os.close(fd)
    try:
        subprocess.run(["gcc", *_CFLAGS, "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    finally:
        if os.path.exists(tmp):
            os.unlink(tmp)
    return _LIB


def lib():
    global _handle
    if _handle is None:
        h = ctypes.CDLL(build())
        p = ctypes.c_void_p
        h.oracle_interpolation.restype = ctypes.c_int64
        h.oracle_interpolation.argtypes = [ctypes.c_int64, p, p, p, p, p, p, p, p, p, p]
        _handle = h
    return _handle
