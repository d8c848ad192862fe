"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Loads ``ga_oracle.c`` (plain C, built with gcc into ``_oracle.so`` next to it)
through ctypes. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the HIP product
path never does, and the two share no code.

The oracle is the plain definition of the guided extension alignment of
Section 2.1 (Eq. 1-3 score table, Eq. 4-7 z-drop termination); see the header
of ``ga_oracle.c`` for the recurrences and the readings taken where the paper
is silent.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ga_oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
# The same source built for the host it runs on (-O3 -march=native): the
# CPU baseline's timing build and the build that computes stored digests.
# Integer arithmetic only, so both builds give identical results; the
# portable one is what the tests load.
_LIB_NATIVE = os.path.join(_HERE, "_oracle_native.so")

RESULT_FIELDS = ("max_score", "max_i", "max_j", "end_score", "end_i", "end_j", "zdropped")


class Scoring(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("a", "b", "q", "e", "q2", "e2", "ambig")]


class Result(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in RESULT_FIELDS]


def build(force: bool = True, native: bool = False) -> str:
    """Compile the oracle with gcc: portable flags by default (the library
    may run on another host than the one that built it), or with ``native``
    -O3 -march=native for the host compiling it (build it on the host that
    runs it)."""
    path = _LIB_NATIVE if native else _LIB
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + f".tmp{os.getpid()}"
        opt = ["-O3", "-march=native"] if native else ["-O2"]
        cmd = ["gcc"] + opt + ["-std=c11", "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return path


_libs = {}


def _load(native: bool = False):
    lib = _libs.get(native)
    if lib is None:
        path = _LIB_NATIVE if native else _LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=True, native=native)
        lib = ctypes.CDLL(path)
        lib.oracle_align.restype = ctypes.c_int
        lib.oracle_align.argtypes = [
            ctypes.c_char_p, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32,
            ctypes.POINTER(Scoring), ctypes.c_int32, ctypes.c_int32,
            ctypes.POINTER(Result), ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_align_batch.restype = ctypes.c_int
        vp = ctypes.c_void_p
        lib.oracle_align_batch.argtypes = [
            ctypes.c_int64, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Scoring),
            ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_int32]
        _libs[native] = lib
    return lib


def scoring(sc: dict) -> Scoring:
    return Scoring(*(int(sc[k]) for k in ("a", "b", "q", "e", "q2", "e2", "ambig")))


def align(T: bytes, Q: bytes, sc: dict, w: int, Z: int) -> Tuple[Tuple[int, ...], int]:
    """Align one pair; returns (7-tuple result, algorithmic cell count)."""
    lib = _load()
    res = Result()
    cells = ctypes.c_int64(0)
    rc = lib.oracle_align(bytes(T), len(T), bytes(Q), len(Q), ctypes.byref(scoring(sc)),
                          int(w), int(Z), ctypes.byref(res), ctypes.byref(cells))
    if rc != 0:
        raise MemoryError("oracle_align failed")
    return tuple(getattr(res, k) for k in RESULT_FIELDS), int(cells.value)


def align_batch(batch, nthreads: Optional[int] = None, w: Optional[int] = None,
                Z: Optional[int] = None, sc: Optional[dict] = None, native: bool = False):
    """Align every pair of a ``seqgen.PairBatch`` (``native``: the
    -O3 -march=native build of the same source).

    Returns (results int32[n_pairs, 7], cells int64[n_pairs])."""
    lib = _load(native)
    n = batch.n_pairs
    out = np.zeros((n, 7), dtype=np.int32)
    cells = np.zeros(n, dtype=np.int64)
    if n == 0:
        return out, cells
    arrs = [np.ascontiguousarray(a) for a in (batch.t_seq, batch.t_off, batch.t_len,
                                              batch.q_seq, batch.q_off, batch.q_len)]
    # zero-length concatenations still need a valid pointer
    arrs = [a if a.size else np.zeros(1, dtype=a.dtype) for a in arrs]
    ptr = [a.ctypes.data for a in arrs]
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    rc = lib.oracle_align_batch(
        n, ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], ptr[5],
        ctypes.byref(scoring(sc if sc is not None else batch.scoring)),
        int(batch.w if w is None else w), int(batch.zdrop if Z is None else Z),
        out.ctypes.data, cells.ctypes.data, int(nthreads))
    if rc != 0:
        raise MemoryError("oracle_align_batch failed")
    return out, cells
