"""ctypes front end of the plain C oracle (oracle/oph_oracle.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Arrays are numpy; the
binomial tail integers come from oracle.tiny.tail_integers.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from fractions import Fraction
from typing import Optional, Sequence, Tuple

import numpy as np

from . import tiny

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oph_oracle.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                        "-Wall", "-Wextra", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        u32, u64, i32, i64, p = C.c_uint32, C.c_uint64, C.c_int32, C.c_int64, C.c_void_p
        L.orc_sketch.argtypes = [C.c_int, u64, u64, u64, p, C.c_int, u32, u32, u32, u32,
                                 p, p, u64, p, u64, p, C.c_int]
        L.orc_sketch.restype = C.c_int
        L.orc_layout_starts.argtypes = [C.c_int, u64, C.c_int, u32, u32, u32, u32, p]
        L.orc_layout_starts.restype = C.c_int
        L.orc_query.argtypes = [C.c_int, u32, u32, u32, u32, p, u64, p, u32, u32, u32, i32, i32,
                                C.c_int, p, p, p, u64, p, p, C.c_int]
        L.orc_query.restype = i64
        L.orc_query_oph_full.argtypes = [u32, p, u64, p, u32, u32, u32, C.c_int, p, p, u64, C.c_int]
        L.orc_query_oph_full.restype = i64
        L.orc_minwise_sketch.argtypes = [C.c_int, u64, u32, p, p, p, p, u64, p, u64, p, C.c_int]
        L.orc_minwise_sketch.restype = C.c_int
        L.orc_minwise_query.argtypes = [u32, p, u64, p, u32, u32, u32, p, p, u64, C.c_int]
        L.orc_minwise_query.restype = i64
        L.orc_pair_counts.argtypes = [p, p, u32, u32, C.c_int, p, p]
        L.orc_pair_counts.restype = None
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    pass


def max_threads() -> int:
    return lib().orc_max_threads()


def layout_starts(hash_kind, universe, layout, k, kp, ra=1, rb=1) -> np.ndarray:
    out = np.zeros(k + 1, dtype=np.uint64)
    rc = lib().orc_layout_starts(hash_kind, universe, layout, k, kp, ra, rb, _ptr(out))
    if rc:
        raise OracleError(f"invalid layout ({rc})")
    return out


def sketch(ids: np.ndarray, offsets: np.ndarray, *, hash_kind: int, universe: int,
           layout: int, k: int, kp: int, ra: int = 1, rb: int = 1, ha: int = 0, hb: int = 0,
           perm: Optional[np.ndarray] = None, which: Optional[np.ndarray] = None,
           nthreads: int = 0, allow_empty: bool = False) -> np.ndarray:
    """Signatures uint32[n][k] of every set (or of the sets listed in which)."""
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n_sets = len(offsets) - 1
    if which is not None:
        which = np.ascontiguousarray(which, dtype=np.uint64)
        if len(which) and int(which.max()) >= n_sets:
            raise OracleError(f"set index {int(which.max())} past the {n_sets} sets")
    n_out = n_sets if which is None else len(which)
    if perm is not None:
        perm = np.ascontiguousarray(perm, dtype=np.uint32)
    out = np.empty((n_out, k), dtype=np.uint32)
    rc = lib().orc_sketch(hash_kind, universe, ha, hb, _ptr(perm), layout, k, kp, ra, rb,
                          _ptr(ids), _ptr(offsets), n_sets, _ptr(which),
                          0 if which is None else len(which), _ptr(out), nthreads)
    if rc == -3 and allow_empty:
        return out
    if rc:
        raise OracleError(f"orc_sketch failed ({rc})")
    return out


def query(sigs: np.ndarray, qsigs: np.ndarray, *, goph: bool, kp: int, T: Fraction,
          eps: Fraction, policy: int = tiny.EMPTY_JOINT, ra: int = 1, rb: int = 1,
          dense: bool = False, nthreads: int = 0):
    """GOPH / HOPH decisions.  Returns (offsets, ids, steps) and, with dense,
    also the dense (n_q, n_sets) decision and step arrays."""
    T, eps = Fraction(T), Fraction(eps)
    sigs = np.ascontiguousarray(sigs, dtype=np.uint32)
    qsigs = np.ascontiguousarray(qsigs, dtype=np.uint32)
    n_sets, k = sigs.shape if sigs.ndim == 2 and sigs.shape[0] else (0, qsigs.shape[1])
    n_q = qsigs.shape[0]
    j_lo, j_hi = tiny.tail_integers(kp, T, eps)
    offs = np.zeros(n_q + 1, dtype=np.uint64)
    dd = np.zeros((n_q, n_sets), dtype=np.uint8) if dense else None
    ds = np.zeros((n_q, n_sets), dtype=np.uint8) if dense else None
    cap = 1 << 16
    while True:
        ids = np.zeros(cap, dtype=np.uint32)
        steps = np.zeros(cap, dtype=np.uint8)
        n = lib().orc_query(1 if goph else 0, k, kp, ra, rb, _ptr(sigs), n_sets, _ptr(qsigs), n_q,
                            T.numerator, T.denominator, j_lo, j_hi, policy, _ptr(offs),
                            _ptr(ids), _ptr(steps), cap, _ptr(dd), _ptr(ds), nthreads)
        if n < 0:
            raise OracleError(f"orc_query failed ({n})")
        if n <= cap:
            break
        cap = int(n)
    res = (offs, ids[:n].copy(), steps[:n].copy())
    if dense:
        return res + (dd, ds)
    return res


def query_oph_full(sigs, qsigs, *, T, policy=tiny.EMPTY_JOINT, nthreads=0):
    T = Fraction(T)
    sigs = np.ascontiguousarray(sigs, dtype=np.uint32)
    qsigs = np.ascontiguousarray(qsigs, dtype=np.uint32)
    n_sets, k = sigs.shape
    n_q = qsigs.shape[0]
    offs = np.zeros(n_q + 1, dtype=np.uint64)
    cap = 1 << 16
    while True:
        ids = np.zeros(cap, dtype=np.uint32)
        n = lib().orc_query_oph_full(k, _ptr(sigs), n_sets, _ptr(qsigs), n_q, T.numerator,
                                     T.denominator, policy, _ptr(offs), _ptr(ids), cap, nthreads)
        if n < 0:
            raise OracleError(f"orc_query_oph_full failed ({n})")
        if n <= cap:
            return offs, ids[:n].copy()
        cap = int(n)


def minwise_sketch(ids, offsets, *, hash_kind, universe, ha: np.ndarray, hb: np.ndarray,
                   which=None, nthreads=0) -> np.ndarray:
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    ha = np.ascontiguousarray(ha, dtype=np.uint64)
    hb = np.ascontiguousarray(hb, dtype=np.uint64)
    k = len(ha)
    n_sets = len(offsets) - 1
    if which is not None:
        which = np.ascontiguousarray(which, dtype=np.uint64)
        if len(which) and int(which.max()) >= n_sets:
            raise OracleError(f"set index {int(which.max())} past the {n_sets} sets")
    n_out = n_sets if which is None else len(which)
    out = np.empty((n_out, k), dtype=np.uint64)
    rc = lib().orc_minwise_sketch(hash_kind, universe, k, _ptr(ha), _ptr(hb), _ptr(ids),
                                  _ptr(offsets), n_sets, _ptr(which),
                                  0 if which is None else len(which), _ptr(out), nthreads)
    if rc:
        raise OracleError(f"orc_minwise_sketch failed ({rc})")
    return out


def minwise_query(sigs, qsigs, *, T, nthreads=0):
    T = Fraction(T)
    sigs = np.ascontiguousarray(sigs, dtype=np.uint64)
    qsigs = np.ascontiguousarray(qsigs, dtype=np.uint64)
    n_sets, k = sigs.shape
    n_q = qsigs.shape[0]
    offs = np.zeros(n_q + 1, dtype=np.uint64)
    cap = 1 << 16
    while True:
        ids = np.zeros(cap, dtype=np.uint32)
        n = lib().orc_minwise_query(k, _ptr(sigs), n_sets, _ptr(qsigs), n_q, T.numerator,
                                    T.denominator, _ptr(offs), _ptr(ids), cap, nthreads)
        if n < 0:
            raise OracleError(f"orc_minwise_query failed ({n})")
        if n <= cap:
            return offs, ids[:n].copy()
        cap = int(n)


def pair_counts(q: np.ndarray, s: np.ndarray, kp: int, policy: int) -> Tuple[np.ndarray, np.ndarray]:
    q = np.ascontiguousarray(q, dtype=np.uint32)
    s = np.ascontiguousarray(s, dtype=np.uint32)
    k = len(q)
    m = np.zeros(k // kp, dtype=np.uint32)
    e = np.zeros(k // kp, dtype=np.uint32)
    lib().orc_pair_counts(_ptr(q), _ptr(s), k, kp, policy, _ptr(m), _ptr(e))
    return m, e
