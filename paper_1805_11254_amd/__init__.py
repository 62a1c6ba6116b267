"""Python binding of libhoph (include/hoph.h): one-permutation hashing (OPH),
grouped OPH (GOPH) and (a:b) hierarchical OPH (HOPH) on MI355X.

The binding only marshals arguments: tensors live in device memory (PyTorch is
used for allocation and streams), every step runs in the library's HIP kernels.
Importing works without a GPU; the device entry points raise if the library is
not built or no GPU is present.  Signatures are uint32 words carried in int32
tensors (same bits).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhoph.so")

HOPH_OK, HOPH_E_INVAL, HOPH_E_RANGE, HOPH_E_CAPACITY = 0, -1, -2, -3
HOPH_E_NOMEM, HOPH_E_UNSUPPORTED, HOPH_E_DEVICE = -4, -5, -6
HASH_TABLE, HASH_MODP31, HASH_MODP32P15 = 0, 1, 2
LAYOUT_OPH, LAYOUT_HIER = 0, 1
EMPTY_JOINT, EMPTY_LITERAL, EMPTY_EITHER = 0, 1, 2
COARSE_CODES, COARSE_WORDS = 0, 1
# coarse-pass kernels as hoph_coarse_plan reports them (HOPH_PLAN_*)
PLAN_NAMES = {0: "none", 1: "words", 2: "codes", 3: "first_group", 4: "first_group_light", 5: "linear",
              6: "linear_light", 7: "oph_full"}
EMPTY = 0xFFFFFFFF

u32, u64, i32, i64, vp = C.c_uint32, C.c_uint64, C.c_int32, C.c_int64, C.c_void_p


class Ratio(C.Structure):
    _fields_ = [("num", u32), ("den", u32)]


class SketchParamsC(C.Structure):
    _fields_ = [("layout", u32), ("k", u32), ("k_group", u32), ("ratio_a", u32), ("ratio_b", u32),
                ("hash", u32), ("universe", u64), ("hash_a", u64), ("hash_b", u64), ("d_perm", vp)]


class QueryParamsC(C.Structure):
    _fields_ = [("T", Ratio), ("eps", Ratio), ("empty_policy", u32), ("coarse_depth", u32),
                ("coarse_filter", u32), ("reserved", u32)]


class ResultsC(C.Structure):
    _fields_ = [("d_offsets", vp), ("d_set_ids", vp), ("capacity", u64), ("needed", u64)]


class MinwiseParamsC(C.Structure):
    _fields_ = [("k", u32), ("hash", u32), ("universe", u64), ("d_hash_a", vp), ("d_hash_b", vp)]


class DecisionTablesC(C.Structure):
    _fields_ = [("L", u32), ("k_group", u32), ("empty_policy", u32), ("goph", u32), ("j_lo", i32), ("j_hi", i32),
                ("lcm", i64), ("wsum", i64), ("W", i64 * 64), ("acc", i64 * 64), ("rej", i64 * 64),
                ("dmul", i64 * 65)]


class PlanConfigC(C.Structure):
    _fields_ = [("kind", u32), ("max_queries", u32), ("max_query_ids", u64), ("max_results", u64),
                ("use_graph", u32), ("tune", u32)]


class PlanInfoC(C.Structure):
    _fields_ = [("q_per_wave", u32), ("coarse_waves_per_cu", u32), ("sketch_chunk", u32),
                ("sketch_waves_per_cu", u32), ("depth", u32), ("graph", u32), ("tuned", u32), ("fallbacks", u32),
                ("tune_ms", C.c_float), ("fallback_causes", u32), ("reserved", u32)]


class ServerConfigC(C.Structure):
    _fields_ = [("kind", u32), ("slots", u32), ("max_batch_queries", u32), ("use_graph", u32),
                ("max_batch_ids", u64), ("max_batch_results", u64), ("device_mem_budget", u64), ("tune", u32),
                ("reserved", u32)]


class ServerStatsC(C.Structure):
    _fields_ = [("submitted", u64), ("completed", u64), ("rejected", u64), ("batches", u64), ("fallbacks", u64),
                ("inserted_sets", u64), ("mean_ms", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("max_ms", C.c_double), ("mean_batch_queries", C.c_double), ("busy_s", C.c_double),
                ("slots", u32), ("reserved", u32), ("slot_bytes", u64)]


# name -> (restype, argtypes); every symbol declared in include/hoph.h
SIGNATURES = {
    "sketch_oph": (C.c_int, [C.POINTER(SketchParamsC), vp, vp, u64, vp, vp]),
    "build_index": (C.c_int, [C.POINTER(SketchParamsC), vp, u64, u64, C.POINTER(vp), vp]),
    "index_append": (C.c_int, [vp, vp, u64, vp]),
    "index_append_sets": (C.c_int, [vp, vp, vp, u64, vp]),
    "hoph_append_timing": (C.c_int, [vp, C.POINTER(C.c_float)]),
    "hoph_stream_timing": (C.c_int, [vp, vp, u64, u32, C.POINTER(C.c_float), vp]),
    "hoph_self_join": (C.c_int, [vp, C.POINTER(QueryParamsC), C.POINTER(ResultsC), vp]),
    "hoph_pair_estimates": (C.c_int, [vp, vp, u32, vp, u64, u32, vp, vp, vp, vp, vp, C.POINTER(C.c_int64), vp]),
    "hoph_index_rows": (C.c_int, [vp, u64, u64, vp, vp]),
    "hoph_index_size": (u64, [vp]),
    "hoph_index_reset": (C.c_int, [vp]),
    "hoph_index_code_planes": (C.c_int, [vp, vp, u64, C.POINTER(u64), vp]),
    "hoph_query_timing": (C.c_int, [vp, C.POINTER(C.c_float)]),
    "hoph_query_counts": (C.c_int, [vp, C.POINTER(C.c_uint64)]),
    "hoph_coarse_plan": (C.c_int, [vp, C.POINTER(C.c_uint32)]),
    "hoph_first_group_plan": (C.c_int, [C.POINTER(SketchParamsC), C.POINTER(QueryParamsC), u32, u32, u32,
                                        C.POINTER(C.c_double), C.POINTER(C.c_uint32)]),
    "hoph_scan_timing": (C.c_int, [vp, vp, u32, C.POINTER(QueryParamsC), u32, vp, u64, C.POINTER(C.c_float), vp]),
    "hoph_index_free": (None, [vp]),
    "query_goph": (C.c_int, [vp, vp, u32, C.POINTER(QueryParamsC), C.POINTER(ResultsC), vp]),
    "query_hoph": (C.c_int, [vp, vp, u32, C.POINTER(QueryParamsC), C.POINTER(ResultsC), vp]),
    "query_oph_full": (C.c_int, [vp, vp, u32, C.POINTER(QueryParamsC), C.POINTER(ResultsC), vp]),
    "query_hoph_noalloc": (C.c_int, [vp, vp, u32, C.POINTER(QueryParamsC), C.POINTER(ResultsC), vp]),
    "minwise_sketch": (C.c_int, [C.POINTER(MinwiseParamsC), vp, vp, u64, vp, vp]),
    "minwise_query": (C.c_int, [C.POINTER(MinwiseParamsC), vp, u64, vp, u32, Ratio, C.POINTER(ResultsC), vp]),
    "hoph_sync": (C.c_int, [vp]),
    "hoph_status_str": (C.c_char_p, [C.c_int]),
    "hoph_last_error": (C.c_char_p, []),
    "hoph_layout_starts": (C.c_int, [C.POINTER(SketchParamsC), vp]),
    "hoph_layout_lookups": (C.c_int, [C.POINTER(SketchParamsC), C.POINTER(u32)]),
    "hoph_tail_integers": (C.c_int, [u32, Ratio, Ratio, C.POINTER(i32), C.POINTER(i32)]),
    "hoph_build_decision_tables": (C.c_int, [C.POINTER(SketchParamsC), C.POINTER(QueryParamsC), u32,
                                             C.POINTER(DecisionTablesC)]),
    "hoph_selftest_bins": (C.c_int, [C.POINTER(SketchParamsC), vp, vp, u64, vp, vp]),
    "hoph_pair_counts": (C.c_int, [vp, vp, u32, vp, u64, u32, vp, vp, vp]),
    "hoph_plan_create": (C.c_int, [vp, C.POINTER(SketchParamsC), C.POINTER(QueryParamsC), C.POINTER(PlanConfigC),
                                   C.POINTER(vp)]),
    "hoph_plan_run": (C.c_int, [vp, vp, vp, u32, u64, vp]),
    "hoph_plan_results": (C.c_int, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(u64), vp]),
    "hoph_plan_query_sigs": (C.c_int, [vp, C.POINTER(vp), C.POINTER(u32)]),
    "hoph_plan_get_info": (C.c_int, [vp, C.POINTER(PlanInfoC)]),
    "hoph_plan_free": (None, [vp]),
    "hoph_server_create": (C.c_int, [vp, C.POINTER(SketchParamsC), C.POINTER(QueryParamsC),
                                     C.POINTER(ServerConfigC), C.POINTER(vp)]),
    "hoph_server_submit": (C.c_int, [vp, vp, u64, C.POINTER(u64)]),
    "hoph_server_wait": (C.c_int, [vp, u64, vp, u64, C.POINTER(u64)]),
    "hoph_server_poll": (C.c_int, [vp, u64, C.POINTER(i32), vp, u64, C.POINTER(u64)]),
    "hoph_server_insert": (C.c_int, [vp, vp, vp, u64]),
    "hoph_server_replay": (C.c_int, [vp, vp, vp, u64, vp, vp, vp, u64]),
    "hoph_server_stats_get": (C.c_int, [vp, C.POINTER(ServerStatsC)]),
    "hoph_server_reset_stats": (C.c_int, [vp]),
    "hoph_server_destroy": (None, [vp]),
}

_lib = None


class HophError(RuntimeError):
    def __init__(self, status: int, message: str, needed: Optional[int] = None):
        self.status = status
        self.needed = needed
        super().__init__(f"{lib().hoph_status_str(status).decode()}: {message}")


def lib():
    """The loaded library; raises ImportError when it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1805_11254_amd.build`")
        # torch's HIP runtime first: the library then binds to that copy
        # (same soname) instead of loading a second runtime into the process
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, needed: Optional[int] = None):
    if status != HOPH_OK:
        raise HophError(status, lib().hoph_last_error().decode(), needed)


def _ratio(r) -> Ratio:
    from fractions import Fraction
    if isinstance(r, Ratio):
        return r
    if isinstance(r, tuple):
        return Ratio(int(r[0]), int(r[1]))
    f = Fraction(str(r)) if isinstance(r, float) else Fraction(r)
    return Ratio(f.numerator, f.denominator)


# ---------------------------------------------------------------------------
# Parameters
# ---------------------------------------------------------------------------
@dataclass
class SketchParams:
    """Sketch layout and permutation (Sec. 3.2 / Sec. 4.1)."""
    layout: int
    k: int
    k_group: int
    hash: int
    universe: int
    ratio_a: int = 1
    ratio_b: int = 1
    hash_a: int = 0
    hash_b: int = 0
    perm: object = None          # torch int32 cuda tensor (HASH_TABLE), or numpy for host helpers

    def c(self, perm_ptr: Optional[int] = None) -> SketchParamsC:
        if perm_ptr is None and self.perm is not None and hasattr(self.perm, "data_ptr"):
            perm_ptr = self.perm.data_ptr()
        return SketchParamsC(self.layout, self.k, self.k_group, self.ratio_a, self.ratio_b, self.hash,
                             self.universe, self.hash_a, self.hash_b, perm_ptr)

    @property
    def groups(self) -> int:
        return self.k // self.k_group


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _need_cuda(t, name, dtypes):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must have dtype in {dtypes}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


# ---------------------------------------------------------------------------
# Device entry points
# ---------------------------------------------------------------------------
def sketch_oph(params: SketchParams, ids, offsets, out=None, stream=None):
    """OPH / HOPH signatures, int32 tensor (n_sets, k) holding uint32 words."""
    import torch
    _need_cuda(ids, "ids", (torch.int32,))
    _need_cuda(offsets, "offsets", (torch.int64,))
    n = offsets.numel() - 1
    if out is None:
        out = torch.empty((max(n, 0), params.k), dtype=torch.int32, device=ids.device)
    else:
        _need_cuda(out, "out", (torch.int32,))
    pc = params.c()
    _check(lib().sketch_oph(C.byref(pc), vp(ids.data_ptr()), vp(offsets.data_ptr()), max(n, 0),
                            vp(out.data_ptr()), _stream(stream)))
    return out


def sync(stream=None):
    """Synchronise and report device-side sketch errors (ids out of range, empty sets)."""
    _check(lib().hoph_sync(_stream(stream)))


class Index:
    """A resident signature index in HBM (library-owned)."""

    def __init__(self, params: SketchParams, sigs, capacity: Optional[int] = None, stream=None):
        import torch
        _need_cuda(sigs, "sigs", (torch.int32,))
        n = sigs.shape[0]
        self.params = params
        self._h = vp()
        pc = params.c()
        _check(lib().build_index(C.byref(pc), vp(sigs.data_ptr()), n, capacity if capacity is not None else n,
                                 C.byref(self._h), _stream(stream)))

    @property
    def handle(self):
        return self._h

    def append(self, sigs, stream=None):
        import torch
        _need_cuda(sigs, "sigs", (torch.int32,))
        _check(lib().index_append(self._h, vp(sigs.data_ptr()), sigs.shape[0], _stream(stream)))

    def append_sets(self, ids, offsets, stream=None):
        """Sketch the sets (CSR on the device) straight into the index."""
        import torch
        _need_cuda(ids, "ids", (torch.int32,))
        _need_cuda(offsets, "offsets", (torch.int64,))
        n = offsets.numel() - 1
        _check(lib().index_append_sets(self._h, vp(ids.data_ptr()), vp(offsets.data_ptr()), max(n, 0),
                                       _stream(stream)))

    def code_planes(self, stream=None):
        """The index's code planes as int32 [code units, capacity / 64, 64, PW]
        (rows past the index size undefined), a copy.  A code unit holds
        min(32 // k', L) whole groups when k' <= 16, else one group."""
        import torch
        dims = (u64 * 3)()
        st = lib().hoph_index_code_planes(self._h, None, 0, dims, _stream(stream))   # sizes only
        if st not in (0, HOPH_E_CAPACITY):
            _check(st)
        cu, rows, pw = int(dims[0]), int(dims[1]), int(dims[2])
        out = torch.empty(max(cu * rows * pw, 1), dtype=torch.int32, device="cuda")
        _check(lib().hoph_index_code_planes(self._h, vp(out.data_ptr()), out.numel(), dims, _stream(stream)))
        return out[:cu * rows * pw].view(cu, rows // 64, 64, pw)

    def rows(self, first=0, n=None, stream=None):
        """Signatures int32[n][k] of index rows first .. first + n - 1 (a copy)."""
        import torch
        if n is None:
            n = len(self) - first
        out = torch.empty((max(n, 0), self.params.k), dtype=torch.int32, device="cuda")
        _check(lib().hoph_index_rows(self._h, first, n, vp(out.data_ptr()), _stream(stream)))
        return out

    def last_append_ms(self):
        """(sketch into the rows, code planes of the new rows) device ms of the
        last append_sets."""
        ms = (C.c_float * 2)()
        _check(lib().hoph_append_timing(self._h, ms))
        return ms[0], ms[1]

    def __len__(self):
        return int(lib().hoph_index_size(self._h)) if self._h else 0

    def reset(self):
        """Size 0, capacity kept (refill with append)."""
        _check(lib().hoph_index_reset(self._h))

    def last_query_ms(self):
        """(coarse, per-survivor, sort+output) device ms of the last query."""
        ms = (C.c_float * 3)()
        _check(lib().hoph_query_timing(self._h, ms))
        return tuple(ms)

    def last_query_counts(self):
        """(coarse-pass survivors, accepted pairs) of the last query."""
        c = (C.c_uint64 * 2)()
        _check(lib().hoph_query_counts(self._h, c))
        return c[0], c[1]

    def last_coarse_plan(self):
        """(depth, kernel, first-phase planes, tiles per wavefront) of the last
        query's coarse pass; kernel is one of the PLAN_* names."""
        c = (C.c_uint32 * 4)()
        _check(lib().hoph_coarse_plan(self._h, c))
        return c[0], PLAN_NAMES.get(c[1], str(c[1])), c[2], c[3]

    def free(self):
        if self._h:
            lib().hoph_index_free(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _run_query(fn, handle, qsigs, qp: QueryParamsC, capacity, stream, device):
    import torch
    n_q = qsigs.shape[0]
    offsets = torch.empty(n_q + 1, dtype=torch.int64, device=device)
    cap = capacity if capacity is not None else max(4096, 64 * n_q)
    while True:
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device=device)
        res = ResultsC(offsets.data_ptr(), ids.data_ptr(), cap, 0)
        st = fn(handle, vp(qsigs.data_ptr()), n_q, C.byref(qp), C.byref(res), _stream(stream))
        if st == HOPH_E_CAPACITY and capacity is None and int(res.needed) > cap:
            cap = int(res.needed)             # the output was too small: retry with what it needs
            continue
        _check(st, int(res.needed))
        return offsets, ids[:int(res.needed)]


def _query(name, index: Index, qsigs, T, eps, policy, capacity, coarse_depth, stream, coarse=COARSE_CODES):
    import torch
    _need_cuda(qsigs, "qsigs", (torch.int32,))
    qp = QueryParamsC(_ratio(T), _ratio(eps), policy, coarse_depth, coarse, 0)
    return _run_query(getattr(lib(), name), index.handle, qsigs, qp, capacity, stream, qsigs.device)


def query_goph(index: Index, qsigs, T=(4, 5), eps=(1, 10000), policy=EMPTY_JOINT, capacity=None,
               coarse_depth=0, stream=None, coarse=COARSE_CODES):
    """Alg. 1 over the index: (offsets int64[n_q+1], set ids int32[...])."""
    return _query("query_goph", index, qsigs, T, eps, policy, capacity, coarse_depth, stream, coarse)


def query_hoph(index: Index, qsigs, T=(4, 5), eps=(1, 10000), policy=EMPTY_JOINT, capacity=None,
               coarse_depth=0, stream=None, coarse=COARSE_CODES):
    """Alg. 2 over the index: (offsets int64[n_q+1], set ids int32[...])."""
    return _query("query_hoph", index, qsigs, T, eps, policy, capacity, coarse_depth, stream, coarse)


def scan_timing(index: Index, qsigs, T=(4, 5), eps=(1, 10000), policy=EMPTY_JOINT, reps=20, coarse_depth=0,
                coarse=COARSE_CODES, flush=None, stream=None) -> float:
    """Mean device time (ms) of one coarse pass over the index for these query
    signatures, reps launches back to back between two HIP events; with a
    flush tensor (device memory larger than the last-level cache, at least
    4 MiB, its first 4 MiB may be overwritten), each pass follows a read of it
    and the reads' own time is subtracted."""
    import torch
    _need_cuda(qsigs, "qsigs", (torch.int32,))
    qp = QueryParamsC(_ratio(T), _ratio(eps), policy, coarse_depth, coarse, 0)
    ms = C.c_float()
    fp, fb = (vp(flush.data_ptr()), flush.numel() * flush.element_size()) if flush is not None else (None, 0)
    _check(lib().hoph_scan_timing(index.handle, vp(qsigs.data_ptr()), qsigs.shape[0], C.byref(qp), reps, fp, fb,
                                  C.byref(ms), _stream(stream)))
    return float(ms.value)


def stream_timing(a, b, reps=10, stream=None):
    """Mean device ms of one read of a, one write of b and one copy a -> b
    (device tensors of equal byte size, at least 4 MiB; a's first 4 MiB may
    be overwritten)."""
    nbytes = a.numel() * a.element_size()
    if b.numel() * b.element_size() != nbytes:
        raise ValueError("a and b must have the same size in bytes")
    ms = (C.c_float * 3)()
    _check(lib().hoph_stream_timing(vp(a.data_ptr()), vp(b.data_ptr()), nbytes, reps, ms, _stream(stream)))
    return float(ms[0]), float(ms[1]), float(ms[2])


def self_join(index: Index, T=(4, 5), eps=(1, 10000), policy=EMPTY_JOINT, capacity=None, coarse_depth=0,
              stream=None, coarse=COARSE_CODES):
    """Near-duplicate pairs i < j inside the index: (offsets int64[n+1], ids int32[...])."""
    import torch
    qp = QueryParamsC(_ratio(T), _ratio(eps), policy, coarse_depth, coarse, 0)
    n = len(index)
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    cap = capacity if capacity is not None else max(4096, 8 * n)
    while True:
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
        res = ResultsC(offsets.data_ptr(), ids.data_ptr(), cap, 0)
        st = lib().hoph_self_join(index.handle, C.byref(qp), C.byref(res), _stream(stream))
        if st == HOPH_E_CAPACITY and capacity is None and int(res.needed) > cap:
            cap = int(res.needed)             # the output was too small: retry with what it needs
            continue
        _check(st, int(res.needed))
        return offsets, ids[:int(res.needed)]


def query_hoph_noalloc(index: Index, qsigs, T=(4, 5), eps=(1, 10000), policy=EMPTY_JOINT, capacity=None,
                       coarse_depth=0, stream=None, coarse=COARSE_CODES):
    """query_hoph through the entry point that allocates no device memory (the
    library's fixed per-device scratch); the output tensors are allocated here."""
    return _query("query_hoph_noalloc", index, qsigs, T, eps, policy, capacity, coarse_depth, stream, coarse)


def query_oph_full(index: Index, qsigs, T=(4, 5), policy=EMPTY_JOINT, capacity=None, stream=None):
    """Plain OPH over all k bins (comparator)."""
    return _query("query_oph_full", index, qsigs, T, (0, 1), policy, capacity, 0, stream)


@dataclass
class MinwiseParams:
    k: int
    hash: int
    universe: int
    hash_a: object               # torch int64 cuda tensor, k entries
    hash_b: object

    def c(self) -> MinwiseParamsC:
        return MinwiseParamsC(self.k, self.hash, self.universe, self.hash_a.data_ptr(), self.hash_b.data_ptr())


def minwise_sketch(params: MinwiseParams, ids, offsets, out=None, stream=None):
    """MinWise signatures, int64 tensor (n_sets, k) holding uint64 minima."""
    import torch
    _need_cuda(ids, "ids", (torch.int32,))
    _need_cuda(offsets, "offsets", (torch.int64,))
    n = offsets.numel() - 1
    if out is None:
        out = torch.empty((max(n, 0), params.k), dtype=torch.int64, device=ids.device)
    pc = params.c()
    _check(lib().minwise_sketch(C.byref(pc), vp(ids.data_ptr()), vp(offsets.data_ptr()), max(n, 0),
                                vp(out.data_ptr()), _stream(stream)))
    return out


def minwise_query(params: MinwiseParams, sigs, qsigs, T=(4, 5), capacity=None, stream=None):
    import torch
    _need_cuda(sigs, "sigs", (torch.int64,))
    _need_cuda(qsigs, "qsigs", (torch.int64,))
    pc = params.c()
    n_q = qsigs.shape[0]
    offsets = torch.empty(n_q + 1, dtype=torch.int64, device=qsigs.device)
    cap = capacity if capacity is not None else max(4096, 64 * n_q)
    while True:
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device=qsigs.device)
        res = ResultsC(offsets.data_ptr(), ids.data_ptr(), cap, 0)
        st = lib().minwise_query(C.byref(pc), vp(sigs.data_ptr()), sigs.shape[0], vp(qsigs.data_ptr()), n_q,
                                 _ratio(T), C.byref(res), _stream(stream))
        if st == HOPH_E_CAPACITY and capacity is None and int(res.needed) > cap:
            cap = int(res.needed)             # the output was too small: retry with what it needs
            continue
        _check(st, int(res.needed))
        return offsets, ids[:int(res.needed)]


_hip = None


def _device_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream):
    """Device-to-device copy on a stream (memory plumbing for plan outputs)."""
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (loads the HIP runtime)
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [vp, vp, C.c_size_t, C.c_int, vp]
        _hip.hipMemcpyAsync.restype = C.c_int
    if nbytes:
        rc = _hip.hipMemcpyAsync(vp(dst_ptr), vp(src_ptr), nbytes, 3, _stream(stream))
        if rc != 0:
            raise RuntimeError(f"hipMemcpyAsync failed ({rc})")


class Plan:
    """Batched GOPH/HOPH over query *sets*: sketch + scan + output per batch,
    persistent kernels, optionally one captured hipGraph replayed per batch and
    tile shapes tuned on the first batch."""

    def __init__(self, index: Index, params: SketchParams, T=(4, 5), eps=(1, 10000), policy=EMPTY_JOINT,
                 kind: Optional[int] = None, max_queries=4096, max_query_ids=1 << 24, max_results=1 << 20,
                 use_graph=True, tune=False, coarse_depth=0, coarse=COARSE_CODES):
        if kind is None:
            kind = 0 if params.layout == LAYOUT_OPH else 1
        self.index = index          # keep the index alive
        self.kind = kind
        self._h = vp()
        pc = params.c()
        qp = QueryParamsC(_ratio(T), _ratio(eps), policy, coarse_depth, coarse, 0)
        cfg = PlanConfigC(kind, max_queries, max_query_ids, max_results, 1 if use_graph else 0, 1 if tune else 0)
        _check(lib().hoph_plan_create(index.handle, C.byref(pc), C.byref(qp), C.byref(cfg), C.byref(self._h)))

    def run(self, ids, offsets, stream=None):
        import torch
        _need_cuda(ids, "ids", (torch.int32,))
        _need_cuda(offsets, "offsets", (torch.int64,))
        n_q = offsets.numel() - 1
        _check(lib().hoph_plan_run(self._h, vp(ids.data_ptr()), vp(offsets.data_ptr()), n_q, ids.numel(),
                                   _stream(stream)))
        self._nq = n_q

    def results(self, stream=None):
        """(offsets int64[n_q+1], set ids int32[...]) of the last batch (copies)."""
        import torch
        po, pi, n = vp(), vp(), u64()
        st = lib().hoph_plan_results(self._h, C.byref(po), C.byref(pi), C.byref(n), _stream(stream))
        _check(st, int(n.value))
        offs = torch.empty(self._nq + 1, dtype=torch.int64, device="cuda")
        ids = torch.empty(max(int(n.value), 1), dtype=torch.int32, device="cuda")
        _device_copy(offs.data_ptr(), po.value, (self._nq + 1) * 8, stream)
        _device_copy(ids.data_ptr(), pi.value, int(n.value) * 4, stream)
        return offs, ids[:int(n.value)]

    def query_sigs(self, k: int, stream=None):
        """Signatures int32[n_q][k] of the last batch's query sets (a copy)."""
        import torch
        pq, n = vp(), u32()
        _check(lib().hoph_plan_query_sigs(self._h, C.byref(pq), C.byref(n)))
        out = torch.empty((int(n.value), k), dtype=torch.int32, device="cuda")
        _device_copy(out.data_ptr(), pq.value, int(n.value) * k * 4, stream)
        return out

    def info(self) -> dict:
        i = PlanInfoC()
        _check(lib().hoph_plan_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in PlanInfoC._fields_ if f != "reserved"}

    def free(self):
        if self._h:
            lib().hoph_plan_free(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Continuous-batching server over a resident index (host query sets in,
    host result lists out)."""

    def __init__(self, index: Index, params: SketchParams, T=(4, 5), eps=(1, 10000), policy=EMPTY_JOINT,
                 kind: Optional[int] = None, slots=2, max_batch_queries=1024, max_batch_ids=1 << 21,
                 max_batch_results=1 << 18, device_mem_budget=0, use_graph=True, tune=False, coarse=COARSE_CODES):
        if kind is None:
            kind = 0 if params.layout == LAYOUT_OPH else 1
        self.index = index
        self._params = params          # keeps a permutation table alive
        self._h = vp()
        pc = params.c()
        qp = QueryParamsC(_ratio(T), _ratio(eps), policy, 0, coarse, 0)
        cfg = ServerConfigC(kind, slots, max_batch_queries, 1 if use_graph else 0, max_batch_ids,
                            max_batch_results, device_mem_budget, 1 if tune else 0, 0)
        _check(lib().hoph_server_create(index.handle, C.byref(pc), C.byref(qp), C.byref(cfg), C.byref(self._h)))

    def submit(self, ids) -> int:
        import numpy as np
        a = np.ascontiguousarray(ids, dtype=np.uint32)
        t = u64()
        _check(lib().hoph_server_submit(self._h, a.ctypes.data_as(vp), a.size, C.byref(t)))
        return t.value

    def wait(self, ticket: int, cap: int = 1 << 20):
        import numpy as np
        out = np.empty(max(cap, 1), dtype=np.uint32)
        n = u64()
        _check(lib().hoph_server_wait(self._h, ticket, out.ctypes.data_as(vp), cap, C.byref(n)), int(n.value))
        return out[:n.value].copy()

    def poll(self, ticket: int, cap: int = 1 << 20):
        import numpy as np
        out = np.empty(max(cap, 1), dtype=np.uint32)
        n, done = u64(), i32()
        _check(lib().hoph_server_poll(self._h, ticket, C.byref(done), out.ctypes.data_as(vp), cap, C.byref(n)))
        return out[:n.value].copy() if done.value else None

    def insert(self, ids, offsets):
        import numpy as np
        i = np.ascontiguousarray(ids, dtype=np.uint32)
        o = np.ascontiguousarray(offsets, dtype=np.uint64)
        _check(lib().hoph_server_insert(self._h, i.ctypes.data_as(vp), o.ctypes.data_as(vp), len(o) - 1))

    def replay(self, ids, offsets, arrival_s, keep_results=False, result_cap=None):
        """Submit request i at arrival_s[i] seconds (native driver), wait for all."""
        import numpy as np
        i = np.ascontiguousarray(ids, dtype=np.uint32)
        o = np.ascontiguousarray(offsets, dtype=np.uint64)
        t = np.ascontiguousarray(arrival_s, dtype=np.float64)
        n = len(o) - 1
        if not keep_results:
            _check(lib().hoph_server_replay(self._h, i.ctypes.data_as(vp), o.ctypes.data_as(vp), n,
                                            t.ctypes.data_as(vp), None, None, 0))
            return None
        cap = result_cap if result_cap is not None else 64 * max(n, 1)
        ro = np.zeros(n + 1, dtype=np.uint64)
        ri = np.zeros(max(cap, 1), dtype=np.uint32)
        _check(lib().hoph_server_replay(self._h, i.ctypes.data_as(vp), o.ctypes.data_as(vp), n,
                                        t.ctypes.data_as(vp), ro.ctypes.data_as(vp), ri.ctypes.data_as(vp), cap))
        return ro, ri[:int(ro[-1])]

    def stats(self) -> dict:
        s = ServerStatsC()
        _check(lib().hoph_server_stats_get(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStatsC._fields_ if f != "reserved"}

    def reset_stats(self):
        _check(lib().hoph_server_reset_stats(self._h))

    def close(self):
        if self._h:
            lib().hoph_server_destroy(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pair_estimates(index: Index, qsigs, pairs, policy=EMPTY_JOINT, unions=None, stream=None):
    """Whole-signature estimates of (query row, set id) pairs: a dict with
    'est' (int64, over 'denominator'), 'mb', 'eb' (int32 holding uint32) and
    'var' (float64, Eq. 8 with the observed 1/(k - N_eb); g from `unions`)."""
    import torch
    _need_cuda(qsigs, "qsigs", (torch.int32,))
    _need_cuda(pairs, "pairs", (torch.int32,))
    if unions is not None:
        _need_cuda(unions, "unions", (torch.float64,))
    n = pairs.shape[0]
    dev = qsigs.device
    est = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    mb = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    eb = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    var = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    den = C.c_int64()
    _check(lib().hoph_pair_estimates(index.handle, vp(qsigs.data_ptr()), qsigs.shape[0], vp(pairs.data_ptr()), n,
                                     policy, vp(unions.data_ptr()) if unions is not None else None,
                                     vp(est.data_ptr()), vp(mb.data_ptr()), vp(eb.data_ptr()), vp(var.data_ptr()),
                                     C.byref(den), _stream(stream)))
    return {"est": est[:n], "mb": mb[:n], "eb": eb[:n], "var": var[:n], "denominator": den.value}


def result_pairs(offsets, ids):
    """(query row, set id) pairs, int32 (n, 2), of a CSR result on the device."""
    import torch
    counts = (offsets[1:] - offsets[:-1]).to(torch.int64)
    rows = torch.repeat_interleave(torch.arange(counts.numel(), device=offsets.device, dtype=torch.int32), counts)
    return torch.stack([rows, ids.to(torch.int32)], dim=1).contiguous()


def pair_counts(index: Index, qsigs, pairs, policy=EMPTY_JOINT, stream=None):
    """Per-group (m, e) for (query row, set id) pairs: two int32 tensors (n_pairs, L)."""
    import torch
    _need_cuda(qsigs, "qsigs", (torch.int32,))
    _need_cuda(pairs, "pairs", (torch.int32,))
    n = pairs.shape[0]
    L = index.params.groups
    m = torch.empty((n, L), dtype=torch.int32, device=pairs.device)
    e = torch.empty((n, L), dtype=torch.int32, device=pairs.device)
    _check(lib().hoph_pair_counts(index.handle, vp(qsigs.data_ptr()), qsigs.shape[0], vp(pairs.data_ptr()), n,
                                  policy, vp(m.data_ptr()), vp(e.data_ptr()), _stream(stream)))
    return m, e


# ---------------------------------------------------------------------------
# Host-only helpers (no GPU)
# ---------------------------------------------------------------------------
def layout_starts(params: SketchParams):
    import numpy as np
    out = np.zeros(params.k + 1, dtype=np.uint64)
    pc = params.c(perm_ptr=0)
    _check(lib().hoph_layout_starts(C.byref(pc), out.ctypes.data_as(vp)))
    return out


LOOKUP_ESTIMATE, LOOKUP_LOG_CELLS, LOOKUP_POW2 = 1, 2, 4


def layout_lookups(params: SketchParams) -> int:
    """Bit mask of the bin lookups the sketch kernels may use for this layout
    (LOOKUP_ESTIMATE | LOOKUP_LOG_CELLS | LOOKUP_POW2)."""
    m = u32()
    pc = params.c(perm_ptr=0)
    _check(lib().hoph_layout_lookups(C.byref(pc), C.byref(m)))
    return int(m.value)


def tail_integers(n: int, T, eps) -> Tuple[int, int]:
    lo, hi = i32(), i32()
    _check(lib().hoph_tail_integers(n, _ratio(T), _ratio(eps), C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def first_group_plan(params: SketchParams, T, eps, policy=EMPTY_JOINT, goph: Optional[bool] = None, tri=False,
                     small_batch=False, keep_rate=None):
    """(first-phase planes, light kernel, tiles per wavefront) of the first-group
    code pass for these parameters (host only); keep_rate: {planes: measured
    phase-1 keep rate} for planes 2..6, or None for independent codes."""
    if goph is None:
        goph = params.layout == LAYOUT_OPH
    pc = params.c()
    qp = QueryParamsC(_ratio(T), _ratio(eps), policy, 0, 0, 0)
    rates = None
    if keep_rate is not None:
        rates = (C.c_double * 8)(*[float(keep_rate.get(i, 0.0)) for i in range(8)])
    out = (C.c_uint32 * 3)()
    _check(lib().hoph_first_group_plan(C.byref(pc), C.byref(qp), 1 if goph else 0, 1 if tri else 0,
                                       1 if small_batch else 0, rates, out))
    return out[0], bool(out[1]), out[2]


def decision_tables(params: SketchParams, T, eps, policy=EMPTY_JOINT, goph: Optional[bool] = None) -> dict:
    if goph is None:
        goph = params.layout == LAYOUT_OPH
    pc = params.c(perm_ptr=0)
    qp = QueryParamsC(_ratio(T), _ratio(eps), policy, 0, COARSE_CODES, 0)
    t = DecisionTablesC()
    _check(lib().hoph_build_decision_tables(C.byref(pc), C.byref(qp), 1 if goph else 0, C.byref(t)))
    L, kp = t.L, t.k_group
    return dict(L=L, k_group=kp, j_lo=t.j_lo, j_hi=t.j_hi, lcm=t.lcm, wsum=t.wsum, W=list(t.W[:L]),
                acc=list(t.acc[:L]), rej=list(t.rej[:L]), dmul=list(t.dmul[:kp + 1]), policy=t.empty_policy)


def selftest_bins(params: SketchParams, ids, perm=None):
    """The library's own hash-and-bin arithmetic run on the host (test hook)."""
    import numpy as np
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    pp = None if perm is None else np.ascontiguousarray(perm, dtype=np.uint32)
    b = np.zeros(len(ids), dtype=np.uint32)
    o = np.zeros(len(ids), dtype=np.uint32)
    pc = params.c(perm_ptr=0)
    _check(lib().hoph_selftest_bins(C.byref(pc), None if pp is None else pp.ctypes.data_as(vp),
                                    ids.ctypes.data_as(vp), len(ids), b.ctypes.data_as(vp), o.ctypes.data_as(vp)))
    return b, o
