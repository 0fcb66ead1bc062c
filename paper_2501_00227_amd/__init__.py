"""Python binding of the MI355X generic tensor-network library (libtn.so).

Argument marshalling only: every step of a contraction runs in the library's
own gfx950 kernels.  The functions below carry the C ABI's names
(include/tn.h); ``Context``, ``Net`` and ``Plan`` are small owners of the
corresponding handles.  PyTorch is used only to hand the library a stream
and a device allocator (its caching allocator), never for arithmetic.

Importing this package never compiles anything; call
``paper_2501_00227_amd.build.build()`` (or ``__graft_entry__.build()``)
first.  A missing library raises ``LibraryMissing``: there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtn.so")

# tn_status
TN_OK, TN_EINVAL, TN_ENOMEM, TN_EDEVICE, TN_EOVERFLOW, TN_ETOOBIG, TN_EBUSY, TN_ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7
# tn_semiring
TN_TROPICAL_I32, TN_TROPICAL_F32, TN_COUNTING_TROPICAL, TN_COUNT_EXACT, TN_PARTITION_F32, TN_PARTITION_BF16 = range(6)
SEMIRING = {
    "tropical_i32": TN_TROPICAL_I32,
    "tropical_f32": TN_TROPICAL_F32,
    "counting_tropical": TN_COUNTING_TROPICAL,
    "count_exact": TN_COUNT_EXACT,
    "partition_f32": TN_PARTITION_F32,
    "partition_bf16": TN_PARTITION_BF16,
}
KERNEL_KIND = {0: "leaf", 1: "permute", 2: "gemm", 3: "gemm_mfma", 4: "accum", 5: "batch", 6: "gemm_big", 7: "gemm_thin",
               8: "gemm_dot"}


class LibraryMissing(RuntimeError):
    pass


class TnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[tn status {code}] {msg}")
        self.code = code


c_int32_p = ctypes.POINTER(ctypes.c_int32)


class tn_allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.c_void_p), ("free", ctypes.c_void_p), ("user", ctypes.c_void_p)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class tn_plan_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("alpha", ctypes.c_double), ("temperature", ctypes.c_double),
                ("nrepeat", ctypes.c_int32), ("seed", ctypes.c_uint64), ("sc_target", ctypes.c_double),
                ("sc_weight", ctypes.c_double), ("rw_weight", ctypes.c_double), ("beta_start", ctypes.c_double),
                ("beta_step", ctypes.c_double), ("beta_stop", ctypes.c_double), ("ntrials", ctypes.c_int32),
                ("niters", ctypes.c_int32), ("nslices", ctypes.c_int32), ("absorb_vertices", ctypes.c_int32),
                ("nthreads", ctypes.c_int32), ("nopen", ctypes.c_int32), ("open", ctypes.POINTER(ctypes.c_int32))]


class tn_plan_info_t(ctypes.Structure):
    _fields_ = [("nleaf", ctypes.c_int32), ("ninner", ctypes.c_int32), ("nsliced", ctypes.c_int32),
                ("max_rank", ctypes.c_int32), ("tc_log2", ctypes.c_double), ("sc_log2", ctypes.c_double),
                ("rwc_log2", ctypes.c_double), ("arena_entries", ctypes.c_uint64), ("npermutes", ctypes.c_int32)]


class tn_solve_opts(ctypes.Structure):
    _fields_ = [("semiring", ctypes.c_int32), ("beta", ctypes.c_double), ("nprimes", ctypes.c_int32),
                ("primes", ctypes.POINTER(ctypes.c_uint32)), ("slice_begin", ctypes.c_int64),
                ("slice_end", ctypes.c_int64), ("executor", ctypes.c_int32)]


class tn_result(ctypes.Structure):
    _fields_ = [("semiring", ctypes.c_int32), ("size_i32", ctypes.c_int32), ("size_f32", ctypes.c_float),
                ("size_is_neg_inf", ctypes.c_int32), ("count_mod_2_64", ctypes.c_uint64),
                ("residues", ctypes.c_uint32 * 16), ("primes", ctypes.c_uint32 * 16), ("nresidues", ctypes.c_int32),
                ("count_limbs", ctypes.c_uint32 * 16), ("count_nlimbs", ctypes.c_int32),
                ("z_mant", ctypes.c_double), ("z_exp2", ctypes.c_int64), ("log_z", ctypes.c_double),
                ("z", ctypes.c_double), ("seconds", ctypes.c_double), ("z_range_log2", ctypes.c_double)]


class tn_kernel_record(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("node", ctypes.c_int32), ("semiring", ctypes.c_int32),
                ("shape", ctypes.c_int32 * 4), ("ms", ctypes.c_float), ("alg_bytes", ctypes.c_double),
                ("ops", ctypes.c_double), ("kernel", ctypes.c_char * 64)]


class tn_task_record(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("job", ctypes.c_int32), ("node", ctypes.c_int32), ("xcc", ctypes.c_int32),
                ("t_start", ctypes.c_float), ("t_ready", ctypes.c_float), ("t_end", ctypes.c_float)]


class tn_server_stats_t(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("peak_admitted_bytes", ctypes.c_uint64),
                ("peak_running", ctypes.c_int32), ("peak_inflight", ctypes.c_int32),
                ("peak_pool_bytes", ctypes.c_uint64), ("rejected", ctypes.c_uint64), ("canceled", ctypes.c_uint64),
                ("requeued", ctypes.c_uint64)]


class tn_tune_record(ctypes.Structure):
    _fields_ = [("dsr", ctypes.c_int32), ("lb", ctypes.c_int32), ("li", ctypes.c_int32), ("lj", ctypes.c_int32),
                ("lk", ctypes.c_int32), ("a_t", ctypes.c_int32), ("b_t", ctypes.c_int32), ("ncand", ctypes.c_int32),
                ("nrejected", ctypes.c_int32), ("heuristic_ms", ctypes.c_float), ("best_ms", ctypes.c_float),
                ("shape", ctypes.c_int32 * 10)]


# (name, restype, argtypes) of every exported symbol of include/tn.h
_P = ctypes.POINTER
_VP = ctypes.c_void_p
SIGNATURES = [
    ("tn_ctx_create", ctypes.c_int, [ctypes.c_int, _VP, _P(tn_allocator), _P(_VP)]),
    ("tn_ctx_destroy", None, [_VP]),
    ("tn_last_error", ctypes.c_char_p, []),
    ("tn_ctx_set_profiling", ctypes.c_int, [_VP, ctypes.c_int]),
    ("tn_ctx_profile", ctypes.c_int, [_VP, _P(tn_kernel_record), ctypes.c_int32, c_int32_p, ctypes.c_int]),
    ("tn_ctx_synchronize", ctypes.c_int, [_VP]),
    ("tn_ctx_set_wait_limit", ctypes.c_int, [_VP, ctypes.c_double]),
    ("tn_ctx_task_trace", ctypes.c_int, [_VP, _P(tn_task_record), ctypes.c_int32, c_int32_p, ctypes.c_int]),
    ("tn_net_independent_set", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, c_int32_p, _P(ctypes.c_float), _P(_VP)]),
    ("tn_net_spin_glass", ctypes.c_int,
     [ctypes.c_int32, ctypes.c_int32, c_int32_p, _P(ctypes.c_float), _P(ctypes.c_float), _P(_VP)]),
    ("tn_net_destroy", None, [_VP]),
    ("tn_net_info", ctypes.c_int, [_VP, c_int32_p, c_int32_p]),
    ("tn_plan_opts_default", None, [_P(tn_plan_opts)]),
    ("tn_plan_create", ctypes.c_int, [_VP, _P(tn_plan_opts), _P(_VP)]),
    ("tn_plan_from_tree", ctypes.c_int, [_VP, ctypes.c_int32, c_int32_p, c_int32_p, ctypes.c_int32, c_int32_p,
                                         c_int32_p, ctypes.c_int32, c_int32_p, _P(_VP)]),
    ("tn_plan_complexity", ctypes.c_int, [_VP, _P(ctypes.c_double), _P(ctypes.c_double), _P(ctypes.c_double)]),
    ("tn_plan_info", ctypes.c_int, [_VP, _P(tn_plan_info_t)]),
    ("tn_plan_peak_bytes", ctypes.c_int, [_VP, ctypes.c_int, _P(ctypes.c_uint64)]),
    ("tn_plan_export", ctypes.c_int, [_VP] + [c_int32_p] * 12),
    ("tn_plan_destroy", None, [_VP]),
    ("tn_net_flat_complexity", ctypes.c_int, [_VP, _P(ctypes.c_double), _P(ctypes.c_double), _P(ctypes.c_double)]),
    ("tn_solve_opts_default", None, [_P(tn_solve_opts)]),
    ("tn_solve", ctypes.c_int, [_VP, _VP, _VP, _P(tn_solve_opts), _P(tn_result)]),
    ("tn_result_combine", ctypes.c_int, [_P(tn_result), _P(tn_result), _P(tn_result)]),
    ("tn_solve_noalloc", ctypes.c_int, [_VP, _VP, _VP, _P(tn_solve_opts), _P(tn_result)]),
    ("tn_solve_batch", ctypes.c_int, [_VP, ctypes.c_int32, _P(_VP), _P(_VP), _P(tn_solve_opts), _P(tn_result)]),
    ("tn_solve_polynomial", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, _P(ctypes.c_uint32), _P(ctypes.c_int32)]),
    ("tn_solve_max_k", ctypes.c_int,
     [_VP, _VP, _VP, ctypes.c_int32, _P(ctypes.c_int32), ctypes.c_int32, _P(ctypes.c_uint32)]),
    ("tn_plan_gemm_shapes", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int32, c_int32_p, c_int32_p]),
    ("tn_net_condition", ctypes.c_int, [_VP, ctypes.c_int32, c_int32_p, c_int32_p, _P(_VP)]),
    ("tn_solve_open", ctypes.c_int, [_VP, _VP, _VP, _P(tn_solve_opts), ctypes.c_int64, _P(tn_result)]),
    ("tn_solve_size_max_k", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_float)]),
    ("tn_solve_counting_max_k", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, c_int32_p,
                                               _P(ctypes.c_uint64)]),
    ("tn_solve_single_config_max", ctypes.c_int, [_VP, _VP, _VP, c_int32_p, _P(ctypes.c_float)]),
    ("tn_tune_plan", ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, c_int32_p]),
    ("tn_tune_save", ctypes.c_int, [ctypes.c_char_p, c_int32_p]),
    ("tn_tune_load", ctypes.c_int, [ctypes.c_char_p, c_int32_p]),
    ("tn_tune_clear", None, []),
    ("tn_tune_records", ctypes.c_int, [_P(tn_tune_record), ctypes.c_int32, c_int32_p]),
    ("tn_server_create", ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_int32, _P(_VP)]),
    ("tn_server_submit", ctypes.c_int, [_VP, _VP, _VP, _P(tn_solve_opts), _P(ctypes.c_uint64)]),
    ("tn_server_poll", ctypes.c_int, [_VP, ctypes.c_uint64, _P(tn_result), c_int32_p, _P(ctypes.c_double)]),
    ("tn_server_drain", ctypes.c_int, [_VP]),
    ("tn_server_cancel", ctypes.c_int, [_VP, ctypes.c_uint64]),
    ("tn_server_job_bytes", ctypes.c_int, [_VP, _VP, _P(tn_solve_opts), _P(ctypes.c_uint64)]),
    ("tn_server_stats", ctypes.c_int, [_VP, _P(tn_server_stats_t)]),
    ("tn_server_destroy", ctypes.c_int, [_VP]),
]

_lib = None
# Contexts and servers still open at interpreter exit are released by an exit
# handler (servers first), while torch's allocator they free into still works.
# The handler is registered when the first context is made, after torch has
# been imported, so that it runs before any exit handler torch registered.
_live: "weakref.WeakSet" = weakref.WeakSet()
_live_servers: "weakref.WeakSet" = weakref.WeakSet()
_exit_hook = False


def _release_all() -> None:
    for s in list(_live_servers):
        try:
            s.close()
        except Exception:
            pass
    for c in list(_live):
        c.close()


def lib():
    """Load libtn.so (never builds; raises LibraryMissing if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # Load PyTorch's HIP runtime first so libtn.so binds to the same
        # libamdhip64 (same soname): streams and allocations are shared.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int) -> None:
    if code != TN_OK:
        raise TnError(code, lib().tn_last_error().decode(errors="replace"))


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _p32(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(c_int32_p)


# ------------------------------------------------------------------ network --

class Net:
    """Independent-set network of a graph (edges: int [m, 2]; weights or None)."""

    def __init__(self, nv: int, edges, weights=None):
        e = _i32(np.asarray(edges).reshape(-1, 2)).reshape(-1)
        self._w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
        h = ctypes.c_void_p()
        _check(lib().tn_net_independent_set(int(nv), int(e.size // 2), _p32(e) if e.size else None,
                                            None if self._w is None else self._w.ctypes.data_as(_P(ctypes.c_float)),
                                            ctypes.byref(h)))
        self.h = h
        self.nv = int(nv)

    @classmethod
    def from_graph(cls, g) -> "Net":
        return cls(g.nv, g.edges, g.weights)

    @classmethod
    def spin_glass(cls, g, J=None, h=None) -> "Net":
        """Spin glass H = sum J_uv s_u s_v + sum h_v s_v on graph g (J per edge,
        default 1; h per vertex, default 0).  Tropical results are -H's maximum
        (minus the ground-state energy)."""
        self = cls.__new__(cls)
        e = _i32(np.asarray(g.edges).reshape(-1, 2)).reshape(-1)
        self._J = None if J is None else np.ascontiguousarray(J, dtype=np.float32)
        self._h = None if h is None else np.ascontiguousarray(h, dtype=np.float32)
        self._w = None
        hdl = ctypes.c_void_p()
        fp = _P(ctypes.c_float)
        _check(lib().tn_net_spin_glass(int(g.nv), int(e.size // 2), _p32(e) if e.size else None,
                                       None if self._J is None else self._J.ctypes.data_as(fp),
                                       None if self._h is None else self._h.ctypes.data_as(fp), ctypes.byref(hdl)))
        self.h = hdl
        self.nv = int(g.nv)
        return self

    def condition(self, fixed) -> "Net":
        """A copy with vertices fixed ({vertex: 0 or 1}); plans of this network
        fit the copy."""
        items = sorted((int(v), int(x)) for v, x in dict(fixed).items())
        vs = np.ascontiguousarray([v for v, _ in items], dtype=np.int32)
        xs = np.ascontiguousarray([x for _, x in items], dtype=np.int32)
        out = Net.__new__(Net)
        hdl = ctypes.c_void_p()
        _check(lib().tn_net_condition(self.h, len(items), _p32(vs) if len(items) else None,
                                      _p32(xs) if len(items) else None, ctypes.byref(hdl)))
        out.h = hdl
        out.nv = self.nv
        return out

    def flat_complexity(self):
        tc, sc, rw = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().tn_net_flat_complexity(self.h, ctypes.byref(tc), ctypes.byref(sc), ctypes.byref(rw)))
        return tc.value, sc.value, rw.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tn_net_destroy(self.h)
            self.h = None


# --------------------------------------------------------------------- plan --

def plan_opts(**kw) -> tn_plan_opts:
    """Plan options; open=[vertices] keeps those vertices to the root (the
    array is attached to the returned struct, which must outlive the call)."""
    o = tn_plan_opts()
    lib().tn_plan_opts_default(ctypes.byref(o))
    method = kw.pop("method", None)
    if method is not None:
        o.method = {"greedy": 0, "treesa": 1, "auto": 2}.get(method, method)
    opn = kw.pop("open", None)
    if opn:
        o._open_buf = _i32(list(opn))
        o.nopen = len(opn)
        o.open = _p32(o._open_buf)
    for k, v in kw.items():
        if k == "absorb":
            k = "absorb_vertices"
        setattr(o, k, v)
    return o


class Plan:
    """A contraction tree plus the executor program derived from it."""

    def __init__(self, net: Net, h: ctypes.c_void_p):
        self.net = net
        self.h = h

    @classmethod
    def create(cls, net: Net, **kw) -> "Plan":
        """Plan options as keywords (method="greedy" | "treesa" | "auto", seed, ntrials,
        niters, sc_target, nslices, ..., open=[vertices])."""
        o = plan_opts(**kw)
        h = ctypes.c_void_p()
        _check(lib().tn_plan_create(net.h, ctypes.byref(o), ctypes.byref(h)))
        p = cls(net, h)
        p.open = [int(v) for v in kw.get("open") or []]
        return p

    @classmethod
    def from_tree(cls, net: Net, leaf_factors: Sequence[Sequence[int]], left: Sequence[int],
                  right: Sequence[int], sliced: Sequence[int] = ()) -> "Plan":
        fac_off = np.zeros(len(leaf_factors) + 1, np.int32)
        fac_off[1:] = np.cumsum([len(x) for x in leaf_factors])
        fac = _i32([c for x in leaf_factors for c in x] or [0])
        L, R = _i32(list(left) or [0]), _i32(list(right) or [0])
        S = _i32(list(sliced) or [0])
        h = ctypes.c_void_p()
        _check(lib().tn_plan_from_tree(net.h, len(leaf_factors), _p32(fac_off), _p32(fac), len(left), _p32(L),
                                       _p32(R), len(sliced), _p32(S), ctypes.byref(h)))
        return cls(net, h)

    def complexity(self):
        tc, sc, rw = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().tn_plan_complexity(self.h, ctypes.byref(tc), ctypes.byref(sc), ctypes.byref(rw)))
        return tc.value, sc.value, rw.value

    def info(self) -> Dict:
        i = tn_plan_info_t()
        _check(lib().tn_plan_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in i._fields_}

    def peak_bytes(self, semiring) -> int:
        b = ctypes.c_uint64()
        _check(lib().tn_plan_peak_bytes(self.h, _sr(semiring), ctypes.byref(b)))
        return b.value

    SHAPE_FIELDS = ("algebra", "node", "lb", "li", "lj", "lk", "a_t", "b_t", "tb", "ti", "tj", "tk", "rm", "rn",
                    "lsplit", "kind", "valid")

    def gemm_shapes(self, semiring) -> List[Dict]:
        """The GEMM launch shape of every inner node (one dict per device
        algebra and node): sizes, tile, kernel kind, and whether the kernels
        accept it."""
        n = ctypes.c_int32()
        _check(lib().tn_plan_gemm_shapes(self.h, _sr(semiring), 0, None, ctypes.byref(n)))
        width = 18
        buf = (ctypes.c_int32 * max(1, n.value * width))()
        _check(lib().tn_plan_gemm_shapes(self.h, _sr(semiring), n.value, buf, ctypes.byref(n)))
        out = []
        for r in range(n.value):
            row = buf[r * width:(r + 1) * width]
            d = dict(zip(self.SHAPE_FIELDS, row))
            d["kind"] = KERNEL_KIND.get(d["kind"], d["kind"])
            out.append(d)
        return out

    def export(self) -> Dict:
        """The tree as plain lists, in the oracle's plan format."""
        nl, ni, nf, nx, ns = (ctypes.c_int32() for _ in range(5))
        L = lib()
        _check(L.tn_plan_export(self.h, ctypes.byref(nl), ctypes.byref(ni), ctypes.byref(nf), ctypes.byref(nx),
                                ctypes.byref(ns), *([None] * 8)))
        fac_off = np.zeros(nl.value + 1, np.int32)
        fac = np.zeros(max(nf.value, 1), np.int32)
        left = np.zeros(max(ni.value, 1), np.int32)
        right = np.zeros(max(ni.value, 1), np.int32)
        idx_off = np.zeros(nl.value + ni.value + 1, np.int32)
        idx = np.zeros(max(nx.value, 1), np.int32)
        sl = np.zeros(max(ns.value, 1), np.int32)
        _check(L.tn_plan_export(self.h, None, None, None, None, None, _p32(fac_off), _p32(fac), _p32(left),
                                _p32(right), _p32(idx_off), _p32(idx), _p32(sl)))
        return {
            "leaf_factors": [fac[fac_off[i]:fac_off[i + 1]].tolist() for i in range(nl.value)],
            "left": left[: ni.value].tolist(),
            "right": right[: ni.value].tolist(),
            "indices": [idx[idx_off[i]:idx_off[i + 1]].tolist() for i in range(nl.value + ni.value)],
            "sliced": sl[: ns.value].tolist(),
        }

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tn_plan_destroy(self.h)
            self.h = None


def _sr(semiring) -> int:
    return SEMIRING[semiring] if isinstance(semiring, str) else int(semiring)


EXECUTOR = {"auto": 0, "stream": 1, "persistent": 2}


def solve_opts(semiring, beta: float = 0.0, primes: Optional[Sequence[int]] = None,
               slices: Optional[Sequence[int]] = None, executor="auto") -> tn_solve_opts:
    o = tn_solve_opts()
    lib().tn_solve_opts_default(ctypes.byref(o))
    o.semiring = _sr(semiring)
    o.beta = float(beta)
    o.executor = EXECUTOR.get(executor, executor) if isinstance(executor, str) else int(executor)
    if primes is not None:
        arr = (ctypes.c_uint32 * len(primes))(*primes)
        o.nprimes = len(primes)
        o.primes = ctypes.cast(arr, ctypes.POINTER(ctypes.c_uint32))
        o._keep = arr
    if slices is not None:
        o.slice_begin, o.slice_end = int(slices[0]), int(slices[1])
    return o


def decode(r: tn_result) -> Dict:
    """tn_result -> dict of plain Python values (exact counts as int)."""
    out = {"semiring": r.semiring, "seconds": r.seconds}
    sr = r.semiring
    if sr in (TN_TROPICAL_I32, TN_COUNTING_TROPICAL):
        out["size"] = float("-inf") if r.size_is_neg_inf else float(r.size_i32)
    if sr == TN_TROPICAL_F32:
        out["size"] = float(r.size_f32)
    if sr == TN_COUNTING_TROPICAL:
        out["count_mod_2_64"] = int(r.count_mod_2_64)
    if sr == TN_COUNT_EXACT:
        out["count_mod_2_64"] = int(r.count_mod_2_64)
        out["count"] = sum(int(r.count_limbs[k]) << (32 * k) for k in range(r.count_nlimbs))
        out["residues"] = [int(r.residues[k]) for k in range(r.nresidues)]
        out["primes"] = [int(r.primes[k]) for k in range(r.nresidues)]
    if sr in (TN_PARTITION_F32, TN_PARTITION_BF16):
        out.update(z=r.z, log_z=r.log_z, z_mant=r.z_mant, z_exp2=int(r.z_exp2), z_range_log2=r.z_range_log2)
    return out


def result_combine(a: tn_result, b: tn_result) -> tn_result:
    """tn_result_combine: a (+) b for results of disjoint slice ranges (the
    raw results of Context.solve_result; bytes(r) stores one, and
    tn_result.from_buffer_copy reads it back)."""
    out = tn_result()
    _check(lib().tn_result_combine(ctypes.byref(a), ctypes.byref(b), ctypes.byref(out)))
    return out


# ---------------------------------------------------------------- autotuner --

TUNE_SHAPE_FIELDS = ("mode", "tb", "ti", "tj", "tk", "rm", "rn", "lsplit", "mfma")


def tune_save(path: str) -> int:
    """Write the process's launch-shape table; returns its entry count."""
    n = ctypes.c_int32()
    _check(lib().tn_tune_save(os.fsencode(path), ctypes.byref(n)))
    return n.value


def tune_load(path: str) -> int:
    """Merge a table file into the process's table; returns the entry count."""
    n = ctypes.c_int32()
    _check(lib().tn_tune_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def tune_clear() -> None:
    """Every node back on the heuristic launch shapes."""
    lib().tn_tune_clear()


def tune_records() -> List[Dict]:
    """One dict per key tuned since the last clear."""
    n = ctypes.c_int32()
    _check(lib().tn_tune_records(None, 0, ctypes.byref(n)))
    recs = (tn_tune_record * max(n.value, 1))()
    _check(lib().tn_tune_records(recs, n.value, ctypes.byref(n)))
    out = []
    for r in recs[: n.value]:
        d = {f: getattr(r, f) for f, _ in r._fields_ if f != "shape"}
        d["shape"] = dict(zip(TUNE_SHAPE_FIELDS, list(r.shape)[:9]))
        out.append(d)
    return out


# ------------------------------------------------------------------ context --

class Context:
    """A device context on one HIP stream.

    With ``use_torch=True`` (default) the stream is torch's current stream on
    the device and device memory comes from torch's caching allocator.
    """

    def __init__(self, device: int = 0, use_torch: bool = True, stream: Optional[int] = None):
        self._cb = None
        alloc = None
        if use_torch:
            import torch

            torch.cuda.set_device(device)
            dev = device
            # bound now: the callbacks must not look torch up at interpreter
            # teardown, when module globals may already be gone
            t_alloc, t_free = torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete

            def _alloc(nbytes, user, stream_ptr):
                try:
                    return t_alloc(int(nbytes), dev, int(stream_ptr or 0))
                except Exception:
                    return None

            def _free(ptr, nbytes, user, stream_ptr):
                t_free(int(ptr))

            a_cb, f_cb = ALLOC_FN(_alloc), FREE_FN(_free)
            self._cb = (a_cb, f_cb)
            alloc = tn_allocator(ctypes.cast(a_cb, ctypes.c_void_p), ctypes.cast(f_cb, ctypes.c_void_p), None)
            if stream is None:
                stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        _check(lib().tn_ctx_create(int(device), ctypes.c_void_p(stream) if stream else None,
                                   ctypes.byref(alloc) if alloc is not None else None, ctypes.byref(h)))
        self.h = h
        global _exit_hook
        if not _exit_hook:
            atexit.register(_release_all)
            _exit_hook = True
        _live.add(self)

    def set_profiling(self, on: bool = True) -> None:
        _check(lib().tn_ctx_set_profiling(self.h, 1 if on else 0))

    def profile(self, clear: bool = True) -> List[Dict]:
        n = ctypes.c_int32()
        _check(lib().tn_ctx_profile(self.h, None, 0, ctypes.byref(n), 0))
        recs = (tn_kernel_record * max(n.value, 1))()
        _check(lib().tn_ctx_profile(self.h, recs, n.value, ctypes.byref(n), 1 if clear else 0))
        return [{"kind": KERNEL_KIND.get(r.kind, r.kind), "node": r.node, "semiring": r.semiring,
                 "shape": list(r.shape), "ms": r.ms, "alg_bytes": r.alg_bytes, "ops": r.ops,
                 "kernel": r.kernel.decode(errors="replace")}
                for r in recs[: n.value]]

    def task_trace(self, clear: bool = True) -> np.ndarray:
        """Per-task timeline of persistent launches (profiling on): structured array."""
        n = ctypes.c_int32()
        _check(lib().tn_ctx_task_trace(self.h, None, 0, ctypes.byref(n), 0))
        recs = (tn_task_record * max(n.value, 1))()
        _check(lib().tn_ctx_task_trace(self.h, recs, n.value, ctypes.byref(n), 1 if clear else 0))
        dt = np.dtype([("kind", np.int32), ("job", np.int32), ("node", np.int32), ("xcc", np.int32),
                       ("t_start", np.float32), ("t_ready", np.float32), ("t_end", np.float32)])
        return np.frombuffer(bytes(recs)[: n.value * dt.itemsize], dtype=dt).copy()

    def set_wait_limit(self, seconds: float) -> None:
        """Longest dependency wait of a persistent launch (tn_ctx_set_wait_limit)."""
        _check(lib().tn_ctx_set_wait_limit(self.h, float(seconds)))

    def synchronize(self) -> None:
        _check(lib().tn_ctx_synchronize(self.h))

    def solve(self, net: Net, plan: Plan, semiring, beta: float = 0.0, primes=None, slices=None,
              executor="auto") -> Dict:
        return decode(self.solve_result(net, plan, semiring, beta, primes, slices, executor))

    def solve_result(self, net: Net, plan: Plan, semiring, beta: float = 0.0, primes=None, slices=None,
                     executor="auto") -> tn_result:
        """As solve, the raw tn_result (for result_combine and decode)."""
        o = solve_opts(semiring, beta, primes, slices, executor)
        r = tn_result()
        _check(lib().tn_solve(self.h, net.h, plan.h, ctypes.byref(o), ctypes.byref(r)))
        return r

    def tune_plan(self, plan: Plan, semiring, min_log2_ops: float = 20.0, reps: int = 3) -> int:
        """Tune the launch shapes of the plan's nodes with at least
        2^min_log2_ops semiring ops (tn_tune_plan); returns the keys added."""
        n = ctypes.c_int32()
        _check(lib().tn_tune_plan(self.h, plan.h, _sr(semiring), float(min_log2_ops), int(reps), ctypes.byref(n)))
        return n.value

    def solve_noalloc(self, net: Net, plan: Plan, semiring, beta: float = 0.0, primes=None, slices=None) -> Dict:
        """tn_solve_noalloc: as solve(..., executor="stream"), every device
        buffer inside the library's fixed scratch array (no allocation)."""
        o = solve_opts(semiring, beta, primes, slices, "stream")
        r = tn_result()
        _check(lib().tn_solve_noalloc(self.h, net.h, plan.h, ctypes.byref(o), ctypes.byref(r)))
        return decode(r)

    def solve_open(self, net: Net, plan: Plan, semiring, beta: float = 0.0, primes=None, slices=None) -> List[Dict]:
        """The result tensor of a plan with open vertices: one dict per
        assignment, entry e has bit q = value of plan.open[q]."""
        o = solve_opts(semiring, beta, primes, slices, "stream")
        n = 1 << len(getattr(plan, "open", []))
        R = (tn_result * n)()
        _check(lib().tn_solve_open(self.h, net.h, plan.h, ctypes.byref(o), n, R))
        return [decode(R[i]) for i in range(n)]

    def solve_batch(self, nets: Sequence[Net], plans: Sequence[Plan], semirings, betas=None) -> List[Dict]:
        n = len(nets)
        if isinstance(semirings, (str, int)):
            semirings = [semirings] * n
        betas = betas if betas is not None else [0.0] * n
        NH = (ctypes.c_void_p * n)(*[x.h.value for x in nets])
        PH = (ctypes.c_void_p * n)(*[x.h.value for x in plans])
        O = (tn_solve_opts * n)(*[solve_opts(s, b) for s, b in zip(semirings, betas)])
        R = (tn_result * n)()
        _check(lib().tn_solve_batch(self.h, n, NH, PH, O, R))
        return [decode(R[i]) for i in range(n)]

    def solve_polynomial(self, net: Net, plan: Plan) -> List[int]:
        """Independence polynomial coefficients c_0 .. c_alpha (exact ints)."""
        limbs = net.nv // 32 + 2
        buf = (ctypes.c_uint32 * ((net.nv + 1) * limbs))()
        deg = ctypes.c_int32(0)
        _check(lib().tn_solve_polynomial(self.h, net.h, plan.h, limbs, buf, ctypes.byref(deg)))
        return [sum(int(buf[k * limbs + l]) << (32 * l) for l in range(limbs)) for k in range(deg.value + 1)]

    def solve_max_k(self, net: Net, plan: Plan, k: int) -> Dict:
        """SizeMax(k) (the k largest sizes, with multiplicity) and CountingMax(k)
        ({size: count} for the k largest sizes), unit weights."""
        limbs = net.nv // 32 + 2
        sizes = (ctypes.c_int32 * k)()
        counts = (ctypes.c_uint32 * (k * limbs))()
        _check(lib().tn_solve_max_k(self.h, net.h, plan.h, int(k), sizes, limbs, counts))
        top = [int(s) for s in sizes]
        alpha = top[0]
        cm = {alpha - d: sum(int(counts[d * limbs + l]) << (32 * l) for l in range(limbs)) for d in range(k)
              if alpha - d >= 0}
        return {"size_max_k": [s if s != -2 ** 31 else float("-inf") for s in top], "counting_max_k": cm}

    def solve_size_max_k(self, net: Net, plan: Plan, k: int, executor="auto") -> List[float]:
        """SizeMax(k) for any weights (k <= 8): the k largest total weights of
        independent sets with multiplicity (spin glass: the k largest -H)."""
        out = (ctypes.c_float * int(k))()
        ex = EXECUTOR.get(executor, executor) if isinstance(executor, str) else int(executor)
        _check(lib().tn_solve_size_max_k(self.h, net.h, plan.h, int(k), int(ex), out))
        return [float(x) for x in out]

    def solve_counting_max_k(self, net: Net, plan: Plan, k: int, executor="auto") -> Dict:
        """CountingMax(k) for integer weights (k <= 4): {"top": the largest
        value (or -inf), "counts": {top - d: count mod 2^64}}."""
        top = ctypes.c_int32(0)
        cnt = (ctypes.c_uint64 * int(k))()
        ex = EXECUTOR.get(executor, executor) if isinstance(executor, str) else int(executor)
        _check(lib().tn_solve_counting_max_k(self.h, net.h, plan.h, int(k), int(ex), ctypes.byref(top), cnt))
        if top.value == -2 ** 31:
            return {"top": float("-inf"), "counts": {}}
        return {"top": top.value, "counts": {top.value - d: int(cnt[d]) for d in range(int(k))}}

    def solve_single_config_max(self, net: Net, plan: Plan) -> Dict:
        """One maximum configuration (SingleConfigMax): {"config": [0/1 per
        vertex], "value": float32 maximum (set weight, or -H for a spin glass)}."""
        cfg = (ctypes.c_int32 * max(1, net.nv))()
        val = ctypes.c_float(0.0)
        _check(lib().tn_solve_single_config_max(self.h, net.h, plan.h, cfg, ctypes.byref(val)))
        return {"config": [int(cfg[v]) for v in range(net.nv)], "value": float(val.value)}

    def close(self) -> None:
        """Release the context (and the device memory it holds) now."""
        if getattr(self, "h", None) and _lib is not None:
            _lib.tn_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def server_job_bytes(net: Net, plan: Plan, semiring, beta: float = 0.0) -> int:
    """Device bytes the job takes in a server (tn_server_job_bytes)."""
    o = solve_opts(semiring, beta)
    b = ctypes.c_uint64()
    _check(lib().tn_server_job_bytes(net.h, plan.h, ctypes.byref(o), ctypes.byref(b)))
    return b.value


class Server:
    """Continuous-batching server over a context (tn_server_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int = 64):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib().tn_server_create(ctx.h, int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)))
        self.h = h
        self._keep = {}
        _live_servers.add(self)

    def submit(self, net: Net, plan: Plan, semiring, beta: float = 0.0) -> int:
        o = solve_opts(semiring, beta)
        jid = ctypes.c_uint64()
        _check(lib().tn_server_submit(self.h, net.h, plan.h, ctypes.byref(o), ctypes.byref(jid)))
        self._keep[jid.value] = (net, plan)
        return jid.value

    def poll(self, job_id: int):
        r = tn_result()
        done = ctypes.c_int32()
        lat = ctypes.c_double()
        code = lib().tn_server_poll(self.h, int(job_id), ctypes.byref(r), ctypes.byref(done), ctypes.byref(lat))
        if code != TN_OK:
            raise TnError(code, lib().tn_last_error().decode(errors="replace"))
        if not done.value:
            return None
        self._keep.pop(job_id, None)
        out = decode(r)
        out["latency_s"] = lat.value
        return out

    def drain(self) -> None:
        _check(lib().tn_server_drain(self.h))

    def cancel(self, job_id: int) -> None:
        """Cancel a job still in the queue (its poll then raises TN_ECANCELED)."""
        _check(lib().tn_server_cancel(self.h, int(job_id)))

    def stats(self) -> Dict:
        s = tn_server_stats_t()
        _check(lib().tn_server_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def close(self) -> None:
        if getattr(self, "h", None):
            _check(lib().tn_server_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
