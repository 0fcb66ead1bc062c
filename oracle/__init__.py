"""CPU oracle for the generic tensor-network independent-set properties.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package, and this package imports nothing from the GPU library.

``oracle.c`` holds three independent programs (brute force, variable
elimination, plan following); this module compiles it with gcc into
``liboracle.so`` next to this file and marshals arguments with ctypes.
Results come back as plain Python values: sizes and partition functions as
floats (plus ln Z), counts as exact Python ints.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SR_TROPICAL, SR_COUNTING_TROPICAL, SR_COUNT, SR_PARTITION = 0, 1, 2, 3
SEMIRINGS = {"tropical": 0, "counting_tropical": 1, "count": 2, "partition": 3}

ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_EOVERFLOW, ORC_ETOOBIG = 0, -1, -2, -4, -5


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        i32p, f64p, u64p = P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_uint64)
        ip = P(ctypes.c_int)
        lib.orc_brute_force.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, ctypes.c_int, f64p,
                                        f64p, u64p, u64p, u64p, f64p, f64p, ctypes.c_int, u64p, ip,
                                        ctypes.c_uint64, ctypes.c_uint64]
        lib.orc_eliminate.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_int, f64p, u64p, f64p, f64p, ip]
        lib.orc_eliminate_poly.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int, u64p, ip, ip]
        lib.orc_eliminate_sg.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, f64p, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_int, f64p, u64p, f64p, f64p, ip]
        lib.orc_brute_force_sg.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, f64p, ctypes.c_int, f64p, f64p,
                                           u64p, f64p, f64p, ctypes.c_uint64, ctypes.c_uint64]
        lib.orc_follow_plan.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_int, i32p, i32p,
                                        i32p, i32p, i32p, i32p, ctypes.c_int, i32p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int, f64p, u64p, f64p, f64p]
        lib.orc_brute_force_topk.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, ctypes.c_int, f64p,
                                             ctypes.c_uint64, ctypes.c_uint64]
        lib.orc_brute_force_sg_topk.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, f64p, ctypes.c_int, f64p,
                                                ctypes.c_uint64, ctypes.c_uint64]
        i64p = P(ctypes.c_int64)
        lib.orc_brute_force_count_top.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, ctypes.c_int, i64p, u64p,
                                                  ip, ctypes.c_uint64, ctypes.c_uint64]
        lib.orc_brute_force_sg_count_top.argtypes = [ctypes.c_int, ctypes.c_int, i32p, f64p, f64p, ctypes.c_int, i64p,
                                                     u64p, ip, ctypes.c_uint64, ctypes.c_uint64]
        for f in (lib.orc_brute_force, lib.orc_eliminate, lib.orc_eliminate_poly, lib.orc_eliminate_sg,
                  lib.orc_brute_force_sg, lib.orc_follow_plan, lib.orc_brute_force_topk, lib.orc_brute_force_sg_topk,
                  lib.orc_brute_force_count_top, lib.orc_brute_force_sg_count_top):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray], ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _graph_arrays(graph):
    edges = np.ascontiguousarray(graph.edges, dtype=np.int32).reshape(-1)
    w = None if graph.weights is None else np.ascontiguousarray(graph.weights, dtype=np.float64)
    return edges, w


def _limbs_to_int(limbs: np.ndarray) -> int:
    return sum(int(x) << (64 * i) for i, x in enumerate(limbs.tolist()))


def _fix_masks(fixed) -> tuple:
    mask = val = 0
    for v, x in (fixed or {}).items():
        mask |= 1 << int(v)
        val |= (int(x) & 1) << int(v)
    return mask, val


def brute_force(graph, betas: Sequence[float] = (), sets_cap: int = 0, fixed=None) -> Dict:
    """O1: enumerate all 2^n subsets (n <= 30; n <= 24 takes about a second).
    fixed: {vertex: 0 or 1}, only subsets that agree with it count."""
    lib = _load()
    fmask, fval = _fix_masks(fixed)
    edges, w = _graph_arrays(graph)
    nb = len(betas)
    b = np.ascontiguousarray(betas, dtype=np.float64) if nb else np.zeros(1)
    mx = np.zeros(1)
    cmax = np.zeros(1, np.uint64)
    tot = np.zeros(1, np.uint64)
    hist = np.zeros(graph.nv + 1, np.uint64)
    z = np.zeros(max(nb, 1))
    lz = np.zeros(max(nb, 1))
    sets = np.zeros(max(sets_cap, 1), np.uint64)
    nsets = ctypes.c_int(0)
    rc = lib.orc_brute_force(graph.nv, graph.ne, _ptr(edges, ctypes.c_int32), _ptr(w, ctypes.c_double),
                             nb, _ptr(b, ctypes.c_double), _ptr(mx, ctypes.c_double),
                             _ptr(cmax, ctypes.c_uint64), _ptr(tot, ctypes.c_uint64),
                             _ptr(hist, ctypes.c_uint64), _ptr(z, ctypes.c_double),
                             _ptr(lz, ctypes.c_double), sets_cap, _ptr(sets, ctypes.c_uint64),
                             ctypes.byref(nsets), fmask, fval)
    if rc != ORC_OK:
        raise OracleError(rc, "brute_force")
    return {
        "size_max": float(mx[0]),
        "count_max": int(cmax[0]),
        "count_all": int(tot[0]),
        "poly": [int(x) for x in hist.tolist()],
        "z": [float(x) for x in z[:nb]],
        "log_z": [float(x) for x in lz[:nb]],
        "max_sets": [int(x) for x in sets[: nsets.value]],
    }


def _result(sr: int, size, limbs, z, lz) -> Dict:
    out: Dict = {}
    if sr in (SR_TROPICAL, SR_COUNTING_TROPICAL):
        out["size"] = float(size[0])
    if sr in (SR_COUNTING_TROPICAL, SR_COUNT):
        out["count"] = _limbs_to_int(limbs)
    if sr == SR_PARTITION:
        out["z"] = float(z[0])
        out["log_z"] = float(lz[0])
    return out


def eliminate(graph, semiring: str, beta: float = 0.0, max_width: int = 26) -> Dict:
    """O2: variable elimination with the oracle's own min-fill order."""
    lib = _load()
    sr = SEMIRINGS[semiring]
    edges, w = _graph_arrays(graph)
    size, z, lz = np.zeros(1), np.zeros(1), np.zeros(1)
    limbs = np.zeros(4, np.uint64)
    width = ctypes.c_int(0)
    rc = lib.orc_eliminate(graph.nv, graph.ne, _ptr(edges, ctypes.c_int32), _ptr(w, ctypes.c_double),
                           sr, float(beta), int(max_width), _ptr(size, ctypes.c_double),
                           _ptr(limbs, ctypes.c_uint64), _ptr(z, ctypes.c_double),
                           _ptr(lz, ctypes.c_double), ctypes.byref(width))
    if rc != ORC_OK:
        raise OracleError(rc, f"eliminate(width={width.value})")
    out = _result(sr, size, limbs, z, lz)
    out["width"] = width.value
    return out


def eliminate_polynomial(graph, max_width: int = 16) -> Dict:
    """O2 over polynomials: the independence polynomial's coefficients
    (c_k = number of independent sets of size k), unit weights, exact."""
    lib = _load()
    edges, _ = _graph_arrays(graph)
    coeffs = np.zeros(4 * (graph.nv + 1), np.uint64)
    degree = ctypes.c_int(0)
    width = ctypes.c_int(0)
    rc = lib.orc_eliminate_poly(graph.nv, graph.ne, _ptr(edges, ctypes.c_int32), int(max_width),
                                _ptr(coeffs, ctypes.c_uint64), ctypes.byref(degree), ctypes.byref(width))
    if rc != ORC_OK:
        raise OracleError(rc, f"eliminate_polynomial(width={width.value})")
    poly = [_limbs_to_int(coeffs[4 * k: 4 * k + 4]) for k in range(degree.value + 1)]
    return {"poly": poly, "degree": degree.value, "width": width.value}


def _sg_arrays(graph, J, h):
    Ja = None if J is None else np.ascontiguousarray(J, dtype=np.float64)
    ha = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
    return Ja, ha


def spin_glass_brute_force(graph, J=None, h=None, betas: Sequence[float] = (), fixed=None) -> Dict:
    """O1 for the spin glass H = sum_(u,v) J_uv s_u s_v + sum_v h_v s_v, s = +-1
    (J per edge in edge order, default 1; h per vertex, default 0); n <= 24.
    fixed: {vertex: 0 (spin down) or 1 (spin up)}."""
    lib = _load()
    fmask, fval = _fix_masks(fixed)
    edges, _ = _graph_arrays(graph)
    Ja, ha = _sg_arrays(graph, J, h)
    nb = len(betas)
    b = np.ascontiguousarray(betas, dtype=np.float64) if nb else np.zeros(1)
    emin = np.zeros(1)
    cnt = np.zeros(1, np.uint64)
    z, lz = np.zeros(max(nb, 1)), np.zeros(max(nb, 1))
    rc = lib.orc_brute_force_sg(graph.nv, graph.ne, _ptr(edges, ctypes.c_int32), _ptr(Ja, ctypes.c_double),
                                _ptr(ha, ctypes.c_double), nb, _ptr(b, ctypes.c_double), _ptr(emin, ctypes.c_double),
                                _ptr(cnt, ctypes.c_uint64), _ptr(z, ctypes.c_double), _ptr(lz, ctypes.c_double),
                                fmask, fval)
    if rc != ORC_OK:
        raise OracleError(rc, "spin_glass_brute_force")
    return {"energy_min": float(emin[0]), "count_min": int(cnt[0]), "z": [float(x) for x in z[:nb]],
            "log_z": [float(x) for x in lz[:nb]]}


def brute_force_topk(graph, k: int, fixed=None) -> List[float]:
    """The k largest independent-set weights with multiplicity (SizeMax(k)),
    by enumeration (n <= 30)."""
    lib = _load()
    edges, w = _graph_arrays(graph)
    fmask, fval = _fix_masks(fixed)
    out = np.zeros(k)
    rc = lib.orc_brute_force_topk(graph.nv, graph.ne, _ptr(edges, ctypes.c_int32), _ptr(w, ctypes.c_double), k,
                                  _ptr(out, ctypes.c_double), fmask, fval)
    if rc != ORC_OK:
        raise OracleError(rc, "brute_force_topk")
    return [float(x) for x in out]


def spin_glass_topk(graph, k: int, J=None, h=None, fixed=None) -> List[float]:
    """The k largest values of -H over all spin configurations, with
    multiplicity (minus the k lowest energies), by enumeration (n <= 30)."""
    lib = _load()
    edges, _ = _graph_arrays(graph)
    Ja, ha = _sg_arrays(graph, J, h)
    fmask, fval = _fix_masks(fixed)
    out = np.zeros(k)
    rc = lib.orc_brute_force_sg_topk(graph.nv, graph.ne, _ptr(edges, ctypes.c_int32), _ptr(Ja, ctypes.c_double),
                                     _ptr(ha, ctypes.c_double), k, _ptr(out, ctypes.c_double), fmask, fval)
    if rc != ORC_OK:
        raise OracleError(rc, "spin_glass_topk")
    return [float(x) for x in out]


def _count_top_result(rc, name, top, cnt, found, k):
    if rc != ORC_OK:
        raise OracleError(rc, name)
    if not found.value:
        return {"top": float("-inf"), "counts": {}}
    t = int(top.value)
    return {"top": t, "counts": {t - d: int(cnt[d]) for d in range(k)}}


def brute_force_counting_max_k(graph, k: int, fixed=None) -> Dict:
    """CountingMax(k) by enumeration (integer weights, n <= 24): {"top": the
    largest set weight, "counts": {top - d: number of independent sets of
    that weight}} (exact; {"top": -inf} if no set meets the fixings)."""
    lib = _load()
    edges, w = _graph_arrays(graph)
    fmask, fval = _fix_masks(fixed)
    top, found = ctypes.c_int64(0), ctypes.c_int(0)
    cnt = np.zeros(k, np.uint64)
    rc = lib.orc_brute_force_count_top(graph.nv, graph.ne, _ptr(edges, ctypes.c_int32), _ptr(w, ctypes.c_double), k,
                                       ctypes.byref(top), _ptr(cnt, ctypes.c_uint64), ctypes.byref(found), fmask, fval)
    return _count_top_result(rc, "brute_force_counting_max_k", top, cnt, found, k)


def spin_glass_counting_max_k(graph, k: int, J=None, h=None, fixed=None) -> Dict:
    """CountingMax(k) of a spin glass with integer J, h by enumeration: the
    largest -H and the number of spin configurations at -H = top - d."""
    lib = _load()
    edges, _ = _graph_arrays(graph)
    Ja, ha = _sg_arrays(graph, J, h)
    fmask, fval = _fix_masks(fixed)
    top, found = ctypes.c_int64(0), ctypes.c_int(0)
    cnt = np.zeros(k, np.uint64)
    rc = lib.orc_brute_force_sg_count_top(graph.nv, graph.ne, _ptr(edges, ctypes.c_int32), _ptr(Ja, ctypes.c_double),
                                          _ptr(ha, ctypes.c_double), k, ctypes.byref(top), _ptr(cnt, ctypes.c_uint64),
                                          ctypes.byref(found), fmask, fval)
    return _count_top_result(rc, "spin_glass_counting_max_k", top, cnt, found, k)


def spin_glass_eliminate(graph, semiring: str, J=None, h=None, beta: float = 0.0, max_width: int = 26) -> Dict:
    """O2 for the spin glass.  tropical / counting_tropical maximise -H:
    "size" is -min H and "count" the number of ground states; "partition"
    gives Z(beta) = sum exp(-beta H); "count" gives 2^n."""
    lib = _load()
    sr = SEMIRINGS[semiring]
    edges, _ = _graph_arrays(graph)
    Ja, ha = _sg_arrays(graph, J, h)
    size, z, lz = np.zeros(1), np.zeros(1), np.zeros(1)
    limbs = np.zeros(4, np.uint64)
    width = ctypes.c_int(0)
    rc = lib.orc_eliminate_sg(graph.nv, graph.ne, _ptr(edges, ctypes.c_int32), _ptr(Ja, ctypes.c_double),
                              _ptr(ha, ctypes.c_double), sr, float(beta), int(max_width), _ptr(size, ctypes.c_double),
                              _ptr(limbs, ctypes.c_uint64), _ptr(z, ctypes.c_double), _ptr(lz, ctypes.c_double),
                              ctypes.byref(width))
    if rc != ORC_OK:
        raise OracleError(rc, f"spin_glass_eliminate(width={width.value})")
    out = _result(sr, size, limbs, z, lz)
    out["width"] = width.value
    return out


def follow_plan(graph, tree: Dict, semiring: str, beta: float = 0.0, max_rank: int = 26,
                slices: Optional[Sequence[int]] = None) -> Dict:
    """O3: evaluate a given contraction tree with literal einsum loops.

    ``tree`` holds plain lists: ``leaf_factors`` (per leaf, factor codes: an
    edge id e >= 0 or a vertex v as -v-1), ``left``/``right`` (children of the
    inner nodes, numbered after the leaves), ``indices`` (output indices of
    every node, leaves first) and ``sliced`` (indices fixed per slice; slice s
    sets sliced[k] to bit k of s).  ``slices=(a, b)`` sums slices a..b-1 only.
    """
    lib = _load()
    sr = SEMIRINGS[semiring]
    edges, w = _graph_arrays(graph)
    lf: List[List[int]] = tree["leaf_factors"]
    nleaf = len(lf)
    ninner = len(tree["left"])
    fac_off = np.zeros(nleaf + 1, np.int32)
    fac_off[1:] = np.cumsum([len(x) for x in lf])
    fac = np.array([c for x in lf for c in x] or [0], np.int32)
    ind: List[List[int]] = tree["indices"]
    idx_off = np.zeros(len(ind) + 1, np.int32)
    idx_off[1:] = np.cumsum([len(x) for x in ind])
    idx = np.array([c for x in ind for c in x] or [0], np.int32)
    left = np.array(list(tree["left"]) or [0], np.int32)
    right = np.array(list(tree["right"]) or [0], np.int32)
    sl = np.array(list(tree.get("sliced", [])) or [0], np.int32)
    nsl = len(tree.get("sliced", []))
    size, z, lz = np.zeros(1), np.zeros(1), np.zeros(1)
    limbs = np.zeros(4, np.uint64)
    I32 = ctypes.c_int32
    rc = lib.orc_follow_plan(graph.nv, graph.ne, _ptr(edges, I32), _ptr(w, ctypes.c_double), sr,
                             float(beta), nleaf, ninner, _ptr(fac_off, I32), _ptr(fac, I32),
                             _ptr(left, I32), _ptr(right, I32), _ptr(idx_off, I32), _ptr(idx, I32),
                             nsl, _ptr(sl, I32), int(slices[0]) if slices else 0, int(slices[1]) if slices else 0,
                             int(max_rank), _ptr(size, ctypes.c_double),
                             _ptr(limbs, ctypes.c_uint64), _ptr(z, ctypes.c_double),
                             _ptr(lz, ctypes.c_double))
    if rc != ORC_OK:
        raise OracleError(rc, "follow_plan")
    return _result(sr, size, limbs, z, lz)
