"""CPU oracle for exact triangle counting (arXiv 1706.05151) — TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. It shares no code with the GPU library and
imports nothing from it. The arithmetic lives in ``oracle.c`` (plain serial C);
this module only marshals numpy arrays.

Routes (each function cites the passage it follows):
  * definitions of Section 2 — ``local_counts_def`` (T_v = edges among the
    neighbours of v; T = sum T_v / 3);
  * NodeIteratorN of Section 3 — ``orient`` (Eq. (1) order, sorted N_v) and
    ``count_nin`` (|N_v ∩ N_u| over oriented edges, per-node counts as in the
    Section 9 local-count figure, listing as in the Section 8 figure);
  * NodeIterator++ of Section 3 — ``count_nodeiterpp``;
  * clustering coefficients of Section 2 — ``clustering``;
  * sparsification of Section 7 — ``sparsify`` and ``estimate``;
  * the k-core order of Section 4 — ``coreness``;
  * the load-balancing schemes of Sections 5 and 6 — ``partition_work``;
  * core-node shards over the orientation order (Section 5 partitions) —
    ``order_positions``, ``shard_bounds``, ``count_nin_pos_range``;
  * sparsification with independent per-shard samples (Section 7, Eq. var2) —
    ``partition_seed``, ``sparsified_count_partitioned``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` (gcc, -O2, OpenMP only for the total-only variant)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    L = ctypes.CDLL(_LIB)
    i32, i64, u64, dbl, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
    sig = {
        "orc_simple": ([vp, vp, i64, i32, vp, vp], i64),
        "orc_degrees": ([vp, vp, i64, i32, vp], None),
        "orc_full_adjacency": ([vp, vp, i64, i32, vp, vp], None),
        "orc_local_counts_def": ([vp, vp, i32, vp], u64),
        "orc_orient": ([vp, vp, i64, vp, i32, vp, vp], None),
        "orc_orient_by_key": ([vp, vp, i64, vp, i32, vp, vp], None),
        "orc_count_nin": ([vp, vp, i32, vp, vp, i64], u64),
        "orc_count_nin_total_omp": ([vp, vp, i32], u64),
        "orc_work": ([vp, vp, i32], u64),
        "orc_count_nodeiterpp": ([vp, vp, vp, i32], u64),
        "orc_sort_triples": ([vp, i64], None),
        "orc_clustering": ([vp, vp, i32, vp, vp, vp], None),
        "orc_keep_threshold": ([dbl], u64),
        "orc_keep": ([i32, i32, dbl, u64], ctypes.c_int),
        "orc_sparsify": ([vp, vp, i64, dbl, u64, vp, vp], i64),
        "orc_estimate": ([u64, dbl], dbl),
        "orc_sampled_local": ([vp, vp, i64, i32, vp, i32, vp, vp], ctypes.c_int),
        "orc_num_threads": ([], ctypes.c_int),
        "orc_coreness": ([vp, vp, i32, vp], None),
        "orc_partition_work": ([vp, vp, vp, i32, ctypes.c_int, i32, vp, vp], None),
        "orc_order_positions": ([vp, i32, vp], None),
        "orc_shard_bounds": ([vp, vp, i32, vp, i32, ctypes.c_int, vp], None),
        "orc_count_nin_pos_range": ([vp, vp, i32, vp, i32, i32], u64),
        "orc_partition_seed": ([u64, i32], u64),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _p(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleRangeError(ValueError):
    pass


# ------------------------------------------------------------ the simple graph

def simple(src, dst, n: int):
    """Unique undirected edges (lo < hi, sorted) of the simple graph of Section 2.
    Self-loops dropped, duplicates merged; raises OracleRangeError for ids outside [0,n)."""
    src, dst = _i32(src), _i32(dst)
    E = src.shape[0]
    lo = np.empty(max(E, 1), np.int32)
    hi = np.empty(max(E, 1), np.int32)
    m = _load().orc_simple(_p(src), _p(dst), E, n, _p(lo), _p(hi))
    if m < 0:
        raise OracleRangeError("vertex id outside [0, n)")
    return lo[:m].copy(), hi[:m].copy()


def degrees(lo, hi, n: int) -> np.ndarray:
    """d_v = |N(v)| (Section 2), int64[n]."""
    deg = np.zeros(max(n, 1), np.int64)
    _load().orc_degrees(_p(lo), _p(hi), lo.shape[0], n, _p(deg))
    return deg[:n]


def full_adjacency(lo, hi, n: int):
    """Full sorted adjacency: (off int64[n+1], nbr int32[2m])."""
    off = np.zeros(n + 1, np.int64)
    nbr = np.empty(max(2 * lo.shape[0], 1), np.int32)
    _load().orc_full_adjacency(_p(lo), _p(hi), lo.shape[0], n, _p(off), _p(nbr))
    return off, nbr[: 2 * lo.shape[0]]


def coreness(off, nbr, n: int) -> np.ndarray:
    """Coreness of every vertex (the k-core order of Section 4) from the full
    adjacency, by bucket peeling; int32[n]."""
    core = np.zeros(max(n, 1), np.int32)
    _load().orc_coreness(_p(off), _p(nbr), n, _p(core))
    return core[:n]


PARTITION_SCHEMES = ("N", "D", "DH", "DDH", "DH2", "DPD", "ANOP")


def partition_work(off, adj, deg, n: int, scheme: int, parts: int):
    """Section 5 load balancing (cost-function table) and the Section 6 cost:
    boundary nodes x_j = argmin F(v) >= j*alpha over ids, and the NodeIteratorN
    merge work of each partition. Returns (bounds int64[parts+1], work uint64[parts])."""
    bounds = np.zeros(parts + 1, np.int64)
    work = np.zeros(parts, np.uint64)
    deg = np.ascontiguousarray(deg, dtype=np.int64)
    _load().orc_partition_work(_p(off), _p(adj), _p(deg), n, scheme, parts, _p(bounds), _p(work))
    return bounds, work


def local_counts_def(off, nbr, n: int):
    """Route (1), Section 2: T_v = |{(u,w) in E : u,w in N(v)}|; returns (T, t uint64[n])."""
    t = np.zeros(max(n, 1), np.uint64)
    T = _load().orc_local_counts_def(_p(off), _p(nbr), n, _p(t))
    return int(T), t[:n]


def orient(lo, hi, deg, n: int):
    """NodeIteratorN preprocessing (Section 3): orient by Eq. (1), sort each N_v by id.
    Returns (off int64[n+1], adj int32[m])."""
    off = np.zeros(n + 1, np.int64)
    adj = np.empty(max(lo.shape[0], 1), np.int32)
    deg = np.ascontiguousarray(deg, dtype=np.int64)
    _load().orc_orient(_p(lo), _p(hi), lo.shape[0], _p(deg), n, _p(off), _p(adj))
    return off, adj[: lo.shape[0]]


def orient_by_key(lo, hi, key, n: int):
    """Orientation by an arbitrary per-vertex key (ties by id): any total order (Section 4)."""
    off = np.zeros(n + 1, np.int64)
    adj = np.empty(max(lo.shape[0], 1), np.int32)
    key = np.ascontiguousarray(key, dtype=np.int64)
    _load().orc_orient_by_key(_p(lo), _p(hi), lo.shape[0], _p(key), n, _p(off), _p(adj))
    return off, adj[: lo.shape[0]]


def count_nin(off, adj, n: int, per_node: bool = False, listing: bool = False, cap: int = -1):
    """NodeIteratorN counting loop (Section 3); per-node counts as in Section 9,
    triangles as in Section 8 (each sorted ascending, list sorted lexicographically).
    Returns (T, t or None, tri or None)."""
    L = _load()
    t = np.zeros(max(n, 1), np.uint64) if per_node else None
    tri = None
    if listing:
        if cap < 0:
            cap = int(L.orc_count_nin(_p(off), _p(adj), n, None, None, 0))
        tri = np.empty((max(cap, 1), 3), np.int32)
    T = int(L.orc_count_nin(_p(off), _p(adj), n, _p(t), _p(tri), cap if listing else 0))
    if listing:
        k = min(T, cap)
        tri = tri[:k].copy()
        L.orc_sort_triples(_p(tri), k)
    return T, (t[:n] if per_node else None), tri


def count_nin_total_omp(off, adj, n: int) -> int:
    return int(_load().orc_count_nin_total_omp(_p(off), _p(adj), n))


def order_positions(key, n: int) -> np.ndarray:
    """Position of every vertex in the total order by (key, id) ascending (Eq. (1) with key = degree); int32[n]."""
    key = np.ascontiguousarray(key, dtype=np.int64)
    pos = np.zeros(max(n, 1), np.int32)
    _load().orc_order_positions(_p(key), n, _p(pos))
    return pos[:n]


def shard_bounds(off, adj, n: int, pos, k: int, cost: int = 0) -> np.ndarray:
    """Boundary positions of k core-node shards: the rule x_j = argmin F >= j*alpha over positions,
    with f(v) = sum_{u in N_v} (dhat_v + dhat_u) (cost 0, Section 5 cost-function table) or
    2 dhat_v (dhat_v - 1) + 16 dhat_v + sum_{u in N_v} dhat_u (cost 1); int64[k+1]."""
    pos = _i32(pos)
    bounds = np.zeros(k + 1, np.int64)
    _load().orc_shard_bounds(_p(off), _p(adj), n, _p(pos), k, int(cost), _p(bounds))
    return bounds


def count_nin_pos_range(off, adj, n: int, pos, p0: int, p1: int) -> int:
    """NodeIteratorN over the core nodes whose position lies in [p0, p1) (triangles by lowest vertex)."""
    pos = _i32(pos)
    return int(_load().orc_count_nin_pos_range(_p(off), _p(adj), n, _p(pos), p0, p1))


def partition_seed(seed: int, i: int) -> int:
    """Output i+1 of SplitMix64 started at seed: the seed of shard i's sample."""
    return int(_load().orc_partition_seed(int(seed) & (2 ** 64 - 1), i))


def work(off, adj, n: int) -> int:
    """W = sum over oriented edges (v,u) of (dhat_v + dhat_u) (Theorem 2)."""
    return int(_load().orc_work(_p(off), _p(adj), n))


def count_nodeiterpp(off_full, nbr, deg, n: int) -> int:
    """NodeIterator++ (Section 3, first figure) with binary-search edge tests."""
    deg = np.ascontiguousarray(deg, dtype=np.int64)
    return int(_load().orc_count_nodeiterpp(_p(off_full), _p(nbr), _p(deg), n))


def clustering(t, deg, n: int):
    """C_v = T_v / C(d_v,2) (Section 2) as (num uint64, den uint64, c float64); d_v<2 -> 0/0, 0.0."""
    t = np.ascontiguousarray(t, dtype=np.uint64)
    deg = np.ascontiguousarray(deg, dtype=np.int64)
    num = np.zeros(max(n, 1), np.uint64)
    den = np.zeros(max(n, 1), np.uint64)
    c = np.zeros(max(n, 1), np.float64)
    _load().orc_clustering(_p(t), _p(deg), n, _p(num), _p(den), _p(c))
    return num[:n], den[:n], c[:n]


def keep_threshold(q: float) -> int:
    return int(_load().orc_keep_threshold(q))


def keep(a: int, b: int, q: float, seed: int) -> bool:
    return bool(_load().orc_keep(a, b, q, seed))


def sparsify(lo, hi, q: float, seed: int):
    """Retained edges of the Section 7 sample (each undirected edge kept independently)."""
    m = lo.shape[0]
    klo = np.empty(max(m, 1), np.int32)
    khi = np.empty(max(m, 1), np.int32)
    k = _load().orc_sparsify(_p(lo), _p(hi), m, q, seed, _p(klo), _p(khi))
    return klo[:k].copy(), khi[:k].copy()


def estimate(Ts: int, q: float) -> float:
    """T_s / q^3 (Section 7)."""
    return float(_load().orc_estimate(Ts, q))


def sampled_local(src, dst, n: int, sample):
    """T_v and d_v by the Section 2 definition for up to 64 sampled vertices, from raw edges."""
    src, dst = _i32(src), _i32(dst)
    sample = _i32(sample)
    k = sample.shape[0]
    t = np.zeros(max(k, 1), np.uint64)
    d = np.zeros(max(k, 1), np.int64)
    rc = _load().orc_sampled_local(_p(src), _p(dst), src.shape[0], n, _p(sample), k, _p(t), _p(d))
    if rc != 0:
        raise ValueError("bad sample")
    return t[:k], d[:k]


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ------------------------------------------------------------------ pipeline

@dataclass
class OracleResult:
    n: int
    m: int
    T: int
    deg: np.ndarray
    off: np.ndarray  # oriented CSR (ids, rows ascending)
    adj: np.ndarray
    t: Optional[np.ndarray] = None
    tri: Optional[np.ndarray] = None
    num: Optional[np.ndarray] = None
    den: Optional[np.ndarray] = None
    cc: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)


def solve(src, dst, n: int, per_node: bool = True, listing: bool = False) -> OracleResult:
    """The whole NodeIteratorN path on the CPU: simple graph, degrees, orientation,
    count, per-node counts, clustering and (optionally) the sorted triangle list."""
    lo, hi = simple(src, dst, n)
    deg = degrees(lo, hi, n)
    off, adj = orient(lo, hi, deg, n)
    T, t, tri = count_nin(off, adj, n, per_node=per_node, listing=listing)
    r = OracleResult(n=n, m=int(lo.shape[0]), T=T, deg=deg, off=off, adj=adj, t=t, tri=tri)
    if per_node:
        r.num, r.den, r.cc = clustering(t, deg, n)
    r.extra["lo"], r.extra["hi"] = lo, hi
    return r


def sparsified_count(lo, hi, deg, n: int, q: float, seed: int):
    """(T_s, m', estimate) on the retained edges, oriented by the original degrees."""
    klo, khi = sparsify(lo, hi, q, seed)
    off, adj = orient(klo, khi, deg, n)
    Ts, _, _ = count_nin(off, adj, n)
    return Ts, int(klo.shape[0]), estimate(Ts, q)


def sparsified_count_partitioned(lo, hi, deg, n: int, q: float, seed: int, parts: int):
    """Section 7 sparsification with overlapping partitions: the core nodes are split into
    `parts` shards (``shard_bounds`` on the degree-ordered graph); shard i keeps each edge
    independently under ``partition_seed(seed, i)`` and counts the triangles of its sample
    whose lowest vertex is one of its core nodes. Returns (T_parts, bounds, sum, estimate)."""
    off, adj = orient(lo, hi, deg, n)
    pos = order_positions(deg, n)
    bounds = shard_bounds(off, adj, n, pos, parts)
    T_parts = []
    for i in range(parts):
        klo, khi = sparsify(lo, hi, q, partition_seed(seed, i))
        soff, sadj = orient(klo, khi, deg, n)
        T_parts.append(count_nin_pos_range(soff, sadj, n, pos, int(bounds[i]), int(bounds[i + 1])))
    Ts = sum(T_parts)
    return T_parts, bounds, Ts, estimate(Ts, q)
