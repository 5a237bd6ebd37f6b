"""ctypes binding of the C ABI in include/tc.h (argument marshalling only).

Every operation runs in the HIP kernels of ``libtc.so``; PyTorch only supplies
device memory and the current HIP stream. There is no CPU fallback: if the
library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_OK, TC_E_INVAL, TC_E_NOMEM, TC_E_DEVICE, TC_E_RANGE, TC_E_TRUNC = 0, -1, -2, -3, -4, -5
TC_IN_DEVICE = 1
OPT_KERNEL, OPT_HUB_DHAT, OPT_ITEM_WORK, OPT_BLOCKS_PER_CU, OPT_HUB_BUCKET_LOAD, OPT_ORDER = 0, 1, 2, 3, 4, 5
ORDER_DEGREE, ORDER_ID, ORDER_RANDOM, ORDER_DEGREE_DESC, ORDER_CORE = 0, 1, 2, 3, 4
SCHEME_N, SCHEME_D, SCHEME_DH, SCHEME_DDH, SCHEME_DH2, SCHEME_DPD, SCHEME_ANOP = range(7)

# (name, argtypes, restype) for every symbol include/tc.h declares
_vp, _i32, _i64, _u32, _u64, _dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_double)
_P = ctypes.POINTER
SIGNATURES = {
    "tc_build_csr": ([_vp, _vp, _i64, _i32, _u32, _vp, _P(_vp)], ctypes.c_int),
    "tc_graph_info": ([_vp, _P(_i32), _P(_i64), _P(_i32), _P(_i32)], ctypes.c_int),
    "tc_graph_free": ([_vp], None),
    "tc_graph_bytes": ([_vp, _P(_u64)], ctypes.c_int),
    "tc_count": ([_vp, _vp, _P(_u64)], ctypes.c_int),
    "tc_count_per_node": ([_vp, _vp, _P(_u64), _vp], ctypes.c_int),
    "tc_count_per_node_noalloc": ([_vp, _vp, _P(_u64), _vp], ctypes.c_int),
    "tc_clustering": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "tc_list": ([_vp, _vp, _vp, _i64, _P(_i64)], ctypes.c_int),
    "tc_sparsify_count": ([_vp, _dbl, _u64, _vp, _P(_u64), _P(_i64), _P(_dbl)], ctypes.c_int),
    "tc_count_plain": ([_vp, _vp, _P(_u64)], ctypes.c_int),
    "tc_graph_work": ([_vp, _vp, _P(_u64), _P(_u64)], ctypes.c_int),
    "tc_graph_degrees": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "tc_graph_order_cost": ([_vp, _vp, _P(_u64), _P(_i32)], ctypes.c_int),
    "tc_graph_coreness": ([_vp, _vp, _vp], ctypes.c_int),
    "tc_count_partitioned": ([_vp, _vp, _i32, _i32, _P(_u64), _vp, _vp], ctypes.c_int),
    "tc_graph_oriented": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "tc_graph_order": ([_vp, _vp, _vp], ctypes.c_int),
    "tc_graph_export_csr": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "tc_count_streamed": ([_vp, _vp, _i32, _i64, _u64, _vp, _P(_u64), _vp], ctypes.c_int),
    "tc_build_csr_host": ([_vp, _vp, _i64, _i32, _u64, _vp, _vp, _vp, _P(_i64), _vp], ctypes.c_int),
    "tc_shard_bounds": ([_vp, _vp, _i32, _i32, _vp], ctypes.c_int),
    "tc_count_shard": ([_vp, _vp, _i32, _i32, _P(_u64)], ctypes.c_int),
    "tc_sparsify_count_partitioned": ([_vp, _dbl, _u64, _i32, _vp, _vp, _vp, _P(_u64), _P(_dbl)], ctypes.c_int),
    "tc_graph_replan": ([_vp, _vp], ctypes.c_int),
    "tc_graph_plan_info": ([_vp, _P(_i64), _P(_i64), _P(_i32)], ctypes.c_int),
    "tc_set_option": ([ctypes.c_int, _i64], ctypes.c_int),
    "tc_get_option": ([ctypes.c_int], _i64),
    "tc_batch_build": ([_vp, _vp, _vp, _vp, _i32, _u32, _vp, _P(_vp)], ctypes.c_int),
    "tc_batch_size": ([_vp, _P(_i32)], ctypes.c_int),
    "tc_batch_count": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "tc_multi_count": ([_vp, _i32, _i32, _vp, _vp, _vp], ctypes.c_int),
    "tc_clustering_from_counts": ([_vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "tc_clustering_digest": ([_vp, _vp, _vp, _i32, _vp, _vp], ctypes.c_int),
    "tc_sparsify_build": ([_vp, _dbl, _u64, _vp, _P(_vp)], ctypes.c_int),
    "tc_sparsify_estimate": ([_u64, _dbl], _dbl),
    "tc_status_str": ([ctypes.c_int], ctypes.c_char_p),
    "tc_last_error": ([], ctypes.c_char_p),
}

_lib = None


class TCError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def lib():
    """Load libtc.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python paper_1706_05151_amd/build_lib.py")
    # PyTorch's HIP runtime is loaded first so that the library shares it (loaded the other
    # way round, a first call such as tc_set_option left no device visible to later calls)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(st: int, where: str):
    if st != TC_OK:
        L = lib()
        raise TCError(st, where, (L.tc_last_error() or b"").decode() or L.tc_status_str(st).decode())


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the triangle-counting library runs on the GPU only")
    return torch


def _stream(stream) -> ctypes.c_void_p:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a) -> ctypes.c_void_p:
    """Address of a torch tensor or a contiguous numpy array."""
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be contiguous")
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.c_void_p(a.data_ptr())


def set_option(key: int, value: int):
    _check(lib().tc_set_option(key, int(value)), "tc_set_option")


def get_option(key: int) -> int:
    return int(lib().tc_get_option(key))


class Graph:
    """A device graph built by tc_build_csr / tc_batch_build (freed on close/del)."""

    def __init__(self, handle: ctypes.c_void_p, device: int):
        self._h = handle
        self.device = device
        n, m, dmax, dhmax = _i32(), _i64(), _i32(), _i32()
        _check(lib().tc_graph_info(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(dmax), ctypes.byref(dhmax)),
               "tc_graph_info")
        self.n, self.m, self.d_max, self.dhat_max = n.value, m.value, dmax.value, dhmax.value
        ng = _i32()
        _check(lib().tc_batch_size(self._h, ctypes.byref(ng)), "tc_batch_size")
        self.num_graphs = ng.value

    # ------------------------------------------------------------ builders
    @classmethod
    def build(cls, src, dst, n: int, stream=None) -> "Graph":
        """src/dst: int32 device tensors, or host numpy arrays (copied by the library)."""
        torch = _torch()
        h = _vp()
        if isinstance(src, np.ndarray):
            s = np.ascontiguousarray(src, dtype=np.int32)
            d = np.ascontiguousarray(dst, dtype=np.int32)
            st = lib().tc_build_csr(s.ctypes.data_as(_vp), d.ctypes.data_as(_vp), s.shape[0], int(n), 0,
                                    _stream(stream), ctypes.byref(h))
        else:
            assert src.dtype == torch.int32 and dst.dtype == torch.int32 and src.is_cuda
            s, d = src.contiguous(), dst.contiguous()
            st = lib().tc_build_csr(_dptr(s), _dptr(d), s.numel(), int(n), TC_IN_DEVICE, _stream(stream),
                                    ctypes.byref(h))
        _check(st, "tc_build_csr")
        return cls(h, torch.cuda.current_device())

    @classmethod
    def build_batch(cls, src, dst, edge_off: np.ndarray, n_per_graph: np.ndarray, stream=None) -> "Graph":
        """Disjoint union of many graphs; ids in src/dst are local to each graph."""
        torch = _torch()
        h = _vp()
        eo = np.ascontiguousarray(edge_off, dtype=np.int64)
        npg = np.ascontiguousarray(n_per_graph, dtype=np.int32)
        if isinstance(src, np.ndarray):
            s = np.ascontiguousarray(src, dtype=np.int32)
            d = np.ascontiguousarray(dst, dtype=np.int32)
            st = lib().tc_batch_build(s.ctypes.data_as(_vp), d.ctypes.data_as(_vp), eo.ctypes.data_as(_vp),
                                      npg.ctypes.data_as(_vp), npg.shape[0], 0, _stream(stream), ctypes.byref(h))
        else:
            s, d = src.contiguous(), dst.contiguous()
            st = lib().tc_batch_build(_dptr(s), _dptr(d), eo.ctypes.data_as(_vp), npg.ctypes.data_as(_vp),
                                      npg.shape[0], TC_IN_DEVICE, _stream(stream), ctypes.byref(h))
        _check(st, "tc_batch_build")
        return cls(h, torch.cuda.current_device())

    # ------------------------------------------------------------- queries
    def bytes(self) -> int:
        """Device bytes the graph holds (tc_graph_bytes)."""
        b = _u64()
        _check(lib().tc_graph_bytes(self._h, ctypes.byref(b)), "tc_graph_bytes")
        return b.value

    def count(self, stream=None) -> int:
        T = _u64()
        _check(lib().tc_count(self._h, _stream(stream), ctypes.byref(T)), "tc_count")
        return T.value

    def count_plain(self, stream=None) -> int:
        T = _u64()
        _check(lib().tc_count_plain(self._h, _stream(stream), ctypes.byref(T)), "tc_count_plain")
        return T.value

    def count_per_node(self, out=None, stream=None) -> Tuple[int, "object"]:
        torch = _torch()
        t = out if out is not None else torch.empty(max(self.n, 1), dtype=torch.int64, device="cuda")
        T = _u64()
        _check(lib().tc_count_per_node(self._h, _stream(stream), ctypes.byref(T), _dptr(t)), "tc_count_per_node")
        return T.value, t[: self.n]

    def count_per_node_noalloc(self, out, stream=None) -> Tuple[int, "object"]:
        """tc_count_per_node_noalloc: the counts of count_per_node with no device allocation in the
        library (static scratch, at most 2^22 vertices); out: int64[n] device tensor."""
        T = _u64()
        _check(lib().tc_count_per_node_noalloc(self._h, _stream(stream), ctypes.byref(T), _dptr(out)),
               "tc_count_per_node_noalloc")
        return T.value, out[: self.n]

    def clustering(self, stream=None):
        torch = _torch()
        k = max(self.n, 1)
        num = torch.empty(k, dtype=torch.int64, device="cuda")
        den = torch.empty(k, dtype=torch.int64, device="cuda")
        c = torch.empty(k, dtype=torch.float64, device="cuda")
        _check(lib().tc_clustering(self._h, _stream(stream), _dptr(num), _dptr(den), _dptr(c)), "tc_clustering")
        return num[: self.n], den[: self.n], c[: self.n]

    def list_size(self, stream=None) -> int:
        cnt = _i64()
        _check(lib().tc_list(self._h, _stream(stream), None, 0, ctypes.byref(cnt)), "tc_list")
        return cnt.value

    def list(self, cap: Optional[int] = None, stream=None):
        torch = _torch()
        if cap is None:
            cap = self.list_size(stream)
        tri = torch.empty((max(cap, 1), 3), dtype=torch.int32, device="cuda")
        cnt = _i64()
        st = lib().tc_list(self._h, _stream(stream), _dptr(tri), int(cap), ctypes.byref(cnt))
        _check(st, "tc_list")
        return tri[: cnt.value]

    def sparsify_count(self, q: float, seed: int, stream=None):
        Ts, mk, est = _u64(), _i64(), _dbl()
        _check(lib().tc_sparsify_count(self._h, float(q), int(seed) & (2 ** 64 - 1), _stream(stream), ctypes.byref(Ts),
                                       ctypes.byref(mk), ctypes.byref(est)), "tc_sparsify_count")
        return Ts.value, mk.value, est.value

    def work(self, stream=None) -> Tuple[int, int]:
        W, P = _u64(), _u64()
        _check(lib().tc_graph_work(self._h, _stream(stream), ctypes.byref(W), ctypes.byref(P)), "tc_graph_work")
        return W.value, P.value

    def order_cost(self, stream=None) -> Tuple[int, int]:
        """(sum_v d_v * dhat_v, order kind the graph was built with)."""
        c, k = _u64(), _i32()
        _check(lib().tc_graph_order_cost(self._h, _stream(stream), ctypes.byref(c), ctypes.byref(k)),
               "tc_graph_order_cost")
        return c.value, k.value

    def count_partitioned(self, scheme: int, parts: int, stream=None):
        """Section 5 static load balancing by cost scheme (0 N, 1 D, 2 DH, 3 DDH, 4 DH^2, 5 DPD,
        6 the Section 6 cost): (T, bounds int64[parts+1], work uint64[parts] as int64) on the device."""
        torch = _torch()
        T = _u64()
        bounds = torch.empty(parts + 1, dtype=torch.int64, device="cuda")
        work = torch.empty(parts, dtype=torch.int64, device="cuda")
        _check(lib().tc_count_partitioned(self._h, _stream(stream), int(scheme), int(parts), ctypes.byref(T),
                                          _dptr(bounds), _dptr(work)), "tc_count_partitioned")
        return T.value, bounds, work

    def coreness(self, stream=None):
        """Coreness of every vertex by caller id (k-core order of Section 4): int32[n] on the device."""
        torch = _torch()
        core = torch.empty(max(self.n, 1), dtype=torch.int32, device="cuda")
        _check(lib().tc_graph_coreness(self._h, _stream(stream), _dptr(core)), "tc_graph_coreness")
        return core[: self.n]

    def order(self, stream=None):
        """Caller id of the vertex at each position of the orientation order: int32[n] on the device."""
        torch = _torch()
        order = torch.empty(max(self.n, 1), dtype=torch.int32, device="cuda")
        _check(lib().tc_graph_order(self._h, _stream(stream), _dptr(order)), "tc_graph_order")
        return order[: self.n]

    def shard_bounds(self, k: int, cost: int = 0, stream=None) -> List[int]:
        """Positions [b[j], b[j+1]) of the core nodes of shard j: the boundary rule over the merge cost
        (cost 0, Section 5) or the pivot kernel's work model (cost 1)."""
        b = (ctypes.c_int32 * (k + 1))()
        _check(lib().tc_shard_bounds(self._h, _stream(stream), int(k), int(cost), b), "tc_shard_bounds")
        return list(b)

    def count_shard(self, lo: int, hi: int, stream=None) -> int:
        """Triangles whose lowest vertex has its position in [lo, hi) of the orientation order."""
        T = _u64()
        _check(lib().tc_count_shard(self._h, _stream(stream), int(lo), int(hi), ctypes.byref(T)), "tc_count_shard")
        return T.value

    def sparsify_count_partitioned(self, q: float, seed: int, parts: int, stream=None):
        """Per-shard independent samples (Section 7 with overlapping partitions):
        (per-shard T_s list, bounds list, sum of T_s, estimate)."""
        tp = (ctypes.c_uint64 * parts)()
        b = (ctypes.c_int32 * (parts + 1))()
        Ts, est = _u64(), _dbl()
        _check(lib().tc_sparsify_count_partitioned(self._h, float(q), int(seed) & (2 ** 64 - 1), int(parts),
                                                   _stream(stream), tp, b, ctypes.byref(Ts), ctypes.byref(est)),
               "tc_sparsify_count_partitioned")
        return list(tp), list(b), Ts.value, est.value

    def export_csr(self, off=None, adj=None, stream=None):
        """Copy the rank-space oriented CSR into off (int64[n+1]) and adj (int32[m]): torch tensors on
        the host (pinned for speed) or the device; allocated as pinned host tensors when omitted."""
        torch = _torch()
        if off is None:
            off = torch.empty(self.n + 1, dtype=torch.int64, pin_memory=True)
        if adj is None:
            adj = torch.empty(max(self.m, 1), dtype=torch.int32, pin_memory=True)
        _check(lib().tc_graph_export_csr(self._h, _stream(stream), _dptr(off), _dptr(adj)), "tc_graph_export_csr")
        return off, adj[: self.m]

    def degrees(self, stream=None):
        torch = _torch()
        k = max(self.n, 1)
        deg = torch.empty(k, dtype=torch.int32, device="cuda")
        dhat = torch.empty(k, dtype=torch.int32, device="cuda")
        _check(lib().tc_graph_degrees(self._h, _stream(stream), _dptr(deg), _dptr(dhat)), "tc_graph_degrees")
        return deg[: self.n], dhat[: self.n]

    def oriented(self, stream=None):
        torch = _torch()
        off = torch.empty(self.n + 1, dtype=torch.int64, device="cuda")
        adj = torch.empty(max(self.m, 1), dtype=torch.int32, device="cuda")
        _check(lib().tc_graph_oriented(self._h, _stream(stream), _dptr(off), _dptr(adj)), "tc_graph_oriented")
        return off, adj[: self.m]

    def replan(self, stream=None):
        """Rebuild the work plan with the current options (refused once a batch count was captured)."""
        _check(lib().tc_graph_replan(self._h, _stream(stream)), "tc_graph_replan")

    def plan_info(self) -> dict:
        """Options the current work plan was built with, and whether a capture froze it."""
        hd, iw, fr = _i64(), _i64(), _i32()
        _check(lib().tc_graph_plan_info(self._h, ctypes.byref(hd), ctypes.byref(iw), ctypes.byref(fr)),
               "tc_graph_plan_info")
        return {"hub_dhat": hd.value, "item_work": iw.value, "frozen": bool(fr.value)}

    def batch_count(self, T_out, t_out=None, stream=None):
        """Per-graph totals (int64[num_graphs]) and optional per-node counts; no host sync."""
        _check(lib().tc_batch_count(self._h, _stream(stream), _dptr(T_out), _dptr(t_out) if t_out is not None else None),
               "tc_batch_count")

    def sparsify_build(self, q: float, seed: int, stream=None) -> "Graph":
        """The Section 7 edge sample as a graph of its own (totals only)."""
        torch = _torch()
        h = _vp()
        _check(lib().tc_sparsify_build(self._h, float(q), int(seed) & (2 ** 64 - 1), _stream(stream), ctypes.byref(h)),
               "tc_sparsify_build")
        return Graph(h, torch.cuda.current_device())

    def clustering_from_counts(self, t, num, den, c, stream=None):
        _check(lib().tc_clustering_from_counts(self._h, _stream(stream), _dptr(t), _dptr(num), _dptr(den), _dptr(c)),
               "tc_clustering_from_counts")

    # ----------------------------------------------------------- lifetime
    def close(self):
        if self._h is not None and self._h.value:
            lib().tc_graph_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def multi_count(graphs, T_out, t_outs=None, stream=None):
    """One launch counting every graph of ``graphs``; T_out int64[k] (device),
    optional per-node outputs t_outs[i] int64[n_i] (device). No host sync."""
    k = len(graphs)
    arr = (_vp * max(k, 1))(*[g._h for g in graphs])
    tp = None
    if t_outs is not None:
        tp = (_vp * max(k, 1))(*[ctypes.c_void_p(t.data_ptr()) for t in t_outs])
    _check(lib().tc_multi_count(arr, k, 1 if t_outs is not None else 0, _stream(stream), _dptr(T_out), tp),
           "tc_multi_count")


def clustering_digest(num, den, c, n: int, out, stream=None):
    """Device digest of a clustering answer (tc_clustering_digest) into out: int64[2] device tensor."""
    _check(lib().tc_clustering_digest(_dptr(num), _dptr(den), _dptr(c), int(n), _stream(stream), _dptr(out)),
           "tc_clustering_digest")


def sparsify_estimate(Ts: int, q: float) -> float:
    return float(lib().tc_sparsify_estimate(int(Ts), float(q)))


def build_csr_host(src, dst, n: int, budget_bytes: int, off=None, adj=None, stream=None):
    """Rank-space oriented CSR of a host edge list (int32 numpy arrays or host tensors) built under a
    device budget (tc_build_csr_host). Returns (off int64[n+1], adj int32[m], info dict); off and adj
    are pinned host tensors unless given (adj needs room for len(src) entries)."""
    torch = _torch()
    E = int(len(src))
    if off is None:
        off = torch.empty(n + 1, dtype=torch.int64, pin_memory=True)
    if adj is None:
        adj = torch.empty(max(E, 1), dtype=torch.int32, pin_memory=True)
    m = _i64()
    info = (ctypes.c_uint64 * 4)()
    _check(lib().tc_build_csr_host(_hptr(src), _hptr(dst), E, int(n), int(budget_bytes), _stream(stream), _hptr(off),
                                   _hptr(adj), ctypes.byref(m), info), "tc_build_csr_host")
    return off, adj[: m.value], {"parts": info[0], "row_ranges": info[1], "bytes_in": info[2], "bytes_out": info[3]}


def count_streamed(off, adj, n: int, budget_bytes: int, stream=None):
    """Exact T of a rank-space oriented CSR held in host memory (off: int64[n+1] host tensor or array,
    adj: int32[m] host or device), streamed through the GPU within budget_bytes of device memory.
    Returns (T, {"partitions", "chunks" (shipped), "pairs" (partition, source range), "bytes_in"})."""
    m = int(off[n])
    T = _u64()
    info = (ctypes.c_uint64 * 4)()
    _check(lib().tc_count_streamed(_hptr(off), _hptr(adj), int(n), m, int(budget_bytes), _stream(stream),
                                   ctypes.byref(T), info), "tc_count_streamed")
    return T.value, {"partitions": info[0], "chunks": info[1], "pairs": info[2], "bytes_in": info[3]}
