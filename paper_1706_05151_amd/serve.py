"""Serving layer: exact-count, clustering and sparsified-estimate requests on a
pool of graphs kept resident in HBM, answered with continuous batching.

* Registry: device-resident graphs (tc_build_csr) and their edge samples
  (tc_sparsify_build), admitted under an HBM byte budget with LRU eviction of
  graphs no in-flight batch uses.
* Scheduler: requests that have arrived are taken in arrival order into the
  next batch while earlier batches still run; up to `streams` batches are in
  flight at once, each on its own HIP stream, so their work overlaps on the
  device. A batch is one tc_multi_count launch for its totals (full graphs and
  samples together), one for its per-node counts, the clustering epilogues and
  asynchronous copies of the answers into pinned host memory.
* Latency: from the request's arrival time to the moment its answer is
  visible on the host; p50/p99 over the trace.

The FIFO baseline answers the same trace one request at a time with the
single-graph calls (tc_count, tc_clustering, tc_count on the cached sample) on
the same resident data.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import tc

COUNT, CLUSTER, SPARSE = "count", "cluster", "sparse"


@dataclass
class Request:
    rid: int
    kind: str
    graph: int
    arrival: float  # seconds since the start of the trace
    q: float = 0.2
    seed: int = 5


@dataclass
class Answer:
    rid: int
    kind: str
    value: object  # int T (count), float estimate (sparse), (num, den, c) arrays (cluster)
    done: float = 0.0
    error: str = ""


_K_V, _K_B = np.uint64(0x434C555354455221), np.uint64(0x4449474553543132)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on uint64 arrays (wrapping arithmetic)."""
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def cc_digest(num, den, c) -> str:
    """128-bit digest of a clustering answer (numerators, denominators and the
    doubles, bit for bit), computed on the host from its arrays: answers are
    compared and stored by digest so the host keeps no per-request arrays. It
    is the digest tc_clustering_digest computes on the device (see tc.h)."""
    num = np.asarray(num).astype(np.uint64, copy=False)
    den = np.asarray(den).astype(np.uint64, copy=False)
    cb = np.ascontiguousarray(np.asarray(c, dtype=np.float64)).view(np.uint64)
    v = np.arange(num.shape[0], dtype=np.uint64)
    with np.errstate(over="ignore"):
        h = _mix64(_mix64(_mix64(_mix64(v ^ _K_V) ^ num) ^ den) ^ cb)
        a = int(h.sum(dtype=np.uint64)) if h.size else 0
        b = int(_mix64(h ^ _K_B).sum(dtype=np.uint64)) if h.size else 0
    return _digest_hex(a, b)


def _digest_hex(a: int, b: int) -> str:
    return f"{a & 0xFFFFFFFFFFFFFFFF:016x}{b & 0xFFFFFFFFFFFFFFFF:016x}"


def device_cc_digest(num, den, c, n: int, out, stream=None):
    """Queue the device digest of a clustering answer into out (int64[2] device tensor)."""
    tc.clustering_digest(num, den, c, n, out, stream)


def footprint_bytes(n: int, m: int) -> int:
    """Estimate of a graph's device bytes before it is built (CSR, in-edge
    records, offsets, ranks and degrees, with headroom for the work plan):
    room is made for this much, and once built the graph is charged what
    tc_graph_bytes reports."""
    return 24 * m + 48 * n + (1 << 16)


class Registry:
    def __init__(self, edge_lists, budget_bytes: int, stream=None):
        self.edge_lists = edge_lists
        self.budget = budget_bytes
        self.used = 0
        self.stream = stream
        self.graphs: "collections.OrderedDict[object, tc.Graph]" = collections.OrderedDict()
        self.sizes: Dict[object, int] = {}
        self.pinned: Dict[object, int] = collections.Counter()
        self.builds = 0
        self.evictions = 0
        self.peak = 0             # largest resident bytes right after a build
        self.peak_after_evict = 0  # largest resident bytes once room was made (> budget only if pinned graphs hold it)

    def _evict_for(self, need: int):
        for key in list(self.graphs.keys()):
            if self.used + need <= self.budget:
                return True
            if self.pinned[key] > 0:
                continue
            g = self.graphs.pop(key)
            g.close()
            self.used -= self.sizes.pop(key)
            self.evictions += 1
        return self.used + need <= self.budget

    def get(self, gid: int, sample=None) -> Optional[tc.Graph]:
        """The resident graph (or its sample (q, seed)); builds it if there is room.
        Returns None when the budget is held by graphs in flight."""
        key = gid if sample is None else (gid, sample[0], sample[1])
        if key in self.graphs:
            self.graphs.move_to_end(key)
            return self.graphs[key]
        el = self.edge_lists[gid]
        need = footprint_bytes(el.n, el.num_edges)
        if sample is not None:
            need = footprint_bytes(el.n, int(el.num_edges * sample[0]) + 1)
            base = self.get(gid)
            if base is None:
                return None
            self.pinned[gid] += 1  # the sample is drawn from the resident graph: keep it while making room
            try:
                ok = self._evict_for(need)
            finally:
                self.pinned[gid] -= 1
            if not ok:
                return None
        elif not self._evict_for(need):
            return None
        if sample is None:
            import torch

            src = torch.from_numpy(el.src).cuda(non_blocking=False)
            dst = torch.from_numpy(el.dst).cuda(non_blocking=False)
            g = tc.Graph.build(src, dst, el.n, self.stream)
            need = footprint_bytes(g.n, g.m)
        else:
            g = self.graphs[gid].sparsify_build(sample[0], sample[1], self.stream)
            need = footprint_bytes(g.n, g.m)
        self.builds += 1
        need = g.bytes()  # what the library really holds for it
        self.graphs[key] = g
        self.sizes[key] = need
        self.used += need
        self.peak = max(self.peak, self.used)
        if self.used > self.budget:  # the estimate was short: make room behind the new graph
            self.pinned[key] += 1
            try:
                self._evict_for(0)
            finally:
                self.pinned[key] -= 1
            self.peak_after_evict = max(self.peak_after_evict, self.used)
        return g

    def pin(self, keys):
        for k in keys:
            self.pinned[k] += 1

    def unpin(self, keys):
        for k in keys:
            self.pinned[k] -= 1

    def close(self):
        for g in self.graphs.values():
            g.close()
        self.graphs.clear()
        self.used = 0


class _Batch:
    def __init__(self, reqs, stream, event, keys, T_host, cc_host, tot_keys, cc_reqs, sparse_q):
        self.reqs = reqs
        self.stream = stream
        self.event = event
        self.keys = keys
        self.T_host = T_host
        self.cc_host = cc_host
        self.tot_keys = tot_keys
        self.cc_reqs = cc_reqs
        self.sparse_q = sparse_q
        self.keep = []


class Server:
    def __init__(self, registry: Registry, max_batch: int = 64, streams: int = 3):
        import torch

        self.torch = torch
        self.reg = registry
        self.max_batch = max_batch
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.inflight: List[_Batch] = []
        self.answers: Dict[int, Answer] = {}
        self.batches = 0
        self.batch_sizes: List[int] = []

    # ------------------------------------------------------------ batching
    def _launch(self, reqs: List[Request], stream) -> Optional[_Batch]:
        torch = self.torch
        keys_tot: List[object] = []     # distinct graphs/samples needing totals
        idx_tot: Dict[object, int] = {}
        cc_keys: List[int] = []         # distinct graphs needing per-node counts
        idx_cc: Dict[int, int] = {}
        graphs_tot, graphs_cc = [], []
        pins: List[object] = []  # graphs are pinned as they are fetched so later fetches cannot evict them
        for r in reqs:
            if r.kind == CLUSTER:
                if r.graph not in idx_cc:
                    g = self.reg.get(r.graph)
                    if g is None:
                        self.reg.unpin(pins)
                        return None
                    self.reg.pin([r.graph])
                    pins.append(r.graph)
                    idx_cc[r.graph] = len(cc_keys)
                    cc_keys.append(r.graph)
                    graphs_cc.append(g)
            else:
                key = r.graph if r.kind == COUNT else (r.graph, r.q, r.seed)
                if key not in idx_tot:
                    g = self.reg.get(r.graph, None if r.kind == COUNT else (r.q, r.seed))
                    if g is None:
                        self.reg.unpin(pins)
                        return None
                    self.reg.pin([key])
                    pins.append(key)
                    idx_tot[key] = len(keys_tot)
                    keys_tot.append(key)
                    graphs_tot.append(g)
        with torch.cuda.stream(stream):
            T_dev = torch.empty(max(len(graphs_tot), 1), dtype=torch.int64, device="cuda")
            T_host = torch.empty(max(len(graphs_tot), 1), dtype=torch.int64, pin_memory=True)
            keep = [T_dev]
            if graphs_tot:
                tc.multi_count(graphs_tot, T_dev, None, stream)
                T_host.copy_(T_dev, non_blocking=True)
            cc_host = None
            if graphs_cc:
                Tc = torch.empty(len(graphs_cc), dtype=torch.int64, device="cuda")
                ts = [torch.empty(max(g.n, 1), dtype=torch.int64, device="cuda") for g in graphs_cc]
                tc.multi_count(graphs_cc, Tc, ts, stream)
                keep += [Tc] + ts
                dig = torch.empty((len(graphs_cc), 2), dtype=torch.int64, device="cuda")
                for i, (g, t) in enumerate(zip(graphs_cc, ts)):
                    num = torch.empty(max(g.n, 1), dtype=torch.int64, device="cuda")
                    den = torch.empty(max(g.n, 1), dtype=torch.int64, device="cuda")
                    c = torch.empty(max(g.n, 1), dtype=torch.float64, device="cuda")
                    g.clustering_from_counts(t, num, den, c, stream)
                    device_cc_digest(num, den, c, g.n, dig[i], stream)
                    keep += [num, den, c]
                cc_host = torch.empty((len(graphs_cc), 2), dtype=torch.int64, pin_memory=True)
                cc_host.copy_(dig, non_blocking=True)
                keep.append(dig)
            ev = torch.cuda.Event()
            ev.record(stream)
        b = _Batch(reqs, stream, ev, pins, T_host, cc_host, idx_tot, idx_cc, None)
        b.keep = keep
        return b

    def _finish(self, b: _Batch, now: float):
        T = b.T_host.numpy()
        for r in b.reqs:
            if r.kind == COUNT:
                val = int(T[b.tot_keys[r.graph]])
            elif r.kind == SPARSE:
                val = tc.sparsify_estimate(int(T[b.tot_keys[(r.graph, r.q, r.seed)]]), r.q)
            else:
                d = b.cc_host[b.cc_reqs[r.graph]]
                val = _digest_hex(int(d[0]), int(d[1]))
            self.answers[r.rid] = Answer(r.rid, r.kind, val, now)
        self.reg.unpin(b.keys)
        b.keep = b.cc_host = b.T_host = None  # pinned and device buffers return to torch's caches
        self.batch_sizes.append(len(b.reqs))

    def _poll(self, clock) -> bool:
        done_any = False
        still = []
        for b in self.inflight:
            if b.event.query():
                self._finish(b, clock())
                done_any = True
            else:
                still.append(b)
        self.inflight = still
        return done_any

    def run(self, trace: List[Request], t0: Optional[float] = None) -> Dict[int, Answer]:
        """Serve an open-loop trace (arrival times relative to the start)."""
        start = time.perf_counter() if t0 is None else t0
        clock = lambda: time.perf_counter() - start  # noqa: E731
        pending = collections.deque(sorted(trace, key=lambda r: r.arrival))
        ready: collections.deque = collections.deque()
        free_streams = list(self.streams)
        while pending or ready or self.inflight:
            now = clock()
            while pending and pending[0].arrival <= now:
                ready.append(pending.popleft())
            if self._poll(clock):
                free_streams = [s for s in self.streams if all(b.stream is not s for b in self.inflight)]
            if ready and free_streams:
                reqs = [ready.popleft() for _ in range(min(self.max_batch, len(ready)))]
                b = self._launch(reqs, free_streams[0])
                if b is None:  # HBM budget held by batches in flight: wait for one to finish
                    if self.inflight:
                        for r in reversed(reqs):
                            ready.appendleft(r)
                        self.inflight[0].event.synchronize()
                        continue
                    if len(reqs) > 1:  # retry the oldest request alone
                        for r in reversed(reqs[1:]):
                            ready.appendleft(r)
                        b = self._launch(reqs[:1], free_streams[0])
                        reqs = reqs[:1]
                    if b is None:  # its graph alone exceeds the budget
                        self.answers[reqs[0].rid] = Answer(reqs[0].rid, reqs[0].kind, None, clock(), "TC_E_NOMEM")
                        continue
                self.inflight.append(b)
                self.batches += 1
                free_streams = free_streams[1:]
                continue
            if not ready and not self.inflight and pending:
                wait = pending[0].arrival - clock()
                if wait > 0:
                    time.sleep(min(wait, 0.002))
            elif self.inflight and (not ready or not free_streams):
                time.sleep(0.0001)
        return self.answers


def _answer_digest(g) -> str:
    """tc_clustering on one graph and the device digest of its answer (16 bytes to the host)."""
    import torch

    num, den, c = g.clustering()
    d = torch.empty(2, dtype=torch.int64, device="cuda")
    device_cc_digest(num, den, c, g.n, d)
    h = d.cpu()
    return _digest_hex(int(h[0]), int(h[1]))


def serve_fifo(registry: Registry, trace: List[Request], t0: Optional[float] = None) -> Dict[int, Answer]:
    """One request at a time, in arrival order, with the single-graph calls."""
    import torch

    start = time.perf_counter() if t0 is None else t0
    answers = {}
    for r in sorted(trace, key=lambda r: r.arrival):
        now = time.perf_counter() - start
        if r.arrival > now:
            time.sleep(r.arrival - now)
        if r.kind == COUNT:
            val = registry.get(r.graph).count()
        elif r.kind == SPARSE:
            val = tc.sparsify_estimate(registry.get(r.graph, (r.q, r.seed)).count(), r.q)
        else:
            g = registry.get(r.graph)
            answers[r.rid] = Answer(r.rid, r.kind, _answer_digest(g), time.perf_counter() - start)
            continue
        torch.cuda.synchronize()
        answers[r.rid] = Answer(r.rid, r.kind, val, time.perf_counter() - start)
    return answers


def serve_plain(edges_dev, trace: List[Request]) -> Tuple[Dict[int, Answer], float]:
    """The plain per-graph launch: for each request in arrival order, as fast as
    possible, build its graph from the edge list already in HBM, answer it with
    the single-graph calls and free the graph (no registry, no batching).
    edges_dev[g] = (src, dst, n) device tensors. Returns (answers, wall seconds)."""
    import torch

    answers = {}
    torch.cuda.synchronize()
    start = time.perf_counter()
    for r in sorted(trace, key=lambda r: r.arrival):
        src, dst, n = edges_dev[r.graph]
        with tc.Graph.build(src, dst, n) as g:
            if r.kind == COUNT:
                val = g.count()
            elif r.kind == SPARSE:
                val = g.sparsify_count(r.q, r.seed)[2]
            else:
                val = _answer_digest(g)
        answers[r.rid] = Answer(r.rid, r.kind, val, time.perf_counter() - start)
    torch.cuda.synchronize()
    return answers, time.perf_counter() - start


def make_trace(num_graphs: int, rate: float, duration: float, seed: int, mix=(0.6, 0.25, 0.15), q: float = 0.2):
    """Poisson arrivals; graph uniform over the pool; kind by the request mix."""
    import synth

    t = synth.poisson_arrivals(rate, duration, seed)
    u = synth.draws(seed, 0x5245515553, 2 * len(t))
    reqs = []
    c1, c2 = mix[0], mix[0] + mix[1]
    for i, a in enumerate(t):
        g = int(u[2 * i] % np.uint64(num_graphs))
        x = float(u[2 * i + 1] >> np.uint64(11)) / 9007199254740992.0
        kind = COUNT if x < c1 else (CLUSTER if x < c2 else SPARSE)
        reqs.append(Request(i, kind, g, float(a), q=q, seed=seed))
    return reqs


def latency_stats(trace: List[Request], answers: Dict[int, Answer], wall: float):
    lat = np.array([answers[r.rid].done - r.arrival for r in trace])
    return {"requests": len(trace), "errors": sum(1 for r in trace if answers[r.rid].error), "wall_s": wall,
            "req_per_s": len(trace) / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


def same_answer(a: Answer, b: Answer) -> bool:
    """Exact equality: counts, estimate doubles and clustering digests."""
    return a.kind == b.kind and a.value == b.value and not a.error and not b.error
