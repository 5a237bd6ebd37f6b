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
    """Device-resident graphs and samples under a byte budget, least recently
    used first out. A graph is charged the estimate of footprint_bytes while it
    is being built and what tc_graph_bytes reports once it is in; pinned graphs
    (used by a batch in flight, or the base of a sample being drawn) are never
    evicted."""

    def __init__(self, edge_lists, budget_bytes: int, stream=None, host_edges=None):
        self.edge_lists = edge_lists
        self.host_edges = host_edges  # optional pinned (src, dst) tensors per graph, from pin_edge_lists
        self.budget = budget_bytes
        self.used = 0
        self.stream = stream
        self.graphs: "collections.OrderedDict[object, tc.Graph]" = collections.OrderedDict()
        self.sizes: Dict[object, int] = {}
        self.reserved: Dict[object, int] = {}
        self.pinned: Dict[object, int] = collections.Counter()
        self.builds = 0
        self.evictions = 0
        self.peak = 0  # largest bytes held (resident and reserved) right after a build

    @staticmethod
    def key_of(gid: int, sample=None):
        return gid if sample is None else (gid, sample[0], sample[1])

    def estimate(self, key) -> int:
        if isinstance(key, tuple):
            el = self.edge_lists[key[0]]
            return footprint_bytes(el.n, int(el.num_edges * key[1]) + 1)
        el = self.edge_lists[key]
        return footprint_bytes(el.n, el.num_edges)

    def _evict_for(self, need: int):
        """Evict unpinned graphs, least recently used first, until need fits; False if it cannot."""
        victims, freed = [], 0
        for key in self.graphs:
            if self.used - freed + need <= self.budget:
                break
            if self.pinned[key] > 0:
                continue
            victims.append(key)
            freed += self.sizes[key]
        if self.used - freed + need > self.budget:
            return False
        for key in victims:
            self.graphs.pop(key).close()
            self.used -= self.sizes.pop(key)
            self.evictions += 1
        return True

    def peek(self, key) -> Optional[tc.Graph]:
        """The resident graph of key, if any, without counting it as a use."""
        return self.graphs.get(key)

    def resident(self, key) -> Optional[tc.Graph]:
        """The resident graph of key, if any, counted as a use (most recently used)."""
        g = self.graphs.get(key)
        if g is not None:
            self.graphs.move_to_end(key)
        return g

    def reserve(self, key, protect=None) -> bool:
        """Make room for the estimate of key and charge it; False if the budget is held by pinned
        graphs. protect (optional) is called only when room must be made, and returns graphs that
        are then kept as if pinned."""
        need = self.estimate(key)
        if self.used + need > self.budget:
            keep = list(protect()) if protect is not None else []
            self.pin(keep)
            try:
                ok = self._evict_for(need)
            finally:
                self.unpin(keep)
            if not ok:
                return False
        self.reserved[key] = need
        self.used += need
        return True

    def cancel(self, key):
        self.used -= self.reserved.pop(key, 0)

    def build(self, key, stream=None, base: Optional[tc.Graph] = None) -> tc.Graph:
        """Build key's graph (or draw its sample from the resident base graph); no accounting."""
        if isinstance(key, tuple):
            base = base if base is not None else self.graphs[key[0]]
            return base.sparsify_build(key[1], key[2], stream if stream is not None else self.stream)
        import torch

        el = self.edge_lists[key]
        if self.host_edges is not None:  # pinned: asynchronous copies on the building stream
            hs, hd = self.host_edges[key]
            src = hs.to("cuda", non_blocking=True)
            dst = hd.to("cuda", non_blocking=True)
        else:
            src = torch.from_numpy(el.src).cuda(non_blocking=False)
            dst = torch.from_numpy(el.dst).cuda(non_blocking=False)
        return tc.Graph.build(src, dst, el.n, stream if stream is not None else self.stream)

    def install(self, key, g: tc.Graph):
        """The built graph replaces its reservation and is charged its real bytes. Nothing
        is evicted here (graphs whose requests are about to run would go): if the estimate
        was short, the next reservation makes the room."""
        self.cancel(key)
        self.builds += 1
        need = g.bytes()
        self.graphs[key] = g
        self.sizes[key] = need
        self.used += need
        self.peak = max(self.peak, self.used)

    def get(self, gid: int, sample=None) -> Optional[tc.Graph]:
        """The resident graph (or its sample (q, seed)), built here if there is room.
        Returns None when the budget is held by pinned graphs."""
        key = self.key_of(gid, sample)
        g = self.resident(key)
        if g is not None:
            return g
        if sample is not None:
            if self.get(gid) is None:
                return None
            self.pinned[gid] += 1  # the sample is drawn from the resident graph: keep it while making room
        try:
            if not self.reserve(key):
                return None
            try:
                g = self.build(key)
            except BaseException:
                self.cancel(key)
                raise
            self.install(key, g)
        finally:
            if sample is not None:
                self.pinned[gid] -= 1
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
        self.sizes.clear()
        self.reserved.clear()
        self.used = 0


def pin_edge_lists(edge_lists):
    """Pinned host copies of the pool's edge lists, (src, dst) per graph, slices of
    one pinned buffer per endpoint array, so graphs are built from them with
    asynchronous copies."""
    import torch

    sizes = [int(el.num_edges) for el in edge_lists]
    total = max(sum(sizes), 1)
    src = torch.empty(total, dtype=torch.int32, pin_memory=True)
    dst = torch.empty(total, dtype=torch.int32, pin_memory=True)
    out, o = [], 0
    for el, e in zip(edge_lists, sizes):
        src[o:o + e].copy_(torch.from_numpy(np.ascontiguousarray(el.src, dtype=np.int32)))
        dst[o:o + e].copy_(torch.from_numpy(np.ascontiguousarray(el.dst, dtype=np.int32)))
        out.append((src[o:o + e], dst[o:o + e]))
        o += e
    return out


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


class _Builder:
    """Builds graphs and samples on threads of its own, each with its own HIP
    stream, so the serving loop keeps batching requests on resident graphs
    meanwhile (the library releases the interpreter lock inside its calls and
    is safe to call from several threads on different streams)."""

    def __init__(self, registry: Registry, threads: int = 2):
        import queue
        import threading

        import torch

        self.reg = registry
        self.todo: "queue.Queue" = queue.Queue()
        self.done: "queue.Queue" = queue.Queue()
        self.spans: List[tuple] = []  # (key, start, end) of every build, perf_counter seconds
        self.device = torch.cuda.current_device()
        self.threads = [threading.Thread(target=self._run, daemon=True) for _ in range(threads)]
        for t in self.threads:
            t.start()

    def _run(self):
        import torch

        torch.cuda.set_device(self.device)
        stream = torch.cuda.Stream()
        while True:
            item = self.todo.get()
            if item is None:
                return
            key, base = item
            try:
                t0 = time.perf_counter()
                with torch.cuda.stream(stream):
                    g = self.reg.build(key, stream, base)
                self.spans.append((key, t0, time.perf_counter()))
                self.done.put((key, g, ""))
            except Exception as e:  # reported with the requests that wait for it
                self.done.put((key, None, getattr(e, "status", None) and tc.lib().tc_status_str(e.status).decode()
                               or "TC_E_DEVICE"))

    def close(self):
        for _ in self.threads:
            self.todo.put(None)
        for t in self.threads:
            t.join()


class Server:
    """Continuous batching over per-graph queues.

    Requests wait in one queue per registry key (a graph, or a graph's sample),
    the queues ordered by their oldest request. Each turn of the loop

    * takes arrivals into their queues, installs what the builders finished and
      retires the batches whose event has fired;
    * when a stream is free, launches one batch holding the queued requests on
      resident keys, oldest queue first, up to max_batch requests;
    * starts builds for the oldest queues whose key is not resident, at most
      two per builder thread at a time (a sample's graph is built first, then
      the sample is drawn from it). Room for a build is made by evicting, least
      recently used first, graphs that no queued request needs; only the oldest
      queue may also evict what younger queues need, and when even that finds
      no room nothing younger starts a build, so no two queues can keep
      evicting each other's graphs. When nothing is in flight, building or
      launchable and the oldest queue's key still does not fit, its requests
      are answered TC_E_NOMEM.
    """

    def __init__(self, registry: Registry, max_batch: int = 64, streams: int = 3, builders: int = 4):
        import torch

        self.torch = torch
        self.reg = registry
        self.max_batch = max_batch
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.inflight: List[_Batch] = []
        self.answers: Dict[int, Answer] = {}
        self.batches = 0
        self.batch_sizes: List[int] = []
        self.queued: "collections.OrderedDict[object, List[Request]]" = collections.OrderedDict()
        self.ready: "collections.OrderedDict[object, None]" = collections.OrderedDict()  # queued keys seen resident
        self.building: Dict[object, object] = {}  # key being built -> graph pinned as its base (or None)
        self.nbuilders = builders
        self.max_building = 2 * builders
        self.builder: Optional[_Builder] = None
        self.timeline: List[tuple] = []  # sampled state, one row per 50 ms of the run
        self.build_spans: List[tuple] = []  # (key, start s, end s) of every build of the last run
        self.started = 0                 # builds started
        self.blocked = 0                 # build starts refused for lack of room

    # ------------------------------------------------------------ building
    @staticmethod
    def _key(r: Request):
        return r.graph if r.kind != SPARSE else (r.graph, r.q, r.seed)

    def _need(self, key):
        """What must be built next for key (None if key is resident): the key, or
        the graph a sample is drawn from while that graph is not resident."""
        if self.reg.peek(key) is not None:
            return None
        if isinstance(key, tuple) and self.reg.peek(key[0]) is None:
            return key[0]
        return key

    def _uses(self, key):
        """The resident graphs a queue needs kept: its key, or the graph its sample is drawn from."""
        if self.reg.peek(key) is not None:
            return (key,)
        if isinstance(key, tuple) and self.reg.peek(key[0]) is not None:
            return (key[0],)
        return ()

    def _start_builds(self, clock) -> bool:
        """Start builds for the oldest queues; True if the oldest queue's key can never fit.
        Only the queues before the last one started are visited (those resident or building,
        then the ones whose build starts), and the graphs every queue needs are listed only
        when a reservation has to evict."""
        if len(self.building) >= self.max_building:
            return False
        uses_all = lambda: [k for key in self.queued for k in self._uses(key)]  # noqa: E731
        older: List[object] = []
        head = True  # still at the oldest queue that needs a build
        for key in self.queued:
            need = self._need(key)
            if need is None or need in self.building:
                older.extend(self._uses(key))
                continue
            base = need[0] if isinstance(need, tuple) else None
            if base is not None:
                self.reg.pinned[base] += 1  # the sample is drawn from it
            ok = self.reg.reserve(need, uses_all) or (head and self.reg.reserve(need, lambda: older))
            if not ok:
                self.blocked += 1
                if base is not None:
                    self.reg.pinned[base] -= 1
                return head and not self.inflight and not self.building and \
                    not any(self.reg.peek(k) is not None for k in self.queued)
            self.building[need] = base
            self.started += 1
            self.builder.todo.put((need, self.reg.peek(base) if base is not None else None))
            head = False
            older.extend(self._uses(key))
            if len(self.building) >= self.max_building:
                break
        return False

    def _collect_builds(self, clock) -> bool:
        import queue

        got = False
        while True:
            try:
                key, g, err = self.builder.done.get_nowait()
            except queue.Empty:
                return got
            got = True
            base = self.building.pop(key)
            if base is not None:
                self.reg.pinned[base] -= 1
            if g is not None:
                self.reg.install(key, g)
                if key in self.queued:
                    self.ready[key] = None
                continue
            self.reg.cancel(key)
            # the requests on key fail, and so do those on samples drawn from it
            for k in [k for k in self.queued if k == key or (isinstance(k, tuple) and k[0] == key)]:
                for r in self.queued.pop(k):
                    self.answers[r.rid] = Answer(r.rid, r.kind, None, clock(), err)

    def _take(self) -> List[Request]:
        """Queued requests on resident keys, at most max_batch, the keys in the order they
        became resident (only keys seen resident are visited)."""
        take: List[Request] = []
        for key in list(self.ready):
            reqs = self.queued.get(key)
            if reqs is None or self.reg.peek(key) is None:  # launched already, or evicted since
                del self.ready[key]
                continue
            room = self.max_batch - len(take)
            take.extend(reqs[:room])
            if room >= len(reqs):
                del self.queued[key]
                del self.ready[key]
            else:
                del reqs[:room]
            if len(take) >= self.max_batch:
                break
        return take

    # ------------------------------------------------------------ batching
    def _launch(self, reqs: List[Request], stream) -> Optional[_Batch]:
        torch = self.torch
        keys_tot: List[object] = []     # distinct graphs/samples needing totals
        idx_tot: Dict[object, int] = {}
        cc_keys: List[int] = []         # distinct graphs needing per-node counts
        idx_cc: Dict[int, int] = {}
        graphs_tot, graphs_cc = [], []
        pins: List[object] = []  # graphs are pinned as they are fetched so later fetches cannot evict them
        batch: List[Request] = []
        for r in reqs:
            key = self._key(r)
            g = self.reg.resident(key)
            if g is None:
                raise RuntimeError("a batch request whose graph is not resident")
            if key not in pins:
                self.reg.pin([key])
                pins.append(key)
            batch.append(r)
            if r.kind == CLUSTER:
                if r.graph not in idx_cc:
                    idx_cc[r.graph] = len(cc_keys)
                    cc_keys.append(r.graph)
                    graphs_cc.append(g)
            elif key not in idx_tot:
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
        b = _Batch(batch, stream, ev, pins, T_host, cc_host, idx_tot, idx_cc, None)
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
        pending = collections.deque(sorted(trace, key=lambda r: (r.arrival, r.rid)))
        free_streams = list(self.streams)
        self.builder = _Builder(self.reg, self.nbuilders)
        changed = True
        next_sample = 0.0
        try:
            while pending or self.queued or self.inflight or self.building:
                now = clock()
                if now >= next_sample:
                    next_sample = now + 0.05
                    self.timeline.append((round(now, 3), self.started, self.reg.builds, len(self.queued),
                                          sum(len(v) for v in self.queued.values()), len(self.building),
                                          len(self.inflight), self.reg.used, sum(self.reg.reserved.values()),
                                          self.reg.evictions, self.blocked))
                while pending and pending[0].arrival <= now:
                    r = pending.popleft()
                    key = self._key(r)
                    q = self.queued.get(key)
                    if q is None:
                        self.queued[key] = [r]
                        if self.reg.peek(key) is not None:
                            self.ready[key] = None
                    else:
                        q.append(r)
                    changed = True
                if self._collect_builds(clock):
                    changed = True
                if self._poll(clock):
                    changed = True
                    free_streams = [s for s in self.streams if all(b.stream is not s for b in self.inflight)]
                more = False
                if changed and free_streams:
                    take = self._take()
                    if take:
                        self.inflight.append(self._launch(take, free_streams[0]))
                        self.batches += 1
                        free_streams = free_streams[1:]
                        more = len(take) == self.max_batch  # launchable requests may remain
                if changed:
                    changed = False
                    if self._start_builds(clock):
                        key = next(iter(self.queued))
                        for r in self.queued.pop(key):
                            self.answers[r.rid] = Answer(r.rid, r.kind, None, clock(), "TC_E_NOMEM")
                        changed = True
                        continue
                if more:
                    changed = True
                    continue
                if self.inflight or self.building:
                    time.sleep(0.0001)
                elif pending:
                    wait = pending[0].arrival - clock()
                    if wait > 0:
                        time.sleep(min(wait, 0.002))
        finally:
            self.builder.close()
            self.build_spans = [(k, a - start, b - start) for k, a, b in self.builder.spans]
            self.builder = None
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


def tail_breakdown(trace: List[Request], answers: Dict[int, Answer], sizes=None, worst: int = 8):
    """Where the latency tail sits: p99 per request kind, p99 over arrivals after the
    first second and the slowest requests (kind, graph, its n, arrival s, latency ms)."""
    lat = np.array([answers[r.rid].done - r.arrival for r in trace])
    arr = np.array([r.arrival for r in trace])
    out = {}
    for kind in (COUNT, CLUSTER, SPARSE):
        sel = np.array([r.kind == kind for r in trace])
        if sel.any():
            out[f"p99_ms_{kind}"] = float(np.percentile(lat[sel], 99) * 1e3)
    late = arr >= 1.0
    if late.any():
        out["p99_ms_after_first_s"] = float(np.percentile(lat[late], 99) * 1e3)
    slow = np.argsort(-lat)[:worst]
    out["slowest"] = [[trace[i].kind, trace[i].graph, int(sizes[trace[i].graph]) if sizes is not None else None,
                       round(float(arr[i]), 3), round(float(lat[i] * 1e3), 1)] for i in slow]
    return out


def same_answer(a: Answer, b: Answer) -> bool:
    """Exact equality: counts, estimate doubles and clustering digests."""
    return a.kind == b.kind and a.value == b.value and not a.error and not b.error
