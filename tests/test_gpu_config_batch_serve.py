"""Oracle parity of the batched and served configurations at their stated size.

* Batch: the 4096-graph mixed batch of seed 4 (n ~ U[64,8192]; ER, PA and
  R-MAT; 1.44e8 edge records), built as one device graph and counted in one
  persistent launch, eagerly and replayed from a HIP graph: every graph's T and
  every t_v against the oracle.
* Serve: the 1024-graph pool of seed 5 (n log-uniform in [1e3, 1e6]) and the
  benchmark's own request trace (Poisson 2000/s for 60 s, 60% counts, 25%
  clustering, 15% estimates at q = 0.2). A seeded subset of 240 requests plus
  every kind of request on the largest pool graph (n close to 1e6) is served
  by the continuous-batching server under a device budget that forces
  evictions; each answer is checked against the oracle (exact T, clustering
  rationals and doubles by digest, the estimate of the oracle's own sample).
"""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pool_threads():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def tcm():
    import torch

    assert torch.cuda.is_available()
    from paper_1706_05151_amd import tc

    return tc


def test_batch4096_seed4_every_graph_against_oracle(tcm):
    import torch

    from paper_1706_05151_amd import batch

    specs = synth.batch_specs(4096, 4)
    els = [s.make() for s in specs]
    packed = batch.pack(els)
    say(f"[batch4096] {len(els)} graphs, {packed['src'].shape[0]} edge records")
    bc = batch.BatchCounter(packed, per_node=True)
    try:
        bc.build()
        bc.count()
        torch.cuda.synchronize()
        T = bc.T.cpu().numpy().astype(np.uint64)
        t = bc.per_graph_t()
        bc.capture()
        bc.T.fill_(-1)
        bc.t.fill_(-1)
        bc.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(bc.T.cpu().numpy().astype(np.uint64), T)
        for a, b in zip(bc.per_graph_t(), t):
            np.testing.assert_array_equal(a, b)
    finally:
        bc.close()
    say(f"[batch4096] counted on the GPU (sum T = {int(T.sum())}); oracle on {_pool_threads()} threads")

    def ref(i):
        e = els[i]
        r = oracle.solve(e.src, e.dst, e.n, per_node=True)
        return i, r.T, r.t

    bad = []
    with ThreadPoolExecutor(_pool_threads()) as ex:
        for i, rT, rt in ex.map(ref, range(len(els))):
            if T[i] != rT or not np.array_equal(t[i], rt):
                bad.append(i)
    assert not bad, f"graphs differing from the oracle: {bad[:10]}"
    say(f"[batch4096] all {len(els)} graphs equal the oracle")


class _LazyPool:
    """Pool graphs made on first use (the registry indexes the pool by graph id)."""

    def __init__(self, specs):
        self.specs = specs
        self.made = {}

    def __len__(self):
        return len(self.specs)

    def __getitem__(self, i):
        if i not in self.made:
            self.made[i] = self.specs[i].make()
        return self.made[i]


def test_serve_pool1024_seed5_subset_against_oracle(tcm):
    from paper_1706_05151_amd import serve

    specs = synth.pool_specs(1024, 5)
    trace = serve.make_trace(len(specs), rate=2000.0, duration=60.0, seed=5)
    big = int(np.argmax([s.n for s in specs]))
    assert specs[big].n > 9e5
    rng = np.random.default_rng(5)
    pick = set(int(i) for i in rng.choice(len(trace), size=240, replace=False))
    for kind in (serve.COUNT, serve.CLUSTER, serve.SPARSE):  # the largest graph, every kind
        pick.add(next(r.rid for r in trace if r.graph == big and r.kind == kind))
    sub = [trace[i] for i in sorted(pick)]
    # the subset keeps the trace's order, arriving at 2000 requests/s
    sub = [serve.Request(r.rid, r.kind, r.graph, 0.0005 * j, r.q, r.seed) for j, r in enumerate(sub)]
    kinds = {r.kind for r in sub}
    assert kinds == {serve.COUNT, serve.CLUSTER, serve.SPARSE}
    pool = _LazyPool(specs)
    gids = sorted({r.graph for r in sub})
    say(f"[serve1024] {len(sub)} requests on {len(gids)} pool graphs (largest n = {specs[big].n})")
    budget = 2 << 30  # below the footprint of the graphs the subset touches: evictions and rebuilds
    reg = serve.Registry(pool, budget_bytes=budget)
    try:
        srv = serve.Server(reg, max_batch=32, streams=3)
        ans = srv.run(sub)
        assert all(not ans[r.rid].error for r in sub), [ans[r.rid].error for r in sub if ans[r.rid].error][:3]
        say(f"[serve1024] served: {reg.builds} builds, {reg.evictions} evictions, {srv.batches} batches")
        assert reg.evictions > 0
    finally:
        reg.close()

    need = {}
    for r in sub:
        need.setdefault(r.graph, set()).add((r.kind, r.q, r.seed) if r.kind == serve.SPARSE else (r.kind,))

    def ref(gid):
        e = pool[gid]
        res = oracle.solve(e.src, e.dst, e.n, per_node=True)
        out = {serve.COUNT: res.T, serve.CLUSTER: serve.cc_digest(res.num, res.den, res.cc)}
        for k in need[gid]:
            if k[0] == serve.SPARSE:
                out[k] = oracle.sparsified_count(res.extra["lo"], res.extra["hi"], res.deg, e.n, k[1], k[2])[2]
        return gid, out

    refs = {}
    with ThreadPoolExecutor(_pool_threads()) as ex:
        for gid, out in ex.map(ref, gids):
            refs[gid] = out
    for r in sub:
        want = refs[r.graph][(r.kind, r.q, r.seed) if r.kind == serve.SPARSE else r.kind]
        assert ans[r.rid].value == want, (r, ans[r.rid].value, want)
    say(f"[serve1024] all {len(sub)} answers equal the oracle")
