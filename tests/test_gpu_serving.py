"""GPU tests of the batched and served paths: every result equals the
single-graph result (exact counts, bit-identical clustering doubles and estimates)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def tcm():
    import torch

    assert torch.cuda.is_available()
    from paper_1706_05151_amd import tc

    keys = (tc.OPT_KERNEL, tc.OPT_HUB_DHAT, tc.OPT_ITEM_WORK, tc.OPT_BLOCKS_PER_CU, tc.OPT_HUB_BUCKET_LOAD)
    saved = {k: tc.get_option(k) for k in keys}
    yield tc
    for k, v in saved.items():
        tc.set_option(k, v)


def _graphs(count, seed):
    return [s.make() for s in synth.batch_specs(count, seed)]


def test_multi_count_matches_single(tcm):
    import torch

    els = _graphs(24, 31) + [synth.complete(10), synth.empty(3), synth.rmat(13, 16, 2)]
    gs = [tcm.Graph.build(torch.from_numpy(e.src).cuda(), torch.from_numpy(e.dst).cuda(), e.n) for e in els]
    say(f"[serving] multi count over {len(gs)} graphs")
    T = torch.zeros(len(gs), dtype=torch.int64, device="cuda")
    ts = [torch.zeros(max(g.n, 1), dtype=torch.int64, device="cuda") for g in gs]
    tcm.multi_count(gs, T, None)
    torch.cuda.synchronize()
    T1 = T.cpu().numpy().copy()
    tcm.multi_count(gs, T, ts)
    torch.cuda.synchronize()
    for i, (e, g) in enumerate(zip(els, gs)):
        ref = oracle.solve(e.src, e.dst, e.n)
        assert T1[i] == ref.T and T[i].item() == ref.T
        np.testing.assert_array_equal(ts[i][: e.n].cpu().numpy().astype(np.uint64), ref.t)
        num = torch.empty(max(e.n, 1), dtype=torch.int64, device="cuda")
        den = torch.empty_like(num)
        c = torch.empty(max(e.n, 1), dtype=torch.float64, device="cuda")
        g.clustering_from_counts(ts[i], num, den, c)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(c[: e.n].cpu().numpy().view(np.uint64), ref.cc.view(np.uint64))
    for g in gs:
        g.close()


def test_concurrent_streams_share_the_block_cache(tcm):
    """Builds, samples and per-node counts on four threads with streams of their own,
    the graphs freed as soon as they are counted: blocks freed on one stream and taken
    on another are reused only once their work is done. Every result equals the one
    computed alone on one stream."""
    import threading

    import torch

    els = [s.make() for s in synth.pool_specs(48, 11, n_lo=1e3, n_hi=2e5)]
    ref = []
    for e in els:
        with tcm.Graph.build(torch.from_numpy(e.src).cuda(), torch.from_numpy(e.dst).cuda(), e.n) as g:
            T, t = g.count_per_node()
            with g.sparsify_build(0.3, 7) as h:
                ref.append((T, t.cpu().numpy(), h.count()))
    say(f"[streams] reference of {len(els)} graphs done")
    host = [(torch.from_numpy(e.src).pin_memory(), torch.from_numpy(e.dst).pin_memory()) for e in els]
    got = [None] * len(els)
    errors = []

    def work(k):
        try:
            torch.cuda.set_device(0)
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for rep in range(3):
                    for i in range(k, len(els), 4):
                        src = host[i][0].to("cuda", non_blocking=True)
                        dst = host[i][1].to("cuda", non_blocking=True)
                        g = tcm.Graph.build(src, dst, els[i].n, st)
                        T, t = g.count_per_node(stream=st)
                        h = g.sparsify_build(0.3, 7, st)
                        Ts = h.count(st)
                        h.close()
                        g.close()  # freed at once: another stream may take these blocks next
                        st.synchronize()
                        got[i] = (T, t.cpu().numpy(), Ts)
        except Exception as ex:  # reported below
            errors.append(ex)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for i, (r, x) in enumerate(zip(ref, got)):
        assert x is not None and x[0] == r[0] and x[2] == r[2], i
        np.testing.assert_array_equal(x[1], r[1])
    # the totals against the oracle for a few of them
    for i in (0, 17, 47):
        e = els[i]
        assert ref[i][0] == oracle.solve(e.src, e.dst, e.n, per_node=False).T


def test_sparsify_build_matches_sparsify_count(tcm):
    import torch

    el = synth.rmat(14, 16, 7)
    with tcm.Graph.build(torch.from_numpy(el.src).cuda(), torch.from_numpy(el.dst).cuda(), el.n) as g:
        Ts, mk, est = g.sparsify_count(0.2, 5)
        with g.sparsify_build(0.2, 5) as h:
            assert h.m == mk and h.count() == Ts
            assert tcm.sparsify_estimate(Ts, 0.2) == est
            with pytest.raises(tcm.TCError):
                h.count_per_node()
    lo, hi = oracle.simple(el.src, el.dst, el.n)
    rTs, rmk, rest = oracle.sparsified_count(lo, hi, oracle.degrees(lo, hi, el.n), el.n, 0.2, 5)
    assert (Ts, mk, est) == (rTs, rmk, rest)


def test_batch_hipgraph_replays(tcm):
    """The captured batched count equals the eager one on every replay, with
    eager work and synchronisations between the replays."""
    import torch

    from paper_1706_05151_amd import batch

    els = _graphs(200, 44)
    packed = batch.pack(els)
    bc = batch.BatchCounter(packed, per_node=True)
    bc.build()
    say(f"[serving] batch of {len(els)} graphs, capture and replay")
    bc.count()
    torch.cuda.synchronize()
    T_ref = bc.T.cpu().numpy().copy()
    t_ref = [x.copy() for x in bc.per_graph_t()]
    for i in (0, 7, 199):
        ref = oracle.solve(els[i].src, els[i].dst, els[i].n)
        assert T_ref[i] == ref.T
        np.testing.assert_array_equal(t_ref[i], ref.t)
    bc.capture()
    # the capture holds the plan's addresses: the plan is frozen, an explicit
    # rebuild is refused, and counting under other options keeps using it
    info = bc.graph.plan_info()
    assert info["frozen"]
    old = batch.current_options()
    try:
        with pytest.raises(tcm.TCError) as e:
            bc.graph.replan()
        assert e.value.status == tcm.TC_E_INVAL
        batch.apply_options((32, 4096, old[2], old[3]))
        assert bc.graph.count() == int(T_ref.sum())
        assert bc.graph.plan_info() == info
    finally:
        batch.apply_options(old)
    for rep in range(4):
        bc.T.fill_(-1)
        bc.t.fill_(-1)
        bc.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(bc.T.cpu().numpy(), T_ref)
        for a, b in zip(bc.per_graph_t(), t_ref):
            np.testing.assert_array_equal(a, b)
        bc.count()  # eager work between replays
        torch.cuda.synchronize()
        np.testing.assert_array_equal(bc.T.cpu().numpy(), T_ref)
    bc.close()


@pytest.mark.parametrize("per_node", [False, True])
def test_autotune_keeps_results(tcm, per_node):
    """The autotuner rebuilds the plan per candidate and leaves the chosen
    candidate's plan on the graph; results never change."""
    import torch

    from paper_1706_05151_amd import batch

    els = _graphs(64, 45)
    bc = batch.BatchCounter(batch.pack(els), per_node=per_node)
    bc.build()
    bc.count()
    torch.cuda.synchronize()
    T0 = bc.T.cpu().numpy().copy()
    t0 = [x.copy() for x in bc.per_graph_t()] if per_node else None
    old = batch.current_options()
    try:
        # the pivot kernel under three partitioner settings and one thread per edge (kernel 1)
        cands = [(128, 16384, 4, 2, 2), (16, 256, 2, 1, 2), (0, 100000, 3, 2, 2), (256, 0, 4, 2, 1)]
        best, table = batch.autotune(bc, candidates=cands, reps=1, persist=False)
        assert len(table) == 4
        info = bc.graph.plan_info()
        assert (info["hub_dhat"], info["item_work"]) == tuple(best["options"][:2])
        assert tcm.get_option(tcm.OPT_KERNEL) == best["options"][4]
        assert not info["frozen"]
        bc.count()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(bc.T.cpu().numpy(), T0)
        if per_node:
            for a, b in zip(bc.per_graph_t(), t0):
                np.testing.assert_array_equal(a, b)
        for i in (0, 31, 63):
            assert T0[i] == oracle.solve(els[i].src, els[i].dst, els[i].n, per_node=False).T
    finally:
        batch.apply_options(old)
        bc.close()


def test_served_results_equal_standalone(tcm):
    """Each request's answer in the continuous-batching server equals its
    one-at-a-time answer, under a budget that forces evictions."""
    from paper_1706_05151_amd import serve

    els = [s.make() for s in synth.pool_specs(24, 9, n_lo=1e3, n_hi=3e4)]
    trace = serve.make_trace(len(els), rate=3000.0, duration=0.4, seed=9)
    say(f"[serving] trace of {len(trace)} requests on {len(els)} graphs")
    # a few graphs at a time, built from pinned host copies (the one-at-a-time run below copies
    # from pageable memory)
    reg = serve.Registry(els, budget_bytes=12 << 20, host_edges=serve.pin_edge_lists(els))
    srv = serve.Server(reg, max_batch=16, streams=3)
    ans = srv.run(trace)
    reg2 = serve.Registry(els, budget_bytes=1 << 34)
    fifo = serve.serve_fifo(reg2, trace)
    assert all(not ans[r.rid].error for r in trace)
    for r in trace:
        assert serve.same_answer(ans[r.rid], fifo[r.rid]), r
    assert reg.evictions > 0
    # every answer against the oracle: counts, clustering (exact rationals and
    # doubles, by digest) and the sparsified estimates of the q = 0.2 samples
    assert {r.kind for r in trace} == {serve.COUNT, serve.CLUSTER, serve.SPARSE}
    refs = {}
    for r in trace:
        if r.graph not in refs:
            e = els[r.graph]
            ref = oracle.solve(e.src, e.dst, e.n)
            lo, hi = ref.extra["lo"], ref.extra["hi"]
            refs[r.graph] = (ref, lo, hi, {})
        ref, lo, hi, sp = refs[r.graph]
        if r.kind == serve.COUNT:
            assert ans[r.rid].value == ref.T, r
        elif r.kind == serve.CLUSTER:
            assert ans[r.rid].value == serve.cc_digest(ref.num, ref.den, ref.cc), r
        else:
            if (r.q, r.seed) not in sp:
                sp[(r.q, r.seed)] = oracle.sparsified_count(lo, hi, ref.deg, els[r.graph].n, r.q, r.seed)[2]
            assert ans[r.rid].value == sp[(r.q, r.seed)], r
    # the plain per-graph launch (build, answer, free per request) gives the same answers
    import torch

    edges = [(torch.from_numpy(e.src).cuda(), torch.from_numpy(e.dst).cuda(), e.n) for e in els]
    plain, _ = serve.serve_plain(edges, trace)
    for r in trace:
        assert serve.same_answer(plain[r.rid], fifo[r.rid]), r
    reg.close()
    reg2.close()


def test_served_oversized_graph_is_refused(tcm):
    from paper_1706_05151_amd import serve

    els = [synth.rmat(12, 16, 1)]
    reg = serve.Registry(els, budget_bytes=1 << 10)
    srv = serve.Server(reg, max_batch=4, streams=2)
    ans = srv.run([serve.Request(0, serve.COUNT, 0, 0.0)])
    assert ans[0].error == "TC_E_NOMEM"
