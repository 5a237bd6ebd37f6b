"""Seeded fuzz parity: many small random graphs of mixed shapes (random, power-law,
dense unions, raw edge lists with loops and repeats) under random partitioner
settings, every output of the library against the CPU oracle."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CASES = 48


def _union(parts, seed):
    """Disjoint union of edge lists, vertex ids shuffled by a seeded permutation."""
    n = sum(p.n for p in parts)
    perm = np.random.default_rng(seed).permutation(max(n, 1)).astype(np.int32)
    src, dst, base = [], [], 0
    for p in parts:
        src.append(p.src.astype(np.int64) + base)
        dst.append(p.dst.astype(np.int64) + base)
        base += p.n
    s = np.concatenate(src) if src else np.zeros(0, np.int64)
    d = np.concatenate(dst) if dst else np.zeros(0, np.int64)
    return synth.EdgeList(n, perm[s].astype(np.int32), perm[d].astype(np.int32), f"union{seed}")


def _random_graph(rng, seed):
    kind = int(rng.integers(0, 6))
    if kind == 0:
        n = int(rng.integers(2, 3000))
        return synth.er(n, float(rng.uniform(0.0005, 0.05)), seed)
    if kind == 1:
        n = int(rng.integers(10, 4000))
        return synth.ba(n, int(rng.integers(1, 12)), seed)
    if kind == 2:
        return synth.rmat(int(rng.integers(4, 12)), int(rng.integers(2, 24)), seed)
    if kind == 3:
        parts = [synth.complete(int(rng.integers(3, 40))) for _ in range(int(rng.integers(1, 4)))]
        parts += [synth.star(int(rng.integers(1, 300))), synth.wheel(int(rng.integers(3, 200)))]
        return _union(parts, seed)
    if kind == 4:
        n = int(rng.integers(5, 2000))
        m = int(rng.integers(0, 20 * n))
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        k = m // 3
        src = np.concatenate([src, dst[:k], np.arange(5, dtype=np.int32)])
        dst = np.concatenate([dst, src[:k], np.arange(5, dtype=np.int32)])
        return synth.EdgeList(n, src, dst, f"raw{seed}")
    hub = int(rng.integers(50, 600))  # one dense hub-heavy core on a sparse rim
    return _union([synth.complete(hub // 8), synth.rmat(10, 8, seed), synth.friendship(hub)], seed)


@pytest.mark.parametrize("case", range(CASES))
def test_fuzz(case):
    import torch

    from paper_1706_05151_amd import tc

    rng = np.random.default_rng(9000 + case)
    el = _random_graph(rng, 9000 + case)
    opts = {tc.OPT_HUB_DHAT: int(rng.choice([0, 16, 64, 256])),
            tc.OPT_ITEM_WORK: int(rng.choice([0, 64, 1024, 65536])),
            tc.OPT_HUB_BUCKET_LOAD: int(rng.choice([1, 2])),
            tc.OPT_KERNEL: int(rng.choice([0, 1, 2]))}
    saved = {k: tc.get_option(k) for k in opts}
    for k, v in opts.items():
        tc.set_option(k, v)
    try:
        ref = oracle.solve(el.src, el.dst, el.n, per_node=True, listing=True)
        print(f"[fuzz] case {case}: {el.name} n={el.n} E={el.num_edges} m={ref.m} T={ref.T} opts={opts}",
              flush=True)
        s = torch.from_numpy(np.ascontiguousarray(el.src)).cuda()
        d = torch.from_numpy(np.ascontiguousarray(el.dst)).cuda()
        with tc.Graph.build(s, d, el.n) as g:
            assert g.m == ref.m
            assert g.count() == ref.T
            T, t = g.count_per_node()
            assert T == ref.T
            np.testing.assert_array_equal(t.cpu().numpy().astype(np.uint64), ref.t)
            num, den, c = g.clustering()
            np.testing.assert_array_equal(c.cpu().numpy().view(np.uint64), ref.cc.view(np.uint64))
            np.testing.assert_array_equal(g.list().cpu().numpy(), ref.tri)
            q = float(rng.choice([0.05, 0.3, 0.7, 1.0]))
            seed = int(rng.integers(0, 2 ** 62))
            Ts, mk, est = g.sparsify_count(q, seed)
            assert (Ts, mk, est) == oracle.sparsified_count(ref.extra["lo"], ref.extra["hi"], ref.deg, el.n, q, seed)
            k = int(rng.integers(1, 9))
            cost = int(rng.integers(0, 2))
            pos = oracle.order_positions(ref.deg, el.n)
            b = oracle.shard_bounds(ref.off, ref.adj, el.n, pos, k, cost)
            assert g.shard_bounds(k, cost) == b.tolist()
            assert [g.count_shard(int(b[j]), int(b[j + 1])) for j in range(k)] == \
                [oracle.count_nin_pos_range(ref.off, ref.adj, el.n, pos, int(b[j]), int(b[j + 1])) for j in range(k)]
            off, adj = g.export_csr()
            budget = int(rng.choice([8 << 10, 64 << 10, 1 << 20]))
            try:
                Tst, _ = tc.count_streamed(off, adj, el.n, budget)
                assert Tst == ref.T
            except tc.TCError as e:  # a row too long for the smallest budgets
                assert "budget" in str(e), e
    finally:
        for k, v in saved.items():
            tc.set_option(k, v)
