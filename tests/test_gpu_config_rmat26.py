"""Parity at the full R-MAT scale-26 size (edge factor 16, seed 3), in the
launch configuration bench.py times: totals, work, degrees and the sparsified
counts against the oracle's stored results (tests/golden/rmat26.json, written
by tests/golden/make_rmat26.py), per-node counts at 64 sampled vertices
computed by the oracle from the definition, and sum_v t_v = 3T; the 8 core-node
shards (boundaries from tests/golden/rmat26_shards.json, written by
tests/golden/make_rmat26_shards.py) adding up to T, the per-shard sampled
counts of the overlapping-partition sparsification, and the streamed count of
the CSR held in host memory."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rmat26.json")
SHARDS = os.path.join(os.path.dirname(__file__), "golden", "rmat26_shards.json")
GOLDEN20 = os.path.join(os.path.dirname(__file__), "golden", "rmat20.json")


def test_rmat20_stored_golden():
    """The same checks at scale 20 against tests/golden/rmat20.json (written by
    tests/golden/make_rmat26.py 20 with the oracle)."""
    import torch

    from paper_1706_05151_amd import tc

    with open(GOLDEN20) as f:
        gold = json.load(f)
    el = synth.rmat(20, 16, 3)
    with tc.Graph.build(torch.from_numpy(el.src).cuda(), torch.from_numpy(el.dst).cuda(), el.n) as g:
        assert (g.n, g.m, g.d_max, g.dhat_max) == (gold["n"], gold["m"], gold["d_max"], gold["dhat_max"])
        assert g.count() == gold["T"] and g.work()[0] == gold["W"]
        T, t = g.count_per_node()
        ids = np.array(gold["sample_ids"], dtype=np.int64)
        np.testing.assert_array_equal(t.cpu().numpy().astype(np.uint64)[ids],
                                      np.array(gold["sample_t"], dtype=np.uint64))
        deg, _ = g.degrees()
        np.testing.assert_array_equal(deg.cpu().numpy()[ids], np.array(gold["sample_deg"], dtype=np.int32))
        for q, ref in gold["sparsified"].items():
            Ts, mk, _ = g.sparsify_count(float(q), ref["seed"])
            assert (Ts, mk) == (ref["T_s"], ref["m_kept"])


@pytest.fixture(scope="module")
def rmat26():
    import torch

    from paper_1706_05151_amd import tc

    with open(GOLDEN) as f:
        gold = json.load(f)
    el = synth.config_rmat(26)
    print(f"[rmat26] generated E={el.num_edges}", flush=True)
    src = torch.from_numpy(el.src).cuda()
    dst = torch.from_numpy(el.dst).cuda()
    n = el.n
    del el
    g = tc.Graph.build(src, dst, n)
    del src, dst
    torch.cuda.empty_cache()
    print(f"[rmat26] built m={g.m}", flush=True)
    yield g, gold
    g.close()


def test_totals(rmat26):
    g, gold = rmat26
    assert g.n == gold["n"] and g.m == gold["m"]
    assert g.d_max == gold["d_max"] and g.dhat_max == gold["dhat_max"]
    assert g.count() == gold["T"]
    W, P = g.work()
    assert W == gold["W"]


def test_per_node_samples(rmat26):
    g, gold = rmat26
    T, t = g.count_per_node()
    assert T == gold["T"]
    assert int(t.sum().item()) == 3 * gold["T"]
    ids = np.array(gold["sample_ids"], dtype=np.int64)
    tt = t.cpu().numpy().astype(np.uint64)
    np.testing.assert_array_equal(tt[ids], np.array(gold["sample_t"], dtype=np.uint64))
    deg, dhat = g.degrees()
    np.testing.assert_array_equal(deg.cpu().numpy()[ids], np.array(gold["sample_deg"], dtype=np.int32))
    assert int(dhat.sum().item()) == gold["m"]


def test_clustering_samples(rmat26):
    """C_v at the 64 sampled vertices: the exact rational T_v / C(d_v, 2) from the stored
    definition-based counts, and its double bit for bit."""
    g, gold = rmat26
    num, den, c = g.clustering()
    ids = np.array(gold["sample_ids"], dtype=np.int64)
    t = np.array(gold["sample_t"], dtype=np.uint64)
    d = np.array(gold["sample_deg"], dtype=np.uint64)
    want_den = np.where(d >= 2, d * (d - np.uint64(1)) // np.uint64(2), np.uint64(0))
    np.testing.assert_array_equal(num.cpu().numpy().astype(np.uint64)[ids], t)
    np.testing.assert_array_equal(den.cpu().numpy().astype(np.uint64)[ids], want_den)
    want_c = np.array([float(a) / float(b) if b else 0.0 for a, b in zip(t, want_den)], dtype=np.float64)
    np.testing.assert_array_equal(c.cpu().numpy()[ids].view(np.uint64), want_c.view(np.uint64))


@pytest.mark.parametrize("q", ["0.1", "0.5"])
def test_sparsified(rmat26, q):
    g, gold = rmat26
    ref = gold["sparsified"][q]
    Ts, mk, est = g.sparsify_count(float(q), ref["seed"])
    assert (Ts, mk) == (ref["T_s"], ref["m_kept"])
    assert est == oracle.estimate(Ts, float(q))


def test_shards_add_up(rmat26):
    g, gold = rmat26
    with open(SHARDS) as f:
        sh = json.load(f)
    b = g.shard_bounds(sh["shards"])
    assert b == sh["bounds"]
    assert sum(g.count_shard(b[j], b[j + 1]) for j in range(sh["shards"])) == gold["T"]


def test_partitioned_sample(rmat26):
    g, _ = rmat26
    with open(SHARDS) as f:
        sh = json.load(f)
    ps = sh["partitioned_sample"]
    T_parts, b, Ts, est = g.sparsify_count_partitioned(ps["q"], ps["seed"], sh["shards"])
    assert b == sh["bounds"]
    assert T_parts == ps["T_parts"] and Ts == ps["T_s"]
    assert est == oracle.estimate(Ts, ps["q"])


def test_streamed_from_host(rmat26):
    """The rank-space CSR in pinned host memory, counted under a 16 GiB device budget (several
    pivot partitions and chunks), gives T."""
    g, gold = rmat26
    from paper_1706_05151_amd import tc

    off, adj = g.export_csr()
    assert int(off[-1]) == gold["m"]
    T, info = tc.count_streamed(off, adj, g.n, 16 << 30)
    print(f"[rmat26] streamed {info}", flush=True)
    assert info["partitions"] > 1 and info["chunks"] > 1
    assert T == gold["T"]
