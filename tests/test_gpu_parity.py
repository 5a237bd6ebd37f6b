"""GPU parity: every output of the HIP library against the CPU oracle, element by element.

Integer results (T, t_v, m', T_s, lists, orientation) must be bit-exact; the
clustering doubles are compared bit for bit as well, beside the exact rationals.
"""
import ctypes
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1706_05151_amd.tc as tcm

    tcm.lib()
    keys = (tcm.OPT_KERNEL, tcm.OPT_HUB_DHAT, tcm.OPT_ITEM_WORK, tcm.OPT_BLOCKS_PER_CU, tcm.OPT_HUB_BUCKET_LOAD)
    saved = {k: tcm.get_option(k) for k in keys}
    yield tcm
    for k, v in saved.items():
        tcm.set_option(k, v)


def to_dev(el):
    import torch

    return (torch.from_numpy(np.ascontiguousarray(el.src)).cuda(), torch.from_numpy(np.ascontiguousarray(el.dst)).cuda())


def u64(t):
    return t.cpu().numpy().astype(np.uint64)


def check_all(tc, el, listing=True, label=""):
    """Build on the GPU and compare every output with the oracle."""
    say(f"[parity] {label or el.name}: n={el.n} E={el.num_edges}")
    ref = oracle.solve(el.src, el.dst, el.n, per_node=True, listing=listing)
    s, d = to_dev(el)
    with tc.Graph.build(s, d, el.n) as g:
        assert g.n == el.n and g.m == ref.m
        assert g.d_max == (int(ref.deg.max()) if el.n else 0)
        assert g.dhat_max == (int(np.diff(ref.off).max()) if el.n else 0)
        assert g.count() == ref.T
        assert g.count_plain() == ref.T
        T, t = g.count_per_node()
        assert T == ref.T
        np.testing.assert_array_equal(u64(t), ref.t)
        num, den, c = g.clustering()
        np.testing.assert_array_equal(u64(num), ref.num)
        np.testing.assert_array_equal(u64(den), ref.den)
        np.testing.assert_array_equal(c.cpu().numpy().view(np.uint64), ref.cc.view(np.uint64))
        if listing:
            tri = g.list()
            np.testing.assert_array_equal(tri.cpu().numpy(), ref.tri)
        deg, dhat = g.degrees()
        np.testing.assert_array_equal(deg.cpu().numpy(), ref.deg.astype(np.int32))
        np.testing.assert_array_equal(dhat.cpu().numpy(), np.diff(ref.off).astype(np.int32))
        off, adj = g.oriented()
        np.testing.assert_array_equal(off.cpu().numpy(), ref.off)
        np.testing.assert_array_equal(adj.cpu().numpy(), ref.adj)
        W, P = g.work()
        assert W == oracle.work(ref.off, ref.adj, el.n)
        dh = np.diff(ref.off).astype(np.int64)
        assert P == int((dh * (dh - 1) // 2).sum())
    return ref


CLOSED = [synth.complete(3), synth.complete(4), synth.complete(30), synth.wheel(4), synth.wheel(3), synth.wheel(200),
          synth.star(300), synth.path(50), synth.cycle(3), synth.cycle(64), synth.complete_bipartite(20, 30),
          synth.hypercube(8), synth.grid(20, 30), synth.random_tree(1000, 5), synth.complete_tripartite(10, 12, 14),
          synth.friendship(100), synth.empty(5), synth.empty(0), synth.complete(2)]


@pytest.mark.parametrize("el", CLOSED, ids=[g.name for g in CLOSED])
def test_closed_forms(tc, el):
    check_all(tc, el)


@pytest.mark.parametrize("seed", range(6))
def test_random_messy(tc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 3000))
    m = int(rng.integers(0, 20 * n))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    k = m // 3
    src = np.concatenate([src, dst[:k], np.arange(min(n, 7), dtype=np.int32)])
    dst = np.concatenate([dst, src[:k], np.arange(min(n, 7), dtype=np.int32)])
    check_all(tc, synth.EdgeList(n, src, dst, f"messy{seed}"))


@pytest.mark.parametrize("spec", ["er", "ba", "rmat13", "rmat15"])
def test_families(tc, spec):
    el = {"er": lambda: synth.er(20000, 0.002, 3), "ba": lambda: synth.ba(50000, 6, 4),
          "rmat13": lambda: synth.rmat(13, 16, 5), "rmat15": lambda: synth.rmat(15, 16, 6)}[spec]()
    ref = check_all(tc, el, listing=True)
    old = tc.get_option(tc.OPT_KERNEL)
    try:
        for k in (1, 2):  # forced plain merge / forced pivot kernel for the total
            tc.set_option(tc.OPT_KERNEL, k)
            with tc.Graph.build(*to_dev(el), el.n) as g:
                assert g.count() == ref.T
    finally:
        tc.set_option(tc.OPT_KERNEL, old)


TINY = [synth.complete(2), synth.path(3), synth.complete(3), synth.star(5), synth.wheel(4)]


@pytest.mark.parametrize("el", TINY, ids=[g.name for g in TINY])
def test_tiny_graphs_on_the_pivot_kernel(tc, el):
    """The pivot kernel forced on graphs of one to eight edges (a work plan of one record sorts
    nothing: the record is made from the key as read): total, per-node counts and the list."""
    ref = oracle.solve(el.src, el.dst, el.n, per_node=True, listing=True)
    old = tc.get_option(tc.OPT_KERNEL)
    try:
        tc.set_option(tc.OPT_KERNEL, 2)
        with tc.Graph.build(*to_dev(el), el.n) as g:
            assert g.count() == ref.T
            T, t = g.count_per_node()
            assert T == ref.T
            np.testing.assert_array_equal(u64(t), ref.t)
            np.testing.assert_array_equal(g.list().cpu().numpy(), ref.tri)
    finally:
        tc.set_option(tc.OPT_KERNEL, old)


@pytest.mark.parametrize("hub,iw,load", [(0, 64, 1), (0, 4096, 2), (16, 64, 2), (256, 100000, 1), (64, 512, 2),
                                         (128, 16384, 1)])
def test_partitioner_settings_identical(tc, hub, iw, load):
    """Every bucket threshold, work-item size and table load gives the same exact results."""
    el = synth.rmat(14, 16, 9)
    ref = oracle.solve(el.src, el.dst, el.n, per_node=True, listing=True)
    old = (tc.get_option(tc.OPT_HUB_DHAT), tc.get_option(tc.OPT_ITEM_WORK), tc.get_option(tc.OPT_HUB_BUCKET_LOAD))
    tc.set_option(tc.OPT_HUB_DHAT, hub)
    tc.set_option(tc.OPT_ITEM_WORK, iw)
    tc.set_option(tc.OPT_HUB_BUCKET_LOAD, load)
    try:
        s, d = to_dev(el)
        with tc.Graph.build(s, d, el.n) as g:
            say(f"[parity] partitioner hub={hub} iw={iw}")
            assert g.count() == ref.T
            T, t = g.count_per_node()
            np.testing.assert_array_equal(u64(t), ref.t)
            np.testing.assert_array_equal(g.list().cpu().numpy(), ref.tri)
    finally:
        tc.set_option(tc.OPT_HUB_DHAT, old[0])
        tc.set_option(tc.OPT_ITEM_WORK, old[1])
        tc.set_option(tc.OPT_HUB_BUCKET_LOAD, old[2])


def test_host_and_device_inputs_agree(tc):
    el = synth.ba(30000, 5, 7)
    s, d = to_dev(el)
    with tc.Graph.build(s, d, el.n) as g1, tc.Graph.build(el.src, el.dst, el.n) as g2:
        assert g1.count() == g2.count()
        np.testing.assert_array_equal(u64(g1.count_per_node()[1]), u64(g2.count_per_node()[1]))


def test_repeatable(tc):
    el = synth.rmat(15, 16, 11)
    s, d = to_dev(el)
    with tc.Graph.build(s, d, el.n) as g:
        T0, t0 = g.count_per_node()
        t0 = u64(t0)
        for _ in range(3):
            assert g.count() == T0
            T, t = g.count_per_node()
            np.testing.assert_array_equal(u64(t), t0)


# -------------------------------------------------------------- sparsify ---

@pytest.mark.parametrize("q,seed", [(0.1, 3), (0.5, 3), (0.2, 5), (1.0, 1), (0.37, 123456789)])
def test_sparsify_matches_oracle(tc, q, seed):
    el = synth.rmat(15, 16, 12)
    lo, hi = oracle.simple(el.src, el.dst, el.n)
    deg = oracle.degrees(lo, hi, el.n)
    Ts, mk, est = oracle.sparsified_count(lo, hi, deg, el.n, q, seed)
    s, d = to_dev(el)
    with tc.Graph.build(s, d, el.n) as g:
        say(f"[parity] sparsify q={q} seed={seed}")
        gTs, gmk, gest = g.sparsify_count(q, seed)
        assert (gTs, gmk) == (Ts, mk)
        assert gest == est


def test_sparsify_relabelled_ids_follow_caller_ids(tc):
    """The sample is a function of the caller's ids, not of the internal ranks."""
    el = synth.ba(20000, 6, 13)
    lo, hi = oracle.simple(el.src, el.dst, el.n)
    deg = oracle.degrees(lo, hi, el.n)
    klo, khi = oracle.sparsify(lo, hi, 0.3, 99)
    s, d = to_dev(el)
    with tc.Graph.build(s, d, el.n) as g:
        _, mk, _ = g.sparsify_count(0.3, 99)
        assert mk == klo.shape[0]
        Ts_ref, _, _ = oracle.count_nin(*oracle.orient(klo, khi, deg, el.n), el.n)
        assert g.sparsify_count(0.3, 99)[0] == Ts_ref


# ----------------------------------------------------------------- errors ---

def test_errors(tc):
    import torch

    s = torch.tensor([0, 1, 5], dtype=torch.int32, device="cuda")
    d = torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(tc.TCError) as e:
        tc.Graph.build(s, d, 5)
    assert e.value.status == tc.TC_E_RANGE
    s = torch.tensor([0, -1], dtype=torch.int32, device="cuda")
    d = torch.tensor([1, 2], dtype=torch.int32, device="cuda")
    with pytest.raises(tc.TCError) as e:
        tc.Graph.build(s, d, 5)
    assert e.value.status == tc.TC_E_RANGE
    el = synth.complete(6)
    with tc.Graph.build(*to_dev(el), el.n) as g:
        with pytest.raises(tc.TCError) as e:
            g.sparsify_count(0.0, 1)
        assert e.value.status == tc.TC_E_RANGE
        with pytest.raises(tc.TCError) as e:
            g.sparsify_count(1.5, 1)
        assert e.value.status == tc.TC_E_RANGE
        assert g.list_size() == 20
        with pytest.raises(tc.TCError) as e:
            g.list(cap=5)
        assert e.value.status == tc.TC_E_TRUNC
        assert g.list(cap=20).shape == (20, 3)
    with pytest.raises(tc.TCError):
        tc.set_option(tc.OPT_KERNEL, 7)
    # more vertices than the int32 vertex loops allow: refused before anything is allocated
    big = 2 ** 31 - 2 ** 25 + 1
    s = torch.tensor([0], dtype=torch.int32, device="cuda")
    d = torch.tensor([1], dtype=torch.int32, device="cuda")
    with pytest.raises(tc.TCError) as e:
        tc.Graph.build(s, d, big)
    assert e.value.status == tc.TC_E_RANGE
    off = np.zeros(2, np.int64)  # n is checked before the offsets are read
    T = ctypes.c_uint64()
    st = tc.lib().tc_count_streamed(tc._hptr(off), None, big, 0, 1 << 20, tc._stream(None), ctypes.byref(T), None)
    assert st == tc.TC_E_RANGE


# ---------------------------------------------------------------- batches ---

def _mixed_batch(count, seed):
    specs = synth.batch_specs(count, seed)
    els = [sp.make() for sp in specs]
    return els


def test_batch_matches_standalone(tc):
    import torch

    els = _mixed_batch(40, 77)
    els += [synth.empty(5), synth.complete(12), synth.wheel(9)]
    src = np.concatenate([e.src for e in els])
    dst = np.concatenate([e.dst for e in els])
    eoff = np.zeros(len(els) + 1, np.int64)
    eoff[1:] = np.cumsum([e.num_edges for e in els])
    npg = np.array([e.n for e in els], np.int32)
    s, d = torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda()
    with tc.Graph.build_batch(s, d, eoff, npg) as g:
        assert g.num_graphs == len(els)
        T = torch.zeros(len(els), dtype=torch.int64, device="cuda")
        t = torch.zeros(int(npg.sum()), dtype=torch.int64, device="cuda")
        g.batch_count(T, t)
        torch.cuda.synchronize()
        T = T.cpu().numpy()
        t = u64(t)
        base = 0
        for i, e in enumerate(els):
            ref = oracle.solve(e.src, e.dst, e.n)
            assert T[i] == ref.T, (i, e.name)
            np.testing.assert_array_equal(t[base:base + e.n], ref.t)
            base += e.n
        assert g.count() == int(T.sum())


def test_batch_range_error(tc):
    import torch

    src = np.array([0, 1, 0, 2], np.int32)
    dst = np.array([1, 2, 1, 3], np.int32)  # graph 1 has 3 vertices: id 3 is out of range
    with pytest.raises(tc.TCError) as e:
        tc.Graph.build_batch(src, dst, np.array([0, 2, 4]), np.array([3, 3]))
    assert e.value.status == tc.TC_E_RANGE


# ---------------------------------------------------------- config sizes ---

def test_config_er10k(tc):
    check_all(tc, synth.config_er10k(), listing=True, label="ER G(10^4, 0.0016) seed 1")


def test_config_ba22(tc):
    """PA n=2^22, 8 edges per new node, seed 2: T, t_v, clustering and the sorted list."""
    check_all(tc, synth.config_ba22(), listing=True, label="BA n=2^22 k=8 seed 2")


@pytest.fixture(scope="module")
def rmat19():
    el = synth.rmat(19, 16, 21)
    return el, oracle.solve(el.src, el.dst, el.n, per_node=True, listing=False)


@pytest.mark.parametrize("hub,load", [(16, 2), (16, 1), (256, 2)])
def test_block_hash_tables(tc, rmat19, hub, load):
    """R-MAT 19 (n = 2^19): with pivots of more than 16 entries on the block path, 93,679 of them span more
    ranks than a block's bitmap holds and take the block hash table (either bucket load); per-node counts
    and clustering in full against the oracle."""
    el, ref = rmat19
    old = (tc.get_option(tc.OPT_HUB_DHAT), tc.get_option(tc.OPT_HUB_BUCKET_LOAD))
    tc.set_option(tc.OPT_HUB_DHAT, hub)
    tc.set_option(tc.OPT_HUB_BUCKET_LOAD, load)
    try:
        with tc.Graph.build(*to_dev(el), el.n) as g:
            say(f"[parity] R-MAT 19 block hash hub={hub} load={load}")
            assert g.m == ref.m
            assert g.count() == ref.T
            T, t = g.count_per_node()
            assert T == ref.T
            np.testing.assert_array_equal(u64(t), ref.t)
            num, den, c = g.clustering()
            np.testing.assert_array_equal(u64(num), ref.num)
            np.testing.assert_array_equal(c.cpu().numpy().view(np.uint64), ref.cc.view(np.uint64))
    finally:
        tc.set_option(tc.OPT_HUB_DHAT, old[0])
        tc.set_option(tc.OPT_HUB_BUCKET_LOAD, old[1])


@pytest.mark.parametrize("hub", [256, 0])
def test_complete_graph_with_lists_past_the_slice_caps(tc, hub):
    """K_5000 by its closed forms: in the degree order (all degrees equal, ties by id) N_v holds the 4999 - v
    later vertices, so the first pivots' lists exceed the 2048- and 4096-entry slices that hub items stage
    and are cut into several slices. T = C(n,3); t_v = C(n-1,2); every clustering coefficient is 1;
    P = sum C(dhat,2) = C(n,3); W = sum over edges of dhat_v + dhat_u = (n-1) m."""
    import torch

    n = 5000
    el = synth.complete(n)
    old = tc.get_option(tc.OPT_HUB_DHAT)
    tc.set_option(tc.OPT_HUB_DHAT, hub)
    try:
        with tc.Graph.build(*to_dev(el), n) as g:
            say(f"[parity] K_{n} hub={hub}")
            m = n * (n - 1) // 2
            assert g.m == m and g.dhat_max == n - 1
            T3 = math.comb(n, 3)
            assert g.count() == T3
            T, t = g.count_per_node()
            assert T == T3
            assert np.all(u64(t) == math.comb(n - 1, 2))
            num, den, c = g.clustering()
            assert np.all(u64(num) == math.comb(n - 1, 2)) and np.all(u64(den) == math.comb(n - 1, 2))
            assert np.all(c.cpu().numpy() == 1.0)
            W, P = g.work()
            assert P == T3 and W == (n - 1) * m
    finally:
        tc.set_option(tc.OPT_HUB_DHAT, old)


def test_sparse_graph_on_a_large_id_range(tc):
    """A small R-MAT graph spread over ids 0 .. n-1 with n = 2^28 + 3 (29-bit ids, 58-bit sort keys). By
    relabelling invariance (pinned in the oracle tests) every output is the compact graph's, mapped through
    the increasing id map; the map keeps the degree-order ties, so W and P are unchanged too. Unused ids are
    isolated: per-node counts and clustering numerators 0."""
    import torch

    small = synth.rmat(11, 8, 77)
    k = small.n
    n = (1 << 28) + 3
    ids = np.arange(k, dtype=np.int64) * ((n - 1) // (k - 1))
    ids[-1] = n - 1
    assert np.all(np.diff(ids) > 0)
    ref = oracle.solve(small.src, small.dst, k, per_node=True, listing=True)
    say(f"[parity] large id range: n={n} k={k} m={ref.m} T={ref.T}")
    s = torch.from_numpy(ids[small.src].astype(np.int32)).cuda()
    d = torch.from_numpy(ids[small.dst].astype(np.int32)).cuda()
    with tc.Graph.build(s, d, n) as g:
        assert g.n == n and g.m == ref.m
        assert g.count() == ref.T
        T, t = g.count_per_node()
        assert T == ref.T
        t = t.cpu().numpy().astype(np.uint64)
        np.testing.assert_array_equal(t[ids], ref.t)
        assert int(t.sum()) == 3 * ref.T
        del t
        num, den, c = g.clustering()
        num = num.cpu().numpy().astype(np.uint64)
        np.testing.assert_array_equal(num[ids], ref.num)
        assert int(num.sum()) == 3 * ref.T
        del num, den
        c = c.cpu().numpy()
        np.testing.assert_array_equal(c[ids].view(np.uint64), ref.cc.view(np.uint64))
        del c
        np.testing.assert_array_equal(g.list().cpu().numpy(), ids[ref.tri].astype(np.int32))
        W, P = g.work()
        assert W == oracle.work(ref.off, ref.adj, k)
        dh = np.diff(ref.off).astype(np.int64)
        assert P == int((dh * (dh - 1) // 2).sum())


# ----------------------------------------------------------------- orders ---

@pytest.mark.parametrize("order", [0, 1, 2, 3, 4])
def test_orders_count_each_triangle_once(tc, order):
    """Theorem 1: every total order gives the same exact outputs; Theorem 3:
    the degree order has the smallest sum_v d_v * dhat_v."""
    el = synth.rmat(13, 16, 17)
    ref = oracle.solve(el.src, el.dst, el.n, per_node=True, listing=True)
    lo, hi = ref.extra["lo"], ref.extra["hi"]
    best = int((ref.deg * np.diff(ref.off)).sum())
    old = tc.get_option(tc.OPT_ORDER)
    tc.set_option(tc.OPT_ORDER, order)
    try:
        s, d = to_dev(el)
        with tc.Graph.build(s, d, el.n) as g:
            say(f"[parity] order {order}")
            assert g.count() == ref.T and g.count_plain() == ref.T
            T, t = g.count_per_node()
            np.testing.assert_array_equal(u64(t), ref.t)
            np.testing.assert_array_equal(g.list().cpu().numpy(), ref.tri)
            cost, kind = g.order_cost()
            assert kind == order and cost >= best
            if order == 0:
                assert cost == best
            if order in (1, 3, 4):  # orders the oracle can reproduce: id, degree descending, coreness (ties by id)
                if order == 4:
                    key = oracle.coreness(*oracle.full_adjacency(lo, hi, el.n), el.n).astype(np.int64)
                else:
                    key = np.zeros(el.n, np.int64) if order == 1 else -ref.deg
                off, adj = oracle.orient_by_key(lo, hi, key, el.n)
                goff, gadj = g.oriented()
                np.testing.assert_array_equal(goff.cpu().numpy(), off)
                np.testing.assert_array_equal(gadj.cpu().numpy(), adj)
                assert cost == int((ref.deg * np.diff(off)).sum())
            Ts, mk, est = g.sparsify_count(0.3, 4)
            assert (Ts, mk) == oracle.sparsified_count(lo, hi, ref.deg, el.n, 0.3, 4)[:2]
    finally:
        tc.set_option(tc.OPT_ORDER, old)


# --------------------------------------------------------------- coreness ---

def _messy_el(n, m, seed):
    """Random raw edge list with loops, repeats and both directions."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    src = np.concatenate([src, dst[: m // 4], np.arange(5, dtype=np.int32)])
    dst = np.concatenate([dst, src[: m // 4], np.arange(5, dtype=np.int32)])
    return synth.EdgeList(n, src, dst, f"messy{seed}")


def _core_ref(el):
    lo, hi = oracle.simple(el.src, el.dst, el.n)
    return oracle.coreness(*oracle.full_adjacency(lo, hi, el.n), el.n)


@pytest.mark.parametrize("name", ["complete", "wheel", "hypercube", "grid", "bipartite", "tripartite", "friendship",
                                  "star", "cycle", "tree", "messy", "rmat", "er", "ba", "empty"])
def test_coreness_matches_oracle(tc, name):
    """Coreness (the k-core order of Section 4) equals the oracle's bucket peeling exactly."""
    el = {
        "complete": lambda: synth.complete(30), "wheel": lambda: synth.wheel(40), "hypercube": lambda: synth.hypercube(7),
        "grid": lambda: synth.grid(17, 23), "bipartite": lambda: synth.complete_bipartite(9, 31),
        "tripartite": lambda: synth.complete_tripartite(5, 8, 13), "friendship": lambda: synth.friendship(25),
        "star": lambda: synth.star(500), "cycle": lambda: synth.cycle(1001), "tree": lambda: synth.random_tree(3000, 8),
        "messy": lambda: _messy_el(700, 5000, 3), "rmat": lambda: synth.rmat(15, 16, 23),
        "er": lambda: synth.er(20000, 0.0008, 6), "ba": lambda: synth.ba(30000, 6, 7), "empty": lambda: synth.empty(50),
    }[name]()
    s, d = to_dev(el)
    with tc.Graph.build(s, d, el.n) as g:
        say(f"[parity] coreness {name} n={el.n}")
        np.testing.assert_array_equal(g.coreness().cpu().numpy(), _core_ref(el))


def test_coreness_of_a_batch(tc):
    """In a disjoint union each graph keeps its own coreness."""
    els = [synth.rmat(11, 8, 30 + i) for i in range(3)] + [synth.wheel(50), synth.complete(12), synth.empty(7)]
    from paper_1706_05151_amd import batch
    packed = batch.pack(els)
    s, d = to_dev(synth.EdgeList(int(packed["n_per_graph"].sum()), packed["src"], packed["dst"], "batch"))
    with tc.Graph.build_batch(s, d, packed["edge_off"], packed["n_per_graph"]) as g:
        core = g.coreness().cpu().numpy()
    ref = np.concatenate([_core_ref(el) for el in els])
    np.testing.assert_array_equal(core, ref)


def test_coreness_refused_on_sample(tc):
    el = synth.rmat(10, 8, 2)
    s, d = to_dev(el)
    with tc.Graph.build(s, d, el.n) as g:
        h = g.sparsify_build(0.5, 1)
        try:
            with pytest.raises(tc.TCError):
                h.coreness()
        finally:
            h.close()


# ------------------------------------------------- load-balancing schemes ---

@pytest.mark.parametrize("scheme", range(7))
def test_partitioned_count_matches_oracle(tc, scheme):
    """Section 5 partitioning: boundaries and per-range merge work equal the oracle's, T is exact."""
    for el, parts in ((synth.rmat(12, 16, 52), 64), (synth.ba(20000, 5, 53), 200), (synth.er(5000, 0.004, 54), 7),
                      (synth.wheel(300), 5)):
        lo, hi = oracle.simple(el.src, el.dst, el.n)
        deg = oracle.degrees(lo, hi, el.n)
        off, adj = oracle.orient(lo, hi, deg, el.n)
        T_ref = oracle.count_nin(off, adj, el.n)[0]
        bounds, work = oracle.partition_work(off, adj, deg, el.n, scheme, parts)
        s, d = to_dev(el)
        with tc.Graph.build(s, d, el.n) as g:
            say(f"[parity] scheme {scheme} {el.name} parts {parts}")
            T, gb, gw = g.count_partitioned(scheme, parts)
            assert T == T_ref
            np.testing.assert_array_equal(gb.cpu().numpy(), bounds)
            np.testing.assert_array_equal(gw.cpu().numpy().astype(np.uint64), work)


def test_partitioned_count_errors(tc):
    el = synth.rmat(9, 8, 1)
    s, d = to_dev(el)
    with tc.Graph.build(s, d, el.n) as g:
        with pytest.raises(tc.TCError):
            g.count_partitioned(7, 4)
        with pytest.raises(tc.TCError):
            g.count_partitioned(0, 0)
        T, b, w = g.count_partitioned(5, 1)  # one range: the whole graph
        assert T == g.count() and b.cpu().tolist() == [0, el.n]


# ----------------------------------------------------------------- shards ---

def _shard_ref(el, k, cost=0):
    """Oracle positions, shard boundaries and per-shard counts (triangles by lowest vertex)."""
    lo, hi = oracle.simple(el.src, el.dst, el.n)
    deg = oracle.degrees(lo, hi, el.n)
    off, adj = oracle.orient(lo, hi, deg, el.n)
    pos = oracle.order_positions(deg, el.n)
    b = oracle.shard_bounds(off, adj, el.n, pos, k, cost)
    T = [oracle.count_nin_pos_range(off, adj, el.n, pos, int(b[j]), int(b[j + 1])) for j in range(k)]
    return pos, b, T, (lo, hi, deg, off, adj)


SHARD_GRAPHS = [synth.rmat(12, 16, 61), synth.ba(20000, 5, 62), synth.er(3000, 0.01, 63), synth.wheel(300),
                synth.complete(40)]


@pytest.mark.parametrize("k,cost", [(1, 0), (3, 0), (8, 0), (3, 1), (8, 1)])
def test_shards_match_oracle(tc, k, cost):
    """Shard boundaries (both costs), each shard's count and the order export equal the oracle's;
    shards add up to T."""
    for el in SHARD_GRAPHS:
        pos, b, T, _ = _shard_ref(el, k, cost)
        s, d = to_dev(el)
        with tc.Graph.build(s, d, el.n) as g:
            say(f"[parity] shards k={k} cost={cost} {el.name}")
            order = g.order().cpu().numpy()
            np.testing.assert_array_equal(pos[order], np.arange(el.n))
            gb = g.shard_bounds(k, cost)
            assert gb == b.tolist()
            gT = [g.count_shard(gb[j], gb[j + 1]) for j in range(k)]
            assert gT == T
            assert sum(gT) == g.count()


@pytest.mark.parametrize("seed", range(4))
def test_shard_ranges_messy(tc, seed):
    """Arbitrary position ranges (empty, single vertex, whole graph) on raw edge lists."""
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(5, 400))
    el = _messy_el(n, int(rng.integers(0, 12 * n)), seed)
    lo, hi = oracle.simple(el.src, el.dst, n)
    deg = oracle.degrees(lo, hi, n)
    off, adj = oracle.orient(lo, hi, deg, n)
    pos = oracle.order_positions(deg, n)
    ranges = [(0, 0), (0, n), (n, n), (n - 1, n)] + [tuple(sorted(rng.integers(0, n + 1, 2).tolist())) for _ in range(8)]
    s, d = to_dev(el)
    with tc.Graph.build(s, d, n) as g:
        say(f"[parity] shard ranges seed {seed} n={n}")
        for a, b in ranges:
            assert g.count_shard(a, b) == oracle.count_nin_pos_range(off, adj, n, pos, a, b), (a, b)


@pytest.mark.parametrize("hub,iw", [(0, 64), (16, 4096), (256, 0)])
def test_shard_partitioner_settings(tc, hub, iw):
    """A shard's own work plan follows the partitioner options and still counts exactly."""
    el = synth.rmat(13, 16, 64)
    pos, b, T, _ = _shard_ref(el, 5)
    s, d = to_dev(el)
    tc.set_option(tc.OPT_HUB_DHAT, hub)
    tc.set_option(tc.OPT_ITEM_WORK, iw)
    try:
        with tc.Graph.build(s, d, el.n) as g:
            say(f"[parity] shard settings hub={hub} iw={iw}")
            assert [g.count_shard(int(b[j]), int(b[j + 1])) for j in range(5)] == T
    finally:
        tc.set_option(tc.OPT_HUB_DHAT, 256)
        tc.set_option(tc.OPT_ITEM_WORK, 0)


def test_shard_of_sampled_graph(tc):
    """Shards of a sampled graph: triangles of the sample by lowest vertex, positions of the full graph."""
    el = synth.rmat(13, 16, 65)
    pos, b, _, (lo, hi, deg, _, _) = _shard_ref(el, 4)
    klo, khi = oracle.sparsify(lo, hi, 0.4, 7)
    koff, kadj = oracle.orient(klo, khi, deg, el.n)
    ref = [oracle.count_nin_pos_range(koff, kadj, el.n, pos, int(b[j]), int(b[j + 1])) for j in range(4)]
    s, d = to_dev(el)
    with tc.Graph.build(s, d, el.n) as g, g.sparsify_build(0.4, 7) as gs:
        say("[parity] shards of a sampled graph")
        assert [gs.count_shard(int(b[j]), int(b[j + 1])) for j in range(4)] == ref
        assert sum(ref) == gs.count()


def test_shard_errors(tc):
    el = synth.rmat(9, 8, 66)
    s, d = to_dev(el)
    with tc.Graph.build(s, d, el.n) as g:
        for a, b in ((-1, 3), (5, 4), (0, el.n + 1)):
            with pytest.raises(tc.TCError):
                g.count_shard(a, b)
        with pytest.raises(tc.TCError):
            g.shard_bounds(0)
        with pytest.raises(tc.TCError):
            g.shard_bounds(4, 2)
        with g.sparsify_build(0.5, 1) as gs:
            with pytest.raises(tc.TCError):
                gs.order()
            with pytest.raises(tc.TCError):
                gs.sparsify_count_partitioned(0.5, 1, 2)
        for q, parts in ((0.0, 2), (1.5, 2), (0.5, 0)):
            with pytest.raises(tc.TCError):
                g.sparsify_count_partitioned(q, 1, parts)


@pytest.mark.parametrize("q,seed,parts", [(0.1, 3, 8), (0.5, 11, 4), (0.3, 2 ** 63 + 5, 1), (1.0, 4, 6),
                                          (0.25, 8, 64)])
def test_partitioned_sample_matches_oracle(tc, q, seed, parts):
    """Per-shard independent samples (Section 7 with overlapping partitions): every shard's T_s,
    the boundaries and the estimate equal the oracle's."""
    for el in (synth.rmat(13, 16, 67), synth.ba(10000, 8, 68)):
        lo, hi = oracle.simple(el.src, el.dst, el.n)
        deg = oracle.degrees(lo, hi, el.n)
        T_parts, b, Ts, est = oracle.sparsified_count_partitioned(lo, hi, deg, el.n, q, seed, parts)
        s, d = to_dev(el)
        with tc.Graph.build(s, d, el.n) as g:
            say(f"[parity] partitioned sample q={q} seed={seed} parts={parts} {el.name}")
            gT, gb, gTs, gest = g.sparsify_count_partitioned(q, seed, parts)
            assert gb == b.tolist()
            assert gT == T_parts
            assert gTs == Ts and gest == est
            if parts == 1:
                assert g.sparsify_count(q, oracle.partition_seed(seed, 0))[0] == Ts


# ------------------------------------------------------ streamed (host CSR) ---

def _rank_csr(el):
    """The rank-space oriented CSR built on the CPU from the oracle's orientation and positions:
    row pos[v] holds pos[u] for u in N_v, ascending. Returns (off int64[n+1], adj int32[m], T)."""
    lo, hi = oracle.simple(el.src, el.dst, el.n)
    deg = oracle.degrees(lo, hi, el.n)
    off, adj = oracle.orient(lo, hi, deg, el.n)
    T = oracle.count_nin(off, adj, el.n)[0]
    pos = oracle.order_positions(deg, el.n).astype(np.int64)
    rows = pos[np.repeat(np.arange(el.n), np.diff(off))]
    cols = pos[adj]
    o = np.lexsort((cols, rows))
    roff = np.zeros(el.n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=el.n), out=roff[1:])
    return roff, np.ascontiguousarray(cols[o], dtype=np.int32), T


STREAM_GRAPHS = [synth.rmat(12, 16, 71), synth.ba(5000, 6, 72), synth.er(2000, 0.01, 73), synth.wheel(500),
                 synth.complete(60)]


def test_export_csr_matches_positions(tc):
    """The exported rank-space CSR equals the one built from the oracle's order and orientation."""
    for el in STREAM_GRAPHS:
        roff, radj, _ = _rank_csr(el)
        s, d = to_dev(el)
        with tc.Graph.build(s, d, el.n) as g:
            say(f"[parity] export csr {el.name}")
            off, adj = g.export_csr()
            np.testing.assert_array_equal(off.numpy(), roff)
            np.testing.assert_array_equal(adj.numpy(), radj)


@pytest.mark.parametrize("budget", [24 << 10, 256 << 10, 64 << 20])
def test_streamed_matches_oracle(tc, budget):
    """The streamed count of a host-resident CSR equals the oracle's T for budgets that split the
    graph into many pivot partitions and chunks and for one that holds it whole."""
    import torch

    for el in STREAM_GRAPHS:
        roff, radj, T = _rank_csr(el)
        say(f"[parity] streamed {el.name} budget {budget}")
        got, info = tc.count_streamed(roff, radj, el.n, budget)
        assert got == T, info
        if budget == 24 << 10 and el.n >= 2000:
            assert info["partitions"] > 1 and info["chunks"] > 1
        # pinned host tensors and a device-resident adj give the same count
        poff = torch.from_numpy(roff).pin_memory()
        padj = torch.from_numpy(radj).pin_memory()
        assert tc.count_streamed(poff, padj, el.n, budget)[0] == T
        assert tc.count_streamed(poff, padj.cuda(), el.n, budget)[0] == T


def test_streamed_edge_cases(tc):
    """Empty graphs, isolated vertices, one edge, one triangle."""
    for n, off, adj, T in ((0, [0], [], 0), (5, [0] * 6, [], 0), (2, [0, 1, 1], [1], 0),
                           (3, [0, 2, 3, 3], [1, 2, 2], 1)):
        got, _ = tc.count_streamed(np.array(off, np.int64), np.array(adj, np.int32), n, 4096)
        assert got == T


def test_streamed_errors(tc):
    n = 4
    good_off = np.array([0, 2, 3, 3, 3], np.int64)
    for adj in ([2, 1, 2], [0, 2, 3], [1, 4, 3], [1, 2, 1]):  # descending, not above its row, >= n, not above row 1
        with pytest.raises(tc.TCError):
            tc.count_streamed(good_off, np.array(adj, np.int32), n, 1 << 20)
    with pytest.raises(tc.TCError):  # offsets that do not start at 0
        tc.count_streamed(np.array([1, 2, 3, 3, 3], np.int64), np.array([1, 2, 3], np.int32), n, 1 << 20)
    with pytest.raises(tc.TCError) as ei:  # decreasing offsets inside a partition (seen on the device)
        tc.count_streamed(np.array([0, 2, 1, 3, 3], np.int64), np.array([1, 2, 3], np.int32), n, 1 << 20)
    assert ei.value.status == tc.TC_E_INVAL
    # decreasing offsets where a budget of about one row per range puts a range's end (seen on the
    # host), and inside one range (seen on the device)
    el = synth.er(2000, 6.0 / 1999, 21)  # rows of at most 7 entries
    roff, radj, _ = _rank_csr(el)
    k = int(np.argmax(np.diff(roff) > 2))
    bad = roff.copy()
    bad[k + 1] = bad[k] - 1  # row k ends before it starts
    for budget in (1 << 20, 8 << 10):
        with pytest.raises(tc.TCError) as ei:
            tc.count_streamed(bad, radj, el.n, budget)
        assert ei.value.status == tc.TC_E_INVAL
    with pytest.raises(tc.TCError):  # budget below the minimum
        tc.count_streamed(good_off, np.array([1, 2, 2], np.int32), n, 1000)
    el = synth.complete(400)  # rows of up to 399 entries: one row needs more than half of 16 KiB
    roff, radj, _ = _rank_csr(el)
    with pytest.raises(tc.TCError):
        tc.count_streamed(roff, radj, el.n, 16 << 10)
