"""GPU tests of the out-of-core path (graphs larger than the device, Section 6):
tc_build_csr_host builds the rank-space oriented CSR of a host edge list under
a device budget, and tc_count_streamed counts it under the same budget. The
lists are checked against the oracle's orientation (mapped through the order
of Eq. (1) the oracle computes), and T against the oracle."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GOLDEN20 = os.path.join(os.path.dirname(__file__), "golden", "rmat20.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    import torch

    assert torch.cuda.is_available()
    import paper_1706_05151_amd.tc as tcm

    tcm.lib()
    return tcm


def _check_against_oracle(el, off, adj):
    """off/adj (rank space) equal the oracle's N_v lists, by id, under the oracle's order."""
    ref = oracle.solve(el.src, el.dst, el.n, per_node=False)
    pos = oracle.order_positions(ref.deg, el.n)
    order = np.empty(el.n, np.int64)
    order[pos] = np.arange(el.n)
    off = np.asarray(off, dtype=np.int64)
    adj = np.asarray(adj, dtype=np.int64)
    assert int(off[-1]) == ref.m and adj.shape[0] == ref.m
    # row r of the rank-space CSR is N_v of v = order[r]; entries are ranks, ascending
    dh = np.diff(off)
    np.testing.assert_array_equal(dh, np.diff(ref.off)[order])
    rows = np.repeat(np.arange(el.n), dh)
    assert np.all(adj > rows)  # entries after their row
    assert np.all((np.diff(adj) > 0) | (np.diff(rows) != 0))  # ascending within rows
    ids = order[adj]
    by_id_rows = order[rows]
    key = by_id_rows * el.n + ids  # (v, w) pairs by id
    ref_rows = np.repeat(np.arange(el.n), np.diff(ref.off))
    np.testing.assert_array_equal(np.sort(key), np.sort(ref_rows * el.n + ref.adj.astype(np.int64)))
    return ref


def test_messy_lists_and_edge_cases(tc):
    """Loops, repeats and reversed pairs at the smallest budget; no edge; one edge."""
    import torch

    rng = np.random.default_rng(7)
    n = 3000
    a = rng.integers(0, n, 40000).astype(np.int32)
    c = (a + rng.integers(-30, 31, 40000)).clip(0, n - 1).astype(np.int32)
    src = np.concatenate([a, c, a[:500], np.arange(50, dtype=np.int32)])
    dst = np.concatenate([c, a, c[:500], np.arange(50, dtype=np.int32)])  # reversed pairs, repeats, loops
    el = synth.EdgeList(n, src, dst, "messy")
    budget = 64 * n + (32 << 20)
    off, adj, info = tc.build_csr_host(src, dst, n, budget)
    say(f"[ooc] messy n={n} E={len(src)}: {info}")
    ref = _check_against_oracle(el, off.numpy(), adj.numpy())
    T, sinfo = tc.count_streamed(off, adj, n, budget)
    assert T == ref.T
    # the same arrays as the in-HBM build
    with tc.Graph.build(torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(), n) as g:
        o2, a2 = g.export_csr()
        np.testing.assert_array_equal(o2.numpy(), off.numpy())
        np.testing.assert_array_equal(a2.numpy(), adj.numpy())
    # no edges; one edge
    off0, adj0, _ = tc.build_csr_host(np.zeros(0, np.int32), np.zeros(0, np.int32), 5, budget)
    assert off0.numpy().tolist() == [0] * 6 and adj0.numel() == 0
    off1, adj1, _ = tc.build_csr_host(np.array([3], np.int32), np.array([1], np.int32), 5, budget)
    assert off1.numpy().tolist() == [0, 0, 0, 0, 1, 1] and adj1.numpy().tolist() == [4]


def test_errors(tc):
    src = np.array([0, 1, 7], np.int32)
    dst = np.array([1, 2, 0], np.int32)
    with pytest.raises(tc.TCError) as e:
        tc.build_csr_host(src, dst, 5, 64 << 20)
    assert e.value.status == tc.TC_E_RANGE
    with pytest.raises(tc.TCError) as e:
        tc.build_csr_host(src[:2], dst[:2], 5, 1 << 20)
    assert e.value.status == tc.TC_E_NOMEM


def test_rmat20_end_to_end_under_a_budget(tc):
    """R-MAT scale 20 (16.8e6 records) under 96 MiB, less than half of the graph's
    resident footprint in HBM: built in parts and row ranges, counted streamed, T
    against the stored oracle result, the lists against the oracle's orientation."""
    import torch

    with open(GOLDEN20) as f:
        gold = json.load(f)
    el = synth.rmat(20, 16, 3)
    budget = 96 << 20
    src = torch.from_numpy(el.src).pin_memory()
    dst = torch.from_numpy(el.dst).pin_memory()
    with tc.Graph.build(src.cuda(), dst.cuda(), el.n) as g:
        resident = g.bytes()
        o2, a2 = g.export_csr()
    say(f"[ooc] R-MAT 20 resident footprint {resident / 2**20:.0f} MiB, budget {budget >> 20} MiB")
    assert resident > 2 * budget
    off, adj, info = tc.build_csr_host(src, dst, el.n, budget)
    say(f"[ooc] build: {info}")
    assert info["parts"] > 1 and info["row_ranges"] > 1
    assert adj.numel() == gold["m"]
    np.testing.assert_array_equal(off.numpy(), o2.numpy())
    np.testing.assert_array_equal(adj.numpy(), a2.numpy())
    T, sinfo = tc.count_streamed(off, adj, el.n, budget)
    say(f"[ooc] count: {sinfo}")
    assert T == gold["T"]
    _check_against_oracle(el, off.numpy(), adj.numpy())


@pytest.mark.parametrize("scale", [16, 17])
def test_row_ranges_streamed_or_split(tc, scale):
    """At the smallest budget (64 n + 32 MiB: 524,288 entries per row range), R-MAT 16 needs two row
    ranges (each streams every unique key through) and R-MAT 17 four (the oriented keys are split by
    range in one pass and each range loads its own part): both give the resident build's CSR, and the
    streamed count of it gives the oracle's T."""
    import torch

    el = synth.rmat(scale, 16, 5)
    ref = oracle.solve(el.src, el.dst, el.n, per_node=False)
    budget = 64 * el.n + (32 << 20)
    src = torch.from_numpy(el.src).pin_memory()
    dst = torch.from_numpy(el.dst).pin_memory()
    say(f"[ooc] R-MAT {scale} at {budget >> 20} MiB")
    off, adj, info = tc.build_csr_host(src, dst, el.n, budget)
    say(f"[ooc] build: {info}")
    if scale == 16:
        assert info["row_ranges"] == 2
    else:
        assert info["row_ranges"] >= 3
    with tc.Graph.build(src.cuda(), dst.cuda(), el.n) as g:
        o2, a2 = g.export_csr()
    np.testing.assert_array_equal(off.numpy(), o2.numpy())
    np.testing.assert_array_equal(adj.numpy(), a2.numpy())
    T, _ = tc.count_streamed(off, adj, el.n, budget)
    assert T == ref.T
