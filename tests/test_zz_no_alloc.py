"""GPU test of tc_count_per_node_noalloc, called through the C ABI: its T and
per-node counts equal tc_count_per_node's (and the oracle's) on two calls in a
row, the second on a smaller graph; the vertex limit is enforced before
anything is written."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

MAX_N = 1 << 22


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1706_05151_amd.tc as tcm

    tcm.lib()
    return tcm


def _build(tc, el):
    import torch

    s = torch.from_numpy(np.ascontiguousarray(el.src)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(el.dst)).cuda()
    return tc.Graph.build(s, d, el.n)


def _noalloc(tc, g, out):
    """One call of the allocation-free entry point through the C ABI."""
    T = ctypes.c_uint64()
    st = tc.lib().tc_count_per_node_noalloc(g._h, tc._stream(None), ctypes.byref(T), tc._dptr(out))
    return st, T.value


def _compare(tc, el, label):
    import torch

    say(f"[no-alloc] {label}: n={el.n} E={el.num_edges}")
    with _build(tc, el) as g:
        T_ref, t_ref = g.count_per_node()
        t_ref = t_ref.cpu().numpy().astype(np.uint64)
        out = torch.full((max(g.n, 1),), -7, dtype=torch.int64, device="cuda")  # fully overwritten
        st, T = _noalloc(tc, g, out)
        assert st == tc.TC_OK, tc.lib().tc_last_error()
        torch.cuda.synchronize()
        assert T == T_ref
        np.testing.assert_array_equal(out[: g.n].cpu().numpy().astype(np.uint64), t_ref)
        return T, t_ref


def test_noalloc_equals_per_node_two_calls(tc):
    """A larger graph, then a smaller one: the second call must not see the first's counts."""
    big = synth.rmat(16, 16, 11)
    small = synth.rmat(12, 16, 3)
    T1, t1 = _compare(tc, big, "R-MAT 16")
    T2, t2 = _compare(tc, small, "R-MAT 12 (smaller, after the larger)")
    for el, T, t in ((big, T1, t1), (small, T2, t2)):
        ref = oracle.solve(el.src, el.dst, el.n, per_node=True)
        assert T == ref.T
        np.testing.assert_array_equal(t, ref.t)


def test_noalloc_degenerate_and_max_size(tc):
    # no edges at all: every count zero, though earlier calls left counts behind
    _compare(tc, synth.empty(5), "5 isolated vertices")
    # exactly the largest accepted vertex count: K_40 on the last ids, the rest isolated
    k = synth.complete(40)
    el = synth.EdgeList(MAX_N, (k.src + (MAX_N - 40)).astype(np.int32), (k.dst + (MAX_N - 40)).astype(np.int32),
                        "K_40 in 2^22 vertices")
    T, t = _compare(tc, el, el.name)
    assert T == 40 * 39 * 38 // 6
    assert int(t.sum()) == 3 * T and int(t[-1]) == 39 * 38 // 2


def test_noalloc_refuses_more_vertices(tc):
    import torch

    el = synth.EdgeList(MAX_N + 1, np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32), "triangle")
    say(f"[no-alloc] refusal: n={el.n}")
    with _build(tc, el) as g:
        out = torch.full((g.n,), -7, dtype=torch.int64, device="cuda")
        st, _ = _noalloc(tc, g, out)
        assert st == tc.TC_E_RANGE
        torch.cuda.synchronize()
        assert bool((out == -7).all())
        # the allocating entry point still serves it
        T, t = g.count_per_node()
        assert T == 1 and int(t[:3].sum()) == 3
