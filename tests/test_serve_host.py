"""CPU checks of the serving layer's host parts: the answer digest (the host
side of tc_clustering_digest) against a scalar restatement of its definition,
and its sensitivity to every array and position; the request trace is a pure
function of its seed."""
import numpy as np

from paper_1706_05151_amd import serve

MASK = (1 << 64) - 1


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def _digest_scalar(num, den, c):
    a = b = 0
    for v in range(len(num)):
        cb = int(np.float64(c[v]).view(np.uint64))
        h = _mix(_mix(_mix(_mix(v ^ 0x434C555354455221) ^ int(num[v])) ^ int(den[v])) ^ cb)
        a = (a + h) & MASK
        b = (b + _mix(h ^ 0x4449474553543132)) & MASK
    return f"{a:016x}{b:016x}"


def _answer(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.integers(0, 50, n).astype(np.uint64)
    den = np.where(d >= 2, d * (d - 1) // 2, 0).astype(np.uint64)
    num = np.array([rng.integers(0, x + 1) if x else 0 for x in den], dtype=np.uint64)
    c = np.where(den > 0, num / np.maximum(den, 1), 0.0)
    return num, den, c


def test_digest_matches_scalar_definition():
    for n, seed in ((0, 1), (1, 2), (7, 3), (300, 4)):
        num, den, c = _answer(n, seed)
        assert serve.cc_digest(num, den, c) == _digest_scalar(num, den, c)


def test_digest_sees_every_array_and_position():
    num, den, c = _answer(200, 9)
    base = serve.cc_digest(num, den, c)
    for arr in (num, den):
        for i in (0, 57, 199):
            x = arr.copy()
            x[i] += np.uint64(1)
            args = (x, den, c) if arr is num else (num, x, c)
            assert serve.cc_digest(*args) != base
    c2 = c.copy()
    c2[13] = np.nextafter(c2[13], 2.0)  # one ulp
    assert serve.cc_digest(num, den, c2) != base
    # the same values at swapped positions are a different answer
    i, j = int(np.argmax(num)), int(np.argmin(num))
    p = np.arange(200)
    p[[i, j]] = p[[j, i]]
    assert serve.cc_digest(num[p], den[p], c[p]) != base


def test_trace_is_seeded():
    a = serve.make_trace(1024, 2000.0, 0.5, 5)
    b = serve.make_trace(1024, 2000.0, 0.5, 5)
    assert [(r.kind, r.graph, r.arrival) for r in a] == [(r.kind, r.graph, r.arrival) for r in b]
    assert {r.kind for r in a} == {serve.COUNT, serve.CLUSTER, serve.SPARSE}
