"""Seeded synthetic graphs: the inputs shared by the CPU oracle and the GPU library.

Nothing here computes triangles or any step of the counting method; the module
only draws edge lists (``src``, ``dst`` as int32 numpy arrays plus a vertex
count ``n``). Random draws come from a counter-based SplitMix64 stream in
``synth.c`` so that every graph is a pure function of its seed.

Recipes follow the paper's workload families (Gnp, PA, and power-law networks
for which R-MAT stands in) at the sizes of the benchmark configurations.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` with gcc + OpenMP (host code only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    vp = ctypes.c_void_p
    lib.synth_er.argtypes = [i32, dbl, u64, vp, vp]
    lib.synth_er.restype = i64
    lib.synth_ba_edges.argtypes = [i32, i32]
    lib.synth_ba_edges.restype = i64
    lib.synth_ba.argtypes = [i32, i32, u64, vp, vp]
    lib.synth_ba.restype = i64
    lib.synth_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, vp, vp]
    lib.synth_rmat.restype = None
    lib.synth_draws.argtypes = [u64, u64, u64, i64, vp]
    lib.synth_draws.restype = None
    lib.synth_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


@dataclass
class EdgeList:
    """A raw undirected edge list on vertex ids ``0..n-1`` (may hold loops/duplicates)."""

    n: int
    src: np.ndarray  # int32 [E]
    dst: np.ndarray  # int32 [E]
    name: str = ""

    @property
    def num_edges(self) -> int:
        return int(self.src.shape[0])


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def er(n: int, q: float, seed: int, name: str = "") -> EdgeList:
    """Erdos-Renyi G(n,q) over all pairs i<j."""
    lib = _load()
    m = lib.synth_er(n, q, seed, None, None)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    if m:
        lib.synth_er(n, q, seed, _ptr(src), _ptr(dst))
    return EdgeList(n, src, dst, name or f"er(n={n},q={q},seed={seed})")


def ba(n: int, k: int, seed: int, name: str = "") -> EdgeList:
    """Preferential attachment: seed clique K_{k+1}, then k distinct targets per new node."""
    lib = _load()
    m = lib.synth_ba_edges(n, k)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    got = lib.synth_ba(n, k, seed, _ptr(src), _ptr(dst)) if m else 0
    assert got == m
    return EdgeList(n, src, dst, name or f"ba(n={n},k={k},seed={seed})")


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19, name: str = "") -> EdgeList:
    """R-MAT on 2^scale vertices with edge_factor * 2^scale draws (no noise, no permutation)."""
    lib = _load()
    n = 1 << scale
    e = edge_factor * n
    src = np.empty(e, dtype=np.int32)
    dst = np.empty(e, dtype=np.int32)
    lib.synth_rmat(scale, e, a, b, c, seed, _ptr(src), _ptr(dst))
    return EdgeList(n, src, dst, name or f"rmat(scale={scale},ef={edge_factor},seed={seed})")


def draws(seed: int, stream: int, count: int, first: int = 0) -> np.ndarray:
    """``count`` raw 64-bit draws of one stream (used for mixes and arrival times)."""
    out = np.empty(count, dtype=np.uint64)
    if count:
        _load().synth_draws(seed, stream, first, count, _ptr(out))
    return out


def uniforms(seed: int, stream: int, count: int) -> np.ndarray:
    """Uniform doubles in [0,1) with 53 random bits."""
    return (draws(seed, stream, count) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def num_threads() -> int:
    return int(_load().synth_num_threads())


# ---------------------------------------------------------- closed forms ---

def _el(n, pairs, name):
    p = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return EdgeList(n, p[:, 0].astype(np.int32).copy(), p[:, 1].astype(np.int32).copy(), name)


def complete(n: int) -> EdgeList:
    return _el(n, [(i, j) for i in range(n) for j in range(i + 1, n)], f"K{n}")


def wheel(r: int) -> EdgeList:
    """Hub 0 joined to a rim cycle 1..r."""
    pairs = [(0, i) for i in range(1, r + 1)] + [(i, i % r + 1) for i in range(1, r + 1)]
    return _el(r + 1, pairs, f"W{r}")


def star(k: int) -> EdgeList:
    return _el(k + 1, [(0, i) for i in range(1, k + 1)], f"star{k}")


def path(n: int) -> EdgeList:
    return _el(n, [(i, i + 1) for i in range(n - 1)], f"P{n}")


def cycle(n: int) -> EdgeList:
    return _el(n, [(i, (i + 1) % n) for i in range(n)], f"C{n}")


def complete_bipartite(a: int, b: int) -> EdgeList:
    return _el(a + b, [(i, a + j) for i in range(a) for j in range(b)], f"K{a},{b}")


def complete_tripartite(a: int, b: int, c: int) -> EdgeList:
    parts = [list(range(a)), list(range(a, a + b)), list(range(a + b, a + b + c))]
    pairs = []
    for x in range(3):
        for y in range(x + 1, 3):
            pairs += [(i, j) for i in parts[x] for j in parts[y]]
    return _el(a + b + c, pairs, f"K{a},{b},{c}")


def friendship(k: int) -> EdgeList:
    """k triangles sharing the centre vertex 0."""
    pairs = []
    for t in range(k):
        x, y = 1 + 2 * t, 2 + 2 * t
        pairs += [(0, x), (0, y), (x, y)]
    return _el(2 * k + 1, pairs, f"F{k}")


def hypercube(d: int) -> EdgeList:
    n = 1 << d
    return _el(n, [(v, v ^ (1 << i)) for v in range(n) for i in range(d) if v < v ^ (1 << i)], f"Q{d}")


def grid(r: int, c: int) -> EdgeList:
    pairs = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                pairs.append((v, v + 1))
            if i + 1 < r:
                pairs.append((v, v + c))
    return _el(r * c, pairs, f"grid{r}x{c}")


def random_tree(n: int, seed: int) -> EdgeList:
    u = draws(seed, 0x5452, max(n - 1, 0))
    pairs = [(v, int(u[v - 1] % np.uint64(v))) for v in range(1, n)]
    return _el(n, pairs, f"tree{n}")


def empty(n: int) -> EdgeList:
    return EdgeList(n, np.zeros(0, np.int32), np.zeros(0, np.int32), f"empty{n}")


# ------------------------------------------------------ workload recipes ---

def config_er10k() -> EdgeList:
    """Plain exact count: G(n=10,000, q=0.0016), seed 1."""
    return er(10_000, 0.0016, 1, "er10k")


def config_ba22() -> EdgeList:
    """Preferential attachment n=2^22, 8 edges per new node, seed 2."""
    return ba(1 << 22, 8, 2, "ba22")


def config_rmat(scale: int = 26) -> EdgeList:
    """R-MAT scale 26, edge factor 16, (0.57,0.19,0.19,0.05), seed 3."""
    return rmat(scale, 16, 3, name=f"rmat{scale}")


@dataclass
class GraphSpec:
    kind: str  # "er" | "ba" | "rmat"
    n: int
    param: float  # q for ER, k for BA, edge factor for R-MAT
    seed: int

    def make(self) -> EdgeList:
        if self.kind == "er":
            return er(self.n, self.param, self.seed)
        if self.kind == "ba":
            return ba(self.n, int(self.param), self.seed)
        scale = int(round(math.log2(self.n)))
        return rmat(scale, int(self.param), self.seed)


def batch_specs(count: int = 4096, seed: int = 4) -> list:
    """Mixed batch: n ~ U[64,8192]; 1/3 ER (avg degree U[8,32]), 1/3 BA (k ~ U{4..16}),
    1/3 R-MAT (edge factor 8, scale = floor(log2 n), n := 2^scale)."""
    d = draws(seed, 0x4241544348, 4 * count)
    specs = []
    for g in range(count):
        kind = ("er", "ba", "rmat")[int(d[4 * g] % np.uint64(3))]
        n = 64 + int(d[4 * g + 1] % np.uint64(8192 - 64 + 1))
        gseed = int(d[4 * g + 3] & np.uint64(0x7FFFFFFFFFFFFFFF))
        if kind == "er":
            deg = 8.0 + 24.0 * float(d[4 * g + 2] >> np.uint64(11)) / 9007199254740992.0
            specs.append(GraphSpec("er", n, deg / (n - 1), gseed))
        elif kind == "ba":
            specs.append(GraphSpec("ba", n, 4 + int(d[4 * g + 2] % np.uint64(13)), gseed))
        else:
            scale = int(math.floor(math.log2(n)))
            specs.append(GraphSpec("rmat", 1 << scale, 8, gseed))
    return specs


def pool_specs(count: int = 1024, seed: int = 5, n_lo: float = 1e3, n_hi: float = 1e6) -> list:
    """Serving pool: n log-uniform in [n_lo, n_hi], average degree 16
    (ER q = 16/(n-1), BA k = 8, R-MAT edge factor 8 with scale = round(log2 n))."""
    d = draws(seed, 0x504f4f4c, 3 * count)
    specs = []
    for g in range(count):
        kind = ("er", "ba", "rmat")[int(d[3 * g] % np.uint64(3))]
        u = float(d[3 * g + 1] >> np.uint64(11)) / 9007199254740992.0
        n = int(round(math.exp(math.log(n_lo) + u * (math.log(n_hi) - math.log(n_lo)))))
        gseed = int(d[3 * g + 2] & np.uint64(0x7FFFFFFFFFFFFFFF))
        if kind == "er":
            specs.append(GraphSpec("er", n, 16.0 / (n - 1), gseed))
        elif kind == "ba":
            specs.append(GraphSpec("ba", n, 8, gseed))
        else:
            scale = int(round(math.log2(n)))
            specs.append(GraphSpec("rmat", 1 << scale, 8, gseed))
    return specs


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate on [0, duration)."""
    expected = int(rate * duration * 1.2 + 100)
    u = uniforms(seed, 0x41525256, expected)
    gaps = -np.log1p(-u) / rate
    t = np.cumsum(gaps)
    return t[t < duration]
