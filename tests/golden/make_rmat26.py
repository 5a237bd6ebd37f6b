#!/usr/bin/env python3
"""Writes tests/golden/rmat26.json: oracle results for the R-MAT scale-26 workload
(edge factor 16, (0.57,0.19,0.19,0.05), seed 3). Calls only oracle/ and synth/.

Contents: n, m, T, W, d_max, dhat_max; the sparsified counts (T_s, m') at
q = 0.1 and 0.5 with sampler seed 3; d_v and T_v of 64 sampled vertices by the
Section 2 definition. Runs for tens of minutes and needs ~45 GB of host memory.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat26.json")
SAMPLE_SEED = 26


def sample_vertices(n: int) -> np.ndarray:
    """60 ids uniform over [0,n) plus 4 low ids (R-MAT hubs sit at low ids)."""
    u = synth.draws(SAMPLE_SEED, 0x53414d50, 60)
    ids = (u % np.uint64(n)).astype(np.int64)
    return np.concatenate([ids, [1, 3, 17, 1000]]).astype(np.int32)


def main(scale: int = 26):
    t0 = time.time()

    def say(msg):
        print(f"[{time.time() - t0:7.1f}s] {msg}", flush=True)

    el = synth.rmat(scale, 16, 3)
    n = el.n
    say(f"generated E={el.num_edges}")
    sample = sample_vertices(n)
    ts, ds = oracle.sampled_local(el.src, el.dst, n, sample)
    say("sampled local counts done")
    lo, hi = oracle.simple(el.src, el.dst, n)
    del el
    say(f"simple graph m={lo.shape[0]}")
    deg = oracle.degrees(lo, hi, n)
    assert np.array_equal(deg[sample], ds)
    off, adj = oracle.orient(lo, hi, deg, n)
    say("oriented")
    W = oracle.work(off, adj, n)
    T = oracle.count_nin_total_omp(off, adj, n)
    say(f"T={T} W={W}")
    res = {
        "workload": f"R-MAT scale {scale}, edge factor 16, (0.57,0.19,0.19,0.05), seed 3",
        "n": n, "m": int(lo.shape[0]), "T": T, "W": W,
        "d_max": int(deg.max()), "dhat_max": int(np.diff(off).max()),
        "sample_ids": sample.tolist(), "sample_deg": ds.tolist(), "sample_t": [int(x) for x in ts],
        "sparsified": {},
    }
    del off, adj
    for q in (0.1, 0.5):
        klo, khi = oracle.sparsify(lo, hi, q, 3)
        koff, kadj = oracle.orient(klo, khi, deg, n)
        Ts = oracle.count_nin_total_omp(koff, kadj, n)
        res["sparsified"][str(q)] = {"seed": 3, "T_s": Ts, "m_kept": int(klo.shape[0]),
                                     "estimate": oracle.estimate(Ts, q)}
        del klo, khi, koff, kadj
        say(f"q={q}: T_s={Ts}")
    res["threads"] = oracle.num_threads()
    res["seconds"] = time.time() - t0
    with open(OUT if scale == 26 else OUT.replace("26", str(scale)), "w") as f:
        json.dump(res, f, indent=1)
    say("written")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 26)
