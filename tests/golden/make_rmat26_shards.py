#!/usr/bin/env python3
"""Writes tests/golden/rmat26_shards.json: oracle results for the core-node
shards of the R-MAT scale-26 workload (edge factor 16, (0.57,0.19,0.19,0.05),
seed 3). Calls only oracle/ and synth/.

Contents: the boundary positions of 8 shards (the rule x_j = argmin F >= j*alpha
over the merge cost f(v) = sum_{u in N_v} (dhat_v + dhat_u), Section 5), and the
per-shard sampled counts T_i of the overlapping-partition sparsification
(Section 7) at q = 0.1, seed 3, 8 shards. Runs for several minutes and needs
~30 GB of host memory.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat26_shards.json")


def main(scale: int = 26, k: int = 8, q: float = 0.1, seed: int = 3):
    t0 = time.time()

    def say(msg):
        print(f"[{time.time() - t0:7.1f}s] {msg}", flush=True)

    el = synth.rmat(scale, 16, 3)
    n = el.n
    lo, hi = oracle.simple(el.src, el.dst, n)
    del el
    deg = oracle.degrees(lo, hi, n)
    off, adj = oracle.orient(lo, hi, deg, n)
    pos = oracle.order_positions(deg, n)
    bounds = oracle.shard_bounds(off, adj, n, pos, k)
    del off, adj
    say(f"bounds {bounds.tolist()}")
    T_parts = []
    for i in range(k):
        klo, khi = oracle.sparsify(lo, hi, q, oracle.partition_seed(seed, i))
        koff, kadj = oracle.orient(klo, khi, deg, n)
        del klo, khi
        T_parts.append(oracle.count_nin_pos_range(koff, kadj, n, pos, int(bounds[i]), int(bounds[i + 1])))
        del koff, kadj
        say(f"shard {i}: T_s={T_parts[-1]}")
    res = {
        "workload": f"R-MAT scale {scale}, edge factor 16, (0.57,0.19,0.19,0.05), seed 3",
        "shards": k, "bounds": [int(x) for x in bounds],
        "partitioned_sample": {"q": q, "seed": seed, "T_parts": T_parts, "T_s": sum(T_parts),
                               "estimate": oracle.estimate(sum(T_parts), q)},
        "seconds": time.time() - t0,
    }
    with open(OUT if scale == 26 else OUT.replace("26", str(scale)), "w") as f:
        json.dump(res, f, indent=1)
    say("written")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 26)
