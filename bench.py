#!/usr/bin/env python3
"""Benchmark of the exact triangle-counting path on one MI355X.

Default workload: R-MAT scale 26, edge factor 16, (a,b,c,d) = (0.57,0.19,0.19,0.05),
seed 3 (1,073,741,824 generated edge records, symmetrised, deduplicated, loops
dropped). One step = tc_build_csr + tc_count on the edge list already resident
in HBM (the whole exact-count job: simple graph, degree order, oriented CSR,
work plan, intersection). value = oriented edges (m) / seconds per step.

Also reported: the count kernel alone, the plain per-edge merge kernel on the
same graph, the sparsified estimates at q = 0.1 and 0.5, the per-node counts
and clustering coefficients, the roofline of the dominant kernel and the CPU
oracle on a bounded sample.

Other workloads (--workload): er10k (G(10^4, 0.0016) seed 1), ba22 (PA n=2^22,
k=8, seed 2; count + per-node + clustering + list), batch (4096 mixed small
graphs in one launch), serve (open-loop Poisson serving), orders (the same
graphs oriented by degree, id, random, reversed degree and coreness), schemes
(the Section 5 load-balancing cost schemes, one id range per workgroup), shards
(the R-MAT graph's core nodes in --shards ranges, each counted with its own
plan: one GPU's share of a sharded count), sampling (one sample against
independent per-shard samples, Section 7), streamed (the rank-space CSR in
pinned host memory counted under device-memory budgets, Section 6 partitions).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact-count oriented edges/s vs plain kernel; served graphs/s + p50/p99 latency"
HBM_PEAK_GBS = 8000.0
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "k_pivot_rmat26_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1706_05151_amd", "csrc", "pivot_kernel.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(launch_bytes_key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    try:
        with open(PROFILE_SUMMARY) as f:
            s = json.load(f)
    except (OSError, ValueError):
        return None
    if s.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return s.get(launch_bytes_key)


def cpu_baseline(scale: int = 20):
    """The CPU oracle on a bounded sample of the same workload family: R-MAT at
    scale 20 with the same edge factor, probabilities and seed (the full
    scale-26 graph takes the serial oracle tens of minutes). Simple graph,
    degrees and orientation run serially; the counting loop of NodeIteratorN
    runs on all host threads (the oracle's OpenMP total-only variant)."""
    import oracle
    import synth

    el = synth.rmat(scale, 16, 3)
    t0 = time.perf_counter()
    lo, hi = oracle.simple(el.src, el.dst, el.n)
    deg = oracle.degrees(lo, hi, el.n)
    off, adj = oracle.orient(lo, hi, deg, el.n)
    t1 = time.perf_counter()
    T = oracle.count_nin_total_omp(off, adj, el.n)
    t2 = time.perf_counter()
    m = int(lo.shape[0])
    W = oracle.work(off, adj, el.n)
    return {
        "value": m / (t2 - t0),
        "unit": "oriented edges/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"R-MAT scale {scale} edge factor 16 (0.57,0.19,0.19,0.05) seed 3: m={m}, T={T}; "
                  f"build {t1 - t0:.2f} s serial + count {t2 - t1:.2f} s on {oracle.num_threads()} threads; "
                  f"count-only {W / (t2 - t1):.3e} merge steps/s (W={W})",
    }


def cached_full_scale_oracle():
    """The oracle's own run on the whole R-MAT scale-26 workload, stored with its
    results by tests/golden/make_rmat26.py (too long to repeat in a bench run)."""
    path = os.path.join(ROOT, "tests", "golden", "rmat26.json")
    try:
        with open(path) as f:
            g = json.load(f)
    except (OSError, ValueError):
        return None
    out = {"m": g["m"], "T": g["T"], "threads": g.get("threads"), "seconds_total": g.get("seconds"),
           "what": "tests/golden/make_rmat26.py on the build container: generation, 64 vertices by the "
                   "definition, simple graph, degrees and orientation (serial), W, T (counting loop on "
                   "all threads) and two sparsified counts"}
    ph = g.get("phase_seconds")
    if ph:
        out["phase_seconds"] = ph
        if "build" in ph and "count" in ph:
            out["value"] = g["m"] / (ph["build"] + ph["count"])
            out["unit"] = "oriented edges/s"
    return out


def make_workload(name: str, scale: int):
    import synth

    if name == "rmat":
        return synth.config_rmat(scale), f"rmat{scale}-exact-count"
    if name == "ba22":
        return synth.config_ba22(), "ba22-count-pernode-cc-list"
    if name == "er10k":
        return synth.config_er10k(), "er10k-count-pernode-cc"
    raise SystemExit(f"unknown workload {name}")


def run_graph_bench(args):
    import torch

    from paper_1706_05151_amd import tc

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    el, wname = make_workload(args.workload, args.scale)
    gen_s = time.perf_counter() - t0
    log(f"[bench] {wname}: n={el.n} E={el.num_edges} generated in {gen_s:.1f} s")
    src = torch.from_numpy(el.src).cuda()
    dst = torch.from_numpy(el.dst).cuda()
    n = el.n
    del el
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        g = tc.Graph.build(src, dst, n, stream)
        if ev:
            ev[1].record(stream)
        T = g.count(stream)
        if ev:
            ev[2].record(stream)
        return g, T

    for i in range(args.warmup):
        g, T = step()
        g.close()
        log(f"[bench] warmup {i + 1}/{args.warmup} done (T={T})")
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    Ts = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        g, T = step(evs[i])
        Ts.append(T)
        m = g.m
        if i + 1 < args.steps:
            g.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    assert len(set(Ts)) == 1, "count differs between steps"
    build_ms = [evs[i][0].elapsed_time(evs[i][1]) for i in range(args.steps)]
    count_ms = [evs[i][1].elapsed_time(evs[i][2]) for i in range(args.steps)]
    ms_per_step = 1e3 * wall / args.steps
    log(f"[bench] {args.steps} steps: {ms_per_step:.1f} ms/step (build {sum(build_ms) / len(build_ms):.1f} ms, "
        f"count {sum(count_ms) / len(count_ms):.1f} ms)")
    W, P = g.work(stream)
    T = Ts[0]
    out = {
        "metric": METRIC,
        "value": m / (ms_per_step / 1e3),
        "unit": "oriented edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wname, "n": n, "m": m, "edge_records": int(src.numel()), "T": T,
                   "d_max": g.d_max, "dhat_max": g.dhat_max, "W": W, "P": P,
                   "step": "tc_build_csr + tc_count from an edge list resident in HBM",
                   "parallelism": "single GPU"},
    }
    cm = sum(count_ms) / len(count_ms)
    bm = sum(build_ms) / len(build_ms)
    out["build_ms"] = bm
    out["count_ms"] = cm
    out["count_edges_per_s"] = m / (cm / 1e3)
    out["count_steps_per_s"] = W / (cm / 1e3)
    # Roofline of the dominant kernel (k_pivot, the persistent intersection
    # kernel of tc_count) on its own algorithmic bytes per launch: every probed
    # suffix element once (4 B each; P = sum_v C(dhat_v, 2) probes), per
    # oriented edge one 8-byte in-edge record and one staged 4-byte entry of
    # the pivot's list, per vertex the two 8-byte offsets of its list and of
    # its in-edge records.
    b_alg = 4 * P + 12 * m + 16 * n
    achieved = b_alg / (cm / 1e3) / 1e9
    traffic = measured_traffic("hbm_bytes_per_launch") if args.workload == "rmat" and args.scale == 26 else None
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                       "kernel": "k_pivot (one launch per tc_count)",
                       "algorithmic_bytes": b_alg,
                       "model": "4*P + 12*m + 16*n bytes per launch (probed suffix elements, in-edge records, "
                                "staged list entries, offsets)"}
    if traffic:
        # measured HBM bytes of one launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated) over this run's time
        out["roofline"]["traffic_gbs"] = traffic / (cm / 1e3) / 1e9
        out["roofline"]["traffic_frac"] = out["roofline"]["traffic_gbs"] / HBM_PEAK_GBS
    # The paper's merge cost model (Theorem 2): 4 B per merge step of W plus 24 B per
    # oriented edge. The pivot kernel does not move these bytes; the rate is the
    # merge-equivalent throughput, beside count_steps_per_s.
    b_merge = 4 * W + 24 * m
    out["merge_equivalent"] = {"bytes": b_merge, "gbs": b_merge / (cm / 1e3) / 1e9,
                               "model": "4*W + 24*m bytes per count (merge model of Theorem 2)"}
    if not args.no_plain:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        Tp = g.count_plain(stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        assert Tp == T, "plain kernel disagrees"
        pm = ev[0].elapsed_time(ev[1])
        out["plain_count_ms"] = pm
        out["plain_edges_per_s"] = m / (pm / 1e3)
        out["count_speedup_vs_plain"] = pm / cm
        log(f"[bench] plain kernel {pm:.1f} ms (speedup {pm / cm:.1f}x)")
    if args.workload == "rmat":
        sp = {}
        for q in (0.1, 0.5):
            # The first call at a given q also grows the memory pool for the
            # sampled graph's arrays; report it apart from the best of three.
            times = []
            for _ in range(4):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Ts_, mk, est = g.sparsify_count(q, 3, stream)
                times.append(1e3 * (time.perf_counter() - t0))
            dt = min(times[1:])
            sp[str(q)] = {"ms": dt, "first_call_ms": times[0], "T_s": Ts_, "m_kept": mk, "estimate": est,
                          "rel_err": est / T - 1}
            log(f"[bench] sparsified q={q}: {dt:.1f} ms (first call {times[0]:.1f} ms), estimate {est:.4e} "
                f"({est / T - 1:+.4%})")
        out["sparsified"] = sp
        # per-node counts (Section 9) and clustering coefficients on the same graph
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Tn, t = g.count_per_node(stream=stream)
            torch.cuda.synchronize()
            times.append(1e3 * (time.perf_counter() - t0))
            assert Tn == T, "per-node count disagrees"
            del t
        out["per_node_ms"] = min(times[1:])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        num, den, c = g.clustering(stream)
        torch.cuda.synchronize()
        out["clustering_ms"] = 1e3 * (time.perf_counter() - t0)
        del num, den, c
        log(f"[bench] per-node counts {out['per_node_ms']:.1f} ms, clustering {out['clustering_ms']:.1f} ms")
    if args.workload in ("ba22", "er10k"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Tn, t = g.count_per_node(stream=stream)
        num, den, c = g.clustering(stream)
        tri = g.list(stream=stream)
        torch.cuda.synchronize()
        out["pernode_cc_list_ms"] = 1e3 * (time.perf_counter() - t0)
        out["listed"] = int(tri.shape[0])
    g.close()
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline()
        if args.workload == "rmat" and args.scale == 26:
            out["cpu_baseline"]["full_scale"] = cached_full_scale_oracle()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat",
                    choices=["rmat", "ba22", "er10k", "batch", "serve", "orders", "schemes", "shards", "sampling",
                             "streamed"])
    ap.add_argument("--parts", type=int, default=1024, help="id ranges for --workload schemes")
    ap.add_argument("--shards", type=int, default=8, help="core-node shards for --workload shards / sampling")
    ap.add_argument("--scale", type=int, default=26, help="R-MAT scale for --workload rmat")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="trace length for --workload serve")
    ap.add_argument("--serve-budget-frac", type=float, default=0.85,
                    help="device budget for --workload serve, as a fraction of the pool's resident footprint")
    ap.add_argument("--budgets", type=int, nargs="+", default=None,
                    help="device budgets in GiB for --workload streamed (default 4 16 64)")
    ap.add_argument("--e2e-budgets", type=int, nargs="+", default=None,
                    help="budgets in GiB of the out-of-core build + count for --workload streamed "
                         "(default 8 16; 0 skips it)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="first run one device-to-device copy of this many GiB (HBM counter calibration)")
    args = ap.parse_args()
    ws = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or ws != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (one process, no collectives); --gpus must be 1"}), flush=True)
        sys.exit(2)
    if args.calibrate_copy_gib > 0:
        import torch

        nbytes = int(args.calibrate_copy_gib * (1 << 30))
        a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {nbytes} bytes done")
        del a, b
        torch.cuda.empty_cache()
    if args.workload in ("batch", "serve", "orders", "schemes", "shards", "sampling", "streamed"):
        from paper_1706_05151_amd import workloads

        out = workloads.run(args)
    else:
        out = run_graph_bench(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
