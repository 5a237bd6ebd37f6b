"""Batched counting of many small graphs: one build of their disjoint union and
one launch of the persistent intersection kernel, optionally captured in a HIP
graph and replayed.

The union keeps each graph's vertices contiguous (graph-major degree ranks), so
per-graph totals come out of the same launch (each work item's pivot belongs to
exactly one graph) and per-node counts are per-graph slices of one array.
The autotuner rebuilds the batch's work plan under each candidate partitioner
setting (options of the C ABI, the choice between the pivot kernel and one
thread per edge among them), times the batched count it deploys and keeps the
fastest; settings change speed only, never results.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import tc

AUTOTUNE_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune.json")

# candidate (hub_dhat, item_work, blocks_per_cu, hub_bucket_load, kernel): the pivot kernel's
# block/wave split, item size, occupancy and hash load, or one thread per edge (kernel 1)
DEFAULT_CANDIDATES = [
    (256, 0, 4, 2, 2), (128, 0, 4, 2, 2), (256, 16384, 4, 2, 2), (256, 65536, 4, 2, 2),
    (128, 16384, 4, 2, 2), (64, 4096, 4, 2, 2), (32, 4096, 4, 2, 2), (256, 0, 3, 1, 2),
    (256, 0, 4, 2, 1),
]
_KEYS = (tc.OPT_HUB_DHAT, tc.OPT_ITEM_WORK, tc.OPT_BLOCKS_PER_CU, tc.OPT_HUB_BUCKET_LOAD, tc.OPT_KERNEL)


def pack(edge_lists: Sequence) -> Dict[str, np.ndarray]:
    """Concatenate graphs (objects with n, src, dst) for tc_batch_build."""
    src = np.concatenate([np.asarray(e.src, np.int32) for e in edge_lists]) if edge_lists else np.zeros(0, np.int32)
    dst = np.concatenate([np.asarray(e.dst, np.int32) for e in edge_lists]) if edge_lists else np.zeros(0, np.int32)
    eoff = np.zeros(len(edge_lists) + 1, np.int64)
    eoff[1:] = np.cumsum([len(e.src) for e in edge_lists])
    npg = np.array([e.n for e in edge_lists], np.int32)
    vbase = np.zeros(len(edge_lists) + 1, np.int64)
    vbase[1:] = np.cumsum(npg)
    return {"src": src, "dst": dst, "edge_off": eoff, "n_per_graph": npg, "vbase": vbase}


def current_options():
    return tuple(tc.get_option(k) for k in _KEYS)


def apply_options(opts):
    for k, v in zip(_KEYS, opts):
        tc.set_option(k, int(v))


class BatchCounter:
    """Device-resident batch of graphs with per-graph totals and per-node counts."""

    def __init__(self, packed: Dict[str, np.ndarray], per_node: bool = True, stream=None):
        import torch

        self.torch = torch
        self.packed = packed
        self.num_graphs = int(packed["n_per_graph"].shape[0])
        self.per_node = per_node
        self.stream = stream
        self.src = torch.from_numpy(packed["src"]).cuda()
        self.dst = torch.from_numpy(packed["dst"]).cuda()
        self.graph: Optional[tc.Graph] = None
        self.T = torch.zeros(self.num_graphs, dtype=torch.int64, device="cuda")
        self.t = None
        self.cuda_graph = None

    def build(self):
        if self.graph is not None:
            self.graph.close()
        self.graph = tc.Graph.build_batch(self.src, self.dst, self.packed["edge_off"], self.packed["n_per_graph"],
                                          self.stream)
        if self.per_node:
            self.t = self.torch.zeros(max(self.graph.n, 1), dtype=self.torch.int64, device="cuda")
        return self.graph

    def count(self):
        """Eager per-graph totals (and per-node counts) on the current stream."""
        self.graph.batch_count(self.T, self.t if self.per_node else None, self.stream)
        return self.T

    def capture(self):
        """Record the batched count in a HIP graph (fill kernels, no memset nodes)."""
        torch = self.torch
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.graph.batch_count(self.T, self.t if self.per_node else None, side)  # warm up on the side stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.graph.batch_count(self.T, self.t if self.per_node else None, torch.cuda.current_stream())
        self.cuda_graph = g
        return g

    def replay(self):
        self.cuda_graph.replay()
        return self.T

    def per_graph_t(self) -> List[np.ndarray]:
        t = self.t[: self.graph.n].cpu().numpy().astype(np.uint64)
        vb = self.packed["vbase"]
        return [t[vb[i]:vb[i + 1]] for i in range(self.num_graphs)]

    def close(self):
        self.cuda_graph = None
        if self.graph is not None:
            self.graph.close()
            self.graph = None


def autotune(bc: BatchCounter, candidates=None, reps: int = 3, key: Optional[str] = None, persist: bool = True):
    """Time candidate partitioner settings on the batch in the mode that is
    deployed (tc_batch_count, with per-node counts when bc.per_node) and keep
    the fastest. For each candidate the graph's work plan is rebuilt with its
    settings (tc_graph_replan; tc_batch_count itself never rebuilds), its
    results are checked against the first candidate's, and the batch count is
    timed. The fastest candidate's plan is rebuilt last and stays on the graph,
    so a later capture() records it. Settings change speed only, never
    results. Returns (best, table)."""
    torch = bc.torch
    candidates = candidates or DEFAULT_CANDIDATES
    g = bc.graph
    T_ref = t_ref = None
    table = []
    for opts in candidates:
        apply_options(opts)
        g.replan(bc.stream)
        bc.count()
        torch.cuda.synchronize()
        if T_ref is None:
            T_ref = bc.T.clone()
            t_ref = bc.t.clone() if bc.per_node else None
        assert torch.equal(bc.T, T_ref), "autotuner setting changed the per-graph totals"
        assert t_ref is None or torch.equal(bc.t, t_ref), "autotuner setting changed the per-node counts"
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bc.count()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        table.append({"options": list(opts), "ms": 1e3 * best})
    best = min(table, key=lambda r: r["ms"])
    apply_options(best["options"])
    g.replan(bc.stream)  # the plan of the chosen settings stays on the graph
    if persist and key:
        data = {}
        if os.path.exists(AUTOTUNE_FILE):
            try:
                with open(AUTOTUNE_FILE) as f:
                    data = json.load(f)
            except (OSError, ValueError):
                data = {}
        data[key] = {"options": best["options"], "ms": best["ms"],
                     "keys": ["hub_dhat", "item_work", "blocks_per_cu", "hub_bucket_load", "kernel"]}
        with open(AUTOTUNE_FILE, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return best, table


def load_tuned(key: str):
    """Apply settings persisted by autotune() for `key`; returns them or None."""
    try:
        with open(AUTOTUNE_FILE) as f:
            entry = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if entry:
        apply_options(entry["options"])
        return entry["options"]
    return None
