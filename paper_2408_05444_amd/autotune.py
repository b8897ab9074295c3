"""Team-size autotuner for ragged batches (mek_solve_multi).

A ragged launch gives instance b a team of W_b work-groups (sum at most the
compute units). The library's default shares them out by per-update work;
this module chooses them by measurement instead:

  * measure(): the kernel time per update of one instance's dense solver at
    a ladder of team sizes (short solves with the residual in device memory,
    the form a ragged launch uses), kept in a persisted table keyed by the
    instance's sizes and precision;
  * allocate(): starting from one work-group each, repeatedly moves the
    instance with the largest predicted time (updates x time per update at
    its team size) to the next measured team size, while that lowers its
    time and the compute units allow;
  * plans_for(): plans with those team sizes, which mek_solve_multi and
    mek_solve_multi_async then use as given.

Only sequencing and bookkeeping live here; every measurement is a library
solve.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence

import torch

import paper_2408_05444_amd as mek

ROWS_PER_WG = 8   # the smallest useful share of R's rows per work-group


def table_path() -> str:
    p = os.environ.get("MEK_AUTOTUNE_TABLE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "mek", "autotune.json")


def shape_key(m: int, p: int, q: int, n: int, precision: str) -> str:
    return f"{precision}:{m}x{p}x{q}x{n}"


def ladder(m: int, cus: int) -> List[int]:
    """Team sizes tried for an instance with m rows: powers of two up to
    about ROWS_PER_WG rows per work-group, plus that end point."""
    top = max(1, min(cus, -(-m // ROWS_PER_WG)))
    out, w = [], 1
    while w < top:
        out.append(w)
        w *= 2
    out.append(top)
    return out


class Table:
    """Persisted measurements: key -> {team size: microseconds per update}."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or table_path()
        self.data: Dict[str, Dict[str, float]] = {}
        try:
            with open(self.path) as f:
                self.data = json.load(f)
        except (OSError, ValueError):
            self.data = {}

    def get(self, key: str) -> Optional[Dict[int, float]]:
        d = self.data.get(key)
        return None if d is None else {int(w): float(t) for w, t in d.items()}

    def put(self, key: str, times: Dict[int, float]):
        self.data[key] = {str(w): float(t) for w, t in times.items()}

    def save(self):
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=0, sort_keys=True)
        os.replace(tmp, self.path)


def measure(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, precision: str,
            sizes: Sequence[int], updates: int = 300, seed: int = 1) -> Dict[int, float]:
    """Kernel microseconds per update of a solve of A X B = C at each team
    size (residual in device memory, as in a ragged launch)."""
    out = {}
    for w in sizes:
        plan = mek.mek_plan_create(A, B, precision=precision, team_wgs=int(w), r_in_lds=0)
        try:
            mek.mek_solve(plan, C, variant="grbk", max_iters=32, seed=seed)   # warm
            r = mek.mek_solve(plan, C, variant="grbk", max_iters=updates, seed=seed,
                              refresh_period=-1)
            out[int(r.team_wgs)] = min(out.get(int(r.team_wgs), float("inf")),
                                       r.kernel_ms * 1e3 / max(r.iters, 1))
        finally:
            mek.mek_plan_destroy(plan)
    return out


def tune(instances: Sequence[tuple], precision: str, table: Optional[Table] = None,
         cus: Optional[int] = None, updates: int = 300) -> List[Dict[int, float]]:
    """instances: (A, B, C) device tensors. Returns each instance's measured
    {team size: us per update}, measuring only shapes the table lacks."""
    table = table or Table()
    cus = cus or torch.cuda.get_device_properties(0).multi_processor_count
    res = []
    for A, B, C in instances:
        m, p = A.shape
        q, n = B.shape
        key = shape_key(m, p, q, n, precision)
        t = table.get(key)
        if t is None:
            t = measure(A, B, C, precision, ladder(m, cus), updates)
            table.put(key, t)
        res.append(t)
    table.save()
    return res


def allocate(times: Sequence[Dict[int, float]], updates: Sequence[float], cus: int) -> List[int]:
    """Team sizes minimising the largest predicted time updates_b x t_b(W_b)
    with sum W_b <= cus (greedy on the slowest instance)."""
    nb = len(times)
    if nb > cus:
        raise ValueError("more instances than compute units")
    ladders = [sorted(t) for t in times]
    pos = [0] * nb
    used = sum(l[0] for l in ladders)
    pred = [updates[b] * times[b][ladders[b][0]] for b in range(nb)]
    while True:
        # Only the slowest instance bounds the batch: stop when it cannot
        # get faster (no larger team measured faster, or no work-groups left).
        b = max(range(nb), key=lambda x: pred[x])
        if pos[b] + 1 >= len(ladders[b]):
            break
        w0, w1 = ladders[b][pos[b]], ladders[b][pos[b] + 1]
        if used + (w1 - w0) > cus or times[b][w1] >= times[b][w0]:
            break
        pos[b] += 1
        used += w1 - w0
        pred[b] = updates[b] * times[b][w1]
    return [ladders[b][pos[b]] for b in range(nb)]


def plans_for(instances: Sequence[tuple], precision: str, teams: Sequence[int]):
    """Plans for a ragged launch with the given team sizes (residual in
    device memory)."""
    return [mek.mek_plan_create(A, B, precision=precision, team_wgs=int(w), r_in_lds=0)
            for (A, B, _), w in zip(instances, teams)]
