"""Autotuner for the persistent batched launch.

For a given set of device shapes and precision it times every candidate tile and
schedule (waves per workgroup x persistent grid size x work-queue order) with HIP
events on the launch stream and keeps the fastest.  Results are cached in a JSON
table keyed by a signature of the workload (block-size histogram, total layers per
block size, precision); ``BatchedPlan(schedule="auto")`` reads the table when it
creates the plan.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Sequence, Tuple

from . import binding

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_table.json")
SCHEDULES = ("longest_first", "interleaved", "input_order")


def signature(shapes: Sequence[Tuple[int, int, int]], precision: str) -> str:
    hist: Dict[int, List[int]] = {}
    for (l, b, ne) in shapes:
        h = hist.setdefault(int(b), [0, 0])
        h[0] += int(ne)
        h[1] += int(l) * int(ne)
    parts = [f"b{b}:n{n}:L{L}" for b, (n, L) in sorted(hist.items())]
    return precision + "|" + ",".join(parts)


def load_table() -> dict:
    try:
        with open(TABLE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(shapes, precision):
    return load_table().get(signature(shapes, precision))


def tune(systems, eta_d: float, precision: str = "fp64", grids=None, reps: int = 2,
         save: bool = True, log=None, waves=(8, 4)) -> dict:
    """Time every candidate on the given GPU inputs; return
    {"schedule", "grid", "waves", "ms", "candidates": {name: ms}} and cache it."""
    import torch
    dev = systems[0][0].device
    shapes = [(H.shape[1], H.shape[2], E.shape[0]) for (H, _, _, E) in systems]
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    n_inst = sum(ne for (_, _, ne) in shapes)
    stream = torch.cuda.current_stream(dev)
    times = {}
    outs = None
    cands = []
    for nw in waves:
        gl = grids or ([cus, (3 * cus) // 4] if nw == 8 else [2 * cus, cus])
        cands += [(sched, min(g, n_inst), nw) for sched in SCHEDULES for g in gl]
    for (sched, g, nw) in cands:
        plan = binding.BatchedPlan(shapes, precision=precision, schedule=sched, grid=g, waves=nw)
        if outs is None:
            outs = binding.solve_batched(systems, eta_d, plan=plan)   # allocates outputs once
        entries = [dict(H=H, sigma_L=sL, sigma_R=sR, energies=E, G_diag=o[0], T=o[1], info=o[2])
                   for (H, sL, sR, E), o in zip(systems, outs)]
        table = binding.device_table(entries, dev)
        ws = torch.empty((plan.workspace_bytes,), dtype=torch.uint8, device=dev)
        binding.rgf_batched_solve(plan, table, eta_d, ws, stream.cuda_stream)   # warm-up
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            binding.rgf_batched_solve(plan, table, eta_d, ws, stream.cuda_stream)
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        times[f"{sched}/grid{g}/waves{nw}"] = min(ms)
        if log:
            log(f"autotune {sched} grid {g} waves {nw}: {min(ms):.2f} ms")
        del ws, plan
        torch.cuda.empty_cache()
    best = min(times, key=times.get)
    sched, g, nw = best.split("/")
    res = {"schedule": sched, "grid": int(g[4:]), "waves": int(nw[5:]), "ms": times[best], "candidates": times}
    if save:
        tab = load_table()
        tab[signature(shapes, precision)] = res
        try:
            with open(TABLE, "w") as f:
                json.dump(tab, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return res
