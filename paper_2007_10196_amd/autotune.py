"""Launch-shape tuner for the stage kernel.

For a set of problems (one batch), every candidate box target (the largest box,
in nodes, the planner's box search may pick for each component grid) is tried
with every candidate cap on resident workgroups per compute unit: the batch is
restricted and admitted, one step is taken, and the stage launches of a few steps
(the three-stage launch of the grids that are one box, the per-stage launches of
the others) are timed with HIP events on the batch stream.  The fastest pair is returned and
cached in a JSON file keyed by the batch's grid shapes and precision.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, Optional, Sequence

import torch

from .solver import Batch, Plan, Solver

CANDIDATES = (512, 1024, 2048)
STEP_STAGES = 3                     # sgw_batch_launch_stage: the stage launches of one step
BLOCKS_PER_CU = (0, 4, 5, 6, 7)     # 0: as many as fit


def default_cache_path() -> str:
    return os.environ.get("SGW_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "sgweno", "tune.json"))


def workload_key(problems: Sequence, precision: int) -> str:
    shapes = sorted({(p.d, p.nr, p.nl, p.flux) for p in problems})
    raw = json.dumps({"shapes": shapes, "n": len(problems), "precision": precision, "tuner": 3})
    return hashlib.sha256(raw.encode()).hexdigest()[:16]


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_stage(problems: Sequence, precision: int, box_target: int, reps: int = 10,
               blocks_per_cu: Iterable[int] = (0,)) -> Dict[int, float]:
    """Average microseconds of the stage launches of one step (all three RK stages) over the
    whole batch, per workgroup cap."""
    stream = torch.cuda.current_stream()
    solvers = [Solver(p, box_target=box_target) for p in problems]
    batch = Batch(max_solvers=len(solvers), precision=precision, hbm_budget=1 << 50,
                  max_items=sum(s.plan.total_nodes // 64 + len(s.plan.grids) for s in solvers) + 16)
    for s in solvers:
        s.restrict()
        batch.admit(s)
    batch.step(1)
    out = {}
    for bpc in blocks_per_cu:
        batch.set_blocks_per_cu(int(bpc))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        batch.launch_stage(STEP_STAGES, 2)
        e0.record(stream)
        batch.launch_stage(STEP_STAGES, reps)
        e1.record(stream)
        torch.cuda.synchronize()
        out[int(bpc)] = e0.elapsed_time(e1) / reps * 1e3
    for slot in list(batch.slots):
        batch.release(slot)
    batch.close()
    for s in solvers:
        s.close()
    return out


def tune_box_target(problems: Sequence, precision: int, candidates: Iterable[int] = CANDIDATES,
                    cache_path: Optional[str] = None, reps: int = 10, force: bool = False,
                    blocks_per_cu: Iterable[int] = BLOCKS_PER_CU) -> Dict:
    """Pick the fastest (box target, workgroups per CU) for this batch; returns
    {"best": target, "blocks_per_cu": cap, "us": {"target/cap": us}, "cached": bool}.  Problems
    whose grids all march as line sweeps (3D and 4D by default) have no stage boxes to shape:
    then nothing is measured and {"best": 0, "blocks_per_cu": 0, "us": {}, "line_sweeps": True}
    comes back (the library's defaults)."""
    if all(not any(info["box"]) for p in problems for info in Plan(p).grids):
        return {"best": 0, "blocks_per_cu": 0, "us": {}, "cached": False, "line_sweeps": True}
    path = cache_path or default_cache_path()
    key = workload_key(problems, precision)
    cache = _load(path)
    if not force and key in cache:
        rec = dict(cache[key])
        rec["cached"] = True
        return rec
    times = {}
    for t in candidates:
        try:
            for bpc, us in time_stage(problems, precision, int(t), reps, blocks_per_cu).items():
                times[f"{int(t)}/{bpc}"] = us
        except Exception as e:  # a target no box satisfies for some grid
            times[f"{int(t)}/0"] = float("inf")
            print(f"[autotune] target {t}: {e}", flush=True)
    best = min(times, key=times.get)
    t_best, b_best = (int(x) for x in best.split("/"))
    rec = {"best": t_best, "blocks_per_cu": b_best, "us": times}
    cache[key] = rec
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    with open(path + ".tmp", "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(path + ".tmp", path)
    out = dict(rec)
    out["cached"] = False
    return out
