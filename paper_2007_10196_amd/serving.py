"""Continuous-batching serving loop over the batch runtime (sgw_batch_*).

Requests arrive over time (each with a problem and an arrival time on the host
monotonic clock).  The loop admits queued requests while a batch slot is free
and the request's device footprint (state + scratch + finest-grid output) fits
the HBM budget, so a request that arrives while others are on the GPU joins the
next time step of the running batch.  Admission goes in arrival order and
backfills: a request that does not fit what is left of the budget is passed
over by later ones that do, until it has waited ``max_bypass_s``; from then on
nothing behind it is admitted before it (no starvation of large requests).  Each tick
advances every admitted solve by a few time steps (graph launches on the batch
stream) and reads the completion flags gathered after the previous tick, whose
copy overlapped this tick's steps.  A finished solve leaves the batch and is prolongated and
combined on a second stream while the batch keeps stepping; its latency is
finish - arrival.  A combination onto a large finest grid (a 256^4 grid is about a second of the
whole GPU) goes in chunks of finest-grid tiles, one chunk in flight at a time for each of the
max_chunked such combinations with the fewest tiles left, so the batch's steps keep running
between them instead of waiting behind them.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional

import torch

from . import binding as B
from .solver import Batch, Plan, Solver


def backfill_choice(footprints: List[int], waits: List[float], used: int, budget: int, free_slots: int,
                    max_bypass_s: float) -> List[int]:
    """Positions (in arrival order) of the queued requests to admit now: every request whose
    footprint fits what is left of the budget, at most ``free_slots`` of them; a request that does
    not fit is passed over while it has waited less than ``max_bypass_s``, and stops the scan once
    it has waited that long (``max_bypass_s = 0``: strict arrival order)."""
    picks: List[int] = []
    for i, (fp, wait) in enumerate(zip(footprints, waits)):
        if len(picks) >= free_slots:
            break
        if used + fp <= budget:
            picks.append(i)
            used += fp
        elif wait >= max_bypass_s:
            break
    return picks


@dataclasses.dataclass
class _Combining:
    """A finished solve whose combination goes in chunks of finest-grid tiles."""
    req: object
    solver: Solver
    admit_s: float
    footprint: int
    out: torch.Tensor
    steps: int
    per_chunk: int                  # tiles per chunk
    next_tile: int = 0
    event: Optional[torch.cuda.Event] = None  # behind the chunk in flight

    @property
    def tiles_left(self) -> int:
        return self.solver.plan.fine_tile_count - self.next_tile


@dataclasses.dataclass
class Result:
    rid: int
    arrival_s: float
    admit_s: float
    finish_s: float
    steps: int
    cell_updates: int
    out: Optional[torch.Tensor]
    kind: str = ""                 # "<dimension>D N_L=<finest level>"

    @property
    def latency_s(self) -> float:
        return self.finish_s - self.arrival_s


class ServingLoop:
    def __init__(self, precision: int = B.FP32_SWEEP, max_active: int = 64, hbm_budget: int = 64 << 30,
                 steps_per_tick: int = 8, keep_outputs: bool = False, box_target: int = 0,
                 blocks_per_cu: int = 0, device: str = "cuda", max_bypass_s: float = 0.5,
                 chunk_fine_nodes: int = 1 << 25, max_chunked: int = 1, sweep_form: int = 0):
        self.precision = precision
        self.max_bypass_s = max_bypass_s
        # combinations onto more than 2 chunk_fine_nodes finest nodes go in chunks of about that many
        self.chunk_fine_nodes = int(chunk_fine_nodes)
        self.max_chunked = max(1, int(max_chunked))
        # the stage form of the requests' plans (sgw_config.sweep_form; 2: 3D grids as stage boxes,
        # whose one-box grids run their three RK stages in one launch; the same latency and
        # throughput as line sweeps on the 512-request mix)
        self.sweep_form = int(sweep_form)
        self.max_active = max_active
        self.budget = int(hbm_budget)
        self.steps_per_tick = steps_per_tick
        self.keep_outputs = keep_outputs
        self.box_target = box_target
        self.device = torch.device(device)
        self.main = torch.cuda.current_stream(self.device)
        self.side = torch.cuda.Stream(device=self.device)
        # solver set-up and restriction: their own stream, so an admission never waits
        # behind the prolongations queued on the side stream
        self.setup = torch.cuda.Stream(device=self.device)
        # host seconds spent per phase of the loop, for tuning
        self.stats: Dict[str, float] = collections.defaultdict(float)
        self.batch = Batch(max_solvers=max_active, precision=precision, hbm_budget=self.budget,
                           max_items=1 << 22, device=device, stream=self.main)
        if blocks_per_cu:
            self.batch.set_blocks_per_cu(blocks_per_cu)

    def run(self, requests: List, clock=time.perf_counter) -> List[Result]:
        """Serve ``requests`` (objects with rid, arrival_s, problem) against the wall clock."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        queue = collections.deque()
        active: Dict[int, tuple] = {}
        finishing: List[tuple] = []
        combining: List[_Combining] = []
        used = 0
        results: List[Result] = []
        plans: Dict[int, Plan] = {}
        t0 = clock()
        polling = False  # a poll_begin whose flags have not been read yet
        while pending or queue or active or finishing or combining:
            now = clock() - t0
            while pending and pending[0].arrival_s <= now:
                queue.append(pending.popleft())
            # admission by slot and device footprint, in arrival order with backfilling
            if queue and len(active) < self.max_active:
                tp = clock()
                for req in queue:
                    if req.rid not in plans:
                        plans[req.rid] = Plan(req.problem, box_target=self.box_target, sweep_form=self.sweep_form)
                self.stats["plan"] += clock() - tp
                for req in queue:
                    if plans[req.rid].footprint > self.budget:
                        raise MemoryError(f"request {req.rid} needs {plans[req.rid].footprint} B, "
                                          f"budget {self.budget} B")
                now = clock() - t0
                picks = backfill_choice([plans[r.rid].footprint for r in queue], [now - r.arrival_s for r in queue],
                                        used, self.budget, self.max_active - len(active), self.max_bypass_s)
                admitted = set()
                for i in picks:
                    req = queue[i]
                    plan = plans[req.rid]
                    tp = clock()
                    with torch.cuda.stream(self.setup):
                        solver = Solver(req.problem, device=str(self.device), stream=self.setup, plan=plan)
                        solver.restrict()
                    slot = self.batch.admit(solver)  # orders the restriction before the batch's next step
                    self.stats["admit"] += clock() - tp
                    used += plan.footprint
                    active[slot] = (req, solver, clock() - t0, plan.footprint)
                    admitted.add(i)
                if admitted:
                    queue = collections.deque(r for i, r in enumerate(queue) if i not in admitted)
            # solves whose combination has completed
            still = []
            for req, solver, admit_s, fp, ev, U, steps in finishing:
                if ev.query():
                    results.append(Result(rid=req.rid, arrival_s=req.arrival_s, admit_s=admit_s,
                                          finish_s=clock() - t0, steps=steps,
                                          cell_updates=steps * solver.plan.total_nodes,
                                          out=U if self.keep_outputs else None,
                                          kind=f"{req.problem.d}D N_L={req.problem.nl}"))
                    used -= fp
                    plans.pop(req.rid, None)
                    # its combination is done (event above); freeing synchronises the solver's
                    # stream, so point it at the set-up stream rather than the busy side stream
                    solver.set_stream(self.setup)
                    solver.close()
                else:
                    still.append((req, solver, admit_s, fp, ev, U, steps))
            finishing = still
            # chunked combinations, the max_chunked with the fewest tiles left (a short one is not
            # held up behind a long one): each one's next chunk once its previous one has run
            combining.sort(key=lambda job: job.tiles_left)
            still = []
            for j, job in enumerate(combining):
                if j < self.max_chunked and (job.event is None or job.event.query()):
                    n = min(job.per_chunk, job.tiles_left)
                    if not (active or queue or pending):
                        n = job.tiles_left  # nothing can wait behind it any more
                    with torch.cuda.stream(self.side):
                        job.solver.prolongate_combine_tiles(job.out, job.next_tile, n)
                        job.event = torch.cuda.Event()
                        job.event.record(self.side)
                    job.next_tile += n
                    if job.tiles_left == 0:
                        finishing.append((job.req, job.solver, job.admit_s, job.footprint, job.event, job.out,
                                          job.steps))
                        continue
                still.append(job)
            combining = still
            if not active:
                if polling:
                    # nothing left to report: a released slot is never reported
                    self.batch.poll_end()
                    polling = False
                if finishing or combining:
                    time.sleep(0.0002)
                elif pending:
                    wait = pending[0].arrival_s - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.005))
                continue
            tp = clock()
            self.batch.step(self.steps_per_tick)
            tq = clock()
            # the flags gathered after the previous tick travel while this tick's steps run
            done = self.batch.poll_end() if polling else []
            self.batch.poll_begin()
            polling = True
            tr = clock()
            self.stats["step_enqueue"] += tq - tp
            self.stats["poll_wait"] += tr - tq
            for slot in done:
                req, solver, admit_s, fp = active.pop(slot)
                self.batch.release(slot)
                t, steps = solver.query()  # cheap: the solver's stream is still the set-up stream
                # the batch stream has finished this solve's steps (poll synchronised it); the
                # set-up stream's restriction was ordered before its admission
                solver.set_stream(self.side)
                plan = solver.plan
                if plan.fine_nodes > 2 * self.chunk_fine_nodes:
                    with torch.cuda.stream(self.side):
                        U = torch.empty(plan.fine_nodes, dtype=torch.float64, device=self.device)
                    tile_nodes = plan.fine_nodes // plan.fine_tile_count
                    combining.append(_Combining(req, solver, admit_s, fp, U, steps,
                                                per_chunk=max(1, self.chunk_fine_nodes // tile_nodes)))
                    continue
                with torch.cuda.stream(self.side):
                    U = solver.prolongate_combine()
                    ev = torch.cuda.Event()
                    ev.record(self.side)
                finishing.append((req, solver, admit_s, fp, ev, U, steps))
            self.stats["finish"] += clock() - tr
            self.stats["ticks"] += 1
        if polling:
            self.batch.poll_end()
        return results

    def close(self):
        self.batch.close()


def latency_summary(results: List[Result]) -> dict:
    import numpy as np
    lat = np.array([r.latency_s for r in results]) * 1e3
    span = max(r.finish_s for r in results) - min(r.arrival_s for r in results)
    cells = sum(r.cell_updates for r in results)
    by_kind = {}
    for kind in sorted({r.kind for r in results}):
        lk = np.array([r.latency_s for r in results if r.kind == kind]) * 1e3
        by_kind[kind] = {"requests": int(lk.size), "p50_ms": float(np.percentile(lk, 50)),
                         "p99_ms": float(np.percentile(lk, 99))}
    return {"requests": len(results), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()),
            "throughput_cell_updates_per_s": cells / span if span > 0 else None, "span_s": span,
            "by_kind": by_kind}
