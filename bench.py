#!/usr/bin/env python
"""Benchmark of the sparse-grid WENO5 hot path on one MI355X.

One step = the whole method over one batch of synthetic solves of the 2D
Burgers workload (u_t + (u^2/2)_x + (u^2/2)_y = 0 on [-1,1]^2, u0 = 0.3 + A
sin(pi(x+y) + phi) with seeded A, phi; root grid 8x8, finest level 5 (256x256),
CFL 0.5, T = 1.5/pi^2): restriction, the shared-dt TVD-RK3 march of all 11
component grids of every solve (batched: one graph per time step, one
persistent stage launch over all boxes), WENO5 prolongation + FP64 combination,
and the L1/Linf norms against the exact solution.  Sweeps run in FP32, the
combination and norms in FP64.

Prints one JSON line.  Extra keys: the plain per-grid FP64 method on the same
workload (equal-L1 comparison), the event-timed stage kernel against its
roofline, the FP64 oracle timed on the host, serving latencies, the same solves
on one full grid, and the same batched path with FP64 sweeps.

--path-workload c3|c4 instead times one 3D advection or 4D Vlasov solve through
the path (stage launches of a step, march, prolongation) and prints its own line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import sgw_inputs as W  # noqa: E402

METRIC = "sparse-grid WENO5 cell-updates/s vs plain at equal L1 err; p50/p99 solve latency"
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
T_FINAL = 1.5 / math.pi ** 2


def flops_per_node_stage(d: int, stage: int) -> int:
    """Algorithmic flops of one RK stage at one node (counted from the paper's formulas):
    per direction two WENO5 reconstructions of 70 flops each (3 candidates x 5, 3 smoothness
    indicators x 12, 3 weights x 3, normalisation 5, combination 5), 6 for the flux and its
    LF split, 3 for the difference of eq. (2.9); plus the RK combination (2, 5, 5)."""
    return d * (2 * 70 + 6 + 3) + (2, 5, 5)[stage]


def make_problems(n, seed=2007_10196):
    """The 2D Burgers workload u0 = 0.3 + 0.7 sin(pi(x+y) + phi_i), phi_i seeded per solve."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed + 1 + i)
        phi = float(rng.uniform(0.0, 2.0 * math.pi))
        out.append(W.c2_burgers_2d(T=T_FINAL, precision=W.PREC_FP32).replace(ic_params=(0.3, 0.7, math.pi, phi)))
    return out


def step_estimate(pb):
    """Steps of the shared-dt loop if the wave speed stayed at its initial bound |c| + |A|."""
    A = abs(pb.ic_params[0]) + abs(pb.ic_params[1])
    denom = sum(A / ((pb.hi[k] - pb.lo[k]) / pb.n_fine) for k in range(pb.d))
    return int(math.ceil(pb.T / (pb.cfl / denom)))


class StepNorms:
    """The norms of every solve of one step travel to pinned host memory behind the step's
    kernels; the host reads them once the next step is queued (or at the end)."""

    def __init__(self, torch, res):
        self.host = torch.empty(tuple(res.shape), dtype=res.dtype, pin_memory=True)
        self.event = None

    def send(self, torch, res, stream):
        with torch.cuda.stream(stream):
            self.host.copy_(res, non_blocking=True)
        self.event = torch.cuda.Event()
        self.event.record(stream)

    def take(self):
        """The norms sent last (waits for them), or None."""
        if self.event is None:
            return None
        self.event.synchronize()
        self.event = None
        return self.host.numpy().copy()


def run_batch_step(torch, batch, solvers, outs, exacts, res, sent):
    """One step of the whole path for every solve.  solvers, outs and exacts are PtrLists:
    marshalled once, so the host builds no pointer arrays between launches.  Returns the
    norms of the previous step (None for the first): they are read only after this step's
    march is queued, so the device never waits for the host between steps."""
    from paper_2007_10196_amd.solver import norms_many, prolongate_combine_many, restrict_many
    # Alg. Step 1 for every solve in one launch
    restrict_many(solvers, stream=batch.stream)
    batch.admit_many(solvers)
    done = set()
    # the wave speed only decays before the shock, so the estimate is an upper bound
    # up to WENO overshoot: march most of it blind, then look every two steps
    batch.step(max(1, step_estimate(solvers[0].problem) - 4))
    prev = sent.take()
    # the flags of each poll travel while the next two steps run (a step of solves
    # that are done does no work)
    batch.poll_begin()
    while True:
        batch.step(2)
        done |= set(batch.poll_end())
        if len(done) == len(solvers):
            break
        batch.poll_begin()
    batch.release_many(list(batch.slots))
    # Alg. Step 3 for every solve in one launch, then the norms of every solve in one launch
    prolongate_combine_many(solvers, outs, stream=batch.stream)
    norms_many(solvers, outs, exacts, res, stream=batch.stream)
    sent.send(torch, res, batch.stream)
    return prev


STAGE_SRC = os.path.join(ROOT, "paper_2007_10196_amd", "csrc", "kernels_stage.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_c2_batch256_traffic.json")


def stage_source_hash():
    import hashlib
    with open(STAGE_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per stage launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE runs,
    or None when the stage kernel source changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != stage_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def copy_calibration():
    """A plain 1 GiB device-to-device copy, three times: the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_copy": x.numel() * 4, "copies": 3}), flush=True)


SERVING_N = 512


def serving_run(box_target, n=None, loads=(0.7,), blocks_per_cu=0):
    """Seeded Poisson stream mixing the 2D advection, 2D Burgers, 3D advection and 4D Vlasov
    workloads at finest levels 2..5 (4D capped at 4), FP32 sweeps.  The mix is first served
    closed-loop (every request queued at t = 0) to measure its saturation throughput; the
    arrival rate of each open-loop run is then `load` x that throughput."""
    import dataclasses
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.serving import ServingLoop, latency_summary
    n = n or SERVING_N
    probe = W.serving_stream(n=n, rate_hz=1.0, max_level_by_family={4: 4})

    def serve(reqs):
        loop = ServingLoop(precision=B.FP32_SWEEP, max_active=64, hbm_budget=96 << 30, steps_per_tick=8,
                           box_target=box_target, blocks_per_cu=blocks_per_cu)
        t0 = time.perf_counter()
        res = loop.run(reqs)
        wall = time.perf_counter() - t0
        loop.close()
        return res, wall

    res, wall = serve([dataclasses.replace(r, arrival_s=0.0) for r in probe])
    cap_hz = n / wall
    closed = latency_summary(res)
    print(f"[bench] serving {n} requests closed-loop: {cap_hz:.1f} requests/s, "
          f"{closed['throughput_cell_updates_per_s']:.3e} cell-updates/s", file=sys.stderr, flush=True)
    runs = []
    for load in loads:
        reqs = W.serving_stream(n=n, rate_hz=load * cap_hz, max_level_by_family={4: 4})
        res, wall = serve(reqs)
        out = latency_summary(res)
        out.update({"arrival_rate_hz": load * cap_hz, "offered_load_of_capacity": load, "wall_s": wall})
        runs.append(out)
        print(f"[bench] serving {n} requests at {load:.1f} of capacity: p50 {out['p50_ms']:.1f} ms "
              f"p99 {out['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    main = dict(runs[0])
    main.update({"capacity_requests_per_s": cap_hz,
                 "capacity_cell_updates_per_s": closed["throughput_cell_updates_per_s"],
                 "other_loads": runs[1:],
                 "mix": "families 2D advection / 2D Burgers / 3D advection / 4D Vlasov, levels 2-5 (4D <= 4), "
                        "seeded phases and amplitudes, FP32 sweeps + FP64 combination; capacity measured "
                        "closed-loop on the same mix"})
    return main


def full_grid_run(torch, probs, box_target, bpc, steps=2):
    """The paper's comparison (Sec. 3 tables): the same solves on one full grid of the finest
    resolution (root 256, finest level 0), batched the same way; time per step of all solves and
    the L1 error against the exact solution."""
    return batch_run(torch, [p.replace(nr=p.n_fine, nl=0) for p in probs], box_target, bpc, steps)


def batch_run(torch, probs, box_target, bpc, steps=2):
    """The batched step of run_batch_step over `probs` (one precision), after one untimed step:
    time per step of all solves and the mean L1 error against the exact solution."""
    from paper_2007_10196_amd.solver import Batch, PtrList, Solver
    solvers = [Solver(p, device="cuda:0", box_target=box_target) for p in probs]
    fine = solvers[0].plan.fine_nodes
    outs = [torch.empty(fine, dtype=torch.float64, device="cuda:0") for _ in solvers]
    exacts = [s.exact(T_FINAL) for s in solvers]
    res = torch.zeros((len(solvers), 2), dtype=torch.float64, device="cuda:0")
    solvers, outs, exacts = PtrList(solvers), PtrList(outs), PtrList(exacts)
    sent = StepNorms(torch, res)
    batch = Batch(max_solvers=len(solvers), precision=probs[0].precision,
                  hbm_budget=sum(s.plan.footprint for s in solvers) + (1 << 30),
                  max_items=sum(s.plan.total_nodes // 32 + 64 for s in solvers))
    batch.set_blocks_per_cu(bpc)
    run_batch_step(torch, batch, solvers, outs, exacts, res, sent)
    sent.take()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run_batch_step(torch, batch, solvers, outs, exacts, res, sent)
    norms = sent.take()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    batch.close()
    return {"ms_per_step": ms, "l1_mean": float(norms[:, 0].mean()), "nodes_per_solve": solvers[0].plan.total_nodes,
            "time_steps": solvers[0].query()[1],
            "cell_updates_per_step": sum(s.query()[1] * s.plan.total_nodes for s in solvers)}


def step_estimate_any(pb):
    """Steps of the shared-dt loop for any workload family (wave-speed bound at t = 0)."""
    if pb.flux == W.FLUX_BURGERS:
        return step_estimate(pb)
    if pb.flux == W.FLUX_ADVECTION:
        A = [abs(a) for a in pb.flux_params[:pb.d]]
    else:
        m = pb.d // 2
        A = [max(abs(pb.lo[m + k]), abs(pb.hi[m + k])) for k in range(m)] + [abs(pb.flux_params[0])] * m
    denom = sum(A[k] / ((pb.hi[k] - pb.lo[k]) / pb.n_fine) for k in range(pb.d))
    return int(math.ceil(pb.T / (pb.cfl / denom)))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s=15.0, single_budget_s=5.0):
    """The oracle on the host: all OpenMP threads for about budget_s, then one thread (the paper's
    setting) for about single_budget_s, on the same solves."""
    import oracle as O
    probs = make_problems(512)

    def run(budget, nthreads):
        t0 = time.perf_counter()
        cells = n = 0
        for p in probs:
            pb = p.replace(precision=W.PREC_FP64)
            _, _, stats = O.solve(pb, nthreads=nthreads)
            cells += stats["steps"] * O.total_nodes(pb)
            n += 1
            if time.perf_counter() - t0 > budget:
                break
        return cells / (time.perf_counter() - t0), n, time.perf_counter() - t0

    cores = O.max_threads()
    v, n, dt = run(budget_s, 0)
    v1, n1, dt1 = run(single_budget_s, 1)
    return {"value": v, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} solves of the same 2D Burgers workload (FP64, full method incl. prolongation), "
                      f"{dt:.1f} s wall, OpenMP over component grids",
            "single_thread_value": v1, "single_thread_sample": f"{n1} solves in {dt1:.1f} s on one thread",
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def path_workload(name, precision, box_target, bpc, reps):
    """One solve of the 3D advection workload (root 8, finest level 5, 46 grids) or the 4D Vlasov
    workload (root 8, finest level 4, 69 grids) through the whole path on one GPU, each part
    timed with HIP events: the stage launches of one time step in the batch's launch shape
    (`reps` repetitions), the march to T as a solver runs it (step graphs), and the WENO5
    prolongation with the signed combination.  Prints one JSON line."""
    import torch
    from paper_2007_10196_amd.solver import Batch, Solver
    torch.cuda.set_device(0)
    make = {"c3": W.c3_advection_3d, "c4": W.c4_vlasov_4d}[name]
    prec = W.PREC_FP64 if precision == "fp64" else W.PREC_FP32
    pb = make(precision=prec)
    if not box_target:
        # the launch shape the autotuner picks for this solve (cached in JSON)
        from paper_2007_10196_amd.autotune import tune_box_target
        tune = tune_box_target([pb], prec, reps=5)
        box_target, bpc = int(tune["best"]), int(tune.get("blocks_per_cu", 0))

    def ev():
        return torch.cuda.Event(enable_timing=True)

    s = Solver(pb, device="cuda:0", box_target=box_target, blocks_per_cu=bpc)
    batch = Batch(max_solvers=1, precision=prec, hbm_budget=1 << 40, max_items=1 << 20)
    if bpc:
        batch.set_blocks_per_cu(bpc)
    s.restrict()
    slot = batch.admit(s)
    batch.step(1)
    st = batch.stream
    e0, e1 = ev(), ev()
    batch.launch_stage(3, 2)
    e0.record(st)
    batch.launch_stage(3, reps)
    e1.record(st)
    torch.cuda.synchronize()
    stage_us = e0.elapsed_time(e1) / reps * 1e3
    info = batch.info()
    batch.release(slot)
    batch.close()
    # the march and the prolongation as one solver runs them; the second of two runs is timed
    # (the first loads the kernels' code)
    s = Solver(pb, device="cuda:0", box_target=box_target, blocks_per_cu=bpc)
    out = torch.empty(s.plan.fine_nodes, dtype=torch.float64, device="cuda:0")
    for _ in range(2):
        s.restrict()
        torch.cuda.synchronize()
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        e0.record(s.stream)
        s.advance()
        e1.record(s.stream)
        t, steps = s.query()
        e2.record(s.stream)
        s.prolongate_combine(out)
        e3.record(s.stream)
        torch.cuda.synchronize()
    march_ms = e0.elapsed_time(e1)
    print(json.dumps({
        "workload": f"{pb.name}: d={pb.d}, root {pb.nr}, finest level {pb.nl}, {len(s.plan.grids)} component grids, "
                    f"{s.plan.total_nodes} nodes, finest grid {s.plan.fine_nodes} nodes, T={pb.T}",
        "precision": precision, "boxes": info["boxes"], "box_target": box_target, "blocks_per_cu": bpc,
        "stage_launches_per_step_us": stage_us, "steps": steps, "t": t, "march_ms": march_ms,
        "march_ms_per_step": march_ms / max(steps, 1),
        "march_cell_updates_per_s": steps * s.plan.total_nodes / (march_ms * 1e-3),
        "prolong_combine_ms": e2.elapsed_time(e3)}), flush=True)


def valu_calibration():
    """Cycles one SIMD spends per wave64 instruction of each class (FP32 FMA, multiply, add;
    INT32 add/xor; FP64 FMA), from event-timed launches of the library's calibration kernels
    over 16 workgroups per compute unit, at the 2.4 GHz peak clock."""
    import ctypes as C
    import torch
    from paper_2007_10196_amd import binding as B
    torch.cuda.set_device(0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = 16 * cus
    out = torch.empty(blocks * 256 * 8, dtype=torch.uint8, device="cuda:0")
    st = torch.cuda.current_stream()
    res = {}
    for op, name in enumerate(("fp32_fma", "fp32_mul", "fp32_add", "int32_add_xor", "fp64_fma")):
        n = C.c_double()
        for rep in range(3):  # the last of three launches is kept
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            B.check(B.lib().sgw_calibrate_valu(op, blocks, C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream),
                                               C.byref(n)))
            e1.record(st)
            torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) * 1e-3 * 2.4e9 / n.value
    print(json.dumps({"valu_cycles_per_wave64_instruction": res, "clock_GHz": 2.4, "compute_units": cus}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--solves", type=int, default=256, help="solves per step (batch size)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--stage-reps", type=int, default=20)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-full", action="store_true", help="skip the single full-grid comparison")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 batched run of the same solves")
    ap.add_argument("--box-target", type=int, default=0,
                    help="0: autotune the stage box target and the workgroups per compute unit")
    ap.add_argument("--blocks-per-cu", type=int, default=0, help="with --box-target: stage workgroups per CU")
    ap.add_argument("--serving-requests", type=int, default=SERVING_N)
    ap.add_argument("--serving-loads", default="0.7,0.5,0.9",
                    help="comma-separated offered loads (the first one is the reported latency)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB copy used to scale the HBM byte counters")
    ap.add_argument("--valu-calibration", action="store_true",
                    help="only time the VALU issue-rate calibration kernels")
    ap.add_argument("--path-workload", choices=("c3", "c4"),
                    help="only run one 3D (c3) or 4D (c4) solve through the path, each part timed")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32", help="with --path-workload")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.valu_calibration:
        valu_calibration()
        return
    if args.path_workload:
        path_workload(args.path_workload, args.precision, args.box_target, args.blocks_per_cu, args.stage_reps)
        return

    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.solver import Batch, PtrList, Solver

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    probs = make_problems(args.solves)
    # box shape for this batch (untimed): fastest of the candidate targets, cached in JSON
    from paper_2007_10196_amd.autotune import tune_box_target
    if args.box_target:
        tune = {"best": args.box_target, "blocks_per_cu": args.blocks_per_cu, "us": None, "cached": True}
    else:
        tune = tune_box_target(probs, B.FP32_SWEEP, reps=5)
    box_target = int(tune["best"])
    bpc = int(tune.get("blocks_per_cu", 0))
    print(f"[bench] launch shape: box target {box_target}, {bpc or 'max'} workgroups per CU "
          f"({'cached' if tune['cached'] else 'measured'})",
          file=sys.stderr, flush=True)
    solvers = [Solver(p, device="cuda:0", box_target=box_target) for p in probs]
    nodes = solvers[0].plan.total_nodes
    fine = solvers[0].plan.fine_nodes
    outs = [torch.empty(fine, dtype=torch.float64, device=dev) for _ in solvers]
    exacts = [s.exact(T_FINAL) for s in solvers]
    res = torch.zeros((len(solvers), 2), dtype=torch.float64, device=dev)
    solvers, outs, exacts = PtrList(solvers), PtrList(outs), PtrList(exacts)
    sent = StepNorms(torch, res)
    budget = sum(s.plan.footprint for s in solvers) + (1 << 30)
    batch = Batch(max_solvers=len(solvers), precision=B.FP32_SWEEP, hbm_budget=budget,
                  max_items=sum(len(s.plan.grids) * 64 for s in solvers))
    batch.set_blocks_per_cu(bpc)
    print(f"[bench] {len(solvers)} solves x {nodes} component nodes, warmup {args.warmup}", file=sys.stderr,
          flush=True)

    for _ in range(args.warmup):
        run_batch_step(torch, batch, solvers, outs, exacts, res, sent)
    sent.take()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norms = None
    for k in range(args.steps):
        run_batch_step(torch, batch, solvers, outs, exacts, res, sent)
    norms = sent.take()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps_each = [s.query()[1] for s in solvers]
    cells_per_step = sum(n * nodes for n in steps_each)
    ms_per_step = elapsed / args.steps * 1e3
    value = cells_per_step / (elapsed / args.steps)
    # the paper's savings view: finest-grid nodes advanced per second
    finest_equiv = sum(n * solvers[0].plan.fine_nodes for n in steps_each) / (elapsed / args.steps)
    l1s = norms[:, 0]
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.3e} cell-updates/s",
          file=sys.stderr, flush=True)

    # ---- the dominant kernel alone, same launch shape, HIP events on the batch stream.  Every
    # component grid of this workload is one stage box, so the stage work of a step is one
    # launch of the three-stage kernel; the split kernel's stage 1 is timed beside it.
    from paper_2007_10196_amd.solver import restrict_many
    restrict_many(solvers, stream=batch.stream)
    batch.admit_many(solvers)
    batch.step(1)
    st = batch.stream

    def timed(stage, reps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        batch.launch_stage(stage, 2)
        ev0.record(st)
        batch.launch_stage(stage, reps)
        ev1.record(st)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    step_ms = timed(3, args.stage_reps)
    split_ms = timed(0, args.stage_reps)
    info = batch.info()
    batch.release_many(list(batch.slots))
    step_flops = info["nodes"] * sum(flops_per_node_stage(2, s) for s in range(3))
    achieved = step_flops / (step_ms * 1e-3) / 1e12
    # algorithmic bytes of a step: u^n read once, u^{n+1} written once (FP32)
    step_bytes = info["nodes"] * 4 * 2
    traffic = measured_traffic()
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                # the HBM side of the same launch: counter bytes (when current) over the event time
                "hbm_GBs": traffic / (step_ms * 1e-3) / 1e9 if traffic else None,
                "hbm_frac": traffic / (step_ms * 1e-3) / 1e9 / PEAK_HBM_GBS if traffic else None,
                "kernel": "stage_kernel<float, 2, fused> (three RK stages of every one-box grid)",
                "avg_launch_us": step_ms * 1e3,
                "flops_per_launch": step_flops, "boxes_per_launch": info["boxes"],
                "algorithmic_bytes_per_launch": step_bytes,
                "achieved_algorithmic_GBs": step_bytes / (step_ms * 1e-3) / 1e9,
                "split_stage_kernel_stage1_us": split_ms * 1e3}

    # ---- plain per-grid FP64 method on the first solve: the equal-L1 reference
    plain = None
    if not args.no_plain:
        p64 = probs[0].replace(precision=W.PREC_FP64)
        sp = Solver(p64, device="cuda:0")
        Up = torch.empty(fine, dtype=torch.float64, device=dev)
        Ep = sp.exact(T_FINAL)
        for rep in range(2):
            torch.cuda.synchronize()
            tp = time.perf_counter()
            sp.restrict()
            sp.advance(mode=B.RUN_PLAIN)
            sp.prolongate_combine(Up)
            l1p, lip = sp.norms(Up, Ep)
            torch.cuda.synchronize()
            tp = time.perf_counter() - tp
        stp = sp.query()[1]
        plain = {"value": stp * nodes / tp, "unit": "cell-updates/s", "mode": "plain: one launch per grid per "
                 "RK stage, no graph, FP64", "ms_per_solve": tp * 1e3, "l1": l1p, "linf": lip,
                 "speedup_of_value": value / (stp * nodes / tp),
                 "equal_l1": bool(abs(l1s[0] - l1p) <= 0.01 * l1p), "l1_batched_fp32_same_solve": float(l1s[0])}

    full = None
    if not args.no_full:
        f = full_grid_run(torch, probs, box_target, bpc)
        full = {"full_grid": "one 256x256 grid (root 256, finest level 0), same solves, same batched FP32 path",
                "full_ms_per_step": f["ms_per_step"], "sparse_ms_per_step": ms_per_step,
                "time_ratio_sparse_over_full": ms_per_step / f["ms_per_step"],
                "l1_full": f["l1_mean"], "l1_sparse": float(l1s.mean()),
                "nodes_full": f["nodes_per_solve"], "nodes_sparse": nodes, "time_steps_full": f["time_steps"],
                "paper_cpu_time_ratio": "2D WENO sparse/single 0.72-0.68 (Table ex3aweno: 0.414/0.572 s at "
                                        "N_h = 80 to 781.990/1149.946 s at 640), 2.3 GHz workstation"}
        print(f"[bench] full grid: {f['ms_per_step']:.2f} ms/step, L1 {f['l1_mean']:.3e} "
              f"(sparse {ms_per_step:.2f} ms/step, L1 {float(l1s.mean()):.3e})", file=sys.stderr, flush=True)

    batched_fp64 = None
    if not args.no_fp64:
        f = batch_run(torch, [p.replace(precision=W.PREC_FP64) for p in probs], box_target, bpc, steps=args.steps)
        v64 = f["cell_updates_per_step"] / (f["ms_per_step"] * 1e-3)
        batched_fp64 = {"value": v64, "unit": "cell-updates/s", "ms_per_step": f["ms_per_step"],
                        "mode": "the same 256 solves and batched path with FP64 sweeps (launch shape of the FP32 run)",
                        "l1_mean": f["l1_mean"], "fp32_speedup": value / v64}
        print(f"[bench] FP64 batched: {f['ms_per_step']:.2f} ms/step, {v64:.3e} cell-updates/s, L1 {f['l1_mean']:.3e}",
              file=sys.stderr, flush=True)

    serving = None if args.no_serving else serving_run(
        box_target, n=args.serving_requests, loads=[float(x) for x in args.serving_loads.split(",")],
        blocks_per_cu=bpc)

    cpu = None if args.no_cpu else cpu_baseline()

    out = {"metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "2D Burgers u0=0.3+A sin(pi(x+y)+phi), [-1,1]^2 periodic, root 8x8, finest "
                                  "level 5 (256x256), 11 component grids, CFL 0.5, T=1.5/pi^2; FP32 sweeps, FP64 "
                                  "combination", "solves_per_step": len(solvers), "component_nodes": nodes,
                      "mode": "batched: one HIP graph per time step, persistent fused WENO5+RK3 stage launch"},
           "l1_mean": float(l1s.mean()), "l1_max": float(l1s.max()),
           "finest_equivalent_cell_updates_per_s": finest_equiv,
           "roofline": roofline, "cpu_baseline": cpu, "plain": plain, "latency": serving, "sparse_vs_full": full,
           "batched_fp64": batched_fp64,
           "autotune": {"box_target": box_target, "blocks_per_cu": bpc, "step_stage_us_by_target_and_cap": tune["us"]}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
