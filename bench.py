#!/usr/bin/env python
"""Benchmark of the sparse-grid WENO5 hot path on one MI355X.

One step = the whole method for one solve of the 4D Vlasov workload at FP64
(f_t + v.grad_x f + E(x).grad_v f = 0, x in [0,4pi]^2, v in [-6,6]^2, periodic,
E = 0.01 (sin(x1/2), sin(x2/2)), f0 = Maxwellian x (1 + 0.01 cos(x1/2) cos(x2/2));
root grid 8^4, finest level 4 (128^4 finest nodes), 69 component grids,
CFL 0.4, T = 1, 307 time steps): restriction, the shared-dt TVD-RK3 march of
every component grid (step graphs; per RK stage a plane launch for directions 1
and 2 and a line sweep for each of directions 3 and 4, each persistent over every
grid), WENO5 prolongation + FP64 combination onto the finest grid, and the
L1/Linf norms against the exact solution (computed once, before timing).

Prints one JSON line.  `value` is component-grid cell-updates per second of
that solve.  Extra keys: the same solve with FP32 sweeps, the plain per-grid
FP64 method on the same solve (equal-L1 comparison), the stage and
prolongation kernels against their rooflines (HIP events), the FP64 oracle on
the host (a bounded sample), the batched 2D Burgers workload (256 solves per
step, FP32 and FP64), the same 2D solves on one full grid, and serving latencies.

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


def flops_per_node_stage(d: int) -> int:
    """Algorithmic flops of one RK stage at one node: per direction two WENO5 reconstructions
    (about 65 flops each: 3 candidate stencils, 3 smoothness indicators, 3 nonlinear weights and
    their normalisation) plus the flux, its Lax-Friedrichs split and the flux difference of
    eq. (2.9), 140 in all; plus 5 for the Runge-Kutta combination."""
    return 140 * d + 5


def flops_per_cell_update(d: int) -> int:
    """One component node advanced one full TVD-RK3 step: three stages."""
    return 3 * flops_per_node_stage(d)


INTERP_FLOPS = 30  # per interpolated point, the smoothness indicators shared by the R points of a coarse interval


def interpolation_count(plan) -> int:
    """Interpolated points of the direction-by-direction prolongation of every component grid
    over whole arrays: the pass along direction k (k = 1..d, refined only where the grid is
    coarser than the finest grid) produces N^k x prod_{k' > k} n_k' points."""
    N = plan.problem.n_fine
    total = 0
    for g in plan.grids:
        n = list(g["shape"])
        for k in range(len(n)):
            if n[k] == N:
                continue
            n[k] = N
            pts = 1
            for x in n:
                pts *= x
            total += pts
    return total


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


CSRC = os.path.join(ROOT, "paper_2007_10196_amd", "csrc")
# HBM bytes per launch from committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs, keyed to the hash of
# the kernel's source file: (summary file under profiles/, source file)
TRAFFIC = {"stage_c2_fp32": ("stage_kernel_c2_batch256_traffic.json", "kernels_stage.hip"),
           "stage_c4_fp64": ("stage_kernel_c4_vlasov_4d_fp64_traffic.json", "kernels_stage.hip"),
           "prolong_c4_fp64": ("prolong_kernel_c4_vlasov_4d_fp64_traffic.json", "kernels_prolong.hip")}


def source_hash(name):
    import hashlib
    with open(os.path.join(CSRC, name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(key, kernel=None):
    """HBM bytes per launch of a kernel from its committed counter summary (`kernel`: one entry of a
    summary that covers several kernels), or None when the kernel's source changed since the
    counters were taken (or none were taken)."""
    fname, src = TRAFFIC[key]
    try:
        with open(os.path.join(ROOT, "profiles", fname)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != source_hash(src):
        return None
    if kernel is not None:
        return rec.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")
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
    workloads at finest levels 2..5 (4D at level 5: 121 grids and a 34.4 GB FP64 finest grid, which
    admission counts), FP32 sweeps.  The mix is first served
    closed-loop (every request queued at t = 0) to measure its saturation throughput; the
    arrival rate of each open-loop run is then `load` x that throughput."""
    import dataclasses
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.serving import ServingLoop, latency_summary
    n = n or SERVING_N
    import torch
    torch.cuda.empty_cache()  # the earlier legs' blocks go back to the device before the 34 GB outputs
    probe = W.serving_stream(n=n, rate_hz=1.0)

    def serve(reqs):
        # each run starts from an empty allocator cache: blocks cached by the previous run (the
        # 34 GB outputs among them) would otherwise meet this run's allocations, and torch's
        # free-and-retry on a full device synchronises it in the middle of the run
        torch.cuda.empty_cache()
        loop = ServingLoop(precision=B.FP32_SWEEP, max_active=64, hbm_budget=160 << 30, steps_per_tick=8,
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
        reqs = W.serving_stream(n=n, rate_hz=load * cap_hz)
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
                 "mix": "families 2D advection / 2D Burgers / 3D advection / 4D Vlasov, levels 2-5, "
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


def cpu_baseline(march_steps=12, single_steps=1):
    """The FP64 oracle on the host for the 4D Vlasov solve of the headline, on a bounded sample:
    `march_steps` time steps on all OpenMP threads (and `single_steps` on one thread, the paper's
    setting), plus the oracle's prolongation + combination of the same workload at finest level 2
    (32^4), scaled to the full solve by the interpolation count.  The estimated solve time is
    307 x (seconds per step) + (seconds per interpolation) x (interpolations of the full solve)."""
    import oracle as O
    from paper_2007_10196_amd.solver import Plan
    pb = W.c4_vlasov_4d(precision=W.PREC_FP64)
    nodes = O.total_nodes(pb)
    steps_full = step_estimate_any(pb)
    interp_full = interpolation_count(Plan(pb))
    st = O.restrict(pb)
    dt = pb.T / steps_full

    def march(nsteps, nthreads):
        t0 = time.perf_counter()
        stats = O.evolve(pb, st, T=(nsteps - 0.5) * dt, nthreads=nthreads)
        return (time.perf_counter() - t0) / stats["steps"], stats["steps"]

    sec_step, n_all = march(march_steps, 0)
    sec_step1, n_one = march(single_steps, 1)
    small = pb.replace(nl=2)
    st_small = O.restrict(small)
    t0 = time.perf_counter()
    O.prolong_combine(small, st_small)
    t_pro_small = time.perf_counter() - t0
    interp_small = interpolation_count(Plan(small))
    sec_interp = t_pro_small / interp_small
    solve_s = steps_full * sec_step + sec_interp * interp_full
    solve_s1 = steps_full * sec_step1 + sec_interp * interp_full
    cells = steps_full * nodes
    return {"value": cells / solve_s, "unit": "cell-updates/s", "cores": O.max_threads(), "kind": "oracle",
            "sample": f"4D Vlasov solve (FP64, root 8, finest level 4, 69 grids): {n_all} time steps on all "
                      f"threads ({sec_step:.3f} s per step) + the prolongation and combination of the same "
                      f"workload at finest level 2 ({interp_small} interpolations in {t_pro_small:.2f} s, one "
                      f"thread), scaled to {steps_full} steps and {interp_full:.3e} interpolations: "
                      f"{solve_s:.0f} s per solve",
            "estimated_solve_s": solve_s, "march_s_per_step": sec_step, "prolong_s_per_interpolation": sec_interp,
            "single_thread_value": cells / solve_s1,
            "single_thread_sample": f"{n_one} time step(s) on one thread ({sec_step1:.2f} s per step), the same "
                                    f"prolongation figure",
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
    batch_stage_us = e0.elapsed_time(e1) / reps * 1e3
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
    pro_ms = e2.elapsed_time(e3)
    # the stage launches of one time step as the solver enqueues them (measurement hook; this
    # spoils the solve's state, which is not read again)
    for stage in range(3):
        s.launch_stage(stage, 0, 1)
    e4, e5 = ev(), ev()
    e4.record(s.stream)
    for _ in range(reps):
        for stage in range(3):
            s.launch_stage(stage, 0, 1)
    e5.record(s.stream)
    torch.cuda.synchronize()
    print(json.dumps({
        "workload": f"{pb.name}: d={pb.d}, root {pb.nr}, finest level {pb.nl}, {len(s.plan.grids)} component grids, "
                    f"{s.plan.total_nodes} nodes, finest grid {s.plan.fine_nodes} nodes, T={pb.T}",
        "precision": precision, "boxes": info["boxes"], "box_target": box_target, "blocks_per_cu": bpc,
        "stage_launches_per_step_us": e4.elapsed_time(e5) / reps * 1e3,
        "batch_stage_launches_per_step_us": batch_stage_us, "steps": steps, "t": t, "march_ms": march_ms,
        "march_ms_per_step": march_ms / max(steps, 1),
        "march_cell_updates_per_s": steps * s.plan.total_nodes / (march_ms * 1e-3),
        "prolong_combine_ms": pro_ms}), flush=True)


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


def ev(torch):
    return torch.cuda.Event(enable_timing=True)


def stage_kernels_us(torch, s, reps):
    """Average launch duration of each kernel of a 4D stage (the plane launch, the line sweeps of
    directions 3 and 4) over the three RK stages, and of a whole time step, each event-timed alone
    on the solver stream through the measurement hook after the solve (whose state it spoils)."""
    out = {}
    for key, part in (("plane", 1), ("line3", 4), ("line4", 5)):
        by_stage = []
        for stage in range(3):
            s.launch_stage(stage, part, 2)
            e0, e1 = ev(torch), ev(torch)
            e0.record(s.stream)
            s.launch_stage(stage, part, reps)
            e1.record(s.stream)
            torch.cuda.synchronize()
            by_stage.append(e0.elapsed_time(e1) * 1e3 / reps)
        out[key] = sum(by_stage) / 3
        out[key + "_by_stage"] = by_stage
    e0, e1 = ev(torch), ev(torch)
    e0.record(s.stream)
    for _ in range(reps):
        for stage in range(3):
            s.launch_stage(stage, 0, 1)
    e1.record(s.stream)
    torch.cuda.synchronize()
    out["step_us"] = e0.elapsed_time(e1) * 1e3 / reps
    return out


def solve_run(torch, pb, steps, warmup, box_target, bpc):
    """`warmup` untimed and `steps` timed solves of pb through the whole path on one stream
    (restriction, march, prolongation + combination, norms against the exact solution, which is
    computed once before timing), then one more solve with each part event-timed."""
    from paper_2007_10196_amd.solver import Solver
    s = Solver(pb, device="cuda:0", box_target=box_target, blocks_per_cu=bpc)
    out = torch.empty(s.plan.fine_nodes, dtype=torch.float64, device="cuda:0")
    exact = s.exact(pb.T)
    res = torch.zeros(2, dtype=torch.float64, device="cuda:0")

    def one():
        s.restrict()
        s.advance()
        s.prolongate_combine(out)
        s.norms_async(out, exact, res)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        one()
        print(f"[bench] {pb.name} solve {k + 1}/{steps} queued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    l1, linf = res.tolist()
    t, nsteps = s.query()
    # one more solve, each part between HIP events on the solver stream
    e = [ev(torch) for _ in range(5)]
    e[0].record(s.stream)
    s.restrict()
    e[1].record(s.stream)
    s.advance()
    e[2].record(s.stream)
    s.prolongate_combine(out)
    e[3].record(s.stream)
    s.norms_async(out, exact, res)
    e[4].record(s.stream)
    torch.cuda.synchronize()
    parts = {name: e[i].elapsed_time(e[i + 1]) for i, name in
             enumerate(("restrict_ms", "march_ms", "prolong_combine_ms", "norms_ms"))}
    return {"solver": s, "out": out, "exact": exact, "ms_per_solve": elapsed / steps * 1e3, "l1": l1, "linf": linf,
            "t": t, "time_steps": nsteps, "parts": parts}


def kernel_roofline(kernel, launch_us, flops, peak, traffic, extra):
    ach = flops / (launch_us * 1e-6) / 1e12
    out = {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
           "traffic": traffic, "kernel": kernel, "avg_launch_us": launch_us, "flops_per_launch": flops,
           "hbm_GBs": traffic / (launch_us * 1e-6) / 1e9 if traffic else None,
           "hbm_frac": traffic / (launch_us * 1e-6) / 1e9 / PEAK_HBM_GBS if traffic else None}
    out.update(extra)
    return out


def c4_headline(args, torch):
    """The 4D Vlasov solve at FP64 (value), its kernels against their rooflines, the same solve with
    FP32 sweeps and the plain per-grid FP64 method on it."""
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.autotune import tune_box_target
    from paper_2007_10196_amd.solver import Solver
    pb = W.c4_vlasov_4d(precision=W.PREC_FP64)
    if args.box_target:
        tune = {"best": args.box_target, "blocks_per_cu": args.blocks_per_cu, "us": None, "cached": True}
    else:
        tune = tune_box_target([pb], pb.precision, reps=5)
    bt, bpc = int(tune["best"]), int(tune.get("blocks_per_cu", 0))
    if tune.get("line_sweeps"):
        print("[bench] 4D Vlasov FP64: line sweeps (no stage boxes to shape)", file=sys.stderr, flush=True)
    else:
        print(f"[bench] 4D Vlasov FP64: box target {bt}, {bpc or 'max'} workgroups per CU "
              f"({'cached' if tune['cached'] else 'measured'})", file=sys.stderr, flush=True)
    r = solve_run(torch, pb, args.steps, args.warmup, bt, bpc)
    s = r["solver"]
    nodes, fine = s.plan.total_nodes, s.plan.fine_nodes
    cells = r["time_steps"] * nodes
    value = cells / (r["ms_per_solve"] * 1e-3)
    print(f"[bench] 4D Vlasov FP64: {r['ms_per_solve']:.1f} ms per solve, {value:.3e} cell-updates/s, "
          f"L1 {r['l1']:.3e}", file=sys.stderr, flush=True)

    # ---- the kernels that take the solve's time, against their rooflines.  A 4D stage is the plane
    # launch (directions 1 and 2 over whole planes in LDS) and the line sweeps of directions 3 and 4;
    # each is event-timed alone on the solver stream through the measurement hook, in each RK stage
    stage_parts = stage_kernels_us(torch, s, args.stage_reps)
    steps = r["time_steps"]
    fl = 140  # flops per node and direction of the WENO5-LF flux difference
    # algorithmic words per node: the plane launch reads the stage input and writes the partial sum;
    # direction 3 reads the input and the partial sum and writes it back; direction 4 reads both and
    # writes the output, and in stages 2 and 3 also reads u^n
    spec = {"plane": ("plane_kernel<double> (directions 1 and 2 of one WENO5-LF stage over whole (x_1, x_2) planes "
                      "staged in LDS)", 2 * fl, 2.0),
            "line3": ("line_kernel<double, 4, 2> (direction 3 of one stage over every grid line)", fl, 3.0),
            "line4": ("line_kernel<double, 4, 3> (direction 4 and the TVD-RK3 combination of one stage)", fl + 5,
                      3.0 + 2.0 / 3.0)}
    stage_k = []
    for key, (name, fpn, words) in spec.items():
        us = stage_parts[key]
        stage_k.append(kernel_roofline(
            name, us, nodes * fpn, PEAK_FP64_TFLOPS, measured_traffic("stage_c4_fp64", key),
            {"launches_per_time_step": 3, "nodes_per_launch": nodes, "flops_per_node": fpn,
             "algorithmic_bytes_per_launch": nodes * 8 * words, "time_per_solve_ms": us * 3 * steps * 1e-3,
             "per_stage_us": stage_parts[key + "_by_stage"]}))
    pro_us = r["parts"]["prolong_combine_ms"] * 1e3
    interps = interpolation_count(s.plan)
    prolong = kernel_roofline(
        "prolong_kernel<double, 4> (WENO5 prolongation of the 69 grids and FP64 combination, one launch)",
        pro_us, interps * INTERP_FLOPS, PEAK_FP64_TFLOPS, measured_traffic("prolong_c4_fp64"),
        {"interpolations_per_launch": interps, "flops_per_interpolation": INTERP_FLOPS,
         "algorithmic_bytes_per_launch": fine * 8 + nodes * 8,
         "achieved_write_GBs": fine * 8 / (pro_us * 1e-6) / 1e9, "time_per_solve_ms": pro_us * 1e-3})
    by_time = sorted(stage_k + [prolong], key=lambda k: -k["time_per_solve_ms"])

    # ---- the same solve with FP32 sweeps (FP64 combination and norms)
    fp32 = None
    if not args.no_fp32:
        p32 = pb.replace(precision=W.PREC_FP32)
        t32 = tune_box_target([p32], p32.precision, reps=5)
        r32 = solve_run(torch, p32, args.steps, 1, int(t32["best"]), int(t32.get("blocks_per_cu", 0)))
        d = (r32["out"] - r["out"]).abs()
        fp32 = {"value": r32["time_steps"] * nodes / (r32["ms_per_solve"] * 1e-3), "unit": "cell-updates/s",
                "ms_per_solve": r32["ms_per_solve"], "parts": r32["parts"], "l1": r32["l1"], "linf": r32["linf"],
                "l1_vs_fp64_solution": float(d.mean()), "linf_vs_fp64_solution": float(d.max()),
                "box_target": int(t32["best"]), "blocks_per_cu": int(t32.get("blocks_per_cu", 0))}
        print(f"[bench] 4D Vlasov FP32 sweeps: {r32['ms_per_solve']:.1f} ms per solve, L1 {r32['l1']:.3e}",
              file=sys.stderr, flush=True)
        del r32, d

    # ---- plain per-grid FP64 method (one launch per grid per RK stage, no graph) on the same solve
    plain = None
    if not args.no_plain:
        sp = Solver(pb, device="cuda:0")
        Up = torch.empty(fine, dtype=torch.float64, device="cuda:0")
        for _ in range(2):
            torch.cuda.synchronize()
            tp = time.perf_counter()
            sp.restrict()
            sp.advance(mode=B.RUN_PLAIN)
            sp.prolongate_combine(Up)
            l1p, lip = sp.norms(Up, r["exact"])
            torch.cuda.synchronize()
            tp = time.perf_counter() - tp
        stp = sp.query()[1]
        plain = {"value": stp * nodes / tp, "unit": "cell-updates/s",
                 "mode": "plain: one launch per grid per RK stage, no graph, FP64", "ms_per_solve": tp * 1e3,
                 "l1": l1p, "linf": lip, "speedup_of_value": value / (stp * nodes / tp),
                 "equal_l1": bool(abs(r["l1"] - l1p) <= 0.01 * l1p)}
        print(f"[bench] plain per-grid FP64: {tp * 1e3:.1f} ms per solve", file=sys.stderr, flush=True)
        del sp, Up

    head = {"value": value, "ms_per_solve": r["ms_per_solve"], "l1": r["l1"], "linf": r["linf"],
            "time_steps": r["time_steps"], "t": r["t"], "nodes": nodes, "fine": fine, "parts": r["parts"],
            "finest_equivalent_cell_updates_per_s": r["time_steps"] * fine / (r["ms_per_solve"] * 1e-3),
            "roofline": by_time[0], "roofline_other": by_time[1:],
            "stage_step_us": stage_parts["step_us"], "fp32": fp32, "plain": plain,
            "autotune": {"box_target": bt, "blocks_per_cu": bpc, "stage_us_by_target_and_cap": tune["us"],
                         "line_sweeps": bool(tune.get("line_sweeps"))}}
    del r
    return head


def c2_batched(args, torch):
    """The batched 2D Burgers workload: 256 solves per step, FP32 sweeps (and FP64), the plain
    per-grid method on one of them, and the same solves on one full 256x256 grid."""
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.autotune import tune_box_target
    from paper_2007_10196_amd.solver import Batch, PtrList, Solver
    dev = torch.device("cuda:0")
    probs = make_problems(args.solves)
    tune = tune_box_target(probs, B.FP32_SWEEP, reps=5)
    box_target, bpc = int(tune["best"]), int(tune.get("blocks_per_cu", 0))
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
    run_batch_step(torch, batch, solvers, outs, exacts, res, sent)
    sent.take()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_batch_step(torch, batch, solvers, outs, exacts, res, sent)
    norms = sent.take()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps_each = [s.query()[1] for s in solvers]
    ms_per_step = elapsed / args.steps * 1e3
    value = sum(n * nodes for n in steps_each) / (elapsed / args.steps)
    l1s = norms[:, 0]
    print(f"[bench] 2D Burgers x {len(probs)}: {ms_per_step:.2f} ms per step, {value:.3e} cell-updates/s",
          file=sys.stderr, flush=True)

    # the three-stage kernel alone (every grid of this workload is one stage box), HIP events on the
    # batch stream, and the split kernel's stage 1 beside it
    from paper_2007_10196_amd.solver import restrict_many
    restrict_many(solvers, stream=batch.stream)
    batch.admit_many(solvers)
    batch.step(1)
    st = batch.stream

    def timed(stage, reps):
        e0, e1 = ev(torch), ev(torch)
        batch.launch_stage(stage, 2)
        e0.record(st)
        batch.launch_stage(stage, reps)
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    step_ms = timed(3, args.stage_reps)
    split_ms = timed(0, args.stage_reps)
    info = batch.info()
    batch.release_many(list(batch.slots))
    batch.close()
    roof = kernel_roofline("stage_kernel<float, 2, fused> (three RK stages of every one-box grid)", step_ms * 1e3,
                           info["nodes"] * flops_per_cell_update(2), PEAK_FP32_TFLOPS,
                           measured_traffic("stage_c2_fp32"),
                           {"boxes_per_launch": info["boxes"], "algorithmic_bytes_per_launch": info["nodes"] * 8,
                            "split_stage_kernel_stage1_us": split_ms * 1e3})

    plain = None
    if not args.no_plain:
        p64 = probs[0].replace(precision=W.PREC_FP64)
        sp = Solver(p64, device="cuda:0")
        Up = torch.empty(fine, dtype=torch.float64, device=dev)
        Ep = sp.exact(T_FINAL)
        for _ in range(2):
            torch.cuda.synchronize()
            tp = time.perf_counter()
            sp.restrict()
            sp.advance(mode=B.RUN_PLAIN)
            sp.prolongate_combine(Up)
            l1p, lip = sp.norms(Up, Ep)
            torch.cuda.synchronize()
            tp = time.perf_counter() - tp
        stp = sp.query()[1]
        plain = {"value": stp * nodes / tp, "ms_per_solve": tp * 1e3, "l1": l1p, "linf": lip,
                 "speedup_of_value": value / (stp * nodes / tp),
                 "equal_l1": bool(abs(l1s[0] - l1p) <= 0.01 * l1p), "l1_batched_fp32_same_solve": float(l1s[0])}

    batched_fp64 = None
    if not args.no_fp64:
        f = batch_run(torch, [p.replace(precision=W.PREC_FP64) for p in probs], box_target, bpc, steps=args.steps)
        v64 = f["cell_updates_per_step"] / (f["ms_per_step"] * 1e-3)
        batched_fp64 = {"value": v64, "ms_per_step": f["ms_per_step"], "l1_mean": f["l1_mean"],
                        "fp32_speedup": value / v64,
                        "plain_fp64_speedup": v64 / plain["value"] if plain else None}
        print(f"[bench] 2D Burgers FP64 batched: {f['ms_per_step']:.2f} ms per step, {v64:.3e} cell-updates/s",
              file=sys.stderr, flush=True)

    full = None
    if not args.no_full:
        f = full_grid_run(torch, probs, box_target, bpc)
        full = {"full_grid": "one 256x256 grid (root 256, finest level 0), same solves, same batched FP32 path",
                "full_ms_per_step": f["ms_per_step"], "sparse_ms_per_step": ms_per_step,
                "time_ratio_sparse_over_full": ms_per_step / f["ms_per_step"],
                "l1_full": f["l1_mean"], "l1_sparse": float(l1s.mean()),
                "nodes_full": f["nodes_per_solve"], "nodes_sparse": nodes, "time_steps_full": f["time_steps"]}

    return {"workload": "2D Burgers u0=0.3+A sin(pi(x+y)+phi), [-1,1]^2 periodic, root 8x8, finest level 5 "
                        "(256x256), 11 component grids, CFL 0.5, T=1.5/pi^2; FP32 sweeps, FP64 combination",
            "solves_per_step": len(probs), "value": value, "unit": "cell-updates/s", "ms_per_step": ms_per_step,
            "l1_mean": float(l1s.mean()), "l1_max": float(l1s.max()),
            "mode": "batched: step graphs of 1..32 time steps, persistent fused WENO5+RK3 stage launch",
            "roofline": roof, "plain_fp64_one_solve": plain, "batched_fp64": batched_fp64, "sparse_vs_full": full,
            "autotune": {"box_target": box_target, "blocks_per_cu": bpc, "step_stage_us_by_target_and_cap": tune["us"]}}


# The paper's own comparison (Sec. 3): CPU seconds of the sparse grid with WENO prolongation and of the
# single grid at equal finest resolution N_h, with their L1 errors, on a 2.3 GHz workstation.
PAPER_SWEEPS = {
    "ex3a_2d_burgers": {"table": "Table ex3aweno", "nl": 3, "n_h": (80, 160, 320, 640),
                        "cpu_sparse_s": (0.414, 4.976, 61.510, 781.990),
                        "cpu_single_s": (0.572, 7.156, 92.854, 1149.946),
                        "l1_sparse": (7.1354e-05, 2.7404e-07, 1.3265e-09, 4.0784e-11),
                        "l1_single": (1.3362e-06, 4.2306e-08, 1.3119e-09, 4.0883e-11)},
    "ex3b_3d_burgers": {"table": "Table ex3-baweno", "nl": 3, "n_h": (80, 160, 320, 640),
                        "cpu_sparse_s": (15.106, 223.450, 4144.632, 96962.960),
                        "cpu_single_s": (26.706, 691.410, 16868.220, 444972.000),
                        "l1_sparse": (1.3225e-04, 7.6655e-07, 2.4830e-09, 6.4883e-11),
                        "l1_single": (2.0866e-06, 6.6687e-08, 2.0836e-09, 6.5107e-11)},
}


def timed_solve(torch, pb, reps=2):
    """Restriction, march, prolongation + combination of one FP64 solve on one stream, the last of
    `reps` runs timed with HIP events; L1 / Linf against the exact solution at T."""
    from paper_2007_10196_amd.solver import Solver
    s = Solver(pb, device="cuda:0")
    out = torch.empty(s.plan.fine_nodes, dtype=torch.float64, device="cuda:0")
    for _ in range(reps):
        e0, e1 = ev(torch), ev(torch)
        e0.record(s.stream)
        s.restrict()
        s.advance()
        s.prolongate_combine(out)
        e1.record(s.stream)
        torch.cuda.synchronize()
    t, steps = s.query()
    exact = s.exact(t)
    l1, linf = s.norms(out, exact)
    res = {"ms": e0.elapsed_time(e1), "l1": l1, "linf": linf, "time_steps": steps, "nodes": s.plan.total_nodes}
    del s, out, exact
    torch.cuda.empty_cache()
    return res


def paper_sweep(torch):
    """Sparse grid against single grid on the GPU at the paper's N_h (Tables ex3aweno and ex3-baweno
    settings, FP64, dt = dx^(5/3)), the 4D Vlasov workload at root 10, level 3 (80^4, the resolution
    of Table tb:ex5bcpu) against its single grid, and the 2D Burgers workload's single grid at the
    resolution whose L1 matches the sparse grid's (equal error), with FP32 sweeps as in the batched leg."""
    out = {}
    for name, spec in PAPER_SWEEPS.items():
        make = W.paper_example3a if name.startswith("ex3a") else W.paper_example3b
        rows = []
        for i, nh in enumerate(spec["n_h"]):
            sp = timed_solve(torch, make(nh, nl=spec["nl"]))
            si = timed_solve(torch, make(nh, nl=0))
            rows.append({"n_h": nh, "sparse_ms": sp["ms"], "single_ms": si["ms"], "gpu_ratio": sp["ms"] / si["ms"],
                         "l1_sparse": sp["l1"], "l1_single": si["l1"], "time_steps": sp["time_steps"],
                         "paper_l1_sparse": spec["l1_sparse"][i], "paper_l1_single": spec["l1_single"][i],
                         "paper_cpu_ratio": spec["cpu_sparse_s"][i] / spec["cpu_single_s"][i],
                         "nodes_sparse": sp["nodes"], "nodes_single": si["nodes"]})
            print(f"[bench] {name} N_h {nh}: sparse {sp['ms']:.1f} ms L1 {sp['l1']:.4e}, single {si['ms']:.1f} ms "
                  f"L1 {si['l1']:.4e}", file=sys.stderr, flush=True)
        out[name] = {"table": spec["table"], "rows": rows}
    v4 = []
    for nl in (3, 0):
        pb = W.c4_vlasov_4d(nr=10 << (3 - nl), nl=nl, precision=W.PREC_FP64)
        v4.append(timed_solve(torch, pb, reps=1 if nl == 0 else 2))
    out["vlasov_4d_80"] = {"setting": "4D Vlasov workload (fixed field, periodic), N_h = 80: sparse root 10, "
                                      "level 3 against one 80^4 grid, FP64, CFL 0.4, T = 1",
                           "sparse_ms": v4[0]["ms"], "single_ms": v4[1]["ms"], "gpu_ratio": v4[0]["ms"] / v4[1]["ms"],
                           "l1_sparse": v4[0]["l1"], "l1_single": v4[1]["l1"],
                           "nodes_sparse": v4[0]["nodes"], "nodes_single": v4[1]["nodes"],
                           "paper_cpu_ratio": "0.064-0.070 (Table tb:ex5bcpu: 4D Vlasov-Boltzmann, zero boundary, "
                                              "t = 0.5 to 3)"}
    print(f"[bench] 4D N_h 80: sparse {v4[0]['ms']:.1f} ms, single {v4[1]['ms']:.1f} ms", file=sys.stderr, flush=True)
    # equal error, 2D Burgers workload, 256 solves per step (FP32 sweeps)
    probs = make_problems(256)
    sparse = batch_run(torch, probs, 0, 0, steps=2)
    fulls = []
    for nh in (32, 48, 64, 96, 128):
        f = batch_run(torch, [p.replace(nr=nh, nl=0) for p in probs], 0, 0, steps=2)
        fulls.append({"n_h": nh, "ms_per_step": f["ms_per_step"], "l1_mean": f["l1_mean"]})
        print(f"[bench] 2D Burgers single {nh}^2: {f['ms_per_step']:.2f} ms/step L1 {f['l1_mean']:.3e}",
              file=sys.stderr, flush=True)
    match = next((f for f in fulls if f["l1_mean"] <= sparse["l1_mean"]), None)
    out["equal_error_2d_burgers"] = {
        "sparse": {"n_h": 256, "ms_per_step": sparse["ms_per_step"], "l1_mean": sparse["l1_mean"]},
        "single_grids": fulls, "single_at_equal_error": match,
        "sparse_over_single_time_at_equal_error": sparse["ms_per_step"] / match["ms_per_step"] if match else None}
    return out


# The paper's Vlasov-Boltzmann comparison (Sec. 3.4, Example 5): CPU seconds of the sparse-grid and
# single-grid computations to time t (Tables tb:ex5acpu, tb:ex5bcpu).
EX5_TABLES = {
    "ex5a_2d": {"table": "Table tb:ex5acpu", "d": 2, "nr": 40, "nl": 3, "t": (0.5, 1.0, 2.0, 3.0, 6.0),
                "cpu_single_s": (13111.313, 25185.141, 50756.395, 82253.965, 153593.745),
                "cpu_sparse_s": (11720.746, 21371.762, 39493.979, 57898.835, 110626.464)},
    "ex5b_4d": {"table": "Table tb:ex5bcpu", "d": 4, "nr": 10, "nl": 3, "t": (0.5, 1.0, 2.0, 3.0),
                "cpu_single_s": (56231.125, 112539.000, 225612.000, 332706.250),
                "cpu_sparse_s": (3918.468, 7876.233, 14468.500, 22821.125)},
}


def example5_run(torch, pb, times):
    """One FP64 solve of the Vlasov-Boltzmann model marched through `times`: at each t the GPU
    time of restriction + march to t + one prolongation and combination (HIP events on the solver
    stream around each piece; the entropy reductions between checkpoints are not counted), and
    the entropy functionals and mass of the combined solution."""
    from paper_2007_10196_amd.solver import Solver
    s = Solver(pb, device="cuda:0")
    out = torch.empty(s.plan.fine_nodes, dtype=torch.float64, device="cuda:0")
    # warm-up: graph capture and first launches, then start over
    s.restrict()
    s.advance(min(times[0], 0.01))
    s.prolongate_combine(out)
    torch.cuda.synchronize()
    rows = []
    r0, r1 = ev(torch), ev(torch)
    r0.record(s.stream)
    s.restrict()
    r1.record(s.stream)
    torch.cuda.synchronize()
    march_ms = r0.elapsed_time(r1)
    cell = (10.0 / pb.n_fine) ** pb.d
    # analysis only: H_2 over the ball |(x, v)| <= 4 (M >= e^-8 M(0)), where the far field's
    # division by M (down to e^-50 M(0) at the 4D corners) does not weigh in
    n, m = pb.n_fine, pb.d // 2
    g = -5.0 + (10.0 / n) * torch.arange(n, dtype=torch.float64, device="cuda:0")
    r2 = torch.zeros((), dtype=torch.float64, device="cuda:0")
    for k in range(pb.d):
        r2 = r2.unsqueeze(-1) + (g * g).reshape((1,) * k + (n,))
    r2 = r2.reshape(-1)
    zx = (math.sqrt(2.0 * math.pi) * math.erf(5.0 / math.sqrt(2.0))) ** m
    Minv = torch.exp(0.5 * r2) * ((2.0 * math.pi) ** (m / 2) * zx)
    inner = r2 <= 16.0
    del r2
    for t in times:
        e0, e1, e2 = ev(torch), ev(torch), ev(torch)
        e0.record(s.stream)
        s.advance(t)
        e1.record(s.stream)
        s.prolongate_combine(out)
        e2.record(s.stream)
        torch.cuda.synchronize()
        march_ms += e0.elapsed_time(e1)
        h2, hl = s.entropies(out)
        mass = float(out.sum().item()) * cell
        h2_inner = float((out * out * Minv)[inner].sum().item()) * cell
        _, steps = s.query()
        rows.append({"t": t, "ms": march_ms + e1.elapsed_time(e2), "march_ms": march_ms,
                     "prolong_ms": e1.elapsed_time(e2), "time_steps": steps, "H2": h2, "Hlog": hl, "mass": mass,
                     "H2_inner_ball_r4": h2_inner})
    res = {"nodes": s.plan.total_nodes, "fine_nodes": s.plan.fine_nodes, "rows": rows}
    del s, out, Minv, inner
    torch.cuda.empty_cache()
    return res


def example5(torch):
    """Sparse grid against single grid for the Vlasov-Boltzmann model at the paper's settings
    (Example 5(a): 2D, root 40, level 3, 320^2; (b): 4D, root 10, level 3, 80^4; theta = tau = 1,
    zero boundaries, CFL 0.4, FP64) at the times of Tables tb:ex5acpu and tb:ex5bcpu, with the
    entropy decay of both computations."""
    out = {}
    for name, spec in EX5_TABLES.items():
        d, nr, nl = spec["d"], spec["nr"], spec["nl"]
        sp = example5_run(torch, W.paper_example5(d, nr=nr, nl=nl), spec["t"])
        si = example5_run(torch, W.paper_example5(d, nr=nr << nl, nl=0), spec["t"])
        rows = []
        for i, t in enumerate(spec["t"]):
            a, b = sp["rows"][i], si["rows"][i]
            rows.append({"t": t, "sparse_ms": a["ms"], "single_ms": b["ms"], "gpu_ratio": a["ms"] / b["ms"],
                         "paper_cpu_ratio": spec["cpu_sparse_s"][i] / spec["cpu_single_s"][i],
                         "time_steps": a["time_steps"], "H2_sparse": a["H2"], "H2_single": b["H2"],
                         "Hlog_sparse": a["Hlog"], "Hlog_single": b["Hlog"], "mass_sparse": a["mass"],
                         "mass_single": b["mass"], "prolong_ms_sparse": a["prolong_ms"],
                         "H2_inner_sparse": a["H2_inner_ball_r4"], "H2_inner_single": b["H2_inner_ball_r4"]})
            print(f"[bench] {name} t={t}: sparse {a['ms']:.1f} ms, single {b['ms']:.1f} ms "
                  f"(ratio {a['ms'] / b['ms']:.3f}, paper {rows[-1]['paper_cpu_ratio']:.3f}); "
                  f"H2 {a['H2']:.5f}/{b['H2']:.5f} (|z|<=4: {a['H2_inner_ball_r4']:.5f}/{b['H2_inner_ball_r4']:.5f}), "
                  f"Hlog {a['Hlog']:.5f}/{b['Hlog']:.5f}",
                  file=sys.stderr, flush=True)
        out[name] = {"table": spec["table"], "nodes_sparse": sp["nodes"], "nodes_single": si["nodes"],
                     "finest_nodes": sp["fine_nodes"], "rows": rows}
    return out


def example6_run(torch, pb):
    """One FP64 Vlasov-Maxwell solve to T: GPU time of restriction + march + prolongation and
    combination of f + combination of the fields (HIP events on the solver stream), the field
    energies and the distribution's mass, kinetic energy and extrema."""
    from paper_2007_10196_amd.solver import Solver
    s = Solver(pb, device="cuda:0")
    out = torch.empty(s.plan.fine_nodes, dtype=torch.float64, device="cuda:0")
    s.restrict()
    s.advance(min(pb.T, 0.5))
    s.prolongate_combine(out)
    s.fields_combine()
    torch.cuda.synchronize()
    e0, e1, e2, e3 = ev(torch), ev(torch), ev(torch), ev(torch)
    e0.record(s.stream)
    s.restrict()
    s.advance()
    e1.record(s.stream)
    s.prolongate_combine(out)
    e2.record(s.stream)
    F = s.fields_combine()
    e3.record(s.stream)
    torch.cuda.synchronize()
    t, steps = s.query()
    n = pb.n_fine
    hx, hv = (pb.hi[0] - pb.lo[0]) / n, 2.4 / n
    xi = -1.2 + hv * torch.arange(n, dtype=torch.float64, device="cuda:0")
    f3 = out.view(n, n, n)  # [xi_2, xi_1, x_2]
    kinetic = 0.5 * float(((xi * xi).view(n, 1, 1) * f3).sum() + ((xi * xi).view(1, n, 1) * f3).sum()) * hx * hv * hv
    res = {"ms": e0.elapsed_time(e3), "march_ms": e0.elapsed_time(e1), "prolong_ms": e1.elapsed_time(e2),
           "fields_combine_ms": e2.elapsed_time(e3), "time_steps": steps, "t": t, "nodes": s.plan.total_nodes,
           "mass": float(out.sum()) * hx * hv * hv, "kinetic_energy": kinetic,
           "field_energy_B3": 0.5 * float((F[0] * F[0]).sum()) * hx,
           "field_energy_E1": 0.5 * float((F[1] * F[1]).sum()) * hx,
           "field_energy_E2": 0.5 * float((F[2] * F[2]).sum()) * hx,
           "f_min": float(out.min()), "f_max": float(out.max())}
    res["fields"] = F
    res["f"] = out
    return res


def example6(torch):
    """Sparse grid against single grid for the 3D Vlasov-Maxwell system at the paper's setting
    (Example 6: root 20, level 3 against 160^3, CFL 0.4, T = 10, FP64); the paper prints CPU times
    3585.81 s (sparse) and 10331.04 s (single)."""
    sp = example6_run(torch, W.paper_example6(nr=20, nl=3))
    si = example6_run(torch, W.paper_example6(nr=160, nl=0))
    df = (sp["f"] - si["f"]).abs()
    dF = (sp["fields"] - si["fields"]).abs()
    out = {"table": "Example 6 (CPU 3585.81 s sparse, 10331.04 s single)", "paper_cpu_ratio": 3585.81 / 10331.04,
           "sparse": {k: v for k, v in sp.items() if k not in ("f", "fields")},
           "single": {k: v for k, v in si.items() if k not in ("f", "fields")},
           "gpu_ratio": sp["ms"] / si["ms"],
           "f_sparse_minus_single": {"l1": float(df.mean()), "linf": float(df.max())},
           "fields_sparse_minus_single_linf": [float(dF[q].max()) for q in range(3)]}
    print(f"[bench] example6: sparse {sp['ms']:.1f} ms ({sp['time_steps']} steps), single {si['ms']:.1f} ms "
          f"({si['time_steps']} steps), ratio {out['gpu_ratio']:.3f} (paper {out['paper_cpu_ratio']:.3f}); "
          f"f sparse-single L1 {out['f_sparse_minus_single']['l1']:.3e} Linf {out['f_sparse_minus_single']['linf']:.3e}",
          file=sys.stderr, flush=True)
    del sp, si, df, dF
    torch.cuda.empty_cache()
    return out


def large_roofline(torch, reps=10):
    """Stage launches of one time step on the scaled cases whose state exceeds the 256 MB MALL: 3D
    advection at root 32 (32.5 M nodes) and the 4D Vlasov workload at root 16 (50.3 M nodes), both as
    line sweeps, one launch per direction and stage, FP64 and FP32, event-timed through the batch
    measurement hook."""
    from paper_2007_10196_amd.solver import Batch, Solver
    out = []
    for name, make in (("c3_large", lambda p: W.c3_advection_3d(nr=32, precision=p)),
                       ("c4_large", lambda p: W.c4_vlasov_4d(nr=16, precision=p))):
        for prec in (W.PREC_FP64, W.PREC_FP32):
            pb = make(prec)
            s = Solver(pb, device="cuda:0")
            batch = Batch(max_solvers=1, precision=prec, hbm_budget=1 << 40, max_items=1 << 24)
            s.restrict()
            slot = batch.admit(s)
            batch.step(1)
            st = batch.stream
            e0, e1 = ev(torch), ev(torch)
            batch.launch_stage(3, 2)
            e0.record(st)
            batch.launch_stage(3, reps)
            e1.record(st)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / reps * 1e3
            nodes = s.plan.total_nodes
            esz = 8 if prec == W.PREC_FP64 else 4
            flops = nodes * flops_per_cell_update(pb.d)
            # stage boxes, fused 3-stage minimum: stage 1 reads u and writes u1, stages 2 and 3 also read
            # u^n (8 words); the line sweep (3D and 4D, one launch per direction in a batch) also moves
            # its partial sums: 3 (3d - 1/3) words per step
            boxes = s.plan.grids[0]["box"] != (0,) * pb.d
            words = 8.0 if boxes else 3 * (3 * pb.d - 1.0 / 3.0)
            peak = PEAK_FP64_TFLOPS if prec == W.PREC_FP64 else PEAK_FP32_TFLOPS
            row = {"case": name, "precision": "fp64" if prec == W.PREC_FP64 else "fp32", "nodes": nodes,
                   "state_MB": 3 * nodes * esz / 1e6, "step_stage_us": us,
                   "cell_updates_per_s": nodes / (us * 1e-6), "tflops": flops / (us * 1e-6) / 1e12,
                   "valu_frac_of_peak": flops / (us * 1e-6) / 1e12 / peak,
                   "algorithmic_bytes_per_cell_update": words * esz,
                   "algorithmic_GBs": nodes * words * esz / (us * 1e-6) / 1e9,
                   "algorithmic_hbm_frac": nodes * words * esz / (us * 1e-6) / 1e9 / PEAK_HBM_GBS}
            out.append(row)
            print(f"[bench] {name} {row['precision']}: {us:.1f} us per step, {row['algorithmic_GBs']:.0f} GB/s "
                  f"algorithmic, {row['tflops']:.1f} TFLOP/s", file=sys.stderr, flush=True)
            batch.release(slot)
            batch.close()
            del s
            torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed solves of the 4D workload (and timed 2D batch steps)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--solves", type=int, default=256, help="2D solves per batched step")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-sweep run of the 4D solve")
    ap.add_argument("--no-c2", action="store_true", help="skip the batched 2D Burgers workload")
    ap.add_argument("--stage-reps", type=int, default=20)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-full", action="store_true", help="skip the single full-grid comparison")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 batched run of the 2D solves")
    ap.add_argument("--box-target", type=int, default=0,
                    help="0: autotune the stage box target and the workgroups per compute unit")
    ap.add_argument("--blocks-per-cu", type=int, default=0, help="with --box-target: stage workgroups per CU")
    ap.add_argument("--serving-requests", type=int, default=SERVING_N)
    ap.add_argument("--serving-loads", default="0.7",
                    help="comma-separated offered loads (the first one is the reported latency)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB copy used to scale the HBM byte counters")
    ap.add_argument("--valu-calibration", action="store_true",
                    help="only time the VALU issue-rate calibration kernels")
    ap.add_argument("--path-workload", choices=("c3", "c4"),
                    help="only run one 3D (c3) or 4D (c4) solve through the path, each part timed")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32", help="with --path-workload")
    ap.add_argument("--paper-sweep", action="store_true",
                    help="only run sparse against single grid at the paper's resolutions (and equal error)")
    ap.add_argument("--example5", action="store_true",
                    help="only run the Vlasov-Boltzmann sparse/single comparison of Tables tb:ex5acpu, tb:ex5bcpu")
    ap.add_argument("--example6", action="store_true",
                    help="only run the Vlasov-Maxwell sparse/single comparison of Example 6")
    ap.add_argument("--large-roofline", action="store_true",
                    help="only time the stage launches of the scaled 3D/4D cases that exceed the MALL")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU; --gpus must be 1", file=sys.stderr)
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
    if args.paper_sweep or args.large_roofline or args.example5 or args.example6:
        import torch
        torch.cuda.set_device(0)
        if args.example5:
            res = {"example5": example5(torch)}
        elif args.example6:
            res = {"example6": example6(torch)}
        else:
            res = {"paper_sweep": paper_sweep(torch)} if args.paper_sweep else {"large_roofline": large_roofline(torch)}
        print(json.dumps(res), flush=True)
        return

    import torch
    torch.cuda.set_device(0)
    head = c4_headline(args, torch)
    c2 = None if args.no_c2 else c2_batched(args, torch)
    serving = None if args.no_serving else serving_run(
        0, n=args.serving_requests, loads=[float(x) for x in args.serving_loads.split(",")])
    cpu = None if args.no_cpu else cpu_baseline()
    out = {"metric": METRIC, "value": head["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_solve"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "4D Vlasov with fixed field, f_t + v.grad_x f + E(x).grad_v f = 0, x in [0,4pi]^2, "
                                  "v in [-6,6]^2 periodic, E = 0.01 (sin(x1/2), sin(x2/2)), f0 = Maxwellian x "
                                  "(1 + 0.01 cos(x1/2) cos(x2/2)); root 8^4, finest level 4 (128^4), 69 component "
                                  "grids, CFL 0.4, T = 1; FP64 throughout; one solve per step",
                      "component_nodes": head["nodes"], "finest_nodes": head["fine"],
                      "time_steps": head["time_steps"],
                      "mode": "step graphs; per RK stage one plane launch (directions 1, 2) and one line sweep "
                              "for each of directions 3, 4, each persistent over every grid; WENO5 prolongation "
                              "(line form) with FP64 combination in one launch"},
           "l1": head["l1"], "linf": head["linf"], "parts_ms": head["parts"],
           "finest_equivalent_cell_updates_per_s": head["finest_equivalent_cell_updates_per_s"],
           "roofline": head["roofline"], "roofline_other": head["roofline_other"],
           "stage_step_us": head["stage_step_us"], "cpu_baseline": cpu,
           "fp32_sweeps": head["fp32"], "plain": head["plain"], "latency": serving, "batched_2d_burgers": c2,
           "autotune": head["autotune"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
