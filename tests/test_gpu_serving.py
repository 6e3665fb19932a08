"""Serving loop and autotuner on the GPU.

Each request's combined solution must be bit-for-bit the one the same solve
produces alone (same kernels, per-solve time stepping), whatever else shares
the batch; requests are admitted by device footprint as memory frees up.
"""
import math

import numpy as np
import pytest

import oracle as O
import sgw_inputs as W

pytestmark = pytest.mark.gpu


def _mixed_stream(n=12, rate=400.0, seed=77, levels=(2, 3)):
    reqs = W.serving_stream(n=n, rate_hz=rate, seed=seed, levels=levels, precision=W.PREC_FP32)
    for r in reqs:  # keep the GPU time of the test small
        r.problem = r.problem.replace(T=min(r.problem.T, 0.15))
    return reqs


def test_serving_results_equal_solo_results():
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.serving import ServingLoop, latency_summary
    from paper_2007_10196_amd.solver import Solver
    reqs = _mixed_stream()
    assert len({r.family for r in reqs}) >= 3
    loop = ServingLoop(precision=B.FP32_SWEEP, max_active=5, hbm_budget=8 << 30, steps_per_tick=4,
                       keep_outputs=True)
    res = loop.run(reqs)
    torch.cuda.synchronize()
    assert sorted(r.rid for r in res) == [r.rid for r in reqs]
    summ = latency_summary(res)
    print("\n[gpu] serving", summ, flush=True)
    assert summ["p99_ms"] >= summ["p50_ms"] > 0
    by_id = {r.rid: r for r in reqs}
    for r in res:
        pb = by_id[r.rid].problem
        solo = Solver(pb).solve(mode=B.RUN_GRAPH).cpu().numpy()
        assert np.array_equal(r.out.cpu().numpy(), solo), r.rid
        assert r.steps > 0 and r.finish_s >= r.admit_s >= r.arrival_s - 1e-3
    loop.close()


def test_chunked_combinations_equal_solo_results():
    """Every combination forced into chunks of a few finest-grid tiles (chunk_fine_nodes tiny): the
    served results are still bitwise the solo ones."""
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.serving import ServingLoop
    from paper_2007_10196_amd.solver import Solver
    reqs = _mixed_stream(n=6, seed=41)
    loop = ServingLoop(precision=B.FP32_SWEEP, max_active=4, hbm_budget=8 << 30, steps_per_tick=4,
                       keep_outputs=True, chunk_fine_nodes=3000)
    res = loop.run(reqs)
    torch.cuda.synchronize()
    assert sorted(r.rid for r in res) == [r.rid for r in reqs]
    by_id = {r.rid: r for r in reqs}
    for r in res:
        solo = Solver(by_id[r.rid].problem).solve(mode=B.RUN_GRAPH).cpu().numpy()
        assert np.array_equal(r.out.cpu().numpy(), solo), r.rid
    loop.close()


def test_serving_fp32_results_close_to_fp64_oracle():
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.serving import ServingLoop
    reqs = _mixed_stream(n=6, seed=5, levels=(2,))
    loop = ServingLoop(precision=B.FP32_SWEEP, max_active=8, hbm_budget=8 << 30, keep_outputs=True)
    res = loop.run(reqs)
    by_id = {r.rid: r for r in reqs}
    for r in res:
        pb = by_id[r.rid].problem.replace(precision=W.PREC_FP64)
        U, _, _ = O.solve(pb)
        err = np.abs(r.out.cpu().numpy() - U)
        print(f"  request {r.rid} {pb.name} nl={pb.nl}: fp32 L1 {err.mean():.2e} Linf {err.max():.2e}")
        assert err.max() < 5e-5 * max(1.0, np.abs(U).max())
    loop.close()


def test_serving_fp64_results_match_fp64_oracle():
    """Served FP64 solves of mixed dimension and level, admitted while others run: each combined
    solution matches the FP64 oracle within 1e-11 max-abs."""
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.serving import ServingLoop
    reqs = W.serving_stream(n=6, rate_hz=400.0, seed=9, levels=(2,), precision=W.PREC_FP64)
    for r in reqs:
        r.problem = r.problem.replace(T=min(r.problem.T, 0.1))
    assert len({r.problem.d for r in reqs}) >= 2
    loop = ServingLoop(precision=B.FP64, max_active=3, hbm_budget=8 << 30, steps_per_tick=4, keep_outputs=True)
    res = loop.run(reqs)
    torch.cuda.synchronize()
    assert sorted(r.rid for r in res) == [r.rid for r in reqs]
    by_id = {r.rid: r for r in reqs}
    for r in res:
        pb = by_id[r.rid].problem
        U, _, _ = O.solve(pb)
        err = np.abs(r.out.cpu().numpy() - U).max()
        print(f"  request {r.rid} {pb.name} d={pb.d} nl={pb.nl}: fp64 max-abs {err:.2e}")
        assert err <= 1e-11, (r.rid, err)
    loop.close()


def test_admission_waits_for_memory_and_rejects_oversize():
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.serving import ServingLoop
    from paper_2007_10196_amd.solver import Plan
    reqs = _mixed_stream(n=8, seed=9, levels=(3,))
    fps = [Plan(r.problem).footprint for r in reqs]
    big = sorted(fps)[-2:]
    budget = int(big[1] + big[0] // 2)  # the two largest solves never fit together
    loop = ServingLoop(precision=B.FP32_SWEEP, max_active=8, hbm_budget=budget)
    res = loop.run(reqs)
    assert len(res) == len(reqs)
    # resident footprints never exceeded the budget (from the admit / finish stamps)
    fp_of = {q.rid: f for q, f in zip(reqs, fps)}
    events = sorted([(r.admit_s, 1, fp_of[r.rid]) for r in res] + [(r.finish_s, -1, fp_of[r.rid]) for r in res])
    resident, peak = 0, 0
    for _, kind, f in events:
        resident += kind * f
        peak = max(peak, resident)
    assert peak <= budget
    assert peak < sum(fps) and peak < big[0] + big[1]  # the two largest never ran at once
    loop.close()
    tiny = ServingLoop(precision=B.FP32_SWEEP, max_active=2, hbm_budget=min(fps) // 2)
    with pytest.raises(MemoryError):
        tiny.run(reqs[:1])
    tiny.close()


def test_admission_backfills_past_a_request_that_does_not_fit():
    """Three requests queued at once, the largest first: the second largest does not fit beside it,
    the smallest does.  With backfilling the smallest is admitted before the second largest; with a
    bypass bound of 0 admission keeps arrival order.  Every result is bitwise the same either way."""
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.serving import ServingLoop
    from paper_2007_10196_amd.solver import Plan
    pool = _mixed_stream(n=12, seed=9, levels=(3,))
    pool.sort(key=lambda r: Plan(r.problem).footprint)
    small, big2, big1 = pool[0], pool[-2], pool[-1]
    fp = {r.rid: Plan(r.problem).footprint for r in (small, big2, big1)}
    assert fp[big2.rid] > fp[small.rid]
    budget = fp[big1.rid] + fp[small.rid] + (fp[big2.rid] - fp[small.rid]) // 2
    reqs = [W.Request(rid=i, arrival_s=0.0, problem=r.problem, family=r.family)
            for i, r in enumerate((big1, big2, small))]
    runs = {}
    for bound in (10.0, 0.0):
        loop = ServingLoop(precision=B.FP32_SWEEP, max_active=8, hbm_budget=budget, keep_outputs=True,
                           max_bypass_s=bound)
        runs[bound] = {r.rid: r for r in loop.run(reqs)}
        loop.close()
    bf, fifo = runs[10.0], runs[0.0]
    assert bf[2].admit_s < bf[1].admit_s
    assert fifo[2].admit_s >= fifo[1].admit_s
    for rid in range(3):
        assert torch.equal(bf[rid].out, fifo[rid].out)


def test_autotuner_picks_and_caches(tmp_path):
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.autotune import tune_box_target
    probs = [W.c2_burgers_2d(nl=4, precision=W.PREC_FP32).replace(ic_params=(0.3, 0.7, math.pi, 0.1 * i))
             for i in range(16)]
    path = str(tmp_path / "tune.json")
    rec = tune_box_target(probs, B.FP32_SWEEP, candidates=(256, 1024), cache_path=path, reps=3,
                          blocks_per_cu=(0, 2))
    assert rec["best"] in (256, 1024) and rec["blocks_per_cu"] in (0, 2) and not rec["cached"]
    assert len(rec["us"]) == 4 and all(v > 0 for v in rec["us"].values())
    again = tune_box_target(probs, B.FP32_SWEEP, candidates=(256, 1024), cache_path=path, reps=3,
                            blocks_per_cu=(0, 2))
    assert again["cached"] and again["best"] == rec["best"] and again["blocks_per_cu"] == rec["blocks_per_cu"]


def test_serving_mix_with_a_4d_level5_request_equals_solo_bitwise():
    """A short FP32 stream with one 4D Vlasov request at finest level 5 (121 grids, a 256^4 FP64 finest
    grid of 34.4 GB that admission counts) among 2D/3D/4D requests at levels 2-3, full final times:
    every served solution equals the same solve run alone, bit for bit."""
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.serving import ServingLoop, latency_summary
    from paper_2007_10196_amd.solver import Plan, Solver
    reqs = W.serving_stream(n=6, rate_hz=200.0, seed=31, levels=(2, 3), precision=W.PREC_FP32)
    big = W.randomized(4, 5, np.random.default_rng(2007_10196 + 999), precision=W.PREC_FP32)
    reqs.append(W.Request(rid=6, arrival_s=reqs[2].arrival_s, problem=big, family=4))
    fp_big = Plan(big).footprint
    assert fp_big >= 256 ** 4 * 8  # the FP64 finest grid is counted
    loop = ServingLoop(precision=B.FP32_SWEEP, max_active=8, hbm_budget=fp_big + (8 << 30), steps_per_tick=8,
                       keep_outputs=True)
    print(f"\n[gpu] serving 7 requests incl. 4D N_L=5 ({fp_big / 1e9:.1f} GB footprint)", flush=True)
    res = loop.run(reqs)
    torch.cuda.synchronize()
    assert sorted(r.rid for r in res) == list(range(7))
    print("[gpu] serving", latency_summary(res), flush=True)
    by_id = {r.rid: r for r in reqs}
    for r in sorted(res, key=lambda x: x.rid):
        pb = by_id[r.rid].problem
        solo = Solver(pb).solve(mode=B.RUN_GRAPH)
        same = bool(torch.equal(r.out, solo))
        print(f"  request {r.rid} {pb.d}D N_L={pb.nl}: served == alone: {same}", flush=True)
        assert same, r.rid
        del solo
        r.out = None
        torch.cuda.empty_cache()
    loop.close()


def test_served_stream_at_full_final_time_fp64():
    """24 seeded requests at their full final times and levels 2-5 (one 4D N_L = 5), FP64, served with
    admissions while others run: members whose oracle solve is quick (2D, 3D up to N_L = 3, 4D up to
    N_L = 2) match the FP64 oracle within 1e-11 max-abs; every member equals its solve run alone, bit
    for bit."""
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.serving import ServingLoop, latency_summary
    from paper_2007_10196_amd.solver import Solver
    reqs = W.serving_stream(n=24, rate_hz=50.0, seed=119, precision=W.PREC_FP64)
    mix = [(r.problem.d, r.problem.nl) for r in reqs]
    assert (4, 5) in mix and (3, 5) in mix and len({r.family for r in reqs}) == 4
    loop = ServingLoop(precision=B.FP64, max_active=12, hbm_budget=64 << 30, steps_per_tick=8, keep_outputs=True)
    print(f"\n[gpu] serving 24 FP64 requests at full T: {sorted(mix)}", flush=True)
    res = loop.run(reqs)
    torch.cuda.synchronize()
    assert sorted(r.rid for r in res) == list(range(24))
    print("[gpu] serving", latency_summary(res), flush=True)
    by_id = {r.rid: r for r in reqs}
    checked = 0
    for r in sorted(res, key=lambda x: x.rid):
        pb = by_id[r.rid].problem
        if pb.d == 2 or (pb.d == 3 and pb.nl <= 3) or (pb.d == 4 and pb.nl <= 2):
            U, _, stats = O.solve(pb)
            assert r.steps == stats["steps"]
            err = float(np.abs(r.out.cpu().numpy() - U).max())
            print(f"  request {r.rid} {pb.d}D N_L={pb.nl}: max-abs vs oracle {err:.2e}", flush=True)
            assert err <= 1e-11, (r.rid, err)
            checked += 1
        solo = Solver(pb).solve(mode=B.RUN_GRAPH)
        assert bool(torch.equal(r.out, solo)), r.rid
        del solo
        r.out = None
        torch.cuda.empty_cache()
    assert checked >= 16
    loop.close()
