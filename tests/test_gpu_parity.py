"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

FP64 runs must match the oracle within 1e-11 max-abs on every component grid
and on the combined solution.  FP32-sweep runs report their L1/Linf error
against the FP64 oracle and must stay within the stated bound.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import sgw_inputs as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lib():
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.solver import Solver, Batch
    return torch, B, Solver, Batch


def _announce(what):
    print(f"\n[gpu] {what}", flush=True)


def gpu_solve(pb, mode=2, **kw):
    torch, B, Solver, _ = _lib()
    s = Solver(pb, **kw)
    s.restrict()
    s.advance(mode=mode)
    U = s.prolongate_combine()
    t, steps = s.query()
    state = s.state_copy().double().cpu().numpy().copy()
    return s, state, U, t, steps


def oracle_solve(pb):
    st = O.restrict(pb)
    stats = O.evolve(pb, st)
    U = O.prolong_combine(pb, st)
    return st, U, stats


def _check_fp64(pb, mode=2, tol=TOL64, **kw):
    _announce(f"{pb.name} d={pb.d} nr={pb.nr} nl={pb.nl} T={pb.T:.6g} mode={mode} kw={kw}")
    pb = pb.replace(precision=W.PREC_FP64)
    s, st_g, U_g, t_g, steps_g = gpu_solve(pb, mode, **kw)
    st_o, U_o, stats = oracle_solve(pb)
    assert steps_g == stats["steps"]
    assert abs(t_g - stats["t"]) < 1e-14
    assert np.max(np.abs(st_g - st_o)) <= tol
    U_g = U_g.cpu().numpy()
    assert np.max(np.abs(U_g - U_o)) <= tol
    return s, U_g, U_o, stats


# --------------------------------------------------------------------------- small, full oracle

@pytest.mark.parametrize("mode", [0, 1, 2])
def test_c1_full_size_all_modes(mode):
    _check_fp64(W.c1_advection_2d(), mode=mode)


SMALL = [
    ("c2_smooth_nl3", lambda: W.c2_burgers_2d(nl=3, T=0.5 / math.pi ** 2)),
    ("c2_steep_nl3", lambda: W.c2_burgers_2d(nl=3, T=1.5 / math.pi ** 2)),
    ("c2_shock_nl3", lambda: W.c2_burgers_2d(nl=3, T=0.30)),
    ("c3_nl3", lambda: W.c3_advection_3d(nl=3)),
    ("c3_nr5_ragged", lambda: W.c3_advection_3d(nr=5, nl=2, T=0.3)),
    ("c3_nr6_burgers", lambda: W.c3_advection_3d(nr=6, nl=2, T=0.2).replace(
        flux=W.FLUX_BURGERS, flux_params=(), ic_params=(0.3, 0.6, math.pi, 0.4))),
    ("c4_nl2", lambda: W.c4_vlasov_4d(nl=2, T=0.5)),
    ("single_grid_3d", lambda: W.c3_advection_3d(nr=16, nl=0, T=0.25)),
    ("one_dim_burgers", lambda: W.Problem(d=1, lo=(-1.0,), hi=(1.0,), flux=W.FLUX_BURGERS, flux_params=(),
                                          ic=W.IC_SINE, ic_params=(0.2, 0.8, math.pi, 0.0), nr=12, nl=4,
                                          T=0.4)),
    ("linear_lagrange_ex1", lambda: W.paper_example1(40, nr=10, nl=2)),
    ("pow53_ex3a", lambda: W.paper_example3a(40, nr=10, nl=2)),
    ("negative_speed", lambda: W.c3_advection_3d(nl=2, T=0.3).replace(flux_params=(-1.0, 0.5, -0.25))),
]


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_small_configs_fp64(name, make):
    _check_fp64(make())


@pytest.mark.parametrize("name,make", [s for s in SMALL if s[0].startswith(("c3", "single_grid_3d", "negative"))],
                         ids=[s[0] for s in SMALL if s[0].startswith(("c3", "single_grid_3d", "negative"))])
def test_small_3d_configs_as_stage_boxes_fp64(name, make):
    """The 3D configurations with stage boxes (sweep_form 2) instead of the default line sweeps."""
    _check_fp64(make(), sweep_form=2)


@pytest.mark.parametrize("prec", [0, 1])
def test_3d_sweep_forms_give_the_same_bits(prec):
    """3D: line sweeps with the plane launch (default), one line launch per direction, and stage
    boxes give the same bits, in a solve and in a batch."""
    torch, B, Solver, Batch = _lib()
    pb = W.c3_advection_3d(nr=8, nl=3, T=0.2, precision=prec).replace(
        flux=W.FLUX_BURGERS, flux_params=(), ic_params=(0.3, 0.6, math.pi, 0.4))
    outs = {}
    for sf in (0, 1, 2):
        _announce(f"3D sweep form {sf} precision {prec}")
        outs[sf] = Solver(pb, sweep_form=sf).solve().cpu().numpy()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    for sf in (0, 2):
        batch = Batch(max_solvers=2, precision=B.FP64 if prec == 0 else B.FP32_SWEEP, hbm_budget=1 << 34)
        s = Solver(pb, sweep_form=sf)
        s.restrict()
        slot = batch.admit(s)
        other = Solver(pb, sweep_form=2 - sf)
        other.restrict()
        with pytest.raises(B.SgwError) as e:
            batch.admit(other)
        assert e.value.status == -2
        for _ in range(200):
            batch.step(8)
            if slot in batch.poll():
                break
        batch.release(slot)
        assert np.array_equal(s.prolongate_combine().cpu().numpy(), outs[0])
        batch.close()


def test_boxes_smaller_than_the_automatic_choice():
    # several boxes per grid, halos in every direction, odd box extents
    _check_fp64(W.c3_advection_3d(nr=6, nl=2, T=0.2), box=[3, 3, 3])
    _check_fp64(W.c2_burgers_2d(nl=3, T=0.1), box=[4, 4], fine_tile=[8, 4])


def _four_d_cases(prec):
    """4D workloads with each kind of flux: the Vlasov one (coefficients per line), advection with
    unequal speeds of both signs (constant coefficients) and Burgers (state-dependent wave speed)."""
    adv = W.Problem(d=4, lo=(0.0,) * 4, hi=(2.0,) * 4, flux=W.FLUX_ADVECTION, flux_params=(1.0, -0.5, 0.75, 0.25),
                    ic=W.IC_SINE, ic_params=(0.1, 1.0, math.pi, 0.3), nr=8, nl=2, T=0.05, cfl=0.5,
                    precision=prec, name="advection_4d")
    burg = adv.replace(flux=W.FLUX_BURGERS, flux_params=(), ic_params=(0.3, 0.7, math.pi, 0.0), name="burgers_4d")
    return [W.c4_vlasov_4d(nl=2, T=0.1, precision=prec), adv, burg, adv.replace(nr=5, nl=1, name="advection_4d_nr5")]


def test_4d_line_sweep_equals_box_kernel_bitwise():
    """4D grids march as line sweeps (one launch per direction, no halo, partial sums in a free state
    copy); manual stage boxes select the box kernel, which stages halo slabs in LDS.  Both give the
    same bits on every component grid and on the combined solution, FP64 and FP32, and the FP64
    line sweep matches the oracle."""
    for prec in (W.PREC_FP64, W.PREC_FP32):
        for pb in _four_d_cases(prec):
            _announce(f"4D line sweep vs boxes {pb.name} nr={pb.nr} nl={pb.nl} precision={prec}")
            s_l, st_l, U_l, t_l, n_l = gpu_solve(pb)
            s_b, st_b, U_b, t_b, n_b = gpu_solve(pb, box=[4, 4, 4, 2] if pb.nr % 4 == 0 else [5, 5, 5, 5])
            assert n_l == n_b and t_l == t_b
            assert np.array_equal(st_l, st_b)
            assert bool((U_l == U_b).all())
            if prec == W.PREC_FP64 and pb.name != "advection_4d_nr5":
                st_o, U_o, stats = oracle_solve(pb)
                assert n_l == stats["steps"]
                assert np.max(np.abs(st_l - st_o)) <= TOL64
                assert np.max(np.abs(U_l.cpu().numpy() - U_o)) <= TOL64


def test_4d_plane_launch_equals_four_line_launches_bitwise():
    """4D stages run directions 1 and 2 in one launch over whole (x_1, x_2) planes in LDS, then line
    sweeps for directions 3 and 4 (sweep_form 0); sweep_form 1 runs four line sweeps.  The two give
    the same bits for every flux kind, linear weights, zero boundaries with relaxation, FP64 and FP32,
    in the graph and the per-grid modes."""
    cases = []
    for prec in (W.PREC_FP64, W.PREC_FP32):
        cases += [(pb, 2) for pb in _four_d_cases(prec)]
        cases.append((W.paper_example5(4, nr=4, nl=2, T=0.1, precision=prec), 2))
    cases.append((W.c4_vlasov_4d(nl=2, T=0.1, precision=W.PREC_FP64).replace(linear=True), 2))
    cases.append((W.c4_vlasov_4d(nl=2, T=0.1, precision=W.PREC_FP64), 0))
    for pb, mode in cases:
        _announce(f"4D plane launch vs line launches {pb.name} nr={pb.nr} nl={pb.nl} precision={pb.precision} "
                  f"mode={mode}")
        _, st_p, U_p, t_p, n_p = gpu_solve(pb, mode)
        _, st_l, U_l, t_l, n_l = gpu_solve(pb, mode, sweep_form=1)
        assert n_p == n_l and t_p == t_l
        assert np.array_equal(st_p, st_l)
        assert bool((U_p == U_l).all())


def test_paper_sparse_weno_row_on_gpu():
    # Table ex3aweno, sparse grid with WENO prolongation, N_r = 10, N_L = 3 (N_h = 80)
    pb = W.paper_example3a(80, nr=10, nl=3)
    s, U_g, U_o, stats = _check_fp64(pb)
    torch, *_ = _lib()
    ex = s.exact(stats["t"])
    l1, li = s.norms(torch.from_numpy(U_g).cuda(), ex)
    assert l1 == pytest.approx(7.1354e-05, rel=2e-4)
    assert li == pytest.approx(5.4916e-04, rel=2e-4)


@pytest.mark.parametrize("make,nh,nl,paper_l1", [
    (W.paper_example3a, 320, 0, 1.3119e-09), (W.paper_example3a, 320, 3, 1.3265e-09),
    (W.paper_example3a, 640, 0, 4.0883e-11), (W.paper_example3a, 640, 3, 4.0784e-11),
    (W.paper_example3b, 160, 0, 6.6687e-08), (W.paper_example3b, 160, 3, 7.6655e-07),
    (W.paper_example3b, 320, 3, 2.4830e-09)])
def test_paper_rows_beyond_the_oracle_on_gpu(make, nh, nl, paper_l1):
    """Rows of Tables ex3aweno (2D) and ex3-baweno (3D) at resolutions the oracle does not run in a
    test: the GPU's FP64 L1 against the exact solution matches the printed value (the 640 rows to the
    paper's rounding floor)."""
    torch, B, Solver, _ = _lib()
    pb = make(nh, nl=nl)
    _announce(f"{pb.name} N_h={nh} N_L={nl}")
    s = Solver(pb)
    U = s.solve(mode=B.RUN_GRAPH)
    t, steps = s.query()
    l1, _ = s.norms(U, s.exact(t))
    print(f"  L1 {l1:.5e} (printed {paper_l1:.4e})", flush=True)
    assert l1 == pytest.approx(paper_l1, rel=5e-4 if nh == 640 else 2e-4)


def test_exact_and_norms_match_oracle():
    torch, *_ = _lib()
    for pb in (W.c2_burgers_2d(nl=3, T=0.1, precision=0), W.c3_advection_3d(nl=2, T=0.4, precision=0),
               W.c4_vlasov_4d(nl=1, T=0.3, precision=0)):
        _announce(f"exact {pb.name}")
        s, st, U, t, steps = gpu_solve(pb)
        ex_g = s.exact(t)
        ex_o = O.exact_fine(pb, t)
        assert np.max(np.abs(ex_g.cpu().numpy() - ex_o)) < 1e-13
        l1g, lig = s.norms(U, ex_g)
        l1o, lio = O.norms(U.cpu().numpy(), ex_o)
        assert l1g == pytest.approx(l1o, rel=1e-12, abs=1e-300)
        assert lig == pytest.approx(lio, rel=1e-12, abs=1e-300)


# --------------------------------------------------------------------------- benchmark workload (2D Burgers)

@pytest.mark.parametrize("T", [0.5 / math.pi ** 2, 1.5 / math.pi ** 2])
def test_c2_full_size(T):
    pb = W.c2_burgers_2d(T=T)
    _check_fp64(pb)
    # FP32 sweeps, FP64 combination, as benchmarked: error against the FP64 oracle
    _announce(f"c2 fp32 T={T}")
    s, st32, U32, t32, steps32 = gpu_solve(pb.replace(precision=W.PREC_FP32))
    st_o, U_o, stats = oracle_solve(pb.replace(precision=W.PREC_FP64))
    e = np.abs(U32.cpu().numpy() - U_o)
    print(f"  c2 T={T:.4f}: fp32 L1 {e.mean():.3e} Linf {e.max():.3e} against the fp64 oracle")
    assert e.mean() < 2e-6 and e.max() < 2e-5, (e.mean(), e.max())


def test_fp32_errors_are_reported_and_bounded():
    for pb in (W.c1_advection_2d(), W.c3_advection_3d(nl=3), W.c4_vlasov_4d(nl=2, T=0.5)):
        _announce(f"fp32 {pb.name}")
        s, st, U, t, steps = gpu_solve(pb.replace(precision=W.PREC_FP32))
        st_o, U_o, stats = oracle_solve(pb.replace(precision=W.PREC_FP64))
        scale = max(1.0, np.max(np.abs(U_o)))
        e = np.abs(U.cpu().numpy() - U_o)
        print(f"  {pb.name}: fp32 L1 {e.mean():.3e} Linf {e.max():.3e}")
        assert e.max() < 5e-5 * scale


# --------------------------------------------------------------------------- full sizes, sampled

def _golden(name):
    path = os.path.join(GOLDEN, f"oracle_{name}_full.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("name,make", [("c3", lambda: W.c3_advection_3d(precision=0)),
                                       ("c4", lambda: W.c4_vlasov_4d(precision=0))])
def test_full_size_sampled(name, make):
    gd = _golden(name)
    pb = make()
    assert gd["eps_flux"] == pb.eps_flux and gd["nl"] == pb.nl and gd["nr"] == pb.nr
    _announce(f"full {name}")
    s, st, U, t, steps = gpu_solve(pb)
    assert steps == gd["steps"]
    for g in gd["grids"]:
        vals = st[g["offset"] + np.array(g["idx"])]
        assert np.max(np.abs(vals - np.array(g["val"]))) <= TOL64
        n = int(np.prod(g["shape"]))
        assert abs(st[g["offset"]:g["offset"] + n].sum() - g["sum"]) <= TOL64 * n
    J = np.array(gd["fine_J"])
    N = pb.n_fine
    flat = sum(J[:, k] * N ** k for k in range(pb.d))
    Ug = U.cpu().numpy()[flat]
    assert np.max(np.abs(Ug - np.array(gd["fine_val"]))) <= TOL64
    ex = s.exact(t).cpu().numpy()[flat]
    assert np.max(np.abs(ex - np.array(gd["fine_exact"]))) < 1e-13


@pytest.mark.parametrize("name,make", [("2d", lambda: W.c2_burgers_2d(nl=4, precision=0)),
                                       ("3d", lambda: W.c3_advection_3d(nr=8, nl=3, precision=1)),
                                       ("4d", lambda: W.c4_vlasov_4d(nl=3, precision=0))])
def test_prolongation_over_tile_ranges_equals_one_call(name, make):
    """sgw_prolongate_combine_tiles over uneven ranges that cover every finest-grid tile once (an
    empty range among them) gives sgw_prolongate_combine's output bitwise, leaves the entries of
    other tiles untouched, and refuses ranges outside 0..count."""
    torch, B, Solver, _ = _lib()
    pb = make()
    _announce(f"tile ranges {name}")
    s = Solver(pb)
    noise = W.component_noise(s.plan.total_nodes, seed=23)
    dev = torch.from_numpy(noise).cuda()
    for g, info in enumerate(s.plan.grids):
        n = int(np.prod(info["shape"]))
        s.set_grid(g, dev[info["offset"]: info["offset"] + n].to(dtype=s.real))
    whole = s.prolongate_combine()
    nt = s.plan.fine_tile_count
    assert nt == s.plan.fine_nodes // int(np.prod(s.plan.fine_tile))
    out = torch.full_like(whole, float("nan"))
    cuts = sorted({0, nt, 1, nt // 3, nt // 3, nt // 2 + 1, nt - 1})
    cuts = [c for c in cuts if 0 <= c <= nt]
    first_part = None
    for a, b in zip(cuts[:-1], cuts[1:]):
        s.prolongate_combine_tiles(out, a, b - a)
        if first_part is None:
            torch.cuda.synchronize()
            first_part = int(torch.isnan(out).sum().item())
    s.prolongate_combine_tiles(out, nt // 3, 0)
    torch.cuda.synchronize()
    assert first_part == (nt - cuts[1]) * int(np.prod(s.plan.fine_tile))
    assert torch.equal(out, whole)
    for a, n in ((-1, 1), (0, nt + 1), (nt, 1), (2, -1)):
        with pytest.raises(B.SgwError) as e:
            s.prolongate_combine_tiles(out, a, n)
        assert e.value.status == -1


@pytest.mark.parametrize("name,make", [("c3", lambda: W.c3_advection_3d(precision=0)),
                                       ("c4", lambda: W.c4_vlasov_4d(precision=0))])
def test_full_size_prolongation_whole_tiles(name, make):
    """The prolongation and combination at full size, in the finest-grid tile shape the planner picks
    for the bench: every component grid holds seeded noise (set through sgw_set_grid), and whole
    tiles of the output -- the corner tile (periodic wrap in every direction), the far-corner tile
    and two interior ones, their corners and edges included -- match the oracle's pointwise
    prolongation of the same values within 1e-11."""
    torch, B, Solver, _ = _lib()
    pb = make()
    s = Solver(pb)
    noise = W.component_noise(s.plan.total_nodes, seed=2007_10196 + 17)
    dev = torch.from_numpy(noise).cuda()
    for g, info in enumerate(s.plan.grids):
        n = int(np.prod(info["shape"]))
        s.set_grid(g, dev[info["offset"]: info["offset"] + n].clone())
    U = s.prolongate_combine()
    torch.cuda.synchronize()
    T = s.plan.fine_tile
    N = pb.n_fine
    ntile = [N // t for t in T]
    rng = np.random.default_rng(2007_10196 + 18)
    picks = [[0] * pb.d, [n - 1 for n in ntile], [int(rng.integers(1, n - 1)) for n in ntile],
             [int(rng.integers(1, n - 1)) for n in ntile]]
    local = np.stack(np.meshgrid(*[np.arange(t) for t in T], indexing="ij"), -1).reshape(-1, pb.d)
    for tile in picks:
        J = (local + np.array(tile) * np.array(T)).astype(np.int32)
        _announce(f"full {name} tile {tile} of shape {T}: {len(J)} nodes")
        flat = torch.from_numpy(sum(J[:, k].astype(np.int64) * N ** k for k in range(pb.d))).cuda()
        got = U[flat].cpu().numpy()
        ref = O.prolong_combine_points(pb, noise, J)
        err = float(np.max(np.abs(got - ref)))
        print(f"  max-abs {err:.2e}", flush=True)
        assert err <= TOL64, (tile, err)


@pytest.mark.parametrize("name,make", [("c3", lambda: W.c3_advection_3d(precision=1)),
                                       ("c4", lambda: W.c4_vlasov_4d(precision=1))])
def test_full_size_fp32_against_fp64_oracle_samples(name, make):
    """FP32 sweeps + FP64 combination at the full sizes: the sampled finest-grid values stay within
    a stated bound of the FP64 oracle (the error is reported)."""
    gd = _golden(name)
    pb = make()
    _announce(f"full {name} fp32")
    s, st, U, t, steps = gpu_solve(pb)
    J = np.array(gd["fine_J"])
    N = pb.n_fine
    flat = sum(J[:, k] * N ** k for k in range(pb.d))
    ref = np.array(gd["fine_val"])
    e = np.abs(U.cpu().numpy()[flat] - ref)
    scale = max(1e-300, np.max(np.abs(ref)))
    print(f"  {name} fp32 vs fp64 oracle on {len(ref)} samples: L1 {e.mean():.3e} Linf {e.max():.3e} "
          f"(max |u| {scale:.3e})")
    assert abs(steps - gd["steps"]) <= 1
    assert e.max() <= 1e-4 * scale


# --------------------------------------------------------------------------- batching and determinism

def test_batched_results_equal_solo_results_bitwise():
    torch, B, Solver, Batch = _lib()
    rng = np.random.default_rng(5)
    probs = [W.randomized(f, nl, rng, precision=W.PREC_FP32) for f, nl in
             [(1, 3), (2, 3), (3, 2), (4, 2), (2, 4), (3, 3)]]
    probs = [p.replace(T=min(p.T, 0.2)) for p in probs]
    solo = []
    for p in probs:
        _announce(f"solo {p.name} nl={p.nl}")
        s = Solver(p)
        solo.append(s.solve(mode=B.RUN_GRAPH).cpu().numpy())
    _announce("batch")
    batch = Batch(max_solvers=8, precision=B.FP32_SWEEP, hbm_budget=1 << 34)
    solvers = []
    for p in probs:
        s = Solver(p)
        s.restrict()
        batch.admit(s)
        solvers.append(s)
    done = set()
    for _ in range(400):
        batch.step(8)
        done |= set(batch.poll())
        if len(done) == len(probs):
            break
    assert len(done) == len(probs)
    for s, ref in zip(solvers, solo):
        U = s.prolongate_combine().cpu().numpy()
        assert np.array_equal(U, ref)
    for slot in list(batch.slots):
        batch.release(slot)


def test_pipelined_polls_and_multi_step_graphs_match_single_steps():
    """Steps queued in runs (8-step graphs plus single ones) with the completion flags
    polled while the next steps run give the same solutions as one step per poll."""
    torch, B, Solver, Batch = _lib()
    rng = np.random.default_rng(11)
    probs = [W.randomized(f, nl, rng, precision=W.PREC_FP64) for f, nl in [(1, 3), (2, 3), (3, 2)]]
    probs = [p.replace(T=min(p.T, 0.15)) for p in probs]

    def run(pipelined):
        _announce(f"batch pipelined={pipelined}")
        batch = Batch(max_solvers=4, precision=B.FP64, hbm_budget=1 << 34)
        solvers = []
        for p in probs:
            s = Solver(p)
            s.restrict()
            batch.admit(s)
            solvers.append(s)
        done = set()
        if pipelined:
            with pytest.raises(B.SgwError):
                batch.poll_end()  # nothing in flight
            batch.step(13)
            batch.poll_begin()
            with pytest.raises(B.SgwError):
                batch.poll_begin()  # one poll at a time
            for _ in range(400):
                batch.step(3)
                done |= set(batch.poll_end())
                if len(done) == len(probs):
                    break
                batch.poll_begin()
        else:
            for _ in range(4000):
                batch.step(1)
                done |= set(batch.poll())
                if len(done) == len(probs):
                    break
        assert len(done) == len(probs)
        out = [(s.query()[1], s.prolongate_combine().cpu().numpy()) for s in solvers]
        batch.release_many(list(batch.slots))
        batch.close()
        return out

    a, b = run(False), run(True)
    for (sa, ua), (sb, ub) in zip(a, b):
        assert sa == sb
        assert np.array_equal(ua, ub)


def test_repeat_runs_are_bitwise_identical():
    pb = W.c2_burgers_2d(nl=4, T=0.1, precision=W.PREC_FP64)
    a = gpu_solve(pb)[2].cpu().numpy()
    b = gpu_solve(pb)[2].cpu().numpy()
    assert np.array_equal(a, b)


def test_non_finite_wave_speed_is_reported():
    torch, B, Solver, _ = _lib()
    pb = W.c2_burgers_2d(nl=2, T=0.05).replace(ic_params=(float("nan"), 0.7, math.pi, 0.0))
    s = Solver(pb)
    s.restrict()
    with pytest.raises(B.SgwError) as e:
        s.advance()
    assert e.value.status == -4


def test_advance_before_restrict_is_refused():
    torch, B, Solver, _ = _lib()
    s = Solver(W.c1_advection_2d())
    with pytest.raises(B.SgwError) as e:
        s.advance()
    assert e.value.status == -6


def test_batched_prolongation_and_async_norms_match_single_calls():
    torch, B, Solver, _ = _lib()
    from paper_2007_10196_amd.solver import prolongate_combine_many
    rng = np.random.default_rng(11)
    for fam, nl in ((2, 3), (3, 2), (4, 2)):
        probs = [W.randomized(fam, nl, rng, precision=W.PREC_FP32) for _ in range(3)]
        probs = [p.replace(T=min(p.T, 0.1)) for p in probs]
        solvers = [Solver(p) for p in probs]
        singles = []
        for s in solvers:
            s.restrict()
            s.advance()
            singles.append(s.prolongate_combine())
        outs = [torch.empty_like(u) for u in singles]
        prolongate_combine_many(solvers, outs)
        res = torch.zeros((len(solvers), 2), dtype=torch.float64, device="cuda")
        for i, s in enumerate(solvers):
            assert torch.equal(outs[i], singles[i])
            ex = s.exact(s.query()[0])
            s.norms_async(outs[i], ex, res[i])
            l1, li = s.norms(singles[i], ex)
            torch.cuda.synchronize()
            assert res[i, 0].item() == l1 and res[i, 1].item() == li


def test_restrict_many_and_norms_many_match_single_calls():
    """One-launch restriction and norms over solves of mixed dimension equal the per-solve calls bitwise;
    a used solver restricted again starts from t = 0 with cleared wave speeds."""
    torch, B, Solver, _ = _lib()
    from paper_2007_10196_amd.solver import norms_many, restrict_many
    rng = np.random.default_rng(23)
    for prec in (W.PREC_FP32, W.PREC_FP64):
        _announce(f"restrict_many / norms_many precision {prec}")
        probs = [W.randomized(fam, nl, rng, precision=prec) for fam, nl in ((1, 3), (2, 4), (3, 2), (4, 2), (2, 2))]
        probs = [p.replace(T=min(p.T, 0.05)) for p in probs]
        single = [Solver(p) for p in probs]
        many = [Solver(p) for p in probs]
        for s in many:  # leave state, time and wave speeds behind, to be reset
            s.restrict()
            s.advance()
        outs_s, outs_m = [], []
        for s in single:
            s.restrict()
        restrict_many(many)
        for a, b in zip(single, many):
            assert torch.equal(a.state_copy(0), b.state_copy(0))
            assert b.query() == (0.0, 0)
        for a, b in zip(single, many):
            a.advance()
            b.advance()
            assert a.query() == b.query()
            outs_s.append(a.prolongate_combine())
            outs_m.append(b.prolongate_combine())
            assert torch.equal(outs_s[-1], outs_m[-1])
        exacts = [s.exact(s.query()[0]) for s in single]
        res = torch.full((len(many), 2), -1.0, dtype=torch.float64, device="cuda")
        norms_many(many, outs_m, exacts, res)
        for i, s in enumerate(single):
            l1, li = s.norms(outs_s[i], exacts[i])
            assert res[i, 0].item() == l1 and res[i, 1].item() == li
            assert 0.0 < l1 <= li


def test_pointer_lists_marshalled_once_match_plain_lists():
    """The many-solve calls and admit_many take PtrLists (pointer arrays built once) with the same
    results as plain lists, bitwise, on two calls in a row."""
    torch, B, Solver, Batch = _lib()
    from paper_2007_10196_amd.solver import PtrList, norms_many, prolongate_combine_many, restrict_many
    rng = np.random.default_rng(31)
    probs = [W.randomized(2, 3, rng, precision=W.PREC_FP32).replace(T=0.05) for _ in range(4)]
    ref = []
    for p in probs:
        s = Solver(p)
        s.restrict()
        s.advance()
        ref.append(s.prolongate_combine())
    solvers = [Solver(p) for p in probs]
    outs = [torch.empty_like(u) for u in ref]
    exacts = [s.exact(p.T) for s, p in zip(solvers, probs)]
    pl_s, pl_o, pl_e = PtrList(solvers), PtrList(outs), PtrList(exacts)
    assert len(pl_s) == 4 and pl_s[1] is solvers[1] and list(pl_o) == outs
    batch = Batch(max_solvers=4, precision=B.FP32_SWEEP, hbm_budget=1 << 32)
    for rep in range(2):
        _announce(f"ptrlist call {rep}")
        for o in outs:
            o.fill_(-1.0)
        restrict_many(pl_s, stream=batch.stream)
        batch.admit_many(pl_s)
        done = set()
        for _ in range(200):
            batch.step(4)
            done |= set(batch.poll())
            if len(done) == 4:
                break
        assert len(done) == 4
        batch.release_many(list(batch.slots))
        prolongate_combine_many(pl_s, pl_o, stream=batch.stream)
        res = torch.full((4, 2), -1.0, dtype=torch.float64, device="cuda")
        norms_many(pl_s, pl_o, pl_e, res, stream=batch.stream)
        res_plain = torch.full((4, 2), -1.0, dtype=torch.float64, device="cuda")
        norms_many(solvers, outs, exacts, res_plain, stream=batch.stream)
        torch.cuda.synchronize()
        for i in range(4):
            assert torch.equal(outs[i], ref[i])
        assert torch.equal(res, res_plain)
    batch.close()


def test_release_many_orders_solver_streams_after_queued_steps():
    """Solvers on two side streams, released while steps are still queued, prolongate on their own
    streams at once: release_many's single event makes both streams wait, so the results equal a run
    that synchronises before releasing, bitwise."""
    torch, B, Solver, Batch = _lib()
    from paper_2007_10196_amd.solver import restrict_many
    rng = np.random.default_rng(37)
    probs = [W.randomized(2, 4, rng, precision=W.PREC_FP32).replace(T=1.0) for _ in range(4)]
    results = []
    for sync in (True, False):
        _announce(f"release ordering sync={sync}")
        side = [torch.cuda.Stream(), torch.cuda.Stream()]
        solvers = [Solver(p, stream=side[i % 2]) for i, p in enumerate(probs)]
        batch = Batch(max_solvers=4, precision=B.FP32_SWEEP, hbm_budget=1 << 32)
        restrict_many(solvers, stream=batch.stream)
        batch.admit_many(solvers)
        batch.step(6)
        if sync:
            torch.cuda.synchronize()
        batch.release_many(sorted(batch.slots))
        outs = []
        for s in solvers:
            with torch.cuda.stream(s.stream):
                outs.append(s.prolongate_combine())
        torch.cuda.synchronize()
        assert all(s.query()[1] == 6 for s in solvers)
        results.append(outs)
        batch.close()
    for a, b in zip(*results):
        assert torch.equal(a, b)


def test_poll_in_flight_skips_a_slot_refilled_by_the_same_solver():
    """Flags gathered before a slot is released and refilled, even by the same solver, are not
    reported for it; the refilled solve then runs to the same result as a solo solve.  The solver
    sits on its own stream, so admission orders the batch after its restriction by an event."""
    torch, B, Solver, Batch = _lib()
    rng = np.random.default_rng(41)
    p = W.randomized(2, 3, rng, precision=W.PREC_FP32).replace(T=0.05)
    solo = Solver(p)
    solo.restrict()
    solo.advance()
    ref = solo.prolongate_combine()
    side = torch.cuda.Stream()
    s = Solver(p, stream=side)
    batch = Batch(max_solvers=2, precision=B.FP32_SWEEP, hbm_budget=1 << 32)
    s.restrict()
    slot = batch.admit(s)
    done = []
    for _ in range(400):
        batch.step(4)
        done = batch.poll()
        if done:
            break
    assert done == [slot]
    _announce("poll in flight across release and re-admission")
    batch.poll_begin()
    batch.release(slot)
    s.restrict()
    assert batch.admit(s) == slot
    assert batch.poll_end() == []
    done = []
    for _ in range(400):
        batch.step(4)
        done = batch.poll()
        if done:
            break
    assert done == [slot]
    batch.release(slot)
    with torch.cuda.stream(side):
        out = s.prolongate_combine()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    batch.close()


def test_many_solve_calls_order_solver_streams_both_ways():
    """restrict_many and prolongate_combine_many on a third stream, with no host synchronisation:
    the solvers' own streams (two side streams) run their advance after the restriction, and a
    restriction enqueued on them right after the prolongation does not disturb it."""
    torch, B, Solver, _ = _lib()
    from paper_2007_10196_amd.solver import prolongate_combine_many, restrict_many
    rng = np.random.default_rng(43)
    probs = [W.randomized(2, 4, rng, precision=W.PREC_FP32).replace(T=0.05) for _ in range(4)]
    ref = []
    for p in probs:
        s = Solver(p)
        s.restrict()
        s.advance()
        ref.append(s.prolongate_combine())
    side = [torch.cuda.Stream(), torch.cuda.Stream()]
    call = torch.cuda.Stream()
    solvers = [Solver(p, stream=side[i % 2]) for i, p in enumerate(probs)]
    outs = [torch.empty_like(u) for u in ref]
    _announce("many-solve calls across three streams")
    restrict_many(solvers, stream=call)
    for s in solvers:
        s.advance()
    prolongate_combine_many(solvers, outs, stream=call)
    for s in solvers:
        s.restrict()
    torch.cuda.synchronize()
    for a, b in zip(outs, ref):
        assert torch.equal(a, b)


def test_bench_configuration_against_fp64_oracle_samples():
    """The benchmark's own step (256 batched 2D Burgers solves, FP32 sweeps, box target 2048 and
    7 workgroups per CU, as bench.py times it): four of the 256 combined solutions, spread over the
    batch, are within the FP32 bounds of the FP64 oracle, and the device norms equal the norms of
    the returned solutions."""
    torch, B, Solver, Batch = _lib()
    import bench
    from paper_2007_10196_amd.solver import PtrList
    probs = bench.make_problems(256)
    solvers = [Solver(p, device="cuda:0", box_target=2048) for p in probs]
    fine = solvers[0].plan.fine_nodes
    outs = [torch.empty(fine, dtype=torch.float64, device="cuda:0") for _ in solvers]
    exacts = [s.exact(bench.T_FINAL) for s in solvers]
    res = torch.zeros((256, 2), dtype=torch.float64, device="cuda:0")
    S, O_, E = PtrList(solvers), PtrList(outs), PtrList(exacts)
    sent = bench.StepNorms(torch, res)
    batch = Batch(max_solvers=256, precision=B.FP32_SWEEP, hbm_budget=sum(s.plan.footprint for s in solvers) + (1 << 30),
                  max_items=sum(len(s.plan.grids) * 64 for s in solvers))
    batch.set_blocks_per_cu(7)
    _announce("bench step, 256 solves")
    bench.run_batch_step(torch, batch, S, O_, E, res, sent)
    norms = sent.take()
    torch.cuda.synchronize()
    for i in (0, 85, 170, 255):
        _announce(f"oracle solve {i}")
        st_o, U_o, stats = oracle_solve(probs[i].replace(precision=W.PREC_FP64))
        U = outs[i].cpu().numpy()
        e = np.abs(U - U_o)
        print(f"  solve {i}: fp32 L1 {e.mean():.3e} Linf {e.max():.3e} against the fp64 oracle")
        assert e.mean() < 2e-6 and e.max() < 2e-5, (i, e.mean(), e.max())
        ex = exacts[i].cpu().numpy()
        assert abs(norms[i, 0] - np.abs(U - ex).mean()) <= 1e-12 * max(1.0, norms[i, 0])
        assert norms[i, 1] == np.abs(U - ex).max()
    batch.release_many(list(batch.slots))
    batch.close()


def test_valu_calibration_hook_runs_every_class():
    """The issue-rate measurement hook launches each instruction class and reports the wave64
    instructions per SIMD that its timing is divided by."""
    import ctypes as C
    torch, B, _, _ = _lib()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = torch.empty(cus * 256 * 8, dtype=torch.uint8, device="cuda")
    for op in range(5):
        n = C.c_double()
        B.check(B.lib().sgw_calibrate_valu(op, cus, C.c_void_p(out.data_ptr()), None, C.byref(n)))
        torch.cuda.synchronize()
        assert n.value == cus * 4 * 4096 * (16 if op == 3 else 8) / (4.0 * cus)


def test_restrict_many_rejects_mixed_precision():
    torch, B, Solver, _ = _lib()
    from paper_2007_10196_amd.solver import restrict_many
    a = Solver(W.c1_advection_2d())
    b = Solver(W.c1_advection_2d().replace(precision=W.PREC_FP32))
    with pytest.raises(B.SgwError) as e:
        restrict_many([a, b])
    assert e.value.status == -1


def test_batch_admit_many_and_release_many():
    """Many-solver admission equals one-by-one admission (bitwise results); a refused solver stops the
    list with the earlier ones admitted; release_many rejects a repeated slot before releasing any."""
    torch, B, Solver, Batch = _lib()
    from paper_2007_10196_amd.solver import restrict_many
    rng = np.random.default_rng(5)
    probs = [W.randomized(2, 3, rng, precision=W.PREC_FP32) for _ in range(6)]
    ref = []
    for p in probs:
        s = Solver(p)
        s.restrict()
        s.advance()
        ref.append(s.prolongate_combine())
    solvers = [Solver(p) for p in probs]
    restrict_many(solvers)
    fp = [s.plan.footprint for s in solvers]
    batch = Batch(max_solvers=8, precision=B.FP32_SWEEP, hbm_budget=sum(fp[:4]) + fp[4] // 2)
    with pytest.raises(B.SgwError) as e:
        batch.admit_many(solvers)
    assert e.value.status == -3 and len(batch.slots) == 4
    with pytest.raises(B.SgwError) as e:
        batch.release_many([0, 0])
    assert e.value.status == -1 and len(batch.slots) == 4
    batch.release_many(sorted(batch.slots))
    assert not batch.slots
    big = Batch(max_solvers=8, precision=B.FP32_SWEEP, hbm_budget=sum(fp) + (1 << 20))
    restrict_many(solvers)
    slots = big.admit_many(solvers)
    assert sorted(slots) == list(range(6))
    done = set()
    while len(done) < 6:
        big.step(4)
        done |= set(big.poll())
    big.release_many(slots)
    for s, r in zip(solvers, ref):
        assert torch.equal(s.prolongate_combine(), r)


@pytest.mark.parametrize("prec", [W.PREC_FP32, W.PREC_FP64])
def test_launch_shape_does_not_change_results(prec):
    """Box target (box decomposition) and workgroups per CU change only who computes each interface
    flux, not the arithmetic: batched results are bitwise identical across launch shapes."""
    torch, B, Solver, Batch = _lib()
    from paper_2007_10196_amd.solver import restrict_many
    rng = np.random.default_rng(31)
    probs = [W.randomized(fam, nl, rng, precision=prec) for fam, nl in ((2, 4), (3, 3), (4, 2), (1, 4))]
    probs = [p.replace(T=min(p.T, 0.05)) for p in probs]
    outs = []
    for target, bpc in ((256, 0), (1024, 3), (2048, 7)):
        _announce(f"launch shape target {target} bpc {bpc} prec {prec}")
        solvers = [Solver(p, box_target=target) for p in probs]
        batch = Batch(max_solvers=8, precision=prec, hbm_budget=1 << 40)
        batch.set_blocks_per_cu(bpc)
        restrict_many(solvers)
        batch.admit_many(solvers)
        done = set()
        while len(done) < len(solvers):
            batch.step(4)
            done |= set(batch.poll())
        batch.release_many(sorted(batch.slots))
        outs.append([s.prolongate_combine() for s in solvers])
    bad = []
    for j, other in enumerate(outs[1:], 1):
        for i, (a, b) in enumerate(zip(outs[0], other)):
            if not torch.equal(a, b):
                bad.append((j, probs[i].name, probs[i].nl, float((a - b).abs().max()), int((a != b).sum())))
    assert not bad, bad


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32])
def test_three_stage_launch_equals_split_stages_bitwise(prec):
    """Grids that are one stage box run all three RK stages in one launch (results kept in
    LDS, wave speeds as workgroup maxima); the per-grid split launches of the plain mode give
    the same bits, with and without state-dependent wave speeds, and with a mix of one-box
    and many-box grids in one solve."""
    cases = [W.c2_burgers_2d(nl=4, T=0.05), W.c1_advection_2d(nl=4).replace(T=0.05),
             W.c3_advection_3d(nr=6, nl=2, T=0.05).replace(flux=W.FLUX_BURGERS, flux_params=(),
                                                          ic_params=(0.3, 0.6, math.pi, 0.4)),
             W.c4_vlasov_4d(nr=4, nl=2, T=0.05)]
    for pb in cases:
        pb = pb.replace(precision=prec)
        for target in (512, 2048):
            _announce(f"three-stage vs split {pb.name} d={pb.d} prec={prec} target={target}")
            s_plain, _, u_plain, _, n_plain = gpu_solve(pb, mode=0, box_target=target)
            s_graph, _, u_graph, _, n_graph = gpu_solve(pb, mode=2, box_target=target)
            assert n_plain == n_graph
            assert bool((u_plain == u_graph).all()), (pb.name, target)
            for s in (s_plain, s_graph):
                s.close()


def test_set_grid_equals_restriction_bitwise():
    """Caller-sampled initial values through sgw_set_grid give the same solve as sgw_restrict_initial."""
    torch, B, Solver, _ = _lib()
    for pb in (W.c2_burgers_2d(nl=3, T=0.05, precision=W.PREC_FP64), W.c4_vlasov_4d(nl=2, T=0.1)):
        _announce(f"set_grid {pb.name}")
        a = Solver(pb).restrict()
        b = Solver(pb)
        init = a.state_copy(0).clone()
        for g, info in enumerate(b.plan.grids):
            n = int(np.prod(info["shape"]))
            b.set_grid(g, init[info["offset"]: info["offset"] + n].clone())
        a.advance()
        b.advance()
        assert a.query() == b.query()
        assert torch.equal(a.prolongate_combine(), b.prolongate_combine())


def test_snapshot_and_restore_are_refused_while_in_a_batch():
    """A batch advances its solvers on the batch stream, so a checkpoint copy on the solver's own
    stream could mix two steps: both calls are refused until the solver is released."""
    torch, B, Solver, Batch = _lib()
    pb = W.c2_burgers_2d(nl=2, T=0.05, precision=W.PREC_FP32)
    _announce("snapshot refused in a batch")
    s = Solver(pb).restrict()
    snap = s.snapshot()
    batch = Batch(4, pb.precision, 1 << 30)
    slot = batch.admit(s)
    for call in (lambda: s.snapshot(), lambda: s.restore(snap)):
        with pytest.raises(B.SgwError) as e:
            call()
        assert e.value.status == -6
    batch.step(4)
    batch.release(slot)
    s.snapshot()
    torch.cuda.synchronize()


def test_snapshot_restore_resumes_bitwise():
    """A solve stopped at T/2 and checkpointed, then resumed in another solver, ends bitwise where the
    original solver ends when it simply continues (stopping at T/2 itself adds a clipped step)."""
    torch, B, Solver, _ = _lib()
    for pb in (W.c2_burgers_2d(nl=3, T=0.1, precision=W.PREC_FP32), W.c3_advection_3d(nl=2, T=0.2)):
        _announce(f"snapshot {pb.name}")
        a = Solver(pb).restrict().advance(t_final=pb.T / 2)
        snap = a.snapshot()
        t_half, steps_half = a.query()
        a.advance()
        b = Solver(pb).restore(snap)
        assert b.query() == (t_half, steps_half)
        b.advance()
        assert a.query() == b.query()
        assert a.query()[0] == pb.T
        assert torch.equal(a.prolongate_combine(), b.prolongate_combine())


# --------------------------------------------------------------------------- translation and canaries

def _adv4():
    """4D advection (line sweeps with the plane launch) on a small sparse grid."""
    return W.Problem(d=4, lo=(0.0,) * 4, hi=(2.0,) * 4, flux=W.FLUX_ADVECTION, flux_params=(1.0, -0.5, 0.75, 0.25),
                     ic=W.IC_SINE, ic_params=(0.0, 1.0, math.pi, 0.3), nr=4, nl=2, T=0.1, cfl=0.5,
                     precision=W.PREC_FP64, name="advection_4d")


def _shifted_grids(s, pb, k):
    """u^n of every grid of solver s cyclically shifted by one root cell along direction k (2^{l_k}
    nodes), as a list of device tensors in the solver's precision."""
    torch = __import__("torch")
    out = []
    for info in s.plan.grids:
        shape = info["shape"]
        n = int(np.prod(shape))
        a = s.state_copy()[info["offset"]: info["offset"] + n].reshape(tuple(reversed(shape)))
        out.append(torch.roll(a, shifts=1 << info["level"][k], dims=pb.d - 1 - k).contiguous().reshape(-1))
    return out


@pytest.mark.parametrize("name,make,k", [
    ("burgers_2d_x", lambda: W.c2_burgers_2d(nl=4, T=0.05, precision=0), 0),
    ("burgers_2d_y", lambda: W.c2_burgers_2d(nl=4, T=0.05, precision=1), 1),
    ("advection_3d_z", lambda: W.c3_advection_3d(nr=8, nl=3, T=0.1, precision=0), 2),
    ("advection_4d_x", lambda: _adv4(), 0),
    ("advection_4d_w", lambda: _adv4(), 3),
])
def test_translation_by_one_root_cell_is_exact(name, make, k):
    """Translation invariance on the GPU: initial grids shifted cyclically by one root cell along
    direction k (set through sgw_set_grid) march to the shifted component grids and combine to the
    finest-grid solution shifted by 2^{N_L} nodes, bit for bit (the shift moves every node across
    stage-box and prolongation-tile edges, which do not move)."""
    torch, B, Solver, _ = _lib()
    pb = make()
    _announce(f"translation {name}")
    a = Solver(pb)
    a.restrict()
    shifted = _shifted_grids(a, pb, k)
    a.advance()
    Ua = a.prolongate_combine()
    b = Solver(pb)
    for g, v in enumerate(shifted):
        b.set_grid(g, v)
    b.advance()
    Ub = b.prolongate_combine()
    assert a.query() == b.query()
    for ga, gb in zip(_shifted_grids(a, pb, k), (b.grid(g) for g in range(len(b.plan.grids)))):
        assert torch.equal(ga, gb)
    n = pb.n_fine
    Ua_s = torch.roll(Ua.reshape((n,) * pb.d), shifts=1 << pb.nl, dims=pb.d - 1 - k).reshape(-1)
    assert torch.equal(Ua_s, Ub)


@pytest.mark.parametrize("k", [0, 3])
def test_4d_prolongation_translation_by_one_root_cell_is_exact(k):
    """The 4D line-form prolongation of seeded noise: grids shifted by one root cell along direction
    k combine to the finest grid shifted by 2^{N_L} nodes, bit for bit."""
    torch, B, Solver, _ = _lib()
    pb = W.c4_vlasov_4d(nl=3, precision=0)
    _announce(f"4D prolongation translation along direction {k + 1}")
    a = Solver(pb)
    noise = torch.from_numpy(W.component_noise(a.plan.total_nodes, seed=29)).cuda()
    for g, info in enumerate(a.plan.grids):
        n = int(np.prod(info["shape"]))
        a.set_grid(g, noise[info["offset"]: info["offset"] + n].clone())
    Ua = a.prolongate_combine()
    b = Solver(pb)
    for g, v in enumerate(_shifted_grids(a, pb, k)):
        b.set_grid(g, v)
    Ub = b.prolongate_combine()
    n = pb.n_fine
    assert torch.equal(torch.roll(Ua.reshape((n,) * 4), shifts=1 << pb.nl, dims=3 - k).reshape(-1), Ub)


@pytest.mark.parametrize("name,make", [("2d", lambda: W.c2_burgers_2d(nl=4, T=0.02, precision=1)),
                                       ("4d", lambda: W.c4_vlasov_4d(nl=2, T=0.02, precision=0))])
def test_outputs_leave_canaries_beyond_the_finest_grid(name, make):
    """Output canaries: the combination, its tile-range form, the exact solution and the batched
    combination write the finest grid and nothing after it (a canary tail of 4096 entries)."""
    torch, B, Solver, _ = _lib()
    from paper_2007_10196_amd.solver import prolongate_combine_many
    pb = make()
    _announce(f"canaries {name}")
    s = Solver(pb)
    s.restrict()
    s.advance()
    nf, tail = s.plan.fine_nodes, 4096
    canary = -1.2345e300
    for fill in ("combine", "tiles", "exact", "many"):
        out = torch.full((nf + tail,), canary, dtype=torch.float64, device="cuda")
        if fill == "combine":
            s.prolongate_combine(out)
        elif fill == "tiles":
            s.prolongate_combine_tiles(out, 0, s.plan.fine_tile_count)
        elif fill == "exact":
            s.exact(pb.T, out)
        else:
            prolongate_combine_many([s], [out])
        torch.cuda.synchronize()
        assert bool((out[nf:] == canary).all()), fill
        assert not bool((out[:nf] == canary).any()), fill


@pytest.mark.parametrize("name,make", [("2d_fp32", lambda: W.c2_burgers_2d(nr=10, nl=3, T=0.05, precision=1)),
                                       ("3d_fp64", lambda: W.c3_advection_3d(nr=6, nl=2, T=0.1, precision=0)),
                                       ("4d_fp64", lambda: _adv4().replace(nr=5))])
def test_state_padding_canaries(name, make):
    """Pad canaries: the bytes after the component grids in each of the three state copies (up to
    the 256-byte aligned copy size) hold NaN patterns through a whole solve; they are never written,
    and never read into a result (bitwise the same solve without them)."""
    torch, B, Solver, _ = _lib()
    pb = make()
    _announce(f"pad canaries {name}")
    esz = 8 if pb.precision == W.PREC_FP64 else 4
    a = Solver(pb)
    copy = a.plan.state_bytes // 3
    used = a.plan.total_nodes * esz
    if copy - used < esz:
        pytest.skip(f"no padding after the grids ({copy} = {used} bytes)")
    a.restrict()
    pads = [a.state[c * copy + used: (c + 1) * copy] for c in range(3)]
    for p in pads:
        p.fill_(0xFF)
    a.advance()
    Ua = a.prolongate_combine()
    b = Solver(pb)
    b.restrict()
    b.advance()
    Ub = b.prolongate_combine()
    torch.cuda.synchronize()
    assert all(bool((p == 0xFF).all()) for p in pads)
    assert torch.equal(Ua, Ub) and torch.equal(a.state_copy(), b.state_copy())


def test_cancelled_solve_leaves_the_others_and_resumes_alone_bitwise():
    """A solve released from a running batch halfway (a cancel) leaves the other solves' results
    bitwise equal to their solo runs, and itself resumes alone to the same bits as its solo run."""
    torch, B, Solver, Batch = _lib()
    rng = np.random.default_rng(17)
    probs = [W.randomized(f, nl, rng, precision=W.PREC_FP64) for f, nl in [(1, 3), (2, 3), (3, 2)]]
    probs = [p.replace(T=min(p.T, 0.15)) for p in probs]
    solo = [Solver(p).solve(mode=B.RUN_GRAPH).cpu().numpy() for p in probs]
    _announce("cancel in a batch")
    batch = Batch(max_solvers=4, precision=B.FP64, hbm_budget=1 << 34)
    solvers, slots = [], []
    for p in probs:
        s = Solver(p)
        s.restrict()
        slots.append(batch.admit(s))
        solvers.append(s)
    batch.step(3)
    cancelled = batch.release(slots[1])
    assert cancelled is solvers[1]
    t_mid, steps_mid = cancelled.query()
    assert 0 < t_mid < probs[1].T and steps_mid == 3
    done = set()
    for _ in range(400):
        batch.step(4)
        done |= set(batch.poll())
        if done >= {slots[0], slots[2]}:
            break
    assert done >= {slots[0], slots[2]} and slots[1] not in done
    for i in (0, 2):
        assert np.array_equal(solvers[i].prolongate_combine().cpu().numpy(), solo[i])
    cancelled.advance()
    assert np.array_equal(cancelled.prolongate_combine().cpu().numpy(), solo[1])
    for sl in (slots[0], slots[2]):
        batch.release(sl)
    batch.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_zero_wave_speed_takes_one_step(prec):
    """With every wave speed 0 the CFL step has no bound: the solve takes one step to T (dt = T - t),
    as the oracle does, and the fluxes vanish, so the combined solution is the initial one up to the
    rounding of the Runge-Kutta combinations (3/4 u + 1/4 u, 1/3 u + 2/3 u)."""
    torch, B, Solver, _ = _lib()
    pb = W.c1_advection_2d(nr=8, nl=3).replace(flux_params=(0.0, 0.0), T=0.7, precision=prec)
    _announce(f"zero speed precision {prec}")
    s = Solver(pb)
    s.restrict()
    U0 = s.prolongate_combine().clone()
    s.advance()
    t, steps = s.query()
    stats = O.evolve(pb.replace(precision=W.PREC_FP64), O.restrict(pb.replace(precision=W.PREC_FP64)))
    assert steps == 1 == stats["steps"] and t == pb.T == stats["t"]
    tol = 1e-14 if prec == 0 else 1e-6
    assert float((s.prolongate_combine() - U0).abs().max()) <= tol
