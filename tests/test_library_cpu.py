"""Host-side checks of libsgweno that need no GPU: exports, planner, validation."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import sgw_inputs as W
from paper_2007_10196_amd import binding as B
from paper_2007_10196_amd.solver import Plan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def _declared():
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(INCLUDE, h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(sgw_[a-z_0-9]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    L = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    assert names == set(B.EXPORTED)


@pytest.mark.parametrize("d,nl", [(1, 3), (2, 0), (2, 3), (2, 5), (3, 5), (4, 4), (4, 5)])
def test_plan_grid_set_matches_oracle(d, nl):
    if d == 4:
        pb = W.c4_vlasov_4d(nl=nl)
    elif d == 3:
        pb = W.c3_advection_3d(nl=nl)
    elif d == 2:
        pb = W.c2_burgers_2d(nl=nl)
    else:
        pb = W.Problem(d=1, lo=(0.0,), hi=(1.0,), flux=W.FLUX_ADVECTION, flux_params=(1.0,), ic=W.IC_SINE,
                       ic_params=(0, 1, 2 * np.pi, 0), nr=8, nl=nl, T=0.1)
    plan = Plan(pb)
    lv, cf = O.grid_set(d, nl)
    assert plan.num_grids == len(lv)
    off = 0
    for g, info in enumerate(plan.grids):
        assert info["level"] == tuple(int(x) for x in lv[g])
        assert info["coef"] == int(cf[g])
        assert info["shape"] == tuple(pb.nr << int(x) for x in lv[g])
        assert info["offset"] == off
        off += int(np.prod(info["shape"]))
        if d >= 3:
            # 3D and 4D grids march as line sweeps by default: no stage boxes
            assert info["box"] == (0,) * d
            continue
        for n, t in zip(info["shape"], info["box"]):
            assert n % t == 0
        assert int(np.prod(info["box"])) <= 2048
    assert plan.total_nodes == off == O.total_nodes(pb)
    assert plan.fine_nodes == pb.n_fine ** d
    esz = 8 if pb.precision == W.PREC_FP64 else 4
    assert plan.state_bytes >= 3 * off * esz


@pytest.mark.parametrize("nr", [4, 5, 6, 7, 10, 12])
def test_plan_handles_non_power_of_two_roots(nr):
    """Stage boxes (3D with sweep_form 2) divide every extent; the default line sweeps plan for
    the same roots."""
    pb = W.c3_advection_3d(nr=nr, nl=3)
    plan = Plan(pb, sweep_form=2)
    for info in plan.grids:
        for n, t in zip(info["shape"], info["box"]):
            assert n % t == 0
    assert all(info["box"] == (0, 0, 0) for info in Plan(pb).grids)


def _expect_status(pb, status, **kw):
    with pytest.raises(B.SgwError) as e:
        Plan(pb, **kw)
    assert e.value.status == status


def test_plan_rejects_invalid_arguments():
    good = W.c1_advection_2d()
    _expect_status(good.replace(d=5, lo=(0,) * 4, hi=(1,) * 4), -1)
    _expect_status(good.replace(d=0), -1)
    _expect_status(good.replace(nr=3), -1)
    _expect_status(good.replace(nl=13), -1)
    _expect_status(good.replace(cfl=0.0), -1)
    _expect_status(good.replace(cfl=2.0), -1)
    _expect_status(good.replace(eps_flux=0.0), -1)
    _expect_status(good.replace(hi=(0.0, 2.0)), -1)
    _expect_status(W.c4_vlasov_4d().replace(d=3, lo=(0,) * 3, hi=(1,) * 3), -1)
    _expect_status(good, -2, box=[3, 3])          # 3 does not divide 4 << l
    _expect_status(good, -2, fine_tile=[5, 5])    # 5 does not divide 32
    _expect_status(good, -1, box_target=32)
    _expect_status(good.replace(bc=(0, 2)), -1)     # unknown boundary condition
    _expect_status(good.replace(bc=(0, 1)), -2, box=[4, 4])  # zero boundary: line sweeps, no manual boxes
    Plan(good.replace(bc=(0, 0, 1, 1)))            # entries beyond dim are ignored
    vb = W.paper_example5(2, nr=8, nl=2)
    _expect_status(vb.replace(relax_tau=-1.0), -1)
    _expect_status(vb.replace(relax_tau=float("inf")), -1)
    _expect_status(vb.replace(relax_theta=0.0), -1)
    _expect_status(vb.replace(d=3, lo=(-5.0,) * 3, hi=(5.0,) * 3, bc=(1,) * 3), -1)  # phase space: even dim
    _expect_status(vb.replace(flux=4), -1)
    _expect_status(vb.replace(ic=3), -1)
    Plan(vb.replace(relax_theta=0.0, relax_tau=0.0))  # theta is not read without relaxation


@pytest.mark.parametrize("d,bc,tau", [(2, (1, 1), 1.0), (2, (1, 0), 0.0), (3, (1, 1, 1), 0.0), (4, (1,) * 4, 1.0)])
def test_zero_boundary_and_relaxation_plans_run_line_sweeps(d, bc, tau):
    """Plans with a zero boundary or relaxation march every grid as line sweeps (no boxes), in
    any dimension, and the same component grids as the oracle."""
    if d in (2, 4):
        pb = W.paper_example5(d, nr=8, nl=2).replace(bc=bc, relax_tau=tau)
    else:
        pb = W.c3_advection_3d(nr=4, nl=2).replace(bc=bc)
    plan = Plan(pb)
    assert plan.total_nodes == O.total_nodes(pb)
    for info in plan.grids:
        assert info["box"] == (0,) * d


def test_error_strings():
    L = B.lib()
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert L.sgw_status_string(s)
    try:
        Plan(W.c1_advection_2d().replace(nr=2))
    except B.SgwError:
        pass
    assert b"root_cells" in L.sgw_last_error()


def test_footprints_scale_with_precision():
    p64 = Plan(W.c3_advection_3d(precision=W.PREC_FP64))
    p32 = Plan(W.c3_advection_3d(precision=W.PREC_FP32))
    assert p64.total_nodes == p32.total_nodes == 507904
    assert p64.state_bytes >= 2 * p32.state_bytes - 1024
    assert p64.fine_bytes == 8 * 256 ** 3


def _coarse_extent(pb, level, T):
    """Coarse values a tile row of extent T needs per direction: T without refinement, else the
    most coarse centres its nodes J0..J0+T-1 reach over the tile positions (node J has centre
    floor(J/R + 1/2), Sec. 2.2.1) plus the two stencil nodes on either side, by brute force."""
    out = []
    N = pb.n_fine
    for k in range(pb.d):
        m = pb.nl - level[k]
        if m == 0:
            out.append(T[k])
            continue
        R = 1 << m
        centre = lambda J: (2 * J + R) >> (m + 1)
        out.append(max(centre(J0 + T[k] - 1) - centre(J0) + 1 for J0 in range(0, N, T[k])) + 4)
    return out


@pytest.mark.parametrize("make", [lambda: W.c1_advection_2d(), lambda: W.c2_burgers_2d(),
                                  lambda: W.c3_advection_3d(), lambda: W.c3_advection_3d(precision=1),
                                  lambda: W.c4_vlasov_4d(), lambda: W.c4_vlasov_4d(precision=0),
                                  lambda: W.c2_burgers_2d(nr=10, nl=3)])
def test_prolongation_tile_fits_and_divides(make):
    """The searched finest-grid tile divides N in every direction, holds at most 16 nodes per thread,
    and its two LDS buffers (largest coarse block or pass output) stay within 64 KB."""
    pb = make()
    plan = Plan(pb)
    T = plan.fine_tile
    N = pb.n_fine
    assert len(T) == pb.d and all(N % t == 0 for t in T)
    assert int(np.prod(T)) <= 256 * 16
    esz = 8 if pb.precision == W.PREC_FP64 else 4
    biggest = 0
    for info in plan.grids:
        c = _coarse_extent(pb, info["level"], T)
        biggest = max(biggest, int(np.prod(c)))
        for k in range(pb.d):
            biggest = max(biggest, int(np.prod([T[j] if j <= k else c[j] for j in range(pb.d)])))
    assert 2 * esz * biggest <= 64 * 1024


def test_prolongation_tile_prefers_late_directions():
    """Directions are refined in increasing order, so halo work of early passes is multiplied by the
    coarse extents of the later directions: the search makes the last extent at least the first."""
    for pb in (W.c3_advection_3d(precision=1), W.c4_vlasov_4d()):
        T = Plan(pb).fine_tile
        assert T[-1] >= T[0], T


def test_blocks_per_cu_is_validated():
    _expect_status(W.c1_advection_2d(), -1, blocks_per_cu=65)
    _expect_status(W.c1_advection_2d(), -1, blocks_per_cu=-1)
    Plan(W.c1_advection_2d(), blocks_per_cu=6)  # accepted


def test_pointer_list_marshals_once_and_validates_lazily():
    """PtrList (binding side, no GPU): the pointer array holds each tensor's data pointer in order,
    it behaves as the sequence it was built from, and records what the norm call checks."""
    import torch
    from paper_2007_10196_amd.solver import PtrList, _ptrs
    xs = [torch.zeros(n, dtype=torch.float64) for n in (5, 3, 7)]
    pl = PtrList(xs)
    assert len(pl) == 3 and pl[1] is xs[1] and list(pl) == xs
    assert [pl.arr[i] for i in range(3)] == [x.data_ptr() for x in xs]
    assert pl.min_numel == 3
    assert pl.all_fp64 is False  # host tensors: the norm call would refuse them
    assert _ptrs(pl, "tensor") is pl.arr
    plain = _ptrs(xs, "tensor")
    assert [plain[i] for i in range(3)] == [x.data_ptr() for x in xs]
    assert len(PtrList([])) == 0


def test_valu_calibration_hook_validates_before_launching():
    """sgw_calibrate_valu refuses an unknown instruction class or a bad size before any GPU call."""
    import ctypes as C
    n = C.c_double()
    for op, blocks, out in ((5, 1, 1), (-1, 1, 1), (0, 0, 1), (0, 1, None)):
        st = B.lib().sgw_calibrate_valu(op, blocks, C.c_void_p(out), None, C.byref(n))
        assert st == -1  # SGW_ERR_INVALID_ARG


def test_vlasov_maxwell_plans():
    """The Vlasov-Maxwell system: dim 3 with its own initial condition, periodic, no relaxation and no
    manual boxes; its plans march as line sweeps and carry 3 n_1 FP64 field values per grid after
    the nodes of each state copy."""
    vm = W.paper_example6(nr=8, nl=2)
    plan = Plan(vm)
    assert plan.fields_count == O.total_fields(vm) == sum(3 * g["shape"][0] for g in plan.grids)
    assert plan.fields_offset % 256 == 0 and plan.fields_offset >= 8 * plan.total_nodes
    assert plan.state_bytes >= 3 * (plan.fields_offset + 8 * plan.fields_count)
    assert all(g["box"] == (0, 0, 0) for g in plan.grids)
    _expect_status(vm.replace(ic=W.IC_SINE), -1)                         # the flux needs its initial condition
    _expect_status(W.c3_advection_3d(nr=8, nl=2).replace(ic=W.IC_VM), -1)  # and the other way round
    _expect_status(vm.replace(relax_tau=1.0), -1)
    _expect_status(vm.replace(bc=(1, 0, 0)), -2)
    _expect_status(vm, -2, box=[8, 8, 8])
    assert Plan(W.c3_advection_3d(nr=8, nl=2)).fields_count == 0


def test_autotuner_skips_plans_without_stage_boxes():
    """3D and 4D plans march as line sweeps by default: the launch-shape tuner has no box to shape
    and returns the library's defaults without measuring (no GPU needed)."""
    from paper_2007_10196_amd.autotune import tune_box_target
    for pb in (W.c4_vlasov_4d(nl=2), W.c3_advection_3d(nl=2)):
        rec = tune_box_target([pb], pb.precision)
        assert rec["line_sweeps"] and rec["best"] == 0 and rec["blocks_per_cu"] == 0 and rec["us"] == {}
