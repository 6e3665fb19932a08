"""The work counts the benchmark prices its rooflines with (CPU only).

One flop count per cell-update everywhere: 3 TVD-RK3 stages of 140 flops per direction (two
WENO5 reconstructions, the flux, its Lax-Friedrichs split and the flux difference of eq. (2.9))
plus 5 for the Runge-Kutta combination.  The prolongation count is checked against the grid set of
the combination technique (Sec. 2.2, eq. (genformusgc)): the component grids of root 8 and finest
level 4 in 4D are the level vectors with 1 <= |l|_1 <= 4 (69 grids), each refined direction by
direction, so the pass along direction k of grid l produces N^k prod_{j>k} n_{l,j} points with
n_{l,j} = 8 * 2^{l_j} and N = 128."""
import itertools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import sgw_inputs as W  # noqa: E402


def test_flops_per_cell_update():
    assert [bench.flops_per_cell_update(d) for d in (2, 3, 4)] == [855, 1275, 1695]


def test_interpolation_count_of_the_4d_headline():
    from paper_2007_10196_amd.solver import Plan
    plan = Plan(W.c4_vlasov_4d(precision=W.PREC_FP64))
    N, nr, nl = 128, 8, 4
    levels = [l for l in itertools.product(range(nl + 1), repeat=4) if 1 <= sum(l) <= nl]
    assert len(levels) == len(plan.grids) == 69
    want = 0
    for l in levels:
        n = [nr << x for x in l]
        for k in range(4):
            if l[k] == nl:
                continue
            pts = N ** (k + 1)
            for j in range(k + 1, 4):
                pts *= n[j]
            want += pts
    got = bench.interpolation_count(plan)
    assert got == want
    assert got == pytest.approx(2.13e10, rel=2e-3)
