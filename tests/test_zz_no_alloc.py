"""The error norms of many solves without allocation (sgw_norms_many_static) against
sgw_norms_many, through the C ABI: bitwise equal on two calls in a row, the second
with fewer and smaller pairs, and more than the stated maximum of pairs refused."""
import numpy as np
import pytest

import sgw_inputs as W

pytestmark = pytest.mark.gpu


def _solved(probs):
    from paper_2007_10196_amd.solver import Solver
    solvers, outs, exacts = [], [], []
    for p in probs:
        s = Solver(p)
        s.restrict()
        s.advance()
        outs.append(s.prolongate_combine())
        exacts.append(s.exact(s.query()[0]))
        solvers.append(s)
    return solvers, outs, exacts


def test_norms_many_static_equals_norms_many_on_two_calls():
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.solver import norms_many, norms_many_static
    rng = np.random.default_rng(31)
    # first call: five pairs of 2D/3D/4D solves; second: two smaller 2D pairs
    first = [W.randomized(fam, nl, rng, precision=W.PREC_FP64) for fam, nl in ((2, 5), (3, 3), (4, 2), (1, 4), (2, 3))]
    second = [W.randomized(fam, nl, rng, precision=W.PREC_FP64) for fam, nl in ((1, 2), (2, 2))]
    for call, probs in enumerate((first, second)):
        probs = [p.replace(T=min(p.T, 0.05)) for p in probs]
        print(f"\n[gpu] norms_many_static call {call}: {[(p.name, p.d, p.nl) for p in probs]}", flush=True)
        solvers, outs, exacts = _solved(probs)
        ref = torch.full((len(probs), 2), -1.0, dtype=torch.float64, device="cuda")
        got = torch.full((len(probs), 2), -2.0, dtype=torch.float64, device="cuda")
        norms_many(solvers, outs, exacts, ref)
        norms_many_static(solvers, outs, exacts, got)
        torch.cuda.synchronize()
        assert torch.equal(ref, got), (ref, got)
        assert bool((got[:, 0] > 0).all()) and bool((got[:, 0] <= got[:, 1]).all())
    assert int(B.lib().sgw_norms_many_static_max_bytes()) <= 1 << 20


def test_norms_many_static_refuses_more_pairs_than_its_maximum():
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.solver import norms_many_static
    probs = [W.c1_advection_2d(precision=W.PREC_FP64).replace(nl=1, T=0.01)] * 33
    solvers, outs, exacts = _solved(probs[:1])
    res = torch.zeros((33, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(B.SgwError) as ei:
        norms_many_static(solvers * 33, outs * 33, exacts * 33, res)
    assert ei.value.status == -1  # invalid argument
