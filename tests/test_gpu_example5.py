"""GPU parity of the Vlasov-Boltzmann model (Sec. 3.4, Example 5) and of zero boundaries: the HIP
path (through the C ABI) against the FP64 oracle within 1e-11 max-abs on every component grid
and on the combined solution, and the entropy functionals H_2, H_log of the combined solution
within 1e-10 relative: both are sums of up to 4.1e7 terms in different orders (sequential on the
CPU, a tree on the GPU), whose rounding grows like sqrt(n) u ~ 1e-12 in practice and at most
n u ~ 5e-9."""
import math

import numpy as np
import pytest

import oracle as O
import sgw_inputs as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
ENT_REL = 1e-10


def _lib():
    import torch
    from paper_2007_10196_amd import binding as B
    from paper_2007_10196_amd.solver import Solver
    return torch, B, Solver


def _announce(what):
    print(f"\n[gpu] {what}", flush=True)


def _solve_both(pb, mode=2, sample=0, **kw):
    """Both paths on pb; with sample > 0 the combined solution is compared at that many seeded
    finest nodes (the faces and corners included) instead of everywhere."""
    torch, B, Solver = _lib()
    pb = pb.replace(precision=W.PREC_FP64)
    _announce(f"{pb.name} d={pb.d} nr={pb.nr} nl={pb.nl} T={pb.T:.6g} bc={pb.bc} tau={pb.relax_tau} mode={mode}")
    s = Solver(pb, **kw)
    s.restrict()
    s.advance(mode=mode)
    U = s.prolongate_combine()
    t, steps = s.query()
    st_g = s.state_copy().double().cpu().numpy().copy()
    st_o = O.restrict(pb)
    stats = O.evolve(pb, st_o)
    assert steps == stats["steps"]
    assert abs(t - stats["t"]) < 1e-14
    assert np.max(np.abs(st_g - st_o)) <= TOL64
    if sample:
        n, d = pb.n_fine, pb.d
        rng = np.random.default_rng(2007)
        J = rng.integers(0, n, size=(sample, d)).astype(np.int32)
        J[:2 ** d] = [[(c >> k & 1) * (n - 1) for k in range(d)] for c in range(2 ** d)]
        U_o = O.prolong_combine_points(pb, st_o, J)
        idx = sum(J[:, k].astype(np.int64) * n ** k for k in range(d))
        assert np.max(np.abs(U.cpu().numpy()[idx] - U_o)) <= TOL64
        return s, U, None
    U_o = O.prolong_combine(pb, st_o)
    assert np.max(np.abs(U.cpu().numpy() - U_o)) <= TOL64
    return s, U, U_o


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_example5_2d_small_all_modes(mode):
    _solve_both(W.paper_example5(2, nr=10, nl=3, T=0.25), mode=mode)


def test_example5_2d_paper_size():
    """Example 5(a) at the paper's size: 40^2 root grid, finest level 3 (320^2), to t = 0.5."""
    s, U, U_o = _solve_both(W.paper_example5(2, nr=40, nl=3, T=0.5))
    pb = W.paper_example5(2, nr=40, nl=3)
    h2, hl = s.entropies(U)
    h2o, hlo = O.entropies(pb, U_o)
    assert abs(h2 - h2o) <= ENT_REL * abs(h2o)
    assert abs(hl - hlo) <= ENT_REL * abs(hlo)


def test_example5_4d_small():
    _solve_both(W.paper_example5(4, nr=4, nl=2, T=0.2))


def test_example5_4d_paper_grids_short_time():
    """Example 5(b)'s grids (10^4 root, finest level 3, 80^4 finest) over 40 steps: every component
    grid, the combined solution at 3000 sampled finest nodes (the corners among them), and the
    entropies of the GPU's combined solution as the oracle computes them."""
    pb = W.paper_example5(4, nr=10, nl=3, T=0.1)
    s, U, _ = _solve_both(pb, sample=3000)
    h2, hl = s.entropies(U)
    h2o, hlo = O.entropies(pb, U.cpu().numpy())
    assert abs(h2 - h2o) <= ENT_REL * abs(h2o)
    assert abs(hl - hlo) <= ENT_REL * abs(hlo)


@pytest.mark.parametrize("name,make", [
    ("advection_2d_zero_x", lambda: W.c1_advection_2d(nr=8, nl=3).replace(bc=(1, 0), T=0.6,
                                                                           flux_params=(1.0, -0.5))),
    ("burgers_2d_zero_both", lambda: W.c2_burgers_2d(nl=3, T=0.5 / math.pi ** 2).replace(bc=(1, 1))),
    ("advection_3d_zero", lambda: W.c3_advection_3d(nr=6, nl=2, T=0.3).replace(bc=(1, 1, 1),
                                                                               flux_params=(1.0, -0.5, 0.25))),
    ("burgers_3d_mixed", lambda: W.c3_advection_3d(nr=8, nl=3, T=0.1).replace(
        bc=(1, 0, 1), flux=W.FLUX_BURGERS, flux_params=(), ic_params=(0.3, 0.6, math.pi, 0.4))),
    ("vlasov_4d_zero_v", lambda: W.c4_vlasov_4d(nl=2, T=0.3).replace(bc=(0, 0, 1, 1))),
    ("lagrange_zero", lambda: W.paper_example1(40, nr=10, nl=2).replace(bc=(1, 1))),
])
def test_zero_boundary_without_relaxation(name, make):
    _solve_both(make())


@pytest.mark.parametrize("d,n,theta", [(2, 16, 1.0), (2, 24, 0.5), (4, 8, 0.7)])
def test_relaxation_alone(d, n, theta):
    """Zero-speed transport plus the source: the density pass and the source term alone."""
    pb = W.Problem(d=d, lo=(-5.0,) * d, hi=(5.0,) * d, flux=W.FLUX_ADVECTION, flux_params=(0.0,) * d,
                   ic=W.IC_VB, ic_params=(1.0,), nr=n, nl=0, T=3.0, dt_mode=W.DT_POW53, bc=(1,) * d,
                   relax_tau=0.8, relax_theta=theta, name="relaxation_alone")
    _solve_both(pb)


def test_relaxation_with_periodic_boundaries_and_sparse_grids():
    _solve_both(W.paper_example5(2, nr=8, nl=4, T=0.2).replace(bc=(0, 0)))


def test_example5_repeat_runs_are_bitwise_identical():
    """The density pass sums in a fixed order (arrival counter, ordered chunk sums)."""
    torch, B, Solver = _lib()
    pb = W.paper_example5(4, nr=8, nl=2, T=0.1)
    outs = []
    for _ in range(2):
        s = Solver(pb)
        s.restrict()
        s.advance()
        outs.append(s.prolongate_combine().cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_example5_fp32_against_fp64_oracle():
    torch, B, Solver = _lib()
    pb = W.paper_example5(2, nr=10, nl=3, T=0.25)
    s = Solver(pb.replace(precision=W.PREC_FP32))
    s.restrict()
    s.advance()
    U = s.prolongate_combine().cpu().numpy()
    U_o = O.solve(pb)[0]
    assert np.max(np.abs(U - U_o)) < 1e-5 * np.max(np.abs(U_o))


def test_exact_is_refused_and_batches_refuse_the_model():
    torch, B, Solver = _lib()
    from paper_2007_10196_amd.solver import Batch
    s = Solver(W.paper_example5(2, nr=8, nl=2, T=0.1))
    s.restrict()
    with pytest.raises(B.SgwError) as e:
        s.exact(0.1)
    assert e.value.status == -2
    b = Batch(4, W.PREC_FP64, 1 << 30)
    with pytest.raises(B.SgwError) as e:
        b.admit(s)
    assert e.value.status == -2
    b.close()


def test_entropies_of_the_stationary_state():
    """H = f/M = 1 at f = M: H_2 = int M (1 up to the Gaussian's tail), H_log = 0; at 2M, 4 and
    2 log 2 times that."""
    torch, B, Solver = _lib()
    for d, nr in ((2, 10), (4, 5)):
        pb = W.paper_example5(d, nr=nr, nl=2)
        s = Solver(pb)
        n = pb.n_fine
        g = -5.0 + 10.0 / n * np.arange(n)
        axes = np.meshgrid(*([g] * d), indexing="ij")
        c = [axes[d - 1 - k].ravel() for k in range(d)]
        m = d // 2
        from scipy.special import erf
        zx = (math.sqrt(2 * math.pi) * erf(5 / math.sqrt(2))) ** m
        M = np.exp(-0.5 * sum(a * a for a in c)) / ((2 * math.pi) ** (m / 2) * zx)
        Mt = torch.from_numpy(M).cuda()
        h2, hl = s.entropies(Mt)
        h2o, hlo = O.entropies(pb, M)
        assert abs(h2 - h2o) <= ENT_REL and abs(hl - hlo) <= ENT_REL
        assert abs(h2 - 1.0) < 1e-4 and abs(hl) < 1e-12
        h2, hl = s.entropies(2 * Mt)
        h2o, hlo = O.entropies(pb, 2 * M)
        assert abs(h2 - h2o) <= 4 * ENT_REL and abs(hl - hlo) <= ENT_REL


@pytest.mark.parametrize("name,make,tile", [
    ("3d_line_form", lambda: W.c3_advection_3d(nr=8, nl=2, T=0.2).replace(bc=(1, 1, 1)), [16, 16, 8]),
    ("3d_pass_form", lambda: W.c3_advection_3d(nr=8, nl=2, T=0.2).replace(bc=(1, 1, 1)), [8, 8, 8]),
    ("3d_mixed_line_form", lambda: W.c3_advection_3d(nr=8, nl=2, T=0.2).replace(bc=(0, 1, 1)), [16, 16, 4]),
    ("4d_line_form", lambda: W.paper_example5(4, nr=4, nl=2, T=0.1), [8, 8, 4, 2]),
    ("4d_pass_form", lambda: W.paper_example5(4, nr=4, nl=2, T=0.1), [4, 4, 4, 4]),
])
def test_zero_boundary_prolongation_tile_forms(name, make, tile):
    """Both prolongation forms (staged passes; one lane per line with the direct first pass) read
    0 beyond a zero boundary: tiles whose first d-1 extents hold 256 nodes take the line form."""
    _solve_both(make(), fine_tile=tile)
