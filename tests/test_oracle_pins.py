"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them retypes the oracle's own
formulas: they compare it with printed values (tests/golden/paper_errors.txt),
closed forms derived independently (Fourier symbol of the linear scheme,
integral definition of the smoothness indicators, degree-4 Lagrange
interpolation), exact invariants (conservation, shift and mirror symmetry) and
convergence rates.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import sgw_inputs as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_errors.txt")


def _paper_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            c = line.split()
            rows.append(dict(case=c[0], ex=c[1], scheme=c[2], prolong=c[3], d=int(c[4]), nr=int(c[5]),
                             nl=int(c[6]), nh=int(c[7]), l1=float(c[8]), linf=float(c[9])))
    return rows


# --------------------------------------------------------------------------- grid set (Sec. 2.2)

@pytest.mark.parametrize("d,nl,count", [(2, 3, 7), (2, 5, 11), (3, 5, 46), (4, 4, 69), (4, 5, 121), (1, 4, 1)])
def test_grid_counts(d, nl, count):
    # 2D: 2 N_L + 1 grids (Sec. 2.2); general d: sum_q C(N_L-q+d-1, d-1), the number of
    # compositions of N_L - q into d non-negative parts.
    assert O.num_grids(d, nl) == count
    assert count == sum(math.comb(nl - q + d - 1, d - 1) for q in range(d) if nl - q >= 0)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("nl", [0, 1, 2, 3, 5, 7])
def test_combination_coefficients(d, nl):
    lv, cf = O.grid_set(d, nl)
    # every index appears once, with |l| in [N_L-d+1, N_L]
    assert len({tuple(r) for r in lv}) == len(lv)
    s = lv.sum(axis=1)
    assert np.all(s <= nl) and np.all(s >= nl - d + 1)
    # printed 2D / 3D / 4D formulas (Sec. 2.2.2): signs and binomials per q = N_L - |l|
    printed = {1: [1], 2: [1, -1], 3: [1, -2, 1], 4: [1, -3, 3, -1]}[d]
    for l, c in zip(lv, cf):
        assert c == printed[nl - int(l.sum())]
    # the coefficients sum to one for every d and N_L
    assert int(cf.sum()) == 1


def test_grid_order_lexicographic():
    lv, _ = O.grid_set(3, 4)
    keys = [(4 - int(l.sum()),) + tuple(int(x) for x in l) for l in lv]
    assert keys == sorted(keys)


# --------------------------------------------------------------------------- WENO5 flux (Sec. 2.1)

def test_linear_weights_give_upwind5():
    # eq. (2.7.1) with w_r = d_r collapses to the fifth-order upwind flux
    # (2 f_{i-2} - 13 f_{i-1} + 47 f_i + 27 f_{i+1} - 3 f_{i+2}) / 60.
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b, c, d, e = rng.normal(size=5)
        ref = (2 * a - 13 * b + 47 * c + 27 * d - 3 * e) / 60
        assert O.weno5(a, b, c, d, e, linear=True) == pytest.approx(ref, rel=1e-13, abs=1e-14)


def test_smoothness_indicators_match_integral_definition():
    # eq. (si): beta_k = sum_{l=1,2} h^{2l-1} int_{x_{i-1/2}}^{x_{i+1/2}} (P_k^{(l)})^2 dx, P_k the
    # quadratic through substencil S_k; in units of h the integral runs over s in [-1/2, 1/2].
    rng = np.random.default_rng(2)
    P = np.polynomial.Polynomial
    for _ in range(50):
        u = rng.normal(size=5)
        beta = O.smoothness(*u)
        for k in range(3):
            p = P.fit(np.arange(k - 2, k + 1), u[k:k + 3], 2).convert()
            tot = 0.0
            for der in (1, 2):
                q = (p.deriv(der) ** 2).integ()
                tot += q(0.5) - q(-0.5)
            assert beta[k] == pytest.approx(tot, rel=1e-11, abs=1e-12)


def test_weno5_essentially_non_oscillatory_on_a_step():
    # Across a jump only the smooth substencil keeps weight: (0,0,0,1,1) -> q0 = 0.
    v = O.weno5(0.0, 0.0, 0.0, 1.0, 1.0, eps=1e-6)
    assert abs(v) < 1e-10
    v = O.weno5(1.0, 1.0, 0.0, 0.0, 0.0, eps=1e-6)   # jump on the left: q2 = 0
    assert abs(v) < 1e-10


def test_constant_state_has_zero_rhs():
    pb = W.c3_advection_3d(nr=4, nl=2)
    lv, _ = O.grid_set(3, 2)
    for l in lv:
        n = int(np.prod(O.grid_shape(pb, l)))
        assert np.all(O.rhs(pb, l, np.full(n, 0.37)) == 0.0)


def test_negative_wind_is_the_mirror_image():
    # the negative-wind flux uses the big stencil mirrored about x_{i+1/2}: speed -1 on the
    # reflected data gives the reflected operator, bit for bit.
    rng = np.random.default_rng(3)
    n = 16
    u = rng.normal(size=n)
    ur = u[(-np.arange(n)) % n]
    pbp = W.Problem(d=1, lo=(0.0,), hi=(1.0,), flux=W.FLUX_ADVECTION, flux_params=(1.0,), ic=W.IC_SINE,
                    ic_params=(0, 1, 2 * math.pi, 0), nr=n, nl=0, T=0.1)
    pbm = pbp.replace(flux_params=(-1.0,))
    Lp = O.rhs(pbp, (0,), u)
    Lm = O.rhs(pbm, (0,), ur)
    assert np.array_equal(Lm, Lp[(-np.arange(n)) % n])


# --------------------------------------------------------------------------- RK3 + linear scheme (closed form)

def _upwind5_symbol(theta):
    # Fourier symbol of the upwind-5 interface flux, derived independently of the oracle
    z = np.exp(1j * theta)
    return (2 * z ** -2 - 13 * z ** -1 + 47 + 27 * z - 3 * z ** 2) / 60


def _linear_closed_form(pb, steps_dt):
    """c + A Im(G e^{i(kappa sum x + phi)}) with G = prod_n R(lambda dt_n), R(z) = 1+z+z^2/2+z^3/6
    (any three-stage third-order Runge-Kutta method on a linear system)."""
    c0, A, kap, ph = pb.ic_params[:4]
    lam = 0j
    for k in range(pb.d):
        h = (pb.hi[k] - pb.lo[k]) / pb.nr
        th = kap * h
        a = pb.flux_params[k]
        lam += -a * _upwind5_symbol(th) * (1 - np.exp(-1j * th)) / h
    G = 1.0 + 0j
    for dt in steps_dt:
        z = lam * dt
        G *= 1 + z + z * z / 2 + z ** 3 / 6
    n = pb.nr
    j = np.indices((n,) * pb.d)
    xs = sum(pb.lo[k] + j[k] * (pb.hi[k] - pb.lo[k]) / n for k in range(pb.d))
    # direction 1 fastest in the oracle's layout -> transpose the meshgrid
    val = c0 + A * np.imag(G * np.exp(1j * (kap * xs + ph)))
    return val.transpose(tuple(reversed(range(pb.d)))).ravel()


def test_linear_scheme_rk3_matches_fourier_closed_form():
    pb = W.Problem(d=2, lo=(0.0, 0.0), hi=(2 * math.pi, 2 * math.pi), flux=W.FLUX_ADVECTION,
                   flux_params=(1.0, 0.7), ic=W.IC_SINE, ic_params=(0.25, 0.8, 1.0, 0.3), nr=20, nl=0,
                   T=0.37, dt_mode=W.DT_POW53, linear=True)
    st = O.restrict(pb)
    stats = O.evolve(pb, st)
    h = 2 * math.pi / 20
    dt0 = h ** (5.0 / 3.0)
    dts, t = [], 0.0
    while pb.T - t > 1e-12:
        dt = min(dt0, pb.T - t)
        dts.append(dt)
        t += dt
    assert stats["steps"] == len(dts)
    ref = _linear_closed_form(pb, dts)
    assert np.max(np.abs(st - ref)) < 1e-13


# --------------------------------------------------------------------------- printed table rows

def _problem_for_row(r):
    lin = r["scheme"] == "linear"
    pro = W.PROLONG_LAGRANGE5 if r["prolong"] == "lagrange" else W.PROLONG_WENO5
    if r["ex"] == "ex1":
        return W.paper_example1(r["nh"], nr=r["nr"], nl=r["nl"])
    if r["ex"] == "ex3a":
        return W.paper_example3a(r["nh"], nr=r["nr"], nl=r["nl"], linear=lin, prolong=pro)
    return W.paper_example3b(r["nh"], nr=r["nr"], nl=r["nl"], linear=lin, prolong=pro)


_ROWS = _paper_rows()
_SLOW = {"t1_single_320", "t3aweno_single_320"}


@pytest.mark.parametrize("row", _ROWS, ids=[r["case"] for r in _ROWS])
def test_paper_printed_errors(row):
    if row["case"] in _SLOW and not os.environ.get("SGW_SLOW_TESTS"):
        pytest.skip("set SGW_SLOW_TESTS=1 for the 320^2 rows (about 15 s each)")
    pb = _problem_for_row(row)
    l1, li, _ = O.solve_errors(pb)
    # 5 significant digits are printed; Table 1's single-grid 80^2 row sits one unit of the
    # last digit away (rounding of the paper's own FP64 run), hence 2e-4 relative.
    assert l1 == pytest.approx(row["l1"], rel=2e-4)
    assert li == pytest.approx(row["linf"], rel=2e-4)


# --------------------------------------------------------------------------- WENO5 interpolation (Sec. 2.2.1)

def test_lagrange_mode_is_the_degree4_interpolant():
    # eq. (lwlag): sum_k C_k(x) P_k(x) reproduces the degree-4 Lagrange polynomial on the big stencil
    rng = np.random.default_rng(4)
    P = np.polynomial.Polynomial
    for _ in range(100):
        u = rng.normal(size=5)
        s = rng.uniform(-0.5, 0.5)
        ref = P.fit(np.arange(-2, 3), u, 4).convert()(s)
        assert O.interp(u, s, lagrange=True) == pytest.approx(ref, rel=1e-12, abs=1e-13)


def test_linear_weights_at_known_points():
    # at the midpoint s = -1/2 the degree-4 Lagrange basis on nodes -2..2 takes the values
    # (-5, 60, 90, -20, 3)/128 (products prod_{m != j} (s - m)/(j - m) worked by hand).
    for j, wt in enumerate(np.array([-5, 60, 90, -20, 3]) / 128.0):
        e = np.zeros(5)
        e[j] = 1.0
        assert O.interp(e, -0.5, lagrange=True) == pytest.approx(wt, abs=1e-15)


def test_weno_interpolation_exact_for_quadratics():
    # every P_k reproduces a quadratic and the nonlinear weights sum to one
    rng = np.random.default_rng(5)
    for _ in range(50):
        c = rng.normal(size=3)
        u = np.polyval(c, np.arange(-2, 3))
        s = rng.uniform(-0.5, 0.5)
        assert O.interp(u, s) == pytest.approx(np.polyval(c, s), rel=1e-12, abs=1e-12)


def test_weno_interpolation_is_non_oscillatory_on_a_step():
    # a jump between x_{i+1} and x_{i+2}: the value near x_i follows the smooth side
    u = np.array([0.0, 0.0, 0.0, 0.0, 1.0])
    for s in (-0.5, -0.25, 0.0, 0.25, 0.49):
        assert abs(O.interp(u, s, eps=1e-6)) < 1e-6


def test_midpoint_goes_to_the_right_node():
    # x in [x_{i-1/2}, x_{i+1/2}) (Sec. 2.2.1): the midpoint between coarse nodes i-1 and i
    # belongs to node i with s = -1/2, i.e. stencil u_{i-2..i+2}.
    pb = W.Problem(d=1, lo=(0.0,), hi=(1.0,), flux=W.FLUX_ADVECTION, flux_params=(1.0,), ic=W.IC_SINE,
                   ic_params=(0, 1, 2 * math.pi, 0), nr=8, nl=1, T=0.1, prolong=W.PROLONG_LAGRANGE5)
    rng = np.random.default_rng(6)
    u = rng.normal(size=8)
    fine = O.prolong(pb, (0,), u)          # coarse n = 8 -> fine 16
    P = np.polynomial.Polynomial
    for i in range(2, 6):
        J = 2 * i - 1                      # midpoint between i-1 and i
        right = P.fit(np.arange(-2, 3), u[i - 2:i + 3], 4).convert()(-0.5)
        assert fine[J] == pytest.approx(right, abs=1e-13)
        assert fine[2 * i] == pytest.approx(u[i], abs=1e-14)


def test_prolongation_of_tensor_quartics_is_exact_inside():
    # Lagrange prolongation reproduces tensor products of quartics wherever no stencil wraps
    pb = W.c3_advection_3d(nr=8, nl=2).replace(prolong=W.PROLONG_LAGRANGE5, lo=(0.0,) * 3, hi=(1.0,) * 3)
    rng = np.random.default_rng(7)
    polys = [rng.normal(size=5) for _ in range(3)]
    lay = O.grid_layout(pb)
    st = np.zeros(O.total_nodes(pb))
    for lev, c, shp, off in lay:
        x = [np.arange(n) / n for n in shp]
        vals = np.einsum("i,j,k->kji", *[np.polyval(polys[k], x[k]) for k in range(3)])
        st[off:off + vals.size] = vals.ravel()
    U = O.prolong_combine(pb, st).reshape((32,) * 3)
    xf = np.arange(32) / 32
    ref = np.einsum("i,j,k->kji", *[np.polyval(polys[k], xf) for k in range(3)])
    sl = slice(10, 19)                     # coarse stencils i-2..i+2 stay inside [0, 8)
    assert np.max(np.abs(U[sl, sl, sl] - ref[sl, sl, sl])) < 1e-12


def test_pointwise_combination_matches_full_combination():
    pb = W.c2_burgers_2d(nr=4, nl=3, precision=W.PREC_FP64, T=0.05)
    U, st, _ = O.solve(pb)
    rng = np.random.default_rng(8)
    J = rng.integers(0, pb.n_fine, size=(40, 2)).astype(np.int32)
    pts = O.prolong_combine_points(pb, st, J)
    full = U.reshape(pb.n_fine, pb.n_fine)
    assert np.max(np.abs(pts - full[J[:, 1], J[:, 0]])) < 1e-14


# --------------------------------------------------------------------------- invariants and convergence

def test_burgers_conserves_each_grid_sum():
    # periodic telescoping of eq. (2.9): sum_j U_g[j] is constant in time (any weights)
    pb = W.c2_burgers_2d(nr=8, nl=3, precision=W.PREC_FP64, T=0.3)
    st0 = O.restrict(pb)
    st = st0.copy()
    O.evolve(pb, st)
    for lev, c, shp, off in O.grid_layout(pb):
        n = int(np.prod(shp))
        assert abs(st[off:off + n].sum() - st0[off:off + n].sum()) < 1e-12 * n


def test_shift_by_one_root_cell_shifts_the_result_exactly():
    pb = W.c2_burgers_2d(nr=8, nl=3, precision=W.PREC_FP64, T=0.05)
    st = O.restrict(pb)
    sh = st.copy()
    for lev, c, shp, off in O.grid_layout(pb):
        a = sh[off:off + int(np.prod(shp))].reshape(tuple(reversed(shp)))
        a = np.roll(a, 1 << lev[0], axis=1)       # one root cell along x (direction 1)
        sh[off:off + a.size] = a.ravel()
    O.evolve(pb, st)
    O.evolve(pb, sh)
    U = O.prolong_combine(pb, st).reshape(pb.n_fine, pb.n_fine)
    Us = O.prolong_combine(pb, sh).reshape(pb.n_fine, pb.n_fine)
    assert np.array_equal(np.roll(U, 1 << pb.nl, axis=1), Us)


def test_single_grid_weno5_converges_at_fifth_order():
    # Sec. 3 opening: dt = dx^(5/3) exposes the fifth-order spatial error
    errs = []
    for n in (20, 40, 80):
        pb = W.Problem(d=2, lo=(0.0, 0.0), hi=(2.0, 2.0), flux=W.FLUX_ADVECTION, flux_params=(1.0, 1.0),
                       ic=W.IC_SINE, ic_params=(0.0, 1.0, math.pi, 0.0), nr=n, nl=0, T=0.25,
                       dt_mode=W.DT_POW53)
        errs.append(O.solve_errors(pb)[0])
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 4.5 < orders[-1] < 5.5, orders


def test_c1_exact_solution_is_the_initial_condition():
    # translation by (1, 1) on the period-2 square returns u0
    pb = W.c1_advection_2d()
    ex = O.exact_fine(pb, 1.0)
    j = np.arange(pb.n_fine) * 2.0 / pb.n_fine
    u0 = np.sin(math.pi * (j[None, :] + j[:, None]))
    assert np.max(np.abs(ex.reshape(pb.n_fine, pb.n_fine) - u0)) < 1e-12


def test_c1_full_solve_is_accurate():
    l1, li, stats = O.solve_errors(W.c1_advection_2d())
    assert stats["steps"] == 64                   # dt = 0.5 / (1/h + 1/h) = 1/64
    assert l1 < 0.05 and li < 0.2               # root grid of 4 cells: 4 nodes per wavelength


def test_burgers_exact_solution_satisfies_the_characteristics():
    pb = W.c2_burgers_2d(precision=W.PREC_FP64, T=0.15)
    rng = np.random.default_rng(9)
    for _ in range(20):
        x = rng.uniform(-1, 1, size=2)
        w = O.exact(pb, x, 0.15)
        c0, A, kap, ph = pb.ic_params
        assert w == pytest.approx(c0 + A * math.sin(kap * (x.sum() - 2 * w * 0.15) + ph), abs=1e-14)


def test_vlasov_exact_solution_follows_the_characteristics():
    # x' = v, v' = E(x): with a zero field the solution is free streaming f0(x - v t, v); with the
    # field, f is constant along characteristics, so it stays positive and bounded by max f0.
    pb = W.c4_vlasov_4d(precision=W.PREC_FP64)
    pb0 = pb.replace(flux_params=(0.0, 0.5))
    x = np.array([1.0, 2.0, 0.5, -0.25])
    y = x.copy()
    y[:2] -= x[2:] * 1.0
    assert O.exact(pb0, x, 1.0) == pytest.approx(O.exact(pb0, y, 0.0), rel=1e-13)
    rng = np.random.default_rng(10)
    fmax = (1 + pb.ic_params[0]) / (2 * math.pi)
    for _ in range(10):
        x = rng.uniform([0, 0, -3, -3], [12, 12, 3, 3])
        f = O.exact(pb, x, 1.0)
        assert 0 < f <= fmax


def test_sparse_grid_burgers_converges():
    # sparse-grid WENO errors fall quickly with the root grid (Table ex3aweno trend)
    e = [O.solve_errors(W.paper_example3a(nr * 8, nr=nr, nl=3))[0] for nr in (5, 10)]
    assert e[1] < e[0] / 10


# --------------------------------------------------------------------------- 4D Vlasov branch (Sec. 3.4 setting)

def _vlasov_single(n, T=0.5, amp=0.01):
    """The 4D phase-space workload on one full grid of n^4 nodes (finest level 0)."""
    return W.c4_vlasov_4d(nr=n, nl=0, precision=W.PREC_FP64, T=T).replace(flux_params=(amp, 0.5))


def _foot_by_scipy(x, t, amp, kE):
    """Foot of the characteristic through x at time t: x_k' = v_k, v_k' = amp sin(kE x_k), integrated
    back to 0 by a library ODE solver (DOP853), independently of the oracle's own integrator."""
    from scipy.integrate import solve_ivp
    y = np.array(x, dtype=float)
    m = len(x) // 2
    for k in range(m):
        sol = solve_ivp(lambda s, z: [z[1], amp * math.sin(kE * z[0])], (t, 0.0), [x[k], x[m + k]],
                        method="DOP853", rtol=1e-13, atol=1e-14)
        y[k], y[m + k] = sol.y[0, -1], sol.y[1, -1]
    return y


def _maxwell_cos(pb, y):
    """f0 of the 4D workload written out: exp(-|v|^2/2)/(2 pi) (1 + a cos(k x1 + p1) cos(k x2 + p2))."""
    a, k, p1, p2 = pb.ic_params[:4]
    return math.exp(-0.5 * (y[2] ** 2 + y[3] ** 2)) / (2 * math.pi) * (
        1 + a * math.cos(k * y[0] + p1) * math.cos(k * y[1] + p2))


@pytest.mark.parametrize("amp", [0.01, 0.3, -0.3])
def test_vlasov_exact_solution_matches_an_independent_characteristic_solve(amp):
    # f is constant along x' = v, v' = E(x): the oracle's exact value is f0 at the foot.  The foot
    # here comes from scipy's DOP853 and f0 is written out; a flipped field sign, swapped x/v
    # roles or a wrong Maxwellian normalisation in the oracle's exact solution fails this.
    pb = W.c4_vlasov_4d(precision=W.PREC_FP64).replace(flux_params=(amp, 0.5), ic_params=(0.05, 0.5, 0.3, 1.1))
    rng = np.random.default_rng(20)
    for _ in range(6):
        x = rng.uniform([0, 0, -4, -4], [4 * math.pi, 4 * math.pi, 4, 4])
        for t in (0.4, 1.0):
            ref = _maxwell_cos(pb, _foot_by_scipy(x, t, amp, 0.5))
            assert O.exact(pb, x, t) == pytest.approx(ref, rel=1e-11, abs=1e-15)


def test_vlasov_characteristics_conserve_the_pendulum_energy():
    # Each (x_k, v_k) pair is a pendulum x'' = amp sin(kE x): H = v^2/2 + (amp/kE) cos(kE x) is
    # constant along it.  Read the foot back through f0 = exp(-|v|^2/2)(...) with the x perturbation
    # switched off and one velocity zero, so f0 = exp(-v_1^2/2)/(2 pi) fixes |v_1| at the foot.
    amp, kE = 0.3, 0.5
    pb = W.c4_vlasov_4d(precision=W.PREC_FP64).replace(flux_params=(amp, kE), ic_params=(0.0, 0.5, 0.0, 0.0))
    rng = np.random.default_rng(21)
    for _ in range(10):
        x1, v1 = rng.uniform(0, 4 * math.pi), rng.uniform(-2, 2)
        t = 1.0
        f = O.exact(pb, np.array([x1, 0.0, v1, 0.0]), t)
        v_foot_sq = -2.0 * math.log(f * 2 * math.pi)
        # x_2 = 0, v_2 = 0 is a fixed point of the second pendulum (sin 0 = 0), so only pair 1 moves
        x_foot = _foot_by_scipy([x1, 0.0, v1, 0.0], t, amp, kE)[0]
        H_now = 0.5 * v1 * v1 + amp / kE * math.cos(kE * x1)
        H_foot = 0.5 * v_foot_sq + amp / kE * math.cos(kE * x_foot)
        assert H_foot == pytest.approx(H_now, abs=1e-10)


def test_vlasov_maxwellian_has_unit_velocity_integral():
    # the Maxwellian exp(-|v|^2/2)/(2 pi) integrates to 1 over v in R^2; the periodic node sum over
    # [-6, 6) misses the tail beyond |v_k| = 6 and the node v_k = 6 (together 7e-9); the perturbation
    # 1 + a cos(x1/2) cos(x2/2) averages to 1 over the x period 4 pi
    n = 24
    pb = W.c4_vlasov_4d(nr=n, nl=0, precision=W.PREC_FP64).replace(ic_params=(0.3, 0.5, 0.7, 0.2))
    f = O.restrict(pb).reshape(n, n, n, n)           # axes (v2, v1, x2, x1)
    hx, hv = 4 * math.pi / n, 12.0 / n
    rho = f.sum(axis=(0, 1)) * hv * hv               # density at every x node
    a, k, p1, p2 = pb.ic_params
    xs = np.arange(n) * hx
    pert = 1 + a * np.cos(k * xs[None, :] + p1) * np.cos(k * xs[:, None] + p2)
    assert np.max(np.abs(rho - pert)) < 1e-8
    assert rho.sum() * hx * hx == pytest.approx((4 * math.pi) ** 2, rel=1e-8)


def test_vlasov_solve_converges_to_the_characteristic_solution():
    # The oracle's march (flux v_k f in x_k, E_k(x_k) f in v_k, eq. (1) in phase space) on full
    # grids n^4 at T = 0.5 against the exact solution: errors fall with n (observed 1.0e-5, 4.4e-6,
    # 1.5e-6 at n = 8, 12, 16; pre-asymptotic on these coarse grids, local order > 3 at the end).
    errs = []
    for n in (8, 12, 16):
        l1, _, st = O.solve_errors(_vlasov_single(n))
        errs.append(l1)
    assert errs[0] < 2e-5 and errs[2] < 2e-6, errs
    order = math.log(errs[1] / errs[2]) / math.log(16 / 12)
    assert order > 3.0, (errs, order)


@pytest.mark.parametrize("amp", [0.01, 0.3])
def test_vlasov_solve_follows_the_field_sign(amp):
    # the same solve measured against the exact solution of the opposite field is far worse: a sign
    # error in E_k f (or a field in the wrong direction) would swap these two errors
    n = 16 if amp == 0.01 else 12
    pb = _vlasov_single(n, amp=amp)
    U, _, st = O.solve(pb)
    l1 = O.norms(U, O.exact_fine(pb, st["t"]))[0]
    l1_flip = O.norms(U, O.exact_fine(pb.replace(flux_params=(-amp, 0.5)), st["t"]))[0]
    l1_free = O.norms(U, O.exact_fine(pb.replace(flux_params=(0.0, 0.5)), st["t"]))[0]
    assert l1_flip > 8 * l1 and l1_free > 4 * l1, (l1, l1_flip, l1_free)
