"""Pins of the oracle's Vlasov-Boltzmann model (Sec. 3.4, Example 5): the field E = -x, the linear
relaxation source (mu_inf(v) rho(x) - f) / tau, zero boundary values, and the entropy functionals
H_2 and H_log relative to the stationary state M.

Each pin comes from outside the oracle's own formulas: the exact characteristics of the harmonic
field (a rotation in phase space), the moments a Maxwellian must have, the stationary state
printed in the paper, the polynomial a three-stage third-order Runge-Kutta step applies to a linear
system, and, for the zero boundary, the same grid padded with zeros inside a periodic one."""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle as O
import sgw_inputs as I


def _node_axis(n, lo=-5.0, hi=5.0):
    return lo + (hi - lo) / n * np.arange(n)


def _coords(d, n):
    """Node coordinates of an n^d grid, direction 0 fastest: one flat array per direction."""
    g = _node_axis(n)
    axes = np.meshgrid(*([g] * d), indexing="ij")  # axes[k] varies along array axis k
    return [axes[d - 1 - k].ravel() for k in range(d)]


def _stationary(d, n, theta=1.0):
    """The stationary state of Example 5 on the nodes: exp(-(|v|^2/2 + |x|^2/2)/theta) over
    (2 pi theta)^(m/2) times the integral of exp(-|x|^2/(2 theta)) over the x domain, m = d/2."""
    m = d // 2
    c = _coords(d, n)
    x2 = sum(a * a for a in c[:m])
    v2 = sum(a * a for a in c[m:])
    zx = (math.sqrt(2.0 * math.pi * theta) * erf(5.0 / math.sqrt(2.0 * theta))) ** m
    return np.exp(-(0.5 * v2 + 0.5 * x2) / theta) / ((2.0 * math.pi * theta) ** (m / 2) * zx)


def test_normalisation_makes_unit_mass():
    """The constant s of the initial condition gives a unit integral; the nodal sum approximates it
    to within the Gaussian's tail."""
    for d, n in ((2, 80), (4, 20)):
        pb = I.paper_example5(d, nr=n, nl=0)
        f0 = O.restrict(pb)
        assert abs(f0.sum() * (10.0 / n) ** d - 1.0) < 1e-4


def test_harmonic_field_rotates_phase_space():
    """Without relaxation, E = -x makes the characteristics x(t) = x0 cos t + v0 sin t,
    v(t) = -x0 sin t + v0 cos t, so f(t, x, v) = f0(x cos t - v sin t, x sin t + v cos t).
    The single-grid solution converges to that at better than third order."""
    errs = []
    for n in (40, 80):
        pb = I.paper_example5(2, nr=n, nl=0, T=math.pi / 2).replace(relax_tau=0.0)
        U, _, stats = O.solve(pb)
        x, v = _coords(2, n)
        t = stats["t"]
        x0 = x * math.cos(t) - v * math.sin(t)
        v0 = x * math.sin(t) + v * math.cos(t)
        ex = pb.ic_params[0] * np.sin(0.5 * x0 ** 2) ** 2 * np.exp(-0.5 * (x0 ** 2 + v0 ** 2))
        errs.append(np.abs(U - ex).mean())
    assert errs[1] < 3e-4
    assert errs[0] / errs[1] > 2 ** 3.5


def test_harmonic_4d_transport_separates_into_two_planes():
    """In 4D the transport acts on the planes (x1, v1) = directions (1, 3) and (x2, v2) =
    directions (2, 4) separately: with linear weights the operator is linear, so on a product
    f(x1, v1) g(x2, v2) it is L2(f) g + f L2(g), where L2 is the 2D operator."""
    n = 12
    rng = np.random.default_rng(11)
    p4 = I.paper_example5(4, nr=n, nl=0).replace(relax_tau=0.0, linear=True)
    p2 = I.paper_example5(2, nr=n, nl=0).replace(relax_tau=0.0, linear=True)
    f = rng.uniform(0.0, 1.0, (n, n))  # [v1, x1]
    g = rng.uniform(0.0, 1.0, (n, n))  # [v2, x2]
    Lf = O.rhs(p2, [0, 0], f.ravel()).reshape(n, n)
    Lg = O.rhs(p2, [0, 0], g.ravel()).reshape(n, n)
    # 4D array axes [v2, v1, x2, x1]
    u = np.einsum("ac,bd->badc", f, g)
    L4 = O.rhs(p4, [0] * 4, u.ravel()).reshape(n, n, n, n)
    want = np.einsum("ac,bd->badc", Lf, g) + np.einsum("ac,bd->badc", f, Lg)
    assert np.abs(L4 - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("flux,fp", [(I.FLUX_BURGERS, ()), (I.FLUX_ADVECTION, (1.0, 0.0)),
                                     (I.FLUX_ADVECTION, (-0.7, 0.0))])
def test_zero_boundary_sweep_equals_zero_padded_periodic(flux, fp):
    """A zero boundary reads 0 beyond either end: the spatial operator equals that of the same
    line padded with three zeros on each side inside a periodic grid (same spacing), on the
    original nodes.  The data are constant along direction 2, whose flux is then 0."""
    rng = np.random.default_rng(3)
    n, h = 12, 0.25
    pb = I.Problem(d=2, lo=(0.0, 0.0), hi=(n * h, n * h), flux=flux, flux_params=fp, ic=0, ic_params=(), nr=n,
                   nl=0, T=0.1, bc=(I.BC_ZERO, I.BC_PERIODIC))
    row = rng.uniform(0.2, 1.0, n)
    L = O.rhs(pb, [0, 0], np.tile(row, n)).reshape(n, n)
    m = n + 6
    pp = pb.replace(lo=(-3 * h, -3 * h), hi=((n + 3) * h, (n + 3) * h), nr=m, bc=())
    rowp = np.concatenate([np.zeros(3), row, np.zeros(3)])
    Lp = O.rhs(pp, [0, 0], np.tile(rowp, m)).reshape(m, m)
    assert np.array_equal(L[0], Lp[0, 3:-3])
    assert np.array_equal(L, np.tile(L[0], (n, 1)))
    # and it is not the periodic operator
    Lper = O.rhs(pb.replace(bc=()), [0, 0], np.tile(row, n)).reshape(n, n)
    assert np.abs(Lper[0] - L[0]).max() > 1e-3


@pytest.mark.parametrize("lev,nrp,off", [((0, 0), 14, 12), ((1, 0), 11, 6)])
def test_zero_boundary_prolongation_equals_zero_padded_periodic(lev, nrp, off):
    """The prolongation reads 0 beyond the ends of a zero-boundary direction: it equals the
    prolongation of the line padded with three coarse zeros on each side in a periodic grid, on
    the fine nodes of the original line.  Direction 2 holds constants (reproduced by the
    interpolation to rounding)."""
    rng = np.random.default_rng(7)
    n, nl = 8, 2
    pb = I.Problem(d=2, lo=(0.0, 0.0), hi=(1.0, 1.0), flux=0, flux_params=(1.0, 1.0), ic=0, ic_params=(), nr=n,
                   nl=nl, T=0.1, bc=(I.BC_ZERO, I.BC_PERIODIC))
    row = rng.uniform(-1.0, 1.0, n << lev[0])
    fine = O.prolong(pb, list(lev), np.tile(row, n << lev[1])).reshape(n << nl, n << nl)
    pp = pb.replace(nr=nrp, bc=())
    rowp = np.concatenate([np.zeros(3), row, np.zeros(3)])
    assert rowp.size == nrp << lev[0]
    finep = O.prolong(pp, list(lev), np.tile(rowp, nrp << lev[1])).reshape(nrp << nl, nrp << nl)
    assert np.array_equal(fine[0], finep[0, off:off + (n << nl)])
    assert np.abs(fine - fine[0]).max() < 1e-15 * 16


@pytest.mark.parametrize("d,nr,nl", [(2, 4, 3), (3, 4, 2)])
def test_zero_boundary_point_prolongation_matches_sweeps(d, nr, nl):
    """The tensor-product point evaluation and the direction-by-direction refinement read the same
    zeros beyond the ends."""
    rng = np.random.default_rng(5)
    pb = I.Problem(d=d, lo=(0.0,) * d, hi=(1.0,) * d, flux=0, flux_params=(1.0,) * d, ic=0, ic_params=(),
                   nr=nr, nl=nl, T=0.1, bc=(I.BC_ZERO,) * d)
    st = rng.uniform(0.0, 1.0, O.total_nodes(pb))
    U = O.prolong_combine(pb, st)
    nf = nr << nl
    J = rng.integers(0, nf, size=(300, d)).astype(np.int32)
    J[:d, :] = 0
    J[d:2 * d, :] = nf - 1
    P = O.prolong_combine_points(pb, st, J)
    idx = sum(J[:, k].astype(np.int64) * nf ** k for k in range(d))
    assert np.abs(P - U[idx]).max() < 1e-14


def _relax_problem(d, n, theta, T):
    """Relaxation alone: zero-speed advection (no transport) plus the source, dt = h^(5/3)."""
    return I.Problem(d=d, lo=(-5.0,) * d, hi=(5.0,) * d, flux=I.FLUX_ADVECTION, flux_params=(0.0,) * d, ic=0,
                     ic_params=(), nr=n, nl=0, T=T, dt_mode=I.DT_POW53, bc=(I.BC_ZERO,) * d, relax_tau=1.0,
                     relax_theta=theta)


@pytest.mark.parametrize("d,n,theta,tol", [(2, 16, 1.0, 1e-4), (2, 24, 0.5, 1e-7), (4, 16, 1.0, 1e-4),
                                           (4, 16, 0.5, 1e-7)])
def test_relaxation_drives_to_the_maxwellian_at_fixed_density(d, n, theta, tol):
    """Relaxation keeps rho and drives f to mu_inf(v) rho(x): long after tau the velocity profile
    at each x is a Maxwellian of unit mass whose second moment per velocity direction is theta
    (up to the Gaussian's tail beyond |v| = 5 and the nodal quadrature)."""
    rng = np.random.default_rng(9)
    pb = _relax_problem(d, n, theta, 20.0)
    f0 = rng.uniform(0.0, 1.0, n ** d)
    st = f0.copy()
    O.evolve(pb, st)
    h = 10.0 / n
    hv = h ** (d // 2)
    nx = n ** (d // 2)
    F0, F = f0.reshape(-1, nx), st.reshape(-1, nx)  # [velocity node, x node]
    rho0, rho = F0.sum(0) * hv, F.sum(0) * hv
    assert np.abs(rho / rho0 - 1.0).max() < tol
    vc = _coords(d // 2, n)
    for vk in vc:
        second = (vk[:, None] ** 2 * F).sum(0) * hv / rho
        assert np.abs(second - theta).max() < tol
        first = (vk[:, None] * F).sum(0) * hv / rho
        assert np.abs(first).max() < 0.01  # the node set is symmetric up to the end node at -5


def test_relaxation_step_is_the_rk3_polynomial():
    """One Runge-Kutta step of du/dt = A u with A u = (mu_inf rho(u) - u)/tau applies
    P(dt A) = I + dt A + (dt A)^2/2 + (dt A)^3/6, the third-order TVD scheme's stability polynomial;
    the source must take rho from each stage's input."""
    d, n, theta, tau = 2, 10, 0.7, 0.5
    pb = _relax_problem(d, n, theta, 1.0).replace(relax_tau=tau)
    h = 10.0 / n
    dt = h ** (5.0 / 3.0)
    pb = pb.replace(T=dt)
    rng = np.random.default_rng(13)
    f0 = rng.uniform(0.0, 1.0, n * n)
    st = f0.copy()
    stats = O.evolve(pb, st)
    assert stats["steps"] == 1
    v = _coords(1, n)[0]
    mu = np.exp(-v * v / (2 * theta)) / math.sqrt(2 * math.pi * theta)

    def A(u):
        F = u.reshape(n, n)  # [v, x]
        rho = F.sum(0) * h
        return ((mu[:, None] * rho[None, :] - F) / tau).ravel()

    a1 = A(f0)
    a2 = A(a1)
    a3 = A(a2)
    want = f0 + dt * a1 + dt ** 2 / 2 * a2 + dt ** 3 / 6 * a3
    assert np.abs(st - want).max() < 1e-14


def test_stationary_state_is_a_fixed_point():
    """M(x, v) is the stationary state of the full model: the spatial operator, transport and
    relaxation together, vanishes on it up to the discretisation error, which falls faster than
    h^3 (in 2D); a field of another sign or shape leaves an O(1) residual."""
    res = []
    for n in (20, 40, 80):
        pb = I.paper_example5(2, nr=n, nl=0)
        res.append(np.abs(O.rhs(pb, [0, 0], _stationary(2, n))).max())
    assert res[0] / res[1] > 8 and res[1] / res[2] > 8
    assert res[2] < 1e-4
    pb = I.paper_example5(2, nr=80, nl=0)
    assert np.abs(O.rhs(pb.replace(flux=I.FLUX_VLASOV, flux_params=(-1.0, 1.0)), [0, 0],
                        _stationary(2, 80))).max() > 1e-2
    r4 = [np.abs(O.rhs(I.paper_example5(4, nr=n, nl=0), [0] * 4, _stationary(4, n))).max() for n in (10, 20)]
    assert r4[0] / r4[1] > 8


def test_entropies_at_the_stationary_state():
    """H = f/M is 1 at f = M: H_2 is the mass of M (1 up to the tail) and H_log is 0; at f = 2M
    they are 4 and 2 log 2 times that mass."""
    for d, n in ((2, 40), (4, 12)):
        pb = I.paper_example5(d, nr=n, nl=0)
        M = _stationary(d, n)
        mass = M.sum() * (10.0 / n) ** d
        assert abs(mass - 1.0) < 1e-4
        h2, hl = O.entropies(pb, M)
        assert abs(h2 - mass) < 1e-12 and abs(hl) < 1e-14
        h2, hl = O.entropies(pb, 2 * M)
        assert abs(h2 - 4 * mass) < 1e-12 and abs(hl - 2 * math.log(2) * mass) < 1e-12
        # H log H is taken as 0 where f <= 0
        z = M.copy()
        z[: z.size // 2] = -1.0
        _, hl = O.entropies(pb, z)
        assert abs(hl) < 1e-14


def test_example5_mass_and_entropy_decay():
    """The model conserves mass up to the boundary outflow of the Gaussian's tail, and both entropy
    functionals decay towards equilibrium; the sparse-grid solution follows the single grid."""
    out = {}
    for nl, nr in ((0, 80), (3, 10)):
        pb = I.paper_example5(2, nr=nr, nl=nl)
        vals = []
        for T in (0.25, 0.5):
            U, _, _ = O.solve(pb.replace(T=T))
            vals.append((U.sum() * (10.0 / 80) ** 2, *O.entropies(pb, U)))
        U0 = O.prolong_combine(pb, O.restrict(pb))
        vals.insert(0, (U0.sum() * (10.0 / 80) ** 2, *O.entropies(pb, U0)))
        for m, h2, hl in vals:
            assert abs(m - 1.0) < 1e-3
        assert vals[0][1] > vals[1][1] > vals[2][1]
        assert vals[0][2] > vals[1][2] > vals[2][2]
        out[nl] = U
    assert np.abs(out[3] - out[0]).mean() < 2e-3
