"""Pins of the oracle's Vlasov-Maxwell system (Sec. 3.4, Example 6): transport in (x_2, xi_1, xi_2)
with the Lorentz force (E_1 + xi_2 B_3, E_2 - xi_1 B_3), the field equations B_3' = dE_1/dx_2,
E_1' = dB_3/dx_2 - j_1, E_2' = -j_2 with the currents j = int f xi dxi, and the combination of the
grids' fields.

Each pin is a closed form of the continuous system that the discretisation must approach: a
standing electromagnetic wave without particles, the moment equations of a uniform plasma in a
uniform magnetic field (a linear ODE solved by the matrix exponential), free streaming along x_2,
and the combination of exactly sampled fields."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
import sgw_inputs as I


def _single(n, T, L=2 * math.pi / 0.2, beta=0.05, b=0.0):
    return I.Problem(d=3, lo=(0.0, -1.2, -1.2), hi=(L, 1.2, 1.2), flux=I.FLUX_VLASOV_MAXWELL, flux_params=(),
                     ic=I.IC_VM, ic_params=(beta, b, 1.0, 0.0, 0.0, 0.2), nr=n, nl=0, T=T, cfl=0.4)


def test_initial_condition_has_unit_density_and_opposite_drifts():
    """f0 integrates to 1 over xi (per x_2) and its beams drift at +v01 and -v02, so with delta =
    1/2 the current is 0; B_3 = b sin(k0 x_2)."""
    pb = I.paper_example6(nr=40, nl=0)
    f = O.restrict(pb).reshape(40, 40, 40)  # [xi_2, xi_1, x_2]
    h = 2.4 / 40
    xi = -1.2 + h * np.arange(40)
    rho = f.sum(axis=(0, 1)) * h * h
    assert np.abs(rho - 1.0).max() < 1e-6
    j1 = (f * xi[None, :, None]).sum(axis=(0, 1)) * h * h
    assert np.abs(j1).max() < 1e-12
    one = pb.replace(ic_params=(0.01, 0.001, 1.0, 0.3, 0.3, 0.2))  # delta = 1: one beam at +0.3
    f1 = O.restrict(one).reshape(40, 40, 40)
    assert abs((f1 * xi[None, :, None]).sum(axis=(0, 1))[0] * h * h - 0.3) < 1e-6
    fl = O.fields_init(pb)
    x = pb.hi[0] / 40 * np.arange(40)
    assert np.array_equal(fl[:40], 0.001 * np.sin(0.2 * x)) and not fl[40:].any()


def test_standing_wave_without_particles():
    """f = 0: no currents, and B_3 = b sin(k0 x) cos(k0 t), E_1 = b cos(k0 x) sin(k0 t) solve the
    field equations; the single-grid fields converge to it at better than h^4, E_2 stays 0."""
    errs = []
    for n in (16, 32):
        pb = _single(n, 2.0, b=0.1)
        st = np.zeros(O.total_nodes(pb))
        fl = O.fields_init(pb)
        t = O.evolve(pb, st, fields=fl)["t"]
        x = pb.hi[0] / n * np.arange(n)
        eB = np.abs(fl[:n] - 0.1 * np.sin(0.2 * x) * np.cos(0.2 * t)).max()
        eE = np.abs(fl[n:2 * n] - 0.1 * np.cos(0.2 * x) * np.sin(0.2 * t)).max()
        assert not fl[2 * n:].any() and not st.any()
        errs.append(max(eB, eE))
    assert errs[1] < 1e-6
    assert errs[0] / errs[1] > 2 ** 4


def test_uniform_plasma_in_a_uniform_magnetic_field():
    """f independent of x_2, uniform E and B_3: B_3 stays constant, and the moments obey
    E' = -j, j_1' = n E_1 + B_3 j_2, j_2' = n E_2 - B_3 j_1 (n = int f dxi), a linear ODE whose
    solution is the matrix exponential.  A wrong sign of the electric or magnetic force, or of the
    current in the field equations, moves E by 0.05 or more."""
    n, beta, u, Bc, e = 24, 0.05, (0.2, -0.1), 0.5, (0.05, -0.03)
    pb = _single(n, 2.0, L=100.0, beta=beta)
    h = 2.4 / n
    xi = -1.2 + h * np.arange(n)
    X1, X2 = np.meshgrid(xi, xi, indexing="xy")  # [xi_2, xi_1]
    f2 = np.exp(-((X1 - u[0]) ** 2 + (X2 - u[1]) ** 2) / beta) / (math.pi * beta)
    st = np.ascontiguousarray(np.broadcast_to(f2.reshape(n, n, 1), (n, n, n)).ravel())
    fl = np.zeros(3 * n)
    fl[:n], fl[n:2 * n], fl[2 * n:] = Bc, e[0], e[1]
    dens = f2.sum() * h * h
    j0 = ((X1 * f2).sum() * h * h, (X2 * f2).sum() * h * h)
    t = O.evolve(pb, st, fields=fl)["t"]
    A = np.array([[0, 0, -1, 0], [0, 0, 0, -1], [dens, 0, 0, Bc], [0, dens, -Bc, 0]])
    y = expm(A * t) @ np.array([e[0], e[1], j0[0], j0[1]])
    assert np.all(fl[:n] == Bc)
    assert np.ptp(fl[n:2 * n]) == 0.0 and np.ptp(fl[2 * n:]) == 0.0
    assert abs(fl[n] - y[0]) < 2e-3 and abs(fl[2 * n] - y[1]) < 2e-3
    assert abs(y[0] - e[0]) > 0.1  # the fields moved


def test_free_streaming_along_x2():
    """No fields and a dilute f = A g(x_2) h(xi_1) k(xi_2), h even: f(t) = f0(x_2 - xi_2 t, xi) up to
    the fields its own current raises (order A^2)."""
    n, A, k0 = 24, 1e-4, 0.2
    pb = _single(n, 3.0)
    x = pb.hi[0] / n * np.arange(n)
    xi = -1.2 + 2.4 / n * np.arange(n)

    def f_of(t):
        X2, XI1, XI2 = np.meshgrid(x, xi, xi, indexing="ij")  # [x_2, xi_1, xi_2]
        v = A * (1 + 0.5 * np.sin(k0 * (X2 - XI2 * t))) * np.exp(-XI1 ** 2 / 0.1) * np.exp(-XI2 ** 2 / 0.2)
        return np.ascontiguousarray(v.transpose(2, 1, 0)).ravel()

    st = f_of(0.0)
    fl = np.zeros(3 * n)
    t = O.evolve(pb, st, fields=fl)["t"]
    ex = f_of(t)
    assert np.abs(st - ex).max() < 2e-5 * np.abs(ex).max()
    assert np.abs(fl).max() < 1e-5


def test_fields_combination_of_exact_samples():
    """Grids holding exact samples of smooth fields combine to those fields on the finest x_2 grid,
    to the interpolation error of the coarsest x_2 grid; grids at the finest x_2 level enter
    unchanged."""
    pb = I.paper_example6(nr=8, nl=3)
    lay = O.grid_layout(pb)
    fl = np.zeros(O.total_fields(pb))
    o = 0
    for level, coef, shape, off in lay:
        n0 = shape[0]
        x = pb.hi[0] / n0 * np.arange(n0)
        fl[o:o + n0] = np.sin(0.2 * x)
        fl[o + n0:o + 2 * n0] = np.cos(0.4 * x)
        fl[o + 2 * n0:o + 3 * n0] = 0.3
        o += 3 * n0
    out = O.fields_combine(pb, fl)
    X = pb.hi[0] / pb.n_fine * np.arange(pb.n_fine)
    assert np.abs(out[0] - np.sin(0.2 * X)).max() < 1e-4
    assert np.abs(out[1] - np.cos(0.4 * X)).max() < 1e-3
    assert np.abs(out[2] - 0.3).max() < 1e-14
    # only finest-level grids: the combination of the grids with l_1 = N_L is their signed sum
    fl2 = np.zeros_like(fl)
    o, want = 0, np.zeros(pb.n_fine)
    rng = np.random.default_rng(3)
    for level, coef, shape, off in lay:
        n0 = shape[0]
        if level[0] == pb.nl:
            v = rng.uniform(-1, 1, n0)
            fl2[o:o + n0] = v
            want += coef * v
        o += 3 * n0
    assert np.abs(O.fields_combine(pb, fl2)[0] - want).max() < 1e-15


@pytest.mark.parametrize("nl", [1, 2])
def test_sparse_grids_conserve_mass_per_grid(nl):
    """The conservative flux differences keep each grid's sum of f over a periodic domain."""
    pb = I.paper_example6(nr=8, nl=nl, T=2.0)
    st = O.restrict(pb)
    fl = O.fields_init(pb)
    st0 = st.copy()
    O.evolve(pb, st, fields=fl)
    for level, coef, shape, off in O.grid_layout(pb):
        size = int(np.prod(shape))
        a, b = st0[off:off + size].sum(), st[off:off + size].sum()
        assert abs(a - b) < 1e-12 * abs(a)


def test_evolve_refuses_the_system_without_fields():
    pb = I.paper_example6(nr=8, nl=1, T=0.1)
    with pytest.raises(ValueError):
        O.evolve(pb, O.restrict(pb))
