"""FP64 CPU oracle of the sparse-grid WENO5 method (ctypes wrapper over liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the GPU library.  The C source
(``oracle.c``) follows the paper step by step; see its header for the readings
of the points the paper leaves open.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None


class _Problem(C.Structure):
    _fields_ = [("d", C.c_int32), ("flux", C.c_int32), ("ic", C.c_int32), ("pad_", C.c_int32),
                ("lo", C.c_double * 4), ("hi", C.c_double * 4), ("fp", C.c_double * 4),
                ("ip", C.c_double * 8), ("bc", C.c_int32 * 4), ("relax_tau", C.c_double),
                ("relax_theta", C.c_double)]


class _Config(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nl", C.c_int32), ("dt_mode", C.c_int32), ("prolong", C.c_int32),
                ("linear", C.c_int32), ("nthreads", C.c_int32), ("cfl", C.c_double),
                ("eps_flux", C.c_double), ("eps_interp", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("t", C.c_double), ("last_dt", C.c_double),
                ("min_dt", C.c_double), ("max_dt", C.c_double)]


_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_num_grids.argtypes = [C.c_int, C.c_int]
        L.orc_num_grids.restype = C.c_int
        L.orc_grid_set.argtypes = [C.c_int, C.c_int, _ip, _ip]
        L.orc_grid_set.restype = C.c_int
        L.orc_smoothness.argtypes = [C.c_double] * 5 + [_dp]
        L.orc_weno5.argtypes = [C.c_double] * 6 + [C.c_int]
        L.orc_weno5.restype = C.c_double
        L.orc_interp.argtypes = [_dp, C.c_double, C.c_double, C.c_int]
        L.orc_interp.restype = C.c_double
        L.orc_total_nodes.argtypes = [C.POINTER(_Problem), C.POINTER(_Config)]
        L.orc_total_nodes.restype = C.c_int64
        L.orc_restrict.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), _dp]
        L.orc_rhs.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), _ip, _dp, _dp]
        L.orc_evolve.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), C.c_double, _dp, C.c_void_p,
                                 C.POINTER(_Stats)]
        L.orc_evolve.restype = C.c_int
        L.orc_prolong.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), _ip, _dp, _dp]
        L.orc_prolong_combine.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), _dp, _dp]
        L.orc_prolong_combine_points.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), _dp, C.c_int64,
                                                 _ip, _dp]
        L.orc_exact.argtypes = [C.POINTER(_Problem), _dp, C.c_double]
        L.orc_exact.restype = C.c_double
        L.orc_exact_fine.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), C.c_double, _dp]
        L.orc_norms.argtypes = [_dp, _dp, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_max_threads.restype = C.c_int
        L.orc_entropies.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), _dp, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]
        L.orc_evolve_fields.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), C.c_double, _dp, C.c_void_p,
                                        C.c_void_p, C.POINTER(_Stats)]
        L.orc_evolve_fields.restype = C.c_int
        L.orc_total_fields.argtypes = [C.POINTER(_Problem), C.POINTER(_Config)]
        L.orc_total_fields.restype = C.c_int64
        L.orc_fields_init.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), _dp]
        L.orc_fields_combine.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), _dp, _dp]
        L.orc_rhs_vm.argtypes = [C.POINTER(_Problem), C.POINTER(_Config), _ip, _dp, _dp, _dp, _dp]
        _lib = L
    return _lib


def _pad(v, n, fill=0.0):
    v = list(v)[:n]
    return v + [fill] * (n - len(v))


def _structs(pb, nthreads: int = 0):
    p = _Problem()
    p.d = pb.d
    p.flux = pb.flux
    p.ic = pb.ic
    p.lo[:] = _pad(pb.lo, 4)
    p.hi[:] = _pad(pb.hi, 4)
    p.fp[:] = _pad(pb.flux_params, 4)
    p.ip[:] = _pad(pb.ic_params, 8)
    p.bc[:] = [int(b) for b in _pad(getattr(pb, "bc", ()) or (), 4, 0)]
    p.relax_tau = float(getattr(pb, "relax_tau", 0.0))
    p.relax_theta = float(getattr(pb, "relax_theta", 1.0))
    c = _Config()
    c.nr = pb.nr
    c.nl = pb.nl
    c.dt_mode = pb.dt_mode
    c.prolong = pb.prolong
    c.linear = 1 if pb.linear else 0
    c.nthreads = nthreads
    c.cfl = pb.cfl
    c.eps_flux = pb.eps_flux
    c.eps_interp = pb.eps_interp
    return p, c


# --------------------------------------------------------------------------- primitives

def num_grids(d: int, nl: int) -> int:
    return lib().orc_num_grids(d, nl)


def grid_set(d: int, nl: int) -> Tuple[np.ndarray, np.ndarray]:
    """(levels[G, d], coefs[G]) in the order the combination accumulates them."""
    G = num_grids(d, nl)
    lv = np.zeros((max(G, 1), 4), dtype=np.int32)
    cf = np.zeros(max(G, 1), dtype=np.int32)
    lib().orc_grid_set(d, nl, lv, cf)
    return lv[:G, :d].copy(), cf[:G].copy()


def smoothness(a, b, c, d, e) -> np.ndarray:
    out = np.zeros(3)
    lib().orc_smoothness(a, b, c, d, e, out)
    return out


def weno5(a, b, c, d, e, eps: float = 1e-6, linear: bool = False) -> float:
    return lib().orc_weno5(a, b, c, d, e, eps, 1 if linear else 0)


def interp(u5, s: float, eps: float = 1e-6, lagrange: bool = False) -> float:
    return lib().orc_interp(np.ascontiguousarray(u5, dtype=np.float64), s, eps, 1 if lagrange else 0)


def grid_shape(pb, level) -> Tuple[int, ...]:
    return tuple(pb.nr << int(l) for l in level)


def grid_layout(pb):
    """[(level, coef, shape, offset)] for every component grid of the problem."""
    lv, cf = grid_set(pb.d, pb.nl)
    out, off = [], 0
    for l, c in zip(lv, cf):
        shp = grid_shape(pb, l)
        out.append((tuple(int(x) for x in l), int(c), shp, off))
        off += int(np.prod(shp))
    return out


def total_nodes(pb) -> int:
    p, c = _structs(pb)
    return lib().orc_total_nodes(C.byref(p), C.byref(c))


def restrict(pb) -> np.ndarray:
    """Alg. Step 1: the initial condition on every component grid, back to back."""
    p, c = _structs(pb)
    st = np.zeros(total_nodes(pb))
    lib().orc_restrict(C.byref(p), C.byref(c), st)
    return st


def rhs(pb, level, u: np.ndarray) -> np.ndarray:
    """Spatial operator L(u) of one component grid (u flat, direction 1 fastest)."""
    p, c = _structs(pb)
    lv = np.array(_pad([int(x) for x in level], 4, 0), dtype=np.int32)
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    L = np.zeros_like(u)
    lib().orc_rhs(C.byref(p), C.byref(c), lv, u, L)
    return L


def evolve(pb, state: np.ndarray, T: Optional[float] = None, mask=None, nthreads: int = 0,
           fields: Optional[np.ndarray] = None):
    """Alg. Step 2 in place on ``state`` (and, for the Vlasov-Maxwell system, on ``fields``, the
    grids' B_3, E_1, E_2 back to back); returns a stats dict."""
    p, c = _structs(pb, nthreads)
    st = _Stats()
    mptr = None
    if mask is not None:
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        mptr = m.ctypes.data_as(C.c_void_p)
    fptr = None
    if fields is not None:
        assert fields.dtype == np.float64 and fields.flags.c_contiguous and fields.size == total_fields(pb)
        fptr = fields.ctypes.data_as(C.c_void_p)
    rc = lib().orc_evolve_fields(C.byref(p), C.byref(c), pb.T if T is None else T, state, fptr, mptr,
                                 C.byref(st))
    if rc == -5:
        raise ValueError("oracle: the Vlasov-Maxwell system needs dim 3 and its fields")
    if rc != 0:
        raise FloatingPointError("oracle: non-finite wave speed")
    return {"steps": st.steps, "t": st.t, "last_dt": st.last_dt, "min_dt": st.min_dt, "max_dt": st.max_dt}


def total_fields(pb) -> int:
    """Field values over all component grids: 3 n_1 per grid (Vlasov-Maxwell), else 0."""
    p, c = _structs(pb)
    return int(lib().orc_total_fields(C.byref(p), C.byref(c)))


def fields_init(pb) -> np.ndarray:
    """Initial fields of every grid (B_3 = b sin(k0 x_2), E = 0), grids back to back."""
    p, c = _structs(pb)
    out = np.zeros(total_fields(pb))
    lib().orc_fields_init(C.byref(p), C.byref(c), out)
    return out


def fields_combine(pb, fields: np.ndarray) -> np.ndarray:
    """(3, N) array: B_3, E_1, E_2 combined on the finest x_2 grid."""
    p, c = _structs(pb)
    out = np.zeros(3 * pb.n_fine)
    lib().orc_fields_combine(C.byref(p), C.byref(c), np.ascontiguousarray(fields, dtype=np.float64), out)
    return out.reshape(3, pb.n_fine)


def rhs_vm(pb, level, u: np.ndarray, fld: np.ndarray):
    """Spatial operators of f and of the fields of one Vlasov-Maxwell component grid."""
    p, c = _structs(pb)
    lv = np.array(_pad([int(x) for x in level], 4, 0), dtype=np.int32)
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    fld = np.ascontiguousarray(fld, dtype=np.float64).ravel()
    L = np.zeros_like(u)
    Lf = np.zeros_like(fld)
    lib().orc_rhs_vm(C.byref(p), C.byref(c), lv, u, fld, L, Lf)
    return L, Lf


def solve_vm(pb, nthreads: int = 0):
    """Vlasov-Maxwell: restrict, initial fields, march, combine.  Returns (U_hat, state, fields,
    combined fields (3, N), stats)."""
    st = restrict(pb)
    fl = fields_init(pb)
    stats = evolve(pb, st, nthreads=nthreads, fields=fl)
    return prolong_combine(pb, st), st, fl, fields_combine(pb, fl), stats


def prolong(pb, level, u: np.ndarray) -> np.ndarray:
    p, c = _structs(pb)
    lv = np.array(_pad([int(x) for x in level], 4, 0), dtype=np.int32)
    out = np.zeros(pb.n_fine ** pb.d)
    lib().orc_prolong(C.byref(p), C.byref(c), lv, np.ascontiguousarray(u, dtype=np.float64).ravel(), out)
    return out


def prolong_combine(pb, state: np.ndarray) -> np.ndarray:
    """Alg. Step 3: the combined solution on the finest grid (flat, direction 1 fastest)."""
    p, c = _structs(pb)
    out = np.zeros(pb.n_fine ** pb.d)
    lib().orc_prolong_combine(C.byref(p), C.byref(c), state, out)
    return out


def prolong_combine_points(pb, state: np.ndarray, J: np.ndarray) -> np.ndarray:
    """The combined solution at fine nodes J[npts, d] only."""
    p, c = _structs(pb)
    J = np.asarray(J, dtype=np.int32).reshape(-1, pb.d)
    J4 = np.zeros((J.shape[0], 4), dtype=np.int32)
    J4[:, :pb.d] = J
    out = np.zeros(J.shape[0])
    lib().orc_prolong_combine_points(C.byref(p), C.byref(c), state, J.shape[0], J4, out)
    return out


def exact(pb, x, t: float) -> float:
    p, _ = _structs(pb)
    return lib().orc_exact(C.byref(p), np.array(_pad(list(x), 4), dtype=np.float64), t)


def exact_fine(pb, t: Optional[float] = None) -> np.ndarray:
    p, c = _structs(pb)
    out = np.zeros(pb.n_fine ** pb.d)
    lib().orc_exact_fine(C.byref(p), C.byref(c), pb.T if t is None else t, out)
    return out


def norms(a: np.ndarray, b: np.ndarray) -> Tuple[float, float]:
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    l1, li = C.c_double(), C.c_double()
    lib().orc_norms(a, b, a.size, C.byref(l1), C.byref(li))
    return l1.value, li.value


def entropies(pb, fine: np.ndarray) -> Tuple[float, float]:
    """(H_2, H_log) of a finest-grid solution relative to the stationary state (Sec. 3.4, Example 5)."""
    p, c = _structs(pb)
    fine = np.ascontiguousarray(fine, dtype=np.float64).ravel()
    assert fine.size == pb.n_fine ** pb.d
    h2, hl = C.c_double(), C.c_double()
    lib().orc_entropies(C.byref(p), C.byref(c), fine, C.byref(h2), C.byref(hl))
    return h2.value, hl.value


def max_threads() -> int:
    return lib().orc_max_threads()


def solve(pb, nthreads: int = 0):
    """Full method: restrict, evolve to T, prolongate + combine.  Returns (U_hat, state, stats)."""
    st = restrict(pb)
    stats = evolve(pb, st, nthreads=nthreads)
    U = prolong_combine(pb, st)
    return U, st, stats


def solve_errors(pb, nthreads: int = 0):
    """(L1, Linf, stats) of the combined solution against the exact solution at T."""
    U, _, stats = solve(pb, nthreads=nthreads)
    ex = exact_fine(pb, stats["t"])
    l1, li = norms(U, ex)
    return l1, li, stats
