"""ctypes binding of libsgweno (include/sgweno.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; PyTorch only
provides device memory and the HIP stream.  Loading fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgweno.so")

SGW_OK = 0
ERRORS = {-1: "invalid argument", -2: "unsupported", -3: "out of memory", -4: "non-finite",
          -5: "HIP error", -6: "call out of order"}

FLUX_ADVECTION, FLUX_BURGERS, FLUX_VLASOV_FIXED_E, FLUX_VLASOV_HARMONIC, FLUX_VLASOV_MAXWELL = 0, 1, 2, 3, 4
IC_SINE, IC_MAXWELL_COS, IC_VLASOV_BOLTZMANN, IC_VLASOV_MAXWELL = 0, 1, 2, 3
DT_CFL, DT_POW53 = 0, 1
PROLONG_WENO5, PROLONG_LAGRANGE5 = 0, 1
FP64, FP32_SWEEP = 0, 1
BC_PERIODIC, BC_ZERO = 0, 1
RUN_PLAIN, RUN_FUSED, RUN_GRAPH = 0, 1, 2


class SgwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sgweno: {ERRORS.get(status, status)}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("flux", C.c_int32), ("ic", C.c_int32), ("reserved0", C.c_int32),
                ("bc", C.c_int32 * 4), ("lo", C.c_double * 4), ("hi", C.c_double * 4), ("flux_params", C.c_double * 4),
                ("ic_params", C.c_double * 8), ("relax_tau", C.c_double), ("relax_theta", C.c_double)]


class Config(C.Structure):
    _fields_ = [("root_cells", C.c_int32), ("finest_level", C.c_int32), ("dt_mode", C.c_int32),
                ("prolong", C.c_int32), ("linear_weights", C.c_int32), ("precision", C.c_int32),
                ("cfl", C.c_double), ("eps_flux", C.c_double), ("eps_interp", C.c_double),
                ("box", C.c_int32 * 4), ("fine_tile", C.c_int32 * 4), ("box_target", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("sweep_form", C.c_int32)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "sgw_plan_create": (C.c_int32, [C.POINTER(Problem), C.POINTER(Config), C.POINTER(C.c_void_p)]),
    "sgw_plan_free": (None, [C.c_void_p]),
    "sgw_plan_footprint": (C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                       C.POINTER(C.c_uint64)]),
    "sgw_plan_info": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sgw_plan_grid": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32 * 4, C.c_int32 * 4, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int64)]),
    "sgw_plan_fine_tile": (C.c_int32, [C.c_void_p, C.c_int32 * 4]),
    "sgw_plan_fine_tile_count": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64)]),
    "sgw_plan_grid_box": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32 * 4]),
    "sgw_solver_create": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "sgw_solver_free": (None, [C.c_void_p]),
    "sgw_solver_set_stream": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "sgw_restrict_initial": (C.c_int32, [C.c_void_p]),
    "sgw_advance": (C.c_int32, [C.c_void_p, C.c_double, C.c_int32]),
    "sgw_prolongate_combine": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "sgw_prolongate_combine_tiles": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64]),
    "sgw_exact": (C.c_int32, [C.c_void_p, C.c_double, C.c_void_p]),
    "sgw_norms": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "sgw_entropies": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "sgw_fields_combine": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "sgw_plan_fields": (C.c_int32, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_int64)]),
    "sgw_query": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "sgw_set_grid": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "sgw_snapshot_bytes": (C.c_uint64, [C.c_void_p]),
    "sgw_snapshot": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "sgw_restore": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "sgw_norms_async": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sgw_prolongate_combine_many": (C.c_int32, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32,
                                                C.c_void_p, C.c_uint64, C.c_void_p]),
    "sgw_prolongate_many_scratch_bytes": (C.c_uint64, [C.POINTER(C.c_void_p), C.c_int32]),
    "sgw_restrict_initial_many": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_uint64,
                                              C.c_void_p]),
    "sgw_restrict_many_scratch_bytes": (C.c_uint64, [C.POINTER(C.c_void_p), C.c_int32]),
    "sgw_norms_many": (C.c_int32, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32,
                                   C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p]),
    "sgw_norms_many_scratch_bytes": (C.c_uint64, [C.POINTER(C.c_void_p), C.c_int32]),
    "sgw_norms_many_static": (C.c_int32, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                          C.c_int32, C.c_void_p, C.c_void_p]),
    "sgw_norms_many_static_max_bytes": (C.c_uint64, []),
    "sgw_batch_create": (C.c_int32, [C.c_int32, C.c_int32, C.c_uint64, C.c_void_p, C.c_void_p, C.c_uint64,
                                     C.POINTER(C.c_void_p)]),
    "sgw_batch_free": (None, [C.c_void_p]),
    "sgw_batch_scratch_bytes": (C.c_uint64, [C.c_int32, C.c_int64]),
    "sgw_batch_admit": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.POINTER(C.c_int32)]),
    "sgw_batch_admit_many": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_double),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "sgw_batch_release_many": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32]),
    "sgw_batch_step": (C.c_int32, [C.c_void_p, C.c_int32]),
    "sgw_batch_poll": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "sgw_batch_poll_begin": (C.c_int32, [C.c_void_p]),
    "sgw_batch_poll_end": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "sgw_batch_release": (C.c_int32, [C.c_void_p, C.c_int32]),
    "sgw_batch_launch_stage": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32]),
    "sgw_solver_launch_stage": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]),
    "sgw_calibrate_valu": (C.c_int32, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "sgw_batch_set_blocks_per_cu": (C.c_int32, [C.c_void_p, C.c_int32]),
    "sgw_batch_info": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sgw_status_string": (C.c_char_p, [C.c_int32]),
    "sgw_last_error": (C.c_char_p, []),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libsgweno.so (built in-tree); raises when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2007_10196_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != SGW_OK:
        raise SgwError(status, lib().sgw_last_error().decode(errors="replace"))


def _pad(v, n, fill=0.0):
    v = list(v)[:n]
    return v + [fill] * (n - len(v))


def make_structs(pb, box=None, fine_tile=None, box_target=0, blocks_per_cu=0, sweep_form=0):
    """Problem/Config structs from a problem description with the fields of
    sgw_inputs.Problem (d, lo, hi, flux, flux_params, ic, ic_params, nr, nl, cfl,
    dt_mode, prolong, linear, precision, eps_flux, eps_interp, bc, relax_tau, relax_theta)."""
    p = Problem()
    p.dim = pb.d
    p.flux = pb.flux
    p.ic = pb.ic
    p.reserved0 = 0
    p.bc[:] = _pad(getattr(pb, "bc", ()) or (), 4, BC_PERIODIC)
    p.lo[:] = _pad(pb.lo, 4)
    p.hi[:] = _pad(pb.hi, 4)
    p.flux_params[:] = _pad(pb.flux_params, 4)
    p.ic_params[:] = _pad(pb.ic_params, 8)
    p.relax_tau = float(getattr(pb, "relax_tau", 0.0))
    p.relax_theta = float(getattr(pb, "relax_theta", 1.0))
    c = Config()
    c.root_cells = pb.nr
    c.finest_level = pb.nl
    c.dt_mode = pb.dt_mode
    c.prolong = pb.prolong
    c.linear_weights = 1 if pb.linear else 0
    c.precision = pb.precision
    c.cfl = pb.cfl
    c.eps_flux = pb.eps_flux
    c.eps_interp = pb.eps_interp
    c.box[:] = _pad(box or [], 4, 0)
    c.fine_tile[:] = _pad(fine_tile or [], 4, 0)
    c.box_target = int(box_target or 0)
    c.blocks_per_cu = int(blocks_per_cu or 0)
    c.sweep_form = int(sweep_form or 0)
    return p, c
