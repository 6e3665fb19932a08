"""Python front end of libsgweno: one sparse-grid solve on one GPU.

Device memory comes from PyTorch (uint8 tensors sized by sgw_plan_footprint)
and work is enqueued on the current PyTorch (HIP) stream; the computation is
the library's.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Tuple

import torch

from . import binding as B


class Plan:
    """Host-only plan: the component grids of the index set, their layout and tiling."""

    def __init__(self, problem, box=None, fine_tile=None, box_target=0, blocks_per_cu=0, sweep_form=0):
        self.problem = problem
        self._pb, self._cfg = B.make_structs(problem, box, fine_tile, box_target, blocks_per_cu, sweep_form)
        h = C.c_void_p()
        B.check(B.lib().sgw_plan_create(C.byref(self._pb), C.byref(self._cfg), C.byref(h)))
        self.handle = h
        st, sc, fi = C.c_uint64(), C.c_uint64(), C.c_uint64()
        B.check(B.lib().sgw_plan_footprint(h, C.byref(st), C.byref(sc), C.byref(fi)))
        self.state_bytes, self.scratch_bytes, self.fine_bytes = st.value, sc.value, fi.value
        g, tn, fn = C.c_int32(), C.c_int64(), C.c_int64()
        B.check(B.lib().sgw_plan_info(h, C.byref(g), C.byref(tn), C.byref(fn)))
        self.num_grids, self.total_nodes, self.fine_nodes = g.value, tn.value, fn.value
        fo, fc = C.c_uint64(), C.c_int64()
        B.check(B.lib().sgw_plan_fields(h, C.byref(fo), C.byref(fc)))
        self.fields_offset, self.fields_count = fo.value, fc.value
        ft = (C.c_int32 * 4)()
        B.check(B.lib().sgw_plan_fine_tile(h, ft))
        self.fine_tile = tuple(ft[:problem.d])
        ntile = C.c_int64()
        B.check(B.lib().sgw_plan_fine_tile_count(h, C.byref(ntile)))
        self.fine_tile_count = ntile.value
        self.grids = []
        for i in range(self.num_grids):
            lv, sh = (C.c_int32 * 4)(), (C.c_int32 * 4)()
            cf, off = C.c_int32(), C.c_int64()
            B.check(B.lib().sgw_plan_grid(h, i, lv, sh, C.byref(cf), C.byref(off)))
            bx = (C.c_int32 * 4)()
            B.check(B.lib().sgw_plan_grid_box(h, i, bx))
            d = problem.d
            self.grids.append(dict(level=tuple(lv[:d]), shape=tuple(sh[:d]), coef=cf.value, offset=off.value,
                                   box=tuple(bx[:d])))

    @property
    def footprint(self) -> int:
        return self.state_bytes + self.scratch_bytes + self.fine_bytes

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                B.lib().sgw_plan_free(h)
            except Exception:
                pass
            self.handle = C.c_void_p()


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Solver:
    """Bound solve: caller-owned device buffers + a HIP stream."""

    def __init__(self, problem, device: str = "cuda", stream: Optional[torch.cuda.Stream] = None,
                 box=None, fine_tile=None, plan: Optional[Plan] = None, box_target: int = 0,
                 blocks_per_cu: int = 0, sweep_form: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("sgweno needs a ROCm GPU; none is visible")
        self.problem = problem
        self.plan = plan or Plan(problem, box, fine_tile, box_target, blocks_per_cu, sweep_form)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # torch's caching allocator returns 512-byte aligned blocks
        self.state = torch.empty(self.plan.state_bytes, dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(self.plan.scratch_bytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        B.check(B.lib().sgw_solver_create(self.plan.handle, C.c_void_p(self.state.data_ptr()),
                                          C.c_void_p(self.scratch.data_ptr()), _stream_handle(self.stream),
                                          C.byref(h)))
        self.handle = h
        self.real = torch.float64 if problem.precision == B.FP64 else torch.float32

    def set_stream(self, stream: torch.cuda.Stream):
        """Enqueue later calls on `stream` (earlier work is not waited for)."""
        B.check(B.lib().sgw_solver_set_stream(self.handle, C.c_void_p(stream.cuda_stream)))
        self.stream = stream
        return self

    # --- the algorithm
    def restrict(self):
        B.check(B.lib().sgw_restrict_initial(self.handle))
        return self

    def advance(self, t_final: Optional[float] = None, mode: int = B.RUN_GRAPH):
        B.check(B.lib().sgw_advance(self.handle, self.problem.T if t_final is None else t_final, mode))
        return self

    def prolongate_combine(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.plan.fine_nodes, dtype=torch.float64, device=self.device)
        assert out.dtype == torch.float64 and out.numel() >= self.plan.fine_nodes and out.is_contiguous()
        B.check(B.lib().sgw_prolongate_combine(self.handle, C.c_void_p(out.data_ptr())))
        return out

    def prolongate_combine_tiles(self, out: torch.Tensor, first_tile: int, num_tiles: int) -> torch.Tensor:
        """Step 3 at finest-grid tiles first_tile .. first_tile + num_tiles - 1 of ``out``."""
        assert out.dtype == torch.float64 and out.numel() >= self.plan.fine_nodes and out.is_contiguous()
        B.check(B.lib().sgw_prolongate_combine_tiles(self.handle, C.c_void_p(out.data_ptr()), int(first_tile),
                                                     int(num_tiles)))
        return out

    def exact(self, t: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.plan.fine_nodes, dtype=torch.float64, device=self.device)
        B.check(B.lib().sgw_exact(self.handle, float(t), C.c_void_p(out.data_ptr())))
        return out

    def norms(self, a: torch.Tensor, b: torch.Tensor) -> Tuple[float, float]:
        assert a.dtype == torch.float64 and b.dtype == torch.float64
        assert a.numel() >= self.plan.fine_nodes and b.numel() >= self.plan.fine_nodes
        res = (C.c_double * 2)()
        B.check(B.lib().sgw_norms(self.handle, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), res))
        return res[0], res[1]

    def launch_stage(self, stage: int, part: int = 0, reps: int = 1):
        """Measurement hook: reps repetitions of one part of RK stage `stage` on the solver stream
        (part 0 the whole stage, 1 the 4D plane launch, 2 + k the line sweep of direction k + 1);
        leaves the solve's state meaningless."""
        B.check(B.lib().sgw_solver_launch_stage(self.handle, stage, part, reps))

    def fields(self, which: int = 0) -> torch.Tensor:
        """Vlasov-Maxwell: the FP64 fields of every grid (B_3, E_1, E_2 at its x_2 nodes, grids back
        to back) in state copy `which` (0: u^n), a view into the state buffer."""
        assert self.plan.fields_count > 0
        copy = self.plan.state_bytes // 3
        start = which * copy + self.plan.fields_offset
        return self.state[start:start + 8 * self.plan.fields_count].view(torch.float64)

    def fields_combine(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Vlasov-Maxwell: (3, N) FP64 combination of the fields of u^n on the finest x_2 grid."""
        n = self.problem.nr << self.problem.nl
        if out is None:
            out = torch.empty(3 * n, dtype=torch.float64, device=self.device)
        assert out.dtype == torch.float64 and out.numel() >= 3 * n
        B.check(B.lib().sgw_fields_combine(self.handle, C.c_void_p(out.data_ptr())))
        return out[:3 * n].view(3, n)

    def entropies(self, f: torch.Tensor) -> Tuple[float, float]:
        """(H_2, H_log) of a finest-grid solution (FP64) relative to the stationary state of the
        Vlasov-Boltzmann model."""
        assert f.dtype == torch.float64 and f.is_cuda and f.numel() >= self.plan.fine_nodes
        res = (C.c_double * 2)()
        B.check(B.lib().sgw_entropies(self.handle, C.c_void_p(f.data_ptr()), res))
        return res[0], res[1]

    def norms_async(self, a: torch.Tensor, b: torch.Tensor, result: torch.Tensor):
        """L1, Linf into result[0:2] (device FP64) without synchronising."""
        assert result.dtype == torch.float64 and result.numel() >= 2 and result.is_cuda
        B.check(B.lib().sgw_norms_async(self.handle, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                        C.c_void_p(result.data_ptr())))

    def set_grid(self, g: int, values: torch.Tensor):
        """Initial values of grid g sampled by the caller (solver precision, plan shape)."""
        info = self.plan.grids[g]
        n = 1
        for x in info["shape"]:
            n *= x
        assert values.dtype == self.real and values.is_cuda and values.is_contiguous() and values.numel() == n
        B.check(B.lib().sgw_set_grid(self.handle, int(g), C.c_void_p(values.data_ptr())))
        return self

    def snapshot(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Checkpoint (device bytes) of u^n, wave speeds and time record."""
        nbytes = int(B.lib().sgw_snapshot_bytes(self.handle))
        if out is None:
            out = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        assert out.dtype == torch.uint8 and out.numel() >= nbytes and out.is_contiguous()
        B.check(B.lib().sgw_snapshot(self.handle, C.c_void_p(out.data_ptr())))
        return out

    def restore(self, snap: torch.Tensor):
        """Resume from a snapshot of a solver with the same plan."""
        assert snap.dtype == torch.uint8 and snap.numel() >= int(B.lib().sgw_snapshot_bytes(self.handle))
        B.check(B.lib().sgw_restore(self.handle, C.c_void_p(snap.data_ptr())))
        return self

    def query(self) -> Tuple[float, int]:
        t, n = C.c_double(), C.c_int64()
        B.check(B.lib().sgw_query(self.handle, C.byref(t), C.byref(n)))
        return t.value, n.value

    # --- views of the caller-owned state
    def state_copy(self, which: int = 0) -> torch.Tensor:
        """Copy ``which`` (0 = u^n) of every component grid, back to back in plan order."""
        esz = 8 if self.real == torch.float64 else 4
        copy_bytes = self.plan.state_bytes // 3
        raw = self.state[which * copy_bytes: which * copy_bytes + self.plan.total_nodes * esz]
        return raw.view(self.real)

    def grid(self, g: int) -> torch.Tensor:
        info = self.plan.grids[g]
        n = 1
        for s in info["shape"]:
            n *= s
        return self.state_copy()[info["offset"]: info["offset"] + n]

    def solve(self, mode: int = B.RUN_GRAPH, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self.restrict()
        self.advance(mode=mode)
        return self.prolongate_combine(out)

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            B.lib().sgw_solver_free(h)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many solves advanced together (sgw_batch_*): one graph launch per step."""

    def __init__(self, max_solvers: int, precision: int, hbm_budget: int, max_items: int = 1 << 20,
                 device: str = "cuda", stream: Optional[torch.cuda.Stream] = None):
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = B.lib().sgw_batch_scratch_bytes(max_solvers, max_items)
        self.scratch = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        B.check(B.lib().sgw_batch_create(max_solvers, precision, int(hbm_budget), _stream_handle(self.stream),
                                         C.c_void_p(self.scratch.data_ptr()), int(nbytes), C.byref(h)))
        self.handle = h
        self.max_solvers = max_solvers
        self.slots = {}

    def admit(self, solver: Solver, t_final: Optional[float] = None) -> int:
        slot = C.c_int32()
        B.check(B.lib().sgw_batch_admit(self.handle, solver.handle,
                                        solver.problem.T if t_final is None else t_final, C.byref(slot)))
        self.slots[slot.value] = solver
        return slot.value

    def try_admit(self, solver: Solver, t_final: Optional[float] = None) -> Optional[int]:
        try:
            return self.admit(solver, t_final)
        except B.SgwError as e:
            if e.status == -3:
                return None
            raise

    def admit_many(self, solvers, t_final=None):
        """Admit solvers (a list or a PtrList) in order; raises at the first refused one (those
        before it stay admitted)."""
        n = len(solvers)
        hs = _ptrs(solvers, "solver")
        if t_final is None and isinstance(solvers, PtrList):
            tf = solvers.t_final()
        else:
            tf = (C.c_double * n)(*[s.problem.T if t_final is None else float(t_final[i])
                                    for i, s in enumerate(solvers)])
        slots = (C.c_int32 * n)()
        got = C.c_int32()
        st = B.lib().sgw_batch_admit_many(self.handle, hs, n, tf, slots, C.byref(got))
        for i in range(got.value):
            self.slots[slots[i]] = solvers[i]
        B.check(st)
        return list(slots[:n])

    def release_many(self, slots):
        """Release the given slots; returns their solvers."""
        n = len(slots)
        arr = (C.c_int32 * n)(*slots)
        B.check(B.lib().sgw_batch_release_many(self.handle, arr, n))
        return [self.slots.pop(s) for s in slots]

    def step(self, nsteps: int = 1):
        B.check(B.lib().sgw_batch_step(self.handle, nsteps))

    def poll(self):
        buf = (C.c_int32 * self.max_solvers)()
        n = C.c_int32()
        B.check(B.lib().sgw_batch_poll(self.handle, buf, C.byref(n)))
        return list(buf[:n.value])

    def poll_begin(self):
        """Enqueue the gathering of the completion flags; poll_end() reads them."""
        B.check(B.lib().sgw_batch_poll_begin(self.handle))

    def poll_end(self):
        buf = (C.c_int32 * self.max_solvers)()
        n = C.c_int32()
        B.check(B.lib().sgw_batch_poll_end(self.handle, buf, C.byref(n)))
        return list(buf[:n.value])

    def set_blocks_per_cu(self, n: int):
        B.check(B.lib().sgw_batch_set_blocks_per_cu(self.handle, int(n)))

    def launch_stage(self, stage: int, reps: int = 1):
        B.check(B.lib().sgw_batch_launch_stage(self.handle, stage, reps))

    def info(self):
        a, b, n = C.c_int32(), C.c_int64(), C.c_int64()
        B.check(B.lib().sgw_batch_info(self.handle, C.byref(a), C.byref(b), C.byref(n)))
        return dict(active=a.value, boxes=b.value, nodes=n.value)

    def release(self, slot: int) -> Solver:
        B.check(B.lib().sgw_batch_release(self.handle, slot))
        return self.slots.pop(slot)

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            B.lib().sgw_batch_free(h)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PtrList:
    """A list of solvers or of device tensors, marshalled once into the C pointer array that the
    many-solve calls take.  With hundreds of solves, building that array from Python costs
    0.1-0.3 ms of host time per call, which a caller that repeats the same call on the same
    solvers and buffers (a benchmark or serving loop) pays only once this way.  The list keeps
    its items alive; it must not be changed after construction."""

    def __init__(self, items):
        self.items = tuple(items)
        if self.items and isinstance(self.items[0], Solver):
            vals = [x.handle.value for x in self.items]
            self.min_numel = None
            self.all_fp64 = None
        else:
            vals = [x.data_ptr() for x in self.items]
            self.min_numel = min((x.numel() for x in self.items), default=0)
            self.all_fp64 = all(x.dtype == torch.float64 and x.is_cuda for x in self.items)
        self.arr = (C.c_void_p * len(vals))(*vals)
        self._t_final = None
        self._max_fine = None

    def __len__(self):
        return len(self.items)

    def __iter__(self):
        return iter(self.items)

    def __getitem__(self, i):
        return self.items[i]

    def max_fine_nodes(self):
        """The largest finest-grid size over a list of solvers."""
        if self._max_fine is None:
            self._max_fine = max((s.plan.fine_nodes for s in self.items), default=0)
        return self._max_fine

    def t_final(self):
        """The final times of a list of solvers, as the C array admit_many takes."""
        if self._t_final is None:
            self._t_final = (C.c_double * len(self.items))(*[s.problem.T for s in self.items])
        return self._t_final


def _ptrs(items, kind):
    if isinstance(items, PtrList):
        return items.arr
    if kind == "solver":
        return (C.c_void_p * len(items))(*[s.handle.value for s in items])
    return (C.c_void_p * len(items))(*[x.data_ptr() for x in items])


def _call_scratch(nbytes: int, device, stream: Optional[torch.cuda.Stream]) -> torch.Tensor:
    """Device scratch for one many-solve call.  The call returns before its kernels
    run, so the allocator is told the scratch is in use on the call's stream."""
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if stream is not None and stream != torch.cuda.current_stream(t.device):
        t.record_stream(stream)
    return t


def prolongate_combine_many(solvers, outs, stream: Optional[torch.cuda.Stream] = None):
    """Combined solutions of many solves (same dimension and precision) in one launch.
    `solvers` and `outs` are lists or PtrLists."""
    n = len(solvers)
    assert len(outs) == n
    hs = _ptrs(solvers, "solver")
    os_ = _ptrs(outs, "tensor")
    nbytes = int(B.lib().sgw_prolongate_many_scratch_bytes(hs, n))
    scratch = _call_scratch(nbytes, outs[0].device, stream)
    B.check(B.lib().sgw_prolongate_combine_many(hs, os_, n, C.c_void_p(scratch.data_ptr()), nbytes,
                                                _stream_handle(stream)))
    return outs


def restrict_many(solvers, stream: Optional[torch.cuda.Stream] = None):
    """Initial values of many solves (one precision) in one launch (a list or a PtrList)."""
    n = len(solvers)
    hs = _ptrs(solvers, "solver")
    nbytes = int(B.lib().sgw_restrict_many_scratch_bytes(hs, n))
    scratch = _call_scratch(nbytes, solvers[0].device, stream)
    B.check(B.lib().sgw_restrict_initial_many(hs, n, C.c_void_p(scratch.data_ptr()), nbytes, _stream_handle(stream)))
    return solvers


def norms_many(solvers, a, b, result: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
    """L1, Linf of (a[i] - b[i]) over solve i's finest grid into result[i, 0:2] (device FP64).
    `solvers`, `a` and `b` are lists or PtrLists."""
    n = len(solvers)
    assert len(a) == n and len(b) == n
    assert result.dtype == torch.float64 and result.is_cuda and result.is_contiguous() and result.numel() >= 2 * n
    for v in (a, b):
        if isinstance(v, PtrList):
            need = (solvers.max_fine_nodes() if isinstance(solvers, PtrList)
                    else max((s.plan.fine_nodes for s in solvers), default=0))
            assert v.all_fp64 and v.min_numel >= need
        else:
            for x, s in zip(v, solvers):
                assert x.dtype == torch.float64 and x.numel() >= s.plan.fine_nodes
    hs = _ptrs(solvers, "solver")
    pa = _ptrs(a, "tensor")
    pb = _ptrs(b, "tensor")
    nbytes = int(B.lib().sgw_norms_many_scratch_bytes(hs, n))
    scratch = _call_scratch(nbytes, result.device, stream)
    B.check(B.lib().sgw_norms_many(hs, pa, pb, n, C.c_void_p(result.data_ptr()), C.c_void_p(scratch.data_ptr()),
                                   nbytes, _stream_handle(stream)))
    return result


def norms_many_static(solvers, a, b, result: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
    """norms_many for at most 32 pairs without any allocation: the library keeps the pair list
    and partial sums in its own device array.  Runs on `stream` (default: the current stream)
    only, so the caller orders the writes of a and b before it."""
    n = len(solvers)
    assert len(a) == n and len(b) == n
    assert result.dtype == torch.float64 and result.is_cuda and result.is_contiguous() and result.numel() >= 2 * n
    for x, y, s in zip(a, b, solvers):
        assert x.dtype == torch.float64 and x.numel() >= s.plan.fine_nodes
        assert y.dtype == torch.float64 and y.numel() >= s.plan.fine_nodes
    B.check(B.lib().sgw_norms_many_static(_ptrs(solvers, "solver"), _ptrs(a, "tensor"), _ptrs(b, "tensor"), n,
                                          C.c_void_p(result.data_ptr()), _stream_handle(stream)))
    return result
