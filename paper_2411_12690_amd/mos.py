"""ctypes binding of the C ABI in include/mos.h (argument marshalling only).

Every stage runs in the HIP library ``libmos.so``; this module converts
Python descriptors to the C structs, passes device pointers of torch tensors,
routes device allocations through torch's caching allocator and turns status
codes into exceptions.  Importing it fails loudly when the library is absent.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmos.so")

MOS_OK, MOS_EINVAL, MOS_ENOMEM, MOS_ENOCONV, MOS_ESINGULAR, MOS_EHIP, MOS_EBUSY = 0, -1, -2, -3, -4, -5, -6
MOS_FP64, MOS_MIXED = 0, 1
MOS_CELL_TSV, MOS_CELL_BUMP = 0, 1
MOS_BC_CLAMP_BOTTOM, MOS_BC_CLAMP_TOP, MOS_BC_LIST_ON_DEVICE = 1, 2, 4
MOS_OUT_VM, MOS_OUT_SIGMA6 = 1, 2
(MOS_Q_N, MOS_Q_CELL_DOFS, MOS_Q_CELL_ELEMS, MOS_Q_CELL_NNZ, MOS_Q_FREE_DOFS, MOS_Q_BANDWIDTH,
 MOS_Q_GLOBAL_DOFS, MOS_Q_ITERS, MOS_Q_REFINES, MOS_Q_DEVICE_BYTES) = range(1, 11)

EXPORTED = ("mos_ctx_create", "mos_ctx_destroy", "mos_build_cell", "mos_reduce", "mos_solve_array",
            "mos_reconstruct", "mos_reconstruct_noalloc", "mos_reconstruct_plane", "mos_reconstruct_displacement", "mos_get_solution", "mos_get_cond_estimate", "mos_query", "mos_cell_export", "mos_rom_export",
            "mos_array_layout", "mos_engine_create", "mos_engine_submit", "mos_engine_progress",
            "mos_engine_result", "mos_engine_cond_estimate", "mos_engine_option", "mos_engine_stats", "mos_engine_graph_stats", "mos_engine_destroy", "mos_timing_start", "mos_timing_stop",
            "mos_cell_free", "mos_rom_free", "mos_sol_free", "mos_last_error")
MOS_K_CELL_GEMM, MOS_K_PCG_SCALARS, MOS_K_PCG_UPDATE, MOS_K_RECON = 1, 2, 3, 4
MOS_OPT_CELL_GEMM = 1
GEMM_AUTO, GEMM_TILES, GEMM_ROWS, GEMM_ROWS_LDS = 0, 1, 2, 3
MOS_OPT_GEMM_SPLIT = 2
MOS_OPT_UPDATE_WIDTH = 3
MOS_OPT_PRECOND = 4
MOS_OPT_GRAPH = 5
MOS_OPT_COARSE_TABLE = 6


class MosError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Material(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("nu", ctypes.c_double), ("alpha", ctypes.c_double)]


class CellDesc(ctypes.Structure):
    _fields_ = [("pitch_x", ctypes.c_double), ("pitch_y", ctypes.c_double), ("height", ctypes.c_double),
                ("mesh", ctypes.c_int32 * 3), ("tsv_diameter", ctypes.c_double),
                ("liner_thickness", ctypes.c_double), ("matrix", Material), ("via", Material),
                ("liner", Material), ("interp", ctypes.c_int32 * 3), ("structure", ctypes.c_int32),
                ("pad_thickness", ctypes.c_double), ("skew", ctypes.c_double)]


class ArrayDesc(ctypes.Structure):
    _fields_ = [("nx_cells", ctypes.c_int32), ("ny_cells", ctypes.c_int32),
                ("cell_type", ctypes.POINTER(ctypes.c_uint8)), ("delta_T", ctypes.c_double),
                ("bc_flags", ctypes.c_uint32), ("n_prescribed", ctypes.c_int64),
                ("prescribed_dof", ctypes.POINTER(ctypes.c_int64)),
                ("prescribed_value", ctypes.POINTER(ctypes.c_double)), ("precision", ctypes.c_int),
                ("rtol", ctypes.c_double), ("max_iters", ctypes.c_int32), ("nz_cells", ctypes.c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, vp = ctypes.POINTER, ctypes.c_void_p
    sig = {
        "mos_ctx_create": (ctypes.c_int, [ctypes.c_int, vp, P(Allocator), P(vp)]),
        "mos_ctx_destroy": (None, [vp]),
        "mos_build_cell": (ctypes.c_int, [vp, P(CellDesc), P(vp)]),
        "mos_reduce": (ctypes.c_int, [vp, vp, P(vp)]),
        "mos_solve_array": (ctypes.c_int, [vp, P(ArrayDesc), P(vp), ctypes.c_int32, P(vp)]),
        "mos_reconstruct": (ctypes.c_int, [vp, vp, ctypes.c_uint32, vp, vp]),
        "mos_reconstruct_noalloc": (ctypes.c_int, [vp, vp, ctypes.c_uint32, vp, vp]),
        "mos_reconstruct_plane": (ctypes.c_int, [vp, vp, ctypes.c_int32, vp]),
        "mos_reconstruct_displacement": (ctypes.c_int, [vp, vp, vp]),
        "mos_get_solution": (ctypes.c_int, [vp, vp, P(ctypes.c_double), P(ctypes.c_int32)]),
        "mos_get_cond_estimate": (ctypes.c_int, [vp, P(ctypes.c_double), P(ctypes.c_int32)]),
        "mos_engine_cond_estimate": (ctypes.c_int, [vp, ctypes.c_int64, P(ctypes.c_double), P(ctypes.c_int32)]),
        "mos_query": (ctypes.c_int, [vp, ctypes.c_int, P(ctypes.c_int64)]),
        "mos_cell_export": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
        "mos_rom_export": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "mos_array_layout": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                            P(ctypes.c_int64), vp, vp, vp, vp]),
        "mos_engine_create": (ctypes.c_int, [vp, P(vp), ctypes.c_int32, ctypes.c_int, ctypes.c_size_t, P(vp)]),
        "mos_engine_submit": (ctypes.c_int, [vp, P(ArrayDesc), vp, vp, vp, P(ctypes.c_int64)]),
        "mos_engine_progress": (ctypes.c_int, [vp, ctypes.c_int32, vp, ctypes.c_int32, P(ctypes.c_int32)]),
        "mos_engine_result": (ctypes.c_int, [vp, ctypes.c_int64, P(ctypes.c_int32), P(ctypes.c_double),
                                             P(ctypes.c_int32), P(ctypes.c_int32)]),
        "mos_engine_option": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int64]),
        "mos_engine_stats": (ctypes.c_int, [vp, P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64),
                                            P(ctypes.c_int64)]),
        "mos_engine_graph_stats": (ctypes.c_int, [vp, P(ctypes.c_int64), P(ctypes.c_int64)]),
        "mos_engine_destroy": (None, [vp]),
        "mos_timing_start": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int]),
        "mos_timing_stop": (ctypes.c_int, [vp, P(ctypes.c_int64), P(ctypes.c_double), P(ctypes.c_int64)]),
        "mos_cell_free": (None, [vp]),
        "mos_rom_free": (None, [vp]),
        "mos_sol_free": (None, [vp]),
        "mos_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


def _check(status, what):
    if status != MOS_OK:
        msg = lib().mos_last_error().decode(errors="replace")
        raise MosError(status, f"{what}: {msg}")


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def cell_desc(spec):
    d = CellDesc()
    d.pitch_x, d.pitch_y, d.height = float(spec.pitch_x), float(spec.pitch_y), float(spec.height)
    d.mesh[:] = [int(v) for v in spec.mesh]
    d.tsv_diameter, d.liner_thickness = float(spec.tsv_diameter), float(spec.liner_thickness)
    d.matrix, d.via, d.liner = (Material(*map(float, m)) for m in (spec.matrix, spec.via, spec.liner))
    d.interp[:] = [int(v) for v in spec.interp]
    kind = getattr(spec, "structure", "tsv")
    d.structure = {"tsv": MOS_CELL_TSV, "bump": MOS_CELL_BUMP}[kind] if isinstance(kind, str) else int(kind)
    d.pad_thickness = float(getattr(spec, "pad_thickness", 0.0))
    d.skew = float(getattr(spec, "skew", 0.0))
    return d


class _Handle:
    _free = None

    def __init__(self, ptr, ctx):
        self.ptr = ptr
        self.ctx = ctx

    def query(self, what):
        v = ctypes.c_int64()
        _check(lib().mos_query(self.ptr, what, ctypes.byref(v)), "mos_query")
        return v.value

    def close(self):
        if self.ptr:
            getattr(lib(), self._free)(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cell(_Handle):
    _free = "mos_cell_free"


class Rom(_Handle):
    _free = "mos_rom_free"


class Solution(_Handle):
    _free = "mos_sol_free"
    precision = MOS_FP64


class Context:
    """A library context on one device and torch stream.  Device memory goes
    through torch's caching allocator unless ``torch_allocator`` is False."""

    def __init__(self, device=0, stream=None, torch_allocator=True):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._alloc = None
        alloc_p = None
        if torch_allocator:
            dev, st = device, self.stream

            def _a(size, user):
                try:
                    return torch.cuda.caching_allocator_alloc(size, dev, st)
                except Exception:
                    return None

            def _f(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            self._alloc = Allocator(ALLOC_FN(_a), FREE_FN(_f), None)
            alloc_p = ctypes.byref(self._alloc)
        h = ctypes.c_void_p()
        _check(lib().mos_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream), alloc_p, ctypes.byref(h)),
               "mos_ctx_create")
        self.ptr = h

    def close(self):
        if self.ptr:
            lib().mos_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mos_build_cell(ctx, spec):
    d = cell_desc(spec)
    h = ctypes.c_void_p()
    _check(lib().mos_build_cell(ctx.ptr, ctypes.byref(d), ctypes.byref(h)), "mos_build_cell")
    return Cell(h, ctx)


def mos_reduce(ctx, cell):
    h = ctypes.c_void_p()
    _check(lib().mos_reduce(ctx.ptr, cell.ptr, ctypes.byref(h)), "mos_reduce")
    return Rom(h, ctx)


def array_desc(nx_cells, ny_cells, cell_type, delta_T, clamp_bottom=True, clamp_top=False,
               prescribed_dofs=None, prescribed_values=None, mixed=False, rtol=0.0, max_iters=0, nz_cells=1):
    """Build the C descriptor; returns (desc, keep-alive arrays)."""
    ct = np.ascontiguousarray(cell_type, dtype=np.uint8)
    if ct.size != nx_cells * ny_cells * nz_cells:
        raise ValueError("cell_type must have nx_cells * ny_cells * nz_cells entries")
    d = ArrayDesc()
    d.nx_cells, d.ny_cells, d.nz_cells = int(nx_cells), int(ny_cells), int(nz_cells)
    d.cell_type = ct.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    d.delta_T = float(delta_T)
    d.bc_flags = (MOS_BC_CLAMP_BOTTOM if clamp_bottom else 0) | (MOS_BC_CLAMP_TOP if clamp_top else 0)
    keep = [ct]
    if prescribed_dofs is not None and getattr(prescribed_dofs, "is_cuda", False):
        # Device-resident list (torch tensors on the context's device).
        pd, pv = prescribed_dofs, prescribed_values
        if (str(pd.dtype) != "torch.int64" or str(pv.dtype) != "torch.float64" or not pv.is_cuda
                or pd.shape != pv.shape or not pd.is_contiguous() or not pv.is_contiguous()):
            raise ValueError("device prescribed lists must be contiguous int64 / float64 tensors of one shape")
        d.bc_flags |= MOS_BC_LIST_ON_DEVICE
        d.n_prescribed = pd.numel()
        d.prescribed_dof = ctypes.cast(ctypes.c_void_p(pd.data_ptr()), ctypes.POINTER(ctypes.c_int64))
        d.prescribed_value = ctypes.cast(ctypes.c_void_p(pv.data_ptr()), ctypes.POINTER(ctypes.c_double))
        keep += [pd, pv]
    elif prescribed_dofs is not None and len(prescribed_dofs):
        pd = np.ascontiguousarray(prescribed_dofs, dtype=np.int64)
        pv = np.ascontiguousarray(prescribed_values, dtype=np.float64)
        if pd.shape != pv.shape:
            raise ValueError("prescribed dofs and values differ in length")
        d.n_prescribed = pd.size
        d.prescribed_dof = pd.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        d.prescribed_value = pv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        keep += [pd, pv]
    d.precision = MOS_MIXED if mixed else MOS_FP64
    d.rtol, d.max_iters = float(rtol), int(max_iters)
    return d, keep


def _rom_array(roms):
    return (ctypes.c_void_p * len(roms))(*[r.ptr.value for r in roms])


def mos_solve_array(ctx, roms, nx_cells, ny_cells, cell_type, delta_T, clamp_bottom=True, clamp_top=False,
                    prescribed_dofs=None, prescribed_values=None, mixed=False, rtol=0.0, max_iters=0, nz_cells=1):
    d, keep = array_desc(nx_cells, ny_cells, cell_type, delta_T, clamp_bottom, clamp_top, prescribed_dofs,
                         prescribed_values, mixed, rtol, max_iters, nz_cells)
    h = ctypes.c_void_p()
    _check(lib().mos_solve_array(ctx.ptr, ctypes.byref(d), _rom_array(roms), len(roms), ctypes.byref(h)),
           "mos_solve_array")
    s = Solution(h, ctx)
    s.precision = d.precision
    s.n_cells = nx_cells * ny_cells * nz_cells
    s.n_elem = roms[0].query(MOS_Q_CELL_ELEMS)
    s.roms = list(roms)
    return s


class Engine:
    """Batched / served global stage (mos_engine_*): submit problems, call
    progress() until their tickets complete."""

    def __init__(self, ctx, roms, mixed=False, device_bytes=8 << 30, gemm=None, precond=None, graph=None):
        self.ctx = ctx
        self.roms = list(roms)
        self.mixed = mixed
        self.ptr = None
        self._keep = {}
        h = ctypes.c_void_p()
        _check(lib().mos_engine_create(ctx.ptr, _rom_array(roms), len(roms), MOS_MIXED if mixed else MOS_FP64,
                                       int(device_bytes), ctypes.byref(h)), "mos_engine_create")
        self.ptr = h
        if gemm is not None:
            self.option(MOS_OPT_CELL_GEMM, gemm)
        if precond is not None:
            self.option(MOS_OPT_PRECOND, precond)
        if graph is not None:
            self.option(MOS_OPT_GRAPH, int(graph))

    def submit(self, nx_cells, ny_cells, cell_type, delta_T, vm=None, sigma6=None, u=None, **kw):
        d, keep = array_desc(nx_cells, ny_cells, cell_type, delta_T, mixed=self.mixed, **kw)
        t = ctypes.c_int64()
        ptr = (lambda x: ctypes.c_void_p(x.data_ptr()) if x is not None else None)
        _check(lib().mos_engine_submit(self.ptr, ctypes.byref(d), ptr(vm), ptr(sigma6), ptr(u), ctypes.byref(t)),
               "mos_engine_submit")
        self._keep[t.value] = (keep, vm, sigma6, u)
        return t.value

    def progress(self, iterations=16, max_completed=4096):
        out = np.zeros(max_completed, dtype=np.int64)
        n = ctypes.c_int32()
        _check(lib().mos_engine_progress(self.ptr, iterations, _ptr(out), max_completed, ctypes.byref(n)),
               "mos_engine_progress")
        return [int(v) for v in out[:n.value]]

    def result(self, ticket):
        """(status, relative residual, iterations, sweeps); forgets the ticket."""
        st, res, it, sw = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().mos_engine_result(self.ptr, ticket, ctypes.byref(st), ctypes.byref(res), ctypes.byref(it),
                                       ctypes.byref(sw)), "mos_engine_result")
        self._keep.pop(ticket, None)
        self.last_error = lib().mos_last_error().decode(errors="replace") if st.value != MOS_OK else ""
        return st.value, res.value, it.value, sw.value

    def cond_estimate(self, ticket):
        """(kappa, steps): the Lanczos condition estimate of a completed
        ticket's first PCG sweep; call it before result()."""
        k, n = ctypes.c_double(), ctypes.c_int32()
        _check(lib().mos_engine_cond_estimate(self.ptr, ticket, ctypes.byref(k), ctypes.byref(n)),
               "mos_engine_cond_estimate")
        return k.value, n.value

    def option(self, option, value):
        _check(lib().mos_engine_option(self.ptr, option, int(value)), "mos_engine_option")

    def graph_stats(self):
        """(captures, replays) of iteration-chunk graphs so far."""
        c = ctypes.c_int64()
        r = ctypes.c_int64()
        _check(lib().mos_engine_graph_stats(self.ptr, ctypes.byref(c), ctypes.byref(r)), "mos_engine_graph_stats")
        return c.value, r.value

    def stats(self):
        a, q, cd, cs = (ctypes.c_int64() for _ in range(4))
        _check(lib().mos_engine_stats(self.ptr, ctypes.byref(a), ctypes.byref(q), ctypes.byref(cd), ctypes.byref(cs)),
               "mos_engine_stats")
        return dict(active=a.value, queued=q.value, capacity_dofs=cd.value, capacity_slots=cs.value)

    def close(self):
        if self.ptr:
            lib().mos_engine_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mos_engine_create(ctx, roms, mixed=False, device_bytes=8 << 30):
    return Engine(ctx, roms, mixed, device_bytes)


def mos_engine_submit(engine, *args, **kw):
    return engine.submit(*args, **kw)


def mos_engine_progress(engine, iterations=16):
    return engine.progress(iterations)


def mos_engine_result(engine, ticket):
    return engine.result(ticket)


def mos_engine_option(engine, option, value):
    engine.option(option, value)


def mos_engine_stats(engine):
    return engine.stats()


def mos_engine_destroy(engine):
    engine.close()


def mos_reconstruct(ctx, sol, vm=None, sigma6=None, noalloc=False):
    """Write von Mises and/or the six stress components into caller-owned
    device tensors ([n_cells, n_elem] and [n_cells, n_elem, 6]); float64 for
    an FP64 solution, float32 for a mixed one.  noalloc=True calls
    mos_reconstruct_noalloc (the library's static scratch, no device
    allocation)."""
    torch = ctx.torch
    want = torch.float32 if sol.precision == MOS_MIXED else torch.float64
    flags = 0
    for t, shape, flag in ((vm, (sol.n_cells, sol.n_elem), MOS_OUT_VM),
                           (sigma6, (sol.n_cells, sol.n_elem, 6), MOS_OUT_SIGMA6)):
        if t is None:
            continue
        if t.dtype != want or tuple(t.shape) != shape or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"output must be a contiguous {want} device tensor of shape {shape}")
        flags |= flag
    fn = lib().mos_reconstruct_noalloc if noalloc else lib().mos_reconstruct
    _check(fn(ctx.ptr, sol.ptr, flags, ctypes.c_void_p(vm.data_ptr() if vm is not None else 0),
              ctypes.c_void_p(sigma6.data_ptr() if sigma6 is not None else 0)),
           "mos_reconstruct_noalloc" if noalloc else "mos_reconstruct")


def mos_reconstruct_noalloc(ctx, sol, vm=None, sigma6=None):
    """mos_reconstruct through the allocation-free entry point."""
    mos_reconstruct(ctx, sol, vm=vm, sigma6=sigma6, noalloc=True)


def mos_reconstruct_displacement(ctx, sol, u_nodal):
    """Fine-mesh displacement of every cell (eq. 15) into a caller-owned
    contiguous float64 device tensor [n_cells, n_fe_dofs]."""
    torch = ctx.torch
    shape = (sol.n_cells, sol.roms[0].query(MOS_Q_CELL_DOFS))
    if u_nodal.dtype != torch.float64 or tuple(u_nodal.shape) != shape or not u_nodal.is_contiguous() \
            or not u_nodal.is_cuda:
        raise ValueError(f"output must be a contiguous float64 device tensor of shape {shape}")
    _check(lib().mos_reconstruct_displacement(ctx.ptr, sol.ptr, ctypes.c_void_p(u_nodal.data_ptr())),
           "mos_reconstruct_displacement")


def mos_reconstruct_plane(ctx, sol, grid, vm):
    """Von Mises at grid x grid points of every cell's mid-height plane into a
    caller-owned contiguous device tensor [n_cells, grid * grid]; float64 for
    an FP64 solution, float32 for a mixed one."""
    torch = ctx.torch
    want = torch.float32 if sol.precision == MOS_MIXED else torch.float64
    shape = (sol.n_cells, int(grid) * int(grid))
    if vm.dtype != want or tuple(vm.shape) != shape or not vm.is_contiguous() or not vm.is_cuda:
        raise ValueError(f"output must be a contiguous {want} device tensor of shape {shape}")
    _check(lib().mos_reconstruct_plane(ctx.ptr, sol.ptr, int(grid), ctypes.c_void_p(vm.data_ptr())),
           "mos_reconstruct_plane")


def mos_get_solution(sol):
    n = sol.query(MOS_Q_GLOBAL_DOFS)
    u = np.empty(n)
    res = ctypes.c_double()
    it = ctypes.c_int32()
    _check(lib().mos_get_solution(sol.ptr, _ptr(u), ctypes.byref(res), ctypes.byref(it)), "mos_get_solution")
    return u, res.value, it.value


def mos_get_cond_estimate(sol):
    """(kappa, steps): Lanczos estimate of the condition number of the
    preconditioned reduced system from the first PCG sweep's steps."""
    k, n = ctypes.c_double(), ctypes.c_int32()
    _check(lib().mos_get_cond_estimate(sol.ptr, ctypes.byref(k), ctypes.byref(n)), "mos_get_cond_estimate")
    return k.value, n.value


def mos_engine_cond_estimate(engine, ticket):
    return engine.cond_estimate(ticket)


def mos_cell_export(cell):
    n_dofs = cell.query(MOS_Q_CELL_DOFS)
    nnz = cell.query(MOS_Q_CELL_NNZ)
    n_elem = cell.query(MOS_Q_CELL_ELEMS)
    indptr = np.empty(n_dofs + 1, dtype=np.int64)
    indices = np.empty(nnz, dtype=np.int32)
    data = np.empty(nnz)
    b = np.empty(n_dofs)
    mat = np.empty(n_elem, dtype=np.uint8)
    _check(lib().mos_cell_export(cell.ptr, _ptr(indptr), _ptr(indices), _ptr(data), _ptr(b), _ptr(mat)),
           "mos_cell_export")
    return indptr, indices, data, b, mat


def mos_rom_export(rom):
    n = rom.query(MOS_Q_N)
    n_dofs = rom.query(MOS_Q_CELL_DOFS)
    phi = np.empty((n_dofs, n))
    fT = np.empty(n_dofs)
    Kr = np.empty((n, n))
    br = np.empty(n)
    _check(lib().mos_rom_export(rom.ptr, _ptr(phi), _ptr(fT), _ptr(Kr), _ptr(br)), "mos_rom_export")
    return phi, fT, Kr, br


def mos_array_layout(ctx, nx_cells, ny_cells, rom, pattern=False, nz_cells=1):
    n_nodes = ctypes.c_int64()
    f = lib().mos_array_layout
    _check(f(ctx.ptr, nx_cells, ny_cells, nz_cells, rom.ptr, ctypes.byref(n_nodes), None, None, None, None),
           "mos_array_layout")
    nn = n_nodes.value
    S = rom.query(MOS_Q_N) // 3
    coords = np.empty((nn, 3))
    conn = np.empty((nx_cells * ny_cells * nz_cells, S), dtype=np.int32)
    indptr = indices = None
    if pattern:
        indptr = np.empty(3 * nn + 1, dtype=np.int64)
        _check(f(ctx.ptr, nx_cells, ny_cells, nz_cells, rom.ptr, ctypes.byref(n_nodes), None, None, _ptr(indptr),
                 None), "mos_array_layout")
        indices = np.empty(int(indptr[-1]), dtype=np.int32)
    _check(f(ctx.ptr, nx_cells, ny_cells, nz_cells, rom.ptr, ctypes.byref(n_nodes), _ptr(coords), _ptr(conn),
             _ptr(indptr), _ptr(indices)), "mos_array_layout")
    return coords, conn, indptr, indices


def mos_timing_start(ctx, kernel, every=1):
    _check(lib().mos_timing_start(ctx.ptr, kernel, every), "mos_timing_start")


def mos_timing_stop(ctx):
    """Returns (timed launches, their total milliseconds, launches seen)."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    seen = ctypes.c_int64()
    _check(lib().mos_timing_stop(ctx.ptr, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(seen)), "mos_timing_stop")
    return n.value, ms.value, seen.value
