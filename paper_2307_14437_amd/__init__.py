"""Python binding of libgofd (the GoFD fractional-Laplacian library for MI355X).

Argument marshalling only: every step of the method runs in the HIP library
behind the C ABI declared in ``include/gofd.h``.  PyTorch supplies device
memory and the current stream.  There is no CPU fallback: importing this
module fails loudly when the compiled library is missing.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgofd.so")

# status codes
OK = 0
E_ARG, E_DEGENERATE, E_RANK, E_ZERO_COLSUM, E_NOT_CONVERGED = -1, -2, -3, -4, -5
E_BREAKDOWN, E_HIP, E_OOM, E_NUMERIC, E_UNSUPPORTED = -6, -7, -8, -9, -10

# transfer parts
TR_ELEM, TR_ELL_VERTS, TR_ELL_WEIGHTS, TR_CSC_OFFSETS = 0, 1, 2, 3
TR_CSC_NODES, TR_CSC_WEIGHTS, TR_D, TR_BOUNDARY = 4, 5, 6, 7

# apply flags
FP32_GRID, SYMMETRIC, UNSCALED, SCALE_H2S, INTERIOR = 1, 2, 4, 8, 16

# preconditioners
PC_NONE, PC_DIAG, PC_IC1_5, PC_IC1_9, PC_IC1_27 = 0, 1, 5, 9, 27
PC_MULTICOLOR = 256
PC_LAPLACIAN = 512
PC_BLOCK_MULTICOLOR = 1024
PC_BY_NAME = {"NONE": PC_NONE, "DIAG": PC_DIAG}
for _p, _k in (("5", PC_IC1_5), ("9", PC_IC1_9), ("27", PC_IC1_27)):
    # IC1_<p>: A_FD on the pattern; _LAP: the discrete Laplacian on it; _MC: multicolour order, _BMC: block
    # multicolour order
    for _lap, _fl in (("", 0), ("_LAP", PC_LAPLACIAN)):
        PC_BY_NAME[f"IC1_{_p}{_lap}"] = _k | _fl
        PC_BY_NAME[f"IC1_{_p}{_lap}_MC"] = _k | _fl | PC_MULTICOLOR
        PC_BY_NAME[f"IC1_{_p}{_lap}_BMC"] = _k | _fl | PC_BLOCK_MULTICOLOR

F_GRID, F_VERTEX = 0, 1
MODE_FP64, MODE_FP32_REFINE, MODE_FP32_RELIABLE = 0, 1, 2


class GofdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("N", ctypes.c_int), ("R", ctypes.c_double),
                ("center", ctypes.c_double * 3)]


class TransferInfo(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_inside", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("n_interior", ctypes.c_int64), ("n_boundary", ctypes.c_int64),
                ("dmin_interior", ctypes.c_double), ("a_h", ctypes.c_double), ("h_bound", ctypes.c_double),
                ("exact_tests", ctypes.c_int64), ("max_col_count", ctypes.c_int64),
                ("rp_slots", ctypes.c_int64), ("rp_entries", ctypes.c_int64), ("rp_seg_rows", ctypes.c_int64),
                ("kernel_us", ctypes.c_double * 8)]


TRANSFER_KERNELS = ("records", "locate", "count", "scan", "fill", "sort", "rows", "colsum")


class CgTapeInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("checkpoints", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("converged", ctypes.c_int)]


class Info1D(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int), ("L", ctypes.c_int), ("h", ctypes.c_double), ("a_h", ctypes.c_double),
                ("dmin_interior", ctypes.c_double), ("n_inside", ctypes.c_int64)]


class SolveInfo1D(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double), ("converged", ctypes.c_int)]


GOFD1D_ELEM, GOFD1D_WEIGHTS, GOFD1D_D, GOFD1D_T = 0, 1, 2, 3


MMPDE_KERNELS = ("hess_fd", "field", "energy", "cg_elem", "cg_vert", "cg_update")


class MmpdeKernelStats(ctypes.Structure):
    _fields_ = [("avg_us", ctypes.c_double * len(MMPDE_KERNELS)), ("launches", ctypes.c_int64 * len(MMPDE_KERNELS))]


class MmpdeOpts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("t_end", ctypes.c_double), ("dt0", ctypes.c_double),
                ("max_steps", ctypes.c_int), ("fixed_dt", ctypes.c_double), ("gtol", ctypes.c_double),
                ("cg_tol", ctypes.c_double), ("max_cg", ctypes.c_int),
                ("stats", ctypes.POINTER(MmpdeKernelStats))]


class MmpdeInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("rejected", ctypes.c_int), ("t", ctypes.c_double),
                ("energy_start", ctypes.c_double), ("energy_end", ctypes.c_double),
                ("cg_iterations", ctypes.c_int64), ("grad_start", ctypes.c_double), ("grad_end", ctypes.c_double)]


class FdwOpts(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("richardson", ctypes.c_int)]


class PrecondInfo(ctypes.Structure):
    _fields_ = [("shift", ctypes.c_double), ("nnz_L", ctypes.c_int64), ("levels", ctypes.c_int),
                ("setup_ms", ctypes.c_double), ("colours", ctypes.c_int), ("apply_bytes", ctypes.c_int64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("max_iter", ctypes.c_int), ("check_every", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("stage_ms", ctypes.POINTER(ctypes.c_double)),
                ("x0", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("refinements", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("time_ms", ctypes.c_double), ("status", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libgofd.so is not built ({LIB_PATH}); run __graft_entry__.build() or "
                          "python paper_2307_14437_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "gofd_create": [ctypes.POINTER(vp), vp],
        "gofd_destroy": [vp],
        "gofd_set_stream": [vp, vp],
        "gofd_build_transfer": [vp, i32, i64, vp, i64, vp, ctypes.POINTER(_Grid), ctypes.POINTER(vp),
                                ctypes.POINTER(TransferInfo)],
        "gofd_transfer_free": [vp],
        "gofd_transfer_export": [vp, vp, i32, vp],
        "gofd_fd_weights": [vp, dbl, ctypes.POINTER(_Grid), ctypes.POINTER(FdwOpts), ctypes.POINTER(vp)],
        "gofd_fdop_from_table": [vp, dbl, ctypes.POINTER(_Grid), ctypes.POINTER(dbl), ctypes.POINTER(vp)],
        "gofd_fdop_get_table": [vp, vp, ctypes.POINTER(dbl)],
        "gofd_fdop_free": [vp],
        "gofd_apply_afd": [vp, vp, i32, vp, vp, i32],
        "gofd_apply_Ah": [vp, vp, vp, i32, vp, vp, i32],
        "gofd_apply_Ah_noalloc": [vp, vp, vp, i32, vp, vp, i32],
        "gofd_precond_create": [vp, vp, vp, i32, ctypes.POINTER(vp), ctypes.POINTER(PrecondInfo)],
        "gofd_precond_free": [vp],
        "gofd_precond_export": [vp, vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(dbl)],
        "gofd_precond_export_order": [vp, vp, ctypes.POINTER(ctypes.c_int32)],
        "gofd_solve": [vp, vp, vp, vp, i32, vp, i32, dbl, ctypes.POINTER(SolveOpts), vp,
                       ctypes.POINTER(SolveInfo)],
        "gofd_solve_batched": [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                               ctypes.POINTER(i32), ctypes.POINTER(vp), i32, dbl, ctypes.POINTER(SolveOpts),
                               ctypes.POINTER(vp), ctypes.POINTER(SolveInfo)],
        "gofd_solve_adjoint": [vp, vp, vp, vp, vp, vp, vp, dbl, ctypes.POINTER(SolveOpts), vp, vp, vp,
                               ctypes.POINTER(SolveInfo)],
        "gofd_time_kernel": [vp, vp, vp, i32, i32, vp, i32, i32, ctypes.POINTER(dbl)],
        "gofd_cg_checkpointed": [vp, vp, vp, vp, vp, i32, dbl, i32, vp, ctypes.POINTER(vp),
                                 ctypes.POINTER(CgTapeInfo)],
        "gofd_cg_unrolled_grad": [vp, vp, vp, vp, vp, vp],
        "gofd_cg_tape_read": [vp, vp, i32, vp, vp, vp, ctypes.POINTER(dbl)],
        "gofd_cg_tape_free": [vp],
        "gofd_autotune": [vp, ctypes.POINTER(_Grid), i32, ctypes.POINTER(i32), ctypes.POINTER(dbl)],
        "gofd_set_schedule": [vp, ctypes.POINTER(_Grid), i32, i32],
        "gofd1d_create": [vp, i64, vp, i32, dbl, dbl, dbl, ctypes.POINTER(vp), ctypes.POINTER(Info1D)],
        "gofd1d_free": [vp],
        "gofd1d_export": [vp, vp, i32, vp],
        "gofd1d_apply_Ah": [vp, vp, i32, vp, vp],
        "gofd1d_solve": [vp, vp, i32, vp, dbl, i32, i32, vp, ctypes.POINTER(SolveInfo1D)],
        "gofd_mmpde_create": [vp, i64, i64, vp, i32, ctypes.POINTER(vp)],
        "gofd_mmpde_free": [vp],
        "gofd_mmpde_metric": [vp, vp, vp, vp, vp, vp, ctypes.POINTER(dbl)],
        "gofd_mmpde_energy": [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(dbl)],
        "gofd_mmpde_element_hessians": [vp, vp, vp, vp, vp],
        "gofd_mmpde_move": [vp, vp, vp, vp, ctypes.POINTER(MmpdeOpts), ctypes.POINTER(MmpdeInfo)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.gofd_last_error.argtypes = [vp]
    lib.gofd_last_error.restype = ctypes.c_char_p
    lib.gofd_strerror.argtypes = [ctypes.c_int]
    lib.gofd_strerror.restype = ctypes.c_char_p
    return lib


lib = _load()

EXPORTED = [
    "gofd_create", "gofd_destroy", "gofd_set_stream", "gofd_last_error", "gofd_strerror",
    "gofd_build_transfer", "gofd_transfer_free", "gofd_transfer_export", "gofd_fd_weights",
    "gofd_fdop_from_table", "gofd_fdop_get_table", "gofd_fdop_free", "gofd_apply_afd", "gofd_apply_Ah",
    "gofd_apply_Ah_noalloc",
    "gofd_precond_create", "gofd_precond_free", "gofd_precond_export", "gofd_precond_export_order",
    "gofd_solve", "gofd_solve_batched",
    "gofd_solve_adjoint", "gofd_time_kernel", "gofd_cg_checkpointed", "gofd_cg_unrolled_grad",
    "gofd_cg_tape_read", "gofd_cg_tape_free",
    "gofd1d_create", "gofd1d_free", "gofd1d_export", "gofd1d_apply_Ah", "gofd1d_solve",
    "gofd_mmpde_create", "gofd_mmpde_free", "gofd_mmpde_metric", "gofd_mmpde_energy",
    "gofd_mmpde_element_hessians", "gofd_mmpde_move",
]

K_PASS_A, K_PASS_B, K_PASS_C, K_SCATTER, K_GATHER = 0, 1, 2, 3, 4


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _grid(grid) -> _Grid:
    c = list(grid.center) + [0.0] * (3 - len(grid.center))
    return _Grid(int(grid.d), int(grid.N), float(grid.R), (ctypes.c_double * 3)(*c))


class Context:
    """A library context bound to torch's current HIP stream on the current device."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the GoFD library runs on the GPU only")
        self._torch = torch
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        h = ctypes.c_void_p()
        self._check(lib.gofd_create(ctypes.byref(h), ctypes.c_void_p(s.cuda_stream)), None)
        self.handle = h

    def _check(self, code, h="self"):
        if code != OK:
            msg = lib.gofd_last_error(self.handle).decode() if h == "self" and getattr(self, "handle", None) \
                else lib.gofd_strerror(code).decode()
            raise GofdError(code, msg)

    def check(self, code):
        self._check(code)

    def close(self):
        if getattr(self, "handle", None):
            lib.gofd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Transfer:
    def __init__(self, ctx: Context, X, elems, grid):
        torch = ctx._torch
        if X.dtype != torch.float64 or elems.dtype != torch.int32 or not X.is_cuda or not elems.is_cuda:
            raise TypeError("X must be a CUDA float64 tensor and elems a CUDA int32 tensor")
        X = X.contiguous()
        elems = elems.contiguous()
        self.ctx, self.grid = ctx, grid
        self.d = int(X.shape[1])
        self.nv = int(X.shape[0])
        self.ne = int(elems.shape[0])
        self.W = 2 * grid.N + 1
        self.n_nodes = self.W ** self.d
        h = ctypes.c_void_p()
        info = TransferInfo()
        g = _grid(grid)
        ctx.check(lib.gofd_build_transfer(ctx.handle, self.d, self.nv, _ptr(X), self.ne, _ptr(elems),
                                          ctypes.byref(g), ctypes.byref(h), ctypes.byref(info)))
        self.handle = h
        self.info = {k: getattr(info, k) for k, _ in TransferInfo._fields_}
        self.info["kernel_us"] = dict(zip(TRANSFER_KERNELS, list(info.kernel_us)))

    def export(self, part):
        torch = self.ctx._torch
        nnz = self.info["nnz"]
        d1 = self.d + 1
        spec = {
            TR_ELEM: (self.n_nodes, torch.int32), TR_ELL_VERTS: (self.n_nodes * d1, torch.int32),
            TR_ELL_WEIGHTS: (self.n_nodes * d1, torch.float64), TR_CSC_OFFSETS: (self.nv + 1, torch.int32),
            TR_CSC_NODES: (nnz, torch.int32), TR_CSC_WEIGHTS: (nnz, torch.float64),
            TR_D: (self.nv, torch.float64), TR_BOUNDARY: (self.nv, torch.uint8),
        }[part]
        out = torch.empty(max(spec[0], 1), dtype=spec[1], device="cuda")
        self.ctx.check(lib.gofd_transfer_export(self.ctx.handle, self.handle, part, _ptr(out)))
        return out[: spec[0]]

    def close(self):
        if getattr(self, "handle", None):
            lib.gofd_transfer_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FdOp:
    def __init__(self, ctx: Context, s, grid, T=None, M=0, richardson=True):
        self.ctx, self.s, self.grid = ctx, float(s), grid
        self.W = 2 * grid.N + 1
        h = ctypes.c_void_p()
        g = _grid(grid)
        if T is None:
            opts = FdwOpts(int(M), 1 if richardson else 0)
            ctx.check(lib.gofd_fd_weights(ctx.handle, self.s, ctypes.byref(g), ctypes.byref(opts), ctypes.byref(h)))
        else:
            T = np.ascontiguousarray(T, dtype=np.float64)
            if T.size != self.W ** grid.d:
                raise ValueError("T must hold (2N+1)^d values")
            ctx.check(lib.gofd_fdop_from_table(ctx.handle, self.s, ctypes.byref(g),
                                               T.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               ctypes.byref(h)))
        self.handle = h

    def table(self):
        out = np.empty((self.W,) * self.grid.d, dtype=np.float64)
        self.ctx.check(lib.gofd_fdop_get_table(self.ctx.handle, self.handle,
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib.gofd_fdop_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def apply_afd(ctx: Context, op: FdOp, v, flags=0):
    v = v.contiguous()
    nrhs = v.numel() // (op.W ** op.grid.d)
    y = ctx._torch.empty_like(v)
    ctx.check(lib.gofd_apply_afd(ctx.handle, op.handle, nrhs, _ptr(v), _ptr(y), int(flags)))
    return y


def apply_Ah(ctx: Context, tr: Transfer, op: FdOp, u, flags=0):
    u = u.contiguous()
    nrhs = u.numel() // tr.nv
    y = ctx._torch.empty_like(u)
    ctx.check(lib.gofd_apply_Ah(ctx.handle, tr.handle, op.handle, nrhs, _ptr(u), _ptr(y), int(flags)))
    return y


def apply_Ah_noalloc(ctx: Context, tr: Transfer, op: FdOp, u, y, flags=0):
    """gofd_apply_Ah_noalloc: y (caller-allocated, like u) = A_h u with the product's workspaces in the
    library's static device array (the call allocates nothing; calls on one GPU must not overlap)."""
    if not (u.is_contiguous() and y.is_contiguous()) or y.numel() != u.numel():
        raise ValueError("u and y must be contiguous and of the same size")
    nrhs = u.numel() // tr.nv
    ctx.check(lib.gofd_apply_Ah_noalloc(ctx.handle, tr.handle, op.handle, nrhs, _ptr(u), _ptr(y), int(flags)))
    return y


class Precond:
    def __init__(self, ctx: Context, tr: Transfer, op: FdOp, kind):
        if isinstance(kind, str):
            kind = PC_BY_NAME[kind]
        self.ctx, self.kind, self.nv = ctx, int(kind), tr.nv
        h = ctypes.c_void_p()
        info = PrecondInfo()
        ctx.check(lib.gofd_precond_create(ctx.handle, tr.handle, op.handle, self.kind, ctypes.byref(h),
                                          ctypes.byref(info)))
        self.handle = h
        self.info = {k: getattr(info, k) for k, _ in PrecondInfo._fields_}

    def export(self):
        import scipy.sparse as sp
        nnz = int(self.info["nnz_L"])
        rp = np.empty(self.nv + 1, dtype=np.int32)
        ci = np.empty(nnz, dtype=np.int32)
        va = np.empty(nnz, dtype=np.float64)
        self.ctx.check(lib.gofd_precond_export(self.ctx.handle, self.handle,
                                               rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                               ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                               va.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return sp.csr_matrix((va, ci, rp), shape=(self.nv, self.nv))

    def order(self):
        """Elimination order of the factor: row i of export() is vertex order()[i]."""
        perm = np.empty(self.nv, dtype=np.int32)
        self.ctx.check(lib.gofd_precond_export_order(self.ctx.handle, self.handle,
                                                     perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return perm

    def close(self):
        if getattr(self, "handle", None):
            lib.gofd_precond_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STAGES = ("gather", "passA", "passB", "passC", "scatter", "precond")


def _torch_float64():
    import torch
    return torch.float64


def _opts(mode=MODE_FP64, max_iter=0, check_every=0, inner_tol=0.0, max_refine=0, use_graph=0, history=None,
          stage_ms=None, x0=None):
    o = SolveOpts(int(mode), int(max_iter), int(check_every), float(inner_tol), int(max_refine), int(use_graph),
                  None, None, None)
    if x0 is not None:
        if not x0.is_contiguous() or x0.dtype != _torch_float64():
            raise ValueError("x0 must be a contiguous float64 device tensor")
        o.x0 = x0.data_ptr()
    if history is not None:
        o.history = history.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if stage_ms is not None:
        if stage_ms.dtype != np.float64 or stage_ms.size < len(STAGES):
            raise ValueError("stage_ms must be a float64 array of 6 entries")
        o.stage_ms = stage_ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return o


def solve(ctx: Context, tr: Transfer, op: FdOp, f, tol=1e-10, pc: Precond | None = None, f_loc=F_GRID,
          raise_on_error=True, **kw):
    """Solve eq. GoFD-2 (f on the grid) or GoFD-3 (f on the vertices); returns (u, [info dicts])."""
    torch = ctx._torch
    f = f.contiguous()
    per = tr.n_nodes if f_loc == F_GRID else tr.nv
    nrhs = f.numel() // per
    u = torch.empty(nrhs * tr.nv, dtype=torch.float64, device=f.device)
    infos = (SolveInfo * nrhs)()
    opts = _opts(**kw)
    code = lib.gofd_solve(ctx.handle, tr.handle, op.handle, pc.handle if pc else None, nrhs, _ptr(f), int(f_loc),
                          float(tol), ctypes.byref(opts), _ptr(u), infos)
    if code != OK and raise_on_error:
        ctx.check(code)
    return u.view(nrhs, tr.nv) if nrhs > 1 else u, [infos[i].as_dict() for i in range(nrhs)]


def solve_batched(ctx: Context, trs, ops, pcs, fs, tol=1e-8, f_loc=F_GRID, raise_on_error=True, **kw):
    """Many problems in one call: fs[q] holds nrhs[q] right-hand sides of problem q."""
    torch = ctx._torch
    n = len(trs)
    nr = []
    us = []
    for q in range(n):
        per = trs[q].n_nodes if f_loc == F_GRID else trs[q].nv
        nr.append(fs[q].numel() // per)
        us.append(torch.empty(nr[-1] * trs[q].nv, dtype=torch.float64, device=fs[q].device))
    fs = [f.contiguous() for f in fs]
    arr = lambda xs: (ctypes.c_void_p * n)(*[x.handle if x is not None else None for x in xs])
    fp = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
    up = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
    nrr = (ctypes.c_int * n)(*nr)
    infos = (SolveInfo * sum(nr))()
    opts = _opts(**kw)
    code = lib.gofd_solve_batched(ctx.handle, n, arr(trs), arr(ops), arr(pcs if pcs else [None] * n), nrr, fp,
                                  int(f_loc), float(tol), ctypes.byref(opts), up, infos)
    if code != OK and raise_on_error:
        ctx.check(code)
    return us, [infos[i].as_dict() for i in range(sum(nr))]


def solve_adjoint(ctx: Context, tr: Transfer, op: FdOp, dLdu, u, f, tol=1e-10, pc: Precond | None = None,
                  want_f=True, want_X=True, **kw):
    torch = ctx._torch
    gf = torch.empty(tr.n_nodes, dtype=torch.float64, device=u.device) if want_f else None
    gX = torch.empty(tr.nv * tr.d, dtype=torch.float64, device=u.device) if want_X else None
    lam = torch.empty(tr.nv, dtype=torch.float64, device=u.device)
    info = SolveInfo()
    opts = _opts(**kw)
    ctx.check(lib.gofd_solve_adjoint(ctx.handle, tr.handle, op.handle, pc.handle if pc else None,
                                     _ptr(dLdu.contiguous()), _ptr(u.contiguous()), _ptr(f.contiguous()),
                                     float(tol), ctypes.byref(opts), _ptr(gf) if gf is not None else None,
                                     _ptr(gX) if gX is not None else None, _ptr(lam), ctypes.byref(info)))
    return gf, (gX.view(tr.nv, tr.d) if gX is not None else None), lam, info.as_dict()


class CgTape:
    """Truncated CG of eq. GoFD-2 with checkpointed iterates (gofd_cg_checkpointed); x holds x_n."""

    def __init__(self, ctx: Context, tr: Transfer, op: FdOp, f, x0=None, max_iter=100, tol=0.0, ckpt_every=8):
        torch = ctx._torch
        self.ctx, self.tr, self.op, self.max_iter = ctx, tr, op, int(max_iter)
        f = f.contiguous()
        self.x = torch.empty(tr.nv, dtype=torch.float64, device=f.device)
        h = ctypes.c_void_p()
        info = CgTapeInfo()
        ctx.check(lib.gofd_cg_checkpointed(ctx.handle, tr.handle, op.handle, _ptr(f),
                                           _ptr(x0.contiguous()) if x0 is not None else None, self.max_iter,
                                           float(tol), int(ckpt_every), _ptr(self.x), ctypes.byref(h),
                                           ctypes.byref(info)))
        self.handle = h
        self.info = {k: getattr(info, k) for k, _ in CgTapeInfo._fields_}

    def grad(self, xbar, want_f=True, want_X=True, want_x0=False):
        """Unrolled gradients (grad_f on the grid, grad_X as N_v x d, grad_x0) of a loss with dL/dx_n = xbar."""
        torch = self.ctx._torch
        dev = xbar.device
        gf = torch.empty(self.tr.n_nodes, dtype=torch.float64, device=dev) if want_f else None
        gX = torch.empty(self.tr.nv * self.tr.d, dtype=torch.float64, device=dev) if want_X else None
        g0 = torch.empty(self.tr.nv, dtype=torch.float64, device=dev) if want_x0 else None
        self.ctx.check(lib.gofd_cg_unrolled_grad(self.ctx.handle, self.handle, _ptr(xbar.contiguous()),
                                                 _ptr(gf) if gf is not None else None,
                                                 _ptr(gX) if gX is not None else None,
                                                 _ptr(g0) if g0 is not None else None))
        return gf, (gX.view(self.tr.nv, self.tr.d) if gX is not None else None), g0

    def checkpoint(self, j):
        """(x, r, p) of checkpoint j and the scalar record (gamma, delta, alpha, beta arrays)."""
        torch = self.ctx._torch
        x, r, p = (torch.empty(self.tr.nv, dtype=torch.float64, device=self.x.device) for _ in range(3))
        sc = np.empty(4 * (self.max_iter + 1), dtype=np.float64)
        self.ctx.check(lib.gofd_cg_tape_read(self.ctx.handle, self.handle, int(j), _ptr(x), _ptr(r), _ptr(p),
                                             sc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return x, r, p, sc.reshape(4, self.max_iter + 1)

    def close(self):
        if getattr(self, "handle", None):
            lib.gofd_cg_tape_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Gofd1D:
    """GoFD in one dimension (the 1D example of Section 5): a mesh of an interval given by its increasing
    vertices, the grid (N, R, center), T by the closed form eq. T-1D-0; products and CG solves of eq. GoFD-2
    run one workgroup per field or right-hand side (FFT length <= 4096)."""

    def __init__(self, ctx: Context, x, N, R, center, s):
        torch = ctx._torch
        if x.dtype != torch.float64 or not x.is_cuda or x.dim() != 1:
            raise TypeError("x must be a 1D CUDA float64 tensor")
        x = x.contiguous()
        self.ctx, self.nv, self.N, self.R, self.center, self.s = ctx, int(x.numel()), int(N), float(R), \
            float(center), float(s)
        h = ctypes.c_void_p()
        info = Info1D()
        ctx.check(lib.gofd1d_create(ctx.handle, self.nv, _ptr(x), self.N, self.R, self.center, self.s,
                                    ctypes.byref(h), ctypes.byref(info)))
        self.handle = h
        self.info = {k: getattr(info, k) for k, _ in Info1D._fields_}
        self.W = self.info["W"]

    def export(self, part):
        torch = self.ctx._torch
        n, dt = {GOFD1D_ELEM: (self.W, torch.int32), GOFD1D_WEIGHTS: (2 * self.W, torch.float64),
                 GOFD1D_D: (self.nv, torch.float64), GOFD1D_T: (2 * self.N + 1, torch.float64)}[part]
        out = torch.empty(n, dtype=dt, device="cuda")
        self.ctx.check(lib.gofd1d_export(self.ctx.handle, self.handle, int(part), _ptr(out)))
        return out

    def apply_Ah(self, u):
        """D^{-1} I^T A_FD I u for u of shape (N_v,) or (fields, N_v)."""
        u = u.contiguous()
        nf = 1 if u.dim() == 1 else int(u.shape[0])
        y = self.ctx._torch.empty_like(u)
        self.ctx.check(lib.gofd1d_apply_Ah(self.ctx.handle, self.handle, nf, _ptr(u), _ptr(y)))
        return y

    def solve(self, f, tol=1e-10, max_iter=0, precond=0, raise_on_error=True):
        """u (nrhs, N_v) and per-rhs info for f of shape (W,) or (nrhs, W) on the grid."""
        torch = self.ctx._torch
        f = f.contiguous()
        nrhs = 1 if f.dim() == 1 else int(f.shape[0])
        u = torch.empty(nrhs, self.nv, dtype=torch.float64, device=f.device)
        infos = (SolveInfo1D * nrhs)()
        code = lib.gofd1d_solve(self.ctx.handle, self.handle, nrhs, _ptr(f), float(tol), int(max_iter),
                                int(precond), _ptr(u), infos)
        if raise_on_error:
            self.ctx.check(code)
        return u, [{k: getattr(i, k) for k, _ in SolveInfo1D._fields_} for i in infos]

    def close(self):
        if getattr(self, "handle", None):
            lib.gofd1d_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MMPDE_BOUNDARY_CIRCLE, MMPDE_BOUNDARY_FIXED = 0, 1


class Mmpde:
    """MMPDE mesh adaptation on a fixed triangulation (Section 4): vertex metrics of eq. MK-1 from a solution,
    the energy of eq. I-h in the metric field of a background mesh and its gradient, and the moving mesh
    equations (eq. x-1) integrated in place.  Metrics are N x 3 (m11, m12, m22), coordinates N_v x 2, all
    float64 on the device."""

    def __init__(self, ctx: Context, nv, elems, boundary=MMPDE_BOUNDARY_CIRCLE):
        torch = ctx._torch
        if elems.dtype != torch.int32 or not elems.is_cuda:
            raise TypeError("elems must be a CUDA int32 tensor")
        elems = elems.contiguous()
        self.ctx, self.nv, self.ne = ctx, int(nv), int(elems.shape[0])
        h = ctypes.c_void_p()
        ctx.check(lib.gofd_mmpde_create(ctx.handle, self.nv, self.ne, _ptr(elems), int(boundary), ctypes.byref(h)))
        self.handle = h

    def _x(self, X):
        torch = self.ctx._torch
        if X.dtype != torch.float64 or not X.is_cuda or tuple(X.shape) != (self.nv, 2):
            raise TypeError("X must be a CUDA float64 tensor of shape (N_v, 2)")
        return X.contiguous()

    def metric(self, X, u, with_hessian=False):
        """(vertex metrics Mv, alpha_h[, vertex Hessians N_v x 3])."""
        torch = self.ctx._torch
        X = self._x(X)
        M = torch.empty(self.nv, 3, dtype=torch.float64, device=X.device)
        H = torch.empty(self.nv, 3, dtype=torch.float64, device=X.device) if with_hessian else None
        a = ctypes.c_double()
        self.ctx.check(lib.gofd_mmpde_metric(self.ctx.handle, self.handle, _ptr(X), _ptr(u.contiguous()), _ptr(M),
                                             _ptr(H) if H is not None else None, ctypes.byref(a)))
        return (M, a.value, H) if with_hessian else (M, a.value)

    def energy(self, Xb, Mv, X, grad=True):
        """(I_h, dI_h/dX or None, element metrics M_K) of the mesh X in the metric field of (Xb, Mv)."""
        torch = self.ctx._torch
        Xb, X = self._x(Xb), self._x(X)
        G = torch.empty(self.nv, 2, dtype=torch.float64, device=X.device) if grad else None
        MK = torch.empty(self.ne, 3, dtype=torch.float64, device=X.device)
        e = ctypes.c_double()
        self.ctx.check(lib.gofd_mmpde_energy(self.ctx.handle, self.handle, _ptr(Xb), _ptr(Mv.contiguous()), _ptr(X),
                                             _ptr(G) if G is not None else None, _ptr(MK), ctypes.byref(e)))
        return e.value, G, MK

    def element_hessians(self, X, MK):
        """N_e x 6 x 6 Hessians of the elements' terms of I_h for the element metrics MK (central differences,
        symmetrised)."""
        torch = self.ctx._torch
        X = self._x(X)
        H = torch.empty(self.ne, 6, 6, dtype=torch.float64, device=X.device)
        self.ctx.check(lib.gofd_mmpde_element_hessians(self.ctx.handle, self.handle, _ptr(X), _ptr(MK.contiguous()),
                                                       _ptr(H)))
        return H

    def move(self, X, Mv, tau=1e-2, t_end=1.0, dt0=1e-3, max_steps=400, fixed_dt=0.0, gtol=1e-6, cg_tol=1e-10,
             max_cg=20000, kernel_stats=False):
        """Moves X (contiguous, modified in place) by eq. x-1 for its vertex metrics Mv; returns the info dict
        (with kernel_stats: also "kernels", name -> (mean us of the first launches, launches))."""
        if not X.is_contiguous():
            raise TypeError("X must be contiguous (it is moved in place)")
        self._x(X)
        ks = MmpdeKernelStats() if kernel_stats else None
        o = MmpdeOpts(float(tau), float(t_end), float(dt0), int(max_steps), float(fixed_dt), float(gtol),
                      float(cg_tol), int(max_cg), ctypes.pointer(ks) if ks is not None else None)
        info = MmpdeInfo()
        self.ctx.check(lib.gofd_mmpde_move(self.ctx.handle, self.handle, _ptr(X), _ptr(Mv.contiguous()),
                                           ctypes.byref(o), ctypes.byref(info)))
        out = {k: getattr(info, k) for k, _ in MmpdeInfo._fields_}
        if ks is not None:
            out["kernels"] = {n: (ks.avg_us[i], ks.launches[i]) for i, n in enumerate(MMPDE_KERNELS)}
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib.gofd_mmpde_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


N_COL_SCHED = 4
COL_SCHEDULES = ((16, 2), (16, 1), (8, 2), (16, 4))     # (values per thread, column slots per block)


def fft_period(N: int) -> int:
    """FFT length of the embedding for a grid of half-width N (as the library computes it)."""
    L = 1
    while L < 4 * N:
        L <<= 1
    return max(8, L)


def _cache_key(arch: str, grid, fp32: bool) -> str:
    return f"{arch}/d{grid.d}/L{fft_period(grid.N)}/{'fp32' if fp32 else 'fp64'}"


def cache_lookup(path, key, full=False):
    """Schedule stored under key in the JSON tuning cache at path (the whole entry with full=True), or None."""
    import json
    if not path or not os.path.exists(path):
        return None
    with open(path) as fh:
        entry = json.load(fh).get(key)
    if entry is None:
        return None
    return entry if full else int(entry["schedule"])


def cache_store(path, key, sched, times, row=0):
    """Record a tuning result under key in the JSON cache at path (other keys are kept)."""
    import json
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data[key] = {"schedule": int(sched), "row": int(row), "ms": [None if t is None else float(t) for t in times]}
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


N_TUNE_TIMES = 6
SCHED_ROWS = 256


def autotune_all(ctx: Context, grid, fp32=True, cache=None):
    """Tune every schedulable pass for the grid's FFT length and precision: 2D the column pass and the first
    row pass of the products, 3D the y/z/y passes.  From the JSON cache when it holds this device
    architecture, dimension, length and precision, else timed on the device (and stored in the cache).
    Returns {"col": .., "row": .., "times": [...] or None} (2D) or {"yzy": .., "times": ...} (3D)."""
    import torch
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    key = _cache_key(arch, grid, fp32)
    g = _grid(grid)
    flags = FP32_GRID if fp32 else 0
    hit = cache_lookup(cache, key, full=True)
    if hit is not None:
        ctx.check(lib.gofd_set_schedule(ctx.handle, ctypes.byref(g), flags, int(hit["schedule"])))
        if grid.d == 2 and hit.get("row"):
            ctx.check(lib.gofd_set_schedule(ctx.handle, ctypes.byref(g), flags | SCHED_ROWS, int(hit["row"])))
        out = {"times": None}
    else:
        sch = (ctypes.c_int * 2)()
        t = (ctypes.c_double * N_TUNE_TIMES)()
        ctx.check(lib.gofd_autotune(ctx.handle, ctypes.byref(g), flags, sch, t))
        hit = {"schedule": sch[0], "row": sch[1]}
        out = {"times": [x if x != float("inf") else None for x in t]}
        if cache:
            cache_store(cache, key, sch[0], out["times"], row=sch[1])
    if grid.d == 3:
        out["yzy"] = int(hit["schedule"])
    else:
        out["col"], out["row"] = int(hit["schedule"]), int(hit.get("row", 0))
    return out


def autotune(ctx: Context, grid, fp32=True, cache=None):
    """Tune the grid's passes (autotune_all) and return (column schedule, its candidate times in ms or None)
    for 2D, (y/z/y schedule, times or None) for 3D."""
    r = autotune_all(ctx, grid, fp32, cache)
    t = r["times"]
    if grid.d == 3:
        return r["yzy"], (None if t is None else [x for x in t[:2] if x is not None])
    return r["col"], (None if t is None else t[:N_COL_SCHED])


def set_schedule(ctx: Context, grid, sched, fp32=True, rows=False):
    """Install a schedule for the grid's FFT length and precision: 2D the column pass (0..N_COL_SCHED-1) or,
    with rows=True, the first row pass's values per thread (0, 8, 16); 3D the y/z/y passes (0, 1)."""
    g = _grid(grid)
    flags = (FP32_GRID if fp32 else 0) | (SCHED_ROWS if rows else 0)
    ctx.check(lib.gofd_set_schedule(ctx.handle, ctypes.byref(g), flags, int(sched)))


def time_kernel(ctx: Context, tr: Transfer, op: FdOp, which, u, flags=0, reps=20):
    """Average duration (ms) of one kernel of the K product, timed with HIP events on the library stream."""
    u = u.contiguous()
    nrhs = u.numel() // tr.nv
    ms = ctypes.c_double()
    ctx.check(lib.gofd_time_kernel(ctx.handle, tr.handle, op.handle, int(which), nrhs, _ptr(u), int(flags),
                                   int(reps), ctypes.byref(ms)))
    return ms.value
