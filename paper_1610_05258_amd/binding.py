"""Thin ctypes binding of libp2m.so (the C ABI in include/p2m.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory and the stream.  The
functions carry the names of the C entry points; they take torch tensors on the
context's device and return torch tensors plus a decoded report.

If libp2m.so is missing this module raises on first use: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import sys
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libp2m.so")

P2M_F32, P2M_F64 = 0, 1
DELTA, FLIP, PIC = 0, 1, 2
START_FLIP, START_ZERO, START_USER, START_LEARNED, START_DELTA1D = 0, 1, 2, 3, 4
FLAG_ORPHAN = 1 << 0
FLAG_NOT_CONVERGED = 1 << 1
FLAG_BREAKDOWN = 1 << 2
FLAG_RANGE = 1 << 3
FLAG_NONFINITE = 1 << 4
FLAG_LEARNED_FALLBACK = 1 << 5
FLAG_BIN_TIMEOUT = 1 << 6
FLAG_TRIANGULATION = 1 << 7
REPORT_BYTES = 144
MAX_FIELDS = 8
SOLVER_AUTO, SOLVER_STREAMING, SOLVER_RESIDENT, SOLVER_TILES, SOLVER_RESIDENT_CHEB = 0, 1, 2, 3, 4
OPT_SOLVER, OPT_PLANS, OPT_SCAN_SPIN, OPT_SOLVE_SPIN, OPT_FFT = 0, 1, 2, 3, 4

EXPORTS = ("p2m_status_string", "p2m_create", "p2m_destroy", "p2m_workspace_size", "p2m_bin",
           "p2m_assemble", "p2m_assign", "p2m_interpolate", "p2m_mass_assign", "p2m_mass_solve",
           "p2m_set_option", "p2m_batch_workspace_size", "p2m_mass_assign_batched",
           "p2m_set_learned", "p2m_learned_features", "p2m_learned_forward",
           "p2m_learned_workspace_size", "p2m_learned_train_step", "p2m_tune", "p2m_tune_batched",
           "p2m_plan_get", "p2m_plan_get_batched",
           "p2m_plan_save", "p2m_plan_load", "p2m_plan_clear", "p2m_mass_assign_noalloc",
           "p2m_x1d_workspace_size", "p2m_x1d_assign", "p2m_x1d_interpolate", "p2m_x1d_volumes",
           "p2m_x2d_workspace_size", "p2m_x2d_triangulation", "p2m_x2d_volumes", "p2m_x2d_assign",
           "p2m_x2d_interpolate", "p2m_x2d_round_trip",
           "p2m_ns_workspace_size", "p2m_ns_step")
QUAD_EXACT, QUAD_APPB = 0, 1
X1D_DELTA, X1D_FLIP, X1D_PIC, X1D_MASS, X1D_LUMPED = 0, 1, 2, 3, 4
X2D_MAXDEG = 32
NS_FLIP, NS_MASS = 0, 1
ERR_SCRATCH = 7
SCRATCH_BYTES = 64 << 20
LEARNED_KMAX, LEARNED_NIN, LEARNED_HIDDEN, LEARNED_NPARAM = 48, 160, 64, 18689


class P2MError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}")


class CProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("np", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("vol", ctypes.c_void_p)]


class CPlan(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int32), ("groups", ctypes.c_int32), ("scatter_tile", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("inner_rtol", ctypes.c_double), ("time_ms", ctypes.c_double)]

    def __repr__(self):
        return (f"CPlan(solver={self.solver}, groups={self.groups}, scatter_tile={self.scatter_tile}, "
                f"inner_rtol={self.inner_rtol:g}, time_ms={self.time_ms:.4f})")


class CSolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("maxit", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("start", ctypes.c_int32), ("reserved", ctypes.c_int32)]


assert ctypes.sizeof(CProblem) == 64 and ctypes.sizeof(CSolveOpts) == 32

_lib = None


def lib():
    """Open libp2m.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(or python -m paper_1610_05258_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        pprob = ctypes.POINTER(CProblem)
        L.p2m_status_string.restype = ctypes.c_char_p
        L.p2m_status_string.argtypes = [ctypes.c_int]
        L.p2m_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        L.p2m_destroy.argtypes = [vp]
        L.p2m_set_option.argtypes = [vp, i32, i32]
        L.p2m_workspace_size.argtypes = [vp, pprob, i32, ctypes.POINTER(sz)]
        L.p2m_bin.argtypes = [vp, pprob, vp, vp, vp, vp, sz, vp]
        L.p2m_assemble.argtypes = [vp, pprob, vp, i32, vp, vp, vp, vp, vp, sz, vp]
        L.p2m_assign.argtypes = [vp, pprob, ctypes.c_int, vp, i32, vp, vp, vp, sz, vp]
        L.p2m_interpolate.argtypes = [vp, pprob, vp, i32, vp, vp, vp, sz, vp]
        L.p2m_mass_assign.argtypes = [vp, pprob, vp, i32, ctypes.POINTER(CSolveOpts), vp, vp, vp,
                                      sz, vp]
        L.p2m_mass_solve.argtypes = [vp, pprob, i32, vp, vp, vp, ctypes.POINTER(CSolveOpts), vp, vp,
                                     vp, sz, vp]
        L.p2m_mass_assign_noalloc.argtypes = [vp, pprob, vp, i32, ctypes.POINTER(CSolveOpts), vp, vp, vp]
        L.p2m_x1d_workspace_size.argtypes = [vp, pprob, i32, ctypes.POINTER(sz)]
        L.p2m_x1d_assign.argtypes = [vp, pprob, i32, i32, vp, i32, ctypes.POINTER(CSolveOpts), vp, vp,
                                     vp, sz, vp]
        L.p2m_x1d_interpolate.argtypes = [vp, pprob, i32, i32, vp, i32, ctypes.POINTER(CSolveOpts), vp,
                                          vp, vp, sz, vp]
        L.p2m_x1d_volumes.argtypes = [vp, pprob, vp, vp, vp, sz, vp]
        L.p2m_x2d_workspace_size.argtypes = [vp, pprob, i32, ctypes.POINTER(sz)]
        L.p2m_x2d_triangulation.argtypes = [vp, pprob, vp, vp, vp, vp, vp, sz, vp]
        L.p2m_x2d_volumes.argtypes = [vp, pprob, vp, vp, vp, sz, vp]
        L.p2m_x2d_assign.argtypes = [vp, pprob, i32, vp, i32, ctypes.POINTER(CSolveOpts), vp, vp, vp,
                                     sz, vp]
        L.p2m_x2d_interpolate.argtypes = [vp, pprob, i32, vp, i32, ctypes.POINTER(CSolveOpts), vp, vp,
                                          vp, sz, vp]
        L.p2m_x2d_round_trip.argtypes = [vp, pprob, i32, i32, vp, i32, ctypes.POINTER(CSolveOpts), vp,
                                         vp, vp, vp, sz, vp]
        L.p2m_ns_workspace_size.argtypes = [vp, pprob, ctypes.POINTER(sz)]
        L.p2m_ns_step.argtypes = [vp, pprob, i32, ctypes.c_double, ctypes.c_double,
                                  ctypes.POINTER(CSolveOpts), vp, vp, vp, vp, vp, vp, sz, vp]
        L.p2m_batch_workspace_size.argtypes = [vp, pprob, i32, i32, ctypes.POINTER(sz)]
        L.p2m_mass_assign_batched.argtypes = [vp, pprob, i32, ctypes.POINTER(vp), i32,
                                              ctypes.POINTER(CSolveOpts), ctypes.POINTER(vp), vp, vp,
                                              sz, vp]
        fp = ctypes.POINTER(ctypes.c_float)
        L.p2m_set_learned.argtypes = [vp, vp]
        L.p2m_learned_features.argtypes = [vp, pprob, vp, i32, vp, i32, vp, vp, vp, vp, vp, sz, vp]
        L.p2m_learned_forward.argtypes = [vp, vp, vp, i32, vp, vp]
        L.p2m_learned_workspace_size.argtypes = [vp, i32, ctypes.POINTER(sz)]
        L.p2m_learned_train_step.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp, vp, vp, i32,
                                             vp, vp, i32, vp, sz, vp]
        del fp
        pplan = ctypes.POINTER(CPlan)
        L.p2m_tune.argtypes = [vp, pprob, vp, i32, ctypes.POINTER(CSolveOpts), vp, vp, vp, sz, vp, pplan]
        L.p2m_plan_get_batched.argtypes = [vp, pprob, i32, i32, pplan]
        L.p2m_tune_batched.argtypes = [vp, pprob, i32, ctypes.POINTER(vp), i32, ctypes.POINTER(CSolveOpts),
                                       ctypes.POINTER(vp), vp, vp, sz, vp, pplan]
        L.p2m_plan_get.argtypes = [vp, pprob, i32, pplan]
        L.p2m_plan_save.argtypes = [vp, ctypes.c_char_p]
        L.p2m_plan_load.argtypes = [vp, ctypes.c_char_p]
        L.p2m_plan_clear.argtypes = [vp]
        for name in EXPORTS[1:]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(s):
    return lib().p2m_status_string(int(s)).decode()


def _check(status, where):
    if status != 0:
        raise P2MError(status, where)


@dataclass
class Report:
    iters: np.ndarray
    refines: np.ndarray
    rel_residual: np.ndarray
    flags: int
    n_orphan: int
    n_invalid: int

    @staticmethod
    def decode(raw: bytes, nfields=MAX_FIELDS):
        a = np.frombuffer(raw, dtype=np.uint8)
        iters = a[0:32].view(np.int32)[:nfields].copy()
        refines = a[32:64].view(np.int32)[:nfields].copy()
        relres = a[64:128].view(np.float64)[:nfields].copy()
        tail = a[128:144].view(np.int32)
        return Report(iters, refines, relres, int(np.uint32(tail[0])), int(tail[1]), int(tail[2]))


@dataclass
class Particles:
    """One periodic P1 problem: mesh size, box and particle arrays on the device."""
    dim: int
    nx: int
    ny: int
    lx: float
    ly: float
    x: torch.Tensor
    y: torch.Tensor | None = None
    vol: torch.Tensor | None = None

    @property
    def n_nodes(self):
        return self.nx * (self.ny if self.dim == 2 else 1)

    @property
    def n_particles(self):
        return int(self.x.numel())

    @property
    def dtype(self):
        return self.x.dtype

    def cstruct(self):
        dt = self.x.dtype
        if dt not in (torch.float32, torch.float64):
            raise TypeError("positions must be float32 or float64")
        for t in (self.x, self.y, self.vol):
            if t is not None:
                if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() != self.x.numel():
                    raise TypeError("x, y, vol must be contiguous device tensors of one dtype and length")
        return CProblem(self.dim, self.nx, self.ny if self.dim == 2 else 1,
                        P2M_F64 if dt == torch.float64 else P2M_F32, float(self.lx),
                        float(self.ly if self.dim == 2 else 1.0), self.x.numel(),
                        self.x.data_ptr(),
                        self.y.data_ptr() if (self.dim == 2 and self.y is not None) else None,
                        self.vol.data_ptr() if self.vol is not None else None)


def particles_from(prob: dict, device="cuda", dtype=None) -> Particles:
    """Build a device problem from a dict of host arrays (keys dim, nx, ny, lx, ly, x, y, vol)."""
    def dev(a):
        if a is None:
            return None
        t = torch.as_tensor(np.ascontiguousarray(a))
        if dtype is not None:
            t = t.to(dtype)
        return t.to(device).contiguous()
    return Particles(prob["dim"], prob["nx"], prob.get("ny", 1), prob["lx"], prob.get("ly", 1.0),
                     dev(prob["x"]), dev(prob.get("y")) if prob["dim"] == 2 else None,
                     dev(prob.get("vol")))


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """A library context on one device plus a cached workspace."""

    def __init__(self, device=0):
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().p2m_create(ctypes.byref(h), int(device)), "p2m_create")
        self.handle = h
        self._ws = None

    def close(self):
        if self.handle:
            lib().p2m_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP call while the interpreter shuts down: the runtime (or a profiler
        # attached to it) may already be finalised; the process exit releases it
        # (the check is bound at definition: module globals may be gone by then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def set_solver(self, kind: int):
        """SOLVER_AUTO, SOLVER_STREAMING, SOLVER_RESIDENT, SOLVER_TILES or SOLVER_RESIDENT_CHEB."""
        _check(lib().p2m_set_option(self.handle, OPT_SOLVER, int(kind)), "p2m_set_option")

    def use_plans(self, on: bool):
        _check(lib().p2m_set_option(self.handle, OPT_PLANS, 1 if on else 0), "p2m_set_option")

    def set_scan_spin(self, value: int):
        """Bound of the binning scan's wait (0: default; < 0: end every wait at once)."""
        _check(lib().p2m_set_option(self.handle, OPT_SCAN_SPIN, int(value)), "p2m_set_option")

    def set_fft(self, on: bool):
        """Direct FFT solves of the circulant mesh systems where the sides allow (default)
        or always the iterative mass-matrix solver."""
        _check(lib().p2m_set_option(self.handle, OPT_FFT, 1 if on else 0), "p2m_set_option")

    def set_solve_spin(self, value: int):
        """Bound of a mass solve's grid-barrier wait (0: default; < 0: end every wait at once)."""
        _check(lib().p2m_set_option(self.handle, OPT_SOLVE_SPIN, int(value)), "p2m_set_option")

    def plan(self, prob, nfields):
        """The stored plan of the problem's shape class, or None."""
        p = CPlan()
        cp = prob.cstruct()
        st = lib().p2m_plan_get(self.handle, ctypes.byref(cp), int(nfields), ctypes.byref(p))
        return p if st == 0 else None

    def save_plans(self, path):
        _check(lib().p2m_plan_save(self.handle, str(path).encode()), "p2m_plan_save")

    def load_plans(self, path):
        _check(lib().p2m_plan_load(self.handle, str(path).encode()), "p2m_plan_load")

    def clear_plans(self):
        _check(lib().p2m_plan_clear(self.handle), "p2m_plan_clear")

    def workspace_size(self, prob: Particles, nfields: int) -> int:
        n = ctypes.c_size_t()
        cp = prob.cstruct()
        _check(lib().p2m_workspace_size(self.handle, ctypes.byref(cp), int(nfields), ctypes.byref(n)),
               "p2m_workspace_size")
        return int(n.value)

    def workspace(self, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def new_report(self):
        return torch.zeros(REPORT_BYTES, dtype=torch.uint8, device=f"cuda:{self.device}")


def read_report(rep: torch.Tensor, nfields=MAX_FIELDS) -> Report:
    return Report.decode(rep.cpu().numpy().tobytes(), nfields)


def _values_tensor(values, prob: Particles):
    if values.dim() == 1:
        values = values[None, :]
    if values.dtype != prob.dtype or not values.is_cuda or values.shape[1] != prob.n_particles:
        raise TypeError("values must be a [F, np] device tensor of the positions' dtype")
    F = values.shape[0]
    if not 1 <= F <= MAX_FIELDS:
        raise ValueError("1 <= F <= 8 fields")
    return values.contiguous(), F


def _ws_args(ctx, prob, F, ws):
    need = ctx.workspace_size(prob, F)
    w = ws if ws is not None else ctx.workspace(need)
    return ctypes.c_void_p(w.data_ptr()), ctypes.c_size_t(w.numel())


def p2m_bin(ctx: Context, prob: Particles, stream=None, ws=None, rep=None):
    """Stable binning: (perm [np] int32, cell_start [ncells+1] int32, report tensor)."""
    cp = prob.cstruct()
    perm = torch.empty(max(prob.n_particles, 1), dtype=torch.int32, device=prob.x.device)
    cs = torch.empty(prob.n_nodes + 1, dtype=torch.int32, device=prob.x.device)
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _ws_args(ctx, prob, 1, ws)
    _check(lib().p2m_bin(ctx.handle, ctypes.byref(cp), ctypes.c_void_p(perm.data_ptr()),
                         ctypes.c_void_p(cs.data_ptr()), ctypes.c_void_p(rep.data_ptr()), wp, wn,
                         _stream_ptr(stream)), "p2m_bin")
    return perm[: prob.n_particles], cs, rep


def p2m_assemble(ctx: Context, prob: Particles, values, want_coef=True, stream=None, ws=None, rep=None):
    """(b [F, nn], w [nn], coef [4 or 2, nn] or None, report tensor)."""
    values, F = _values_tensor(values, prob)
    cp = prob.cstruct()
    nn = prob.n_nodes
    dev = prob.x.device
    b = torch.empty((F, nn), dtype=prob.dtype, device=dev)
    w = torch.empty(nn, dtype=prob.dtype, device=dev)
    coef = torch.empty((4 if prob.dim == 2 else 2, nn), dtype=prob.dtype, device=dev) if want_coef else None
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _ws_args(ctx, prob, F, ws)
    _check(lib().p2m_assemble(ctx.handle, ctypes.byref(cp), ctypes.c_void_p(values.data_ptr()), F,
                              ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                              ctypes.c_void_p(coef.data_ptr()) if coef is not None else None,
                              ctypes.c_void_p(rep.data_ptr()), wp, wn, _stream_ptr(stream)),
           "p2m_assemble")
    return b, w, coef, rep


def p2m_assign(ctx: Context, prob: Particles, kind: int, values, stream=None, ws=None, rep=None, out=None):
    """Particle->mesh by DELTA (1D), FLIP or PIC: (nodal [F, nn], report tensor)."""
    values, F = _values_tensor(values, prob)
    cp = prob.cstruct()
    out = torch.empty((F, prob.n_nodes), dtype=prob.dtype, device=prob.x.device) if out is None else out
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _ws_args(ctx, prob, F, ws)
    _check(lib().p2m_assign(ctx.handle, ctypes.byref(cp), int(kind), ctypes.c_void_p(values.data_ptr()),
                            F, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(rep.data_ptr()), wp, wn,
                            _stream_ptr(stream)), "p2m_assign")
    return out, rep


def p2m_interpolate(ctx: Context, prob: Particles, nodal, stream=None, rep=None, out=None, ws=None):
    """Mesh->particle interpolation: (values [F, np], report tensor).  ws: optional device
    workspace (uint8 tensor) for the node-major path of 2D, 2-4 field gathers."""
    if nodal.dim() == 1:
        nodal = nodal[None, :]
    if nodal.dtype != prob.dtype or nodal.shape[1] != prob.n_nodes or not nodal.is_cuda:
        raise TypeError("nodal must be a [F, nnodes] device tensor of the positions' dtype")
    nodal = nodal.contiguous()
    F = nodal.shape[0]
    cp = prob.cstruct()
    out = torch.empty((F, prob.n_particles), dtype=prob.dtype, device=prob.x.device) if out is None else out
    rep = ctx.new_report() if rep is None else rep
    _check(lib().p2m_interpolate(ctx.handle, ctypes.byref(cp), ctypes.c_void_p(nodal.data_ptr()), F,
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(rep.data_ptr()),
                                 None if ws is None else ctypes.c_void_p(ws.data_ptr()),
                                 0 if ws is None else ws.numel(), _stream_ptr(stream)), "p2m_interpolate")
    return out, rep


def solve_opts(tol=1e-6, inner_rtol=None, maxit=1000, max_refine=8, start=START_FLIP, fp64=False):
    if inner_rtol is None:
        inner_rtol = 0.0 if fp64 else 1e-4
    return CSolveOpts(float(tol), float(inner_rtol), int(maxit), int(max_refine), int(start), 0)


def p2m_mass_assign(ctx: Context, prob: Particles, values, opts: CSolveOpts | None = None,
                    x0=None, stream=None, ws=None, rep=None, out=None):
    """Mass assignment: (nodal [F, nn], report tensor).  x0 is read when opts.start is USER."""
    values, F = _values_tensor(values, prob)
    cp = prob.cstruct()
    opts = opts if opts is not None else solve_opts(fp64=prob.dtype == torch.float64)
    if out is None:
        out = torch.empty((F, prob.n_nodes), dtype=prob.dtype, device=prob.x.device)
    if x0 is not None:
        out.copy_(x0)
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _ws_args(ctx, prob, F, ws)
    _check(lib().p2m_mass_assign(ctx.handle, ctypes.byref(cp), ctypes.c_void_p(values.data_ptr()), F,
                                 ctypes.byref(opts), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(rep.data_ptr()), wp, wn, _stream_ptr(stream)),
           "p2m_mass_assign")
    return out, rep


def p2m_mass_assign_noalloc(ctx: Context, prob: Particles, values, opts: CSolveOpts | None = None,
                            x0=None, stream=None, rep=None, out=None):
    """Mass assignment on the library's static device scratch (no workspace argument):
    (nodal [F, nn], report tensor).  Raises P2MError with ERR_SCRATCH when the problem
    needs more than SCRATCH_BYTES of workspace."""
    values, F = _values_tensor(values, prob)
    cp = prob.cstruct()
    opts = opts if opts is not None else solve_opts(fp64=prob.dtype == torch.float64)
    if out is None:
        out = torch.empty((F, prob.n_nodes), dtype=prob.dtype, device=prob.x.device)
    if x0 is not None:
        out.copy_(x0)
    rep = ctx.new_report() if rep is None else rep
    _check(lib().p2m_mass_assign_noalloc(ctx.handle, ctypes.byref(cp),
                                         ctypes.c_void_p(values.data_ptr()), F, ctypes.byref(opts),
                                         ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(rep.data_ptr()), _stream_ptr(stream)),
           "p2m_mass_assign_noalloc")
    return out, rep


# ----------------------------------------------------------------------------
# paper-exact 1D (FP64 1D problems; particle volumes from the sorted particles)
# ----------------------------------------------------------------------------
def x1d_workspace_size(ctx, prob, F):
    n = ctypes.c_size_t()
    cp = prob.cstruct()
    _check(lib().p2m_x1d_workspace_size(ctx.handle, ctypes.byref(cp), int(F), ctypes.byref(n)),
           "p2m_x1d_workspace_size")
    return int(n.value)


def _x1d_ws(ctx, prob, F, ws):
    if ws is None:
        ws = ctx.workspace(x1d_workspace_size(ctx, prob, F))
    return ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel())


def _opts_ptr(opts):
    return ctypes.byref(opts) if opts is not None else None


def p2m_x1d_assign(ctx: Context, prob: Particles, kind: int, quad: int, values, opts=None,
                   stream=None, ws=None, rep=None, out=None):
    """Paper-exact 1D particle->mesh of kind X1D_* with QUAD_EXACT / QUAD_APPB integrals:
    (nodal [F, nx] FP64, report tensor)."""
    values, F = _values_tensor(values, prob)
    cp = prob.cstruct()
    if out is None:
        out = torch.empty((F, prob.n_nodes), dtype=torch.float64, device=prob.x.device)
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _x1d_ws(ctx, prob, F, ws)
    _check(lib().p2m_x1d_assign(ctx.handle, ctypes.byref(cp), int(kind), int(quad),
                                ctypes.c_void_p(values.data_ptr()), F, _opts_ptr(opts),
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(rep.data_ptr()),
                                wp, wn, _stream_ptr(stream)), "p2m_x1d_assign")
    return out, rep


def p2m_x1d_interpolate(ctx: Context, prob: Particles, kind: int, quad: int, nodal, opts=None,
                        stream=None, ws=None, rep=None, out=None):
    """Paper-exact 1D mesh->particle of kind X1D_DELTA / X1D_MASS / X1D_LUMPED:
    (values [F, np] FP64 in caller order, report tensor)."""
    nodal = nodal.contiguous()
    F = int(nodal.shape[0])
    cp = prob.cstruct()
    if out is None:
        out = torch.empty((F, prob.n_particles), dtype=torch.float64, device=prob.x.device)
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _x1d_ws(ctx, prob, F, ws)
    _check(lib().p2m_x1d_interpolate(ctx.handle, ctypes.byref(cp), int(kind), int(quad),
                                     ctypes.c_void_p(nodal.data_ptr()), F, _opts_ptr(opts),
                                     ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(rep.data_ptr()),
                                     wp, wn, _stream_ptr(stream)), "p2m_x1d_interpolate")
    return out, rep


def p2m_x1d_volumes(ctx: Context, prob: Particles, stream=None, ws=None, rep=None):
    """Particle volumes of eq. (4) in caller order (FP64)."""
    cp = prob.cstruct()
    out = torch.empty(prob.n_particles, dtype=torch.float64, device=prob.x.device)
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _x1d_ws(ctx, prob, 1, ws)
    _check(lib().p2m_x1d_volumes(ctx.handle, ctypes.byref(cp), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(rep.data_ptr()), wp, wn, _stream_ptr(stream)),
           "p2m_x1d_volumes")
    return out


def x2d_workspace_size(ctx, prob, F):
    n = ctypes.c_size_t()
    cp = prob.cstruct()
    _check(lib().p2m_x2d_workspace_size(ctx.handle, ctypes.byref(cp), int(F), ctypes.byref(n)),
           "p2m_x2d_workspace_size")
    return int(n.value)


def _x2d_ws(ctx, prob, F, ws):
    if ws is None:
        ws = ctx.workspace(x2d_workspace_size(ctx, prob, F))
    return ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel())


def p2m_x2d_triangulation(ctx: Context, prob: Particles, stream=None, ws=None, rep=None):
    """Periodic Delaunay triangulation of the particles: (deg [np], nbr [np, X2D_MAXDEG],
    shift [np, X2D_MAXDEG] packed (sx + 128) | (sy + 128) << 8, report tensor), int32."""
    cp = prob.cstruct()
    dev = prob.x.device
    deg = torch.empty(prob.n_particles, dtype=torch.int32, device=dev)
    nbr = torch.empty((prob.n_particles, X2D_MAXDEG), dtype=torch.int32, device=dev)
    sh = torch.empty((prob.n_particles, X2D_MAXDEG), dtype=torch.int32, device=dev)
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _x2d_ws(ctx, prob, 1, ws)
    _check(lib().p2m_x2d_triangulation(ctx.handle, ctypes.byref(cp), ctypes.c_void_p(deg.data_ptr()),
                                       ctypes.c_void_p(nbr.data_ptr()), ctypes.c_void_p(sh.data_ptr()),
                                       ctypes.c_void_p(rep.data_ptr()), wp, wn, _stream_ptr(stream)),
           "p2m_x2d_triangulation")
    return deg, nbr, sh, rep


def p2m_x2d_volumes(ctx: Context, prob: Particles, stream=None, ws=None, rep=None):
    """Particle volumes int psi_mu on the particle triangulation, caller order (FP64)."""
    cp = prob.cstruct()
    out = torch.empty(prob.n_particles, dtype=torch.float64, device=prob.x.device)
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _x2d_ws(ctx, prob, 1, ws)
    _check(lib().p2m_x2d_volumes(ctx.handle, ctypes.byref(cp), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(rep.data_ptr()), wp, wn, _stream_ptr(stream)),
           "p2m_x2d_volumes")
    return out, rep


def p2m_x2d_assign(ctx: Context, prob: Particles, kind: int, values, opts=None, stream=None,
                   ws=None, rep=None, out=None):
    """Paper-exact 2D particle->mesh of kind X1D_* (the same kinds): (nodal [F, nn] FP64,
    report tensor)."""
    values, F = _values_tensor(values, prob)
    cp = prob.cstruct()
    if out is None:
        out = torch.empty((F, prob.n_nodes), dtype=torch.float64, device=prob.x.device)
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _x2d_ws(ctx, prob, F, ws)
    _check(lib().p2m_x2d_assign(ctx.handle, ctypes.byref(cp), int(kind),
                                ctypes.c_void_p(values.data_ptr()), F, _opts_ptr(opts),
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(rep.data_ptr()),
                                wp, wn, _stream_ptr(stream)), "p2m_x2d_assign")
    return out, rep


def p2m_x2d_interpolate(ctx: Context, prob: Particles, kind: int, nodal, opts=None, stream=None,
                        ws=None, rep=None, out=None):
    """Paper-exact 2D mesh->particle of kind X1D_DELTA / X1D_MASS / X1D_LUMPED:
    (values [F, np] FP64 in caller order, report tensor)."""
    nodal = nodal.contiguous()
    F = int(nodal.shape[0])
    cp = prob.cstruct()
    if out is None:
        out = torch.empty((F, prob.n_particles), dtype=torch.float64, device=prob.x.device)
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _x2d_ws(ctx, prob, F, ws)
    _check(lib().p2m_x2d_interpolate(ctx.handle, ctypes.byref(cp), int(kind),
                                     ctypes.c_void_p(nodal.data_ptr()), F, _opts_ptr(opts),
                                     ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(rep.data_ptr()),
                                     wp, wn, _stream_ptr(stream)), "p2m_x2d_interpolate")
    return out, rep


def p2m_x2d_round_trip(ctx: Context, prob: Particles, kind_p2m: int, kind_m2p: int, values,
                       opts=None, stream=None, ws=None, reps=None, nodal=None, out=None):
    """Paper-exact 2D P2M of kind_p2m then M2P of kind_m2p at one set of positions, one
    binning and triangulation: (nodal [F, nn], values [F, np], reports [2, REPORT_BYTES])."""
    values, F = _values_tensor(values, prob)
    cp = prob.cstruct()
    dev = prob.x.device
    if nodal is None:
        nodal = torch.empty((F, prob.n_nodes), dtype=torch.float64, device=dev)
    if out is None:
        out = torch.empty((F, prob.n_particles), dtype=torch.float64, device=dev)
    if reps is None:
        reps = torch.zeros((2, REPORT_BYTES), dtype=torch.uint8, device=dev)
    wp, wn = _x2d_ws(ctx, prob, F, ws)
    _check(lib().p2m_x2d_round_trip(ctx.handle, ctypes.byref(cp), int(kind_p2m), int(kind_m2p),
                                    ctypes.c_void_p(values.data_ptr()), F, _opts_ptr(opts),
                                    ctypes.c_void_p(nodal.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(reps.data_ptr()), wp, wn, _stream_ptr(stream)),
           "p2m_x2d_round_trip")
    return nodal, out, reps


def ns_workspace_size(ctx: Context, prob: Particles) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().p2m_ns_workspace_size(ctx.handle, ctypes.byref(prob.cstruct()), ctypes.byref(n)),
           "p2m_ns_workspace_size")
    return int(n.value)


def p2m_ns_step(ctx: Context, prob: Particles, vel, assign: int, dt: float, nu: float,
                opts: CSolveOpts | None = None, x_out=None, y_out=None, mesh_vel=None, reps=None,
                stream=None, ws=None):
    """One step of the particle fluid solver (p2m_ns_step).  vel [2, np] (FP32, device) is
    updated in place; the advected positions go to x_out, y_out (default: prob.x, prob.y,
    in place).  Returns (mesh velocity [2, nn] or None, reports [3, REPORT_BYTES])."""
    if vel.dtype != torch.float32 or not vel.is_cuda or not vel.is_contiguous():
        raise TypeError("vel must be a contiguous FP32 device tensor [2, np]")
    cp = prob.cstruct()
    opts = opts if opts is not None else solve_opts()
    x_out = prob.x if x_out is None else x_out
    y_out = prob.y if y_out is None else y_out
    reps = torch.zeros((3, REPORT_BYTES), dtype=torch.uint8, device=vel.device) if reps is None else reps
    if ws is None:
        ws = ctx.workspace(ns_workspace_size(ctx, prob))
    mv = ctypes.c_void_p(mesh_vel.data_ptr()) if mesh_vel is not None else None
    _check(lib().p2m_ns_step(ctx.handle, ctypes.byref(cp), int(assign), float(dt), float(nu),
                             ctypes.byref(opts), ctypes.c_void_p(vel.data_ptr()),
                             ctypes.c_void_p(x_out.data_ptr()), ctypes.c_void_p(y_out.data_ptr()), mv,
                             ctypes.c_void_p(reps.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                             ctypes.c_size_t(ws.numel()), _stream_ptr(stream)), "p2m_ns_step")
    return mesh_vel, reps


def p2m_mass_solve(ctx: Context, prob: Particles, b, w, coef, opts: CSolveOpts | None = None,
                   x0=None, stream=None, ws=None, rep=None, out=None):
    """Solve step alone on a system from p2m_assemble (b and coef are modified in place:
    orphan rows become identity rows).  Returns (nodal [F, nn], report tensor)."""
    F = b.shape[0]
    for t in (b, w, coef):
        if t.dtype != prob.dtype or not t.is_cuda or not t.is_contiguous():
            raise TypeError("b, w, coef must be contiguous device tensors of the positions' dtype")
    cp = prob.cstruct()
    opts = opts if opts is not None else solve_opts(fp64=prob.dtype == torch.float64)
    if out is None:
        out = torch.empty((F, prob.n_nodes), dtype=prob.dtype, device=prob.x.device)
    if x0 is not None:
        out.copy_(x0)
    rep = ctx.new_report() if rep is None else rep
    wp, wn = _ws_args(ctx, prob, F, ws)
    _check(lib().p2m_mass_solve(ctx.handle, ctypes.byref(cp), F, ctypes.c_void_p(b.data_ptr()),
                                ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(coef.data_ptr()),
                                ctypes.byref(opts), ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(rep.data_ptr()), wp, wn, _stream_ptr(stream)),
           "p2m_mass_solve")
    return out, rep


class Batch:
    """A batch of independent 2D FP32 problems for p2m_mass_assign_batched, with its
    value tensors, outputs ([F, nn_k] each), reports ([nprob] x 144 bytes) and
    workspace.  Every run() passes the same instance table, so after the first call
    the library relaunches its cached graph."""

    def __init__(self, ctx: Context, probs, values, opts: CSolveOpts | None = None):
        if len(probs) != len(values) or not probs:
            raise ValueError("one value tensor per problem")
        self.ctx = ctx
        self.probs = list(probs)
        self.values = []
        F = None
        for p, v in zip(self.probs, values):
            v, f = _values_tensor(v, p)
            if F is not None and f != F:
                raise ValueError("every instance needs the same field count")
            F = f
            self.values.append(v)
        self.F = F
        self.n = len(self.probs)
        self.opts = opts if opts is not None else solve_opts()
        dev = f"cuda:{ctx.device}"
        self.out = [torch.empty((F, p.n_nodes), dtype=torch.float32, device=dev) for p in self.probs]
        self.reps = torch.zeros((self.n, REPORT_BYTES), dtype=torch.uint8, device=dev)
        self._cprobs = (CProblem * self.n)(*[p.cstruct() for p in self.probs])
        self._vptr = (ctypes.c_void_p * self.n)(*[v.data_ptr() for v in self.values])
        self._optr = (ctypes.c_void_p * self.n)(*[o.data_ptr() for o in self.out])
        nb = ctypes.c_size_t()
        _check(lib().p2m_batch_workspace_size(ctx.handle, self._cprobs, self.n, F, ctypes.byref(nb)),
               "p2m_batch_workspace_size")
        self.ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=dev)

    def run(self, stream=None):
        _check(lib().p2m_mass_assign_batched(
            self.ctx.handle, self._cprobs, self.n, self._vptr, self.F, ctypes.byref(self.opts),
            self._optr, ctypes.c_void_p(self.reps.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
            ctypes.c_size_t(self.ws.numel()), _stream_ptr(stream)), "p2m_mass_assign_batched")
        return self.out

    def tune(self, stream=None):
        """Time the batch under each inner_rtol candidate and keep the fastest plan for
        its shape class (applied by later run() calls while plans are on)."""
        plan = CPlan()
        _check(lib().p2m_tune_batched(
            self.ctx.handle, self._cprobs, self.n, self._vptr, self.F, ctypes.byref(self.opts),
            self._optr, ctypes.c_void_p(self.reps.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
            ctypes.c_size_t(self.ws.numel()), _stream_ptr(stream), ctypes.byref(plan)),
            "p2m_tune_batched")
        return plan

    def plan(self):
        """The stored plan of this batch's shape class, or None."""
        p = CPlan()
        st = lib().p2m_plan_get_batched(self.ctx.handle, self._cprobs, self.n, self.F, ctypes.byref(p))
        return p if st == 0 else None

    def reports(self):
        raw = self.reps.cpu().numpy()
        return [Report.decode(raw[k].tobytes(), self.F) for k in range(self.n)]


def p2m_mass_assign_batched(ctx: Context, probs, values, opts: CSolveOpts | None = None, x0=None,
                            stream=None):
    """Mass assignment of a batch in one graph launch: (list of nodal [F, nn_k], Batch).
    x0 (a list) is read when opts.start is USER."""
    b = Batch(ctx, probs, values, opts)
    if x0 is not None:
        for o, x in zip(b.out, x0):
            o.copy_(x)
    b.run(stream)
    return b.out, b


# ----------------------------------------------------------------------------
# learned warm start
# ----------------------------------------------------------------------------
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def set_learned(ctx: Context, params):
    """Parameters (FP32 device tensor of LEARNED_NPARAM) for START_LEARNED, or None."""
    if params is not None:
        if params.dtype != torch.float32 or not params.is_cuda or params.numel() != LEARNED_NPARAM:
            raise TypeError("params must be a float32 device tensor of LEARNED_NPARAM entries")
        params = params.contiguous()
    ctx._learned = params
    _check(lib().p2m_set_learned(ctx.handle, _ptr(params)), "p2m_set_learned")


def learned_features(ctx: Context, prob: Particles, values, nodes=None, stream=None, ws=None):
    """Feature rows of the nodes (all when None): X [nrows, F, 160] bfloat16, base and
    scale [nrows, F] (scale 0 = node not usable)."""
    values, F = _values_tensor(values, prob)
    dev = prob.x.device
    nrows = prob.n_nodes if nodes is None else int(nodes.numel())
    if nodes is not None:
        nodes = nodes.to(device=dev, dtype=torch.int32).contiguous()
    X = torch.empty((nrows, F, LEARNED_NIN), dtype=torch.bfloat16, device=dev)
    base = torch.empty((nrows, F), dtype=torch.float32, device=dev)
    scale = torch.empty((nrows, F), dtype=torch.float32, device=dev)
    rep = ctx.new_report()
    cp = prob.cstruct()
    wp, wn = _ws_args(ctx, prob, F, ws)
    _check(lib().p2m_learned_features(ctx.handle, ctypes.byref(cp), _ptr(values), F, _ptr(nodes),
                                      nrows, _ptr(X), _ptr(base), _ptr(scale), _ptr(rep), wp, wn,
                                      _stream_ptr(stream)), "p2m_learned_features")
    return X, base, scale


def learned_forward(ctx: Context, params, X, stream=None):
    """Network outputs of rows X [n, 160] (bfloat16)."""
    X = X.reshape(-1, LEARNED_NIN).contiguous()
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(lib().p2m_learned_forward(ctx.handle, _ptr(params), _ptr(X), X.shape[0], _ptr(y),
                                     _stream_ptr(stream)), "p2m_learned_forward")
    return y


class Trainer:
    """Adam state and workspace for p2m_learned_train_step on one feature table."""

    def __init__(self, ctx: Context, params, batch):
        self.ctx = ctx
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step = 0
        self.batch = int(batch)
        n = ctypes.c_size_t()
        _check(lib().p2m_learned_workspace_size(ctx.handle, self.batch, ctypes.byref(n)),
               "p2m_learned_workspace_size")
        self.ws = torch.empty(int(n.value), dtype=torch.uint8, device=params.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)

    def run(self, X, target, rows, lr=1e-3, apply=True, grad=None, stream=None):
        """One step on rows of X [N, 160] with targets [N]; returns the loss tensor."""
        if rows.numel() > self.batch:
            raise ValueError("more rows than the batch size")
        if apply:
            self.step += 1
        _check(lib().p2m_learned_train_step(
            self.ctx.handle, _ptr(self.params), _ptr(self.m), _ptr(self.v), max(self.step, 1),
            float(lr), _ptr(X), _ptr(target), _ptr(rows), int(rows.numel()), _ptr(self.loss),
            _ptr(grad), 1 if apply else 0, _ptr(self.ws), ctypes.c_size_t(self.ws.numel()),
            _stream_ptr(stream)), "p2m_learned_train_step")
        return self.loss


def p2m_tune(ctx: Context, prob: Particles, values, opts: CSolveOpts | None = None, stream=None):
    """Time every applicable plan on this problem, keep the fastest for its shape class.
    Returns (plan, nodal [F, nn] of the chosen plan, report tensor)."""
    values, F = _values_tensor(values, prob)
    cp = prob.cstruct()
    opts = opts if opts is not None else solve_opts(fp64=prob.dtype == torch.float64)
    out = torch.empty((F, prob.n_nodes), dtype=prob.dtype, device=prob.x.device)
    rep = ctx.new_report()
    wp, wn = _ws_args(ctx, prob, F, None)
    plan = CPlan()
    _check(lib().p2m_tune(ctx.handle, ctypes.byref(cp), _ptr(values), F, ctypes.byref(opts), _ptr(out),
                          _ptr(rep), wp, wn, _stream_ptr(stream), ctypes.byref(plan)), "p2m_tune")
    return plan, out, rep
