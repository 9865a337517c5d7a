"""Python binding of libnfa (ctypes).

Argument marshalling only: every step of the projection runs in the HIP
library.  torch supplies device memory (tensors) and the stream (the current
torch stream).  If the library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnfa.so")

NFA_OK = 0
NFA_NOT_CONVERGED = 1
NFA_F64, NFA_F32, NFA_BF16 = 0, 1, 2
NFA_PROF_MG_DOWN, NFA_PROF_MG_UP = 2, 3
NFA_PROF_F32_FLEX, NFA_PROF_UNET = 4, 5
NFA_PROF_F64_X2, NFA_PROF_F32_X2 = 6, 7
NFA_PC_JACOBI, NFA_PC_UNET, NFA_PC_TEST_SABOTAGE, NFA_PC_JACOBI_FCG, NFA_PC_MG = 1, 2, 3, 4, 5
NFA_PREC_F64, NFA_PREC_MIXED = 0, 1

EXPORT = {
    "frac_x": 1, "frac_y": 2, "frac_z": 3, "vfrac": 4, "open_x": 5, "open_y": 6, "open_z": 7,
    "active": 8, "root": 9, "reduced": 10,
    "rho": 20, "tx": 21, "ty": 22, "tz": 23, "dinv": 24, "tx32": 25, "ty32": 26, "tz32": 27,
    "dinv32": 28,
}


class NFAError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (python -m paper_1410_1937_amd.build)")
    return ctypes.CDLL(LIB_PATH)


lib = _load()

c_void_p, c_int, c_double, c_ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong


class GridInfo(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int), ("cells", c_ll), ("active", c_ll),
                ("reduced", c_ll), ("groups", c_int), ("slaves", c_int), ("all_neumann", c_int)]


class AssembleParams(ctypes.Structure):
    _fields_ = [("rho_liquid", c_double), ("rho_gas", c_double), ("smooth", c_int),
                ("phi_dtype", c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("max_iters", c_int), ("precond", c_int), ("precision", c_int),
                ("replace_drop", c_double), ("fcg_m", c_int),
                ("fallback_ratio", c_double), ("fallback_window", c_int), ("warm_start", c_int),
                ("check_every", c_int), ("unet", c_void_p), ("history", ctypes.POINTER(c_double)),
                ("history_cap", c_int), ("mg", c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", c_int), ("outer", c_int), ("fallback", c_int),
                ("history_len", c_int), ("relres", c_double), ("ms", c_double)]


class RK2Params(ctypes.Structure):
    _fields_ = [("dt", c_double), ("body_vel", c_double * 3), ("rho", AssembleParams)]


class KernelStats(ctypes.Structure):
    _fields_ = [("launches", c_ll), ("ms", c_double), ("cells", c_ll)]


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("nfa_last_error", ctypes.c_char_p, [])
_sig("nfa_version", c_int, [])
_sig("nfa_stream_copy", c_int, [c_void_p, c_void_p, ctypes.c_size_t, c_void_p])
_sig("nfa_stream_fill", c_int, [c_void_p, ctypes.c_uint, ctypes.c_size_t, c_void_p])
_sig("nfa_grid_create", c_int, [c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                ctypes.POINTER(c_void_p)])
_sig("nfa_grid_set_body", c_int, [c_void_p, c_void_p, c_double, c_int, c_void_p])
_sig("nfa_grid_get_info", c_int, [c_void_p, ctypes.POINTER(GridInfo)])
_sig("nfa_grid_export", c_int, [c_void_p, c_int, c_void_p, c_void_p])
_sig("nfa_grid_destroy", None, [c_void_p])
_sig("nfa_poisson_create", c_int, [c_void_p, c_void_p, ctypes.c_size_t, ctypes.POINTER(c_void_p)])
_sig("nfa_poisson_workspace_bytes", ctypes.c_size_t, [c_void_p])
_sig("nfa_poisson_assemble", c_int, [c_void_p, c_void_p, ctypes.POINTER(AssembleParams), c_void_p])
_sig("nfa_poisson_apply", c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p])
_sig("nfa_poisson_rhs", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                                c_void_p, c_void_p])
_sig("nfa_poisson_project", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                    c_void_p, c_void_p, c_void_p, c_void_p])
_sig("nfa_poisson_divergence", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_void_p])
_sig("nfa_solve_opts_default", None, [ctypes.POINTER(SolveOpts)])
_sig("nfa_poisson_solve", c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveOpts),
                                  c_void_p, ctypes.POINTER(SolveInfo)])
_sig("nfa_poisson_export", c_int, [c_void_p, c_int, c_void_p, c_void_p])
_sig("nfa_poisson_destroy", None, [c_void_p])
_sig("nfa_poisson_profile", c_int, [c_void_p, c_int])
_sig("nfa_poisson_residual", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double), c_void_p])
_sig("nfa_unet_create", c_int, [c_int, c_int, c_int, c_int, c_int, c_void_p, ctypes.c_size_t,
                                ctypes.POINTER(c_void_p)])
_sig("nfa_unet_workspace_bytes", ctypes.c_size_t, [c_int, c_int, c_int, c_int])
_sig("nfa_unet_bind", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int])
_sig("nfa_unet_param_count", c_ll, [c_int])
_sig("nfa_unet_levels", c_int, [c_void_p])
_sig("nfa_unet_get_params", c_int, [c_void_p, c_void_p])
_sig("nfa_unet_set_params", c_int, [c_void_p, c_void_p])
_sig("nfa_unet_get_grads", c_int, [c_void_p, c_void_p])
_sig("nfa_unet_forward", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p])
_sig("nfa_unet_grad", c_int, [c_void_p, c_void_p, c_void_p, c_double, ctypes.POINTER(c_double), c_void_p])
_sig("nfa_unet_train_step", c_int, [c_void_p, c_void_p, c_void_p, c_double, ctypes.c_float, c_int,
                                    ctypes.POINTER(c_double), c_void_p])
_sig("nfa_unet_backward", c_int, [c_void_p, c_void_p, c_void_p, c_void_p])
_sig("nfa_unet_adam_step", c_int, [c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, c_int,
                                   c_void_p])
_sig("nfa_unet_export", c_int, [c_void_p, c_int, c_void_p, c_void_p])
_sig("nfa_unet_destroy", None, [c_void_p])
_sig("nfa_poisson_profile_read", c_int, [c_void_p, c_int, ctypes.POINTER(KernelStats)])
_sig("nfa_poisson_velocity", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double,
                                     c_void_p, c_void_p, c_void_p, c_void_p])
_sig("nfa_faces_combine", c_int, [c_ll, c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p])
_sig("nfa_poisson_rhs_cells", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p])
_sig("nfa_exit_velocity", c_int, [c_void_p, c_void_p, c_double, c_double, c_void_p, c_void_p])
_sig("nfa_mg_create", c_int, [c_void_p, ctypes.POINTER(c_void_p)])
_sig("nfa_mg_destroy", None, [c_void_p])
_sig("nfa_mg_setup", c_int, [c_void_p, c_void_p])
_sig("nfa_mg_apply", c_int, [c_void_p, c_void_p, c_void_p, c_void_p])
_sig("nfa_mg_info", c_int, [c_void_p, ctypes.POINTER(c_int), c_void_p])
_sig("nfa_mg_set_tail", c_int, [c_void_p, c_int])
_sig("nfa_mg_set_params", c_int, [c_void_p, c_double, c_double])
_sig("nfa_mg_set_coef", c_int, [c_void_p, c_int])
_sig("nfa_mg_side_rows", c_int, [c_void_p, c_int, ctypes.POINTER(c_int)])
_sig("nfa_mg_export", c_int, [c_void_p, c_int, c_void_p, c_void_p])
_sig("nfa_stretch_axis", c_int, [c_double, c_double, c_int, c_int, c_void_p, c_void_p, c_double, c_int, c_void_p,
                                 ctypes.POINTER(c_int)])
_sig("nfa_panels_psi", c_int, [c_void_p, c_void_p, c_ll, c_void_p, c_void_p])
_sig("nfa_panels_psi_noalloc", c_int, [c_void_p, c_void_p, c_ll, c_void_p, c_void_p])
_sig("nfa_vof_create", c_int, [c_void_p, ctypes.POINTER(c_void_p)])
_sig("nfa_vof_destroy", None, [c_void_p])
_sig("nfa_vof_sweep", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int, c_int,
                              c_void_p, c_void_p])
_sig("nfa_vof_advect", c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int, c_void_p,
                               c_void_p])
_sig("nfa_rk2_cycle", c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(RK2Params),
                              ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                              ctypes.POINTER(c_void_p), c_void_p, c_void_p, ctypes.POINTER(c_void_p),
                              ctypes.POINTER(SolveOpts), c_void_p, ctypes.POINTER(SolveInfo)])


def faces_combine(a, b, s, c, out=None):
    """out = (a + b) + s c, or a + s c when b is None (nfa_faces_combine)."""
    out = torch.empty_like(a) if out is None else out
    n = a.numel()
    for name, t in (("a", a), ("c", c), ("out", out)) + ((("b", b),) if b is not None else ()):
        _dev(t, torch.float64, a.shape, name)
    _check(lib.nfa_faces_combine(n, c_void_p(a.data_ptr()), None if b is None else c_void_p(b.data_ptr()),
                                 s, c_void_p(c.data_ptr()), c_void_p(out.data_ptr()), _stream()),
           "nfa_faces_combine")
    return out


def stream_copy(dst, src):
    """dst = src (same-size contiguous device tensors, 16-byte aligned) with
    the library's plain streaming copy (nfa_stream_copy); on the current
    stream."""
    if not (isinstance(dst, torch.Tensor) and isinstance(src, torch.Tensor) and dst.is_cuda and src.is_cuda):
        raise TypeError("dst and src must be CUDA (HIP) tensors")
    if not (dst.is_contiguous() and src.is_contiguous()):
        raise TypeError("dst and src must be contiguous")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src differ in size")
    _check(lib.nfa_stream_copy(c_void_p(dst.data_ptr()), c_void_p(src.data_ptr()), nbytes, _stream()),
           "nfa_stream_copy")
    return dst


def stream_fill(dst, value=0):
    """Every 32-bit word of dst (a contiguous device tensor, 16-byte aligned)
    set to the unsigned `value` with the library's plain streaming write
    (nfa_stream_fill); on the current stream."""
    if not (isinstance(dst, torch.Tensor) and dst.is_cuda):
        raise TypeError("dst must be a CUDA (HIP) tensor")
    if not dst.is_contiguous():
        raise TypeError("dst must be contiguous")
    nbytes = dst.numel() * dst.element_size()
    _check(lib.nfa_stream_fill(c_void_p(dst.data_ptr()), int(value) & 0xFFFFFFFF, nbytes, _stream()),
           "nfa_stream_fill")
    return dst


def stretch_axis(a, b, n, levels, zones=(), tol=1e-13, max_iter=500):
    """Nodes of one stretched axis and the sweeps taken (nfa_stretch_axis);
    zones is a sequence of (x0, x1) transitions between consecutive levels.
    Raises if the iteration did not converge."""
    lv = np.ascontiguousarray(levels, dtype=np.float64)
    zn = np.ascontiguousarray(np.asarray(zones, dtype=np.float64).reshape(-1))
    if len(lv) != len(zn) // 2 + 1:
        raise ValueError("need one more level than transition zones")
    out = np.empty(n + 1)
    it = c_int()
    st = lib.nfa_stretch_axis(a, b, n, len(zn) // 2, lv.ctypes.data, zn.ctypes.data if len(zn) else None, tol,
                              max_iter, out.ctypes.data, ctypes.byref(it))
    _check(st, "nfa_stretch_axis")
    if st != 0:
        raise NFAError(f"nfa_stretch_axis did not converge in {it.value} sweeps")
    return out, it.value


def _check(st, what):
    if st < 0:
        msg = lib.nfa_last_error().decode()
        raise NFAError(f"{what} failed ({st}): {msg}")
    return st


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, shape=None, name="array"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Grid:
    """Stretched cartesian grid with an optional immersed body."""

    def __init__(self, xf, yf, zf, bc):
        xf, yf, zf = (np.ascontiguousarray(a, dtype=np.float64) for a in (xf, yf, zf))
        bc = np.ascontiguousarray(bc, dtype=np.int32)
        h = c_void_p()
        _check(lib.nfa_grid_create(len(xf) - 1, len(yf) - 1, len(zf) - 1, xf.ctypes.data,
                                   yf.ctypes.data, zf.ctypes.data, bc.ctypes.data, ctypes.byref(h)),
               "nfa_grid_create")
        self.h = h
        self.nx, self.ny, self.nz = len(xf) - 1, len(yf) - 1, len(zf) - 1
        self.shape = (self.nz, self.ny, self.nx)

    def set_body(self, psi, theta=0.25, samples=8):
        ptr = None if psi is None else _dev(psi, torch.float64,
                                             (self.nz + 1, self.ny + 1, self.nx + 1), "psi")
        _check(lib.nfa_grid_set_body(self.h, ptr, theta, samples, _stream()), "nfa_grid_set_body")

    def panels_psi(self, panels, out=None, noalloc=False):
        """Signed distance of a triangulated body at the nodes (nfa_panels_psi,
        or nfa_panels_psi_noalloc when noalloc: no device allocation, at most
        65536 panels); panels: (m, 3, 3) FP64 device tensor."""
        if panels.ndim != 3 or tuple(panels.shape[1:]) != (3, 3):
            raise ValueError("panels must have shape (m, 3, 3)")
        shape = (self.nz + 1, self.ny + 1, self.nx + 1)
        out = torch.empty(shape, dtype=torch.float64, device=panels.device) if out is None else out
        name = "nfa_panels_psi_noalloc" if noalloc else "nfa_panels_psi"
        _check(getattr(lib, name)(self.h, _dev(panels, torch.float64, None, "panels"), panels.shape[0],
                                  _dev(out, torch.float64, shape, "psi"), _stream()), name)
        return out

    def exit_velocity(self, uk_x, uc, dt, ut_x=None):
        """Exit-plane x-velocity of the radiation condition (nfa_exit_velocity);
        writes the +x boundary plane of ut_x (a copy of uk_x when not given)."""
        sh = self.face_shape(0)
        ut = uk_x.clone() if ut_x is None else ut_x
        _check(lib.nfa_exit_velocity(self.h, _dev(uk_x, torch.float64, sh, "uk_x"), uc, dt,
                                     _dev(ut, torch.float64, sh, "ut_x"), _stream()), "nfa_exit_velocity")
        return ut

    def info(self):
        gi = GridInfo()
        _check(lib.nfa_grid_get_info(self.h, ctypes.byref(gi)), "nfa_grid_get_info")
        return {f: getattr(gi, f) for f, _ in GridInfo._fields_}

    def face_shape(self, axis):
        nz, ny, nx = self.shape
        return [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)][axis]

    def export(self, what):
        code = EXPORT[what]
        shape = {1: self.face_shape(0), 2: self.face_shape(1), 3: self.face_shape(2),
                 5: self.face_shape(0), 6: self.face_shape(1), 7: self.face_shape(2)}.get(code, self.shape)
        dtype = {8: torch.uint8, 9: torch.int32, 10: torch.uint8}.get(code, torch.float64)
        out = torch.empty(shape, dtype=dtype, device="cuda")
        _check(lib.nfa_grid_export(self.h, code, c_void_p(out.data_ptr()), _stream()), "nfa_grid_export")
        return out

    def __del__(self, _destroy=lib.nfa_grid_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


class Multigrid:
    """Aggregation multigrid preconditioner of an operator (nfa_mg_*)."""

    def __init__(self, op):
        self.op = op
        h = c_void_p()
        _check(lib.nfa_mg_create(op.h, ctypes.byref(h)), "nfa_mg_create")
        self.h = h

    def setup(self):
        _check(lib.nfa_mg_setup(self.h, _stream()), "nfa_mg_setup")

    def set_tail(self, max_cells):
        """First level of the single-workgroup tail: at most max_cells cells
        (0: the coarsest only; negative: the default)."""
        _check(lib.nfa_mg_set_tail(self.h, int(max_cells)), "nfa_mg_set_tail")

    def apply(self, r, out=None):
        """z = V(r), one V-cycle (FP32 cell arrays)."""
        z = torch.empty_like(r) if out is None else out
        _check(lib.nfa_mg_apply(self.h, _dev(r, torch.float32, self.op.shape, "r"),
                                _dev(z, torch.float32, self.op.shape, "z"), _stream()), "nfa_mg_apply")
        return z

    def levels(self):
        L = c_int()
        dims = (c_int * 48)()
        _check(lib.nfa_mg_info(self.h, ctypes.byref(L), dims), "nfa_mg_info")
        return [tuple(dims[3 * l:3 * l + 3]) for l in range(L.value)]

    def set_params(self, omega=0.9, alpha=1.0):
        """Jacobi damping and coarse-correction scale of the V-cycle."""
        _check(lib.nfa_mg_set_params(self.h, float(omega), float(alpha)), "nfa_mg_set_params")

    def set_coef(self, dtype):
        """Precision of the level-0 coefficients the cycle reads: "f32" or "bf16"."""
        _check(lib.nfa_mg_set_coef(self.h, {"f32": NFA_F32, "bf16": NFA_BF16}[dtype]), "nfa_mg_set_coef")

    def side_rows(self, level):
        """Rows of a level held in the side list (couplings beyond 7 points)."""
        m = c_int()
        _check(lib.nfa_mg_side_rows(self.h, level, ctypes.byref(m)), "nfa_mg_side_rows")
        return m.value

    def export(self, level):
        """Level >= 1's FP64 stencil as (27, nz, ny, nx)."""
        shape = self.levels()[level]
        out = torch.empty((27,) + shape, dtype=torch.float64, device="cuda")
        _check(lib.nfa_mg_export(self.h, level, c_void_p(out.data_ptr()), _stream()), "nfa_mg_export")
        return out

    def __del__(self, _destroy=lib.nfa_mg_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


class Vof:
    """Split VOF advection on a grid (nfa_vof_*); the handle owns the plane
    table, the cell lists and a fraction buffer."""

    def __init__(self, grid: Grid):
        self.grid = grid
        h = c_void_p()
        _check(lib.nfa_vof_create(grid.h, ctypes.byref(h)), "nfa_vof_create")
        self.h = h

    def _args(self, phi, u, v, w):
        g = self.grid
        return (_dev(phi, torch.float64, g.shape, "phi"), _dev(u, torch.float64, g.face_shape(0), "u"),
                _dev(v, torch.float64, g.face_shape(1), "v"), _dev(w, torch.float64, g.face_shape(2), "w"))

    def sweep(self, phi, u, v, w, dt, direction, implicit, out=None):
        """One directional sweep (nfa_vof_sweep)."""
        out = torch.empty_like(phi) if out is None else out
        _check(lib.nfa_vof_sweep(self.h, *self._args(phi, u, v, w), dt, direction, int(bool(implicit)),
                                 _dev(out, torch.float64, self.grid.shape, "out"), _stream()), "nfa_vof_sweep")
        return out

    def advect(self, phi, u, v, w, dt, step=0, out=None):
        """One time step (nfa_vof_advect): face velocities u, v, w relative to
        the body, the order of the sweeps set by the parity of step."""
        out = torch.empty_like(phi) if out is None else out
        _check(lib.nfa_vof_advect(self.h, *self._args(phi, u, v, w), dt, step,
                                  _dev(out, torch.float64, self.grid.shape, "out"), _stream()), "nfa_vof_advect")
        return out

    def __del__(self, _destroy=lib.nfa_vof_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


@dataclasses.dataclass
class SolveResult:
    status: int
    iterations: int
    outer: int
    fallback: bool
    relres: float
    ms: float
    history: np.ndarray | None = None


class Poisson:
    """Assembled pressure operator and its solvers on a Grid."""

    def __init__(self, grid: Grid):
        """The operator's device memory is one torch tensor (the workspace),
        owned here and handed to the library."""
        self.grid = grid
        nbytes = int(lib.nfa_poisson_workspace_bytes(grid.h))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = c_void_p()
        _check(lib.nfa_poisson_create(grid.h, c_void_p(self.workspace.data_ptr()), nbytes, ctypes.byref(h)),
               "nfa_poisson_create")
        self.h = h
        self.shape = grid.shape

    def assemble(self, phi, rho_l=1000.0, rho_g=1.2, smooth=True):
        if phi.dtype == torch.float64:
            dt = NFA_F64
        elif phi.dtype == torch.float32:
            dt = NFA_F32
        else:
            raise TypeError("phi must be float64 or float32")
        prm = AssembleParams(rho_l, rho_g, 1 if smooth else 0, dt)
        _check(lib.nfa_poisson_assemble(self.h, _dev(phi, phi.dtype, self.shape, "phi"),
                                        ctypes.byref(prm), _stream()), "nfa_poisson_assemble")

    def apply(self, x, out=None):
        dt = NFA_F64 if x.dtype == torch.float64 else NFA_F32
        y = torch.empty_like(x) if out is None else out
        _check(lib.nfa_poisson_apply(self.h, _dev(x, x.dtype, self.shape, "x"),
                                     _dev(y, x.dtype, self.shape, "y"), dt, _stream()),
               "nfa_poisson_apply")
        return y

    def rhs(self, u, v, w, dt=1.0, body_vel=(0.0, 0.0, 0.0), out=None):
        g = self.grid
        b = torch.empty(self.shape, dtype=torch.float64, device="cuda") if out is None else out
        vel = np.ascontiguousarray(body_vel, dtype=np.float64)
        _check(lib.nfa_poisson_rhs(self.h, _dev(u, torch.float64, g.face_shape(0), "u"),
                                   _dev(v, torch.float64, g.face_shape(1), "v"),
                                   _dev(w, torch.float64, g.face_shape(2), "w"), dt, vel.ctypes.data,
                                   _dev(b, torch.float64, self.shape, "b"), _stream()), "nfa_poisson_rhs")
        return b

    def rhs_cells(self, u, v, w, dt, vb, out=None):
        """nfa_poisson_rhs with a per-cell body velocity vb = (vx, vy, vz) cells."""
        g = self.grid
        b = torch.empty(self.shape, dtype=torch.float64, device="cuda") if out is None else out
        _check(lib.nfa_poisson_rhs_cells(self.h, _dev(u, torch.float64, g.face_shape(0), "u"),
                                         _dev(v, torch.float64, g.face_shape(1), "v"),
                                         _dev(w, torch.float64, g.face_shape(2), "w"), dt,
                                         *[_dev(a, torch.float64, self.shape, "vb") for a in vb],
                                         _dev(b, torch.float64, self.shape, "b"), _stream()), "nfa_poisson_rhs_cells")
        return b

    def project(self, u, v, w, p, dt=1.0):
        g = self.grid
        fu, fv, fw = torch.empty_like(u), torch.empty_like(v), torch.empty_like(w)
        _check(lib.nfa_poisson_project(self.h, _dev(u, torch.float64, g.face_shape(0), "u"),
                                       _dev(v, torch.float64, g.face_shape(1), "v"),
                                       _dev(w, torch.float64, g.face_shape(2), "w"),
                                       _dev(p, torch.float64, self.shape, "p"), dt,
                                       _dev(fu, torch.float64), _dev(fv, torch.float64),
                                       _dev(fw, torch.float64), _stream()), "nfa_poisson_project")
        return fu, fv, fw

    def divergence(self, fu, fv, fw, body_vel=(0.0, 0.0, 0.0)):
        g = self.grid
        div = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        vel = np.ascontiguousarray(body_vel, dtype=np.float64)
        _check(lib.nfa_poisson_divergence(self.h, _dev(fu, torch.float64, g.face_shape(0), "fu"),
                                          _dev(fv, torch.float64, g.face_shape(1), "fv"),
                                          _dev(fw, torch.float64, g.face_shape(2), "fw"),
                                          vel.ctypes.data, _dev(div, torch.float64), _stream()),
               "nfa_poisson_divergence")
        return div

    def multigrid(self):
        """The operator's multigrid preconditioner (created on first use)."""
        if getattr(self, "_mg", None) is None:
            self._mg = Multigrid(self)
        return self._mg

    def solve(self, b, x=None, tol=1e-8, precision="f64", precond="jacobi", max_iters=200000,
              replace_drop=0.1, warm_start=False, check_every=16, unet=None,
              fallback_ratio=0.99, fallback_window=10, history=0, mg=None):
        o = SolveOpts()
        lib.nfa_solve_opts_default(ctypes.byref(o))
        o.tol = tol
        o.max_iters = max_iters
        o.precision = {"f64": NFA_PREC_F64, "mixed": NFA_PREC_MIXED}[precision]
        o.precond = {"jacobi": NFA_PC_JACOBI, "unet": NFA_PC_UNET, "jacobi_fcg": NFA_PC_JACOBI_FCG,
                     "sabotage": NFA_PC_TEST_SABOTAGE, "mg": NFA_PC_MG}[precond]
        if precond == "mg":
            o.mg = (mg if mg is not None else self.multigrid()).h
        o.replace_drop = replace_drop
        o.warm_start = 1 if warm_start else 0
        o.check_every = check_every
        o.fallback_ratio = fallback_ratio
        o.fallback_window = fallback_window
        o.unet = None if unet is None else unet.h
        hist = None
        if history:
            hist = np.zeros(history, dtype=np.float64)
            o.history = hist.ctypes.data_as(ctypes.POINTER(c_double))
            o.history_cap = history
        if x is None:
            x = torch.zeros(self.shape, dtype=torch.float64, device="cuda")
        info = SolveInfo()
        st = _check(lib.nfa_poisson_solve(self.h, _dev(b, torch.float64, self.shape, "b"),
                                          _dev(x, torch.float64, self.shape, "x"), ctypes.byref(o),
                                          _stream(), ctypes.byref(info)), "nfa_poisson_solve")
        res = SolveResult(st, info.iterations, info.outer, bool(info.fallback), info.relres, info.ms,
                          None if hist is None else hist[:info.history_len].copy())
        return x, res

    def residual(self, b, x, out=None):
        """(r = b' - A'x in FP64, ||r||^2)."""
        r = torch.empty_like(b) if out is None else out
        rr = c_double()
        _check(lib.nfa_poisson_residual(self.h, _dev(b, torch.float64, self.shape, "b"),
                                        _dev(x, torch.float64, self.shape, "x"),
                                        _dev(r, torch.float64, self.shape, "r"), ctypes.byref(rr), _stream()),
               "nfa_poisson_residual")
        return r, rr.value

    def velocity(self, ut, p, dt=1.0, scale=1.0):
        """Velocity form of the projection on the three face sets:
        scale * (u~ - dt beta grad p), closed and Neumann faces keep scale * u~."""
        g = self.grid
        shapes = [g.face_shape(a) for a in range(3)]
        ins = [_dev(t, torch.float64, sh, f"ut[{a}]") for a, (t, sh) in enumerate(zip(ut, shapes))]
        out = [torch.empty(sh, dtype=torch.float64, device="cuda") for sh in shapes]
        _check(lib.nfa_poisson_velocity(self.h, *ins, _dev(p, torch.float64, self.shape, "p"), dt, scale,
                                        *[_dev(o, torch.float64) for o in out], _stream()),
               "nfa_poisson_velocity")
        return tuple(out)

    def rk2_cycle(self, phi_k, phi_star, uk, R, dt, body_vel=(0.0, 0.0, 0.0), rho_l=1000.0, rho_g=1.2,
                  smooth=True, tol=1e-8, precision="f64", precond="jacobi", max_iters=200000,
                  pstar=None, p=None, warm_start=False, unet=None):
        """One Runge-Kutta projection cycle (nfa_rk2_cycle).  Returns a dict with
        u* ('ustar'), u^{k+1} ('unext'), the pressures 'pstar' and 'p', and the
        two stages' SolveResult.  Leaves the operator assembled with phi_star."""
        g = self.grid
        if phi_k.dtype != phi_star.dtype or phi_k.dtype not in (torch.float64, torch.float32):
            raise TypeError("phi_k and phi_star must share a float64 or float32 dtype")
        dtp = NFA_F64 if phi_k.dtype == torch.float64 else NFA_F32
        shapes = [g.face_shape(a) for a in range(3)]
        trip = lambda ts, name: (c_void_p * 3)(*[_dev(t, torch.float64, sh, f"{name}[{a}]")
                                                 for a, (t, sh) in enumerate(zip(ts, shapes))])
        ut = [torch.empty(sh, dtype=torch.float64, device="cuda") for sh in shapes]
        ustar = [torch.empty(sh, dtype=torch.float64, device="cuda") for sh in shapes]
        unext = [torch.empty(sh, dtype=torch.float64, device="cuda") for sh in shapes]
        pstar = torch.zeros(self.shape, dtype=torch.float64, device="cuda") if pstar is None else pstar
        p = torch.zeros(self.shape, dtype=torch.float64, device="cuda") if p is None else p
        prm = RK2Params(dt, (c_double * 3)(*body_vel), AssembleParams(rho_l, rho_g, 1 if smooth else 0, dtp))
        o = SolveOpts()
        lib.nfa_solve_opts_default(ctypes.byref(o))
        o.tol = tol
        o.max_iters = max_iters
        o.precision = {"f64": NFA_PREC_F64, "mixed": NFA_PREC_MIXED}[precision]
        o.precond = {"jacobi": NFA_PC_JACOBI, "unet": NFA_PC_UNET, "jacobi_fcg": NFA_PC_JACOBI_FCG,
                     "mg": NFA_PC_MG}[precond]
        if precond == "mg":
            o.mg = self.multigrid().h
        o.warm_start = 1 if warm_start else 0
        o.unet = None if unet is None else unet.h
        info = (SolveInfo * 2)()
        st = _check(lib.nfa_rk2_cycle(self.h, _dev(phi_k, phi_k.dtype, self.shape, "phi_k"),
                                      _dev(phi_star, phi_star.dtype, self.shape, "phi_star"), ctypes.byref(prm),
                                      trip(uk, "uk"), trip(R, "R"), trip(ut, "ut"), trip(ustar, "ustar"),
                                      _dev(pstar, torch.float64, self.shape, "pstar"),
                                      _dev(p, torch.float64, self.shape, "p"), trip(unext, "unext"),
                                      ctypes.byref(o), _stream(), info), "nfa_rk2_cycle")
        res = [SolveResult(st, i.iterations, i.outer, bool(i.fallback), i.relres, i.ms) for i in info]
        return {"ustar": tuple(ustar), "unext": tuple(unext), "pstar": pstar, "p": p, "ut2": tuple(ut),
                "stage1": res[0], "stage2": res[1], "status": st}

    def profile(self, enable=True):
        _check(lib.nfa_poisson_profile(self.h, 1 if enable else 0), "nfa_poisson_profile")

    def profile_read(self, dtype):
        ks = KernelStats()
        code = {"f64": NFA_F64, "f32": NFA_F32, "mg_down": NFA_PROF_MG_DOWN, "mg_up": NFA_PROF_MG_UP,
                "f32_flex": NFA_PROF_F32_FLEX, "unet": NFA_PROF_UNET, "f64_x2": NFA_PROF_F64_X2,
                "f32_x2": NFA_PROF_F32_X2}[dtype]
        _check(lib.nfa_poisson_profile_read(self.h, code, ctypes.byref(ks)), "nfa_poisson_profile_read")
        return {"launches": ks.launches, "ms": ks.ms, "cells": ks.cells}

    def export(self, what):
        code = EXPORT[what]
        g = self.grid
        shape = {21: g.face_shape(0), 22: g.face_shape(1), 23: g.face_shape(2),
                 25: g.face_shape(0), 26: g.face_shape(1), 27: g.face_shape(2)}.get(code, self.shape)
        dtype = torch.float32 if code in (25, 26, 27, 28) else torch.float64
        out = torch.empty(shape, dtype=dtype, device="cuda")
        _check(lib.nfa_poisson_export(self.h, code, c_void_p(out.data_ptr()), _stream()),
               "nfa_poisson_export")
        return out

    def __del__(self, _destroy=lib.nfa_poisson_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


def unet_channels(levels):
    return [16, 32, 64][:levels] + [64] * max(0, levels - 3)


def unet_taps(levels=3):
    """Taps per convolution in parameter order: 27 each, 1 for the head."""
    return [27] * (len(unet_shapes(levels)) - 1) + [1]


def unet_shapes(levels=3):
    c = unet_channels(levels)
    out = [(2, c[0])] + [(c[l - 1], c[l]) for l in range(1, levels)]
    out.append((c[levels - 1], c[levels - 2]))
    out += [(c[l], c[l - 1]) for l in range(levels - 2, 0, -1)]
    out.append((c[0], c[0]))
    out.append((c[0], 1))
    return out


class UNet:
    """The learned preconditioner (see include/nfa_unet.h)."""

    def __init__(self, nx, ny, nz, seed=0, levels=3):
        """Device memory: one workspace tensor for the network, and four FP32
        tensors (params, grads, adam_m, adam_v) bound as its parameter state;
        all owned here."""
        nbytes = int(lib.nfa_unet_workspace_bytes(nx, ny, nz, levels))
        if nbytes == 0:
            raise NFAError("nfa_unet_workspace_bytes: invalid network size")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = c_void_p()
        _check(lib.nfa_unet_create(nx, ny, nz, levels, seed, c_void_p(self.workspace.data_ptr()), nbytes,
                                   ctypes.byref(h)), "nfa_unet_create")
        self.h = h
        self.shape = (nz, ny, nx)
        self.levels = levels
        n = self.param_count()
        self.params, self.grads, self.adam_m, self.adam_v = (
            torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(4))
        self._bind(copy=True)

    def _bind(self, copy):
        _check(lib.nfa_unet_bind(self.h, *(c_void_p(t.data_ptr()) for t in
                                           (self.params, self.grads, self.adam_m, self.adam_v)), int(copy)),
               "nfa_unet_bind")

    def state(self):
        """Parameters and Adam moments as host arrays (a training checkpoint)."""
        torch.cuda.synchronize()
        return {k: getattr(self, k).cpu().numpy() for k in ("params", "adam_m", "adam_v")}

    def load_state(self, state):
        """Resume from state(): the arrays become the bound parameter state."""
        for k in ("params", "adam_m", "adam_v"):
            getattr(self, k).copy_(torch.as_tensor(np.asarray(state[k], dtype=np.float32)))
        torch.cuda.synchronize()
        self._bind(copy=False)

    def param_count(self):
        return int(lib.nfa_unet_param_count(self.levels))

    def _flat(self, fn, what):
        a = np.empty(self.param_count(), dtype=np.float32)
        _check(fn(self.h, a.ctypes.data), what)
        return a

    def get_params(self):
        return self._flat(lib.nfa_unet_get_params, "nfa_unet_get_params")

    def get_grads(self):
        return self._flat(lib.nfa_unet_get_grads, "nfa_unet_get_grads")

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != self.param_count():
            raise ValueError("wrong parameter count")
        _check(lib.nfa_unet_set_params(self.h, a.ctypes.data), "nfa_unet_set_params")

    def unflatten(self, flat):
        out, o = [], 0
        for (ci, co), nt in zip(unet_shapes(self.levels), unet_taps(self.levels)):
            w = flat[o:o + nt * ci * co].reshape(nt, ci, co)
            o += nt * ci * co
            b = flat[o:o + co]
            o += co
            out.append((w, b))
        return out

    @staticmethod
    def flatten(params):
        return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)

    def forward(self, op, r, out=None, keep=False):
        """z = network(r); keep=True also stores every activation for export()."""
        z = torch.empty_like(r) if out is None else out
        _check(lib.nfa_unet_forward(self.h, op.h, _dev(r, torch.float32, self.shape, "r"),
                                    _dev(z, torch.float32, self.shape, "z"), int(bool(keep)), _stream()),
               "nfa_unet_forward")
        return z

    def grad(self, op, r, eAe):
        loss = c_double()
        _check(lib.nfa_unet_grad(self.h, op.h, _dev(r, torch.float32, self.shape, "r"), float(eAe),
                                 ctypes.byref(loss), _stream()), "nfa_unet_grad")
        return loss.value

    def train_step(self, op, r, eAe, lr, t):
        loss = c_double()
        _check(lib.nfa_unet_train_step(self.h, op.h, _dev(r, torch.float32, self.shape, "r"), float(eAe),
                                       float(lr), int(t), ctypes.byref(loss), _stream()), "nfa_unet_train_step")
        return loss.value

    def backward(self, op, dz):
        """Gradients for dL/dz = dz (FP32 cells) at the output of the last
        forward with keep=True on `op` (nfa_unet_backward)."""
        _check(lib.nfa_unet_backward(self.h, op.h, _dev(dz, torch.float32, self.shape, "dz"), _stream()),
               "nfa_unet_backward")

    def adam_step(self, lr, t, b1=0.9, b2=0.999, eps=1e-8):
        """One Adam step on the current gradients (nfa_unet_adam_step)."""
        _check(lib.nfa_unet_adam_step(self.h, float(lr), float(b1), float(b2), float(eps), int(t), _stream()),
               "nfa_unet_adam_step")

    def export(self, what):
        """Activations 'x0', 'a<l>', 'p<l>', 'd<l>' of the last forward with keep,
        or gradients 'dz' (FP32 cells), 'dd<l>', 'skip<l>', 'da<l>', 'dp<l>' of
        the last grad / train_step, as channels-last bfloat16 tensors."""
        c = unet_channels(self.levels)
        nz, ny, nx = self.shape
        if what == "dz":
            out = torch.empty(self.shape, dtype=torch.float32, device="cuda")
            _check(lib.nfa_unet_export(self.h, 64, c_void_p(out.data_ptr()), _stream()), "nfa_unet_export")
            return out
        if what == "x0":
            code, level, ch = 0, 0, 2
        else:
            kind = what.rstrip("0123456789")
            l = int(what[len(kind):])
            code = {"a": 16, "p": 32, "d": 48, "dd": 80, "skip": 96, "da": 112, "dp": 128}[kind] + l
            level = l + 1 if kind in ("p", "dp") else l
            ch = (c[l - 1] if l > 0 else c[0]) if kind in ("d", "dd") else c[l]
        f = 2 ** level
        out = torch.empty((nz // f, ny // f, nx // f, ch), dtype=torch.bfloat16, device="cuda")
        _check(lib.nfa_unet_export(self.h, code, c_void_p(out.data_ptr()), _stream()), "nfa_unet_export")
        return out

    def __del__(self, _destroy=lib.nfa_unet_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


def from_workload(wl, device_phi_dtype=torch.float64):
    """Grid + body + assembled operator + right-hand side for a fixtures.Workload."""
    g = Grid(wl.xf, wl.yf, wl.zf, wl.bc)
    if wl.psi is not None:
        g.set_body(torch.as_tensor(wl.psi, device="cuda"), wl.theta, wl.samples)
    op = Poisson(g)
    phi = torch.as_tensor(wl.phi, device="cuda").to(device_phi_dtype).contiguous()
    op.assemble(phi, wl.rho_l, wl.rho_g, wl.smooth)
    if wl.b is not None:
        b = torch.as_tensor(wl.b, device="cuda").contiguous()
    else:
        b = op.rhs(torch.as_tensor(wl.u, device="cuda"), torch.as_tensor(wl.v, device="cuda"),
                   torch.as_tensor(wl.w, device="cuda"), wl.dt, wl.body_vel)
    return g, op, b
