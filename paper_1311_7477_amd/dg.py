"""Thin ctypes binding of libdgark (include/dgark.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Fields are torch float64 CUDA tensors of shape
(ny, nx, n, n) (layout [cy][cx][j][i]); the current torch stream is passed
to every call.  If the library is missing, the first call raises: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgark.so")

DG_OK = 0
DG_E_INVAL, DG_E_ALIAS, DG_E_NOMEM, DG_E_HIP = -1, -2, -3, -4
DG_E_NOCONV, DG_E_UNSUPPORTED, DG_E_WORKSPACE = -5, -6, -7
DG_BC_PERIODIC, DG_BC_DIRICHLET = 0, 1
DG_PREC_FP64, DG_PREC_MIXED = 0, 1
DG_WS_FD = 0x10
DG_WS_FD_PRODUCTS = 0x20      # with DG_WS_FD: folded matrix products, no rocFFT plans
DG_PRECOND_NONE, DG_PRECOND_FD = 0, 1
DG_FORM_ARAKAWA, DG_FORM_PP, DG_FORM_PX, DG_FORM_XP = 0, 1, 2, 3

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


class CgOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("precond", ctypes.c_int),
                ("check_every", ctypes.c_int)]


class CgStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("converged", ctypes.c_int)]


class StepOpts(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("D", ctypes.c_double), ("cg", CgOpts),
                ("record_times", ctypes.c_int), ("form", ctypes.c_int)]


class StepStats(ctypes.Structure):
    _fields_ = [("cg_iters", ctypes.c_int * 3), ("stage_ms", ctypes.c_float * 3),
                ("converged", ctypes.c_int)]


class DgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dgark error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Open libdgark.so (once); raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "dg_last_error": (ctypes.c_char_p, []),
        "dg_grid_create": (ctypes.c_int, [ctypes.c_int] * 3 + [ctypes.c_double] * 4
                           + [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
        "dg_grid_destroy": (None, [_vp]),
        "dg_field_elems": (ctypes.c_size_t, [_vp]),
        "dg_grid_tables": (ctypes.c_int, [_vp, _dp, ctypes.c_int]),
        "dg_workspace_bytes": (ctypes.c_int, [_vp, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_size_t)]),
        "dg_workspace_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_vp)]),
        "dg_workspace_destroy": (None, [_vp]),
        "dg_workspace_held_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
        "dg_poisson_bracket": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
        "dg_bracket_form": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, _vp]),
        "dg_laplace_apply": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
        "dg_cg_solve_poisson": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(CgOpts),
                                               ctypes.POINTER(CgStats), _vp, _vp]),
        "dg_precond_apply": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
        "dg_ab_state_create": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double,
                                              ctypes.POINTER(_vp)]),
        "dg_ab_state_destroy": (None, [_vp]),
        "dg_ab_time": (ctypes.c_double, [_vp]),
        "dg_ab_psi_state": (_vp, [_vp]),
        "dg_ab_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(StepOpts),
                                      ctypes.POINTER(StepStats), _vp, _vp]),
        "dg_grid_set_tiles": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
        "dg_grid_tiles": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int)]),
        "dg_grid_tune": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _dp, _vp]),
        "dg_grid_fd_basis": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp,
                                            ctypes.POINTER(ctypes.c_int)]),
        "dg_grid_axis_operator": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
        "dg_state_create": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.POINTER(_vp)]),
        "dg_state_destroy": (None, [_vp]),
        "dg_state_psi": (_vp, [_vp]),
        "dg_state_copy_psi": (ctypes.c_int, [_vp, _vp, _vp]),
        "dg_state_time": (ctypes.c_double, [_vp]),
        "dg_rk_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(StepOpts),
                                      ctypes.POINTER(StepStats), _vp, _vp]),
        "dg_invariants": (ctypes.c_int, [_vp, _vp, _vp, _dp, _vp, _vp]),
        "dg_invariants_dev": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "dg_invariants_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
        "dg_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
        "dg_profile_read": (ctypes.c_int, [_vp, _dp]),
        "dg_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp)]),
        "dg_batch_destroy": (None, [_vp]),
        "dg_batch_attach": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double,
                                           ctypes.POINTER(ctypes.c_int)]),
        "dg_batch_detach": (ctypes.c_int, [_vp, ctypes.c_int]),
        "dg_batch_member_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
        "dg_batch_use_graphs": (ctypes.c_int, [_vp, ctypes.c_int]),
        "dg_batch_use_precond": (ctypes.c_int, [_vp, ctypes.c_int]),
        "dg_batch_rk_step": (ctypes.c_int, [_vp, ctypes.POINTER(CgOpts),
                                            ctypes.POINTER(ctypes.c_int), _vp]),
        "dg_batch_copy_psi": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp]),
        "dg_batch_slot_converged": (ctypes.c_int, [_vp, ctypes.c_int]),
        "dg_batch_time": (ctypes.c_double, [_vp, ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int, allow=()):
    if rc != DG_OK and rc not in allow:
        raise DgError(rc, lib().dg_last_error().decode())
    return rc


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return _vp(s.cuda_stream)


class Grid:
    """Periodic grid: n polynomials per cell and direction, nx x ny cells."""

    def __init__(self, n, nx, ny, x0=0.0, x1=None, y0=0.0, y1=None,
                 bc_x=DG_BC_PERIODIC, bc_y=DG_BC_PERIODIC):
        import math
        x1 = 2 * math.pi if x1 is None else x1
        y1 = 2 * math.pi if y1 is None else y1
        h = _vp()
        _check(lib().dg_grid_create(n, nx, ny, x0, x1, y0, y1, bc_x, bc_y,
                                    ctypes.byref(h)))
        self._h = h
        self.n, self.nx, self.ny = n, nx, ny
        self.shape = (ny, nx, n, n)
        self.elems = int(lib().dg_field_elems(h))

    @property
    def handle(self):
        return self._h

    def tables(self):
        out = (ctypes.c_double * 256)()
        k = _check_count(lib().dg_grid_tables(self._h, out, 256))
        return [out[i] for i in range(k)]

    def set_tiles(self, cw, rw):
        """Cell tile height cw in {4, 8, 16}, bracket tile height rw in {8, 16}."""
        _check(lib().dg_grid_set_tiles(self._h, cw, rw))

    def tiles(self):
        cw, rw = ctypes.c_int(), ctypes.c_int()
        _check(lib().dg_grid_tiles(self._h, ctypes.byref(cw), ctypes.byref(rw)))
        return cw.value, rw.value

    def tune(self, omega, reps=20):
        """Time every tile shape on this grid (omega: a device field with a
        nonzero mean-free part), keep the fastest; returns ((cw, rw), ms) with
        ms = per-iteration / per-bracket times of cw = 4, 8, 16 and rw = 8, 16."""
        ms = (ctypes.c_double * 5)()
        _check(lib().dg_grid_tune(self._h, _field(omega, self, "omega"), reps, ms, _stream()))
        return self.tiles(), list(ms)

    def fd_basis(self, axis=0):
        """(V, lam, zero) of the fast-diagonalisation basis along one axis
        (host numpy arrays; V[:, k] is mode k)."""
        import numpy as np
        N = self.nx if axis == 0 else self.ny
        NN = N * self.n
        V = np.empty(NN * NN)
        lam = np.empty(NN)
        z = ctypes.c_int()
        _check(lib().dg_grid_fd_basis(self._h, axis, V.ctypes.data_as(_dp),
                                      lam.ctypes.data_as(_dp), ctypes.byref(z)))
        return V.reshape(NN, NN).T.copy(), lam, z.value

    def axis_operator(self, axis=0):
        """The 1D LDG second derivative of one axis as a dense host numpy
        array (rows and columns c * n + i)."""
        import numpy as np
        N = self.nx if axis == 0 else self.ny
        NN = N * self.n
        L = np.empty(NN * NN)
        _check(lib().dg_grid_axis_operator(self._h, axis, L.ctypes.data_as(_dp)))
        return L.reshape(NN, NN).T.copy()

    def workspace_bytes(self, mode=DG_PREC_FP64):
        b = ctypes.c_size_t()
        _check(lib().dg_workspace_bytes(self._h, mode, ctypes.byref(b)))
        return b.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dg_grid_destroy(self._h)
            self._h = None


def _check_count(rc):
    if rc < 0:
        raise DgError(rc, lib().dg_last_error().decode())
    return rc


class Workspace:
    def __init__(self, grid: Grid, mode=DG_PREC_FP64):
        h = _vp()
        _check(lib().dg_workspace_create(grid.handle, mode, ctypes.byref(h)))
        self._h, self.grid, self.mode = h, grid, mode

    @property
    def handle(self):
        return self._h

    def held_bytes(self):
        """Device bytes this workspace holds, library work buffers included."""
        b = ctypes.c_size_t()
        _check(lib().dg_workspace_held_bytes(self._h, ctypes.byref(b)))
        return b.value

    def profile(self, on=True):
        _check(lib().dg_profile_enable(self._h, 1 if on else 0))

    def read_profile(self):
        """(mean ms direction kernel, samples, mean ms residual kernel, samples)"""
        out = (ctypes.c_double * 4)()
        _check(lib().dg_profile_read(self._h, out))
        a, na, b, nb = out
        return (a / na if na else float("nan"), int(na), b / nb if nb else float("nan"), int(nb))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dg_workspace_destroy(self._h)
            self._h = None


class State:
    def __init__(self, grid: Grid, t0=0.0):
        h = _vp()
        _check(lib().dg_state_create(grid.handle, t0, ctypes.byref(h)))
        self._h, self.grid = h, grid

    @property
    def handle(self):
        return self._h

    @property
    def t(self):
        return lib().dg_state_time(self._h)

    def psi(self):
        """The most recent Poisson solution as a new tensor (a copy)."""
        import torch
        if not lib().dg_state_psi(self._h):
            return None
        out = torch.empty(self.grid.shape, dtype=torch.float64, device="cuda")
        _check(lib().dg_state_copy_psi(self._h, _vp(out.data_ptr()), _stream()))
        return out

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dg_state_destroy(self._h)
            self._h = None


def _field(t, grid: Grid, name: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() != grid.elems:
        raise ValueError(f"{name} has {t.numel()} elements, grid needs {grid.elems}")
    return _vp(t.data_ptr())


def poisson_bracket(grid: Grid, f, g, out=None):
    """out = J(f, g), the conservative dG Arakawa bracket."""
    import torch
    out = torch.empty_like(f) if out is None else out
    _check(lib().dg_poisson_bracket(grid.handle, _field(f, grid, "f"),
                                    _field(g, grid, "g"), _field(out, grid, "out"),
                                    _stream()))
    return out


def bracket_form(grid: Grid, f, g, form, out=None):
    import torch
    out = torch.empty_like(f) if out is None else out
    _check(lib().dg_bracket_form(grid.handle, _field(f, grid, "f"),
                                 _field(g, grid, "g"), _field(out, grid, "out"),
                                 form, _stream()))
    return out


def laplace_apply(grid: Grid, f, out=None):
    import torch
    out = torch.empty_like(f) if out is None else out
    _check(lib().dg_laplace_apply(grid.handle, _field(f, grid, "f"),
                                  _field(out, grid, "out"), _stream()))
    return out


def cg_opts(rtol=1e-12, max_iter=100000, precision=DG_PREC_FP64,
            precond=DG_PRECOND_NONE, check_every=0):
    return CgOpts(rtol, max_iter, precision, precond, check_every)


def precond_apply(grid: Grid, r, ws: Workspace, out=None):
    """z = (-Lap_h)^+ r by fast diagonalisation (ws made with DG_WS_FD)."""
    import torch
    out = torch.empty_like(r) if out is None else out
    _check(lib().dg_precond_apply(grid.handle, _field(r, grid, "r"),
                                  _field(out, grid, "z"), ws.handle, _stream()))
    return out


@dataclass
class SolveResult:
    iters: int
    outer_iters: int
    rel_residual: float
    converged: bool
    stalled: bool = False     # mixed mode: stopped at the attainable FP64 accuracy


def cg_solve_poisson(grid: Grid, omega, psi, ws: Workspace, opts: CgOpts = None):
    """Solve -Lap psi = omega - mean(omega) in place (psi holds the guess)."""
    st = CgStats()
    opts = cg_opts() if opts is None else opts
    _check(lib().dg_cg_solve_poisson(grid.handle, _field(omega, grid, "omega"),
                                     _field(psi, grid, "psi"), ctypes.byref(opts),
                                     ctypes.byref(st), ws.handle, _stream()),
           allow=(DG_E_NOCONV,))
    return SolveResult(st.iters, st.outer_iters, st.rel_residual, bool(st.converged),
                       st.converged == 2)


@dataclass
class StepResult:
    cg_iters: tuple
    stage_ms: tuple
    converged: bool
    stalled: bool = False     # a mixed-mode solve stopped at the attainable FP64 accuracy


def rk_step(grid: Grid, omega, state: State, ws: Workspace, dt, D,
            opts: CgOpts = None, record_times=False, form=DG_FORM_ARAKAWA):
    so = StepOpts(dt, D, cg_opts() if opts is None else opts, 1 if record_times else 0,
                  form)
    st = StepStats()
    _check(lib().dg_rk_step(grid.handle, _field(omega, grid, "omega"), state.handle,
                            ctypes.byref(so), ctypes.byref(st), ws.handle, _stream()),
           allow=(DG_E_NOCONV,))
    return StepResult(tuple(st.cg_iters), tuple(st.stage_ms), bool(st.converged),
                      st.converged == 2)


class AbState:
    """K-step Adams-Bashforth state (dg_ab_*): K right-hand sides and the
    psi history."""

    def __init__(self, grid: Grid, K: int, t0=0.0):
        h = _vp()
        _check(lib().dg_ab_state_create(grid.handle, K, t0, ctypes.byref(h)))
        self._h, self.grid, self.K = h, grid, K

    @property
    def handle(self):
        return self._h

    @property
    def t(self):
        return lib().dg_ab_time(self._h)

    def psi(self):
        """The most recent Poisson solution as a new tensor (a copy)."""
        import torch
        st = lib().dg_ab_psi_state(self._h)
        if not lib().dg_state_psi(st):
            return None
        out = torch.empty(self.grid.shape, dtype=torch.float64, device="cuda")
        _check(lib().dg_state_copy_psi(st, _vp(out.data_ptr()), _stream()))
        return out

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dg_ab_state_destroy(self._h)
            self._h = None


def ab_step(grid: Grid, omega, ab: AbState, ws: Workspace, dt, D, opts: CgOpts = None,
            form=DG_FORM_ARAKAWA):
    so = StepOpts(dt, D, cg_opts() if opts is None else opts, 0, form)
    st = StepStats()
    _check(lib().dg_ab_step(grid.handle, _field(omega, grid, "omega"), ab.handle,
                            ctypes.byref(so), ctypes.byref(st), ws.handle, _stream()),
           allow=(DG_E_NOCONV,))
    return StepResult(tuple(st.cg_iters), tuple(st.stage_ms), bool(st.converged),
                      st.converged == 2)


def invariants(grid: Grid, omega, psi, ws: Workspace):
    out = (ctypes.c_double * 3)()
    _check(lib().dg_invariants(grid.handle, _field(omega, grid, "omega"),
                               _field(psi, grid, "psi"), out, ws.handle, _stream()))
    return tuple(out)


def invariants_dev(grid: Grid, omega, psi, ws: Workspace, out=None):
    """(V, E, Omega) into a device tensor of 3 doubles (asynchronous)."""
    import torch
    out = torch.empty(3, dtype=torch.float64, device="cuda") if out is None else out
    _check(lib().dg_invariants_dev(grid.handle, _field(omega, grid, "omega"),
                                   _field(psi, grid, "psi"), _vp(out.data_ptr()),
                                   ws.handle, _stream()))
    return out


def invariants_noalloc(grid: Grid, omega, psi, out):
    """(V, E, Omega) into the caller's device tensor `out` (3 doubles) with
    no workspace and no allocation (dg_invariants_noalloc)."""
    _check(lib().dg_invariants_noalloc(grid.handle, _field(omega, grid, "omega"),
                                       _field(psi, grid, "psi"), _vp(out.data_ptr()),
                                       _stream()))
    return out


class Batch:
    """Instances advanced together by batched fused launches (see
    dg_batch_* in include/dgark.h).  Members keep references to their grid
    and omega tensor while attached."""

    def __init__(self, capacity: int, use_graphs: bool = True):
        h = _vp()
        _check(lib().dg_batch_create(capacity, ctypes.byref(h)))
        self._h, self.capacity = h, capacity
        self.members = {}
        _check(lib().dg_batch_use_graphs(h, 1 if use_graphs else 0))

    def use_precond(self, ws_fd_flags: int = DG_WS_FD):
        """Members attached from now on get the fast-diagonalisation
        preconditioner (call before attaching), so that rk_step can take
        cg_opts(precond=DG_PRECOND_FD)."""
        _check(lib().dg_batch_use_precond(self._h, ws_fd_flags))

    def attach(self, grid: Grid, omega, dt: float, D: float, t0: float = 0.0) -> int:
        slot = ctypes.c_int()
        _check(lib().dg_batch_attach(self._h, grid.handle, _field(omega, grid, "omega"),
                                     dt, D, t0, ctypes.byref(slot)))
        self.members[slot.value] = (grid, omega)
        return slot.value

    def detach(self, slot: int):
        _check(lib().dg_batch_detach(self._h, slot))
        self.members.pop(slot, None)

    def rk_step(self, opts: CgOpts = None):
        """One SSP-RK3 step of every member; returns {slot: (iters stage 1..3)}
        and whether every solve converged."""
        it = (ctypes.c_int * (3 * self.capacity))()
        rc = _check(lib().dg_batch_rk_step(self._h, ctypes.byref(cg_opts() if opts is None else opts),
                                           it, _stream()), allow=(DG_E_NOCONV,))
        return {s: tuple(it[3 * s:3 * s + 3]) for s in self.members}, rc == DG_OK

    def psi(self, slot: int):
        import torch
        grid = self.members[slot][0]
        out = torch.empty(grid.shape, dtype=torch.float64, device="cuda")
        _check(lib().dg_batch_copy_psi(self._h, slot, _vp(out.data_ptr()), _stream()))
        return out

    def time(self, slot: int) -> float:
        return lib().dg_batch_time(self._h, slot)

    def converged(self, slot: int) -> bool:
        """Whether every solve of the slot's last step converged."""
        return _check_count(lib().dg_batch_slot_converged(self._h, slot)) == 1

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dg_batch_destroy(self._h)
            self._h = None


def batch_member_bytes(grid: Grid) -> int:
    b = ctypes.c_size_t()
    _check(lib().dg_batch_member_bytes(grid.handle, ctypes.byref(b)))
    return b.value
