"""fvib: FV + immersed-boundary time step and its discrete adjoint on MI355X.

Thin Python binding over libfvib.so (include/fvib.h).  PyTorch provides
device memory and the HIP stream; every step of the method runs in the
library's HIP kernels.  The binding fails loudly if the library is missing.

Module-level functions carry the names of the C entry points
(``fvib_create_grid``, ``fvib_step``, ...); :class:`Grid` wraps a handle
with tensor-friendly helpers.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _abi
from ._abi import BC, BODY, CONV, PREC, SOLVER, STATUS_NAMES

__all__ = ["Grid", "FvibError", "fvib_create_grid", "fvib_destroy_grid", "fvib_field_layout",
           "fvib_ib_set_body", "fvib_step", "fvib_step_adjoint", "fvib_step_strong",
           "fvib_step_strong_adjoint", "fvib_step_rk", "fvib_step_rk_adjoint", "fvib_set_dt",
           "fvib_cfl_dt", "fvib_loss_wall_shear",
           "fvib_loss_wall_shear_noalloc", "fvib_loss_rms_lift", "fvib_last_error", "fvib_version", "lib"]


class FvibError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fvib status {code} ({STATUS_NAMES.get(code, '?')}): {msg}")
        self.code = code


def lib() -> C.CDLL:
    return _abi.load()


def _ptr(t) -> int:
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _check(rc: int, handle=None):
    if rc != 0:
        msg = lib().fvib_last_error(handle).decode()
        raise FvibError(rc, msg)


# ------------------------------------------------------------ C-name wrappers
def fvib_create_grid(desc: _abi.GridDesc, stream: int = 0):
    h = C.c_void_p()
    _check(lib().fvib_create_grid(C.byref(desc), C.c_void_p(stream), C.byref(h)))
    return h


def fvib_destroy_grid(h) -> None:
    _check(lib().fvib_destroy_grid(h))


def fvib_field_layout(h, comp: int):
    shape = (C.c_int64 * 3)()
    strides = (C.c_int64 * 3)()
    dt = C.c_int()
    _check(lib().fvib_field_layout(h, comp, shape, strides, C.byref(dt)), h)
    return tuple(shape), tuple(strides), dt.value


def fvib_ib_set_body(h, body: Optional[_abi.BodyDesc]) -> None:
    _check(lib().fvib_ib_set_body(h, C.byref(body) if body is not None else None), h)


def fvib_step(h, fin: _abi.Fields, fout: _abi.Fields, info_ptr: int = 0) -> int:
    return lib().fvib_step(h, C.byref(fin), C.byref(fout), C.c_void_p(info_ptr))


def fvib_step_strong(h, fin: _abi.Fields, fout: _abi.Fields, max_iters: int, tol: float,
                     omega_ptr: int = 0, info_ptr: int = 0) -> int:
    return lib().fvib_step_strong(h, C.byref(fin), C.byref(fout), int(max_iters), float(tol),
                                  C.c_void_p(omega_ptr), C.c_void_p(info_ptr))


def fvib_step_strong_adjoint(h, fin: _abi.Fields, omega_ptr: int, bar_out: _abi.Adjoint,
                             dF_ptr: int, bar_in: _abi.Adjoint, info_ptr: int = 0) -> int:
    return lib().fvib_step_strong_adjoint(h, C.byref(fin), C.c_void_p(omega_ptr),
                                          C.byref(bar_out), C.c_void_p(dF_ptr), C.byref(bar_in),
                                          C.c_void_p(info_ptr))


def fvib_step_rk(h, fin: _abi.Fields, fout: _abi.Fields, scheme: int, info_ptr: int = 0) -> int:
    return lib().fvib_step_rk(h, C.byref(fin), C.byref(fout), int(scheme), C.c_void_p(info_ptr))


def fvib_step_rk_adjoint(h, fin: _abi.Fields, bar_out: _abi.Adjoint, bar_in: _abi.Adjoint,
                         scheme: int, info_ptr: int = 0) -> int:
    return lib().fvib_step_rk_adjoint(h, C.byref(fin), C.byref(bar_out), C.byref(bar_in),
                                      int(scheme), C.c_void_p(info_ptr))


def fvib_set_dt(h, dt: float) -> int:
    return lib().fvib_set_dt(h, float(dt))


def fvib_cfl_dt(h, u_ptrs, cfl: float, dt_max: float):
    vp = C.c_void_p * 3
    out = C.c_double()
    rc = lib().fvib_cfl_dt(h, vp(*(list(u_ptrs) + [0] * (3 - len(u_ptrs)))), float(cfl),
                           float(dt_max), C.byref(out))
    return rc, out.value


def fvib_step_adjoint(h, fin: _abi.Fields, bar_out: _abi.Adjoint, dF_ptr: int,
                      bar_in: _abi.Adjoint, info_ptr: int = 0) -> int:
    return lib().fvib_step_adjoint(h, C.byref(fin), C.byref(bar_out), C.c_void_p(dF_ptr),
                                   C.byref(bar_in), C.c_void_p(info_ptr))


def fvib_loss_wall_shear(h, u0_ptr: int, J_ptr: int, ubar_ptr: int = 0) -> int:
    return lib().fvib_loss_wall_shear(h, C.c_void_p(u0_ptr), C.c_void_p(J_ptr),
                                      C.c_void_p(ubar_ptr))


def fvib_loss_wall_shear_noalloc(h, u0_ptr: int, J_ptr: int, ubar_ptr: int = 0) -> int:
    return lib().fvib_loss_wall_shear_noalloc(h, C.c_void_p(u0_ptr), C.c_void_p(J_ptr),
                                              C.c_void_p(ubar_ptr))


def fvib_loss_rms_lift(h, Fh_ptr: int, nsteps: int, stride: int, offset: int, u_ref: float,
                       diameter: float, J_ptr: int, dFh_ptr: int = 0) -> int:
    return lib().fvib_loss_rms_lift(h, C.c_void_p(Fh_ptr), nsteps, stride, offset, u_ref,
                                    diameter, C.c_void_p(J_ptr), C.c_void_p(dFh_ptr))


def fvib_last_error(h=None) -> str:
    return lib().fvib_last_error(h).decode()


def fvib_version() -> str:
    return lib().fvib_version().decode()


# ------------------------------------------------------------------ Grid
INFO_DOUBLES = 8      # fvib_step_info is 64 bytes


def parse_info(t: torch.Tensor) -> dict:
    """Decode one or more fvib_step_info records held in a float64 tensor."""
    raw = t.detach().cpu().contiguous().view(-1, INFO_DOUBLES)
    ints = raw.view(torch.int32).view(-1, 2 * INFO_DOUBLES)
    out = []
    for r in range(raw.shape[0]):
        fl = int(ints[r, 3])
        out.append({"status": int(ints[r, 0]), "cg_iters": int(ints[r, 1]),
                    "ir_iters": int(ints[r, 2]), "flags": fl, "clamp": fl & 1,
                    "coupling_iters": (fl >> 8) & 0xFFFF,
                    "res": float(raw[r, 2]), "div_max": float(raw[r, 3]),
                    "force": [float(raw[r, 4]), float(raw[r, 5]), float(raw[r, 6])],
                    "xi": float(raw[r, 7])})
    return out[0] if len(out) == 1 else out


class Grid:
    """A libfvib grid handle bound to the current HIP stream of `device`."""

    def __init__(self, dim: int, n: Sequence[int], faces: Sequence[np.ndarray],
                 bc: Sequence[Sequence[str]], bc_vel=None, nu: float = 0.01, rho: float = 1.0,
                 dt: float = 1e-3, u_conv: float = 1.0, convection: str = "central",
                 precision: str = "fp64", poisson_tol: float = 1e-10,
                 poisson_maxit: int = 100000, ir_maxit: int = 30, inner_rtol: float = 1e-4,
                 check_every: int = 64, solver: str = "fdm", device: str = "cuda:0"):
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dim = int(dim)
        self.n = tuple(int(x) for x in n)
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        d = _abi.GridDesc()
        d.dim = self.dim
        for a in range(3):
            d.n[a] = self.n[a]
        self._faces = []
        for a in range(self.dim):
            f = np.ascontiguousarray(np.asarray(faces[a], dtype=np.float64))
            self._faces.append(f)
            d.faces[a] = f.ctypes.data
        for a in range(3):
            for s in range(2):
                d.bc[a][s] = BC[bc[a][s]] if a < self.dim else 0
        bv = np.zeros((3, 2, 3)) if bc_vel is None else np.asarray(bc_vel, dtype=np.float64)
        for a in range(3):
            for s in range(2):
                for c in range(3):
                    d.bc_vel[a][s][c] = float(bv[a, s, c])
        d.nu, d.rho, d.dt, d.u_conv = nu, rho, dt, u_conv
        d.convection = CONV[convection]
        d.precision = PREC[precision]
        d.poisson_tol = poisson_tol
        d.poisson_maxit = poisson_maxit
        d.ir_maxit = ir_maxit
        d.inner_rtol = inner_rtol
        d.check_every = check_every
        d.solver = SOLVER[solver]
        self.solver = solver
        self.desc = d
        self.nu, self.rho, self.dt = nu, rho, dt
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.h = fvib_create_grid(d, self.stream.cuda_stream)
        self.layouts = [fvib_field_layout(self.h, c) for c in range(self.dim)]
        self.pshape = fvib_field_layout(self.h, 3)[0]
        self.has_body = False
        self.has_box = False
        self.has_les = False
        self._info = torch.zeros(INFO_DOUBLES, dtype=torch.float64, device=self.device)

    @classmethod
    def from_workload(cls, w, **kw):
        """Build from any object with the attributes of a workload description."""
        args = dict(dim=w.dim, n=w.n, faces=w.faces, bc=w.bc, bc_vel=w.bc_vel, nu=w.nu,
                    rho=w.rho, dt=w.dt, u_conv=w.u_conv, convection=w.conv,
                    precision=w.precision)
        args.update(kw)
        g = cls(**args)
        if w.body is not None:
            b = w.body
            g.set_body(b.kind, b.X0, b.ds, b.free_dof, b.m)
        if getattr(w, "box", None) is not None:
            g.set_box(w.box[0], w.box[1])
        if getattr(w, "les", None) is not None:
            g.set_les(**w.les)
        return g

    def close(self):
        if getattr(self, "h", None):
            fvib_destroy_grid(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ tensors
    def zeros_u(self, dtype=None) -> List[torch.Tensor]:
        dt = self.dtype if dtype is None else dtype
        return [torch.zeros(self.layouts[c][0], dtype=dt, device=self.device) for c in range(self.dim)]

    def zeros_p(self) -> torch.Tensor:
        return torch.zeros(self.pshape, dtype=torch.float64, device=self.device)

    def to_u(self, arrays) -> List[torch.Tensor]:
        out = []
        for c in range(self.dim):
            t = torch.as_tensor(np.asarray(arrays[c]), dtype=self.dtype).to(self.device).contiguous()
            assert tuple(t.shape) == tuple(self.layouts[c][0]), (t.shape, self.layouts[c][0])
            out.append(t)
        return out

    def _check_u(self, u, name="u"):
        if u is None or len(u) != self.dim:
            raise ValueError(f"{name} needs {self.dim} components")
        for c in range(self.dim):
            t = u[c]
            if not isinstance(t, torch.Tensor) or tuple(t.shape) != tuple(self.layouts[c][0]) \
                    or t.dtype != self.dtype or not t.is_contiguous() or t.device != self.device:
                raise ValueError(f"{name}[{c}] must be a contiguous {self.dtype} tensor of shape "
                                 f"{self.layouts[c][0]} on {self.device}")

    def _check_comp(self, t, c, name):
        """One velocity-like component c: contiguous, grid dtype and shape."""
        if not isinstance(t, torch.Tensor) or tuple(t.shape) != tuple(self.layouts[c][0]) \
                or t.dtype != self.dtype or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape "
                             f"{self.layouts[c][0]} on {self.device}")

    def _check_t(self, t, name, shape=None, min_numel=None, required=True):
        """A float64 tensor passed by pointer: contiguous, on the grid's
        device, of the given shape or with at least min_numel elements.
        Raises ValueError before anything is launched."""
        if t is None:
            if required:
                raise ValueError(f"{name} is required")
            return
        ok = isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_contiguous() \
            and t.device == self.device
        if ok and shape is not None:
            ok = tuple(t.shape) == tuple(shape)
        if ok and min_numel is not None:
            ok = t.numel() >= min_numel
        if not ok:
            what = f"shape {tuple(shape)}" if shape is not None else f">= {min_numel} elements"
            raise ValueError(f"{name} must be a contiguous float64 tensor with {what} on "
                             f"{self.device}")

    # ------------------------------------------------------------ body
    def set_box(self, lo, hi) -> None:
        """Static immersed box (3D grids): half-open [lo, hi) per axis
        (fvib_ib_set_box); lo = None removes it."""
        if lo is None:
            _check(lib().fvib_ib_set_box(self.h, None, None), self.h)
            self.has_box = False
            return
        lo_a = (C.c_double * 3)(*[float(x) for x in lo])
        hi_a = (C.c_double * 3)(*[float(x) for x in hi])
        _check(lib().fvib_ib_set_box(self.h, lo_a, hi_a), self.h)
        self.has_box = True

    def set_les(self, cs: Optional[float], wall_model: bool = False, kappa: float = 0.4,
                B: float = 5.0, eps: float = 1e-6) -> None:
        """Constant Smagorinsky subgrid model, with the equilibrium wall
        model on the y walls if wall_model (fvib_les_set); cs = None turns
        the model off."""
        if cs is None:
            _check(lib().fvib_les_set(self.h, None), self.h)
            self.has_les = False
            return
        d = _abi.LesDesc()
        d.cs = float(cs)
        d.wall_model = 1 if wall_model else 0
        d.reserved = 0
        d.kappa, d.B, d.eps = float(kappa), float(B), float(eps)
        _check(lib().fvib_les_set(self.h, C.byref(d)), self.h)
        self.has_les = True

    def set_body(self, kind: str, X0, ds, free_dof=(0, 0, 0), m: float = 1.0):
        X0 = np.ascontiguousarray(np.asarray(X0, dtype=np.float64))
        ds = np.ascontiguousarray(np.asarray(ds, dtype=np.float64))
        b = _abi.BodyDesc()
        b.kind = BODY[kind]
        b.n_markers = int(X0.shape[0])
        b.X0 = X0.ctypes.data
        b.ds = ds.ctypes.data
        for a in range(3):
            b.free_dof[a] = int(free_dof[a])
        b.m = float(m)
        fvib_ib_set_body(self.h, b)
        self.has_body = True

    # ------------------------------------------------------------ step
    def _fields(self, u, p, fb=None, body=None, kc=None) -> _abi.Fields:
        f = _abi.Fields()
        for c in range(self.dim):
            f.u[c] = _ptr(u[c])
            f.fb[c] = _ptr(fb[c]) if fb is not None else 0
        f.p = _ptr(p)
        f.body = _ptr(body)
        f.kc = _ptr(kc)
        return f

    def step(self, u, p, fb=None, body=None, kc=None, u_out=None, p_out=None, body_out=None,
             info: Optional[torch.Tensor] = None, check: bool = True, coupling=None,
             omega: Optional[torch.Tensor] = None, scheme: Optional[str] = None) -> int:
        """One time step; in place unless *_out are given.  Returns the status.
        coupling = (max_iters, tol) makes it the strongly coupled step
        (fvib_step_strong); omega (6 doubles) then receives the iterate the
        fluid saw last, which its adjoint needs.  scheme ("fe", "rk2", "rk3")
        makes it an explicit Runge-Kutta step (fvib_step_rk)."""
        self._check_u(u)
        if fb is not None:
            self._check_u(fb, "fb")
        u_out = u if u_out is None else u_out
        p_out = p if p_out is None else p_out
        body_out = body if body_out is None else body_out
        self._check_u(u_out, "u_out")
        self._check_t(p, "p", shape=self.pshape)
        self._check_t(p_out, "p_out", shape=self.pshape)
        self._check_t(body, "body", min_numel=6, required=self.has_body)
        self._check_t(body_out, "body_out", min_numel=6, required=self.has_body)
        self._check_t(kc, "kc", min_numel=6, required=False)
        self._check_t(info, "info", min_numel=INFO_DOUBLES, required=False)
        self._check_t(omega, "omega", min_numel=6, required=False)
        fin = self._fields(u, p, fb, body, kc)
        fout = self._fields(u_out, p_out, fb, body_out, kc)
        ip = _ptr(info if info is not None else self._info)
        if scheme is not None:
            if coupling is not None:
                raise ValueError("a Runge-Kutta step has no coupling iterations")
            rc = fvib_step_rk(self.h, fin, fout, _abi.TIME[scheme], ip)
        elif coupling is None:
            rc = fvib_step(self.h, fin, fout, ip)
        else:
            nmax, tol = coupling
            rc = fvib_step_strong(self.h, fin, fout, nmax, tol, _ptr(omega), ip)
        if check:
            _check(rc, self.h)
        return rc

    def last_info(self) -> dict:
        return parse_info(self._info)

    # --------------------------------------------------------- adjoint
    def step_adjoint(self, u, fb, body, kc, ubar_out, bodybar_out, dF, ubar_in, bodybar_in,
                     fbbar=None, kcbar=None, check: bool = True,
                     info: Optional[torch.Tensor] = None,
                     mu: Optional[torch.Tensor] = None,
                     omega: Optional[torch.Tensor] = None, scheme: Optional[str] = None,
                     p: Optional[torch.Tensor] = None) -> int:
        """Adjoint of one step (fvib_step_adjoint).  mu (optional, float64,
        pressure layout) warm-starts the adjoint Poisson solve and receives
        its solution.  With omega (the iterate a strongly coupled step
        returned) it is the adjoint of that step (fvib_step_strong_adjoint)."""
        self._check_u(u)
        if fb is not None:
            self._check_u(fb, "fb")
        self._check_u(ubar_out, "ubar_out")
        self._check_u(ubar_in, "ubar_in")
        if fbbar is not None:
            self._check_u(fbbar, "fbbar")
        self._check_t(body, "body", min_numel=6, required=self.has_body)
        self._check_t(kc, "kc", min_numel=6, required=False)
        self._check_t(bodybar_out, "bodybar_out", min_numel=6, required=False)
        self._check_t(bodybar_in, "bodybar_in", min_numel=6, required=self.has_body)
        self._check_t(kcbar, "kcbar", min_numel=6, required=False)
        self._check_t(dF, "dF", min_numel=3, required=False)
        self._check_t(mu, "mu", shape=self.pshape, required=False)
        self._check_t(info, "info", min_numel=INFO_DOUBLES, required=False)
        fin = self._fields(u, None, fb, body, kc)
        fin.p = 0
        bo = _abi.Adjoint()
        bi = _abi.Adjoint()
        for c in range(self.dim):
            bo.u[c] = _ptr(ubar_out[c])
            bi.u[c] = _ptr(ubar_in[c])
            bi.fb[c] = _ptr(fbbar[c]) if fbbar is not None else 0
        bo.body = _ptr(bodybar_out)
        bi.body = _ptr(bodybar_in)
        bi.kc = _ptr(kcbar)
        bi.mu = _ptr(mu)
        ip = _ptr(info if info is not None else self._info)
        if scheme is not None:
            self._check_t(p, "p", shape=self.pshape, required=False)
            fin.p = _ptr(p)
            rc = fvib_step_rk_adjoint(self.h, fin, bo, bi, _abi.TIME[scheme], ip)
        elif omega is None:
            rc = fvib_step_adjoint(self.h, fin, bo, _ptr(dF), bi, ip)
        else:
            self._check_t(omega, "omega", min_numel=6)
            rc = fvib_step_strong_adjoint(self.h, fin, _ptr(omega), bo, _ptr(dF), bi, ip)
        if check:
            _check(rc, self.h)
        return rc

    # --------------------------------------------------------- losses
    def loss_wall_shear(self, u0: torch.Tensor, ubar0: Optional[torch.Tensor] = None):
        self._check_comp(u0, 0, "u0")
        if ubar0 is not None:
            self._check_comp(ubar0, 0, "ubar0")
        J = torch.zeros(1, dtype=torch.float64, device=self.device)
        _check(fvib_loss_wall_shear(self.h, _ptr(u0), _ptr(J), _ptr(ubar0)), self.h)
        return J

    def loss_wall_shear_noalloc(self, u0: torch.Tensor, J: torch.Tensor,
                                ubar0: Optional[torch.Tensor] = None) -> None:
        """The allocation-free entry point: J (1 double on the device) and
        ubar0 are the caller's; nothing is allocated by the call."""
        self._check_comp(u0, 0, "u0")
        if ubar0 is not None:
            self._check_comp(ubar0, 0, "ubar0")
        if not (isinstance(J, torch.Tensor) and J.dtype == torch.float64 and J.numel() >= 1
                and J.device == self.device):
            raise ValueError("J must be a float64 tensor of at least 1 element on the grid's device")
        _check(fvib_loss_wall_shear_noalloc(self.h, _ptr(u0), _ptr(J), _ptr(ubar0)), self.h)

    def loss_rms_lift(self, Fh: torch.Tensor, stride: int, offset: int, u_ref: float = 1.0,
                      diameter: float = 1.0, dFh: Optional[torch.Tensor] = None):
        J = torch.zeros(1, dtype=torch.float64, device=self.device)
        nsteps = Fh.numel() // stride
        _check(fvib_loss_rms_lift(self.h, _ptr(Fh), nsteps, stride, offset, u_ref, diameter,
                                  _ptr(J), _ptr(dFh)), self.h)
        return J

    # --------------------------------------------------------- deferred status
    def defer_status(self, on: bool = True) -> None:
        """Steps return once enqueued; their status is only in the info
        records (see check_infos)."""
        _check(lib().fvib_defer_status(self.h, 1 if on else 0), self.h)

    def check_infos(self, infos: torch.Tensor, what: str = "step") -> None:
        """Raise if any fvib_step_info record (rows of a float64 tensor)
        holds a non-zero status (synchronises with the device)."""
        # the records are copied whole (contiguous), then read on the host
        st = infos.reshape(-1, INFO_DOUBLES).cpu().view(torch.int32)[:, 0]
        bad = torch.nonzero(st).flatten()
        if bad.numel():
            n = int(bad[0])
            raise RuntimeError(f"libfvib {what} {n}: status {int(st[n])}")

    # --------------------------------------------------------- timing
    def timing_enable(self, on: bool = True, classes=None, every: int = 1) -> None:
        """Start (totals cleared) or stop event timing; `classes` (names of
        _abi.K_CLASSES) restricts it to those kernel classes, `every` times
        one launch in `every` of each class."""
        mask = 0xFFFFFFFF
        if classes is not None:
            mask = 0
            for name in classes:
                mask |= 1 << _abi.K_CLASSES[name]
        _check(lib().fvib_timing_select(self.h, mask), self.h)
        _check(lib().fvib_timing_sample(self.h, int(every)), self.h)
        _check(lib().fvib_timing_enable(self.h, 1 if on else 0), self.h)

    def timing_read(self, skipped: bool = False) -> dict:
        """{kernel class: (total_ms, launches)} since the last enable; with
        skipped, the launches of refinement sweeps that the device skipped
        (excluded from the default figures)."""
        fn = lib().fvib_timing_read_skipped if skipped else lib().fvib_timing_read
        out = {}
        for name, k in _abi.K_CLASSES.items():
            ms = C.c_double()
            n = C.c_int64()
            _check(fn(self.h, k, C.byref(ms), C.byref(n)), self.h)
            out[name] = (ms.value, n.value)
        return out

    # --------------------------------------------------------- test hooks
    def test_momentum(self, u, fb=None) -> List[torch.Tensor]:
        R = self.zeros_u()
        vp = C.c_void_p * 3
        ua = vp(*([_ptr(u[c]) for c in range(self.dim)] + [0] * (3 - self.dim)))
        fa = vp(*([_ptr(fb[c]) if fb is not None else 0 for c in range(self.dim)] + [0] * (3 - self.dim)))
        ra = vp(*([_ptr(R[c]) for c in range(self.dim)] + [0] * (3 - self.dim)))
        _check(lib().fvib_test_momentum(self.h, ua, fa, ra), self.h)
        return R

    def test_ppe_rhs(self, ustar) -> torch.Tensor:
        b = self.zeros_p()
        vp = C.c_void_p * 3
        ua = vp(*([_ptr(ustar[c]) for c in range(self.dim)] + [0] * (3 - self.dim)))
        _check(lib().fvib_test_ppe_rhs(self.h, ua, _ptr(b)), self.h)
        return b

    def test_poisson(self, b: torch.Tensor, p0: Optional[torch.Tensor] = None):
        p = self.zeros_p() if p0 is None else p0.clone()
        it = C.c_int32()
        _check(lib().fvib_test_poisson(self.h, _ptr(b), _ptr(p), C.byref(it)), self.h)
        return p, it.value

    def test_apply_A(self, p: torch.Tensor) -> torch.Tensor:
        y = torch.empty_like(p)
        _check(lib().fvib_test_apply_A(self.h, _ptr(p), _ptr(y)), self.h)
        return y

    def _arr3(self, ts):
        vp = C.c_void_p * 3
        return vp(*([_ptr(t) for t in ts] + [0] * (3 - len(ts))))

    def test_project(self, ustar, p: torch.Tensor):
        """Eq. 10 alone: returns (u, div_max)."""
        self._check_u(ustar, "ustar")
        self._check_t(p, "p", shape=self.pshape)
        u = self.zeros_u()
        dm = torch.zeros(1, dtype=torch.float64, device=self.device)
        _check(lib().fvib_test_project(self.h, self._arr3(ustar), _ptr(p), self._arr3(u),
                                       _ptr(dm)), self.h)
        return u, float(dm[0])

    def test_project_adjoint(self, ubar) -> torch.Tensor:
        self._check_u(ubar, "ubar")
        pbar = self.zeros_p()
        _check(lib().fvib_test_project_adjoint(self.h, self._arr3(ubar), _ptr(pbar)), self.h)
        return pbar

    def test_ib_target(self, body: torch.Tensor) -> List[torch.Tensor]:
        self._check_t(body, "body", min_numel=6)
        us = self.zeros_u()
        _check(lib().fvib_test_ib_target(self.h, _ptr(body), self._arr3(us)), self.h)
        return us

    def test_ib_target_adjoint(self, body: torch.Tensor, usbar, bodybar: torch.Tensor) -> None:
        self._check_t(body, "body", min_numel=6)
        self._check_u(usbar, "usbar")
        self._check_t(bodybar, "bodybar", min_numel=6)
        _check(lib().fvib_test_ib_target_adjoint(self.h, _ptr(body), self._arr3(usbar),
                                                 _ptr(bodybar)), self.h)

    def test_ib_loads(self, body: torch.Tensor, f) -> torch.Tensor:
        self._check_t(body, "body", min_numel=6)
        self._check_u(f, "f")
        F = torch.zeros(3, dtype=torch.float64, device=self.device)
        _check(lib().fvib_test_ib_loads(self.h, _ptr(body), self._arr3(f), _ptr(F)), self.h)
        return F

    def test_ib_loads_adjoint(self, body: torch.Tensor, f, Fbar: torch.Tensor,
                              bodybar: torch.Tensor) -> List[torch.Tensor]:
        self._check_t(body, "body", min_numel=6)
        self._check_u(f, "f")
        self._check_t(Fbar, "Fbar", min_numel=3)
        self._check_t(bodybar, "bodybar", min_numel=6)
        fbar = self.zeros_u()
        _check(lib().fvib_test_ib_loads_adjoint(self.h, _ptr(body), self._arr3(f), _ptr(Fbar),
                                                self._arr3(fbar), _ptr(bodybar)), self.h)
        return fbar

    def test_body_rk4(self, body: torch.Tensor, F: torch.Tensor, kc: torch.Tensor) -> torch.Tensor:
        for t, n, m in ((body, "body", 6), (F, "F", 3), (kc, "kc", 6)):
            self._check_t(t, n, min_numel=m)
        out = torch.zeros(6, dtype=torch.float64, device=self.device)
        _check(lib().fvib_test_body_rk4(self.h, _ptr(body), _ptr(F), _ptr(kc), _ptr(out)), self.h)
        return out

    def test_body_rk4_adjoint(self, body, F, kc, bodybar_out, kcbar):
        """Returns (bodybar_in, Fbar); adds into kcbar."""
        for t, n, m in ((body, "body", 6), (F, "F", 3), (kc, "kc", 6),
                        (bodybar_out, "bodybar_out", 6), (kcbar, "kcbar", 6)):
            self._check_t(t, n, min_numel=m)
        bin_ = torch.zeros(6, dtype=torch.float64, device=self.device)
        Fbar = torch.zeros(3, dtype=torch.float64, device=self.device)
        _check(lib().fvib_test_body_rk4_adjoint(self.h, _ptr(body), _ptr(F), _ptr(kc),
                                                _ptr(bodybar_out), _ptr(bin_), _ptr(Fbar),
                                                _ptr(kcbar)), self.h)
        return bin_, Fbar

    def set_dt(self, dt: float) -> None:
        """Time step of every later step (fvib_set_dt)."""
        _check(fvib_set_dt(self.h, dt), self.h)
        self.dt = float(dt)

    def cfl_dt(self, u, cfl: float, dt_max: float) -> float:
        """min(dt_max, cfl h_min / max |u|) from a device reduction (fvib_cfl_dt)."""
        self._check_u(u)
        rc, dt = fvib_cfl_dt(self.h, [_ptr(x) for x in u], cfl, dt_max)
        _check(rc, self.h)
        return dt

    def clear_error(self) -> None:
        """Reset the handle after a device-side failure (fvib_clear_error)."""
        _check(lib().fvib_clear_error(self.h), self.h)

    def test_ib_classify(self, body: torch.Tensor) -> List[torch.Tensor]:
        cls = [torch.zeros(self.layouts[c][0], dtype=torch.uint8, device=self.device) for c in range(2)]
        vp = C.c_void_p * 3
        ca = vp(_ptr(cls[0]), _ptr(cls[1]), 0)
        _check(lib().fvib_test_ib_classify(self.h, _ptr(body), ca), self.h)
        return cls
