"""Seeded synthetic workloads for the FV + IBM time step.

This module only *describes* problems: grid face coordinates, boundary
conditions, physical constants, immersed-body markers and initial fields.
It holds none of the solver's arithmetic, so both the CPU oracle and the
GPU path can read the same inputs without sharing any method code.

Workloads (all nondimensional, rho = 1, see the paper's validation cases):

* ``tgv2d``    -- 2D Taylor-Green vortex, periodic, 2pi x 2pi (validation of
                  the fluid solver; analytic decay of the discrete mode).
* ``tgv3d``    -- 3D Taylor-Green vortex, periodic, Re = 1600.
* ``cylinder`` -- 2D flow past a stationary cylinder through direct-forcing
                  IBM, Re = 100, inflow / convective outflow / free-slip
                  lateral walls (Sec. 3.1 of the paper).
* ``channel``  -- 3D plane channel at Re_tau = 180 on a tanh-stretched
                  wall-normal grid, driven by a uniform body force
                  (Sec. 3.4.1 of the paper, Table 4).
* ``wmles``    -- wall-modelled LES of a plane channel, uniform 64^3 grid on
                  2pi x 2 x pi, Re_tau = 2000, constant Smagorinsky model and
                  equilibrium wall model (Sec. 3.4.5, Table 5).
* ``viv``      -- 2D elastically mounted cylinder, 1-DOF transverse spring
                  (or 2-DOF, equal springs in-line and cross-flow), m* = 2,
                  U_r = 5, zeta = 0, Re = 150 (Sec. 3.2, Table 2); weak or
                  strong coupling (Alg. 1 with N sub-iterations at most).

Face arrays use the staggered (MAC) layout: component ``c`` lives on the
faces normal to axis ``c``; arrays are C-contiguous in (z, y, x) order with
x fastest; along its own axis a component has ``N`` faces on a periodic
axis and ``N + 1`` faces otherwise.  2D problems use nz = 1 and two
components.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

BC_NAMES = ("periodic", "noslip", "freeslip", "inflow", "outflow_conv",
            "outflow_neumann")


@dataclass
class Body:
    """Rigid body described by a closed polygon of Lagrangian markers."""
    kind: str                      # "static" or "spring"
    X0: np.ndarray                 # (M, 2) marker positions at zero displacement
    ds: np.ndarray                 # (M,) arc-length element per marker
    free_dof: tuple = (0, 0, 0)    # 1 where the DOF is free (x, y, z)
    m: float = 1.0
    k: tuple = (0.0, 0.0, 0.0)
    c: tuple = (0.0, 0.0, 0.0)
    d0: tuple = (0.0, 0.0, 0.0)    # initial displacement
    v0: tuple = (0.0, 0.0, 0.0)    # initial velocity
    diameter: float = 1.0
    u_ref: float = 1.0
    coupling_iters: int = 1        # sub-iterations per step at most (1 = weak coupling)
    coupling_tol: float = 1e-5     # coupling error that ends the sub-iterations


@dataclass
class Workload:
    name: str
    dim: int
    n: tuple                       # (nx, ny, nz); nz = 1 in 2D
    faces: List[np.ndarray]        # 3 arrays of face coordinates (len n+1)
    bc: List[List[str]]            # bc[axis][side], side 0 = low, 1 = high
    bc_vel: np.ndarray             # (3, 2, 3): velocity vector per boundary
    nu: float
    rho: float
    dt: float
    steps: int
    u_conv: float = 1.0            # convective-outflow speed
    conv: str = "central"          # "central" or "upwind"
    precision: str = "fp64"        # "fp64" or "fp32"
    body: Optional[Body] = None
    # static immersed box (3D grids): ((x0, y0, z0), (x1, y1, z1)), or None
    box: Optional[tuple] = None
    # large-eddy simulation: {"cs": Smagorinsky constant, "wall_model": bool,
    # "kappa", "B": Spalding-law constants, "eps": Eq. 28 regulariser}, or None
    les: Optional[dict] = None
    meta: dict = field(default_factory=dict)

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def face_shape(self, c: int) -> tuple:
        """Shape (nz, ny, nx) of the array holding velocity component c."""
        ext = [self.n[0], self.n[1], self.n[2]]
        if self.bc[c][0] != "periodic":
            ext[c] += 1
        return (ext[2], ext[1], ext[0])

    def cell_shape(self) -> tuple:
        return (self.n[2], self.n[1], self.n[0])


def _uniform(n: int, lo: float, hi: float) -> np.ndarray:
    return lo + (hi - lo) * np.arange(n + 1, dtype=np.float64) / n


def tanh_faces(n: int, gamma: float) -> np.ndarray:
    """Wall-normal faces on [-1, 1]: y_j = tanh(gamma (2j/n - 1)) / tanh(gamma)."""
    s = 2.0 * np.arange(n + 1, dtype=np.float64) / n - 1.0
    y = np.tanh(gamma * s) / math.tanh(gamma)
    y[0], y[-1] = -1.0, 1.0
    return y


def _bcv():
    return np.zeros((3, 2, 3), dtype=np.float64)


def circle_markers(xc: float, yc: float, diameter: float, m: int):
    """M markers uniform in angle on a circle, counter-clockwise."""
    th = 2.0 * np.pi * np.arange(m, dtype=np.float64) / m
    X0 = np.stack([xc + 0.5 * diameter * np.cos(th),
                   yc + 0.5 * diameter * np.sin(th)], axis=1)
    ds = np.full(m, np.pi * diameter / m, dtype=np.float64)
    return X0, ds


# --------------------------------------------------------------------------
# workload constructors
# --------------------------------------------------------------------------

def tgv2d(n: int = 64, steps: int = 100, dt: float = 1e-3, nu: float = 0.01,
          precision: str = "fp64") -> Workload:
    L = 2.0 * np.pi
    faces = [_uniform(n, 0.0, L), _uniform(n, 0.0, L), np.array([0.0, 1.0])]
    bc = [["periodic", "periodic"]] * 2 + [["periodic", "periodic"]]
    return Workload("tgv2d", 2, (n, n, 1), faces, [list(b) for b in bc], _bcv(),
                    nu=nu, rho=1.0, dt=dt, steps=steps, precision=precision)


def tgv3d(n: int = 128, steps: int = 500, dt: float = 1e-3,
          nu: float = 1.0 / 1600.0, precision: str = "fp32") -> Workload:
    L = 2.0 * np.pi
    faces = [_uniform(n, 0.0, L) for _ in range(3)]
    bc = [["periodic", "periodic"] for _ in range(3)]
    return Workload("tgv3d", 3, (n, n, n), faces, bc, _bcv(), nu=nu, rho=1.0,
                    dt=dt, steps=steps, precision=precision)


def channel(nx: int = 192, ny: int = 128, nz: int = 160, steps: int = 200,
            dt: float = 1e-5, gamma: float = 1.45, precision: str = "fp32",
            seed: int = 20250530) -> Workload:
    faces = [_uniform(nx, 0.0, 2.0 * np.pi), tanh_faces(ny, gamma),
             _uniform(nz, 0.0, np.pi)]
    bc = [["periodic", "periodic"], ["noslip", "noslip"], ["periodic", "periodic"]]
    cf = 8.0e-3
    w = Workload("channel", 3, (nx, ny, nz), faces, bc, _bcv(), nu=1.0 / 180.0,
                 rho=1.0, dt=dt, steps=steps, precision=precision,
                 meta={"seed": seed, "u_bulk": math.sqrt(2.0 / cf),
                       "fb": (1.0, 0.0, 0.0), "perturb": 0.1})
    return w


def wmles(n: int = 64, re_tau: float = 2000.0, cs: float = 0.1, steps: int = 100,
          dt: float = 1e-3, wall_model: bool = True, precision: str = "fp32",
          seed: int = 20250531, kappa: float = 0.4, B: float = 5.0,
          eps: float = 1e-6) -> Workload:
    """Wall-modelled LES of a plane channel (Sec. 3.4.5, Table 5): uniform
    n^3 grid on 2pi x 2 x pi, nu = 1 / Re_tau (u_tau = 1, half height 1),
    driven by the uniform body force 1 that balances the mean wall stress."""
    faces = [_uniform(n, 0.0, 2.0 * np.pi), _uniform(n, -1.0, 1.0), _uniform(n, 0.0, np.pi)]
    bc = [["periodic", "periodic"], ["noslip", "noslip"], ["periodic", "periodic"]]
    w = Workload("wmles", 3, (n, n, n), faces, bc, _bcv(), nu=1.0 / re_tau, rho=1.0,
                 dt=dt, steps=steps, precision=precision,
                 les={"cs": cs, "wall_model": wall_model, "kappa": kappa, "B": B, "eps": eps},
                 meta={"seed": seed, "re_tau": re_tau, "fb": (1.0, 0.0, 0.0), "perturb": 0.1})
    return w


def channel_cube(nx: int = 192, ny: int = 128, nz: int = 160, steps: int = 200,
                 dt: float = 1e-5, precision: str = "fp32") -> Workload:
    """The channel with one cube-like roughness element standing on its
    floor (Sec. 3.4.2 places a layer of cubes on the wall): a box 0.4 wide
    in x and z reaching from the lower wall to y = -0.6."""
    w = channel(nx=nx, ny=ny, nz=nz, steps=steps, dt=dt, precision=precision)
    w.name = "channel"              # same initial fields
    w.box = ((2.0, -1.5, 1.2), (2.4, -0.6, 1.6))
    w.meta["variant"] = "cube"
    return w


def cylinder(nx: int = 512, ny: int = 256, steps: int = 5000, dt: float = 5e-3,
             markers: int = 160, re: float = 100.0, precision: str = "fp32",
             lx: float = 32.0, ly: float = 16.0, center=(8.0, 8.0)) -> Workload:
    faces = [_uniform(nx, 0.0, lx), _uniform(ny, 0.0, ly), np.array([0.0, 1.0])]
    bc = [["inflow", "outflow_conv"], ["freeslip", "freeslip"],
          ["periodic", "periodic"]]
    bcv = _bcv()
    bcv[0, 0, 0] = 1.0                                 # uniform inflow u = 1
    X0, ds = circle_markers(center[0], center[1], 1.0, markers)
    body = Body("static", X0, ds)
    return Workload("cylinder", 2, (nx, ny, 1), faces, bc, bcv, nu=1.0 / re,
                    rho=1.0, dt=dt, steps=steps, u_conv=1.0, precision=precision,
                    body=body)


def viv(nx: int = 1024, ny: int = 512, steps: int = 4000, dt: float = 4e-3,
        markers: int = 256, re: float = 150.0, mass_ratio: float = 2.0,
        u_r: float = 5.0, zeta: float = 0.0, d0: float = 0.1,
        precision: str = "fp32", lx: float = 32.0, ly: float = 16.0,
        center=(8.0, 8.0), dof: int = 1, coupling_iters: int = 1,
        coupling_tol: float = 1e-5) -> Workload:
    w = cylinder(nx=nx, ny=ny, steps=steps, dt=dt, markers=markers, re=re,
                 precision=precision, lx=lx, ly=ly, center=center)
    D = 1.0
    m = mass_ratio * np.pi * D * D / 4.0               # rho = 1
    fn = 1.0 / (D * u_r)                               # U = 1
    k = m * (2.0 * np.pi * fn) ** 2
    c = 2.0 * m * (2.0 * np.pi * fn) * zeta
    w.name = "viv"
    if dof == 1:          # transverse (cross-flow) spring only
        free, kk, cc = (0, 1, 0), (0.0, k, 0.0), (0.0, c, 0.0)
    elif dof == 2:        # equal springs in-line and cross-flow (Sec. 3.2.2)
        free, kk, cc = (1, 1, 0), (k, k, 0.0), (c, c, 0.0)
    else:
        raise ValueError(dof)
    w.body = Body("spring", w.body.X0, w.body.ds, free_dof=free, m=m, k=kk, c=cc,
                  d0=(0.0, d0, 0.0), coupling_iters=coupling_iters, coupling_tol=coupling_tol)
    w.meta.update({"fn": fn, "mass_ratio": mass_ratio, "u_r": u_r, "dof": dof})
    return w


def generic(dim: int, n: tuple, faces, bc, bc_vel=None, nu=0.01, dt=1e-3,
            steps=1, conv="central", precision="fp64", u_conv=1.0, body=None,
            name="generic") -> Workload:
    """Free-form workload for tests (walls, stretching, upwinding, ...)."""
    bcv = _bcv() if bc_vel is None else np.asarray(bc_vel, dtype=np.float64)
    faces = [np.asarray(f, dtype=np.float64) for f in faces]
    if dim == 2:
        faces = faces[:2] + [np.array([0.0, 1.0])]
        bc = [list(bc[0]), list(bc[1]), ["periodic", "periodic"]]
    return Workload(name, dim, tuple(n), faces, [list(b) for b in bc], bcv,
                    nu=nu, rho=1.0, dt=dt, steps=steps, u_conv=u_conv,
                    conv=conv, precision=precision, body=body)


# --------------------------------------------------------------------------
# initial fields (values only: analytic profiles and seeded noise)
# --------------------------------------------------------------------------

def centres(f: np.ndarray) -> np.ndarray:
    return 0.5 * (f[:-1] + f[1:])


def face_points(w: Workload, c: int):
    """Coordinates (x, y, z) broadcastable to the shape of component c."""
    pts = []
    for a in range(3):
        f = w.faces[a]
        if a == c:
            p = f if w.bc[a][0] != "periodic" else f[:-1]
        else:
            p = centres(f)
        shape = [1, 1, 1]
        shape[2 - a] = p.size
        pts.append(p.reshape(shape))
    return pts


def initial_fields(w: Workload):
    """Return (u, fb): lists of `dim` float64 arrays in the face layout."""
    ncomp = w.dim
    u = [np.zeros(w.face_shape(c)) for c in range(ncomp)]
    fb = [np.zeros(w.face_shape(c)) for c in range(ncomp)]
    if w.name == "tgv2d":
        x, y, _ = face_points(w, 0)
        u[0] = np.broadcast_to(np.sin(x) * np.cos(y), u[0].shape).copy()
        x, y, _ = face_points(w, 1)
        u[1] = np.broadcast_to(-np.cos(x) * np.sin(y), u[1].shape).copy()
    elif w.name == "tgv3d":
        x, y, z = face_points(w, 0)
        u[0] = np.broadcast_to(np.sin(x) * np.cos(y) * np.cos(z), u[0].shape).copy()
        x, y, z = face_points(w, 1)
        u[1] = np.broadcast_to(-np.cos(x) * np.sin(y) * np.cos(z), u[1].shape).copy()
    elif w.name == "channel":
        ub = w.meta["u_bulk"]
        _, y, _ = face_points(w, 0)
        u[0] = np.broadcast_to(1.5 * ub * (1.0 - y * y), u[0].shape).copy()
        rng = np.random.default_rng(w.meta["seed"])
        amp = w.meta["perturb"] * ub
        for c in range(3):
            xi = rng.random(u[c].shape)
            pert = amp * (2.0 * xi - 1.0)
            if c == 1:                    # wall-normal faces on the walls stay 0
                pert[:, 0, :] = 0.0
                pert[:, -1, :] = 0.0
            u[c] = u[c] + pert
        for c in range(3):
            fb[c][...] = w.meta["fb"][c]
    elif w.name == "wmles":
        # Reichardt's mean profile in wall units (u_tau = 1) plus seeded noise
        re = w.meta["re_tau"]
        _, y, _ = face_points(w, 0)
        yp = (1.0 - np.abs(y)) * re
        k = 0.41
        up = np.log1p(k * yp) / k + 7.8 * (1.0 - np.exp(-yp / 11.0) - yp / 11.0 * np.exp(-yp / 3.0))
        u[0] = np.broadcast_to(up, u[0].shape).copy()
        rng = np.random.default_rng(w.meta["seed"])
        amp = w.meta["perturb"] * float(up.mean())
        for c in range(3):
            pert = amp * (2.0 * rng.random(u[c].shape) - 1.0)
            if c == 1:
                pert[:, 0, :] = 0.0
                pert[:, -1, :] = 0.0
            u[c] = u[c] + pert
        for c in range(3):
            fb[c][...] = w.meta["fb"][c]
    elif w.name in ("cylinder", "viv"):
        u[0][...] = w.bc_vel[0, 0, 0]
    return u, fb


def body_state0(w: Workload) -> np.ndarray:
    """Body state vector [d_x, d_y, d_z, v_x, v_y, v_z] (float64)."""
    s = np.zeros(6, dtype=np.float64)
    if w.body is not None:
        s[:3] = w.body.d0
        s[3:] = w.body.v0
    return s


def random_fields(w: Workload, seed: int, scale: float = 1.0):
    """Seeded uniform(-scale, scale) arrays in the face layout (test inputs)."""
    rng = np.random.default_rng(seed)
    return [scale * (2.0 * rng.random(w.face_shape(c)) - 1.0) for c in range(w.dim)]


def random_cells(w: Workload, seed: int, scale: float = 1.0):
    rng = np.random.default_rng(seed)
    return scale * (2.0 * rng.random(w.cell_shape()) - 1.0)


def by_name(name: str, size: str = "full") -> Workload:
    """Named workloads at full size or reduced sizes for parity tests."""
    if name == "tgv2d":
        return tgv2d() if size == "full" else tgv2d(n=32, steps=20)
    if name == "tgv3d":
        return tgv3d() if size == "full" else tgv3d(n=24, steps=10)
    if name == "channel":
        return channel() if size == "full" else channel(nx=24, ny=16, nz=20, steps=10)
    if name == "channel_cube":
        return channel_cube() if size == "full" else channel_cube(nx=24, ny=16, nz=20, steps=10)
    if name == "wmles":
        return wmles() if size == "full" else wmles(n=16, steps=5)
    if name == "cylinder":
        if size == "full":
            return cylinder()
        return cylinder(nx=128, ny=64, steps=20, markers=40)
    if name == "viv":
        if size == "full":
            return viv()
        return viv(nx=256, ny=128, steps=20, markers=64, dt=4e-3)
    if name == "viv2dof":       # 2-DOF, strongly coupled (Alg. 1, N <= 100, tol 1e-5)
        if size == "full":
            return viv(dof=2, coupling_iters=100)
        return viv(nx=256, ny=128, steps=20, markers=64, dt=4e-3, dof=2, coupling_iters=100)
    raise KeyError(name)
