"""Pins of the oracle's static 3D immersed box (oracle/ibm3d.py):

* a box spanning a z-periodic domain gives, plane by plane, the flow of the
  2D step with a static square body (the pinned polygon classification and
  2D step), with w = 0;
* from rest under a uniform body force the first step's force is
  rho f_b times the forced volume, whose face count follows from the box's
  cell range in closed form;
* the corrected field is divergence free with a body present;
* the gradient through box steps equals central differences.
"""
import numpy as np
import pytest
import torch

import fvib_workloads as W
from oracle import Grid, fluid, init_state, make_params, step
from oracle.step import rollout

F64 = torch.float64


def _square_body(x0, y0, x1, y1, per_side=8):
    pts = []
    for t in np.linspace(0, 1, per_side, endpoint=False):
        pts.append((x0 + t * (x1 - x0), y0))
    for t in np.linspace(0, 1, per_side, endpoint=False):
        pts.append((x1, y0 + t * (y1 - y0)))
    for t in np.linspace(0, 1, per_side, endpoint=False):
        pts.append((x1 - t * (x1 - x0), y1))
    for t in np.linspace(0, 1, per_side, endpoint=False):
        pts.append((x0, y1 - t * (y1 - y0)))
    X0 = np.asarray(pts)
    ds = np.full(len(pts), 2 * ((x1 - x0) + (y1 - y0)) / len(pts))
    return W.Body("static", X0, ds)


def test_extruded_box_equals_2d_square():
    nx, ny, nz = 32, 16, 4
    fx, fy, fz = np.linspace(0, 4, nx + 1), np.linspace(0, 2, ny + 1), np.linspace(0, 1, nz + 1)
    bcv = np.zeros((3, 2, 3))
    bcv[0, 0, 0] = 1.0
    bc2 = [["inflow", "outflow_conv"], ["freeslip", "freeslip"]]
    x0, y0, x1, y1 = 1.03, 0.71, 1.58, 1.29
    w2 = W.generic(2, (nx, ny, 1), [fx, fy, fz], bc2, bc_vel=bcv, nu=0.02, dt=2e-3,
                   body=_square_body(x0, y0, x1, y1))
    w3 = W.generic(3, (nx, ny, nz), [fx, fy, fz], bc2 + [["periodic", "periodic"]], bc_vel=bcv,
                   nu=0.02, dt=2e-3)
    w3.box = ((x0, y0, -1.0), (x1, y1, 2.0))
    g2, g3 = Grid(w2), Grid(w3)
    rng = np.random.default_rng(4)
    u2 = [1.0 + 0.1 * rng.standard_normal(g2.face_shape(0)),
          0.1 * rng.standard_normal(g2.face_shape(1))]
    u3 = [np.repeat(u2[0], nz, axis=0), np.repeat(u2[1], nz, axis=0),
          np.zeros(g3.face_shape(2))]
    with torch.no_grad():
        s2, F2, _ = rollout(g2, init_state(g2, u2), make_params(g2), 5)
        s3, F3, _ = rollout(g3, init_state(g3, u3), make_params(g3), 5)
    for k in range(nz):
        for c in range(2):
            d = float((s3["u"][c][k] - s2["u"][c][0]).abs().max())
            assert d < 1e-12, (k, c, d)
        assert float((s3["p"][k] - s2["p"][0]).abs().max()) < 1e-10 * float(s2["p"].abs().max())
    assert float(s3["u"][2].abs().max()) < 1e-13
    # the forced faces are the square's (the body is there)
    assert float(F3.abs().max()) > 0.0


def test_force_from_rest_closed_form():
    n, L = 16, 2.0
    h = L / n
    f = np.linspace(0, L, n + 1)
    w = W.generic(3, (n, n, n), [f, f, f], [["periodic", "periodic"]] * 3, nu=0.05, dt=1e-3)
    i0, i1, j0, j1, k0, k1 = 5, 9, 6, 11, 4, 7
    w.box = (((i0 - 0.25) * h, (j0 - 0.25) * h, (k0 - 0.25) * h),
             ((i1 - 0.25) * h, (j1 - 0.25) * h, (k1 - 0.25) * h))
    g = Grid(w)
    fb_c = (0.7, -0.4, 1.3)
    fb = [np.full(g.face_shape(c), fb_c[c]) for c in range(3)]
    u0 = [np.zeros(g.face_shape(c)) for c in range(3)]
    with torch.no_grad():
        _, aux = step(g, init_state(g, u0), make_params(g, fb))
    nx_, ny_, nz_ = i1 - i0, j1 - j0, k1 - k0
    count = nx_ * ny_ * nz_ + 2 * (ny_ * nz_ + nx_ * nz_ + nx_ * ny_)
    for c in range(3):
        exact = w.rho * fb_c[c] * h ** 3 * count
        assert abs(float(aux["F"][c]) - exact) <= 1e-12 * abs(exact), (c, float(aux["F"][c]), exact)
        assert int(aux["eps"][c].sum()) == count


def test_force_from_rest_box_on_wall():
    """A box standing on the lower wall (the roughness cubes of Sec. 3.4.2):
    the six-neighbour shell has no layer below the wall, and the wall-normal
    faces on the wall keep their boundary condition, so they are not forced."""
    n, L = 16, 2.0
    h = L / n
    f = np.linspace(0, L, n + 1)
    bc = [["periodic", "periodic"], ["noslip", "noslip"], ["periodic", "periodic"]]
    w = W.generic(3, (n, n, n), [f, f, f], bc, nu=0.05, dt=1e-3)
    i0, i1, j1, k0, k1 = 5, 9, 4, 3, 7
    w.box = (((i0 - 0.25) * h, -0.5, (k0 - 0.25) * h), ((i1 - 0.25) * h, (j1 - 0.25) * h,
                                                       (k1 - 0.25) * h))
    g = Grid(w)
    fb_c = (0.7, -0.4, 1.3)
    fb = [np.full(g.face_shape(c), fb_c[c]) for c in range(3)]
    u0 = [np.zeros(g.face_shape(c)) for c in range(3)]
    with torch.no_grad():
        _, aux = step(g, init_state(g, u0), make_params(g, fb))
    nx_, ny_, nz_ = i1 - i0, j1, k1 - k0
    total = nx_ * ny_ * nz_ + 2 * ny_ * nz_ + 2 * nx_ * ny_ + nx_ * nz_
    count = [total, total - (nx_ * nz_ + 2 * nz_ + 2 * nx_), total]
    for c in range(3):
        exact = w.rho * fb_c[c] * h ** 3 * count[c]
        assert int(aux["eps"][c].sum()) == count[c], (c, int(aux["eps"][c].sum()), count[c])
        assert abs(float(aux["F"][c]) - exact) <= 1e-12 * abs(exact), (c, float(aux["F"][c]), exact)


def test_divergence_free_with_box():
    w = W.channel(nx=16, ny=12, nz=10, steps=1, dt=1e-5)
    w.box = ((2.0, -0.5, 1.0), (3.2, 0.3, 2.2))
    g = Grid(w)
    u0, fb = W.initial_fields(w)
    with torch.no_grad():
        st, aux = step(g, init_state(g, u0), make_params(g, fb))
    d = fluid.divergence(g, st["u"])
    scale = max(float(x.abs().max()) for x in st["u"]) / float(min(x.min() for x in g.dx))
    assert float(d.abs().max()) < 1e-11 * scale
    assert int(sum(e.sum() for e in aux["eps"])) > 0


def test_box_gradient_vs_central_differences():
    n = 8
    f = np.linspace(0, 2.0, n + 1)
    w = W.generic(3, (n, n, n), [f, f, f], [["periodic", "periodic"]] * 3, nu=0.05, dt=2e-3)
    w.box = ((0.6, 0.7, 0.55), (1.2, 1.3, 1.1))
    g = Grid(w)
    u0 = W.random_fields(w, 3)
    rng = np.random.default_rng(8)
    ub = [torch.tensor(rng.standard_normal(g.face_shape(c))) for c in range(3)]
    Fb = torch.tensor(rng.standard_normal(3))
    fbv = [0.1 * rng.standard_normal(g.face_shape(c)) for c in range(3)]

    def J(fb):
        st, Fh, _ = rollout(g, init_state(g, u0), make_params(g, fb), 3)
        return sum((a * b).sum() for a, b in zip(st["u"], ub)) + (Fh.sum(0) * Fb).sum()

    fbt = [torch.tensor(x, requires_grad=True) for x in fbv]
    J(fbt).backward()
    for comp, idx in ((0, (1, 2, 3)), (2, (4, 4, 1)), (1, (3, 3, 3))):
        d = 1e-6
        vals = []
        for s in (+1, -1):
            arr = [x.copy() for x in fbv]
            arr[comp][idx] += s * d
            with torch.no_grad():
                vals.append(float(J(arr)))
        fd = (vals[0] - vals[1]) / (2 * d)
        ad = float(fbt[comp].grad[idx])
        assert abs(fd - ad) <= 1e-7 * max(1.0, abs(fd)), (comp, idx, fd, ad)


def test_force_from_rest_stretched_volumes():
    """The same closed form on the tanh-stretched channel grid: the forced
    faces are the box's index range plus its six-neighbour shell, and each
    face's volume is its centre spacing along the component's axis times
    the transverse cell widths, computed here from the face coordinates."""
    w = W.channel(nx=16, ny=12, nz=10, steps=1, dt=1e-5)
    f = [np.asarray(w.faces[a]) for a in range(3)]
    xc = [0.5 * (x[1:] + x[:-1]) for x in f]
    rng = [(5, 9), (3, 7), (4, 7)]                       # cell index ranges per axis
    lo = tuple(0.5 * (xc[a][rng[a][0] - 1] + f[a][rng[a][0]]) for a in range(3))
    hi = tuple(0.5 * (xc[a][rng[a][1] - 1] + f[a][rng[a][1]]) for a in range(3))
    w.box = (lo, hi)
    g = Grid(w)
    fb_c = (0.9, -0.6, 0.4)
    fb = [np.full(g.face_shape(c), fb_c[c]) for c in range(3)]
    u0 = [np.zeros(g.face_shape(c)) for c in range(3)]
    with torch.no_grad():
        _, aux = step(g, init_state(g, u0), make_params(g, fb))
    width = [x[1:] - x[:-1] for x in f]
    for c in range(3):
        forced = set()
        I = [range(*rng[a]) for a in range(3)]
        for i in I[0]:
            for j in I[1]:
                for k in I[2]:
                    forced.add((i, j, k))
        shell = set()
        for (i, j, k) in forced:
            for a in range(3):
                for s in (-1, 1):
                    q = [i, j, k]
                    q[a] += s
                    if tuple(q) not in forced:
                        shell.add(tuple(q))
        total = 0.0
        for q in forced | shell:
            dv = 1.0
            for a in range(3):
                if a == c:
                    # centre spacing at face q[a] of a wall-bounded or periodic axis
                    i = q[a]
                    lo_c = xc[a][i - 1] if i > 0 else xc[a][-1] - (f[a][-1] - f[a][0])
                    dv *= xc[a][i] - lo_c
                else:
                    dv *= width[a][q[a]]
            total += dv
        exact = w.rho * fb_c[c] * total
        assert abs(float(aux["F"][c]) - exact) <= 1e-12 * abs(exact), (c, float(aux["F"][c]), exact)
