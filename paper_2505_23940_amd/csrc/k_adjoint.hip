// Discrete adjoint of one time step (reverse mode of every sub-step, with
// the point classes of the step frozen; they are piecewise constant in the
// body position).
//
// Forward, per step:  u* = (1 - eps)(u + dt R(u)) + eps u_s  (Eqs. 4-5),
// boundary faces, outflow correction, b = -(rho/dt) S u~ with
// u~ = (1 - eps) u* + eps u_c, p = A^+ b, u^{n+1} = u* - (dt/rho) G p
// (Eqs. 9-10), F = -rho h^2 sum_k dV_k sum_f f_f delta_h(x_f - X_k)
// (Eq. 20), body^{n+1} = RK4(body^n, F; k, c) (Eq. 12).
//
// Reverse:
//   RK4^T gives the force adjoint Fbar and (kbar, cbar);
//   loads^T gives fbar on forced faces and the marker-position part of dbar;
//   projection^T: one extra solve A mu = G^T ubar^{n+1} (A = A^T, so the
//     implicit-function adjoint of the PPE is the same solver), then
//     u~bar = S^T mu, ustar_bar = ubar^{n+1} + (1 - eps) u~bar and the
//     forced faces feed the body-velocity adjoint;
//   boundary^T: outflow correction, zero-gradient and convective outflow;
//   predictor^T: Rbar = (1 - eps) dt ustar_bar - eps fbar, then the
//     transposed momentum stencil written as a gather (each thread owns one
//     input face and collects every output face that read it), so no
//     atomics are needed and the result is deterministic.
#include "fvib_kernels.h"

namespace fvib {

// Threads of the body-load adjoint: its marker-position gather takes one
// item per (marker, component, stencil row).
constexpr int kAdjLoadsBlock = 1024;

// ---------------------------------------------- RK4^T and loads^T (1 block)
// The RK4 of the step starts from st_rk; the markers sit at st_pos (the
// same state in a weakly coupled step; the converged structural iterate in
// a strongly coupled one).  stbar_out = adjoint of the state after the
// step; dF direct force adjoint (may be NULL).  parts & 1: RK4^T, written
// into stbar_rk (the body-velocity part from the fluid is added later),
// kcbar accumulated, force adjoint = dF + RK4^T part; parts & 2: the
// marker-position part of loads^T for that force adjoint, added into
// stbar_pos[0..1]; parts & 4: the step's force (which RK4^T linearises
// about) gathered here from the recomputed forcing with the markers at
// st_pos, else read from sc->force.  The total force adjoint is left in
// sc->force.
template <typename T>
__global__ void __launch_bounds__(kAdjLoadsBlock)
k_adj_body_loads(IbGeo B, IbView<T> ib, const double* st_rk, const double* st_pos,
                 const double* stbar_out, const double* __restrict__ dF,
                 const double* __restrict__ kc, double* stbar_rk, double* stbar_pos,
                 double* __restrict__ kcbar, SolverScalars* sc, int parts) {
  __shared__ double Fbar_s[3];
  if (parts & 4) {
    double q[2] = {0.0, 0.0};
    ib_loads_share<T>(B, ib, st_pos, threadIdx.x, kAdjLoadsBlock, q);
    block_sum_n<2, kAdjLoadsBlock>(q);
    if (threadIdx.x == 0) {
      sc->force[0] = -B.rho * q[0];
      sc->force[1] = -B.rho * q[1];
      sc->force[2] = 0.0;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double* st = st_rk;
    double sb[6];
    for (int a = 0; a < 6; ++a) sb[a] = stbar_out ? stbar_out[a] : 0.0;
    double Fb[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a) Fb[a] = dF ? dF[a] : 0.0;
    double out[6];
    for (int a = 0; a < 6; ++a) out[a] = sb[a];
    if ((parts & 1) && B.kind == FVIB_BODY_RIGID_SPRING) {
      const double m = B.m, h = B.dt;
      for (int a = 0; a < 3; ++a) {
        if (!B.free_dof[a]) continue;
        const double k = kc ? kc[a] : 0.0, c = kc ? kc[3 + a] : 0.0;
        const double F = sc->force[a];
        const double d = st[a], v = st[3 + a];
        // forward stages
        const double k1d = v, k1v = (F - c * v - k * d) / m;
        const double d2 = d + 0.5 * h * k1d, v2 = v + 0.5 * h * k1v;
        const double k2v = (F - c * v2 - k * d2) / m;
        const double k2d = v2;
        const double d3 = d + 0.5 * h * k2d, v3 = v + 0.5 * h * k2v;
        const double k3v = (F - c * v3 - k * d3) / m;
        const double k3d = v3;
        const double d4 = d + h * k3d, v4 = v + h * k3v;
        (void)k1d;
        // reverse
        const double d1b = sb[a], v1b = sb[3 + a];
        double db = d1b, vb = v1b, Fbar = 0.0, kb = 0.0, cb = 0.0;
        double k1db = h / 6.0 * d1b, k2db = h / 3.0 * d1b, k3db = h / 3.0 * d1b, k4db = h / 6.0 * d1b;
        double k1vb = h / 6.0 * v1b, k2vb = h / 3.0 * v1b, k3vb = h / 3.0 * v1b, k4vb = h / 6.0 * v1b;
        // stage 4
        double v4b = k4db - c * k4vb / m, d4b = -k * k4vb / m;
        Fbar += k4vb / m;
        cb -= v4 * k4vb / m;
        kb -= d4 * k4vb / m;
        db += d4b;
        k3db += h * d4b;
        vb += v4b;
        k3vb += h * v4b;
        // stage 3
        double v3b = k3db - c * k3vb / m, d3b = -k * k3vb / m;
        Fbar += k3vb / m;
        cb -= v3 * k3vb / m;
        kb -= d3 * k3vb / m;
        db += d3b;
        k2db += 0.5 * h * d3b;
        vb += v3b;
        k2vb += 0.5 * h * v3b;
        // stage 2
        double v2b = k2db - c * k2vb / m, d2b = -k * k2vb / m;
        Fbar += k2vb / m;
        cb -= v2 * k2vb / m;
        kb -= d2 * k2vb / m;
        db += d2b;
        k1db += 0.5 * h * d2b;
        vb += v2b;
        k1vb += 0.5 * h * v2b;
        // stage 1
        Fbar += k1vb / m;
        cb -= v * k1vb / m;
        kb -= d * k1vb / m;
        db += -k * k1vb / m;
        vb += -c * k1vb / m + k1db;
        out[a] = db;
        out[3 + a] = vb;
        Fb[a] += Fbar;
        if (kcbar) {
          kcbar[a] += kb;
          kcbar[3 + a] += cb;
        }
      }
    }
    if (parts & 1)
      for (int a = 0; a < 6; ++a) stbar_rk[a] = out[a];
    for (int a = 0; a < 3; ++a) Fbar_s[a] = Fb[a];
  }
  __syncthreads();
  if (!(parts & 2)) {
    if (threadIdx.x == 0)
      for (int a = 0; a < 3; ++a) sc->force[a] = Fbar_s[a];   // total force adjoint
    return;
  }
  // marker-position part: dF_c/dX_k,a = rho h^2 dV_k sum_f f_f d(delta)/dr_a
  const double dxb = st_pos[0], dyb = st_pos[1];
  const double h = B.h;
  // one item per (marker, component, stencil row), as the loads gather
  double g[2] = {0.0, 0.0};
  for (int it = threadIdx.x; it < 8 * B.M; it += kAdjLoadsBlock) {
    const int k = it >> 3, c = (it >> 2) & 1, dj = it & 3;
    const double Fb = Fbar_s[c];
    if (Fb == 0.0) continue;
    const double Xx = B.X0[2 * k] + dxb, Xy = B.X0[2 * k + 1] + dyb;
    const double dV = B.ds[k] * h;
    const int i0 = (int)floor((Xx - B.fx[c][0]) / h) - 1;
    const int j0 = (int)floor((Xy - B.fy[c][0]) / h) - 1;
    const int ox = ib.origin[2 * c], oy = ib.origin[2 * c + 1];
    const int lj = j0 + dj - oy;
    if (lj < 0 || lj >= B.W[c][1]) continue;
    const double ry = B.fy[c][j0 + dj] - Xy;
    const double wy = ib_dh(ry, h), gy = ib_ddh(ry, h);
    double ax = 0.0, ay = 0.0;
    for (int di = 0; di < 4; ++di) {
      const int li = i0 + di - ox;
      if (li < 0 || li >= B.W[c][0]) continue;
      const int l = lj * B.W[c][0] + li;
      if (!ib.cls[c][l]) continue;
      const double rx = B.fx[c][i0 + di] - Xx;
      const double f = (double)ib.f[c][l];
      ax += f * ib_ddh(rx, h) * wy;
      ay += f * ib_dh(rx, h) * gy;
    }
    g[0] += Fb * B.rho * h * h * dV * ax;
    g[1] += Fb * B.rho * h * h * dV * ay;
  }
  block_sum_n<2, kAdjLoadsBlock>(g);
  if (threadIdx.x == 0) {
    stbar_pos[0] += g[0];
    stbar_pos[1] += g[1];
    for (int a = 0; a < 3; ++a) sc->force[a] = Fbar_s[a];   // total force adjoint
  }
}

// fbar on forced faces: -rho h^2 Fbar_c sum_k dV_k delta_h(x_f - X_k)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_fbar(IbGeo B, const double* __restrict__ st, const SolverScalars* sc, T* __restrict__ fb0,
           T* __restrict__ fb1) {
  T* fbar[2] = {fb0, fb1};
  const int n0 = B.W[0][0] * B.W[0][1];
  const int n1 = B.W[1][0] * B.W[1][1];
  const double h = B.h;
  // one wavefront per window face, its lanes over the markers
  const int lane = threadIdx.x & 63;
  const int wpb = kBlock / 64;
  for (int t = blockIdx.x * wpb + (threadIdx.x >> 6); t < n0 + n1; t += gridDim.x * wpb) {
    const int c = (t < n0) ? 0 : 1;
    const int l = (c == 0) ? t : t - n0;
    if (!B.cls[c][l]) {
      if (lane == 0) fbar[c][l] = T(0);
      continue;
    }
    const int li = l % B.W[c][0], lj = l / B.W[c][0];
    const int i = B.origin[2 * c] + li, j = B.origin[2 * c + 1] + lj;
    const double px = B.fx[c][i], py = B.fy[c][j];
    double s = 0.0;
    for (int k = lane; k < B.M; k += 64) {
      const double Xx = B.X0[2 * k] + st[0], Xy = B.X0[2 * k + 1] + st[1];
      s += B.ds[k] * h * ib_dh(px - Xx, h) * ib_dh(py - Xy, h);
    }
    s = wave_sum(s);
    if (lane == 0) fbar[c][l] = (T)(-B.rho * h * h * sc->force[c] * s);
  }
}

// ------------------------------------------ strong coupling (Eq. 24)
// One classic RK4 step of (d, v) with d' = v, v' = (F - c v - k d) / m.
__device__ __forceinline__ void rk4_dv(double m, double k, double c, double dt, double d,
                                       double v, double F, double* d1, double* v1) {
  const double k1d = v, k1v = (F - c * v - k * d) / m;
  const double d2 = d + 0.5 * dt * k1d, v2 = v + 0.5 * dt * k1v;
  const double k2d = v2, k2v = (F - c * v2 - k * d2) / m;
  const double d3 = d + 0.5 * dt * k2d, v3 = v + 0.5 * dt * k2v;
  const double k3d = v3, k3v = (F - c * v3 - k * d3) / m;
  const double d4 = d + dt * k3d, v4 = v + dt * k3v;
  const double k4d = v4, k4v = (F - c * v4 - k * d4) / m;
  *d1 = d + (dt / 6.0) * (k1d + 2.0 * k2d + 2.0 * k3d + k4d);
  *v1 = v + (dt / 6.0) * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
}

// Jacobians of one coupling sub-iteration at the iterate om the fluid saw
// (its point classes and forcing in the window, frozen):
//   DF = dF/d(om), 3 x 6 row-major: positions through the kernel weights of
//        the loads, velocities through the forcing, whose target on forced
//        faces is the rigid velocity (df/dU_c = 1/dt there);
//   RF = d body^{n+1} / dF, 6 x 3 row-major: the RK4 of Eq. 12 is linear in
//        the state and the force, so its force column is RK4 of a unit force
//        from rest (free degrees of freedom only).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_strong_jac(IbGeo B, IbView<T> ib, const double* __restrict__ om,
             const double* __restrict__ kc, double* __restrict__ DF, double* __restrict__ RF) {
  const double h = B.h;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // per component: dF/dd_x, dF/dd_y, dF/dv_c
  for (int k = threadIdx.x; k < B.M; k += kBlock) {
    const double Xx = B.X0[2 * k] + om[0], Xy = B.X0[2 * k + 1] + om[1];
    const double wgt = B.rho * h * h * (B.ds[k] * h);
    for (int c = 0; c < 2; ++c) {
      const int i0 = (int)floor((Xx - B.fx[c][0]) / h) - 1;
      const int j0 = (int)floor((Xy - B.fy[c][0]) / h) - 1;
      const int ox = ib.origin[2 * c], oy = ib.origin[2 * c + 1];
      double ax = 0.0, ay = 0.0, s0 = 0.0;
      for (int dj = 0; dj < 4; ++dj) {
        const int lj = j0 + dj - oy;
        if (lj < 0 || lj >= B.W[c][1]) continue;
        const double ry = B.fy[c][j0 + dj] - Xy;
        for (int di = 0; di < 4; ++di) {
          const int li = i0 + di - ox;
          if (li < 0 || li >= B.W[c][0]) continue;
          const int l = lj * B.W[c][0] + li;
          if (!ib.cls[c][l]) continue;
          const double rx = B.fx[c][i0 + di] - Xx;
          const double f = (double)ib.f[c][l];
          ax += f * ib_ddh(rx, h) * ib_dh(ry, h);
          ay += f * ib_dh(rx, h) * ib_ddh(ry, h);
          s0 += ib_dh(rx, h) * ib_dh(ry, h);
        }
      }
      s[3 * c + 0] += wgt * ax;
      s[3 * c + 1] += wgt * ay;
      s[3 * c + 2] -= wgt * s0 / B.dt;
    }
  }
  block_sum<6>(s);
  if (threadIdx.x != 0) return;
  for (int i = 0; i < 18; ++i) DF[i] = 0.0;
  for (int c = 0; c < 2; ++c) {
    DF[c * 6 + 0] = s[3 * c + 0];
    DF[c * 6 + 1] = s[3 * c + 1];
    DF[c * 6 + 3 + c] = s[3 * c + 2];
  }
  for (int i = 0; i < 18; ++i) RF[i] = 0.0;
  if (B.kind != FVIB_BODY_RIGID_SPRING) return;
  for (int a = 0; a < 3; ++a) {
    if (!B.free_dof[a]) continue;
    double d1, v1;
    rk4_dv(B.m, kc ? kc[a] : 0.0, kc ? kc[3 + a] : 0.0, B.dt, 0.0, 0.0, 1.0, &d1, &v1);
    RF[a * 3 + a] = d1;
    RF[(3 + a) * 3 + a] = v1;
  }
}

// Adjoint of the coupling fixed point w* = Phi(w*), Phi(w) = RK4(w^n, F(w))
// (Eq. 24 with the residual w - Phi(w)): lam solves (I - J^T) lam = a with
// J = RF DF and a = wbar + ubody + DF^T dF, the direct derivative of the
// loss with respect to the iterate (wbar: adjoint of the body state after
// the step; ubody: the fluid's body-velocity adjoint; dF: the direct force
// adjoint, nullable).  Dense 6 x 6 Gaussian elimination with partial
// pivoting, one thread.
__global__ void k_strong_lambda(const double* __restrict__ DF, const double* __restrict__ RF,
                                const double* __restrict__ wbar, const double* __restrict__ ubody,
                                const double* __restrict__ dF, double* __restrict__ lam,
                                SolverScalars* sc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double M[6][7];
  for (int i = 0; i < 6; ++i) {
    double r = (wbar ? wbar[i] : 0.0) + ubody[i];
    for (int a = 0; a < 3; ++a) r += DF[a * 6 + i] * (dF ? dF[a] : 0.0);
    M[i][6] = r;
    for (int j = 0; j < 6; ++j) {
      double Jji = 0.0;                     // J[j][i] = sum_a RF[j][a] DF[a][i]
      for (int a = 0; a < 3; ++a) Jji += RF[j * 3 + a] * DF[a * 6 + i];
      M[i][j] = (i == j ? 1.0 : 0.0) - Jji;
    }
  }
  for (int col = 0; col < 6; ++col) {
    int piv = col;
    for (int r = col + 1; r < 6; ++r)
      if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
    if (piv != col)
      for (int j = 0; j < 7; ++j) {
        const double t = M[col][j];
        M[col][j] = M[piv][j];
        M[piv][j] = t;
      }
    const double d = M[col][col];
    if (!(fabs(d) > 0.0)) {              // singular: the sub-iterations cannot converge
      sc->status = FVIB_ENONFINITE;
      for (int i = 0; i < 6; ++i) lam[i] = 0.0;
      return;
    }
    for (int r = col + 1; r < 6; ++r) {
      const double f = M[r][col] / d;
      for (int j = col; j < 7; ++j) M[r][j] -= f * M[col][j];
    }
  }
  for (int i = 5; i >= 0; --i) {
    double x = M[i][6];
    for (int j = i + 1; j < 6; ++j) x -= M[i][j] * lam[j];
    lam[i] = x / M[i][i];
  }
}

// ------------------------------------------------- static box (3D)
// Control volume of face (i, j, k) of component C: centre spacing along C
// times the transverse cell widths.
template <typename T>
__device__ __forceinline__ double box_face_volume(const Geo<double>& G, int c, int i, int j,
                                                  int k) {
  const int I[3] = {i, j, k};
  double v = 1.0;
  for (int a = 0; a < 3; ++a) v *= (a == c) ? G.dc[a][I[a]] : G.dx[a][I[a]];
  return v;
}

// Force on the box: F = -rho sum over forced faces of f dv (block partial
// sums, combined in block order by a one-block epilogue).
struct FinBoxForce {
  double rho;
  __device__ bool skip(const SolverScalars*) const { return false; }
  __device__ void apply(const double* t, SolverScalars* sc) const {
    for (int a = 0; a < 3; ++a) sc->force[a] = -rho * t[a];
  }
};

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_box_force(Geo<double> G, IbView<T> ib, double* __restrict__ partial) {
  double F[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < 3; ++c) {
    const int W0 = ib.bw[c][0], W1 = ib.bw[c][1], n = W0 * W1 * ib.bw[c][2];
    for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
      if (!ib.bcls[c][l]) continue;
      const int i = ib.bo[c][0] + l % W0, j = ib.bo[c][1] + (l / W0) % W1,
                k = ib.bo[c][2] + l / (W0 * W1);
      F[c] += (double)ib.bf[c][l] * box_face_volume<T>(G, c, i, j, k);
    }
  }
  block_partials<3, 3>(F, partial);
}

// Forcing adjoint on the box's forced faces for a force adjoint dF
// (nullable: zero): fbar = -rho dv dF_c.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_box_fbar(Geo<double> G, IbView<T> ib, double rho, const double* __restrict__ dF) {
  for (int c = 0; c < 3; ++c) {
    const int W0 = ib.bw[c][0], W1 = ib.bw[c][1], n = W0 * W1 * ib.bw[c][2];
    const double g = dF ? -rho * dF[c] : 0.0;
    for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
      const int i = ib.bo[c][0] + l % W0, j = ib.bo[c][1] + (l / W0) % W1,
                k = ib.bo[c][2] + l / (W0 * W1);
      ib.bf[c][l] = (T)(ib.bcls[c][l] ? g * box_face_volume<T>(G, c, i, j, k) : 0.0);
    }
  }
}

// Forward: on the forced faces the predictor's u* = u + dt R becomes the
// target 0, and the forcing of Eq. 5 is f = -R - u / dt = -u* / dt.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_box_fix(Geo<T> G, IbView<T> ib, T* __restrict__ s0, T* __restrict__ s1, T* __restrict__ s2) {
  T* us[3] = {s0, s1, s2};
  for (int c = 0; c < 3; ++c) {
    const int W0 = ib.bw[c][0], W1 = ib.bw[c][1], n = W0 * W1 * ib.bw[c][2];
    for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
      if (!ib.bcls[c][l]) continue;
      const int i = ib.bo[c][0] + l % W0, j = ib.bo[c][1] + (l / W0) % W1,
                k = ib.bo[c][2] + l / (W0 * W1);
      const int64_t id = fidx(G.ext[c], i, j, k);
      ib.bf[c][l] = -us[c][id] / G.dt;
      us[c][id] = T(0);
    }
  }
}

// Adjoint: on the forced faces the momentum adjoint reads the forcing
// adjoint -fbar / dt in place of ustar_bar (u* there is the constant
// target; R reaches the loss only through f).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_box_rbar(Geo<T> G, IbView<T> ib, T* __restrict__ s0, T* __restrict__ s1, T* __restrict__ s2) {
  T* usb[3] = {s0, s1, s2};
  for (int c = 0; c < 3; ++c) {
    const int W0 = ib.bw[c][0], W1 = ib.bw[c][1], n = W0 * W1 * ib.bw[c][2];
    for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
      if (!ib.bcls[c][l]) continue;
      const int i = ib.bo[c][0] + l % W0, j = ib.bo[c][1] + (l / W0) % W1,
                k = ib.bo[c][2] + l / (W0 * W1);
      usb[c][fidx(G.ext[c], i, j, k)] = -ib.bf[c][l] / G.dt;
    }
  }
}

static int box_blocks(const IbView<float>& ib) {
  int64_t n = 0;
  for (int c = 0; c < 3; ++c) n = std::max<int64_t>(n, (int64_t)ib.bw[c][0] * ib.bw[c][1] * ib.bw[c][2]);
  int64_t b = (n + kBlock - 1) / kBlock;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), kMaxRedBlocks);
}
static int box_blocks(const IbView<double>& ib) {
  int64_t n = 0;
  for (int c = 0; c < 3; ++c) n = std::max<int64_t>(n, (int64_t)ib.bw[c][0] * ib.bw[c][1] * ib.bw[c][2]);
  int64_t b = (n + kBlock - 1) / kBlock;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), kMaxRedBlocks);
}

template <typename T>
int launch_box_force(const Geo<double>& G, const IbView<T>& ib, double rho, RedBuf red,
                     SolverScalars* sc, hipStream_t s) {
  const int nb = box_blocks(ib);
  launch_kernel((k_box_force<T>), dim3(nb), dim3(kBlock), 0, s, G, ib, red.partial);
  FVIB_HIP(hipGetLastError());
  FVIB_HIP((launch_finish<3, 3>(red.partial, nb, sc, FinBoxForce{rho}, s)));
  return FVIB_OK;
}

template <typename T>
int launch_box_fix(const Geo<T>& G, const IbView<T>& ib, T* us[3], hipStream_t s) {
  launch_kernel((k_box_fix<T>), dim3(box_blocks(ib)), dim3(kBlock), 0, s, G, ib, us[0], us[1],
                us[2]);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_box_rbar(const Geo<T>& G, const IbView<T>& ib, T* usb[3], hipStream_t s) {
  launch_kernel((k_box_rbar<T>), dim3(box_blocks(ib)), dim3(kBlock), 0, s, G, ib, usb[0], usb[1],
                usb[2]);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_box_fbar(const Geo<double>& G, const IbView<T>& ib, double rho, const double* dF,
                    hipStream_t s) {
  launch_kernel((k_box_fbar<T>), dim3(64), dim3(kBlock), 0, s, G, ib, rho, dF);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template int launch_box_force<float>(const Geo<double>&, const IbView<float>&, double, RedBuf,
                                     SolverScalars*, hipStream_t);
template int launch_box_force<double>(const Geo<double>&, const IbView<double>&, double, RedBuf,
                                      SolverScalars*, hipStream_t);
template int launch_box_fix<float>(const Geo<float>&, const IbView<float>&, float* [3],
                                   hipStream_t);
template int launch_box_fix<double>(const Geo<double>&, const IbView<double>&, double* [3],
                                    hipStream_t);
template int launch_box_rbar<float>(const Geo<float>&, const IbView<float>&, float* [3],
                                    hipStream_t);
template int launch_box_rbar<double>(const Geo<double>&, const IbView<double>&, double* [3],
                                     hipStream_t);
template int launch_box_fbar<float>(const Geo<double>&, const IbView<float>&, double,
                                    const double*, hipStream_t);
template int launch_box_fbar<double>(const Geo<double>&, const IbView<double>&, double,
                                     const double*, hipStream_t);

// --------------------------------------------------------- projection^T
// y_c = (G^T ubar)_c = sum over interior faces of c of (+-) ubar_f / dc_f,
// + for the low face, - for the high face.  Records sum(y) and max |y / V|.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock)
k_adj_rhs(Geo<T> G, PGeo<double> P, Tiling tl, const T* __restrict__ b0,
          const T* __restrict__ b1, const T* __restrict__ b2, double* __restrict__ y,
          RedBuf red, SolverScalars* sc) {
  const T* ub[3] = {b0, b1, b2};
  const int nx_ = G.n[0], ny_ = G.n[1];
  double sum = 0.0, mx = 0.0;
  for (int t_ = xcd_block(blockIdx.x, gridDim.x); t_ < tl.ntiles; t_ += gridDim.x) {
    const int i = (t_ % tl.ntx) * kTileX + (threadIdx.x & (kTileX - 1));
    const int j = ((t_ / tl.ntx) % tl.nty) * kTileY + (threadIdx.x / kTileX);
    const int k = t_ / (tl.ntx * tl.nty);
    if (i >= nx_ || j >= ny_) continue;
    const int I[3] = {i, j, k};
    double lo[DIM], hi[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int ic = I[c], nc = G.n[c];
      int H[3] = {i, j, k};
      H[c] = (G.per[c] && ic + 1 == nc) ? 0 : ic + 1;
      lo[c] = (double)ub[c][fidx(G.ext[c], i, j, k)];
      hi[c] = (double)ub[c][fidx(G.ext[c], H[0], H[1], H[2])];
    }
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int ic = I[c], nc = G.n[c];
      // boundary faces of a bounded axis carry no flux (selected, not
      // multiplied, so whatever the adjoint holds there cannot leak in)
      const double tl_ = lo[c] * P.idc[c][ic], th_ = hi[c] * P.idc[c][ic + 1];
      acc += (G.per[c] || ic > 0) ? tl_ : 0.0;
      acc -= (G.per[c] || ic + 1 < nc) ? th_ : 0.0;
    }
    y[((int64_t)k * ny_ + j) * nx_ + i] = acc;
    sum += acc;
    double iv = (double)P.iv[0][i] * (double)P.iv[1][j];
    if (DIM == 3) iv *= (double)P.iv[2][k];
    mx = fmax(mx, fabs(acc) * iv);
  }
  double v[2] = {sum, mx};
  block_partials<2, 1>(v, red.partial);
}

// 3D column march of k_adj_rhs (same terms, same order): each thread walks
// one (i, j) column of a chunk of z-planes, carrying the upper w face of
// plane k over as the lower face of plane k + 1 and fetching the faces of
// the next plane while it evaluates this one.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_rhs_col(Geo<T> G, PGeo<double> P, ColTiling ct, const T* __restrict__ b0,
              const T* __restrict__ b1, const T* __restrict__ b2, double* __restrict__ y,
              RedBuf red) {
  const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
  const int64_t sxy = (int64_t)nx * ny;
  double sum = 0.0, mx = 0.0;
  const int lx = threadIdx.x & (kTileX - 1), ly = threadIdx.x / kTileX;
  for (int u = xcd_block(blockIdx.x, gridDim.x); u < ct.nunits; u += gridDim.x) {
    const int tx = u % ct.ntx, ty = (u / ct.ntx) % ct.nty, zc = u / (ct.ntx * ct.nty);
    const int i = tx * kTileX + lx, j = ty * kTileY + ly;
    if (i >= nx || j >= ny) continue;
    const int k0 = zc * ct.zchunk, k1 = min(k0 + ct.zchunk, nz);
    const int ex0 = G.ext[0][0], ex1 = G.ext[0][1];
    const int ey0 = G.ext[1][0], ey1 = G.ext[1][1];
    const int ez0 = G.ext[2][0], ez1 = G.ext[2][1];
    const int iH = (G.per[0] && i + 1 == nx) ? 0 : i + 1;
    const int jH = (G.per[1] && j + 1 == ny) ? 0 : j + 1;
    const int64_t uL = (int64_t)j * ex0 + i, uH = (int64_t)j * ex0 + iH;
    const int64_t vL = (int64_t)j * ey0 + i, vH = (int64_t)jH * ey0 + i;
    const int64_t wL = (int64_t)j * ez0 + i;
    const int64_t su = (int64_t)ex0 * ex1, sv = (int64_t)ey0 * ey1, sw = (int64_t)ez0 * ez1;
    // boundary faces of a bounded axis carry no flux (selected, not
    // multiplied, so whatever the adjoint holds there cannot leak in)
    const bool xl = G.per[0] || i > 0, xh = G.per[0] || i + 1 < nx;
    const bool yl = G.per[1] || j > 0, yh = G.per[1] || j + 1 < ny;
    const double cxl = P.idc[0][i], cxh = P.idc[0][i + 1];
    const double cyl = P.idc[1][j], cyh = P.idc[1][j + 1];
    const double ivxy = (double)P.iv[0][i] * (double)P.iv[1][j];
    auto kup = [&](int k) { return (G.per[2] && k + 1 == nz) ? 0 : k + 1; };
    double ulo = (double)b0[(int64_t)k0 * su + uL], uhi = (double)b0[(int64_t)k0 * su + uH];
    double vlo = (double)b1[(int64_t)k0 * sv + vL], vhi = (double)b1[(int64_t)k0 * sv + vH];
    double wlo = (double)b2[(int64_t)k0 * sw + wL], whi = (double)b2[(int64_t)kup(k0) * sw + wL];
    for (int k = k0; k < k1; ++k) {
      // faces of plane k + 1 (its lower w face is this plane's upper one)
      double ulo2 = 0.0, uhi2 = 0.0, vlo2 = 0.0, vhi2 = 0.0, whi2 = 0.0;
      if (k + 1 < k1) {
        const int64_t kn = k + 1;
        ulo2 = (double)b0[kn * su + uL];
        uhi2 = (double)b0[kn * su + uH];
        vlo2 = (double)b1[kn * sv + vL];
        vhi2 = (double)b1[kn * sv + vH];
        whi2 = (double)b2[(int64_t)kup(k + 1) * sw + wL];
      }
      const bool zl = G.per[2] || k > 0, zh = G.per[2] || k + 1 < nz;
      double acc = 0.0;
      acc += xl ? ulo * cxl : 0.0;
      acc -= xh ? uhi * cxh : 0.0;
      acc += yl ? vlo * cyl : 0.0;
      acc -= yh ? vhi * cyh : 0.0;
      acc += zl ? wlo * P.idc[2][k] : 0.0;
      acc -= zh ? whi * P.idc[2][k + 1] : 0.0;
      y[(int64_t)k * sxy + (int64_t)j * nx + i] = acc;
      sum += acc;
      mx = fmax(mx, fabs(acc) * (ivxy * (double)P.iv[2][k]));
      ulo = ulo2;
      uhi = uhi2;
      vlo = vlo2;
      vhi = vhi2;
      wlo = whi;
      whi = whi2;
    }
  }
  double v[2] = {sum, mx};
  block_partials<2, 1>(v, red.partial);
}

// 3D column march of k_adj_rhs_col fused with the first residual of the
// adjoint solve: y = G^T ubar is stored for the later residuals and
// r = y - A mu_in is handed to the fast-diagonalisation sweep without the mean
// of y (the sweep drops the constant mode); the criterion is
// max |r| / V + |mean y| max (1 / V), an upper bound of the mean-free one.
// Same terms in the same order as k_adj_rhs_col (y) and k_residual (A mu).
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock)
k_adj_rhs_res_col(Geo<T> G, PGeo<double> P, ColTiling ct, const T* __restrict__ b0,
                  const T* __restrict__ b1, const T* __restrict__ b2,
                  const double* __restrict__ x, double* __restrict__ y,
                  double* __restrict__ r64, float* __restrict__ r32, RedBuf red) {
  const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
  const int64_t sxy = (int64_t)nx * ny;
  double rr = 0.0, sx = 0.0, sy = 0.0, mr = 0.0, my = 0.0;
  const int lx = threadIdx.x & (kTileX - 1), ly = threadIdx.x / kTileX;
  for (int u = xcd_block(blockIdx.x, gridDim.x); u < ct.nunits; u += gridDim.x) {
    const int tx = u % ct.ntx, ty = (u / ct.ntx) % ct.nty, zc = u / (ct.ntx * ct.nty);
    const int i = tx * kTileX + lx, j = ty * kTileY + ly;
    if (i >= nx || j >= ny) continue;
    const int k0 = zc * ct.zchunk, k1 = min(k0 + ct.zchunk, nz);
    const int ex0 = G.ext[0][0], ex1 = G.ext[0][1];
    const int ey0 = G.ext[1][0], ey1 = G.ext[1][1];
    const int ez0 = G.ext[2][0], ez1 = G.ext[2][1];
    const int iH = (G.per[0] && i + 1 == nx) ? 0 : i + 1;
    const int jH = (G.per[1] && j + 1 == ny) ? 0 : j + 1;
    const int64_t uL = (int64_t)j * ex0 + i, uH = (int64_t)j * ex0 + iH;
    const int64_t vL = (int64_t)j * ey0 + i, vH = (int64_t)jH * ey0 + i;
    const int64_t wL = (int64_t)j * ez0 + i;
    const int64_t su = (int64_t)ex0 * ex1, sv = (int64_t)ey0 * ey1, sw = (int64_t)ez0 * ez1;
    const bool xl = G.per[0] || i > 0, xh = G.per[0] || i + 1 < nx;
    const bool yl = G.per[1] || j > 0, yh = G.per[1] || j + 1 < ny;
    const double cxl = P.idc[0][i], cxh = P.idc[0][i + 1];
    const double cyl = P.idc[1][j], cyh = P.idc[1][j + 1];
    const double ivxy = (double)P.iv[0][i] * (double)P.iv[1][j];
    auto kup = [&](int k) { return (G.per[2] && k + 1 == nz) ? 0 : k + 1; };
    // adjoint pressure column: x-y neighbours and coefficients
    const int64_t cC = (int64_t)j * nx + i;
    const int64_t cW = (int64_t)j * nx + (i > 0 ? i - 1 : (P.per[0] ? nx - 1 : 0));
    const int64_t cE = (int64_t)j * nx + (i < nx - 1 ? i + 1 : (P.per[0] ? 0 : nx - 1));
    const int64_t cS = (int64_t)(j > 0 ? j - 1 : (P.per[1] ? ny - 1 : 0)) * nx + i;
    const int64_t cN = (int64_t)(j < ny - 1 ? j + 1 : (P.per[1] ? 0 : ny - 1)) * nx + i;
    const double dxi = P.dx[0][i], dyj = P.dx[1][j];
    const double kxl = P.kf[0][i], kxh = P.kf[0][i + 1];
    const double kyl = P.kf[1][j], kyh = P.kf[1][j + 1];
    const int pz = P.per[2];
    auto klo = [&](int k) { return k > 0 ? k - 1 : (pz ? nz - 1 : 0); };
    auto khi = [&](int k) { return k < nz - 1 ? k + 1 : (pz ? 0 : nz - 1); };
    auto at = [&](int64_t off, int k) { return x[(int64_t)k * sxy + off]; };
    double xm = at(cC, klo(k0)), xc = at(cC, k0), xp = at(cC, khi(k0));
    double xw = at(cW, k0), xe = at(cE, k0), xs = at(cS, k0), xn = at(cN, k0);
    double ulo = (double)b0[(int64_t)k0 * su + uL], uhi = (double)b0[(int64_t)k0 * su + uH];
    double vlo = (double)b1[(int64_t)k0 * sv + vL], vhi = (double)b1[(int64_t)k0 * sv + vH];
    double wlo = (double)b2[(int64_t)k0 * sw + wL], whi = (double)b2[(int64_t)kup(k0) * sw + wL];
    for (int k = k0; k < k1; ++k) {
      double ulo2 = 0.0, uhi2 = 0.0, vlo2 = 0.0, vhi2 = 0.0, whi2 = 0.0;
      double xp2 = 0.0, xw2 = 0.0, xe2 = 0.0, xs2 = 0.0, xn2 = 0.0;
      if (k + 1 < k1) {
        const int64_t kn = k + 1;
        ulo2 = (double)b0[kn * su + uL];
        uhi2 = (double)b0[kn * su + uH];
        vlo2 = (double)b1[kn * sv + vL];
        vhi2 = (double)b1[kn * sv + vH];
        whi2 = (double)b2[(int64_t)kup(k + 1) * sw + wL];
        xp2 = at(cC, khi(k + 1));
        xw2 = at(cW, k + 1);
        xe2 = at(cE, k + 1);
        xs2 = at(cS, k + 1);
        xn2 = at(cN, k + 1);
      }
      const bool zl = G.per[2] || k > 0, zh = G.per[2] || k + 1 < nz;
      double acc = 0.0;
      acc += xl ? ulo * cxl : 0.0;
      acc -= xh ? uhi * cxh : 0.0;
      acc += yl ? vlo * cyl : 0.0;
      acc -= yh ? vhi * cyh : 0.0;
      acc += zl ? wlo * P.idc[2][k] : 0.0;
      acc -= zh ? whi * P.idc[2][k + 1] : 0.0;
      const double dzk = P.dx[2][k], kzl = P.kf[2][k], kzh = P.kf[2][k + 1];
      double ax_ = 0.0;
      const double ax = dyj * dzk, ay = dxi * dzk, az = dxi * dyj;
      ax_ += ax * kxl * (xc - xw);
      ax_ += ax * kxh * (xc - xe);
      ax_ += ay * kyl * (xc - xs);
      ax_ += ay * kyh * (xc - xn);
      ax_ += az * kzl * (xc - xm);
      ax_ += az * kzh * (xc - xp);
      const double r = acc - ax_;
      const double iv = ivxy * (double)P.iv[2][k];
      const int64_t c = (int64_t)k * sxy + (int64_t)j * nx + i;
      y[c] = acc;
      if (MODE == 3)
        r64[c] = r;
      else
        r32[c] = (float)r;
      rr += r * r;
      sx += xc;
      sy += acc;
      mr = fmax(mr, fabs(r) * iv);
      my = fmax(my, fabs(acc) * iv);
      ulo = ulo2;
      uhi = uhi2;
      vlo = vlo2;
      vhi = vhi2;
      wlo = whi;
      whi = whi2;
      xm = xc;
      xc = xp;
      xp = xp2;
      xw = xw2;
      xe = xe2;
      xs = xs2;
      xn = xn2;
    }
  }
  double v[5] = {rr, sx, sy, mr, my};
  block_partials<5, 3>(v, red.partial);
}

// k_adj_rhs_res_col on a 2D grid (one cell per thread): y = G^T ubar (the
// terms of k_adj_rhs) and the first residual r = y - A mu_in (the terms of
// k_residual) in one pass.
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock)
k_adj_rhs_res_2d(Geo<T> G, PGeo<double> P, ColTiling ct, const T* __restrict__ b0,
                 const T* __restrict__ b1, const double* __restrict__ x,
                 double* __restrict__ y, double* __restrict__ r64, float* __restrict__ r32,
                 RedBuf red) {
  const int nx = G.n[0], ny = G.n[1];
  double rr = 0.0, sx = 0.0, sy = 0.0, mr = 0.0, my = 0.0;
  const int lx = threadIdx.x & (kTileX - 1), ly = threadIdx.x / kTileX;
  for (int u = xcd_block(blockIdx.x, gridDim.x); u < ct.nunits; u += gridDim.x) {
    const int tx = u % ct.ntx, ty = (u / ct.ntx) % ct.nty;
    const int i = tx * kTileX + lx, j = ty * kTileY + ly;
    if (i >= nx || j >= ny) continue;
    const int iH = (G.per[0] && i + 1 == nx) ? 0 : i + 1;
    const int jH = (G.per[1] && j + 1 == ny) ? 0 : j + 1;
    const double ulo = (double)b0[(int64_t)j * G.ext[0][0] + i];
    const double uhi = (double)b0[(int64_t)j * G.ext[0][0] + iH];
    const double vlo = (double)b1[(int64_t)j * G.ext[1][0] + i];
    const double vhi = (double)b1[(int64_t)jH * G.ext[1][0] + i];
    const bool xl = G.per[0] || i > 0, xh = G.per[0] || i + 1 < nx;
    const bool yl = G.per[1] || j > 0, yh = G.per[1] || j + 1 < ny;
    double acc = 0.0;
    acc += xl ? ulo * P.idc[0][i] : 0.0;
    acc -= xh ? uhi * P.idc[0][i + 1] : 0.0;
    acc += yl ? vlo * P.idc[1][j] : 0.0;
    acc -= yh ? vhi * P.idc[1][j + 1] : 0.0;
    const int64_t cC = (int64_t)j * nx + i;
    const double xc = x[cC];
    const double xw = x[(int64_t)j * nx + (i > 0 ? i - 1 : (P.per[0] ? nx - 1 : 0))];
    const double xe = x[(int64_t)j * nx + (i < nx - 1 ? i + 1 : (P.per[0] ? 0 : nx - 1))];
    const double xs = x[(int64_t)(j > 0 ? j - 1 : (P.per[1] ? ny - 1 : 0)) * nx + i];
    const double xn = x[(int64_t)(j < ny - 1 ? j + 1 : (P.per[1] ? 0 : ny - 1)) * nx + i];
    const double dxi = P.dx[0][i], dyj = P.dx[1][j];
    double ax_ = 0.0;
    ax_ += dyj * P.kf[0][i] * (xc - xw);
    ax_ += dyj * P.kf[0][i + 1] * (xc - xe);
    ax_ += dxi * P.kf[1][j] * (xc - xs);
    ax_ += dxi * P.kf[1][j + 1] * (xc - xn);
    const double r = acc - ax_;
    const double iv = (double)P.iv[0][i] * (double)P.iv[1][j];
    y[cC] = acc;
    if (MODE == 3)
      r64[cC] = r;
    else
      r32[cC] = (float)r;
    rr += r * r;
    sx += xc;
    sy += acc;
    mr = fmax(mr, fabs(r) * iv);
    my = fmax(my, fabs(acc) * iv);
  }
  double v[5] = {rr, sx, sy, mr, my};
  block_partials<5, 3>(v, red.partial);
}

// Epilogue of k_adj_rhs_res_col: mean of y, the relative target of the
// adjoint solve, then what FinResidual does for the first residual.
struct FinAdjRhsResidual {
  double inv_ncell, rtol, dt_over_rho, inner_rtol, max_iv;
  SolverScalars* mirror;
  __device__ bool skip(const SolverScalars*) const { return false; }
  __device__ void apply(const double* t, SolverScalars* sc) const {
    const double mb = t[2] * inv_ncell;
    sc->meanb = mb;
    sc->ymax = t[4];
    sc->tol_dev = rtol * t[4] * dt_over_rho;
    sc->sweeps = 0;
    const double crit = (t[3] + fabs(mb) * max_iv) * dt_over_rho;
    sc->rr = t[0];
    sc->rr0 = t[0];
    sc->beta = 0.0;
    sc->iters = 0;
    sc->crit = crit;
    sc->sumx = t[1];
    sc->tol_rr = inner_rtol * inner_rtol * t[0];
    const bool bad = !(t[0] == t[0]) || !(crit == crit);
    if (bad) sc->status = FVIB_ENONFINITE;
    const bool conv = bad || crit <= sc->tol_dev || t[0] == 0.0;
    sc->done = conv ? 1 : 0;
    sc->outer_done = conv ? 1 : 0;
    if (mirror) *mirror = *sc;
  }
};

struct FinAdjRhs {          // mean of G^T ubar, max |y / V| and the solve target
  double inv_ncell, rtol, dt_over_rho;
  __device__ bool skip(const SolverScalars*) const { return false; }
  __device__ void apply(const double* t, SolverScalars* sc) const {
    sc->meanb = t[0] * inv_ncell;
    sc->crit = t[1];
    sc->ymax = t[1];
    sc->tol_dev = rtol * t[1] * dt_over_rho;
  }
};

template <int C, typename T>
__device__ __forceinline__ int forced_cls(const IbView<T>& ib, int i, int j, int* lidx) {
  if (!ib.active || ib.box || C > 1) return 0;
  const int li = i - ib.origin[2 * C + 0];
  const int lj = j - ib.origin[2 * C + 1];
  if (li < 0 || lj < 0 || li >= ib.W[C][0] || lj >= ib.W[C][1]) return 0;
  *lidx = lj * ib.W[C][0] + li;
  return ib.cls[C][*lidx];
}

// (S^T mu)_f = A_f (mu_{f-1} - mu_f) with the cells that exist, mu taken at
// zero mean (mu - shift).
template <int C, typename T>
__device__ __forceinline__ double st_mu(const Geo<T>& G, const PGeo<double>& P,
                                        const double* mu, int i, int j, int k, double shift) {
  const int I[3] = {i, j, k};
  const int ic = I[C], nc = G.n[C];
  double A = 1.0;
  for (int a = 0; a < G.dim; ++a)
    if (a != C) A *= P.dx[a][I[a]];
  const int nx = G.n[0], ny = G.n[1];
  double lo = 0.0, hi = 0.0;
  int L[3] = {i, j, k};
  if (G.per[C] || ic > 0) {
    L[C] = (ic == 0) ? nc - 1 : ic - 1;
    lo = mu[((int64_t)L[2] * ny + L[1]) * nx + L[0]] - shift;
  }
  if (G.per[C] || ic < nc) {
    int H[3] = {i, j, k};
    H[C] = (ic == nc) ? 0 : ic;
    hi = mu[((int64_t)H[2] * ny + H[1]) * nx + H[0]] - shift;
  }
  return A * (lo - hi);
}

// ustar_bar = ubar^{n+1} + (1 - eps) S^T mu on every face, all components
// in one launch.  Each thread walks a z-column of a tile chunk and owns the
// low faces of its cells (and the high face of the last cell of a bounded
// axis); mu is taken at zero mean (its mean is the solve's last measured
// sum / n, so the solve itself needs no gauge pass).
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock)
k_adj_ustar(Geo<T> G, PGeo<double> P, ColTiling ct, const T* __restrict__ b0,
            const T* __restrict__ b1, const T* __restrict__ b2, const double* __restrict__ mu,
            IbView<T> ib, T* __restrict__ s0, T* __restrict__ s1, T* __restrict__ s2,
            const SolverScalars* sc, fvib_step_info* info, const double* body_src,
            double* body_dst, int* sticky) {
  const T* ub[3] = {b0, b1, b2};
  T* us[3] = {s0, s1, s2};
  if (info && blockIdx.x == 0) {
    // the step record (the scalars are final once the solve has converged;
    // a repeated launch writes the same record again) and the adjoint body
    // state of a step without a body, passed through
    if (body_dst && threadIdx.x < 6) body_dst[threadIdx.x] = body_src ? body_src[threadIdx.x] : 0.0;
    if (threadIdx.x == 0) put_record(sc, info, 0, sc->sweeps, sticky, 0);
  }
  const double shift = sc->sumx * P.inv_ncell;
  const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
  const int64_t sxy = (int64_t)nx * ny;
  const int lx = threadIdx.x & (kTileX - 1), ly = threadIdx.x / kTileX;
  for (int u = xcd_block(blockIdx.x, gridDim.x); u < ct.nunits; u += gridDim.x) {
    const int tx = u % ct.ntx, ty = (u / ct.ntx) % ct.nty, zc = u / (ct.ntx * ct.nty);
    const int i = tx * kTileX + lx, j = ty * kTileY + ly;
    if (i >= nx || j >= ny) continue;
    const int k0 = zc * ct.zchunk, k1 = min(k0 + ct.zchunk, nz);
    const int64_t cC = (int64_t)j * nx + i;
    const int64_t cW = (int64_t)j * nx + (i > 0 ? i - 1 : nx - 1);
    const int64_t cS = (int64_t)(j > 0 ? j - 1 : ny - 1) * nx + i;
    const bool hasW = G.per[0] || i > 0, hasS = G.per[1] || j > 0;
    const double dxi = P.dx[0][i], dyj = P.dx[1][j];
    double mzm = 0.0;
    bool hasZ = false;
    if (DIM == 3) {
      hasZ = G.per[2] || k0 > 0;
      if (hasZ) mzm = mu[(int64_t)(k0 > 0 ? k0 - 1 : nz - 1) * sxy + cC] - shift;
    }
    for (int k = k0; k < k1; ++k) {
      const int64_t c = (int64_t)k * sxy + cC;
      const double mc = mu[c] - shift;
      const double mw = hasW ? mu[(int64_t)k * sxy + cW] - shift : 0.0;
      const double ms = hasS ? mu[(int64_t)k * sxy + cS] - shift : 0.0;
      const double dzk = (DIM == 3) ? (double)P.dx[2][k] : 1.0;
      const int I[3] = {i, j, k};
      const double lo[3] = {mw, ms, hasZ ? mzm : 0.0};
      const double area[3] = {dyj * dzk, dxi * dzk, dxi * dyj};
#pragma unroll
      for (int C = 0; C < DIM; ++C) {
        // low face of the cell
        const int64_t id = fidx(G.ext[C], i, j, k);
        double v = (double)ub[C][id];
        int li = 0;
        bool forced = false;
        if (C == 0) forced = forced_cls<0>(ib, i, j, &li);
        else if (C == 1) forced = forced_cls<1>(ib, i, j, &li);
        if (DIM == 3 && ib.box) {
          if (C == 0) forced = forced_box<0>(ib, i, j, k, &li);
          else if (C == 1) forced = forced_box<1>(ib, i, j, k, &li);
          else forced = forced_box<2>(ib, i, j, k, &li);
        }
        if (!forced) v += area[C] * (lo[C] - mc);
        // streamed past the caches (measured 31.0 -> 29.7 us on the channel;
        // the transposed momentum kernel that reads it did not slow)
        __builtin_nontemporal_store((T)v, &us[C][id]);
        // high face of the last cell of a bounded axis
        if (!G.per[C] && I[C] == G.n[C] - 1) {
          int H[3] = {i, j, k};
          H[C] += 1;
          const int64_t ih = fidx(G.ext[C], H[0], H[1], H[2]);
          double vh = (double)ub[C][ih];
          bool fh = false;
          if (C == 0) fh = forced_cls<0>(ib, H[0], H[1], &li);
          else if (C == 1) fh = forced_cls<1>(ib, H[0], H[1], &li);
          if (DIM == 3 && ib.box) {
            if (C == 0) fh = forced_box<0>(ib, H[0], H[1], H[2], &li);
            else if (C == 1) fh = forced_box<1>(ib, H[0], H[1], H[2], &li);
            else fh = forced_box<2>(ib, H[0], H[1], H[2], &li);
          }
          if (!fh) vh += area[C] * mc;
          __builtin_nontemporal_store((T)vh, &us[C][ih]);
        }
      }
      mzm = mc;
      hasZ = true;
    }
  }
}

// Body-velocity adjoint from the forced faces: u_s and u_c equal the rigid
// velocity there, so Ubar_c = sum_forced [ubar^{n+1} + S^T mu + fbar/dt].
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_ubody(Geo<T> G, PGeo<double> P, IbGeo B, const T* __restrict__ ub0,
            const T* __restrict__ ub1, const double* __restrict__ mu, IbView<T> ib,
            double* __restrict__ stbar, const SolverScalars* sc) {
  const T* ub[2] = {ub0, ub1};
  const double shift = sc->sumx * P.inv_ncell;
  double s[2] = {0.0, 0.0};
  for (int c = 0; c < 2; ++c) {
    const int W0 = B.W[c][0], W1 = B.W[c][1];
    for (int l = threadIdx.x; l < W0 * W1; l += kBlock) {
      if (!B.cls[c][l]) continue;
      const int i = B.origin[2 * c] + l % W0, j = B.origin[2 * c + 1] + l / W0;
      const double sm = (c == 0) ? st_mu<0>(G, P, mu, i, j, 0, shift)
                                 : st_mu<1>(G, P, mu, i, j, 0, shift);
      s[c] += (double)ub[c][fidx(G.ext[c], i, j, 0)] + sm + (double)ib.f[c][l] / (double)G.dt;
    }
  }
  block_sum<2>(s);
  if (threadIdx.x == 0) {
    stbar[3] += s[0];
    stbar[4] += s[1];
  }
}

// ------------------------------------------------------------ boundary^T
// Outflow correction: ustar_bar_b += s_b A_b K, K = -(1/A_out) sum_out s_b ustar_bar_b;
// zero-gradient outflow then hands its adjoint to the advanced neighbour.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_outflow_sum(Geo<T> G, Planes PL, const T* __restrict__ u0, const T* __restrict__ u1,
                  const T* __restrict__ u2, RedBuf red, SolverScalars* sc) {
  const T* us[3] = {u0, u1, u2};
  int64_t total = 0;
  for (int q = 0; q < PL.np; ++q) total += PL.p[q].count;
  double acc = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < total;
       r += (int64_t)gridDim.x * kBlock) {
    int q = 0;
    while (q + 1 < PL.np && r >= PL.p[q + 1].start) ++q;
    const Plane& Pn = PL.p[q];
    if (Pn.kind != FVIB_BC_OUTFLOW_CONVECTIVE && Pn.kind != FVIB_BC_OUTFLOW_NEUMANN) continue;
    int I[3];
    int64_t rem = r - Pn.start;
    for (int a = 0; a < 3; ++a) {
      if (a == Pn.c) { I[a] = (Pn.side == 0) ? 0 : G.n[a]; continue; }
      I[a] = (int)(rem % G.n[a]);
      rem /= G.n[a];
    }
    const double sign = (Pn.side == 0) ? -1.0 : 1.0;
    acc += sign * (double)us[Pn.c][fidx(G.ext[Pn.c], I[0], I[1], I[2])];
  }
  double v[1] = {acc};
  block_partials<1, 1>(v, red.partial);
}

struct FinAdjOutflow {      // K = -(1/A_out) sum_out s_b ustar_bar_b
  double area_out;
  __device__ bool skip(const SolverScalars*) const { return false; }
  __device__ void apply(const double* t, SolverScalars* sc) const { sc->meanb = -t[0] / area_out; }
};

// mode 0: outflow correction + zero-gradient hand-off (before the momentum
// adjoint); mode 1: convective outflow into ubar^n (after it).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_outflow_apply(Geo<T> G, Planes PL, int mode, T* us0, T* us1, T* us2, T* un0, T* un1,
                    T* un2, const SolverScalars* sc) {
  T* us[3] = {us0, us1, us2};
  T* un[3] = {un0, un1, un2};
  const double K = sc->meanb;
  int64_t total = 0;
  for (int q = 0; q < PL.np; ++q) total += PL.p[q].count;
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < total;
       r += (int64_t)gridDim.x * kBlock) {
    int q = 0;
    while (q + 1 < PL.np && r >= PL.p[q + 1].start) ++q;
    const Plane& Pn = PL.p[q];
    const bool conv = Pn.kind == FVIB_BC_OUTFLOW_CONVECTIVE;
    const bool neum = Pn.kind == FVIB_BC_OUTFLOW_NEUMANN;
    if (!conv && !neum) continue;
    int I[3];
    int64_t rem = r - Pn.start;
    for (int a = 0; a < 3; ++a) {
      if (a == Pn.c) { I[a] = (Pn.side == 0) ? 0 : G.n[a]; continue; }
      I[a] = (int)(rem % G.n[a]);
      rem /= G.n[a];
    }
    const int c = Pn.c;
    const int64_t id = fidx(G.ext[c], I[0], I[1], I[2]);
    int In[3] = {I[0], I[1], I[2]};
    In[c] += (Pn.side == 0) ? 1 : -1;
    const int64_t inner = fidx(G.ext[c], In[0], In[1], In[2]);
    if (mode == 0) {
      double A = 1.0;
      for (int a = 0; a < G.dim; ++a)
        if (a != c) A *= (double)G.dx[a][I[a]];
      const double sign = (Pn.side == 0) ? -1.0 : 1.0;
      const double v = (double)us[c][id] + sign * A * K;
      us[c][id] = (T)v;
      if (neum) us[c][inner] = (T)((double)us[c][inner] + v);
    } else if (conv) {
      const double a = (double)G.dt * PL.u_conv / Pn.h;
      const double v = (double)us[c][id];
      un[c][id] = (T)((double)un[c][id] + (1.0 - a) * v);
      un[c][inner] = (T)((double)un[c][inner] + a * v);
    }
  }
}

// ----------------------------------------------------------- momentum^T
template <typename T>
struct AdjCtx {
  Geo<T> G;
  const T* u[3];      // u^n
  const T* usb[3];    // ustar_bar
  IbView<T> ib;       // point classes; ib.f holds fbar on forced faces
};

// Rbar / dt of component C at face (i, j, k), i.e. ustar_bar, or -fbar / dt
// on a forced face; indices may lie one step outside the array (periodic
// wrap, else zero).  The momentum adjoint gathers with this scaled Rbar and
// multiplies the sum by dt once.
template <int C, int DIM, typename T>
__device__ __forceinline__ T rbar(const AdjCtx<T>& X, int i, int j, int k) {
  int I[3] = {i, j, k};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int e = X.G.ext[C][a];
    if (I[a] < 0) {
      if (!X.G.per[a]) return T(0);
      I[a] += e;
    } else if (I[a] >= e) {
      if (!X.G.per[a]) return T(0);
      I[a] -= e;
    }
  }
  if (!X.G.per[C] && (I[C] < 1 || I[C] > X.G.n[C] - 1)) return T(0);
  if constexpr (C < 2) {
    int li;
    if (forced_cls<C>(X.ib, I[0], I[1], &li)) return -X.ib.f[C][li] / X.G.dt;
  }
  return X.usb[C][fidx(X.G.ext[C], I[0], I[1], I[2])];
}

template <int A_, int DIM, typename T>
__device__ __forceinline__ T ldu(const AdjCtx<T>& X, int i, int j, int k) {
  return ld<A_, DIM>(X.G, X.u[A_], i, j, k);
}

// Generic accessors by runtime component (a small switch).
template <int DIM, typename T>
__device__ __forceinline__ T rbar_c(const AdjCtx<T>& X, int c, int i, int j, int k) {
  if (c == 0) return rbar<0, DIM>(X, i, j, k);
  if (c == 1) return rbar<1, DIM>(X, i, j, k);
  return rbar<2, DIM>(X, i, j, k);
}

template <int DIM, typename T>
__device__ __forceinline__ T ldu_c(const AdjCtx<T>& X, int c, int i, int j, int k) {
  if (c == 0) return ldu<0, DIM>(X, i, j, k);
  if (c == 1) return ldu<1, DIM>(X, i, j, k);
  return ldu<2, DIM>(X, i, j, k);
}

// Gather of every use of u_C(J) in R (convection and diffusion, ghost
// preimages included).  RB(c, di, dj, dk) / U(c, di, dj, dk) return Rbar and
// u^n of component c at an offset of at most one step per axis from J
// (Rbar is zero outside the domain and on faces R does not advance, so the
// terms of stencils that do not exist vanish without a branch; the padded
// coefficient tables keep every index in range).
template <int C, int DIM, bool UPW, typename T, typename RBL, typename UL, typename ML>
__device__ __forceinline__ T adj_gather(const Geo<T>& G, const RBL& RB, const UL& U, const ML& M,
                                        const int J[3]) {
  constexpr int cx = (C == 0), cy = (C == 1), cz = (C == 2);
  const T u0 = U(C, 0, 0, 0), r0 = RB(C, 0, 0, 0);
  const T nu = G.nu;
  const Met4<T> fcm = M.mf(C, -1), fc0 = M.mf(C, 0), fcp = M.mf(C, 1);
  T acc;
  // ---- own axis: convective fluxes at the centres of cells jc-1 and jc,
  // F = Q^2 (central) or Q u_upwind, Q the mean of the two faces; Fbar of a
  // cell is the difference of the scaled Rbar of its two faces
  {
    const T um = U(C, -cx, -cy, -cz), up = U(C, cx, cy, cz);
    const T rm = RB(C, -cx, -cy, -cz), rp = RB(C, cx, cy, cz);
    const T Pb0 = r0 * fc0.x - rm * fcm.x;
    const T Pb1 = rp * fcp.x - r0 * fc0.x;
    const T Q0 = T(0.5) * (um + u0), Q1 = T(0.5) * (u0 + up);
    if constexpr (!UPW) {
      acc = Q0 * Pb0 + Q1 * Pb1;
    } else {
      // J is the upper face of cell jc-1 and the lower face of cell jc
      const T w0 = Q0 > T(0) ? um : (Q0 < T(0) ? u0 : T(0));
      const T w1 = Q1 > T(0) ? u0 : (Q1 < T(0) ? up : T(0));
      const T d0 = T(0.5) * w0 + (Q0 < T(0) ? Q0 : T(0));
      const T d1 = T(0.5) * w1 + (Q1 > T(0) ? Q1 : T(0));
      acc = d0 * Pb0 + d1 * Pb1;
    }
    // own-axis diffusion
    acc += nu * (rm * fcm.y + rp * fcp.z - r0 * (fc0.y + fc0.z));
  }
  // ---- cross axes: the edge at a-face ja (e = 0, J the upper cell) and at
  // a-face ja + 1 (e = 1, J the lower cell).  The edge carries F_C = U V for
  // the C-equation (U: u_C along a, V: u_a along C) and F_a for the
  // a-equation.  Behind a bounded a-boundary the ghost of J sits on the
  // other side of the same edge, so the ghost preimage is the same edge
  // term with the ghost's weight and sign (the a-equation has no flux
  // there: its boundary face is not advanced).
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (a == C) continue;
    const int ax = (a == 0), ay = (a == 1), az = (a == 2);
    const int ja = J[a];
    const Met4<T> cam = M.mc(a, -1), ca0 = M.mc(a, 0), cap = M.mc(a, 1);
    const T ixc_lo = M.mc(C, -1).x, ixc_hi = M.mc(C, 0).x;
    const T wc = fc0.w;
    const bool gb = !G.per[a];
    const T sg_lo = (gb && ja == 0) ? (G.dir[a][0] ? T(-1) : T(1)) : T(0);
    const T sg_hi = (gb && ja == G.n[a] - 1) ? (G.dir[a][1] ? T(-1) : T(1)) : T(0);
    const T rca = RB(C, -ax, -ay, -az), rcb = RB(C, ax, ay, az);
    const T uca = U(C, -ax, -ay, -az), ucb = U(C, ax, ay, az);
    T cross = T(0);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const T wa = M.mf(a, e).w;
      // u_C below / above the edge along a, Rbar_C likewise
      const T cL = e ? u0 : uca, cR = e ? ucb : u0;
      const T rL = e ? r0 : rca, rR = e ? rcb : r0;
      const T FbC = rR * (e ? cap.x : ca0.x) - rL * (e ? ca0.x : cam.x);
      // u_a and Rbar_a on the edge's a-face, C-cells jc-1 and jc
      const T aL = U(a, ax * e - cx, ay * e - cy, az * e - cz);
      const T aR = U(a, ax * e, ay * e, az * e);
      const T Fba = RB(a, ax * e, ay * e, az * e) * ixc_hi -
                    RB(a, ax * e - cx, ay * e - cy, az * e - cz) * ixc_lo;
      const T V = (T(1) - wc) * aL + wc * aR;
      const T wJ = e ? (T(1) - wa) : wa;      // weight of J in U
      const T wG = e ? wa : (T(1) - wa);      // weight of J's ghost in U
      const T sg = e ? sg_hi : sg_lo;
      if constexpr (!UPW) {
        cross += V * (wJ * (FbC + Fba) + sg * wG * FbC);
      } else {
        // F_C = V u_C(upwind of V), F_a = U u_a(upwind of U)
        const bool selJ = e ? (V > T(0)) : (V < T(0));
        const bool selG = e ? (V < T(0)) : (V > T(0));
        const T Uv = (T(1) - wa) * cL + wa * cR;
        const T upa = Uv > T(0) ? aL : (Uv < T(0) ? aR : T(0));
        cross += (selJ ? V * FbC : T(0)) + wJ * upa * Fba + sg * (selG ? V * FbC : T(0));
      }
    }
    acc += cross;
    // cross diffusion, the ghost of J behind a bounded boundary included
    acc += nu * (rca * cam.y + rcb * cap.z - r0 * (ca0.y + ca0.z) +
                   r0 * (sg_lo * ca0.z + sg_hi * ca0.y));
  }
  return acc;
}

// The direct predictor term of an advanced face J, (1 - eps) ustar_bar -
// eps fbar / dt, is the scaled Rbar of J itself (zero on faces that are not
// advanced); the body-force adjoint takes fbbar += Rbar(J) = dt * that.

// Cell-based transposed momentum stencil with LDS halo planes of u^n and
// Rbar (same tiling and z-march as the predictor).  Each thread writes the
// low face of its cell for every component, and the thread of the last cell
// of a bounded axis also the high boundary face of that axis' component.
template <typename T, int DIM>
struct AdjRings {
  T u[DIM][3][kLY][kLX];
  T r[DIM][3][kLY][kLX];
};

// Scaled Rbar for a halo slot: the same values as rbar, with the index arithmetic
// done by selects (zero outside a bounded axis and on faces R does not
// advance).
template <int C, int DIM, typename T>
__device__ __forceinline__ T rb_halo(const AdjCtx<T>& X, int i, int j, int k) {
  const Geo<T>& G = X.G;
  int I[3] = {i, j, k};
  bool out = false;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int e = G.ext[C][a];
    const bool lo = I[a] < 0, hi = I[a] >= e;
    const bool per = G.per[a] != 0;
    I[a] = per ? (lo ? I[a] + e : (hi ? I[a] - e : I[a])) : (lo ? 0 : (hi ? e - 1 : I[a]));
    out = out || (!per && (lo || hi));
  }
  const bool evolved = G.per[C] || (I[C] >= 1 && I[C] <= G.n[C] - 1);
  T v = X.usb[C][fidx(G.ext[C], I[0], I[1], I[2])];
  if constexpr (C < 2) {
    if (X.ib.active) {
      int li = 0;
      if (forced_cls<C>(X.ib, I[0], I[1], &li)) v = -X.ib.f[C][li] / G.dt;
    }
  }
  return (out || !evolved) ? T(0) : v;
}

// Halo slots of one plane in registers (two per thread at most), so the
// loads of plane k + 3 can be in flight while plane k + 1 is computed.
template <typename T, int DIM>
struct AdjRegs {
  T u[2][DIM], r[2][DIM];
};

// The x-y part of the halo rules of this thread's slots, which does not
// change along the z-march: the in-plane offset of each slot per component
// (wrapped on periodic axes, clamped on bounded ones), the ghost rule of u
// (negated about 2 g behind a Dirichlet boundary) and whether the scaled
// Rbar vanishes (outside a bounded axis, or an own-axis face that is not
// advanced), plus the forced-face index of the 2D immersed boundary.  Each
// plane then only adds its (uniform) z part.
template <typename T, int DIM>
struct AdjHalo {
  int xy[2][DIM];
  T goff[2][DIM];                // ghost offset 2 g of u (x-y), used when negated
  uint32_t neg;                  // bit 3 h + c: u negated by an x-y ghost
  uint32_t zr;                   // bit 3 h + c: Rbar zero by the x-y rules
  int li[2][2];                  // forced index of components 0, 1 or -1
};

template <int DIM, typename T>
__device__ __forceinline__ void adj_halo_init(const AdjCtx<T>& X, AdjHalo<T, DIM>& Hh, int i0,
                                              int j0) {
  const Geo<T>& G = X.G;
  Hh.neg = 0u;
  Hh.zr = 0u;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int s = threadIdx.x + h * kBlock;
    const int sy = s / kLX, sx = s - sy * kLX;
    const int gi = min(i0 - 1 + sx, G.n[0]), gj = min(j0 - 1 + sy, G.n[1]);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      int I[2] = {gi, gj};
      T off = T(0);
      bool neg = false, out = false;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int e = G.ext[c][a];
        const bool lo = I[a] < 0, hi = I[a] >= e;
        const bool per = G.per[a] != 0;
        const int wrapped = lo ? I[a] + e : (hi ? I[a] - e : I[a]);
        const int clamped = lo ? 0 : (hi ? e - 1 : I[a]);
        I[a] = per ? wrapped : clamped;
        const bool ghost = !per && (lo || hi);
        const bool dir = lo ? (G.dir[a][0] != 0) : (G.dir[a][1] != 0);
        const T g2 = T(2) * (lo ? G.gv[c][a][0] : G.gv[c][a][1]);
        neg = (ghost && dir) ? true : (ghost ? false : neg);
        off = (ghost && dir) ? g2 : off;
        out = out || ghost;
      }
      Hh.xy[h][c] = I[1] * G.ext[c][0] + I[0];
      Hh.goff[h][c] = off;
      // own-axis face not advanced (x or y component; z is per plane)
      const bool notev = c < 2 && !G.per[c] && (I[c] < 1 || I[c] > G.n[c] - 1);
      Hh.neg |= (neg ? 1u : 0u) << (3 * h + c);
      Hh.zr |= ((out || notev) ? 1u : 0u) << (3 * h + c);
      if (c < 2) {
        int li = -1;
        if (X.ib.active) {
          int l = 0;
          const int f = c == 0 ? forced_cls<0>(X.ib, I[0], I[1], &l) : forced_cls<1>(X.ib, I[0], I[1], &l);
          li = f ? l : -1;
        }
        Hh.li[h][c] = li;
      }
    }
  }
}

template <int DIM, typename T>
__device__ __forceinline__ void adj_load(const AdjCtx<T>& X, const AdjHalo<T, DIM>& Hh,
                                         AdjRegs<T, DIM>& P, int kk) {
  const Geo<T>& G = X.G;
  // z part of the rules for this plane (uniform across the block)
  // (per component: w has one more face than cells along a bounded z)
  int64_t pbase[DIM];
  bool gz[DIM], dz[DIM], zoff[DIM];
  T g2z[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    int kz = 0;
    gz[c] = dz[c] = zoff[c] = false;
    g2z[c] = T(0);
    if constexpr (DIM == 3) {
      const int e = G.ext[c][2];
      const bool lo = kk < 0, hi = kk >= e;
      const bool per = G.per[2] != 0;
      kz = per ? (lo ? kk + e : (hi ? kk - e : kk)) : (lo ? 0 : (hi ? e - 1 : kk));
      gz[c] = !per && (lo || hi);
      dz[c] = lo ? (G.dir[2][0] != 0) : (G.dir[2][1] != 0);
      g2z[c] = T(2) * (lo ? G.gv[c][2][0] : G.gv[c][2][1]);
      zoff[c] = gz[c] || (c == 2 && !G.per[2] && (kz < 1 || kz > G.n[2] - 1));
    }
    pbase[c] = (int64_t)kz * G.ext[c][0] * G.ext[c][1];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int s = threadIdx.x + h * kBlock;
    if (s >= kLX * kLY) break;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int64_t id = pbase[c] + Hh.xy[h][c];
      const T v = X.u[c][id];
      const bool negxy = (Hh.neg >> (3 * h + c)) & 1u;
      const bool neg = gz[c] ? dz[c] : negxy;
      const T off = (gz[c] && dz[c]) ? g2z[c] : Hh.goff[h][c];
      P.u[h][c] = neg ? off - v : v;
      T rv = X.usb[c][id];
      if (c < 2) {
        const int li = Hh.li[h][c];
        if (li >= 0) rv = -X.ib.f[c][li] / G.dt;
      }
      const bool zero = ((Hh.zr >> (3 * h + c)) & 1u) || zoff[c];
      P.r[h][c] = zero ? T(0) : rv;
    }
  }
}

template <int DIM, typename T>
__device__ __forceinline__ void adj_store(AdjRings<T, DIM>& S, int slot, const AdjRegs<T, DIM>& P) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int s = threadIdx.x + h * kBlock;
    if (s >= kLX * kLY) break;
    const int sy = s / kLX, sx = s - sy * kLX;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      S.u[c][slot][sy][sx] = P.u[h][c];
      S.r[c][slot][sy][sx] = P.r[h][c];
    }
  }
}

template <int DIM, typename T>
__device__ __forceinline__ void adj_fill(const AdjCtx<T>& X, const AdjHalo<T, DIM>& Hh,
                                         AdjRings<T, DIM>& S, int slot, int kk) {
  AdjRegs<T, DIM> P;
  adj_load<DIM>(X, Hh, P, kk);
  adj_store<DIM>(S, slot, P);
}

// At most 128 registers (four waves per SIMD): a channel-sized grid then
// runs in one round of blocks.
template <typename T, int DIM, bool UPW>
__global__ void __launch_bounds__(kBlock, 4)
k_adj_momentum_lds(AdjCtx<T> X, int ntx, int nty, int nzc, T* __restrict__ ub0,
                   T* __restrict__ ub1, T* __restrict__ ub2, T* __restrict__ fb0,
                   T* __restrict__ fb1, T* __restrict__ fb2) {
  __shared__ AdjRings<T, DIM> S;
  __shared__ TileMet<T> TM;
  const Geo<T>& G = X.G;
  T* ubar[3] = {ub0, ub1, ub2};
  T* fbb[3] = {fb0, fb1, fb2};
  const int b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= ntx * nty * nzc) return;
  const int tx = b % ntx, ty = (b / ntx) % nty, zc = b / (ntx * nty);
  const int i0 = tx * kTileX, j0 = ty * kTileY;
  // one wavefront per tile row: ly (and so j) is uniform across the wave
  const int lx = threadIdx.x & (kTileX - 1);
  const int ly = __builtin_amdgcn_readfirstlane(threadIdx.x / kTileX);
  const int i = i0 + lx, j = j0 + ly;
  const int k0 = (DIM == 3) ? zc * kZChunk : 0;
  const int k1 = (DIM == 3) ? min(k0 + kZChunk, G.n[2]) : 1;
  const bool inside = i < G.n[0] && j < G.n[1];
  load_tile_met<DIM>(G, TM, i0, j0, k0);
  AdjHalo<T, DIM> Hh;
  adj_halo_init<DIM>(X, Hh, i0, j0);
  AdjRegs<T, DIM> nxt;
  if (DIM == 3) {
    adj_fill<DIM>(X, Hh, S, ring_slot(k0 - 1), k0 - 1);
    adj_fill<DIM>(X, Hh, S, ring_slot(k0), k0);
    adj_fill<DIM>(X, Hh, S, ring_slot(k0 + 1), k0 + 1);
    if (k0 + 1 < k1) adj_load<DIM>(X, Hh, nxt, k0 + 2);
  } else {
    adj_fill<DIM>(X, Hh, S, 0, 0);
  }
  for (int k = k0; k < k1; ++k) {
    __syncthreads();
    const int sc = (DIM == 3) ? ring_slot(k) : 0;
    const int sm = (DIM == 3) ? ring_slot(k - 1) : 0;
    const int sp = (DIM == 3) ? ring_slot(k + 1) : 0;
    if (inside) {
      auto Ul = [&](int c, int di, int dj, int dk) -> T {
        const int sl = dk < 0 ? sm : (dk > 0 ? sp : sc);
        return S.u[c][sl][ly + 1 + dj][lx + 1 + di];
      };
      auto Rl = [&](int c, int di, int dj, int dk) -> T {
        const int sl = dk < 0 ? sm : (dk > 0 ? sp : sc);
        return S.r[c][sl][ly + 1 + dj][lx + 1 + di];
      };
      const int J[3] = {i, j, k};
      const MetLds<T> M{&TM, {lx + 1, ly + 1, k - k0 + 1}};
      // body-force adjoint of the three faces first: its loads overlap the
      // gathers
      int64_t id[3];
      T fbo[3] = {T(0), T(0), T(0)};
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        id[c] = fidx(G.ext[c], i, j, k);
        if (fbb[c]) fbo[c] = fbb[c][id[c]];
      }
#define FVIB_ADJ_COMP(CC)                                                           \
      if (CC < DIM) {                                                               \
        const T rJ = Rl(CC, 0, 0, 0);                                               \
        ubar[CC][id[CC]] = G.dt * adj_gather<CC, DIM, UPW, T>(G, Rl, Ul, M, J) + rJ; \
        if (fbb[CC]) fbb[CC][id[CC]] = fbo[CC] + G.dt * rJ;                         \
      }
      FVIB_ADJ_COMP(0)
      FVIB_ADJ_COMP(1)
      FVIB_ADJ_COMP(2)
#undef FVIB_ADJ_COMP
      // The face on the high boundary of a bounded own axis (index n[C]) is
      // gathered by the thread of the last cell.  Its stencil reaches one
      // step past the tile only for values that multiply its own zero Rbar
      // (a boundary face is not advanced) or the zero Rbar outside, so
      // those indices are clamped into the tile.
#define FVIB_ADJ_HI(CC, SX, SY, SZ)                                                     \
      {                                                                                 \
        auto Uh = [&](int c, int di, int dj, int dk) -> T {                             \
          const int dd = dk + SZ;                                                       \
          const int sl = dd < 0 ? sm : (dd > 0 ? sp : sc);                              \
          return S.u[c][sl][min(ly + 1 + dj + SY, kLY - 1)][min(lx + 1 + di + SX, kLX - 1)]; \
        };                                                                              \
        auto Rh = [&](int c, int di, int dj, int dk) -> T {                             \
          const int dd = dk + SZ;                                                       \
          const int sl = dd < 0 ? sm : (dd > 0 ? sp : sc);                              \
          return S.r[c][sl][min(ly + 1 + dj + SY, kLY - 1)][min(lx + 1 + di + SX, kLX - 1)]; \
        };                                                                              \
        const MetLdsClamp<T> Mh{&TM, {lx + 1 + SX, ly + 1 + SY, k - k0 + 1 + SZ}};      \
        const int Jh[3] = {i + SX, j + SY, k + SZ};                                     \
        ubar[CC][fidx(G.ext[CC], Jh[0], Jh[1], Jh[2])] =                                \
            G.dt * adj_gather<CC, DIM, UPW, T>(G, Rh, Uh, Mh, Jh);                     \
      }
      if (!G.per[0] && i == G.n[0] - 1) FVIB_ADJ_HI(0, 1, 0, 0)
      if (!G.per[1] && j == G.n[1] - 1) FVIB_ADJ_HI(1, 0, 1, 0)
      if constexpr (DIM == 3) {
        if (!G.per[2] && k == G.n[2] - 1) FVIB_ADJ_HI(2, 0, 0, 1)
      }
#undef FVIB_ADJ_HI
    }
    if (DIM == 3 && k + 1 < k1) {
      __syncthreads();
      adj_store<DIM>(S, sm, nxt);                     // slot of plane k-1 takes k+2
      if (k + 2 < k1) adj_load<DIM>(X, Hh, nxt, k + 3);
    }
  }
}


// ============================================================== launchers
template <typename T>
int launch_adj_body_loads(const IbGeo& B, const IbView<T>& ib, const double* st_rk,
                          const double* st_pos, const double* stbar_out, const double* dF,
                          const double* kc, double* stbar_rk, double* stbar_pos, double* kcbar,
                          SolverScalars* sc, int parts, hipStream_t s) {
  launch_kernel((k_adj_body_loads<T>), dim3(1), dim3(kAdjLoadsBlock), 0, s, B, ib, st_rk, st_pos,
                stbar_out, dF, kc, stbar_rk, stbar_pos, kcbar, sc, parts);
  FVIB_HIP(hipGetLastError());
  const int n = B.W[0][0] * B.W[0][1] + B.W[1][0] * B.W[1][1];
  launch_kernel((k_adj_fbar<T>), dim3((n + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0, s, B, st_pos,
                     (const SolverScalars*)sc, (T*)ib.f[0], (T*)ib.f[1]);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_strong_jac(const IbGeo& B, const IbView<T>& ib, const double* om, const double* kc,
                      double* DF, double* RF, hipStream_t s) {
  launch_kernel((k_strong_jac<T>), dim3(1), dim3(kBlock), 0, s, B, ib, om, kc, DF, RF);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

int launch_strong_lambda(const double* DF, const double* RF, const double* wbar,
                         const double* ubody, const double* dF, double* lam, SolverScalars* sc,
                         hipStream_t s) {
  launch_kernel(k_strong_lambda, dim3(1), dim3(64), 0, s, DF, RF, wbar, ubody, dF, lam, sc);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_adj_rhs_residual(const Geo<T>& G, const PGeo<double>& P, const T* const ub[3],
                            const double* x, double* y, double* r64, float* r32, RedBuf red,
                            SolverScalars* sc, double rtol, double max_iv, hipStream_t s,
                            SolverScalars* mirror) {
  const ColTiling ct = make_col_tiling(G.n[0], G.n[1], G.n[2]);
  if (G.dim == 2) {
    if (r64)
      launch_kernel((k_adj_rhs_res_2d<T, 3>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct,
                    ub[0], ub[1], x, y, r64, r32, red);
    else
      launch_kernel((k_adj_rhs_res_2d<T, 2>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct,
                    ub[0], ub[1], x, y, r64, r32, red);
  } else if (r64) {
    launch_kernel((k_adj_rhs_res_col<T, 3>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct,
                  ub[0], ub[1], ub[2], x, y, r64, r32, red);
  } else {
    launch_kernel((k_adj_rhs_res_col<T, 2>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct,
                  ub[0], ub[1], ub[2], x, y, r64, r32, red);
  }
  FVIB_HIP(hipGetLastError());
  FVIB_HIP((launch_finish<5, 3>(red.partial, ct.nblocks, sc,
                                FinAdjRhsResidual{P.inv_ncell, rtol, P.dt_over_rho, 0.5, max_iv,
                                                  mirror},
                                s)));
  return FVIB_OK;
}

template <typename T>
int launch_adj_rhs(const Geo<T>& G, const PGeo<double>& P, const T* const ub[3], double* y,
                   RedBuf red, SolverScalars* sc, double rtol, hipStream_t s) {
  if (G.dim == 3) {
    const ColTiling ct = make_col_tiling(G.n[0], G.n[1], G.n[2]);
    launch_kernel((k_adj_rhs_col<T>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct, ub[0],
                  ub[1], ub[2], y, red);
    FVIB_HIP(hipGetLastError());
    FVIB_HIP((launch_finish<2, 1>(red.partial, ct.nblocks, sc,
                                  FinAdjRhs{P.inv_ncell, rtol, P.dt_over_rho}, s)));
    return FVIB_OK;
  }
  const Tiling tl = make_tiling(G.n[0], G.n[1], G.n[2]);
  launch_kernel((k_adj_rhs<T, 2>), dim3(tl.nblocks), dim3(kBlock), 0, s, G, P, tl, ub[0],
                ub[1], ub[2], y, red, sc);
  FVIB_HIP(hipGetLastError());
  FVIB_HIP((launch_finish<2, 1>(red.partial, tl.nblocks, sc,
                                FinAdjRhs{P.inv_ncell, rtol, P.dt_over_rho}, s)));
  return FVIB_OK;
}

static inline int nblk(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 8 * kMaxRedBlocks) b = 8 * kMaxRedBlocks;
  return (int)(b < 1 ? 1 : b);
}

template <typename T>
int launch_adj_ustar(const Geo<T>& G, const PGeo<double>& P, const T* const ub1[3],
                     const double* mu, const IbView<T>& ib, T* usb[3], const SolverScalars* sc,
                     hipStream_t s, fvib_step_info* info, const double* body_src,
                     double* body_dst, int* sticky) {
  const ColTiling ct = make_col_tiling(G.n[0], G.n[1], G.n[2]);
  if (G.dim == 2)
    launch_kernel((k_adj_ustar<T, 2>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct, ub1[0],
                  ub1[1], ub1[2], mu, ib, usb[0], usb[1], usb[2], sc, info, body_src, body_dst,
                  sticky);
  else
    launch_kernel((k_adj_ustar<T, 3>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct, ub1[0],
                  ub1[1], ub1[2], mu, ib, usb[0], usb[1], usb[2], sc, info, body_src, body_dst,
                  sticky);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_adj_ubody(const Geo<T>& G, const PGeo<double>& P, const IbGeo& B, const T* const ub1[3],
                     const double* mu, const IbView<T>& ib, double* stbar,
                     const SolverScalars* sc, hipStream_t s) {
  launch_kernel((k_adj_ubody<T>), dim3(1), dim3(kBlock), 0, s, G, P, B, ub1[0], ub1[1], mu, ib,
                     stbar, sc);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_adj_outflow(const Geo<T>& G, const Planes& PL, int mode, T* usb[3], T* ubar[3],
                       RedBuf red, SolverScalars* sc, hipStream_t s) {
  if (!PL.any_outflow) return FVIB_OK;
  int64_t total = 0;
  for (int q = 0; q < PL.np; ++q) total += PL.p[q].count;
  int nb = (int)((total + kBlock - 1) / kBlock);
  if (nb > kMaxRedBlocks) nb = kMaxRedBlocks;
  if (nb < 1) nb = 1;
  if (mode == 0) {
    launch_kernel((k_adj_outflow_sum<T>), dim3(nb), dim3(kBlock), 0, s, G, PL, usb[0], usb[1],
                       usb[2], red, sc);
    FVIB_HIP(hipGetLastError());
    FVIB_HIP((launch_finish<1, 1>(red.partial, nb, sc, FinAdjOutflow{PL.area_out}, s)));
  }
  launch_kernel((k_adj_outflow_apply<T>), dim3(nb), dim3(kBlock), 0, s, G, PL, mode, usb[0],
                     usb[1], usb[2], ubar[0], ubar[1], ubar[2], (const SolverScalars*)sc);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <bool UPW, typename T>
static int launch_adj_momentum_t(const AdjCtx<T>& X, T* ubar[3], T* fbbar[3], hipStream_t s);

template <typename T>
int launch_adj_momentum(const Geo<T>& G, const T* const u[3], const T* const usb[3],
                        const IbView<T>& ib, T* ubar[3], T* fbbar[3], hipStream_t s) {
  AdjCtx<T> X;
  X.G = G;
  for (int c = 0; c < 3; ++c) {
    X.u[c] = u[c];
    X.usb[c] = usb[c];
  }
  X.ib = ib;
  if (G.upwind) return launch_adj_momentum_t<true>(X, ubar, fbbar, s);
  return launch_adj_momentum_t<false>(X, ubar, fbbar, s);
}

template <bool UPW, typename T>
static int launch_adj_momentum_t(const AdjCtx<T>& X, T* ubar[3], T* fbbar[3], hipStream_t s) {
  const Geo<T>& G = X.G;
  const int ntx = (G.n[0] + kTileX - 1) / kTileX;
  const int nty = (G.n[1] + kTileY - 1) / kTileY;
  const int nzc = (G.dim == 3) ? (G.n[2] + kZChunk - 1) / kZChunk : 1;
  int nb = ntx * nty * nzc;
  nb = (nb + kXcds - 1) / kXcds * kXcds;
  if (G.dim == 2)
    launch_kernel((k_adj_momentum_lds<T, 2, UPW>), dim3(nb), dim3(kBlock), 0, s, X, ntx,
                  nty, nzc, ubar[0], ubar[1], ubar[2], fbbar[0], fbbar[1], fbbar[2]);
  else
    launch_kernel((k_adj_momentum_lds<T, 3, UPW>), dim3(nb), dim3(kBlock), 0, s, X, ntx,
                  nty, nzc, ubar[0], ubar[1], ubar[2], fbbar[0], fbbar[1], fbbar[2]);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

#define FVIB_INST(T)                                                                            \
  template int launch_adj_body_loads<T>(const IbGeo&, const IbView<T>&, const double*,          \
                                        const double*, const double*, const double*,            \
                                        const double*, double*, double*, double*,               \
                                        SolverScalars*, int, hipStream_t);                      \
  template int launch_strong_jac<T>(const IbGeo&, const IbView<T>&, const double*,              \
                                    const double*, double*, double*, hipStream_t);              \
  template int launch_adj_rhs_residual<T>(const Geo<T>&, const PGeo<double>&,                  \
                                          const T* const[3], const double*, double*, double*,   \
                                          float*, RedBuf, SolverScalars*, double, double,       \
                                          hipStream_t, SolverScalars*);                         \
  template int launch_adj_rhs<T>(const Geo<T>&, const PGeo<double>&, const T* const[3],         \
                                 double*, RedBuf, SolverScalars*, double, hipStream_t);         \
  template int launch_adj_ustar<T>(const Geo<T>&, const PGeo<double>&, const T* const[3],       \
                                   const double*, const IbView<T>&, T* [3],                     \
                                   const SolverScalars*, hipStream_t, fvib_step_info*,        \
                                   const double*, double*, int*);                               \
  template int launch_adj_ubody<T>(const Geo<T>&, const PGeo<double>&, const IbGeo&,            \
                                   const T* const[3], const double*, const IbView<T>&,          \
                                   double*, const SolverScalars*, hipStream_t);                 \
  template int launch_adj_outflow<T>(const Geo<T>&, const Planes&, int, T* [3], T* [3],         \
                                     RedBuf, SolverScalars*, hipStream_t);                      \
  template int launch_adj_momentum<T>(const Geo<T>&, const T* const[3], const T* const[3],      \
                                      const IbView<T>&, T* [3], T* [3], hipStream_t);
FVIB_INST(float)
FVIB_INST(double)
#undef FVIB_INST

}  // namespace fvib
