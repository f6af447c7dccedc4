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

// ------------------------------------------------------------------ kernel
__device__ __forceinline__ double phi4a(double s) {
  s = fabs(s);
  if (s <= 1.0) return (3.0 - 2.0 * s + sqrt(1.0 + 4.0 * s - 4.0 * s * s)) / 8.0;
  if (s <= 2.0) return (5.0 - 2.0 * s - sqrt(-7.0 + 12.0 * s - 4.0 * s * s)) / 8.0;
  return 0.0;
}

// d phi / d s for s >= 0 (the kernel is even; phi'(0) = 0)
__device__ __forceinline__ double dphi4(double s) {
  if (s <= 1.0) return (-2.0 + (4.0 - 8.0 * s) / (2.0 * sqrt(1.0 + 4.0 * s - 4.0 * s * s))) / 8.0;
  if (s <= 2.0) return (-2.0 - (12.0 - 8.0 * s) / (2.0 * sqrt(-7.0 + 12.0 * s - 4.0 * s * s))) / 8.0;
  return 0.0;
}

__device__ __forceinline__ double dh(double r, double h) { return phi4a(r / h) / h; }

// d/dr of d_h(r) = phi(|r|/h)/h
__device__ __forceinline__ double ddh(double r, double h) {
  const double s = fabs(r) / h;
  const double g = dphi4(s) / (h * h);
  return r < 0.0 ? -g : g;
}

// ---------------------------------------------- RK4^T and loads^T (1 block)
// body state st = [d(3), v(3)]; stbar_out = adjoint of the state after the
// step; dF direct force adjoint (may be NULL).  Writes stbar_in (partial:
// the body-velocity part from the fluid is added later), accumulates
// kcbar, stores the total force adjoint in sc->force.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_body_loads(IbGeo B, IbView<T> ib, const double* __restrict__ st,
                 const double* __restrict__ stbar_out, const double* __restrict__ dF,
                 const double* __restrict__ kc, double* __restrict__ stbar_in,
                 double* __restrict__ kcbar, SolverScalars* sc) {
  __shared__ double Fbar_s[3];
  __shared__ double F_s[3];
  if (threadIdx.x == 0) {
    double sb[6];
    for (int a = 0; a < 6; ++a) sb[a] = stbar_out ? stbar_out[a] : 0.0;
    double Fb[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a) Fb[a] = dF ? dF[a] : 0.0;
    double out[6];
    for (int a = 0; a < 6; ++a) out[a] = sb[a];
    if (B.kind == FVIB_BODY_RIGID_SPRING) {
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
    for (int a = 0; a < 6; ++a) stbar_in[a] = out[a];
    for (int a = 0; a < 3; ++a) {
      Fbar_s[a] = Fb[a];
      F_s[a] = sc->force[a];
    }
  }
  __syncthreads();
  // marker-position part: dF_c/dX_k,a = rho h^2 dV_k sum_f f_f d(delta)/dr_a
  const double dxb = st[0], dyb = st[1];
  const double h = B.h;
  double g[2] = {0.0, 0.0};
  for (int k = threadIdx.x; k < B.M; k += kBlock) {
    const double Xx = B.X0[2 * k] + dxb, Xy = B.X0[2 * k + 1] + dyb;
    const double dV = B.ds[k] * h;
    for (int c = 0; c < 2; ++c) {
      const double Fb = Fbar_s[c];
      if (Fb == 0.0) continue;
      const int i0 = (int)floor((Xx - B.fx[c][0]) / h) - 1;
      const int j0 = (int)floor((Xy - B.fy[c][0]) / h) - 1;
      const int ox = ib.origin[2 * c], oy = ib.origin[2 * c + 1];
      double ax = 0.0, ay = 0.0;
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
          ax += f * ddh(rx, h) * dh(ry, h);
          ay += f * dh(rx, h) * ddh(ry, h);
        }
      }
      g[0] += Fb * B.rho * h * h * dV * ax;
      g[1] += Fb * B.rho * h * h * dV * ay;
    }
  }
  block_sum<2>(g);
  if (threadIdx.x == 0) {
    stbar_in[0] += g[0];
    stbar_in[1] += g[1];
    for (int a = 0; a < 3; ++a) sc->force[a] = Fbar_s[a];   // total force adjoint
    (void)F_s;
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
  for (int t = blockIdx.x * kBlock + threadIdx.x; t < n0 + n1; t += gridDim.x * kBlock) {
    const int c = (t < n0) ? 0 : 1;
    const int l = (c == 0) ? t : t - n0;
    if (!B.cls[c][l]) {
      fbar[c][l] = T(0);
      continue;
    }
    const int li = l % B.W[c][0], lj = l / B.W[c][0];
    const int i = B.origin[2 * c] + li, j = B.origin[2 * c + 1] + lj;
    const double px = B.fx[c][i], py = B.fy[c][j];
    double s = 0.0;
    for (int k = 0; k < B.M; ++k) {
      const double Xx = B.X0[2 * k] + st[0], Xy = B.X0[2 * k + 1] + st[1];
      s += B.ds[k] * h * dh(px - Xx, h) * dh(py - Xy, h);
    }
    fbar[c][l] = (T)(-B.rho * h * h * sc->force[c] * s);
  }
}

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
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int ic = I[c], nc = G.n[c];
      if (G.per[c] || ic > 0)
        acc += (double)ub[c][fidx(G.ext[c], i, j, k)] * P.idc[c][ic];
      if (G.per[c] || ic + 1 < nc) {
        int H[3] = {i, j, k};
        H[c] = (ic + 1 == nc) ? 0 : ic + 1;
        acc -= (double)ub[c][fidx(G.ext[c], H[0], H[1], H[2])] * P.idc[c][ic + 1];
      }
    }
    y[((int64_t)k * ny_ + j) * nx_ + i] = acc;
    sum += acc;
    double v = (double)P.dx[0][i] * (double)P.dx[1][j];
    if (DIM == 3) v *= (double)P.dx[2][k];
    mx = fmax(mx, fabs(acc) / v);
  }
  double v[2] = {sum, mx}, tot[2];
  if (grid_reduce<2, 1>(v, red.partial, red.ticket, tot)) {
    if (threadIdx.x == 0) {
      sc->meanb = tot[0] * P.inv_ncell;
      sc->crit = tot[1];
    }
  }
}

template <int C, typename T>
__device__ __forceinline__ int forced_cls(const IbView<T>& ib, int i, int j, int* lidx) {
  if (!ib.active || C > 1) return 0;
  const int li = i - ib.origin[2 * C + 0];
  const int lj = j - ib.origin[2 * C + 1];
  if (li < 0 || lj < 0 || li >= ib.W[C][0] || lj >= ib.W[C][1]) return 0;
  *lidx = lj * ib.W[C][0] + li;
  return ib.cls[C][*lidx];
}

// (S^T mu)_f = A_f (mu_{f-1} - mu_f) with the cells that exist.
template <int C, typename T>
__device__ __forceinline__ double st_mu(const Geo<T>& G, const PGeo<double>& P,
                                        const double* mu, int i, int j, int k) {
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
    lo = mu[((int64_t)L[2] * ny + L[1]) * nx + L[0]];
  }
  if (G.per[C] || ic < nc) {
    int H[3] = {i, j, k};
    H[C] = (ic == nc) ? 0 : ic;
    hi = mu[((int64_t)H[2] * ny + H[1]) * nx + H[0]];
  }
  return A * (lo - hi);
}

// ustar_bar = ubar^{n+1} + (1 - eps) S^T mu on every face of component C.
template <int C, typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_ustar(Geo<T> G, PGeo<double> P, const T* __restrict__ ubar1, const double* __restrict__ mu,
            IbView<T> ib, T* __restrict__ usb) {
  const int e0 = G.ext[C][0], e1 = G.ext[C][1], e2 = G.ext[C][2];
  const int64_t n = (int64_t)e0 * e1 * e2;
  for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < n;
       id += (int64_t)gridDim.x * kBlock) {
    const int i = (int)(id % e0);
    const int j = (int)((id / e0) % e1);
    const int k = (int)(id / ((int64_t)e0 * e1));
    double v = (double)ubar1[id];
    int li;
    if (!forced_cls<C>(ib, i, j, &li)) v += st_mu<C>(G, P, mu, i, j, k);
    usb[id] = (T)v;
  }
}

// Body-velocity adjoint from the forced faces: u_s and u_c equal the rigid
// velocity there, so Ubar_c = sum_forced [ubar^{n+1} + S^T mu + fbar/dt].
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_ubody(Geo<T> G, PGeo<double> P, IbGeo B, const T* __restrict__ ub0,
            const T* __restrict__ ub1, const double* __restrict__ mu, IbView<T> ib,
            double* __restrict__ stbar) {
  const T* ub[2] = {ub0, ub1};
  double s[2] = {0.0, 0.0};
  for (int c = 0; c < 2; ++c) {
    const int W0 = B.W[c][0], W1 = B.W[c][1];
    for (int l = threadIdx.x; l < W0 * W1; l += kBlock) {
      if (!B.cls[c][l]) continue;
      const int i = B.origin[2 * c] + l % W0, j = B.origin[2 * c + 1] + l / W0;
      const double sm = (c == 0) ? st_mu<0>(G, P, mu, i, j, 0) : st_mu<1>(G, P, mu, i, j, 0);
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
  double v[1] = {acc}, tot[1];
  if (grid_reduce<1, 1>(v, red.partial, red.ticket, tot)) {
    if (threadIdx.x == 0) sc->meanb = -tot[0] / PL.area_out;
  }
}

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

// Rbar of component C at face (i, j, k); indices may lie one step outside
// the array (periodic wrap, else zero).
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
    if (forced_cls<C>(X.ib, I[0], I[1], &li)) return -X.ib.f[C][li];
  }
  return X.G.dt * X.usb[C][fidx(X.G.ext[C], I[0], I[1], I[2])];
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
// (Rbar is zero outside the domain and on faces R does not advance).
template <int C, int DIM, typename T, typename RBL, typename UL>
__device__ __forceinline__ T adj_gather(const Geo<T>& G, const RBL& RB, const UL& U,
                                        const int J[3]) {
  const int jc = J[C];
  const bool upw = G.upwind != 0;
  T acc = T(0);
  // ---- own-direction convection: J is the right face of cell jc-1 and the
  // left face of cell jc
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int m = jc - 1 + side;            // cell index along C
    if (!G.per[C] && (m < 0 || m > G.n[C] - 1)) continue;
    const int oL = side - 1, oR = side;     // offsets of faces m, m+1 from J
    const T uL = U(C, C == 0 ? oL : 0, C == 1 ? oL : 0, C == 2 ? oL : 0);
    const T uR = U(C, C == 0 ? oR : 0, C == 1 ? oR : 0, C == 2 ? oR : 0);
    int mm = m;
    if (G.per[C] && mm < 0) mm += G.n[C];
    // Pbar(m) = Cbar(face m)/dc[m] - Cbar(face m+1)/dc[m+1], Cbar = -Rbar
    const T Pb = -RB(C, C == 0 ? oL : 0, C == 1 ? oL : 0, C == 2 ? oL : 0) / G.dc[C][mm] +
                 RB(C, C == 0 ? oR : 0, C == 1 ? oR : 0, C == 2 ? oR : 0) / G.dc[C][m + 1];
    const T Q = T(0.5) * (uL + uR);
    T d;
    if (upw) {
      const T up = Q > T(0) ? uL : (Q < T(0) ? uR : T(0));
      d = T(0.5) * up + (side == 0 ? (Q < T(0) ? Q : T(0)) : (Q > T(0) ? Q : T(0)));
    } else {
      d = Q;
    }
    acc += d * Pb;
  }
  // ---- cross-direction convection through the edge fluxes
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (a == C) continue;
    const int ja = J[a];
    const int na = G.n[a];
    const int nc = G.n[C];
    const T wc = G.wi[C][jc];
    const int ax = (a == 0), ay = (a == 1), az = (a == 2);
    const int cx = (C == 0), cy = (C == 1), cz = (C == 2);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int jj;          // a-face index of the edge
      T sg = T(1);     // ghost sign (1 for a real use)
      bool lower;      // J (or its ghost) is the lower cell jj-1 of the edge
      if (e == 0) { jj = ja; lower = false; }
      else if (e == 1) { jj = ja + 1; lower = true; }
      else if (e == 2) {                // ghost below the low boundary
        if (G.per[a] || ja != 0) continue;
        jj = 0; lower = true;
        sg = G.dir[a][0] ? T(-1) : T(1);
      } else {                          // ghost above the high boundary
        if (G.per[a] || ja != na - 1) continue;
        jj = na; lower = false;
        sg = G.dir[a][1] ? T(-1) : T(1);
      }
      const int oa = jj - ja;           // 0 or 1
      const T wa = G.wi[a][jj];
      const T wJ = lower ? (T(1) - wa) : wa;
      // U = u_C carried along a (cells jj-1, jj), V = u_a carried along C
      const T cL = U(C, ax * (oa - 1), ay * (oa - 1), az * (oa - 1));
      const T cR = U(C, ax * oa, ay * oa, az * oa);
      const T Uv = (T(1) - wa) * cL + wa * cR;
      const T aL = U(a, ax * oa - cx, ay * oa - cy, az * oa - cz);
      const T aR = U(a, ax * oa, ay * oa, az * oa);
      const T V = (T(1) - wc) * aL + wc * aR;
      // flux adjoints of the C-equation (cells jj-1, jj along a) and of the
      // a-equation (cells jc-1, jc along C)
      T FbC = T(0);
      {
        int c0 = jj - 1, c1 = jj;
        if (G.per[a]) {
          if (c0 < 0) c0 += na;
          if (c1 >= na) c1 -= na;
        }
        if (G.per[a] || jj - 1 >= 0)
          FbC += -RB(C, ax * (oa - 1), ay * (oa - 1), az * (oa - 1)) / G.dx[a][c0];
        if (G.per[a] || jj <= na - 1) FbC -= -RB(C, ax * oa, ay * oa, az * oa) / G.dx[a][c1];
      }
      T Fba = T(0);
      {
        int c0 = jc - 1, c1 = jc;
        if (G.per[C]) {
          if (c0 < 0) c0 += nc;
          if (c1 >= nc) c1 -= nc;
        }
        if (G.per[C] || jc - 1 >= 0)
          Fba += -RB(a, ax * oa - cx, ay * oa - cy, az * oa - cz) / G.dx[C][c0];
        if (G.per[C] || jc <= nc - 1) Fba -= -RB(a, ax * oa, ay * oa, az * oa) / G.dx[C][c1];
      }
      T contrib;
      if (!upw) {
        contrib = wJ * V * (FbC + Fba);
      } else {
        // C-equation: F_C = V * (V > 0 ? u_C(jj-1) : V < 0 ? u_C(jj) : 0)
        const bool sel = lower ? (V > T(0)) : (V < T(0));
        const T partC = sel ? V * FbC : T(0);
        // a-equation: F_a = U * (U > 0 ? u_a(jc-1) : U < 0 ? u_a(jc) : 0)
        const T upa = Uv > T(0) ? aL : (Uv < T(0) ? aR : T(0));
        contrib = partC + wJ * upa * Fba;
      }
      acc += sg * contrib;
    }
  }
  // ---- diffusion (transpose), with ghost preimages
  const T nu = G.nu;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int ja = J[a];
    const int na = (a == C) ? G.ext[C][C] : G.n[a];
    const int ax = (a == 0), ay = (a == 1), az = (a == 2);
#pragma unroll
    for (int o = -1; o <= 1; ++o) {
      int ia = ja + o;
      if (G.per[a]) {
        if (ia < 0) ia += na;
        if (ia >= na) ia -= na;
      } else if (ia < 0 || ia >= na) {
        continue;
      }
      const T rb = RB(C, ax * o, ay * o, az * o);
      if (rb == T(0)) continue;
      T hp, hm, H;
      if (a == C) {
        hp = G.dxe[C][ia + 1];
        hm = G.dxe[C][ia];
        H = G.dc[C][ia];
      } else {
        hp = G.dc[a][ia + 1];
        hm = G.dc[a][ia];
        H = G.dx[a][ia];
      }
      T coef;
      if (o == -1) coef = T(1) / (hp * H);           // J = I + e_a
      else if (o == 1) coef = T(1) / (hm * H);       // J = I - e_a
      else coef = -(T(1) / hp + T(1) / hm) / H;
      acc += nu * rb * coef;
      // I = J at a bounded tangential boundary reads a ghost made from J
      if (o == 0 && a != C && !G.per[a]) {
        if (ia == 0) acc += nu * rb * (G.dir[a][0] ? T(-1) : T(1)) / (hm * H);
        if (ia == na - 1) acc += nu * rb * (G.dir[a][1] ? T(-1) : T(1)) / (hp * H);
      }
    }
  }
  return acc;
}

// Direct predictor term of an advanced face J and its body-force adjoint:
// ubar += (1 - eps) ustar_bar - eps fbar / dt,  fbbar += Rbar(J).
template <int C, int DIM, typename T>
__device__ __forceinline__ T adj_direct(const AdjCtx<T>& X, const int J[3], int64_t id, T rJ,
                                        T* __restrict__ fbbar) {
  const Geo<T>& G = X.G;
  const bool evolvedJ = G.per[C] || (J[C] >= 1 && J[C] <= G.n[C] - 1);
  if (!evolvedJ) return T(0);
  T direct = X.usb[C][id];
  if constexpr (C < 2) {
    int li = 0;
    if (forced_cls<C>(X.ib, J[0], J[1], &li)) direct = -X.ib.f[C][li] / G.dt;
  }
  if (fbbar) fbbar[id] += rJ;
  return direct;
}

// Cell-based transposed momentum stencil with LDS halo planes of u^n and
// Rbar (same tiling and z-march as the predictor).  Each thread writes the
// low face of its cell for every component; faces on the high boundary of
// a bounded own axis are left to k_adj_momentum_plane.
template <typename T, int DIM>
struct AdjRings {
  T u[DIM][3][kLY][kLX];
  T r[DIM][3][kLY][kLX];
};

template <int DIM, typename T>
__device__ __forceinline__ void adj_fill(const AdjCtx<T>& X, AdjRings<T, DIM>& S, int slot,
                                         int i0, int j0, int kk) {
  const Geo<T>& G = X.G;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    for (int s = threadIdx.x; s < kLX * kLY; s += kBlock) {
      const int sy = s / kLX, sx = s - sy * kLX;
      const int gi = min(i0 - 1 + sx, G.n[0]), gj = min(j0 - 1 + sy, G.n[1]);
      S.u[c][slot][sy][sx] = ldu_c<DIM>(X, c, gi, gj, kk);
      S.r[c][slot][sy][sx] = rbar_c<DIM>(X, c, gi, gj, kk);
    }
  }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock)
k_adj_momentum_lds(AdjCtx<T> X, int ntx, int nty, int nzc, T* __restrict__ ub0,
                   T* __restrict__ ub1, T* __restrict__ ub2, T* __restrict__ fb0,
                   T* __restrict__ fb1, T* __restrict__ fb2) {
  __shared__ AdjRings<T, DIM> S;
  const Geo<T>& G = X.G;
  T* ubar[3] = {ub0, ub1, ub2};
  T* fbb[3] = {fb0, fb1, fb2};
  const int b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= ntx * nty * nzc) return;
  const int tx = b % ntx, ty = (b / ntx) % nty, zc = b / (ntx * nty);
  const int i0 = tx * kTileX, j0 = ty * kTileY;
  const int lx = threadIdx.x & (kTileX - 1), ly = threadIdx.x / kTileX;
  const int i = i0 + lx, j = j0 + ly;
  const int k0 = (DIM == 3) ? zc * kZChunk : 0;
  const int k1 = (DIM == 3) ? min(k0 + kZChunk, G.n[2]) : 1;
  const bool inside = i < G.n[0] && j < G.n[1];
  if (DIM == 3) {
    adj_fill<DIM>(X, S, ring_slot(k0 - 1), i0, j0, k0 - 1);
    adj_fill<DIM>(X, S, ring_slot(k0), i0, j0, k0);
    adj_fill<DIM>(X, S, ring_slot(k0 + 1), i0, j0, k0 + 1);
  } else {
    adj_fill<DIM>(X, S, 0, i0, j0, 0);
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
#define FVIB_ADJ_COMP(CC)                                                           \
      if (CC < DIM) {                                                               \
        const int64_t id = fidx(G.ext[CC], i, j, k);                                \
        T acc = adj_gather<CC, DIM, T>(G, Rl, Ul, J);                               \
        acc += adj_direct<CC, DIM, T>(X, J, id, Rl(CC, 0, 0, 0), fbb[CC]);          \
        ubar[CC][id] = acc;                                                         \
      }
      FVIB_ADJ_COMP(0)
      FVIB_ADJ_COMP(1)
      FVIB_ADJ_COMP(2)
#undef FVIB_ADJ_COMP
    }
    if (DIM == 3 && k + 1 < k1) {
      __syncthreads();
      adj_fill<DIM>(X, S, sm, i0, j0, k + 2);
    }
  }
}

// Faces on the high boundary of a bounded own axis (face index n[C]).
template <int C, int DIM, typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_momentum_plane(AdjCtx<T> X, T* __restrict__ ubar) {
  const Geo<T>& G = X.G;
  int64_t count = 1;
  for (int a = 0; a < 3; ++a)
    if (a != C) count *= G.n[a];
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < count;
       r += (int64_t)gridDim.x * kBlock) {
    int J[3];
    int64_t rem = r;
    for (int a = 0; a < 3; ++a) {
      if (a == C) { J[a] = G.n[C]; continue; }
      J[a] = (int)(rem % G.n[a]);
      rem /= G.n[a];
    }
    auto Ug = [&](int c, int di, int dj, int dk) -> T {
      return ldu_c<DIM>(X, c, J[0] + di, J[1] + dj, J[2] + dk);
    };
    auto Rg = [&](int c, int di, int dj, int dk) -> T {
      return rbar_c<DIM>(X, c, J[0] + di, J[1] + dj, J[2] + dk);
    };
    ubar[fidx(G.ext[C], J[0], J[1], J[2])] = adj_gather<C, DIM, T>(G, Rg, Ug, J);
  }
}

// ============================================================== launchers
template <typename T>
int launch_adj_body_loads(const IbGeo& B, const IbView<T>& ib, const double* st,
                          const double* stbar_out, const double* dF, const double* kc,
                          double* stbar_in, double* kcbar, SolverScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL((k_adj_body_loads<T>), dim3(1), dim3(kBlock), 0, s, B, ib, st, stbar_out, dF,
                     kc, stbar_in, kcbar, sc);
  FVIB_HIP(hipGetLastError());
  const int n = B.W[0][0] * B.W[0][1] + B.W[1][0] * B.W[1][1];
  hipLaunchKernelGGL((k_adj_fbar<T>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, B, st,
                     (const SolverScalars*)sc, (T*)ib.f[0], (T*)ib.f[1]);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_adj_rhs(const Geo<T>& G, const PGeo<double>& P, const T* const ub[3], double* y,
                   RedBuf red, SolverScalars* sc, hipStream_t s) {
  const Tiling tl = make_tiling(G.n[0], G.n[1], G.n[2]);
  if (G.dim == 2)
    hipLaunchKernelGGL((k_adj_rhs<T, 2>), dim3(tl.nblocks), dim3(kBlock), 0, s, G, P, tl, ub[0],
                       ub[1], ub[2], y, red, sc);
  else
    hipLaunchKernelGGL((k_adj_rhs<T, 3>), dim3(tl.nblocks), dim3(kBlock), 0, s, G, P, tl, ub[0],
                       ub[1], ub[2], y, red, sc);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

static inline int nblk(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 8 * kMaxRedBlocks) b = 8 * kMaxRedBlocks;
  return (int)(b < 1 ? 1 : b);
}

template <typename T>
int launch_adj_ustar(const Geo<T>& G, const PGeo<double>& P, const T* const ub1[3],
                     const double* mu, const IbView<T>& ib, T* usb[3], hipStream_t s) {
  for (int c = 0; c < G.dim; ++c) {
    const int64_t n = (int64_t)G.ext[c][0] * G.ext[c][1] * G.ext[c][2];
    if (c == 0)
      hipLaunchKernelGGL((k_adj_ustar<0, T>), dim3(nblk(n)), dim3(kBlock), 0, s, G, P, ub1[0], mu, ib, usb[0]);
    else if (c == 1)
      hipLaunchKernelGGL((k_adj_ustar<1, T>), dim3(nblk(n)), dim3(kBlock), 0, s, G, P, ub1[1], mu, ib, usb[1]);
    else
      hipLaunchKernelGGL((k_adj_ustar<2, T>), dim3(nblk(n)), dim3(kBlock), 0, s, G, P, ub1[2], mu, ib, usb[2]);
    FVIB_HIP(hipGetLastError());
  }
  return FVIB_OK;
}

template <typename T>
int launch_adj_ubody(const Geo<T>& G, const PGeo<double>& P, const IbGeo& B, const T* const ub1[3],
                     const double* mu, const IbView<T>& ib, double* stbar, hipStream_t s) {
  hipLaunchKernelGGL((k_adj_ubody<T>), dim3(1), dim3(kBlock), 0, s, G, P, B, ub1[0], ub1[1], mu, ib,
                     stbar);
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
    hipLaunchKernelGGL((k_adj_outflow_sum<T>), dim3(nb), dim3(kBlock), 0, s, G, PL, usb[0], usb[1],
                       usb[2], red, sc);
    FVIB_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL((k_adj_outflow_apply<T>), dim3(nb), dim3(kBlock), 0, s, G, PL, mode, usb[0],
                     usb[1], usb[2], ubar[0], ubar[1], ubar[2], (const SolverScalars*)sc);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

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
  const int ntx = (G.n[0] + kTileX - 1) / kTileX;
  const int nty = (G.n[1] + kTileY - 1) / kTileY;
  const int nzc = (G.dim == 3) ? (G.n[2] + kZChunk - 1) / kZChunk : 1;
  int nb = ntx * nty * nzc;
  nb = (nb + kXcds - 1) / kXcds * kXcds;
  if (G.dim == 2)
    hipLaunchKernelGGL((k_adj_momentum_lds<T, 2>), dim3(nb), dim3(kBlock), 0, s, X, ntx, nty, nzc,
                       ubar[0], ubar[1], ubar[2], fbbar[0], fbbar[1], fbbar[2]);
  else
    hipLaunchKernelGGL((k_adj_momentum_lds<T, 3>), dim3(nb), dim3(kBlock), 0, s, X, ntx, nty, nzc,
                       ubar[0], ubar[1], ubar[2], fbbar[0], fbbar[1], fbbar[2]);
  FVIB_HIP(hipGetLastError());
  for (int c = 0; c < G.dim; ++c) {
    if (G.per[c]) continue;
    int64_t count = 1;
    for (int a = 0; a < 3; ++a)
      if (a != c) count *= G.n[a];
    const dim3 gr(nblk(count)), bl(kBlock);
    if (G.dim == 2) {
      if (c == 0) hipLaunchKernelGGL((k_adj_momentum_plane<0, 2, T>), gr, bl, 0, s, X, ubar[0]);
      else hipLaunchKernelGGL((k_adj_momentum_plane<1, 2, T>), gr, bl, 0, s, X, ubar[1]);
    } else {
      if (c == 0) hipLaunchKernelGGL((k_adj_momentum_plane<0, 3, T>), gr, bl, 0, s, X, ubar[0]);
      else if (c == 1) hipLaunchKernelGGL((k_adj_momentum_plane<1, 3, T>), gr, bl, 0, s, X, ubar[1]);
      else hipLaunchKernelGGL((k_adj_momentum_plane<2, 3, T>), gr, bl, 0, s, X, ubar[2]);
    }
    FVIB_HIP(hipGetLastError());
  }
  return FVIB_OK;
}

#define FVIB_INST(T)                                                                            \
  template int launch_adj_body_loads<T>(const IbGeo&, const IbView<T>&, const double*,          \
                                        const double*, const double*, const double*, double*,   \
                                        double*, SolverScalars*, hipStream_t);                  \
  template int launch_adj_rhs<T>(const Geo<T>&, const PGeo<double>&, const T* const[3],         \
                                 double*, RedBuf, SolverScalars*, hipStream_t);                 \
  template int launch_adj_ustar<T>(const Geo<T>&, const PGeo<double>&, const T* const[3],       \
                                   const double*, const IbView<T>&, T* [3], hipStream_t);       \
  template int launch_adj_ubody<T>(const Geo<T>&, const PGeo<double>&, const IbGeo&,            \
                                   const T* const[3], const double*, const IbView<T>&,          \
                                   double*, hipStream_t);                                       \
  template int launch_adj_outflow<T>(const Geo<T>&, const Planes&, int, T* [3], T* [3],         \
                                     RedBuf, SolverScalars*, hipStream_t);                      \
  template int launch_adj_momentum<T>(const Geo<T>&, const T* const[3], const T* const[3],      \
                                      const IbView<T>&, T* [3], T* [3], hipStream_t);
FVIB_INST(float)
FVIB_INST(double)
#undef FVIB_INST

}  // namespace fvib
