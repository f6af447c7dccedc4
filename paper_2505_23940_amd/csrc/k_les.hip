// Large-eddy simulation terms: the constant-coefficient Smagorinsky
// subgrid stress (Sec. 2.5, Table 1) and the equilibrium wall-stress model
// with the Spalding law (Sec. 3.4.5, Eqs. 27-29), forward and adjoint.
//
// Discretisation on the MAC grid (3D; every axis periodic or a no-slip
// wall pair):
//   * nu_t = (C_s Delta)^2 |S| at cell centres, Delta = (dx dy dz)^(1/3),
//     |S| = sqrt(2 S_ij S_ij); the diagonal of S from the cell's two faces,
//     an off-diagonal entry as the mean of (d_a u_c + d_c u_a) / 2 on the
//     four edges around the centre in that plane;
//   * edge gradient G = d_a u_c + d_c u_a: differences of the two values
//     beside the edge over their centre spacing, behind a wall the mirrored
//     ghost 2 g - u_0 (as in the molecular term);
//   * the subgrid term added to R on the evolved faces is the divergence of
//     2 nu_t S: normal stresses 2 nu_t d_c u_c at the cells, shear stresses
//     nu_e G on the edges, nu_e the mean of the four cells around an
//     interior edge, zero on a wall edge unless the wall model sets it;
//   * wall model (walls normal to y, x and z periodic): at each streamwise
//     and spanwise face of the first cell row, U = |(u, w) - wall velocity|
//     with the other component the mean of its four nearest faces in the
//     row, u_tau from the Spalding law at the half height of the wall cell
//     (Newton-Raphson on ln u+, safeguarded by bisection), tau_w = u_tau^2,
//     the component tau_w u_i / U (Eq. 29), and the wall-edge viscosity
//     tau_i / (du_i/dn + eps) - nu (Eq. 28), du_i/dn = (u_i - u_wall)/y.
// The forward pass hands the predictor g = fb + subgrid term as its body
// force, so the direct forcing and every later sub-step see the full R.
//
// Adjoint: with gbar the adjoint of g, the subgrid term is bilinear in
// (viscosity, velocity gradients).  Sites (cells and edges) first collect
// the stress adjoint from the faces they feed (tau_bar); a cell then sums
// its viscosity adjoint (its own normal stresses and a quarter of each
// interior edge around it), pushes it through |S|, and the edges gather
// the strain adjoint of the four cells around them; the wall faces push the
// wall-edge viscosity adjoint through Eqs. 27-29; finally every face
// gathers the coefficients of the gradients it appears in.  Every pass is a
// gather (one writer per output), so the result is deterministic.
//
// The kernels are grid-stride loops over plain global loads: the subgrid
// passes are small next to the pressure solve of the same step.
#include <math.h>

#include "fvib_internal.h"
#include "fvib_kernels.h"

namespace fvib {

namespace {

template <typename T>
struct U3 {
  const T* c[3];
};

template <int C, typename T>
__device__ __forceinline__ T ldu(const Geo<T>& G, const T* __restrict__ q, const int P[3]) {
  return ld<C, 3, T>(G, q, P[0], P[1], P[2]);
}

// 1 / centre spacing at face f and 1 / cell width at cell i (tables hold
// entries -1 .. n + 1 and -1 .. n, wrapped on periodic axes).
template <typename T>
__device__ __forceinline__ T idc(const Geo<T>& G, int a, int f) { return G.mf[a][f].x; }
template <typename T>
__device__ __forceinline__ T idx(const Geo<T>& G, int a, int i) { return G.mc[a][i].x; }

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ int64_t cidx(const Geo<T>& G, int i, int j, int k) {
  return ((int64_t)k * G.n[1] + j) * G.n[0] + i;
}

template <typename T>
__device__ __forceinline__ int64_t eidx(const Geo<T>& G, const int E[3]) {
  return ((int64_t)E[2] * (G.n[1] + 1) + E[1]) * (G.n[0] + 1) + E[0];
}

// nu_t of cell P (periodic axes wrapped; bounded indices in range).
template <typename T>
__device__ __forceinline__ T nut_at(const Geo<T>& G, const T* __restrict__ nut, const int P[3]) {
  int I[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) I[a] = G.per[a] ? wrapi(P[a], G.n[a]) : P[a];
  return nut[cidx(G, I[0], I[1], I[2])];
}

// G = d_A u_C + d_C u_A on edge E (E[C], E[A] face indices, E[B] cell).
template <int C, int A, typename T>
__device__ __forceinline__ T edge_grad(const Geo<T>& G, const U3<T>& u, const int E[3]) {
  int P[3] = {E[0], E[1], E[2]};
  const T c1 = ldu<C>(G, u.c[C], P);
  P[A] = E[A] - 1;
  const T c0 = ldu<C>(G, u.c[C], P);
  int Q[3] = {E[0], E[1], E[2]};
  const T a1 = ldu<A>(G, u.c[A], Q);
  Q[C] = E[C] - 1;
  const T a0 = ldu<A>(G, u.c[A], Q);
  return (c1 - c0) * idc(G, A, E[A]) + (a1 - a0) * idc(G, C, E[C]);
}

template <int C, int A, typename T>
__device__ __forceinline__ bool edge_on_wall(const Geo<T>& G, const int E[3]) {
  return (!G.per[C] && (E[C] == 0 || E[C] == G.n[C])) ||
         (!G.per[A] && (E[A] == 0 || E[A] == G.n[A]));
}

// Viscosity on edge E of the (C, A) plane.
template <int C, int A, typename T>
__device__ __forceinline__ T edge_nu(const Geo<T>& G, const LesView<T>& L, const int E[3]) {
  if (edge_on_wall<C, A>(G, E)) {
    if constexpr ((C == 0 && A == 1) || (C == 1 && A == 2)) {
      if (L.wall) {
        // the y walls: x-y edges carry u's, y-z edges w's wall viscosity
        const int side = E[1] == 0 ? 0 : 1;
        const int i = (C == 0 && E[0] == G.n[0]) ? 0 : E[0];
        const int k = (A == 2 && E[2] == G.n[2]) ? 0 : E[2];
        return (T)L.nuw[C == 0 ? 0 : 1][side][(int64_t)k * G.n[0] + i];
      }
    }
    return T(0);
  }
  T s = T(0);
#pragma unroll
  for (int dc = -1; dc <= 0; ++dc)
#pragma unroll
    for (int da = -1; da <= 0; ++da) {
      int P[3] = {E[0], E[1], E[2]};
      P[C] += dc;
      P[A] += da;
      s += nut_at(G, L.nut, P);
    }
  return T(0.25) * s;
}

// Cell strain: diagonal and the three off-diagonal entries (x-y, x-z, y-z),
// the latter from the edge gradients stored by k_les_grad.
template <typename T>
__device__ __forceinline__ void cell_strain(const Geo<T>& G, const LesView<T>& L, const U3<T>& u,
                                            int i, int j, int k, T sd[3], T so[3]) {
  const int P0[3] = {i, j, k};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int P[3] = {i, j, k};
    P[c] += 1;
    T hi, lo;
    if (c == 0) { hi = ldu<0>(G, u.c[0], P); lo = ldu<0>(G, u.c[0], P0); }
    else if (c == 1) { hi = ldu<1>(G, u.c[1], P); lo = ldu<1>(G, u.c[1], P0); }
    else { hi = ldu<2>(G, u.c[2], P); lo = ldu<2>(G, u.c[2], P0); }
    sd[c] = (hi - lo) * idx(G, c, P0[c]);
  }
  T s01 = 0, s02 = 0, s12 = 0;
#pragma unroll
  for (int p = 0; p <= 1; ++p)
#pragma unroll
    for (int q = 0; q <= 1; ++q) {
      const int E01[3] = {i + p, j + q, k};
      const int E02[3] = {i + p, j, k + q};
      const int E12[3] = {i, j + p, k + q};
      s01 += L.ge[0][eidx(G, E01)];
      s02 += L.ge[1][eidx(G, E02)];
      s12 += L.ge[2][eidx(G, E12)];
    }
  so[0] = T(0.125) * s01;
  so[1] = T(0.125) * s02;
  so[2] = T(0.125) * s12;
}

template <typename T>
__device__ __forceinline__ T delta2(const Geo<T>& G, int i, int j, int k) {
  const T v = G.dx[0][i] * G.dx[1][j] * G.dx[2][k];
  const T d = cbrt(v);
  return d * d;
}

// ------------------------------------------------------------ Spalding law
// u+ of Eq. 27 for Re = U y / nu > 0 (u+ below 200), and du+/dRe.
// Newton-Raphson on h(t) = t + ln y+(e^t) - ln Re with t = ln u+ (u+ y+ =
// Re): first in float from the upper end of the bracket [t_hi - 80, t_hi],
// t_hi = min(ln sqrt(Re), ln 200) (y+ >= u+ puts the root below sqrt(Re)),
// a step leaving the bracket replaced by bisection, until |h| or a step is
// below about 2e-5 (h' >= 1, so t is then that close to the root); then
// three Newton steps in double.  du+/dRe = 1 / (y+ + u+ dy+/du+),
// from differentiating Re = u+ y+(u+).
__device__ double spalding_uplus(double re, double kappa, double B, double* dup_dre) {
  const double lre = log(re);
  const double e = exp(-kappa * B);
  // bracketed phase in float (hardware exp / log): the root to ~1e-6 in t
  const float lref = (float)lre, kf = (float)kappa, ef = (float)e;
  float hi = fminf(0.5f * lref, 5.298317f), lo = hi - 80.0f, tf = hi;    // ln 200
  for (int it = 0; it < 100; ++it) {
    const float up = __expf(tf), k = kf * up, ek = __expf(k);
    const float yp = up + ef * (ek - 1.0f - k - 0.5f * k * k - k * k * k * (1.0f / 6.0f));
    const float dyp = 1.0f + ef * kf * (ek - 1.0f - k - 0.5f * k * k);
    const float h = tf + __logf(yp) - lref, dh = 1.0f + up * dyp / yp;
    if (fabsf(h) <= 3e-5f) break;      // dh >= 1: within 3e-5 of the root
    if (h < 0.0f) lo = tf;
    if (h > 0.0f) hi = tf;
    float tn = tf - h / dh;
    if (!(tn > lo && tn < hi)) tn = 0.5f * (lo + hi);
    const bool done = fabsf(tn - tf) <= 2e-5f;
    tf = tn;
    if (done) break;
  }
  // Newton in double from there: quadratic convergence takes the 1e-6
  // start to rounding level in two steps; a third confirms it
  auto eval = [&](double tt, double* h, double* dh) {
    const double up = exp(tt), k = kappa * up, ek = exp(k);
    const double yp = up + e * (ek - 1.0 - k - 0.5 * k * k - k * k * k / 6.0);
    const double dyp = 1.0 + e * kappa * (ek - 1.0 - k - 0.5 * k * k);
    *h = tt + log(yp) - lre;
    *dh = 1.0 + up * dyp / yp;
  };
  double t = tf;
  for (int it = 0; it < 3; ++it) {
    double h, dh;
    eval(t, &h, &dh);
    t -= h / dh;
  }
  const double up = exp(t), k = kappa * up, ek = exp(k);
  const double yp = up + e * (ek - 1.0 - k - 0.5 * k * k - k * k * k / 6.0);
  const double dyp = 1.0 + e * kappa * (ek - 1.0 - k - 0.5 * k * k);
  *dup_dre = 1.0 / (yp + up * dyp);
  return up;
}

// Wall face (comp 0: u at x-face i, comp 1: w at z-face k) of the first
// row next to wall `side`: its own velocity and the other component's
// four-face mean, both relative to the wall.
template <typename T>
__device__ __forceinline__ void wall_pair(const Geo<T>& G, const LesView<T>& L, const U3<T>& u,
                                          int comp, int side, int i, int k, double* own,
                                          double* oth) {
  const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
  const int j = side == 0 ? 0 : ny - 1;
  auto at = [&](const T* q, int ii, int kk) {
    return (double)q[((int64_t)wrapi(kk, nz) * ny + j) * nx + wrapi(ii, nx)];
  };
  if (comp == 0) {
    *own = at(u.c[0], i, k) - L.uw[side][0];
    *oth = 0.25 * (at(u.c[2], i - 1, k) + at(u.c[2], i, k) + at(u.c[2], i - 1, k + 1) +
                   at(u.c[2], i, k + 1)) - L.uw[side][2];
  } else {
    *own = at(u.c[2], i, k) - L.uw[side][2];
    *oth = 0.25 * (at(u.c[0], i, k - 1) + at(u.c[0], i + 1, k - 1) + at(u.c[0], i, k) +
                   at(u.c[0], i + 1, k)) - L.uw[side][0];
  }
}

// u+ (Eq. 27) at tangential speed U > 0 and du+/dRe.
template <typename T>
__device__ __forceinline__ double wall_uplus(const LesView<T>& L, int side, double U, double* dup) {
  return spalding_uplus(U * L.yw[side] / L.nu, L.kappa, L.B, dup);
}

// Wall-edge viscosity (Eq. 28) and its partial derivatives in the own and
// the other velocity, given u+ and du+/dRe at U = |(own, oth)| (unused
// when U = 0: no stress).
template <typename T>
__device__ __forceinline__ double wall_nu(const LesView<T>& L, int side, double own, double oth,
                                          double up, double dup, double* d_own, double* d_oth) {
  const double y = L.yw[side];
  const double U = sqrt(own * own + oth * oth);
  double taui = 0.0, dti_own = 0.0, dti_oth = 0.0;
  if (U > 0.0) {
    const double tau = (U / up) * (U / up);
    // d tau / dU with u+ = u+(U y / nu)
    const double dtau = 2.0 * U / (up * up) - 2.0 * U * U / (up * up * up) * dup * (y / L.nu);
    const double r = own / U, s = oth / U;
    taui = tau * r;
    dti_own = dtau * r * r + tau * (1.0 - r * r) / U;
    dti_oth = dtau * r * s - tau * r * s / U;
  }
  const double den = own / y + L.eps;
  *d_own = dti_own / den - taui / (den * den * y);
  *d_oth = dti_oth / den;
  return taui / den - L.nu;
}

// ----------------------------------------------------------------- forward
template <int C, int A, typename T>
__device__ __forceinline__ void store_grad(const Geo<T>& G, const LesView<T>& L, const U3<T>& u,
                                           const int E[3]) {
  constexpr int B = 3 - C - A;
  if (E[B] >= G.n[B]) return;
  L.ge[C + A - 1][eidx(G, E)] = edge_grad<C, A>(G, u, E);
}

// Edge gradients of the three planes on the whole edge lattice.
template <typename T>
__device__ __forceinline__ void les_grad_sites(const Geo<T>& G, const LesView<T>& L,
                                               const U3<T>& u, int blk, int nblk) {
  const int l0 = G.n[0] + 1, l1 = G.n[1] + 1;
  const int64_t n = (int64_t)l0 * l1 * (G.n[2] + 1);
  for (int64_t id = (int64_t)blk * kBlock + threadIdx.x; id < n; id += (int64_t)nblk * kBlock) {
    const int E[3] = {(int)(id % l0), (int)((id / l0) % l1), (int)(id / ((int64_t)l0 * l1))};
    store_grad<0, 1>(G, L, u, E);
    store_grad<0, 2>(G, L, u, E);
    store_grad<1, 2>(G, L, u, E);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_les_nut(Geo<T> G, LesView<T> L, U3<T> u) {
  const int64_t n = (int64_t)G.n[0] * G.n[1] * G.n[2];
  for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < n;
       id += (int64_t)gridDim.x * kBlock) {
    const int i = (int)(id % G.n[0]);
    const int j = (int)((id / G.n[0]) % G.n[1]);
    const int k = (int)(id / ((int64_t)G.n[0] * G.n[1]));
    T sd[3], so[3];
    cell_strain(G, L, u, i, j, k, sd, so);
    const T ss = sd[0] * sd[0] + sd[1] * sd[1] + sd[2] * sd[2] +
                 T(2) * (so[0] * so[0] + so[1] * so[1] + so[2] * so[2]);
    L.nut[id] = L.cs2 * delta2(G, i, j, k) * sqrt(T(2) * ss);
  }
}

template <typename T>
__device__ __forceinline__ void les_wall_faces(const Geo<T>& G, const LesView<T>& L,
                                               const U3<T>& u, int blk, int nblk) {
  const int nx = G.n[0], nz = G.n[2];
  const int64_t n = 4 * (int64_t)nx * nz;
  for (int64_t id = (int64_t)blk * kBlock + threadIdx.x; id < n; id += (int64_t)nblk * kBlock) {
    const int i = (int)(id % nx);
    const int k = (int)((id / nx) % nz);
    const int side = (int)((id / ((int64_t)nx * nz)) % 2);
    const int comp = (int)(id / (2 * (int64_t)nx * nz));
    double own, oth, d1, d2, dup = 0.0, up = 1.0;
    wall_pair(G, L, u, comp, side, i, k, &own, &oth);
    const double U = sqrt(own * own + oth * oth);
    if (U > 0.0) up = wall_uplus(L, side, U, &dup);
    const int64_t w = (int64_t)k * nx + i;
    L.upl[comp][side][w] = up;       // kept for the adjoint of this state
    L.dupl[comp][side][w] = dup;
    L.nuw[comp][side][w] = wall_nu(L, side, own, oth, up, dup, &d1, &d2);
  }
}

// The edge gradients and, with the wall model, the wall faces' Eq. 27 solve
// in one launch: both read u only.  Blocks [0, bg) take the edge lattice,
// the rest the wall faces.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_les_grad(Geo<T> G, LesView<T> L, U3<T> u, int bg) {
  const int b = blockIdx.x;
  if (b < bg)
    les_grad_sites(G, L, u, b, bg);
  else
    les_wall_faces(G, L, u, b - bg, (int)gridDim.x - bg);
}

template <int C, int A, typename T>
__device__ __forceinline__ T shear(const Geo<T>& G, const LesView<T>& L, const int E[3]) {
  constexpr int lo = C < A ? C : A, hi = C < A ? A : C;
  return edge_nu<lo, hi>(G, L, E) * L.ge[lo + hi - 1][eidx(G, E)];
}

// The faces of component C taken by blocks blk = 0 .. nblk - 1 of a range.
template <int C, typename T>
__device__ __forceinline__ void les_force_faces(const Geo<T>& G, const LesView<T>& L,
                                                const U3<T>& u, const T* __restrict__ fb,
                                                T* __restrict__ g, int blk, int nblk) {
  constexpr int A1 = (C + 1) % 3, A2 = (C + 2) % 3;
  const int e0 = G.ext[C][0], e1 = G.ext[C][1], e2 = G.ext[C][2];
  const int64_t n = (int64_t)e0 * e1 * e2;
  for (int64_t id = (int64_t)blk * kBlock + threadIdx.x; id < n; id += (int64_t)nblk * kBlock) {
    const int F[3] = {(int)(id % e0), (int)((id / e0) % e1), (int)(id / ((int64_t)e0 * e1))};
    const T base = fb ? fb[id] : T(0);
    const bool ev = G.per[C] || (F[C] >= 1 && F[C] <= G.n[C] - 1);
    if (!ev) {
      g[id] = base;
      continue;
    }
    // normal stress 2 nu_t d_C u_C at cells F[C] - 1 and F[C]
    T tn[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      int P[3] = {F[0], F[1], F[2]};
      const int cell = G.per[C] ? wrapi(F[C] - 1 + s, G.n[C]) : F[C] - 1 + s;
      P[C] = cell;
      const T lo = ldu<C>(G, u.c[C], P);
      P[C] = cell + 1;
      const T hi = ldu<C>(G, u.c[C], P);
      P[C] = cell;
      tn[s] = T(2) * nut_at(G, L.nut, P) * (hi - lo) * idx(G, C, cell);
    }
    T D = (tn[1] - tn[0]) * idc(G, C, F[C]);
    {
      int Eh[3] = {F[0], F[1], F[2]};
      Eh[A1] += 1;
      D += (shear<C, A1>(G, L, Eh) - shear<C, A1>(G, L, F)) * idx(G, A1, F[A1]);
    }
    {
      int Eh[3] = {F[0], F[1], F[2]};
      Eh[A2] += 1;
      D += (shear<C, A2>(G, L, Eh) - shear<C, A2>(G, L, F)) * idx(G, A2, F[A2]);
    }
    g[id] = base + D;
  }
}

// All three components in one launch: blocks [0, b0) take u, [b0, b0 + b1)
// take v and the rest w (the component is uniform across a block).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_les_force(Geo<T> G, LesView<T> L, U3<T> u, U3<T> fb, T* __restrict__ g0, T* __restrict__ g1,
            T* __restrict__ g2, int b0, int b1) {
  const int b = blockIdx.x;
  if (b < b0)
    les_force_faces<0>(G, L, u, fb.c[0], g0, b, b0);
  else if (b < b0 + b1)
    les_force_faces<1>(G, L, u, fb.c[1], g1, b - b0, b1);
  else
    les_force_faces<2>(G, L, u, fb.c[2], g2, b - b0 - b1, (int)gridDim.x - b0 - b1);
}

// ----------------------------------------------------------------- adjoint
// gbar of component C at face P if that face is evolved (0 otherwise);
// periodic axes wrapped, bounded transverse indices in range.
template <int C, typename T>
__device__ __forceinline__ T gbar_at(const Geo<T>& G, const T* __restrict__ gb, const int P[3]) {
  int I[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) I[a] = G.per[a] ? wrapi(P[a], G.ext[C][a]) : P[a];
  if (!G.per[C] && (I[C] < 1 || I[C] > G.n[C] - 1)) return T(0);
  return gb[fidx(G.ext[C], I[0], I[1], I[2])];
}

// Stress adjoint of an edge of the (C, A) plane: the C-equation faces on
// either side along A and the A-equation faces on either side along C.
template <int C, int A, typename T>
__device__ __forceinline__ T edge_tbar(const Geo<T>& G, const U3<T>& gb, const int E[3]) {
  T tb = T(0);
  if (G.per[A] || E[A] - 1 >= 0) {
    int P[3] = {E[0], E[1], E[2]};
    P[A] = E[A] - 1;
    tb += gbar_at<C>(G, gb.c[C], P) * idx(G, A, E[A] - 1);
  }
  if (G.per[A] || E[A] < G.n[A]) tb -= gbar_at<C>(G, gb.c[C], E) * idx(G, A, E[A]);
  if (G.per[C] || E[C] - 1 >= 0) {
    int P[3] = {E[0], E[1], E[2]};
    P[C] = E[C] - 1;
    tb += gbar_at<A>(G, gb.c[A], P) * idx(G, C, E[C] - 1);
  }
  if (G.per[C] || E[C] < G.n[C]) tb -= gbar_at<A>(G, gb.c[A], E) * idx(G, C, E[C]);
  return tb;
}

template <int C, int A, typename T>
__device__ __forceinline__ void site_edge(const Geo<T>& G, const LesView<T>& L, const U3<T>& u,
                                          const U3<T>& gb, const int E[3]) {
  constexpr int B = 3 - C - A;
  if (E[B] >= G.n[B]) return;
  const T tb = edge_tbar<C, A>(G, gb, E);
  const int64_t e = eidx(G, E);
  L.pe[C + A - 1][e] = tb * edge_nu<C, A>(G, L, E);
  L.qe[C + A - 1][e] = tb * L.ge[C + A - 1][e];
}

// Pass 1 over the lattice: cells (normal stresses) and edges.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_les_adj_sites(Geo<T> G, LesView<T> L, U3<T> u, U3<T> gb) {
  const int l0 = G.n[0] + 1, l1 = G.n[1] + 1;
  const int64_t n = (int64_t)l0 * l1 * (G.n[2] + 1);
  for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < n;
       id += (int64_t)gridDim.x * kBlock) {
    const int E[3] = {(int)(id % l0), (int)((id / l0) % l1), (int)(id / ((int64_t)l0 * l1))};
    if (E[0] < G.n[0] && E[1] < G.n[1] && E[2] < G.n[2]) {
      const int64_t ci = cidx(G, E[0], E[1], E[2]);
      const T nu = L.nut[ci];
      T nb = T(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        int P[3] = {E[0], E[1], E[2]};
        P[c] += 1;
        T hi, lo, tb;
        if (c == 0) {
          hi = ldu<0>(G, u.c[0], P); lo = ldu<0>(G, u.c[0], E);
          tb = gbar_at<0>(G, gb.c[0], E) * idc(G, 0, E[0]) - gbar_at<0>(G, gb.c[0], P) * idc(G, 0, E[0] + 1);
        } else if (c == 1) {
          hi = ldu<1>(G, u.c[1], P); lo = ldu<1>(G, u.c[1], E);
          tb = gbar_at<1>(G, gb.c[1], E) * idc(G, 1, E[1]) - gbar_at<1>(G, gb.c[1], P) * idc(G, 1, E[1] + 1);
        } else {
          hi = ldu<2>(G, u.c[2], P); lo = ldu<2>(G, u.c[2], E);
          tb = gbar_at<2>(G, gb.c[2], E) * idc(G, 2, E[2]) - gbar_at<2>(G, gb.c[2], P) * idc(G, 2, E[2] + 1);
        }
        L.wcc[c][ci] = T(2) * tb * nu;
        nb += T(2) * tb * (hi - lo) * idx(G, c, E[c]);
      }
      L.nbar[ci] = nb;
    }
    site_edge<0, 1>(G, L, u, gb, E);
    site_edge<0, 2>(G, L, u, gb, E);
    site_edge<1, 2>(G, L, u, gb, E);
  }
}

template <int C, int A, typename T>
__device__ __forceinline__ T cell_edge_qsum(const Geo<T>& G, const LesView<T>& L, int i, int j,
                                            int k) {
  T s = T(0);
#pragma unroll
  for (int p = 0; p <= 1; ++p)
#pragma unroll
    for (int q = 0; q <= 1; ++q) {
      int E[3] = {i, j, k};
      E[C] += p;
      E[A] += q;
      if (!edge_on_wall<C, A>(G, E)) s += L.qe[C + A - 1][eidx(G, E)];
    }
  return s;
}

// Pass 2 over the cells: viscosity adjoint through |S|.
template <typename T>
__device__ __forceinline__ void les_adj_cells(const Geo<T>& G, const LesView<T>& L,
                                              const U3<T>& u, int blk, int nblk) {
  const int64_t n = (int64_t)G.n[0] * G.n[1] * G.n[2];
  for (int64_t id = (int64_t)blk * kBlock + threadIdx.x; id < n; id += (int64_t)nblk * kBlock) {
    const int i = (int)(id % G.n[0]);
    const int j = (int)((id / G.n[0]) % G.n[1]);
    const int k = (int)(id / ((int64_t)G.n[0] * G.n[1]));
    const T nb = L.nbar[id] + T(0.25) * (cell_edge_qsum<0, 1>(G, L, i, j, k) +
                                         cell_edge_qsum<0, 2>(G, L, i, j, k) +
                                         cell_edge_qsum<1, 2>(G, L, i, j, k));
    T sd[3], so[3];
    cell_strain(G, L, u, i, j, k, sd, so);
    const T ss = sd[0] * sd[0] + sd[1] * sd[1] + sd[2] * sd[2] +
                 T(2) * (so[0] * so[0] + so[1] * so[1] + so[2] * so[2]);
    const T mag = sqrt(T(2) * ss);
    // d|S|/dS_cc = 2 S_cc / |S|, d|S|/dS_ca = 4 S_ca / |S| (a != c, once each)
    const T f = mag > T(0) ? L.cs2 * delta2(G, i, j, k) * nb / mag : T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) L.wcc[c][id] += T(2) * f * sd[c];
#pragma unroll
    for (int t = 0; t < 3; ++t) L.soff[t][id] = T(4) * f * so[t];
  }
}

// Pass 2b over the wall faces: Eqs. 27-29 adjoint.
template <typename T>
__device__ __forceinline__ void les_adj_wall(const Geo<T>& G, const LesView<T>& L,
                                             const U3<T>& u, int blk, int nblk) {
  const int nx = G.n[0], nz = G.n[2];
  const int64_t n = 4 * (int64_t)nx * nz;
  for (int64_t id = (int64_t)blk * kBlock + threadIdx.x; id < n; id += (int64_t)nblk * kBlock) {
    const int i = (int)(id % nx);
    const int k = (int)((id / nx) % nz);
    const int side = (int)((id / ((int64_t)nx * nz)) % 2);
    const int comp = (int)(id / (2 * (int64_t)nx * nz));
    const int E[3] = {i, side == 0 ? 0 : G.n[1], k};
    const double nub = (double)L.qe[comp == 0 ? 0 : 2][eidx(G, E)];
    double own, oth, dn_own, dn_oth;
    wall_pair(G, L, u, comp, side, i, k, &own, &oth);
    const int64_t w = (int64_t)k * nx + i;
    (void)wall_nu(L, side, own, oth, L.upl[comp][side][w], L.dupl[comp][side][w], &dn_own, &dn_oth);
    L.wown[comp][side][w] = nub * dn_own;
    L.woth[comp][side][w] = nub * dn_oth;
  }
}

// Passes 2 and 2b in one launch (they read the stress sites' output only):
// blocks [0, bc) take the cells, the rest the wall faces.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_les_adj_cells(Geo<T> G, LesView<T> L, U3<T> u,
                                                          int bc) {
  const int b = blockIdx.x;
  if (b < bc)
    les_adj_cells(G, L, u, b, bc);
  else
    les_adj_wall(G, L, u, b - bc, (int)gridDim.x - bc);
}

template <int C, int A, typename T>
__device__ __forceinline__ void edge_finish(const Geo<T>& G, const LesView<T>& L, const int E[3]) {
  constexpr int B = 3 - C - A;
  if (E[B] >= G.n[B]) return;
  T s = T(0);
#pragma unroll
  for (int dc = -1; dc <= 0; ++dc)
#pragma unroll
    for (int da = -1; da <= 0; ++da) {
      int P[3] = {E[0], E[1], E[2]};
      P[C] += dc;
      P[A] += da;
      if (!G.per[C] && (P[C] < 0 || P[C] >= G.n[C])) continue;
      if (!G.per[A] && (P[A] < 0 || P[A] >= G.n[A])) continue;
      int I[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) I[a] = G.per[a] ? wrapi(P[a], G.n[a]) : P[a];
      s += L.soff[C + A - 1][cidx(G, I[0], I[1], I[2])];
    }
  // S_ca of a cell is 1/8 of the sum of G over its four edges
  L.pe[C + A - 1][eidx(G, E)] += T(0.125) * s;
}

// Pass 3 over the edges: gradient coefficients.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_les_adj_edges(Geo<T> G, LesView<T> L) {
  const int l0 = G.n[0] + 1, l1 = G.n[1] + 1;
  const int64_t n = (int64_t)l0 * l1 * (G.n[2] + 1);
  for (int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x; id < n;
       id += (int64_t)gridDim.x * kBlock) {
    const int E[3] = {(int)(id % l0), (int)((id / l0) % l1), (int)(id / ((int64_t)l0 * l1))};
    edge_finish<0, 1>(G, L, E);
    edge_finish<0, 2>(G, L, E);
    edge_finish<1, 2>(G, L, E);
  }
}

// Coefficient of u_C at face F through the edges of the (C, A) plane:
// d_A u_C on the edges at F[A] (+) and F[A] + 1 (-); behind a Dirichlet
// boundary the mirrored ghost doubles the weight.
template <int C, int A, typename T>
__device__ __forceinline__ T face_from_edges(const Geo<T>& G, const LesView<T>& L,
                                             const int F[3]) {
  constexpr int lo = C < A ? C : A, hi = C < A ? A : C;
  int Eh[3] = {F[0], F[1], F[2]};
  Eh[A] += 1;
  T wl = T(1), wh = T(1);
  if (!G.per[A]) {
    if (F[A] == 0) wl = G.dir[A][0] ? T(2) : T(0);
    if (F[A] == G.n[A] - 1) wh = G.dir[A][1] ? T(2) : T(0);
  }
  return L.pe[lo + hi - 1][eidx(G, F)] * idc(G, A, F[A]) * wl -
         L.pe[lo + hi - 1][eidx(G, Eh)] * idc(G, A, F[A] + 1) * wh;
}

// Pass 4 over the faces of component C (blocks blk = 0 .. nblk - 1 of a
// range): ubar += the subgrid VJP.
template <int C, typename T>
__device__ __forceinline__ void les_adj_faces(const Geo<T>& G, const LesView<T>& L,
                                              T* __restrict__ ub, const T* __restrict__ gb,
                                              T* __restrict__ fbar, int blk, int nblk) {
  constexpr int A1 = (C + 1) % 3, A2 = (C + 2) % 3;
  const int e0 = G.ext[C][0], e1 = G.ext[C][1], e2 = G.ext[C][2];
  const int64_t n = (int64_t)e0 * e1 * e2;
  for (int64_t id = (int64_t)blk * kBlock + threadIdx.x; id < n; id += (int64_t)nblk * kBlock) {
    const int F[3] = {(int)(id % e0), (int)((id / e0) % e1), (int)(id / ((int64_t)e0 * e1))};
    T acc = T(0);
    if (G.per[C] || F[C] - 1 >= 0) {
      int P[3] = {F[0], F[1], F[2]};
      P[C] = G.per[C] ? wrapi(F[C] - 1, G.n[C]) : F[C] - 1;
      acc += L.wcc[C][cidx(G, P[0], P[1], P[2])] * idx(G, C, P[C]);
    }
    if (G.per[C] || F[C] < G.n[C]) acc -= L.wcc[C][cidx(G, F[0], F[1], F[2])] * idx(G, C, F[C]);
    acc += face_from_edges<C, A1>(G, L, F) + face_from_edges<C, A2>(G, L, F);
    if constexpr (C == 0 || C == 2) {
      if (L.wall && (F[1] == 0 || F[1] == G.n[1] - 1)) {
        const int nx = G.n[0], nz = G.n[2];
        const int i = F[0], k = F[2];
        double w = 0.0;
        for (int side = 0; side < 2; ++side) {
          if (F[1] != (side == 0 ? 0 : G.n[1] - 1)) continue;
          if (C == 0) {
            w += L.wown[0][side][(int64_t)k * nx + i];
            // w faces whose mean of u includes this face: cells i-1, i; faces k, k+1
            for (int di = -1; di <= 0; ++di)
              for (int dk = 0; dk <= 1; ++dk)
                w += 0.25 * L.woth[1][side][(int64_t)wrapi(k + dk, nz) * nx + wrapi(i + di, nx)];
          } else {
            w += L.wown[1][side][(int64_t)k * nx + i];
            // u faces whose mean of w includes this face: faces i, i+1; cells k-1, k
            for (int di = 0; di <= 1; ++di)
              for (int dk = -1; dk <= 0; ++dk)
                w += 0.25 * L.woth[0][side][(int64_t)wrapi(k + dk, nz) * nx + wrapi(i + di, nx)];
          }
        }
        acc += (T)w;
      }
    }
    ub[id] += acc;
    if (fbar) fbar[id] += gb[id];     // g = fb + subgrid term: fbar gets gbar
  }
}

// All three components in one launch (block ranges as k_les_force).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_les_adj_face(Geo<T> G, LesView<T> L, T* __restrict__ ub0, T* __restrict__ ub1,
               T* __restrict__ ub2, U3<T> gb, T* __restrict__ fb0, T* __restrict__ fb1,
               T* __restrict__ fb2, int b0, int b1) {
  const int b = blockIdx.x;
  if (b < b0)
    les_adj_faces<0>(G, L, ub0, gb.c[0], fb0, b, b0);
  else if (b < b0 + b1)
    les_adj_faces<1>(G, L, ub1, gb.c[1], fb1, b - b0, b1);
  else
    les_adj_faces<2>(G, L, ub2, gb.c[2], fb2, b - b0 - b1, (int)gridDim.x - b0 - b1);
}

inline int grid_for(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

template <typename T>
int launch_les_forward(const Geo<T>& G, const LesView<T>& L, const T* const u[3],
                       const T* const fb[3], T* const g[3], hipStream_t s) {
  const U3<T> U{{u[0], u[1], u[2]}};
  const int64_t nc = (int64_t)G.n[0] * G.n[1] * G.n[2];
  const int64_t nl = (int64_t)(G.n[0] + 1) * (G.n[1] + 1) * (G.n[2] + 1);
  const int bg = grid_for(nl);
  const int bw = L.wall ? grid_for(4 * (int64_t)G.n[0] * G.n[2]) : 0;
  launch_kernel(k_les_grad<T>, dim3(bg + bw), dim3(kBlock), 0, s, G, L, U, bg);
  FVIB_HIP(hipGetLastError());
  launch_kernel(k_les_nut<T>, dim3(grid_for(nc)), dim3(kBlock), 0, s, G, L, U);
  FVIB_HIP(hipGetLastError());
  const int64_t nf[3] = {(int64_t)G.ext[0][0] * G.ext[0][1] * G.ext[0][2],
                         (int64_t)G.ext[1][0] * G.ext[1][1] * G.ext[1][2],
                         (int64_t)G.ext[2][0] * G.ext[2][1] * G.ext[2][2]};
  const int b0 = grid_for(nf[0]), b1 = grid_for(nf[1]), b2 = grid_for(nf[2]);
  const U3<T> FB{{fb[0], fb[1], fb[2]}};
  launch_kernel(k_les_force<T>, dim3(b0 + b1 + b2), dim3(kBlock), 0, s, G, L, U, FB, g[0], g[1],
                g[2], b0, b1);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_les_adjoint(const Geo<T>& G, const LesView<T>& L, const T* const u[3],
                       const T* const gbar[3], T* const ubar[3], T* const fbar[3],
                       hipStream_t s) {
  const U3<T> U{{u[0], u[1], u[2]}};
  const U3<T> GB{{gbar[0], gbar[1], gbar[2]}};
  const int64_t nc = (int64_t)G.n[0] * G.n[1] * G.n[2];
  const int64_t nl = (int64_t)(G.n[0] + 1) * (G.n[1] + 1) * (G.n[2] + 1);
  const int64_t nw = 4 * (int64_t)G.n[0] * G.n[2];
  const int bg = grid_for(nl), bw = L.wall ? grid_for(nw) : 0;
  launch_kernel(k_les_grad<T>, dim3(bg + bw), dim3(kBlock), 0, s, G, L, U, bg);
  FVIB_HIP(hipGetLastError());
  launch_kernel(k_les_nut<T>, dim3(grid_for(nc)), dim3(kBlock), 0, s, G, L, U);
  FVIB_HIP(hipGetLastError());
  launch_kernel(k_les_adj_sites<T>, dim3(grid_for(nl)), dim3(kBlock), 0, s, G, L, U, GB);
  FVIB_HIP(hipGetLastError());
  const int bc = grid_for(nc);
  launch_kernel(k_les_adj_cells<T>, dim3(bc + bw), dim3(kBlock), 0, s, G, L, U, bc);
  FVIB_HIP(hipGetLastError());
  launch_kernel(k_les_adj_edges<T>, dim3(grid_for(nl)), dim3(kBlock), 0, s, G, L);
  FVIB_HIP(hipGetLastError());
  const int64_t nf[3] = {(int64_t)G.ext[0][0] * G.ext[0][1] * G.ext[0][2],
                         (int64_t)G.ext[1][0] * G.ext[1][1] * G.ext[1][2],
                         (int64_t)G.ext[2][0] * G.ext[2][1] * G.ext[2][2]};
  const int b0 = grid_for(nf[0]), b1 = grid_for(nf[1]), b2 = grid_for(nf[2]);
  launch_kernel(k_les_adj_face<T>, dim3(b0 + b1 + b2), dim3(kBlock), 0, s, G, L, ubar[0], ubar[1],
                ubar[2], GB, fbar[0], fbar[1], fbar[2], b0, b1);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template int launch_les_forward<float>(const Geo<float>&, const LesView<float>&,
                                       const float* const[3], const float* const[3],
                                       float* const[3], hipStream_t);
template int launch_les_forward<double>(const Geo<double>&, const LesView<double>&,
                                        const double* const[3], const double* const[3],
                                        double* const[3], hipStream_t);
template int launch_les_adjoint<float>(const Geo<float>&, const LesView<float>&,
                                       const float* const[3], const float* const[3],
                                       float* const[3], float* const[3], hipStream_t);
template int launch_les_adjoint<double>(const Geo<double>&, const LesView<double>&,
                                        const double* const[3], const double* const[3],
                                        double* const[3], double* const[3], hipStream_t);

}  // namespace fvib
