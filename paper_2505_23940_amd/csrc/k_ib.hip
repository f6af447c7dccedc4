// Immersed-boundary kernels (2D): point classes, target velocities, loads
// on the body and the rigid-body update (paper Sec. 2.2, Eqs. 12, 18-22).
//
// Point classes (Sec. 2.2, Fig. 2) are evaluated per velocity component on
// that component's own face points inside a fixed-size window that follows
// the body: solid = inside the closed marker polygon (crossing number,
// half-open rule y_a <= y < y_b, double precision, no contraction of the
// multiply-add so the decision is reproducible); immersed-boundary point =
// not solid with a solid axis neighbour.  Both are forced (Eq. 5).
//
// Target velocity on IB points: the marker velocity interpolated with the
// normalised 4-point-kernel weights w_k = delta_h(x - X_k) dV_k
// (Eqs. 18-19, Shepard form), which for a rigid body (every marker moving
// with the body velocity) is the body velocity itself, written directly;
// on solid points the body velocity (Eq. 23).
//
// Loads (Eq. 20): q_k = -sum_x f(x) delta_h(x - X_k) h^2 over forced faces,
// F = rho sum_k q_k dV_k with dV_k = ds_k h; then classic RK4 of
// m w'' + c w' + k w = F with F held over the step (Eq. 12).
#include "fvib_kernels.h"

namespace fvib {


__device__ __forceinline__ void window_origin(const IbGeo& B, const double* body, int c,
                                              int* ox, int* oy, bool* clamped) {
  const double dx = body[0], dy = body[1];
  int x0 = (int)floor((B.xmin0 + dx - B.fx[c][0]) / B.h) - B.margin;
  int y0 = (int)floor((B.ymin0 + dy - B.fy[c][0]) / B.h) - B.margin;
  const int xmax = B.ext[c][0] - B.W[c][0];
  const int ymax = B.ext[c][1] - B.W[c][1];
  bool cl = false;
  if (x0 < 0) { x0 = 0; cl = true; }
  if (y0 < 0) { y0 = 0; cl = true; }
  if (x0 > xmax) { x0 = xmax; cl = true; }
  if (y0 > ymax) { y0 = ymax; cl = true; }
  *ox = x0;
  *oy = y0;
  *clamped = *clamped || cl;
}

// Crossing parity of the polygon edges k0, k0 + dk, ... with the ray from
// (px, py) towards +x (the parity over all edges decides inside).
__device__ bool crossings_odd(const IbGeo& B, double dxb, double dyb, double px, double py,
                              int k0, int dk) {
#pragma clang fp contract(off)
  bool inside = false;
  const int M = B.M;
  for (int k = k0; k < M; k += dk) {
    const int kn = (k + 1 == M) ? 0 : k + 1;
    const double ax = B.X0[2 * k] + dxb, ay = B.X0[2 * k + 1] + dyb;
    const double bx = B.X0[2 * kn] + dxb, by = B.X0[2 * kn + 1] + dyb;
    if ((ay <= py && py < by) || (by <= py && py < ay)) {
      double t = (py - ay) * (bx - ax);
      t = t / (by - ay);
      const double xint = ax + t;
      if (px < xint) inside = !inside;
    }
  }
  return inside;
}

// Point classes of the window and their targets in one launch, and the
// window origins.  One wavefront per window face; its lanes take every 64th
// polygon edge and the crossing parities combine through a ballot.  The
// wavefront tests the face itself and, for a fluid face, its axis
// neighbours inside the window, so that an immersed-boundary point (a fluid
// face with a solid neighbour) is found without a second pass.  Every marker
// of a rigid body moves with the body velocity, so the normalised
// interpolation of Eqs. 18-19 returns that velocity exactly: the target of
// an immersed-boundary point is the body velocity, as on solid points
// (Eq. 23).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_ib_classify(IbGeo B, const double* __restrict__ body, SolverScalars* sc, T* __restrict__ us0,
              T* __restrict__ us1) {
  T* us[2] = {us0, us1};
  int org[4];
  bool clamped = false;
  window_origin(B, body, 0, &org[0], &org[1], &clamped);
  window_origin(B, body, 1, &org[2], &org[3], &clamped);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int q = 0; q < 4; ++q) B.origin[q] = org[q];
    if (clamped) sc->clamp = 1;
  }
  const int n0 = B.W[0][0] * B.W[0][1];
  const int n1 = B.W[1][0] * B.W[1][1];
  const int lane = threadIdx.x & 63;
  const int wpb = kBlock / 64;
  const double dxb = body[0], dyb = body[1];
  const double tolb = 1e-6 * B.h;
  for (int t = blockIdx.x * wpb + (threadIdx.x >> 6); t < n0 + n1; t += gridDim.x * wpb) {
    const int c = (t < n0) ? 0 : 1;
    const int l = (c == 0) ? t : t - n0;
    const int Wx = B.W[c][0], Wy = B.W[c][1];
    const int li = l % Wx, lj = l / Wx;
    const int i = org[2 * c] + li, j = org[2 * c + 1] + lj;
    // solid flag of face (ii, jj) of component c (uniform across the wave).
    // Outside the polygon's box the crossing test cannot report inside (a
    // horizontal line meets a closed polygon an even number of times, or
    // not at all), so points farther out than a rounding margin skip it.
    auto solid = [&](int ii, int jj) -> bool {
      const double px = B.fx[c][ii], py = B.fy[c][jj];
      if (!(px >= B.xmin0 + dxb - tolb && px <= B.xmax0 + dxb + tolb &&
            py >= B.ymin0 + dyb - tolb && py <= B.ymax0 + dyb + tolb))
        return false;
      const bool odd = crossings_odd(B, dxb, dyb, px, py, lane, 64);
      return (__popcll(__ballot(odd ? 1 : 0)) & 1) != 0;
    };
    int cls = solid(i, j) ? 1 : 0;
    if (cls == 0) {
      bool nb = false;
      if (li > 0) nb = nb || solid(i - 1, j);
      if (!nb && li + 1 < Wx) nb = nb || solid(i + 1, j);
      if (!nb && lj > 0) nb = nb || solid(i, j - 1);
      if (!nb && lj + 1 < Wy) nb = nb || solid(i, j + 1);
      cls = nb ? 2 : 0;
    }
    if (lane == 0) {
      B.cls[c][l] = (uint8_t)cls;
      if (cls) us[c][l] = (T)body[3 + c];
    }
  }
}

// Classic RK4 of m w'' + c w' + k w = F per free degree of freedom, F held
// over the step; fixed degrees of freedom keep their values.
__device__ void body_rk4(const IbGeo& B, const double* st_in, const double* F,
                         const double* __restrict__ kc, double* st) {
  for (int a = 0; a < 6; ++a) st[a] = st_in[a];
  if (B.kind != FVIB_BODY_RIGID_SPRING) return;
  const double m = B.m, dt = B.dt;
  for (int a = 0; a < 3; ++a) {
    if (!B.free_dof[a]) continue;
    const double kk = kc ? kc[a] : 0.0, cc = kc ? kc[3 + a] : 0.0;
    const double d = st[a], v = st[3 + a], Fa = F[a];
    const double k1d = v, k1v = (Fa - cc * v - kk * d) / m;
    const double d2 = d + 0.5 * dt * k1d, v2 = v + 0.5 * dt * k1v;
    const double k2d = v2, k2v = (Fa - cc * v2 - kk * d2) / m;
    const double d3 = d + 0.5 * dt * k2d, v3 = v + 0.5 * dt * k2v;
    const double k3d = v3, k3v = (Fa - cc * v3 - kk * d3) / m;
    const double d4 = d + dt * k3d, v4 = v + dt * k3v;
    const double k4d = v4, k4v = (Fa - cc * v4 - kk * d4) / m;
    st[a] = d + (dt / 6.0) * (k1d + 2.0 * k2d + 2.0 * k3d + k4d);
    st[3 + a] = v + (dt / 6.0) * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
  }
}

// Loads on the body (markers placed by body_pos) and, when body_out is
// given, the RK4 update from body_rk; one block.  Fin (nullable) replaces
// the computed force.  With body_out and the coupling error requested
// (xi != 0), sc->xi = |body_out - body_pos|^2 / max(|body_pos|^2, 1e-30):
// the change of the structural iterate of a coupling sub-iteration.
// info (nullable): the step's record, written last (the step's final
// launch), with the host's iteration counts and sticky word.
// The loads gather takes one item per (marker, component, stencil row):
// kLoadsBlock threads, each summing its items' four faces, then one
// block-wide sum (fixed order).
constexpr int kLoadsBlock = 1024;

template <typename T>
__global__ void __launch_bounds__(kLoadsBlock)
k_loads_body(IbGeo B, IbView<T> ib, const double* body_pos, const double* body_rk,
             double* body_out,
             const double* __restrict__ kc, const double* __restrict__ Fin, int xi,
             SolverScalars* sc, fvib_step_info* info, int cg_iters, int ir_iters, int* sticky) {
  double q[2] = {0.0, 0.0};
  if (!Fin) {
    ib_loads_share<T>(B, ib, body_pos, threadIdx.x, kLoadsBlock, q);
    block_sum_n<2, kLoadsBlock>(q);
  }
  if (threadIdx.x != 0) return;
  double F[3] = {-B.rho * q[0], -B.rho * q[1], 0.0};
  if (Fin)
    for (int a = 0; a < 3; ++a) F[a] = Fin[a];
  for (int a = 0; a < 3; ++a) sc->force[a] = F[a];
  if (body_out) {
    double st[6];
    body_rk4(B, body_rk, F, kc, st);
    if (xi) {
      double num = 0.0, den = 0.0;
      for (int a = 0; a < 6; ++a) {
        const double e = st[a] - body_pos[a];
        num += e * e;
        den += body_pos[a] * body_pos[a];
      }
      sc->xi = num / fmax(den, 1e-30);
    }
    for (int a = 0; a < 6; ++a) body_out[a] = st[a];
  }
  if (info) put_record(sc, info, cg_iters, ir_iters, sticky, 0);
}

// Also copies (or zeroes, src == nullptr) a 6-double body state when dst
// is given (the adjoint body state of a step without a body).
__global__ void k_copy_info(const SolverScalars* sc, fvib_step_info* info, int cg_iters,
                            int ir_iters, const double* body_src, double* body_dst, int* sticky,
                            int cpl_iters) {
  if (body_dst && threadIdx.x < 6) body_dst[threadIdx.x] = body_src ? body_src[threadIdx.x] : 0.0;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  put_record(sc, info, cg_iters, ir_iters, sticky, cpl_iters);
}

// Static box on a 3D grid: forced flags on the window faces of each
// component from the box's face-index ranges [bs0, bs1) per axis (the faces
// whose points lie in the half-open box): solid inside the ranges, immersed
// boundary one step outside along exactly one axis (a solid axis neighbour).
__global__ void __launch_bounds__(kBlock) k_box_classify(BoxGeo B) {
  for (int c = 0; c < 3; ++c) {
    const int W0 = B.bw[c][0], W1 = B.bw[c][1], n = W0 * W1 * B.bw[c][2];
    for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
      const int I[3] = {B.bo[c][0] + l % W0, B.bo[c][1] + (l / W0) % W1,
                        B.bo[c][2] + l / (W0 * W1)};
      bool in[3], near[3];
      for (int a = 0; a < 3; ++a) {
        in[a] = I[a] >= B.bs[c][a][0] && I[a] < B.bs[c][a][1];
        near[a] = I[a] == B.bs[c][a][0] - 1 || I[a] == B.bs[c][a][1];
      }
      const bool solid = in[0] && in[1] && in[2];
      const bool ibp = !solid && ((near[0] && in[1] && in[2]) || (in[0] && near[1] && in[2]) ||
                                  (in[0] && in[1] && near[2]));
      // a boundary-normal face keeps its boundary condition: never forced
      const bool bnd = !B.per[c] && (I[c] == 0 || I[c] == B.nc[c]);
      B.cls[c][l] = ((solid || ibp) && !bnd) ? 1 : 0;
    }
  }
}

int launch_box_classify(const BoxGeo& B, hipStream_t s) {
  launch_kernel(k_box_classify, dim3(64), dim3(kBlock), 0, s, B);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

// ------------------------------------------------------------ launchers
template <typename T>
int launch_ib_classify(const IbGeo& B, const double* body, T* us0, T* us1, SolverScalars* sc,
                       hipStream_t s) {
  const int n = B.W[0][0] * B.W[0][1] + B.W[1][0] * B.W[1][1];
  // one wavefront per window face
  launch_kernel((k_ib_classify<T>), dim3((n + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0,
                s, B, body, sc, us0, us1);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_loads_body(const IbGeo& B, const IbView<T>& ib, const double* body_pos,
                      const double* body_rk, double* body_out, const double* kc,
                      const double* Fin, int xi, SolverScalars* sc, hipStream_t s,
                      fvib_step_info* info, int cg_iters, int ir_iters, int* sticky) {
  launch_kernel((k_loads_body<T>), dim3(1), dim3(kLoadsBlock), 0, s, B, ib, body_pos, body_rk,
                body_out, kc, Fin, xi, sc, info, cg_iters, ir_iters, sticky);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

// The solver scalars cleared at the start of a step: one small launch in
// place of a runtime fill (which issues two fill kernels for this size).
__global__ void k_zero_scalars(SolverScalars* sc) {
  constexpr int kWords = (int)(sizeof(SolverScalars) / sizeof(uint32_t));
  static_assert(sizeof(SolverScalars) % sizeof(uint32_t) == 0 && kWords <= 64, "one wavefront");
  if (threadIdx.x < kWords) reinterpret_cast<uint32_t*>(sc)[threadIdx.x] = 0u;
}

int launch_zero_scalars(SolverScalars* sc, hipStream_t s) {
  launch_kernel(k_zero_scalars, dim3(1), dim3(64), 0, s, sc);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

int launch_copy_info(const SolverScalars* sc, fvib_step_info* info, int cg_iters, int ir_iters,
                     hipStream_t s, const double* body_src, double* body_dst, int* sticky,
                     int cpl_iters) {
  launch_kernel(k_copy_info, dim3(1), dim3(64), 0, s, sc, info, cg_iters, ir_iters, body_src,
                body_dst, sticky, cpl_iters);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template int launch_ib_classify<float>(const IbGeo&, const double*, float*, float*,
                                       SolverScalars*, hipStream_t);
template int launch_ib_classify<double>(const IbGeo&, const double*, double*, double*,
                                        SolverScalars*, hipStream_t);
template int launch_loads_body<float>(const IbGeo&, const IbView<float>&, const double*,
                                      const double*, double*, const double*, const double*, int,
                                      SolverScalars*, hipStream_t, fvib_step_info*, int, int,
                                      int*);
template int launch_loads_body<double>(const IbGeo&, const IbView<double>&, const double*,
                                       const double*, double*, const double*, const double*, int,
                                       SolverScalars*, hipStream_t, fvib_step_info*, int, int,
                                       int*);

}  // namespace fvib
