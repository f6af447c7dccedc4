// Predictor of the projection method with direct forcing (paper Eqs. 4-5)
// and the boundary-normal faces.
//
// R = -div(u (x) u) + nu lap(u) + f_b is evaluated on every face that the
// momentum equation advances.  Convection is in divergence form: along its
// own axis a component is carried to the cell centre as the mean of its two
// faces; across the other axes it is interpolated linearly between cell
// centres to the edge and multiplied by the transverse component
// interpolated along the own axis (central), or the transported value is
// taken from the upwind side (first-order upwind).  Diffusion is the
// central second-order finite-volume Laplacian.
//
// One thread owns one cell and computes the low face of that cell for every
// component, so each velocity array is read once per sweep with the
// stencil neighbours served from L1/L2.
#include "fvib_internal.h"

namespace fvib {

// R of component C at face (i, j, k).  `L(c, di, dj, dk)` returns component
// c at the offset (di, dj, dk) from (i, j, k), boundary rules applied (each
// offset is -1, 0 or +1 per axis).
template <int C, int DIM, bool UPW, typename T, typename Load, typename ML>
__device__ __forceinline__ T momentum_rhs(const Geo<T>& G, const Load& L, const ML& M, T fb) {
  const T q0 = L(C, 0, 0, 0);
  const Met4<T> fc = M.mf(C, 0);
  T conv, visc;
  // along the own axis: convective fluxes at the two adjacent cell centres
  // and the own-axis diffusion
  {
    const T qm = L(C, C == 0 ? -1 : 0, C == 1 ? -1 : 0, C == 2 ? -1 : 0);
    const T qp = L(C, C == 0 ? 1 : 0, C == 1 ? 1 : 0, C == 2 ? 1 : 0);
    const T Qlo = T(0.5) * (qm + q0);
    const T Qhi = T(0.5) * (q0 + qp);
    T Flo, Fhi;
    if constexpr (UPW) {
      Flo = Qlo * (Qlo > T(0) ? qm : (Qlo < T(0) ? q0 : T(0)));
      Fhi = Qhi * (Qhi > T(0) ? q0 : (Qhi < T(0) ? qp : T(0)));
    } else {
      Flo = Qlo * Qlo;
      Fhi = Qhi * Qhi;
    }
    conv = (Fhi - Flo) * fc.x;
    visc = (qp - q0) * fc.y - (q0 - qm) * fc.z;
  }
  // across the other axes: edge fluxes at a-faces ia and ia + 1, and the
  // cross diffusion
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (a == C) continue;
    const int ex = (a == 0), ey = (a == 1), ez = (a == 2);
    const int cx = (C == 0), cy = (C == 1), cz = (C == 2);
    const Met4<T> ca = M.mc(a, 0);
    const T cm = L(C, -ex, -ey, -ez);
    const T cp = L(C, ex, ey, ez);
    // component a at (a-face ia, own cells ic-1, ic) and at a-face ia + 1
    const T a00 = L(a, -cx, -cy, -cz);
    const T a01 = L(a, 0, 0, 0);
    const T a10 = L(a, ex - cx, ey - cy, ez - cz);
    const T a11 = L(a, ex, ey, ez);
    const T wc = fc.w;
    const T V0 = (T(1) - wc) * a00 + wc * a01;
    const T V1 = (T(1) - wc) * a10 + wc * a11;
    T F0, F1;
    if constexpr (UPW) {
      F0 = V0 * (V0 > T(0) ? cm : (V0 < T(0) ? q0 : T(0)));
      F1 = V1 * (V1 > T(0) ? q0 : (V1 < T(0) ? cp : T(0)));
    } else {
      const T w0 = M.mf(a, 0).w, w1 = M.mf(a, 1).w;
      const T U0 = (T(1) - w0) * cm + w0 * q0;
      const T U1 = (T(1) - w1) * q0 + w1 * cp;
      F0 = U0 * V0;
      F1 = U1 * V1;
    }
    conv += (F1 - F0) * ca.x;
    visc += (cp - q0) * ca.y - (q0 - cm) * ca.z;
  }
  return -conv + G.nu * visc + fb;
}

// Is face (i, j, k) of component C advanced by the momentum equation?
template <int C, typename T>
__device__ __forceinline__ bool evolved(const Geo<T>& G, int i, int j, int k) {
  const int I[3] = {i, j, k};
  return G.per[C] || (I[C] >= 1 && I[C] <= G.n[C] - 1);
}

// Forcing class of face (i, j) of component C < 2: 0 fluid, else forced.
template <int C, typename T>
__device__ __forceinline__ int forced(const IbView<T>& ib, int i, int j, int* lidx) {
  if (!ib.active) return 0;
  const int li = i - ib.origin[2 * C + 0];
  const int lj = j - ib.origin[2 * C + 1];
  if (li < 0 || lj < 0 || li >= ib.W[C][0] || lj >= ib.W[C][1]) return 0;
  *lidx = lj * ib.W[C][0] + li;
  return ib.cls[C][*lidx];
}

// Predictor (MODE 0) or right-hand side (MODE 1) of component C at face
// (i, j, k):  u* = u + dt (R + f),  f = eps [ -R + (u_s - u) / dt ], i.e.
// u* = u + dt R off the body and u* = u_s on forced faces.
// UPW: upwind convection; IBA: an immersed body is active (else no face
// is forced and the class lookups are compiled out).
template <int C, int DIM, int MODE, bool UPW, bool IBA, typename T, typename Load, typename ML>
__device__ __forceinline__ void predict_face(const Geo<T>& G, const Load& L, const ML& M, T fbv,
                                             T* out, const IbView<T>& ib, int i, int j, int k) {
  if (C >= DIM || !evolved<C>(G, i, j, k)) return;
  const T R = momentum_rhs<C, DIM, UPW, T>(G, L, M, fbv);
  const int64_t id = fidx(G.ext[C], i, j, k);
  if (MODE == 1) {
    out[id] = R;
    return;
  }
  const T un = L(C, 0, 0, 0);
  if constexpr (DIM == 2 && C < 2 && IBA) {
    int li = 0;
    if (forced<C>(ib, i, j, &li)) {
      // Eq. 5 substituted into Eq. 4: the forced face takes the target
      // exactly, so u* - u_c stays free of rounding on forced faces.
      const T us = ib.us[C][li];
      ib.f[C][li] = -R + (us - un) / G.dt;
      out[id] = us;
      return;
    }
  }
  out[id] = un + G.dt * R;
}

// LDS halo tiles: a block owns a 64 x 4 tile of cells in x-y and marches
// through a chunk of z-planes, keeping planes k-1, k, k+1 of every
// component (with a one-cell halo, boundary rules applied when the halo is
// filled) in a three-slot ring.  Each value is loaded once per plane
// instead of once per use.  The tile's stencil coefficients sit in LDS
// as well.  A plane is brought in two halves: load_plane issues the global loads of
// this thread's (at most two) halo slots into registers, store_plane puts
// them into a ring slot.  The z-march loads plane k + 3 while plane k + 1
// is computed, so the load latency hides behind the stencil arithmetic.
template <typename T, int DIM>
struct PlaneRegs {
  T v[2][DIM];
};

// The x-y part of the halo rules of this thread's slots (fixed along the
// z-march): in-plane offset per component (wrapped / clamped) and the ghost
// rule behind a bounded x or y boundary; each plane adds its uniform z part.
// Halo slots past a ragged tile edge are clamped to one step outside the
// domain (their values are never used), so every load stays in bounds
// however small the axis.
template <typename T, int DIM>
struct PlaneHalo {
  int xy[2][DIM];
  T goff[2][DIM];                // ghost offset 2 g (x-y), used when negated
  uint32_t neg;                  // bit 3 h + c: negated by an x-y ghost
};

template <int DIM, typename T>
__device__ __forceinline__ void plane_halo_init(const Geo<T>& G, PlaneHalo<T, DIM>& Hh, int i0,
                                                int j0) {
  Hh.neg = 0u;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int s = threadIdx.x + h * kBlock;
    const int sy = s / kLX, sx = s - sy * kLX;
    const int gi = min(i0 - 1 + sx, G.n[0]), gj = min(j0 - 1 + sy, G.n[1]);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      int I[2] = {gi, gj};
      T off = T(0);
      bool neg = false;
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
      }
      Hh.xy[h][c] = I[1] * G.ext[c][0] + I[0];
      Hh.goff[h][c] = off;
      Hh.neg |= (neg ? 1u : 0u) << (3 * h + c);
    }
  }
}

template <int DIM, typename T>
__device__ __forceinline__ void load_plane(const Geo<T>& G, const T* const* u,
                                           const PlaneHalo<T, DIM>& Hh, PlaneRegs<T, DIM>& P,
                                           int kk) {
  // (per component: w has one more face than cells along a bounded z)
  int64_t pbase[DIM];
  bool gz[DIM], dz[DIM];
  T g2z[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    int kz = 0;
    gz[c] = dz[c] = false;
    g2z[c] = T(0);
    if constexpr (DIM == 3) {
      const int e = G.ext[c][2];
      const bool lo = kk < 0, hi = kk >= e;
      const bool per = G.per[2] != 0;
      kz = per ? (lo ? kk + e : (hi ? kk - e : kk)) : (lo ? 0 : (hi ? e - 1 : kk));
      gz[c] = !per && (lo || hi);
      dz[c] = lo ? (G.dir[2][0] != 0) : (G.dir[2][1] != 0);
      g2z[c] = T(2) * (lo ? G.gv[c][2][0] : G.gv[c][2][1]);
    }
    pbase[c] = (int64_t)kz * G.ext[c][0] * G.ext[c][1];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int s = threadIdx.x + h * kBlock;
    if (s >= kLX * kLY) break;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const T v = u[c][pbase[c] + Hh.xy[h][c]];
      const bool neg = gz[c] ? dz[c] : (((Hh.neg >> (3 * h + c)) & 1u) != 0);
      const T off = (gz[c] && dz[c]) ? g2z[c] : Hh.goff[h][c];
      P.v[h][c] = neg ? off - v : v;
    }
  }
}

template <int DIM, typename T>
__device__ __forceinline__ void store_plane(PlaneRing<T, DIM>& R, int slot,
                                            const PlaneRegs<T, DIM>& P) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int s = threadIdx.x + h * kBlock;
    if (s >= kLX * kLY) break;
    const int sy = s / kLX, sx = s - sy * kLX;
#pragma unroll
    for (int c = 0; c < DIM; ++c) R.v[c][slot][sy][sx] = P.v[h][c];
  }
}

template <int DIM, typename T>
__device__ __forceinline__ void fill_plane(const Geo<T>& G, const T* const* u,
                                           const PlaneHalo<T, DIM>& Hh, PlaneRing<T, DIM>& R,
                                           int slot, int kk) {
  PlaneRegs<T, DIM> P;
  load_plane<DIM>(G, u, Hh, P, kk);
  store_plane<DIM>(R, slot, P);
}

// MODE 0: predictor (writes u*, and the forcing on forced faces).
// MODE 1: right-hand side only (writes R on advanced faces).
// z-chunk of the predictor's march: ten planes give 1536 blocks on the
// channel grid, six to a CU at this kernel's occupancy, so all of them run
// in one round (16-plane chunks left CUs idle); the tile metrics span more
// planes than that.
constexpr int kZChunkPred = 10;
static_assert(kZChunkPred <= kZChunk, "tile metric tables cover kZChunk + 2 planes");

template <typename T, int DIM, int MODE, bool UPW, bool IBA>
__global__ void __launch_bounds__(kBlock)
k_predictor(Geo<T> G, int ntx, int nty, int nzc, const T* __restrict__ u0,
            const T* __restrict__ u1, const T* __restrict__ u2, const T* __restrict__ fb0,
            const T* __restrict__ fb1, const T* __restrict__ fb2, T* __restrict__ o0,
            T* __restrict__ o1, T* __restrict__ o2, IbView<T> ib) {
  __shared__ PlaneRing<T, DIM> R;
  __shared__ TileMet<T> TM;
  const T* u[3] = {u0, u1, u2};
  const T* fbp[3] = {fb0, fb1, fb2};
  const int b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= ntx * nty * nzc) return;
  const int tx = b % ntx, ty = (b / ntx) % nty, zc = b / (ntx * nty);
  const int i0 = tx * kTileX, j0 = ty * kTileY;
  // one wavefront per tile row: ly (and so j) is uniform across the wave
  const int lx = threadIdx.x & (kTileX - 1);
  const int ly = __builtin_amdgcn_readfirstlane(threadIdx.x / kTileX);
  const int i = i0 + lx, j = j0 + ly;
  const int k0 = (DIM == 3) ? zc * kZChunkPred : 0;
  const int k1 = (DIM == 3) ? min(k0 + kZChunkPred, G.n[2]) : 1;
  const bool inside = i < G.n[0] && j < G.n[1];
  load_tile_met<DIM>(G, TM, i0, j0, k0);
  PlaneHalo<T, DIM> Hh;
  plane_halo_init<DIM>(G, Hh, i0, j0);
  // body force of this thread's faces, fetched one plane ahead
  T fbn[3] = {T(0), T(0), T(0)};
  auto load_fb = [&](int kk) {
#pragma unroll
    for (int c = 0; c < DIM; ++c)
      if (inside && fbp[c]) fbn[c] = fbp[c][fidx(G.ext[c], i, j, kk)];
  };
  load_fb(k0);
  PlaneRegs<T, DIM> nxt;
  if (DIM == 3) {
    fill_plane<DIM>(G, u, Hh, R, ring_slot(k0 - 1), k0 - 1);
    fill_plane<DIM>(G, u, Hh, R, ring_slot(k0), k0);
    fill_plane<DIM>(G, u, Hh, R, ring_slot(k0 + 1), k0 + 1);
    if (k0 + 1 < k1) load_plane<DIM>(G, u, Hh, nxt, k0 + 2);
  } else {
    fill_plane<DIM>(G, u, Hh, R, 0, 0);
  }
  for (int k = k0; k < k1; ++k) {
    __syncthreads();
    const int sc = (DIM == 3) ? ring_slot(k) : 0;
    const int sm = (DIM == 3) ? ring_slot(k - 1) : 0;
    const int sp = (DIM == 3) ? ring_slot(k + 1) : 0;
    T fbv[3] = {fbn[0], fbn[1], fbn[2]};
    if (k + 1 < k1) load_fb(k + 1);
    if (inside) {
      auto L = [&](int c, int di, int dj, int dk) -> T {
        const int sl = dk < 0 ? sm : (dk > 0 ? sp : sc);
        return R.v[c][sl][ly + 1 + dj][lx + 1 + di];
      };
      const MetLds<T> M{&TM, {lx + 1, ly + 1, k - k0 + 1}};
      predict_face<0, DIM, MODE, UPW, IBA, T>(G, L, M, fbv[0], o0, ib, i, j, k);
      predict_face<1, DIM, MODE, UPW, IBA, T>(G, L, M, fbv[1], o1, ib, i, j, k);
      predict_face<2, DIM, MODE, UPW, IBA, T>(G, L, M, fbv[2], o2, ib, i, j, k);
    }
    if (DIM == 3 && k + 1 < k1) {
      __syncthreads();
      store_plane<DIM>(R, sm, nxt);                   // slot of plane k-1 takes k+2
      if (k + 2 < k1) load_plane<DIM>(G, u, Hh, nxt, k + 3);
    }
  }
}

// ------------------------------------------------------ boundary faces
// Faces normal to a bounded axis: walls / inflow hold bc_vel, a convective
// outflow advects u_b with U_conv, a zero-gradient outflow copies the
// advanced neighbour.  The outward flux of every boundary face is summed
// (double) for the outflow correction.
template <typename T>
__device__ __forceinline__ double face_area(const Geo<T>& G, int c, int i, int j, int k) {
  const int I[3] = {i, j, k};
  double A = 1.0;
  for (int a = 0; a < G.dim; ++a)
    if (a != c) A *= (double)G.dx[a][I[a]];
  return A;
}

template <typename T>
__device__ __forceinline__ void plane_face(const Geo<T>& G, const Plane& P, int64_t r,
                                           int& i, int& j, int& k) {
  // enumerate the plane with the other two axes in (x, y, z) order
  int I[3];
  const int c = P.c;
  const int b = (P.side == 0) ? 0 : G.n[c];
  int64_t rem = r;
  for (int a = 0; a < 3; ++a) {
    if (a == c) { I[a] = b; continue; }
    const int na = G.n[a];
    I[a] = (int)(rem % na);
    rem /= na;
  }
  i = I[0]; j = I[1]; k = I[2];
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_boundary_faces(Geo<T> G, Planes PL, const T* __restrict__ un0, const T* __restrict__ un1,
                 const T* __restrict__ un2, T* us0, T* us1, T* us2, RedBuf red,
                 SolverScalars* sc) {
  const T* un[3] = {un0, un1, un2};
  T* us[3] = {us0, us1, us2};
  int64_t total = 0;
  for (int q = 0; q < PL.np; ++q) total += PL.p[q].count;
  double flux = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < total;
       r += (int64_t)gridDim.x * kBlock) {
    int q = 0;
    while (q + 1 < PL.np && r >= PL.p[q + 1].start) ++q;
    const Plane& P = PL.p[q];
    int i, j, k;
    plane_face(G, P, r - P.start, i, j, k);
    const int c = P.c;
    const int64_t id = fidx(G.ext[c], i, j, k);
    int In[3] = {i, j, k};
    In[c] += (P.side == 0) ? 1 : -1;
    const int64_t inner = fidx(G.ext[c], In[0], In[1], In[2]);
    T val;
    if (P.kind == FVIB_BC_OUTFLOW_CONVECTIVE) {
      const T ub = un[c][id];
      val = ub - G.dt * T(PL.u_conv) * (ub - un[c][inner]) / T(P.h);
    } else if (P.kind == FVIB_BC_OUTFLOW_NEUMANN) {
      val = us[c][inner];
    } else {
      val = T(P.value);
    }
    us[c][id] = val;
    const double sign = (P.side == 0) ? -1.0 : 1.0;
    flux += sign * (double)val * face_area(G, c, i, j, k);
  }
  if (!PL.any_outflow) return;
  double v[1] = {flux};
  block_partials<1, 1>(v, red.partial);
}

struct FinOutflow {         // net boundary flux per unit outflow area
  double area_out;
  __device__ bool skip(const SolverScalars*) const { return false; }
  __device__ void apply(const double* t, SolverScalars* sc) const { sc->meanb = t[0] / area_out; }
};

// Uniform correction of the outflow faces: u_b -= sign * net / area_out.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_outflow_correct(Geo<T> G, Planes PL, T* us0, T* us1, T* us2, const SolverScalars* sc) {
  T* us[3] = {us0, us1, us2};
  const double corr = sc->meanb;
  int64_t total = 0;
  for (int q = 0; q < PL.np; ++q) total += PL.p[q].count;
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < total;
       r += (int64_t)gridDim.x * kBlock) {
    int q = 0;
    while (q + 1 < PL.np && r >= PL.p[q + 1].start) ++q;
    const Plane& P = PL.p[q];
    if (P.kind != FVIB_BC_OUTFLOW_CONVECTIVE && P.kind != FVIB_BC_OUTFLOW_NEUMANN) continue;
    int i, j, k;
    plane_face(G, P, r - P.start, i, j, k);
    const int64_t id = fidx(G.ext[P.c], i, j, k);
    const double sign = (P.side == 0) ? -1.0 : 1.0;
    us[P.c][id] = (T)((double)us[P.c][id] - sign * corr);
  }
}

// ------------------------------------------------------------ launchers
template <typename T>
int launch_predictor(const Geo<T>& G, const T* const u[3], const T* const fb[3], T* out[3],
                     const IbView<T>& ib, int mode, hipStream_t s) {
  const int ntx = (G.n[0] + kTileX - 1) / kTileX;
  const int nty = (G.n[1] + kTileY - 1) / kTileY;
  const int nzc = (G.dim == 3) ? (G.n[2] + kZChunkPred - 1) / kZChunkPred : 1;
  int nb = ntx * nty * nzc;
  nb = (nb + kXcds - 1) / kXcds * kXcds;
  dim3 grid(nb), block(kBlock);
#define FVIB_PRED4(D, M, U, I)                                                                 \
  launch_kernel((k_predictor<T, D, M, U, I>), grid, block, 0, s, G, ntx, nty, nzc, u[0], u[1],  \
                u[2], fb[0], fb[1], fb[2], out[0], out[1], out[2], ib)
  // marker bodies (2D) force faces inside the predictor; a static box's
  // faces are fixed by a pass of their own afterwards
  const bool iba = ib.active && !ib.box;
#define FVIB_PRED(D, M)                                                                        \
  do {                                                                                         \
    if (G.upwind) {                                                                            \
      if (iba) FVIB_PRED4(D, M, true, true); else FVIB_PRED4(D, M, true, false);              \
    } else {                                                                                   \
      if (iba) FVIB_PRED4(D, M, false, true); else FVIB_PRED4(D, M, false, false);            \
    }                                                                                          \
  } while (0)
#define FVIB_PRED3(M)                                                                          \
  do {                                                                                         \
    if (G.upwind) FVIB_PRED4(3, M, true, false); else FVIB_PRED4(3, M, false, false);          \
  } while (0)
  if (G.dim == 2) {
    if (mode == 0) FVIB_PRED(2, 0); else FVIB_PRED(2, 1);
  } else {
    if (mode == 0) FVIB_PRED3(0); else FVIB_PRED3(1);
  }
#undef FVIB_PRED3
#undef FVIB_PRED
#undef FVIB_PRED4
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_boundary(const Geo<T>& G, const Planes& PL, const T* const un[3], T* us[3],
                    RedBuf red, SolverScalars* sc, hipStream_t s) {
  if (PL.np == 0) return FVIB_OK;
  int64_t total = 0;
  for (int q = 0; q < PL.np; ++q) total += PL.p[q].count;
  int nb = (int)((total + kBlock - 1) / kBlock);
  if (nb > kMaxRedBlocks) nb = kMaxRedBlocks;
  if (nb < 1) nb = 1;
  launch_kernel((k_boundary_faces<T>), dim3(nb), dim3(kBlock), 0, s, G, PL, un[0], un[1],
                     un[2], us[0], us[1], us[2], red, sc);
  FVIB_HIP(hipGetLastError());
  if (PL.any_outflow) {
    FVIB_HIP((launch_finish<1, 1>(red.partial, nb, sc, FinOutflow{PL.area_out}, s)));
    launch_kernel((k_outflow_correct<T>), dim3(nb), dim3(kBlock), 0, s, G, PL, us[0], us[1],
                       us[2], (const SolverScalars*)sc);
    FVIB_HIP(hipGetLastError());
  }
  return FVIB_OK;
}

template int launch_predictor<float>(const Geo<float>&, const float* const[3],
                                     const float* const[3], float* [3], const IbView<float>&,
                                     int, hipStream_t);
template int launch_predictor<double>(const Geo<double>&, const double* const[3],
                                      const double* const[3], double* [3],
                                      const IbView<double>&, int, hipStream_t);
template int launch_boundary<float>(const Geo<float>&, const Planes&, const float* const[3],
                                    float* [3], RedBuf, SolverScalars*, hipStream_t);
template int launch_boundary<double>(const Geo<double>&, const Planes&, const double* const[3],
                                     double* [3], RedBuf, SolverScalars*, hipStream_t);

}  // namespace fvib
