// Internal definitions shared by the fvib HIP translation units.
//
// Staggered (MAC) layout: component c lives on faces normal to axis c and
// face i along axis c is the low face of cell i; arrays are (z, y, x) with
// x fastest (see include/fvib.h).  Everything here is written for gfx950:
// 64-wide wavefronts, 256-thread blocks, eight XCDs with private L2.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fvib.h"

namespace fvib {

// Kernel timing without marker packets: while a timed section is open on
// this thread, launches carry the section's events in their own dispatch
// (the first launch records the start, every launch the end), so the
// measured interval is kernel execution only and the stream gets no extra
// packets between kernels.
struct LaunchTiming {
  hipEvent_t start, stop;
  bool first;                    // no launch has recorded start yet
};
extern thread_local LaunchTiming* t_launch_timing;

template <typename F, typename... Args>
inline void launch_kernel(F kernel, const dim3& grid, const dim3& block, uint32_t shmem,
                          hipStream_t s, Args... args) {
  LaunchTiming* lt = t_launch_timing;
  if (!lt) {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
    return;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, lt->first ? lt->start : nullptr, lt->stop,
                        0u, args...);
  lt->first = false;
}

constexpr int kBlock = 256;          // threads per block (4 wavefronts)
constexpr int kTileX = 64;           // one wavefront spans 64 consecutive x
constexpr int kTileY = 4;            // four wavefronts stacked in y
constexpr int kMaxRedBlocks = 2048;  // partial-sum slots of a reduction
constexpr int kXcds = 8;             // MI355X: 8 XCDs, round-robin dispatch

// ---------------------------------------------------------------- geometry
// Per-axis metrics (see the grid description in the header):
//   dx[i]  cell width (n), dxe[e] widths with one mirrored/periodic ghost on
//   each side (n + 2, dxe[i + 1] = dx[i]), dc[f] centre spacing at face f
//   (n + 1), wi[f] interpolation weight of the upper cell at face f (n + 1).
// Stencil coefficients of one index along an axis, four per entry so one
// vector load fetches them.  Cell entries (index -1 .. n):
//   x = 1/dx, y = 1/(dc[i+1] dx[i]), z = 1/(dc[i] dx[i]), w = 0;
// face entries (index -1 .. n+1):
//   x = 1/dc, y = 1/(dxe[f+1] dc[f]), z = 1/(dxe[f] dc[f]), w = wi[f].
// Entries past the ends wrap on periodic axes and repeat the end entry on
// bounded ones (there they only ever multiply a zero adjoint).
template <typename T>
struct alignas(4 * sizeof(T)) Met4 {
  T x, y, z, w;
};

template <typename T>
struct Geo {
  int dim;
  int n[3];
  int per[3];
  int ext[3][3];       // ext[c][a]: extent of component c along axis a
  int dir[3][2];       // 1: Dirichlet ghost rule on boundary (a, side)
  T gv[3][3][2];       // ghost value g of comp c behind boundary (a, side)
  const T *dx[3], *dxe[3], *dc[3], *wi[3];
  const Met4<T>* mc[3];  // cell coefficients, mc[a][i] valid for i in [-1, n]
  const Met4<T>* mf[3];  // face coefficients, mf[a][f] valid for f in [-1, n+1]
  T nu, dt, rho;
  int upwind;
};

// Immersed-boundary window (2D): per component a fixed-size box of faces
// around the body; its origin follows the body and lives in device memory.
template <typename T>
struct IbView {
  int active;
  int W[2][2];                  // W[c][0] width in x, W[c][1] width in y
  const int *origin;            // origin[2c + 0/1]: first face index x / y
  const uint8_t *cls[2];        // 0 fluid, 1 solid, 2 immersed-boundary point
  const T *us[2];               // target velocity on forced faces
  T *f[2];                      // direct forcing written by the predictor
  const double *body;           // body state [d(3), v(3)]
  // static box on a 3D grid (box != 0): per component a fixed window of
  // faces around the box with a forced flag per face; the predictor writes
  // the forcing there, the adjoint reads the forcing adjoint from it
  int box;
  int bo[3][3];                 // bo[c][a]: first face index of the window
  int bw[3][3];                 // bw[c][a]: window extent
  const uint8_t *bcls[3];       // 1 on forced faces
  T *bf[3];                     // forcing (forward) / its adjoint (adjoint)
};

// Forced face (i, j, k) of component C of a static box: window index in
// *lidx.
template <int C, typename T>
__device__ __forceinline__ int forced_box(const IbView<T>& ib, int i, int j, int k, int* lidx) {
  const int li = i - ib.bo[C][0], lj = j - ib.bo[C][1], lk = k - ib.bo[C][2];
  if (li < 0 || lj < 0 || lk < 0 || li >= ib.bw[C][0] || lj >= ib.bw[C][1] || lk >= ib.bw[C][2])
    return 0;
  *lidx = (lk * ib.bw[C][1] + lj) * ib.bw[C][0] + li;
  return ib.bcls[C][*lidx];
}

__host__ __device__ inline int64_t fidx(const int ext[3], int i, int j, int k) {
  return ((int64_t)k * ext[1] + j) * ext[0] + i;
}

// Load component C at integer index (i, j, k) where at most one index may
// lie one step outside the array: periodic axes wrap, and behind a wall /
// inflow (Dirichlet) the ghost is 2 g - u_0, otherwise (free slip,
// outflow) it is u_0.  Along its own bounded axis a component is never
// addressed outside [0, n].
template <int C, int DIM, typename T>
__device__ __forceinline__ T ld(const Geo<T>& G, const T* __restrict__ q, int i, int j, int k) {
  int I[3] = {i, j, k};
  T off = T(0);
  bool neg = false;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int e = G.ext[C][a];
    if (I[a] < 0) {
      if (G.per[a]) {
        I[a] += e;
      } else {
        I[a] = 0;
        if (G.dir[a][0]) { neg = true; off = T(2) * G.gv[C][a][0]; }
      }
    } else if (I[a] >= e) {
      if (G.per[a]) {
        I[a] -= e;
      } else {
        I[a] = e - 1;
        if (G.dir[a][1]) { neg = true; off = T(2) * G.gv[C][a][1]; }
      }
    }
  }
  const T v = q[fidx(G.ext[C], I[0], I[1], I[2])];
  return neg ? off - v : v;
}

// Branch-free variant of ld for halo fills: the index of each axis is
// wrapped (periodic) or clamped (bounded) with selects, and the ghost rule
// of the last axis found outside is applied.  *outside reports whether any
// bounded axis was left (the index then names the boundary-adjacent face).
template <int C, int DIM, typename T>
__device__ __forceinline__ T ld_halo(const Geo<T>& G, const T* __restrict__ q, int i, int j,
                                     int k, bool* outside) {
  int I[3] = {i, j, k};
  T off = T(0);
  bool neg = false, out = false;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int e = G.ext[C][a];
    const bool lo = I[a] < 0, hi = I[a] >= e;
    const bool per = G.per[a] != 0;
    const int wrapped = lo ? I[a] + e : (hi ? I[a] - e : I[a]);
    const int clamped = lo ? 0 : (hi ? e - 1 : I[a]);
    I[a] = per ? wrapped : clamped;
    const bool ghost = !per && (lo || hi);
    const bool dir = lo ? (G.dir[a][0] != 0) : (G.dir[a][1] != 0);
    const T g2 = T(2) * (lo ? G.gv[C][a][0] : G.gv[C][a][1]);
    neg = (ghost && dir) ? true : (ghost ? false : neg);
    off = (ghost && dir) ? g2 : off;
    out = out || ghost;
  }
  *outside = out;
  const T v = q[fidx(G.ext[C], I[0], I[1], I[2])];
  return neg ? off - v : v;
}

// --------------------------------------------------------- tile iteration
// Logical tiles of kTileX x kTileY cells in one z-plane.  Blocks are
// dispatched round-robin over the XCDs; remapping the block id makes every
// XCD sweep one contiguous slab so stencil neighbours hit its own L2.
struct Tiling {
  int ntx, nty, nz;
  int ntiles;
  int nblocks;      // padded to a multiple of kXcds
};

inline Tiling make_tiling(int nx, int ny, int nz, int max_blocks = kMaxRedBlocks) {
  Tiling t;
  t.ntx = (nx + kTileX - 1) / kTileX;
  t.nty = (ny + kTileY - 1) / kTileY;
  t.nz = nz;
  t.ntiles = t.ntx * t.nty * t.nz;
  int nb = t.ntiles < max_blocks ? t.ntiles : max_blocks;
  nb = (nb + kXcds - 1) / kXcds * kXcds;
  t.nblocks = nb;
  return t;
}

// Column march: a unit is one tile of an x-y plane and a chunk of z-planes;
// each thread owns one (i, j) column of its unit and walks up the chunk,
// so values of plane k + 1 are reused as plane k and k - 1 (each value
// crosses HBM once per chunk) and the next plane is prefetched.
struct ColTiling {
  int ntx, nty, nzc, zchunk;
  int nunits;
  int nblocks;      // multiple of kXcds, at most kMaxRedBlocks
};

inline ColTiling make_col_tiling(int nx, int ny, int nz) {
  ColTiling t;
  t.ntx = (nx + kTileX - 1) / kTileX;
  t.nty = (ny + kTileY - 1) / kTileY;
  const int per_plane = t.ntx * t.nty;
  // chunks of about ten planes: more columns in flight than longer chunks
  // (a march is latency bound), less halo and set-up than shorter ones
  int nzc = (nz + 9) / 10;
  if (per_plane * nzc > kMaxRedBlocks) nzc = kMaxRedBlocks / per_plane > 0 ? kMaxRedBlocks / per_plane : 1;
  t.zchunk = (nz + nzc - 1) / nzc;
  t.nzc = (nz + t.zchunk - 1) / t.zchunk;
  t.nunits = per_plane * t.nzc;
  int nb = t.nunits < kMaxRedBlocks ? t.nunits : kMaxRedBlocks;
  t.nblocks = (nb + kXcds - 1) / kXcds * kXcds;
  return t;
}

__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  const int per = nblocks / kXcds;       // nblocks is a multiple of kXcds
  return (b % kXcds) * per + b / kXcds;
}

// LDS halo planes (tile of kTileX x kTileY cells plus a one-cell halo) kept
// in a three-slot ring for planes k-1, k, k+1 while a block marches in z.
constexpr int kZChunk = 16;
constexpr int kLX = kTileX + 2, kLY = kTileY + 2;

template <typename T, int DIM>
struct PlaneRing {
  T v[DIM][3][kLY][kLX];
};

__device__ __forceinline__ int ring_slot(int k) { return ((k % 3) + 3) % 3; }

// Stencil coefficients of a block's tile in LDS: entries -1 .. 64 of the
// tile along x, -1 .. 4 along y and -1 .. kZChunk along z (relative to the
// tile origin), loaded once per block since they do not change along the
// z-march.  Indices past the grid are clamped (those entries are never
// used for a real face).
constexpr int kMX = (kLX > kZChunk + 2) ? kLX : kZChunk + 2;

template <typename T>
struct TileMet {
  Met4<T> c[3][kMX];
  Met4<T> f[3][kMX];
};

template <int DIM, typename T>
__device__ __forceinline__ void load_tile_met(const Geo<T>& G, TileMet<T>& M, int i0, int j0,
                                              int k0) {
  const int base[3] = {i0 - 1, j0 - 1, k0 - 1};
  for (int e = threadIdx.x; e < DIM * kMX; e += kBlock) {
    const int a = e / kMX, x = e - a * kMX;
    const int n = G.n[a];
    const int gi = base[a] + x;
    M.c[a][x] = G.mc[a][min(gi, n)];        // cell entries exist for -1 .. n
    M.f[a][x] = G.mf[a][min(gi, n + 1)];    // face entries for -1 .. n + 1
  }
}

// Coefficient access relative to a face J: mc(a, off) / mf(a, off) are the
// cell / face entries at index J[a] + off (off in -1 .. 1) along axis a.
template <typename T>
struct MetLds {
  const TileMet<T>* M;
  int o[3];           // LDS index of J along each axis
  __device__ __forceinline__ Met4<T> mc(int a, int off) const { return M->c[a][o[a] + off]; }
  __device__ __forceinline__ Met4<T> mf(int a, int off) const { return M->f[a][o[a] + off]; }
};

// As MetLds with the LDS index clamped to the tile's table (for a face one
// step past the tile, whose out-of-table entries only multiply zero terms).
template <typename T>
struct MetLdsClamp {
  const TileMet<T>* M;
  int o[3];
  __device__ __forceinline__ Met4<T> mc(int a, int off) const { return M->c[a][min(o[a] + off, kMX - 1)]; }
  __device__ __forceinline__ Met4<T> mf(int a, int off) const { return M->f[a][min(o[a] + off, kMX - 1)]; }
};

template <typename T>
struct MetGlobal {
  const Geo<T>* G;
  int J[3];
  __device__ __forceinline__ Met4<T> mc(int a, int off) const { return G->mc[a][J[a] + off]; }
  __device__ __forceinline__ Met4<T> mf(int a, int off) const { return G->mf[a][J[a] + off]; }
};


// ------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide sum of NV values per thread (fixed order: deterministic).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double sh[NV][kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = wave_sum(v[q]);
    if (lane == 0) sh[q][w] = s;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) s += sh[q][k];
    v[q] = s;
  }
  __syncthreads();
}

// As block_sum for a block of NT threads (a multiple of 64).
template <int NV, int NT>
__device__ __forceinline__ void block_sum_n(double (&v)[NV]) {
  __shared__ double sh[NV][NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = wave_sum(v[q]);
    if (lane == 0) sh[q][w] = s;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) s += sh[q][k];
    v[q] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ double block_max(double v) {
  __shared__ double sh[kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double s = wave_max(v);
  if (lane == 0) sh[w] = s;
  __syncthreads();
  double m = sh[0];
#pragma unroll
  for (int k = 1; k < kBlock / 64; ++k) m = fmax(m, sh[k]);
  __syncthreads();
  return m;
}

// Deterministic two-pass grid reduction.  Every block of the producing
// kernel reduces its values in a fixed order and stores one partial per
// value; a one-block kernel launched right after it on the same stream
// combines the partials in block order and hands the totals to an
// epilogue.  The kernel boundary makes the partials visible, so no block
// needs a device-wide fence (on a multi-XCD part such a fence writes back
// and invalidates the XCD's L2 and costs every block that follows it).
// Kinds: the first NS values are sums, the remaining NV - NS are maxima.
template <int NV, int NS>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* partial) {
  double s[NS > 0 ? NS : 1];
  if constexpr (NS > 0) {
#pragma unroll
    for (int q = 0; q < NS; ++q) s[q] = v[q];
    block_sum<NS>(s);
  }
  double mx[NV - NS > 0 ? NV - NS : 1];
#pragma unroll
  for (int q = NS; q < NV; ++q) mx[q - NS] = block_max(v[q]);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NS; ++q) partial[q * kMaxRedBlocks + blockIdx.x] = s[q];
#pragma unroll
    for (int q = NS; q < NV; ++q) partial[q * kMaxRedBlocks + blockIdx.x] = mx[q - NS];
  }
}

struct SolverScalars;

// Second pass: FIN::skip(sc) lets an epilogue stand down with its producer
// (a finished CG solve launches no work); FIN::apply(tot, sc) runs on
// thread 0 with the totals.
template <int NV, int NS, typename FIN>
__global__ void __launch_bounds__(kBlock)
k_reduce_finish(const double* __restrict__ partial, int nb, SolverScalars* sc, FIN fin) {
  if (fin.skip(sc)) return;
  // all loads issued before the (fixed-order) combination
  constexpr int kPer = kMaxRedBlocks / kBlock;
  double x[NV][kPer];
#pragma unroll
  for (int q = 0; q < NV; ++q)
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int b = threadIdx.x + u * kBlock;
      x[q][u] = (b < nb) ? partial[q * kMaxRedBlocks + b] : ((q < NS) ? 0.0 : -1.0);
    }
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double a = (q < NS) ? 0.0 : -1.0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) a = (q < NS) ? a + x[q][u] : fmax(a, x[q][u]);
    acc[q] = a;
  }
  double tot[NV];
  if constexpr (NS > 0) {
    double tmp[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) tmp[q] = acc[q];
    block_sum<NS>(tmp);
#pragma unroll
    for (int q = 0; q < NS; ++q) tot[q] = tmp[q];
  }
#pragma unroll
  for (int q = NS; q < NV; ++q) tot[q] = block_max(acc[q]);
  if (threadIdx.x == 0) fin.apply(tot, sc);
}

// The one-block epilogue is left out of an open timed section, so a
// section times its main kernel alone.
template <int NV, int NS, typename FIN>
inline hipError_t launch_finish(const double* partial, int nb, SolverScalars* sc, const FIN& fin,
                                hipStream_t s) {
  LaunchTiming* saved = t_launch_timing;
  t_launch_timing = nullptr;
  launch_kernel((k_reduce_finish<NV, NS, FIN>), dim3(1), dim3(kBlock), 0, s, partial, nb, sc,
                     fin);
  t_launch_timing = saved;
  return hipGetLastError();
}

// Pressure-operator metrics in the vector type V of the solve.
template <typename V>
struct PGeo {
  int dim;
  int n[3];
  int per[3];
  const V* dx[3];    // cell widths
  const V* idc[3];   // 1 / centre spacing at faces 0..n
  const V* kf[3];    // idc with zeros on the faces of a bounded boundary
  const V* iv[3];    // 1 / cell width
  double dt_over_rho;
  double inv_ncell;
};

// Boundary-normal face planes of bounded axes (at most six).
struct Plane {
  int c, side, kind;
  int64_t count;      // faces in the plane
  int64_t start;      // prefix offset in the flattened plane list
  double value;       // prescribed normal velocity
  double h;           // spacing between the boundary face and its neighbour
};

struct Planes {
  int np;
  Plane p[6];
  int any_outflow;
  double area_out;
  double u_conv;
};

// Device-side scalars of the Poisson solver (one instance per handle).
struct SolverScalars {
  double rr;        // r.r of the current iterate
  double rr0;       // r.r at the start of the (inner) solve
  double pq;        // p.Ap
  double alpha, beta;
  double crit;      // max |r_c / V_c| * dt / rho of the last check
  double meanb;     // mean of the PPE right-hand side
  double sumx;      // sum of the initial iterate of the solve (gauge)
  double sump;      // sum of the current search direction (gauge)
  double tol_rr;    // inner stopping threshold on r.r (mixed inner solve)
  double div_max;   // max |D u^{n+1}| of the projection
  double force[3];
  double loss;
  double ymax;      // adjoint right-hand side: max |y / V|
  double tol_dev;   // stopping target set on the device (tol < 0 on the host)
  double xi;        // coupling error of the last structural sub-iteration
  double cfl_dt;    // CFL-limited time step of the last launch_cfl_dt
  int done;         // current CG solve finished
  int outer_done;   // refinement finished
  int iters;        // iterations of the current CG solve
  int status;       // FVIB_OK or a negative status
  int clamp;        // body window clamped (body left the allowed region)
  int sweeps;       // refinement corrections applied in the current solve
  int pad[2];
};

struct RedBuf {
  double* partial;          // 5 * kMaxRedBlocks doubles
};

// ------------------------------------------------------------ host glue
#define FVIB_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) return fvib::hip_fail(e_, #call, __FILE__, __LINE__); \
  } while (0)

int hip_fail(hipError_t e, const char* what, const char* file, int line);

}  // namespace fvib
