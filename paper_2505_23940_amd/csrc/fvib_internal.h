// Internal definitions shared by the fvib HIP translation units.
//
// Staggered (MAC) layout: component c lives on faces normal to axis c and
// face i along axis c is the low face of cell i; arrays are (z, y, x) with
// x fastest (see include/fvib.h).  Everything here is written for gfx950:
// 64-wide wavefronts, 256-thread blocks, eight XCDs with private L2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fvib.h"

namespace fvib {

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
template <typename T>
struct Geo {
  int dim;
  int n[3];
  int per[3];
  int ext[3][3];       // ext[c][a]: extent of component c along axis a
  int dir[3][2];       // 1: Dirichlet ghost rule on boundary (a, side)
  T gv[3][3][2];       // ghost value g of comp c behind boundary (a, side)
  const T *dx[3], *dxe[3], *dc[3], *wi[3];
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
};

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

// Deterministic grid reduction: every block stores its partials, the last
// block to arrive (atomic ticket) combines them in block order.  Returns
// true in the last block, whose threads then all hold the totals in tot.
// Kinds: first NS values are sums, the remaining NV - NS are maxima.
template <int NV, int NS>
__device__ __forceinline__ bool grid_reduce(double (&v)[NV], double* partial,
                                            unsigned int* ticket, double (&tot)[NV]) {
  __shared__ bool last;
  double s[NS > 0 ? NS : 1];
#pragma unroll
  for (int q = 0; q < NS; ++q) s[q] = v[q];
  if constexpr (NS > 0) {
    double tmp[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) tmp[q] = s[q];
    block_sum<NS>(tmp);
#pragma unroll
    for (int q = 0; q < NS; ++q) s[q] = tmp[q];
  }
  double mx[NV - NS > 0 ? NV - NS : 1];
#pragma unroll
  for (int q = NS; q < NV; ++q) mx[q - NS] = block_max(v[q]);
  const int nb = gridDim.x;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NS; ++q) partial[q * kMaxRedBlocks + blockIdx.x] = s[q];
#pragma unroll
    for (int q = NS; q < NV; ++q) partial[q * kMaxRedBlocks + blockIdx.x] = mx[q - NS];
    __threadfence();
    const unsigned int t = atomicAdd(ticket, 1u);
    last = (t == (unsigned int)(nb - 1));
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double a = (q < NS) ? 0.0 : -1.0;
    const volatile double* pq = partial + q * kMaxRedBlocks;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
      const double x = pq[b];
      a = (q < NS) ? a + x : fmax(a, x);
    }
    acc[q] = a;
  }
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
  if (threadIdx.x == 0) *ticket = 0u;   // ready for the next launch
  return true;
}

// Pressure-operator metrics in the vector type V of the solve.
template <typename V>
struct PGeo {
  int dim;
  int n[3];
  int per[3];
  const V* dx[3];    // cell widths
  const V* idc[3];   // 1 / centre spacing at faces 0..n
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
  int done;         // current CG solve finished
  int outer_done;   // refinement finished
  int iters;        // iterations of the current CG solve
  int status;       // FVIB_OK or a negative status
  int clamp;        // body window clamped (body left the allowed region)
  int pad[3];
};

struct RedBuf {
  double* partial;          // 4 * kMaxRedBlocks doubles
  unsigned int* ticket;     // one counter per reduction site
};

// ------------------------------------------------------------ host glue
#define FVIB_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) return fvib::hip_fail(e_, #call, __FILE__, __LINE__); \
  } while (0)

int hip_fail(hipError_t e, const char* what, const char* file, int line);

}  // namespace fvib
