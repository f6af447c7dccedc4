// Exact solve of the separable PPE operator by fast diagonalisation.
//
// The volume-integrated operator is a Kronecker sum A = sum_a (W_other (x) T_a)
// with T_a the 1D symmetric tridiagonal (periodic: circulant) operator of
// axis a and W_a = diag(dx_a).  With the per-axis generalised eigenpairs
// T_a Phi_a = W_a Phi_a Lambda_a, Phi_a^T W_a Phi_a = I, its pseudo-inverse
// is  A^+ = Phi diag(1 / (lam_x + lam_y + lam_z)) Phi^T  (zero mode -> 0).
//
// On the GPU each factor Phi_a^T (forward) and Phi_a (inverse) is a dense
// contraction over one grid axis, i.e. a GEMM whose small dimension is the
// axis length; it runs on the matrix cores (MFMA 16x16x4, float or double),
// staged through LDS.  The division by the eigenvalue sum is fused into the
// last forward contraction.  The solve is used as the inner solver of the
// double-residual iterative refinement, so the answer is certified by the
// double residual of the operator itself, not by the eigenbases.
#include <math.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "fvib_kernels.h"

namespace fvib {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename V>
struct Mfma;

// Operands (both types): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  The 16x16 result holds D[row][l % 16] in register v
// with row = 4 (l / 16) + v for float and row = 4 v + l / 16 for double
// (measured on gfx950).
template <>
struct Mfma<float> {
  typedef floatx4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <>
struct Mfma<double> {
  typedef doublex4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

constexpr int BM = 64;   // rows of the axis operator per block (output modes)
constexpr int BN = 64;   // grid lines (columns) per block
constexpr int BKc = 16;  // contraction chunk

// Y[o][m][i] = sum_k A[m][k] X[o][k][i] for m < K, columns n = o * inner + i.
// XFAST: inner == 1 (contraction along the contiguous axis).
// DIV:   multiply by 1 / (lam_x[mx] + lam_y[my] + lam_z[mz]) (zero mode 0);
//        used on the last forward contraction (outer == 1, the modes of the
//        other axes are decoded from i).
template <typename V, bool XFAST, bool DIV>
__global__ void __launch_bounds__(kBlock)
k_axis_gemm(const V* __restrict__ X, V* __restrict__ Y, const V* __restrict__ A, int K,
            int inner, int64_t ncols, FdmDiv dv, const int* stop) {
  if (stop && *stop) return;
  __shared__ V As[BKc][BM + 1];
  __shared__ V Bs[BKc][BN + 1];
  typedef typename Mfma<V>::acc_t acc_t;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.x * BM;
  const int64_t n0 = (int64_t)blockIdx.y * BN;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  // per-thread column bases for the B tile
  int64_t colbase[4];
  bool colok[4];
  int bk[4], bn[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (XFAST) {
      bk[r] = t & 15;
      bn[r] = (t >> 4) + 16 * r;
    } else {
      bn[r] = t & 63;
      bk[r] = (t >> 6) + 4 * r;
    }
    const int64_t n = n0 + bn[r];
    colok[r] = n < ncols;
    if (XFAST) {
      colbase[r] = n * (int64_t)K;
    } else {
      const int64_t o = n / inner, i = n - o * inner;
      colbase[r] = o * (int64_t)K * inner + i;
    }
  }
  for (int k0 = 0; k0 < K; k0 += BKc) {
    // A tile: As[k][m] = A[(m0 + m) K + k0 + k]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = t + r * kBlock;         // 0..1023
      const int m = e >> 4, k = e & 15;
      const int gm = m0 + m, gk = k0 + k;
      As[k][m] = (gm < K && gk < K) ? A[(int64_t)gm * K + gk] : V(0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gk = k0 + bk[r];
      V v = V(0);
      if (colok[r] && gk < K)
        v = XFAST ? X[colbase[r] + gk] : X[colbase[r] + (int64_t)gk * inner];
      Bs[bk[r]][bn[r]] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BKc / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      V a0 = As[kr][wm + (lane & 15)];
      V a1 = As[kr][wm + 16 + (lane & 15)];
      V b0 = Bs[kr][wn + (lane & 15)];
      V b1 = Bs[kr][wn + 16 + (lane & 15)];
      acc[0][0] = Mfma<V>::op(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<V>::op(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<V>::op(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<V>::op(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  // epilogue: lane holds D[Mfma<V>::row(lane, v)][col = lane % 16]
#pragma unroll
  for (int ti = 0; ti < 2; ++ti) {
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      const int64_t n = n0 + wn + tj * 16 + (lane & 15);
      if (n >= ncols) continue;
      int64_t o = 0, i = 0, base;
      if (XFAST) {
        base = n * (int64_t)K;
      } else {
        o = n / inner;
        i = n - o * inner;
        base = o * (int64_t)K * inner + i;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + ti * 16 + Mfma<V>::row(lane, v);
        if (m >= K) continue;
        V val = acc[ti][tj][v];
        if (DIV) {
          // last forward axis: modes of the faster axes come from i
          int mm[3] = {0, 0, 0};
          int64_t rem = XFAST ? 0 : i;
          for (int b = 0; b < dv.axis; ++b) {
            mm[b] = (int)(rem % dv.n[b]);
            rem /= dv.n[b];
          }
          mm[dv.axis] = m;
          double ls = 0.0;
          for (int b = 0; b < dv.dim; ++b) ls += dv.lam[b][mm[b]];
          const bool zero = (mm[0] == 0 && mm[1] == 0 && mm[2] == 0);
          val = zero ? V(0) : (V)((double)val / ls);
        }
        // non-temporal: see the note on k_fft_axis' stores
        if (XFAST)
          __builtin_nontemporal_store(val, Y + base + m);
        else
          __builtin_nontemporal_store(val, Y + base + (int64_t)m * inner);
      }
    }
  }
}

// Register-blocked variant for axes of at most 256 cells with K % 4 == 0
// (every axis of the production grids).  A block owns 16 NT grid lines and
// produces all K modes for them, so X is read from HBM once; wave w owns
// the 16-row tiles w, w + 4, ... of the operator.  Both operands go straight
// from L1/L2 into registers: within a batch of 16 contraction indices, lane
// group q holds indices 4q .. 4q + 3 (contiguous in a row of A, and in a
// line of X when the axis is the fast one) and MFMA step s contracts index
// 4q + s, so each operand needs one vector load per batch.  The next batch
// is loaded while the current one is multiplied.
template <typename V>
struct Quad {
  V v[4];
};

template <typename V, bool CONTIG>
__device__ __forceinline__ Quad<V> ld_quad(const V* p, int64_t stride) {
  Quad<V> r;
  if constexpr (CONTIG) {
    if constexpr (sizeof(V) == 4) {
      const float4 t = *reinterpret_cast<const float4*>(p);
      r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
    } else {
      const double2 t0 = *reinterpret_cast<const double2*>(p);
      const double2 t1 = *reinterpret_cast<const double2*>(p + 2);
      r.v[0] = t0.x; r.v[1] = t0.y; r.v[2] = t1.x; r.v[3] = t1.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) r.v[j] = p[j * stride];
  }
  return r;
}

template <typename V, bool XFAST, bool DIV, bool TAIL, int MT, int NT>
__global__ void __launch_bounds__(kBlock)
k_axis_mfma(const V* __restrict__ X, V* __restrict__ Y, const V* __restrict__ A, int K,
            int inner, int64_t ncols, FdmDiv dv, const int* stop) {
  if (stop && *stop) return;
  typedef typename Mfma<V>::acc_t acc_t;
  // quads per batch: 2 (32 contraction indices) in float, 1 in double
  constexpr int QB = sizeof(V) == 4 ? 2 : 1;
  constexpr int KB = 16 * QB;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int q = lane >> 4, r = lane & 15;
  const int ntr = (K + 15) >> 4;
  const int64_t n0 = (int64_t)blockIdx.x * (16 * NT);
  // every wave runs MT row tiles; tiles past K read row K - 1 and are
  // never stored
  const V* ap[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    int m = 16 * (w + 4 * mt) + r;
    if (m >= K) m = K - 1;
    ap[mt] = A + (int64_t)m * K + 4 * q;
  }
  const V* xp[NT];
  int64_t base[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    int64_t n = n0 + 16 * t + r;
    if (n >= ncols) n = ncols - 1;          // lines past ncols likewise
    if (XFAST) {
      base[t] = n * (int64_t)K;
      xp[t] = X + base[t] + 4 * q;
    } else {
      const int64_t o = n / inner, i = n - o * inner;
      base[t] = o * (int64_t)K * inner + i;
      xp[t] = X + base[t] + (int64_t)(4 * q) * inner;
    }
  }
  acc_t acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[mt][t] = acc_t{0, 0, 0, 0};
  auto load = [&](int kb, Quad<V> (*a)[MT], Quad<V> (*b)[NT]) {
#pragma unroll
    for (int j = 0; j < QB; ++j) {
      // K % 4 == 0: a quad is all inside or all past K.  With TAIL, a quad
      // past K is read at k = 0 of its line and its operator part zeroed
      // (the product is then zero whatever the line holds there).
      const int k = kb + 16 * j;
      const bool ok = !TAIL || k + 4 * q < K;
      const int ka = ok ? k : -4 * q;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        a[j][mt] = ld_quad<V, true>(ap[mt] + ka, 1);
        if (TAIL) {
          const V z = ok ? V(1) : V(0);
#pragma unroll
          for (int e = 0; e < 4; ++e) a[j][mt].v[e] *= z;
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t)
        b[j][t] = ld_quad<V, XFAST>(xp[t] + (XFAST ? ka : (int64_t)ka * inner), inner);
    }
  };
  auto compute = [&](const Quad<V> (*a)[MT], const Quad<V> (*b)[NT]) {
#pragma unroll
    for (int j = 0; j < QB; ++j)
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[mt][t] = Mfma<V>::op(a[j][mt].v[s], b[j][t].v[s], acc[mt][t]);
  };
  // two register buffers in ping-pong: batch kb + KB is in flight while
  // batch kb is multiplied
  Quad<V> a0[QB][MT], b0[QB][NT], a1[QB][MT], b1[QB][NT];
  load(0, a0, b0);
  int kb = 0;
  for (; kb + KB < K; kb += 2 * KB) {
    load(kb + KB, a1, b1);
    compute(a0, b0);
    if (kb + 2 * KB < K) load(kb + 2 * KB, a0, b0);
    compute(a1, b1);
  }
  if (kb < K) compute(a0, b0);
  // epilogue: lane holds D[Mfma<V>::row(lane, v)][col r] of each tile
  double lrest[NT];
  if (DIV) {
    // eigenvalue sum of the faster axes' modes of each line (decoded from i)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t n = n0 + 16 * t + r;
      int64_t rem = XFAST ? 0 : (n % inner);
      double ls = 0.0;
      int allz = 1;
      for (int b = 0; b < dv.axis; ++b) {
        const int mb = (int)(rem % dv.n[b]);
        rem /= dv.n[b];
        ls += dv.lam[b][mb];
        allz &= (mb == 0);
      }
      lrest[t] = allz ? -1.0 : ls;          // -1 marks the lines of the zero mode
    }
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    if (w + 4 * mt >= ntr) continue;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t n = n0 + 16 * t + r;
      if (n >= ncols) continue;
      const int mrow0 = 16 * (w + 4 * mt);
      if constexpr (XFAST && !DIV && sizeof(V) == 4) {
        // float layout: this lane's four values are rows 4q .. 4q + 3 of
        // one line, contiguous along the fast axis (K % 4 == 0)
        const int m = mrow0 + 4 * q;
        if (m < K) {
          const acc_t& c = acc[mt][t];
          *reinterpret_cast<float4*>(Y + base[t] + m) = make_float4(c[0], c[1], c[2], c[3]);
        }
        continue;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = mrow0 + Mfma<V>::row(lane, v);
        if (m >= K) continue;
        V val = acc[mt][t][v];
        if (DIV) {
          const bool zero = (lrest[t] < 0.0) && m == 0;
          const double ls = (lrest[t] < 0.0 ? 0.0 : lrest[t]) + dv.lam[dv.axis][m];
          val = zero ? V(0) : (V)((double)val / ls);
        }
        if (XFAST)
          Y[base[t] + m] = val;
        else
          Y[base[t] + (int64_t)m * inner] = val;
      }
    }
  }
}

// LDS-staged variant (K % 32 == 0, K <= 256, and for a strided axis
// blocks of lines that never straddle two outer indices): per chunk of KC
// contraction indices the block loads the operator rows (K x KC) and its
// 16 NT lines (16 NT x KC) with 16-byte coalesced loads into LDS, both
// stored contraction-contiguous, and each wave reads its MFMA operands back
// as 16-byte LDS reads (same quad assignment as above).  The next chunk is
// loaded into registers while the current one is multiplied.  NT is chosen
// per axis so that the blocks spread evenly over the CUs.
template <typename V>
struct LdsGemm {
  static constexpr int KC = sizeof(V) == 4 ? 32 : 16;   // 128 bytes of a row
  static constexpr int VW = 16 / sizeof(V);            // elements per 16 B
  static constexpr int PAD = VW;                       // row padding
  static constexpr int LD = KC + PAD;                  // LDS row stride
  static constexpr int RV = KC / VW;                   // 16-byte vectors per row chunk (8)
};

// FUSE (with DIV): the divided modes stay in LDS and the same block applies
// the inverse operator A2 of this axis at once, so the last forward and the
// first inverse contraction of a sweep share one pass over memory.
template <typename V, bool XFAST, bool DIV, bool FUSE, int MT, int NT>
__global__ void __launch_bounds__(kBlock)
k_axis_lds(const V* __restrict__ X, V* __restrict__ Y, const V* __restrict__ A,
           const V* __restrict__ A2, int K, int inner, int64_t ncols, FdmDiv dv,
           const int* stop) {
  if (stop && *stop) return;
  typedef LdsGemm<V> L;
  typedef typename Mfma<V>::acc_t acc_t;
  constexpr int NC = 16 * NT;
  constexpr int RV = L::RV;
  typedef __attribute__((ext_vector_type(L::VW))) V vec_t;
  constexpr int LDY = 256 + L::VW;                      // stride of the fused modes
  __shared__ __attribute__((aligned(16))) V As[256 * L::LD];
  __shared__ __attribute__((aligned(16))) V Xs[NC * L::LD];
  __shared__ __attribute__((aligned(16))) V Ys[FUSE ? NC * LDY : 1];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int q = lane >> 4, r = lane & 15;
  const int ntr = K >> 4;
  const int64_t n0 = (int64_t)blockIdx.x * NC;
  // strided axis: the block's lines are consecutive inner indices of one
  // outer index
  const int64_t o0 = XFAST ? 0 : n0 / inner;
  const int64_t i0 = XFAST ? 0 : n0 - o0 * inner;
  const V* xbase = XFAST ? X : X + o0 * (int64_t)K * inner + i0;
  // per-thread global chunk loads: operator rows (K * RV vectors, a whole
  // number K / 32 per thread since K % 32 == 0) and lines (NC * RV vectors)
  constexpr int AV = 256 * RV / kBlock;                 // at most 8 per thread
  constexpr int XV = (NC * RV + kBlock - 1) / kBlock;
  const int av = K * RV / kBlock;                       // wave-uniform
  vec_t ra[AV], rx[XV];
  auto gload = [&](const V* Aop, int kc, bool with_x) {
#pragma unroll
    for (int u = 0; u < AV; ++u) {
      if (u < av) {
        const int e = t + u * kBlock;
        const int m = e / RV, f = e - m * RV;
        ra[u] = *reinterpret_cast<const vec_t*>(Aop + (int64_t)m * K + kc + f * L::VW);
      }
    }
    if (!with_x) return;
#pragma unroll
    for (int u = 0; u < XV; ++u) {
      const int e = t + u * kBlock;
      if ((NC * RV) % kBlock == 0 || e < NC * RV) {
        if (XFAST) {
          const int col = e / RV, f = e - col * RV;
          int64_t n = n0 + col;
          if (n >= ncols) n = ncols - 1;
          rx[u] = *reinterpret_cast<const vec_t*>(X + n * (int64_t)K + kc + f * L::VW);
        } else {
          constexpr int CV = NC / L::VW;                  // vectors per index row
          const int k = e / CV, c = e - k * CV;
          rx[u] = *reinterpret_cast<const vec_t*>(xbase + (int64_t)(kc + k) * inner + c * L::VW);
        }
      }
    }
  };
  auto sstore = [&](bool with_x) {
#pragma unroll
    for (int u = 0; u < AV; ++u) {
      if (u < av) {
        const int e = t + u * kBlock;
        const int m = e / RV, f = e - m * RV;
        *reinterpret_cast<vec_t*>(As + m * L::LD + f * L::VW) = ra[u];
      }
    }
    if (!with_x) return;
#pragma unroll
    for (int u = 0; u < XV; ++u) {
      const int e = t + u * kBlock;
      if ((NC * RV) % kBlock == 0 || e < NC * RV) {
        if (XFAST) {
          const int col = e / RV, f = e - col * RV;
          *reinterpret_cast<vec_t*>(Xs + col * L::LD + f * L::VW) = rx[u];
        } else {
          constexpr int CV = NC / L::VW;
          const int k = e / CV, c = e - k * CV;
#pragma unroll
          for (int j = 0; j < L::VW; ++j) Xs[(c * L::VW + j) * L::LD + k] = rx[u][j];
        }
      }
    }
  };
  acc_t acc[MT][NT];
  // one contraction over K: B operand from the staged lines (phase 1) or
  // from the modes kept in LDS (phase 2 of FUSE)
  auto gemm = [&](const V* Aop, bool from_ys) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) acc[mt][tt] = acc_t{0, 0, 0, 0};
    gload(Aop, 0, !from_ys);
    for (int kc = 0; kc < K; kc += L::KC) {
      __syncthreads();                 // previous chunk fully consumed
      sstore(!from_ys);
      __syncthreads();
      if (kc + L::KC < K) gload(Aop, kc + L::KC, !from_ys);
#pragma unroll
      for (int g = 0; g < L::KC / 16; ++g) {
        const int kq = 16 * g + 4 * q;   // this lane group's quad in the chunk
        Quad<V> xa[NT];
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            xa[tt].v[e] = from_ys ? Ys[(16 * tt + r) * LDY + kc + kq + e]
                                  : Xs[(16 * tt + r) * L::LD + kq + e];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int tile = w + 4 * mt;
          if (tile >= ntr) continue;     // wave-uniform
          Quad<V> aa;
#pragma unroll
          for (int e = 0; e < 4; ++e) aa.v[e] = As[(16 * tile + r) * L::LD + kq + e];
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int tt = 0; tt < NT; ++tt)
              acc[mt][tt] = Mfma<V>::op(aa.v[s], xa[tt].v[s], acc[mt][tt]);
        }
      }
    }
  };
  gemm(A, false);
  // division by the eigenvalue sum (last forward axis)
  double lrest[NT];
  if (DIV) {
    // eigenvalue sum of the faster axes' modes of each line (decoded from i)
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const int64_t n = n0 + 16 * tt + r;
      int64_t rem = XFAST ? 0 : (n % inner);
      double ls = 0.0;
      int allz = 1;
      for (int b = 0; b < dv.axis; ++b) {
        const int mb = (int)(rem % dv.n[b]);
        rem /= dv.n[b];
        ls += dv.lam[b][mb];
        allz &= (mb == 0);
      }
      lrest[tt] = allz ? -1.0 : ls;      // -1 marks the lines of the zero mode
    }
  }
  auto divide = [&](int tt, int m, V val) -> V {
    const bool zero = (lrest[tt] < 0.0) && m == 0;
    const double ls = (lrest[tt] < 0.0 ? 0.0 : lrest[tt]) + dv.lam[dv.axis][m];
    return zero ? V(0) : (V)((double)val / ls);
  };
  if constexpr (FUSE) {
    // divided modes into LDS (every row < K of every line), then the inverse
    // operator of the same axis; the barriers at the top of each chunk of
    // the second contraction order these writes before their reads
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int tile = w + 4 * mt;
      if (tile >= ntr) continue;
#pragma unroll
      for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * tile + Mfma<V>::row(lane, v);
          Ys[(16 * tt + r) * LDY + m] = divide(tt, m, acc[mt][tt][v]);
        }
    }
    gemm(A2, true);
  }
  constexpr bool DIVOUT = DIV && !FUSE;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int tile = w + 4 * mt;
    if (tile >= ntr) continue;
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const int64_t n = n0 + 16 * tt + r;
      if (n >= ncols) continue;
      int64_t base;
      if (XFAST) {
        base = n * (int64_t)K;
      } else {
        const int64_t o = n / inner, i = n - o * inner;
        base = o * (int64_t)K * inner + i;
      }
      if constexpr (XFAST && !DIVOUT && sizeof(V) == 4) {
        const acc_t& c = acc[mt][tt];
        typedef __attribute__((ext_vector_type(4))) float f4_t;
        __builtin_nontemporal_store(f4_t{c[0], c[1], c[2], c[3]},
                                    reinterpret_cast<f4_t*>(Y + base + 16 * tile + 4 * q));
        continue;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * tile + Mfma<V>::row(lane, v);
        V val = acc[mt][tt][v];
        if (DIVOUT) val = divide(tt, m, val);
        // non-temporal: see the note on k_fft_axis' stores
        if (XFAST)
          __builtin_nontemporal_store(val, Y + base + m);
        else
          __builtin_nontemporal_store(val, Y + base + (int64_t)m * inner);
      }
    }
  }
}

// Strided axis, float, K = 16 k' <= 128 (no division): the operator stays
// in registers.  Each wave owns row tiles w, w + 4 (MT of them) of the
// K x K operator and loads its rows once from L2 (lane (r, q) holds
// A[16 tile + r][16 g + 4 q + s] for every group g and s < 4, 16-byte loads);
// the block's lines (NT tiles of 16, one outer index) are fetched from HBM
// in one go, transposed into LDS line-major, and contracted with the same
// quad order as k_axis_lds (lane group q takes k = 16 g + 4 q + s in the
// s-th of four consecutive MFMAs).  One HBM latency per block instead of one
// per contraction chunk, and no operator traffic through LDS.
template <int K, int NT>
__global__ void __launch_bounds__(kBlock)
k_axis_reg(const float* __restrict__ X, float* __restrict__ Y, const float* __restrict__ A,
           int inner, int64_t ncols, const int* stop) {
  if (stop && *stop) return;
  static_assert(K % 16 == 0 && K <= 128, "operator rows must fit the registers");
  constexpr int NC = 16 * NT;                    // lines per block
  constexpr int NTR = K / 16;                    // row tiles of the operator
  constexpr int MT = (NTR + 3) / 4;              // row tiles per wave
  constexpr int G = K / 16;                      // contraction groups
  constexpr int LDK = K + 4;                     // LDS line stride (floats)
  constexpr int CV = NC / 4;                     // float4 per index row of the tile
  constexpr int XV = (K * CV + kBlock - 1) / kBlock;
  typedef __attribute__((ext_vector_type(4))) float f4_t;
  typedef typename Mfma<float>::acc_t acc_t;
  __shared__ __attribute__((aligned(16))) float Xs[NC * LDK];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int q = lane >> 4, r = lane & 15;
  const int64_t n0 = (int64_t)blockIdx.x * NC;
  const int64_t o0 = n0 / inner;
  const int64_t i0 = n0 - o0 * inner;
  const float* xb = X + o0 * (int64_t)K * inner + i0;
  // the block's lines: index row k holds NC consecutive floats
  f4_t rx[XV];
#pragma unroll
  for (int u = 0; u < XV; ++u) {
    const int e = t + u * kBlock;
    if ((K * CV) % kBlock == 0 || e < K * CV) {
      const int k = e / CV, c = e - k * CV;
      rx[u] = *reinterpret_cast<const f4_t*>(xb + (int64_t)k * inner + 4 * c);
    }
  }
  // this wave's operator rows
  f4_t ra[MT][G];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int tile = w + 4 * mt;
#pragma unroll
    for (int g = 0; g < G; ++g)
      ra[mt][g] = tile < NTR ? *reinterpret_cast<const f4_t*>(A + (16 * tile + r) * K + 16 * g + 4 * q)
                             : f4_t{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int u = 0; u < XV; ++u) {
    const int e = t + u * kBlock;
    if ((K * CV) % kBlock == 0 || e < K * CV) {
      const int k = e / CV, c = e - k * CV;
#pragma unroll
      for (int j = 0; j < 4; ++j) Xs[(4 * c + j) * LDK + k] = rx[u][j];
    }
  }
  __syncthreads();
  acc_t acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) acc[mt][tt] = acc_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int g = 0; g < G; ++g) {
    f4_t xa[NT];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
      xa[tt] = *reinterpret_cast<const f4_t*>(Xs + (16 * tt + r) * LDK + 16 * g + 4 * q);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      if (w + 4 * mt >= NTR) continue;           // wave-uniform
#pragma unroll
      for (int sidx = 0; sidx < 4; ++sidx)
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
          acc[mt][tt] = Mfma<float>::op(ra[mt][g][sidx], xa[tt][sidx], acc[mt][tt]);
    }
  }
  float* yb = Y + o0 * (int64_t)K * inner + i0;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int tile = w + 4 * mt;
    if (tile >= NTR) continue;
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = 16 * tile + Mfma<float>::row(lane, v);
        __builtin_nontemporal_store(acc[mt][tt][v], yb + (int64_t)m * inner + 16 * tt + r);
      }
  }
}

// Mirror-symmetric bounded axis (float, N = 2H): every eigenvector of a
// 1D operator that commutes with the reflection j -> N - 1 - j is even or
// odd, so the N x N contraction splits into two H x H ones.  Forward:
// even modes from S_j = x_j + x_{N-1-j}, odd modes from D_j = x_j -
// x_{N-1-j} (j < H), written as [even modes | odd modes]; inverse: E = Ie
// c_even, O = Io c_odd and x_j = E_j + O_j, x_{N-1-j} = E_j - O_j.  Half
// the matrix-core work of the dense form; same staging as k_axis_reg (each
// wave holds even and odd row tiles w, w + 4, ... of its operators).
template <int H, bool FWD>
__global__ void __launch_bounds__(kBlock)
k_axis_sym(const float* __restrict__ X, float* __restrict__ Y, const float* __restrict__ Ae,
           const float* __restrict__ Ao, int inner, int64_t ncols, const int* stop) {
  if (stop && *stop) return;
  static_assert(H % 16 == 0 && H <= 128, "half operator rows must fit the registers");
  constexpr int N = 2 * H;
  constexpr int NT = 2, NC = 32;                 // lines per tile
  constexpr int TH = H / 16;                     // row tiles per half
  constexpr int MT = (TH + 3) / 4;               // per wave and half
  constexpr int G = H / 16;                      // contraction groups
  constexpr int LDK = H + 4;
  constexpr int CV = NC / 4;                     // float4 per index row
  constexpr int XP = (H * CV + kBlock - 1) / kBlock;
  typedef __attribute__((ext_vector_type(4))) float f4_t;
  typedef typename Mfma<float>::acc_t acc_t;
  // even and odd operands (line-major), later the tile's output rows
  constexpr int LDY = NC + 4;                    // output row stride (floats)
  constexpr int SMN = (2 * NC * LDK > N * LDY) ? 2 * NC * LDK : N * LDY;
  __shared__ __attribute__((aligned(16))) float SM[SMN];
  float* S0 = SM;
  float* S1 = SM + NC * LDK;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int q = lane >> 4, r = lane & 15;
  const int64_t ntiles = ncols / NC;
  // index rows k and N-1-k (forward) or k and H+k (inverse) of a tile's lines
  f4_t ra[XP], rb[XP];
  auto load_tile = [&](int64_t tile_id) {
    const int64_t n0 = tile_id * NC;
    const int64_t o0 = n0 / inner;
    const float* xb = X + o0 * (int64_t)N * inner + (n0 - o0 * inner);
#pragma unroll
    for (int u = 0; u < XP; ++u) {
      const int e = t + u * kBlock;
      if ((H * CV) % kBlock == 0 || e < H * CV) {
        const int k = e / CV, c = e - k * CV;
        const int k2 = FWD ? N - 1 - k : H + k;
        ra[u] = *reinterpret_cast<const f4_t*>(xb + (int64_t)k * inner + 4 * c);
        rb[u] = *reinterpret_cast<const f4_t*>(xb + (int64_t)k2 * inner + 4 * c);
      }
    }
  };
  int64_t tile_id = blockIdx.x;
  if (tile_id >= ntiles) return;
  load_tile(tile_id);
  f4_t ae[MT][G], ao[MT][G];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int tile = w + 4 * mt;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int off = (16 * tile + r) * H + 16 * g + 4 * q;
      ae[mt][g] = tile < TH ? *reinterpret_cast<const f4_t*>(Ae + off) : f4_t{0.f, 0.f, 0.f, 0.f};
      ao[mt][g] = tile < TH ? *reinterpret_cast<const f4_t*>(Ao + off) : f4_t{0.f, 0.f, 0.f, 0.f};
    }
  }
  // persistent loop over tiles: the next tile's lines are in flight while
  // this one is contracted and stored
  for (; tile_id < ntiles; tile_id += gridDim.x) {
#pragma unroll
    for (int u = 0; u < XP; ++u) {
      const int e = t + u * kBlock;
      if ((H * CV) % kBlock == 0 || e < H * CV) {
        const int k = e / CV, c = e - k * CV;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          S0[(4 * c + j) * LDK + k] = FWD ? ra[u][j] + rb[u][j] : ra[u][j];
          S1[(4 * c + j) * LDK + k] = FWD ? ra[u][j] - rb[u][j] : rb[u][j];
        }
      }
    }
    __syncthreads();
    if (tile_id + gridDim.x < ntiles) load_tile(tile_id + gridDim.x);
    acc_t ce[MT][NT], co[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        ce[mt][tt] = acc_t{0.f, 0.f, 0.f, 0.f};
        co[mt][tt] = acc_t{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      f4_t xe[NT], xo[NT];
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        xe[tt] = *reinterpret_cast<const f4_t*>(S0 + (16 * tt + r) * LDK + 16 * g + 4 * q);
        xo[tt] = *reinterpret_cast<const f4_t*>(S1 + (16 * tt + r) * LDK + 16 * g + 4 * q);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        if (w + 4 * mt >= TH) continue;           // wave-uniform
#pragma unroll
        for (int sidx = 0; sidx < 4; ++sidx)
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) {
            ce[mt][tt] = Mfma<float>::op(ae[mt][g][sidx], xe[tt][sidx], ce[mt][tt]);
            co[mt][tt] = Mfma<float>::op(ao[mt][g][sidx], xo[tt][sidx], co[mt][tt]);
          }
      }
    }
    // output rows through LDS, so each row of the tile (NC lines, 128
    // bytes) leaves as whole 16-byte vectors
    __syncthreads();                             // operands fully consumed
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int tile = w + 4 * mt;
      if (tile >= TH) continue;
#pragma unroll
      for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * tile + Mfma<float>::row(lane, v);
          const float a = ce[mt][tt][v], b = co[mt][tt][v];
          const int row0 = m, row1 = FWD ? H + m : N - 1 - m;
          SM[row0 * LDY + 16 * tt + r] = FWD ? a : a + b;
          SM[row1 * LDY + 16 * tt + r] = FWD ? b : a - b;
        }
    }
    __syncthreads();
    const int64_t n0 = tile_id * NC;
    const int64_t o0 = n0 / inner;
    float* yb = Y + o0 * (int64_t)N * inner + (n0 - o0 * inner);
    constexpr int OV = N * CV;                   // float4 of the tile's output
#pragma unroll
    for (int u = 0; u < (OV + kBlock - 1) / kBlock; ++u) {
      const int e = t + u * kBlock;
      if (OV % kBlock == 0 || e < OV) {
        const int row = e / CV, c = e - row * CV;
        __builtin_nontemporal_store(*reinterpret_cast<const f4_t*>(SM + row * LDY + 4 * c),
                                    reinterpret_cast<f4_t*>(yb + (int64_t)row * inner + 4 * c));
      }
    }
    __syncthreads();                             // output staged out before the next operands
  }
}

// Half sizes with a k_axis_sym kernel.
#define FVIB_SYM_SIZES(X) X(16) X(32) X(48) X(64) X(96) X(128)

bool fdm_sym_size_supported(int n) {
  const int h = n / 2;
  if (n % 2 != 0) return false;
#define FVIB_SYM_IS(HH) if (h == HH) return true;
  FVIB_SYM_SIZES(FVIB_SYM_IS)
#undef FVIB_SYM_IS
  return false;
}

// Operator sizes with a k_axis_reg kernel.
#define FVIB_REG_SIZES(X) X(32) X(64) X(96) X(128)

// p = pin + d (refinement correction, double accumulator; pin == p in
// place).  A skipped sweep still carries pin over into p.
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_add_correction(int64_t n, double* p, const double* pin, const V* __restrict__ d,
                 const int* stop) {
  const bool skip = stop && *stop;
  if (skip && pin == p) return;
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * kBlock)
    p[c] = skip ? pin[c] : pin[c] + (double)d[c];
}

// p -= sum(p) / n with the sum measured by the last residual sweep
__global__ void __launch_bounds__(kBlock)
k_gauge(int64_t n, double* __restrict__ p, const SolverScalars* sc, double inv_n) {
  const double s = sc->sumx * inv_n;
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * kBlock)
    p[c] -= s;
}

// ------------------------------------------------------------- launchers
// Lines per block of k_axis_lds (in units of 16).  A strided axis takes 2
// (its lines are transposed into LDS; wider blocks measured slower on
// gfx950), else 1, and needs blocks that stay inside one outer index.  The
// contiguous axis takes the count whose blocks fill the CUs most evenly by
// a simple model (a block costs its tiles plus a fixed start-up of about
// 1.5 tiles; blocks run in rounds of one per CU).  0: no count fits.
static int lds_line_tiles(int64_t ncols, int inner) {
  constexpr int kCUs = 256;
  if (inner != 1) return inner % 32 == 0 ? 2 : (inner % 16 == 0 ? 1 : 0);
  int best = 0;
  double best_cost = 1e300;
  for (int nt = 1; nt <= 6; ++nt) {
    const int nc = 16 * nt;
    if (inner != 1 && inner % nc != 0) continue;
    const int64_t blocks = (ncols + nc - 1) / nc;
    const int64_t rounds = (blocks + kCUs - 1) / kCUs;
    const double cost = (double)rounds * (nt + 1.5);
    if (cost < best_cost - 1e-9) {
      best_cost = cost;
      best = nt;
    }
  }
  return best;
}

template <typename V>
bool fdm_fuses_last_axis(const FdmPlan<V>& F) {
  const int a = F.dim - 1;
  if (fft_usable(F, a)) return true;
  const int K = F.n[a];
  int inner = 1;
  for (int b = 0; b < a; ++b) inner *= F.n[b];
  int64_t outer = 1;
  for (int b = a + 1; b < 3; ++b) outer *= F.n[b];
  const int nt = (K % 32 == 0 && K <= 256) ? lds_line_tiles(outer * inner, inner) : 0;
  return nt > 0 && inner != 1 && nt <= 2;
}

template <typename V>
int launch_fdm_axis(const FdmPlan<V>& F, int a, bool fwd, const V* in, V* out, const int* stop,
                    hipStream_t s, bool* fused, double* acc, bool* accd, const double* accin) {
  if (fused) *fused = false;
  if (accd) *accd = false;
  if (fft_usable(F, a)) {
    const bool last = fwd && a == F.dim - 1;
    if (!fwd && acc && accd && a == 0) {
      *accd = true;
      return launch_fft_axis<V>(F, a, 1, in, out, stop, s, acc, accin ? accin : acc);
    }
    if (!last) return launch_fft_axis<V>(F, a, fwd ? 0 : 1, in, out, stop, s);
    if (fused) {
      *fused = true;
      return launch_fft_axis<V>(F, a, 2, in, out, stop, s);
    }
    // a division without the fused inverse falls through to the contraction
  }
  const int K = F.n[a];
  int inner = 1;
  for (int b = 0; b < a; ++b) inner *= F.n[b];
  int64_t outer = 1;
  for (int b = a + 1; b < 3; ++b) outer *= F.n[b];
  const int64_t ncols = outer * inner;
  const V* Am = fwd ? F.phiT[a] : F.phi[a];
  const bool div = fwd && a == F.dim - 1;
  if constexpr (sizeof(V) == 4) {
    // mirror-symmetric strided float axis without division: two half-size
    // contractions
    if (F.sym[a].on && !div && inner != 1 && inner % 32 == 0) {
      const int H = K / 2;
      bool done = false;
      // persistent blocks, two tiles of 32 lines each on average
      const dim3 g((unsigned)((ncols / 32 + 1) / 2));
      const float* A0 = fwd ? F.sym[a].fe : F.sym[a].ie;
      const float* A1 = fwd ? F.sym[a].fo : F.sym[a].io;
#define FVIB_SYM(HH)                                                                            \
      if (!done && H == HH) {                                                                   \
        done = true;                                                                            \
        if (fwd)                                                                                \
          launch_kernel((k_axis_sym<HH, true>), g, dim3(kBlock), 0, s, (const float*)in,        \
                        (float*)out, A0, A1, inner, ncols, stop);                               \
        else                                                                                    \
          launch_kernel((k_axis_sym<HH, false>), g, dim3(kBlock), 0, s, (const float*)in,       \
                        (float*)out, A0, A1, inner, ncols, stop);                               \
      }
      FVIB_SYM_SIZES(FVIB_SYM)
#undef FVIB_SYM
      if (done) {
        FVIB_HIP(hipGetLastError());
        return FVIB_OK;
      }
      return FVIB_EINVAL;      // the plan marks only axes with a kernel
    }
    // strided float axis without division: operator in registers
    if (!div && inner != 1 && inner % 32 == 0) {
      bool done = false;
      const dim3 g((unsigned)(ncols / 32));
#define FVIB_REG(KK)                                                                            \
      if (!done && K == KK) {                                                                   \
        done = true;                                                                            \
        launch_kernel((k_axis_reg<KK, 2>), g, dim3(kBlock), 0, s, (const float*)in,             \
                      (float*)out, (const float*)Am, inner, ncols, stop);                       \
      }
      FVIB_REG_SIZES(FVIB_REG)
#undef FVIB_REG
      if (done) {
        FVIB_HIP(hipGetLastError());
        return FVIB_OK;
      }
    }
  }
  const int nt = (K % 32 == 0 && K <= 256) ? lds_line_tiles(ncols, inner) : 0;
  if (nt > 0 && div && fused && inner != 1 && nt <= 2) {
    // last forward axis, division and first inverse axis in one launch
    const dim3 g((unsigned)((ncols + 16 * nt - 1) / (16 * nt)));
    const int mt = (K / 16 + 3) / 4;
#define FVIB_AF(MT, NT)                                                                         \
    launch_kernel((k_axis_lds<V, false, true, true, MT, NT>), g, dim3(kBlock), 0, s, in,   \
                       out, Am, F.phi[a], K, inner, ncols, F.div, stop)
#define FVIB_AFN(MT)                                                                            \
    if (nt == 1) FVIB_AF(MT, 1); else FVIB_AF(MT, 2);
    switch (mt) {
      case 1: FVIB_AFN(1) break;
      case 2: FVIB_AFN(2) break;
      case 3: FVIB_AFN(3) break;
      default: FVIB_AFN(4) break;
    }
#undef FVIB_AFN
#undef FVIB_AF
    FVIB_HIP(hipGetLastError());
    *fused = true;
    return FVIB_OK;
  }
  if (nt > 0) {
    const dim3 g((unsigned)((ncols + 16 * nt - 1) / (16 * nt)));
    const int mt = (K / 16 + 3) / 4;
#define FVIB_AL(XF, DV, MT, NT)                                                                 \
    launch_kernel((k_axis_lds<V, XF, DV, false, MT, NT>), g, dim3(kBlock), 0, s, in, out,  \
                       Am, Am, K, inner, ncols, F.div, stop)
#define FVIB_ALN(XF, DV, MT)                                                                    \
    switch (nt) {                                                                               \
      case 1: FVIB_AL(XF, DV, MT, 1); break;                                                    \
      case 2: FVIB_AL(XF, DV, MT, 2); break;                                                    \
      case 3: FVIB_AL(XF, DV, MT, 3); break;                                                    \
      case 4: FVIB_AL(XF, DV, MT, 4); break;                                                    \
      case 5: FVIB_AL(XF, DV, MT, 5); break;                                                    \
      default: FVIB_AL(XF, DV, MT, 6); break;                                                   \
    }
#define FVIB_ALM(XF, DV)                                                                        \
    switch (mt) {                                                                               \
      case 1: FVIB_ALN(XF, DV, 1) break;                                                        \
      case 2: FVIB_ALN(XF, DV, 2) break;                                                        \
      case 3: FVIB_ALN(XF, DV, 3) break;                                                        \
      default: FVIB_ALN(XF, DV, 4) break;                                                       \
    }
    if (inner == 1) {
      if (div) { FVIB_ALM(true, true) } else { FVIB_ALM(true, false) }
    } else {
      if (div) { FVIB_ALM(false, true) } else { FVIB_ALM(false, false) }
    }
#undef FVIB_ALM
#undef FVIB_ALN
#undef FVIB_AL
    FVIB_HIP(hipGetLastError());
    return FVIB_OK;
  }
  if (K % 4 == 0 && K <= 256) {
    constexpr int NT = 2;
    const dim3 g((unsigned)((ncols + 16 * NT - 1) / (16 * NT)));
    const int mt = (K + 63) / 64;
    const bool tail = K % (sizeof(V) == 4 ? 32 : 16) != 0;
#define FVIB_AX(XF, DV, MT)                                                                     \
    if (tail)                                                                                   \
      launch_kernel((k_axis_mfma<V, XF, DV, true, MT, NT>), g, dim3(kBlock), 0, s, in, out, \
                         Am, K, inner, ncols, F.div, stop);                                     \
    else                                                                                        \
      launch_kernel((k_axis_mfma<V, XF, DV, false, MT, NT>), g, dim3(kBlock), 0, s, in,    \
                         out, Am, K, inner, ncols, F.div, stop)
#define FVIB_AXM(XF, DV)                                                                        \
    switch (mt) {                                                                               \
      case 1: FVIB_AX(XF, DV, 1); break;                                                        \
      case 2: FVIB_AX(XF, DV, 2); break;                                                        \
      case 3: FVIB_AX(XF, DV, 3); break;                                                        \
      default: FVIB_AX(XF, DV, 4); break;                                                       \
    }
    if (inner == 1) {
      if (div) { FVIB_AXM(true, true) } else { FVIB_AXM(true, false) }
    } else {
      if (div) { FVIB_AXM(false, true) } else { FVIB_AXM(false, false) }
    }
#undef FVIB_AXM
#undef FVIB_AX
    FVIB_HIP(hipGetLastError());
    return FVIB_OK;
  }
  dim3 grid((K + BM - 1) / BM, (unsigned)((ncols + BN - 1) / BN));
  if (inner == 1) {
    if (div)
      launch_kernel((k_axis_gemm<V, true, true>), grid, dim3(kBlock), 0, s, in, out, Am, K, inner, ncols, F.div, stop);
    else
      launch_kernel((k_axis_gemm<V, true, false>), grid, dim3(kBlock), 0, s, in, out, Am, K, inner, ncols, F.div, stop);
  } else {
    if (div)
      launch_kernel((k_axis_gemm<V, false, true>), grid, dim3(kBlock), 0, s, in, out, Am, K, inner, ncols, F.div, stop);
    else
      launch_kernel((k_axis_gemm<V, false, false>), grid, dim3(kBlock), 0, s, in, out, Am, K, inner, ncols, F.div, stop);
  }
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename V>
int launch_add_correction(int64_t n, double* p, const double* pin, const V* d, const int* stop,
                          hipStream_t s) {
  int nb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 8 * kMaxRedBlocks);
  launch_kernel((k_add_correction<V>), dim3(nb), dim3(kBlock), 0, s, n, p, pin, d, stop);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

int launch_gauge(int64_t n, double* p, const SolverScalars* sc, hipStream_t s) {
  int nb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 8 * kMaxRedBlocks);
  launch_kernel(k_gauge, dim3(nb), dim3(kBlock), 0, s, n, p, sc, 1.0 / (double)n);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template bool fdm_fuses_last_axis<float>(const FdmPlan<float>&);
template bool fdm_fuses_last_axis<double>(const FdmPlan<double>&);
template int launch_fdm_axis<float>(const FdmPlan<float>&, int, bool, const float*, float*,
                                    const int*, hipStream_t, bool*, double*, bool*,
                                    const double*);
template int launch_fdm_axis<double>(const FdmPlan<double>&, int, bool, const double*, double*,
                                     const int*, hipStream_t, bool*, double*, bool*,
                                     const double*);
template int launch_add_correction<float>(int64_t, double*, const double*, const float*,
                                          const int*, hipStream_t);
template int launch_add_correction<double>(int64_t, double*, const double*, const double*,
                                           const int*, hipStream_t);

// ============================================================ host setup
// Symmetric eigen-decomposition by cyclic Jacobi rotations (stretched axes).
static void jacobi_eigen(int n, std::vector<double>& a, std::vector<double>& lam,
                         std::vector<double>& vec) {
  vec.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) vec[(size_t)i * n + i] = 1.0;
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += A(i, i) * A(i, i);
      for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
    }
    if (off <= 1e-32 * diag) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A(p, q);
        if (fabs(apq) < 1e-300) continue;
        const double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(tt * tt + 1.0), sn = tt * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - sn * akq;
          A(k, q) = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - sn * aqk;
          A(q, k) = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = vec[(size_t)k * n + p], vkq = vec[(size_t)k * n + q];
          vec[(size_t)k * n + p] = c * vkp - sn * vkq;
          vec[(size_t)k * n + q] = sn * vkp + c * vkq;
        }
      }
    }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = A(i, i);
}

// Generalised eigenpairs of axis a: phi (n x n, column m = mode m, row-major
// phi[j * n + m]) with phi^T W phi = I, and lam (ascending, lam[0] = 0 for
// the constant mode).
void axis_eigen(const std::vector<double>& f, bool periodic, std::vector<double>& phi,
                std::vector<double>& lam) {
  const int N = (int)f.size() - 1;
  std::vector<double> dx(N), xc(N);
  for (int i = 0; i < N; ++i) {
    dx[i] = f[i + 1] - f[i];
    xc[i] = 0.5 * (f[i] + f[i + 1]);
  }
  const double h = (f[N] - f[0]) / N;
  bool uniform = true;
  for (int i = 0; i < N; ++i)
    if (fabs(dx[i] - h) > 1e-12 * h) uniform = false;
  phi.assign((size_t)N * N, 0.0);
  lam.assign(N, 0.0);
  const double pi = 3.14159265358979323846;
  if (periodic) {
    // real Fourier basis (uniform periodic axes)
    const double s = 1.0 / sqrt(h);
    int col = 0;
    for (int j = 0; j < N; ++j) phi[(size_t)j * N + col] = s / sqrt((double)N);
    lam[col++] = 0.0;
    for (int m = 1; 2 * m < N; ++m) {
      const double l = 4.0 / (h * h) * pow(sin(pi * m / N), 2);
      for (int j = 0; j < N; ++j) {
        phi[(size_t)j * N + col] = s * sqrt(2.0 / N) * cos(2.0 * pi * m * j / N);
        phi[(size_t)j * N + col + 1] = s * sqrt(2.0 / N) * sin(2.0 * pi * m * j / N);
      }
      lam[col] = l;
      lam[col + 1] = l;
      col += 2;
    }
    if (N % 2 == 0) {
      for (int j = 0; j < N; ++j) phi[(size_t)j * N + col] = s / sqrt((double)N) * ((j % 2) ? -1.0 : 1.0);
      lam[col++] = 4.0 / (h * h);
    }
    return;
  }
  if (uniform) {
    // cosine basis of the Neumann operator (uniform bounded axes)
    const double s = 1.0 / sqrt(h);
    for (int m = 0; m < N; ++m) {
      const double nm = (m == 0) ? sqrt(1.0 / N) : sqrt(2.0 / N);
      for (int j = 0; j < N; ++j) phi[(size_t)j * N + m] = s * nm * cos(pi * m * (j + 0.5) / N);
      lam[m] = 4.0 / (h * h) * pow(sin(pi * m / (2.0 * N)), 2);
    }
    return;
  }
  // stretched bounded axis: C = W^-1/2 T W^-1/2, then phi = W^-1/2 psi
  std::vector<double> C((size_t)N * N, 0.0);
  for (int q = 1; q < N; ++q) {
    const double coef = 1.0 / (xc[q] - xc[q - 1]);
    const int i = q, j = q - 1;
    C[(size_t)i * N + i] += coef;
    C[(size_t)j * N + j] += coef;
    C[(size_t)i * N + j] -= coef;
    C[(size_t)j * N + i] -= coef;
  }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) C[(size_t)i * N + j] /= sqrt(dx[i] * dx[j]);
  std::vector<double> l, v;
  jacobi_eigen(N, C, l, v);
  std::vector<int> ord(N);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return l[x] < l[y]; });
  for (int m = 0; m < N; ++m) {
    const int src = ord[m];
    // sign convention: first nonzero entry positive
    double sg = v[(size_t)0 * N + src] < 0 ? -1.0 : 1.0;
    for (int j = 0; j < N; ++j) phi[(size_t)j * N + m] = sg * v[(size_t)j * N + src] / sqrt(dx[j]);
    lam[m] = (m == 0) ? 0.0 : l[src];
  }
}

// Mirror-symmetric bounded axis (faces symmetric about the middle, N even):
// the Neumann operator T commutes with the reflection, so its generalised
// eigenproblem T phi = lam W phi splits into an even and an odd half of size
// H = N / 2 on the cells j < H: T restricted to them, with the coupling
// across the middle folded in by x_H = +x_{H-1} (even) or -x_{H-1} (odd).
// Solving the halves directly gives an exactly even / odd eigenbasis even
// where the full problem has (numerically) degenerate pairs of wall modes.
// ue, uo: H x H, column s = mode s, entries j < H, scaled so that the full
// mirrored vector has unit W-norm; le, lo ascending (le[0] = 0).
void axis_eigen_sym(const std::vector<double>& f, std::vector<double>& ue, std::vector<double>& le,
                    std::vector<double>& uo, std::vector<double>& lo) {
  const int N = (int)f.size() - 1;
  const int H = N / 2;
  std::vector<double> dx(N), xc(N);
  for (int i = 0; i < N; ++i) {
    dx[i] = f[i + 1] - f[i];
    xc[i] = 0.5 * (f[i] + f[i + 1]);
  }
  for (int par = 0; par < 2; ++par) {
    std::vector<double> C((size_t)H * H, 0.0);
    for (int q = 1; q < H; ++q) {
      const double coef = 1.0 / (xc[q] - xc[q - 1]);
      const int i = q, j = q - 1;
      C[(size_t)i * H + i] += coef;
      C[(size_t)j * H + j] += coef;
      C[(size_t)i * H + j] -= coef;
      C[(size_t)j * H + i] -= coef;
    }
    // coupling of cells H-1 and H: diagonal coef, partner value +-x_{H-1}
    const double cm = 1.0 / (xc[H] - xc[H - 1]);
    C[(size_t)(H - 1) * H + (H - 1)] += par == 0 ? 0.0 : 2.0 * cm;
    for (int i = 0; i < H; ++i)
      for (int j = 0; j < H; ++j) C[(size_t)i * H + j] /= sqrt(dx[i] * dx[j]);
    std::vector<double> l, v;
    jacobi_eigen(H, C, l, v);
    std::vector<int> ord(H);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int x, int y) { return l[x] < l[y]; });
    std::vector<double>& u = par == 0 ? ue : uo;
    std::vector<double>& lam = par == 0 ? le : lo;
    u.assign((size_t)H * H, 0.0);
    lam.assign(H, 0.0);
    for (int m = 0; m < H; ++m) {
      const int src = ord[m];
      const double sg = v[(size_t)0 * H + src] < 0 ? -1.0 : 1.0;
      for (int j = 0; j < H; ++j)
        u[(size_t)j * H + m] = sg * v[(size_t)j * H + src] / sqrt(dx[j]) / sqrt(2.0);
      lam[m] = (par == 0 && m == 0) ? 0.0 : l[src];
    }
  }
}

}  // namespace fvib
