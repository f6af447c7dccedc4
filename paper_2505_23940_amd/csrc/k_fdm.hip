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
            int inner, int64_t ncols, FdmDiv dv) {
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
        if (XFAST)
          Y[base + m] = val;
        else
          Y[base + (int64_t)m * inner] = val;
      }
    }
  }
}

// p += d (refinement correction, double accumulator)
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_add_correction(int64_t n, double* __restrict__ p, const V* __restrict__ d) {
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * kBlock)
    p[c] += (double)d[c];
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
template <typename V>
int launch_fdm_axis(const FdmPlan<V>& F, int a, bool fwd, const V* in, V* out, hipStream_t s) {
  const int K = F.n[a];
  int inner = 1;
  for (int b = 0; b < a; ++b) inner *= F.n[b];
  int64_t outer = 1;
  for (int b = a + 1; b < 3; ++b) outer *= F.n[b];
  const int64_t ncols = outer * inner;
  const V* Am = fwd ? F.phiT[a] : F.phi[a];
  dim3 grid((K + BM - 1) / BM, (unsigned)((ncols + BN - 1) / BN));
  const bool div = fwd && a == F.dim - 1;
  if (inner == 1) {
    if (div)
      hipLaunchKernelGGL((k_axis_gemm<V, true, true>), grid, dim3(kBlock), 0, s, in, out, Am, K, inner, ncols, F.div);
    else
      hipLaunchKernelGGL((k_axis_gemm<V, true, false>), grid, dim3(kBlock), 0, s, in, out, Am, K, inner, ncols, F.div);
  } else {
    if (div)
      hipLaunchKernelGGL((k_axis_gemm<V, false, true>), grid, dim3(kBlock), 0, s, in, out, Am, K, inner, ncols, F.div);
    else
      hipLaunchKernelGGL((k_axis_gemm<V, false, false>), grid, dim3(kBlock), 0, s, in, out, Am, K, inner, ncols, F.div);
  }
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename V>
int launch_add_correction(int64_t n, double* p, const V* d, hipStream_t s) {
  int nb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 8 * kMaxRedBlocks);
  hipLaunchKernelGGL((k_add_correction<V>), dim3(nb), dim3(kBlock), 0, s, n, p, d);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

int launch_gauge(int64_t n, double* p, const SolverScalars* sc, hipStream_t s) {
  int nb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 8 * kMaxRedBlocks);
  hipLaunchKernelGGL(k_gauge, dim3(nb), dim3(kBlock), 0, s, n, p, sc, 1.0 / (double)n);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template int launch_fdm_axis<float>(const FdmPlan<float>&, int, bool, const float*, float*, hipStream_t);
template int launch_fdm_axis<double>(const FdmPlan<double>&, int, bool, const double*, double*, hipStream_t);
template int launch_add_correction<float>(int64_t, double*, const float*, hipStream_t);
template int launch_add_correction<double>(int64_t, double*, const double*, hipStream_t);

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

}  // namespace fvib
