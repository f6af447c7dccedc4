// Real FFT along a uniform periodic axis, in place of the dense contraction
// with that axis' real Fourier eigenbasis (constant, cos / sin pairs of
// increasing wavenumber, alternating sign for even N; the basis of the
// periodic second-difference operator, Sec. 2.4's pressure operator on a
// uniform periodic axis).
//
// Two real lines are packed into one complex line z = x1 + i x2 and
// transformed by a Stockham (self-sorting) FFT of radices 2, 3, 4, 5 in LDS;
// the two real spectra follow from Z_m and Z_{N-m}.  The inverse builds the
// packed Hermitian spectrum Y1 + i Y2 and uses IDFT(Z) = conj(FFT(conj Z)).
// With the division by the eigenvalue sum (last axis), the forward
// transform, the division and the inverse run in one launch.  The work is
// memory bound: every line crosses HBM once per launch.
#include <math.h>

#include <vector>

#include "fvib_kernels.h"

namespace fvib {

template <typename V>
struct FftCfg {
  static constexpr int LPB = sizeof(V) == 4 ? 32 : 16;   // lines per block
  static constexpr int P = LPB / 2;                      // complex lines
};

// R-point DFT (sign -) on (re, im) arrays, R = 2, 3, 4, 5.
template <int R, typename V>
__device__ __forceinline__ void dft_small(V (&xr)[R], V (&xi)[R]) {
  if constexpr (R == 2) {
    const V ar = xr[0], ai = xi[0];
    xr[0] = ar + xr[1]; xi[0] = ai + xi[1];
    xr[1] = ar - xr[1]; xi[1] = ai - xi[1];
  } else if constexpr (R == 4) {
    const V s0r = xr[0] + xr[2], s0i = xi[0] + xi[2];
    const V d0r = xr[0] - xr[2], d0i = xi[0] - xi[2];
    const V s1r = xr[1] + xr[3], s1i = xi[1] + xi[3];
    const V d1r = xr[1] - xr[3], d1i = xi[1] - xi[3];
    xr[0] = s0r + s1r; xi[0] = s0i + s1i;
    xr[2] = s0r - s1r; xi[2] = s0i - s1i;
    // X1 = d0 - i d1, X3 = d0 + i d1
    xr[1] = d0r + d1i; xi[1] = d0i - d1r;
    xr[3] = d0r - d1i; xi[3] = d0i + d1r;
  } else {
    // R = 3 or 5: direct sum with the R-th roots of unity exp(-2 pi i q / R)
    constexpr double c3[3] = {1.0, -0.5, -0.5};
    constexpr double s3[3] = {0.0, -0.86602540378443865, 0.86602540378443865};
    constexpr double c5[5] = {1.0, 0.30901699437494742, -0.80901699437494742,
                              -0.80901699437494742, 0.30901699437494742};
    constexpr double s5[5] = {0.0, -0.95105651629515357, -0.58778525229247313,
                              0.58778525229247313, 0.95105651629515357};
    V yr[R], yi[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      V sr = V(0), si = V(0);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int q = (r * k) % R;
        const V c = (V)(R == 3 ? c3[q % 3] : c5[q % 5]);
        const V sn = (V)(R == 3 ? s3[q % 3] : s5[q % 5]);
        sr += xr[r] * c - xi[r] * sn;
        si += xr[r] * sn + xi[r] * c;
      }
      yr[k] = sr;
      yi[k] = si;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      xr[k] = yr[k];
      xi[k] = yi[k];
    }
  }
}

// Radix plan (compile time, same rule as fft_plan): radix-4 stages, one
// radix-2 stage for an odd power of two, then radix-3 and radix-5 stages.
constexpr int fft_radix_at(int n, int st) {
  int m = n, k = 0;
  while (m % 4 == 0) { if (k == st) return 4; ++k; m /= 4; }
  if (m % 2 == 0) { if (k == st) return 2; ++k; m /= 2; }
  while (m % 3 == 0) { if (k == st) return 3; ++k; m /= 3; }
  while (m % 5 == 0) { if (k == st) return 5; ++k; m /= 5; }
  return 0;
}
constexpr int fft_nstages(int n) {
  int k = 0;
  while (fft_radix_at(n, k) != 0) ++k;
  return k;
}

template <typename V>
struct alignas(2 * sizeof(V)) Cx {
  V r, i;
};

// One Stockham stage of radix R over P complex lines of length N (current
// sub-transform length NS): src -> dst.
template <int R, int N, int NS, int P, typename V>
__device__ __forceinline__ void fft_stage(const Cx<V>* src, Cx<V>* dst, const Cx<V>* tw) {
  constexpr int NR = N / R;
  constexpr int TWS = N / (NS * R);
  for (int e = threadIdx.x; e < P * NR; e += kBlock) {
    const int p = e / NR, j = e - p * NR;
    const int k = j % NS;
    const Cx<V>* s0 = src + p * N;
    Cx<V>* d0 = dst + p * N;
    V xr[R], xi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const Cx<V> v = s0[j + r * NR];
      xr[r] = v.r;
      xi[r] = v.i;
    }
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const Cx<V> w = tw[(r * k * TWS) % N];
      const V vr = xr[r] * w.r - xi[r] * w.i;
      xi[r] = xr[r] * w.i + xi[r] * w.r;
      xr[r] = vr;
    }
    dft_small<R, V>(xr, xi);
    const int idx = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d0[idx + r * NS] = Cx<V>{xr[r], xi[r]};
  }
}

// Stockham FFT of P complex lines of length N in src (dst is scratch);
// returns the buffer that holds the result.
template <typename V, int N, int P, int ST = 0, int NS = 1>
__device__ __forceinline__ Cx<V>* fft_lines(Cx<V>* src, Cx<V>* dst, const Cx<V>* tw) {
  if constexpr (ST == fft_nstages(N)) {
    return src;
  } else {
    constexpr int R = fft_radix_at(N, ST);
    fft_stage<R, N, NS, P, V>(src, dst, tw);
    __syncthreads();
    return fft_lines<V, N, P, ST + 1, NS * R>(dst, src, tw);
  }
}

// Real coefficient c of line part (0: x1, 1: x2) from the packed spectrum Z
// (interleaved, length N) of its pair.
template <typename V>
__device__ __forceinline__ V spec_coeff(const V* Z, int N, int c, int part, double a, double b) {
  if (c == 0) return (V)(b * (double)Z[part]);
  if ((N & 1) == 0 && c == N - 1) return (V)(b * (double)Z[2 * (N / 2) + part]);
  const int m = (c + 1) / 2;
  const V zmr = Z[2 * m], zmi = Z[2 * m + 1];
  const V znr = Z[2 * (N - m)], zni = Z[2 * (N - m) + 1];
  V v;
  if (c & 1) {     // cosine coefficient: a Re X_m
    v = part == 0 ? (zmr + znr) : (zmi + zni);
  } else {         // sine coefficient: -a Im X_m
    v = part == 0 ? (zni - zmi) : (zmr - znr);
  }
  return (V)(0.5 * a * (double)v);
}

// conj of the packed Hermitian spectrum Y1 + i Y2 at index m, from the real
// coefficients y1, y2 (each N long, stride 1).
template <typename V>
__device__ __forceinline__ void herm_pack_conj(const V* y1, const V* y2, int N, int m, double a,
                                               double b, V* zr, V* zi) {
  double y1r, y1i, y2r, y2i;
  if (m == 0) {
    y1r = b * y1[0]; y1i = 0.0; y2r = b * y2[0]; y2i = 0.0;
  } else if ((N & 1) == 0 && m == N / 2) {
    y1r = b * y1[N - 1]; y1i = 0.0; y2r = b * y2[N - 1]; y2i = 0.0;
  } else {
    const int mm = (2 * m < N) ? m : N - m;
    const double sg = (2 * m < N) ? -1.0 : 1.0;    // Y_{N-m} = conj(Y_m)
    y1r = 0.5 * a * y1[2 * mm - 1]; y1i = sg * 0.5 * a * y1[2 * mm];
    y2r = 0.5 * a * y2[2 * mm - 1]; y2i = sg * 0.5 * a * y2[2 * mm];
  }
  // Z = Y1 + i Y2, stored conjugated for the forward transform
  *zr = (V)(y1r - y2i);
  *zi = (V)(-(y1i + y2r));
}

// MODE 0: forward (lines -> basis coefficients), 1: inverse, 2: forward,
// division by the eigenvalue sum, inverse.  N is the axis length.
template <typename V, int N, bool XFAST, int MODE>
__global__ void __launch_bounds__(kBlock)
k_fft_axis(const V* __restrict__ X, V* __restrict__ Y, int inner, int64_t ncols, FftAxis ax,
           const V* __restrict__ twg, FdmDiv dv, const int* stop) {
  if (stop && *stop) return;
  typedef FftCfg<V> C;
  constexpr int LPB = C::LPB, P = C::P;
  __shared__ Cx<V> bufA[P * N];
  __shared__ Cx<V> bufB[P * N];
  __shared__ Cx<V> tw[N];
  __shared__ double lam_s[MODE == 2 ? N : 1];
  __shared__ double lrest_s[MODE == 2 ? LPB : 1];
  V* rowsB = reinterpret_cast<V*>(bufB);        // LPB real rows of N
  const int t = threadIdx.x;
  const int64_t n0 = (int64_t)blockIdx.x * LPB;
  const int64_t o0 = XFAST ? 0 : n0 / inner;
  const int64_t i0 = XFAST ? 0 : n0 - o0 * inner;
  const int64_t base = XFAST ? n0 * (int64_t)N : o0 * (int64_t)N * inner + i0;
  const int nl = (int)((ncols - n0) < LPB ? (ncols - n0) : LPB);   // lines of this block
  for (int e = t; e < N; e += kBlock) tw[e] = Cx<V>{twg[2 * e], twg[2 * e + 1]};
  if (MODE == 2) {
    for (int e = t; e < N; e += kBlock) lam_s[e] = dv.lam[dv.axis][e];
    if (t < LPB) {
      // eigenvalue sum of the faster axes' modes of line t (-1: zero mode)
      int64_t rem = (n0 + t) % inner;
      double ls = 0.0;
      int allz = 1;
      for (int q = 0; q < dv.axis; ++q) {
        const int mq = (int)(rem % dv.n[q]);
        rem /= dv.n[q];
        ls += dv.lam[q][mq];
        allz &= (mq == 0);
      }
      lrest_s[t] = allz ? -1.0 : ls;
    }
  }
  // element (line l, index k) of this block in global memory
  auto gidx = [&](int l, int k) -> int64_t {
    return XFAST ? base + (int64_t)l * N + k : base + (int64_t)k * inner + l;
  };
  auto split = [&](int e, int& l, int& k) {
    if (XFAST) { l = e / N; k = e - l * N; } else { k = e / LPB; l = e - k * LPB; }
  };
  // load: lines as packed complex pairs (MODE 0, 2) or as real rows (MODE 1)
  V* packA = reinterpret_cast<V*>(bufA);
  for (int e = t; e < LPB * N; e += kBlock) {
    int l, k;
    split(e, l, k);
    const V v = l < nl ? X[gidx(l, k)] : V(0);
    if (MODE == 1) rowsB[l * N + k] = v;
    else packA[2 * ((l >> 1) * N + k) + (l & 1)] = v;
  }
  __syncthreads();
  const double a = ax.a, b = ax.b;
  if (MODE != 1) {
    Cx<V>* res = fft_lines<V, N, P>(bufA, bufB, tw);
    // basis coefficients of every line as real rows in the other buffer
    V* rows = reinterpret_cast<V*>(res == bufA ? bufB : bufA);
    const V* Z = reinterpret_cast<const V*>(res);
    for (int e = t; e < LPB * N; e += kBlock) {
      const int l = e / N, c = e - l * N;
      V v = spec_coeff<V>(Z + 2 * (l >> 1) * N, N, c, l & 1, a, b);
      if (MODE == 2) {
        const double lr = lrest_s[l];
        v = (lr < 0.0 && c == 0) ? V(0) : (V)((double)v / ((lr < 0.0 ? 0.0 : lr) + lam_s[c]));
      }
      rows[l * N + c] = v;
    }
    __syncthreads();
    if (MODE == 0) {
      for (int e = t; e < LPB * N; e += kBlock) {
        int l, k;
        split(e, l, k);
        if (l < nl) Y[gidx(l, k)] = rows[l * N + k];
      }
      return;
    }
    if (rows != rowsB) {
      for (int e = t; e < LPB * N; e += kBlock) rowsB[e] = rows[e];
      __syncthreads();
    }
  }
  // inverse: real rows in bufB -> conj of the packed spectra in bufA
  for (int e = t; e < P * N; e += kBlock) {
    const int p = e / N, m = e - p * N;
    V zr, zi;
    herm_pack_conj<V>(rowsB + (2 * p) * N, rowsB + (2 * p + 1) * N, N, m, a, b, &zr, &zi);
    bufA[p * N + m] = Cx<V>{zr, zi};
  }
  __syncthreads();
  Cx<V>* res = fft_lines<V, N, P>(bufA, bufB, tw);
  // x1 = Re conj(FFT) = Re FFT, x2 = Im conj(FFT) = -Im FFT
  for (int e = t; e < LPB * N; e += kBlock) {
    int l, k;
    split(e, l, k);
    const Cx<V> z = res[(l >> 1) * N + k];
    if (l < nl) Y[gidx(l, k)] = (l & 1) ? -z.i : z.r;
  }
}

// Axis lengths with an FFT kernel (every one factors into 2, 3, 5).
#define FVIB_FFT_SIZES(X) X(24) X(32) X(48) X(64) X(96) X(128) X(160) X(192) X(256)

static bool fft_size_supported(int n) {
#define FVIB_FFT_IS(NN) if (n == NN) return true;
  FVIB_FFT_SIZES(FVIB_FFT_IS)
#undef FVIB_FFT_IS
  return false;
}

FftAxis fft_plan(int n, double h) {
  FftAxis ax;
  ax.on = 0;
  ax.nst = 0;
  for (int i = 0; i < kFftMaxStages; ++i) ax.radix[i] = 0;
  ax.a = sqrt(2.0 / n) / sqrt(h);
  ax.b = 1.0 / sqrt(n * h);
  if (n < 2 || n > kFftMaxN) return ax;
  int m = n;
  for (int r : {4, 2, 3, 5}) {
    while (m % r == 0 && !(r == 2 && m % 4 == 0)) {
      if (ax.nst == kFftMaxStages) return ax;
      ax.radix[ax.nst++] = r;
      m /= r;
    }
  }
  if (m != 1) {
    ax.nst = 0;
    return ax;
  }
  ax.on = 1;
  return ax;
}

template <typename V>
int launch_fft_axis(const FdmPlan<V>& F, int a, int mode, const V* in, V* out, const int* stop,
                    hipStream_t s) {
  const int N = F.n[a];
  int inner = 1;
  for (int q = 0; q < a; ++q) inner *= F.n[q];
  int64_t outer = 1;
  for (int q = a + 1; q < 3; ++q) outer *= F.n[q];
  const int64_t ncols = outer * inner;
  constexpr int LPB = FftCfg<V>::LPB;
  const dim3 g((unsigned)((ncols + LPB - 1) / LPB));
  bool done = false;
#define FVIB_FFT(NN, XF, M)                                                                     \
  hipLaunchKernelGGL((k_fft_axis<V, NN, XF, M>), g, dim3(kBlock), 0, s, in, out, inner, ncols,  \
                     F.fft[a], F.tw[a], F.div, stop)
#define FVIB_FFT_N(NN)                                                                          \
  if (!done && N == NN) {                                                                       \
    done = true;                                                                                \
    if (inner == 1) {                                                                           \
      if (mode == 0) FVIB_FFT(NN, true, 0); else FVIB_FFT(NN, true, 1);                         \
    } else {                                                                                    \
      if (mode == 0) FVIB_FFT(NN, false, 0);                                                    \
      else if (mode == 1) FVIB_FFT(NN, false, 1);                                               \
      else FVIB_FFT(NN, false, 2);                                                              \
    }                                                                                           \
  }
  FVIB_FFT_SIZES(FVIB_FFT_N)
#undef FVIB_FFT_N
#undef FVIB_FFT
  if (!done || (inner == 1 && mode == 2)) return FVIB_EINVAL;
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

// A strided axis needs the lines of a block inside one outer index.
template <typename V>
bool fft_usable(const FdmPlan<V>& F, int a) {
  if (!F.fft[a].on || !fft_size_supported(F.n[a])) return false;
  int inner = 1;
  for (int q = 0; q < a; ++q) inner *= F.n[q];
  return inner == 1 || inner % FftCfg<V>::LPB == 0;
}

template int launch_fft_axis<float>(const FdmPlan<float>&, int, int, const float*, float*,
                                    const int*, hipStream_t);
template int launch_fft_axis<double>(const FdmPlan<double>&, int, int, const double*, double*,
                                     const int*, hipStream_t);
template bool fft_usable<float>(const FdmPlan<float>&, int);
template bool fft_usable<double>(const FdmPlan<double>&, int);

}  // namespace fvib
