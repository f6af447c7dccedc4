// Real FFT along a uniform periodic axis, in place of the dense contraction
// with that axis' real Fourier eigenbasis (constant, cos / sin pairs of
// increasing wavenumber, alternating sign for even N; the basis of the
// periodic second-difference operator, Sec. 2.5's pressure operator on a
// uniform periodic axis).
//
// Two real lines are packed into one complex line z = x1 + i x2 and
// transformed by a Stockham (self-sorting) FFT of radices 2, 3, 4, 5 in LDS;
// the two real spectra follow from Z_m and Z_{N-m}.  The inverse builds the
// packed Hermitian spectrum Y1 + i Y2 and uses IDFT(Z) = conj(FFT(conj Z)).
// With the division by the eigenvalue sum (last axis), the forward
// transform, the division and the inverse run in one launch.  The work is
// memory bound: every line crosses HBM once per launch.  Outputs are
// stored non-temporally: a pass writes about as much as the L2s hold, and
// lines left dirty there would be written back at the kernel's end, idling
// the next launch for several microseconds.
#include <math.h>

#include <vector>

#include "fvib_kernels.h"

namespace fvib {

// Lines per block: 16 on the contiguous axis (two buffers of 8 complex
// lines, about 25 KB of LDS for 192 floats, so six blocks fit a CU); the
// strided axis keeps 32 float lines, whose interleaved rows then span 128
// bytes.  Long axes halve the lines until the block's LDS (two line
// buffers, twiddles, eigenvalues) fits 72 KB.
constexpr int fft_lds_bytes(int lpb, int n, int vs) {
  return 2 * (lpb / 2) * n * 2 * vs + n * 2 * vs + n * 8;
}
constexpr int fft_lines_fit(int lpb, int n, int vs) {
  return (lpb > 2 && fft_lds_bytes(lpb, n, vs) > 72 * 1024) ? fft_lines_fit(lpb / 2, n, vs) : lpb;
}
template <typename V, bool XFAST, int N>
struct FftCfg {
  static constexpr int LPB = fft_lines_fit((sizeof(V) == 4 && !XFAST) ? 32 : 16, N, (int)sizeof(V));
  static constexpr int P = LPB / 2;                      // complex lines
};

// Position of entry j of a line in the even-odd reordered sequence of the
// cosine transform: v_m = x_{2m}, v_{N-1-m} = x_{2m+1}.
template <int N>
__device__ __forceinline__ int dct_pos(int j) {
  return (j & 1) ? N - 1 - (j >> 1) : (j >> 1);
}

// sin and cos of 2 pi j / R (compile time): reduction to the nearest
// quarter turn, then Taylor series on |r| <= pi / 4.
constexpr void cx_sincos(int j, int R, double& s, double& c) {
  constexpr double kPi = 3.14159265358979323846;
  const int q8 = 4 * j;                    // angle in quarter turns = 4 j / R
  int quad = (2 * q8 + R) / (2 * R);       // nearest quarter turn
  const double r = 2.0 * kPi * ((double)(q8 - quad * R) / (4.0 * R));
  double sr = 0.0, cr = 0.0, term = r;
  for (int n = 1; n < 30; n += 2) {        // sin r = r - r^3/3! + ...
    sr += term;
    term *= -r * r / ((n + 1) * (n + 2));
  }
  term = 1.0;
  for (int n = 0; n < 30; n += 2) {        // cos r = 1 - r^2/2! + ...
    cr += term;
    term *= -r * r / ((n + 1) * (n + 2));
  }
  quad &= 3;
  s = quad == 0 ? sr : quad == 1 ? cr : quad == 2 ? -sr : -cr;
  c = quad == 0 ? cr : quad == 1 ? -sr : quad == 2 ? -cr : sr;
}

// Roots exp(-2 pi i j / R), j < R.
template <int R>
struct Roots {
  double c[R], s[R];
  constexpr Roots() : c(), s() {
    for (int j = 0; j < R; ++j) {
      double sn = 0.0, cs = 0.0;
      cx_sincos(j, R, sn, cs);
      c[j] = cs;
      s[j] = -sn;
    }
  }
};

// Split of a composite radix R = A B (A the first factor of 4, 2, 3, 5).
constexpr int dft_split(int R) {
  if (R % 4 == 0 && R != 4) return 4;
  if (R % 2 == 0 && R != 2 && R != 4) return 2;
  if (R % 3 == 0 && R != 3) return 3;
  if (R % 5 == 0 && R != 5) return 5;
  return R;
}

// R-point DFT (sign -) in registers on (re, im) arrays.  R = 2, 3, 4, 5
// directly; a composite R = A B by one Cooley-Tukey split: A-point DFTs
// over n1 of x[B n1 + n2], twiddles exp(-2 pi i n2 k1 / R), B-point DFTs
// over n2 into X[k1 + A k2].
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
  } else if constexpr (R == 3 || R == 5) {
    constexpr Roots<R> W{};
    V yr[R], yi[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      V sr = xr[0], si = xi[0];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const V c = (V)W.c[(r * k) % R], sn = (V)W.s[(r * k) % R];
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
  } else {
    constexpr int A = dft_split(R), B = R / A;
    static_assert(A > 1 && B > 1 && A * B == R, "radix without a kernel");
    constexpr Roots<R> W{};
    V yr[B][A], yi[B][A];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      V tr[A], ti[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) {
        tr[n1] = xr[B * n1 + n2];
        ti[n1] = xi[B * n1 + n2];
      }
      dft_small<A, V>(tr, ti);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        const int e = (n2 * k1) % R;
        if (e == 0) {
          yr[n2][k1] = tr[k1];
          yi[n2][k1] = ti[k1];
        } else {
          const V c = (V)W.c[e], sn = (V)W.s[e];
          yr[n2][k1] = tr[k1] * c - ti[k1] * sn;
          yi[n2][k1] = tr[k1] * sn + ti[k1] * c;
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      V tr[B], ti[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) {
        tr[n2] = yr[n2][k1];
        ti[n2] = yi[n2][k1];
      }
      dft_small<B, V>(tr, ti);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) {
        xr[k1 + A * k2] = tr[k2];
        xi[k1 + A * k2] = ti[k2];
      }
    }
  }
}

// Radix plan (compile time): each stage takes the largest radix of
// 16, 12, 10, 8, 6, 5, 4, 3, 2 that divides what is left of n, so the
// common lengths need two passes through LDS.
constexpr int fft_radix_at(int n, int st) {
  constexpr int kR[9] = {16, 12, 10, 8, 6, 5, 4, 3, 2};
  int m = n;
  for (int k = 0; m > 1; ++k) {
    int r = 0;
    for (int q = 0; q < 9 && r == 0; ++q)
      if (m % kR[q] == 0) r = kR[q];
    if (r == 0) return 0;
    if (k == st) return r;
    m /= r;
  }
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

// LDS index of complex entry k of packed line pair p: line-contiguous for a
// contiguous axis, line-interleaved (index-major) for a strided axis, so that
// in both cases a block's global lines land in LDS as one dense image.
template <int N, int P, bool IL>
__device__ __forceinline__ int zidx(int p, int k) {
  return IL ? k * P + p : p * N + k;
}

// One Stockham stage of radix R over P complex lines of length N (current
// sub-transform length NS): src -> dst.  Consecutive threads take
// consecutive entries of the layout.
template <int R, int N, int NS, int P, bool IL, typename V>
__device__ __forceinline__ void fft_stage(const Cx<V>* src, Cx<V>* dst, const Cx<V>* tw) {
  constexpr int NR = N / R;
  constexpr int TWS = N / (NS * R);
  constexpr int NE = P * NR;
#pragma unroll
  for (int e0 = 0; e0 < NE; e0 += kBlock) {
    const int e = e0 + (int)threadIdx.x;
    if (NE % kBlock == 0 || e < NE) {
      int p, j;
      if (IL) { p = e % P; j = e / P; } else { p = e / NR; j = e - p * NR; }
      const int k = j % NS;
      V xr[R], xi[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const Cx<V> v = src[zidx<N, P, IL>(p, j + r * NR)];
        xr[r] = v.r;
        xi[r] = v.i;
      }
      // r k TWS <= (R - 1)(NS - 1) N / (NS R) < N: no wrap; the first
      // stage (NS = 1) has none
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const Cx<V> w = tw[r * k * TWS];
          const V vr = xr[r] * w.r - xi[r] * w.i;
          xi[r] = xr[r] * w.i + xi[r] * w.r;
          xr[r] = vr;
        }
      }
      dft_small<R, V>(xr, xi);
      const int idx = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[zidx<N, P, IL>(p, idx + r * NS)] = Cx<V>{xr[r], xi[r]};
    }
  }
}

// Stockham FFT of P complex lines of length N in src (dst is scratch);
// returns the buffer that holds the result.
template <typename V, int N, int P, bool IL, int ST = 0, int NS = 1>
__device__ __forceinline__ Cx<V>* fft_lines(Cx<V>* src, Cx<V>* dst, const Cx<V>* tw) {
  if constexpr (ST == fft_nstages(N)) {
    return src;
  } else {
    constexpr int R = fft_radix_at(N, ST);
    fft_stage<R, N, NS, P, IL, V>(src, dst, tw);
    __syncthreads();
    return fft_lines<V, N, P, IL, ST + 1, NS * R>(dst, src, tw);
  }
}

// Relations used below (a = sqrt(2 / N) / sqrt(h), b = 1 / sqrt(N h), the
// normalisation of the orthonormal real Fourier basis on a uniform axis of
// spacing h; Z = FFT(x1 + i x2) of a line pair; X1_m = (Z_m + conj Z_{N-m}) / 2,
// X2_m = (Z_m - conj Z_{N-m}) / (2 i)):
//   coefficient 0           b Re X_0
//   coefficient 2m - 1      a Re X_m          (cosine of wavenumber m)
//   coefficient 2m          -a Im X_m         (sine of wavenumber m)
//   coefficient N - 1       b Re X_{N/2}      (N even, alternating sign)
// and back: Y_0 = b y_0, Y_{N/2} = b y_{N-1}, Y_m = (a / 2)(y_{2m-1} - i y_{2m})
// for 0 < m < N / 2, Y_{N-m} = conj Y_m; x = IDFT(Y1 + i Y2) =
// conj FFT(conj(Y1 + i Y2)) splits into the two real lines.

// Uniform bounded axis (ax.dct): the basis is the cosine basis of the
// Neumann operator, phi_m(j) = s_m cos(pi m (j + 1/2) / N) with s_0 = b,
// s_m = a.  A line's coefficients come from one FFT of its even-odd
// reordered sequence v (Makhoul's cosine transform): with Z = FFT(v1 + i v2)
// of a line pair, V1_m = (Z_m + conj Z_{N-m}) / 2, V2_m = (Z_m - conj
// Z_{N-m}) / (2 i) and t_m = pi m / (2N),
//   X_m = cos t_m Re V_m + sin t_m Im V_m,  X_{N-m} = sin t_m Re V_m - cos t_m Im V_m,
// and coefficient m = s_m X_m.  Back: with Y_m = s_m y_m, the sequence
// v_n = sum_m Y_m cos(pi m (2n + 1/2) / N) (read back in the even-odd order)
// is the inverse FFT of the Hermitian H_0 = Y_0, H_m = (1/2) e^{i t_m}
// (Y_m - i Y_{N-m}), H_{N/2} = Y_{N/2} / sqrt 2, H_{N-m} = conj H_m; two
// lines pack into D = H1 + i H2.  The twiddles (cos t_m, sin t_m) for
// m <= N/2 come from the plan.

// MODE 0: forward (lines -> basis coefficients), 1: inverse, 2: forward,
// division by the eigenvalue sum, inverse.  N is the axis length.  ACC
// (contiguous axis, MODE 1): pacc = pin + result, in double, instead of
// the result in Y (the refinement correction of the last pass of a sweep;
// pin == pacc in place, else a skipped launch still copies pin).
template <typename V, int N, bool XFAST, int MODE, bool ACC>
__global__ void __launch_bounds__(kBlock)
k_fft_axis(const V* __restrict__ X, V* __restrict__ Y, int inner, int64_t ncols, FftAxis ax,
           const V* __restrict__ twg, const V* __restrict__ dtw, FdmDiv dv, const int* stop,
           double* pacc, const double* pin) {
  static_assert(!ACC || (XFAST && MODE == 1), "accumulation is for the contiguous inverse");
  if (stop && *stop) {
    if constexpr (ACC) {
      if (pin != pacc) {
        constexpr int L = FftCfg<V, XFAST, N>::LPB;
        const int64_t b0 = (int64_t)blockIdx.x * L * N;
        const int64_t left = ncols - (int64_t)blockIdx.x * L;
        const int64_t ne = (left < L ? left : L) * N;
        for (int64_t e = threadIdx.x; e < ne; e += kBlock) pacc[b0 + e] = pin[b0 + e];
      }
    }
    return;
  }
  constexpr bool IL = !XFAST;
  typedef FftCfg<V, XFAST, N> C;
  constexpr int LPB = C::LPB, P = C::P;
  constexpr int VW = 16 / (int)sizeof(V);            // 16-byte global vectors
  typedef __attribute__((ext_vector_type(VW))) V vec_t;
  __shared__ __attribute__((aligned(16))) Cx<V> bufA[P * N];
  __shared__ __attribute__((aligned(16))) Cx<V> bufB[P * N];
  __shared__ Cx<V> tw[N];
  __shared__ double lam_s[MODE == 2 ? N : 1];
  __shared__ double lrest_s[MODE == 2 ? LPB : 1];
  const int t = threadIdx.x;
  const int64_t n0 = (int64_t)blockIdx.x * LPB;
  const int64_t o0 = XFAST ? 0 : n0 / inner;
  const int64_t i0 = XFAST ? 0 : n0 - o0 * inner;
  const int64_t base = XFAST ? n0 * (int64_t)N : o0 * (int64_t)N * inner + i0;
  const int nl = (int)((ncols - n0) < LPB ? (ncols - n0) : LPB);   // lines of this block
  // Global vectors of the block.  Contiguous axis: slot (p, kv) holds
  // entries VW kv .. VW kv + VW - 1 of lines 2p and 2p + 1 (lines past the
  // end read as zero and are not written); strided axis (every block full):
  // slot e holds lines VW c .. VW c + VW - 1 at index k, e = k LPB / VW + c.
  constexpr int NV = XFAST ? P * N / VW : LPB * N / VW;
  constexpr int PT = (NV + kBlock - 1) / kBlock;
  constexpr int LV = XFAST ? 2 : 1;
  constexpr int KV = N / VW;
  auto gaddr = [&](int e, int h) -> int64_t {
    if (XFAST) {
      const int p = e / KV, kv = e - p * KV;
      return base + (int64_t)(2 * p + h) * N + kv * VW;
    }
    const int k = e / (LPB / VW), c = e - k * (LPB / VW);
    return base + (int64_t)k * inner + c * VW;
  };
  auto gvalid = [&](int e, int h) -> bool { return !XFAST || 2 * (e / KV) + h < nl; };
  vec_t rv[PT][LV];
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int e = t + u * kBlock;
#pragma unroll
    for (int h = 0; h < LV; ++h) {
      rv[u][h] = vec_t{};
      if ((NV % kBlock == 0 || e < NV) && gvalid(e, h))
        rv[u][h] = *reinterpret_cast<const vec_t*>(X + gaddr(e, h));
    }
  }
  // ACC: the accumulator entries of this thread's output slots, fetched
  // with the input
  typedef __attribute__((ext_vector_type(VW))) double dvec_t;
  dvec_t pv[ACC ? PT : 1][ACC ? LV : 1];
  if constexpr (ACC) {
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int e = t + u * kBlock;
#pragma unroll
      for (int h = 0; h < LV; ++h) {
        pv[u][h] = dvec_t{};
        if ((NV % kBlock == 0 || e < NV) && gvalid(e, h))
          pv[u][h] = *reinterpret_cast<const dvec_t*>(pin + gaddr(e, h));
      }
    }
  }
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
  V* fA = reinterpret_cast<V*>(bufA);
  V* fB = reinterpret_cast<V*>(bufB);
  // real row entry (l, c) in LDS, same layout rule as zidx
  auto ridx = [&](int l, int c) -> int { return IL ? c * LPB + l : l * N + c; };
  // LDS image of the block: real rows in bufB (MODE 1) or packed pairs in bufA
  // (for the cosine transform the pairs in the even-odd order)
  const bool dct = ax.dct != 0;
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int e = t + u * kBlock;
    if (NV % kBlock == 0 || e < NV) {
      if (IL) {
        if (MODE != 1 && dct) {
          const int k = e / (LPB / VW), c = e - k * (LPB / VW);
          *reinterpret_cast<vec_t*>(fA + (dct_pos<N>(k) * (LPB / VW) + c) * VW) = rv[u][0];
        } else {
          *reinterpret_cast<vec_t*>((MODE == 1 ? fB : fA) + e * VW) = rv[u][0];
        }
      } else {
        const int p = e / KV, kv = e - p * KV;
        if (MODE != 1 && dct) {
#pragma unroll
          for (int j = 0; j < VW; ++j) {
            V* d = fA + 2 * (p * N + dct_pos<N>(kv * VW + j));
            d[0] = rv[u][0][j];
            d[1] = rv[u][1][j];
          }
        } else if (MODE == 1) {
#pragma unroll
          for (int h = 0; h < 2; ++h)
            *reinterpret_cast<vec_t*>(fB + (2 * p + h) * N + kv * VW) = rv[u][h];
        } else {
          // interleave the pair: (x1_k, x2_k) for k = VW kv ...
          vec_t lo, hi;
#pragma unroll
          for (int j = 0; j < VW / 2; ++j) {
            lo[2 * j] = rv[u][0][j];
            lo[2 * j + 1] = rv[u][1][j];
            hi[2 * j] = rv[u][0][j + VW / 2];
            hi[2 * j + 1] = rv[u][1][j + VW / 2];
          }
          V* d = fA + 2 * (p * N + kv * VW);
          *reinterpret_cast<vec_t*>(d) = lo;
          *reinterpret_cast<vec_t*>(d + VW) = hi;
        }
      }
    }
  }
  __syncthreads();
  const V ha = (V)(0.5 * ax.a), hb = (V)ax.b;
  // work items (p, m), m = 0 .. N / 2: the wavenumber-m pair of lines
  // 2p, 2p + 1 (N is even for every supported length)
  constexpr int H = N / 2;
  constexpr int NI = P * (H + 1);
  auto item = [&](int e, int& p, int& m) {
    if (IL) { p = e % P; m = e / P; } else { p = e / (H + 1); m = e - p * (H + 1); }
  };
  Cx<V>* spec = bufA;              // conj packed spectrum for the inverse
  // cosine transform: coefficients m and N - m of the pair from Z_m, Z_{N-m}
  // (times 2: the halves are in ha), in the order (line 2p: m, N-m; line
  // 2p + 1: m, N-m)
  auto dct_coef = [&](const Cx<V>* Z, int p, int m, V* q) {
    const Cx<V> zm = Z[zidx<N, P, IL>(p, m)], zn = Z[zidx<N, P, IL>(p, N - m)];
    const V c = dtw[2 * m], sn = dtw[2 * m + 1];
    const V rv1 = zm.r + zn.r, iv1 = zm.i - zn.i, rv2 = zm.i + zn.i, iv2 = zn.r - zm.r;
    q[0] = ha * (c * rv1 + sn * iv1);
    q[1] = ha * (sn * rv1 - c * iv1);
    q[2] = ha * (c * rv2 + sn * iv2);
    q[3] = ha * (sn * rv2 - c * iv2);
  };
  const V hq = (V)(ax.a * 0.70710678118654752440);      // a cos(pi / 4)
  if (MODE == 0 && dct) {
    const Cx<V>* Z = fft_lines<V, N, P, IL>(bufA, bufB, tw);
    V* rows = reinterpret_cast<V*>(Z == bufA ? bufB : bufA);
    for (int e = t; e < NI; e += kBlock) {
      int p, m;
      item(e, p, m);
      if (m == 0 || m == H) {
        const Cx<V> z = Z[zidx<N, P, IL>(p, m)];
        const V sc = m == 0 ? hb : hq;
        rows[ridx(2 * p, m)] = sc * z.r;
        rows[ridx(2 * p + 1, m)] = sc * z.i;
      } else {
        V q[4];
        dct_coef(Z, p, m, q);
        rows[ridx(2 * p, m)] = q[0];
        rows[ridx(2 * p, N - m)] = q[1];
        rows[ridx(2 * p + 1, m)] = q[2];
        rows[ridx(2 * p + 1, N - m)] = q[3];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int e = t + u * kBlock;
      if (NV % kBlock == 0 || e < NV) {
#pragma unroll
        for (int h = 0; h < LV; ++h) {
          const int off = IL ? e * VW : (2 * (e / KV) + h) * N + (e % KV) * VW;
          if (gvalid(e, h))
            __builtin_nontemporal_store(*reinterpret_cast<const vec_t*>(rows + off),
                                        reinterpret_cast<vec_t*>(Y + gaddr(e, h)));
        }
      }
    }
    return;
  }
  if (MODE == 0) {
    const Cx<V>* Z = fft_lines<V, N, P, IL>(bufA, bufB, tw);
    V* rows = reinterpret_cast<V*>(Z == bufA ? bufB : bufA);
    for (int e = t; e < NI; e += kBlock) {
      int p, m;
      item(e, p, m);
      if (m == 0 || m == H) {
        const int c = m == 0 ? 0 : N - 1;
        const Cx<V> z = Z[zidx<N, P, IL>(p, m)];
        rows[ridx(2 * p, c)] = hb * z.r;
        rows[ridx(2 * p + 1, c)] = hb * z.i;
      } else {
        const Cx<V> zm = Z[zidx<N, P, IL>(p, m)], zn = Z[zidx<N, P, IL>(p, N - m)];
        rows[ridx(2 * p, 2 * m - 1)] = ha * (zm.r + zn.r);
        rows[ridx(2 * p + 1, 2 * m - 1)] = ha * (zm.i + zn.i);
        rows[ridx(2 * p, 2 * m)] = ha * (zn.i - zm.i);
        rows[ridx(2 * p + 1, 2 * m)] = ha * (zm.r - zn.r);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int e = t + u * kBlock;
      if (NV % kBlock == 0 || e < NV) {
#pragma unroll
        for (int h = 0; h < LV; ++h) {
          const int off = IL ? e * VW : (2 * (e / KV) + h) * N + (e % KV) * VW;
          if (gvalid(e, h))
            __builtin_nontemporal_store(*reinterpret_cast<const vec_t*>(rows + off),
                                        reinterpret_cast<vec_t*>(Y + gaddr(e, h)));
        }
      }
    }
    return;
  }
  // packed conj spectrum entries m and N - m of pair p from the basis
  // coefficients: (c1, s1) cosine and sine of wavenumber m of line 2p,
  // (c2, s2) of line 2p + 1
  auto put_pair = [&](int p, int m, V c1, V s1, V c2, V s2) {
    const V y1r = ha * c1, y2r = ha * c2, y1s = ha * s1, y2s = ha * s2;
    spec[zidx<N, P, IL>(p, m)] = Cx<V>{y1r + y2s, y1s - y2r};
    spec[zidx<N, P, IL>(p, N - m)] = Cx<V>{y1r - y2s, -(y1s + y2r)};
  };
  // cosine transform: packed conj spectrum entries m and N - m of pair p
  // from the coefficients (y1m, y1n) of line 2p and (y2m, y2n) of line
  // 2p + 1 at m and N - m (0 < m < N/2)
  auto dct_put = [&](int p, int m, V y1m, V y1n, V y2m, V y2n) {
    const V c = dtw[2 * m], sn = dtw[2 * m + 1];
    const V h1r = ha * (y1m * c + y1n * sn), h1i = ha * (y1m * sn - y1n * c);
    const V h2r = ha * (y2m * c + y2n * sn), h2i = ha * (y2m * sn - y2n * c);
    spec[zidx<N, P, IL>(p, m)] = Cx<V>{h1r - h2i, -(h1i + h2r)};
    spec[zidx<N, P, IL>(p, N - m)] = Cx<V>{h1r + h2i, h1i - h2r};
  };
  auto divd = [&](V v, int l, int c) -> V {
    const double lr = lrest_s[l];
    if (lr < 0.0 && c == 0) return V(0);
    return v / (V)((lr < 0.0 ? 0.0 : lr) + lam_s[c]);
  };
  if (MODE == 2 && dct) {
    const Cx<V>* Z = fft_lines<V, N, P, IL>(bufA, bufB, tw);
    spec = Z == bufA ? bufB : bufA;
    for (int e = t; e < NI; e += kBlock) {
      int p, m;
      item(e, p, m);
      if (m == 0 || m == H) {
        const Cx<V> z = Z[zidx<N, P, IL>(p, m)];
        const V sc = m == 0 ? hb : hq;
        const V y1 = divd(sc * z.r, 2 * p, m), y2 = divd(sc * z.i, 2 * p + 1, m);
        spec[zidx<N, P, IL>(p, m)] = Cx<V>{sc * y1, -(sc * y2)};
      } else {
        V q[4];
        dct_coef(Z, p, m, q);
        dct_put(p, m, divd(q[0], 2 * p, m), divd(q[1], 2 * p, N - m), divd(q[2], 2 * p + 1, m),
                divd(q[3], 2 * p + 1, N - m));
      }
    }
  } else if (MODE == 1 && dct) {
    for (int e = t; e < NI; e += kBlock) {
      int p, m;
      item(e, p, m);
      if (m == 0 || m == H) {
        const V sc = m == 0 ? hb : hq;
        spec[zidx<N, P, IL>(p, m)] = Cx<V>{sc * fB[ridx(2 * p, m)], -(sc * fB[ridx(2 * p + 1, m)])};
      } else {
        dct_put(p, m, fB[ridx(2 * p, m)], fB[ridx(2 * p, N - m)], fB[ridx(2 * p + 1, m)],
                fB[ridx(2 * p + 1, N - m)]);
      }
    }
  } else if (MODE == 2) {
    const Cx<V>* Z = fft_lines<V, N, P, IL>(bufA, bufB, tw);
    spec = Z == bufA ? bufB : bufA;
    // spectrum -> basis coefficients -> division -> packed conj spectrum
    for (int e = t; e < NI; e += kBlock) {
      int p, m;
      item(e, p, m);
      if (m == 0 || m == H) {
        const int c = m == 0 ? 0 : N - 1;
        const Cx<V> z = Z[zidx<N, P, IL>(p, m)];
        const V y1 = divd(hb * z.r, 2 * p, c), y2 = divd(hb * z.i, 2 * p + 1, c);
        spec[zidx<N, P, IL>(p, m)] = Cx<V>{hb * y1, -(hb * y2)};
      } else {
        const Cx<V> zm = Z[zidx<N, P, IL>(p, m)], zn = Z[zidx<N, P, IL>(p, N - m)];
        const int c1 = 2 * m - 1, c2 = 2 * m;
        put_pair(p, m, divd(ha * (zm.r + zn.r), 2 * p, c1), divd(ha * (zn.i - zm.i), 2 * p, c2),
                 divd(ha * (zm.i + zn.i), 2 * p + 1, c1), divd(ha * (zm.r - zn.r), 2 * p + 1, c2));
      }
    }
  } else {
    // MODE 1: real rows in bufB -> packed conj spectrum in bufA
    for (int e = t; e < NI; e += kBlock) {
      int p, m;
      item(e, p, m);
      if (m == 0 || m == H) {
        const int c = m == 0 ? 0 : N - 1;
        spec[zidx<N, P, IL>(p, m)] =
            Cx<V>{hb * fB[ridx(2 * p, c)], -(hb * fB[ridx(2 * p + 1, c)])};
      } else {
        put_pair(p, m, fB[ridx(2 * p, 2 * m - 1)], fB[ridx(2 * p, 2 * m)],
                 fB[ridx(2 * p + 1, 2 * m - 1)], fB[ridx(2 * p + 1, 2 * m)]);
      }
    }
  }
  __syncthreads();
  Cx<V>* res = fft_lines<V, N, P, IL>(spec, spec == bufA ? bufB : bufA, tw);
  // x1 = Re conj(FFT) = Re FFT, x2 = Im conj(FFT) = -Im FFT
  const V* fr = reinterpret_cast<const V*>(res);
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int e = t + u * kBlock;
    if (NV % kBlock == 0 || e < NV) {
      if (IL) {
        int off = e * VW;
        if (dct) {
          const int k = e / (LPB / VW), c = e - k * (LPB / VW);
          off = (dct_pos<N>(k) * (LPB / VW) + c) * VW;
        }
        vec_t v = *reinterpret_cast<const vec_t*>(fr + off);
#pragma unroll
        for (int j = 1; j < VW; j += 2) v[j] = -v[j];
        __builtin_nontemporal_store(v, reinterpret_cast<vec_t*>(Y + gaddr(e, 0)));
      } else {
        const int p = e / KV, kv = e - p * KV;
        vec_t x1, x2;
        if (dct) {
#pragma unroll
          for (int j = 0; j < VW; ++j) {
            const V* q = fr + 2 * (p * N + dct_pos<N>(kv * VW + j));
            x1[j] = q[0];
            x2[j] = -q[1];
          }
        } else {
          const V* s = fr + 2 * (p * N + kv * VW);
          const vec_t lo = *reinterpret_cast<const vec_t*>(s);
          const vec_t hi = *reinterpret_cast<const vec_t*>(s + VW);
#pragma unroll
          for (int j = 0; j < VW / 2; ++j) {
            x1[j] = lo[2 * j];
            x2[j] = -lo[2 * j + 1];
            x1[j + VW / 2] = hi[2 * j];
            x2[j + VW / 2] = -hi[2 * j + 1];
          }
        }
        if constexpr (ACC) {
          dvec_t q1 = pv[u][0], q2 = pv[u][LV - 1];
#pragma unroll
          for (int j = 0; j < VW; ++j) {
            q1[j] += (double)x1[j];
            q2[j] += (double)x2[j];
          }
          if (gvalid(e, 0)) *reinterpret_cast<dvec_t*>(pacc + gaddr(e, 0)) = q1;
          if (gvalid(e, 1)) *reinterpret_cast<dvec_t*>(pacc + gaddr(e, 1)) = q2;
        } else {
          if (gvalid(e, 0)) __builtin_nontemporal_store(x1, reinterpret_cast<vec_t*>(Y + gaddr(e, 0)));
          if (gvalid(e, 1)) __builtin_nontemporal_store(x2, reinterpret_cast<vec_t*>(Y + gaddr(e, 1)));
        }
      }
    }
  }
}

// Axis lengths with an FFT kernel (every one factors into 2, 3, 5).
#define FVIB_FFT_SIZES(X) X(24) X(32) X(48) X(64) X(96) X(128) X(160) X(192) X(256) X(384) X(512) \
  X(768) X(1024)

static bool fft_size_supported(int n) {
#define FVIB_FFT_IS(NN) if (n == NN) return true;
  FVIB_FFT_SIZES(FVIB_FFT_IS)
#undef FVIB_FFT_IS
  return false;
}

FftAxis fft_plan(int n, double h) {
  FftAxis ax;
  ax.a = sqrt(2.0 / n) / sqrt(h);
  ax.b = 1.0 / sqrt(n * h);
  ax.on = fft_size_supported(n) ? 1 : 0;
  ax.dct = 0;
  return ax;
}

template <typename V>
int launch_fft_axis(const FdmPlan<V>& F, int a, int mode, const V* in, V* out, const int* stop,
                    hipStream_t s, double* acc, const double* accin) {
  const int N = F.n[a];
  if (!accin) accin = acc;
  // the kernel moves 16-byte vectors (32-byte ones of the accumulator)
  if (((uintptr_t)in | (uintptr_t)out) % 16 != 0 || ((uintptr_t)acc | (uintptr_t)accin) % 32 != 0)
    return FVIB_EINVAL;
  int inner = 1;
  for (int q = 0; q < a; ++q) inner *= F.n[q];
  int64_t outer = 1;
  for (int q = a + 1; q < 3; ++q) outer *= F.n[q];
  const int64_t ncols = outer * inner;
  if (acc && !(inner == 1 && mode == 1)) return FVIB_EINVAL;
  if (inner == 1 && mode == 2) return FVIB_EINVAL;
  bool done = false;
#define FVIB_FFT(NN, XF, M, AC)                                                                 \
  launch_kernel((k_fft_axis<V, NN, XF, M, AC>),                                                 \
                dim3((unsigned)((ncols + FftCfg<V, XF, NN>::LPB - 1) / FftCfg<V, XF, NN>::LPB)),  \
                dim3(kBlock), 0, s, in, out, inner, ncols, F.fft[a], F.tw[a], F.dtw[a], F.div,  \
                stop, acc, accin)
#define FVIB_FFT_N(NN)                                                                          \
  if (!done && N == NN) {                                                                       \
    done = true;                                                                                \
    if (inner == 1) {                                                                           \
      if (mode == 0) FVIB_FFT(NN, true, 0, false);                                              \
      else if (acc) FVIB_FFT(NN, true, 1, true);                                                \
      else FVIB_FFT(NN, true, 1, false);                                                        \
    } else {                                                                                    \
      if (mode == 0) FVIB_FFT(NN, false, 0, false);                                             \
      else if (mode == 1) FVIB_FFT(NN, false, 1, false);                                        \
      else FVIB_FFT(NN, false, 2, false);                                                       \
    }                                                                                           \
  }
  FVIB_FFT_SIZES(FVIB_FFT_N)
#undef FVIB_FFT_N
#undef FVIB_FFT
  if (!done) return FVIB_EINVAL;
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

// A strided axis needs the lines of a block inside one outer index.
template <typename V>
bool fft_usable(const FdmPlan<V>& F, int a) {
  if (!F.fft[a].on || !fft_size_supported(F.n[a])) return false;
  int inner = 1;
  for (int q = 0; q < a; ++q) inner *= F.n[q];
  int lpb = 0;
#define FVIB_FFT_LPB(NN) if (F.n[a] == NN) lpb = FftCfg<V, false, NN>::LPB;
  FVIB_FFT_SIZES(FVIB_FFT_LPB)
#undef FVIB_FFT_LPB
  return inner == 1 || (lpb > 0 && inner % lpb == 0);
}

bool fft_size_ok(int n) { return fft_size_supported(n); }

template int launch_fft_axis<float>(const FdmPlan<float>&, int, int, const float*, float*,
                                    const int*, hipStream_t, double*, const double*);
template int launch_fft_axis<double>(const FdmPlan<double>&, int, int, const double*, double*,
                                     const int*, hipStream_t, double*, const double*);
template bool fft_usable<float>(const FdmPlan<float>&, int);
template bool fft_usable<double>(const FdmPlan<double>&, int);

}  // namespace fvib
