// Modified pressure Poisson equation (paper Eq. 9), its solution by
// conjugate gradients (the paper's pressure solver), iterative refinement
// with a float inner solve and a double residual, and the velocity
// correction (Eq. 10).
//
// The PPE is solved in its volume-integrated symmetric form
//   (A p)_c = sum_{interior faces f of c} (A_f / dc_f) (p_c - p_nb)
//   b_c     = -(rho / dt) sum_{faces f of c} (+-) A_f u~_f,
//   u~ = (1 - eps) u* + eps u_c,
// with homogeneous Neumann conditions on bounded axes; A is symmetric
// positive semi-definite with the constants as null space, so b has its
// mean removed and every iterate is kept at zero mean.
//
// Convergence is measured by what the correction leaves behind: for the
// residual r = b - A p the divergence of the corrected field is
// -(dt / rho) r_c / V_c, and the solve stops when its maximum over the
// cells falls below the requested tolerance.
#include <algorithm>

#include "fvib_internal.h"
#include "fvib_kernels.h"

namespace fvib {


// Neighbour cell of index ia along an axis of na cells: wrapped on a
// periodic axis, clamped on a bounded one (where the face between them is a
// boundary face whose coefficient kf is zero).  Every index is valid, so
// all loads of a stencil can be issued before any arithmetic.
__device__ __forceinline__ int nb_lo(int ia, int na, int per) {
  return ia > 0 ? ia - 1 : (per ? na - 1 : 0);
}
__device__ __forceinline__ int nb_hi(int ia, int na, int per) {
  return ia < na - 1 ? ia + 1 : (per ? 0 : na - 1);
}

template <typename V, int DIM, typename Get>
__device__ __forceinline__ V apply_A(const PGeo<V>& P, const Get& get, int i, int j, int k, V xc) {
  const int I[3] = {i, j, k};
  V lo[DIM], hi[DIM], d[DIM], klo[DIM], khi[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const int ia = I[a];
    int J[3] = {i, j, k};
    J[a] = nb_lo(ia, P.n[a], P.per[a]);
    lo[a] = get(J[0], J[1], J[2]);
    J[a] = nb_hi(ia, P.n[a], P.per[a]);
    hi[a] = get(J[0], J[1], J[2]);
    d[a] = P.dx[a][ia];
    klo[a] = P.kf[a][ia];
    khi[a] = P.kf[a][ia + 1];
  }
  V acc = V(0);
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    V area = V(1);
#pragma unroll
    for (int b = 0; b < DIM; ++b)
      if (b != a) area *= d[b];
    acc += area * klo[a] * (xc - lo[a]);
    acc += area * khi[a] * (xc - hi[a]);
  }
  return acc;
}

// 1 / cell volume
template <typename V>
__device__ __forceinline__ double inv_volume(const PGeo<V>& P, int i, int j, int k) {
  double v = (double)P.iv[0][i] * (double)P.iv[1][j];
  if (P.dim == 3) v *= (double)P.iv[2][k];
  return v;
}

#define FVIB_TILE_LOOP(tl)                                                      \
  for (int t_ = xcd_block(blockIdx.x, gridDim.x); t_ < (tl).ntiles; t_ += gridDim.x) { \
    const int i = (t_ % (tl).ntx) * kTileX + (threadIdx.x & (kTileX - 1));   \
    const int j = ((t_ / (tl).ntx) % (tl).nty) * kTileY + (threadIdx.x / kTileX); \
    const int k = t_ / ((tl).ntx * (tl).nty);                                 \
    if (i >= nx_ || j >= ny_) continue;                                       \
    const int64_t c_ = ((int64_t)k * ny_ + j) * nx_ + i;

#define FVIB_TILE_END }

// ------------------------------------------------ reduction epilogues
struct FinMeanB {           // mean of the PPE right-hand side
  double inv_ncell;
  __device__ bool skip(const SolverScalars*) const { return false; }
  __device__ void apply(const double* t, SolverScalars* sc) const { sc->meanb = t[0] * inv_ncell; }
};

template <int MODE>
struct FinResidual {        // start of a solve / refinement sweep
  double tol, inner_rtol, dt_over_rho;
  int first;                // first residual of the solve (never skipped)
  SolverScalars* mirror;    // nullable: device view of the host's pinned copy
  // nullable: a coherent pinned word the host polls for this check: one
  // 64-bit store (no fence) of the ticket with the check's outcome
  unsigned long long* tick;
  unsigned int ticket;
  __device__ void post(const SolverScalars* sc) const {
    unsigned long long w = (unsigned long long)__float_as_uint((float)sc->crit);
    w |= (unsigned long long)(sc->sweeps < 127 ? sc->sweeps : 127) << 32;
    w |= (unsigned long long)(sc->outer_done ? 1 : 0) << 39;
    w |= (unsigned long long)(ticket & 0xFFFFFFu) << 40;
    __hip_atomic_store(tick, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  // a sweep queued after the refinement finished is skipped, but still
  // answers its ticket (with the finished solve's outcome)
  __device__ bool skip(const SolverScalars* sc) const {
    const bool s = !first && sc->outer_done;
    if (s && tick && threadIdx.x == 0) post(sc);
    return s;
  }
  __device__ void apply(const double* t, SolverScalars* sc) const {
    sc->sweeps = first ? 0 : sc->sweeps + 1;
    const double crit = t[2] * dt_over_rho;
    const double tol = this->tol < 0.0 ? sc->tol_dev : this->tol;
    sc->rr = t[0];
    sc->rr0 = t[0];
    sc->beta = 0.0;
    sc->iters = 0;
    sc->crit = crit;
    sc->sumx = t[1];
    sc->tol_rr = inner_rtol * inner_rtol * t[0];
    const bool bad = !(t[0] == t[0]) || !(crit == crit);
    if (bad) sc->status = FVIB_ENONFINITE;
    const bool conv = bad || crit <= tol || t[0] == 0.0;
    sc->done = conv ? 1 : 0;
    if (MODE != 0) sc->outer_done = conv ? 1 : 0;
    // the host's check reads the scalars once the stream has passed this
    // kernel (completion makes the stores visible to it)
    if (mirror) *mirror = *sc;
    if (tick) post(sc);
  }
};

struct FinCgDir {
  __device__ bool skip(const SolverScalars* sc) const { return sc->done != 0; }
  __device__ void apply(const double* t, SolverScalars* sc) const {
    sc->pq = t[0];
    sc->alpha = (t[0] > 0.0) ? sc->rr / t[0] : 0.0;
    sc->sump = t[1];          // sum(p), used to keep x at zero mean
    if (!(t[0] == t[0])) {
      sc->status = FVIB_ENONFINITE;
      sc->done = 1;
      sc->outer_done = 1;
    } else if (!(t[0] > 0.0)) {
      sc->done = 1;           // exact solution reached (p = 0)
    }
  }
};

template <int MODE>
struct FinCgUpdate {
  double tol, dt_over_rho;
  int maxit;
  __device__ bool skip(const SolverScalars* sc) const { return sc->done != 0; }
  __device__ void apply(const double* t, SolverScalars* sc) const {
    const double rrn = t[0];
    sc->beta = (sc->rr > 0.0) ? rrn / sc->rr : 0.0;
    sc->rr = rrn;
    sc->iters += 1;
    bool conv;
    if (MODE == 0) {
      sc->crit = t[1] * dt_over_rho;
      conv = sc->crit <= (tol < 0.0 ? sc->tol_dev : tol);
    } else {
      conv = rrn <= sc->tol_rr;
    }
    if (!(rrn == rrn)) {
      sc->status = FVIB_ENONFINITE;
      sc->outer_done = 1;
      conv = true;
    }
    if (!conv && sc->iters >= maxit) {
      if (MODE == 0) sc->status = FVIB_ENOCONV;
      conv = true;
    }
    sc->done = conv ? 1 : 0;
  }
};

struct FinDivMax {
  // nullable: the step record, written here from the scalars (a solve by
  // fast diagonalisation without a body, whose scalars are final once the
  // projection has run)
  fvib_step_info* info;
  int* sticky;   // nullable: a failed status is also stored here
  __device__ bool skip(const SolverScalars*) const { return false; }
  __device__ void apply(const double* t, SolverScalars* sc) const {
    sc->div_max = t[0];
    if (!info) return;
    int st = sc->status;
    if (st == FVIB_OK && sc->clamp) st = FVIB_EINVAL;
    if (sticky && st != FVIB_OK) *sticky = st;
    info->status = st;
    info->cg_iters = 0;
    info->ir_iters = sc->sweeps;
    info->flags = sc->clamp;
    info->res = sc->crit;
    info->div_max = t[0];
    for (int a = 0; a < 3; ++a) info->force[a] = sc->force[a];
    info->xi = 0.0;
  }
};

// ----------------------------------------------------------------- RHS
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock)
k_ppe_rhs(Geo<T> G, PGeo<double> P, Tiling tl, const T* __restrict__ s0,
          const T* __restrict__ s1, const T* __restrict__ s2, IbView<T> ib,
          double* __restrict__ b, RedBuf red, SolverScalars* sc) {
  const int nx_ = G.n[0], ny_ = G.n[1];
  const T* us[3] = {s0, s1, s2};
  const double scale = -1.0 / P.dt_over_rho;
  double sum = 0.0;
  FVIB_TILE_LOOP(tl)
    const int I[3] = {i, j, k};
    double lo[DIM], hi[DIM], d[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      int H[3] = {i, j, k};
      H[c] += 1;
      if (G.per[c] && H[c] == G.n[c]) H[c] = 0;
      lo[c] = (double)us[c][fidx(G.ext[c], i, j, k)];
      hi[c] = (double)us[c][fidx(G.ext[c], H[0], H[1], H[2])];
      d[c] = P.dx[c][I[c]];
    }
    if (ib.active && !ib.box) {
      // u~ = u_c on the forced faces (a static box has u* = u_c = 0 there)
#pragma unroll
      for (int c = 0; c < (DIM < 2 ? DIM : 2); ++c) {
        const double Uc = ib.body[3 + c];
        const int* o = ib.origin;
        const int W0 = ib.W[c][0], W1 = ib.W[c][1];
        int li = i - o[2 * c], ljj = j - o[2 * c + 1];
        if (li >= 0 && ljj >= 0 && li < W0 && ljj < W1 && ib.cls[c][ljj * W0 + li]) lo[c] = Uc;
        int H[2] = {i + (c == 0), j + (c == 1)};
        if (G.per[c] && H[c] == G.n[c]) H[c] = 0;
        li = H[0] - o[2 * c];
        ljj = H[1] - o[2 * c + 1];
        if (li >= 0 && ljj >= 0 && li < W0 && ljj < W1 && ib.cls[c][ljj * W0 + li]) hi[c] = Uc;
      }
    }
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      double A = 1.0;
#pragma unroll
      for (int a = 0; a < DIM; ++a)
        if (a != c) A *= d[a];
      acc += hi[c] * A - lo[c] * A;
    }
    const double bc = scale * acc;
    b[c_] = bc;
    sum += bc;
  FVIB_TILE_END
  double v[1] = {sum};
  block_partials<1, 1>(v, red.partial);
}

// ------------------------------------------------------------ residual
// r = b - mean(b) - A x in double.  MODE 0 (double CG): writes r (double)
// and starts the solve.  Refinement sweeps decide whether refinement is
// finished and hand r to the inner solve: MODE 1 float CG (r as float, the
// inner iterate cleared), MODE 2 float fast diagonalisation (r as float),
// MODE 3 double fast diagonalisation (r as double).  Also records sum(x)
// for the pressure gauge.
template <int DIM, int MODE>
__global__ void __launch_bounds__(kBlock)
k_residual(PGeo<double> P, ColTiling ct, const double* __restrict__ b,
           const double* __restrict__ x, double* __restrict__ r64, float* __restrict__ r32,
           float* __restrict__ d32, RedBuf red, SolverScalars* sc, int first) {
  if (!first && sc->outer_done) return;
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  const int64_t sxy = (int64_t)nx * ny;
  const double mb = sc->meanb;
  double rr = 0.0, sx = 0.0, mx = 0.0;
  const int lx = threadIdx.x & (kTileX - 1), ly = threadIdx.x / kTileX;
  for (int u = xcd_block(blockIdx.x, gridDim.x); u < ct.nunits; u += gridDim.x) {
    const int tx = u % ct.ntx, ty = (u / ct.ntx) % ct.nty, zc = u / (ct.ntx * ct.nty);
    const int i = tx * kTileX + lx, j = ty * kTileY + ly;
    if (i >= nx || j >= ny) continue;
    const int k0 = zc * ct.zchunk, k1 = min(k0 + ct.zchunk, nz);
    // column constants: x-y neighbours (wrapped / clamped, the boundary
    // faces carry kf = 0) and coefficients
    const int64_t cC = (int64_t)j * nx + i;
    const int64_t cW = (int64_t)j * nx + nb_lo(i, nx, P.per[0]);
    const int64_t cE = (int64_t)j * nx + nb_hi(i, nx, P.per[0]);
    const int64_t cS = (int64_t)nb_lo(j, ny, P.per[1]) * nx + i;
    const int64_t cN = (int64_t)nb_hi(j, ny, P.per[1]) * nx + i;
    const double dxi = P.dx[0][i], dyj = P.dx[1][j];
    const double kxl = P.kf[0][i], kxh = P.kf[0][i + 1];
    const double kyl = P.kf[1][j], kyh = P.kf[1][j + 1];
    const double ivxy = (double)P.iv[0][i] * (double)P.iv[1][j];
    auto emit = [&](int k, double xc, double r, double iv) {
      const int64_t c = (int64_t)k * sxy + cC;
      if (MODE == 0 || MODE == 3) {
        r64[c] = r;
      } else {
        r32[c] = (float)r;
        if (MODE == 1) d32[c] = 0.0f;
      }
      rr += r * r;
      sx += xc;
      mx = fmax(mx, fabs(r) * iv);
    };
    if (DIM == 2) {
      // same term order as apply_A
      const double xc = x[cC];
      double acc = 0.0;
      acc += dyj * kxl * (xc - x[cW]);
      acc += dyj * kxh * (xc - x[cE]);
      acc += dxi * kyl * (xc - x[cS]);
      acc += dxi * kyh * (xc - x[cN]);
      emit(0, xc, b[cC] - mb - acc, ivxy);
      continue;
    }
    const int pz = P.per[2];
    auto at = [&](int64_t off, int k) { return x[(int64_t)k * sxy + off]; };
    double xm = at(cC, nb_lo(k0, nz, pz)), xc = at(cC, k0), xp = at(cC, nb_hi(k0, nz, pz));
    double w = at(cW, k0), e = at(cE, k0), so = at(cS, k0), no = at(cN, k0);
    double bb = b[(int64_t)k0 * sxy + cC];
    for (int k = k0; k < k1; ++k) {
      // plane k + 1 is fetched while plane k is evaluated
      double xp2 = 0.0, w2 = 0.0, e2 = 0.0, so2 = 0.0, no2 = 0.0, bb2 = 0.0;
      if (k + 1 < k1) {
        xp2 = at(cC, nb_hi(k + 1, nz, pz));
        w2 = at(cW, k + 1);
        e2 = at(cE, k + 1);
        so2 = at(cS, k + 1);
        no2 = at(cN, k + 1);
        bb2 = b[(int64_t)(k + 1) * sxy + cC];
      }
      const double dzk = P.dx[2][k], kzl = P.kf[2][k], kzh = P.kf[2][k + 1];
      // same term order as apply_A
      double acc = 0.0;
      const double ax = dyj * dzk, ay = dxi * dzk, az = dxi * dyj;
      acc += ax * kxl * (xc - w);
      acc += ax * kxh * (xc - e);
      acc += ay * kyl * (xc - so);
      acc += ay * kyh * (xc - no);
      acc += az * kzl * (xc - xm);
      acc += az * kzh * (xc - xp);
      emit(k, xc, bb - mb - acc, ivxy * (double)P.iv[2][k]);
      xm = xc;
      xc = xp;
      xp = xp2;
      w = w2;
      e = e2;
      so = so2;
      no = no2;
      bb = bb2;
    }
  }
  double v[3] = {rr, sx, mx};
  block_partials<3, 2>(v, red.partial);
}

// ------------------------------------- RHS and first residual (3D, FDM)
// The right-hand side of Eq. 9 (no immersed body) and the first residual of
// the refinement in one column march: b = -(rho/dt) S u* is stored for the
// later residuals, and r = b - A x_in is handed to the fast-diagonalisation
// sweep without the mean of b, which is not known until the reduction ends
// (the sweep drops the constant mode, so the correction is the same).  The
// stopping criterion is taken as max |r| / V + |mean b| max (1 / V), an
// upper bound of the criterion of the mean-free residual.  Same terms in the
// same order as k_ppe_rhs (b) and k_residual (A x).
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock)
k_rhs_residual_col(Geo<T> G, PGeo<double> P, ColTiling ct, const T* __restrict__ s0,
                   const T* __restrict__ s1, const T* __restrict__ s2,
                   const double* __restrict__ x, double* __restrict__ b,
                   double* __restrict__ r64, float* __restrict__ r32, RedBuf red) {
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  const int64_t sxy = (int64_t)nx * ny;
  const double scale = -1.0 / P.dt_over_rho;
  double rr = 0.0, sx = 0.0, sb = 0.0, mx = 0.0;
  const int lx = threadIdx.x & (kTileX - 1), ly = threadIdx.x / kTileX;
  for (int u = xcd_block(blockIdx.x, gridDim.x); u < ct.nunits; u += gridDim.x) {
    const int tx = u % ct.ntx, ty = (u / ct.ntx) % ct.nty, zc = u / (ct.ntx * ct.nty);
    const int i = tx * kTileX + lx, j = ty * kTileY + ly;
    if (i >= nx || j >= ny) continue;
    const int k0 = zc * ct.zchunk, k1 = min(k0 + ct.zchunk, nz);
    // velocity faces of the column: u at i and its high face, v at j and its
    // high face, w at k and k + 1 (wrapped on periodic axes)
    const int iH = (G.per[0] && i + 1 == nx) ? 0 : i + 1;
    const int jH = (G.per[1] && j + 1 == ny) ? 0 : j + 1;
    const int ex0 = G.ext[0][0], ex1 = G.ext[0][1];
    const int ey0 = G.ext[1][0], ey1 = G.ext[1][1];
    const int ez0 = G.ext[2][0], ez1 = G.ext[2][1];
    const int64_t su = (int64_t)ex0 * ex1, sv = (int64_t)ey0 * ey1, sw = (int64_t)ez0 * ez1;
    const int64_t uL = (int64_t)j * ex0 + i, uH = (int64_t)j * ex0 + iH;
    const int64_t vL = (int64_t)j * ey0 + i, vH = (int64_t)jH * ey0 + i;
    const int64_t wL = (int64_t)j * ez0 + i;
    auto kup = [&](int k) { return (G.per[2] && k + 1 == nz) ? 0 : k + 1; };
    // pressure column: x-y neighbours (wrapped / clamped; kf = 0 on the
    // boundary faces) and coefficients
    const int64_t cC = (int64_t)j * nx + i;
    const int64_t cW = (int64_t)j * nx + nb_lo(i, nx, P.per[0]);
    const int64_t cE = (int64_t)j * nx + nb_hi(i, nx, P.per[0]);
    const int64_t cS = (int64_t)nb_lo(j, ny, P.per[1]) * nx + i;
    const int64_t cN = (int64_t)nb_hi(j, ny, P.per[1]) * nx + i;
    const double dxi = P.dx[0][i], dyj = P.dx[1][j];
    const double kxl = P.kf[0][i], kxh = P.kf[0][i + 1];
    const double kyl = P.kf[1][j], kyh = P.kf[1][j + 1];
    const double ivxy = (double)P.iv[0][i] * (double)P.iv[1][j];
    const int pz = P.per[2];
    auto at = [&](int64_t off, int k) { return x[(int64_t)k * sxy + off]; };
    double xm = at(cC, nb_lo(k0, nz, pz)), xc = at(cC, k0), xp = at(cC, nb_hi(k0, nz, pz));
    double xw = at(cW, k0), xe = at(cE, k0), xs = at(cS, k0), xn = at(cN, k0);
    double ul = (double)s0[(int64_t)k0 * su + uL], uh = (double)s0[(int64_t)k0 * su + uH];
    double vl = (double)s1[(int64_t)k0 * sv + vL], vh = (double)s1[(int64_t)k0 * sv + vH];
    double wl = (double)s2[(int64_t)k0 * sw + wL], wh = (double)s2[(int64_t)kup(k0) * sw + wL];
    for (int k = k0; k < k1; ++k) {
      // plane k + 1 is fetched while plane k is evaluated
      double xp2 = 0.0, xw2 = 0.0, xe2 = 0.0, xs2 = 0.0, xn2 = 0.0;
      double ul2 = 0.0, uh2 = 0.0, vl2 = 0.0, vh2 = 0.0, wh2 = 0.0;
      if (k + 1 < k1) {
        const int64_t kn = k + 1;
        xp2 = at(cC, nb_hi(k + 1, nz, pz));
        xw2 = at(cW, k + 1);
        xe2 = at(cE, k + 1);
        xs2 = at(cS, k + 1);
        xn2 = at(cN, k + 1);
        ul2 = (double)s0[kn * su + uL];
        uh2 = (double)s0[kn * su + uH];
        vl2 = (double)s1[kn * sv + vL];
        vh2 = (double)s1[kn * sv + vH];
        wh2 = (double)s2[(int64_t)kup(k + 1) * sw + wL];
      }
      const double dzk = P.dx[2][k], kzl = P.kf[2][k], kzh = P.kf[2][k + 1];
      // b of this cell (the terms of k_ppe_rhs in its order)
      double fl = 0.0;
      fl += uh * (dyj * dzk) - ul * (dyj * dzk);
      fl += vh * (dxi * dzk) - vl * (dxi * dzk);
      fl += wh * (dxi * dyj) - wl * (dxi * dyj);
      const double bc = scale * fl;
      // A x (the terms of k_residual in its order)
      double acc = 0.0;
      const double ax = dyj * dzk, ay = dxi * dzk, az = dxi * dyj;
      acc += ax * kxl * (xc - xw);
      acc += ax * kxh * (xc - xe);
      acc += ay * kyl * (xc - xs);
      acc += ay * kyh * (xc - xn);
      acc += az * kzl * (xc - xm);
      acc += az * kzh * (xc - xp);
      const double r = bc - acc;
      const int64_t c = (int64_t)k * sxy + cC;
      b[c] = bc;
      if (MODE == 3)
        r64[c] = r;
      else
        r32[c] = (float)r;
      rr += r * r;
      sx += xc;
      sb += bc;
      mx = fmax(mx, fabs(r) * (ivxy * (double)P.iv[2][k]));
      xm = xc;
      xc = xp;
      xp = xp2;
      xw = xw2;
      xe = xe2;
      xs = xs2;
      xn = xn2;
      ul = ul2;
      uh = uh2;
      vl = vl2;
      vh = vh2;
      wl = wh;
      wh = wh2;
    }
  }
  double v[4] = {rr, sx, sb, mx};
  block_partials<4, 3>(v, red.partial);
}

// ------------------------------------- RHS and first residual (2D, FDM)
// As k_rhs_residual_col on a 2D grid (one cell per thread), with the
// immersed body's forced faces taking the body velocity in the divergence
// (Eq. 9's u~ = u_c there, the terms of k_ppe_rhs): one pass in place of
// the right-hand side, its epilogue, the first residual and its epilogue.
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock)
k_rhs_residual_2d(Geo<T> G, PGeo<double> P, ColTiling ct, const T* __restrict__ s0,
                  const T* __restrict__ s1, IbView<T> ib, const double* __restrict__ x,
                  double* __restrict__ b, double* __restrict__ r64, float* __restrict__ r32,
                  RedBuf red) {
  const int nx = P.n[0], ny = P.n[1];
  const double scale = -1.0 / P.dt_over_rho;
  double rr = 0.0, sx = 0.0, sb = 0.0, mx = 0.0;
  const int lx = threadIdx.x & (kTileX - 1), ly = threadIdx.x / kTileX;
  for (int u = xcd_block(blockIdx.x, gridDim.x); u < ct.nunits; u += gridDim.x) {
    const int tx = u % ct.ntx, ty = (u / ct.ntx) % ct.nty;
    const int i = tx * kTileX + lx, j = ty * kTileY + ly;
    if (i >= nx || j >= ny) continue;
    const int iH = (G.per[0] && i + 1 == nx) ? 0 : i + 1;
    const int jH = (G.per[1] && j + 1 == ny) ? 0 : j + 1;
    double lo[2], hi[2];
    lo[0] = (double)s0[(int64_t)j * G.ext[0][0] + i];
    hi[0] = (double)s0[(int64_t)j * G.ext[0][0] + iH];
    lo[1] = (double)s1[(int64_t)j * G.ext[1][0] + i];
    hi[1] = (double)s1[(int64_t)jH * G.ext[1][0] + i];
    if (ib.active && !ib.box) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double Uc = ib.body[3 + c];
        const int* o = ib.origin;
        const int W0 = ib.W[c][0], W1 = ib.W[c][1];
        int li = i - o[2 * c], lj = j - o[2 * c + 1];
        if (li >= 0 && lj >= 0 && li < W0 && lj < W1 && ib.cls[c][lj * W0 + li]) lo[c] = Uc;
        li = (c == 0 ? iH : i) - o[2 * c];
        lj = (c == 1 ? jH : j) - o[2 * c + 1];
        if (li >= 0 && lj >= 0 && li < W0 && lj < W1 && ib.cls[c][lj * W0 + li]) hi[c] = Uc;
      }
    }
    const double dxi = P.dx[0][i], dyj = P.dx[1][j];
    // b of this cell (the terms of k_ppe_rhs in its order)
    double fl = 0.0;
    fl += hi[0] * dyj - lo[0] * dyj;
    fl += hi[1] * dxi - lo[1] * dxi;
    const double bc = scale * fl;
    // A x (the terms of k_residual in its order)
    const int64_t cC = (int64_t)j * nx + i;
    const double xc = x[cC];
    const double xw = x[(int64_t)j * nx + nb_lo(i, nx, P.per[0])];
    const double xe = x[(int64_t)j * nx + nb_hi(i, nx, P.per[0])];
    const double xs = x[(int64_t)nb_lo(j, ny, P.per[1]) * nx + i];
    const double xn = x[(int64_t)nb_hi(j, ny, P.per[1]) * nx + i];
    double acc = 0.0;
    acc += dyj * P.kf[0][i] * (xc - xw);
    acc += dyj * P.kf[0][i + 1] * (xc - xe);
    acc += dxi * P.kf[1][j] * (xc - xs);
    acc += dxi * P.kf[1][j + 1] * (xc - xn);
    const double r = bc - acc;
    b[cC] = bc;
    if (MODE == 3)
      r64[cC] = r;
    else
      r32[cC] = (float)r;
    rr += r * r;
    sx += xc;
    sb += bc;
    mx = fmax(mx, fabs(r) * ((double)P.iv[0][i] * (double)P.iv[1][j]));
  }
  double v[4] = {rr, sx, sb, mx};
  block_partials<4, 3>(v, red.partial);
}

// Epilogue of k_rhs_residual_col: the mean of b, then what FinResidual does
// for the first residual of a solve, on the upper-bound criterion.
struct FinRhsResidual {
  double tol, inner_rtol, dt_over_rho, inv_ncell, max_iv;
  SolverScalars* mirror;
  __device__ bool skip(const SolverScalars*) const { return false; }
  __device__ void apply(const double* t, SolverScalars* sc) const {
    const double mb = t[2] * inv_ncell;
    sc->meanb = mb;
    sc->sweeps = 0;
    const double crit = (t[3] + fabs(mb) * max_iv) * dt_over_rho;
    sc->rr = t[0];
    sc->rr0 = t[0];
    sc->beta = 0.0;
    sc->iters = 0;
    sc->crit = crit;
    sc->sumx = t[1];
    sc->tol_rr = inner_rtol * inner_rtol * t[0];
    const bool bad = !(t[0] == t[0]) || !(crit == crit);
    if (bad) sc->status = FVIB_ENONFINITE;
    const bool conv = bad || crit <= tol || t[0] == 0.0;
    sc->done = conv ? 1 : 0;
    sc->outer_done = conv ? 1 : 0;
    if (mirror) *mirror = *sc;
  }
};

// ------------------------------------------------------ CG direction
// p_new = r + beta p_old (beta = 0 on the first iteration), then p.Ap and
// sum(p).  p_new is formed on the fly at the stencil neighbours, so p_old
// and r are each read once.
template <typename V, int DIM>
__global__ void __launch_bounds__(kBlock)
k_cg_dir(PGeo<V> P, Tiling tl, const V* __restrict__ r, const V* __restrict__ pold,
         V* __restrict__ pnew, RedBuf red, SolverScalars* sc) {
  if (sc->done) return;
  const int nx_ = P.n[0], ny_ = P.n[1];
  const V beta = (V)sc->beta;
  const bool first = (sc->iters == 0);
  double pq = 0.0, sp = 0.0;
  auto get = [&](int a, int b_, int c) {
    const int64_t id = ((int64_t)c * ny_ + b_) * nx_ + a;
    return first ? r[id] : r[id] + beta * pold[id];
  };
  FVIB_TILE_LOOP(tl)
    const V pc = first ? r[c_] : r[c_] + beta * pold[c_];
    const V q = apply_A<V, DIM>(P, get, i, j, k, pc);
    pnew[c_] = pc;
    pq += (double)pc * (double)q;
    sp += (double)pc;
  FVIB_TILE_END
  double v[2] = {pq, sp};
  block_partials<2, 2>(v, red.partial);
}

// --------------------------------------------------------- CG update
// x += alpha (p - mean p), r -= alpha A p; r.r and max |r / V| decide the
// next beta and convergence.  MODE 0: stop on the divergence criterion
// (double solve).  MODE 1: stop on r.r <= inner_rtol^2 r0.r0 (inner solve).
template <typename V, int DIM, int MODE>
__global__ void __launch_bounds__(kBlock)
k_cg_update(PGeo<V> P, Tiling tl, const V* __restrict__ p, V* __restrict__ x,
            V* __restrict__ r, RedBuf red, SolverScalars* sc, double tol, int maxit) {
  if (sc->done) return;
  const int nx_ = P.n[0], ny_ = P.n[1];
  const V alpha = (V)sc->alpha;
  const V shift = (V)(sc->alpha * sc->sump * P.inv_ncell);
  double rr = 0.0, mx = 0.0;
  auto get = [&](int a, int b_, int c) { return p[((int64_t)c * ny_ + b_) * nx_ + a]; };
  FVIB_TILE_LOOP(tl)
    const V pc = p[c_];
    const double ivol = (MODE == 0) ? inv_volume(P, i, j, k) : 0.0;
    const V xo = x[c_], ro = r[c_];
    const V q = apply_A<V, DIM>(P, get, i, j, k, pc);
    x[c_] = xo + (alpha * pc - shift);
    const V rn = ro - alpha * q;
    r[c_] = rn;
    rr += (double)rn * (double)rn;
    if (MODE == 0) mx = fmax(mx, fabs((double)rn) * ivol);
  FVIB_TILE_END
  double v[2] = {rr, mx};
  block_partials<2, 1>(v, red.partial);
}

// ------------------------------------------------ refinement correction
// p64 += d32 - mean(p64): the residual kernel recorded sum(p64) and the
// inner iterate is kept at zero mean by its own updates.
__global__ void __launch_bounds__(kBlock)
k_ir_correct(int64_t n, double* __restrict__ p, const float* __restrict__ d,
             const SolverScalars* sc, double inv_n) {
  const double shift = sc->sumx * inv_n;
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * kBlock)
    p[c] = (p[c] + (double)d[c]) - shift;
}

// --------------------------------------------------------- projection
// u^{n+1} = u* - (dt/rho) (p_c - p_{c-1}) / dc on every face that is not a
// boundary face of a bounded axis (those keep u*: their coefficient is 0).  Each thread owns the
// low faces of its cell and, on the last cell of a bounded axis, the high
// boundary face.  The divergence of the corrected field is evaluated in
// double before rounding to the storage type and its maximum recorded.
template <typename T, int DIM, bool MIX>
__global__ void __launch_bounds__(kBlock)
k_project(Geo<T> G, PGeo<double> P, Tiling tl, const T* __restrict__ s0,
          const T* __restrict__ s1, const T* __restrict__ s2, const double* __restrict__ p,
          T* o0, T* o1, T* o2, RedBuf red, SolverScalars* sc, StageMix mix,
          double* __restrict__ pg) {
  const int nx_ = G.n[0], ny_ = G.n[1];
  const T* us[3] = {s0, s1, s2};
  T* out[3] = {o0, o1, o2};
  // pg (nullable): the pressure minus its mean (the gradient does not see it)
  const double mean = pg ? sc->sumx * P.inv_ncell : 0.0;
  const T* u0[3] = {(const T*)mix.u0[0], (const T*)mix.u0[1], (const T*)mix.u0[2]};
  // stage output: a u0 + b (corrected field), or the corrected field
  auto put = [&](int c, int64_t id, double v) {
    out[c][id] = MIX ? (T)(mix.a * (double)u0[c][id] + mix.b * v) : (T)v;
  };
  const double f = P.dt_over_rho;
  double mx = 0.0;
  FVIB_TILE_LOOP(tl)
    const int I[3] = {i, j, k};
    const double pc = p[c_];
    if (pg) pg[c_] = pc - mean;
    const double ivol = inv_volume(P, i, j, k);
    int64_t lo_id[DIM], hi_id[DIM];
    double ulo[DIM], uhi[DIM], plo[DIM], phi[DIM], d[DIM], klo[DIM], khi[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int ic = I[c], nc = G.n[c];
      int H[3] = {i, j, k};
      H[c] = (G.per[c] && ic + 1 == nc) ? 0 : ic + 1;
      lo_id[c] = fidx(G.ext[c], i, j, k);
      hi_id[c] = fidx(G.ext[c], H[0], H[1], H[2]);
      ulo[c] = (double)us[c][lo_id[c]];
      uhi[c] = (double)us[c][hi_id[c]];
      int J[3] = {i, j, k};
      J[c] = nb_lo(ic, nc, G.per[c]);
      plo[c] = p[((int64_t)J[2] * ny_ + J[1]) * nx_ + J[0]];
      J[c] = nb_hi(ic, nc, G.per[c]);
      phi[c] = p[((int64_t)J[2] * ny_ + J[1]) * nx_ + J[0]];
      d[c] = P.dx[c][ic];
      klo[c] = P.kf[c][ic];
      khi[c] = P.kf[c][ic + 1];
    }
    double div = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const int ic = I[c], nc = G.n[c];
      double A = 1.0;
#pragma unroll
      for (int a = 0; a < DIM; ++a)
        if (a != c) A *= d[a];
      // faces of a bounded boundary have kf = 0 and keep u*
      const double lo = ulo[c] - f * (pc - plo[c]) * klo[c];
      const double hi = uhi[c] - f * (phi[c] - pc) * khi[c];
      put(c, lo_id[c], lo);
      if (!G.per[c] && ic + 1 == nc) put(c, hi_id[c], hi);
      div += (hi - lo) * A;
    }
    mx = fmax(mx, fabs(div) * ivol);
  FVIB_TILE_END
  double v[1] = {mx};
  block_partials<1, 0>(v, red.partial);
}

// 3D projection as a column march: each thread owns an (x, y) column of a
// unit and walks up its z-chunk keeping p at k - 1, k, k + 1 and the w
// faces below and above the cell in registers (the next plane prefetched),
// so p and u* cross HBM once per chunk; the x and y neighbours of a plane
// are shared with the adjacent columns through the caches.  Same arithmetic
// and term order as k_project.  pg (nullable, not p): receives p minus its
// mean (the gradient does not see that constant).
template <typename T, bool MIX>
__global__ void __launch_bounds__(kBlock)
k_project_col(Geo<T> G, PGeo<double> P, ColTiling ct, const T* __restrict__ s0,
              const T* __restrict__ s1, const T* __restrict__ s2, const double* __restrict__ p,
              T* o0, T* o1, T* o2, RedBuf red, double* __restrict__ pg, const SolverScalars* sc,
              StageMix mix) {
  const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
  const T* m0 = (const T*)mix.u0[0];
  const T* m1 = (const T*)mix.u0[1];
  const T* m2 = (const T*)mix.u0[2];
  // stage output: a u0 + b (corrected field), or the corrected field (each
  // element of u0 is read by the thread that writes it, before the write)
  auto put = [&](T* o, const T* m, int64_t id, double v) {
    __builtin_nontemporal_store(MIX ? (T)(mix.a * (double)m[id] + mix.b * v) : (T)v, &o[id]);
  };
  const int64_t sxy = (int64_t)nx * ny;
  const double f = P.dt_over_rho;
  // gauge constant of the pressure copy (the mean of p, from the sum the
  // last residual recorded)
  const double mean = pg ? sc->sumx * P.inv_ncell : 0.0;
  double mx = 0.0;
  const int lx = threadIdx.x & (kTileX - 1), ly = threadIdx.x / kTileX;
  for (int u = xcd_block(blockIdx.x, gridDim.x); u < ct.nunits; u += gridDim.x) {
    const int tx = u % ct.ntx, ty = (u / ct.ntx) % ct.nty, zc = u / (ct.ntx * ct.nty);
    const int i = tx * kTileX + lx, j = ty * kTileY + ly;
    if (i >= nx || j >= ny) continue;
    const int k0 = zc * ct.zchunk, k1 = min(k0 + ct.zchunk, nz);
    // column constants: face extents, neighbours and coefficients along x, y
    const int ex0 = G.ext[0][0], ex1 = G.ext[0][1];       // u faces
    const int ey0 = G.ext[1][0], ey1 = G.ext[1][1];       // v faces
    const int ez0 = G.ext[2][0], ez1 = G.ext[2][1];       // w faces
    const int iH = (G.per[0] && i + 1 == nx) ? 0 : i + 1;
    const int jH = (G.per[1] && j + 1 == ny) ? 0 : j + 1;
    const int64_t cC = (int64_t)j * nx + i;
    const int64_t cW = (int64_t)j * nx + nb_lo(i, nx, P.per[0]);
    const int64_t cE = (int64_t)j * nx + nb_hi(i, nx, P.per[0]);
    const int64_t cS = (int64_t)nb_lo(j, ny, P.per[1]) * nx + i;
    const int64_t cN = (int64_t)nb_hi(j, ny, P.per[1]) * nx + i;
    const int64_t uL = (int64_t)j * ex0 + i, uH = (int64_t)j * ex0 + iH;
    const int64_t vL = (int64_t)j * ey0 + i, vH = (int64_t)jH * ey0 + i;
    const int64_t wL = (int64_t)j * ez0 + i;
    const int64_t su = (int64_t)ex0 * ex1, sv = (int64_t)ey0 * ey1, sw = (int64_t)ez0 * ez1;
    const double dx = P.dx[0][i], dy = P.dx[1][j];
    const double kxl = P.kf[0][i], kxh = P.kf[0][i + 1];
    const double kyl = P.kf[1][j], kyh = P.kf[1][j + 1];
    const double ivxy = (double)P.iv[0][i] * (double)P.iv[1][j];
    const bool xlast = !G.per[0] && i + 1 == nx, ylast = !G.per[1] && j + 1 == ny;
    auto pz = [&](int k) { return p[(int64_t)k * sxy + cC]; };
    double pm = pz(nb_lo(k0, nz, P.per[2])), pc = pz(k0);
    double wlo = (double)s2[(int64_t)k0 * sw + wL];
    for (int k = k0; k < k1; ++k) {
      const int kn = nb_hi(k, nz, P.per[2]);
      const int kH = (G.per[2] && k + 1 == nz) ? 0 : k + 1;
      // plane loads (the z neighbours above come first)
      const double pp = pz(kn);
      const double whi = (double)s2[(int64_t)kH * sw + wL];
      const int64_t pk = (int64_t)k * sxy;
      const double pw = p[pk + cW], pe = p[pk + cE], ps = p[pk + cS], pn = p[pk + cN];
      const double ulo = (double)s0[(int64_t)k * su + uL], uhi = (double)s0[(int64_t)k * su + uH];
      const double vlo = (double)s1[(int64_t)k * sv + vL], vhi = (double)s1[(int64_t)k * sv + vH];
      const double dz = P.dx[2][k], kzl = P.kf[2][k], kzh = P.kf[2][k + 1];
      const double ivol = ivxy * (double)P.iv[2][k];
      // faces of a bounded boundary have kf = 0 and keep u*
      const double lx_ = ulo - f * (pc - pw) * kxl, hx = uhi - f * (pe - pc) * kxh;
      const double ly_ = vlo - f * (pc - ps) * kyl, hy = vhi - f * (pn - pc) * kyh;
      const double lz = wlo - f * (pc - pm) * kzl, hz = whi - f * (pp - pc) * kzh;
      // streaming stores: the next reader is the following step
      if (pg) __builtin_nontemporal_store(pc - mean, &pg[pk + cC]);
      put(o0, m0, (int64_t)k * su + uL, lx_);
      if (xlast) put(o0, m0, (int64_t)k * su + uH, hx);
      put(o1, m1, (int64_t)k * sv + vL, ly_);
      if (ylast) put(o1, m1, (int64_t)k * sv + vH, hy);
      put(o2, m2, (int64_t)k * sw + wL, lz);
      if (!G.per[2] && k + 1 == nz) put(o2, m2, (int64_t)kH * sw + wL, hz);
      double div = 0.0;
      div += (hx - lx_) * (dy * dz);
      div += (hy - ly_) * (dx * dz);
      div += (hz - lz) * (dx * dy);
      mx = fmax(mx, fabs(div) * ivol);
      pm = pc;
      pc = pp;
      wlo = whi;
    }
  }
  double v[1] = {mx};
  block_partials<1, 0>(v, red.partial);
}

// ---------------------------------------------------------- apply A
__global__ void __launch_bounds__(kBlock)
k_apply_A(PGeo<double> P, Tiling tl, const double* __restrict__ x, double* __restrict__ y) {
  const int nx_ = P.n[0], ny_ = P.n[1];
  auto get = [&](int a, int b_, int c) { return x[((int64_t)c * ny_ + b_) * nx_ + a]; };
  FVIB_TILE_LOOP(tl)
    if (P.dim == 3)
      y[c_] = apply_A<double, 3>(P, get, i, j, k, x[c_]);
    else
      y[c_] = apply_A<double, 2>(P, get, i, j, k, x[c_]);
  FVIB_TILE_END
}

// ============================================================ launchers
static inline Tiling red_tiling(const int n[3]) { return make_tiling(n[0], n[1], n[2]); }

template <typename T>
int launch_ppe_rhs(const Geo<T>& G, const PGeo<double>& P, const T* const us[3],
                   const IbView<T>& ib, double* b, RedBuf red, SolverScalars* sc,
                   hipStream_t s) {
  const Tiling tl = red_tiling(G.n);
  if (G.dim == 2)
    launch_kernel((k_ppe_rhs<T, 2>), dim3(tl.nblocks), dim3(kBlock), 0, s, G, P, tl, us[0],
                       us[1], us[2], ib, b, red, sc);
  else
    launch_kernel((k_ppe_rhs<T, 3>), dim3(tl.nblocks), dim3(kBlock), 0, s, G, P, tl, us[0],
                       us[1], us[2], ib, b, red, sc);
  FVIB_HIP(hipGetLastError());
  FVIB_HIP((launch_finish<1, 1>(red.partial, tl.nblocks, sc, FinMeanB{P.inv_ncell}, s)));
  return FVIB_OK;
}

int launch_residual(const PGeo<double>& P, int mode, const double* b, const double* x,
                    double* r64, float* r32, float* d32, RedBuf red, SolverScalars* sc,
                    double tol, double inner_rtol, hipStream_t s, int first,
                    SolverScalars* mirror, unsigned long long* tick, unsigned int ticket) {
  const ColTiling ct = make_col_tiling(P.n[0], P.n[1], P.n[2]);
  dim3 g(ct.nblocks), bl(kBlock);
#define FVIB_RES(D, M)                                                                        \
  launch_kernel((k_residual<D, M>), g, bl, 0, s, P, ct, b, x, r64, r32, d32, red, sc,      \
                     first);                                                                    \
  FVIB_HIP(hipGetLastError());                                                                  \
  FVIB_HIP((launch_finish<3, 2>(red.partial, ct.nblocks, sc,                                    \
                                FinResidual<M>{tol, inner_rtol, P.dt_over_rho, first, mirror,  \
                                               tick, ticket}, s)))
  if (P.dim == 2) {
    switch (mode) {
      case 0: FVIB_RES(2, 0); break;
      case 1: FVIB_RES(2, 1); break;
      case 2: FVIB_RES(2, 2); break;
      default: FVIB_RES(2, 3); break;
    }
  } else {
    switch (mode) {
      case 0: FVIB_RES(3, 0); break;
      case 1: FVIB_RES(3, 1); break;
      case 2: FVIB_RES(3, 2); break;
      default: FVIB_RES(3, 3); break;
    }
  }
#undef FVIB_RES
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_rhs_residual(const Geo<T>& G, const PGeo<double>& P, const T* const us[3],
                        const double* x, double* b, double* r64, float* r32, RedBuf red,
                        SolverScalars* sc, double tol, double max_iv, hipStream_t s,
                        SolverScalars* mirror, const IbView<T>& ib) {
  const ColTiling ct = make_col_tiling(P.n[0], P.n[1], P.n[2]);
  if (G.dim == 2) {
    if (r64)
      launch_kernel((k_rhs_residual_2d<T, 3>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct,
                    us[0], us[1], ib, x, b, r64, r32, red);
    else
      launch_kernel((k_rhs_residual_2d<T, 2>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct,
                    us[0], us[1], ib, x, b, r64, r32, red);
  } else if (ib.active && !ib.box) {
    return FVIB_EINVAL;           // a 3D grid has no immersed rigid body
  } else if (r64)
    launch_kernel((k_rhs_residual_col<T, 3>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct,
                  us[0], us[1], us[2], x, b, r64, r32, red);
  else
    launch_kernel((k_rhs_residual_col<T, 2>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct,
                  us[0], us[1], us[2], x, b, r64, r32, red);
  FVIB_HIP(hipGetLastError());
  FVIB_HIP((launch_finish<4, 3>(red.partial, ct.nblocks, sc,
                                FinRhsResidual{tol, 0.5, P.dt_over_rho, P.inv_ncell, max_iv,
                                               mirror},
                                s)));
  return FVIB_OK;
}

template <typename V>
int launch_cg_iter(const PGeo<V>& P, int mode, const V* r, const V* pold, V* pnew, V* x, V* rw,
                   RedBuf red, SolverScalars* sc, double tol, int maxit, hipStream_t s,
                   hipEvent_t* ev) {
  const Tiling tl = red_tiling(P.n);
  dim3 g(tl.nblocks), bl(kBlock);
  if (ev) FVIB_HIP(hipEventRecord(ev[0], s));
  if (P.dim == 2)
    launch_kernel((k_cg_dir<V, 2>), g, bl, 0, s, P, tl, r, pold, pnew, red, sc);
  else
    launch_kernel((k_cg_dir<V, 3>), g, bl, 0, s, P, tl, r, pold, pnew, red, sc);
  FVIB_HIP(hipGetLastError());
  FVIB_HIP((launch_finish<2, 2>(red.partial, tl.nblocks, sc, FinCgDir{}, s)));
  if (ev) FVIB_HIP(hipEventRecord(ev[1], s));
  if (P.dim == 2) {
    if (mode == 0)
      launch_kernel((k_cg_update<V, 2, 0>), g, bl, 0, s, P, tl, (const V*)pnew, x, rw, red, sc, tol, maxit);
    else
      launch_kernel((k_cg_update<V, 2, 1>), g, bl, 0, s, P, tl, (const V*)pnew, x, rw, red, sc, tol, maxit);
  } else {
    if (mode == 0)
      launch_kernel((k_cg_update<V, 3, 0>), g, bl, 0, s, P, tl, (const V*)pnew, x, rw, red, sc, tol, maxit);
    else
      launch_kernel((k_cg_update<V, 3, 1>), g, bl, 0, s, P, tl, (const V*)pnew, x, rw, red, sc, tol, maxit);
  }
  FVIB_HIP(hipGetLastError());
  if (mode == 0)
    FVIB_HIP((launch_finish<2, 1>(red.partial, tl.nblocks, sc,
                                  FinCgUpdate<0>{tol, P.dt_over_rho, maxit}, s)));
  else
    FVIB_HIP((launch_finish<2, 1>(red.partial, tl.nblocks, sc,
                                  FinCgUpdate<1>{tol, P.dt_over_rho, maxit}, s)));
  if (ev) FVIB_HIP(hipEventRecord(ev[2], s));
  return FVIB_OK;
}

int launch_ir_correct(int64_t n, double* p, const float* d, const SolverScalars* sc,
                      hipStream_t s) {
  int nb = (int)((n + kBlock - 1) / kBlock);
  if (nb > 4 * kMaxRedBlocks) nb = 4 * kMaxRedBlocks;
  launch_kernel(k_ir_correct, dim3(nb), dim3(kBlock), 0, s, n, p, d, sc, 1.0 / (double)n);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template <typename T>
int launch_project(const Geo<T>& G, const PGeo<double>& P, const T* const us[3], const double* p,
                   T* out[3], RedBuf red, SolverScalars* sc, hipStream_t s, double* pg,
                   fvib_step_info* info, int* sticky, const StageMix* mix) {
  const Tiling tl = red_tiling(G.n);
  if (pg && pg == p) return FVIB_EINVAL;
  StageMix m{};
  const bool mx = mix && mix->u0[0];
  if (mx) m = *mix;
  if (G.dim == 2) {
    if (mx)
      launch_kernel((k_project<T, 2, true>), dim3(tl.nblocks), dim3(kBlock), 0, s, G, P, tl,
                    us[0], us[1], us[2], p, out[0], out[1], out[2], red, sc, m, pg);
    else
      launch_kernel((k_project<T, 2, false>), dim3(tl.nblocks), dim3(kBlock), 0, s, G, P, tl,
                    us[0], us[1], us[2], p, out[0], out[1], out[2], red, sc, m, pg);
  } else {
    const ColTiling ct = make_col_tiling(G.n[0], G.n[1], G.n[2]);
    if (mx)
      launch_kernel((k_project_col<T, true>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct,
                    us[0], us[1], us[2], p, out[0], out[1], out[2], red, pg, sc, m);
    else
      launch_kernel((k_project_col<T, false>), dim3(ct.nblocks), dim3(kBlock), 0, s, G, P, ct,
                    us[0], us[1], us[2], p, out[0], out[1], out[2], red, pg, sc, m);
    FVIB_HIP(hipGetLastError());
    FVIB_HIP((launch_finish<1, 0>(red.partial, ct.nblocks, sc, FinDivMax{info, sticky}, s)));
    return FVIB_OK;
  }
  FVIB_HIP(hipGetLastError());
  FVIB_HIP((launch_finish<1, 0>(red.partial, tl.nblocks, sc, FinDivMax{info, sticky}, s)));
  return FVIB_OK;
}

__global__ void __launch_bounds__(kBlock)
k_scale(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * kBlock)
    y[t] = a * x[t];
}

// y = a x + b y over n values of type T (x may be NULL: y = b y; b = 0 does
// not read y)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_axpby(int64_t n, double a, const T* __restrict__ x, double b, T* __restrict__ y) {
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * kBlock)
    y[t] = (T)((x ? a * (double)x[t] : 0.0) + (b != 0.0 ? b * (double)y[t] : 0.0));
}

template <typename T>
int launch_axpby(int64_t n, double a, const T* x, double b, T* y, hipStream_t s) {
  const int64_t nb = std::min<int64_t>((n + kBlock - 1) / kBlock, 8 * kMaxRedBlocks);
  launch_kernel((k_axpby<T>), dim3((int)nb), dim3(kBlock), 0, s, n, a, x, b, y);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

// max over every face value of every component of |u|, then the CFL step
// dt = min(dt_max, cfl h_min / max |u|) into sc->cfl_dt
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_max_speed(int64_t n0, const T* __restrict__ u0, int64_t n1, const T* __restrict__ u1,
            int64_t n2, const T* __restrict__ u2, RedBuf red) {
  double m = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (int64_t t = t0; t < n0; t += stride) m = fmax(m, fabs((double)u0[t]));
  for (int64_t t = t0; t < n1; t += stride) m = fmax(m, fabs((double)u1[t]));
  if (u2)
    for (int64_t t = t0; t < n2; t += stride) m = fmax(m, fabs((double)u2[t]));
  double v[1] = {m};
  block_partials<1, 0>(v, red.partial);
}

struct FinCflDt {
  double cfl, h_min, dt_max;
  __device__ bool skip(const SolverScalars*) const { return false; }
  __device__ void apply(const double* t, SolverScalars* sc) const {
    const double um = t[0];
    sc->cfl_dt = (um > 0.0) ? fmin(dt_max, cfl * h_min / um) : dt_max;
    if (!(um == um)) sc->status = FVIB_ENONFINITE;
  }
};

template <typename T>
int launch_cfl_dt(const int64_t n[3], const T* const u[3], double cfl, double h_min,
                  double dt_max, RedBuf red, SolverScalars* sc, hipStream_t s) {
  const int nb = (int)std::min<int64_t>((n[0] + kBlock - 1) / kBlock, kMaxRedBlocks);
  launch_kernel((k_max_speed<T>), dim3(nb), dim3(kBlock), 0, s, n[0], u[0], n[1], u[1], n[2],
                u[2], red);
  FVIB_HIP(hipGetLastError());
  FVIB_HIP((launch_finish<1, 0>(red.partial, nb, sc, FinCflDt{cfl, h_min, dt_max}, s)));
  return FVIB_OK;
}

template int launch_axpby<float>(int64_t, double, const float*, double, float*, hipStream_t);
template int launch_axpby<double>(int64_t, double, const double*, double, double*, hipStream_t);
template int launch_cfl_dt<float>(const int64_t[3], const float* const[3], double, double, double,
                                  RedBuf, SolverScalars*, hipStream_t);
template int launch_cfl_dt<double>(const int64_t[3], const double* const[3], double, double,
                                   double, RedBuf, SolverScalars*, hipStream_t);

int launch_scale(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  const int64_t nb = std::min<int64_t>((n + kBlock - 1) / kBlock, 8 * kMaxRedBlocks);
  launch_kernel(k_scale, dim3((int)nb), dim3(kBlock), 0, s, n, a, x, y);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

int launch_apply_A(const PGeo<double>& P, const double* x, double* y, hipStream_t s) {
  const Tiling tl = red_tiling(P.n);
  launch_kernel(k_apply_A, dim3(tl.nblocks), dim3(kBlock), 0, s, P, tl, x, y);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template int launch_ppe_rhs<float>(const Geo<float>&, const PGeo<double>&, const float* const[3],
                                   const IbView<float>&, double*, RedBuf, SolverScalars*,
                                   hipStream_t);
template int launch_ppe_rhs<double>(const Geo<double>&, const PGeo<double>&,
                                    const double* const[3], const IbView<double>&, double*,
                                    RedBuf, SolverScalars*, hipStream_t);
template int launch_rhs_residual<float>(const Geo<float>&, const PGeo<double>&,
                                        const float* const[3], const double*, double*, double*,
                                        float*, RedBuf, SolverScalars*, double, double,
                                        hipStream_t, SolverScalars*, const IbView<float>&);
template int launch_rhs_residual<double>(const Geo<double>&, const PGeo<double>&,
                                         const double* const[3], const double*, double*,
                                         double*, float*, RedBuf, SolverScalars*, double, double,
                                         hipStream_t, SolverScalars*, const IbView<double>&);
template int launch_cg_iter<float>(const PGeo<float>&, int, const float*, const float*, float*,
                                   float*, float*, RedBuf, SolverScalars*, double, int,
                                   hipStream_t, hipEvent_t*);
template int launch_cg_iter<double>(const PGeo<double>&, int, const double*, const double*,
                                    double*, double*, double*, RedBuf, SolverScalars*, double,
                                    int, hipStream_t, hipEvent_t*);
template int launch_project<float>(const Geo<float>&, const PGeo<double>&, const float* const[3],
                                   const double*, float* [3], RedBuf, SolverScalars*,
                                   hipStream_t, double*, fvib_step_info*, int*,
                                   const StageMix*);
template int launch_project<double>(const Geo<double>&, const PGeo<double>&,
                                    const double* const[3], const double*, double* [3], RedBuf,
                                    SolverScalars*, hipStream_t, double*, fvib_step_info*,
                                    int*, const StageMix*);

}  // namespace fvib
