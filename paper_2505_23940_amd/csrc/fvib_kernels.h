// Host-side launchers of the fvib kernels (one declaration per entry).
#pragma once

#include <vector>

#include "fvib_internal.h"

namespace fvib {

// Immersed-boundary geometry resident on the device (2D).
struct IbGeo {
  int M;                       // markers
  const double* X0;            // M x 2 reference positions
  const double* ds;            // M arc-length elements
  double xmin0, ymin0;         // lower corner of the reference polygon box
  double xmax0, ymax0;         // its upper corner
  double h;                    // uniform grid spacing
  int margin;                  // cells between the polygon box and the window
  int W[2][2];                 // window widths per component (x, y)
  int ext[2][2];               // array extents per component (x, y)
  const double* fx[2];         // face-point x coordinates per component
  const double* fy[2];         // face-point y coordinates per component
  int* origin;                 // 4 ints: window origin per component
  uint8_t* cls[2];             // window point classes
  int kind;                    // FVIB_BODY_*
  int free_dof[3];
  double m, rho, dt;
};

// The step record from the solver scalars (one thread); a failed status is
// also stored in *sticky (nullable).
__device__ __forceinline__ void put_record(const SolverScalars* sc, fvib_step_info* info,
                                           int cg_iters, int ir_iters, int* sticky,
                                           int cpl_iters) {
  int st = sc->status;
  if (st == FVIB_OK && sc->clamp) st = FVIB_EINVAL;
  if (sticky && st != FVIB_OK) *sticky = st;
  info->status = st;
  info->cg_iters = cg_iters;
  info->ir_iters = ir_iters;
  info->flags = (sc->clamp ? 1 : 0) | (cpl_iters << 8);
  info->res = sc->crit;
  info->div_max = sc->div_max;
  for (int a = 0; a < 3; ++a) info->force[a] = sc->force[a];
  info->xi = cpl_iters ? sc->xi : 0.0;
}

// The 4-point regularised delta of the immersed boundary (Eq. 22): phi of
// the distance in grid spacings, its derivative (s >= 0; the kernel is
// even), the 1D kernel d_h(r) = phi(|r| / h) / h and its derivative in r.
__device__ __forceinline__ double ib_phi4(double s) {
  s = fabs(s);
  if (s <= 1.0) return (3.0 - 2.0 * s + sqrt(1.0 + 4.0 * s - 4.0 * s * s)) / 8.0;
  if (s <= 2.0) return (5.0 - 2.0 * s - sqrt(-7.0 + 12.0 * s - 4.0 * s * s)) / 8.0;
  return 0.0;
}
__device__ __forceinline__ double ib_dphi4(double s) {
  if (s <= 1.0) return (-2.0 + (4.0 - 8.0 * s) / (2.0 * sqrt(1.0 + 4.0 * s - 4.0 * s * s))) / 8.0;
  if (s <= 2.0) return (-2.0 - (12.0 - 8.0 * s) / (2.0 * sqrt(-7.0 + 12.0 * s - 4.0 * s * s))) / 8.0;
  return 0.0;
}
__device__ __forceinline__ double ib_dh(double r, double h) { return ib_phi4(r / h) / h; }
__device__ __forceinline__ double ib_ddh(double r, double h) {
  const double s = fabs(r) / h;
  const double g = ib_dphi4(s) / (h * h);
  return r < 0.0 ? -g : g;
}

// This thread's share of the loads gather of Eq. 20 over the window's
// forcing with the markers at body_pos: q_c += dV_k h^2 sum_faces f d_h d_h
// for the items t, t + nt, ... of the (marker, component, stencil row)
// list (8 M items).
template <typename T>
__device__ __forceinline__ void ib_loads_share(const IbGeo& B, const IbView<T>& ib,
                                               const double* body_pos, int t, int nt,
                                               double q[2]) {
  const double dxb = body_pos[0], dyb = body_pos[1];
  const double h = B.h;
  for (int it = t; it < 8 * B.M; it += nt) {
    const int k = it >> 3, c = (it >> 2) & 1, dj = it & 3;
    const double Xx = B.X0[2 * k] + dxb, Xy = B.X0[2 * k + 1] + dyb;
    const double dV = B.ds[k] * h;
    const int i0 = (int)floor((Xx - B.fx[c][0]) / h) - 1;
    const int j0 = (int)floor((Xy - B.fy[c][0]) / h) - 1;
    const int ox = ib.origin[2 * c], oy = ib.origin[2 * c + 1];
    const int lj = j0 + dj - oy;
    if (lj < 0 || lj >= B.W[c][1]) continue;
    const double wy = ib_dh(B.fy[c][j0 + dj] - Xy, h);
    double acc = 0.0;
    for (int di = 0; di < 4; ++di) {
      const int li = i0 + di - ox;
      if (li < 0 || li >= B.W[c][0]) continue;
      const int l = lj * B.W[c][0] + li;
      if (!ib.cls[c][l]) continue;
      acc += (double)ib.f[c][l] * ib_dh(B.fx[c][i0 + di] - Xx, h) * wy;
    }
    q[c] += acc * (h * h) * dV;
  }
}

// Runge-Kutta stage combination written by the velocity correction:
// out = a u0 + b (corrected field) when u0[0] is not NULL.
struct StageMix {
  const void* u0[3];
  double a, b;
};

// Large-eddy simulation terms on a 3D grid (k_les.hip): Smagorinsky
// viscosity at cell centres, wall-model viscosity on the wall edges of the
// y walls, and the adjoint work arrays.  Edge arrays use the lattice
// (n0 + 1) x (n1 + 1) x (n2 + 1); edge type t = C + A - 1 for the plane of
// axes C < A (0: x-y, 1: x-z, 2: y-z).
template <typename T>
struct LesView {
  int wall;                  // wall model on (walls normal to y, x and z periodic)
  T cs2;                     // C_s^2
  double nu, kappa, B, eps;
  double yw[2];              // matching distance: half height of the wall cells
  double uw[2][3];           // wall velocity per side
  T* nut;                    // cell nu_t
  double* nuw[2][2];         // [0 u / 1 w][side], nz x nx: wall-edge viscosity
  double* upl[2][2];         // u+ of the wall faces (kept for the adjoint)
  double* dupl[2][2];        // du+/dRe there
  T* ge[3];                  // edge: symmetric velocity gradient d_a u_c + d_c u_a
  // adjoint
  T* wcc[3];                 // cell: coefficient of d_c u_c
  T* nbar;                   // cell: nu_t adjoint (normal-stress part)
  T* soff[3];                // cell: strain adjoint of the off-diagonal entries
  T* pe[3];                  // edge: coefficient of the symmetric gradient
  T* qe[3];                  // edge: viscosity adjoint
  double* wown[2][2];        // wall face: adjoint of its own velocity
  double* woth[2][2];        // wall face: adjoint of the averaged other velocity
};

// Forward: nu_t, the wall viscosity and g_c = fb_c + div(2 nu_t S)_c on the
// evolved faces (g_c = fb_c elsewhere; fb may be NULL).
template <typename T>
int launch_les_forward(const Geo<T>& G, const LesView<T>& L, const T* const u[3],
                       const T* const fb[3], T* const g[3], hipStream_t s);
// Adjoint: given gbar (this step's adjoint of g alone), add the subgrid
// term's vector-Jacobian product to ubar and gbar to fbar (entries may be
// NULL); recomputes nu_t and the wall viscosity.
template <typename T>
int launch_les_adjoint(const Geo<T>& G, const LesView<T>& L, const T* const u[3],
                       const T* const gbar[3], T* const ubar[3], T* const fbar[3],
                       hipStream_t s);

// Static box on a 3D grid: windows and face-index ranges per component.
struct BoxGeo {
  int bo[3][3];        // window origin, component c, axis a
  int bw[3][3];        // window extent
  int bs[3][3][2];     // solid face-index range [bs0, bs1) per axis
  int per[3];          // periodic axes
  int nc[3];           // cells per axis (the last face index of a bounded own axis)
  uint8_t* cls[3];     // forced flags of the window faces
};
int launch_box_classify(const BoxGeo& B, hipStream_t s);

// Fast-diagonalisation plan: per-axis eigenbases on the device.
struct FdmDiv {
  int dim, axis;               // axis = last forward axis (dim - 1)
  int n[3];
  const double* lam[3];        // per-axis eigenvalues (ascending, lam[0] = 0)
};

// Uniform axes whose length factors into 2, 3, 5 use an FFT in place of
// the dense contraction with their basis: a real FFT on a periodic axis
// (real Fourier basis), a cosine transform through one FFT on a bounded
// one (cosine basis of the Neumann operator).
struct FftAxis {
  int on;                      // axis transformed by FFT
  int dct;                     // bounded axis: cosine transform
  double a, b;                 // basis scales sqrt(2/N)/sqrt(h), 1/sqrt(N h)
};
// Whether an FFT kernel exists for axis length n.
bool fft_size_ok(int n);

// Mirror-symmetric bounded axis split into even and odd halves (float
// path): half-size operators, row-major H x H, and the mode order
// [even modes | odd modes] of that axis in the transformed array.
template <typename V>
struct FdmSym {
  int on;
  const V* fe;                 // forward even: [s][j] = u_j of even mode s
  const V* fo;                 // forward odd
  const V* ie;                 // inverse even: [j][s] (transpose of fe)
  const V* io;                 // inverse odd
};

template <typename V>
struct FdmPlan {
  int dim;
  int n[3];
  const V* phi[3];             // n x n row-major, column m = mode m
  const V* phiT[3];            // transpose
  FdmDiv div;
  FftAxis fft[3];
  const V* tw[3];              // exp(-2 pi i k / N), k < N, as (re, im) pairs
  const V* dtw[3];             // cosine transform: (cos, sin)(pi m / (2N)), m <= N/2
  FdmSym<V> sym[3];
};

// Whether an axis of length n has a symmetric-split kernel.
bool fdm_sym_size_supported(int n);

// FFT description of a uniform periodic axis of length n and spacing h
// (on = 0 if no FFT kernel exists for n).
FftAxis fft_plan(int n, double h);

// k_fft.hip: mode 0 forward, 1 inverse, 2 forward + division + inverse.
// acc (nullable, contiguous axis, mode 1): store accin + result in acc
// instead of the result in out (accin may equal acc; a skipped launch still
// copies accin into acc when they differ).
template <typename V>
int launch_fft_axis(const FdmPlan<V>& F, int a, int mode, const V* in, V* out, const int* stop,
                    hipStream_t s, double* acc = nullptr, const double* accin = nullptr);
template <typename V>
bool fft_usable(const FdmPlan<V>& F, int a);

// k_momentum.hip
template <typename T>
int launch_predictor(const Geo<T>& G, const T* const u[3], const T* const fb[3], T* out[3],
                     const IbView<T>& ib, int mode, hipStream_t s);
template <typename T>
int launch_boundary(const Geo<T>& G, const Planes& PL, const T* const un[3], T* us[3],
                    RedBuf red, SolverScalars* sc, hipStream_t s);

// k_poisson.hip
template <typename T>
int launch_ppe_rhs(const Geo<T>& G, const PGeo<double>& P, const T* const us[3],
                   const IbView<T>& ib, double* b, RedBuf red, SolverScalars* sc,
                   hipStream_t s);
// first = 0: a refinement sweep launched ahead of the host's check; it
// does nothing once the device scalars say the refinement is finished.
// mirror (nullable): device address of a pinned host SolverScalars that
// receives a copy of the scalars whenever the launch is not skipped.
// tick (nullable): device address of a coherent pinned 64-bit word that
// receives, skipped or not, ticket (low 24 bits) << 40 | converged << 39 |
// min(sweeps, 127) << 32 | the criterion as float bits, in one store.
int launch_residual(const PGeo<double>& P, int mode, const double* b, const double* x,
                    double* r64, float* r32, float* d32, RedBuf red, SolverScalars* sc,
                    double tol, double inner_rtol, hipStream_t s, int first = 1,
                    SolverScalars* mirror = nullptr, unsigned long long* tick = nullptr,
                    unsigned int ticket = 0);
// ev (nullable): three events recorded before the direction kernel, between
// the two kernels and after the update kernel.
template <typename V>
int launch_cg_iter(const PGeo<V>& P, int mode, const V* r, const V* pold, V* pnew, V* x, V* rw,
                   RedBuf red, SolverScalars* sc, double tol, int maxit, hipStream_t s,
                   hipEvent_t* ev);
int launch_ir_correct(int64_t n, double* p, const float* d, const SolverScalars* sc,
                      hipStream_t s);
// pg (nullable, 3D only, distinct from p): also store p minus its mean
// (sc->sumx / ncell) there.  info (nullable): also fill that step record
// from the scalars (refinement sweeps as the iteration count).
template <typename T>
int launch_project(const Geo<T>& G, const PGeo<double>& P, const T* const us[3], const double* p,
                   T* out[3], RedBuf red, SolverScalars* sc, hipStream_t s, double* pg = nullptr,
                   fvib_step_info* info = nullptr, int* sticky = nullptr,
                   const StageMix* mix = nullptr);
int launch_apply_A(const PGeo<double>& P, const double* x, double* y, hipStream_t s);
// Fast diagonalisation: the PPE right-hand side b and the first refinement
// residual r = b - A x (r64 for the double inner solve, else r32) in one
// pass; criterion max |r| / V + |mean b| max_iv.  2D grids take the immersed
// body's forced faces from ib (as launch_ppe_rhs); a 3D grid accepts no
// rigid body (a static box needs no change of the right-hand side).
template <typename T>
int launch_rhs_residual(const Geo<T>& G, const PGeo<double>& P, const T* const us[3],
                        const double* x, double* b, double* r64, float* r32, RedBuf red,
                        SolverScalars* sc, double tol, double max_iv, hipStream_t s,
                        SolverScalars* mirror, const IbView<T>& ib);
// y = a x over n doubles (y may alias x)
int launch_scale(int64_t n, double a, const double* x, double* y, hipStream_t s);
// y = a x + b y over n values (x NULL: y = b y)
template <typename T>
int launch_axpby(int64_t n, double a, const T* x, double b, T* y, hipStream_t s);
// CFL step min(dt_max, cfl h_min / max |u|) into sc->cfl_dt (n: face counts)
template <typename T>
int launch_cfl_dt(const int64_t n[3], const T* const u[3], double cfl, double h_min,
                  double dt_max, RedBuf red, SolverScalars* sc, hipStream_t s);

// k_ib.hip
template <typename T>
int launch_ib_classify(const IbGeo& B, const double* body, T* us0, T* us1, SolverScalars* sc,
                       hipStream_t s);
// Loads of the forcing in the body window with the markers at body_pos
// (force into sc->force; Fin, nullable, replaces it) and, when body_out is
// given, RK4 from body_rk; xi != 0 also stores the coupling error in sc->xi.
// info (nullable): the step record, written by the same launch (in place of
// launch_copy_info when the loads are a step's last launch).
template <typename T>
int launch_loads_body(const IbGeo& B, const IbView<T>& ib, const double* body_pos,
                      const double* body_rk, double* body_out, const double* kc,
                      const double* Fin, int xi, SolverScalars* sc, hipStream_t s,
                      fvib_step_info* info = nullptr, int cg_iters = 0, int ir_iters = 0,
                      int* sticky = nullptr);
// Step record from the solver scalars; a failed status is also stored in
// *sticky (nullable).
int launch_zero_scalars(SolverScalars* sc, hipStream_t s);
int launch_copy_info(const SolverScalars* sc, fvib_step_info* info, int cg_iters, int ir_iters,
                     hipStream_t s, const double* body_src = nullptr, double* body_dst = nullptr,
                     int* sticky = nullptr, int cpl_iters = 0);

// k_adjoint.hip
// RK4^T (parts & 1) and the marker-position part of loads^T (parts & 2) in
// one block; parts & 4 first gathers the step's force from the recomputed
// forcing (else it is read from sc->force).
template <typename T>
int launch_adj_body_loads(const IbGeo& B, const IbView<T>& ib, const double* st_rk,
                          const double* st_pos, const double* stbar_out, const double* dF,
                          const double* kc, double* stbar_rk, double* stbar_pos, double* kcbar,
                          SolverScalars* sc, int parts, hipStream_t s);
// Static box (3D): force F = -rho sum f dv over the forced faces into
// sc->force, and the forcing adjoint -rho dv dF_c on them (dF nullable).
template <typename T>
int launch_box_force(const Geo<double>& G, const IbView<T>& ib, double rho, RedBuf red,
                     SolverScalars* sc, hipStream_t s);
// Forced faces of the box after the predictor: forcing -u*/dt stored, u* = 0.
template <typename T>
int launch_box_fix(const Geo<T>& G, const IbView<T>& ib, T* us[3], hipStream_t s);
// Before the momentum adjoint: ustar_bar = -fbar/dt on the forced faces.
template <typename T>
int launch_box_rbar(const Geo<T>& G, const IbView<T>& ib, T* usb[3], hipStream_t s);
template <typename T>
int launch_box_fbar(const Geo<double>& G, const IbView<T>& ib, double rho, const double* dF,
                    hipStream_t s);
template <typename T>
// Strong coupling: Jacobians of a coupling sub-iteration at the iterate om
// (DF 3 x 6, RF 6 x 3, device) and the fixed-point adjoint lam (6).
int launch_strong_jac(const IbGeo& B, const IbView<T>& ib, const double* om, const double* kc,
                      double* DF, double* RF, hipStream_t s);
int launch_strong_lambda(const double* DF, const double* RF, const double* wbar,
                         const double* ubody, const double* dF, double* lam, SolverScalars* sc,
                         hipStream_t s);
// Fast diagonalisation (2D, or 3D without a rigid body): y = G^T ubar and the
// first residual y - A x of the adjoint solve in one pass (target as
// launch_adj_rhs).
template <typename T>
int launch_adj_rhs_residual(const Geo<T>& G, const PGeo<double>& P, const T* const ub[3],
                            const double* x, double* y, double* r64, float* r32, RedBuf red,
                            SolverScalars* sc, double rtol, double max_iv, hipStream_t s,
                            SolverScalars* mirror);
template <typename T>
// rtol: relative target of the adjoint solve, set on the device as
// rtol * max |y / V| * dt / rho (used by a solve called with tol < 0).
int launch_adj_rhs(const Geo<T>& G, const PGeo<double>& P, const T* const ub[3], double* y,
                   RedBuf red, SolverScalars* sc, double rtol, hipStream_t s);
template <typename T>
// mu is used at zero mean: sc->sumx is its sum (measured by the solve's
// last residual sweep)
// info (nullable): the adjoint step's record, written by block 0 with the
// device's sweep count (and the 6-double body state body_src copied to
// body_dst, zero when body_src is NULL, when body_dst is given).
int launch_adj_ustar(const Geo<T>& G, const PGeo<double>& P, const T* const ub1[3],
                     const double* mu, const IbView<T>& ib, T* usb[3], const SolverScalars* sc,
                     hipStream_t s, fvib_step_info* info = nullptr,
                     const double* body_src = nullptr, double* body_dst = nullptr,
                     int* sticky = nullptr);
template <typename T>
int launch_adj_ubody(const Geo<T>& G, const PGeo<double>& P, const IbGeo& B, const T* const ub1[3],
                     const double* mu, const IbView<T>& ib, double* stbar,
                     const SolverScalars* sc, hipStream_t s);
template <typename T>
int launch_adj_outflow(const Geo<T>& G, const Planes& PL, int mode, T* usb[3], T* ubar[3],
                       RedBuf red, SolverScalars* sc, hipStream_t s);
template <typename T>
int launch_adj_momentum(const Geo<T>& G, const T* const u[3], const T* const usb[3],
                        const IbView<T>& ib, T* ubar[3], T* fbbar[3], hipStream_t s);

// k_fdm.hip
// Whether launch_fdm_axis fuses the last forward and first inverse axis.
template <typename V>
bool fdm_fuses_last_axis(const FdmPlan<V>& F);
// fused (nullable): on the last forward axis, ask for the first inverse
// contraction of the same axis to run in the same launch; *fused tells
// whether it did (out then holds the inverse-transformed values).
// acc (nullable): on an inverse axis, ask for accin + result to be stored
// in the double array acc instead of the result in out (accin nullable:
// acc itself); *accd tells whether it was.
template <typename V>
int launch_fdm_axis(const FdmPlan<V>& F, int a, bool fwd, const V* in, V* out, const int* stop,
                    hipStream_t s, bool* fused = nullptr, double* acc = nullptr,
                    bool* accd = nullptr, const double* accin = nullptr);
// p = pin + d (pin may equal p; with the stop flag set, p = pin)
template <typename V>
int launch_add_correction(int64_t n, double* p, const double* pin, const V* d, const int* stop,
                          hipStream_t s);
int launch_gauge(int64_t n, double* p, const SolverScalars* sc, hipStream_t s);
void axis_eigen(const std::vector<double>& f, bool periodic, std::vector<double>& phi,
                std::vector<double>& lam);
// Even and odd half eigenbases of a mirror-symmetric bounded axis (N even).
void axis_eigen_sym(const std::vector<double>& f, std::vector<double>& ue, std::vector<double>& le,
                    std::vector<double>& uo, std::vector<double>& lo);

// k_loss.hip
template <typename T>
int launch_wall_shear(int nx, int ny, int nz, const T* u, T* ubar, double wlo, double whi,
                      double* J, double* partial, hipStream_t s);
int launch_rms_lift(const double* Fh, int S, int stride, int off, double g, double* J,
                    double* dFh, hipStream_t s);
// Device address of the static scratch of the allocation-free wall-shear
// loss on `device`: looked up once per device by noalloc_scratch_init (the
// device must be current), then returned by noalloc_scratch (nullptr before
// that); *slots receives its capacity in doubles.
int noalloc_scratch_init(int device);
double* noalloc_scratch(int device, int64_t* slots);
// Partial-sum slots a wall-shear launch over an nx x nz wall plane uses.
int64_t wall_shear_slots(int nx, int nz);

}  // namespace fvib
