// Scalar losses used to seed the adjoint: mean wall shear stress of a
// wall-bounded flow and the root-mean-square lift coefficient of a force
// history.  Each writes J and, optionally, its gradient.
#include <algorithm>
#include <mutex>

#include "fvib_kernels.h"

namespace fvib {

// Scratch of the allocation-free wall-shear loss: the block partial sums in
// the layout of block_partials (2 sums x kMaxRedBlocks slots, 32 KiB).  Each
// device holds its own copy until the process ends.  Host code never passes
// the array's name to a kernel: it looks the device address up once per
// device (noalloc_scratch_init) and passes that.
constexpr int kNoAllocSlots = 2 * kMaxRedBlocks;
static __device__ __align__(256) double scratch[kNoAllocSlots];

constexpr int kMaxDevices = 64;
static double* g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

int noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return FVIB_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return FVIB_OK;
  double* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
  g_scratch_ptr[device] = ptr;
  return FVIB_OK;
}

double* noalloc_scratch(int device, int64_t* slots) {
  if (slots) *slots = kNoAllocSlots;
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

// J = (nu / 2) [ <u>_lo / (yc_0 - y_0) + <u>_hi / (y_N - yc_{N-1}) ], the
// x-z means taken over the streamwise faces of the two wall-adjacent rows.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_wall_shear(int nx, int ny, int nz, const T* __restrict__ u, T* __restrict__ ubar, double wlo,
             double whi, double* partial) {
  const int64_t plane = (int64_t)nx * nz;
  double s[2] = {0.0, 0.0};
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < plane;
       r += (int64_t)gridDim.x * kBlock) {
    const int i = (int)(r % nx), k = (int)(r / nx);
    const int64_t lo = ((int64_t)k * ny + 0) * nx + i;
    const int64_t hi = ((int64_t)k * ny + (ny - 1)) * nx + i;
    s[0] += (double)u[lo];
    s[1] += (double)u[hi];
    if (ubar) {
      ubar[lo] = (T)((double)ubar[lo] + wlo / (double)plane);
      ubar[hi] = (T)((double)ubar[hi] + whi / (double)plane);
    }
  }
  block_partials<2, 2>(s, partial);
}

struct FinWallShear {
  double wlo, whi, plane;
  double* J;
  __device__ bool skip(const SolverScalars*) const { return false; }
  __device__ void apply(const double* t, SolverScalars*) const {
    *J = wlo * t[0] / plane + whi * t[1] / plane;
  }
};

// J = sqrt(mean_n C_L^2), C_L = 2 F_y / (rho U^2 D); dJ/dF_y(n) = C_L(n) g / (S J)
// with g = 2 / (rho U^2 D).
__global__ void __launch_bounds__(kBlock)
k_rms_lift(const double* __restrict__ Fh, int S, int stride, int off, double g, double* J,
           double* dFh) {
  double s[1] = {0.0};
  for (int n = threadIdx.x; n < S; n += kBlock) {
    const double cl = g * Fh[(int64_t)n * stride + off];
    s[0] += cl * cl;
  }
  block_sum<1>(s);
  const double j = sqrt(s[0] / (double)S);
  if (threadIdx.x == 0) *J = j;
  if (!dFh) return;
  for (int n = threadIdx.x; n < S; n += kBlock) {
    const double cl = g * Fh[(int64_t)n * stride + off];
    dFh[(int64_t)n * stride + off] = (j > 0.0) ? cl * g / ((double)S * j) : 0.0;
  }
}

static int wall_shear_blocks(int nx, int nz) {
  const int64_t plane = (int64_t)nx * nz;
  return (int)std::min<int64_t>((plane + kBlock - 1) / kBlock, kMaxRedBlocks);
}

// block_partials<2, 2> writes slot q * kMaxRedBlocks + block for q = 0, 1
int64_t wall_shear_slots(int nx, int nz) {
  return (int64_t)kMaxRedBlocks + wall_shear_blocks(nx, nz);
}

template <typename T>
int launch_wall_shear(int nx, int ny, int nz, const T* u, T* ubar, double wlo, double whi,
                      double* J, double* partial, hipStream_t s) {
  const int64_t plane = (int64_t)nx * nz;
  const int nb = wall_shear_blocks(nx, nz);
  launch_kernel((k_wall_shear<T>), dim3(nb), dim3(kBlock), 0, s, nx, ny, nz, u, ubar, wlo,
                     whi, partial);
  FVIB_HIP(hipGetLastError());
  FVIB_HIP((launch_finish<2, 2>(partial, nb, nullptr,
                                FinWallShear{wlo, whi, (double)plane, J}, s)));
  return FVIB_OK;
}

int launch_rms_lift(const double* Fh, int S, int stride, int off, double g, double* J,
                    double* dFh, hipStream_t s) {
  launch_kernel(k_rms_lift, dim3(1), dim3(kBlock), 0, s, Fh, S, stride, off, g, J, dFh);
  FVIB_HIP(hipGetLastError());
  return FVIB_OK;
}

template int launch_wall_shear<float>(int, int, int, const float*, float*, double, double,
                                      double*, double*, hipStream_t);
template int launch_wall_shear<double>(int, int, int, const double*, double*, double, double,
                                       double*, double*, hipStream_t);

}  // namespace fvib
