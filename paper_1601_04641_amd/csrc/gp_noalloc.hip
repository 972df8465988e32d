// gp_raw_sums_noalloc: the observable sums of gp_raw_sums for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  Its kernels are the
// ones gp_raw_sums launches; their reduction scratch (per-block partial sums and the
// final sums) lives in one file-scope device array per GPU instead of a context's
// allocations.  Nothing here calls hipMalloc, hipFree or an allocating library routine.
#include "../../include/gp.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "gp_internal.h"

namespace {

constexpr int kObsBlocks = 2048;  // blocks of the observables kernel (grid-stride: any grid size)
constexpr size_t kScratchDoubles = (size_t)kObsBlocks * 9 + 16;  // partials + final sums: 147,584 B
constexpr int kMaxDevices = 64;

}  // namespace

// Reduction scratch, one copy per GPU, held until the process ends.  Host code never
// uses this name as an address: the per-device pointer from hipGetSymbolAddress is.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {nullptr};

// device address of this GPU's scratch (looked up once per device, with it current)
int scratch_ptr(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return GP_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    double* p = nullptr;
    if (hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return GP_ERR_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GP_OK;
}

bool bad_grid(const gp_params* p) {
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) return true;
  if (!(p->dx > 0) || !(p->dy > 0) || !(p->dz > 0)) return true;
  if (!std::isfinite(p->dx) || !std::isfinite(p->dy) || !std::isfinite(p->dz)) return true;
  if (!(p->nux >= 0) || !(p->nuy >= 0) || !(p->nuz >= 0)) return true;
  if (!std::isfinite(p->nux) || !std::isfinite(p->nuy) || !std::isfinite(p->nuz)) return true;
  return p->precision != GP_C64 && p->precision != GP_C128;
}

}  // namespace

extern "C" int gp_raw_sums_noalloc(const gp_params* p, const void* psi_dev, double* raw_dev, void* hip_stream) {
  if (!p || !psi_dev || !raw_dev || bad_grid(p)) return GP_ERR_INVALID;
  if (p->nx > 2048 || p->ny > 2048 || p->nz > 2048) return GP_ERR_UNSUPPORTED;
  const size_t es = p->precision == GP_C128 ? 16 : 8;
  if (reinterpret_cast<uintptr_t>(psi_dev) % es != 0 || reinterpret_cast<uintptr_t>(raw_dev) % 8 != 0)
    return GP_ERR_INVALID;
  const int64_t npts = (int64_t)p->nx * p->ny * p->nz;
  // the same grid as a context's observables pass, so the sums are bitwise those of
  // gp_raw_sums; it never exceeds the scratch's block count
  const int64_t grid = std::min<int64_t>((npts + 255) / 256, kObsBlocks);
  if (grid < 1 || grid > kObsBlocks) return GP_ERR_UNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return GP_ERR_HIP;
  }
  double* ptr = nullptr;
  int rc = scratch_ptr(dev, &ptr);
  if (rc) return rc;
  gpk::ObsLaunch o{};
  o.psi = psi_dev;
  o.nx = p->nx;
  o.ny = p->ny;
  o.nz = p->nz;
  o.ax = gpk::AxisQ{0.5 * p->nux * p->nux, 0.5 * (p->nx - 1), p->dx};
  o.ay = gpk::AxisQ{0.5 * p->nuy * p->nuy, 0.5 * (p->ny - 1), p->dy};
  o.az = gpk::AxisQ{0.5 * p->nuz * p->nuz, 0.5 * (p->nz - 1), p->dz};
  o.partials = ptr;                       // every block writes its 9 partials: no clearing
  o.grid = (int)grid;
  o.out = ptr + (size_t)kObsBlocks * 9;   // final raw sums, written by one block
  hipStream_t s = (hipStream_t)hip_stream;
  if (gpk::launch_observables(p->precision, o, s) != hipSuccess) return GP_ERR_HIP;
  const double dV = p->dx * p->dy * p->dz;
  const double d2[3] = {p->dx * p->dx, p->dy * p->dy, p->dz * p->dz};
  if (gpk::launch_obs_scale(o.out, raw_dev, dV, d2, s) != hipSuccess) return GP_ERR_HIP;
  return GP_OK;
}
