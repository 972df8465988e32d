// C-ABI of the split-step Crank-Nicolson Gross-Pitaevskii solver (declared in gp.h).
//
// Host side: parameter checks, the per-axis Crank-Nicolson coefficient tables (computed
// in FP64, rounded once to the storage precision), device-resident state, the launch
// sequence of one step, HIP graphs of fixed step counts, per-kernel event timing and the
// FP64 observables.  All compute runs in the HIP kernels of gp_kernels.hip.
#include "../../include/gp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "gp_internal.h"

using gpk::DevState;
typedef std::complex<double> cd;

namespace gpk {

// Constant-pivot Crank-Nicolson solve along one axis (see gp_kernels.hip): c'_inf is the
// root of modulus < 1 of c x^2 + (1+2c) x + c = 0 (taken in the cancellation-free form
// -2c / ((1+2c) +- sqrt((1+2c)^2 - 4c^2))), gamma = 1/(1 + 2c + c c'_inf), a = c gamma,
// b = (1-2c) gamma, kappa = c c'_inf.  omega = kappa w / (1 - kappa w_0) with
// w = A'^{-1} e_0 (forward d_i = gamma a^i, backward w_i = d_i + a w_{i+1}); nw counts
// the leading omega_i above 1/100 of the storage precision's unit roundoff.
void cn_axis_constants(int n, double d, double dt, int mode, int m, bool f32, AxisConst* out) {
  const double k = dt / (4.0 * d * d);
  const cd cc = mode == 0 ? cd(k, 0) : cd(0, k);
  const cd s1 = 1.0 + 2.0 * cc;
  const cd disc = std::sqrt(s1 * s1 - 4.0 * cc * cc);
  const cd q = std::abs(s1 + disc) >= std::abs(s1 - disc) ? s1 + disc : s1 - disc;
  const cd cpinf = -2.0 * cc / q;
  const cd gam = 1.0 / (1.0 + 2.0 * cc + cc * cpinf);
  const cd a = cc * gam, b = (1.0 - 2.0 * cc) * gam, kappa = cc * cpinf;
  cd P(1, 0);
  for (int i = 0; i < m; ++i) P *= a;
  std::vector<cd> w(n);
  cd dd = gam;
  for (int i = 0; i < n; ++i) {
    w[i] = dd;
    dd *= a;
  }
  for (int i = n - 2; i >= 0; --i) w[i] += a * w[i + 1];
  const cd beta = kappa / (1.0 - kappa * w[0]);
  const double thr = 0.01 * (f32 ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53));
  int nw = 0;
  for (int i = 0; i < n; ++i)
    if (std::abs(beta * w[i]) > thr) nw = i + 1;
  auto rnd = [&](cd v) { return f32 ? cd((float)v.real(), (float)v.imag()) : v; };
  const cd rb = rnd(b);
  const cd vals[4] = {rnd(a), rb, f32 ? rnd(b - rb) : cd(0, 0), rnd(P)};
  for (int q2 = 0; q2 < 4; ++q2) {
    out->coef[2 * q2] = vals[q2].real();
    out->coef[2 * q2 + 1] = vals[q2].imag();
  }
  out->nw = nw;
  // truncated back-substitution u_i = sum_{m<=H} a^m d_{i+m}: the dropped tail is at most
  // |a|^(H+1) / (1 - |a|) max|d|; H is the smallest length that puts it below thr
  {
    const double aa = std::abs(a);
    int h = 0;
    double t = aa / (1.0 - aa);
    while (t > thr && h < 64) {
      t *= aa;
      ++h;
    }
    out->hlen = (aa < 1.0) ? h : 64;
  }
  out->omega.resize(nw);
  for (int i = 0; i < nw; ++i) out->omega[i] = beta * w[i];
}

// per-request cap on the library's own device allocations (gp_set_alloc_cap); < 0: none
static std::atomic<int64_t> g_alloc_cap{-1};

hipError_t dev_alloc(void** p, size_t bytes) {
  const int64_t cap = g_alloc_cap.load();
  if (cap >= 0 && (int64_t)bytes > cap) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

void set_alloc_cap(int64_t bytes) { g_alloc_cap.store(bytes < 0 ? -1 : bytes); }

void pack_complex(const std::vector<std::complex<double>>& v, bool f32, std::vector<unsigned char>& out) {
  if (f32) {
    out.resize(v.size() * 2 * sizeof(float));
    float* f = reinterpret_cast<float*>(out.data());
    for (size_t i = 0; i < v.size(); ++i) {
      f[2 * i] = (float)v[i].real();
      f[2 * i + 1] = (float)v[i].imag();
    }
  } else {
    out.resize(v.size() * sizeof(cd));
    std::memcpy(out.data(), v.data(), out.size());
  }
}

}  // namespace gpk


namespace {

constexpr int kGraphSteps = 16;   // steps per captured graph
constexpr int kKinds = 5;         // timing kinds: x, y, z, finalize, other
constexpr int kEventPool = 4096;  // event pairs before a forced harvest

struct Mapping {
  int mx, swx, my, swy;  // x/y: points per thread, segments per wavefront
  int segz, mz;          // z: threads per line (power of two), points per thread
};

struct TimingRec {
  int kind;
  hipEvent_t a, b;
};

}  // namespace

struct gp_ctx {
  gp_params p;
  void* psi = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // private stream used only for graph capture
  int device = 0;
  int64_t npts = 0;
  size_t esize = 0;
  Mapping map{};

  DevState* st = nullptr;      // device
  void* tab[2][3] = {{nullptr}};  // [imag, real][axis]: omega, storage precision, n complex
  int nw[2][3] = {{0}};
  int hlen[2][3] = {{0}};          // truncated back-substitution lengths [imag, real][axis]
  int trunc = 0;                   // 0 exact sweeps; 1 streaming x/y sweeps, truncated back-substitution;
                                   // 2 streaming x sweep + fused y+z pass
  int yz_chunk = 0, yz_nchunks = 0;  // mode 2: rows per block and blocks per plane
  void* work = nullptr;              // mode 2: the x sweep's output, the fused pass's input
  double yzcoef[2][8] = {{0}};       // mode 2: z constants with P = a^mz of the fused kernel
  double coef[2][3][8] = {{{0}}};  // a, b, b_lo, P = a^m as (re, im)
  void* vtab[3] = {nullptr};      // storage-precision 1/2 nu^2 a^2
  double* zpart = nullptr;
  int zgrid = 0;       // z sweep blocks in imaginary time (one FP64 norm partial each)
  int zgrid_real = 0;  // z sweep blocks in real time
  int zw = 4;          // z sweep wavefronts per block (gpk::z_waves)
  int zpart_cap = 0;  // doubles allocated at zpart (z sweep or fused y+z partials)
  double* opart = nullptr;
  int ogrid = 0;
  double* oout = nullptr;
  double* host = nullptr;  // pinned readback buffer (16 doubles)

  hipGraphExec_t gexec[2] = {nullptr, nullptr};  // [imag, real], kGraphSteps steps each
  bool use_graphs = true;

  bool timing = false;
  std::vector<TimingRec> recs;
  std::vector<hipEvent_t> pool;
  double tsum[kKinds] = {0};
  int64_t tcnt[kKinds] = {0};

  int64_t steps_done = 0;
  char err[256] = {0};
};

namespace {

int fail_hip(gp_ctx* c, hipError_t e, const char* where) {
  if (c) snprintf(c->err, sizeof(c->err), "%s: %s", where, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? GP_ERR_OOM : GP_ERR_HIP;
}

#define HIPCHK(c, expr)                                \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return fail_hip(c, e_, #expr); \
  } while (0)

bool bad_params(const gp_params* p) {
  if (!p) return true;
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) return true;
  if (!(p->dx > 0) || !(p->dy > 0) || !(p->dz > 0) || !(p->dt > 0)) return true;
  if (!std::isfinite(p->dx) || !std::isfinite(p->dy) || !std::isfinite(p->dz) || !std::isfinite(p->dt)) return true;
  if (!(p->nux >= 0) || !(p->nuy >= 0) || !(p->nuz >= 0)) return true;
  if (!std::isfinite(p->nux) || !std::isfinite(p->nuy) || !std::isfinite(p->nuz)) return true;
  if (!std::isfinite(p->g)) return true;
  if (p->precision != GP_C64 && p->precision != GP_C128) return true;
  if (p->split != GP_SPLIT_LIE && p->split != GP_SPLIT_STRANG) return true;
  return false;
}

int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Lines of one sweep axis: n points per line, element i of line l at
// (l / inner) n inner + l % inner + i inner.
struct AxisLines {
  int n;
  int64_t inner, nlines;
  size_t esize;
};

AxisLines axis_lines(const gp_params& p, int axis) {
  const size_t es = p.precision == GP_C128 ? 16 : 8;
  if (axis == 0) return AxisLines{p.nx, (int64_t)p.ny * p.nz, (int64_t)p.ny * p.nz, es};
  return AxisLines{p.ny, (int64_t)p.nz, (int64_t)p.nx * p.nz, es};
}

// x/y line mapping: m points per thread (the kernel instance's register count) and sw
// segments per wavefront; a block holds ceil(ceil(n/m)/sw) <= 16 wavefronts.  A
// wavefront addresses its points by 32-bit byte offsets from its first point: its sw*m
// rows plus the spread of its 64/sw lines (which cross into the next plane of the y
// sweep) must stay below 2 GiB.
// Wavefronts whose rows span 2 GiB or more run the 64-bit addressed (WIDE) instances.
bool needs_wide(const AxisLines& a, int m, int sw) {
  const int64_t lw = 64 / sw;
  const int64_t spread = a.nlines > a.inner ? ((lw - 1) / a.inner + 1) * a.inner * a.n : lw - 1;
  return (spread + (int64_t)sw * m * a.inner) * (int64_t)a.esize >= ((int64_t)1 << 31);
}

bool valid_lines(int prec, const AxisLines& a, int m, int sw) {
  if (sw < 1 || sw > 8 || m < 1) return false;
  if (ceil_div(ceil_div(a.n, m), sw) > 16) return false;
  return needs_wide(a, m, sw) ? gpk::sweep_lines_wide_supported(prec, m, sw)
                              : gpk::sweep_lines_supported(prec, m, sw);
}

// Default: 16 points per thread; 4 segments per wavefront once a line has >= 16 segments
// (16-line bundles, 8 wavefronts per block), else the fewest wavefronts-per-segment that
// fit.  complex128 with the fused potential step uses 8 points per thread (register
// budget).  Lines beyond 1024 points (complex64) take 30 or 32 points per thread with 4
// segments per wavefront (128-byte line chunks: 18.7 and 13.5 ms for the x and y sweeps
// of the 1920x1600x1280 grid) before 16 points with 8 segments (64-byte chunks: 31.7 and
// 18.3 ms).  gp_set_mapping / the autotuner can override this.
bool pick_lines(int prec, const AxisLines& a, bool nstep, int* m_out, int* sw_out) {
  const int m0 = (prec == GP_C128 && nstep) ? 8 : 16;
  const int pref_sw = ceil_div(a.n, m0) >= 16 ? 4 : 1;
  auto take = [&](int m, int sw) {
    if (!valid_lines(prec, a, m, sw)) return false;
    *m_out = m;
    *sw_out = sw;
    return true;
  };
  for (int m = m0; m <= 16; m *= 2) {
    if (take(m, pref_sw)) return true;
    for (int sw : {1, 2, 4})
      if (take(m, sw)) return true;
  }
  for (int m : {30, 32})
    for (int sw : {1, 2, 4})
      if (take(m, sw)) return true;
  return take(16, 8);
}

// z mapping: seg threads per line (power of two <= 64), m points per thread (an instance
// size), seg*m >= nz, block LDS (4 wavefronts x 64/seg lines x nz values + 512 B) <= 64 KiB.
// z sweep grid: the blocks that fit on the device at once (LDS bound: each block holds
// 4 L lines of nz points), each walking an equal share of the line groups; a second,
// partial round of blocks would leave most CUs idle at the tail
// complex64 z blocks hold the Sherman-Morrison vector (at most nz values) beside their rows
size_t z_omega_bound(int nz, size_t esize) { return gpk::z_omega_in_lds(esize, 4) ? (size_t)nz * esize : 0; }
int zpad_of(int nz, int seg, int m, size_t esize) {
  return gpk::z_pad(nz, seg, m, esize, gpk::kMaxLdsBlock, z_omega_bound(nz, esize));
}

// z sweep grids.  4-wavefront blocks: complex128 one block per line group (measured
// 723 -> 706 us, with the non-temporal policy 671 -> 654 us on the quench grid); complex64
// the blocks that fit on the device at once, each walking an equal share of the groups
// (one block per group measured 2-4% slower there; a second, partial round of resident
// blocks would leave most CUs idle at the tail).  1-wavefront blocks (long complex128
// lines): one block per group in real time; in imaginary time one block per 16 groups,
// which keeps the norm partials (one per block) few enough for the finalize kernel, but
// never fewer than 8 blocks per CU (a 64^3 grid has 512 groups: 32 blocks measured 57 us
// per sweep against 10 us for 512).
struct ZPlan {
  int zw = 4;
  int64_t groups = 0;
  int grid_imag = 0, grid_real = 0;
};

ZPlan z_plan(const gp_ctx* c, int segz, int mz) {
  ZPlan z;
  const int zpad = zpad_of(c->p.nz, segz, mz, c->esize);
  z.zw = gpk::z_waves(c->p.nz, segz, mz, zpad, c->esize);
  const int64_t per_grp = (int64_t)z.zw * (64 / segz);
  z.groups = ((int64_t)c->p.nx * c->p.ny + per_grp - 1) / per_grp;
  const int64_t one_shot = std::max<int64_t>(1, std::min<int64_t>(z.groups, 0x7fffffff));
  int cus = 0, lds_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1) cus = 256;
  if (z.zw == 1) {
    const int64_t chunked = std::max<int64_t>((z.groups + 15) / 16, (int64_t)8 * cus);
    z.grid_imag = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(z.groups, chunked), 0x7fffffff));
    z.grid_real = (int)one_shot;
    return z;
  }
  if (c->esize == 16) {
    z.grid_imag = z.grid_real = (int)one_shot;
    return z;
  }
  if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->device) != hipSuccess ||
      lds_cu < 65536)
    lds_cu = 65536;
  const int nom = std::max(c->nw[0][2], c->nw[1][2]);
  const size_t lds = gpk::z_lds(c->p.nz, segz, mz, zpad, c->esize, z.zw) +
                     (gpk::z_omega_in_lds(c->esize, z.zw) ? (size_t)nom * c->esize : 0);
  int64_t per_cu = lds_cu / std::max<int64_t>((int64_t)lds + 512, 1);
  per_cu = std::max<int64_t>(1, std::min<int64_t>(per_cu, 8));
  z.grid_imag = z.grid_real = (int)std::max<int64_t>(1, std::min<int64_t>(z.groups, per_cu * cus));
  return z;
}

bool valid_z(int nz, int seg, int m, size_t esize) {
  if (seg < 2 || seg > 64 || (seg & (seg - 1)) != 0) return false;
  if (!gpk::sweep_z_supported(esize == 16 ? 1 : 0, m)) return false;
  if ((size_t)4 * (64 / seg) * nz * esize + z_omega_bound(nz, esize) + 512 > gpk::kMaxLdsBlock) return false;
  return (int64_t)seg * m >= nz;  // trailing positions are zero-coefficient padding
}


bool pick_z(int nz, size_t esize, int* seg_out, int* m_out) {
  const int ms[] = {2, 4, 6, 7, 8, 12, 14, 15, 16, 20, 24, 32};
  int best_seg = 0, best_m = 0;
  long best_score = -1;
  for (int seg = 64; seg >= 2; seg >>= 1)
    for (int m : ms) {
      if (!valid_z(nz, seg, m, esize)) continue;
      const long waste = (long)seg * m - nz;
      const long score = waste * 16 + std::abs(m - 8);
      if (best_score < 0 || score < best_score) {
        best_score = score;
        best_seg = seg;
        best_m = m;
      }
      break;  // smallest m for this seg
    }
  if (best_score < 0) return false;
  *seg_out = best_seg;
  *m_out = best_m;
  return true;
}

int build_axis_table(gp_ctx* c, int mode, int axis) {
  const int n = axis == 0 ? c->p.nx : axis == 1 ? c->p.ny : c->p.nz;
  const double d = axis == 0 ? c->p.dx : axis == 1 ? c->p.dy : c->p.dz;
  const int m = axis == 0 ? c->map.mx : axis == 1 ? c->map.my : c->map.mz;
  const bool f32 = c->p.precision == GP_C64;
  gpk::AxisConst ac;
  gpk::cn_axis_constants(n, d, c->p.dt, mode, m, f32, &ac);
  for (int q = 0; q < 8; ++q) c->coef[mode][axis][q] = ac.coef[q];
  c->nw[mode][axis] = ac.nw;
  c->hlen[mode][axis] = ac.hlen;
  if (ac.nw == 0) return GP_OK;
  std::vector<unsigned char> bytes;
  gpk::pack_complex(ac.omega, f32, bytes);
  HIPCHK(c, hipMemcpy(c->tab[mode][axis], bytes.data(), bytes.size(), hipMemcpyHostToDevice));
  return GP_OK;
}

int build_tables(gp_ctx* c) {
  for (int mode = 0; mode < 2; ++mode)
    for (int a = 0; a < 3; ++a) {
      int rc = build_axis_table(c, mode, a);
      if (rc) return rc;
    }
  return GP_OK;
}

void destroy_graphs(gp_ctx* c) {
  for (auto& g : c->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

gpk::SweepLaunch lines_args(gp_ctx* c, int axis, int mode) {
  gpk::SweepLaunch a{};
  const gp_params& p = c->p;
  a.psi = c->psi;
  a.psi_bytes = c->npts * (int64_t)c->esize;
  a.n = axis == 0 ? p.nx : p.ny;
  a.m = axis == 0 ? c->map.mx : c->map.my;
  a.sw = axis == 0 ? c->map.swx : c->map.swy;
  a.nseg = ceil_div(a.n, a.m);
  for (int q = 0; q < 8; ++q) a.coef[q] = c->coef[mode][axis][q];
  a.omega = c->tab[mode][axis];
  a.nw = c->nw[mode][axis];
  a.nlines = axis == 0 ? (int64_t)p.ny * p.nz : (int64_t)p.nx * p.nz;
  a.inner = axis == 0 ? (int64_t)p.ny * p.nz : (int64_t)p.nz;
  a.wide = needs_wide(axis_lines(p, axis), a.m, a.sw);
  a.hlen = c->hlen[mode][axis];
  a.nstep = 0;
  if (axis == 0) {
    a.nstep = mode == 0 ? 1 : 2;
    a.tau = p.split == GP_SPLIT_LIE ? p.dt : 0.5 * p.dt;
    a.vx = c->vtab[0];
    a.vy = c->vtab[1];
    a.vz = c->vtab[2];
    a.ph = 0.5 * p.nux * p.nux;
    a.pc = 0.5 * (p.nx - 1);
    a.pd = p.dx;
  }
  a.ny = p.ny;
  a.nz = p.nz;
  a.st = c->st;
  return a;
}

gpk::SweepLaunch z_args(gp_ctx* c, int mode) {
  gpk::SweepLaunch a{};
  const gp_params& p = c->p;
  a.psi = c->psi;
  for (int q = 0; q < 8; ++q) a.coef[q] = c->coef[mode][2][q];
  a.omega = c->tab[mode][2];
  a.nw = c->nw[mode][2];
  a.n = p.nz;
  a.m = c->map.mz;
  a.nseg = c->map.segz;
  a.nlines = (int64_t)p.nx * p.ny;
  a.inner = 1;
  a.nstep = p.split == GP_SPLIT_STRANG ? (mode == 0 ? 1 : 2) : 0;
  a.tau = 0.5 * p.dt;
  a.vx = c->vtab[0];
  a.vy = c->vtab[1];
  a.vz = c->vtab[2];
  a.ph = 0.5 * p.nuz * p.nuz;
  a.pc = 0.5 * (p.nz - 1);
  a.pd = p.dz;
  a.ny = p.ny;
  a.nz = p.nz;
  a.st = c->st;
  a.partials = mode == 0 ? c->zpart : nullptr;
  a.grid = mode == 0 ? c->zgrid : c->zgrid_real;
  a.zpad = zpad_of(p.nz, a.nseg, a.m, c->esize);
  a.zw = c->zw;
  return a;
}

hipEvent_t pool_get(gp_ctx* c) {
  if (c->pool.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = c->pool.back();
  c->pool.pop_back();
  return e;
}

int harvest(gp_ctx* c) {
  if (c->recs.empty()) return GP_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& r : c->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->tsum[r.kind] += ms;
      c->tcnt[r.kind] += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->recs.clear();
  return GP_OK;
}

// Launch one kernel (through fn) with optional event bracketing.
template <typename F>
int timed(gp_ctx* c, hipStream_t s, int kind, F fn) {
  if (!c->timing || s != c->stream) {
    hipError_t e = fn(s);
    return e == hipSuccess ? GP_OK : fail_hip(c, e, "kernel launch");
  }
  if ((int)c->recs.size() >= kEventPool) {
    int rc = harvest(c);
    if (rc) return rc;
  }
  hipEvent_t a = pool_get(c), b = pool_get(c);
  if (!a || !b) return fail_hip(c, hipErrorOutOfMemory, "hipEventCreate");
  HIPCHK(c, hipEventRecord(a, s));
  hipError_t e = fn(s);
  if (e != hipSuccess) return fail_hip(c, e, "kernel launch");
  HIPCHK(c, hipEventRecord(b, s));
  c->recs.push_back({kind, a, b});
  return GP_OK;
}

gpk::YZLaunch yz_args(gp_ctx* c, int mode) {
  gpk::YZLaunch a{};
  const gp_params& p = c->p;
  a.src = c->work;
  a.psi = c->psi;
  a.nx = p.nx;
  a.ny = p.ny;
  a.nz = p.nz;
  a.chunk = c->yz_chunk;
  a.nchunks = c->yz_nchunks;
  for (int q = 0; q < 6; ++q) a.ycoef[q] = c->coef[mode][1][q];
  a.yomega = c->tab[mode][1];
  a.ynw = c->nw[mode][1];
  for (int q = 0; q < 8; ++q) a.zcoef[q] = c->yzcoef[mode][q];
  a.zomega = c->tab[mode][2];
  a.znw = c->nw[mode][2];
  a.mz = gpk::yz_mz(p.nz);
  a.hlen = c->hlen[mode][1];
  a.epi = p.split == GP_SPLIT_STRANG ? (mode == 0 ? 1 : 2) : 0;
  a.ph = 0.5 * p.nuz * p.nuz;
  a.pc = 0.5 * (p.nz - 1);
  a.pd = p.dz;
  a.tau = 0.5 * p.dt;
  a.vx = c->vtab[0];
  a.vy = c->vtab[1];
  a.st = c->st;
  a.partials = mode == 0 ? c->zpart : nullptr;
  return a;
}

// One full step on stream s. mode 0 imaginary (renormalising), 1 real.
int enqueue_step(gp_ctx* c, int mode, hipStream_t s) {
  const int prec = c->p.precision;
  const bool cc = mode == 1;
  if (c->trunc == 2) {  // exact x sweep psi -> work, then the fused y+z pass work -> psi
    gpk::SweepLaunch ax = lines_args(c, 0, mode);
    ax.dst = c->work;
    gpk::YZLaunch ayz = yz_args(c, mode);
    int rc = timed(c, s, 0, [&](hipStream_t t) { return gpk::launch_sweep_lines(prec, cc, ax, t); });
    if (rc) return rc;
    rc = timed(c, s, 2, [&](hipStream_t t) { return gpk::launch_stream_yz(prec, cc, ayz, t); });
    if (rc) return rc;
    if (mode == 0) {
      const double dV = c->p.dx * c->p.dy * c->p.dz;
      const int nb = c->p.nx * c->yz_nchunks;
      rc = timed(c, s, 3, [&](hipStream_t t) {
        return gpk::launch_finalize_norm(c->zpart, nb, dV, c->p.dt, c->st, t);
      });
    }
    return rc;
  }
  gpk::SweepLaunch ax = lines_args(c, 0, mode), ay = lines_args(c, 1, mode), az = z_args(c, mode);
  auto lines = c->trunc ? gpk::launch_stream_lines : gpk::launch_sweep_lines;
  int rc = timed(c, s, 0, [&](hipStream_t t) { return lines(prec, cc, ax, t); });
  if (rc) return rc;
  rc = timed(c, s, 1, [&](hipStream_t t) { return lines(prec, cc, ay, t); });
  if (rc) return rc;
  rc = timed(c, s, 2, [&](hipStream_t t) { return gpk::launch_sweep_z(prec, cc, az, t); });
  if (rc) return rc;
  if (mode == 0) {
    const double dV = c->p.dx * c->p.dy * c->p.dz;
    rc = timed(c, s, 3, [&](hipStream_t t) {
      return gpk::launch_finalize_norm(c->zpart, c->zgrid, dV, c->p.dt, c->st, t);
    });
    if (rc) return rc;
  }
  return GP_OK;
}

int ensure_graph(gp_ctx* c, int mode) {
  if (c->gexec[mode]) return GP_OK;
  if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  int rc = GP_OK;
  for (int k = 0; k < kGraphSteps && rc == GP_OK; ++k) rc = enqueue_step(c, mode, c->cap);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail_hip(c, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&c->gexec[mode], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->gexec[mode] = nullptr;
    return fail_hip(c, e, "hipGraphInstantiate");
  }
  return GP_OK;
}

int run_steps(gp_ctx* c, int mode, int32_t n) {
  int32_t left = n;
  if (c->use_graphs && !c->timing && n >= kGraphSteps) {
    int rc = ensure_graph(c, mode);
    if (rc) return rc;
    while (left >= kGraphSteps) {
      HIPCHK(c, hipGraphLaunch(c->gexec[mode], c->stream));
      left -= kGraphSteps;
    }
  }
  for (int32_t k = 0; k < left; ++k) {
    int rc = enqueue_step(c, mode, c->stream);
    if (rc) return rc;
  }
  c->steps_done += n;
  return GP_OK;
}

int observe(gp_ctx* c, double raw[9]) {
  gpk::ObsLaunch o{};
  o.psi = c->psi;
  o.nx = c->p.nx;
  o.ny = c->p.ny;
  o.nz = c->p.nz;
  o.ax = gpk::AxisQ{0.5 * c->p.nux * c->p.nux, 0.5 * (c->p.nx - 1), c->p.dx};
  o.ay = gpk::AxisQ{0.5 * c->p.nuy * c->p.nuy, 0.5 * (c->p.ny - 1), c->p.dy};
  o.az = gpk::AxisQ{0.5 * c->p.nuz * c->p.nuz, 0.5 * (c->p.nz - 1), c->p.dz};
  o.partials = c->opart;
  o.grid = c->ogrid;
  o.out = c->oout;
  int rc = timed(c, c->stream, 4, [&](hipStream_t t) { return gpk::launch_observables(c->p.precision, o, t); });
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->host, c->oout, 9 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double dV = c->p.dx * c->p.dy * c->p.dz;
  const double d2[3] = {c->p.dx * c->p.dx, c->p.dy * c->p.dy, c->p.dz * c->p.dz};
  raw[0] = c->host[0] * dV;
  for (int a = 0; a < 3; ++a) raw[1 + a] = 0.5 * c->host[1 + a] * dV / d2[a];
  for (int q = 4; q < 9; ++q) raw[q] = c->host[q] * dV;
  for (int q = 0; q < 9; ++q)
    if (!std::isfinite(raw[q])) return GP_ERR_NONFINITE;
  if (!(raw[0] > 0)) return GP_ERR_ZERO_NORM;
  return GP_OK;
}

template <typename T>
int dalloc(gp_ctx* c, T** p, size_t bytes) {
  hipError_t e = gpk::dev_alloc((void**)p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail_hip(c, e, "hipMalloc");
  }
  return GP_OK;
}

void release(gp_ctx* c) {
  destroy_graphs(c);
  for (auto& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  (void)hipFree(c->st);
  for (auto& m : c->tab)
    for (auto p : m) (void)hipFree(p);
  for (int a = 0; a < 3; ++a) {
    (void)hipFree(c->vtab[a]);
  }
  (void)hipFree(c->zpart);
  (void)hipFree(c->work);
  (void)hipFree(c->opart);
  (void)hipFree(c->oout);
  if (c->host) (void)hipHostFree(c->host);
}

int check_psi(gp_ctx* c, void* psi) {
  if (!psi) return GP_ERR_INVALID;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, psi) != hipSuccess) {
    (void)hipGetLastError();
    snprintf(c->err, sizeof(c->err), "psi is not a HIP device pointer");
    return GP_ERR_INVALID;
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) {
    snprintf(c->err, sizeof(c->err), "psi is not device memory");
    return GP_ERR_INVALID;
  }
  if (attr.device != c->device) {
    snprintf(c->err, sizeof(c->err), "psi lives on device %d, context on device %d", attr.device, c->device);
    return GP_ERR_INVALID;
  }
  if (reinterpret_cast<uintptr_t>(psi) % c->esize != 0) {
    snprintf(c->err, sizeof(c->err), "psi is not aligned to its complex element size");
    return GP_ERR_INVALID;
  }
  // the grid must end inside the device allocation that holds psi (when the runtime
  // can name that allocation)
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, psi) == hipSuccess && base) {
    const uintptr_t end = reinterpret_cast<uintptr_t>(base) + size;
    if (reinterpret_cast<uintptr_t>(psi) + (uintptr_t)c->npts * c->esize > end) {
      snprintf(c->err, sizeof(c->err), "psi's allocation is smaller than the %lld-point grid",
               (long long)c->npts);
      return GP_ERR_INVALID;
    }
  } else {
    (void)hipGetLastError();
  }
  return GP_OK;
}

// default mapping of a grid; false where no kernel instance covers one of its axes
bool pick_mapping(const gp_params& p, Mapping* m) {
  return pick_lines(p.precision, axis_lines(p, 0), true, &m->mx, &m->swx) &&
         pick_lines(p.precision, axis_lines(p, 1), false, &m->my, &m->swy) &&
         pick_z(p.nz, p.precision == GP_C128 ? 16 : 8, &m->segz, &m->mz);
}

int init_body(gp_ctx* c) {
  const gp_params& p = c->p;
  if (!pick_mapping(p, &c->map)) {
    snprintf(c->err, sizeof(c->err), "grid %dx%dx%d exceeds the supported line lengths", p.nx, p.ny, p.nz);
    return GP_ERR_UNSUPPORTED;
  }
  const int n[3] = {p.nx, p.ny, p.nz};
  const double d[3] = {p.dx, p.dy, p.dz};
  const double nu[3] = {p.nux, p.nuy, p.nuz};
  int rc;
  if ((rc = dalloc(c, &c->st, sizeof(DevState)))) return rc;
  for (int mode = 0; mode < 2; ++mode)
    for (int a = 0; a < 3; ++a)
      if ((rc = dalloc(c, &c->tab[mode][a], (size_t)n[a] * c->esize))) return rc;
  for (int a = 0; a < 3; ++a) {
    if ((rc = dalloc(c, &c->vtab[a], (size_t)n[a] * c->esize / 2))) return rc;
    std::vector<double> v(n[a]);
    std::vector<float> vf(n[a]);
    for (int i = 0; i < n[a]; ++i) {
      const double x = (i - 0.5 * (n[a] - 1)) * d[a];
      v[i] = 0.5 * nu[a] * nu[a] * x * x;
      vf[i] = (float)v[i];
    }
    if (p.precision == GP_C128)
      HIPCHK(c, hipMemcpy(c->vtab[a], v.data(), n[a] * sizeof(double), hipMemcpyHostToDevice));
    else
      HIPCHK(c, hipMemcpy(c->vtab[a], vf.data(), n[a] * sizeof(float), hipMemcpyHostToDevice));
  }
  if ((rc = build_tables(c))) return rc;
  const ZPlan zp = z_plan(c, c->map.segz, c->map.mz);
  c->zw = zp.zw;
  c->zgrid = zp.grid_imag;
  c->zgrid_real = zp.grid_real;
  const int64_t oblocks = (c->npts + 255) / 256;
  c->ogrid = (int)std::min<int64_t>(oblocks, 2048);
  if ((rc = dalloc(c, &c->zpart, (size_t)c->zgrid * sizeof(double)))) return rc;
  c->zpart_cap = c->zgrid;
  if ((rc = dalloc(c, &c->opart, (size_t)c->ogrid * 9 * sizeof(double)))) return rc;
  if ((rc = dalloc(c, &c->oout, 16 * sizeof(double)))) return rc;
  HIPCHK(c, hipHostMalloc((void**)&c->host, 16 * sizeof(double), hipHostMallocDefault));
  DevState s0{};
  s0.s = 1.0;
  s0.g = p.g;
  s0.npre = 1.0;
  HIPCHK(c, hipMemcpy(c->st, &s0, sizeof(s0), hipMemcpyHostToDevice));
  return GP_OK;
}

}  // namespace

extern "C" {

int gp_init(const gp_params* p, void* psi_dev, void* hip_stream, gp_ctx** out) {
  if (!out) return GP_ERR_INVALID;
  *out = nullptr;
  if (bad_params(p) || !psi_dev) return GP_ERR_INVALID;
  if (p->nx > 2048 || p->ny > 2048 || p->nz > 2048) return GP_ERR_UNSUPPORTED;
  Mapping m0{};
  if (!pick_mapping(*p, &m0)) return GP_ERR_UNSUPPORTED;
  gp_ctx* c = new (std::nothrow) gp_ctx;
  if (!c) return GP_ERR_OOM;
  c->p = *p;
  c->stream = (hipStream_t)hip_stream;
  c->npts = (int64_t)p->nx * p->ny * p->nz;
  c->esize = p->precision == GP_C128 ? 16 : 8;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return GP_ERR_HIP;
  }
  int rc = check_psi(c, psi_dev);
  if (rc == GP_OK) {
    c->psi = psi_dev;
    rc = init_body(c);
  }
  if (rc != GP_OK) {
    release(c);
    delete c;
    return rc;
  }
  *out = c;
  return GP_OK;
}

int gp_destroy(gp_ctx* c) {
  if (!c) return GP_ERR_INVALID;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  release(c);
  delete c;
  return GP_OK;
}

int gp_step_imag(gp_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return GP_ERR_INVALID;
  if (nsteps == 0) return GP_OK;
  int rc = run_steps(c, 0, nsteps);
  if (rc) return rc;
  // psi is kept unnormalised between steps (the scale rides into the next potential
  // step); apply it so the caller sees dV sum|psi|^2 = 1.
  return timed(c, c->stream, 4, [&](hipStream_t t) {
    return gpk::launch_scale(c->p.precision, c->psi, c->npts, c->st, t);
  });
}

int gp_step_real(gp_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return GP_ERR_INVALID;
  if (nsteps == 0) return GP_OK;
  return run_steps(c, 1, nsteps);
}

int gp_raw_sums(gp_ctx* c, double raw[9]) {
  if (!c || !raw) return GP_ERR_INVALID;
  return observe(c, raw);
}

int gp_norm(gp_ctx* c, double* norm) {
  if (!c || !norm) return GP_ERR_INVALID;
  double r[9];
  int rc = observe(c, r);
  *norm = r[0];
  return rc;
}

int gp_energy_mu(gp_ctx* c, double* energy, double* mu) {
  if (!c || !energy || !mu) return GP_ERR_INVALID;
  double r[9];
  int rc = observe(c, r);
  if (rc) return rc;
  const double N = r[0];
  const double lin = (r[1] + r[2] + r[3] + r[4]) / N;
  const double nl = c->p.g * r[5] / (N * N);
  *energy = lin + 0.5 * nl;
  *mu = lin + nl;
  return GP_OK;
}

int gp_rms(gp_ctx* c, double rms[4]) {
  if (!c || !rms) return GP_ERR_INVALID;
  double r[9];
  int rc = observe(c, r);
  if (rc) return rc;
  const double N = r[0];
  rms[0] = std::sqrt(r[6] / N);
  rms[1] = std::sqrt(r[7] / N);
  rms[2] = std::sqrt(r[8] / N);
  rms[3] = std::sqrt((r[6] + r[7] + r[8]) / N);
  return GP_OK;
}

int gp_set_g(gp_ctx* c, double g) {
  if (!c || !std::isfinite(g)) return GP_ERR_INVALID;
  c->p.g = g;
  c->host[12] = g;  // staged in pinned memory so the copy is stream-ordered
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpyAsync(&c->st->g, &c->host[12], sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return GP_OK;
}

int gp_set_psi(gp_ctx* c, void* psi_dev) {
  if (!c) return GP_ERR_INVALID;
  int rc = check_psi(c, psi_dev);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->psi = psi_dev;
  destroy_graphs(c);
  return GP_OK;
}

int gp_status(gp_ctx* c, int64_t* steps_done, double* mu_est, int32_t* flags) {
  if (!c) return GP_ERR_INVALID;
  DevState s{};
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(&s, c->st, sizeof(s), hipMemcpyDeviceToHost));
  if (steps_done) *steps_done = c->steps_done;
  if (mu_est) *mu_est = s.mu_est;
  if (flags) *flags = s.flags;
  return GP_OK;
}

int gp_converge_imag(gp_ctx* c, double tol, int32_t check_every, int64_t max_steps, int64_t* steps_taken,
                     double* mu, int32_t* converged) {
  if (!c || !(tol > 0) || max_steps < 0) return GP_ERR_INVALID;
  int32_t K = check_every > 0 ? check_every : (int32_t)std::ceil(0.25 / c->p.dt);
  if (K < 1) K = 1;
  // complex128: the per-check value is the free estimate mu_est = -ln(N_pre)/(2 dt) of the
  // renormalisation (a 40-byte read instead of an observables pass); when it meets the
  // stopping rule, mu itself is evaluated now and after one more check interval, and that
  // change (with the tail the estimate's contraction ratio predicts) must meet tol too.
  // complex64: mu every check (the FP32 rounding of N_pre makes mu_est too noisy).
  const bool est = c->p.precision == GP_C128;
  gpk::StopRule rule;
  int64_t done = 0;
  double cur = NAN, e = 0;
  int32_t conv = 0;
  bool have_mu = false;
  int rc = GP_OK;
  auto advance = [&](int64_t* d) {
    const int32_t n = (int32_t)std::min<int64_t>(K, max_steps - *d);
    int r2 = gp_step_imag(c, n);
    *d += n;
    return r2;
  };
  while (done < max_steps) {
    if ((rc = advance(&done))) return rc;
    double v = NAN;
    have_mu = false;
    if (est) {
      if ((rc = gp_status(c, nullptr, &v, nullptr))) return rc;
    } else {
      if ((rc = gp_energy_mu(c, &e, &cur))) return rc;
      v = cur;
      have_mu = true;
    }
    if (!rule.update(v, tol)) continue;
    if (!est) {
      conv = 1;
      break;
    }
    if ((rc = gp_energy_mu(c, &e, &cur))) return rc;
    have_mu = true;
    if (done >= max_steps) break;
    const double m0 = cur;
    if ((rc = advance(&done))) return rc;
    if ((rc = gp_energy_mu(c, &e, &cur))) return rc;
    const double d = cur - m0, lim = tol * std::fabs(cur);
    if (std::fabs(d) <= lim && rule.tail(d) <= 0.5 * lim) {
      conv = 1;
      break;
    }
    rule.reset();  // not yet: monitor again from fresh estimates
  }
  if (!have_mu && (rc = gp_energy_mu(c, &e, &cur))) return rc;
  if (steps_taken) *steps_taken = done;
  if (mu) *mu = cur;
  if (converged) *converged = conv;
  return GP_OK;
}

int gp_stop_rule_eval(const double* values, int32_t n, double tol, int32_t* stop_index) {
  if (n < 0 || (n > 0 && (!values || !stop_index))) return GP_ERR_INVALID;
  if (stop_index) *stop_index = -1;
  gpk::StopRule rule;
  for (int32_t k = 0; k < n; ++k)
    if (rule.update(values[k], tol)) {
      *stop_index = k;
      break;
    }
  return GP_OK;
}

int gp_set_timing(gp_ctx* c, int32_t enable) {
  if (!c) return GP_ERR_INVALID;
  int rc = harvest(c);
  if (rc) return rc;
  c->timing = enable != 0;
  for (int k = 0; k < kKinds; ++k) {
    c->tsum[k] = 0;
    c->tcnt[k] = 0;
  }
  return GP_OK;
}

int gp_get_timing(gp_ctx* c, double ms_mean[5], int64_t launches[5]) {
  if (!c) return GP_ERR_INVALID;
  int rc = harvest(c);
  if (rc) return rc;
  for (int k = 0; k < kKinds; ++k) {
    if (ms_mean) ms_mean[k] = c->tcnt[k] ? c->tsum[k] / c->tcnt[k] : 0.0;
    if (launches) launches[k] = c->tcnt[k];
  }
  return GP_OK;
}

int gp_get_mapping(gp_ctx* c, int32_t map[6]) {
  if (!c || !map) return GP_ERR_INVALID;
  map[0] = c->map.mx;
  map[1] = c->map.swx;
  map[2] = c->map.my;
  map[3] = c->map.swy;
  map[4] = c->map.segz;
  map[5] = c->map.mz;
  return GP_OK;
}

int gp_set_mapping(gp_ctx* c, const int32_t map[6]) {
  if (!c || !map) return GP_ERR_INVALID;
  Mapping nm = c->map;
  const int prec = c->p.precision;
  // x and y: points per thread and segments per wavefront (0 keeps the current value)
  auto lines = [&](int axis, int m_in, int sw_in, int* m, int* sw) {
    const AxisLines al = axis_lines(c->p, axis);
    const int mm = m_in > 0 ? m_in : *m;  // must be an instance size (sweep_lines_supported)
    if (sw_in > 0) {
      if (!valid_lines(prec, al, mm, sw_in)) return false;
      *m = mm;
      *sw = sw_in;
      return true;
    }
    for (int s : {1, 2, 4, 8})
      if (valid_lines(prec, al, mm, s)) {
        *m = mm;
        *sw = s;
        return true;
      }
    return false;
  };
  if ((map[0] > 0 || map[1] > 0) && !lines(0, map[0], map[1], &nm.mx, &nm.swx)) return GP_ERR_INVALID;
  if ((map[2] > 0 || map[3] > 0) && !lines(1, map[2], map[3], &nm.my, &nm.swy)) return GP_ERR_INVALID;
  if (map[4] > 0 || map[5] > 0) {
    const int seg = map[4] > 0 ? map[4] : nm.segz;
    int m = map[5];
    if (m <= 0) {  // smallest instance size that covers the line
      for (int cand : {2, 4, 6, 7, 8, 12, 14, 15, 16, 20, 24, 32})
        if ((int64_t)seg * cand >= c->p.nz && gpk::sweep_z_supported(c->esize == 16 ? 1 : 0, cand)) {
          m = cand;
          break;
        }
    }
    if (!valid_z(c->p.nz, seg, m, c->esize)) return GP_ERR_INVALID;
    nm.segz = seg;
    nm.mz = m;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const Mapping old = c->map;
  c->map = nm;
  const ZPlan zp = z_plan(c, nm.segz, nm.mz);
  const int zgrid = zp.grid_imag;
  if (zgrid > c->zpart_cap) {
    double* np = nullptr;
    int rc = dalloc(c, &np, (size_t)zgrid * sizeof(double));
    if (rc) {
      c->map = old;
      return rc;
    }
    (void)hipFree(c->zpart);
    c->zpart = np;
    c->zpart_cap = zgrid;
  }
  const int old_zgrid = c->zgrid, old_zgrid_real = c->zgrid_real, old_zw = c->zw;
  c->zgrid = zgrid;
  c->zgrid_real = zp.grid_real;
  c->zw = zp.zw;
  destroy_graphs(c);
  int rc = build_tables(c);
  if (rc) {  // back to the previous mapping (its tables fit: they were built before)
    c->map = old;
    c->zgrid = old_zgrid;
    c->zgrid_real = old_zgrid_real;
    c->zw = old_zw;
    (void)build_tables(c);
  }
  return rc;
}

// ---------------------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------------------
namespace {

struct TuneKey {
  int nx, ny, nz, prec, mode;
};

bool cache_lookup(const char* path, const TuneKey& k, int32_t map[6]) {
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    TuneKey e;
    int32_t m[6];
    if (sscanf(line, "gfx950 %d %d %d %d %d : %d %d %d %d %d %d", &e.nx, &e.ny, &e.nz, &e.prec, &e.mode, &m[0],
               &m[1], &m[2], &m[3], &m[4], &m[5]) == 11 &&
        e.nx == k.nx && e.ny == k.ny && e.nz == k.nz && e.prec == k.prec && e.mode == k.mode) {
      for (int q = 0; q < 6; ++q) map[q] = m[q];
      found = true;  // the last matching entry wins
    }
  }
  fclose(f);
  return found;
}

void cache_store(const char* path, const TuneKey& k, const int32_t map[6]) {
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "gfx950 %d %d %d %d %d : %d %d %d %d %d %d\n", k.nx, k.ny, k.nz, k.prec, k.mode, map[0], map[1], map[2],
          map[3], map[4], map[5]);
  fclose(f);
}

// Mean duration (ms) of kernel kind `kind` over `steps` steps with mapping `map`.
int time_mapping(gp_ctx* c, int mode, const int32_t map[6], int kind, int steps, double* ms) {
  int rc = gp_set_mapping(c, map);
  if (rc) return rc;
  if ((rc = run_steps(c, mode, 2))) return rc;
  if ((rc = gp_set_timing(c, 1))) return rc;
  if ((rc = run_steps(c, mode, steps))) return rc;
  double mean[5];
  int64_t n[5];
  if ((rc = gp_get_timing(c, mean, n))) return rc;
  *ms = mean[kind];
  return gp_set_timing(c, 0);
}

}  // namespace

extern "C" int gp_autotune(gp_ctx* c, int32_t mode, int32_t steps, const char* cache_path, int32_t map_out[6]) {
  if (!c || (mode != 0 && mode != 1) || steps < 1) return GP_ERR_INVALID;
  const TuneKey key{c->p.nx, c->p.ny, c->p.nz, c->p.precision, mode};
  int32_t best[6];
  if (cache_lookup(cache_path, key, best)) {
    int rc = gp_set_mapping(c, best);
    if (rc == GP_OK) {
      if (map_out)
        for (int q = 0; q < 6; ++q) map_out[q] = best[q];
      return GP_OK;
    }
  }
  // work on the caller's psi, then restore it, the device state, the step count, the
  // mapping and the timing switch on every path out
  int32_t orig[6];
  gp_get_mapping(c, orig);
  const bool timing0 = c->timing;
  const int64_t steps_done = c->steps_done;
  const size_t bytes = (size_t)c->npts * c->esize;
  void* saved = nullptr;
  int rc = dalloc(c, &saved, bytes);
  if (rc) return rc;
  DevState st0{};
  bool have_copy = false;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemcpy(&st0, c->st, sizeof(st0), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpyAsync(saved, c->psi, bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) rc = fail_hip(c, e, "autotune: saving psi");
  else have_copy = true;
  const int prec = c->p.precision;
  for (int q = 0; q < 6; ++q) best[q] = orig[q];
  double best_ms[3] = {1e300, 1e300, 1e300};
  const int ms_lines[] = {8, 10, 12, 16, 30, 32};
  for (int axis = 0; axis < 2 && rc == GP_OK; ++axis) {
    const AxisLines al = axis_lines(c->p, axis);
    for (int m : ms_lines)
      for (int sw : {1, 2, 4, 8}) {
        if (!valid_lines(prec, al, m, sw)) continue;
        int32_t cand[6];
        for (int q = 0; q < 6; ++q) cand[q] = best[q];
        cand[2 * axis] = m;
        cand[2 * axis + 1] = sw;
        double ms = 0;
        rc = time_mapping(c, mode, cand, axis, steps, &ms);
        if (rc) break;
        if (ms < best_ms[axis]) {
          best_ms[axis] = ms;
          best[2 * axis] = m;
          best[2 * axis + 1] = sw;
        }
      }
  }
  for (int seg = 2; seg <= 64 && rc == GP_OK; seg <<= 1)
    for (int m : {2, 4, 6, 7, 8, 12, 14, 15, 16, 20, 24, 32}) {
      if (!valid_z(c->p.nz, seg, m, c->esize)) continue;
      if ((int64_t)seg * m - c->p.nz >= m) continue;  // a whole trailing segment would be empty
      int32_t cand[6];
      for (int q = 0; q < 6; ++q) cand[q] = best[q];
      cand[4] = seg;
      cand[5] = m;
      double ms = 0;
      rc = time_mapping(c, mode, cand, 2, steps, &ms);
      if (rc) break;
      if (ms < best_ms[2]) {
        best_ms[2] = ms;
        best[4] = seg;
        best[5] = m;
      }
    }
  // timing off (drops any pending events), then the winner or, on failure, the original
  (void)gp_set_timing(c, 0);
  if (rc == GP_OK) rc = gp_set_mapping(c, best);
  if (rc != GP_OK) (void)gp_set_mapping(c, orig);
  if (have_copy) {
    (void)hipMemcpyAsync(c->psi, saved, bytes, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(c->st, &st0, sizeof(st0), hipMemcpyHostToDevice, c->stream);
  }
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(saved);
  c->steps_done = steps_done;
  (void)gp_set_timing(c, timing0 ? 1 : 0);
  if (rc) return rc;
  cache_store(cache_path, key, best);
  if (map_out)
    for (int q = 0; q < 6; ++q) map_out[q] = best[q];
  return GP_OK;
}

int gp_set_truncation(gp_ctx* c, int32_t mode) {
  if (!c || mode < 0 || mode > 2) return GP_ERR_INVALID;
  const gp_params& p = c->p;
  for (int m = 0; m < 2 && mode == 1; ++m)
    for (int a = 0; a < 2; ++a)
      if (gpk::stream_h(c->hlen[m][a]) < 0) {
        snprintf(c->err, sizeof(c->err), "truncation length %d exceeds the streaming kernels' 15", c->hlen[m][a]);
        return GP_ERR_UNSUPPORTED;
      }
  int chunk = 0, nchunks = 0;
  if (mode == 2) {
    if (gpk::yz_mz(p.nz) < 0) {
      snprintf(c->err, sizeof(c->err), "the fused y+z pass holds z lines of at most 1024 points");
      return GP_ERR_UNSUPPORTED;
    }
    int nwy = 0;
    for (int m = 0; m < 2; ++m) {
      if (gpk::yz_h(c->hlen[m][1]) < 0) {
        snprintf(c->err, sizeof(c->err), "y truncation length %d exceeds the fused kernels' 15", c->hlen[m][1]);
        return GP_ERR_UNSUPPORTED;
      }
      nwy = std::max(nwy, c->nw[m][1]);
      const size_t lds = gpk::yz_lds(p.nz, c->hlen[m][1], c->esize, c->nw[m][2]);
      if (lds > gpk::kMaxLdsBlock) {  // the rows of one group of z lines must fit one block's LDS
        snprintf(c->err, sizeof(c->err), "the fused y+z pass would need %zu bytes of LDS per block (at most %zu)",
                 lds, gpk::kMaxLdsBlock);
        return GP_ERR_UNSUPPORTED;
      }
    }
    // enough blocks to fill the device (about 2048), chunks of at least 32 rows, and the
    // y head correction inside the first chunk (the only block that holds u_0)
    nchunks = std::max(1, std::min(ceil_div(2048, p.nx), p.ny / 32));
    chunk = ceil_div(p.ny, nchunks);
    if (chunk < nwy) {
      nchunks = 1;
      chunk = p.ny;
    }
    nchunks = ceil_div(p.ny, chunk);
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (mode == 2 && !c->work) {  // the x sweep's output array (one more psi-sized buffer)
    int rc = dalloc(c, &c->work, (size_t)c->npts * c->esize);
    if (rc) return rc;
  }
  if (mode != 2 && c->work) {
    (void)hipFree(c->work);
    c->work = nullptr;
  }
  if (mode == 2) {
    const int nb = p.nx * nchunks;
    if (nb > c->zpart_cap) {  // room for the fused pass's norm partials
      double* np = nullptr;
      int rc = dalloc(c, &np, (size_t)nb * sizeof(double));
      if (rc) return rc;
      (void)hipFree(c->zpart);
      c->zpart = np;
      c->zpart_cap = nb;
    }
    for (int m = 0; m < 2; ++m) {
      gpk::AxisConst ac;
      gpk::cn_axis_constants(p.nz, p.dz, p.dt, m, gpk::yz_mz(p.nz), p.precision == GP_C64, &ac);
      for (int q = 0; q < 8; ++q) c->yzcoef[m][q] = ac.coef[q];
    }
    c->yz_chunk = chunk;
    c->yz_nchunks = nchunks;
  }
  c->trunc = mode;
  destroy_graphs(c);
  return GP_OK;
}

int gp_get_truncation(gp_ctx* c, int32_t* mode, int32_t hlen[6]) {
  if (!c) return GP_ERR_INVALID;
  if (mode) *mode = c->trunc;
  if (hlen)
    for (int m = 0; m < 2; ++m)
      for (int a = 0; a < 3; ++a) hlen[3 * m + a] = c->hlen[m][a];
  return GP_OK;
}

int gp_set_alloc_cap(int64_t bytes) {
  gpk::set_alloc_cap(bytes);
  return GP_OK;
}

int gp_eval_sincos(int32_t precision, const void* x_dev, int64_t n, void* sin_dev, void* cos_dev, void* hip_stream) {
  if ((precision != GP_C64 && precision != GP_C128) || n < 0) return GP_ERR_INVALID;
  if (n == 0) return GP_OK;
  if (!x_dev || !sin_dev || !cos_dev) return GP_ERR_INVALID;
  const size_t es = precision == GP_C128 ? 8 : 4;
  for (const void* q : {x_dev, (const void*)sin_dev, (const void*)cos_dev})
    if (reinterpret_cast<uintptr_t>(q) % es != 0) return GP_ERR_INVALID;
  hipError_t e = gpk::launch_eval_sincos(precision, x_dev, n, sin_dev, cos_dev, (hipStream_t)hip_stream);
  return e == hipSuccess ? GP_OK : GP_ERR_HIP;
}

int gp_stream_copy(const void* src_dev, void* dst_dev, int64_t bytes, void* hip_stream) {
  if (bytes < 0 || bytes % 16 != 0) return GP_ERR_INVALID;
  if (bytes == 0) return GP_OK;
  if (!src_dev || !dst_dev || reinterpret_cast<uintptr_t>(src_dev) % 16 != 0 ||
      reinterpret_cast<uintptr_t>(dst_dev) % 16 != 0)
    return GP_ERR_INVALID;
  hipError_t e = gpk::launch_stream_copy(src_dev, dst_dev, bytes, (hipStream_t)hip_stream);
  return e == hipSuccess ? GP_OK : GP_ERR_HIP;
}

const char* gp_strerror(int code) {
  switch (code) {
    case GP_OK: return "ok";
    case GP_ERR_INVALID: return "invalid argument";
    case GP_ERR_HIP: return "HIP runtime error";
    case GP_ERR_OOM: return "out of device memory";
    case GP_ERR_NONFINITE: return "non-finite norm or observable";
    case GP_ERR_ZERO_NORM: return "zero norm";
    case GP_ERR_UNSUPPORTED: return "unsupported grid size";
    default: return "unknown error code";
  }
}

const char* gp_last_error(gp_ctx* c) { return c ? c->err : "null context"; }

}  // extern "C"
