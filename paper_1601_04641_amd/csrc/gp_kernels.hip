// HIP kernels (gfx950, wave64) of the split-step Crank-Nicolson Gross-Pitaevskii step.
//
// One step streams psi through three kernels (paper: "Summary of revisions", the
// sub-steps calcnu, calclux, calcluy, calcluz):
//   k_sweep_lines  x sweep with the potential/nonlinear step fused into its load, then
//                  the y sweep (same kernel, no potential step).  Lanes run over the
//                  contiguous line index, so every row of a line bundle is one coalesced
//                  512 B (complex64) / 1 KB (complex128) access.
//   k_sweep_z      z sweep over the contiguous axis: line blocks staged through LDS with
//                  coalesced copies, each z line split over a group of lanes; in
//                  imaginary time it also emits FP64 per-block sums of |psi|^2.
//   k_finalize_norm  fixed-order FP64 sum of those partials -> renormalisation scale,
//                  which the next potential step applies (paper: renormalisation of the
//                  wavefunction after each imaginary-time step).
//
// Each Crank-Nicolson solve along a line,
//   -c u_{i-1} + (1+2c) u_i - c u_{i+1} = c p_{i-1} + (1-2c) p_i + c p_{i+1},
// is the Thomas algorithm written as two first-order linear recurrences with the
// constant tables a_i = c gamma_i and b_i = (1-2c) gamma_i of the forward sweep
// (in complex64 storage b, which is close to unit modulus, is carried as an FP32 hi+lo
// pair: rounding it to one float would make every real-time sweep non-unitary by ~1e-7
// in the same direction, a norm drift linear in the step count):
//   forward   d_i = a_i (p_{i-1} + p_{i+1} + d_{i-1}) + b_i p_i,   d_{-1} = 0
//   backward  u_i = d_i + a_i u_{i+1},                             u_n = 0
// A line is cut into segments of m points, one segment per thread.  Each thread runs
// both recurrences over its segment from a zero start; the true start values follow
// from composing the segments' affine maps x -> A x + B (A = product of a over the
// segment), and the fix-ups d_i += (a_s..a_i) D_in, u_i += (a_i..a_e-1) U_in run as
// running products.  This is algebraically the same elimination as the
// serial Thomas sweep (only rounding order differs) and needs no d' storage beyond the
// segment held in registers, so psi is read once and written once per sweep.
#include "gp_device.h"

#include <algorithm>

namespace gpk {

// ---------------------------------------------------------------------------------------
// single-grid kernels (bodies in gp_device.h)
// ---------------------------------------------------------------------------------------
#ifndef GP_XCD_REMAP
#define GP_XCD_REMAP 1
#endif

// MAXW: the most wavefronts a block of this instance may have.  1024-thread blocks cap a
// thread at 128 VGPRs; complex128 with 16 points per thread needs more in the x sweep (the
// potential step's phase factor), and spilling there cost 30% extra HBM traffic (scratch
// reads and writes), so blocks of at most 8 wavefronts run an instance bounded at 512
// (256 VGPRs).  The same holds for 30 and 32 points per thread in either precision.
// LONGHC: the Sherman-Morrison correction reaches past the first segment and is applied
// in the kernel (u_0 through LDS) instead of by a separate pass (k_head_correction).
template <typename R, int M, int SW, bool CC, int NSTEP, bool WIDE, int MAXW, bool LONGHC = false>
__global__ void __launch_bounds__(64 * MAXW)
k_sweep_lines(const typename VecOf<R>::T* psi, typename VecOf<R>::T* dst, int64_t psi_bytes, typename VecOf<R>::T ca,
              typename VecOf<R>::T cb, typename VecOf<R>::T cbl, typename VecOf<R>::T cP,
              const typename VecOf<R>::T* __restrict__ omega, int nwi, int n, int nseg, int64_t nlines,
              int64_t inner, Pot1D<R> px, const R* __restrict__ vy, const R* __restrict__ vz, int nz,
              R tau, const DevState* __restrict__ st) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R scale = 1, g = 0;
  if (NSTEP != 0) {
    scale = (R)st->s;
    g = (R)st->g;
  }
  const int64_t b = GP_XCD_REMAP ? xcd_bundle(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  lines_body<R, M, SW, CC, NSTEP, WIDE, LONGHC>(psi, dst, psi_bytes, ca, cb, cbl, cP, omega, nwi, n, nseg, nlines, inner,
                                                px, vy, vz, nz, tau, scale, g, b, smem_raw);
}

// Streaming x or y sweep with the truncated back-substitution (stream_line): thread =
// line; lines l = j*nz + k (x sweep, inner = ny*nz) or i*nz + k (y sweep, inner = nz).
template <typename R, int H, bool CC, int NSTEP>
__global__ void __launch_bounds__(256)
k_stream_lines(typename VecOf<R>::T* __restrict__ psi, typename VecOf<R>::T ca, typename VecOf<R>::T cb,
               typename VecOf<R>::T cbl, const typename VecOf<R>::T* __restrict__ omega, int nw, int n,
               int64_t nlines, int64_t inner, Pot1D<R> px, const R* __restrict__ vy, const R* __restrict__ vz,
               int nz, R tau, const DevState* __restrict__ st) {
  const int64_t b = GP_XCD_REMAP ? xcd_bundle(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
  const int64_t line = b * 256 + threadIdx.x;
  if (line >= nlines) return;
  R scale = 1, g = 0, vperp = 0;
  if (NSTEP != 0) {
    scale = (R)st->s;
    g = (R)st->g;
    vperp = vy[line / nz] + vz[line % nz];  // x-sweep line index = j*nz + k
  }
  const int64_t base = (line / inner) * (inner * n) + (line % inner);
  Coef<typename VecOf<R>::T> cf;
  cf.a = ca;
  cf.b = cb;
  cf.bl = cbl;
  stream_line<R, H, CC, NSTEP>(psi + base, n, inner, cf, omega, nw, px, vperp, tau, scale, g);
}

template <typename R, int MZ, bool CC, bool NORM, int EPI, int NW>
__global__ void __launch_bounds__(64 * NW)
k_sweep_z(typename VecOf<R>::T* __restrict__ psi, typename VecOf<R>::T ca, typename VecOf<R>::T cb,
          typename VecOf<R>::T cbl, typename VecOf<R>::T cP, const typename VecOf<R>::T* __restrict__ omega, int nwi,
          int nz, int nseg, int64_t nlines, double* __restrict__ partials, const R* __restrict__ vx,
          const R* __restrict__ vy, Pot1D<R> pz, int ny, R tau, const DevState* __restrict__ st, int zpad) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[4];
  R g = 0;
  if (EPI != 0) g = (R)st->g;
  // Sherman-Morrison vector from LDS or global memory: z_omega_in_lds
  const double acc = z_body<R, MZ, CC, NORM, EPI, NW, (NW == 1 || sizeof(R) == 4)>(psi, ca, cb, cbl, cP, omega, nwi, nz, nseg, nlines, vx,
                                                               vy, pz, ny, tau, g, blockIdx.x, gridDim.x, zpad,
                                                               smem_raw);
  if (NORM) {
    const double t = block_sum_w<NW>(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------------------
// reductions and small kernels
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_finalize_norm(const double* __restrict__ partials, int nb, double dV, double dt, DevState* st) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int q = threadIdx.x; q < nb; q += 256) acc += partials[q];
  const double tot = block_sum_256(acc, red);
  if (threadIdx.x == 0) {
    const double npre = tot * dV;
    int f = 0;
    if (!isfinite(npre)) f = 1;
    else if (!(npre > 0.0)) f = 2;
    st->npre = npre;
    st->mu_est = (f == 0) ? -log(npre) / (2.0 * dt) : 0.0;
    st->flags |= f;
    st->s = (f == 0) ? 1.0 / sqrt(npre) : 1.0;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_scale(typename VecOf<R>::T* __restrict__ psi, int64_t n, DevState* st) {
  const R s = (R)st->s;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
    typename VecOf<R>::T v = psi[q];
    v.x *= s;
    v.y *= s;
    psi[q] = v;
  }
}

__global__ void k_reset_scale(DevState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->s = 1.0;
}

template <typename R>
__global__ void __launch_bounds__(256)
k_observables(const typename VecOf<R>::T* __restrict__ psi, int nx, int ny, int nz, AxisQ ax, AxisQ ay, AxisQ az,
              double* __restrict__ partials) {
  __shared__ double red[4];
  const int64_t total = (int64_t)nx * ny * nz;
  const int64_t sx = (int64_t)ny * nz;
  double acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = 0.0;
  const int64_t qs = (int64_t)gridDim.x * 256;
  Idx3 ix((int64_t)blockIdx.x * 256 + threadIdx.x, qs, ny, nz);
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += qs, ix.advance()) {
    const int i = ix.i, j = ix.j, k = ix.k;
    const double re = psi[q].x, im = psi[q].y;
    const double n2 = re * re + im * im;
    double ex = 0, ey = 0, ez = 0, fx = 0, fy = 0, fz = 0;
    if (i + 1 < nx) { ex = psi[q + sx].x; fx = psi[q + sx].y; }
    if (j + 1 < ny) { ey = psi[q + nz].x; fy = psi[q + nz].y; }
    if (k + 1 < nz) { ez = psi[q + 1].x; fz = psi[q + 1].y; }
    double lx = (ex - re) * (ex - re) + (fx - im) * (fx - im);
    double ly = (ey - re) * (ey - re) + (fy - im) * (fy - im);
    double lz = (ez - re) * (ez - re) + (fz - im) * (fz - im);
    if (i == 0) lx += n2;  // link from the zero ghost at -1
    if (j == 0) ly += n2;
    if (k == 0) lz += n2;
    acc[0] += n2;
    acc[1] += lx;
    acc[2] += ly;
    acc[3] += lz;
    // coordinates and potentials from their closed forms: six FP64 table loads per point
    // made this kernel bound by its load instructions
    // (rounded operations, no contraction: the values the host computes in FP64)
    const double xi = ((double)i - ax.c) * ax.d, yj = ((double)j - ay.c) * ay.d, zk = ((double)k - az.c) * az.d;
    const double v = __dadd_rn(__dadd_rn(__dmul_rn(__dmul_rn(ax.h, xi), xi), __dmul_rn(__dmul_rn(ay.h, yj), yj)),
                               __dmul_rn(__dmul_rn(az.h, zk), zk));
    acc[4] += v * n2;
    acc[5] += n2 * n2;
    acc[6] += __dmul_rn(xi, xi) * n2;
    acc[7] += __dmul_rn(yj, yj) * n2;
    acc[8] += __dmul_rn(zk, zk) * n2;
  }
  for (int c = 0; c < 9; ++c) {
    const double t = block_sum_256(acc[c], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 9 + c] = t;
  }
}

__global__ void __launch_bounds__(256) k_obs_final(const double* __restrict__ partials, int nb, double* __restrict__ out) {
  __shared__ double red[4];
  for (int c = 0; c < 9; ++c) {
    double acc = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) acc += partials[(int64_t)q * 9 + c];
    const double t = block_sum_256(acc, red);
    if (threadIdx.x == 0) out[c] = t;
  }
}

// raw sums -> the scaled values of gp_raw_sums: N, kinetic link sums x 1/(2 d^2), U, I and
// the second moments, each times dV (the host formulas, same operations and order)
__global__ void k_obs_scale(const double* __restrict__ sums, double* __restrict__ raw, double dV, double d2x,
                            double d2y, double d2z) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double d2[3] = {d2x, d2y, d2z};
  raw[0] = __dmul_rn(sums[0], dV);
  for (int a = 0; a < 3; ++a) raw[1 + a] = __ddiv_rn(__dmul_rn(__dmul_rn(0.5, sums[1 + a]), dV), d2[a]);
  for (int q = 4; q < 9; ++q) raw[q] = __dmul_rn(sums[q], dV);
}

// the real-time phase factor's sin and cos on given arguments (error-bound checks)
template <typename R>
__global__ void __launch_bounds__(256)
k_eval_sincos(const R* __restrict__ x, int64_t n, R* __restrict__ sn, R* __restrict__ cs) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
    R s, c;
    dsincos(x[q], &s, &c);
    sn[q] = s;
    cs[q] = c;
  }
}

// Streaming copy of 16-byte units with raw buffer loads and stores, the access width of
// the sweeps' row loads, marked non-temporal: one unit per thread and one launch wide
// enough for the whole array (measured on the MI355X, 2 GiB: 6.37 TB/s, against 5.7 TB/s
// for grid-stride loops of 4 units per thread and 5.5 TB/s without the non-temporal
// hint).  Each block's resource starts at its own 4 KiB chunk.
__global__ void __launch_bounds__(256)
k_stream_copy(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int64_t nunits) {
  const int64_t c0 = (int64_t)blockIdx.x * 256;
  const int64_t left = min(nunits - c0, (int64_t)256);
  if ((int64_t)threadIdx.x >= left) return;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(src + c0 * 16, (uint32_t)(left * 16));
  const __amdgpu_buffer_rsrc_t rd = make_rsrc(dst + c0 * 16, (uint32_t)(left * 16));
  const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)threadIdx.x * 16, 0, 2);
  __builtin_amdgcn_raw_buffer_store_b128(v, rd, (int)threadIdx.x * 16, 0, 2);
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
template <typename R> static typename VecOf<R>::T cval(const double* c) {
  typename VecOf<R>::T v;
  v.x = (R)c[0];
  v.y = (R)c[1];
  return v;
}

template <typename R, int M, int SW, bool CC, int NSTEP, bool WIDE>
static hipError_t go_lines(const SweepLaunch& a, hipStream_t s) {
  typedef typename VecOf<R>::T V;
  constexpr int LW = 64 / SW;
  const int waves = (a.nseg + SW - 1) / SW;
  const size_t lds = (size_t)3 * waves * SW * LW * sizeof(V);
  const int64_t blocks = (a.nlines + LW - 1) / LW;
  // Corrections longer than a segment: in the kernel for 8 and 16 points per thread on
  // grids of up to 2^23 points, where the separate pass is mostly launch overhead; else a
  // separate pass.  Measured: 512 complex128 64^3 imaginary-time problems one after another
  // (8 points per thread along x, 16 along y) 12.7 -> 10.1 s, the same step counts and mu;
  // on the 512x480x448 grid (8 points per thread, 1024-thread blocks) the x sweep with the
  // separate pass took 800 us, in-kernel 882 us.
  constexpr bool kLong = !WIDE && (M == 8 || M == 16);
  const bool lng = kLong && a.nw > M && a.nlines * (int64_t)a.n <= ((int64_t)1 << 23);
  const int nwi = (a.nw <= M || lng) ? a.nw : 0;
  constexpr bool kMax8 = (sizeof(R) == 8 && M == 16 && NSTEP != 0) || M >= 30;
  auto kern = k_sweep_lines<R, M, SW, CC, NSTEP, WIDE, 16>;
  if constexpr (kMax8)
    if (waves <= 8) kern = k_sweep_lines<R, M, SW, CC, NSTEP, WIDE, 8>;
  if constexpr (kLong) {
    if (lng) {
      kern = k_sweep_lines<R, M, SW, CC, NSTEP, WIDE, 16, true>;
      if constexpr (kMax8)
        if (waves <= 8) kern = k_sweep_lines<R, M, SW, CC, NSTEP, WIDE, 8, true>;
    }
  }
  V* dst = (V*)(a.dst ? a.dst : a.psi);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(waves * 64), lds, s,
                     (const V*)a.psi, dst, a.psi_bytes, cval<R>(a.coef), cval<R>(a.coef + 2), cval<R>(a.coef + 4),
                     cval<R>(a.coef + 6), (const V*)a.omega, nwi, a.n, a.nseg, a.nlines, a.inner,
                     Pot1D<R>{(R)a.ph, (R)a.pc, (R)a.pd}, (const R*)a.vy, (const R*)a.vz, a.nz, (R)a.tau, a.st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nwi > 0 || a.nw == 0) return e;
  const int64_t want = (a.nlines + 255) / 256;
  hipLaunchKernelGGL((k_head_correction<R, CC>), dim3((unsigned)(want < 2048 ? want : 2048)), dim3(256), 0, s,
                     dst, (const V*)a.omega, a.nw, a.n, a.nlines, a.inner);
  return hipGetLastError();
}

template <typename R, int M, int SW, bool WIDE = false>
static hipError_t go_lines_mode(bool cc, const SweepLaunch& a, hipStream_t s) {
  if (!cc) return a.nstep ? go_lines<R, M, SW, false, 1, WIDE>(a, s) : go_lines<R, M, SW, false, 0, WIDE>(a, s);
  return a.nstep ? go_lines<R, M, SW, true, 2, WIDE>(a, s) : go_lines<R, M, SW, true, 0, WIDE>(a, s);
}

// Instances: complex64 M in {8, 10, 12, 16, 32}, complex128 M in {8, 16}, SW in {1, 2, 4}
// (32 complex doubles per thread would not fit the 128 VGPRs of 1024-thread blocks);
// M = 10 and 12 keep the real-time x sweep (with the phase factor) at <= 64 VGPRs, i.e.
// 8 waves per SIMD, where M = 16 needs 80 (6 waves).  For lines of up to 2048 points:
// SW = 8 with M = 16, 30, 32 in both precisions (M = 30, 32: at most 8 wavefronts, so the
// 512-thread bound and no spills), and complex64 M = 30 with SW = 4 (128-byte line chunks).
bool sweep_lines_supported(int precision, int m, int sw) {
  if (sw == 8) return m == 16 || m == 30 || m == 32;
  if (m == 30) return precision == 0 && sw == 4;
  if (sw != 1 && sw != 2 && sw != 4) return false;
  if (precision == 0) return m == 8 || m == 10 || m == 12 || m == 16 || m == 32;
  return m == 8 || m == 16;
}

#define GP_LINES_SW(R, M)                                                    \
  do {                                                                       \
    if (a.sw == 1) return go_lines_mode<R, M, 1>(cc, a, s);                 \
    if (a.sw == 2) return go_lines_mode<R, M, 2>(cc, a, s);                 \
    if (a.sw == 4) return go_lines_mode<R, M, 4>(cc, a, s);                 \
  } while (0)

// 64-bit addressed instances: the mappings that cover lines of 513-2048 points (and
// complex128 lines of up to 1024 with 8 points per thread) on grids whose planes are so
// large that a wavefront's rows span 2 GiB or more
bool sweep_lines_wide_supported(int precision, int m, int sw) {
  if ((m == 30 || m == 32) && sw == 8) return true;
  if (precision == 0) return (m == 16 && (sw == 4 || sw == 8)) || ((m == 30 || m == 32) && sw == 4);
  return (m == 16 && (sw == 4 || sw == 8)) || (m == 8 && sw == 4);
}

hipError_t launch_sweep_lines(int precision, bool cc, const SweepLaunch& a, hipStream_t s) {
  if (a.wide) {
    if (precision == 0) {
      if (a.m == 16 && a.sw == 4) return go_lines_mode<float, 16, 4, true>(cc, a, s);
      if (a.m == 16 && a.sw == 8) return go_lines_mode<float, 16, 8, true>(cc, a, s);
      if (a.m == 30 && a.sw == 4) return go_lines_mode<float, 30, 4, true>(cc, a, s);
      if (a.m == 32 && a.sw == 4) return go_lines_mode<float, 32, 4, true>(cc, a, s);
      if (a.m == 30 && a.sw == 8) return go_lines_mode<float, 30, 8, true>(cc, a, s);
      if (a.m == 32 && a.sw == 8) return go_lines_mode<float, 32, 8, true>(cc, a, s);
    } else {
      if (a.m == 16 && a.sw == 4) return go_lines_mode<double, 16, 4, true>(cc, a, s);
      if (a.m == 16 && a.sw == 8) return go_lines_mode<double, 16, 8, true>(cc, a, s);
      if (a.m == 8 && a.sw == 4) return go_lines_mode<double, 8, 4, true>(cc, a, s);
      if (a.m == 30 && a.sw == 8) return go_lines_mode<double, 30, 8, true>(cc, a, s);
      if (a.m == 32 && a.sw == 8) return go_lines_mode<double, 32, 8, true>(cc, a, s);
    }
    return hipErrorInvalidValue;
  }
  if (precision == 0) {
    if (a.m == 8) GP_LINES_SW(float, 8);
    if (a.m == 16 && a.sw == 8) return go_lines_mode<float, 16, 8>(cc, a, s);
    if (a.m == 30 && a.sw == 4) return go_lines_mode<float, 30, 4>(cc, a, s);
    if (a.m == 30 && a.sw == 8) return go_lines_mode<float, 30, 8>(cc, a, s);
    if (a.m == 32 && a.sw == 8) return go_lines_mode<float, 32, 8>(cc, a, s);
    if (a.m == 16) GP_LINES_SW(float, 16);
    if (a.m == 12) GP_LINES_SW(float, 12);
    if (a.m == 10) GP_LINES_SW(float, 10);
    if (a.m == 32) GP_LINES_SW(float, 32);
  } else {
    if (a.m == 16 && a.sw == 8) return go_lines_mode<double, 16, 8>(cc, a, s);
    if (a.m == 30 && a.sw == 8) return go_lines_mode<double, 30, 8>(cc, a, s);
    if (a.m == 32 && a.sw == 8) return go_lines_mode<double, 32, 8>(cc, a, s);
    if (a.m == 8) GP_LINES_SW(double, 8);
    if (a.m == 16) GP_LINES_SW(double, 16);
  }
  return hipErrorInvalidValue;
}
#undef GP_LINES_SW

template <typename R, int H, bool CC, int NSTEP>
static hipError_t go_stream(const SweepLaunch& a, hipStream_t s) {
  typedef typename VecOf<R>::T V;
  const int64_t blocks = (a.nlines + 255) / 256;
  hipLaunchKernelGGL((k_stream_lines<R, H, CC, NSTEP>), dim3((unsigned)blocks), dim3(256), 0, s, (V*)a.psi,
                     cval<R>(a.coef), cval<R>(a.coef + 2), cval<R>(a.coef + 4), (const V*)a.omega, a.nw, a.n,
                     a.nlines, a.inner, Pot1D<R>{(R)a.ph, (R)a.pc, (R)a.pd}, (const R*)a.vy, (const R*)a.vz, a.nz,
                     (R)a.tau, a.st);
  return hipGetLastError();
}

template <typename R, int H>
static hipError_t go_stream_mode(bool cc, const SweepLaunch& a, hipStream_t s) {
  if (!cc) return a.nstep ? go_stream<R, H, false, 1>(a, s) : go_stream<R, H, false, 0>(a, s);
  return a.nstep ? go_stream<R, H, true, 2>(a, s) : go_stream<R, H, true, 0>(a, s);
}

// truncation lengths with kernel instances: the smallest one >= the required H is used
int stream_h(int h) {
  for (int v : {3, 5, 7, 11, 15})
    if (h <= v) return v;
  return -1;
}

hipError_t launch_stream_lines(int precision, bool cc, const SweepLaunch& a, hipStream_t s) {
  const int h = stream_h(a.hlen);
  if (precision == 0) {
    switch (h) {
      case 3: return go_stream_mode<float, 3>(cc, a, s);
      case 5: return go_stream_mode<float, 5>(cc, a, s);
      case 7: return go_stream_mode<float, 7>(cc, a, s);
      case 11: return go_stream_mode<float, 11>(cc, a, s);
      case 15: return go_stream_mode<float, 15>(cc, a, s);
    }
  } else {
    switch (h) {
      case 3: return go_stream_mode<double, 3>(cc, a, s);
      case 5: return go_stream_mode<double, 5>(cc, a, s);
      case 7: return go_stream_mode<double, 7>(cc, a, s);
      case 11: return go_stream_mode<double, 11>(cc, a, s);
      case 15: return go_stream_mode<double, 15>(cc, a, s);
    }
  }
  return hipErrorInvalidValue;
}

template <typename R, int MZ, bool CC, bool NORM, int EPI, int NW>
static hipError_t go_z_w(const SweepLaunch& a, hipStream_t s) {
  typedef typename VecOf<R>::T V;
  const int zpad = (MZ % 2 == 0) ? a.zpad : 0;
  // the block's line rows, then (z_omega_in_lds) the Sherman-Morrison vector
  const size_t lds =
      z_lds(a.nz, a.nseg, MZ, zpad, sizeof(V), NW) + (z_omega_in_lds(sizeof(V), NW) ? (size_t)a.nw * sizeof(V) : 0);
  if (lds > 65536 - 512) {  // more than the default 64 KiB per block: opt in (up to 160 KiB)
    static size_t granted = 0;
    if (lds > granted) {
      hipError_t e = hipFuncSetAttribute((const void*)k_sweep_z<R, MZ, CC, NORM, EPI, NW>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      granted = lds;
    }
  }
  hipLaunchKernelGGL((k_sweep_z<R, MZ, CC, NORM, EPI, NW>), dim3(a.grid), dim3(64 * NW), lds, s, (V*)a.psi,
                     cval<R>(a.coef), cval<R>(a.coef + 2), cval<R>(a.coef + 4), cval<R>(a.coef + 6),
                     (const V*)a.omega, a.nw, a.nz, a.nseg, a.nlines, a.partials, (const R*)a.vx, (const R*)a.vy,
                     Pot1D<R>{(R)a.ph, (R)a.pc, (R)a.pd}, a.ny, (R)a.tau, a.st, zpad);
  return hipGetLastError();
}

// one-wavefront blocks exist for the instances of long lines (z_waves picks them)
template <int MZ> constexpr bool kZOneWave = MZ >= 8;

template <typename R, int MZ, bool CC, bool NORM, int EPI>
static hipError_t go_z(const SweepLaunch& a, hipStream_t s) {
  if constexpr (kZOneWave<MZ>)
    if (a.zw == 1) return go_z_w<R, MZ, CC, NORM, EPI, 1>(a, s);
  if (a.zw != 4) return hipErrorInvalidValue;
  return go_z_w<R, MZ, CC, NORM, EPI, 4>(a, s);
}

template <typename R, int MZ>
static hipError_t go_z_mode(bool cc, const SweepLaunch& a, hipStream_t s) {
  if (!cc) {  // imaginary time: FP64 norm partials
    return a.nstep ? go_z<R, MZ, false, true, 1>(a, s) : go_z<R, MZ, false, true, 0>(a, s);
  }
  return a.nstep ? go_z<R, MZ, true, false, 2>(a, s) : go_z<R, MZ, true, false, 0>(a, s);
}

// z instances: points per thread MZ in {2, 4, 6, 7, 8, 12, 14, 16}, {20, 24, 32} for
// lines longer than 1024 points (64 segments; complex128 blocks of such lines hold more
// than 64 KiB of LDS and opt in to up to 160 KiB) and 15 (960 = 64 x 15 with packed,
// conflict-free LDS rows and 5 complex64 blocks per CU)
bool sweep_z_supported(int precision, int mz) {
  (void)precision;
  return mz == 2 || mz == 4 || mz == 6 || mz == 7 || mz == 8 || mz == 12 || mz == 14 || mz == 15 || mz == 16 ||
         mz == 20 || mz == 24 || mz == 32;
}

#define GP_Z_M(R)                                              \
  do {                                                         \
    switch (a.m) {                                             \
      case 2: return go_z_mode<R, 2>(cc, a, s);                \
      case 4: return go_z_mode<R, 4>(cc, a, s);                \
      case 6: return go_z_mode<R, 6>(cc, a, s);                \
      case 7: return go_z_mode<R, 7>(cc, a, s);                \
      case 8: return go_z_mode<R, 8>(cc, a, s);                \
      case 12: return go_z_mode<R, 12>(cc, a, s);              \
      case 14: return go_z_mode<R, 14>(cc, a, s);              \
      case 16: return go_z_mode<R, 16>(cc, a, s);              \
      default: return hipErrorInvalidValue;                    \
    }                                                          \
  } while (0)

hipError_t launch_sweep_z(int precision, bool cc, const SweepLaunch& a, hipStream_t s) {
  if (precision == 0) {
    if (a.m == 15) return go_z_mode<float, 15>(cc, a, s);
    if (a.m == 20) return go_z_mode<float, 20>(cc, a, s);
    if (a.m == 24) return go_z_mode<float, 24>(cc, a, s);
    if (a.m == 32) return go_z_mode<float, 32>(cc, a, s);
    GP_Z_M(float);
  }
  if (a.m == 15) return go_z_mode<double, 15>(cc, a, s);
  if (a.m == 20) return go_z_mode<double, 20>(cc, a, s);
  if (a.m == 24) return go_z_mode<double, 24>(cc, a, s);
  if (a.m == 32) return go_z_mode<double, 32>(cc, a, s);
  GP_Z_M(double);
}
#undef GP_Z_M


hipError_t launch_finalize_norm(const double* partials, int nb, double dV, double dt, DevState* st,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_norm, dim3(1), dim3(256), 0, s, partials, nb, dV, dt, st);
  return hipGetLastError();
}

hipError_t launch_scale(int precision, void* psi, int64_t n, DevState* st, hipStream_t s) {
  const int64_t want = (n + 255) / 256;
  const unsigned blocks = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  if (precision == 0)
    hipLaunchKernelGGL(k_scale<float>, dim3(blocks), dim3(256), 0, s, (float2*)psi, n, st);
  else
    hipLaunchKernelGGL(k_scale<double>, dim3(blocks), dim3(256), 0, s, (double2*)psi, n, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reset_scale, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_obs_scale(const double* sums, double* raw, double dV, const double d2[3], hipStream_t s) {
  hipLaunchKernelGGL(k_obs_scale, dim3(1), dim3(64), 0, s, sums, raw, dV, d2[0], d2[1], d2[2]);
  return hipGetLastError();
}

hipError_t launch_eval_sincos(int precision, const void* x, int64_t n, void* sn, void* cs, hipStream_t s) {
  const int64_t want = (n + 255) / 256;
  const unsigned blocks = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  if (precision == 0)
    hipLaunchKernelGGL(k_eval_sincos<float>, dim3(blocks), dim3(256), 0, s, (const float*)x, n, (float*)sn,
                       (float*)cs);
  else
    hipLaunchKernelGGL(k_eval_sincos<double>, dim3(blocks), dim3(256), 0, s, (const double*)x, n, (double*)sn,
                       (double*)cs);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
  const int64_t units = bytes / 16;
  const int64_t blocks = (units + 255) / 256;  // < 2^31 for any array below 32 TiB
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, s,
                     (const unsigned char*)src, (unsigned char*)dst, units);
  return hipGetLastError();
}

hipError_t launch_observables(int precision, const ObsLaunch& a, hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(k_observables<float>, dim3(a.grid), dim3(256), 0, s, (const float2*)a.psi, a.nx, a.ny, a.nz,
                       a.ax, a.ay, a.az, a.partials);
  else
    hipLaunchKernelGGL(k_observables<double>, dim3(a.grid), dim3(256), 0, s, (const double2*)a.psi, a.nx, a.ny,
                       a.nz, a.ax, a.ay, a.az, a.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, s, a.partials, a.grid, a.out);
  return hipGetLastError();
}

}  // namespace gpk
