// Internal interface between the C-ABI host code (gp_api.cpp) and the HIP kernels
// (gp_kernels.hip).  Not installed; not part of the C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace gpk {

// Device-resident solver state, read by the kernels through a pointer so that captured
// graphs stay valid when g or the renormalisation scale change.
struct DevState {
  double s;       // pending renormalisation scale, applied by the next potential step
  double g;       // nonlinearity
  double npre;    // dV sum|psi|^2 before the last renormalisation
  double mu_est;  // -ln(npre) / (2 dt)
  int32_t flags;  // GP_FLAG_* bits
  int32_t pad;
};

// Per-axis Crank-Nicolson constants of the constant-pivot solve (see gp_kernels.hip):
// coef = {a, b, b_lo, P} as (re, im) pairs, P = a^m; omega[nw] (storage precision,
// device) the Sherman-Morrison head correction.
// z sweep LDS layout.  A block holds 4 L lines of nz values (L = 64 / seg lines per
// wavefront); lane p of a line reads and writes points p*mz .. p*mz + mz - 1, so with
// packed rows the lanes of a wavefront are mz values apart and an even mz puts many of
// them on the same LDS banks (mz = 16: every lane of a half-wavefront on two banks).
// zpad = 1 leaves one empty slot after each segment: segments start mz + 1 (odd) values
// apart and a wavefront's accesses spread over all banks.  Taken for mz a multiple of 4
// (4-way or worse conflicts when packed; 1280-point lines: z sweep 20.2 -> 15.2 ms)
// whenever the padded block still fits 64 KiB; other even mz conflict 2-way at most,
// which measured no slower packed.
__host__ __device__ inline int z_pitch(int nz, int mz, int zpad) { return nz + zpad * ((nz + mz - 1) / mz); }
inline size_t z_lds(int nz, int seg, int mz, int zpad, size_t esize, int nw = 4) {
  return (size_t)nw * (64 / seg) * (size_t)z_pitch(nz, mz, zpad) * esize;
}
// Wavefronts per z block: 4, or 1 for long complex128 lines (mz >= 8) whose 4-wavefront
// block would hold more than 32 KiB of LDS.  The LDS of a CU then holds fewer than five
// 4-wavefront blocks, and a block's phases (copy in, solve, copy out) stop overlapping
// with other blocks' memory traffic; one-wavefront blocks keep about the same lines per
// CU in flight in independent units.  Measured (1000 steps): 1280-point lines 48.2 ->
// 37.8 ms (imaginary time), 960-point lines 18.3 -> 15.4 ms (real time); the quench
// grid's 448-point lines take 572 us as 32 segments of 14 points in one-wavefront blocks
// against 619 us as 64 of 7 in 4-wavefront blocks (under 32 KiB).  complex64 ran slower in
// one-wavefront blocks (1280-point lines 14.2 -> 20.3 ms, the quench grid 317 -> 324 us)
// and keeps 4 wavefronts.
inline int z_waves(int nz, int seg, int mz, int zpad, size_t esize) {
  return (esize == 16 && mz >= 8 && z_lds(nz, seg, mz, zpad, esize, 4) + 512 > 32768) ? 1 : 4;
}
// z blocks that hold the Sherman-Morrison vector in LDS after their line rows (read there by
// every line's head correction): one-wavefront blocks and complex64 blocks.  Measured,
// omega from global memory -> LDS: 1280-point complex128 lines 37.9 -> 32.6 ms together
// with the batched copy-in; complex64 quench z sweep 322 -> 313 us (real time); complex128
// 4-wavefront blocks ran 654 -> 677 us that way and read it from global memory.
inline bool z_omega_in_lds(size_t esize, int zw) { return zw == 1 || esize == 8; }
// Blocks whose packed rows already need more than 64 KiB (complex128 lines beyond 1016
// points, complex64 beyond 2032) take the padded layout whenever it fits max_lds.  extra:
// further bytes the block holds (the Sherman-Morrison vector).
inline int z_pad(int nz, int seg, int mz, size_t esize, size_t max_lds = 65536, size_t extra = 0) {
  if (mz % 4 != 0) return 0;
  const size_t packed = z_lds(nz, seg, mz, 0, esize) + 512 + extra;
  const size_t padded = z_lds(nz, seg, mz, 1, esize) + 512 + extra;
  if (padded <= 65536) return 1;
  return (packed > 65536 && padded <= max_lds) ? 1 : 0;
}
// LDS one workgroup may hold on gfx950 (160 KiB); z blocks above 64 KiB opt in per kernel
constexpr size_t kMaxLdsBlock = 163840;

struct SweepLaunch {
  void* psi;
  void* dst;        // x/y kernels: output array (null: in place)
  int64_t psi_bytes;  // size of psi in bytes
  double coef[8];
  const void* omega;
  int nw;
  int n;            // points along the swept axis
  int m;            // points per thread segment (= the kernel instance's register count)
  int nseg;         // segments per line
  int64_t nlines;   // number of lines
  int64_t inner;    // x sweep: ny*nz; y sweep: nz (line l -> base (l/inner)*n*inner + l%inner)
  int sw;           // segments per wavefront (x/y kernels)
  bool wide;        // x/y kernels: 64-bit addressing (a wavefront's rows span >= 2 GiB)
  int hlen;         // streaming kernels: terms kept of the back-substitution (H)
  // potential step fused into the load (x sweep) or store (z sweep, Strang)
  double ph, pc, pd;  // potential of the swept axis: V(i) = ph ((i - pc) pd)^2
  int nstep;        // 0 none, 1 imaginary, 2 real
  double tau;
  const void* vx;   // storage-precision potential tables 1/2 nu^2 a^2
  const void* vy;
  const void* vz;
  int ny, nz;
  const DevState* st;
  double* partials; // z sweep: per-block FP64 sum |psi|^2 (imaginary time), else null
  int grid;         // z sweep: number of blocks
  int zpad;         // z sweep: one empty LDS slot after each segment (z_pad)
  int zw;           // z sweep: wavefronts per block (z_waves)
};

// precision: 0 complex64, 1 complex128; cc: complex coefficients (real time)
hipError_t launch_sweep_lines(int precision, bool cc, const SweepLaunch& a, hipStream_t s);
hipError_t launch_sweep_z(int precision, bool cc, const SweepLaunch& a, hipStream_t s);
// Streaming x/y sweep with the back-substitution truncated after a.hlen terms
hipError_t launch_stream_lines(int precision, bool cc, const SweepLaunch& a, hipStream_t s);
int stream_h(int h);  // instance size for a required truncation length (-1: none)

// Fused y + z sweep with the truncated y back-substitution (gp_stream.hip)
struct YZLaunch {
  const void* src;        // input: the x sweep's output (a separate array)
  void* psi;              // output
  int nx, ny, nz;
  int chunk, nchunks;     // rows per block, blocks per plane
  double ycoef[6];        // y: a, b, b_lo as (re, im)
  const void* yomega;
  int ynw;
  double zcoef[8];        // z: a, b, b_lo, P = a^mz as (re, im)
  const void* zomega;
  int znw;
  int mz;                 // z points per lane (yz_mz(nz))
  int hlen;               // y truncation length
  int epi;                // Strang: trailing half potential step (1 imaginary, 2 real)
  double ph, pc, pd, tau; // z potential V(k) = ph ((k - pc) pd)^2; half step tau
  const void* vx;
  const void* vy;
  const DevState* st;
  double* partials;       // imaginary time: one FP64 sum per block
};
hipError_t launch_stream_yz(int precision, bool cc, const YZLaunch& a, hipStream_t s);
int yz_h(int h);    // instance size for a y truncation length (-1: none)
int yz_mz(int nz);  // z points per lane of the fused kernel (-1: nz > 1024)
// LDS bytes of one fused block (the rows of one group of z lines) for a y truncation
// length h; 0 when no instance covers (nz, h)
size_t yz_lds(int nz, int h, size_t esize, int znw);

hipError_t launch_finalize_norm(const double* partials, int nb, double dV, double dt, DevState* st,
                                hipStream_t s);
hipError_t launch_scale(int precision, void* psi, int64_t n, DevState* st, hipStream_t s);

// Observables: 9 FP64 sums per block into partials[nb][9], then a fixed-order final sum
// into out[9] (raw, without dV or 1/(2 d^2) factors).
// One axis of the harmonic potential in FP64: x_i = (i - c) d, V_i = (h x_i) x_i with
// h = nu^2 / 2 and c = (n - 1) / 2 (the host tables' operations in the same order).
struct AxisQ {
  double h, c, d;
};

struct ObsLaunch {
  const void* psi;
  int nx, ny, nz;
  AxisQ ax, ay, az;  // coordinates and potentials evaluated in place (no table loads)
  double* partials;
  int grid;
  double* out;
};
hipError_t launch_observables(int precision, const ObsLaunch& a, hipStream_t s);

// Host: constants of the constant-pivot CN solve along one axis (computed in FP64).
struct AxisConst {
  double coef[8];                             // a, b, b_lo, P = a^m as (re, im), rounded
  int nw;                                     // Sherman-Morrison correction length
  int hlen;                                   // terms of a truncated back-substitution
  std::vector<std::complex<double>> omega;    // FP64 correction coefficients
};
void cn_axis_constants(int n, double d, double dt, int mode, int m, bool f32, AxisConst* out);
void pack_complex(const std::vector<std::complex<double>>& v, bool f32, std::vector<unsigned char>& out);

// Device allocation of the library's own buffers (contexts, batches, networks).  Fails
// with hipErrorOutOfMemory, without calling the runtime, when a cap set by
// gp_set_alloc_cap is exceeded by this one request.
hipError_t dev_alloc(void** p, size_t bytes);
void set_alloc_cap(int64_t bytes);

// Device sin/cos of the real-time phase factor on n arguments (gp_eval_sincos)
hipError_t launch_eval_sincos(int precision, const void* x, int64_t n, void* s, void* c, hipStream_t st);
// Plain streaming copy with 16-byte buffer loads and stores (gp_stream_copy)
hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t st);
// raw observable sums -> the scaled raw[9] of gp_raw_sums, on the device
hipError_t launch_obs_scale(const double* sums, double* raw, double dV, const double d2[3], hipStream_t st);

// Stopping rule of the imaginary-time convergence loops, fed one value (mu) per check.
// delta_n = mu_n - mu_{n-1}, q_n = delta_n / delta_{n-1}.  mu approaches its limit
// geometrically when one decaying mode dominates: then q_n lies in (0, 1) and stays put.
// The rule asks for that at two successive checks, |q_n - q_{n-1}| <= q_n / 10, and prices
// the distance to the limit with the larger ratio r = max(q_n, q_{n-1}) (Aitken's
// extrapolation): |delta_n| r / (1 - r) <= tol |mu_n| / 2, |delta_n| <= tol |mu_n|, and the
// extrapolated limit mu_n + delta_n r / (1 - r) within tol |mu_n| / 2 of the previous
// check's.  The band on q rejects the two ways a mix of modes imitates a converged tail:
// a slower mode of opposite sign emerging makes q fall (towards a turning point of mu(t),
// where the changes are small while mu is still far from its limit), and a slower mode of
// the same sign makes q rise (its tail is then underpriced by the current ratio).
// Otherwise (mu turning, alternating, or at its rounding floor) |delta| <= tol |mu_n| / 10
// must hold at three successive checks.
struct StopRule {
  double prev = NAN, prev2 = NAN;
  double q = -1.0;        // last ratio delta_n / delta_{n-1} (-1: none, or not in (0, 1))
  double r = -1.0;        // ratio the tail is priced with (-1: not geometric at this check)
  double lim_prev = NAN;  // extrapolated limit at the previous check (NaN: not geometric)
  int hits = 0;
  void reset() {
    prev = prev2 = lim_prev = NAN;
    q = r = -1.0;
    hits = 0;
  }
  // distance to the limit that the ratio r predicts for a change d (0 when not geometric)
  double tail(double d) const { return (r > 0.0 && r < 1.0) ? std::fabs(d) * r / (1.0 - r) : 0.0; }
  bool update(double cur, double tol) {
    bool done = false;
    if (std::isfinite(prev) && std::isfinite(cur)) {
      const double d1 = cur - prev, lim = tol * std::fabs(cur);
      hits = std::fabs(d1) <= 0.1 * lim ? hits + 1 : 0;
      const double qp = q;
      q = r = -1.0;
      double extrap = NAN;
      if (std::isfinite(prev2)) {
        const double d0 = prev - prev2;
        const double qn = d0 != 0.0 ? d1 / d0 : -1.0;
        if (qn > 0.0 && qn < 1.0) {
          q = qn;
          if (qp > 0.0 && qp < 1.0 && std::fabs(qn - qp) <= 0.1 * qn) {
            r = std::max(qn, qp);
            extrap = cur + d1 * r / (1.0 - r);
            done = std::fabs(d1) <= lim && tail(d1) <= 0.5 * lim && std::isfinite(lim_prev) &&
                   std::fabs(extrap - lim_prev) <= 0.5 * lim;
          }
        }
      }
      lim_prev = extrap;
      done = done || hits >= 3;
    } else {
      hits = 0;
      q = r = -1.0;
      lim_prev = NAN;
    }
    prev2 = prev;
    prev = cur;
    return done;
  }
};

// Supported line mappings (x/y kernels: points per thread and segments per wavefront)
bool sweep_lines_supported(int precision, int m, int sw);
bool sweep_lines_wide_supported(int precision, int m, int sw);
bool sweep_z_supported(int precision, int mz);

}  // namespace gpk
