// Internal interface between the C-ABI host code (gp_api.cpp) and the HIP kernels
// (gp_kernels.hip).  Not installed; not part of the C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
inline size_t z_lds(int nz, int seg, int mz, int zpad, size_t esize) {
  return (size_t)4 * (64 / seg) * (size_t)z_pitch(nz, mz, zpad) * esize;
}
inline int z_pad(int nz, int seg, int mz, size_t esize) {
  return (mz % 4 == 0 && z_lds(nz, seg, mz, 1, esize) + 512 <= 65536) ? 1 : 0;
}

struct SweepLaunch {
  void* psi;
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
};

// precision: 0 complex64, 1 complex128; cc: complex coefficients (real time)
hipError_t launch_sweep_lines(int precision, bool cc, const SweepLaunch& a, hipStream_t s);
hipError_t launch_sweep_z(int precision, bool cc, const SweepLaunch& a, hipStream_t s);

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
  std::vector<std::complex<double>> omega;    // FP64 correction coefficients
};
void cn_axis_constants(int n, double d, double dt, int mode, int m, bool f32, AxisConst* out);
void pack_complex(const std::vector<std::complex<double>>& v, bool f32, std::vector<unsigned char>& out);

// Supported line mappings (x/y kernels: points per thread and segments per wavefront)
bool sweep_lines_supported(int precision, int m, int sw);
bool sweep_z_supported(int precision, int mz);

}  // namespace gpk
