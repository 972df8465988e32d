// Device-side helpers shared by the single-grid and batched kernels: complex arithmetic,
// the potential/nonlinear step, sin/cos and exp, raw buffer access, the sweep bodies.
// Included by gp_kernels.hip and gp_batch.hip only.
#pragma once
#include "gp_internal.h"

namespace gpk {


template <typename R> struct VecOf;
template <> struct VecOf<float> { typedef float2 T; };
template <> struct VecOf<double> { typedef double2 T; };

template <typename V> __device__ __forceinline__ V vmake(decltype(V::x) x, decltype(V::x) y) {
  V r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename V> __device__ __forceinline__ V vzero() { return vmake<V>(0, 0); }
template <typename V> __device__ __forceinline__ V vone() { return vmake<V>(1, 0); }
template <typename V> __device__ __forceinline__ V vadd(V a, V b) { return vmake<V>(a.x + b.x, a.y + b.y); }

// coefficient * value; with real coefficients (CC = false) only a.x is used
template <bool CC, typename V> __device__ __forceinline__ V cmul(V a, V b) {
  if (CC) return vmake<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  return vmake<V>(a.x * b.x, a.x * b.y);
}
// a * b + c
template <bool CC, typename V> __device__ __forceinline__ V cfma(V a, V b, V c) {
  if (CC) return vmake<V>(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
  return vmake<V>(fma(a.x, b.x, c.x), fma(a.x, b.y, c.y));
}

__device__ __forceinline__ float dexp(float v) { return expf(v); }
__device__ __forceinline__ double dexp(double v) { return exp(v); }

// sin and cos for the real-time phase factor.  Cody and Waite's additive reduction
// x = k pi/2 + r with pi/2 split into three parts (each k * part exact inside an FMA),
// |r| <= pi/4, then the Taylor series of sin and cos in r (through r^9 / r^10 in FP32,
// r^17 / r^18 in FP64; truncation below 1e-10 resp. 1e-20 on [-pi/4, pi/4]), and the
// quadrant k mod 4.  FP32 arguments beyond 1e4 are reduced in FP64 with the FP64 parts
// (the residual of pi/2 after three FP64 parts is ~1e-49, so k stays exact to |x| ~ 1e15);
// FP64 arguments use the same reduction up to |x| ~ 2^52.  Worst error measured on dense
// samples of |x| <= 1e4 against an 80-bit extended-precision reference, in ulps of the
// correctly rounded value: 1.46 (sin) / 1.47 (cos) in FP32, 1.47 / 1.48 in FP64.  There is no
// out-of-line fallback: a call inside the unrolled sweeps would force the calling
// convention on every live register (94 instead of 77 VGPRs in the x sweep).  The phase
// of one real-time step is usually far below 1/8; there the series is used directly.
__device__ __forceinline__ void quadrant(int q, float sp, float cp, float* s, float* c) {
  float ss = (q & 1) ? cp : sp, cc = (q & 1) ? sp : cp;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}
__device__ __forceinline__ void quadrant(int q, double sp, double cp, double* s, double* c) {
  double ss = (q & 1) ? cp : sp, cc = (q & 1) ? sp : cp;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// k mod 4 of an integer-valued double, without converting k itself to int
__device__ __forceinline__ int quad_of(double k) { return (int)(k - 4.0 * floor(0.25 * k)); }

// x = k pi/2 + r in FP64, |r| <= pi/4 (pi/2 = Q1 + Q2 + Q3, each part 53 bits)
__device__ __forceinline__ double reduce_pio2(double x, double* k) {
  *k = rint(x * 0.6366197723675814);  // 2/pi
  double r = fma(-*k, 1.5707963267948966, x);
  r = fma(-*k, 6.123233995736766e-17, r);
  return fma(-*k, -1.4973849048591698e-33, r);
}

__device__ __forceinline__ void dsincos(float x, float* s, float* c) {
  if (fabsf(x) < 0.125f) {  // typical step: no reduction, series through x^5 / x^6
    const float x2 = x * x;  // truncation < (1/8)^7/7! / (1/8) = 7.6e-10 (sin), 1.5e-12 (cos)
    *s = fmaf(x * x2, fmaf(x2, 1.0f / 120.0f, -1.0f / 6.0f), x);
    *c = fmaf(x2, fmaf(x2, fmaf(x2, -1.0f / 720.0f, 1.0f / 24.0f), -0.5f), 1.0f);
    return;
  }
  float r;
  int q;
  if (fabsf(x) <= 1.0e4f) {
    const float k = rintf(x * 0.636619772f);  // 2/pi
    r = fmaf(-k, 1.57079637f, x);             // pi/2 = 1.57079637 - 4.37113883e-8 - 1.71512451e-15
    r = fmaf(-k, -4.37113883e-08f, r);
    r = fmaf(-k, -1.71512451e-15f, r);
    q = (int)k & 3;
  } else {
    double k;
    r = (float)reduce_pio2((double)x, &k);
    q = quad_of(k);
  }
  const float r2 = r * r;
  const float ps = fmaf(r2, fmaf(r2, fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f), 1.0f / 120.0f), -1.0f / 6.0f);
  const float sp = fmaf(r * r2, ps, r);
  const float pc = fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -1.0f / 3628800.0f, 1.0f / 40320.0f), -1.0f / 720.0f),
                             1.0f / 24.0f), -0.5f);
  const float cp = fmaf(r2, pc, 1.0f);
  quadrant(q, sp, cp, s, c);
}

__device__ __forceinline__ void dsincos(double x, double* s, double* c) {
  if (fabs(x) < 0.125) {  // typical step: series through x^11 / x^12, truncation < 1e-20
    const double x2 = x * x;
    double ps = fma(x2, -1.0 / 39916800.0, 1.0 / 362880.0);  // sin: -1/11!, 1/9!, ...
    ps = fma(x2, ps, -1.0 / 5040.0);
    ps = fma(x2, ps, 1.0 / 120.0);
    ps = fma(x2, ps, -1.0 / 6.0);
    *s = fma(x * x2, ps, x);
    double pc = fma(x2, 1.0 / 479001600.0, -1.0 / 3628800.0);  // cos: 1/12!, -1/10!, ...
    pc = fma(x2, pc, 1.0 / 40320.0);
    pc = fma(x2, pc, -1.0 / 720.0);
    pc = fma(x2, pc, 1.0 / 24.0);
    pc = fma(x2, pc, -0.5);
    *c = fma(x2, pc, 1.0);
    return;
  }
  double k;
  const double r = reduce_pio2(x, &k);
  const double r2 = r * r;
  // ps = 1/3! - r^2/5! + ... - r^14/17!, sin r = r - r^3 ps; pc likewise, cos r = 1 - r^2 pc
  double ps = -1.0 / 355687428096000.0;               // -1/17!
  ps = fma(r2, ps, 1.0 / 1307674368000.0);            //  1/15!
  ps = fma(r2, ps, -1.0 / 6227020800.0);              // -1/13!
  ps = fma(r2, ps, 1.0 / 39916800.0);                 //  1/11!
  ps = fma(r2, ps, -1.0 / 362880.0);                  // -1/9!
  ps = fma(r2, ps, 1.0 / 5040.0);                     //  1/7!
  ps = fma(r2, ps, -1.0 / 120.0);                     // -1/5!
  ps = fma(r2, ps, 1.0 / 6.0);
  const double sp = fma(r * r2, -ps, r);
  double pc = 1.0 / 6402373705728000.0;               //  1/18!
  pc = fma(r2, pc, -1.0 / 20922789888000.0);          // -1/16!
  pc = fma(r2, pc, 1.0 / 87178291200.0);              //  1/14!
  pc = fma(r2, pc, -1.0 / 479001600.0);               // -1/12!
  pc = fma(r2, pc, 1.0 / 3628800.0);                  //  1/10!
  pc = fma(r2, pc, -1.0 / 40320.0);                   // -1/8!
  pc = fma(r2, pc, 1.0 / 720.0);                      //  1/6!
  pc = fma(r2, pc, -1.0 / 24.0);                      // -1/4!
  pc = fma(r2, pc, 0.5);
  const double cp = fma(r2, -pc, 1.0);
  quadrant(quad_of(k), sp, cp, s, c);
}

// Potential + nonlinear step on one value (calcnu): p <- scale p, then
// imaginary time p <- exp(-tau (V + g|p|^2)) p, real time p <- exp(-i tau (V + g|p|^2)) p.
template <int MODE, typename R, typename V>
__device__ __forceinline__ V nstep(V v, R scale, R pot, R g, R tau) {
  const R re = v.x * scale, im = v.y * scale;
  const R w = fma(g, fma(re, re, im * im), pot);
  if (MODE == 1) {
    const R f = dexp(-tau * w);
    return vmake<V>(f * re, f * im);
  }
  R sn, cs;
  dsincos(-tau * w, &sn, &cs);
  return vmake<V>(cs * re - sn * im, fma(cs, im, sn * re));
}

// Raw buffer access: an SGPR resource for the whole array, a 32-bit per-lane byte offset
// (VGPR) and a uniform per-row byte offset (SGPR), so a strided line costs one VGPR of
// addressing instead of a 64-bit address per element.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((__vector_size__(8)));
typedef unsigned int u32x4 __attribute__((__vector_size__(16)));

// Cache policy of psi's loads and stores: non-temporal (cache-policy value 2), since psi
// streams through once per sweep and nothing re-reads it from the caches.  Measured on the
// 512x480x448 quench: y and z sweeps 1-7% faster (complex128 y 666 -> 626 us, z 723 ->
// 671 us; complex64 z 348 -> 324 us); the x sweeps' loads keep the default policy
// (kLdLines, kStLines below).
#ifndef GP_NT
#define GP_NT 2
#endif
template <int AUX = GP_NT>
__device__ __forceinline__ void bload(float2& v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, AUX));
}
template <int AUX = GP_NT>
__device__ __forceinline__ void bload(double2& v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, AUX));
}
template <int AUX = GP_NT>
__device__ __forceinline__ void bstore(const float2& v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)vo, (int)so, AUX);
}
template <int AUX = GP_NT>
__device__ __forceinline__ void bstore(const double2& v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)vo, (int)so, AUX);
}
// Cache policy of a line sweep's loads and stores.  The sweep with the potential step (the
// x sweep) loads with the default policy and stores non-temporally; the y sweep does both
// non-temporally.  Measured on the 512x480x448 quench (x sweep, loads / stores):
// complex128 NT / NT 702 us, default / NT 673-675 us, default / default 680 us, NT /
// default 677 us (y sweep after it 642 instead of 626 us); complex64 default / default
// 333 us, default / NT 329 us (y 316 instead of 318 us), NT / default 324 us (y 328 us),
// NT / NT 365 us.  Non-temporal loads in the y sweep stay (default loads: 645 instead of
// 626 us in complex128, 328 instead of 318 us in complex64).  The 64-bit-addressed (WIDE)
// instances access psi through gld / gst below, non-temporally in both directions.
template <typename R, int NSTEP> constexpr int kLdLines = NSTEP != 0 ? 0 : GP_NT;
template <typename R, int NSTEP> constexpr int kStLines = GP_NT;
// The batched sweeps (many small instances per launch) keep non-temporal loads and stores,
// except the complex64 x sweep, which keeps the default policy for both: with the single
// grid's x-sweep policy the batched complex128 x sweep of the ground-state runs took 277.5
// instead of 262.1 us.
template <typename R, int NSTEP> constexpr int kBatchLines = (sizeof(R) == 4 && NSTEP != 0) ? 0 : GP_NT;
// plain global loads and stores of psi values (8 or 16 bytes) under the same policy
template <typename T> __device__ __forceinline__ T gld(const T* p) {
  static_assert(sizeof(T) == 8 || sizeof(T) == 16, "8- or 16-byte values");
  if constexpr (GP_NT != 0) {
    if constexpr (sizeof(T) == 16) return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p)));
    else return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p)));
  } else {
    return *p;
  }
}
template <typename T> __device__ __forceinline__ void gst(T* p, const T& v) {
  static_assert(sizeof(T) == 8 || sizeof(T) == 16, "8- or 16-byte values");
  if constexpr (GP_NT != 0) {
    if constexpr (sizeof(T) == 16) __builtin_nontemporal_store(__builtin_bit_cast(u32x4, v), reinterpret_cast<u32x4*>(p));
    else __builtin_nontemporal_store(__builtin_bit_cast(u32x2, v), reinterpret_cast<u32x2*>(p));
  } else {
    *p = v;
  }
}

template <typename V> __device__ __forceinline__ V shfl_up_v(V v, int off, int width) {
  return vmake<V>(__shfl_up(v.x, off, width), __shfl_up(v.y, off, width));
}
template <typename V> __device__ __forceinline__ V shfl_down_v(V v, int off, int width) {
  return vmake<V>(__shfl_down(v.x, off, width), __shfl_down(v.y, off, width));
}

// ---------------------------------------------------------------------------------------
// Constant-pivot form of the solve.  The Thomas pivots of A = tridiag(-c, 1+2c, -c)
// converge to gamma_inf = 1/(1 + 2c + c c'_inf), c'_inf the root of modulus < 1 of
// c x^2 + (1+2c) x + c = 0.  Running the elimination with gamma_inf from the first row on
// solves A' = A + kappa e_0 e_0^T, kappa = c c'_inf, exactly; the solution of A follows
// from the Sherman-Morrison identity u = u' + omega u'_0 with
// omega = kappa A'^{-1} e_0 / (1 - kappa (A'^{-1} e_0)_0), which decays like c'_inf^i,
// so only the first nw points of a line are corrected (nw: last |omega_i| above the
// storage precision's rounding level).  The sweeps therefore use three constants:
//   a = c gamma_inf, b = (1-2c) gamma_inf (complex64 storage: b as an FP32 hi+lo pair)
// and P = a^M, the product of a over a full segment.  Points past the end of a line
// (padding of a last segment) are forced to zero in the backward recurrence, which is
// all the exact solve needs (their forward values never reach a stored point).
// ---------------------------------------------------------------------------------------
template <typename V> struct Coef {
  V a, b, bl;
};

// one forward-recurrence point: d = a (prev + next + d) + (b + b_lo) p
template <bool CC, typename R, typename V>
__device__ __forceinline__ V fwd_point(const Coef<V>& c, V prev, V nxt, V d, V p) {
  const V sum = vadd(vadd(prev, nxt), d);
  V dn = cmul<CC>(c.a, sum);
  if (sizeof(R) == 4) dn = cfma<CC>(c.bl, p, dn);  // low part of b (complex64 storage)
  return cfma<CC>(c.b, p, dn);
}

// Harmonic potential along one axis, V(i) = h x^2 with x = (i - c) d, h = nu^2 / 2,
// c = (n - 1) / 2: evaluated in place of a table load (the same operations, in the same
// order, as the host tables, so FP64 values are identical to them).
template <typename R> struct Pot1D {
  R h, c, d;
  __device__ __forceinline__ R at(int i) const {
    const R x = ((R)i - c) * d;
    return h * x * x;
  }
};

// ---------------------------------------------------------------------------------------
// x / y sweep.  Block = ceil(nseg/SW) wavefronts; a wavefront holds SW segments of
// LW = 64/SW consecutive lines (lane = segment-in-wave * LW + line).  Lines l of a block
// are bidx*LW + [0, LW) (lanes past the last line repeat it: they compute and store
// identical values); element i of line l sits at base(l) + i*inner.  Each thread holds M
// consecutive points of one line in registers.  nwi > 0: the omega correction is applied
// here (nwi <= M, so it stays inside segment 0); otherwise k_head_correction follows.
// Each wavefront addresses psi from its own first point (first line of the block, first
// segment of the wavefront: the smallest element index any of its lanes touches), so the
// 32-bit byte offsets span only the wavefront's own rows and lines, whatever the size of
// psi; the host keeps that span below 2 GiB.  WIDE instances (for wavefronts whose rows
// span more, e.g. complex128 x lines of the paper's 1920x1600x1280 grid: 128 rows of
// 32.8 MB) address every point with a 64-bit pointer instead.  The sweep reads psi and
// writes dst (the same array for the in-place sweeps; another one for the x sweep ahead of
// the fused y+z pass, which must not read values another block has already replaced).
// ---------------------------------------------------------------------------------------
template <typename R, int M, int SW, bool CC, int NSTEP, bool WIDE = false, bool LONGHC = false,
          int LDP = kLdLines<R, NSTEP>, int STP = kStLines<R, NSTEP>>
__device__ __forceinline__ void lines_body(const typename VecOf<R>::T* psi, typename VecOf<R>::T* dst,
                                           int64_t psi_bytes,
                                           typename VecOf<R>::T ca, typename VecOf<R>::T cb,
                                           typename VecOf<R>::T cbl, typename VecOf<R>::T cP,
                                           const typename VecOf<R>::T* __restrict__ omega, int nwi, int n,
                                           int nseg, int64_t nlines, int64_t inner, Pot1D<R> px,
                                           const R* __restrict__ vy, const R* __restrict__ vz, int nz, R tau,
                                           R scale, R g, int64_t bidx, unsigned char* smem_raw) {
  typedef typename VecOf<R>::T V;
  constexpr int LW = 64 / SW;
  const int nslot = (int)(blockDim.x >> 6) * SW;  // segment slots in this block
  V* sh_first = reinterpret_cast<V*>(smem_raw);  // reused for the backward exchange
  V* sh_last = sh_first + nslot * LW;
  V* sh_B = sh_last + nslot * LW;
  V* sh_U = sh_first;

  const int lane = threadIdx.x & 63;
  const int li = lane % LW;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int p = (SW == 1) ? w : w * SW + lane / LW;
  const int64_t line = min(bidx * LW + li, nlines - 1);
  const int64_t base = (line / inner) * (inner * n) + (line % inner);
  const int s = p * M;
  const int len = max(0, min(M, n - s));
  Coef<V> cf;
  cf.a = ca;
  cf.b = cb;
  cf.bl = cbl;

  // e0: this wavefront's first point, (first line of the block, first row of the
  // wavefront's first segment).  With the early loads (below) a wavefront past the line's
  // end (batched blocks are sized for the largest instance) takes the line's last row, so
  // that e0 is always a point of psi.
  constexpr bool kEarly = M >= 24;
  const int64_t line0 = min(bidx * LW, nlines - 1);
  const int row0 = kEarly ? min(w * SW * M, n - 1) : w * SW * M;
  const int64_t e0 = (line0 / inner) * (inner * n) + (line0 % inner) + (int64_t)row0 * inner;
  const int64_t left_bytes = psi_bytes - e0 * (int64_t)sizeof(V);
  const uint32_t span = (uint32_t)min(left_bytes, (int64_t)0xffffffff);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(psi + e0, span);
  const __amdgpu_buffer_rsrc_t rd = (dst == psi) ? rs : make_rsrc(dst + e0, span);
  const uint32_t voff = (uint32_t)((base + (int64_t)s * inner - e0) * (int64_t)sizeof(V));
  const uint32_t srow = (uint32_t)(inner * (int64_t)sizeof(V));
  const V* const lp = psi + base + (int64_t)s * inner;  // WIDE: this lane's first point
  V* const lq = dst + base + (int64_t)s * inner;
  // Two load schemes.  Guarded (M < 24): each row's load sits behind a per-lane branch
  // (t < len), and the compiler then waits for all rows before the first use.  Early
  // (M >= 24, the long lines of the paper's grids): loads complete in issue order and each
  // use waits only for the loads issued before it, so the potential tables go first (every
  // point's potential step needs them), then the segment's first and last rows (the
  // neighbour exchange and its barrier need only those), then the rows between, whose
  // potential steps and forward recurrence run while later rows are still in flight; no
  // row load sits behind a branch (a branch around them all also made the compiler wait
  // for all of them): a row past the line's end (t >= len) loads the point e0 instead and
  // is zeroed before its first use.  Measured (per sweep): 1920x1600x1280 complex128
  // imaginary x 32.1 -> 28.8 ms, 1600x1280x960 complex64 y 7.41 -> 5.38 ms; on the
  // 512x480x448 quench (M = 16) the early scheme ran 0-3% slower.
  R vyz = 0;
  if (NSTEP != 0 && kEarly) vyz = vy[line / nz] + vz[line % nz];  // x-sweep line index = j*nz + k
  V v[M];
  if constexpr (kEarly) {
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const int t = (q == 0) ? 0 : (q == 1 ? M - 1 : q - 1);
      if (WIDE) v[t] = gld(t < len ? lp + (int64_t)t * inner : psi + e0);
      else bload<LDP>(v[t], rs, t < len ? voff + (uint32_t)t * srow : 0u, 0u);
    }
#pragma unroll
    for (int q = 0; q < 2 && q < M; ++q) {
      const int t = (q == 0) ? 0 : M - 1;
      if (t >= len) v[t] = vzero<V>();
      if (NSTEP != 0) {
        v[t] = nstep<NSTEP, R, V>(v[t], scale, px.at(min(s + t, n - 1)) + vyz, g, tau);  // padding stays 0
        if constexpr (sizeof(R) == 8) __builtin_amdgcn_sched_barrier(0);
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < M; ++t) {
      v[t] = vzero<V>();
      if (t < len) {
        if (WIDE) v[t] = gld(lp + (int64_t)t * inner);
        else bload<LDP>(v[t], rs, voff, (uint32_t)t * srow);
      }
    }
    if (NSTEP != 0) {
      vyz = vy[line / nz] + vz[line % nz];
#pragma unroll
      for (int t = 0; t < M; ++t) {
        const int pos = min(s + t, n - 1);
        v[t] = nstep<NSTEP, R, V>(v[t], scale, px.at(pos) + vyz, g, tau);  // padding stays 0
      }
    }
  }

  // neighbours across segment boundaries (right-hand side of the first and last rows);
  // a segment that ends early is the line's last, so nobody reads its last value
  sh_first[p * LW + li] = v[0];
  sh_last[p * LW + li] = v[M - 1];
  __syncthreads();
  if constexpr (kEarly) {
#pragma unroll
    for (int t = 1; t < M - 1; ++t)
      if (t >= len) v[t] = vzero<V>();
    if (NSTEP != 0) {
#pragma unroll
      for (int t = 1; t < M - 1; ++t) {
        v[t] = nstep<NSTEP, R, V>(v[t], scale, px.at(min(s + t, n - 1)) + vyz, g, tau);
        // complex128: one point's exp or sin/cos at a time, else the scheduler overlaps
        // many of them and the live temporaries exceed even 256 VGPRs (spills; complex64
        // keeps the overlap, which measured 9% faster there)
        if constexpr (sizeof(R) == 8) __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  const V left = (p > 0 && p < nseg) ? sh_last[(p - 1) * LW + li] : vzero<V>();
  const V right = (p < nseg - 1) ? sh_first[(p + 1) * LW + li] : vzero<V>();

  // forward recurrence over the segment from d_{s-1} = 0
  {
    V prev = left, d = vzero<V>();
#pragma unroll
    for (int t = 0; t < M; ++t) {
      V nxt = right;
      if (t + 1 < M) nxt = v[t + 1];
      const V dn = fwd_point<CC, R, V>(cf, prev, nxt, d, v[t]);
      prev = v[t];
      v[t] = dn;
      d = dn;
    }
    sh_B[p * LW + li] = d;
  }
  __syncthreads();
  // incoming d_{s-1}: compose the earlier segments' maps D -> P D + B_q, then add
  // a^(t+1) D_in as a running product
  {
    V D = vzero<V>();
    for (int q = 0; q < p && q < nseg; ++q) D = cfma<CC>(cP, D, sh_B[q * LW + li]);
    V r = D;
#pragma unroll
    for (int t = 0; t < M; ++t) {
      r = cmul<CC>(ca, r);
      v[t] = vadd(v[t], r);
    }
  }
  // backward recurrence over the segment from u_e = 0 (u = 0 past the end of the line)
  {
    V u = vzero<V>();
#pragma unroll
    for (int t = M - 1; t >= 0; --t) {
      u = cfma<CC>(ca, u, v[t]);
      if (t >= len) u = vzero<V>();
      v[t] = u;
    }
    sh_U[p * LW + li] = u;  // every halo read of sh_first precedes the barrier above
  }
  __syncthreads();
  {
    V U = vzero<V>();
    for (int q = nseg - 1; q > p; --q) U = cfma<CC>(cP, U, sh_U[q * LW + li]);
    V r = U;
#pragma unroll
    for (int t = M - 1; t >= 0; --t) {
      r = cmul<CC>(ca, r);
      v[t] = vadd(v[t], r);
    }
  }
  // Sherman-Morrison head correction of segment 0
  if (!LONGHC || nwi <= M) {
    if (w == 0 && nwi > 0) {
      const bool mine = (SW == 1) || (lane < LW);
      const V u0 = v[0];
#pragma unroll
      for (int t = 0; t < M; ++t) {
        if (t < nwi) {
          const V c = cfma<CC>(omega[t], u0, v[t]);
          if (mine) v[t] = c;
        }
      }
    }
  } else {
    // LONGHC instances, correction longer than a segment (large c, e.g. imaginary time on
    // coarse grids): u_0 reaches the other segments through LDS (sh_B is free: its last
    // reads precede the barrier above).  A separate pass over the first nw points of every
    // line, as the single-grid sweeps take, cost the batched ground-state runs about a
    // fifth of their time in extra launches.  (Instances without it keep the registers of
    // this path free: the omega loads of a general path raised the complex128 sweeps by
    // 18-36 VGPRs.)
    if (p == 0) sh_B[li] = v[0];
    __syncthreads();
    const V u0 = sh_B[li];
    if (s < nwi) {
#pragma unroll
      for (int t = 0; t < M; ++t)
        if (s + t < nwi) v[t] = cfma<CC>(omega[s + t], u0, v[t]);
    }
  }

#pragma unroll
  for (int t = 0; t < M; ++t)
    if (t < len) {
      if (WIDE) gst(lq + (int64_t)t * inner, v[t]);
      else bstore<STP>(v[t], rd, voff, (uint32_t)t * srow);
    }
}

// ---------------------------------------------------------------------------------------
// Streaming line solve with the back-substitution truncated after H terms (halo-truncated
// Crank-Nicolson inverse).  One thread per line; the thread walks its line once, reading
// p_{j+1} and writing u_{j-H} at step j:
//   forward   d_j = a (p_{j-1} + p_{j+1} + d_{j-1}) + b p_j   (exact, from the line start)
//   backward  u_j = sum_{m=0}^{H} a^m d_{j+m}                  (the exact sum runs to the
//             line end; the dropped terms are below |a|^{H+1} / (1 - |a|) max|d|, and the
//             host picks H so that this is 1/100 of the storage precision's unit roundoff)
// followed by the head correction u_j += omega_j u_0 (j < nw, u_0 kept in a register).
// Near the line end the sum stops at the last point, so it is exact there.  The loop is
// unrolled by L = H + 1: the ring of the last L values of d and the queue of the next L
// rows in flight are indexed by compile-time positions.  psi is read once and written
// once, in 64-lane rows of consecutive lines (one coalesced access per row), with no LDS
// and no barriers.  NSTEP: the potential step applied to each value as it is consumed.
// ---------------------------------------------------------------------------------------
template <typename R, int H, bool CC, int NSTEP>
__device__ __forceinline__ void stream_line(typename VecOf<R>::T* __restrict__ lp, int n, int64_t inner,
                                            const Coef<typename VecOf<R>::T>& cf,
                                            const typename VecOf<R>::T* __restrict__ omega, int nw, Pot1D<R> px,
                                            R vperp, R tau, R scale, R g) {
  typedef typename VecOf<R>::T V;
  constexpr int L = H + 1;
  const V ca = cf.a;
  auto load = [&](int j) { return gld(lp + (int64_t)j * inner); };
  auto prep = [&](V v, int j) {
    if (NSTEP != 0) v = nstep<NSTEP, R, V>(v, scale, px.at(j) + vperp, g, tau);
    return v;
  };
  V q[L];     // rows j+1 .. j+L in flight (slot (j+1) % L holds p_{j+1})
  V ring[L];  // d_{j-H} .. d_j (slot j % L holds d_j)
#pragma unroll
  for (int t = 0; t < L; ++t) {
    ring[t] = vzero<V>();
    q[(1 + t) % L] = (1 + t < n) ? load(1 + t) : vzero<V>();
  }
  V pm = vzero<V>(), pc = prep(load(0), 0), dprev = vzero<V>(), u0 = vzero<V>();
  const int total = n + H;  // the last H steps only emit (d past the line end is zero)
  for (int jb = 0; jb < total; jb += L) {
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int j = jb + t;
      if (j < total) {
        V d = vzero<V>();
        if (j < n) {
          const int s1 = (t + 1) % L;
          const V pn = (j + 1 < n) ? prep(q[s1], j + 1) : vzero<V>();
          if (j + 1 + L < n) q[s1] = load(j + 1 + L);
          d = fwd_point<CC, R, V>(cf, pm, pn, dprev, pc);
          pm = pc;
          pc = pn;
          dprev = d;
        }
        ring[t] = d;
        const int r = j - H;
        if (r >= 0) {
          V u = ring[t];
#pragma unroll
          for (int m = H - 1; m >= 0; --m) u = cfma<CC>(ca, u, ring[(t + 1 + m) % L]);
          if (r == 0) u0 = u;
          if (r < nw) u = cfma<CC>(omega[r], u0, u);
          gst(lp + (int64_t)r * inner, u);
        }
      }
    }
  }
}

// Line bundle of block b when blocks are dealt to the XCDs round-robin (block b runs on
// XCD b mod 8): XCD x takes one contiguous stretch of bundles, so the blocks resident on
// one XCD (sharing its L2 and address-translation caches) read adjacent row chunks
// instead of chunks eight bundles apart.  A bijection of [0, nb).
__device__ __forceinline__ int64_t xcd_bundle(int64_t b, int64_t nb) {
  const int64_t x = b & 7, k = b >> 3, per = nb >> 3, rem = nb & 7;
  return x * per + min(x, rem) + k;
}

// Sherman-Morrison head correction u_i += omega_i u_0, i < nw, one thread per line, for
// x/y lines when the correction reaches past the first segment (large c).  Lines as in
// k_sweep_lines.
template <typename R, bool CC>
__global__ void __launch_bounds__(256)
k_head_correction(typename VecOf<R>::T* __restrict__ psi, const typename VecOf<R>::T* __restrict__ omega, int nw,
                  int n, int64_t nlines, int64_t inner) {
  typedef typename VecOf<R>::T V;
  for (int64_t line = (int64_t)blockIdx.x * 256 + threadIdx.x; line < nlines; line += (int64_t)gridDim.x * 256) {
    const int64_t base = (line / inner) * (inner * n) + (line % inner);
    const V u0 = psi[base];
    for (int i = nw - 1; i >= 0; --i) psi[base + i * inner] = cfma<CC>(omega[i], u0, psi[base + i * inner]);
  }
}

// Solve of one z line held in LDS (row: its values, point q at q + zp (q / MZ)) by the
// nseg lanes of line group l: lane p holds points s .. s + len - 1 (s = p MZ, LDS position
// ss) in registers, runs both recurrences over them, and composes the segments' affine maps
// across lanes by Hillis-Steele scans of shuffles; then the Sherman-Morrison head
// correction.  The solution is left in v (registers); act = false lanes hold zeros.
template <typename R, int MZ, bool CC>
__device__ __forceinline__ void z_line_solve(typename VecOf<R>::T (&v)[MZ], const typename VecOf<R>::T* row, bool act,
                                             int s, int ss, int zp, int len, int nz, int nseg, int l, int p,
                                             const Coef<typename VecOf<R>::T>& cf, typename VecOf<R>::T cP,
                                             const typename VecOf<R>::T* __restrict__ omega, int nwi) {
  typedef typename VecOf<R>::T V;
  const V ca = cf.a;
#pragma unroll
  for (int t = 0; t < MZ; ++t) {
    v[t] = vzero<V>();
    if (act && t < len) v[t] = row[ss + t];
  }
  // neighbours: the previous segment's last point and (for a full segment) the next
  // segment's first point
  const V left = (act && s > 0) ? row[ss - 1 - zp] : vzero<V>();
  const V right = (act && s + len < nz) ? row[ss + len + zp] : vzero<V>();

  V d = vzero<V>();
  {
    V prev = left;
#pragma unroll
    for (int t = 0; t < MZ; ++t) {
      V nxt = right;
      if (t + 1 < MZ) nxt = v[t + 1];
      const V dn = fwd_point<CC, R, V>(cf, prev, nxt, d, v[t]);
      prev = v[t];
      v[t] = dn;
      d = dn;
    }
  }
  // inclusive scan of the segment maps x -> P x + B along the line.  Every segment
  // before an active lane is full, so a span of `off` segments multiplies by P^off:
  // the products are powers of P and only B travels between lanes.
  V B = act ? d : vzero<V>();
  {
    V Apow = cP;
    for (int off = 1; off < nseg; off <<= 1) {
      const V Bp = shfl_up_v(B, off, nseg);
      if (p >= off) B = cfma<CC>(Apow, Bp, B);
      Apow = cmul<CC>(Apow, Apow);
    }
  }
  V D = shfl_up_v(B, 1, nseg);
  if (p == 0) D = vzero<V>();
  {
    V r = D;
#pragma unroll
    for (int t = 0; t < MZ; ++t) {
      r = cmul<CC>(ca, r);
      v[t] = vadd(v[t], r);
    }
  }
  V u = vzero<V>();
#pragma unroll
  for (int t = MZ - 1; t >= 0; --t) {
    u = cfma<CC>(ca, u, v[t]);
    if (t >= len) u = vzero<V>();
    v[t] = u;
  }
  // backward scan likewise; a span reaching into the empty lanes past the line's last
  // segment gets P^off instead of the true product, but it only ever multiplies the
  // zero contribution of those lanes
  V Bu = act ? u : vzero<V>();
  {
    V Apow = cP;
    for (int off = 1; off < nseg; off <<= 1) {
      const V Bp = shfl_down_v(Bu, off, nseg);
      if (p + off < nseg) Bu = cfma<CC>(Apow, Bp, Bu);
      Apow = cmul<CC>(Apow, Apow);
    }
  }
  V U = shfl_down_v(Bu, 1, nseg);
  if (p == nseg - 1) U = vzero<V>();
  {
    V r = U;
#pragma unroll
    for (int t = MZ - 1; t >= 0; --t) {
      r = cmul<CC>(ca, r);
      v[t] = vadd(v[t], r);
    }
  }
  // Sherman-Morrison head correction: u_i += omega_i u_0 for i < nwi
  if (nwi > 0) {
    const V u0 = vmake<V>(__shfl(v[0].x, l * nseg, 64), __shfl(v[0].y, l * nseg, 64));
#pragma unroll
    for (int t = 0; t < MZ; ++t) {
      if (t < nwi) {  // uniform: segment-0 lanes need it whenever t < nwi
        const int pos = s + t;
        const V om = omega[min(pos, nwi - 1)];
        const V c = cfma<CC>(om, u0, v[t]);
        if (pos < nwi) v[t] = c;
      }
    }
  }

}

// ---------------------------------------------------------------------------------------
// z sweep.  Block = NW wavefronts (4, or 1 for long lines); a wavefront holds L = 64/nseg
// z lines, lane = line-in-wave * nseg + segment, MZ points per thread.  Each iteration
// copies NW L consecutive lines (contiguous in memory) into LDS, solves them, and copies
// them back.
// The omega correction runs here (any nw), u'_0 broadcast along the line by a shuffle.
// Processes line groups grp_begin, grp_begin + grp_step, ...; returns this thread's FP64
// sum of |psi|^2 over the stored points when NORM.
// ---------------------------------------------------------------------------------------
template <typename R, int MZ, bool CC, bool NORM, int EPI, int NW = 4, bool OML = false>
__device__ __forceinline__ double z_body(typename VecOf<R>::T* __restrict__ psi, typename VecOf<R>::T ca,
                                         typename VecOf<R>::T cb, typename VecOf<R>::T cbl,
                                         typename VecOf<R>::T cP, const typename VecOf<R>::T* __restrict__ omega,
                                         int nwi, int nz, int nseg, int64_t nlines, const R* __restrict__ vx,
                                         const R* __restrict__ vy, Pot1D<R> pz, int ny, R tau, R g,
                                         int64_t grp_begin, int64_t grp_step, int zpad,
                                         unsigned char* smem_raw) {
  typedef typename VecOf<R>::T V;
  V* sdata = reinterpret_cast<V*>(smem_raw);
  // LDS rows of `pitch` values; with zp = 1 point q of a line sits at q + q / MZ (one empty
  // slot after each segment, even MZ only, so the two points of a 16-byte pair share one)
  const int zp = (MZ % 2 == 0) ? zpad : 0;
  const int pitch = z_pitch(nz, MZ, zp);

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int L = 64 / nseg;
  const int l = lane / nseg, p = lane % nseg;
  constexpr int NT = 64 * NW;  // threads per block
  const int lines_per_grp = NW * L;
  const int64_t ngrp = (nlines + lines_per_grp - 1) / lines_per_grp;
  const int s = p * MZ;
  const int ss = s + zp * p;  // LDS position of the segment's first point
  const int len = max(0, min(MZ, nz - s));
  Coef<V> cf;
  cf.a = ca;
  cf.b = cb;
  cf.bl = cbl;
  double acc = 0.0;
  // this thread's copy positions advance by NT points (or pairs) per iteration: their
  // (line, point) digits advance by the step's own digits with one carry
  const int half = nz >> 1;
  // 16-byte copies need a 16-byte aligned grid base (a batched instance may start at any
  // complex64 element); otherwise every copy moves one 8-byte value
  const bool al16 = (reinterpret_cast<uintptr_t>(psi) & 15) == 0;
  const bool pairs = sizeof(V) == 8 && (nz & 1) == 0 && al16;  // with zp = 1 (MZ even)
  const int cn = pairs ? half : nz;
  const int dl = NT / cn, dq = NT % cn;
  // complex128 blocks issue their copies KB at a time, all loads before the LDS stores: one
  // copy per iteration waits out a whole memory latency per value (the compiler keeps one
  // load in flight).  Measured: 4-wavefront blocks of 448-point lines (7 copies per
  // thread) z sweep 650 -> 607 us (real time), 696 -> 593 us (imaginary time); KB = 2, 3
  // and 4 within 1-4% of that, 8 slower (635 / 624 us).  One-wavefront blocks (long
  // lines, 15-20 copies per thread) take 8.  complex64 blocks ran 3-25% slower batched.
  constexpr int KB = (sizeof(R) == 4) ? 1 : (NW == 1 ? 8 : 6);
  // OML: the Sherman-Morrison vector is read from LDS (staged after the line rows once per
  // block) instead of global memory: each lane's read of it depends on its segment, so the
  // global loads were issued one at a time, each waiting out a cache latency, per group.
  const V* om = omega;
  if constexpr (OML) {
    V* s_om = sdata + (size_t)lines_per_grp * pitch;
    for (int q = tid; q < nwi; q += NT) s_om[q] = omega[q];
    om = s_om;  // visible to every wavefront after the first group's copy-in barrier
  }

  for (int64_t grp = grp_begin; grp < ngrp; grp += grp_step) {
    const int64_t line0 = grp * lines_per_grp;
    const int nl = (int)min((int64_t)lines_per_grp, nlines - line0);
    const int cnt = nl * nz;
    const V* src = psi + line0 * nz;
    if (zp == 0) {
      if (sizeof(V) == 8 && al16 && ((line0 * nz) & 1) == 0 && (cnt & 1) == 0) {  // 16-byte copies
        const float4* s4 = reinterpret_cast<const float4*>(src);
        float4* d4 = reinterpret_cast<float4*>(sdata);
        for (int q = tid; q < (cnt >> 1); q += NT) d4[q] = gld(s4 + q);
      } else if constexpr (KB > 1) {
        for (int q0 = tid; q0 < cnt; q0 += KB * NT) {
          V tmp[KB];
#pragma unroll
          for (int k = 0; k < KB; ++k)
            if (q0 + k * NT < cnt) tmp[k] = gld(src + q0 + k * NT);
#pragma unroll
          for (int k = 0; k < KB; ++k)
            if (q0 + k * NT < cnt) sdata[q0 + k * NT] = tmp[k];
        }
      } else {
        for (int q = tid; q < cnt; q += NT) sdata[q] = gld(src + q);
      }
    } else if (pairs) {  // 16-byte global loads; a pair never straddles a line or segment
      const float4* s4 = reinterpret_cast<const float4*>(src);
      int cl = tid / cn, cq = tid % cn;
      for (int f = tid; f < (cnt >> 1); f += NT) {
        const int q = 2 * cq, at = cl * pitch + q + q / MZ;
        const float4 x = gld(s4 + f);
        sdata[at] = vmake<V>(x.x, x.y);
        sdata[at + 1] = vmake<V>(x.z, x.w);
        cq += dq;
        cl += dl;
        if (cq >= cn) {
          cq -= cn;
          ++cl;
        }
      }
    } else if constexpr (KB > 1) {
      int cl = tid / cn, cq = tid % cn;
      for (int f0 = tid; f0 < cnt; f0 += KB * NT) {
        V tmp[KB];
        int at[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          at[k] = cl * pitch + cq + cq / MZ;
          if (f0 + k * NT < cnt) tmp[k] = gld(src + f0 + k * NT);
          cq += dq;
          cl += dl;
          if (cq >= cn) {
            cq -= cn;
            ++cl;
          }
        }
#pragma unroll
        for (int k = 0; k < KB; ++k)
          if (f0 + k * NT < cnt) sdata[at[k]] = tmp[k];
      }
    } else {
      int cl = tid / cn, cq = tid % cn;
      for (int f = tid; f < cnt; f += NT) {
        sdata[cl * pitch + cq + cq / MZ] = gld(src + f);
        cq += dq;
        cl += dl;
        if (cq >= cn) {
          cq -= cn;
          ++cl;
        }
      }
    }
    __syncthreads();

    const int ll = w * L + l;
    const bool act = (ll < nl) && (len > 0);
    V* row = sdata + (act ? ll * pitch : 0);
    V v[MZ];
    z_line_solve<R, MZ, CC>(v, row, act, s, ss, zp, len, nz, nseg, l, p, cf, cP, om, nwi);

    if (act) {
      R vxy = 0;
      if (EPI != 0) {
        const int64_t zl = line0 + ll;  // z line index = i*ny + j
        vxy = vx[zl / ny] + vy[zl % ny];
      }
#pragma unroll
      for (int t = 0; t < MZ; ++t) {
        if (t < len) {
          if (EPI != 0) v[t] = nstep<EPI, R, V>(v[t], (R)1, vxy + pz.at(s + t), g, tau);
          if (NORM) acc = fma((double)v[t].x, (double)v[t].x, fma((double)v[t].y, (double)v[t].y, acc));
          row[ss + t] = v[t];
        }
      }
    }
    __syncthreads();
    V* dst = psi + line0 * nz;
    if (zp == 0) {
      if (sizeof(V) == 8 && al16 && ((line0 * nz) & 1) == 0 && (cnt & 1) == 0) {
        float4* d4 = reinterpret_cast<float4*>(dst);
        const float4* s4 = reinterpret_cast<const float4*>(sdata);
        for (int q = tid; q < (cnt >> 1); q += NT) gst(d4 + q, s4[q]);
      } else {
        for (int q = tid; q < cnt; q += NT) gst(dst + q, sdata[q]);
      }
    } else if (pairs) {
      float4* d4 = reinterpret_cast<float4*>(dst);
      int cl = tid / cn, cq = tid % cn;
      for (int f = tid; f < (cnt >> 1); f += NT) {
        const int q = 2 * cq, at = cl * pitch + q + q / MZ;
        const V a = sdata[at], b = sdata[at + 1];
        gst(d4 + f, make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y));
        cq += dq;
        cl += dl;
        if (cq >= cn) {
          cq -= cn;
          ++cl;
        }
      }
    } else {
      int cl = tid / cn, cq = tid % cn;
      for (int f = tid; f < cnt; f += NT) {
        gst(dst + f, sdata[cl * pitch + cq + cq / MZ]);
        cq += dq;
        cl += dl;
        if (cq >= cn) {
          cq -= cn;
          ++cl;
        }
      }
    }
    __syncthreads();
  }
  return acc;
}


// (i, j, k) of a flat index q = (i ny + j) nz + k, advanced by a fixed stride without a
// division per point: the stride's own (di, dj, dk) digits are added with carries (each
// digit below its radix, so at most one carry per digit)
struct Idx3 {
  int i, j, k;
  int di, dj, dk;
  int ny, nz;
  __device__ __forceinline__ Idx3(int64_t q, int64_t stride, int ny_, int nz_) : ny(ny_), nz(nz_) {
    k = (int)(q % nz);
    const int64_t r = q / nz;
    j = (int)(r % ny);
    i = (int)(r / ny);
    dk = (int)(stride % nz);
    const int64_t rs = stride / nz;
    dj = (int)(rs % ny);
    di = (int)(rs / ny);
  }
  __device__ __forceinline__ void advance() {
    k += dk;
    int c = k >= nz;
    k -= c ? nz : 0;
    j += dj + c;
    c = j >= ny;
    j -= c ? ny : 0;
    i += di + c;
  }
};

__device__ __forceinline__ double block_sum_256(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// sum over a block of NW = 1 or 4 wavefronts (red: 4 doubles of LDS), fixed order
template <int NW> __device__ __forceinline__ double block_sum_w(double v, double* red) {
  static_assert(NW == 1 || NW == 4, "z blocks are 1 or 4 wavefronts");
  if constexpr (NW == 4) return block_sum_256(v, red);
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

}  // namespace gpk
