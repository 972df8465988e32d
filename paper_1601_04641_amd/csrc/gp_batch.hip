// Batched split-step Crank-Nicolson: many independent grids of different sizes advanced by
// the same launches.  One step of a batch is four launches whatever the number of
// instances: x sweep (+ potential step), y sweep, z sweep (+ norm partials), per-instance
// finalize.  A per-block work table maps each block to (instance, block within the
// instance); per-instance descriptors hold the dimensions, the offset of the instance's
// psi in the caller's concatenated buffer, the Crank-Nicolson constants and the offsets
// of its potential tables.  The launch boundaries are the instance-wide barriers between
// the x, y and z phases; converged instances are masked by a flag in their descriptor,
// so captured graphs stay valid.  The sweep bodies are those of the single-grid kernels.
#include "../../include/gp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "gp_device.h"

namespace gpk {

struct BInst {
  int nx, ny, nz, active;
  int64_t off;     // element offset of this instance's psi in the concatenated buffer
  uint32_t bytes;  // size of this instance's psi in bytes
  int split;
  int zpad;              // z sweep LDS layout (z_pad)
  int nseg[3];           // segments per line: x, y (m points each), z (power of two)
  int nw[2][3];          // Sherman-Morrison correction length [imag, real][axis]
  int omega_off[2][3];   // element offsets into the omega table
  int v_off[3];          // element offsets of the x, y, z potential tables
  int zb0, zb1;          // z-sweep blocks of this instance (norm partials)
  int ob0, ob1;          // observables / scale blocks of this instance
  double dt, dV;
  double id2[3];         // 1 / dx^2, 1 / dy^2, 1 / dz^2
  double ph[3], pc[3];   // potential per axis: V(i) = ph ((i - pc) d)^2
  double pd[3];          // grid spacing per axis
  double coef[2][3][8];  // a, b, b_lo, P as (re, im) [imag, real][axis]
};

struct BWork {
  int inst;
  int blk;
};

constexpr int kChunk = 8192;  // points per block of the pointwise batched kernels (32 per thread:
                              // amortises the per-block FP64 reductions of the observables)
constexpr int kMF = 8;        // points per lane of the fused y+z kernel's in-LDS line solves
constexpr int kZGroups = 4;   // consecutive line groups per block of the batched z sweep
constexpr int kYZThreads = 256;  // threads of a fused y+z block (one plane in LDS; 1024 measured slower)

// coordinate and potential of point i along axis a of instance I, from their closed forms
// with rounded operations (no contraction): the values the host computes in FP64
__device__ __forceinline__ double bcoord(const BInst& I, int a, int i) { return ((double)i - I.pc[a]) * I.pd[a]; }
__device__ __forceinline__ double bpot(const BInst& I, int a, double x) { return __dmul_rn(__dmul_rn(I.ph[a], x), x); }

template <typename R> __device__ __forceinline__ typename VecOf<R>::T dval(const double* c) {
  typename VecOf<R>::T v;
  v.x = (R)c[0];
  v.y = (R)c[1];
  return v;
}

template <typename R, int M, int SW, bool CC, int NSTEP, bool LONGHC>
__global__ void __launch_bounds__(1024)
kb_sweep_lines(typename VecOf<R>::T* __restrict__ psi_all, const BInst* __restrict__ inst,
               const BWork* __restrict__ work, int axis, const R* __restrict__ vtab,
               const typename VecOf<R>::T* __restrict__ omega_all, const DevState* __restrict__ st) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const BWork wk = work[blockIdx.x];
  const BInst& I = inst[wk.inst];
  if (!I.active) return;
  constexpr int mode = CC ? 1 : 0;
  const int n = axis == 0 ? I.nx : I.ny;
  const int64_t nlines = axis == 0 ? (int64_t)I.ny * I.nz : (int64_t)I.nx * I.nz;
  const int64_t inner = axis == 0 ? (int64_t)I.ny * I.nz : (int64_t)I.nz;
  const double* cf = I.coef[mode][axis];
  R scale = 1, g = 0, tau = 0;
  if (NSTEP != 0) {
    scale = (R)st[wk.inst].s;
    g = (R)st[wk.inst].g;
    tau = (R)(I.split ? 0.5 * I.dt : I.dt);
  }
  const int nw = I.nw[mode][axis];
  lines_body<R, M, SW, CC, NSTEP, false, LONGHC, kBatchLines<R, NSTEP>, kBatchLines<R, NSTEP>>(psi_all + I.off, psi_all + I.off, I.bytes, dval<R>(cf), dval<R>(cf + 2),
                                  dval<R>(cf + 4), dval<R>(cf + 6), omega_all + I.omega_off[mode][axis],
                                  (LONGHC || nw <= M) ? nw : 0, n,
                                  I.nseg[axis], nlines, inner, Pot1D<R>{(R)I.ph[0], (R)I.pc[0], (R)I.pd[0]},
                                  vtab + I.v_off[1], vtab + I.v_off[2], I.nz, tau, scale, g, wk.blk, smem_raw);
}

template <typename R, int MZ, bool CC, bool NORM, int EPI>
__global__ void __launch_bounds__(256)
kb_sweep_z(typename VecOf<R>::T* __restrict__ psi_all, const BInst* __restrict__ inst, const BWork* __restrict__ work,
           const R* __restrict__ vtab, const typename VecOf<R>::T* __restrict__ omega_all,
           const DevState* __restrict__ st, double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[4];
  const BWork wk = work[blockIdx.x];
  const BInst& I = inst[wk.inst];
  if (!I.active) {
    if (NORM && threadIdx.x == 0) partials[blockIdx.x] = 0.0;
    return;
  }
  constexpr int mode = CC ? 1 : 0;
  const double* cf = I.coef[mode][2];
  R g = 0;
  if (EPI != 0) g = (R)st[wk.inst].g;
  const double acc = z_body<R, MZ, CC, NORM, EPI>(
      psi_all + I.off, dval<R>(cf), dval<R>(cf + 2), dval<R>(cf + 4), dval<R>(cf + 6),
      omega_all + I.omega_off[mode][2], I.nw[mode][2], I.nz, I.nseg[2],
      min((int64_t)I.nx * I.ny, (int64_t)(wk.blk + 1) * kZGroups * 4 * (64 / I.nseg[2])), vtab + I.v_off[0],
      vtab + I.v_off[1], Pot1D<R>{(R)I.ph[2], (R)I.pc[2], (R)I.pd[2]}, I.ny, (R)(0.5 * I.dt), g,
      (int64_t)wk.blk * kZGroups, 1, I.zpad, smem_raw);
  if (NORM) {
    const double t = block_sum_256(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

// Crank-Nicolson solves of nl lines held in LDS (line l, element i at L0 + l * lstride +
// i * stride, n points) in registers, as the register sweeps do it: a wavefront takes
// 64 / nseg lines at a time, lane = line * nseg + segment, MZ consecutive points per lane
// (nseg = the smallest power of two with nseg * MZ >= n).  Each segment runs the
// constant-pivot recurrences from a zero start; the segments of a line are joined by
// shuffle scans of the affine maps (every segment before an active one is full, so spans
// multiply by powers of P = a^MZ and only the offsets travel); the Sherman-Morrison head
// correction u_i += omega_i u_0 (i < nw) comes last.  A lane reads its points and both
// neighbours before any lane of its wavefront writes, and no two wavefronts share a line,
// so no barrier is needed inside; the caller separates passes with barriers.
template <typename R, int MZ, bool CC>
__device__ __forceinline__ void lds_lines_regs(typename VecOf<R>::T* L0, int lstride, int stride, int n, int nl,
                                               const Coef<typename VecOf<R>::T>& cf,
                                               const typename VecOf<R>::T* __restrict__ omega, int nw) {
  typedef typename VecOf<R>::T V;
  int nseg = 1;
  while (nseg * MZ < n) nseg *= 2;
  const int LW = 64 / nseg;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, nwave = (int)(blockDim.x >> 6);
  const int l = lane / nseg, p = lane % nseg;
  const int s = p * MZ;
  const int len = max(0, min(MZ, n - s));
  V cP = cf.a;  // a^MZ
#pragma unroll
  for (int k = 1; k < MZ; ++k) cP = cmul<CC>(cf.a, cP);
  for (int l0 = 0; l0 < nl; l0 += nwave * LW) {
    const int line = l0 + w * LW + l;
    const bool act = line < nl && len > 0;
    V* row = L0 + (int64_t)(act ? line : 0) * lstride;
    V v[MZ];
#pragma unroll
    for (int t = 0; t < MZ; ++t) {
      v[t] = vzero<V>();
      if (act && t < len) v[t] = row[(s + t) * stride];
    }
    const V left = (act && s > 0) ? row[(s - 1) * stride] : vzero<V>();
    const V right = (act && s + len < n) ? row[(s + len) * stride] : vzero<V>();
    V d = vzero<V>();
    {
      V prev = left;
#pragma unroll
      for (int t = 0; t < MZ; ++t) {
        V nxt = right;
        if (t + 1 < MZ) nxt = v[t + 1];
        // past len: zeros in, values never stored (the backward pass restarts from zero
        // there and no later segment of the line is active)
        const V dn = fwd_point<CC, R, V>(cf, prev, nxt, d, v[t]);
        prev = v[t];
        v[t] = dn;
        d = dn;
      }
    }
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
        r = cmul<CC>(cf.a, r);
        v[t] = vadd(v[t], r);
      }
    }
    V u = vzero<V>();
#pragma unroll
    for (int t = MZ - 1; t >= 0; --t) {
      u = cfma<CC>(cf.a, u, v[t]);
      if (t >= len) u = vzero<V>();
      v[t] = u;
    }
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
        r = cmul<CC>(cf.a, r);
        v[t] = vadd(v[t], r);
      }
    }
    if (nw > 0) {
      const V u0 = vmake<V>(__shfl(v[0].x, l * nseg, 64), __shfl(v[0].y, l * nseg, 64));
#pragma unroll
      for (int t = 0; t < MZ; ++t) {
        const int pos = s + t;
        const V c = cfma<CC>(omega[min(pos, nw - 1)], u0, v[t]);
        if (pos < nw) v[t] = c;
      }
    }
    if (act) {
#pragma unroll
      for (int t = 0; t < MZ; ++t)
        if (t < len) row[(s + t) * stride] = v[t];
    }
  }
}

// Fused y and z sweeps of one x-plane of one instance (the plane [y][z] is contiguous in
// psi): load the plane into LDS (row pitch nz + 1, so the z lines of consecutive threads
// fall in different banks), solve the nz y-lines, then the ny z-lines, store, and
// (imaginary time) the FP64 sum |psi|^2 of the plane.  psi crosses HBM twice per step for
// y and z together instead of four times.
template <typename R, bool CC, bool NORM>
__global__ void __launch_bounds__(kYZThreads)
kb_sweep_yz(typename VecOf<R>::T* __restrict__ psi_all, const BInst* __restrict__ inst, const BWork* __restrict__ work,
            const typename VecOf<R>::T* __restrict__ omega_all, double* __restrict__ partials) {
  typedef typename VecOf<R>::T V;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[kYZThreads / 64];
  V* plane = reinterpret_cast<V*>(smem_raw);
  const BWork wk = work[blockIdx.x];
  const BInst& I = inst[wk.inst];
  if (!I.active) {
    if (NORM && threadIdx.x == 0) partials[blockIdx.x] = 0.0;
    return;
  }
  constexpr int mode = CC ? 1 : 0;
  const int ny = I.ny, nz = I.nz, pitch = nz + 1;
  const int np = ny * nz;
  V* g = psi_all + I.off + (int64_t)wk.blk * np;
  // plane in: 16-byte units (E values each), 8 loads in flight per thread; a unit never
  // straddles a row when nz is a multiple of E (else the scalar loop)
  constexpr int E = 16 / (int)sizeof(V);
  const bool vec = (nz % E) == 0 && (reinterpret_cast<uintptr_t>(g) & 15) == 0;
  if (vec) {
    const int nu = np / E;
    const uint4* g4 = reinterpret_cast<const uint4*>(g);
    for (int base = threadIdx.x; base < nu; base += kYZThreads * 8) {
      uint4 r[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (base + k * kYZThreads < nu) r[k] = g4[base + k * kYZThreads];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int u = base + k * kYZThreads;
        if (u < nu) {
          const int q = u * E;
          const V* e = reinterpret_cast<const V*>(&r[k]);
          V* dst = plane + (q / nz) * pitch + q % nz;
#pragma unroll
          for (int h = 0; h < E; ++h) dst[h] = e[h];
        }
      }
    }
  } else {
    for (int q = threadIdx.x; q < np; q += kYZThreads) plane[(q / nz) * pitch + q % nz] = g[q];
  }
  __syncthreads();
  {
    const double* c = I.coef[mode][1];
    const Coef<V> cf{dval<R>(c), dval<R>(c + 2), dval<R>(c + 4)};
    lds_lines_regs<R, kMF, CC>(plane, 1, pitch, ny, nz, cf, omega_all + I.omega_off[mode][1], I.nw[mode][1]);
  }
  __syncthreads();
  {
    const double* c = I.coef[mode][2];
    const Coef<V> cf{dval<R>(c), dval<R>(c + 2), dval<R>(c + 4)};
    lds_lines_regs<R, kMF, CC>(plane, pitch, 1, nz, ny, cf, omega_all + I.omega_off[mode][2], I.nw[mode][2]);
  }
  __syncthreads();
  double acc = 0.0;
  if (vec) {
    const int nu = np / E;
    uint4* g4 = reinterpret_cast<uint4*>(g);
    for (int u = threadIdx.x; u < nu; u += kYZThreads) {
      const int q = u * E;
      uint4 w;
      V* e = reinterpret_cast<V*>(&w);
      const V* src = plane + (q / nz) * pitch + q % nz;
#pragma unroll
      for (int h = 0; h < E; ++h) {
        e[h] = src[h];
        if (NORM) acc += (double)e[h].x * (double)e[h].x + (double)e[h].y * (double)e[h].y;
      }
      g4[u] = w;
    }
  } else {
    for (int q = threadIdx.x; q < np; q += kYZThreads) {
      const V u = plane[(q / nz) * pitch + q % nz];
      g[q] = u;
      if (NORM) acc += (double)u.x * (double)u.x + (double)u.y * (double)u.y;
    }
  }
  if (NORM) {
    // fixed-order sum over the block's wavefronts
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < kYZThreads / 64; ++k) t += red[k];
      partials[blockIdx.x] = t;
    }
  }
}

__global__ void __launch_bounds__(256)
kb_finalize_norm(const double* __restrict__ partials, const BInst* __restrict__ inst, DevState* st) {
  __shared__ double red[4];
  const BInst& I = inst[blockIdx.x];
  if (!I.active) return;
  double acc = 0.0;
  for (int q = I.zb0 + threadIdx.x; q < I.zb1; q += 256) acc += partials[q];
  const double tot = block_sum_256(acc, red);
  if (threadIdx.x == 0) {
    DevState& S = st[blockIdx.x];
    const double npre = tot * I.dV;
    int f = 0;
    if (!isfinite(npre)) f = 1;
    else if (!(npre > 0.0)) f = 2;
    S.npre = npre;
    S.mu_est = (f == 0) ? -log(npre) / (2.0 * I.dt) : 0.0;
    S.flags |= f;
    S.s = (f == 0) ? 1.0 / sqrt(npre) : 1.0;
  }
}

template <typename R>
__global__ void __launch_bounds__(256)
kb_scale(typename VecOf<R>::T* __restrict__ psi_all, const BInst* __restrict__ inst, const BWork* __restrict__ work,
         const DevState* __restrict__ st) {
  const BWork wk = work[blockIdx.x];
  const BInst& I = inst[wk.inst];
  if (!I.active) return;
  const R s = (R)st[wk.inst].s;
  const int64_t npts = (int64_t)I.nx * I.ny * I.nz;
  const int64_t q0 = (int64_t)wk.blk * kChunk, q1 = min(q0 + kChunk, npts);
  typename VecOf<R>::T* psi = psi_all + I.off;
  for (int64_t q = q0 + threadIdx.x; q < q1; q += 256) {
    typename VecOf<R>::T v = psi[q];
    v.x *= s;
    v.y *= s;
    psi[q] = v;
  }
}

__global__ void kb_reset_scale(const BInst* __restrict__ inst, DevState* st, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n && inst[i].active) st[i].s = 1.0;
}

template <typename R>
__global__ void __launch_bounds__(256)
kb_observables(const typename VecOf<R>::T* __restrict__ psi_all, const BInst* __restrict__ inst,
               const BWork* __restrict__ work, double* __restrict__ partials) {
  __shared__ double red[4];
  const BWork wk = work[blockIdx.x];
  const BInst& I = inst[wk.inst];
  const int nx = I.nx, ny = I.ny, nz = I.nz;
  const int64_t npts = (int64_t)nx * ny * nz, sx = (int64_t)ny * nz;
  const typename VecOf<R>::T* psi = psi_all + I.off;
  double acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = 0.0;
  const int64_t q0 = (int64_t)wk.blk * kChunk, q1 = min(q0 + kChunk, npts);
  Idx3 ix(q0 + threadIdx.x, 256, ny, nz);
  for (int64_t q = q0 + threadIdx.x; q < q1; q += 256, ix.advance()) {
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
    const double xi = bcoord(I, 0, i), yj = bcoord(I, 1, j), zk = bcoord(I, 2, k);
    acc[4] += __dadd_rn(__dadd_rn(bpot(I, 0, xi), bpot(I, 1, yj)), bpot(I, 2, zk)) * n2;
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

__global__ void __launch_bounds__(256)
kb_obs_final(const double* __restrict__ partials, const BInst* __restrict__ inst, double* __restrict__ out) {
  __shared__ double red[4];
  const BInst& I = inst[blockIdx.x];
  for (int c = 0; c < 9; ++c) {
    double acc = 0.0;
    for (int q = I.ob0 + threadIdx.x; q < I.ob1; q += 256) acc += partials[(int64_t)q * 9 + c];
    const double t = block_sum_256(acc, red);
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * 9 + c] = t;
  }
}

// Residual sums of the stationary equation, per block: with L = -1/2 lap_h psi + V psi
// (3-point Laplacian, zero ghosts) and Q = |psi|^2 psi:
// { sum|psi|^2, sum|L|^2, sum Re(L* Q), sum|Q|^2, sum Re(psi* L), sum|psi|^4 }.
constexpr int kResSums = 6;

template <typename R>
__global__ void __launch_bounds__(256)
kb_residual(const typename VecOf<R>::T* __restrict__ psi_all, const BInst* __restrict__ inst,
            const BWork* __restrict__ work, double* __restrict__ partials) {
  __shared__ double red[4];
  const BWork wk = work[blockIdx.x];
  const BInst& I = inst[wk.inst];
  const int nx = I.nx, ny = I.ny, nz = I.nz;
  const int64_t npts = (int64_t)nx * ny * nz, sx = (int64_t)ny * nz;
  const typename VecOf<R>::T* psi = psi_all + I.off;
  double acc[kResSums];
#pragma unroll
  for (int c = 0; c < kResSums; ++c) acc[c] = 0.0;
  const int64_t q0 = (int64_t)wk.blk * kChunk, q1 = min(q0 + kChunk, npts);
  Idx3 ix(q0 + threadIdx.x, 256, ny, nz);
  for (int64_t q = q0 + threadIdx.x; q < q1; q += 256, ix.advance()) {
    const int i = ix.i, j = ix.j, k = ix.k;
    const double re = psi[q].x, im = psi[q].y;
    double sr[3] = {0, 0, 0}, si[3] = {0, 0, 0};  // neighbour sums per axis
    if (i > 0) { sr[0] += psi[q - sx].x; si[0] += psi[q - sx].y; }
    if (i + 1 < nx) { sr[0] += psi[q + sx].x; si[0] += psi[q + sx].y; }
    if (j > 0) { sr[1] += psi[q - nz].x; si[1] += psi[q - nz].y; }
    if (j + 1 < ny) { sr[1] += psi[q + nz].x; si[1] += psi[q + nz].y; }
    if (k > 0) { sr[2] += psi[q - 1].x; si[2] += psi[q - 1].y; }
    if (k + 1 < nz) { sr[2] += psi[q + 1].x; si[2] += psi[q + 1].y; }
    const double v =
        __dadd_rn(__dadd_rn(bpot(I, 0, bcoord(I, 0, i)), bpot(I, 1, bcoord(I, 1, j))), bpot(I, 2, bcoord(I, 2, k)));
    double lr = v * re, li = v * im;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lr -= 0.5 * I.id2[a] * (sr[a] - 2.0 * re);
      li -= 0.5 * I.id2[a] * (si[a] - 2.0 * im);
    }
    const double n2 = re * re + im * im;
    const double qr = n2 * re, qi = n2 * im;
    acc[0] += n2;
    acc[1] += lr * lr + li * li;
    acc[2] += lr * qr + li * qi;
    acc[3] += qr * qr + qi * qi;
    acc[4] += re * lr + im * li;
    acc[5] += n2 * n2;
  }
  for (int c = 0; c < kResSums; ++c) {
    const double t = block_sum_256(acc[c], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * kResSums + c] = t;
  }
}

__global__ void __launch_bounds__(256)
kb_res_final(const double* __restrict__ partials, const BInst* __restrict__ inst, double* __restrict__ out) {
  __shared__ double red[4];
  const BInst& I = inst[blockIdx.x];
  for (int c = 0; c < kResSums; ++c) {
    double acc = 0.0;
    for (int q = I.ob0 + threadIdx.x; q < I.ob1; q += 256) acc += partials[(int64_t)q * kResSums + c];
    const double t = block_sum_256(acc, red);
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * kResSums + c] = t;
  }
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
struct BLaunch {
  void* psi;
  const BInst* inst;
  const BWork* work;
  int nblocks;
  int threads;
  size_t lds;
  int axis;
  const void* vtab;
  const void* omega;
  const DevState* st;
  double* partials;
  int m, sw;
  int nstep;    // 0 none, 1 imaginary, 2 real
  bool longhc;  // some instance's head correction is longer than a segment (x/y sweeps)
};

template <typename R, int M, int SW, bool CC, int NSTEP>
static hipError_t gob_lines(const BLaunch& a, hipStream_t s) {
  typedef typename VecOf<R>::T V;
  if (a.longhc)
    hipLaunchKernelGGL((kb_sweep_lines<R, M, SW, CC, NSTEP, true>), dim3(a.nblocks), dim3(a.threads), a.lds, s,
                       (V*)a.psi, a.inst, a.work, a.axis, (const R*)a.vtab, (const V*)a.omega, a.st);
  else
    hipLaunchKernelGGL((kb_sweep_lines<R, M, SW, CC, NSTEP, false>), dim3(a.nblocks), dim3(a.threads), a.lds, s,
                       (V*)a.psi, a.inst, a.work, a.axis, (const R*)a.vtab, (const V*)a.omega, a.st);
  return hipGetLastError();
}
template <typename R, int M, int SW>
static hipError_t gob_lines_mode(bool cc, const BLaunch& a, hipStream_t s) {
  if (!cc) return a.nstep ? gob_lines<R, M, SW, false, 1>(a, s) : gob_lines<R, M, SW, false, 0>(a, s);
  return a.nstep ? gob_lines<R, M, SW, true, 2>(a, s) : gob_lines<R, M, SW, true, 0>(a, s);
}
#define GPB_LINES_SW(R, M)                                 \
  do {                                                     \
    if (a.sw == 1) return gob_lines_mode<R, M, 1>(cc, a, s); \
    if (a.sw == 2) return gob_lines_mode<R, M, 2>(cc, a, s); \
    if (a.sw == 4) return gob_lines_mode<R, M, 4>(cc, a, s); \
  } while (0)
static hipError_t launch_b_lines(int prec, bool cc, const BLaunch& a, hipStream_t s) {
  if (prec == 0) {
    if (a.m == 8) GPB_LINES_SW(float, 8);
    if (a.m == 16) GPB_LINES_SW(float, 16);
    if (a.m == 32) GPB_LINES_SW(float, 32);
  } else {
    if (a.m == 8) GPB_LINES_SW(double, 8);
    if (a.m == 16) GPB_LINES_SW(double, 16);
  }
  return hipErrorInvalidValue;
}
#undef GPB_LINES_SW

template <typename R, int MZ, bool CC, bool NORM, int EPI>
static hipError_t gob_z(const BLaunch& a, hipStream_t s) {
  typedef typename VecOf<R>::T V;
  hipLaunchKernelGGL((kb_sweep_z<R, MZ, CC, NORM, EPI>), dim3(a.nblocks), dim3(256), a.lds, s, (V*)a.psi, a.inst,
                     a.work, (const R*)a.vtab, (const V*)a.omega, a.st, a.partials);
  return hipGetLastError();
}
template <typename R, int MZ>
static hipError_t gob_z_mode(bool cc, const BLaunch& a, hipStream_t s) {
  if (!cc) return a.nstep ? gob_z<R, MZ, false, true, 1>(a, s) : gob_z<R, MZ, false, true, 0>(a, s);
  return a.nstep ? gob_z<R, MZ, true, false, 2>(a, s) : gob_z<R, MZ, true, false, 0>(a, s);
}
#define GPB_Z(R)                                   \
  do {                                             \
    switch (a.m) {                                 \
      case 4: return gob_z_mode<R, 4>(cc, a, s);   \
      case 6: return gob_z_mode<R, 6>(cc, a, s);   \
      case 8: return gob_z_mode<R, 8>(cc, a, s);   \
      case 12: return gob_z_mode<R, 12>(cc, a, s); \
      default: return hipErrorInvalidValue;        \
    }                                              \
  } while (0)
static hipError_t launch_b_z(int prec, bool cc, const BLaunch& a, hipStream_t s) {
  if (prec == 0) GPB_Z(float);
  GPB_Z(double);
}
#undef GPB_Z

static bool b_lines_supported(int prec, int m, int sw) {
  if (sw != 1 && sw != 2 && sw != 4) return false;
  return prec == 0 ? (m == 8 || m == 16 || m == 32) : (m == 8 || m == 16);
}
static bool b_z_supported(int m) { return m == 4 || m == 6 || m == 8 || m == 12; }

}  // namespace gpk

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
using gpk::BInst;
using gpk::BWork;
using gpk::DevState;

namespace {
constexpr int kBGraphSteps = 16;
constexpr int kBKinds = 5;  // x, y, z, finalize, other
}  // namespace

struct gp_batch {
  int n = 0;
  int prec = 0;
  size_t esize = 8;
  std::vector<gp_params> p;
  std::vector<int64_t> off;
  void* psi = nullptr;
  hipStream_t stream = nullptr, cap = nullptr;
  int device = 0;
  int map[5] = {16, 1, 16, 1, 8};  // m_x, sw_x, m_y, sw_y, m_z

  std::vector<BInst> hinst;
  BInst* dinst = nullptr;
  DevState* st = nullptr;
  void* vtab = nullptr;    // storage precision potentials, per instance x | y | z
  void* omega = nullptr;   // storage precision, per instance [mode][axis]
  BWork *wx = nullptr, *wy = nullptr, *wz = nullptr, *wo = nullptr, *wyz = nullptr;
  int nbx = 0, nby = 0, nbz = 0, nbo = 0, nbyz = 0;
  int yz_fuse = 0;          // fuse the y and z sweeps of instances whose x-plane fits in LDS
  int nfused = 0;           // instances on the fused path
  size_t max_lds = 65536;   // dynamic LDS per block available to the fused kernel
  size_t ldsyz = 0;
  // fused y+z launches, one per plane-size class: blocks [start, start + count) of wyz,
  // dynamic LDS of the class's largest plane
  struct YZClass {
    int start, count;
    size_t lds;
  };
  std::vector<YZClass> yzcls;
  int lds_cu = 65536;  // LDS per CU
  int thrx = 64, thry = 64;
  bool need_hc[2][2] = {{false, false}, {false, false}};  // [mode][axis]: nw > m somewhere
  size_t ldsx = 0, ldsy = 0, ldsz = 0;
  double* zpart = nullptr;
  double* opart = nullptr;
  double* oout = nullptr;
  double* host = nullptr;  // pinned, 9n doubles
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::vector<uint8_t> active;
  std::vector<int64_t> steps;

  bool timing = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  double tsum[kBKinds] = {0};
  int64_t tcnt[kBKinds] = {0};
  char err[256] = {0};
};

namespace {

int bfail(gp_batch* b, hipError_t e, const char* where) {
  if (b) snprintf(b->err, sizeof(b->err), "%s: %s", where, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? GP_ERR_OOM : GP_ERR_HIP;
}
#define BCHK(b, expr)                                 \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return bfail(b, e_, #expr); \
  } while (0)

int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

bool bad_inst(const gp_params& p) {
  if (p.nx < 3 || p.ny < 3 || p.nz < 3 || p.nx > 1024 || p.ny > 1024 || p.nz > 1024) return true;
  if (!(p.dx > 0) || !(p.dy > 0) || !(p.dz > 0) || !(p.dt > 0)) return true;
  if (!std::isfinite(p.dx) || !std::isfinite(p.dy) || !std::isfinite(p.dz) || !std::isfinite(p.dt)) return true;
  if (!(p.nux >= 0) || !(p.nuy >= 0) || !(p.nuz >= 0) || !std::isfinite(p.g)) return true;
  if (!std::isfinite(p.nux) || !std::isfinite(p.nuy) || !std::isfinite(p.nuz)) return true;
  if (p.split != GP_SPLIT_LIE && p.split != GP_SPLIT_STRANG) return true;
  return false;
}

void bfree(gp_batch* b) {
  for (auto& g : b->gexec)
    if (g) (void)hipGraphExecDestroy(g), g = nullptr;
  for (auto& r : b->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  b->recs.clear();
  if (b->cap) (void)hipStreamDestroy(b->cap);
  (void)hipFree(b->dinst);
  (void)hipFree(b->st);
  (void)hipFree(b->vtab);
  (void)hipFree(b->omega);
  (void)hipFree(b->wx);
  (void)hipFree(b->wy);
  (void)hipFree(b->wz);
  (void)hipFree(b->wo);
  (void)hipFree(b->wyz);
  (void)hipFree(b->zpart);
  (void)hipFree(b->opart);
  (void)hipFree(b->oout);
  if (b->host) (void)hipHostFree(b->host);
}

template <typename T>
int bdalloc(gp_batch* b, T** ptr, size_t bytes) {
  hipError_t e = gpk::dev_alloc((void**)ptr, bytes > 0 ? bytes : 16);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return bfail(b, e, "hipMalloc");
  }
  return GP_OK;
}

template <typename T>
int upload(gp_batch* b, T** dptr, const std::vector<T>& v) {
  (void)hipFree(*dptr);
  *dptr = nullptr;
  int rc = bdalloc(b, dptr, v.size() * sizeof(T));
  if (rc) return rc;
  if (!v.empty()) BCHK(b, hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return GP_OK;
}

// Lay out descriptors, constants, work tables and scratch for the current mapping.
int configure(gp_batch* b) {
  for (auto& g : b->gexec)
    if (g) (void)hipGraphExecDestroy(g), g = nullptr;
  const int mx = b->map[0], swx = b->map[1], my = b->map[2], swy = b->map[3], mz = b->map[4];
  if (!gpk::b_lines_supported(b->prec, mx, swx) || !gpk::b_lines_supported(b->prec, my, swy) ||
      !gpk::b_z_supported(mz))
    return GP_ERR_INVALID;
  const bool f32 = b->prec == GP_C64;
  std::vector<BInst> hi(b->n);
  std::vector<BWork> wx, wy, wz, wo, wyz;
  std::vector<int> yzb0(b->n, 0), yzb1(b->n, 0);
  std::vector<size_t> lyzv(b->n, 0);
  std::vector<unsigned char> omega;
  size_t ldsyz = 0;
  int nfused = 0;
  bool need_hc[2][2] = {{false, false}, {false, false}};
  int wavesx = 1, wavesy = 1;
  size_t ldsz = 0;
  int voff = 0;
  for (int i = 0; i < b->n; ++i) {
    const gp_params& p = b->p[i];
    BInst& I = hi[i];
    I.nx = p.nx;
    I.ny = p.ny;
    I.nz = p.nz;
    I.active = b->active[i];
    I.off = b->off[i];
    I.bytes = (uint32_t)((int64_t)p.nx * p.ny * p.nz * b->esize);
    I.split = p.split;
    I.dt = p.dt;
    I.dV = p.dx * p.dy * p.dz;
    I.id2[0] = 1.0 / (p.dx * p.dx);
    I.id2[1] = 1.0 / (p.dy * p.dy);
    I.id2[2] = 1.0 / (p.dz * p.dz);
    {
      const double nu3[3] = {p.nux, p.nuy, p.nuz}, d3[3] = {p.dx, p.dy, p.dz};
      const int n3[3] = {p.nx, p.ny, p.nz};
      for (int a = 0; a < 3; ++a) {
        I.ph[a] = 0.5 * nu3[a] * nu3[a];
        I.pc[a] = 0.5 * (n3[a] - 1);
        I.pd[a] = d3[a];
      }
    }
    const int n[3] = {p.nx, p.ny, p.nz};
    const double d[3] = {p.dx, p.dy, p.dz};
    I.nseg[0] = cdiv(p.nx, mx);
    I.nseg[1] = cdiv(p.ny, my);
    int seg = 2;
    while (seg < 64 && (int64_t)seg * mz < p.nz) seg <<= 1;
    if ((int64_t)seg * mz < p.nz) return GP_ERR_UNSUPPORTED;
    I.nseg[2] = seg;
    const size_t lyz = (size_t)p.ny * (p.nz + 1) * b->esize;
    const bool fuse = b->yz_fuse && p.split == GP_SPLIT_LIE && p.ny <= 256 && p.nz <= 256 && lyz <= b->max_lds;
    if (cdiv(I.nseg[0], swx) > 16 || (!fuse && cdiv(I.nseg[1], swy) > 16)) return GP_ERR_UNSUPPORTED;
    I.zpad = gpk::z_pad(p.nz, seg, mz, b->esize);
    const size_t lz = gpk::z_lds(p.nz, seg, mz, I.zpad, b->esize);
    if (!fuse && lz + 512 > 65536) return GP_ERR_UNSUPPORTED;
    if (!fuse) ldsz = std::max(ldsz, lz);
    if (fuse) ldsyz = std::max(ldsyz, lyz);
    nfused += fuse ? 1 : 0;
    wavesx = std::max(wavesx, cdiv(I.nseg[0], swx));
    if (!fuse) wavesy = std::max(wavesy, cdiv(I.nseg[1], swy));
    const int m[3] = {mx, my, mz};
    for (int mode = 0; mode < 2; ++mode)
      for (int a = 0; a < 3; ++a) {
        gpk::AxisConst ac;
        gpk::cn_axis_constants(n[a], d[a], p.dt, mode, m[a], f32, &ac);
        if (a < 2 && ac.nw > m[a]) need_hc[mode][a] = true;  // LONGHC sweep instances
        for (int q = 0; q < 8; ++q) I.coef[mode][a][q] = ac.coef[q];
        I.nw[mode][a] = ac.nw;
        I.omega_off[mode][a] = (int)(omega.size() / b->esize);
        std::vector<unsigned char> bytes;
        gpk::pack_complex(ac.omega, f32, bytes);
        omega.insert(omega.end(), bytes.begin(), bytes.end());
      }
    for (int a = 0; a < 3; ++a) {
      I.v_off[a] = voff;
      voff += n[a];
    }
    const int bx = cdiv((int64_t)p.ny * p.nz, 64 / swx), by = cdiv((int64_t)p.nx * p.nz, 64 / swy);
    const int bz = cdiv((int64_t)p.nx * p.ny, 4 * (64 / seg) * gpk::kZGroups);
    const int bo = cdiv((int64_t)p.nx * p.ny * p.nz, gpk::kChunk);
    for (int k = 0; k < bx; ++k) wx.push_back({i, k});
    if (fuse) {
      lyzv[i] = lyz;  // blocks added below, grouped by plane-size class
      I.zb0 = I.zb1 = -1;  // set below: fused partials follow the z-sweep partials
    } else {
      for (int k = 0; k < by; ++k) wy.push_back({i, k});
      I.zb0 = (int)wz.size();
      for (int k = 0; k < bz; ++k) wz.push_back({i, k});
      I.zb1 = (int)wz.size();
    }
    I.ob0 = (int)wo.size();
    for (int k = 0; k < bo; ++k) wo.push_back({i, k});
    I.ob1 = (int)wo.size();
  }
  // fused instances grouped by how many of their blocks fit on a CU (LDS bound), so that
  // small planes are not launched with the LDS of the largest one; one block per x-plane
  struct YZClassH {
    int start, count;
    size_t lds;
    int bpc;
  };
  std::vector<YZClassH> cls;
  {
    std::vector<int> order;
    for (int i = 0; i < b->n; ++i)
      if (lyzv[i] > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return lyzv[u] < lyzv[v]; });
    auto bpc = [&](size_t l) { return (int)std::min<size_t>(8, (size_t)b->lds_cu / l); };
    for (int i : order) {
      if (cls.empty() || bpc(lyzv[i]) != cls.back().bpc) cls.push_back({(int)wyz.size(), 0, 0, bpc(lyzv[i])});
      yzb0[i] = (int)wyz.size();
      for (int k = 0; k < b->p[i].nx; ++k) wyz.push_back({i, k});
      yzb1[i] = (int)wyz.size();
      cls.back().count = (int)wyz.size() - cls.back().start;
      cls.back().lds = std::max(cls.back().lds, lyzv[i]);
    }
  }
  for (int i = 0; i < b->n; ++i)
    if (hi[i].zb0 < 0) {
      hi[i].zb0 = (int)wz.size() + yzb0[i];
      hi[i].zb1 = (int)wz.size() + yzb1[i];
    }
  // potential tables (storage precision; the FP64 reductions evaluate the closed forms)
  std::vector<double> vd(voff);
  std::vector<float> vf(voff);
  for (int i = 0; i < b->n; ++i) {
    const gp_params& p = b->p[i];
    const int n[3] = {p.nx, p.ny, p.nz};
    const double d[3] = {p.dx, p.dy, p.dz}, nu[3] = {p.nux, p.nuy, p.nuz};
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < n[a]; ++k) {
        const double x = (k - 0.5 * (n[a] - 1)) * d[a];
        vd[hi[i].v_off[a] + k] = 0.5 * nu[a] * nu[a] * x * x;
        vf[hi[i].v_off[a] + k] = (float)(0.5 * nu[a] * nu[a] * x * x);
      }
  }
  int rc;
  (void)hipFree(b->vtab);
  b->vtab = nullptr;
  if (f32) {
    float* t = nullptr;
    if ((rc = upload(b, &t, vf))) return rc;
    b->vtab = t;
  } else {
    double* t = nullptr;
    if ((rc = upload(b, &t, vd))) return rc;
    b->vtab = t;
  }
  unsigned char* om = nullptr;
  if ((rc = upload(b, &om, omega))) return rc;
  (void)hipFree(b->omega);
  b->omega = om;
  if ((rc = upload(b, &b->wx, wx)) || (rc = upload(b, &b->wy, wy)) || (rc = upload(b, &b->wz, wz)) ||
      (rc = upload(b, &b->wo, wo)) || (rc = upload(b, &b->wyz, wyz)) || (rc = upload(b, &b->dinst, hi)))
    return rc;
  if (ldsyz > 65536) {  // opt in to the large LDS allocation for the kernels this batch uses
    hipError_t e;
    if (f32) {
      e = hipFuncSetAttribute((const void*)gpk::kb_sweep_yz<float, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsyz);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)gpk::kb_sweep_yz<float, true, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsyz);
    } else {
      e = hipFuncSetAttribute((const void*)gpk::kb_sweep_yz<double, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsyz);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)gpk::kb_sweep_yz<double, true, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsyz);
    }
    if (e != hipSuccess) return bfail(b, e, "hipFuncSetAttribute");
  }
  b->hinst = hi;
  for (int mode = 0; mode < 2; ++mode)
    for (int a = 0; a < 2; ++a) b->need_hc[mode][a] = need_hc[mode][a];
  b->nbx = (int)wx.size();
  b->nby = (int)wy.size();
  b->nbz = (int)wz.size();
  b->nbo = (int)wo.size();
  b->nbyz = (int)wyz.size();
  b->ldsyz = ldsyz;
  b->yzcls.clear();
  for (const YZClassH& c : cls) b->yzcls.push_back({c.start, c.count, c.lds});
  b->nfused = nfused;
  b->thrx = wavesx * 64;
  b->thry = wavesy * 64;
  b->ldsx = (size_t)3 * wavesx * swx * (64 / swx) * b->esize;
  b->ldsy = (size_t)3 * wavesy * swy * (64 / swy) * b->esize;
  b->ldsz = ldsz;
  (void)hipFree(b->zpart);
  (void)hipFree(b->opart);
  b->zpart = b->opart = nullptr;
  if ((rc = bdalloc(b, &b->zpart, (size_t)(b->nbz + b->nbyz + 1) * sizeof(double)))) return rc;
  if ((rc = bdalloc(b, &b->opart, (size_t)b->nbo * 9 * sizeof(double)))) return rc;
  return GP_OK;
}

template <typename F>
int btimed(gp_batch* b, hipStream_t s, int kind, F fn) {
  if (!b->timing || s != b->stream) {
    hipError_t e = fn(s);
    return e == hipSuccess ? GP_OK : bfail(b, e, "kernel launch");
  }
  hipEvent_t e0, e1;
  BCHK(b, hipEventCreate(&e0));
  BCHK(b, hipEventCreate(&e1));
  BCHK(b, hipEventRecord(e0, s));
  hipError_t e = fn(s);
  if (e != hipSuccess) return bfail(b, e, "kernel launch");
  BCHK(b, hipEventRecord(e1, s));
  b->recs.push_back({kind, e0, e1});
  return GP_OK;
}

int bharvest(gp_batch* b) {
  if (b->recs.empty()) return GP_OK;
  BCHK(b, hipStreamSynchronize(b->stream));
  for (auto& r : b->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      b->tsum[r.kind] += ms;
      b->tcnt[r.kind] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  b->recs.clear();
  return GP_OK;
}

int benqueue_step(gp_batch* b, int mode, hipStream_t s) {
  const bool cc = mode == 1;
  const int strang = b->p[0].split == GP_SPLIT_STRANG;
  gpk::BLaunch ax{b->psi, b->dinst, b->wx, b->nbx, b->thrx, b->ldsx, 0, b->vtab, b->omega, b->st, nullptr,
                  b->map[0], b->map[1], mode == 0 ? 1 : 2, b->need_hc[mode][0]};
  gpk::BLaunch ay{b->psi, b->dinst, b->wy, b->nby, b->thry, b->ldsy, 1, b->vtab, b->omega, b->st, nullptr,
                  b->map[2], b->map[3], 0, b->need_hc[mode][1]};
  gpk::BLaunch az{b->psi, b->dinst, b->wz, b->nbz, 256, b->ldsz, 2, b->vtab, b->omega, b->st, b->zpart,
                  b->map[4], 0, strang ? (mode == 0 ? 1 : 2) : 0, false};
  int rc = btimed(b, s, 0, [&](hipStream_t t) {
    return gpk::launch_b_lines(b->prec, cc, ax, t);
  });
  if (rc) return rc;
  if (b->nby > 0) {
    rc = btimed(b, s, 1, [&](hipStream_t t) {
      return gpk::launch_b_lines(b->prec, cc, ay, t);
    });
    if (rc) return rc;
  }
  if (b->nbz > 0) {
    rc = btimed(b, s, 2, [&](hipStream_t t) { return gpk::launch_b_z(b->prec, cc, az, t); });
    if (rc) return rc;
  }
  if (b->nbyz > 0) {  // fused y+z sweeps (timed with the z sweeps), one launch per plane-size class
    rc = btimed(b, s, 2, [&](hipStream_t t) {
      for (const auto& c : b->yzcls) {
        double* part = b->zpart + b->nbz + c.start;
        const gpk::BWork* wk = b->wyz + c.start;
        const dim3 grid(c.count), blk(gpk::kYZThreads);
        if (b->prec == GP_C64) {
          if (cc)
            hipLaunchKernelGGL((gpk::kb_sweep_yz<float, true, false>), grid, blk, c.lds, t, (float2*)b->psi, b->dinst,
                               wk, (const float2*)b->omega, part);
          else
            hipLaunchKernelGGL((gpk::kb_sweep_yz<float, false, true>), grid, blk, c.lds, t, (float2*)b->psi,
                               b->dinst, wk, (const float2*)b->omega, part);
        } else {
          if (cc)
            hipLaunchKernelGGL((gpk::kb_sweep_yz<double, true, false>), grid, blk, c.lds, t, (double2*)b->psi,
                               b->dinst, wk, (const double2*)b->omega, part);
          else
            hipLaunchKernelGGL((gpk::kb_sweep_yz<double, false, true>), grid, blk, c.lds, t, (double2*)b->psi,
                               b->dinst, wk, (const double2*)b->omega, part);
        }
      }
      return hipGetLastError();
    });
    if (rc) return rc;
  }
  if (mode == 0) {
    rc = btimed(b, s, 3, [&](hipStream_t t) {
      hipLaunchKernelGGL(gpk::kb_finalize_norm, dim3(b->n), dim3(256), 0, t, b->zpart, b->dinst, b->st);
      return hipGetLastError();
    });
    if (rc) return rc;
  }
  return GP_OK;
}

int bensure_graph(gp_batch* b, int mode) {
  if (b->gexec[mode]) return GP_OK;
  if (!b->cap) BCHK(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  BCHK(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  int rc = GP_OK;
  for (int k = 0; k < kBGraphSteps && rc == GP_OK; ++k) rc = benqueue_step(b, mode, b->cap);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return bfail(b, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->gexec[mode], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->gexec[mode] = nullptr;
    return bfail(b, e, "hipGraphInstantiate");
  }
  return GP_OK;
}

int bset_active(gp_batch* b, const uint8_t* active) {
  if (!active) return GP_OK;
  bool changed = false;
  for (int i = 0; i < b->n; ++i) {
    const int a = active[i] ? 1 : 0;
    if (b->hinst[i].active != a) {
      b->hinst[i].active = a;
      b->active[i] = (uint8_t)a;
      changed = true;
    }
  }
  if (!changed) return GP_OK;
  BCHK(b, hipStreamSynchronize(b->stream));
  BCHK(b, hipMemcpy(b->dinst, b->hinst.data(), b->hinst.size() * sizeof(BInst), hipMemcpyHostToDevice));
  return GP_OK;
}

int brun(gp_batch* b, int mode, int32_t n) {
  int32_t left = n;
  if (!b->timing && n >= kBGraphSteps) {
    int rc = bensure_graph(b, mode);
    if (rc) return rc;
    while (left >= kBGraphSteps) {
      BCHK(b, hipGraphLaunch(b->gexec[mode], b->stream));
      left -= kBGraphSteps;
    }
  }
  for (int32_t k = 0; k < left; ++k) {
    int rc = benqueue_step(b, mode, b->stream);
    if (rc) return rc;
  }
  for (int i = 0; i < b->n; ++i)
    if (b->active[i]) b->steps[i] += n;
  return GP_OK;
}

int bobserve(gp_batch* b) {
  int rc = btimed(b, b->stream, 4, [&](hipStream_t t) {
    if (b->prec == GP_C64)
      hipLaunchKernelGGL(gpk::kb_observables<float>, dim3(b->nbo), dim3(256), 0, t, (const float2*)b->psi, b->dinst,
                         b->wo, b->opart);
    else
      hipLaunchKernelGGL(gpk::kb_observables<double>, dim3(b->nbo), dim3(256), 0, t, (const double2*)b->psi,
                         b->dinst, b->wo, b->opart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gpk::kb_obs_final, dim3(b->n), dim3(256), 0, t, b->opart, b->dinst, b->oout);
    return hipGetLastError();
  });
  if (rc) return rc;
  BCHK(b, hipMemcpyAsync(b->host, b->oout, (size_t)b->n * 9 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  // scale to raw sums: N, Tx, Ty, Tz, U, I, X2, Y2, Z2
  int status = GP_OK;
  for (int i = 0; i < b->n; ++i) {
    const gp_params& p = b->p[i];
    double* r = b->host + (size_t)9 * i;
    const double dV = p.dx * p.dy * p.dz;
    const double d2[3] = {p.dx * p.dx, p.dy * p.dy, p.dz * p.dz};
    r[0] *= dV;
    for (int a = 0; a < 3; ++a) r[1 + a] *= 0.5 * dV / d2[a];
    for (int q = 4; q < 9; ++q) r[q] *= dV;
    for (int q = 0; q < 9; ++q)
      if (!std::isfinite(r[q])) status = GP_ERR_NONFINITE;
    if (status == GP_OK && !(r[0] > 0)) status = GP_ERR_ZERO_NORM;
  }
  return status;
}

}  // namespace

extern "C" {

int gp_batch_init(const gp_params* p, int32_t n, void* psi_dev, const int64_t* offsets, void* hip_stream,
                  gp_batch** out) {
  if (!out) return GP_ERR_INVALID;
  *out = nullptr;
  if (!p || n < 1 || !psi_dev || !offsets) return GP_ERR_INVALID;
  const int prec = p[0].precision;
  if (prec != GP_C64 && prec != GP_C128) return GP_ERR_INVALID;
  const int64_t es = prec == GP_C128 ? 16 : 8;
  if (reinterpret_cast<uintptr_t>(psi_dev) % (uintptr_t)es != 0) return GP_ERR_INVALID;
  for (int i = 0; i < n; ++i) {
    if (bad_inst(p[i]) || p[i].precision != prec || p[i].split != p[0].split) return GP_ERR_INVALID;
    if (offsets[i] < 0) return GP_ERR_INVALID;
    if ((int64_t)p[i].nx * p[i].ny * p[i].nz * es >= (int64_t)1 << 32) return GP_ERR_UNSUPPORTED;
  }
  // instance regions [off, off + size) must not overlap, and must lie inside the device
  // allocation that holds psi_dev (when the runtime can name it)
  {
    std::vector<std::pair<int64_t, int64_t>> reg(n);
    for (int i = 0; i < n; ++i) reg[i] = {offsets[i], offsets[i] + (int64_t)p[i].nx * p[i].ny * p[i].nz};
    std::sort(reg.begin(), reg.end());
    for (int i = 1; i < n; ++i)
      if (reg[i].first < reg[i - 1].second) return GP_ERR_INVALID;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, psi_dev) == hipSuccess && base) {
      const uintptr_t end = reinterpret_cast<uintptr_t>(base) + size;
      const uintptr_t last = reinterpret_cast<uintptr_t>(psi_dev) + (uintptr_t)(reg[n - 1].second * es);
      if (last > end) return GP_ERR_INVALID;
    } else {
      (void)hipGetLastError();
    }
  }
  gp_batch* b = new (std::nothrow) gp_batch;
  if (!b) return GP_ERR_OOM;
  b->n = n;
  b->prec = prec;
  b->esize = prec == GP_C128 ? 16 : 8;
  b->p.assign(p, p + n);
  b->off.assign(offsets, offsets + n);
  b->psi = psi_dev;
  b->stream = (hipStream_t)hip_stream;
  b->active.assign(n, 1);
  b->steps.assign(n, 0);
  if (prec == GP_C128) {
    b->map[0] = 8;
    b->map[2] = 8;
  }
  int rc = GP_OK;
  hipPointerAttribute_t attr;
  if (hipGetDevice(&b->device) != hipSuccess || hipPointerGetAttributes(&attr, psi_dev) != hipSuccess ||
      (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)) {
    (void)hipGetLastError();
    rc = GP_ERR_INVALID;
  }
  if (rc == GP_OK) {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device) == hipSuccess && lds > 0)
      b->max_lds = (size_t)lds - 512;  // the fused kernel's static shared array
    else
      (void)hipGetLastError();
    int ldc = 0;
    if (hipDeviceGetAttribute(&ldc, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, b->device) == hipSuccess &&
        ldc >= 65536)
      b->lds_cu = ldc;
    else
      (void)hipGetLastError();
  }
  if (rc == GP_OK) rc = configure(b);
  if (rc == GP_OK) rc = bdalloc(b, &b->st, (size_t)n * sizeof(DevState));
  if (rc == GP_OK) rc = bdalloc(b, &b->oout, (size_t)n * 9 * sizeof(double));
  if (rc == GP_OK) {
    if (hipHostMalloc((void**)&b->host, (size_t)n * 9 * sizeof(double), hipHostMallocDefault) != hipSuccess)
      rc = GP_ERR_OOM;
  }
  if (rc == GP_OK) {
    std::vector<DevState> s0(n);
    for (int i = 0; i < n; ++i) {
      s0[i] = DevState{};
      s0[i].s = 1.0;
      s0[i].g = p[i].g;
      s0[i].npre = 1.0;
    }
    if (hipMemcpy(b->st, s0.data(), n * sizeof(DevState), hipMemcpyHostToDevice) != hipSuccess) rc = GP_ERR_HIP;
  }
  if (rc != GP_OK) {
    bfree(b);
    delete b;
    return rc;
  }
  *out = b;
  return GP_OK;
}

int gp_batch_destroy(gp_batch* b) {
  if (!b) return GP_ERR_INVALID;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  bfree(b);
  delete b;
  return GP_OK;
}

int gp_batch_step_imag(gp_batch* b, int32_t nsteps, const uint8_t* active) {
  if (!b || nsteps < 0) return GP_ERR_INVALID;
  int rc = bset_active(b, active);
  if (rc || nsteps == 0) return rc;
  if ((rc = brun(b, 0, nsteps))) return rc;
  return btimed(b, b->stream, 4, [&](hipStream_t t) {
    if (b->prec == GP_C64)
      hipLaunchKernelGGL(gpk::kb_scale<float>, dim3(b->nbo), dim3(256), 0, t, (float2*)b->psi, b->dinst, b->wo, b->st);
    else
      hipLaunchKernelGGL(gpk::kb_scale<double>, dim3(b->nbo), dim3(256), 0, t, (double2*)b->psi, b->dinst, b->wo,
                         b->st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gpk::kb_reset_scale, dim3((b->n + 255) / 256), dim3(256), 0, t, b->dinst, b->st, b->n);
    return hipGetLastError();
  });
}

int gp_batch_step_real(gp_batch* b, int32_t nsteps, const uint8_t* active) {
  if (!b || nsteps < 0) return GP_ERR_INVALID;
  int rc = bset_active(b, active);
  if (rc || nsteps == 0) return rc;
  return brun(b, 1, nsteps);
}

int gp_batch_raw_sums(gp_batch* b, double* raw) {
  if (!b || !raw) return GP_ERR_INVALID;
  int rc = bobserve(b);
  std::memcpy(raw, b->host, (size_t)b->n * 9 * sizeof(double));
  return rc;
}

int gp_batch_norm(gp_batch* b, double* norm) {
  if (!b || !norm) return GP_ERR_INVALID;
  int rc = bobserve(b);
  for (int i = 0; i < b->n; ++i) norm[i] = b->host[(size_t)9 * i];
  return rc;
}

int gp_batch_energy_mu(gp_batch* b, double* energy, double* mu) {
  if (!b || !energy || !mu) return GP_ERR_INVALID;
  int rc = bobserve(b);
  for (int i = 0; i < b->n; ++i) {
    const double* r = b->host + (size_t)9 * i;
    const double N = r[0];
    const double lin = (r[1] + r[2] + r[3] + r[4]) / N;
    const double nl = b->p[i].g * r[5] / (N * N);
    energy[i] = lin + 0.5 * nl;
    mu[i] = lin + nl;
  }
  return rc;
}

int gp_batch_residual(gp_batch* b, double* res, double* mu) {
  if (!b || !res) return GP_ERR_INVALID;
  int rc = btimed(b, b->stream, 4, [&](hipStream_t t) {
    if (b->prec == GP_C64)
      hipLaunchKernelGGL(gpk::kb_residual<float>, dim3(b->nbo), dim3(256), 0, t, (const float2*)b->psi, b->dinst,
                         b->wo, b->opart);
    else
      hipLaunchKernelGGL(gpk::kb_residual<double>, dim3(b->nbo), dim3(256), 0, t, (const double2*)b->psi, b->dinst,
                         b->wo, b->opart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gpk::kb_res_final, dim3(b->n), dim3(256), 0, t, b->opart, b->dinst, b->oout);
    return hipGetLastError();
  });
  if (rc) return rc;
  BCHK(b, hipMemcpyAsync(b->host, b->oout, (size_t)b->n * gpk::kResSums * sizeof(double), hipMemcpyDeviceToHost,
                         b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  int status = GP_OK;
  for (int i = 0; i < b->n; ++i) {
    const double* r = b->host + (size_t)gpk::kResSums * i;
    const double g = b->p[i].g, dV = b->p[i].dx * b->p[i].dy * b->p[i].dz;
    const double N = dV * r[0];
    // phi = psi / sqrt(N):  H phi = L / sqrt(N) + g Q / N^{3/2}
    const double hh = dV * (r[1] / N + 2.0 * g * r[2] / (N * N) + g * g * r[3] / (N * N * N));
    const double m = dV * (r[4] / N + g * r[5] / (N * N));
    const double r2 = hh - m * m;
    res[i] = std::sqrt(r2 > 0.0 ? r2 : 0.0);
    if (mu) mu[i] = m;
    if (!std::isfinite(res[i]) || !std::isfinite(m)) status = GP_ERR_NONFINITE;
    else if (!(N > 0)) status = GP_ERR_ZERO_NORM;
  }
  return status;
}

int gp_batch_rms(gp_batch* b, double* rms4) {
  if (!b || !rms4) return GP_ERR_INVALID;
  int rc = bobserve(b);
  for (int i = 0; i < b->n; ++i) {
    const double* r = b->host + (size_t)9 * i;
    rms4[4 * i] = std::sqrt(r[6] / r[0]);
    rms4[4 * i + 1] = std::sqrt(r[7] / r[0]);
    rms4[4 * i + 2] = std::sqrt(r[8] / r[0]);
    rms4[4 * i + 3] = std::sqrt((r[6] + r[7] + r[8]) / r[0]);
  }
  return rc;
}

int gp_batch_status(gp_batch* b, int64_t* steps_done, double* mu_est, int32_t* flags) {
  if (!b) return GP_ERR_INVALID;
  std::vector<DevState> s(b->n);
  BCHK(b, hipStreamSynchronize(b->stream));
  BCHK(b, hipMemcpy(s.data(), b->st, b->n * sizeof(DevState), hipMemcpyDeviceToHost));
  for (int i = 0; i < b->n; ++i) {
    if (steps_done) steps_done[i] = b->steps[i];
    if (mu_est) mu_est[i] = s[i].mu_est;
    if (flags) flags[i] = s[i].flags;
  }
  return GP_OK;
}

int gp_batch_converge_imag(gp_batch* b, double tol, int32_t check_every, int64_t max_steps, int64_t* steps_taken,
                           double* mu, int32_t* converged) {
  if (!b || !(tol > 0) || max_steps < 0 || check_every < 0) return GP_ERR_INVALID;
  int32_t K = check_every;
  if (K == 0) {
    double dtmin = b->p[0].dt;
    for (auto& q : b->p) dtmin = std::min(dtmin, q.dt);
    K = std::max(1, (int32_t)std::ceil(0.25 / dtmin));
  }
  const int n = b->n;
  std::vector<double> cur(n, NAN), e(n);
  std::vector<uint8_t> act(n, 1);
  std::vector<int64_t> taken(n, 0);
  std::vector<int32_t> conv(n, 0);
  std::vector<gpk::StopRule> rule(n);
  int rc = bset_active(b, act.data());
  if (rc) return rc;
  int64_t done = 0;
  int remaining = n;
  while (done < max_steps && remaining > 0) {
    const int32_t k = (int32_t)std::min<int64_t>(K, max_steps - done);
    if ((rc = gp_batch_step_imag(b, k, act.data()))) break;
    done += k;
    for (int i = 0; i < n; ++i)
      if (act[i]) taken[i] += k;
    if ((rc = gp_batch_energy_mu(b, e.data(), cur.data())) && rc != GP_ERR_NONFINITE && rc != GP_ERR_ZERO_NORM)
      break;
    rc = GP_OK;
    for (int i = 0; i < n; ++i) {
      if (!act[i]) continue;
      // the stopping rule of gp_converge_imag on mu of every check
      if (rule[i].update(cur[i], tol)) {
        conv[i] = 1;
        act[i] = 0;
        --remaining;
      } else if (!std::isfinite(cur[i])) {
        act[i] = 0;  // diverged: stop it, report not converged
        --remaining;
      }
    }
  }
  std::vector<uint8_t> all(n, 1);
  int rc2 = bset_active(b, all.data());
  if (rc == GP_OK) rc = rc2;
  for (int i = 0; i < n; ++i) {
    if (steps_taken) steps_taken[i] = taken[i];
    if (mu) mu[i] = cur[i];
    if (converged) converged[i] = conv[i];
  }
  return rc;
}

int gp_batch_set_yz_fusion(gp_batch* b, int32_t enable) {
  if (!b) return GP_ERR_INVALID;
  BCHK(b, hipStreamSynchronize(b->stream));
  const int old = b->yz_fuse;
  b->yz_fuse = enable ? 1 : 0;
  int rc = configure(b);
  if (rc) {
    b->yz_fuse = old;
    (void)configure(b);
  }
  return rc;
}

int gp_batch_get_yz_fusion(gp_batch* b, int32_t* enabled, int32_t* fused_instances) {
  if (!b) return GP_ERR_INVALID;
  if (enabled) *enabled = b->yz_fuse;
  if (fused_instances) *fused_instances = b->nfused;
  return GP_OK;
}

int gp_batch_get_mapping(gp_batch* b, int32_t map[5]) {
  if (!b || !map) return GP_ERR_INVALID;
  for (int q = 0; q < 5; ++q) map[q] = b->map[q];
  return GP_OK;
}

int gp_batch_set_mapping(gp_batch* b, const int32_t map[5]) {
  if (!b || !map) return GP_ERR_INVALID;
  BCHK(b, hipStreamSynchronize(b->stream));
  int old[5];
  for (int q = 0; q < 5; ++q) {
    old[q] = b->map[q];
    if (map[q] > 0) b->map[q] = map[q];
  }
  int rc = configure(b);
  if (rc) {
    for (int q = 0; q < 5; ++q) b->map[q] = old[q];
    int rc2 = configure(b);
    (void)rc2;
    return rc == GP_ERR_UNSUPPORTED ? GP_ERR_INVALID : rc;
  }
  return GP_OK;
}

int gp_batch_set_timing(gp_batch* b, int32_t enable) {
  if (!b) return GP_ERR_INVALID;
  int rc = bharvest(b);
  if (rc) return rc;
  b->timing = enable != 0;
  for (int k = 0; k < kBKinds; ++k) {
    b->tsum[k] = 0;
    b->tcnt[k] = 0;
  }
  return GP_OK;
}

int gp_batch_get_timing(gp_batch* b, double ms_mean[5], int64_t launches[5]) {
  if (!b) return GP_ERR_INVALID;
  int rc = bharvest(b);
  if (rc) return rc;
  for (int k = 0; k < kBKinds; ++k) {
    if (ms_mean) ms_mean[k] = b->tcnt[k] ? b->tsum[k] / b->tcnt[k] : 0.0;
    if (launches) launches[k] = b->tcnt[k];
  }
  return GP_OK;
}

}  // extern "C"

namespace {

// Autotuner cache key of a batch: FNV-1a over the instances' grid sizes, in order, with
// the instance count, precision, splitting and step kind beside it.
uint64_t batch_key(const gp_batch* b) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int q = 0; q < 8; ++q) {
      h ^= (uint64_t)((v >> (8 * q)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  for (const gp_params& p : b->p) {
    mix(p.nx);
    mix(p.ny);
    mix(p.nz);
  }
  return h;
}

bool bcache_lookup(const char* path, const gp_batch* b, int mode, int32_t map[5], int* fuse) {
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  const unsigned long long key = batch_key(b);
  char line[256];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    unsigned long long k = 0;
    int n = 0, prec = 0, split = 0, md = 0, m[5], fz = 0;
    if (sscanf(line, "gfx950-batch %llx %d %d %d %d : %d %d %d %d %d %d", &k, &n, &prec, &split, &md, &m[0], &m[1],
               &m[2], &m[3], &m[4], &fz) == 11 &&
        k == key && n == b->n && prec == b->prec && split == b->p[0].split && md == mode) {
      for (int q = 0; q < 5; ++q) map[q] = m[q];
      *fuse = fz;
      found = true;  // the last matching entry wins
    }
  }
  fclose(f);
  return found;
}

void bcache_store(const char* path, const gp_batch* b, int mode, const int32_t map[5], int fuse) {
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "gfx950-batch %llx %d %d %d %d : %d %d %d %d %d %d\n", (unsigned long long)batch_key(b), b->n, b->prec,
          b->p[0].split, mode, map[0], map[1], map[2], map[3], map[4], fuse);
  fclose(f);
}

}  // namespace

extern "C" {

int gp_batch_autotune(gp_batch* b, int32_t mode, int32_t steps, const char* cache_path, int32_t map_out[5]) {
  if (!b || (mode != 0 && mode != 1) || steps < 1) return GP_ERR_INVALID;
  {
    int32_t cm[5];
    int cf = 0;
    if (bcache_lookup(cache_path, b, mode, cm, &cf) && gp_batch_set_mapping(b, cm) == GP_OK &&
        gp_batch_set_yz_fusion(b, cf) == GP_OK) {
      if (map_out)
        for (int q = 0; q < 5; ++q) map_out[q] = b->map[q];
      return GP_OK;
    }
  }
  // tune on a copy of psi; restore psi, state and step counts afterwards
  int64_t total = 0;
  for (int i = 0; i < b->n; ++i)
    total = std::max<int64_t>(total, b->off[i] + (int64_t)b->p[i].nx * b->p[i].ny * b->p[i].nz);
  const size_t bytes = (size_t)total * b->esize;
  void* saved = nullptr;
  int rc = bdalloc(b, &saved, bytes);
  if (rc) return rc;
  std::vector<DevState> st0(b->n);
  {
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipMemcpy(st0.data(), b->st, b->n * sizeof(DevState), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(saved, b->psi, bytes, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
      (void)hipFree(saved);
      return bfail(b, e, "autotune: saving psi");
    }
  }
  const std::vector<int64_t> steps0 = b->steps;
  int best[5];
  for (int q = 0; q < 5; ++q) best[q] = b->map[q];
  double best_ms[3] = {1e300, 1e300, 1e300};
  const int fuse_in = b->yz_fuse;
  b->yz_fuse = 0;  // tune the separate sweeps' mappings first (set_mapping reconfigures)
  auto trial = [&](int kind, const int* cand, double* ms) -> int {
    int rc2 = gp_batch_set_mapping(b, cand);
    if (rc2) return rc2;
    if ((rc2 = brun(b, mode, 1))) return rc2;
    if ((rc2 = gp_batch_set_timing(b, 1))) return rc2;
    if ((rc2 = brun(b, mode, steps))) return rc2;
    double mean[5];
    int64_t cnt[5];
    if ((rc2 = gp_batch_get_timing(b, mean, cnt))) return rc2;
    *ms = mean[kind];
    return gp_batch_set_timing(b, 0);
  };
  const int ms_lines[] = {8, 16, 32};
  for (int axis = 0; axis < 2 && rc == GP_OK; ++axis)
    for (int m : ms_lines)
      for (int sw : {1, 2, 4}) {
        if (!gpk::b_lines_supported(b->prec, m, sw)) continue;
        int cand[5];
        for (int q = 0; q < 5; ++q) cand[q] = best[q];
        cand[2 * axis] = m;
        cand[2 * axis + 1] = sw;
        double ms = 0;
        int r2 = trial(axis, cand, &ms);
        if (r2 == GP_ERR_INVALID) continue;  // mapping does not fit every instance
        if (r2) {
          rc = r2;
          break;
        }
        if (ms < best_ms[axis]) {
          best_ms[axis] = ms;
          best[2 * axis] = m;
          best[2 * axis + 1] = sw;
        }
      }
  for (int m : {4, 6, 8, 12}) {
    if (rc) break;
    int cand[5];
    for (int q = 0; q < 5; ++q) cand[q] = best[q];
    cand[4] = m;
    double ms = 0;
    int r2 = trial(2, cand, &ms);
    if (r2 == GP_ERR_INVALID) continue;
    if (r2) {
      rc = r2;
      break;
    }
    if (ms < best_ms[2]) {
      best_ms[2] = ms;
      best[4] = m;
    }
  }
  if (rc == GP_OK) rc = gp_batch_set_mapping(b, best);
  // fused y+z sweeps against separate ones: whole-step time, keep the faster
  if (rc == GP_OK) {
    double step_ms[2] = {1e300, 1e300};
    const int fuse0 = fuse_in;
    for (int f = 0; f < 2 && rc == GP_OK; ++f) {
      if ((rc = gp_batch_set_yz_fusion(b, f))) break;
      if ((rc = brun(b, mode, 1)) || (rc = gp_batch_set_timing(b, 1)) || (rc = brun(b, mode, steps))) break;
      double mean[5];
      int64_t cnt[5];
      if ((rc = gp_batch_get_timing(b, mean, cnt)) || (rc = gp_batch_set_timing(b, 0))) break;
      double tot = 0.0;
      for (int k = 0; k < 4; ++k) tot += mean[k] * (double)cnt[k];
      step_ms[f] = tot / steps;
    }
    if (rc == GP_OK) rc = gp_batch_set_yz_fusion(b, step_ms[1] <= step_ms[0] ? 1 : 0);
    else (void)gp_batch_set_yz_fusion(b, fuse0);
  } else {
    b->yz_fuse = fuse_in;
    (void)configure(b);
  }
  (void)hipMemcpy(b->psi, saved, bytes, hipMemcpyDeviceToDevice);
  (void)hipMemcpy(b->st, st0.data(), b->n * sizeof(DevState), hipMemcpyHostToDevice);
  (void)hipFree(saved);
  b->steps = steps0;
  if (rc) return rc;
  bcache_store(cache_path, b, mode, best, b->yz_fuse);
  if (map_out)
    for (int q = 0; q < 5; ++q) map_out[q] = best[q];
  return GP_OK;
}

const char* gp_batch_last_error(gp_batch* b) { return b ? b->err : "null batch"; }

}  // extern "C"
