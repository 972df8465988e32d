// Fused y + z sweep with the halo-truncated y back-substitution (gp_set_truncation mode 2).
//
// A y line of plane i is the column k of that plane; its elimination is a recurrence over
// the rows j, and a row (i, j, .) is a whole z line.  A block takes one plane and a chunk
// of rows [j0, j1) and walks the rows in order with one thread per column k:
//   forward   d_j = a (p_{j-1} + p_{j+1} + d_{j-1}) + b p_j   (started H rows before j0,
//             from d = p = 0: the start's error decays like a^(H+1) by row j0; exact
//             from the line start when j0 <= H)
//   backward  u_r = sum_{m=0}^{H} a^m d_{r+m}                  (emitted at step r + H)
// with the y head correction u_r += omega_r u_0 near the line start.  Every emitted row is
// at once a complete z line: the block's waves solve the rows of each group of
// L ceil(W / L) steps (L = H + 1, W wavefronts; one row per wave at a time, 64 lanes x MZ
// points, the z sweep's scans) in LDS, add the
// Strang half potential step if asked, and store them.  psi is read once (plus 2H halo
// rows per chunk) and written once for the y and z sweeps together: 16 B per point
// (complex64) instead of the 32 B of two separate sweeps.  Imaginary time: FP64 sums of
// |psi|^2 per block for the renormalisation.  The pass reads one array (the x sweep's
// output) and writes another: chunks read H rows beyond their own on each side, rows that
// the neighbouring chunk's block writes, so in place the result would depend on block order.
#include "gp_device.h"

#include <algorithm>

namespace gpk {

// MAXW: the most wavefronts (z columns / 64) of a block; complex128 blocks of at most 8
// wavefronts are bounded at 512 threads, which leaves 256 VGPRs per thread (no spills).
template <typename R, int H, int MZ, bool CC, bool NORM, int EPI, int MAXW>
__global__ void __launch_bounds__(64 * MAXW)
k_stream_yz(const typename VecOf<R>::T* __restrict__ src, typename VecOf<R>::T* __restrict__ psi, int ny, int nz,
            int chunk, int nchunks,
            typename VecOf<R>::T ya, typename VecOf<R>::T yb, typename VecOf<R>::T ybl,
            const typename VecOf<R>::T* __restrict__ yomega, int ynw, typename VecOf<R>::T za,
            typename VecOf<R>::T zb, typename VecOf<R>::T zbl, typename VecOf<R>::T zP,
            const typename VecOf<R>::T* __restrict__ zomega, int znw, const R* __restrict__ vx,
            const R* __restrict__ vy, Pot1D<R> pz, R tau, const DevState* __restrict__ st,
            double* __restrict__ partials, int zp) {
  typedef typename VecOf<R>::T V;
  constexpr int L = H + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  V* sdata = reinterpret_cast<V*>(smem_raw);
  const int pitch = z_pitch(nz, MZ, zp);
  const int W = blockDim.x >> 6;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x / nchunks;
  const int c = blockIdx.x % nchunks;
  const int j0 = c * chunk, j1 = min(ny, j0 + chunk);
  const int js = max(0, j0 - H);
  const int k = threadIdx.x;
  const bool kin = k < nz;
  const int kpos = k + zp * (k / MZ);  // LDS position of column k in a row slot
  const V* splane = src + i * (int64_t)ny * nz;  // input (the x sweep's output)
  V* plane = psi + i * (int64_t)ny * nz;         // output
  auto load = [&](int j) { return kin ? gld(splane + (int64_t)j * nz + k) : vzero<V>(); };
  Coef<V> cy, cz;
  cy.a = ya;
  cy.b = yb;
  cy.bl = ybl;
  cz.a = za;
  cz.b = zb;
  cz.bl = zbl;
  R g = 0;
  if (EPI != 0) g = (R)st->g;
  // z-line layout of the solving wave: lane = segment p, MZ points each
  const int s = lane * MZ, ss = s + zp * lane;
  const int len = max(0, min(MZ, nz - s));

  // rows past the last one the chunk needs (j1 + H) are not read (they were, L rows per
  // chunk: 6% of the reads of 120-row chunks; quench grid complex128 real time 1391 ->
  // 1355 us, complex64 576 -> 570 us)
  const int jend = min(ny, j1 + H + 1);
  V q[L], ring[L];
#pragma unroll
  for (int t = 0; t < L; ++t) {
    ring[t] = vzero<V>();
    q[(1 + t) % L] = (js + 1 + t < jend) ? load(js + 1 + t) : vzero<V>();
  }
  V pm = vzero<V>(), pc = load(js), dprev = vzero<V>(), u0 = vzero<V>();
  double acc = 0.0;
  const int total = j1 + H - js;  // steps js .. j1 - 1 + H
  // rows are solved along z in groups of G = L ceil(W / L) steps, so that every wave has a
  // row to solve; LDS slot of step jj: jj - gstart
  const int G = L * ((W + L - 1) / L);
  // the z Sherman-Morrison vector, staged after the group's rows: read from global memory,
  // each lane's value depends on its segment and the loads of a z solve waited out a cache
  // latency in every group (quench grid, fused pass: complex128 imaginary time 858 -> 829
  // us, complex64 real 570 -> 540 us, imaginary 439 -> 418 us; complex128 real unchanged)
  V* s_om = sdata + (size_t)G * pitch;
  for (int q2 = threadIdx.x; q2 < znw; q2 += blockDim.x) s_om[q2] = zomega[q2];  // seen after the first barrier
  int gstart = 0;
  for (int jb = 0; jb < total; jb += L) {
#pragma unroll
    for (int t = 0; t < L; ++t) {
      const int jj = jb + t, j = js + jj;
      if (jj < total) {
        V d = vzero<V>();
        if (j < ny) {
          const int s1 = (t + 1) % L;
          const V pn = (j + 1 < ny) ? q[s1] : vzero<V>();
          if (j + 1 + L < jend) q[s1] = load(j + 1 + L);
          d = fwd_point<CC, R, V>(cy, pm, pn, dprev, pc);
          pm = pc;
          pc = pn;
          dprev = d;
        }
        ring[t] = d;
        const int r = j - H;
        if (r >= j0) {
          V u = ring[t];
#pragma unroll
          for (int m = H - 1; m >= 0; --m) u = cfma<CC>(ya, u, ring[(t + 1 + m) % L]);
          if (r == 0) u0 = u;
          if (r < ynw) u = cfma<CC>(yomega[r], u0, u);
          if (kin) sdata[(jj - gstart) * pitch + kpos] = u;
        }
      }
    }
    const int gend = min(jb + L, total);
    if (gend - gstart < G && gend < total) continue;  // group not full yet (uniform)
    // the rows emitted in this group: slot q holds row js + gstart + q - H
    __syncthreads();
    for (int slot = w; slot < gend - gstart; slot += W) {
      const int r = js + gstart + slot - H;
      if (r >= j0) {
        V* row = sdata + slot * pitch;
        V v[MZ];
        z_line_solve<R, MZ, CC>(v, row, len > 0, s, ss, zp, len, nz, 64, 0, lane, cz, zP, s_om, znw);
        if (len > 0) {
          R vxy = 0;
          if (EPI != 0) vxy = vx[i] + vy[r];
#pragma unroll
          for (int t = 0; t < MZ; ++t) {
            if (t < len) {
              if (EPI != 0) v[t] = nstep<EPI, R, V>(v[t], (R)1, vxy + pz.at(s + t), g, tau);
              if (NORM) acc = fma((double)v[t].x, (double)v[t].x, fma((double)v[t].y, (double)v[t].y, acc));
              row[ss + t] = v[t];
            }
          }
        }
      }
    }
    __syncthreads();
    for (int slot = 0; slot < gend - gstart; ++slot) {
      const int r = js + gstart + slot - H;
      if (r >= j0 && kin) gst(plane + (int64_t)r * nz + k, sdata[slot * pitch + kpos]);
    }
    __syncthreads();
    gstart = gend;
  }
  if (NORM) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) red[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
      for (int q2 = 0; q2 < W; ++q2) tot += red[q2];
      partials[blockIdx.x] = tot;
    }
  }
}

namespace {

template <typename R> typename VecOf<R>::T cv(const double* c) {
  typename VecOf<R>::T v;
  v.x = (R)c[0];
  v.y = (R)c[1];
  return v;
}

template <typename R, int H, int MZ, bool CC, bool NORM, int EPI>
hipError_t go_yz(const YZLaunch& a, hipStream_t s) {
  typedef typename VecOf<R>::T V;
  const int zp = (MZ % 4 == 0) ? 1 : 0;
  constexpr int L = H + 1;
  // ceil(nz / 64) wavefronts cover the columns; if they do not divide the group of
  // G = L ceil(W / L) rows that they solve along z one row per wave, the group's last round
  // of z solves leaves waves idle.  Launch instead the fewest waves W >= ceil(nz / 64) (up
  // to the instance's bound) that divide their own G (the extra waves only solve rows):
  // G is unchanged, since W = G itself divides it.  Quench grid, nz = 448 (7 columns of
  // waves): complex128 real time (H = 7) 8 waves, fused pass 1504 -> 1391 us; complex64
  // real time (H = 3) 8 waves, 684 -> 576 us; complex64 imaginary time (H = 5) 12 waves,
  // 446 -> 438 us.
  int waves = (a.nz + 63) / 64;
  for (int w2 = waves; w2 <= (sizeof(R) == 8 ? 8 : 16); ++w2)
    if ((L * ((w2 + L - 1) / L)) % w2 == 0) {
      waves = w2;
      break;
    }
  const int group = L * ((waves + H) / L);  // L ceil(W / L) row slots
  const size_t lds = ((size_t)group * z_pitch(a.nz, MZ, zp) + a.znw) * sizeof(V);
  auto kern = k_stream_yz<R, H, MZ, CC, NORM, EPI, 16>;
  int which = 0;
  if constexpr (sizeof(R) == 8)
    if (waves <= 8) {
      kern = k_stream_yz<R, H, MZ, CC, NORM, EPI, 8>;
      which = 1;
    }
  if (lds > 65536 - 256) {  // more than the default 64 KiB per block: opt in (up to 160 KiB)
    static size_t granted[2] = {0, 0};
    if (lds > granted[which]) {
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      granted[which] = lds;
    }
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)((int64_t)a.nx * a.nchunks)), dim3(64 * waves), lds, s, (const V*)a.src,
                     (V*)a.psi, a.ny, a.nz, a.chunk, a.nchunks, cv<R>(a.ycoef), cv<R>(a.ycoef + 2), cv<R>(a.ycoef + 4),
                     (const V*)a.yomega, a.ynw, cv<R>(a.zcoef), cv<R>(a.zcoef + 2), cv<R>(a.zcoef + 4),
                     cv<R>(a.zcoef + 6), (const V*)a.zomega, a.znw, (const R*)a.vx, (const R*)a.vy,
                     Pot1D<R>{(R)a.ph, (R)a.pc, (R)a.pd}, (R)a.tau, a.st, a.partials, zp);
  return hipGetLastError();
}

template <typename R, int H, int MZ>
hipError_t go_yz_mode(bool cc, int epi, const YZLaunch& a, hipStream_t s) {
  if (!cc) return epi ? go_yz<R, H, MZ, false, true, 1>(a, s) : go_yz<R, H, MZ, false, true, 0>(a, s);
  return epi ? go_yz<R, H, MZ, true, false, 2>(a, s) : go_yz<R, H, MZ, true, false, 0>(a, s);
}

template <typename R, int H>
hipError_t go_yz_m(bool cc, int epi, const YZLaunch& a, hipStream_t s) {
  switch (a.mz) {
    case 4: return go_yz_mode<R, H, 4>(cc, epi, a, s);
    case 6: return go_yz_mode<R, H, 6>(cc, epi, a, s);
    case 7: return go_yz_mode<R, H, 7>(cc, epi, a, s);
    case 8: return go_yz_mode<R, H, 8>(cc, epi, a, s);
    case 12: return go_yz_mode<R, H, 12>(cc, epi, a, s);
    case 16: return go_yz_mode<R, H, 16>(cc, epi, a, s);
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t go_yz_h(bool cc, int epi, const YZLaunch& a, hipStream_t s) {
  switch (yz_h(a.hlen)) {
    case 3: return go_yz_m<R, 3>(cc, epi, a, s);
    case 5: return go_yz_m<R, 5>(cc, epi, a, s);
    case 7: return go_yz_m<R, 7>(cc, epi, a, s);
    case 11: return go_yz_m<R, 11>(cc, epi, a, s);
    case 15: return go_yz_m<R, 15>(cc, epi, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int yz_h(int h) {
  for (int v : {3, 5, 7, 11, 15})
    if (h <= v) return v;
  return -1;
}

size_t yz_lds(int nz, int h, size_t esize, int znw) {
  const int H = yz_h(h), mz = yz_mz(nz);
  if (H < 0 || mz < 0) return 0;
  const int waves = (nz + 63) / 64;
  const int group = (H + 1) * ((waves + H) / (H + 1));
  const int zp = (mz % 4 == 0) ? 1 : 0;
  return ((size_t)group * z_pitch(nz, mz, zp) + znw) * esize;
}

int yz_mz(int nz) {
  for (int m : {4, 6, 7, 8, 12, 16})
    if (64 * m >= nz) return m;
  return -1;
}

hipError_t launch_stream_yz(int precision, bool cc, const YZLaunch& a, hipStream_t s) {
  return precision == 0 ? go_yz_h<float>(cc, a.epi, a, s) : go_yz_h<double>(cc, a.epi, a, s);
}

}  // namespace gpk
