// Warm-start network on gfx950: BF16 MFMA convolutions (implicit GEMM) with FP32
// accumulation, split-K weight gradients through LDS, fused pointwise layers and Adam.
//
// Matrix-core tiles (wave64): v_mfma_f32_16x16x32_bf16 (cin multiple of 32) and
// v_mfma_f32_16x16x16_bf16 (cin multiple of 16).  For the 16x16xK tile, lane l holds
// A[row l%16][k (l/16)*K/4 ...] and B[k (l/16)*K/4 ...][col l%16] (K/4 consecutive
// values each) and receives D[row (l/16)*4 + i][col l%16], i = 0..3.
//
// Convolution as GEMM: rows = output positions, columns = output channels,
// K = taps x input channels.  Channels-last storage makes every A fragment (K/4
// consecutive input channels of one position) and every B fragment (K/4 consecutive
// input channels of one output channel, weights [tap][cout][cin]) one 16- or 8-byte
// load.  The backward pass with respect to the input is the same kernel applied to the
// output gradient with the weights transposed and the taps mirrored
// (W'[26 - t][i][o] = W[t][o][i]), so one kernel serves both.
#include "../../include/gpnn.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gp_internal.h"

namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kFMax = 10.0f;   // psi = exp(min(f, kFMax))
constexpr int kChunkMin = 2048;  // fewest positions per split-K block of the weight gradient
constexpr int kMaxChunks = 128;  // most split-K blocks (partial sums to reduce) per tap
constexpr int kConvBlocks = 768;  // blocks of the tiled convolution (about 3 per CU)

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even (the gfx950 conversion instruction); NaN stays NaN
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }

// hardware reciprocal (1 ulp): the result is rounded to BF16 afterwards
__device__ __forceinline__ float sigm(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }
__device__ __forceinline__ float silu(float x) { return x * sigm(x); }
__device__ __forceinline__ float silu_d(float x) {
  const float s = sigm(x);
  return s * (1.0f + x * (1.0f - s));
}

template <int KC> struct Frag;
template <> struct Frag<32> {
  typedef bf16x8 T;
  static __device__ __forceinline__ T load(const uint16_t* p) { return *reinterpret_cast<const T*>(p); }
  static __device__ __forceinline__ T zero() { return T{}; }
  static __device__ __forceinline__ f32x4 mma(T a, T b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Frag<16> {
  typedef bf16x4 T;
  static __device__ __forceinline__ T load(const uint16_t* p) { return *reinterpret_cast<const T*>(p); }
  static __device__ __forceinline__ T zero() { return T{}; }
  static __device__ __forceinline__ f32x4 mma(T a, T b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};

// y[p, o] = epilogue(sum_t sum_i w[t][o][i] x[nbr_t(p)][i]).  Block: 4 waves, 64 positions
// (16 per wave) x 64 output channels (blockIdx.y selects the 64-channel slice).
template <int KS, int KC>
__global__ void __launch_bounds__(256)
k_conv(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w, const float* __restrict__ bias,
       int64_t P, int D, int cin, int cout, int act, const uint16_t* __restrict__ gate,
       uint16_t* __restrict__ y, uint16_t* __restrict__ pre) {
  typedef Frag<KC> F;
  constexpr int KQ = KC / 4;  // consecutive K values per lane
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const int64_t p0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int co0 = blockIdx.y * 64;
  const int nb = min(4, (cout - co0) >> 4);
  const int64_t p = p0 + r;
  const bool pv = p < P;
  int pi = 0, pj = 0, pk = 0;
  if (KS == 3 && pv) {
    int64_t q = p;
    pk = (int)(q % D);
    q /= D;
    pj = (int)(q % D);
    q /= D;
    pi = (int)(q % D);
  }
  f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int t = 0; t < KS * KS * KS; ++t) {
    bool ok = pv;
    int64_t nbr = p;
    if (KS == 3) {
      const int a = t / 9 - 1, b = (t / 3) % 3 - 1, c = t % 3 - 1;
      ok = ok && (unsigned)(pi + a) < (unsigned)D && (unsigned)(pj + b) < (unsigned)D &&
           (unsigned)(pk + c) < (unsigned)D;
      nbr = p + ((int64_t)a * D + b) * D + c;
    }
    const uint16_t* xr = x + (ok ? nbr : 0) * (int64_t)cin + kq * KQ;
    const uint16_t* wt = w + ((int64_t)t * cout + co0 + r) * cin + kq * KQ;
    for (int k0 = 0; k0 < cin; k0 += KC) {
      const typename F::T av = ok ? F::load(xr + k0) : F::zero();
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < nb) acc[j] = F::mma(av, F::load(wt + (int64_t)j * 16 * cin + k0), acc[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j >= nb) continue;
    const int co = co0 + j * 16 + r;
    const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t pos = p0 + kq * 4 + i;
      if (pos >= P) continue;
      const int64_t o = pos * cout + co;
      float v = acc[j][i] + bv;
      if (pre) pre[o] = f2bf(v);
      if (gate) v *= silu_d(bf2f(gate[o]));
      else if (act) v = silu(v);
      y[o] = f2bf(v);
    }
  }
}

// Dense layer for few positions (a batch of problems), split over the input channels:
// block (16 positions, 64 output channels, input-channel slice blockIdx.z); its 4 waves
// take interleaved 32-channel steps of the slice, are summed in LDS, and the slice sum goes
// to part[z][p][cout] for k_dense_finish.  A plain one-tap launch would leave 3 of 4 waves
// idle at 16 positions and walk all input channels in one wave.
__global__ void __launch_bounds__(256)
k_dense_sk(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w, int P, int cin, int cout, int kslice,
           float* __restrict__ part) {
  __shared__ float red[4][16][65];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const int p0 = blockIdx.x * 16, co0 = blockIdx.y * 64;
  const int nb = min(4, (cout - co0) >> 4);
  const int kb = blockIdx.z * kslice, ke = min(cin, kb + kslice);
  const int p = p0 + r;
  const bool pv = p < P;
  f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* xr = x + (int64_t)(pv ? p : 0) * cin + kq * 8;
  const uint16_t* wr = w + (int64_t)(co0 + r) * cin + kq * 8;
  for (int k0 = kb + wave * 32; k0 < ke; k0 += 128) {
    const bf16x8 av = pv ? *reinterpret_cast<const bf16x8*>(xr + k0) : bf16x8{};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < nb)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            av, *reinterpret_cast<const bf16x8*>(wr + (int64_t)j * 16 * cin + k0), acc[j], 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wave][kq * 4 + i][j * 16 + r] = acc[j][i];
  __syncthreads();
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int e = threadIdx.x + 256 * it;
    const int pr = e >> 6, c = e & 63;
    if (p0 + pr < P && c < nb * 16)
      part[((int64_t)blockIdx.z * P + p0 + pr) * cout + co0 + c] = red[0][pr][c] + red[1][pr][c] + red[2][pr][c] +
                                                                      red[3][pr][c];
  }
}

// y[p][o] = epilogue(bias[o] + sum_z part[z][p][o]), epilogue as k_conv
__global__ void __launch_bounds__(256)
k_dense_finish(const float* __restrict__ part, int S, int P, int cout, const float* __restrict__ bias, int act,
               const uint16_t* __restrict__ gate, uint16_t* __restrict__ y, uint16_t* __restrict__ pre) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)P * cout) return;
  float v = bias ? bias[e % cout] : 0.0f;
  for (int z = 0; z < S; ++z) v += part[(int64_t)z * P * cout + e];
  if (pre) pre[e] = f2bf(v);
  if (gate) v *= silu_d(bf2f(gate[e]));
  else if (act) v = silu(v);
  y[e] = f2bf(v);
}

// 3x3x3 convolution with the input tile staged in LDS, for D^3 grids with D a power of
// two >= 8.  Work item: a TI x TJ x TK = 256-position brick of one sample (TK = min(D, 16)
// along z, TJ = 4, TI = 256 / (TJ TK)), 16 NB output channels (blockIdx.y), one chunk of
// KC input channels.  For each item a block stages the brick's halo ((TI+2)(TJ+2)(TK+2)
// positions, KC channels, row pitch KC + 8 so the 16 lanes of a fragment hit distinct
// banks), then runs the 27 taps from LDS; each wave owns 4 tiles of 16 positions x NB
// tiles of 16 output channels, so every A fragment (LDS) feeds NB MFMAs and every B
// fragment (weights, global/L1) feeds 4.  A block walks several bricks; for single output
// tiles the next item's halo loads are in flight while the current item's MFMAs run, and
// always the next tap's weight and halo fragments while the current tap's do.  Bricks are dealt so that the blocks on
// one XCD (workgroups go round-robin to the 8 XCDs) work on one contiguous stretch of the
// grid at a time, sharing halos through that XCD's L2.  UP: the input is given on the 2x
// coarser grid (D/2)^3 and read as its nearest-neighbour upsampling, so the upsampled
// tensor is never stored.  Epilogue as k_conv.
template <int KC, int TK, int NB, bool UP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB <= 2 ? 3 : 1)))
k_conv3_tiled(const uint16_t* __restrict__ x, const uint16_t* __restrict__ w, const float* __restrict__ bias, int D,
              int cin, int cout, int act, const uint16_t* __restrict__ gate, uint16_t* __restrict__ y,
              uint16_t* __restrict__ pre, int nbrick) {
  typedef Frag<KC> F;
  typedef typename F::T FT;
  constexpr int KQ = KC / 4;
  constexpr int PITCH = KC + 8;  // bf16 per halo position
  constexpr int U = KC / 8;      // 16-byte units per position
  constexpr int TJ = 4, TI = 256 / (TJ * TK);
  constexpr int HK = TK + 2, HJ = TJ + 2, HI = TI + 2;
  constexpr int nhalo = HI * HJ * HK;
  constexpr int NE = (nhalo * U + 255) / 256;  // staged 16-byte units per thread
  extern __shared__ __align__(16) uint16_t halo[];
  // this block's bricks: brick(it) for it = 0, 1, ... while < nmine
  const int G = gridDim.x, b = blockIdx.x;
  int first, stride, nmine;
  if (nbrick % 8 == 0 && G % 8 == 0) {
    const int per = nbrick / 8, nslot = G / 8, slot = b / 8;
    first = (b % 8) * per + slot;
    stride = nslot;
    nmine = slot < per ? (per - slot + nslot - 1) / nslot : 0;
  } else {
    first = b;
    stride = G;
    nmine = b < nbrick ? (nbrick - b + G - 1) / G : 0;
  }
  const int nchunk = cin / KC;
  const int nitem = nmine * nchunk;
  const int tkn = D / TK, tjn = D / TJ, tin = D / TI;
  const int co0 = blockIdx.y * 16 * NB;
  const int nb = min(NB, (cout - co0) >> 4);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  int hbase[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const int tp = wave * 64 + mb * 16 + r;
    const int tk = tp % TK, tj = (tp / TK) % TJ, ti = tp / (TK * TJ);
    hbase[mb] = (((ti + 1) * HJ + (tj + 1)) * HK + (tk + 1)) * PITCH + kq * KQ;
  }
  struct Brick {
    int i0, j0, k0;
    int64_t sbase;  // first output position of the sample
    int64_t xbase;  // first input position of the sample (UP: on the coarse grid)
  };
  const int Dc = D >> 1;
  auto brick = [&](int it) {
    Brick o;
    int q = first + it * stride;
    o.k0 = (q % tkn) * TK;
    q /= tkn;
    o.j0 = (q % tjn) * TJ;
    q /= tjn;
    o.i0 = (q % tin) * TI;
    o.sbase = (int64_t)(q / tin) * D * D * D;
    o.xbase = UP ? (int64_t)(q / tin) * Dc * Dc * Dc : o.sbase;
    return o;
  };
  uint4 v[NE];
  auto load_item = [&](int item, int m0, int m1) {
    const Brick o = brick(item / nchunk);
    const int ci0 = (item % nchunk) * KC;
    const uint16_t* xs = x + o.xbase * cin + ci0;
#pragma unroll
    for (int m = 0; m < NE; ++m) {
      if (m < m0 || m >= m1) continue;
      const int e = threadIdx.x + 256 * m;
      v[m] = make_uint4(0, 0, 0, 0);
      if (e < nhalo * U) {
        const int hp = e / U, u = e % U;
        const int hk = hp % HK, hj = (hp / HK) % HJ, hi = hp / (HK * HJ);
        const int gi = o.i0 - 1 + hi, gj = o.j0 - 1 + hj, gk = o.k0 - 1 + hk;
        if ((unsigned)gi < (unsigned)D && (unsigned)gj < (unsigned)D && (unsigned)gk < (unsigned)D) {
          // UP: the input is the 2x coarser grid, read as its nearest-neighbour upsampling
          const int idx = UP ? ((gi >> 1) * Dc + (gj >> 1)) * Dc + (gk >> 1) : (gi * D + gj) * D + gk;
          v[m] = *reinterpret_cast<const uint4*>(xs + (int64_t)idx * cin + u * 8);
        }
      }
    }
  };
  f32x4 acc[4][NB];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[mb][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto store_item = [&](int m0, int m1) {
#pragma unroll
    for (int m = 0; m < NE; ++m) {
      if (m < m0 || m >= m1) continue;
      const int e = threadIdx.x + 256 * m;
      if (e < nhalo * U) *reinterpret_cast<uint4*>(halo + (e / U) * PITCH + (e % U) * 8) = v[m];
    }
  };
  // prefetching the whole next item costs NE x 4 registers: single output tiles only;
  // wider tiles issue their first NE1 loads before the barrier that frees the LDS
  constexpr bool PIPE = NB == 1;
  constexpr int NE1 = PIPE ? NE : (NE < 6 ? NE : 6);
  if (PIPE && nitem > 0) load_item(0, 0, NE);
  for (int item = 0; item < nitem; ++item) {
    if (!PIPE) load_item(item, 0, NE1);
    const int ci0 = (item % nchunk) * KC;
    const uint16_t* wbase = w + ((int64_t)co0 + r) * cin + ci0 + kq * KQ;
    FT bv[NB], bn[NB], av[4], an[4];
#pragma unroll
    for (int j = 0; j < NB; ++j) bv[j] = j < nb ? F::load(wbase + (int64_t)j * 16 * cin) : F::zero();
    __syncthreads();
    store_item(0, NE1);
    if (!PIPE && NE > NE1) {
      load_item(item, NE1, NE);
      store_item(NE1, NE);
    }
    __syncthreads();
    if (PIPE && item + 1 < nitem) load_item(item + 1, 0, NE);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) av[mb] = F::load(halo + hbase[mb] + (((-1) * HJ + (-1)) * HK + (-1)) * PITCH);
    auto fetch = [&](int tn, FT* ax, FT* bx) {
      const int toffn = ((tn / 9 - 1) * HJ + ((tn / 3) % 3 - 1)) * HK + (tn % 3 - 1);
      const uint16_t* wt = wbase + (int64_t)tn * cout * cin;
#pragma unroll
      for (int j = 0; j < NB; ++j) bx[j] = j < nb ? F::load(wt + (int64_t)j * 16 * cin) : F::zero();
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) ax[mb] = F::load(halo + hbase[mb] + toffn * PITCH);
    };
    auto mfmas = [&](const FT* ac, const FT* bc) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (j < nb) acc[mb][j] = F::mma(ac[mb], bc[j], acc[mb][j]);
    };
    if constexpr (KC == 16) {
      // 16 input channels: two taps per 16x16x32 MFMA (lanes kq < 2 carry tap 2p, kq >= 2
      // tap 2p + 1, 8 channels each), 14 steps instead of 27 K = 16 ones; the missing
      // 28th tap has zero weights (its A fragment repeats tap 26, finite times zero)
      const uint16_t* wpair = w + ((int64_t)co0 + r) * cin + ci0 + (kq & 1) * 8;
      bf16x8 pa[4], pna[4], pb[NB], pnb[NB];
      auto pfetch = [&](int pn, bf16x8* ax, bf16x8* bx) {
        const int mt = 2 * pn + (kq >> 1);
        const int ta = mt < 27 ? mt : 26;
        const int toffa = ((ta / 9 - 1) * HJ + ((ta / 3) % 3 - 1)) * HK + (ta % 3 - 1);
        const uint16_t* wt = wpair + (int64_t)ta * cout * cin;
#pragma unroll
        for (int j = 0; j < NB; ++j)
          bx[j] = (j < nb && mt < 27) ? *reinterpret_cast<const bf16x8*>(wt + (int64_t)j * 16 * cin) : bf16x8{};
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
          ax[mb] = *reinterpret_cast<const bf16x8*>(halo + hbase[mb] - kq * KQ + toffa * PITCH + (kq & 1) * 8);
      };
      pfetch(0, pa, pb);
#pragma unroll 1
      for (int pn = 0; pn < 14; ++pn) {
        if (pn + 1 < 14) pfetch(pn + 1, pna, pnb);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
          for (int j = 0; j < NB; ++j)
            if (j < nb) acc[mb][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pa[mb], pb[j], acc[mb][j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < NB; ++j) pb[j] = pnb[j];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) pa[mb] = pna[mb];
      }
    } else if constexpr (NB == 1) {
      // taps in pairs with two register sets and no copies between them
#pragma unroll 1
      for (int t = 0; t < 26; t += 2) {
        fetch(t + 1, an, bn);
        mfmas(av, bv);
        fetch(t + 2, av, bv);
        mfmas(an, bn);
      }
      mfmas(av, bv);  // tap 26
    } else {
      // wider output tiles: one register set plus copies keeps the occupancy
#pragma unroll 1
      for (int t = 0; t < 27; ++t) {
        if (t + 1 < 27) fetch(t + 1, an, bn);
        mfmas(av, bv);
#pragma unroll
        for (int j = 0; j < NB; ++j) bv[j] = bn[j];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) av[mb] = an[mb];
      }
    }
    if (item % nchunk != nchunk - 1) continue;
    // epilogue of the brick
    const Brick o = brick(item / nchunk);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j >= nb) continue;
        const int co = co0 + j * 16 + r;
        const float bvv = bias ? bias[co] : 0.0f;
        // the 4 rows of a lane are consecutive positions along z
        const int tp = wave * 64 + mb * 16 + kq * 4;
        const int tk = tp % TK, tj = (tp / TK) % TJ, ti = tp / (TK * TJ);
        const int64_t o0 = (o.sbase + ((int64_t)(o.i0 + ti) * D + (o.j0 + tj)) * D + (o.k0 + tk)) * cout + co;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t oi = o0 + (int64_t)i * cout;
          float vv = acc[mb][j][i] + bvv;
          if (pre) pre[oi] = f2bf(vv);
          if (gate) vv *= silu_d(bf2f(gate[oi]));
          else if (act) vv = silu(vv);
          y[oi] = f2bf(vv);
        }
        acc[mb][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
  }
}

// Split-K weight gradient: block (chunk of positions, group of 4 taps, 64x64 tile of
// (cout, cin)); partial sums over the chunk's positions written to
// part[chunk][tap][cout][cin].  Each 64-position sub-tile of dy is staged in LDS once and
// the x sub-tiles of the group's 4 taps (shifted, zero outside the grid) next to it, all
// transposed ([channel][position]) so both MFMA operands are 16-byte LDS reads; wave w
// accumulates tap 4 g + w for the whole 64x64 tile.  The block holding the centre tap and
// the first input-channel tile also sums the staged dy rows: the bias gradient's partial
// sums, dbpart[chunk][cout] (nullable).
template <int KS, int MCO, int MCI>
__global__ void __launch_bounds__(256)
k_wgrad(const uint16_t* __restrict__ dy, const uint16_t* __restrict__ x, int64_t P, int D, int cin, int cout,
        int64_t chunk, float* __restrict__ part, float* __restrict__ dbpart) {
  // a tile covers up to MCO x MCI blocks of 16 output x 16 input channels (MCO, MCI <= 4)
  constexpr int NB = MCO * MCI;
  constexpr int LD = 72;  // 64 positions + 8 pad (row = 144 B, 16-byte aligned)
  constexpr int T = KS * KS * KS;
  constexpr int G = T < 4 ? T : 4;  // taps per block
  extern __shared__ __align__(16) uint16_t smem[];
  const int cot = (cout + 63) / 64;
  const int co0 = (blockIdx.z % cot) * 64, ci0 = (blockIdx.z / cot) * 64;
  const int nco = min(64, cout - co0), nci = min(64, cin - ci0);
  uint16_t* sdy = smem;              // [nco][LD]
  uint16_t* sxb = smem + nco * LD;   // [G][nci][LD]
  const int t0 = blockIdx.y * G;
  const int64_t q0 = (int64_t)blockIdx.x * chunk;
  const int64_t q1 = min(P, q0 + chunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const int tw = t0 + wave;  // this wave's tap
  const bool wact = wave < G && tw < T;
  const bool do_db = dbpart != nullptr && ci0 == 0 && T / 2 >= t0 && T / 2 < t0 + G;
  float dbacc = 0.0f;  // channel threadIdx.x / 4, positions (threadIdx.x % 4) * 16 ... + 15
  f32x4 acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // staging: thread -> positions 2 pq, 2 pq + 1 of the sub-tile and 8 channels c8 .. c8 + 7;
  // each channel's pair of positions is one 32-bit LDS word (consecutive lanes, consecutive
  // words: conflict-free)
  const int pq = threadIdx.x & 31;
  const int c8 = (threadIdx.x >> 5) * 8;
  for (int64_t s0 = q0; s0 < q1; s0 += 64) {
    __syncthreads();
    {
      int64_t pos[2];
      bool pv[2];
      int pi[2] = {0, 0}, pj[2] = {0, 0}, pk[2] = {0, 0};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        pos[h] = s0 + 2 * pq + h;
        pv[h] = pos[h] < q1;
        if (KS == 3 && pv[h]) {
          int64_t q = pos[h];
          pk[h] = (int)(q % D);
          q /= D;
          pj[h] = (int)(q % D);
          q /= D;
          pi[h] = (int)(q % D);
        }
      }
      {
        uint4 v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          v[h] = make_uint4(0, 0, 0, 0);
          if (pv[h] && c8 < nco) v[h] = *reinterpret_cast<const uint4*>(dy + pos[h] * cout + co0 + c8);
        }
        const uint16_t* e0 = reinterpret_cast<const uint16_t*>(&v[0]);
        const uint16_t* e1 = reinterpret_cast<const uint16_t*>(&v[1]);
        if (c8 < nco)
#pragma unroll
          for (int q = 0; q < 8; ++q)
            *reinterpret_cast<uint32_t*>(sdy + (c8 + q) * LD + 2 * pq) = (uint32_t)e0[q] | ((uint32_t)e1[q] << 16);
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int t = t0 + g;
        uint4 v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          bool ok = pv[h] && t < T && c8 < nci;
          int64_t nbr = pos[h];
          if (KS == 3 && ok) {
            const int a = t / 9 - 1, b = (t / 3) % 3 - 1, c = t % 3 - 1;
            ok = (unsigned)(pi[h] + a) < (unsigned)D && (unsigned)(pj[h] + b) < (unsigned)D &&
                 (unsigned)(pk[h] + c) < (unsigned)D;
            nbr = pos[h] + ((int64_t)a * D + b) * D + c;
          }
          v[h] = make_uint4(0, 0, 0, 0);
          if (ok) v[h] = *reinterpret_cast<const uint4*>(x + nbr * cin + ci0 + c8);
        }
        const uint16_t* e0 = reinterpret_cast<const uint16_t*>(&v[0]);
        const uint16_t* e1 = reinterpret_cast<const uint16_t*>(&v[1]);
        if (c8 < nci)
#pragma unroll
          for (int q = 0; q < 8; ++q)
            *reinterpret_cast<uint32_t*>(sxb + (g * nci + c8 + q) * LD + 2 * pq) =
                (uint32_t)e0[q] | ((uint32_t)e1[q] << 16);
      }
    }
    __syncthreads();
    if (do_db && (threadIdx.x >> 2) < nco) {
      const uint16_t* row = sdy + (threadIdx.x >> 2) * LD + (threadIdx.x & 3) * 16;
#pragma unroll
      for (int e = 0; e < 16; ++e) dbacc += bf2f(row[e]);
    }
    if (wact) {
      const uint16_t* sxw = sxb + (wave < G ? wave : 0) * nci * LD;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
        for (int blk = 0; blk < NB; ++blk) {
          const int bco = blk % MCO, bci = blk / MCO;
          if (bco * 16 >= nco || bci * 16 >= nci) continue;
          const bf16x8 av = *reinterpret_cast<const bf16x8*>(sdy + (bco * 16 + r) * LD + ks * 32 + kq * 8);
          const bf16x8 bv = *reinterpret_cast<const bf16x8*>(sxw + (bci * 16 + r) * LD + ks * 32 + kq * 8);
          acc[blk] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[blk], 0, 0, 0);
        }
      }
    }
  }
  if (do_db) {
    dbacc += __shfl_xor(dbacc, 1);
    dbacc += __shfl_xor(dbacc, 2);
    const int co = threadIdx.x >> 2;
    if ((threadIdx.x & 3) == 0 && co < nco) dbpart[(int64_t)blockIdx.x * cout + co0 + co] = dbacc;
  }
  if (!wact) return;
  float* out = part + ((int64_t)blockIdx.x * T + tw) * (int64_t)cout * cin;
#pragma unroll
  for (int blk = 0; blk < NB; ++blk) {
    const int bco = blk % MCO, bci = blk / MCO;
    if (bco * 16 >= nco || bci * 16 >= nci) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      out[(int64_t)(co0 + bco * 16 + kq * 4 + i) * cin + ci0 + bci * 16 + r] = acc[blk][i];
  }
}

// Weight gradient of the 3x3x3 convolution on power-of-two grids (D >= 8, whole samples),
// tiled like k_conv3_tiled.  A block walks a run of 256-position bricks (TI x TJ x TK,
// z fastest).  Per brick it stages dy transposed ([channel][position], 264-element rows)
// and the x halo of one input-channel tile transposed ([channel][hi][hj][hk]: rows of HK
// z-values, HK >= TK + 2 and a multiple of 8; channel stride CS = 8 mod 128 elements so
// the 16 rows of a fragment hit distinct banks).  Position pairs are packed into 32-bit
// LDS words on the way in.  A wave owns units (one (x, y) tap offset pair x one 16-channel
// input block) and, for each, the three z offsets: one 16-byte plus one 4-byte LDS read
// gives the eight z-consecutive halo values of all three (shifted by 0, 1 or 2 elements
// with funnel shifts), so every staged value feeds three MFMAs.  The A fragments (dy)
// are shared by all of a wave's units.  Partial sums over the block's bricks go to
// part[chunk][tap][cout][cin]; blocks of the first tap group and input tile also sum the
// staged dy rows into dbpart[chunk][cout] (nullable).
template <int MCO, int MCI, int NU, bool UP>
__global__ void __launch_bounds__(256)
k_wgrad3_tiled(const uint16_t* __restrict__ dy, const uint16_t* __restrict__ x, int D, int lg, int cin, int cout,
               int nab, int ntiles, int tpb, float* __restrict__ part, float* __restrict__ dbpart) {
  constexpr int MU = 6;    // x staging units per thread (<= 6 * 256 16-byte pairs per brick)
  constexpr int DP = 264;  // dy row pitch (elements)
  constexpr int CIT = 16 * MCI;
  extern __shared__ __align__(16) uint16_t smem[];
  const int TK = D < 16 ? D : 16, TJ = 4, TI = 256 / (TJ * TK);
  const int lgk = TK == 16 ? 4 : 3;
  const int HK = TK == 16 ? 24 : 16, HJ = TJ + 2, HI = TI + 2;
  const int HR = HI * HJ * HK;
  const int CS = HR + ((8 - HR) % 128 + 128) % 128;
  const int NP = (TK + 2) / 2;
  uint16_t* sdy = smem;                // [16 MCO][DP]
  uint16_t* sx = smem + 16 * MCO * DP;  // [CIT][CS]
  const int cit = (cin + CIT - 1) / CIT;
  const int co0 = (blockIdx.z / cit) * 16 * MCO, ci0 = (blockIdx.z % cit) * CIT;
  const int nco = min(16 * MCO, cout - co0), nci = min(CIT, cin - ci0);
  const int ab0 = blockIdx.y * nab, nabb = min(nab, 9 - ab0), nunit = nabb * MCI;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const bool do_db = dbpart != nullptr && blockIdx.y == 0 && ci0 == 0;
  // x staging units of this thread: unit n -> (channel group cg, halo row, z pair pr)
  int xl[MU], xg[MU];
  const int nxu = (CIT / 8) * HI * HJ * NP;
#pragma unroll
  for (int m = 0; m < MU; ++m) {
    const int n = threadIdx.x + 256 * m;
    xl[m] = -1;
    xg[m] = 0;
    if (n < nxu) {
      const int pr = n % NP, rest = n / NP, row = rest % (HI * HJ), cg = rest / (HI * HJ);
      if (cg * 8 < nci) {
        xl[m] = (cg * 8 * CS + row * HK + 2 * pr) >> 1;
        xg[m] = (row / HJ) | ((row % HJ) << 8) | ((2 * pr) << 16) | (cg << 24);
      }
    }
  }
  // this wave's units: u = wave + 4 j -> (tap pair ab, input block mci); uoff = LDS offset
  int uoff[NU];
  bool uact[NU];
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const int u = wave + 4 * j;
    const int abl = u / MCI, mci = u % MCI, ab = ab0 + abl;
    uact[j] = u < nunit && mci * 16 < nci;
    uoff[j] = uact[j] ? (mci * 16 + r) * CS + ((ab / 3) * HJ + ab % 3) * HK : 0;
  }
  f32x4 acc[NU][3][MCO];
#pragma unroll
  for (int j = 0; j < NU; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int b = 0; b < MCO; ++b) acc[j][c][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbacc = 0.0f;
  const int tkn = D / TK, tjn = D / TJ, tin = D / TI;
  const int tb0 = blockIdx.x * tpb, tb1 = min(ntiles, tb0 + tpb);
  // staging of a brick: global loads into registers, then position pairs packed into
  // 32-bit LDS words.  Where the accumulators leave room for it at two waves per SIMD, the
  // next brick's loads are in flight while the current one is computed.
  struct Org {
    int i0, j0, k0;
    int64_t sbase;  // first position of the sample (UP: xbase on the coarse grid)
    int64_t xbase;
  };
  auto origin = [&](int tb) {
    Org o;
    int q = tb;
    o.k0 = (q % tkn) * TK;
    q /= tkn;
    o.j0 = (q % tjn) * TJ;
    q /= tjn;
    o.i0 = (q % tin) * TI;
    o.sbase = (int64_t)(q / tin) << (3 * lg);
    o.xbase = UP ? (int64_t)(q / tin) << (3 * (lg - 1)) : o.sbase;
    return o;
  };
  // dy: 128 position pairs x (16 MCO / 8) channel groups
  auto load_dy = [&](int m, const Org& o, uint4& v0, uint4& v1) {
    const int n = threadIdx.x + 256 * m;
    const int pp = n & 127, cg = n >> 7;
    if (cg * 8 >= nco) return;
    const int p = 2 * pp;
    const int kk = p & (TK - 1), jj = (p >> lgk) & 3, ii = p >> (lgk + 2);
    const int64_t g = o.sbase + ((int64_t)(o.i0 + ii) << (2 * lg)) + ((o.j0 + jj) << lg) + (o.k0 + kk);
    v0 = *reinterpret_cast<const uint4*>(dy + g * cout + co0 + cg * 8);
    v1 = *reinterpret_cast<const uint4*>(dy + (g + 1) * cout + co0 + cg * 8);
  };
  auto store_dy = [&](int m, const uint4& v0, const uint4& v1) {
    const int n = threadIdx.x + 256 * m;
    const int pp = n & 127, cg = n >> 7;
    if (cg * 8 >= nco) return;
    const uint16_t* e0 = reinterpret_cast<const uint16_t*>(&v0);
    const uint16_t* e1 = reinterpret_cast<const uint16_t*>(&v1);
    uint32_t* d32 = reinterpret_cast<uint32_t*>(sdy);
#pragma unroll
    for (int e = 0; e < 8; ++e) d32[((cg * 8 + e) * DP >> 1) + pp] = (uint32_t)e0[e] | ((uint32_t)e1[e] << 16);
  };
  // x halo of the input tile, zero outside the grid
  auto load_x = [&](int m, const Org& o, uint4& v0, uint4& v1) {
    v0 = make_uint4(0, 0, 0, 0);
    v1 = v0;
    if (xl[m] < 0) return;
    const int gi = o.i0 + (xg[m] & 255) - 1, gj = o.j0 + ((xg[m] >> 8) & 255) - 1;
    const int gk = o.k0 + ((xg[m] >> 16) & 255) - 1, cg = xg[m] >> 24;
    if ((unsigned)gi < (unsigned)D && (unsigned)gj < (unsigned)D) {
      if (UP) {  // x on the 2x coarser grid, read as its nearest-neighbour upsampling
        const int lc = lg - 1;
        const int64_t g = o.xbase + ((int64_t)(gi >> 1) << (2 * lc)) + ((gj >> 1) << lc);
        const uint16_t* src = x + g * cin + ci0 + cg * 8;
        if ((unsigned)gk < (unsigned)D) v0 = *reinterpret_cast<const uint4*>(src + (int64_t)(gk >> 1) * cin);
        if ((unsigned)(gk + 1) < (unsigned)D)
          v1 = *reinterpret_cast<const uint4*>(src + (int64_t)((gk + 1) >> 1) * cin);
      } else {
        const int64_t g = o.sbase + ((int64_t)gi << (2 * lg)) + (gj << lg) + gk;
        const uint16_t* src = x + g * cin + ci0 + cg * 8;
        if ((unsigned)gk < (unsigned)D) v0 = *reinterpret_cast<const uint4*>(src);
        if ((unsigned)(gk + 1) < (unsigned)D) v1 = *reinterpret_cast<const uint4*>(src + cin);
      }
    }
  };
  auto store_x = [&](int m, const uint4& v0, const uint4& v1) {
    if (xl[m] < 0) return;
    const uint16_t* e0 = reinterpret_cast<const uint16_t*>(&v0);
    const uint16_t* e1 = reinterpret_cast<const uint16_t*>(&v1);
    uint32_t* x32 = reinterpret_cast<uint32_t*>(sx);
#pragma unroll
    for (int e = 0; e < 8; ++e) x32[xl[m] + e * (CS >> 1)] = (uint32_t)e0[e] | ((uint32_t)e1[e] << 16);
  };
  constexpr bool PIPE = MCO <= 2 && MCO * NU * 12 <= 72;
  uint4 rdy[PIPE ? MCO : 1][2], rx[PIPE ? MU : 1][2];
  if constexpr (PIPE) {
    if (tb0 < tb1) {
      const Org o = origin(tb0);
#pragma unroll
      for (int m = 0; m < MCO; ++m) load_dy(m, o, rdy[m][0], rdy[m][1]);
#pragma unroll
      for (int m = 0; m < MU; ++m) load_x(m, o, rx[m][0], rx[m][1]);
    }
  }
  for (int tb = tb0; tb < tb1; ++tb) {
    __syncthreads();
    if constexpr (PIPE) {
#pragma unroll
      for (int m = 0; m < MCO; ++m) store_dy(m, rdy[m][0], rdy[m][1]);
#pragma unroll
      for (int m = 0; m < MU; ++m) store_x(m, rx[m][0], rx[m][1]);
      if (tb + 1 < tb1) {
        const Org o = origin(tb + 1);
#pragma unroll
        for (int m = 0; m < MCO; ++m) load_dy(m, o, rdy[m][0], rdy[m][1]);
#pragma unroll
        for (int m = 0; m < MU; ++m) load_x(m, o, rx[m][0], rx[m][1]);
      }
    } else {
      const Org o = origin(tb);
#pragma unroll
      for (int m = 0; m < MCO; ++m) {
        uint4 v0, v1;
        load_dy(m, o, v0, v1);
        store_dy(m, v0, v1);
      }
#pragma unroll
      for (int m = 0; m < MU; ++m) {
        uint4 v0, v1;
        load_x(m, o, v0, v1);
        store_x(m, v0, v1);
      }
    }
    __syncthreads();
    if (do_db && (threadIdx.x >> 2) < nco) {
      const uint16_t* row = sdy + (threadIdx.x >> 2) * DP + (threadIdx.x & 3) * 64;
#pragma unroll
      for (int e = 0; e < 64; e += 8) {
        const uint4 v = *reinterpret_cast<const uint4*>(row + e);
        const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) dbacc += bf2f((uint16_t)(wv[h] & 0xffffu)) + bf2f((uint16_t)(wv[h] >> 16));
      }
    }
#pragma unroll 2
    for (int ks = 0; ks < 8; ++ks) {
      const int p0 = ks * 32 + kq * 8;
      const int posoff = ((p0 >> (lgk + 2)) * HJ + ((p0 >> lgk) & 3)) * HK + (p0 & (TK - 1));
      bf16x8 av[MCO];
#pragma unroll
      for (int b = 0; b < MCO; ++b)
        av[b] = b * 16 < nco ? *reinterpret_cast<const bf16x8*>(sdy + (b * 16 + r) * DP + p0) : bf16x8{};
#pragma unroll
      for (int j = 0; j < NU; ++j) {
        if (!uact[j]) continue;
        const uint16_t* src = sx + uoff[j] + posoff;
        const uint4 w4 = *reinterpret_cast<const uint4*>(src);
        const uint32_t w5 = *reinterpret_cast<const uint32_t*>(src + 8);
        const uint32_t wv[5] = {w4.x, w4.y, w4.z, w4.w, w5};
        uint32_t sh[3][4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          sh[0][d] = wv[d];
          sh[1][d] = __builtin_amdgcn_alignbit(wv[d + 1], wv[d], 16);
          sh[2][d] = wv[d + 1];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          bf16x8 bv;
          __builtin_memcpy(&bv, sh[c], 16);
#pragma unroll
          for (int b = 0; b < MCO; ++b)
            if (b * 16 < nco) acc[j][c][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[b], bv, acc[j][c][b], 0, 0, 0);
        }
      }
    }
  }
  if (do_db) {
    dbacc += __shfl_xor(dbacc, 1);
    dbacc += __shfl_xor(dbacc, 2);
    const int co = threadIdx.x >> 2;
    if ((threadIdx.x & 3) == 0 && co < nco) dbpart[(int64_t)blockIdx.x * cout + co0 + co] = dbacc;
  }
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    if (!uact[j]) continue;
    const int u = wave + 4 * j;
    const int ab = ab0 + u / MCI, ci = ci0 + (u % MCI) * 16 + r;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float* out = part + ((int64_t)blockIdx.x * 27 + ab * 3 + c) * (int64_t)cout * cin;
#pragma unroll
      for (int b = 0; b < MCO; ++b) {
        if (b * 16 >= nco) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) out[(int64_t)(co0 + b * 16 + kq * 4 + i) * cin + ci] = acc[j][c][b][i];
      }
    }
  }
}

// partial sums of up to 128 consecutive chunks: out[c2][e] = sum_{k < 128} part[c2 * 128 + k][e]
__global__ void __launch_bounds__(256)
k_reduce_chunks_pre(const float* __restrict__ part, int nchunk, int64_t per_chunk, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= per_chunk) return;
  const int k0 = blockIdx.y * 128, k1 = min(nchunk, k0 + 128);
  float s = 0.0f;
  for (int k = k0; k < k1; ++k) s += part[(int64_t)k * per_chunk + e];
  out[(int64_t)blockIdx.y * per_chunk + e] = s;
}

// out[(t * rows + o) * keep + i] = sum_chunks part[chunk][t][o][i], i < keep (fixed order)
__global__ void __launch_bounds__(256)
k_reduce_chunks(const float* __restrict__ part, int nchunk, int64_t per_chunk, int cols, int keep,
                float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= per_chunk) return;
  const int i = (int)(e % cols);
  if (i >= keep) return;
  float s = 0.0f;
#pragma unroll 8
  for (int k = 0; k < nchunk; ++k) s += part[(int64_t)k * per_chunk + e];
  out[(e / cols) * keep + i] = s;
}

// nearest x2 upsampling, channels last, 8 channels (16 B) per thread
__global__ void __launch_bounds__(256)
k_up2(const uint16_t* __restrict__ a, int n, int D, int C, uint16_t* __restrict__ u) {
  const int D2 = 2 * D, c8n = C / 8;
  const int64_t tot = (int64_t)n * D2 * D2 * D2 * c8n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= tot) return;
  int64_t q = e;
  const int c8 = (int)(q % c8n);
  q /= c8n;
  const int k = (int)(q % D2);
  q /= D2;
  const int j = (int)(q % D2);
  q /= D2;
  const int i = (int)(q % D2);
  const int64_t s = q / D2;
  const int64_t src = (((s * D + (i >> 1)) * D + (j >> 1)) * D + (k >> 1)) * C + c8 * 8;
  reinterpret_cast<uint4*>(u)[e] = *reinterpret_cast<const uint4*>(a + src);
}

// dh[coarse] = silu'(pre[coarse]) * sum of the 8 fine children of du (adjoint of k_up2,
// then the activation's derivative)
__global__ void __launch_bounds__(256)
k_pool2_gate(const uint16_t* __restrict__ du, int n, int D, int C, const uint16_t* __restrict__ pre,
             uint16_t* __restrict__ dh) {
  const int D2 = 2 * D, c8n = C / 8;
  const int64_t tot = (int64_t)n * D * D * D * c8n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= tot) return;
  int64_t q = e;
  const int c8 = (int)(q % c8n);
  q /= c8n;
  const int k = (int)(q % D);
  q /= D;
  const int j = (int)(q % D);
  q /= D;
  const int i = (int)(q % D);
  const int64_t s = q / D;
  float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int di = 0; di < 2; ++di)
    for (int dj = 0; dj < 2; ++dj)
      for (int dk = 0; dk < 2; ++dk) {
        const int64_t f = (((s * D2 + 2 * i + di) * D2 + 2 * j + dj) * D2 + 2 * k + dk) * C + c8 * 8;
        const uint4 v = *reinterpret_cast<const uint4*>(du + f);
        const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
        for (int q2 = 0; q2 < 8; ++q2) acc[q2] += bf2f(h[q2]);
      }
  const uint4 pv = reinterpret_cast<const uint4*>(pre)[e];
  const uint16_t* ph = reinterpret_cast<const uint16_t*>(&pv);
  uint4 o;
  uint16_t* oh = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
  for (int q2 = 0; q2 < 8; ++q2) oh[q2] = f2bf(acc[q2] * silu_d(bf2f(ph[q2])));
  reinterpret_cast<uint4*>(dh)[e] = o;
}

// standardised features, zero-padded to 32 channels
__global__ void k_features(const float* __restrict__ prm, int n, const float* __restrict__ mean_std,
                           uint16_t* __restrict__ z0) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * 32) return;
  const int s = e / 32, f = e % 32;
  float v = 0.0f;
  if (f < 4) {
    float q = prm[s * 4 + f];
    if (f == 3) q = logf(q);
    v = (q - mean_std[f]) / mean_std[4 + f];
  }
  z0[e] = f2bf(v);
}

__device__ __forceinline__ float log_prior(const float* prm, int s, int i, int j, int k, int N, float dx) {
  const float nx = prm[s * 4], ny = prm[s * 4 + 1], nz = prm[s * 4 + 2];
  const float h = 0.5f * (float)(N - 1);
  const float x = ((float)i - h) * dx, y = ((float)j - h) * dx, z = ((float)k - h) * dx;
  return 0.25f * (logf(nx * 0.31830988618379067f) + logf(ny * 0.31830988618379067f) +
                  logf(nz * 0.31830988618379067f)) -
         0.5f * (nx * x * x + ny * y * y + nz * z * z);
}

// psi = exp(min(wh . a + bh + ln G, FMAX)); C multiple of 8
__global__ void __launch_bounds__(256)
k_head_fwd(const uint16_t* __restrict__ aL, int64_t P, int N, int C, const float* __restrict__ whb,
           const float* __restrict__ prm, float dx, void* __restrict__ out, int cplx) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  int64_t q = p;
  const int k = (int)(q % N);
  q /= N;
  const int j = (int)(q % N);
  q /= N;
  const int i = (int)(q % N);
  const int s = (int)(q / N);
  float f = whb[C];
  for (int c8 = 0; c8 < C; c8 += 8) {
    const uint4 v = *reinterpret_cast<const uint4*>(aL + p * C + c8);
    const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
    for (int e = 0; e < 8; ++e) f += whb[c8 + e] * bf2f(h[e]);
  }
  f += log_prior(prm, s, i, j, k, N, dx);
  const float psi = __expf(fminf(f, kFMax));
  if (cplx == 2) reinterpret_cast<double2*>(out)[p] = make_double2((double)psi, 0.0);
  else if (cplx) reinterpret_cast<float2*>(out)[p] = make_float2(psi, 0.0f);
  else reinterpret_cast<float*>(out)[p] = psi;
}

// loss and the head's backward: df = dL/dpsi * psi (zero where clamped);
// dh[p][c] = df wh[c] silu'(pre[p][c]); per-block partials of sum (psi - t)^2, of
// df a[p][c] and of df (wave shuffles, then the 4 waves in fixed order).
// LOSS: dL/dpsi = 2 (psi - t) scale from the target (t = tgt); otherwise dL/dpsi is
// given per point (tgt holds it) and the loss partials are zero.
template <int C, bool LOSS>
__global__ void __launch_bounds__(256)
k_head_bwd(const float* __restrict__ psi, const float* __restrict__ tgt, const uint16_t* __restrict__ aL,
           const uint16_t* __restrict__ preL, int64_t P, const float* __restrict__ whb, float scale,
           uint16_t* __restrict__ dh, float* __restrict__ gpart, double* __restrict__ lpart) {
  __shared__ float sred[4][C + 1];
  __shared__ double dred[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float df = 0.0f;
  double d2 = 0.0;
  float ga[C];
  const bool pv = p < P;
  if (pv) {
    const float ps = psi[p];
    if (LOSS) {
      const float d = ps - tgt[p];
      d2 = (double)d * (double)d;
      df = ps < __expf(kFMax) ? 2.0f * d * scale * ps : 0.0f;
    } else {
      df = ps < __expf(kFMax) ? tgt[p] * ps : 0.0f;
    }
  }
#pragma unroll
  for (int c8 = 0; c8 < C; c8 += 8) {
    uint4 av = make_uint4(0, 0, 0, 0), hv = make_uint4(0, 0, 0, 0);
    if (pv) {
      av = *reinterpret_cast<const uint4*>(aL + p * C + c8);
      hv = *reinterpret_cast<const uint4*>(preL + p * C + c8);
    }
    const uint16_t* ah = reinterpret_cast<const uint16_t*>(&av);
    const uint16_t* hh = reinterpret_cast<const uint16_t*>(&hv);
    uint4 o;
    uint16_t* oh = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      ga[c8 + e] = df * bf2f(ah[e]);
      oh[e] = f2bf(df * whb[c8 + e] * silu_d(bf2f(hh[e])));
    }
    if (pv) *reinterpret_cast<uint4*>(dh + p * C + c8) = o;
  }
#pragma unroll
  for (int c = 0; c <= C; ++c) {
    float v = c < C ? ga[c] : df;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) sred[wave][c] = v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d2 += __shfl_xor(d2, off);
  if (lane == 0) dred[wave] = d2;
  __syncthreads();
  if ((int)threadIdx.x <= C)
    gpart[(int64_t)blockIdx.x * (C + 1) + threadIdx.x] =
        ((sred[0][threadIdx.x] + sred[1][threadIdx.x]) + sred[2][threadIdx.x]) + sred[3][threadIdx.x];
  if (threadIdx.x == 0) lpart[blockIdx.x] = ((dred[0] + dred[1]) + dred[2]) + dred[3];
}

__global__ void k_sum_double(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += part[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// BF16 copies of a weight [T][rows][cols]: dst [T][rows][cpad] (zero padded columns) and,
// if dst_t, the mirrored transpose dst_t[T-1-t][cols][rows]
__global__ void k_pack(const float* __restrict__ src, int T, int rows, int cols, int cpad, uint16_t* __restrict__ dst,
                       uint16_t* __restrict__ dst_t) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t tot = (int64_t)T * rows * cpad;
  if (e >= tot) return;
  const int i = (int)(e % cpad);
  const int64_t q = e / cpad;
  const int o = (int)(q % rows);
  const int t = (int)(q / rows);
  const float v = i < cols ? src[((int64_t)t * rows + o) * cols + i] : 0.0f;
  dst[e] = f2bf(v);
  if (dst_t && i < cols) dst_t[((int64_t)(T - 1 - t) * cols + i) * rows + o] = f2bf(v);
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const float gv = g[e];
  const float mv = b1 * m[e] + (1.0f - b1) * gv;
  const float vv = b2 * v[e] + (1.0f - b2) * gv * gv;
  m[e] = mv;
  v[e] = vv;
  w[e] -= lr * (mv * c1) / (sqrtf(vv * c2) + eps);
}

}  // namespace nn

using namespace nn;

// ------------------------------------------------------------------------------- host
namespace {

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// input-channel slice of the split dense layer: a multiple of 128 (4 waves x 32), at most
// 8 slices
int dense_kslice(int cin) {
  const int ks = (cin + 7) / 8;
  return ((ks + 127) / 128) * 128;
}
int64_t dense_ws_floats(int64_t P, int cin, int cout) {
  const int kslice = dense_kslice(cin);
  return (int64_t)((cin + kslice - 1) / kslice) * P * cout;
}

// ws (nullable): FP32 workspace of ws_floats; with room for dense_ws_floats, one-tap
// layers over at most 64 positions take the split path
// tiled 3x3x3 path: D a power of two >= 8 and P a whole number of D^3 samples
bool conv_tiled(int64_t P, int D) {
  return D >= 8 && (D & (D - 1)) == 0 && P % ((int64_t)D * D * D) == 0;
}

// up: x is given on the 2x coarser grid and upsampled on the fly (tiled path only)
hipError_t launch_conv(int ks, int64_t P, int D, int cin, int cout, const uint16_t* x, const uint16_t* w,
                       const float* bias, int act, const uint16_t* gate, uint16_t* y, uint16_t* pre,
                       hipStream_t st, float* ws = nullptr, int64_t ws_floats = 0, bool up = false) {
  if (up && !(ks == 3 && conv_tiled(P, D))) return hipErrorInvalidValue;
  if (ks == 1 && P <= 64 && cin % 32 == 0 && ws && dense_ws_floats(P, cin, cout) <= ws_floats) {
    const int kslice = dense_kslice(cin);
    const int S = (cin + kslice - 1) / kslice;
    dim3 g((unsigned)((P + 15) / 16), (unsigned)((cout + 63) / 64), (unsigned)S);
    hipLaunchKernelGGL(k_dense_sk, g, dim3(256), 0, st, x, w, (int)P, cin, cout, kslice, ws);
    hipLaunchKernelGGL(k_dense_finish, dim3(nblk(P * cout)), dim3(256), 0, st, ws, S, (int)P, cout, bias, act, gate,
                       y, pre);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((P + 63) / 64), (unsigned)((cout + 63) / 64));
  const bool k32 = cin % 32 == 0;
  if (ks == 3 && conv_tiled(P, D)) {
    const int TK = D < 16 ? D : 16, TJ = 4, TI = 256 / (TJ * TK);
    const size_t lds = (size_t)(TI + 2) * (TJ + 2) * (TK + 2) * ((k32 ? 32 : 16) + 8) * sizeof(uint16_t);
    const int64_t nbrick = P / 256;
    // 16-channel output blocks per wave; on small grids (fewer bricks than about two per
    // CU) one per block, so that more blocks share the work
    const int nbt = nbrick * ((cout + 63) / 64) < 512 ? 1 : cout <= 16 ? 1 : cout <= 32 ? 2 : 4;
    // about three resident blocks per CU walk the bricks (a multiple of 8 blocks so the
    // XCD dealing applies)
    const int64_t gy = (cout + 16 * nbt - 1) / (16 * nbt);
    int64_t gx = (kConvBlocks + gy - 1) / gy;
    gx = (gx + 7) / 8 * 8;
    // (measured: 16-channel inputs and four-tile outputs run faster one brick per block)
    if (gx > nbrick || !k32 || nbt == 4) gx = nbrick;
    dim3 tg((unsigned)gx, (unsigned)gy);
#define CT(A, B, C)                                                                                         \
  do {                                                                                                      \
    if (up)                                                                                                 \
      hipLaunchKernelGGL((k_conv3_tiled<A, B, C, true>), tg, dim3(256), lds, st, x, w, bias, D, cin, cout, act, \
                         gate, y, pre, (int)nbrick);                                                        \
    else                                                                                                    \
      hipLaunchKernelGGL((k_conv3_tiled<A, B, C, false>), tg, dim3(256), lds, st, x, w, bias, D, cin, cout, act, \
                         gate, y, pre, (int)nbrick);                                                        \
  } while (0)
#define CTN(A, B)     \
  do {                \
    if (nbt == 1) CT(A, B, 1); \
    else if (nbt == 2) CT(A, B, 2); \
    else CT(A, B, 4); \
  } while (0)
    if (k32) {
      if (TK == 16) CTN(32, 16);
      else CTN(32, 8);
    } else {
      if (TK == 16) CTN(16, 16);
      else CTN(16, 8);
    }
#undef CTN
#undef CT
    return hipGetLastError();
  }
  if (ks == 3) {
    if (k32) hipLaunchKernelGGL((k_conv<3, 32>), grid, dim3(256), 0, st, x, w, bias, P, D, cin, cout, act, gate, y, pre);
    else hipLaunchKernelGGL((k_conv<3, 16>), grid, dim3(256), 0, st, x, w, bias, P, D, cin, cout, act, gate, y, pre);
  } else {
    if (k32) hipLaunchKernelGGL((k_conv<1, 32>), grid, dim3(256), 0, st, x, w, bias, P, 1, cin, cout, act, gate, y, pre);
    else hipLaunchKernelGGL((k_conv<1, 16>), grid, dim3(256), 0, st, x, w, bias, P, 1, cin, cout, act, gate, y, pre);
  }
  return hipGetLastError();
}

// positions per split-K block: at least kChunkMin, and at most kMaxChunks blocks per tap
int64_t wgrad_chunk(int64_t P) {
  const int64_t c = ((P + kMaxChunks - 1) / kMaxChunks + 63) / 64 * 64;
  return c > kChunkMin ? c : kChunkMin;
}
int64_t wgrad_nch(int64_t P) { return (P + wgrad_chunk(P) - 1) / wgrad_chunk(P); }

// Launch shape of one weight gradient.  Tiled (k_wgrad3_tiled) for 3x3x3 taps on a
// power-of-two grid D >= 8 holding whole samples: units of (tap pair, 16 input channels)
// spread over the 4 waves with at most 120 accumulators per lane, the rest of the grid
// split into runs of bricks so that about kTiledBlocks blocks are in flight.
constexpr int kTiledBlocks = 512;
struct WgPlan {
  bool tiled = false;
  int mco = 1, mci = 1, nu = 1, nab = 9, groups = 1, zt = 1, ntiles = 0, tpb = 0;
  int64_t nch = 0;
  size_t lds = 0;
};

WgPlan wgrad_plan(int ks, int64_t P, int D, int cin, int cout) {
  WgPlan w;
  w.tiled = ks == 3 && D >= 8 && (D & (D - 1)) == 0 && P % ((int64_t)D * D * D) == 0 && P / 256 < (1ll << 30);
  if (!w.tiled) {
    w.nch = wgrad_nch(P);
    return w;
  }
  const int tco = cout < 64 ? cout : 64;
  w.mco = tco <= 16 ? 1 : 2;  // 32-channel output tiles at most: the wider tile measured slower
  w.mci = cin >= 32 ? 2 : 1;
  w.nab = 9;
  w.nu = (w.nab * w.mci + 3) / 4;
  w.groups = (9 + w.nab - 1) / w.nab;
  w.zt = ((cout + 16 * w.mco - 1) / (16 * w.mco)) * ((cin + 16 * w.mci - 1) / (16 * w.mci));
  w.ntiles = (int)(P / 256);
  int64_t want = (kTiledBlocks + w.groups * w.zt - 1) / (w.groups * w.zt);
  if (want < 1) want = 1;
  if (want > w.ntiles) want = w.ntiles;
  w.tpb = (int)((w.ntiles + want - 1) / want);
  w.nch = (w.ntiles + w.tpb - 1) / w.tpb;
  const int TK = D < 16 ? D : 16, TJ = 4, TI = 256 / (TJ * TK);
  const int HR = (TI + 2) * (TJ + 2) * (TK == 16 ? 24 : 16);
  const int CS = HR + ((8 - HR) % 128 + 128) % 128;
  w.lds = ((size_t)16 * w.mco * 264 + (size_t)16 * w.mci * CS) * sizeof(uint16_t);
  return w;
}

int64_t wgrad_part_floats(int ks, int64_t P, int D, int cin, int cout) {
  return wgrad_plan(ks, P, D, cin, cout).nch * (int64_t)ks * ks * ks * cout * cin;
}

// dw[t][o][i < keep] (row stride keep) and db[o] (nullable) from dy [P][cout], x [P][cin];
// part holds wgrad_part_floats, cpart wgrad_plan(...).nch * cout floats
// up: x is given on the 2x coarser grid and upsampled on the fly (tiled path only)
hipError_t launch_wgrad(int ks, int64_t P, int D, int cin, int cout, int keep, const uint16_t* dy, const uint16_t* x,
                        float* part, float* dw, float* cpart, float* db, hipStream_t st, bool up = false) {
  const int T = ks * ks * ks;
  float* dbp = db ? cpart : nullptr;
  const WgPlan pl = wgrad_plan(ks, P, D, cin, cout);
  const int nch = (int)pl.nch;
  if (up && !pl.tiled) return hipErrorInvalidValue;
  if (pl.tiled) {
    int lg = 0;
    while ((1 << lg) < D) ++lg;
    dim3 grid((unsigned)nch, (unsigned)pl.groups, (unsigned)pl.zt);
#define WT1(A, B, U, UPV)                                                                                      \
  do {                                                                                                         \
    if (pl.lds > 65536) { /* opt in to the large LDS allocation (on the current device) */                    \
      hipError_t ea = hipFuncSetAttribute((const void*)k_wgrad3_tiled<A, B, U, UPV>,                           \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);            \
      if (ea != hipSuccess) return ea;                                                                         \
    }                                                                                                          \
    hipLaunchKernelGGL((k_wgrad3_tiled<A, B, U, UPV>), grid, dim3(256), pl.lds, st, dy, x, D, lg, cin, cout,   \
                       pl.nab, pl.ntiles, pl.tpb, part, dbp);                                                  \
  } while (0)
#define WT(A, B, U)          \
  do {                       \
    if (up) WT1(A, B, U, true); \
    else WT1(A, B, U, false); \
  } while (0)
    if (pl.mco == 1) {
      if (pl.mci == 2) WT(1, 2, 5);
      else WT(1, 1, 3);
    } else {
      if (pl.mci == 2) WT(2, 2, 5);
      else WT(2, 1, 3);
    }
#undef WT
#undef WT1
  } else {
  const int64_t chunk = wgrad_chunk(P);
  dim3 grid((unsigned)nch, (unsigned)((T + 3) / 4), (unsigned)(((cout + 63) / 64) * ((cin + 63) / 64)));
  // accumulators for the largest tile of this launch; LDS for its rows
  const int tco = cout < 64 ? cout : 64, tci = cin < 64 ? cin : 64;
  const int G = T < 4 ? T : 4;
  const size_t lds = (size_t)(tco + G * tci) * 72 * sizeof(uint16_t);
  const int mco = tco <= 16 ? 1 : tco <= 32 ? 2 : 4, mci = tci <= 16 ? 1 : tci <= 32 ? 2 : 4;
#define WG(A, B)                                                                                                   \
  do {                                                                                                             \
    if (ks == 3)                                                                                                   \
      hipLaunchKernelGGL((k_wgrad<3, A, B>), grid, dim3(256), lds, st, dy, x, P, D, cin, cout, chunk, part, dbp); \
    else                                                                                                           \
      hipLaunchKernelGGL((k_wgrad<1, A, B>), grid, dim3(256), lds, st, dy, x, P, 1, cin, cout, chunk, part, dbp); \
  } while (0)
#define WGB(A)            \
  do {                    \
    if (mci == 1) WG(A, 1); \
    else if (mci == 2) WG(A, 2); \
    else WG(A, 4);        \
  } while (0)
  if (mco == 1) WGB(1);
  else if (mco == 2) WGB(2);
  else WGB(4);
#undef WGB
#undef WG
  }
  const int64_t per = (int64_t)T * cout * cin;
  hipLaunchKernelGGL(k_reduce_chunks, dim3(nblk(per)), dim3(256), 0, st, part, nch, per, cin, keep, dw);
  if (db)
    hipLaunchKernelGGL(k_reduce_chunks, dim3(nblk(cout)), dim3(256), 0, st, cpart, nch, (int64_t)cout, cout, cout, db);
  return hipGetLastError();
}

}  // namespace

struct gpnn {
  gpnn_arch a{};
  hipStream_t st = nullptr;
  std::string err;
  int S = 0, N = 0, F2 = 0;
  int64_t np = 0;
  // offsets into the FP32 parameter vector
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oC[7] = {}, oc[7] = {}, owh = 0;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *ms = nullptr;
  uint16_t *W1p = nullptr, *W2 = nullptr, *W2t = nullptr, *Cb[7] = {}, *Ct[7] = {};
  // activations
  uint16_t *z0 = nullptr, *h1 = nullptr, *a1 = nullptr, *h2 = nullptr, *a2 = nullptr;
  uint16_t *u[7] = {}, *h[7] = {}, *act[7] = {};
  uint16_t *dA = nullptr, *dB = nullptr, *dU = nullptr;
  float *part = nullptr, *cpart = nullptr, *gpart = nullptr;
  int64_t npart = 0;  // floats in part
  double *lpart = nullptr, *lsum = nullptr;
  std::vector<void*> allocs;
  // last forward
  int n = 0;
  const float* prm = nullptr;
  const void* out = nullptr;
  int out_cplx = 0;
};

namespace {

int set_err(gpnn* m, int code, const std::string& s) {
  if (m) m->err = s;
  return code;
}

int hip_chk(gpnn* m, hipError_t e, const char* what) {
  if (e == hipSuccess) return GPNN_OK;
  return set_err(m, GPNN_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T> int alloc(gpnn* m, T** p, int64_t count) {
  void* q = nullptr;
  if (gpk::dev_alloc(&q, (size_t)count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(m, GPNN_ERR_OOM, "device allocation failed");
  }
  m->allocs.push_back(q);
  *p = (T*)q;
  return GPNN_OK;
}

int64_t vol(int D) { return (int64_t)D * D * D; }

hipError_t refresh_bf16(gpnn* m) {
  const gpnn_arch& a = m->a;
  hipStream_t st = m->st;
  hipLaunchKernelGGL(k_pack, dim3(nblk((int64_t)a.hidden * 32)), dim3(256), 0, st, m->w + m->oW1, 1, a.hidden, 4, 32,
                     m->W1p, (uint16_t*)nullptr);
  hipLaunchKernelGGL(k_pack, dim3(nblk((int64_t)m->F2 * a.hidden)), dim3(256), 0, st, m->w + m->oW2, 1, m->F2,
                     a.hidden, a.hidden, m->W2, m->W2t);
  for (int s = 1; s <= m->S; ++s)
    hipLaunchKernelGGL(k_pack, dim3(nblk((int64_t)27 * a.ch[s] * a.ch[s - 1])), dim3(256), 0, st, m->w + m->oC[s], 27,
                       a.ch[s], a.ch[s - 1], a.ch[s - 1], m->Cb[s], m->Ct[s]);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int gpnn_create(const gpnn_arch* a, void* hip_stream, gpnn** out) {
  if (!a || !out) return GPNN_ERR_INVALID;
  *out = nullptr;
  const int S = a->nstage;
  if (S < 1 || S > 6 || a->base < 1 || a->max_batch < 1 || a->hidden < 16 || a->hidden % 16 || !(a->dx > 0))
    return GPNN_ERR_INVALID;
  for (int s = 0; s <= S; ++s)
    if (a->ch[s] < 16 || a->ch[s] % 16) return GPNN_ERR_INVALID;
  if (a->ch[S] != 16 && a->ch[S] != 32 && a->ch[S] != 64) return GPNN_ERR_INVALID;
  for (int f = 0; f < 4; ++f)
    if (!(a->in_std[f] > 0)) return GPNN_ERR_INVALID;
  const int64_t N = (int64_t)a->base << S;
  if (N > 1024 || (int64_t)a->max_batch * vol((int)N) * a->ch[S - 1] > ((int64_t)1 << 34)) return GPNN_ERR_INVALID;
  gpnn* m = new (std::nothrow) gpnn();
  if (!m) return GPNN_ERR_OOM;
  m->a = *a;
  m->st = (hipStream_t)hip_stream;
  m->S = S;
  m->N = (int)N;
  m->F2 = a->base * a->base * a->base * a->ch[0];
  int64_t o = 0;
  m->oW1 = o; o += (int64_t)a->hidden * 4;
  m->ob1 = o; o += a->hidden;
  m->oW2 = o; o += (int64_t)m->F2 * a->hidden;
  m->ob2 = o; o += m->F2;
  for (int s = 1; s <= S; ++s) {
    m->oC[s] = o; o += (int64_t)27 * a->ch[s] * a->ch[s - 1];
    m->oc[s] = o; o += a->ch[s];
  }
  m->owh = o; o += a->ch[S] + 1;
  m->np = o;
  const int B = a->max_batch;
  int rc = GPNN_OK;
  auto A = [&](auto** p, int64_t cnt) { if (rc == GPNN_OK) rc = alloc(m, p, cnt); };
  A(&m->w, o); A(&m->g, o); A(&m->m, o); A(&m->v, o); A(&m->ms, 8);
  A(&m->W1p, (int64_t)a->hidden * 32);
  A(&m->W2, (int64_t)m->F2 * a->hidden);
  A(&m->W2t, (int64_t)m->F2 * a->hidden);
  A(&m->z0, (int64_t)B * 32);
  A(&m->h1, (int64_t)B * a->hidden); A(&m->a1, (int64_t)B * a->hidden);
  A(&m->h2, (int64_t)B * m->F2); A(&m->a2, (int64_t)B * m->F2);
  int64_t maxd = (int64_t)B * std::max(m->F2, a->hidden), maxu = 0, maxpart = 0, maxc = 0;
  maxpart = std::max(wgrad_part_floats(1, B, 1, a->hidden, m->F2), wgrad_part_floats(1, B, 1, 32, a->hidden));
  maxc = std::max<int64_t>(m->F2, a->hidden);
  for (int s = 1; s <= S; ++s) {
    const int D = a->base << s;
    const int64_t P = (int64_t)B * vol(D);
    A(&m->Cb[s], (int64_t)27 * a->ch[s] * a->ch[s - 1]);
    A(&m->Ct[s], (int64_t)27 * a->ch[s] * a->ch[s - 1]);
    if (!conv_tiled(P, D)) A(&m->u[s], P * a->ch[s - 1]);  // tiled layers upsample on the fly
    A(&m->h[s], P * a->ch[s]);
    A(&m->act[s], P * a->ch[s]);
    maxd = std::max(maxd, P * a->ch[s]);
    maxd = std::max(maxd, (int64_t)B * vol(D / 2) * a->ch[s - 1]);
    maxu = std::max(maxu, P * a->ch[s - 1]);
    maxpart = std::max(maxpart, wgrad_part_floats(3, P, D, a->ch[s - 1], a->ch[s]));
    maxc = std::max(maxc, wgrad_plan(3, P, D, a->ch[s - 1], a->ch[s]).nch * a->ch[s]);
  }
  const int64_t PS = (int64_t)B * vol(m->N);
  const int64_t hblocks = (PS + 255) / 256;
  maxc = std::max(maxc, ((hblocks + 127) / 128) * (a->ch[S] + 1));  // head partials, first stage
  A(&m->dA, maxd); A(&m->dB, maxd); A(&m->dU, maxu);
  maxpart = std::max(maxpart, std::max(dense_ws_floats(B, 32, a->hidden),
                                       std::max(dense_ws_floats(B, a->hidden, m->F2), dense_ws_floats(B, m->F2, a->hidden))));
  m->npart = maxpart;
  A(&m->part, maxpart); A(&m->cpart, maxc);
  A(&m->gpart, hblocks * (a->ch[S] + 1));
  A(&m->lpart, hblocks); A(&m->lsum, 1);
  if (rc == GPNN_OK) {
    float hms[8];
    for (int f = 0; f < 4; ++f) {
      hms[f] = (float)a->in_mean[f];
      hms[4 + f] = (float)a->in_std[f];
    }
    rc = hip_chk(m, hipMemcpyAsync(m->ms, hms, sizeof(hms), hipMemcpyHostToDevice, m->st), "copy");
    if (rc == GPNN_OK) rc = hip_chk(m, hipStreamSynchronize(m->st), "sync");
  }
  if (rc != GPNN_OK) {
    gpnn_destroy(m);
    return rc;
  }
  *out = m;
  return GPNN_OK;
}

int gpnn_destroy(gpnn* m) {
  if (!m) return GPNN_ERR_INVALID;
  if (m->st) (void)hipStreamSynchronize(m->st);
  else (void)hipDeviceSynchronize();
  for (void* p : m->allocs) (void)hipFree(p);
  delete m;
  return GPNN_OK;
}

int gpnn_param_count(gpnn* m, int64_t* n) {
  if (!m || !n) return GPNN_ERR_INVALID;
  *n = m->np;
  return GPNN_OK;
}

int gpnn_set_params(gpnn* m, const float* host, int64_t n) {
  if (!m || !host || n != m->np) return set_err(m, GPNN_ERR_INVALID, "parameter count mismatch");
  int rc = hip_chk(m, hipMemcpyAsync(m->w, host, n * sizeof(float), hipMemcpyHostToDevice, m->st), "copy");
  if (!rc) rc = hip_chk(m, hipMemsetAsync(m->m, 0, n * sizeof(float), m->st), "memset");
  if (!rc) rc = hip_chk(m, hipMemsetAsync(m->v, 0, n * sizeof(float), m->st), "memset");
  if (!rc) rc = hip_chk(m, hipMemsetAsync(m->g, 0, n * sizeof(float), m->st), "memset");
  if (!rc) rc = hip_chk(m, refresh_bf16(m), "pack");
  if (!rc) rc = hip_chk(m, hipStreamSynchronize(m->st), "sync");
  return rc;
}

static int get_vec(gpnn* m, const float* src, float* host, int64_t n) {
  if (!m || !host || n != m->np) return set_err(m, GPNN_ERR_INVALID, "parameter count mismatch");
  int rc = hip_chk(m, hipMemcpyAsync(host, src, n * sizeof(float), hipMemcpyDeviceToHost, m->st), "copy");
  if (!rc) rc = hip_chk(m, hipStreamSynchronize(m->st), "sync");
  return rc;
}

int gpnn_get_params(gpnn* m, float* host, int64_t n) { return m ? get_vec(m, m->w, host, n) : GPNN_ERR_INVALID; }
int gpnn_get_grads(gpnn* m, float* host, int64_t n) { return m ? get_vec(m, m->g, host, n) : GPNN_ERR_INVALID; }

int gpnn_forward(gpnn* m, const float* prm, int32_t n, void* out, int32_t out_complex64) {
  if (!m || !prm || !out || n < 1 || n > m->a.max_batch) return set_err(m, GPNN_ERR_INVALID, "bad forward arguments");
  if (out_complex64 < 0 || out_complex64 > 2) return set_err(m, GPNN_ERR_INVALID, "bad output kind");
  const gpnn_arch& a = m->a;
  hipStream_t st = m->st;
  hipLaunchKernelGGL(k_features, dim3(nblk((int64_t)n * 32)), dim3(256), 0, st, prm, n, m->ms, m->z0);
  hipError_t e = launch_conv(1, n, 1, 32, a.hidden, m->z0, m->W1p, m->w + m->ob1, 1, nullptr, m->a1, m->h1, st,
                             m->part, m->npart);
  if (e == hipSuccess)
    e = launch_conv(1, n, 1, a.hidden, m->F2, m->a1, m->W2, m->w + m->ob2, 1, nullptr, m->a2, m->h2, st, m->part,
                    m->npart);
  const uint16_t* prev = m->a2;
  for (int s = 1; s <= m->S && e == hipSuccess; ++s) {
    const int Dc = a.base << (s - 1), D = a.base << s;
    const int64_t Ps = (int64_t)n * vol(D);
    if (conv_tiled(Ps, D)) {  // nearest x2 upsampling read on the fly by the convolution
      e = launch_conv(3, Ps, D, a.ch[s - 1], a.ch[s], prev, m->Cb[s], m->w + m->oc[s], 1, nullptr, m->act[s], m->h[s],
                      st, nullptr, 0, true);
    } else {
      const int64_t tot = Ps * (a.ch[s - 1] / 8);
      hipLaunchKernelGGL(k_up2, dim3(nblk(tot)), dim3(256), 0, st, prev, n, Dc, a.ch[s - 1], m->u[s]);
      e = launch_conv(3, Ps, D, a.ch[s - 1], a.ch[s], m->u[s], m->Cb[s], m->w + m->oc[s], 1, nullptr, m->act[s],
                      m->h[s], st);
    }
    prev = m->act[s];
  }
  if (e == hipSuccess) {
    const int64_t P = (int64_t)n * vol(m->N);
    hipLaunchKernelGGL(k_head_fwd, dim3(nblk(P)), dim3(256), 0, st, prev, P, m->N, a.ch[m->S], m->w + m->owh, prm,
                       (float)a.dx, out, out_complex64);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_chk(m, e, "forward");
  m->n = n;
  m->prm = prm;
  m->out = out;
  m->out_cplx = out_complex64;
  return GPNN_OK;
}

}  // extern "C"

namespace {

// Backward pass from the head: LOSS takes dL/dpsi from the L2 loss against `src` (the
// target), otherwise `src` is dL/dpsi itself.  Overwrites every parameter gradient.
template <bool LOSS> int backward_from(gpnn* m, const float* src, double* loss) {
  const gpnn_arch& a = m->a;
  hipStream_t st = m->st;
  const int n = m->n, S = m->S;
  const int64_t P = (int64_t)n * vol(m->N);
  const unsigned hb = nblk(P);
  const float scale = (float)(a.dx * a.dx * a.dx / n);
  const float* psi = (const float*)m->out;
  if (a.ch[S] == 16)
    hipLaunchKernelGGL((k_head_bwd<16, LOSS>), dim3(hb), dim3(256), 0, st, psi, src, m->act[S], m->h[S], P,
                       m->w + m->owh, scale, m->dA, m->gpart, m->lpart);
  else if (a.ch[S] == 32)
    hipLaunchKernelGGL((k_head_bwd<32, LOSS>), dim3(hb), dim3(256), 0, st, psi, src, m->act[S], m->h[S], P,
                       m->w + m->owh, scale, m->dA, m->gpart, m->lpart);
  else
    hipLaunchKernelGGL((k_head_bwd<64, LOSS>), dim3(hb), dim3(256), 0, st, psi, src, m->act[S], m->h[S], P,
                       m->w + m->owh, scale, m->dA, m->gpart, m->lpart);
  {  // head partials: groups of 128 blocks first (into the bias-partials buffer, free here)
    const int per = a.ch[S] + 1, n2 = (int)((hb + 127) / 128);
    hipLaunchKernelGGL(k_reduce_chunks_pre, dim3(nblk(per), (unsigned)n2), dim3(256), 0, st, m->gpart, (int)hb,
                       (int64_t)per, m->cpart);
    hipLaunchKernelGGL(k_reduce_chunks, dim3(nblk(per)), dim3(256), 0, st, m->cpart, n2, (int64_t)per, per, per,
                       m->g + m->owh);
  }
  hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(256), 0, st, m->lpart, (int)hb, m->lsum);
  hipError_t e = hipGetLastError();
  uint16_t* dh = m->dA;  // gradient w.r.t. the pre-activation of the current layer
  uint16_t* other = m->dB;
  for (int s = S; s >= 1 && e == hipSuccess; --s) {
    const int D = a.base << s, Dc = a.base << (s - 1);
    const int64_t Ps = (int64_t)n * vol(D);
    const bool up = conv_tiled(Ps, D);  // the layer's input: the coarse activations, upsampled on the fly
    const uint16_t* xin = up ? (s > 1 ? m->act[s - 1] : m->a2) : m->u[s];
    e = launch_wgrad(3, Ps, D, a.ch[s - 1], a.ch[s], a.ch[s - 1], dh, xin, m->part, m->g + m->oC[s], m->cpart,
                     m->g + m->oc[s], st, up);
    if (e != hipSuccess) break;
    e = launch_conv(3, Ps, D, a.ch[s], a.ch[s - 1], dh, m->Ct[s], nullptr, 0, nullptr, m->dU, nullptr, st);
    if (e != hipSuccess) break;
    const uint16_t* pre_prev = s > 1 ? m->h[s - 1] : m->h2;
    const int64_t tot = (int64_t)n * vol(Dc) * (a.ch[s - 1] / 8);
    hipLaunchKernelGGL(k_pool2_gate, dim3(nblk(tot)), dim3(256), 0, st, m->dU, n, Dc, a.ch[s - 1], pre_prev, other);
    e = hipGetLastError();
    std::swap(dh, other);
  }
  // dense layers: dh = dL/dh2 [n][F2]
  if (e == hipSuccess)
    e = launch_wgrad(1, n, 1, a.hidden, m->F2, a.hidden, dh, m->a1, m->part, m->g + m->oW2, m->cpart, m->g + m->ob2,
                     st);
  if (e == hipSuccess)
    e = launch_conv(1, n, 1, m->F2, a.hidden, dh, m->W2t, nullptr, 0, m->h1, other, nullptr, st, m->part, m->npart);
  if (e == hipSuccess)
    e = launch_wgrad(1, n, 1, 32, a.hidden, 4, other, m->z0, m->part, m->g + m->oW1, m->cpart, m->g + m->ob1, st);
  if (e != hipSuccess) return hip_chk(m, e, "backward");
  if (loss) {
    int rc = hip_chk(m, hipMemcpyAsync(loss, m->lsum, sizeof(double), hipMemcpyDeviceToHost, st), "copy");
    if (!rc) rc = hip_chk(m, hipStreamSynchronize(st), "sync");
    if (rc) return rc;
    *loss *= a.dx * a.dx * a.dx / n;
  }
  return GPNN_OK;
}

}  // namespace

extern "C" {

int gpnn_loss_backward(gpnn* m, const float* tgt, double* loss) {
  if (!m || !tgt) return set_err(m, GPNN_ERR_INVALID, "bad backward arguments");
  if (m->n < 1 || m->out_cplx) return set_err(m, GPNN_ERR_STATE, "no FP32 forward pass to differentiate");
  return backward_from<true>(m, tgt, loss);
}

int gpnn_backward(gpnn* m, const void* grad_psi_dev) {
  if (!m || !grad_psi_dev) return set_err(m, GPNN_ERR_INVALID, "bad backward arguments");
  if (m->n < 1 || m->out_cplx) return set_err(m, GPNN_ERR_STATE, "no FP32 forward pass to differentiate");
  if (reinterpret_cast<uintptr_t>(grad_psi_dev) % sizeof(float) != 0)
    return set_err(m, GPNN_ERR_INVALID, "grad_psi is not aligned to float");
  return backward_from<false>(m, static_cast<const float*>(grad_psi_dev), nullptr);
}

int gpnn_adam_step(gpnn* m, float lr, float b1, float b2, float eps, int64_t t) {
  if (!m || t < 1 || !(lr >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps >= 0))
    return set_err(m, GPNN_ERR_INVALID, "bad Adam arguments");
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)t)));
  hipLaunchKernelGGL(k_adam, dim3(nblk(m->np)), dim3(256), 0, m->st, m->w, m->g, m->m, m->v, m->np, lr, b1, b2, eps,
                     c1, c2);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = refresh_bf16(m);
  return hip_chk(m, e, "adam");
}

int gpnn_conv(int32_t ks, int32_t n, int32_t d, int32_t cin, int32_t cout, const void* x, const void* w,
              const float* bias, int32_t act, const void* gate, void* y, void* pre, void* hip_stream) {
  if ((ks != 1 && ks != 3) || n < 1 || (ks == 3 && (d < 1 || d > 1024)) || cin < 16 || cin % 16 || cout < 16 ||
      cout % 16 || !x || !w || !y)
    return GPNN_ERR_INVALID;
  const int64_t P = ks == 3 ? (int64_t)n * vol(d) : n;
  hipStream_t st = (hipStream_t)hip_stream;
  float* ws = nullptr;
  const int64_t nws = ks == 1 ? dense_ws_floats(P, cin, cout) : 0;
  if (nws > 0 && hipMalloc((void**)&ws, (size_t)nws * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return GPNN_ERR_OOM;
  }
  hipError_t e = launch_conv(ks, P, ks == 3 ? d : 1, cin, cout, (const uint16_t*)x, (const uint16_t*)w, bias, act,
                             (const uint16_t*)gate, (uint16_t*)y, (uint16_t*)pre, st, ws, nws);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (ws) (void)hipFree(ws);
  return e == hipSuccess ? GPNN_OK : GPNN_ERR_HIP;
}

int gpnn_conv_wgrad(int32_t ks, int32_t n, int32_t d, int32_t cin, int32_t cout, const void* dy, const void* x,
                    float* dw, float* db, void* hip_stream) {
  if ((ks != 1 && ks != 3) || n < 1 || (ks == 3 && (d < 1 || d > 1024)) || cin < 16 || cin % 16 || cout < 16 ||
      cout % 16 || !dy || !x || !dw)
    return GPNN_ERR_INVALID;
  const int64_t P = ks == 3 ? (int64_t)n * vol(d) : n;
  hipStream_t st = (hipStream_t)hip_stream;
  float *part = nullptr, *cpart = nullptr;
  const int64_t nch = wgrad_plan(ks, P, ks == 3 ? d : 1, cin, cout).nch;
  if (hipMalloc((void**)&part, (size_t)wgrad_part_floats(ks, P, ks == 3 ? d : 1, cin, cout) * sizeof(float)) !=
          hipSuccess ||
      hipMalloc((void**)&cpart, (size_t)nch * cout * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    if (part) (void)hipFree(part);
    return GPNN_ERR_OOM;
  }
  hipError_t e = launch_wgrad(ks, P, ks == 3 ? d : 1, cin, cout, cin, (const uint16_t*)dy, (const uint16_t*)x, part,
                              dw, cpart, db, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(part);
  (void)hipFree(cpart);
  return e == hipSuccess ? GPNN_OK : GPNN_ERR_HIP;
}

const char* gpnn_last_error(gpnn* m) { return m ? m->err.c_str() : "null model"; }

}  // extern "C"
