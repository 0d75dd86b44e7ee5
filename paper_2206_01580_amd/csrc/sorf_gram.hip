// Normal-equation accumulation G += Z^T Z, Zty += Z^T y on gfx950 MFMA.
//
// Paper: arXiv 2206.01580, RFF subsection (regularised normal equation; the
// Z^T Z product dominates training) and Timings (FP32 Z^T Z suffers cumulative
// round-off, which the paper counters with Kahan summation; DP training).
//
// Modes. FP32: FP32 operands on v_mfma_f32_32x32x2f32. BF16/FP16 x1: one
// 16-bit product hi^T hi. hi+lo: z = hi + lo with hi = round(z),
// lo = round(z - hi) in bf16 or fp16 and G accumulates all four products
// hi^T hi + hi^T lo + lo^T hi + lo^T lo, i.e. the Gram of hi + lo, which is
// positive semidefinite (dropping lo^T lo is not).
//
// Accumulation. A matrix-core accumulator that has grown large loses the low
// bits of small addends with a bias: over 20,000 QM9-like rows the single
// running accumulator of the hi+lo modes drifted by about -3e-7 sqrt(G_ii
// G_jj) off the diagonal, enough to make G + 1e-6 I indefinite. Here every
// mode accumulates 256 rows at a time in a fresh MFMA
// accumulator P and adds P into an FP32 sum S with round-to-nearest adds (a blocked
// summation in the spirit of the paper's compensated sum); this also cuts
// the FP32 mode's error by an order of magnitude.
//
// Work split. FP32 modes: 16 waves (four per SIMD) per 256 x 128 tile (I, J)
// of the lower triangle, each wave 32 x 64 (1 x 2 MFMA 32x32 blocks), as two
// 8-wave workgroups of 128 x 128 that share a compute unit, rows staged
// through a global-to-LDS ring; when the tiles alone would leave
// compute units idle, a tile's rows are split into slices whose sums are
// combined in slice order. hi+lo modes (and the split mode's tail): 8 waves (4 x 2, two
// per SIMD) per 256 x 128 tile, each wave 64 x 64 (2 x 2 blocks). Single
// product modes (and the split mode's int8 head): 8 waves (2 x 4) per 256 x 256
// tile, each wave 128 x 64. The 256 x 128 tiles are dealt to the XCDs in
// super-tiles of 4 x 8 tiles, so the tiles running together on one XCD share
// their A and B panels in its L2.
// The 16-bit modes first pack Z once into MFMA fragment order (one 1 KB
// fragment per 16 rows x 32 columns: lane l holds rows 8(l/32)..8(l/32)+7 of
// column l%32), so the Gram kernel streams contiguous fragments through LDS
// with no per-tile conversion. The pack kernel also forms Z^T y in FP64
// (per-chunk partials summed in a fixed order); the FP32 mode runs it for
// Z^T y only and stages row-major Z slabs directly.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "sorf_internal.h"

namespace sorf {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

// Modes 0..5 are the public precisions. The split mode (FP64 output) runs two
// internal ones: kSplitHead, the integer head products on int8 matrix cores,
// and kSplitCross, the three fp16 products that involve the tail.
enum GramMode { kFP32 = 0, kBF16 = 1, kFP16 = 2, kBF16HiLo = 3, kFP16HiLo = 4, kFP32Kahan = 5,
                kSplitCross = 6, kSplitHead = 7 };

constexpr int KB = 16;                 // rows per fragment / FP32 stage
constexpr int TM = 256, TN = 128;      // workgroup tile
constexpr int kFlushRows = 256;        // rows per fresh MFMA accumulator
constexpr int kPackSlabs = 64;         // 16-row slabs per pack workgroup (Z^T y chunk)
// FP32 ring kernel (both FP32 modes): half tiles, two 8-wave workgroups per
// CU, 32-row stages
constexpr int kFP32Waves = 8;
constexpr bool kFP32Half = true;
constexpr int kFP32StageRows = 32;

__host__ __device__ constexpr bool is_hilo(int mode) {
  return mode == kBF16HiLo || mode == kFP16HiLo || mode == kSplitCross;
}
__host__ __device__ constexpr bool is_bf(int mode) { return mode == kBF16 || mode == kBF16HiLo; }

// round-to-nearest-even conversions, returned as raw 16-bit patterns
__device__ __forceinline__ unsigned short to_bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(r >> 16);
}
__device__ __forceinline__ float from_bf16_bits(unsigned short h) {
  return __uint_as_float(uint32_t(h) << 16);
}

template <int MODE>
__device__ __forceinline__ void split(float z, unsigned short& hi, unsigned short& lo) {
  if constexpr (is_bf(MODE)) {
    hi = to_bf16_bits(z);
    lo = to_bf16_bits(z - from_bf16_bits(hi));
  } else {
    const _Float16 h = (_Float16)z;
    const _Float16 l = (_Float16)(z - (float)h);
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, l);
  }
}

template <int MODE>
__device__ __forceinline__ f32x16 mma16(u16x8 a, u16x8 b, f32x16 c) {
  if constexpr (is_bf(MODE))
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

__host__ __device__ inline int64_t gram_tiles(int64_t D, int64_t& nI, int64_t& nJ) {
  nI = (D + TM - 1) / TM;
  nJ = (D + TN - 1) / TN;
  const int64_t last = 2 * nI < nJ ? 2 * nI : nJ;
  return (nI - 1) * nI + last;
}

// Workgroups are dealt round-robin to the 8 XCDs, and each XCD runs 32 of
// them at a time (one per compute unit). Block b therefore gets XCD b % 8
// and local slot q = b / 8; 32 consecutive slots of one XCD form a
// super-tile of 4 x 8 tiles (1024 x 1024 entries of G), so the tiles that
// run together on one XCD share 4 A panels and 8 B panels in its L2.
// Super-tiles strictly below the diagonal come first, the lighter diagonal
// ones last. Returns false for slots whose tile is outside the lower
// triangle or the matrix.
constexpr int SR_T = 4, SC_T = 8;   // tiles per super-tile (rows, columns)

__host__ __device__ inline int64_t gram_super_tiles(int64_t D) {
  const int64_t nS = (D + SR_T * TM - 1) / (SR_T * TM);
  return nS * (nS + 1) / 2;
}

__device__ __forceinline__ bool super_tile(int64_t b, int64_t D, int64_t nI, int64_t nJ,
                                           int64_t& I, int64_t& J) {
  const int64_t nS = (D + SR_T * TM - 1) / (SR_T * TM);
  const int64_t q = b / 8;
  const int64_t G = (q / (SR_T * SC_T)) * 8 + b % 8;
  const int pos = int(q % (SR_T * SC_T));
  const int64_t off = nS * (nS - 1) / 2;
  int64_t R, C;
  if (G < off) {
    int64_t r = int64_t((1.0 + std::sqrt(1.0 + 8.0 * double(G))) * 0.5);
    while (r * (r - 1) / 2 > G) --r;
    while ((r + 1) * r / 2 <= G) ++r;
    R = r;
    C = G - r * (r - 1) / 2;
  } else if (G < off + nS) {
    R = C = G - off;
  } else {
    return false;
  }
  I = R * SR_T + pos / SC_T;
  J = C * SC_T + pos % SC_T;
  return I < nI && J < nJ && J * TN <= I * TM + TM - 1;
}

// Row slices of the 256 x 128 tile kernels. One workgroup fills a compute
// unit, so a launch of n_tiles tiles runs in ceil(n_tiles / 256) rounds; at
// D = 8192 (1056 tiles) the fifth round holds 32 tiles and a fifth of the
// launch leaves most of the chip idle. Splitting the rows of every tile into
// n_split slices makes n_split * n_tiles shorter items (8448 at D = 8192, 33
// whole rounds). Slice sp covers rows [sp * rows_per, (sp + 1) * rows_per) and
// is dealt blocks [sp * grid1, (sp + 1) * grid1), each slice in the super-tile
// order, so the slices run one after another and neighbouring tiles of one
// slice share their panels in an XCD's L2. With n_split > 1 each item writes
// its 256 x 128 sum to a partial tile and gram_slices_combine_kernel adds the
// n_split partials of every entry into G in slice order (deterministic).
struct SlicePlan {
  int32_t n_split;    // row slices per tile (1: items add into G themselves)
  int64_t rows_per;   // rows per slice, a multiple of the flush block
  int64_t grid1;      // blocks per slice
};

// Index of lower-triangle tile (I, J) of 256 x 128 tiles: row I holds
// J = 0 .. 2 I + 1, so the rows before it hold I (I + 1) tiles.
__host__ __device__ inline int64_t tile_index(int64_t I, int64_t J) { return I * (I + 1) + J; }

// ------------------------------------------------------------------- packing
// Fragment (ks, cb) -> u16x8 index ((ks * ncb + cb) * 64 + lane).
// One workgroup per 128 columns (4 column blocks) x kPackSlabs slabs. Row
// tiles of 4 slabs x 128 columns are read with coalesced 16-byte loads (the
// next tile's loads are issued before the current one is processed), staged
// in LDS and re-read by column: wave w forms the fragments of slab w, lane l
// holding column 32 cb + l % 32 and rows 8 (l / 32) .. + 7 of each block. Z^T y
// is summed per lane in FP64 and combined over the 8 partial sums of a column
// in a fixed order.
constexpr int kPackLds = 128 + 4;   // LDS row stride (floats): conflict-free column reads

template <int MODE>
__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ Z, int64_t M,
                                                   int32_t D, int64_t n_slabs, int32_t ncb,
                                                   float zscale, u16x8* __restrict__ hi,
                                                   u16x8* __restrict__ lo,
                                                   const float* __restrict__ y,
                                                   double* __restrict__ zpart) {
  __shared__ float tile[64][kPackLds];
  __shared__ double red[8][128];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int64_t c0 = int64_t(blockIdx.x) * 128;
  const int64_t ks0 = int64_t(blockIdx.y) * kPackSlabs;
  const int64_t ks1 = ks0 + kPackSlabs < n_slabs ? ks0 + kPackSlabs : n_slabs;
  const bool vec = (D % 4 == 0) && (c0 + 128 <= D);
  // loader role: float4 f = tid + 256 i of the tile: row tid / 32 + 8 i, columns 4 (tid % 32)
  const int lrow = tid >> 5, lcol = (tid & 31) * 4;
  float4 buf[8];
  auto load = [&](int64_t ks) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t r = ks * KB + lrow + 8 * i;
      const int64_t rc = r < M ? r : M - 1;
      const float* src = Z + rc * D + c0 + lcol;
      float4 v;
      if (vec) {
        v = *reinterpret_cast<const float4*>(src);
      } else {
        v.x = c0 + lcol + 0 < D ? src[0] : 0.0f;
        v.y = c0 + lcol + 1 < D ? src[1] : 0.0f;
        v.z = c0 + lcol + 2 < D ? src[2] : 0.0f;
        v.w = c0 + lcol + 3 < D ? src[3] : 0.0f;
      }
      buf[i] = r < M ? v : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  };
  double zacc[4] = {0.0, 0.0, 0.0, 0.0};
  if (ks0 < ks1) load(ks0);
  for (int64_t ks = ks0; ks < ks1; ks += 4) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
      *reinterpret_cast<float4*>(&tile[lrow + 8 * i][lcol]) = buf[i];
    __syncthreads();
    if (ks + 4 < ks1) load(ks + 4);
    const int64_t slab = ks + wv;
    if (slab < ks1) {
      const int rr = 16 * wv + 8 * (lane >> 5);
      float yv[8];
      if (y != nullptr) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int64_t r = slab * KB + 8 * (lane >> 5) + j;
          const float t = y[r < M ? r : M - 1];
          yv[j] = r < M ? t : 0.0f;
        }
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int c = cb * 32 + (lane & 31);
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = tile[rr + j][c];
        if (y != nullptr) {
#pragma unroll
          for (int j = 0; j < 8; ++j) zacc[cb] += double(v[j]) * double(yv[j]);
        }
        if constexpr (MODE != kFP32) {
          u16x8 h, l;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            unsigned short a, b;
            split<MODE>(v[j] * zscale, a, b);
            h[j] = a;
            l[j] = b;
          }
          const int64_t idx = (slab * ncb + blockIdx.x * 4 + cb) * 64 + lane;
          hi[idx] = h;
          if constexpr (is_hilo(MODE)) lo[idx] = l;
        }
      }
    }
    __syncthreads();
  }
  if (y != nullptr) {
    // partial of column 32 cb + l % 32 from wave w, half l / 32 -> red[2 w + half][col]
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) red[2 * wv + (lane >> 5)][cb * 32 + (lane & 31)] = zacc[cb];
    __syncthreads();
    if (tid < 128 && c0 + tid < D) {
      double t = 0.0;
#pragma unroll
      for (int p = 0; p < 8; ++p) t += red[p][tid];
      zpart[int64_t(blockIdx.y) * D + c0 + tid] = t;
    }
  }
}

template <typename T>
__global__ void zty_finalize_kernel(const double* __restrict__ zpart, int64_t chunks, int32_t D,
                                    T* __restrict__ Zty) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= D) return;
  double t = 0.0;
  for (int64_t k = 0; k < chunks; ++k) t += zpart[k * D + c];
  Zty[c] += T(t);
}

// ------------------------------------------------------- split mode (FP64 G)
// Every column f of Z gets a power-of-two scale 2^e_f, e_f the largest
// exponent with max_m |Z[m][f]| 2^e_f <= 127. The scaled value w = z 2^e_f
// (exact) is split into an integer head h = rint(w), |h| <= 127, and a tail
// t = w - h (exact, |t| <= 1/2) rounded to fp16. The Gram of h + t is
//   h^T h  (int8 products, int32 sums: exact while rows * 127^2 < 2^31)
// + h^T t + t^T h + t^T t  (fp16 products, FP32 block sums),
// each entry scaled by 2^-(e_i + e_j) into an FP64 G. Only the tail's fp16
// rounding (at most 2^-13 2^-e_f, below 2^-19 of the column's maximum) and the
// FP32 sums of the tail products (2^-7 of G in size) are inexact.

// Column maxima of |Z| over row chunks (a wave reads consecutive columns of
// one row); partial maxima [chunk][D].
__global__ __launch_bounds__(256) void colmax_kernel(const float* __restrict__ Z, int64_t M,
                                                     int32_t D, int64_t rows_per,
                                                     float* __restrict__ part) {
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= D) return;
  const int64_t r0 = int64_t(blockIdx.y) * rows_per;
  const int64_t r1 = r0 + rows_per < M ? r0 + rows_per : M;
  float m = 0.0f;
  for (int64_t r = r0; r < r1; ++r) m = fmaxf(m, fabsf(Z[r * D + c]));
  part[int64_t(blockIdx.y) * D + c] = m;
}

// e_f from the chunk maxima: with max = mant 2^k (1 <= mant < 2), the largest
// e with max 2^e <= 127 is 6 - k when mant * 64 <= 127, else 5 - k. An all-zero
// column gets e = 0.
__global__ __launch_bounds__(256) void split_exps_kernel(const float* __restrict__ part,
                                                         int64_t chunks, int32_t D,
                                                         int32_t* __restrict__ exps) {
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= D) return;
  float m = 0.0f;
  for (int64_t k = 0; k < chunks; ++k) m = fmaxf(m, part[k * D + c]);
  int e = 0;
  if (m > 0.0f) {
    const int k = ilogbf(m);
    e = ldexpf(m, 6 - k) <= 127.0f ? 6 - k : 5 - k;
  }
  exps[c] = e;
}

// pack_kernel's tiling for the split mode: per 16-row slab and 32-column block
// the fp16 head and tail fragments (lane l: column l % 32, rows 8 (l / 32)
// .. + 7), and the int8 head in 32-row fragments of 16 bytes per lane whose
// bytes 0..7 are the lane's rows of the first slab and bytes 8..15 those of the
// second (the same rows as its two fp16 fragments; A and B use one layout, so
// the order of the K index within a fragment is free). Z^T y in FP64 partials.
__global__ __launch_bounds__(256) void pack_split_kernel(
    const float* __restrict__ Z, int64_t M, int32_t D, int64_t n_slabs, int32_t ncb,
    const int32_t* __restrict__ exps, u16x8* __restrict__ hi, u16x8* __restrict__ lo,
    uint2* __restrict__ hi8, const float* __restrict__ y, double* __restrict__ zpart) {
  __shared__ float tile[64][kPackLds];
  __shared__ double red[8][128];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int64_t c0 = int64_t(blockIdx.x) * 128;
  const int64_t ks0 = int64_t(blockIdx.y) * kPackSlabs;
  const int64_t ks1 = ks0 + kPackSlabs < n_slabs ? ks0 + kPackSlabs : n_slabs;
  const bool vec = (D % 4 == 0) && (c0 + 128 <= D);
  const int lrow = tid >> 5, lcol = (tid & 31) * 4;
  int ex[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int64_t c = c0 + cb * 32 + (lane & 31);
    ex[cb] = c < D ? exps[c] : 0;
  }
  float4 buf[8];
  auto load = [&](int64_t ks) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t r = ks * KB + lrow + 8 * i;
      const int64_t rc = r < M ? r : M - 1;
      const float* src = Z + rc * D + c0 + lcol;
      float4 v;
      if (vec) {
        v = *reinterpret_cast<const float4*>(src);
      } else {
        v.x = c0 + lcol + 0 < D ? src[0] : 0.0f;
        v.y = c0 + lcol + 1 < D ? src[1] : 0.0f;
        v.z = c0 + lcol + 2 < D ? src[2] : 0.0f;
        v.w = c0 + lcol + 3 < D ? src[3] : 0.0f;
      }
      buf[i] = r < M ? v : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  };
  double zacc[4] = {0.0, 0.0, 0.0, 0.0};
  if (ks0 < ks1) load(ks0);
  for (int64_t ks = ks0; ks < ks1; ks += 4) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
      *reinterpret_cast<float4*>(&tile[lrow + 8 * i][lcol]) = buf[i];
    __syncthreads();
    if (ks + 4 < ks1) load(ks + 4);
    const int64_t slab = ks + wv;
    if (slab < ks1) {
      const int rr = 16 * wv + 8 * (lane >> 5);
      float yv[8];
      if (y != nullptr) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int64_t r = slab * KB + 8 * (lane >> 5) + j;
          const float t = y[r < M ? r : M - 1];
          yv[j] = r < M ? t : 0.0f;
        }
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int c = cb * 32 + (lane & 31);
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = tile[rr + j][c];
        if (y != nullptr) {
#pragma unroll
          for (int j = 0; j < 8; ++j) zacc[cb] += double(v[j]) * double(yv[j]);
        }
        u16x8 h, l;
        uint32_t b8[2] = {0u, 0u};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float w = ldexpf(v[j], ex[cb]);
          const float hv = rintf(w);
          h[j] = __builtin_bit_cast(unsigned short, (_Float16)hv);
          l[j] = __builtin_bit_cast(unsigned short, (_Float16)(w - hv));
          b8[j >> 2] |= (uint32_t(int32_t(hv)) & 0xFFu) << (8 * (j & 3));
        }
        const int64_t cbg = int64_t(blockIdx.x) * 4 + cb;
        const int64_t idx = (slab * ncb + cbg) * 64 + lane;
        hi[idx] = h;
        lo[idx] = l;
        hi8[(((slab >> 1) * ncb + cbg) * 64 + lane) * 2 + (slab & 1)] = make_uint2(b8[0], b8[1]);
      }
    }
    __syncthreads();
  }
  if (y != nullptr) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) red[2 * wv + (lane >> 5)][cb * 32 + (lane & 31)] = zacc[cb];
    __syncthreads();
    if (tid < 128 && c0 + tid < D) {
      double t = 0.0;
#pragma unroll
      for (int p = 0; p < 8; ++p) t += red[p][tid];
      zpart[int64_t(blockIdx.y) * D + c0 + tid] = t;
    }
  }
}

// Direct global -> LDS copies (16 bytes per lane; a wave fills 1 KB at a
// wave-uniform LDS address, lane i at byte 16 i). Their completion is tracked
// by vmcnt only, so the kernels below wait on vmcnt themselves before the
// barrier that publishes a stage; loads return in issue order.
__device__ __forceinline__ void dma16(const void* g, void* lds) {
  __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
// Wait until at most `ahead` stages of PW copies each are still in flight.
template <int PW>
__device__ __forceinline__ void wait_stage(int64_t ahead) {
  if (ahead >= 3) wait_vm<3 * PW>();
  else if (ahead == 2) wait_vm<2 * PW>();
  else if (ahead == 1) wait_vm<PW>();
  else wait_vm<0>();
}
__device__ __forceinline__ void stage_barrier() {
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// ------------------------------------------------------ 16-bit modes (packed)
// Stage = 2 slabs (32 rows): 16 A fragments (rows 256 I .. +255 of G) and 8 B
// fragments per part, copied into a ring of NS stages; wave w copies the
// fragments w, w + 8, ... of each part. Eight waves (4 x 2), two per SIMD,
// each owning 64 x 64 of the 256 x 128 tile: while one wave of a SIMD waits
// on a barrier, a copy or LDS, the other keeps the matrix core busy.
constexpr int kPackedWaves = 8;
template <int MODE>
__global__ __launch_bounds__(64 * kPackedWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gram_packed_kernel(const u16x8* __restrict__ hi, const u16x8* __restrict__ lo,
                        int64_t n_slabs, int32_t ncb, int32_t D, int64_t n_tiles, int64_t nI,
                        int64_t nJ, float gscale, float* __restrict__ G,
                        double* __restrict__ G64, const int32_t* __restrict__ exps) {
  constexpr bool HILO = is_hilo(MODE);
  constexpr bool CROSS = MODE == kSplitCross;   // tail products only, FP64 output
  constexpr int NP = HILO ? 2 : 1;            // parts per operand
  constexpr int AF = 2 * (TM / 32);           // A fragments per stage
  constexpr int BF = 2 * (TN / 32);           // B fragments per stage
  constexpr int NF = AF + BF;
  constexpr int NW = kPackedWaves;
  constexpr int WR = TM / (NW / 2), WC = TN / 2;   // wave tile: 64 x 64
  constexpr int BA = WR / 32, BB = WC / 32;        // 32 x 32 blocks per wave
  constexpr int FW = NF / NW;                 // fragments per wave per part
  constexpr int PW = NP * FW;                 // copies per wave per stage
  constexpr int NS = HILO ? 3 : 4;            // ring depth (stages)
  constexpr int KC = kFlushRows / (2 * KB);   // stages per flush
  __shared__ u16x8 ring[NS][NP][NF][64];

  int64_t I, J;
  if (!super_tile(blockIdx.x, D, nI, nJ, I, J)) return;
  (void)n_tiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv >> 1, wx = wv & 1;
  const bool active = I * TM + wy * WR + WR - 1 >= J * TN + wx * WC;

  int64_t src[FW];
#pragma unroll
  for (int c = 0; c < FW; ++c) {
    const int f = wv + NW * c;
    const int slab = f < AF ? f / (TM / 32) : (f - AF) / (TN / 32);
    const int64_t cbf = f < AF ? I * (TM / 32) + f % (TM / 32) : J * (TN / 32) + (f - AF) % (TN / 32);
    src[c] = (int64_t(slab) * ncb + cbf) * 64 + lane;
  }
  const int64_t stage_stride = int64_t(2) * ncb * 64;
  const int64_t n_st = n_slabs / 2;
  auto issue = [&](int64_t st, int slot) {
    const int64_t off = st * stage_stride;
#pragma unroll
    for (int c = 0; c < FW; ++c) {
      dma16(hi + src[c] + off, &ring[slot][0][wv + NW * c][0]);
      if constexpr (HILO) dma16(lo + src[c] + off, &ring[slot][NP - 1][wv + NW * c][0]);
    }
  };

  f32x16 P[BA][BB], S[BA][BB];
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        P[a][b][r] = 0.0f;
        S[a][b][r] = 0.0f;
      }

  // Groups of KC stages accumulate in P; P is added into S after each group.
  // Waves whose block lies above the diagonal compute too (their result is
  // dropped): keeping the loop free of per-wave branches keeps P in the
  // accumulation registers. Software pipeline over half-stages as in the
  // single-product kernel: the fragments of one half-stage are read from LDS
  // while the products of the previous half-stage run; all NS slots are
  // filled up front and the slot of stage s takes stage s + NS after the
  // barrier that publishes stage s + 1.
  u16x8 ah0[BA], al0[BA], bh0[BB], bl0[BB], ah1[BA], al1[BA], bh1[BB], bl1[BB];
  auto read_half = [&](int sl, int kk, u16x8 (&ah)[BA], u16x8 (&al)[BA], u16x8 (&bh)[BB],
                       u16x8 (&bl)[BB]) {
#pragma unroll
    for (int a = 0; a < BA; ++a) {
      ah[a] = ring[sl][0][kk * (TM / 32) + wy * BA + a][lane];
      if constexpr (HILO) al[a] = ring[sl][NP - 1][kk * (TM / 32) + wy * BA + a][lane];
    }
#pragma unroll
    for (int b = 0; b < BB; ++b) {
      bh[b] = ring[sl][0][AF + kk * (TN / 32) + wx * BB + b][lane];
      if constexpr (HILO) bl[b] = ring[sl][NP - 1][AF + kk * (TN / 32) + wx * BB + b][lane];
    }
  };
  auto mma_half = [&](const u16x8 (&ah)[BA], const u16x8 (&al)[BA], const u16x8 (&bh)[BB],
                      const u16x8 (&bl)[BB]) {
#pragma unroll
    for (int a = 0; a < BA; ++a)
#pragma unroll
      for (int b = 0; b < BB; ++b) {
        if constexpr (!CROSS) P[a][b] = mma16<MODE>(ah[a], bh[b], P[a][b]);
        if constexpr (HILO) {
          P[a][b] = mma16<MODE>(ah[a], bl[b], P[a][b]);
          P[a][b] = mma16<MODE>(al[a], bh[b], P[a][b]);
          P[a][b] = mma16<MODE>(al[a], bl[b], P[a][b]);
        }
      }
  };
  // the next half-stage's LDS reads interleaved with the first products
  auto interleave = [] {
    constexpr int NR = (BA + BB) * NP, NM = BA * BB * (CROSS ? 3 : HILO ? 4 : 1);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, NM - NR, 0);
  };
  auto flush = [&] {
#pragma unroll
    for (int a = 0; a < BA; ++a)
#pragma unroll
      for (int b = 0; b < BB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          S[a][b][r] += P[a][b][r];
          P[a][b][r] = 0.0f;
        }
  };

#pragma unroll
  for (int j = 0; j < NS; ++j)
    if (j < n_st) issue(j, j);
  if (n_st > 0) {
    wait_stage<PW>(n_st - 1 < NS - 1 ? n_st - 1 : NS - 1);
    stage_barrier();
    read_half(0, 0, ah0, al0, bh0, bl0);
  }
  int64_t s = 0;
  int slot = 0;
  while (s + 1 < n_st) {
    const int64_t g_end = (s / KC + 1) * KC < n_st - 1 ? (s / KC + 1) * KC : n_st - 1;
    for (; s < g_end; ++s) {
      const int nslot = slot + 1 == NS ? 0 : slot + 1;
      read_half(slot, 1, ah1, al1, bh1, bl1);
      mma_half(ah0, al0, bh0, bl0);
      interleave();
      const int64_t ahead = n_st - 2 - s;
      wait_stage<PW>(ahead < NS - 2 ? ahead : NS - 2);
      // this wave's reads of stage s have landed before its slot is reused
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      stage_barrier();
      if (s + NS < n_st) issue(s + NS, slot);
      read_half(nslot, 0, ah0, al0, bh0, bl0);
      mma_half(ah1, al1, bh1, bl1);
      interleave();
      slot = nslot;
    }
    if (s % KC == 0) flush();
  }
  if (n_st > 0) {
    read_half(slot, 1, ah1, al1, bh1, bl1);
    mma_half(ah0, al0, bh0, bl0);
    mma_half(ah1, al1, bh1, bl1);
    flush();
  }

  if (!active) return;
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gi = I * TM + wy * WR + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t gj = J * TN + wx * WC + b * 32 + (lane & 31);
        if (gi < D && gj < D && gi >= gj) {
          if constexpr (CROSS)
            G64[gi * D + gj] += ldexp(double(S[a][b][r]), -(exps[gi] + exps[gj]));
          else
            G[gi * D + gj] += S[a][b][r] * gscale;
        }
      }
}

// ------------------------------------------ 16-bit single-product modes
// One workgroup per 256 x 256 square tile of the lower triangle. bf16/fp16:
// 16 waves (4 x 4, four per SIMD), each owning 64 x 64 (2 x 2 blocks of
// 32 x 32, 128 registers), so that while one wave of a SIMD waits on a
// barrier or a copy three others can keep the matrix core busy (1.88 against
// 1.93 ms at 20,000 x 8192 and 29.2 against 30.5 ms at 100,000 x 16384 with
// 8 waves of 128 x 64). The split mode's int8 head keeps 8 waves of 128 x 64
// (two per SIMD): with 16 its FP64 epilogue would spill 32 registers.
// Ring: 16-bit stages of 4 slabs (64 rows, 64 KB), 2 deep; the int8 head's
// stages of 2 slabs (64 rows, 32 KB), 5 deep (64-row 16-bit stages took
// 1.85-1.88 against 1.88-1.90 ms with 32-row stages 5 deep at 20,000 x 8192).
// A launch covers at most kX1LaunchStages stages (8192 rows) and adds its
// tiles to G, so the matrix-core accumulators never run over more rows than
// that: a single accumulator over a long row range drifts enough to make
// G + lambda I indefinite (100,000 rows, lambda = 1e-8); G itself is summed
// in FP32 with round-to-nearest.
//
// Scheduling: with one 160 KB workgroup per CU, the tiles run in rounds of
// kX1Slots. The first n_whole tiles (whole rounds) are computed over all rows
// and added to G directly; each remaining tail tile is split into n_split
// slices of the rows so that the last round is filled with short items.
// Slices write partial tiles and gram_combine_kernel adds them to G in a
// fixed order, so results stay deterministic. Every XCD receives a
// contiguous run of whole tiles (neighbouring tiles share operand blocks in
// its L2) followed by a contiguous run of slices.
constexpr int TX = 256;        // square tile of the single-product kernel
constexpr int kX1Slots = 256;  // concurrent workgroups: one per CU of the chip
// waves per workgroup of the single-product kernel, by mode
__host__ __device__ constexpr int x1_waves(int mode) { return mode == kSplitHead ? 8 : 16; }
// fragment slabs per ring stage: 16-bit slabs hold 16 rows, int8 head slabs 32
__host__ __device__ constexpr int x1_stage_slabs(int mode) { return mode == kSplitHead ? 2 : 4; }
// 8192 rows per launch: stages of x1_stage_slabs(kBF16) 16-row slabs
constexpr int64_t kX1LaunchStages = 8192 / (KB * x1_stage_slabs(kBF16));

__host__ __device__ inline int64_t x1_tiles(int64_t D) {
  const int64_t n = (D + TX - 1) / TX;
  return n * (n + 1) / 2;
}

// Order of the tiles (I, J), J <= I, of the n x n tile grid: bands of 4 tile
// rows; in band b first the 8-column blocks that lie wholly below the band's
// diagonal (b / 2 of them, 32 tiles each, row-major inside), then the band's
// remaining tiles row by row; the last band, when n is not a multiple of 4,
// row by row. Consecutive tiles, which run together on one XCD, then form 4 x 8
// blocks that read 4 + 8 column panels of Z through that XCD's L2 (row-major
// order: a run of 32 tiles of one or two rows reads about 33).
// Band b holds 16 b + 10 tiles, so 8 b^2 + 2 b tiles precede it.
__device__ __forceinline__ void x1_tile_of(int64_t t, int64_t n, int64_t& I, int64_t& J) {
  const int64_t nfull = n / 4;
  const int64_t base = 8 * nfull * nfull + 2 * nfull;
  int64_t u, r, c0;
  if (t >= base) {   // last, partial band
    u = t - base;
    r = 4 * nfull;
    c0 = 0;
  } else {
    int64_t b = int64_t((std::sqrt(4.0 + 32.0 * double(t)) - 2.0) / 16.0);
    while (8 * b * b + 2 * b > t) --b;
    while (8 * (b + 1) * (b + 1) + 2 * (b + 1) <= t) ++b;
    u = t - (8 * b * b + 2 * b);
    const int64_t nf = b / 2;   // whole 8-column blocks below the band's diagonal
    if (u < 32 * nf) {
      I = 4 * b + (u % 32) / 8;
      J = 8 * (u / 32) + u % 8;
      return;
    }
    u -= 32 * nf;
    r = 4 * b;
    c0 = 8 * nf;
  }
  while (u >= r - c0 + 1) {   // rows of the remaining region, columns c0 .. r
    u -= r - c0 + 1;
    ++r;
  }
  I = r;
  J = c0 + u;
}

struct X1Plan {
  int64_t n_tiles;   // tiles of the lower triangle
  int64_t n_whole;   // tiles computed over all rows
  int32_t n_split;   // row slices per tail tile (1: no tail)
};

// Items of XCD x: its whole tiles, then its slices (both contiguous runs).
__host__ __device__ inline void x1_xcd_items(const X1Plan& p, int x, int64_t& w0, int64_t& nw,
                                             int64_t& q0, int64_t& nq) {
  const int64_t n_pieces = (p.n_tiles - p.n_whole) * p.n_split;
  w0 = p.n_whole * x / 8;
  nw = p.n_whole * (x + 1) / 8 - w0;
  q0 = n_pieces * x / 8;
  nq = n_pieces * (x + 1) / 8 - q0;
}

template <int MODE>
__global__ __launch_bounds__(64 * x1_waves(MODE))
__attribute__((amdgpu_waves_per_eu(x1_waves(MODE) / 4, x1_waves(MODE) / 4)))
void gram_x1_kernel(const u16x8* __restrict__ hi, int64_t st_begin, int64_t st_count,
                    int32_t ncb, int32_t D, X1Plan plan, float gscale, float* __restrict__ G,
                    float* __restrict__ part, double* __restrict__ G64,
                    const int32_t* __restrict__ exps) {
  // kSplitHead: 16-byte lanes hold 16 int8 head values of 32 rows (one
  // v_mfma_i32_32x32x32_i8 per 32 x 32 block and fragment row); the int32
  // sums are exact, and the result goes to the FP64 G scaled by 2^-(e_i + e_j)
  constexpr bool HEAD = MODE == kSplitHead;
  using Acc = std::conditional_t<HEAD, i32x16, f32x16>;
  constexpr int SL = x1_stage_slabs(MODE);   // fragment slabs per stage
  constexpr int AF = SL * (TX / 32);  // A fragments per stage
  constexpr int NF = 2 * AF;          // A and B
  constexpr int NW = x1_waves(MODE);
  constexpr int WR = TX / (NW / 4);   // wave rows: NW / 4 x 4 waves of WR x 64
  constexpr int BA = WR / 32, BB = 2;  // 32 x 32 blocks per wave
  constexpr int FW = NF / NW;         // copies per wave per stage
  static_assert(FW * NW == NF, "copies per stage");
  constexpr int NS = 160 / NF;        // ring depth: the whole LDS of a CU (NF KB per stage)
  __shared__ u16x8 ring[NS][NF][64];

  int64_t w0, nw, q0, nq;
  x1_xcd_items(plan, int(blockIdx.x % 8), w0, nw, q0, nq);
  const int64_t k = blockIdx.x / 8;
  if (k >= nw + nq) return;
  const int64_t n_tail = plan.n_tiles - plan.n_whole;
  const bool whole = k < nw;
  // slices are split-major: concurrent slices of one XCD share their rows
  const int64_t piece = whole ? 0 : q0 + (k - nw);
  const int64_t t = whole ? w0 + k : plan.n_whole + piece % n_tail;
  const int sp = whole ? 0 : int(piece / n_tail);
  const int n_split = whole ? 1 : plan.n_split;
  int64_t I, J;
  x1_tile_of(t, (D + TX - 1) / TX, I, J);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv >> 2, wx = wv & 3;   // rows [WR wy, +WR), columns [64 wx, +64)
  const bool active = I * TX + wy * WR + WR - 1 >= J * TX + wx * 64;

  // the slice of stages this item accumulates
  const int64_t s0 = st_begin + st_count * sp / n_split;
  const int64_t n_st = st_begin + st_count * (sp + 1) / n_split - s0;

  int64_t src[FW];
#pragma unroll
  for (int c = 0; c < FW; ++c) {
    const int f = wv + NW * c;
    const int slab = (f % AF) / (TX / 32);
    const int64_t cbf = (f < AF ? I : J) * (TX / 32) + (f % AF) % (TX / 32);
    src[c] = ((SL * s0 + slab) * int64_t(ncb) + cbf) * 64 + lane;
  }
  const int64_t stage_stride = int64_t(SL) * ncb * 64;
  auto issue = [&](int64_t st, int slot) {
    const int64_t off = st * stage_stride;
#pragma unroll
    for (int c = 0; c < FW; ++c) dma16(hi + src[c] + off, &ring[slot][wv + NW * c][0]);
  };

  Acc P[BA][BB];
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) P[a][b][r] = 0;

  // Software pipeline over the SL slabs of a stage: the fragments of one slab
  // are read from LDS while the MFMAs of the previous slab run. All NS slots
  // are filled up front; after the barrier that publishes stage st + 1 every
  // wave has read all of stage st, so its slot takes stage st + NS.
  static_assert(SL % 2 == 0, "slabs per stage");
  u16x8 a0[BA], b0[BB], a1[BA], b1[BB];
  auto read_half = [&](int slot, int kk, u16x8 (&af)[BA], u16x8 (&bf)[BB]) {
#pragma unroll
    for (int q = 0; q < BA; ++q) af[q] = ring[slot][kk * (TX / 32) + wy * BA + q][lane];
#pragma unroll
    for (int q = 0; q < BB; ++q) bf[q] = ring[slot][AF + kk * (TX / 32) + wx * BB + q][lane];
  };
  auto mma_half = [&](const u16x8 (&af)[BA], const u16x8 (&bf)[BB]) {
#pragma unroll
    for (int a = 0; a < BA; ++a)
#pragma unroll
      for (int b = 0; b < BB; ++b) {
        if constexpr (HEAD)
          P[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(i32x4, af[a]),
                                                          __builtin_bit_cast(i32x4, bf[b]),
                                                          P[a][b], 0, 0, 0);
        else
          P[a][b] = mma16<MODE>(af[a], bf[b], P[a][b]);
      }
  };
  // the next slab's BA + BB LDS reads interleaved with the first MFMAs
  auto interleave = [] {
#pragma unroll
    for (int i = 0; i < BA + BB; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    if constexpr (BA * BB > BA + BB)
      __builtin_amdgcn_sched_group_barrier(0x008, BA * BB - (BA + BB), 0);
  };

#pragma unroll
  for (int j = 0; j < NS; ++j)
    if (j < n_st) issue(j, j);
  if (n_st > 0) {
    wait_stage<FW>(n_st - 1 < NS - 1 ? n_st - 1 : NS - 1);
    stage_barrier();
    read_half(0, 0, a0, b0);
  }
  // slabs 0 .. SL - 2 of a stage whose slab 0 sits in a0/b0; slab SL - 1 is
  // left in a1/b1
  auto inner = [&](int sl) {
#pragma unroll
    for (int j = 0; j + 2 < SL; j += 2) {
      read_half(sl, j + 1, a1, b1);
      mma_half(a0, b0);
      interleave();
      read_half(sl, j + 2, a0, b0);
      mma_half(a1, b1);
      interleave();
    }
    read_half(sl, SL - 1, a1, b1);
  };
  int slot = 0;
  for (int64_t st = 0; st + 1 < n_st; ++st) {
    const int nslot = slot + 1 == NS ? 0 : slot + 1;
    inner(slot);
    mma_half(a0, b0);
    interleave();
    const int64_t ahead = n_st - 2 - st;
    wait_stage<FW>(ahead < NS - 2 ? ahead : NS - 2);
    // this wave's reads of stage st have landed before its slot is reused
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    stage_barrier();
    if (st + NS < n_st) issue(st + NS, slot);
    read_half(nslot, 0, a0, b0);
    mma_half(a1, b1);
    interleave();
    slot = nslot;
  }
  if (n_st > 0) {
    inner(slot);
    mma_half(a0, b0);
    mma_half(a1, b1);
  }

  if (!active) return;
  if (whole) {
#pragma unroll
    for (int a = 0; a < BA; ++a)
#pragma unroll
      for (int b = 0; b < BB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t gi = I * TX + wy * WR + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int64_t gj = J * TX + wx * 64 + b * 32 + (lane & 31);
          if (gi < D && gj < D && gi >= gj) {
            if constexpr (HEAD)
              G64[gi * D + gj] += ldexp(double(P[a][b][r]), -(exps[gi] + exps[gj]));
            else
              G[gi * D + gj] += P[a][b][r] * gscale;
          }
        }
    return;
  }
  using Part = std::conditional_t<HEAD, int32_t, float>;
  Part* out = reinterpret_cast<Part*>(part) + (int64_t(sp) * n_tail + (t - plan.n_whole)) * TX * TX;
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = wy * WR + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = wx * 64 + b * 32 + (lane & 31);
        out[i * TX + j] = P[a][b][r];
      }
}

// G += sum over the slices of a tail tile's partials, slice 0 first. One
// workgroup per 4 rows of a tile, 4 columns per thread. Partial entries of
// waves above the diagonal are never written; they are read but discarded.
__global__ __launch_bounds__(256) void gram_combine_kernel(const float* __restrict__ part,
                                                          X1Plan plan, int32_t D, float gscale,
                                                          float* __restrict__ G) {
  const int64_t n_tail = plan.n_tiles - plan.n_whole;
  const int64_t tt = blockIdx.x;
  int64_t I, J;
  x1_tile_of(plan.n_whole + tt, (D + TX - 1) / TX, I, J);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int j = (threadIdx.x & 63) * 4;
  const int64_t gi = I * TX + i;
  if (gi >= D) return;
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int sp = 0; sp < plan.n_split; ++sp) {
    const float4 v = *reinterpret_cast<const float4*>(
        part + (int64_t(sp) * n_tail + tt) * TX * TX + int64_t(i) * TX + j);
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  const float a4[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t gj = J * TX + j + c;
    if (gj < D && gi >= gj) G[gi * D + gj] += a4[c] * gscale;
  }
}

// The split head's slices: exact int64 sums of the int32 partials, slice
// order irrelevant, then scaled into the FP64 G.
__global__ __launch_bounds__(256) void gram_combine_head_kernel(const int32_t* __restrict__ part,
                                                               X1Plan plan, int32_t D,
                                                               const int32_t* __restrict__ exps,
                                                               double* __restrict__ G64) {
  const int64_t n_tail = plan.n_tiles - plan.n_whole;
  const int64_t tt = blockIdx.x;
  int64_t I, J;
  x1_tile_of(plan.n_whole + tt, (D + TX - 1) / TX, I, J);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int j = (threadIdx.x & 63) * 4;
  const int64_t gi = I * TX + i;
  if (gi >= D) return;
  int64_t acc[4] = {0, 0, 0, 0};
  for (int sp = 0; sp < plan.n_split; ++sp) {
    const int4 v = *reinterpret_cast<const int4*>(
        part + (int64_t(sp) * n_tail + tt) * TX * TX + int64_t(i) * TX + j);
    acc[0] += v.x;
    acc[1] += v.y;
    acc[2] += v.z;
    acc[3] += v.w;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t gj = J * TX + j + c;
    if (gj < D && gi >= gj) G64[gi * D + gj] += ldexp(double(acc[c]), -(exps[gi] + exps[gj]));
  }
}

// Tail split of the single-product kernel: keep whole rounds of kX1Slots
// tiles (all of them, or all but one round) and split the remaining tiles
// into the slice count that minimises the rounds of work, in units of one
// whole tile. Slices keep at least 8 stages of rows, and at most 1024
// partial tiles (256 MB) are written.
static X1Plan x1_plan(int64_t D, int64_t n_stages) {
  X1Plan best{x1_tiles(D), x1_tiles(D), 1};
  const int64_t nt = best.n_tiles;
  const int64_t q = nt / kX1Slots;
  if (nt % kX1Slots == 0) return best;
  double best_cost = double(q + 1);
  for (int64_t k = q; k >= 0 && k >= q - 1; --k) {
    const int64_t tail = nt - k * kX1Slots;
    for (int st = 2; st <= 16; ++st) {
      if (n_stages < 8 * int64_t(st) || tail * st > 1024) break;
      const double cost = double(k) + double((tail * st + kX1Slots - 1) / kX1Slots) / st;
      if (cost < best_cost - 1e-9) {
        best_cost = cost;
        best = X1Plan{nt, nt - tail, st};
      }
    }
  }
  return best;
}

static int64_t x1_grid(const X1Plan& p) {
  int64_t m = 0;
  for (int x = 0; x < 8; ++x) {
    int64_t w0, nw, q0, nq;
    x1_xcd_items(p, x, w0, nw, q0, nq);
    m = std::max(m, nw + nq);
  }
  return 8 * m;
}

// Flush of the block sum P (kFlushRows rows on the matrix cores) into the
// running FP32 sum S. With KAHAN (the paper's FP32 training mode) the flush is
// compensated: the rounding error of each S += P is carried in C and
// subtracted from the next block (y = P - C; t = S + y; C = (t - S) - y; S = t).
template <bool KAHAN, int BA, int BB, int NA>
__device__ __forceinline__ void flush_sum(f32x16 (&P)[BA][BB], f32x16 (&S)[BA][BB],
                                          f32x16 (&C)[NA][BB]) {
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if constexpr (KAHAN) {
          const float y = P[a][b][r] - C[a][b][r];
          const float t = S[a][b][r] + y;
          C[a][b][r] = (t - S[a][b][r]) - y;
          S[a][b][r] = t;
        } else {
          S[a][b][r] += P[a][b][r];
        }
        P[a][b][r] = 0.0f;
      }
}
// After the last flush of the Kahan mode: the sum with its carried rounding
// error taken back, S - C, which is what leaves the kernel.
template <int BA, int BB>
__device__ __forceinline__ void fold_compensation(f32x16 (&S)[BA][BB], const f32x16 (&C)[BA][BB]) {
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) S[a][b][r] -= C[a][b][r];
}

// ------------------------------------------------ FP32 mode, D % 4 == 0
// Stage = SR rows of Z: SR A rows of 256 floats (one wave copy each) and SR B
// rows of 128 floats (one copy per pair of rows), in a ring of 4 stages of 16
// rows, 3 of 32 or 2 of 48 (96, 144, 144 KB of LDS: one workgroup per CU).
// With two stages the copies of stage s + 2 are issued after the barrier that
// publishes s + 1 and have the products of s + 1 to land.
// Rows past M are copied from a 1 KB block of zeros; columns past D are
// clamped into the row (they only reach G entries that are never written).
// Waves: NW / 2 x 2 waves of (2 TA / NW) x 64, TA the A columns of a workgroup.
// HALF: the two row halves of a 256 x 128 tile (TA = 128) go to two
// workgroups of 8 waves of 32 x 64 with a 64 KB ring (2 stages of 32 rows),
// so two workgroups share a compute unit and each passes its stage barriers
// on its own: while one waits on a barrier or a copy, the other's waves keep
// the matrix cores busy. Each entry of G is summed in the same order either
// way (bitwise the same G). Plain FP32 uses half tiles: 12.6 ms at 20,000 x
// 8192 against 13.4 with one 16-wave workgroup per tile (four waves per SIMD,
// 3 stages of 32 rows), 13.7 with eight waves of 64 x 64 and 2 stages of 48,
// and 13.3 with half tiles and 16-row stages; 216 against 232 ms at 100,000
// x 16384. The Kahan mode likewise: 13.6 ms against 14.4 in whole 16-wave
// tiles and 14.7 with eight waves of 64 x 64 and 4 stages of 16 (it spills
// about 24 registers around the flushes). The block size of the products stays 32 x 32
// (v_mfma_f32_32x32x2f32): v_mfma_f32_16x16x4f32 with the same wave tiles
// took 13.5 ms (sixteen waves) and 13.8 ms (eight).
template <bool KAHAN, int NW, int SR, bool HALF>
__global__ __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(HALF ? NW / 2 : NW / 4, HALF ? NW / 2 : NW / 4)))
void gram_fp32_ring_kernel(const float* __restrict__ Z, int64_t M, int32_t D, int64_t n_tiles,
                           int64_t nI, int64_t nJ, const float* __restrict__ zeros,
                           float* __restrict__ G, SlicePlan plan, float* __restrict__ part) {
  static_assert(SR == 16 || SR == 32 || SR == 48, "stage rows");
  constexpr int TA = HALF ? TM / 2 : TM;      // A columns (rows of G) per workgroup
  // ring depth: 96, 144, 144 KB of LDS for whole tiles, 64 KB for half tiles
  constexpr int NS = HALF ? 64 / SR : (SR == 16 ? 4 : (SR == 32 ? 3 : 2));
  // copies per stage: SR A rows (HALF: SR / 2 pairs) and SR / 2 pairs of B rows
  constexpr int NCP = HALF ? SR : SR + SR / 2;
  constexpr int PW = NCP / NW;                 // copies per wave per stage
  static_assert(PW * NW == NCP && NS >= 2, "copies per stage, ring depth");
  // stages per flush: 256 rows, or 240 with 48-row stages
  constexpr int KC = SR == 48 ? 5 : kFlushRows / SR;
  constexpr int WR = TA / (NW / 2), WC = TN / 2;   // wave tile
  constexpr int BA = WR / 32, BB = WC / 32;
  __shared__ float ra[NS][SR][TA];
  __shared__ float rb[NS][SR][TN];

  // HALF: workgroups b and b + 8 of each group of 16 take the two row halves
  // of the same item, on the same XCD (b mod 8)
  int64_t I, J;
  const int64_t hb = HALF ? (blockIdx.x / 8) & 1 : 0;
  const int64_t bid = HALF ? (blockIdx.x / 16) * 8 + blockIdx.x % 8 : blockIdx.x;
  const int64_t sp = bid / plan.grid1;
  if (!super_tile(bid % plan.grid1, D, nI, nJ, I, J)) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv >> 1, wx = wv & 1;
  const int64_t A0 = I * TM + hb * TA, B0 = J * TN;
  const bool active = A0 + wy * WR + WR - 1 >= B0 + wx * WC;
  const int la = HALF ? (lane & 31) : lane;
  const int64_t colA = (A0 + 4 * la < D - 4 ? A0 + 4 * la : D - 4);
  const int64_t colB = (B0 + 4 * (lane & 31) < D - 4 ? B0 + 4 * (lane & 31) : D - 4);
  // this item's rows [r0, r1)
  const int64_t r0 = sp * plan.rows_per;
  const int64_t r1 = r0 + plan.rows_per < M ? r0 + plan.rows_per : M;
  const int64_t n_st = r1 > r0 ? (r1 - r0 + SR - 1) / SR : 0;
  // copy c of a stage (c = wv + NW i): c < NA is A row c (HALF: rows 2 c + (0, 1)),
  // else B rows 2 (c - NA) + (0, 1)
  auto issue = [&](int64_t st, int slot) {
    const int64_t m0 = r0 + st * SR;
#pragma unroll
    for (int i = 0; i < PW; ++i) {
      const int c = wv + NW * i;
      constexpr int NA = HALF ? SR / 2 : SR;
      if (c < NA) {
        const int k = HALF ? 2 * c + (lane >> 5) : c;
        const int64_t m = m0 + k;
        const float* g = m < r1 ? Z + m * D + colA : zeros + 4 * lane;
        dma16(g, &ra[slot][HALF ? 2 * c : c][0]);
      } else {
        const int k = 2 * (c - NA) + (lane >> 5);
        const int64_t m = m0 + k;
        const float* g = m < r1 ? Z + m * D + colB : zeros + 4 * lane;
        dma16(g, &rb[slot][2 * (c - NA)][0]);
      }
    }
  };

  f32x16 P[BA][BB], S[BA][BB];
  f32x16 Cc[KAHAN ? BA : 1][BB];   // Kahan compensation of S (mode 5 only)
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        P[a][b][r] = 0.0f;
        S[a][b][r] = 0.0f;
        if (KAHAN) Cc[KAHAN ? a : 0][b][r] = 0.0f;
      }

  // Software pipeline over sub-stages of 8 rows (4 k steps): the LDS reads of
  // one sub-stage are issued while the products of the previous one run, so
  // the matrix core keeps working across the stage barrier. All NS slots are
  // filled up front; after the barrier that publishes stage s + 1 every wave
  // has read all of stage s, so its slot takes stage s + NS.
  constexpr int HK = 4;            // k steps (of 2 rows) per sub-stage
  constexpr int NSUB = SR / 8;     // sub-stages per stage (even)
  float a0[HK][BA], b0[HK][BB], a1[HK][BA], b1[HK][BB];
  auto read_sub = [&](int sl, int j, float (&af)[HK][BA], float (&bf)[HK][BB]) {
#pragma unroll
    for (int kk = 0; kk < HK; ++kk) {
      const int k = 2 * (j * HK + kk) + (lane >> 5);
#pragma unroll
      for (int a = 0; a < BA; ++a) af[kk][a] = ra[sl][k][wy * WR + a * 32 + (lane & 31)];
#pragma unroll
      for (int b = 0; b < BB; ++b) bf[kk][b] = rb[sl][k][wx * WC + b * 32 + (lane & 31)];
    }
  };
  auto mma_sub = [&](const float (&af)[HK][BA], const float (&bf)[HK][BB]) {
#pragma unroll
    for (int kk = 0; kk < HK; ++kk)
#pragma unroll
      for (int a = 0; a < BA; ++a)
#pragma unroll
        for (int b = 0; b < BB; ++b)
          P[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[kk][a], bf[kk][b], P[a][b], 0, 0, 0);
  };
  // sum r of a lane sits in row 4 (lane / 32) + rr(r) of its 32 x 32 block,
  // column lane % 32 (the lane-dependent offsets are formed once, outside the
  // unrolled stores: indexing each store from the lane kept more registers live)
  auto rr = [](int r) { return 8 * (r >> 2) + (r & 3); };
  // the next sub-stage's LDS reads interleaved with the first products
  auto interleave = [] {
    constexpr int NR = HK * (BA + BB), NM = HK * BA * BB;
#pragma unroll
    for (int i = 0; i < (NR < NM ? NR : NM); ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    if constexpr (NM > NR) __builtin_amdgcn_sched_group_barrier(0x008, NM - NR, 0);
    if constexpr (NR > NM) __builtin_amdgcn_sched_group_barrier(0x100, NR - NM, 0);
  };

#pragma unroll
  for (int j = 0; j < NS; ++j)
    if (j < n_st) issue(j, j);
  if (n_st > 0) {
    wait_stage<PW>(n_st - 1 < NS - 1 ? n_st - 1 : NS - 1);
    stage_barrier();
    read_sub(0, 0, a0, b0);
  }
  int slot = 0;
  int64_t s = 0;
  while (s < n_st) {
    const int64_t g_end = s + KC < n_st ? s + KC : n_st;
    for (; s < g_end; ++s) {
      // sub-stages 0 .. NSUB - 2 of stage s; sub-stage j sits in a0/b0 when j is even
#pragma unroll
      for (int j = 0; j + 2 < NSUB; j += 2) {
        read_sub(slot, j + 1, a1, b1);
        mma_sub(a0, b0);
        interleave();
        read_sub(slot, j + 2, a0, b0);
        mma_sub(a1, b1);
        interleave();
      }
      read_sub(slot, NSUB - 1, a1, b1);
      mma_sub(a0, b0);
      interleave();
      const bool more = s + 1 < n_st;
      const int nslot = more ? (slot + 1 == NS ? 0 : slot + 1) : slot;
      if (more) {
        const int64_t ahead = n_st - 2 - s;
        wait_stage<PW>(ahead < NS - 2 ? ahead : NS - 2);
        // this wave's reads of stage s have landed before its slot is reused
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        stage_barrier();
        if (s + NS < n_st) issue(s + NS, slot);
      }
      // after the last stage this re-reads a published slot with no copy in
      // flight; the values are not used
      read_sub(nslot, 0, a0, b0);
      mma_sub(a1, b1);
      interleave();
      slot = nslot;
    }
    flush_sum<KAHAN>(P, S, Cc);
  }
  if constexpr (KAHAN) fold_compensation(S, Cc);

  if (!active) return;
  if (sp > 0) {
    float* out = part + ((sp - 1) * n_tiles + tile_index(I, J)) * (TM * TN) +
                 (hb * TA + wy * WR + 4 * (lane >> 5)) * TN + wx * WC + (lane & 31);
#pragma unroll
    for (int a = 0; a < BA; ++a)
#pragma unroll
      for (int b = 0; b < BB; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) out[(a * 32 + rr(r)) * TN + b * 32] = S[a][b][r];
    return;
  }
  const int64_t i0 = A0 + wy * WR + 4 * (lane >> 5), j0 = B0 + wx * WC + (lane & 31);
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gi = i0 + a * 32 + rr(r);
        const int64_t gj = j0 + b * 32;
        if (gi < D && gj < D && gi >= gj) G[gi * D + gj] += S[a][b][r];
      }
}

// G += the partial tiles of slices 1 .. n_split - 1 of every 256 x 128 tile
// (slice 0 added its sum into G itself), summed in slice order; in the Kahan
// mode G and the partials are summed with compensation, so that combining the
// slices rounds once, as the unsliced kernel's final G += S does. One workgroup
// per 4 rows of a tile, two columns per thread. Entries of waves above the
// diagonal are never written to the partials; they are not read.
template <bool KAHAN>
__global__ __launch_bounds__(256) void gram_slices_combine_kernel(const float* __restrict__ part,
                                                                 int64_t n_tiles, int32_t n_split,
                                                                 int32_t D,
                                                                 float* __restrict__ G) {
  const int64_t t = blockIdx.x;
  int64_t I = int64_t((std::sqrt(4.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) > t) --I;
  while ((I + 1) * (I + 2) <= t) ++I;
  const int64_t J = t - I * (I + 1);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int j = (threadIdx.x & 63) * 2;
  const int64_t gi = I * TM + i, gj = J * TN + j;
  if (gi >= D || gj > gi) return;
  const bool second = gj + 1 < D && gj + 1 <= gi;
  if constexpr (KAHAN) {
    // G (which holds slice 0) and the partials in slice order, compensated
    float2 sum = make_float2(G[gi * D + gj], second ? G[gi * D + gj + 1] : 0.0f);
    float2 c = make_float2(0.0f, 0.0f);
    for (int sp = 1; sp < n_split; ++sp) {
      const float2 v = *reinterpret_cast<const float2*>(
          part + (int64_t(sp - 1) * n_tiles + t) * (TM * TN) + int64_t(i) * TN + j);
      const float yx = v.x - c.x, yy = v.y - c.y;
      const float tx = sum.x + yx, ty = sum.y + yy;
      c.x = (tx - sum.x) - yx;
      c.y = (ty - sum.y) - yy;
      sum.x = tx;
      sum.y = ty;
    }
    G[gi * D + gj] = sum.x - c.x;
    if (second) G[gi * D + gj + 1] = sum.y - c.y;
  } else {
    float2 acc = make_float2(0.0f, 0.0f);
    for (int sp = 1; sp < n_split; ++sp) {
      const float2 v = *reinterpret_cast<const float2*>(
          part + (int64_t(sp - 1) * n_tiles + t) * (TM * TN) + int64_t(i) * TN + j);
      acc.x += v.x;
      acc.y += v.y;
    }
    G[gi * D + gj] += acc.x;
    if (second) G[gi * D + gj + 1] += acc.y;
  }
}

// ------------------------------------------------ FP32 mode, any D
// Row-major slabs of 16 rows staged through registers into LDS ([k][column],
// padded) with masked loads; the 32x32x2 f32 MFMA reads lane l = column l%32
// of slab row k0 + l/32. Used when D is not a multiple of 4.
template <bool VEC4, bool KAHAN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gram_fp32_kernel(const float* __restrict__ Z, int64_t M, int32_t D, int64_t n_tiles,
                      int64_t nI, int64_t nJ, float* __restrict__ G) {
  constexpr int LDA = TM + 4, LDB = TN + 4;
  constexpr int KC = kFlushRows / KB;
  constexpr int CA = KB * TM / 4 / 256;        // float4 chunks per thread (A)
  constexpr int CB = KB * TN / 4 / 256;        // (B)
  __shared__ float sA[2][KB][LDA];
  __shared__ float sB[2][KB][LDB];

  int64_t I, J;
  if (!super_tile(blockIdx.x, D, nI, nJ, I, J)) return;
  (void)n_tiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv >> 1, wx = wv & 1;
  const bool active = I * TM + wy * 128 + 127 >= J * TN + wx * 64;
  const int64_t A0 = I * TM, B0 = J * TN;

  f32x16 P[4][2], S[4][2];
  f32x16 Cc[KAHAN ? 4 : 1][2];   // Kahan compensation of S (mode 5 only)
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        P[a][b][r] = 0.0f;
        S[a][b][r] = 0.0f;
        if (KAHAN) Cc[KAHAN ? a : 0][b][r] = 0.0f;
      }

  float4 pa[CA], pb[CB];
  // chunk q: slab row q / (width / 4), column 4 (q % (width / 4))
  auto load = [&](int64_t m0) {
#pragma unroll
    for (int c = 0; c < CA + CB; ++c) {
      const bool isA = c < CA;
      const int q = tid + 256 * (isA ? c : c - CA);
      const int w4 = (isA ? TM : TN) / 4;
      const int k = q / w4;
      const int64_t col = (isA ? A0 : B0) + 4 * (q % w4);
      const int64_t m = m0 + k;
      float4 v;
      if (VEC4 && m < M && col + 4 <= D) {
        v = *reinterpret_cast<const float4*>(Z + m * D + col);
      } else {
        const int64_t mc = m < M ? m : M - 1;
        float e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float zl = Z[mc * D + (col + u < D ? col + u : D - 1)];
          e[u] = (m < M && col + u < D) ? zl : 0.0f;
        }
        v = make_float4(e[0], e[1], e[2], e[3]);
      }
      if (isA) pa[c] = v; else pb[c - CA] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int c = 0; c < CA; ++c) {
      const int q = tid + 256 * c;
      *reinterpret_cast<float4*>(&sA[buf][q / (TM / 4)][4 * (q % (TM / 4))]) = pa[c];
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int q = tid + 256 * c;
      *reinterpret_cast<float4*>(&sB[buf][q / (TN / 4)][4 * (q % (TN / 4))]) = pb[c];
    }
  };

  const int64_t n_stages = (M + KB - 1) / KB;
  load(0);
  store(0);
  __syncthreads();
  for (int64_t s = 0; s < n_stages; ++s) {
    const int buf = int(s & 1);
    if (s + 1 < n_stages) load((s + 1) * KB);
    if (active) {
#pragma unroll
      for (int kk = 0; kk < KB; kk += 2) {
        const int k = kk + (lane >> 5);
        float af[4], bf[2];
#pragma unroll
        for (int a = 0; a < 4; ++a) af[a] = sA[buf][k][wy * 128 + a * 32 + (lane & 31)];
#pragma unroll
        for (int b = 0; b < 2; ++b) bf[b] = sB[buf][k][wx * 64 + b * 32 + (lane & 31)];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            P[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a], bf[b], P[a][b], 0, 0, 0);
      }
      if ((s + 1) % KC == 0 || s + 1 == n_stages) flush_sum<KAHAN>(P, S, Cc);
    }
    if (s + 1 < n_stages) store(buf ^ 1);
    __syncthreads();
  }
  if constexpr (KAHAN) fold_compensation(S, Cc);

  if (!active) return;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gi = A0 + wy * 128 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t gj = B0 + wx * 64 + b * 32 + (lane & 31);
        if (gi < D && gj < D && gi >= gj) G[gi * D + gj] += S[a][b][r];
      }
}

// Square tiles of the FP64 mode: t = I (I + 1) / 2 + J, I >= J.
__device__ __forceinline__ void tile_of_square(int64_t t, int64_t& I, int64_t& J) {
  int64_t i = int64_t((std::sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

// ----------------------------------------------------------------- FP64 mode
// The paper's double-precision training: Z (FP32) promoted to FP64 in LDS and
// multiplied on the FP64 matrix cores; G is FP64. 64 x 64 tiles, 4 waves of
// 32 x 32 (2 x 2 blocks of v_mfma_f64_16x16x4f64).
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void gram_fp64_kernel(const float* __restrict__ Z, int64_t M,
                                                       int32_t D, double* __restrict__ G,
                                                       const float* __restrict__ y,
                                                       double* __restrict__ Zty) {
  constexpr int T64 = 64;
  __shared__ double sA[KB][T64 + 1];
  __shared__ double sB[KB][T64 + 1];
  __shared__ double zred[KB][T64];
  int64_t I, J;
  tile_of_square(blockIdx.x, I, J);
  const bool diag = (I == J);
  const int64_t I0 = I * T64, J0 = J * T64;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv >> 1, wx = wv & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int lk = tid >> 4;        // slab row 0..15
  const int li = (tid & 15) * 4;  // 4 consecutive columns
  const bool want_zty = diag && y != nullptr;
  double zacc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t m0 = 0; m0 < M; m0 += KB) {
    const int64_t m = m0 + lk;
    const double yl = want_zty ? double(y[m < M ? m : M - 1]) : 0.0;
    const double ym = (m < M) ? yl : 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t ci = I0 + li + c, cj = J0 + li + c;
      const int64_t mc = m < M ? m : M - 1;
      const float zil = Z[mc * D + (ci < D ? ci : D - 1)];
      const float zjl = Z[mc * D + (cj < D ? cj : D - 1)];
      const double zi = (m < M && ci < D) ? double(zil) : 0.0;
      sA[lk][li + c] = zi;
      zacc[c] += zi * ym;
      if (!diag) sB[lk][li + c] = (m < M && cj < D) ? double(zjl) : 0.0;
    }
    __syncthreads();
    const double (*sb)[T64 + 1] = diag ? sA : sB;
#pragma unroll
    for (int kk = 0; kk < KB; kk += 4) {
      const int k = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        av[b] = sA[k][wy * 32 + b * 16 + (lane & 15)];
        bv[b] = sb[k][wx * 32 + b * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // v_mfma_f64_16x16x4f64: lane l, register r holds row l/16 + 4 r, column l%16
        const int64_t gi = I0 + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int64_t gj = J0 + wx * 32 + b * 16 + (lane & 15);
        if (gi < D && gj < D && gi >= gj) G[gi * D + gj] += acc[a][b][r];
      }
  if (want_zty) {
#pragma unroll
    for (int c = 0; c < 4; ++c) zred[lk][li + c] = zacc[c];
    __syncthreads();
    if (tid < T64 && I0 + tid < D) {
      double t = 0.0;
      for (int r = 0; r < KB; ++r) t += zred[r][tid];
      Zty[I0 + tid] += t;
    }
  }
}

}  // namespace sorf

using namespace sorf;

namespace {
size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
// Workspace: [Z^T y partials][1 KB of zeros][packed hi][packed lo]
struct GramLayout {
  int64_t n_slabs;   // 16-row slabs, padded to whole 4-slab stages
  int32_t ncb;       // 32-column blocks, padded to whole 256-column tiles
  int64_t chunks;    // Z^T y partial chunks
  size_t part_bytes, zpart_bytes;
};
constexpr size_t kZeroBytes = 1024;
GramLayout gram_layout(int64_t M, int32_t D) {
  GramLayout g;
  g.n_slabs = ((M + 4 * KB - 1) / (4 * KB)) * 4;
  g.ncb = int32_t(((int64_t(D) + TM - 1) / TM) * (TM / 32));
  g.chunks = (g.n_slabs + kPackSlabs - 1) / kPackSlabs;
  g.part_bytes = al256(size_t(g.n_slabs) * size_t(g.ncb) * 1024);
  g.zpart_bytes = al256(size_t(g.chunks) * size_t(D) * sizeof(double));
  return g;
}
}  // namespace

// Row ranges of the single-product launches: [k R, min((k + 1) R, n)).
static size_t x1_plan_partial_bytes(const X1Plan& p) {
  return size_t(p.n_split > 1 ? p.n_split : 0) * size_t(p.n_tiles - p.n_whole) * TX * TX *
         sizeof(float);
}

size_t x1_partial_bytes(int64_t n_rows, int32_t D) {
  const GramLayout g = gram_layout(n_rows, D);
  const int64_t n_st = g.n_slabs / x1_stage_slabs(kBF16);
  const int64_t full = n_st < kX1LaunchStages ? n_st : kX1LaunchStages;
  const int64_t last = n_st % kX1LaunchStages;
  size_t b = x1_plan_partial_bytes(x1_plan(D, full));
  if (last > 0) b = std::max(b, x1_plan_partial_bytes(x1_plan(D, last)));
  return al256(b);
}

// Row-slice plan of the FP32 tile kernel: the slice count in 1..8 with the
// least estimated time, counted in rounds of 256 items (one per compute unit,
// each a slice of one tile at the FP32 matrix-core rate) plus the partial
// tiles' HBM traffic (written once, read once, at 5 TB/s). Ties: fewer
// slices. Slices keep at least 2048 rows; the partials stay within 4 GB.
static SlicePlan slice_plan(int64_t M, int32_t D) {
  int64_t nI, nJ;
  const int64_t T = gram_tiles(D, nI, nJ);
  const int64_t grid1 = ((gram_super_tiles(D) + 7) / 8) * 8 * SR_T * SC_T;
  const double tile_s = 2.0 * TM * TN * double(M) / (157.3e12 / kX1Slots);   // whole tile
  const double part_s = double(TM * TN * sizeof(float)) * 2.0 / 5e12;       // per partial tile
  SlicePlan best{1, M, grid1};
  double best_cost = double((T + kX1Slots - 1) / kX1Slots) * tile_s;
  for (int s = 2; s <= 8; ++s) {
    const int64_t rows = ((M + s - 1) / s + kFlushRows - 1) / kFlushRows * kFlushRows;
    const int64_t n = (M + rows - 1) / rows;
    if (rows < 2048 || size_t(n - 1) * size_t(T) * TM * TN * sizeof(float) > (size_t(4) << 30))
      break;
    const double cost = double((T * n + kX1Slots - 1) / kX1Slots) * tile_s * double(rows) / double(M) +
                        double((n - 1) * T) * part_s;
    if (cost < best_cost - 1e-9) {
      best_cost = cost;
      best = SlicePlan{int32_t(n), rows, grid1};
    }
  }
  return best;
}

static size_t slice_partial_bytes(int64_t M, int32_t D) {
  const SlicePlan p = slice_plan(M, D);
  if (p.n_split <= 1) return 0;
  int64_t nI, nJ;
  return al256(size_t(p.n_split - 1) * size_t(gram_tiles(D, nI, nJ)) * TM * TN * sizeof(float));
}

size_t sorf_gram_ws_bytes(int64_t n_rows, int32_t D, int mode) {
  if (n_rows <= 0 || D <= 0) return 0;
  const GramLayout g = gram_layout(n_rows, D);
  size_t b = g.zpart_bytes + kZeroBytes;
  if ((mode == kFP32 || mode == kFP32Kahan) && D % 4 == 0) b += slice_partial_bytes(n_rows, D);
  if (mode != kFP32 && mode != kFP32Kahan) b += g.part_bytes * (is_hilo(mode) ? 2 : 1);
  if (mode == kBF16 || mode == kFP16) b += x1_partial_bytes(n_rows, D);
  return b;
}

hipError_t sorf_launch_gram(int64_t n_rows, int32_t D, const float* Z, const float* y, int mode,
                            int32_t scale_exp, float* G, float* Zty, void* ws, hipStream_t st) {
  if (n_rows == 0 || D == 0) return hipSuccess;
  const GramLayout g = gram_layout(n_rows, D);
  char* w = static_cast<char*>(ws);
  double* zpart = reinterpret_cast<double*>(w);
  float* zeros = reinterpret_cast<float*>(w + g.zpart_bytes);
  u16x8* hi = reinterpret_cast<u16x8*>(w + g.zpart_bytes + kZeroBytes);
  u16x8* lo = reinterpret_cast<u16x8*>(w + g.zpart_bytes + kZeroBytes + g.part_bytes);
  const float zs = std::ldexp(1.0f, scale_exp);
  const float gs = std::ldexp(1.0f, -2 * scale_exp);
  const dim3 pgrid{unsigned(g.ncb / 4), unsigned(g.chunks)}, blk{256};
  switch (mode) {
    case kFP32:
    case kFP32Kahan:
      if (y != nullptr)
        hipLaunchKernelGGL(pack_kernel<kFP32>, pgrid, blk, 0, st, Z, n_rows, D, g.n_slabs, g.ncb,
                           1.0f, hi, lo, y, zpart);
      break;
    case kBF16:
      hipLaunchKernelGGL(pack_kernel<kBF16>, pgrid, blk, 0, st, Z, n_rows, D, g.n_slabs, g.ncb,
                         zs, hi, lo, y, zpart);
      break;
    case kFP16:
      hipLaunchKernelGGL(pack_kernel<kFP16>, pgrid, blk, 0, st, Z, n_rows, D, g.n_slabs, g.ncb,
                         zs, hi, lo, y, zpart);
      break;
    case kBF16HiLo:
      hipLaunchKernelGGL(pack_kernel<kBF16HiLo>, pgrid, blk, 0, st, Z, n_rows, D, g.n_slabs,
                         g.ncb, zs, hi, lo, y, zpart);
      break;
    case kFP16HiLo:
      hipLaunchKernelGGL(pack_kernel<kFP16HiLo>, pgrid, blk, 0, st, Z, n_rows, D, g.n_slabs,
                         g.ncb, zs, hi, lo, y, zpart);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (y != nullptr) {
    hipLaunchKernelGGL(zty_finalize_kernel<float>, dim3(unsigned((D + 255) / 256)), dim3(256), 0,
                       st, zpart, g.chunks, D, Zty);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  int64_t nI, nJ;
  const int64_t n_tiles = gram_tiles(D, nI, nJ);
  const dim3 grid{unsigned(((gram_super_tiles(D) + 7) / 8) * 8 * SR_T * SC_T)};
  switch (mode) {
    case kFP32:
    case kFP32Kahan:
      if (D % 4 == 0) {
        if ((e = sorf_launch_fill(zeros, int64_t(kZeroBytes / sizeof(float)), 0.0f, st)) !=
            hipSuccess)
          return e;
        const SlicePlan plan = slice_plan(n_rows, D);
        float* part = reinterpret_cast<float*>(w + g.zpart_bytes + kZeroBytes);
        const dim3 rgrid{unsigned(plan.grid1 * plan.n_split)};
        if (mode == kFP32Kahan)
          hipLaunchKernelGGL((gram_fp32_ring_kernel<true, kFP32Waves, kFP32StageRows, kFP32Half>),
                             dim3((kFP32Half ? 2 : 1) * rgrid.x), dim3(64 * kFP32Waves), 0, st, Z,
                             n_rows, D, n_tiles, nI, nJ, zeros, G, plan, part);
        else
          hipLaunchKernelGGL((gram_fp32_ring_kernel<false, kFP32Waves, kFP32StageRows, kFP32Half>),
                             dim3((kFP32Half ? 2 : 1) * rgrid.x), dim3(64 * kFP32Waves), 0, st, Z,
                             n_rows, D, n_tiles, nI, nJ, zeros, G, plan, part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (plan.n_split > 1 && mode == kFP32Kahan)
          hipLaunchKernelGGL(gram_slices_combine_kernel<true>,
                             dim3(unsigned(n_tiles), unsigned(TM / 4)), blk, 0, st, part, n_tiles,
                             plan.n_split, D, G);
        else if (plan.n_split > 1)
          hipLaunchKernelGGL(gram_slices_combine_kernel<false>,
                             dim3(unsigned(n_tiles), unsigned(TM / 4)), blk, 0, st, part, n_tiles,
                             plan.n_split, D, G);
      } else if (mode == kFP32Kahan) {
        hipLaunchKernelGGL((gram_fp32_kernel<false, true>), grid, blk, 0, st, Z, n_rows, D,
                           n_tiles, nI, nJ, G);
      } else {
        hipLaunchKernelGGL((gram_fp32_kernel<false, false>), grid, blk, 0, st, Z, n_rows, D,
                           n_tiles, nI, nJ, G);
      }
      break;
    case kBF16:
    case kFP16: {
      float* part = reinterpret_cast<float*>(w + g.zpart_bytes + kZeroBytes + g.part_bytes);
      const int64_t n_st = g.n_slabs / x1_stage_slabs(kBF16);
      for (int64_t s0 = 0; s0 < n_st; s0 += kX1LaunchStages) {
        const int64_t cnt = n_st - s0 < kX1LaunchStages ? n_st - s0 : kX1LaunchStages;
        const X1Plan plan = x1_plan(D, cnt);
        const dim3 xg{unsigned(x1_grid(plan))};
        if (mode == kBF16)
          hipLaunchKernelGGL(gram_x1_kernel<kBF16>, xg, dim3(64 * x1_waves(kBF16)), 0, st, hi, s0,
                             cnt, g.ncb, D, plan, gs, G, part, nullptr, nullptr);
        else
          hipLaunchKernelGGL(gram_x1_kernel<kFP16>, xg, dim3(64 * x1_waves(kFP16)), 0, st, hi, s0,
                             cnt, g.ncb, D, plan, gs, G, part, nullptr, nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (plan.n_split > 1) {
          const dim3 cg{unsigned(plan.n_tiles - plan.n_whole), unsigned(TX / 4)};
          hipLaunchKernelGGL(gram_combine_kernel, cg, blk, 0, st, part, plan, D, gs, G);
          if ((e = hipGetLastError()) != hipSuccess) return e;
        }
      }
      break;
    }
    case kBF16HiLo:
      hipLaunchKernelGGL(gram_packed_kernel<kBF16HiLo>, grid, dim3(64 * kPackedWaves), 0, st, hi,
                         lo, g.n_slabs, g.ncb, D, n_tiles, nI, nJ, gs, G, nullptr, nullptr);
      break;
    case kFP16HiLo:
      hipLaunchKernelGGL(gram_packed_kernel<kFP16HiLo>, grid, dim3(64 * kPackedWaves), 0, st, hi,
                         lo, g.n_slabs, g.ncb, D, n_tiles, nI, nJ, gs, G, nullptr, nullptr);
      break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------- split mode launch
namespace {
// Head launches: 64-row stages, exact while rows * 127^2 < 2^31.
constexpr int64_t kHeadLaunchStages = 2048;   // 131,072 rows
// Workspace: [Z^T y partials][column maxima][exponents][fp16 head][fp16 tail]
// [int8 head][head slice partials]
struct SplitLayout {
  int64_t n_slabs;   // 16-row slabs, padded to whole 64-row head stages
  int32_t ncb;       // 32-column blocks, padded to whole 256-column tiles
  int64_t chunks;    // Z^T y partial chunks
  int64_t cm_chunks, cm_rows;
  size_t zpart, cmax, exps, frag16, frag8, head_part;
};
SplitLayout split_layout(int64_t M, int32_t D) {
  SplitLayout g;
  g.n_slabs = ((M + 4 * KB - 1) / (4 * KB)) * 4;
  g.ncb = int32_t(((int64_t(D) + TM - 1) / TM) * (TM / 32));
  g.chunks = (g.n_slabs + kPackSlabs - 1) / kPackSlabs;
  g.cm_chunks = std::min<int64_t>(256, (M + 511) / 512);
  g.cm_rows = (M + g.cm_chunks - 1) / g.cm_chunks;
  g.zpart = al256(size_t(g.chunks) * size_t(D) * sizeof(double));
  g.cmax = al256(size_t(g.cm_chunks) * size_t(D) * sizeof(float));
  g.exps = al256(size_t(D) * sizeof(int32_t));
  g.frag16 = al256(size_t(g.n_slabs) * size_t(g.ncb) * 1024);
  g.frag8 = al256(size_t(g.n_slabs / 2) * size_t(g.ncb) * 1024);
  const int64_t n_st = g.n_slabs / 4;
  const int64_t full = n_st < kHeadLaunchStages ? n_st : kHeadLaunchStages;
  const int64_t last = n_st % kHeadLaunchStages;
  size_t b = x1_plan_partial_bytes(x1_plan(D, full));
  if (last > 0) b = std::max(b, x1_plan_partial_bytes(x1_plan(D, last)));
  g.head_part = al256(b);
  return g;
}
}  // namespace

size_t sorf_gram_split_ws_bytes(int64_t n_rows, int32_t D) {
  if (n_rows <= 0 || D <= 0) return 0;
  const SplitLayout g = split_layout(n_rows, D);
  return g.zpart + g.cmax + g.exps + 2 * g.frag16 + g.frag8 + g.head_part;
}

hipError_t sorf_launch_gram_split(int64_t n_rows, int32_t D, const float* Z, const float* y,
                                  double* G, double* Zty, void* ws, hipStream_t st) {
  if (n_rows == 0 || D == 0) return hipSuccess;
  const SplitLayout g = split_layout(n_rows, D);
  char* w = static_cast<char*>(ws);
  double* zpart = reinterpret_cast<double*>(w);
  w += g.zpart;
  float* cmax = reinterpret_cast<float*>(w);
  w += g.cmax;
  int32_t* exps = reinterpret_cast<int32_t*>(w);
  w += g.exps;
  u16x8* hi = reinterpret_cast<u16x8*>(w);
  w += g.frag16;
  u16x8* lo = reinterpret_cast<u16x8*>(w);
  w += g.frag16;
  u16x8* hi8 = reinterpret_cast<u16x8*>(w);
  w += g.frag8;
  int32_t* hpart = reinterpret_cast<int32_t*>(w);
  const dim3 blk{256};
  const unsigned cgrid = unsigned((D + 255) / 256);
  hipLaunchKernelGGL(colmax_kernel, dim3(cgrid, unsigned(g.cm_chunks)), blk, 0, st, Z, n_rows, D,
                     g.cm_rows, cmax);
  hipLaunchKernelGGL(split_exps_kernel, dim3(cgrid), blk, 0, st, cmax, g.cm_chunks, D, exps);
  hipLaunchKernelGGL(pack_split_kernel, dim3(unsigned(g.ncb / 4), unsigned(g.chunks)), blk, 0, st,
                     Z, n_rows, D, g.n_slabs, g.ncb, exps, hi, lo, reinterpret_cast<uint2*>(hi8),
                     y, zpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (y != nullptr) {
    hipLaunchKernelGGL(zty_finalize_kernel<double>, dim3(cgrid), blk, 0, st, zpart, g.chunks, D,
                       Zty);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // head: h^T h on the int8 matrix cores, whole 64-row stages per launch
  const int64_t n_st = g.n_slabs / 4;
  for (int64_t s0 = 0; s0 < n_st; s0 += kHeadLaunchStages) {
    const int64_t cnt = n_st - s0 < kHeadLaunchStages ? n_st - s0 : kHeadLaunchStages;
    const X1Plan plan = x1_plan(D, cnt);
    hipLaunchKernelGGL(gram_x1_kernel<kSplitHead>, dim3(unsigned(x1_grid(plan))),
                       dim3(64 * x1_waves(kSplitHead)), 0, st, hi8, s0, cnt, g.ncb, D, plan, 1.0f,
                       nullptr, reinterpret_cast<float*>(hpart), G, exps);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (plan.n_split > 1) {
      const dim3 cg{unsigned(plan.n_tiles - plan.n_whole), unsigned(TX / 4)};
      hipLaunchKernelGGL(gram_combine_head_kernel, cg, blk, 0, st, hpart, plan, D, exps, G);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  // tail: h^T t + t^T h + t^T t on the fp16 matrix cores
  int64_t nI, nJ;
  const int64_t n_tiles = gram_tiles(D, nI, nJ);
  const dim3 grid{unsigned(((gram_super_tiles(D) + 7) / 8) * 8 * SR_T * SC_T)};
  hipLaunchKernelGGL(gram_packed_kernel<kSplitCross>, grid, dim3(64 * kPackedWaves), 0, st, hi, lo,
                     g.n_slabs, g.ncb, D, n_tiles, nI, nJ, 1.0f, nullptr, G, exps);
  return hipGetLastError();
}

hipError_t sorf_launch_gram_f64(int64_t n_rows, int32_t D, const float* Z, const float* y,
                                double* G, double* Zty, hipStream_t st) {
  if (n_rows == 0 || D == 0) return hipSuccess;
  const int64_t nt = (D + 63) / 64;
  hipLaunchKernelGGL(gram_fp64_kernel, dim3(unsigned(nt * (nt + 1) / 2)), dim3(256), 0, st, Z,
                     n_rows, D, G, y, Zty);
  return hipGetLastError();
}
