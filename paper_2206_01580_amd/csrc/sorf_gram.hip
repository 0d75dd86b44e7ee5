// Normal-equation accumulation G += Z^T Z, Zty += Z^T y on gfx950 MFMA.
//
// Paper: arXiv 2206.01580, RFF subsection (regularised normal equation; the
// Z^T Z product dominates training) and Training-time discussion (FP32 Z^T Z
// suffers cumulative round-off; the paper uses Kahan summation). Here the
// reduced-precision modes split each FP32 value z into hi = round(z) and
// lo = round(z - hi) in bf16 or fp16 and accumulate (hi + lo)^T (hi + lo) =
// hi^T hi + hi^T lo + lo^T hi + lo^T lo in FP32 on the matrix cores. All four
// products are kept: without lo^T lo the result is G - lo^T lo, which is not
// positive semidefinite, and on the QM9-like workload its smallest
// eigenvalues fall below zero by more than any useful ridge term.
//
// Tiling: one workgroup (4 waves) per 128 x 128 tile (I, J) of the lower
// triangle of G; the tile walks all rows of Z in slabs of 16 rows staged
// through LDS; each wave owns a 64 x 64 quadrant = 2 x 2 MFMA 32x32 blocks.
// Z^T y is accumulated (in FP64) by the diagonal tiles, which already read
// every row of their column block, and added once per call in FP32.
#include <cmath>

#include "sorf_internal.h"

namespace sorf {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

enum GramMode { kFP32 = 0, kBF16 = 1, kFP16 = 2, kBF16HiLo = 3, kFP16HiLo = 4 };

constexpr int TILE = 128;
constexpr int KB = 16;

__device__ __forceinline__ void tile_of(int64_t t, int64_t& I, int64_t& J) {
  // t enumerates (I, J), I >= J, row by row: t = I (I + 1) / 2 + J
  int64_t i = int64_t((std::sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

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
  if constexpr (MODE == kBF16 || MODE == kBF16HiLo) {
    hi = to_bf16_bits(z);
    lo = to_bf16_bits(z - from_bf16_bits(hi));
  } else {
    const _Float16 h = (_Float16)z;
    const _Float16 l = (_Float16)(z - (float)h);
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, l);
  }
}

// ----------------------------------------------------------------- FP32 mode
template <bool VEC4>
__global__ __launch_bounds__(256) void gram_fp32_kernel(const float* __restrict__ Z, int64_t M,
                                                       int32_t D, float* __restrict__ G,
                                                       const float* __restrict__ y,
                                                       float* __restrict__ Zty) {
  __shared__ float sA[KB][TILE + 4];
  __shared__ float sB[KB][TILE + 4];
  __shared__ double zred[KB][TILE];
  int64_t I, J;
  tile_of(blockIdx.x, I, J);
  const bool diag = (I == J);
  const int64_t I0 = I * TILE, J0 = J * TILE;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv >> 1, wx = wv & 1;

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  const int lk = tid >> 4;         // slab row 0..15
  const int li = (tid & 15) * 8;   // 8 consecutive columns
  // Z^T y rides on the diagonal tiles, which stream every row of their columns
  const bool want_zty = diag && y != nullptr;
  double zacc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) zacc[c] = 0.0;
  for (int64_t m0 = 0; m0 < M; m0 += KB) {
    const int64_t m = m0 + lk;
    const bool mok = m < M;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t col0 = (h == 0 ? I0 : J0) + li;
      float v[8];
      if (VEC4 && mok && col0 + 8 <= D) {
        const float4* p = reinterpret_cast<const float4*>(Z + m * D + col0);
        const float4 a = p[0], b = p[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
      } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const float zl = Z[(mok ? m : M - 1) * D + (col0 + c < D ? col0 + c : D - 1)];
          v[c] = (mok && col0 + c < D) ? zl : 0.0f;
        }
      }
      float* dst = (h == 0 ? &sA[lk][li] : &sB[lk][li]);
#pragma unroll
      for (int c = 0; c < 8; ++c) dst[c] = v[c];
      if (diag) {
        if (want_zty && mok) {
          const double ym = double(y[m]);
#pragma unroll
          for (int c = 0; c < 8; ++c) zacc[c] += double(v[c]) * ym;
        }
        break;
      }
    }
    __syncthreads();
    const float (*sb)[TILE + 4] = diag ? sA : sB;
#pragma unroll
    for (int kk = 0; kk < KB; kk += 2) {
      const int k = kk + (lane >> 5);
      float af[2], bf[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        af[b] = sA[k][wy * 64 + b * 32 + (lane & 31)];
        bf[b] = sb[k][wx * 64 + b * 32 + (lane & 31)];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gi = I0 + wy * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t gj = J0 + wx * 64 + b * 32 + (lane & 31);
        if (gi < D && gj < D && gi >= gj) G[gi * D + gj] += acc[a][b][r];
      }
  if (want_zty) {
#pragma unroll
    for (int c = 0; c < 8; ++c) zred[lk][li + c] = zacc[c];
    __syncthreads();
    if (tid < TILE && I0 + tid < D) {
      double t = 0.0;
      for (int r = 0; r < KB; ++r) t += zred[r][tid];
      Zty[I0 + tid] += float(t);
    }
  }
}

// ------------------------------------------------- bf16 / fp16 (x1 and hi+lo)
template <int MODE>
__global__ __launch_bounds__(256) void gram_half_kernel(const float* __restrict__ Z, int64_t M,
                                                       int32_t D, float zscale, float gscale,
                                                       float* __restrict__ G,
                                                       const float* __restrict__ y,
                                                       float* __restrict__ Zty) {
  __shared__ double zred[2][TILE];
  constexpr bool HILO = (MODE == kBF16HiLo || MODE == kFP16HiLo);
  constexpr int KP = KB + 8;  // padded k stride (in 16-bit elements)
  __shared__ __attribute__((aligned(16))) unsigned short sAh[TILE][KP];
  __shared__ __attribute__((aligned(16))) unsigned short sBh[TILE][KP];
  __shared__ __attribute__((aligned(16))) unsigned short sAl[HILO ? TILE : 1][KP];
  __shared__ __attribute__((aligned(16))) unsigned short sBl[HILO ? TILE : 1][KP];
  int64_t I, J;
  tile_of(blockIdx.x, I, J);
  const bool diag = (I == J);
  const int64_t I0 = I * TILE, J0 = J * TILE;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv >> 1, wx = wv & 1;

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  const int li = tid & (TILE - 1);  // column within the tile
  const int lk = (tid >> 7) * 8;    // 8 consecutive slab rows
  const bool want_zty = diag && y != nullptr;
  double zacc = 0.0;
  for (int64_t m0 = 0; m0 < M; m0 += KB) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t col = (h == 0 ? I0 : J0) + li;
      u16x8 hi, lo;
      // clamped addresses: every load is issued unconditionally, then masked
      const int64_t colc = col < D ? col : D - 1;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int64_t m = m0 + lk + c;
        const bool ok = m < M && col < D;
        const float zl = Z[(m < M ? m : M - 1) * D + colc];
        const float zr = ok ? zl : 0.0f;
        if (h == 0 && want_zty && ok) zacc += double(zr) * double(y[m]);
        unsigned short a, b;
        split<MODE>(zr * zscale, a, b);
        hi[c] = a;
        lo[c] = b;
      }
      if (h == 0) {
        *reinterpret_cast<u16x8*>(&sAh[li][lk]) = hi;
        if constexpr (HILO) *reinterpret_cast<u16x8*>(&sAl[li][lk]) = lo;
      } else {
        *reinterpret_cast<u16x8*>(&sBh[li][lk]) = hi;
        if constexpr (HILO) *reinterpret_cast<u16x8*>(&sBl[li][lk]) = lo;
      }
      if (diag) break;
    }
    __syncthreads();
    const unsigned short (*bh)[KP] = diag ? sAh : sBh;
    const unsigned short (*bl)[KP] = diag ? sAl : sBl;
    const int ko = 8 * (lane >> 5);
    u16x8 ah[2], bhv[2], al[2], blv[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int ra = wy * 64 + b * 32 + (lane & 31);
      const int rb = wx * 64 + b * 32 + (lane & 31);
      ah[b] = *reinterpret_cast<const u16x8*>(&sAh[ra][ko]);
      bhv[b] = *reinterpret_cast<const u16x8*>(&bh[rb][ko]);
      if constexpr (HILO) {
        al[b] = *reinterpret_cast<const u16x8*>(&sAl[ra][ko]);
        blv[b] = *reinterpret_cast<const u16x8*>(&bl[rb][ko]);
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if constexpr (MODE == kBF16 || MODE == kBF16HiLo) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(bf16x8, ah[a]), __builtin_bit_cast(bf16x8, bhv[b]), acc[a][b], 0, 0, 0);
          if constexpr (HILO) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, ah[a]), __builtin_bit_cast(bf16x8, blv[b]), acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, al[a]), __builtin_bit_cast(bf16x8, bhv[b]), acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, al[a]), __builtin_bit_cast(bf16x8, blv[b]), acc[a][b], 0, 0, 0);
          }
        } else {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
              __builtin_bit_cast(f16x8, ah[a]), __builtin_bit_cast(f16x8, bhv[b]), acc[a][b], 0, 0, 0);
          if constexpr (HILO) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                __builtin_bit_cast(f16x8, ah[a]), __builtin_bit_cast(f16x8, blv[b]), acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                __builtin_bit_cast(f16x8, al[a]), __builtin_bit_cast(f16x8, bhv[b]), acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                __builtin_bit_cast(f16x8, al[a]), __builtin_bit_cast(f16x8, blv[b]), acc[a][b], 0, 0, 0);
          }
        }
      }
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gi = I0 + wy * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t gj = J0 + wx * 64 + b * 32 + (lane & 31);
        if (gi < D && gj < D && gi >= gj) G[gi * D + gj] += acc[a][b][r] * gscale;
      }
  if (want_zty) {
    zred[lk >> 3][li] = zacc;
    __syncthreads();
    if (tid < TILE && I0 + tid < D) Zty[I0 + tid] += float(zred[0][tid] + zred[1][tid]);
  }
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
  tile_of(blockIdx.x, I, J);
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

hipError_t sorf_launch_gram(int64_t n_rows, int32_t D, const float* Z, const float* y, int mode,
                            int32_t scale_exp, float* G, float* Zty, hipStream_t st) {
  if (n_rows == 0 || D == 0) return hipSuccess;
  const int64_t nt = (D + TILE - 1) / TILE;
  const dim3 grid{unsigned(nt * (nt + 1) / 2)}, block{256};
  const float zs = std::ldexp(1.0f, scale_exp);
  const float gs = std::ldexp(1.0f, -2 * scale_exp);
  switch (mode) {
    case kFP32:
      if (D % 4 == 0)
        hipLaunchKernelGGL(gram_fp32_kernel<true>, grid, block, 0, st, Z, n_rows, D, G, y, Zty);
      else
        hipLaunchKernelGGL(gram_fp32_kernel<false>, grid, block, 0, st, Z, n_rows, D, G, y, Zty);
      break;
    case kBF16:
      hipLaunchKernelGGL(gram_half_kernel<kBF16>, grid, block, 0, st, Z, n_rows, D, zs, gs, G, y, Zty);
      break;
    case kFP16:
      hipLaunchKernelGGL(gram_half_kernel<kFP16>, grid, block, 0, st, Z, n_rows, D, zs, gs, G, y, Zty);
      break;
    case kBF16HiLo:
      hipLaunchKernelGGL(gram_half_kernel<kBF16HiLo>, grid, block, 0, st, Z, n_rows, D, zs, gs, G,
                         y, Zty);
      break;
    case kFP16HiLo:
      hipLaunchKernelGGL(gram_half_kernel<kFP16HiLo>, grid, block, 0, st, Z, n_rows, D, zs, gs, G,
                         y, Zty);
      break;
    default:
      return hipErrorInvalidValue;
  }
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
