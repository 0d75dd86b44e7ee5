// Derivative feature matrix of the force-trained normal equation (arXiv
// 2206.01580, Theory section, RFF subsection): one row per atomic coordinate,
//
//   dZ[3 a + k][s d + j] = sqrt(2/D) sum_{i in m} sin(u_{i,f}) (W_{e_i,s} J_i)[j][3 (a - a0) + k]
//
// with f = s d + j, u_i = W_{e_i} x_i + b_{e_i} the atom's phases and J_i =
// dx_i/dr_m (d x 3 N_m) the atom's Jacobian block. The rows are minus the
// coordinate derivatives of the molecule's feature row, so dZ alpha = F.
//
// Cost. Every column of every J_i goes through the SORF chain W_{e_i,s}
// (T rounds of signs and a fast Hadamard transform, SORF subsection):
// N_m * 3 N_m transforms per molecule and stack, each followed by one FMA
// per entry into the output row. The N_m phase transforms of the atoms are
// 1 / (3 N_m) of that. The work is VALU issue; J (read once from HBM) and
// dZ (written once) are small beside it.
//
// Work split. One workgroup (4 waves) per (molecule, stack). A wave holds 64 /
// K column vectors in the lane layout of the other feature kernels (K lanes
// of EPL entries each) and keeps their d output sums in registers while it
// walks the molecule's atoms, so every output row is summed in registers in
// atom order and written once (no atomics, deterministic). sin(u_i) of up to
// 4 * (64 / K) atoms is formed by the four waves together and kept in LDS;
// molecules with more atoms are processed in atom chunks, the column
// groups in lockstep.
//
// Blocks are ordered so that the S stacks of one molecule run on one XCD
// (workgroups are dispatched to the 8 XCDs round robin): the molecule's
// Jacobian block is then read from HBM into that XCD's L2 once and re-read
// by the other stacks from there.
#include <cmath>

#include "sorf_internal.h"

namespace sorf {

// Lane layout of this kernel: entry j of a d-vector sits in lane q = j % K of
// its group, register r = j / K (K = d / EPL lanes per vector). The butterfly
// stages over the register bits run in registers and those over the lane bits
// across lanes, as in the other feature kernels; the Hadamard matrix in
// natural order is unchanged by this relabelling of the index bits, since it
// relabels rows and columns alike. The point of the layout: the K sign bits
// of register r of a group are one K-bit chunk of the sign vector, and when
// every group of a wave transforms a column of the same atom (same element
// and stack), the sign mask of register r across the wave is that chunk
// repeated 64 / K times: a wave-uniform value in scalar registers, applied
// with one v_cndmask per entry.

template <int K>
__host__ __device__ constexpr uint32_t lane_repeat() {  // sum over k < 32/K of 2^(kK)
  uint32_t v = 0;
  for (int k = 0; k < 32 / K; ++k) v |= 1u << (k * K);
  return v;
}

template <int K>
__host__ __device__ constexpr uint32_t odd_lanes() {    // bit q set iff popcount(q) is odd, q < K
  uint32_t v = 0;
  for (int q = 0; q < K && q < 32; ++q)
    if (__builtin_popcount(q) & 1) v |= 1u << q;
  return v;
}

// v[r] = -v[r] where the sign bit of entry r K + q is set; `pending` also
// flips the lanes that carry the pending sign of the previous transform's
// cross-lane stages. `sw` points at the W sign words of the vector and must
// be the same for the whole wave.
template <int EPL, int K>
__device__ __forceinline__ void apply_signs_wave(float (&v)[EPL], const uint32_t* __restrict__ sw,
                                                 bool pending) {
  constexpr uint32_t KMASK = K >= 32 ? 0xFFFFFFFFu : ((1u << K) - 1u);
  constexpr uint32_t REP = lane_repeat<K>();
  constexpr uint32_t FLIP = odd_lanes<K>() * REP;
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    const uint32_t word = __builtin_amdgcn_readfirstlane(sw[(r * K) >> 5]);
    uint32_t m32 = ((word >> ((r * K) & 31)) & KMASK) * REP;
    if (pending) m32 ^= FLIP;
    const uint64_t m = (uint64_t(m32) << 32) | m32;
    asm("v_cndmask_b32_e64 %0, %1, -%1, %2" : "=v"(v[r]) : "v"(v[r]), "s"(m));
  }
}

// The same for a lane group whose vector differs from the other groups'.
// `flip` is 0x80000000 on lanes that carry a pending sign, else 0.
template <int EPL, int K>
__device__ __forceinline__ void apply_signs_group(float (&v)[EPL], const uint32_t* __restrict__ sw,
                                                  uint32_t q, uint32_t flip) {
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    const uint32_t bit = (sw[(r * K) >> 5] >> (((r * K) & 31) + q)) << 31;
    v[r] = __uint_as_float(__float_as_uint(v[r]) ^ bit ^ flip);
  }
}

template <int LOG_D, int LOG_EPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void dz_kernel(
    const float* __restrict__ x, const int32_t* __restrict__ element,
    const int64_t* __restrict__ mol_ptr, const uint32_t* __restrict__ signs,
    const float* __restrict__ bias, const float* __restrict__ J, const int64_t* __restrict__ J_ptr,
    float* __restrict__ dZ, int64_t m_begin, int64_t m_end, int32_t S, int32_t T, float c_rev,
    float out_scale) {
  constexpr int DV = 1 << LOG_D;
  constexpr int EPL = 1 << LOG_EPL;
  constexpr int LOGK = LOG_D - LOG_EPL;
  constexpr int K = 1 << LOGK;                       // lanes per vector
  constexpr int VPW = 64 >> LOGK;                    // column vectors per wave
  constexpr int W = (DV + 31) / 32;                  // sign words per vector
  constexpr int PADL = EPL % 4 == 0 ? EPL + 4 : EPL; // LDS stride of one lane's share
  constexpr int ROW = K * PADL;                      // LDS floats per atom
  constexpr int CH = 4 * VPW;                        // atoms per LDS chunk
  __shared__ __attribute__((aligned(16))) float sinbuf[CH * ROW];

  // block -> (molecule, stack): the S blocks of a molecule share blockIdx.x % 8
  const int64_t b = blockIdx.x;
  const int64_t rr = b >> 3;
  const int64_t m = m_begin + (rr / S) * 8 + (b & 7);
  const int32_t s = int32_t(rr % S);
  if (m >= m_end) return;
  const int64_t a0 = mol_ptr[m];
  const int64_t n = mol_ptr[m + 1] - a0;
  if (n <= 0) return;

  const int wv = int(threadIdx.x >> 6);
  const uint32_t lane = lane_id();
  const uint32_t q = lane & (K - 1u);
  const int g = int(lane >> LOGK);
  const bool odd = (__builtin_popcount(q) & 1) != 0;
  const uint32_t flip = odd ? 0x80000000u : 0u;  // pending sign after cross-lane stages
  const float c_lane = odd ? -c_rev : c_rev;
  const float o_lane = odd ? -out_scale : out_scale;
  const int64_t Dtot = int64_t(S) * DV;
  const int64_t tstride = int64_t(S) * W;
  const int64_t ncol = 3 * n;
  const float* __restrict__ jm = J + J_ptr[m];
  const int64_t n_cg = (ncol + VPW - 1) / VPW;

  // sin(u_i) of atoms i0 .. i0 + CH - 1 into LDS (atom i0 + wv VPW + g per group;
  // groups past the molecule's end repeat its last atom and store nothing)
  auto sin_chunk = [&](int64_t i0) {
    const int64_t i = i0 + wv * VPW + g;
    const int64_t a = a0 + (i < n ? i : n - 1);
    const int32_t e = element[a];
    const float* xa = x + a * DV + q;
    float v[EPL];
#pragma unroll
    for (int r = 0; r < EPL; ++r) v[r] = xa[r * K];
    const uint32_t* sv = signs + (int64_t(e) * T * S + s) * W;
    for (int t = 0; t < T; ++t) {
      apply_signs_group<EPL, K>(v, sv + t * tstride, q, t > 0 ? flip : 0u);
      fwht<LOGK, EPL>(v, q);
    }
    const float* bp = bias + int64_t(e) * Dtot + int64_t(s) * DV + q;
#pragma unroll
    for (int r = 0; r < EPL; ++r)
      v[r] = __builtin_amdgcn_sinf(__builtin_fmaf(v[r], c_lane, bp[r * K] * kInv2Pi));
    if (i < n) {
      float* dst = sinbuf + (wv * VPW + g) * ROW + q * PADL;
      if constexpr (EPL % 4 == 0) {
#pragma unroll
        for (int r = 0; r < EPL; r += 4)
          *reinterpret_cast<float4*>(dst + r) = make_float4(v[r], v[r + 1], v[r + 2], v[r + 3]);
      } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r) dst[r] = v[r];
      }
    }
  };

  // acc += sin(u_i) * (W_{e_i,s} J_i[:, col]) over atoms i0 .. i1 - 1 (LDS chunk at i0).
  // Every group of the wave takes the same atom, so the sign masks and the row
  // base of each J load are wave-uniform; only the lane's row and column vary.
  auto col_pass = [&](int64_t cg, int64_t i0, int64_t i1, float (&acc)[EPL]) {
    const int64_t col = cg * VPW + g;
    const int64_t colc = col < ncol ? col : ncol - 1;
    // the atom's block through a buffer descriptor: the wave-uniform row offset
    // of each load goes in a scalar register, so loads need no address VALU
    const uint32_t vofs = uint32_t((int64_t(q) * ncol + colc) * 4);   // bytes
    // (a block below 2^32 bytes, d * 3 N_m * 4, as the interface requires)
    const uint32_t blk_bytes = uint32_t(int64_t(DV) * ncol * 4);
    const uint32_t row_bytes = uint32_t(int64_t(K) * ncol * 4);
    for (int64_t i = i0; i < i1; ++i) {
      const int32_t e = __builtin_amdgcn_readfirstlane(element[a0 + i]);
      const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(jm + i * DV * ncol), int16_t(0), int32_t(blk_bytes), 0x00020000);
      float v[EPL];
#pragma unroll
      for (int r = 0; r < EPL; ++r)
        v[r] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc, vofs, r * row_bytes, 0));
      const uint32_t* sv = signs + (int64_t(e) * T * S + s) * W;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        if (t < T) {
          apply_signs_wave<EPL, K>(v, sv + t * tstride, t > 0);
          fwht<LOGK, EPL>(v, q);
        }
      }
      const float* sp = sinbuf + (i - i0) * ROW + q * PADL;
      if constexpr (EPL % 4 == 0) {
#pragma unroll
        for (int r = 0; r < EPL; r += 4) {
          const float4 sn = *reinterpret_cast<const float4*>(sp + r);
          acc[r] = __builtin_fmaf(sn.x, v[r], acc[r]);
          acc[r + 1] = __builtin_fmaf(sn.y, v[r + 1], acc[r + 1]);
          acc[r + 2] = __builtin_fmaf(sn.z, v[r + 2], acc[r + 2]);
          acc[r + 3] = __builtin_fmaf(sn.w, v[r + 3], acc[r + 3]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < EPL; ++r) acc[r] = __builtin_fmaf(sp[r], v[r], acc[r]);
      }
    }
  };

  auto store_row = [&](int64_t cg, const float (&acc)[EPL]) {
    const int64_t col = cg * VPW + g;
    if (col < ncol) {
      float* out = dZ + (3 * a0 + col) * Dtot + int64_t(s) * DV + q;
#pragma unroll
      for (int r = 0; r < EPL; ++r) out[r * K] = acc[r] * o_lane;
    }
  };

  if (n <= CH) {
    sin_chunk(0);
    __syncthreads();
    for (int64_t cg = wv; cg < n_cg; cg += 4) {
      float acc[EPL];
#pragma unroll
      for (int r = 0; r < EPL; ++r) acc[r] = 0.0f;
      col_pass(cg, 0, n, acc);
      store_row(cg, acc);
    }
  } else {
    for (int64_t cg0 = 0; cg0 < n_cg; cg0 += 4) {
      const int64_t cg = cg0 + wv;
      float acc[EPL];
#pragma unroll
      for (int r = 0; r < EPL; ++r) acc[r] = 0.0f;
      for (int64_t i0 = 0; i0 < n; i0 += CH) {
        __syncthreads();  // the previous chunk's sin values are no longer read
        sin_chunk(i0);
        __syncthreads();
        if (cg < n_cg) col_pass(cg, i0, i0 + CH < n ? i0 + CH : n, acc);
      }
      if (cg < n_cg) store_row(cg, acc);
    }
  }
}

template <int LOG_D>
static hipError_t dz_dispatch(const SorfFeatureArgs& a, const float* J, const int64_t* J_ptr,
                              float* dZ, hipStream_t st) {
  constexpr int LOG_EPL = LOG_D < 5 ? LOG_D : 5;
  const double D = double(a.d) * a.n_stacks;
  const double c = std::sqrt(double(a.d)) / double(a.sigma) *
                   std::pow(double(a.d), -0.5 * a.n_transforms);
  const float c_f = float(c);  // the same rounded c as the other feature kernels
  const float c_rev = float(double(c_f) * (1.0 / (2.0 * M_PI)));
  const float out_scale = float(double(c_f) * std::sqrt(2.0 / D));
  // at most 2^30 blocks per launch
  const int64_t per_launch = ((int64_t(1) << 27) / a.n_stacks) * 8;
  for (int64_t m0 = 0; m0 < a.n_mols; m0 += per_launch) {
    const int64_t m1 = m0 + per_launch < a.n_mols ? m0 + per_launch : a.n_mols;
    const int64_t blocks = ((m1 - m0 + 7) / 8) * 8 * a.n_stacks;
    hipLaunchKernelGGL((dz_kernel<LOG_D, LOG_EPL>), dim3(unsigned(blocks)), dim3(256), 0, st,
                       a.x, a.element, a.mol_ptr, a.signs, a.bias, J, J_ptr, dZ, m0, m1,
                       a.n_stacks, a.n_transforms, c_rev, out_scale);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace sorf

using namespace sorf;

hipError_t sorf_launch_dz(const SorfFeatureArgs& a, const float* J, const int64_t* J_ptr,
                          float* dZ, hipStream_t st) {
  if (a.n_mols == 0 || a.n_atoms == 0) return hipSuccess;
  switch (a.d) {
    case 2: return dz_dispatch<1>(a, J, J_ptr, dZ, st);
    case 4: return dz_dispatch<2>(a, J, J_ptr, dZ, st);
    case 8: return dz_dispatch<3>(a, J, J_ptr, dZ, st);
    case 16: return dz_dispatch<4>(a, J, J_ptr, dZ, st);
    case 32: return dz_dispatch<5>(a, J, J_ptr, dZ, st);
    case 64: return dz_dispatch<6>(a, J, J_ptr, dZ, st);
    case 128: return dz_dispatch<7>(a, J, J_ptr, dZ, st);
    case 256: return dz_dispatch<8>(a, J, J_ptr, dZ, st);
    case 512: return dz_dispatch<9>(a, J, J_ptr, dZ, st);
    case 1024: return dz_dispatch<10>(a, J, J_ptr, dZ, st);
    default: return hipErrorInvalidValue;
  }
}
