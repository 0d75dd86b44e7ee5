// SORF feature kernels for gfx950: forward features (Z), the per-atom adjoint
// (dE/dx and per-atom energies) and the per-molecule reduction that turns
// per-atom results into energies and forces.
//
// Paper: arXiv 2206.01580, Theory section (RFF feature map, atomic energy
// decomposition, derivative features) and SORF subsection (W ~ (sqrt(d)/sigma)
// [H_i D_i]_{N_transform}, stacked N_F/d times, fast Hadamard transform).
//
// Work split. sorf_forward: one lane group per (molecule, stack); the group
// walks the molecule's atoms and keeps the stack's d running sums of cos in
// registers, so the atom->molecule sum needs no atomics and no second pass and
// Z is written once, coalesced per lane (EPL contiguous floats).
// Adjoint: one wave per atom; its lane groups cover the stacks in passes and
// the stack sum is a wave reduction at the end.
#include <cmath>

#include "sorf_internal.h"

namespace sorf {

// ---------------------------------------------------------------------------
// Forward features
// ---------------------------------------------------------------------------
template <int LOG_D, int LOG_EPL>
__global__ __launch_bounds__(256) void forward_kernel(
    const float* __restrict__ x, const int32_t* __restrict__ element,
    const int64_t* __restrict__ mol_ptr, const uint32_t* __restrict__ signs,
    const float* __restrict__ bias, float* __restrict__ Z, int64_t n_mols, int32_t S, int32_t T,
    float c_rev, float out_scale) {
  constexpr int DV = 1 << LOG_D;
  constexpr int EPL = 1 << LOG_EPL;
  constexpr int LOGK = LOG_D - LOG_EPL;
  constexpr int VPW = 64 >> LOGK;               // vectors per wave
  constexpr int W = (DV + 31) / 32;             // sign words per vector
  constexpr int LW = EPL >= 32 ? EPL / 32 : 1;  // sign words per lane

  const uint32_t lane = lane_id();
  const uint32_t q = lane & ((1u << LOGK) - 1u);
  const uint32_t grp = lane >> LOGK;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t item = wave * VPW + grp;
  if (item >= n_mols * int64_t(S)) return;  // whole lane groups leave together
  const int64_t m = item / S;
  const int32_t s = int32_t(item - m * S);
  const int64_t a0 = mol_ptr[m];
  const int64_t a1 = mol_ptr[m + 1];
  const int64_t Dtot = int64_t(S) * DV;

  const bool odd = (__builtin_popcount(q) & 1) != 0;
  const uint32_t flip = odd ? 0xFFFFFFFFu : 0u;      // pending sign after cross-lane stages
  const float c_lane = odd ? -c_rev : c_rev;
  const int64_t tstride = int64_t(S) * W;

  float acc[EPL];
#pragma unroll
  for (int r = 0; r < EPL; ++r) acc[r] = 0.0f;

  for (int64_t a = a0; a < a1; ++a) {
    const int32_t e = element[a];
    float v[EPL];
    load_vec<EPL>(v, x + a * DV + q * EPL);
    const uint32_t* sv = signs + (int64_t(e) * T * S + s) * W;
    for (int t = 0; t < T; ++t) {
      uint32_t w[LW];
      load_sign_words<EPL>(w, sv + t * tstride, q, t > 0 ? flip : 0u);
      apply_signs<EPL>(v, w);
      fwht<LOGK, EPL>(v, q);
    }
    float b[EPL];
    load_vec<EPL>(b, bias + int64_t(e) * Dtot + int64_t(s) * DV + q * EPL);
#pragma unroll
    for (int r = 0; r < EPL; ++r) {
      const float u = __builtin_fmaf(v[r], c_lane, b[r] * kInv2Pi);  // phase in revolutions
      acc[r] += __builtin_amdgcn_cosf(u);
    }
  }
  store_vec<EPL>(Z + m * Dtot + int64_t(s) * DV + q * EPL, acc, out_scale);
}

// ---------------------------------------------------------------------------
// Per-atom adjoint: dE/dx_i (and the atom's energy share)
// ---------------------------------------------------------------------------
template <int LOG_D, int LOG_EPL, bool WANT_E, bool WANT_G>
__global__ __launch_bounds__(256) void atom_adjoint_kernel(
    const float* __restrict__ x, const int32_t* __restrict__ element,
    const int64_t* __restrict__ mol_ptr, const uint32_t* __restrict__ signs,
    const float* __restrict__ bias, const float* __restrict__ alpha,
    const float* __restrict__ dE, float* __restrict__ grad_x, float* __restrict__ e_atom,
    int64_t n_atoms, int64_t n_mols, int32_t S, int32_t T, float c_rev, float g_scale,
    float e_scale) {
  constexpr int DV = 1 << LOG_D;
  constexpr int EPL = 1 << LOG_EPL;
  constexpr int LOGK = LOG_D - LOG_EPL;
  constexpr int VPW = 64 >> LOGK;
  constexpr int W = (DV + 31) / 32;
  constexpr int LW = EPL >= 32 ? EPL / 32 : 1;

  const uint32_t lane = lane_id();
  const uint32_t q = lane & ((1u << LOGK) - 1u);
  const uint32_t grp = lane >> LOGK;
  const int64_t a = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (a >= n_atoms) return;  // whole waves leave together

  const int32_t e = element[a];
  const int64_t Dtot = int64_t(S) * DV;
  const bool odd = (__builtin_popcount(q) & 1) != 0;
  const uint32_t flip = odd ? 0xFFFFFFFFu : 0u;
  const float c_lane = odd ? -c_rev : c_rev;
  const int64_t tstride = int64_t(S) * W;

  float xin[EPL];
  load_vec<EPL>(xin, x + a * DV + q * EPL);

  float gacc[EPL];
#pragma unroll
  for (int r = 0; r < EPL; ++r) gacc[r] = 0.0f;
  float eacc = 0.0f;

  for (int32_t s0 = 0; s0 < S; s0 += VPW) {
    const int32_t s = s0 + int32_t(grp);
    if (s < S) {
      float v[EPL];
#pragma unroll
      for (int r = 0; r < EPL; ++r) v[r] = xin[r];
      const uint32_t* sv = signs + (int64_t(e) * T * S + s) * W;
      for (int t = 0; t < T; ++t) {
        uint32_t w[LW];
        load_sign_words<EPL>(w, sv + t * tstride, q, t > 0 ? flip : 0u);
        apply_signs<EPL>(v, w);
        fwht<LOGK, EPL>(v, q);
      }
      float b[EPL], al[EPL];
      load_vec<EPL>(b, bias + int64_t(e) * Dtot + int64_t(s) * DV + q * EPL);
      load_vec<EPL>(al, alpha + int64_t(s) * DV + q * EPL);
#pragma unroll
      for (int r = 0; r < EPL; ++r) {
        const float u = __builtin_fmaf(v[r], c_lane, b[r] * kInv2Pi);
        if constexpr (WANT_E) eacc = __builtin_fmaf(al[r], __builtin_amdgcn_cosf(u), eacc);
        if constexpr (WANT_G) v[r] = al[r] * __builtin_amdgcn_sinf(u);
      }
      if constexpr (WANT_G) {
        // transposed chain: H first, then D_{T-1}, ..., H, then D_0
        for (int t = T - 1; t >= 0; --t) {
          fwht<LOGK, EPL>(v, q);
          uint32_t w[LW];
          load_sign_words<EPL>(w, sv + t * tstride, q, flip);
          apply_signs<EPL>(v, w);
        }
#pragma unroll
        for (int r = 0; r < EPL; ++r) gacc[r] += v[r];
      }
    }
  }

  if constexpr (WANT_G) {
    // sum over the lane groups (stacks) of the wave: lane bits LOGK .. 5
    if constexpr (LOGK <= 0) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<0>(gacc[r]); }
    if constexpr (LOGK <= 1) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<1>(gacc[r]); }
    if constexpr (LOGK <= 2) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<2>(gacc[r]); }
    if constexpr (LOGK <= 3) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<3>(gacc[r]); }
    if constexpr (LOGK <= 4) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<4>(gacc[r]); }
    if constexpr (LOGK <= 5) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<5>(gacc[r]); }
    if (grp == 0) {
      float w_m = 1.0f;
      if (dE != nullptr) w_m = dE[molecule_of(mol_ptr, n_mols, a)];
      store_vec<EPL>(grad_x + a * DV + q * EPL, gacc, g_scale * w_m);
    }
  }
  if constexpr (WANT_E) {
    eacc += lane_xor<0>(eacc);
    eacc += lane_xor<1>(eacc);
    eacc += lane_xor<2>(eacc);
    eacc += lane_xor<3>(eacc);
    eacc += lane_xor<4>(eacc);
    eacc += lane_xor<5>(eacc);
    if (lane == 0) e_atom[a] = eacc * e_scale;
  }
}

// ---------------------------------------------------------------------------
// Per-molecule reduction: E_m = sum of the atoms' shares; F = -sum_i J_i^T g_i
// grid.x = molecule, grid.y strides over 64-column blocks of the molecule's
// 3 N_m force components; the four waves split the N_m * d Jacobian rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void molecule_reduce_kernel(
    const int64_t* __restrict__ mol_ptr, const float* __restrict__ e_atom,
    const float* __restrict__ grad, const float* __restrict__ J, const int64_t* __restrict__ J_ptr,
    float* __restrict__ E, float* __restrict__ F, int32_t d) {
  __shared__ float red[4][64];
  const int64_t m = blockIdx.x;
  const int64_t a0 = mol_ptr[m];
  const int64_t n = mol_ptr[m + 1] - a0;
  if (blockIdx.y == 0 && threadIdx.x == 0 && E != nullptr) {
    float s = 0.0f;
    for (int64_t i = 0; i < n; ++i) s += e_atom[a0 + i];
    E[m] = s;
  }
  if (J == nullptr || n == 0) return;
  const int64_t ncol = 3 * n;
  const int64_t rows = n * d;
  const float* __restrict__ blk = J + J_ptr[m];
  const float* __restrict__ g = grad + a0 * d;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  for (int64_t cb = blockIdx.y; cb * 64 < ncol; cb += gridDim.y) {
    const int64_t col = cb * 64 + lane;
    const bool ok = col < ncol;
    float acc = 0.0f;
    int64_t r = wv;
    for (; r + 12 < rows; r += 16) {
      float j0 = 0, j1 = 0, j2 = 0, j3 = 0;
      if (ok) {
        j0 = blk[(r + 0) * ncol + col];
        j1 = blk[(r + 4) * ncol + col];
        j2 = blk[(r + 8) * ncol + col];
        j3 = blk[(r + 12) * ncol + col];
      }
      acc = __builtin_fmaf(j0, g[r + 0], acc);
      acc = __builtin_fmaf(j1, g[r + 4], acc);
      acc = __builtin_fmaf(j2, g[r + 8], acc);
      acc = __builtin_fmaf(j3, g[r + 12], acc);
    }
    for (; r < rows; r += 4) {
      const float jv = ok ? blk[r * ncol + col] : 0.0f;
      acc = __builtin_fmaf(jv, g[r], acc);
    }
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && ok) {
      F[3 * a0 + col] = -(((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
    }
    __syncthreads();
  }
}

__global__ void validate_kernel(const int64_t* __restrict__ mol_ptr,
                                const int32_t* __restrict__ element, int64_t n_atoms,
                                int64_t n_mols, int32_t n_elements, int32_t* __restrict__ result) {
  __shared__ int32_t flags;
  if (threadIdx.x == 0) flags = 0;
  __syncthreads();
  int32_t f = 0;
  if (threadIdx.x == 0) {
    if (mol_ptr[0] != 0) f |= 1;
    if (mol_ptr[n_mols] != n_atoms) f |= 4;
  }
  for (int64_t m = threadIdx.x; m < n_mols; m += blockDim.x)
    if (mol_ptr[m + 1] < mol_ptr[m]) f |= 2;
  for (int64_t i = threadIdx.x; i < n_atoms; i += blockDim.x) {
    const int32_t e = element[i];
    if (e < 0 || e >= n_elements) f |= 8;
  }
  if (f) atomicOr(&flags, f);
  __syncthreads();
  if (threadIdx.x == 0) *result = flags;
}

__global__ void fill_kernel(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// Dispatch on d (compile-time lane layout per d)
// ---------------------------------------------------------------------------
template <int LOG_D>
constexpr int default_log_epl() {
  return LOG_D < 5 ? LOG_D : 5;  // 32 entries per lane, d/32 lanes per vector
}

inline float sorf_c(const SorfFeatureArgs& a) {
  // c = (sqrt(d)/sigma) * d^(-T/2), computed in double then rounded once
  return float(std::sqrt(double(a.d)) / double(a.sigma) * std::pow(double(a.d), -0.5 * a.n_transforms));
}

template <int LOG_D>
static hipError_t forward_dispatch(const SorfFeatureArgs& a, float* Z, hipStream_t st) {
  constexpr int LOG_EPL = default_log_epl<LOG_D>();
  constexpr int VPW = 64 >> (LOG_D - LOG_EPL);
  const int64_t items = a.n_mols * int64_t(a.n_stacks);
  const int64_t waves = (items + VPW - 1) / VPW;
  const int64_t blocks = (waves + 3) / 4;
  const double D = double(a.d) * a.n_stacks;
  const float c_rev = float(double(sorf_c(a)) * (1.0 / (2.0 * M_PI)));
  hipLaunchKernelGGL((forward_kernel<LOG_D, LOG_EPL>), dim3(unsigned(blocks)), dim3(256), 0, st,
                     a.x, a.element, a.mol_ptr, a.signs, a.bias, Z, a.n_mols, a.n_stacks,
                     a.n_transforms, c_rev, float(std::sqrt(2.0 / D)));
  return hipGetLastError();
}

template <int LOG_D>
static hipError_t adjoint_dispatch(const SorfFeatureArgs& a, const float* alpha, const float* dE,
                                   float* grad_x, float* e_atom, hipStream_t st) {
  constexpr int LOG_EPL = default_log_epl<LOG_D>();
  const int64_t blocks = (a.n_atoms + 3) / 4;
  const double D = double(a.d) * a.n_stacks;
  const double c = double(sorf_c(a));
  const float c_rev = float(c * (1.0 / (2.0 * M_PI)));
  const float g_scale = float(-std::sqrt(2.0 / D) * c);
  const float e_scale = float(std::sqrt(2.0 / D));
  const dim3 grid{unsigned(blocks)}, block{256};
#define SORF_ADJ(WE, WG)                                                                        \
  hipLaunchKernelGGL((atom_adjoint_kernel<LOG_D, LOG_EPL, WE, WG>), grid, block, 0, st, a.x,   \
                     a.element, a.mol_ptr, a.signs, a.bias, alpha, dE, grad_x, e_atom,        \
                     a.n_atoms, a.n_mols, a.n_stacks, a.n_transforms, c_rev, g_scale, e_scale)
  if (e_atom && grad_x) SORF_ADJ(true, true);
  else if (e_atom) SORF_ADJ(true, false);
  else SORF_ADJ(false, true);
#undef SORF_ADJ
  return hipGetLastError();
}

}  // namespace sorf

using namespace sorf;

#define SORF_LOGD_SWITCH(LOGD, CALL) \
  switch (LOGD) {                    \
    case 1: return CALL(1);          \
    case 2: return CALL(2);          \
    case 3: return CALL(3);          \
    case 4: return CALL(4);          \
    case 5: return CALL(5);          \
    case 6: return CALL(6);          \
    case 7: return CALL(7);          \
    case 8: return CALL(8);          \
    case 9: return CALL(9);          \
    case 10: return CALL(10);        \
    default: return hipErrorInvalidValue; \
  }

static int log2i(int d) {
  int l = 0;
  while ((1 << l) < d) ++l;
  return l;
}

hipError_t sorf_launch_forward(const SorfFeatureArgs& a, float* Z, hipStream_t st) {
  if (a.n_mols == 0) return hipSuccess;
#define CALL(L) forward_dispatch<L>(a, Z, st)
  SORF_LOGD_SWITCH(log2i(a.d), CALL)
#undef CALL
}

hipError_t sorf_launch_atom_adjoint(const SorfFeatureArgs& a, const float* alpha, const float* dE,
                                    float* grad_x, float* e_atom, hipStream_t st) {
  if (a.n_atoms == 0) return hipSuccess;
#define CALL(L) adjoint_dispatch<L>(a, alpha, dE, grad_x, e_atom, st)
  SORF_LOGD_SWITCH(log2i(a.d), CALL)
#undef CALL
}

hipError_t sorf_launch_molecule_reduce(const SorfFeatureArgs& a, const float* e_atom,
                                       const float* grad, const float* J, const int64_t* J_ptr,
                                       float* E, float* F, hipStream_t st) {
  if (a.n_mols == 0) return hipSuccess;
  unsigned gy = 1;
  if (J != nullptr) {
    const int64_t want = 2048 / (a.n_mols > 0 ? a.n_mols : 1);
    gy = unsigned(want < 1 ? 1 : (want > 16 ? 16 : want));
  }
  hipLaunchKernelGGL(molecule_reduce_kernel, dim3(unsigned(a.n_mols), gy), dim3(256), 0, st,
                     a.mol_ptr, e_atom, grad, J, J_ptr, E, F, a.d);
  return hipGetLastError();
}

hipError_t sorf_launch_validate(const SorfFeatureArgs& a, int32_t* result, hipStream_t st) {
  hipLaunchKernelGGL(validate_kernel, dim3(1), dim3(1024), 0, st, a.mol_ptr, a.element, a.n_atoms,
                     a.n_mols, a.n_elements, result);
  return hipGetLastError();
}

hipError_t sorf_launch_fill(float* p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
