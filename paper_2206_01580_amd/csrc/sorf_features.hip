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
// Z is written once, coalesced per lane (EPL contiguous floats). Energies
// without forces use the same kernel with the dot product against alpha in
// place of the store (one partial per molecule and stack).
// Adjoint: one wave per atom; its lane groups cover the stacks in passes and
// the stack sum is a wave reduction at the end.
#include <cmath>

#include "sorf_internal.h"

namespace sorf {

// LDS writes of a wave visible to all its lanes (no workgroup barrier)
__device__ __forceinline__ void lds_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Forward features
// ---------------------------------------------------------------------------
// With DOT, the group does not store its features: it writes the stack's
// share of the molecule's energy, part[m S + s] = sum_f alpha_f z_f over the
// stack's features, summed over the group's lanes in a fixed order.
// SHARED (the stack count a multiple of the groups per wave, so that all
// groups of a wave walk the same molecule): the wave loads the next atom's x
// row cooperatively (d / 64 floats per lane) while it transforms the current
// one, and parks it in a double-buffered LDS row that the groups read from.
template <int LOG_D, int LOG_EPL, bool DOT, bool SHARED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void forward_kernel(
    const float* __restrict__ x, const int32_t* __restrict__ element,
    const int64_t* __restrict__ mol_ptr, const uint32_t* __restrict__ signs,
    const float* __restrict__ bias, float* __restrict__ Z, const float* __restrict__ alpha,
    int64_t n_mols, int32_t S, int32_t T, float c_rev, float out_scale) {
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

  constexpr int XR = SHARED ? DV / 64 : 1;   // floats of a row per lane
  __shared__ float xrow[SHARED ? 4 : 1][2][SHARED ? DV : 1];
  const int wv = int(threadIdx.x >> 6);
  if constexpr (SHARED) {
    if (a0 < a1) {
#pragma unroll
      for (int i = 0; i < XR; ++i) xrow[wv][0][lane + 64 * i] = x[a0 * DV + lane + 64 * i];
      lds_wave_sync();
    }
  }
  // the next atom's element is read one atom ahead, and all T sign words of
  // an atom are requested before its first transform
  int32_t e_next = a0 < a1 ? element[a0] : 0;
  for (int64_t a = a0; a < a1; ++a) {
    const int32_t e = e_next;
    if (a + 1 < a1) e_next = element[a + 1];
    float v[EPL];
    float xn[XR];
    const int buf = int(a - a0) & 1;
    if constexpr (SHARED) {
#pragma unroll
      for (int r = 0; r < EPL; ++r) v[r] = xrow[wv][buf][q * EPL + r];
    } else {
      load_vec<EPL>(v, x + a * DV + q * EPL);
    }
    const uint32_t* sv = signs + (int64_t(e) * T * S + s) * W;
    uint32_t w[3][LW];
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (t < T) load_sign_words<EPL>(w[t], sv + t * tstride, q, t > 0 ? flip : 0u);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if (t < T) {
        apply_signs<EPL>(v, w[t]);
        fwht<LOGK, EPL>(v, q);
      }
    }
    // the next atom's row is requested here, to arrive during the cosines
    if constexpr (SHARED) {
      if (a + 1 < a1) {
#pragma unroll
        for (int i = 0; i < XR; ++i) xn[i] = x[(a + 1) * DV + lane + 64 * i];
      }
    }
    // bias in chunks of (at most) 8 entries, so that few of them are live at once
    constexpr int CH = EPL < 8 ? EPL : 8;
    const float* bp = bias + int64_t(e) * Dtot + int64_t(s) * DV + q * EPL;
#pragma unroll
    for (int r0 = 0; r0 < EPL; r0 += CH) {
      float b[CH];
      load_vec<CH>(b, bp + r0);
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        const float u = __builtin_fmaf(v[r0 + r], c_lane, b[r] * kInv2Pi);  // phase in revolutions
        acc[r0 + r] += __builtin_amdgcn_cosf(u);
      }
    }
    if constexpr (SHARED) {
      // the next atom's row goes to the other buffer, whose last reads (one
      // atom ago) are behind the previous sync
      if (a + 1 < a1) {
#pragma unroll
        for (int i = 0; i < XR; ++i) xrow[wv][buf ^ 1][lane + 64 * i] = xn[i];
      }
      lds_wave_sync();
    }
  }
  if constexpr (DOT) {
    float al[EPL];
    load_vec<EPL>(al, alpha + int64_t(s) * DV + q * EPL);
    float p = 0.0f;
#pragma unroll
    for (int r = 0; r < EPL; ++r) p = __builtin_fmaf(al[r], acc[r], p);
    if constexpr (LOGK > 0) p += lane_xor<0>(p);
    if constexpr (LOGK > 1) p += lane_xor<1>(p);
    if constexpr (LOGK > 2) p += lane_xor<2>(p);
    if constexpr (LOGK > 3) p += lane_xor<3>(p);
    if constexpr (LOGK > 4) p += lane_xor<4>(p);
    if constexpr (LOGK > 5) p += lane_xor<5>(p);
    if (q == 0) Z[m * S + s] = p * out_scale;
  } else {
    store_vec<EPL>(Z + m * Dtot + int64_t(s) * DV + q * EPL, acc, out_scale);
  }
}

// E[m] = sum over the stacks of part[m S + s], in stack order.
__global__ __launch_bounds__(256) void energy_sum_kernel(const float* __restrict__ part,
                                                        int64_t n_mols, int32_t S,
                                                        float* __restrict__ E) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= n_mols) return;
  float e = 0.0f;
  for (int32_t s = 0; s < S; ++s) e += part[m * S + s];
  E[m] = e;
}

// ---------------------------------------------------------------------------
// Per-atom adjoint: dE/dx_i (and the atom's energy share)
// ---------------------------------------------------------------------------
// The stacks s = s_begin, s_begin + s_step, ... of atom a (element e) for the
// lane group grp of a wave (lane q inside the group): the forward chain, the
// phase, the energy share sum_f alpha_f cos(u_f) into eacc and, for the
// gradient, alpha_f sin(u_f) taken back through the transposed chain and
// added into gacc (per lane, before any sum over the groups).
template <int LOG_D, int LOG_EPL, bool WANT_E, bool WANT_G>
__device__ __forceinline__ void adjoint_stacks(const float* __restrict__ xrow,
                                               const uint32_t* __restrict__ signs_e,
                                               const float* __restrict__ bias_e,
                                               const float* __restrict__ alpha, int32_t S,
                                               int32_t T, int32_t s_begin, int32_t s_step,
                                               uint32_t q, uint32_t grp, float c_rev,
                                               float (&gacc)[1 << LOG_EPL], float& eacc) {
  constexpr int DV = 1 << LOG_D;
  constexpr int EPL = 1 << LOG_EPL;
  constexpr int LOGK = LOG_D - LOG_EPL;
  constexpr int W = (DV + 31) / 32;
  constexpr int LW = EPL >= 32 ? EPL / 32 : 1;
  const bool odd = (__builtin_popcount(q) & 1) != 0;
  const uint32_t flip = odd ? 0xFFFFFFFFu : 0u;
  const float c_lane = odd ? -c_rev : c_rev;
  const int64_t tstride = int64_t(S) * W;
  for (int32_t s0 = s_begin; s0 < S; s0 += s_step) {
    const int32_t s = s0 + int32_t(grp);
    if (s < S) {
      float v[EPL];
      load_vec<EPL>(v, xrow);
      const uint32_t* sv = signs_e + int64_t(s) * W;
      for (int t = 0; t < T; ++t) {
        uint32_t w[LW];
        load_sign_words<EPL>(w, sv + t * tstride, q, t > 0 ? flip : 0u);
        apply_signs<EPL>(v, w);
        fwht<LOGK, EPL>(v, q);
      }
      // bias and alpha in chunks of (at most) 8 entries, so that few of them
      // are live at once
      constexpr int CH = EPL < 8 ? EPL : 8;
      const float* bp = bias_e + int64_t(s) * DV + q * EPL;
      const float* ap = alpha + int64_t(s) * DV + q * EPL;
#pragma unroll
      for (int r0 = 0; r0 < EPL; r0 += CH) {
        float b[CH], al[CH];
        load_vec<CH>(b, bp + r0);
        load_vec<CH>(al, ap + r0);
#pragma unroll
        for (int r = 0; r < CH; ++r) {
          const float u = __builtin_fmaf(v[r0 + r], c_lane, b[r] * kInv2Pi);
          if constexpr (WANT_E) eacc = __builtin_fmaf(al[r], __builtin_amdgcn_cosf(u), eacc);
          if constexpr (WANT_G) v[r0 + r] = al[r] * __builtin_amdgcn_sinf(u);
        }
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
}

// Sum of gacc over the lane groups of a wave (lane bits LOGK .. 5) and of
// eacc over all its lanes, in a fixed order.
template <int LOGK, int EPL, bool WANT_E, bool WANT_G>
__device__ __forceinline__ void adjoint_wave_sums(float (&gacc)[EPL], float& eacc) {
  if constexpr (WANT_G) {
    if constexpr (LOGK <= 0) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<0>(gacc[r]); }
    if constexpr (LOGK <= 1) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<1>(gacc[r]); }
    if constexpr (LOGK <= 2) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<2>(gacc[r]); }
    if constexpr (LOGK <= 3) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<3>(gacc[r]); }
    if constexpr (LOGK <= 4) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<4>(gacc[r]); }
    if constexpr (LOGK <= 5) { for (int r = 0; r < EPL; ++r) gacc[r] += lane_xor<5>(gacc[r]); }
  }
  if constexpr (WANT_E) {
    eacc += lane_xor<0>(eacc);
    eacc += lane_xor<1>(eacc);
    eacc += lane_xor<2>(eacc);
    eacc += lane_xor<3>(eacc);
    eacc += lane_xor<4>(eacc);
    eacc += lane_xor<5>(eacc);
  }
}

// One wave per atom: its lane groups cover the stacks in passes of VPW.
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

  const uint32_t lane = lane_id();
  const uint32_t q = lane & ((1u << LOGK) - 1u);
  const uint32_t grp = lane >> LOGK;
  const int64_t a = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (a >= n_atoms) return;  // whole waves leave together

  const int32_t e = element[a];
  const int64_t Dtot = int64_t(S) * DV;
  // x is re-read (from cache) for every stack pass rather than held: with
  // the gradient sums live, fewer registers per lane let more waves share a
  // SIMD
  const float* xrow = x + a * DV + q * EPL;

  float gacc[EPL];
#pragma unroll
  for (int r = 0; r < EPL; ++r) gacc[r] = 0.0f;
  float eacc = 0.0f;
  adjoint_stacks<LOG_D, LOG_EPL, WANT_E, WANT_G>(xrow, signs + int64_t(e) * T * S * W,
                                                 bias + int64_t(e) * Dtot, alpha, S, T, 0, VPW,
                                                 q, grp, c_rev, gacc, eacc);
  adjoint_wave_sums<LOGK, EPL, WANT_E, WANT_G>(gacc, eacc);
  if constexpr (WANT_G) {
    if (grp == 0) {
      float w_m = 1.0f;
      if (dE != nullptr) w_m = dE[molecule_of(mol_ptr, n_mols, a)];
      store_vec<EPL>(grad_x + a * DV + q * EPL, gacc, g_scale * w_m);
    }
  }
  if constexpr (WANT_E) {
    if (lane == 0) e_atom[a] = eacc * e_scale;
  }
}

// Latency form of the energy + gradient adjoint (sorf_predict with forces):
// one workgroup of NWAVE waves per atom, wave w taking the stack passes
// w, w + NWAVE, ...; the waves' sums are added in wave order through LDS.
// A small batch (a served request) then spreads over NWAVE times as many
// SIMDs and finishes in about 1 / NWAVE of the one-wave time. NWAVE depends
// only on the model (the pass count, at most 8), so a molecule's results do
// not depend on the batch it is in.
constexpr int kAdjMaxWaves = 8;
template <int LOG_D, int LOG_EPL>
__global__ __launch_bounds__(64 * kAdjMaxWaves) __attribute__((amdgpu_waves_per_eu(3))) void atom_adjoint_split_kernel(
    const float* __restrict__ x, const int32_t* __restrict__ element,
    const uint32_t* __restrict__ signs, const float* __restrict__ bias,
    const float* __restrict__ alpha, float* __restrict__ grad_x, float* __restrict__ e_atom,
    int64_t n_atoms, int32_t S, int32_t T, float c_rev, float g_scale, float e_scale) {
  constexpr int DV = 1 << LOG_D;
  constexpr int EPL = 1 << LOG_EPL;
  constexpr int LOGK = LOG_D - LOG_EPL;
  constexpr int VPW = 64 >> LOGK;
  constexpr int W = (DV + 31) / 32;
  __shared__ float red[kAdjMaxWaves][DV];
  __shared__ float ered[kAdjMaxWaves];

  const int nw = int(blockDim.x >> 6);
  const int wv = int(threadIdx.x >> 6);
  const uint32_t lane = lane_id();
  const uint32_t q = lane & ((1u << LOGK) - 1u);
  const uint32_t grp = lane >> LOGK;
  // workgroup-uniform loop over atoms (one per workgroup at a time)
  for (int64_t a = blockIdx.x; a < n_atoms; a += gridDim.x) {
    const int32_t e = element[a];
    const float* xrow = x + a * DV + q * EPL;

    float gacc[EPL];
#pragma unroll
    for (int r = 0; r < EPL; ++r) gacc[r] = 0.0f;
    float eacc = 0.0f;
    adjoint_stacks<LOG_D, LOG_EPL, true, true>(xrow, signs + int64_t(e) * T * S * W,
                                               bias + int64_t(e) * int64_t(S) * DV, alpha, S, T,
                                               wv * VPW, nw * VPW, q, grp, c_rev, gacc, eacc);
    adjoint_wave_sums<LOGK, EPL, true, true>(gacc, eacc);
    if (grp == 0) {
#pragma unroll
      for (int r = 0; r < EPL; ++r) red[wv][q * EPL + r] = gacc[r];
    }
    if (lane == 0) ered[wv] = eacc;
    __syncthreads();
    if (wv == 0) {
      if (grp == 0) {
#pragma unroll
        for (int r = 0; r < EPL; ++r) {
          float g = red[0][q * EPL + r];
          for (int w = 1; w < nw; ++w) g += red[w][q * EPL + r];
          gacc[r] = g;
        }
        store_vec<EPL>(grad_x + a * DV + q * EPL, gacc, g_scale);
      }
      if (lane == 0) {
        float es = ered[0];
        for (int w = 1; w < nw; ++w) es += ered[w];
        e_atom[a] = es * e_scale;
      }
    }
    __syncthreads();   // red[] and ered[] are rewritten for the next atom
  }
}

// ---------------------------------------------------------------------------
// Per-molecule reduction: E_m = sum of the atoms' shares; F_m = -sum_i J_i^T g_i.
//
// The force contraction is a transposed GEMV per molecule: J_m is
// [N_m d rows][3 N_m columns] row-major, g_m the N_m d gradient entries. A
// molecule is cut into tiles of (64 columns) x (row chunk); the number of
// row chunks depends on N_m only (min(ceil(N_m d / 256), 32)), so every
// molecule is summed in the same order whatever batch it is in: results are
// bitwise independent of batching. Three launches:
//   plan    one block scans the molecules' tile and partial counts;
//   partial a persistent grid walks the tile list; in a tile the four waves
//           take every fourth row, lanes own columns, the waves are combined
//           through LDS in fixed order into one partial row;
//   final   F = -(sum of a molecule's partial rows in chunk order); E_m is
//           summed over the atoms in order.
// ---------------------------------------------------------------------------
constexpr int64_t kForceRowChunk = 256;
constexpr int64_t kForceMaxChunks = 32;

struct ForceShape {
  int64_t nrc;    // row chunks
  int64_t ncb;    // 64-column blocks
  int64_t chunk;  // rows per chunk (last may be shorter)
};

__device__ __forceinline__ ForceShape force_shape(int64_t n, int32_t d) {
  ForceShape f;
  const int64_t rows = n * d;
  const int64_t c = (rows + kForceRowChunk - 1) / kForceRowChunk;
  f.nrc = c < kForceMaxChunks ? c : kForceMaxChunks;
  f.chunk = f.nrc > 0 ? (rows + f.nrc - 1) / f.nrc : 0;
  f.ncb = (3 * n + 63) / 64;
  return f;
}

// Largest index m in [0, count) with ptr[m] <= v, for nondecreasing ptr with
// ptr[0] <= v < ptr[count]: that entry has ptr[m] <= v < ptr[m + 1].
__device__ __forceinline__ int64_t upper_segment(const int64_t* __restrict__ ptr, int64_t count,
                                                 int64_t v) {
  int64_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (ptr[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(1024) void force_plan_kernel(const int64_t* __restrict__ mol_ptr,
                                                          int64_t n_mols, int32_t d,
                                                          int64_t* __restrict__ tile_start,
                                                          int64_t* __restrict__ part_start) {
  __shared__ int64_t st[1024];
  __shared__ int64_t sp[1024];
  const int tid = threadIdx.x;
  const int64_t per = (n_mols + 1023) / 1024;
  const int64_t b0 = int64_t(tid) * per;
  const int64_t m0 = b0 < n_mols ? b0 : n_mols;
  const int64_t m1 = m0 + per < n_mols ? m0 + per : n_mols;
  int64_t t = 0, q = 0;
  for (int64_t m = m0; m < m1; ++m) {
    const int64_t n = mol_ptr[m + 1] - mol_ptr[m];
    const ForceShape f = force_shape(n, d);
    t += f.nrc * f.ncb;
    q += f.nrc * 3 * n;
  }
  st[tid] = t;
  sp[tid] = q;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t vt = tid >= off ? st[tid - off] : 0;
    const int64_t vp = tid >= off ? sp[tid - off] : 0;
    __syncthreads();
    st[tid] += vt;
    sp[tid] += vp;
    __syncthreads();
  }
  int64_t tb = st[tid] - t, pb = sp[tid] - q;
  for (int64_t m = m0; m < m1; ++m) {
    const int64_t n = mol_ptr[m + 1] - mol_ptr[m];
    const ForceShape f = force_shape(n, d);
    tile_start[m] = tb;
    part_start[m] = pb;
    tb += f.nrc * f.ncb;
    pb += f.nrc * 3 * n;
  }
  if (tid == 1023) {
    tile_start[n_mols] = st[1023];
    part_start[n_mols] = sp[1023];
  }
}

__global__ __launch_bounds__(256) void force_partial_kernel(
    const int64_t* __restrict__ mol_ptr, int64_t n_mols, const int64_t* __restrict__ tile_start,
    const int64_t* __restrict__ part_start, const float* __restrict__ grad,
    const float* __restrict__ J, const int64_t* __restrict__ J_ptr, float* __restrict__ partial,
    int32_t d) {
  __shared__ float red[4][64];
  const int64_t total = tile_start[n_mols];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int64_t m = upper_segment(tile_start, n_mols, t);
    const int64_t a0 = mol_ptr[m];
    const int64_t n = mol_ptr[m + 1] - a0;
    const ForceShape f = force_shape(n, d);
    const int64_t local = t - tile_start[m];
    const int64_t rc = local / f.ncb;
    const int64_t cb = local - rc * f.ncb;
    const int64_t ncol = 3 * n;
    const int64_t rows = n * d;
    const int64_t r0 = rc * f.chunk < rows ? rc * f.chunk : rows;
    const int64_t r1 = r0 + f.chunk < rows ? r0 + f.chunk : rows;
    const int64_t col = cb * 64 + lane;
    const bool ok = col < ncol;
    // out-of-range lanes read the last column (in bounds) and discard it
    const float* __restrict__ blk = J + J_ptr[m] + (ok ? col : ncol - 1);
    const float* __restrict__ g = grad + a0 * d;
    float acc = 0.0f;
    int64_t r = r0 + wv;
    for (; r + 28 < r1; r += 32) {
      float jv[8], gv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        jv[k] = blk[(r + 4 * k) * ncol];
        gv[k] = g[r + 4 * k];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) acc = __builtin_fmaf(jv[k], gv[k], acc);
    }
    for (; r < r1; r += 4) acc = __builtin_fmaf(blk[r * ncol], g[r], acc);
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && ok)
      partial[part_start[m] + rc * ncol + col] =
          ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void molecule_final_kernel(
    const int64_t* __restrict__ mol_ptr, int64_t n_atoms, int64_t n_mols,
    const int64_t* __restrict__ part_start, const float* __restrict__ partial,
    const float* __restrict__ e_atom, float* __restrict__ E, float* __restrict__ F, int32_t d) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (F != nullptr) {
    for (int64_t k = tid; k < 3 * n_atoms; k += stride) {
      const int64_t i = k / 3;
      const int64_t m = upper_segment(mol_ptr, n_mols, i);
      const int64_t a0 = mol_ptr[m];
      const int64_t n = mol_ptr[m + 1] - a0;
      const ForceShape f = force_shape(n, d);
      const int64_t ncol = 3 * n;
      const float* __restrict__ p = partial + part_start[m] + (k - 3 * a0);
      // all chunk partials are loaded before the sum (one memory round trip
      // instead of nrc dependent ones); the sum keeps chunk order
      float v[kForceMaxChunks];
#pragma unroll
      for (int rc = 0; rc < kForceMaxChunks; ++rc) v[rc] = rc < f.nrc ? p[rc * ncol] : 0.0f;
      float s = 0.0f;
#pragma unroll
      for (int rc = 0; rc < kForceMaxChunks; ++rc)
        if (rc < f.nrc) s += v[rc];
      F[k] = -s;
    }
  }
  if (E != nullptr) {
    for (int64_t m = tid; m < n_mols; m += stride) {
      const int64_t a0 = mol_ptr[m], a1 = mol_ptr[m + 1];
      float s = 0.0f;
      // loads in groups of 16 ahead of the in-order sum
      for (int64_t i0 = a0; i0 < a1; i0 += 16) {
        float v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = i0 + j < a1 ? e_atom[i0 + j] : 0.0f;
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (i0 + j < a1) s += v[j];
      }
      E[m] = s;
    }
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
static hipError_t forward_dispatch(const SorfFeatureArgs& a, float* Z, const float* alpha,
                                   hipStream_t st) {
  constexpr int LOG_EPL = default_log_epl<LOG_D>();
  constexpr int VPW = 64 >> (LOG_D - LOG_EPL);
  const int64_t items = a.n_mols * int64_t(a.n_stacks);
  const int64_t waves = (items + VPW - 1) / VPW;
  const int64_t blocks = (waves + 3) / 4;
  const double D = double(a.d) * a.n_stacks;
  const float c_rev = float(double(sorf_c(a)) * (1.0 / (2.0 * M_PI)));
  const float scale = float(std::sqrt(2.0 / D));
  // the shared-row form needs whole rows per wave (d >= 64) and every wave's
  // groups on one molecule (n_stacks a multiple of the groups per wave)
  constexpr bool kCanShare = LOG_D >= 6 && LOG_D <= 8;
  const bool share = kCanShare && a.n_stacks % VPW == 0;
#define SORF_FWD(DOTV, SH)                                                                     \
  hipLaunchKernelGGL((forward_kernel<LOG_D, LOG_EPL, DOTV, SH>), dim3(unsigned(blocks)),     \
                     dim3(256), 0, st, a.x, a.element, a.mol_ptr, a.signs, a.bias, Z, alpha, \
                     a.n_mols, a.n_stacks, a.n_transforms, c_rev, scale)
  if (alpha == nullptr) {
    if (share) SORF_FWD(false, kCanShare);
    else SORF_FWD(false, false);
  } else {
    if (share) SORF_FWD(true, kCanShare);
    else SORF_FWD(true, false);
  }
#undef SORF_FWD
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
  if (e_atom && grad_x && dE == nullptr) {
    // energies with forces: the latency form, one pass of stacks per wave
    constexpr int VPW = 64 >> (LOG_D - LOG_EPL);
    const int64_t passes = (a.n_stacks + VPW - 1) / VPW;
    const int nw = int(passes < kAdjMaxWaves ? passes : kAdjMaxWaves);
    const int64_t grid = a.n_atoms < (int64_t(1) << 20) ? a.n_atoms : (int64_t(1) << 20);
    hipLaunchKernelGGL((atom_adjoint_split_kernel<LOG_D, LOG_EPL>), dim3(unsigned(grid)),
                       dim3(64 * nw), 0, st, a.x, a.element, a.signs, a.bias, alpha, grad_x,
                       e_atom, a.n_atoms, a.n_stacks, a.n_transforms, c_rev, g_scale, e_scale);
  } else if (e_atom && grad_x) SORF_ADJ(true, true);
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
#define CALL(L) forward_dispatch<L>(a, Z, nullptr, st)
  SORF_LOGD_SWITCH(log2i(a.d), CALL)
#undef CALL
}

static hipError_t energy_parts(const SorfFeatureArgs& a, const float* alpha, float* part,
                               hipStream_t st) {
#define CALL(L) forward_dispatch<L>(a, part, alpha, st)
  SORF_LOGD_SWITCH(log2i(a.d), CALL)
#undef CALL
}

hipError_t sorf_launch_energies(const SorfFeatureArgs& a, const float* alpha, float* part,
                                float* E, hipStream_t st) {
  if (a.n_mols == 0) return hipSuccess;
  hipError_t e = energy_parts(a, alpha, part, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(energy_sum_kernel, dim3(unsigned((a.n_mols + 255) / 256)), dim3(256), 0, st,
                     part, a.n_mols, a.n_stacks, E);
  return hipGetLastError();
}

hipError_t sorf_launch_atom_adjoint(const SorfFeatureArgs& a, const float* alpha, const float* dE,
                                    float* grad_x, float* e_atom, hipStream_t st) {
  if (a.n_atoms == 0) return hipSuccess;
#define CALL(L) adjoint_dispatch<L>(a, alpha, dE, grad_x, e_atom, st)
  SORF_LOGD_SWITCH(log2i(a.d), CALL)
#undef CALL
}

size_t sorf_force_plan_bytes(int64_t n_atoms, int64_t n_mols) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return 2 * al(sizeof(int64_t) * size_t(n_mols + 1)) +
         al(sizeof(float) * size_t(kForceMaxChunks) * 3 * size_t(n_atoms));
}

hipError_t sorf_launch_molecule_reduce(const SorfFeatureArgs& a, const float* e_atom,
                                       const float* grad, const float* J, const int64_t* J_ptr,
                                       float* E, float* F, void* plan_ws, hipStream_t st) {
  if (a.n_mols == 0) return hipSuccess;
  const float* partial = nullptr;
  const int64_t* part_start = nullptr;
  if (J != nullptr && a.n_atoms > 0) {
    const size_t idx = ((sizeof(int64_t) * size_t(a.n_mols + 1)) + 255) & ~size_t(255);
    int64_t* tile_start = static_cast<int64_t*>(plan_ws);
    int64_t* pstart = reinterpret_cast<int64_t*>(static_cast<char*>(plan_ws) + idx);
    float* part = reinterpret_cast<float*>(static_cast<char*>(plan_ws) + 2 * idx);
    hipLaunchKernelGGL(force_plan_kernel, dim3(1), dim3(1024), 0, st, a.mol_ptr, a.n_mols, a.d,
                       tile_start, pstart);
    // tiles <= sum_m 32 (3 N_m / 64 + 1) = 1.5 A + 32 M bounds the useful grid
    const int64_t bound = (3 * a.n_atoms) / 2 + 32 * a.n_mols + 1;
    const unsigned grid = unsigned(bound < 4096 ? bound : 4096);
    hipLaunchKernelGGL(force_partial_kernel, dim3(grid), dim3(256), 0, st, a.mol_ptr, a.n_mols,
                       tile_start, pstart, grad, J, J_ptr, part, a.d);
    partial = part;
    part_start = pstart;
  }
  const int64_t work = (F != nullptr ? 3 * a.n_atoms : 0) > a.n_mols
                           ? 3 * a.n_atoms : a.n_mols;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(molecule_final_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, a.mol_ptr,
                     a.n_atoms, a.n_mols, part_start, partial, e_atom, E,
                     (J != nullptr && a.n_atoms > 0) ? F : nullptr, a.d);
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
