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
// share of the energy of one chunk of at most kEnergyChunkAtoms atoms of a
// molecule, part[c S + s] = sum_f alpha_f z_f over the stack's features for
// chunk c (chunk_ptr[m] .. chunk_ptr[m + 1] - 1 are molecule m's), summed
// over the group's lanes in a fixed order. A molecule's atoms are walked by
// one lane group per chunk and stack, so a single large molecule still
// spreads over the chip; a molecule of at most kEnergyChunkAtoms atoms is one
// chunk.
// SHARED (the stack count a multiple of the groups per wave, so that all
// groups of a wave walk the same molecule): the wave loads the next atom's x
// row cooperatively (d / 64 floats per lane) while it transforms the current
// one, and parks it in a double-buffered LDS row that the groups read from.
template <int LOG_D, int LOG_EPL, bool DOT, bool SHARED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void forward_kernel(
    const float* __restrict__ x, const int32_t* __restrict__ element,
    const int64_t* __restrict__ mol_ptr, const uint32_t* __restrict__ signs,
    const float* __restrict__ bias, float* __restrict__ Z, const float* __restrict__ alpha,
    const int64_t* __restrict__ chunk_ptr, int64_t n_mols, int32_t S, int32_t T, float c_rev,
    float out_scale) {
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
  int64_t m, c = 0, a0, a1;
  int32_t s;
  if constexpr (DOT) {
    // item = (chunk, stack); the molecule of chunk c is the m with
    // chunk_ptr[m] <= c < chunk_ptr[m + 1]
    if (item >= chunk_ptr[n_mols] * int64_t(S)) return;   // whole lane groups leave together
    c = item / S;
    s = int32_t(item - c * S);
    int64_t lo = 0, hi = n_mols;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (chunk_ptr[mid] <= c) lo = mid;
      else hi = mid;
    }
    m = lo;
    const int64_t m1 = mol_ptr[m + 1];
    a0 = mol_ptr[m] + (c - chunk_ptr[m]) * kEnergyChunkAtoms;
    a1 = a0 + kEnergyChunkAtoms < m1 ? a0 + kEnergyChunkAtoms : m1;
  } else {
    if (item >= n_mols * int64_t(S)) return;  // whole lane groups leave together
    m = item / S;
    s = int32_t(item - m * S);
    a0 = mol_ptr[m];
    a1 = mol_ptr[m + 1];
  }
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
    if (q == 0) Z[c * S + s] = p * out_scale;
  } else {
    store_vec<EPL>(Z + m * Dtot + int64_t(s) * DV + q * EPL, acc, out_scale);
  }
}

// E[m] = the sum of molecule m's chunk partials: one wave per molecule, lane j
// adding the stacks j, j + 64, ... (inside a stack its chunks in order), then
// the 64 lane sums by a fixed butterfly.
__global__ __launch_bounds__(256) void energy_sum_kernel(const float* __restrict__ part,
                                                        const int64_t* __restrict__ chunk_ptr,
                                                        int64_t n_mols, int32_t S,
                                                        float* __restrict__ E) {
  const int64_t m = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = int(threadIdx.x & 63);
  if (m >= n_mols) return;   // whole waves
  const int64_t c0 = chunk_ptr[m], c1 = chunk_ptr[m + 1];
  float e = 0.0f;
  for (int32_t s = lane; s < S; s += 64)
    for (int64_t c = c0; c < c1; ++c) e += part[c * S + s];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
  if (lane == 0) E[m] = e;
}

// chunk_ptr[m] = sum over the molecules before m of ceil(N / kEnergyChunkAtoms)
// (one workgroup of 1024 threads: each thread sums a contiguous run of
// molecules, the runs' totals are scanned in LDS, then each thread writes its
// run's offsets; chunk_ptr[n_mols] is the total).
__global__ __launch_bounds__(1024) void energy_chunks_kernel(const int64_t* __restrict__ mol_ptr,
                                                            int64_t n_mols,
                                                            int64_t* __restrict__ chunk_ptr) {
  __shared__ int64_t tot[1024];
  const int t = threadIdx.x;
  const int64_t per = (n_mols + 1023) / 1024;
  const int64_t m0 = t * per < n_mols ? t * per : n_mols;
  const int64_t m1 = m0 + per < n_mols ? m0 + per : n_mols;
  int64_t sum = 0;
  for (int64_t m = m0; m < m1; ++m)
    sum += (mol_ptr[m + 1] - mol_ptr[m] + kEnergyChunkAtoms - 1) / kEnergyChunkAtoms;
  tot[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan
    const int64_t v = t >= off ? tot[t - off] : 0;
    __syncthreads();
    tot[t] += v;
    __syncthreads();
  }
  int64_t run = tot[t] - sum;   // exclusive prefix of this thread's run
  for (int64_t m = m0; m < m1; ++m) {
    chunk_ptr[m] = run;
    run += (mol_ptr[m + 1] - mol_ptr[m] + kEnergyChunkAtoms - 1) / kEnergyChunkAtoms;
  }
  if (t == 1023) chunk_ptr[n_mols] = tot[1023];
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
// Atom a with waves 0 .. nw - 1 of the workgroup (waves at or above nw only
// take part in the barriers); red/ered are the workgroup's LDS scratch.
template <int LOG_D, int LOG_EPL>
__device__ __forceinline__ void adjoint_split_atom(
    int64_t a, int nw, const float* __restrict__ x, const int32_t* __restrict__ element,
    const uint32_t* __restrict__ signs, const float* __restrict__ bias,
    const float* __restrict__ alpha, float* __restrict__ grad_x, float* __restrict__ e_atom,
    int32_t S, int32_t T, float c_rev, float g_scale, float e_scale,
    float (&red)[kAdjMaxWaves][1 << LOG_D], float (&ered)[kAdjMaxWaves]) {
  constexpr int DV = 1 << LOG_D;
  constexpr int EPL = 1 << LOG_EPL;
  constexpr int LOGK = LOG_D - LOG_EPL;
  constexpr int VPW = 64 >> LOGK;
  constexpr int W = (DV + 31) / 32;
  const int wv = int(threadIdx.x >> 6);
  const uint32_t lane = lane_id();
  const uint32_t q = lane & ((1u << LOGK) - 1u);
  const uint32_t grp = lane >> LOGK;
  if (wv < nw) {
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
  }
  __syncthreads();
  if (wv == 0) {
    if (grp == 0) {
      float g[EPL];
#pragma unroll
      for (int r = 0; r < EPL; ++r) {
        float v = red[0][q * EPL + r];
        for (int w = 1; w < nw; ++w) v += red[w][q * EPL + r];
        g[r] = v;
      }
      store_vec<EPL>(grad_x + a * DV + q * EPL, g, g_scale);
    }
    if (lane == 0) {
      float es = ered[0];
      for (int w = 1; w < nw; ++w) es += ered[w];
      e_atom[a] = es * e_scale;
    }
  }
  __syncthreads();   // red[] and ered[] are rewritten for the next atom
}

// Latency form of the energy + gradient adjoint (sorf_predict with forces):
// one workgroup of nw waves per atom, wave w taking the stack passes
// w, w + nw, ...; the waves' sums are added in wave order through LDS.
// A small batch (a served request) then spreads over nw times as many SIMDs
// and finishes in about 1 / nw of the one-wave time. nw depends only on the
// model (the pass count, at most 8), so a molecule's results do not depend
// on the batch it is in.
template <int LOG_D, int LOG_EPL>
__global__ __launch_bounds__(64 * kAdjMaxWaves) __attribute__((amdgpu_waves_per_eu(3))) void atom_adjoint_split_kernel(
    const float* __restrict__ x, const int32_t* __restrict__ element,
    const uint32_t* __restrict__ signs, const float* __restrict__ bias,
    const float* __restrict__ alpha, float* __restrict__ grad_x, float* __restrict__ e_atom,
    int64_t n_atoms, int32_t S, int32_t T, float c_rev, float g_scale, float e_scale) {
  __shared__ float red[kAdjMaxWaves][1 << LOG_D];
  __shared__ float ered[kAdjMaxWaves];
  const int nw = int(blockDim.x >> 6);
  // workgroup-uniform loop over atoms (one per workgroup at a time)
  for (int64_t a = blockIdx.x; a < n_atoms; a += gridDim.x)
    adjoint_split_atom<LOG_D, LOG_EPL>(a, nw, x, element, signs, bias, alpha, grad_x, e_atom, S,
                                       T, c_rev, g_scale, e_scale, red, ered);
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

// Tile t of the force contraction by four waves (wq = 0..3, lane = 0..63)
// sharing red[4][64]: in the tile (64 columns, one row chunk of molecule m),
// wave wq takes rows r0 + wq, r0 + wq + 4, ..., lanes own columns, and the
// waves are combined in fixed order into one partial row. Both barriers are
// reached by every caller's thread, active or not.
__device__ __forceinline__ void force_tile(bool active, int64_t t,
                                           const int64_t* __restrict__ mol_ptr, int64_t n_mols,
                                           const int64_t* __restrict__ tile_start,
                                           const int64_t* __restrict__ part_start,
                                           const float* __restrict__ grad,
                                           const float* __restrict__ J,
                                           const int64_t* __restrict__ J_ptr,
                                           float* __restrict__ partial, int32_t d, int wq, int lane,
                                           float (&red)[4][64]) {
  int64_t m = 0, rc = 0, col = 0, ncol = 1;
  bool ok = false;
  if (active) {
    m = upper_segment(tile_start, n_mols, t);
    const int64_t a0 = mol_ptr[m];
    const int64_t n = mol_ptr[m + 1] - a0;
    const ForceShape f = force_shape(n, d);
    const int64_t local = t - tile_start[m];
    rc = local / f.ncb;
    const int64_t cb = local - rc * f.ncb;
    ncol = 3 * n;
    const int64_t rows = n * d;
    const int64_t r0 = rc * f.chunk < rows ? rc * f.chunk : rows;
    const int64_t r1 = r0 + f.chunk < rows ? r0 + f.chunk : rows;
    col = cb * 64 + lane;
    ok = col < ncol;
    // out-of-range lanes read the last column (in bounds) and discard it
    const float* __restrict__ blk = J + J_ptr[m] + (ok ? col : ncol - 1);
    const float* __restrict__ g = grad + a0 * d;
    float acc = 0.0f;
    int64_t r = r0 + wq;
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
    red[wq][lane] = acc;
  }
  __syncthreads();
  if (active && wq == 0 && ok)
    partial[part_start[m] + rc * ncol + col] =
        ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
  __syncthreads();
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
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x)
    force_tile(true, t, mol_ptr, n_mols, tile_start, part_start, grad, J, J_ptr, partial, d, wv,
               lane, red);
}

// F[k] = -(sum of the molecule's partial rows at column k - 3 a0, in chunk
// order), for force entry k of atom k / 3 of the batch. All chunk partials are
// loaded before the sum (one memory round trip instead of nrc dependent ones).
__device__ __forceinline__ float force_entry(int64_t k, const int64_t* __restrict__ mol_ptr,
                                             int64_t n_mols,
                                             const int64_t* __restrict__ part_start,
                                             const float* __restrict__ partial, int32_t d) {
  const int64_t i = k / 3;
  const int64_t m = upper_segment(mol_ptr, n_mols, i);
  const int64_t a0 = mol_ptr[m];
  const int64_t n = mol_ptr[m + 1] - a0;
  const ForceShape f = force_shape(n, d);
  const int64_t ncol = 3 * n;
  const float* __restrict__ p = partial + part_start[m] + (k - 3 * a0);
  float v[kForceMaxChunks];
#pragma unroll
  for (int rc = 0; rc < kForceMaxChunks; ++rc) v[rc] = rc < f.nrc ? p[rc * ncol] : 0.0f;
  float s = 0.0f;
#pragma unroll
  for (int rc = 0; rc < kForceMaxChunks; ++rc)
    if (rc < f.nrc) s += v[rc];
  return -s;
}

// E_m = sum of the atoms' shares in atom order, loads in groups of 16 ahead
// of the in-order sum.
__device__ __forceinline__ float molecule_energy(int64_t a0, int64_t a1,
                                                 const float* __restrict__ e_atom) {
  float s = 0.0f;
  for (int64_t i0 = a0; i0 < a1; i0 += 16) {
    float v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = i0 + j < a1 ? e_atom[i0 + j] : 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (i0 + j < a1) s += v[j];
  }
  return s;
}

__global__ __launch_bounds__(256) void molecule_final_kernel(
    const int64_t* __restrict__ mol_ptr, int64_t n_atoms, int64_t n_mols,
    const int64_t* __restrict__ part_start, const float* __restrict__ partial,
    const float* __restrict__ e_atom, float* __restrict__ E, float* __restrict__ F, int32_t d) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (F != nullptr) {
    for (int64_t k = tid; k < 3 * n_atoms; k += stride)
      F[k] = force_entry(k, mol_ptr, n_mols, part_start, partial, d);
  }
  if (E != nullptr) {
    for (int64_t m = tid; m < n_mols; m += stride)
      E[m] = molecule_energy(mol_ptr[m], mol_ptr[m + 1], e_atom);
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
                                   const int64_t* chunk_ptr, hipStream_t st) {
  constexpr int LOG_EPL = default_log_epl<LOG_D>();
  constexpr int VPW = 64 >> (LOG_D - LOG_EPL);
  // energies: at most n_mols + ceil(n_atoms / kEnergyChunkAtoms) chunks per stack
  const int64_t items = (alpha == nullptr ? a.n_mols : energy_chunk_bound(a.n_atoms, a.n_mols)) *
                        int64_t(a.n_stacks);
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
                     chunk_ptr, a.n_mols, a.n_stacks, a.n_transforms, c_rev, scale)
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

// latency: energies with gradients in the latency form (several waves per
// atom); otherwise one wave per atom.
template <int LOG_D>
static hipError_t adjoint_dispatch(const SorfFeatureArgs& a, const float* alpha, const float* dE,
                                   float* grad_x, float* e_atom, bool latency, hipStream_t st) {
  constexpr int LOG_EPL = default_log_epl<LOG_D>();
  const int64_t blocks = (a.n_atoms + 3) / 4;
  float c_rev, g_scale, e_scale;
  sorf_adjoint_scales(a, &c_rev, &g_scale, &e_scale);
  const dim3 grid{unsigned(blocks)}, block{256};
#define SORF_ADJ(WE, WG)                                                                        \
  hipLaunchKernelGGL((atom_adjoint_kernel<LOG_D, LOG_EPL, WE, WG>), grid, block, 0, st, a.x,   \
                     a.element, a.mol_ptr, a.signs, a.bias, alpha, dE, grad_x, e_atom,        \
                     a.n_atoms, a.n_mols, a.n_stacks, a.n_transforms, c_rev, g_scale, e_scale)
  if (e_atom && grad_x && dE == nullptr && latency) {
    // energies with forces: the latency form, one pass of stacks per wave
    const int nw = sorf_adjoint_waves(a.d, a.n_stacks);
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

// ---------------------------------------------------------------------------
// Persistent serving kernel
// ---------------------------------------------------------------------------
// One workgroup of 8 waves per compute unit, all resident (cooperative
// launch). Per batch, with grid-wide barriers between the phases:
//   B0  workgroup 0 waits until every workgroup has finished the previous
//       batch, publishes it as done, waits for the host to publish the next
//       one and copies its descriptor into device memory;
//   A   energy + gradient adjoint of the batch's atoms (adjoint_split_atom,
//       the sorf_predict kernel's per-atom work);
//   B   force tiles (force_tile, two tiles per workgroup at a time);
//   C   forces and energies (force_entry, molecule_energy) written straight
//       into the batch's host-coherent result slot.
// Every result is summed in the order sorf_predict uses, so a request's
// energy and forces are bitwise those of sorf_predict on it alone. Every wait
// is bounded: a wait that exceeds its limit ends the kernel with state 3.
__device__ __forceinline__ unsigned long long serve_poll(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// constant-rate real-time counter (the device's wall clock)
__device__ __forceinline__ int64_t serve_now() {
  return int64_t(__builtin_amdgcn_s_memrealtime());
}

// Grid-wide barrier number `n` (counted from 0 over the kernel's life):
// returns false when the wait limit was reached.
// One thread per workgroup carries the synchronisation: after the workgroup
// barrier (every wave's stores have reached the compute unit's L2) it
// releases at device scope, which writes the L2 back once for the whole
// workgroup, and after the wait it acquires once (one L2 invalidation)
// before the second workgroup barrier lets the other waves read. The wait
// itself polls with relaxed loads: an acquire load would invalidate the L2
// on every poll and make the workgroups that are still working miss.
__device__ __forceinline__ bool serve_barrier(unsigned long long* bar, unsigned long long n,
                                              int64_t limit, int* lds_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(&bar[0], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long target = (n + 1) * gridDim.x;
    const int64_t t0 = serve_now();
    int ok = 1;
    while (serve_poll(&bar[0]) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (serve_now() - t0 > limit) { ok = 0; break; }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *lds_ok = ok;
  }
  __syncthreads();
  return *lds_ok != 0;
}

template <int LOG_D, int LOG_EPL>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void serve_kernel(
    ServeKernelArgs a) {
  constexpr int DV = 1 << LOG_D;
  __shared__ float red[kAdjMaxWaves][DV];
  __shared__ float ered[kAdjMaxWaves];
  __shared__ float fred[2][4][64];
  __shared__ int s_ok;
  __shared__ int64_t s_flag;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t G = gridDim.x, b = blockIdx.x;
  unsigned long long nbar = 0;   // barriers passed
  for (int64_t k = 0;; ++k) {
    // ---- B0: batch boundary. The workgroup's result writes (host memory)
    // are released at system scope by one thread, after the workgroup barrier.
    __syncthreads();
    if (tid == 0)
      __hip_atomic_fetch_add(&a.bar[0], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    if (b == 0) {
      if (tid == 0) {
        int64_t flag = 1;   // 1: run, 0: exit (stop or idle), -1: exit (limit)
        const unsigned long long target = (nbar + 1) * G;
        int64_t t0 = serve_now();
        while (serve_poll(&a.bar[0]) < target) {
          __builtin_amdgcn_s_sleep(1);
          if (serve_now() - t0 > a.wait_ticks) { flag = -1; break; }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");   // every workgroup's results, system scope
        if (flag == 1) {
          // batches before k are complete and their results written
          __hip_atomic_store(&a.ctl->done, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
          t0 = serve_now();
          while (__hip_atomic_load(&a.ctl->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) <= k) {
            if (__hip_atomic_load(&a.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
              flag = 0;
              __hip_atomic_store(&a.ctl->state, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
              break;
            }
            __builtin_amdgcn_s_sleep(2);
            if (serve_now() - t0 > a.idle_ticks) {
              flag = 0;
              __hip_atomic_store(&a.ctl->state, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
              break;
            }
          }
        } else {
          __hip_atomic_store(&a.ctl->state, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");   // the descriptor published with head
        s_flag = flag;
      }
      __syncthreads();
      // copy the descriptor (or an exit command) into device memory
      const int64_t words = int64_t(sizeof(ServeDesc) / sizeof(int64_t));
      const int64_t* src = reinterpret_cast<const int64_t*>(&a.ring[k % a.ring_slots]);
      int64_t* dst = reinterpret_cast<int64_t*>(a.dev_desc);
      for (int64_t w = tid; w < words; w += blockDim.x) {
        int64_t v = 0;
        if (s_flag == 1)
          v = __hip_atomic_load(&src[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (w == 2 && s_flag != 1) v = -1;   // n_req < 0: exit
        dst[w] = v;
      }
      __syncthreads();
      if (tid == 0)
        __hip_atomic_store(&a.bar[1], nbar + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else if (tid == 0) {
      // covers workgroup 0's two waits: the arrivals and the host
      const int64_t t0 = serve_now();
      int ok = 1;
      while (serve_poll(&a.bar[1]) < nbar + 1) {
        __builtin_amdgcn_s_sleep(2);
        if (serve_now() - t0 > a.idle_ticks + 2 * a.wait_ticks) { ok = 0; break; }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the descriptor
      s_ok = ok;
    }
    __syncthreads();
    if (b != 0 && !s_ok) return;
    ++nbar;
    const ServeDesc* d = a.dev_desc;
    const int64_t n_req = d->n_req;
    if (n_req < 0) return;
    const int64_t n_atoms = d->n_atoms, atom0 = d->atom0;

    // ---- A: adjoint of every atom, one atom per workgroup at a time
    for (int64_t i = b; i < n_atoms; i += G)
      adjoint_split_atom<LOG_D, LOG_EPL>(i, a.n_waves, a.x_pool + atom0 * DV, a.element_pool + atom0,
                                         a.signs, a.bias, a.alpha, a.grad, a.e_atom, a.n_stacks,
                                         a.n_transforms, a.c_rev, a.g_scale, a.e_scale, red, ered);
    if (!serve_barrier(a.bar, nbar++, a.wait_ticks, &s_ok)) return;

    // ---- B: force tiles, two per workgroup at a time (waves 0-3 and 4-7)
    const int64_t total = d->tile_start[n_req];
    const int half = wv >> 2, wq = wv & 3;
    const int64_t rounds = (total + 2 * G - 1) / (2 * G);
    for (int64_t r = 0; r < rounds; ++r) {
      const int64_t t = 2 * (r * G + b) + half;
      force_tile(t < total, t, d->mol_ptr, n_req, d->tile_start, d->part_start, a.grad, a.J_pool,
                 d->j_ptr, a.partial, DV, wq, lane, fred[half]);
    }
    if (!serve_barrier(a.bar, nbar++, a.wait_ticks, &s_ok)) return;

    // ---- C: forces and energies into the host result slot [E (max requests) | F]
    float* out = a.results + d->slot * a.slot_floats;
    for (int64_t q = b * blockDim.x + tid; q < 3 * n_atoms; q += G * blockDim.x)
      out[kServeMaxRequests + q] = force_entry(q, d->mol_ptr, n_req, d->part_start, a.partial, DV);
    for (int64_t m = b * blockDim.x + tid; m < n_req; m += G * blockDim.x)
      out[m] = molecule_energy(d->mol_ptr[m], d->mol_ptr[m + 1], a.e_atom);
  }
}

template <int LOG_D>
static hipError_t serve_dispatch(const ServeKernelArgs& a, int grid, hipStream_t st) {
  constexpr int LOG_EPL = default_log_epl<LOG_D>();
  ServeKernelArgs args = a;
  void* params[] = {&args};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&serve_kernel<LOG_D, LOG_EPL>),
                                    dim3(unsigned(grid)), dim3(512), params, 0, st);
}

}  // namespace sorf

using namespace sorf;

size_t sorf_serve_scratch_bytes(int32_t d, int64_t max_atoms) {
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  return al(sizeof(ServeDesc)) + al(2 * sizeof(unsigned long long)) +
         al(sizeof(float) * size_t(max_atoms) * size_t(d)) + al(sizeof(float) * size_t(max_atoms)) +
         al(sizeof(float) * size_t(kForceMaxChunks) * 3 * size_t(max_atoms));
}


int sorf_adjoint_waves(int32_t d, int32_t n_stacks) {
  int log_d = 0;
  while ((1 << log_d) < d) ++log_d;
  const int log_epl = log_d < 5 ? log_d : 5;
  const int vpw = 64 >> (log_d - log_epl);
  const int64_t passes = (int64_t(n_stacks) + vpw - 1) / vpw;
  return int(passes < kAdjMaxWaves ? passes : kAdjMaxWaves);
}

void sorf_adjoint_scales(const SorfFeatureArgs& a, float* c_rev, float* g_scale, float* e_scale) {
  const double D = double(a.d) * a.n_stacks;
  const double c = double(sorf_c(a));
  *c_rev = float(c * (1.0 / (2.0 * M_PI)));
  *g_scale = float(-std::sqrt(2.0 / D) * c);
  *e_scale = float(std::sqrt(2.0 / D));
}


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
#define CALL(L) forward_dispatch<L>(a, Z, nullptr, nullptr, st)
  SORF_LOGD_SWITCH(log2i(a.d), CALL)
#undef CALL
}

static hipError_t energy_parts(const SorfFeatureArgs& a, const float* alpha,
                               const int64_t* chunk_ptr, float* part, hipStream_t st) {
#define CALL(L) forward_dispatch<L>(a, part, alpha, chunk_ptr, st)
  SORF_LOGD_SWITCH(log2i(a.d), CALL)
#undef CALL
}

hipError_t sorf_launch_energies(const SorfFeatureArgs& a, const float* alpha, int64_t* chunk_ptr,
                                float* part, float* E, hipStream_t st) {
  if (a.n_mols == 0) return hipSuccess;
  hipLaunchKernelGGL(energy_chunks_kernel, dim3(1), dim3(1024), 0, st, a.mol_ptr, a.n_mols,
                     chunk_ptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = energy_parts(a, alpha, chunk_ptr, part, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(energy_sum_kernel, dim3(unsigned((a.n_mols + 3) / 4)), dim3(256), 0, st,
                     part, chunk_ptr, a.n_mols, a.n_stacks, E);
  return hipGetLastError();
}

hipError_t sorf_launch_atom_adjoint(const SorfFeatureArgs& a, const float* alpha, const float* dE,
                                    float* grad_x, float* e_atom, hipStream_t st) {
  if (a.n_atoms == 0) return hipSuccess;
#define CALL(L) adjoint_dispatch<L>(a, alpha, dE, grad_x, e_atom, true, st)
  SORF_LOGD_SWITCH(log2i(a.d), CALL)
#undef CALL
}

hipError_t sorf_launch_energy_grad(const SorfFeatureArgs& a, const float* alpha, float* grad_x,
                                   float* e_atom, float* E, hipStream_t st) {
  if (a.n_atoms > 0) {
    hipError_t e;
#define CALL(L) adjoint_dispatch<L>(a, alpha, nullptr, grad_x, e_atom, false, st)
    auto adj = [&]() -> hipError_t { SORF_LOGD_SWITCH(log2i(a.d), CALL) };
#undef CALL
    if ((e = adj()) != hipSuccess) return e;
  }
  return sorf_launch_molecule_reduce(a, e_atom, grad_x, nullptr, nullptr, E, nullptr, nullptr, st);
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

hipError_t sorf_launch_serve(const ServeKernelArgs& a, int grid, hipStream_t st) {
#define CALL(L) serve_dispatch<L>(a, grid, st)
  SORF_LOGD_SWITCH(log2i(a.d), CALL)
#undef CALL
}
