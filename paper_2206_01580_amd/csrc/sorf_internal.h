// Internal device helpers and launcher declarations of the SORF library.
//
// Data layout of one SORF vector (one atom, one stack) inside a wave64:
// the d entries are split over K = d / EPL consecutive lanes ("a lane group"),
// lane q of the group holding entries j = q * EPL + r, r = 0 .. EPL-1, in
// registers. A wave therefore carries 64 / K vectors at once. The fast
// Walsh-Hadamard transform (SORF subsection: O(d log d) in-place butterflies)
// runs its first log2(EPL) stages inside each lane and the last log2(K)
// stages across the lanes of the group with DPP / swizzle exchanges.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sorf {

constexpr float kInv2Pi = 0.159154943091895336f;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Value of `x` held by lane (lane ^ (1 << BIT)) of the same wave.
template <int BIT>
__device__ __forceinline__ float lane_xor(float x) {
  int i = __float_as_int(x);
  if constexpr (BIT == 0) {
    i = __builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  } else if constexpr (BIT == 1) {
    i = __builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  } else if constexpr (BIT <= 4) {
    // bitmask swizzle inside 32 lanes: and = 0x1f, or = 0, xor = 1 << BIT
    i = __builtin_amdgcn_ds_swizzle(i, 0x1F | ((1 << BIT) << 10));
  } else {
    i = __builtin_amdgcn_ds_bpermute(int((lane_id() ^ 32u) << 2), i);
  }
  return __int_as_float(i);
}

// Butterfly stages of the Hadamard transform over the EPL entries of a lane
// (index bits 0 .. log2(EPL)-1): (a, b) -> (a + b, a - b), natural order.
template <int EPL>
__device__ __forceinline__ void fwht_in_lane(float (&v)[EPL]) {
#pragma unroll
  for (int h = 1; h < EPL; h <<= 1) {
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      if ((i & h) == 0) {
        const float a = v[i];
        const float b = v[i + h];
        v[i] = a + b;
        v[i + h] = a - b;
      }
    }
  }
}

// Butterfly stages over the lane bits of the group (index bits log2(EPL) ..).
// Every lane computes v + m * partner with m = +1 on the low lane of a pair and
// m = -1 on the high lane. The low lane gets a + b; the high lane gets
// b - a = -(a - b): its value is carried with a pending sign. After all stages
// lane q holds (-1)^popcount(q) times the true entries; the caller folds that
// sign into the next sign diagonal or into the final scale.
//
// Inside a quad (lane bits 0 and 1) the exchange and the multiply-add are one
// v_fmac_f32 with a DPP quad_perm on src0 (v += dpp(v) * m). The compiler does
// not fuse a separate DPP move into the FMA, hence the inline assembly. The
// leading s_nop covers the 2 wait states required between a VALU write of a
// VGPR and a DPP read of it; inside a block every instruction reads a
// different register than the previous one wrote.
#define SORF_DPP_FMAC(CTRL, R) \
  "v_fmac_f32_dpp %" #R ", %" #R ", %16 " CTRL " row_mask:0xf bank_mask:0xf\n\t"
#define SORF_DPP_BLOCK16(CTRL)                                                                  \
  "s_nop 1\n\t" SORF_DPP_FMAC(CTRL, 0) SORF_DPP_FMAC(CTRL, 1) SORF_DPP_FMAC(CTRL, 2)           \
      SORF_DPP_FMAC(CTRL, 3) SORF_DPP_FMAC(CTRL, 4) SORF_DPP_FMAC(CTRL, 5)                      \
          SORF_DPP_FMAC(CTRL, 6) SORF_DPP_FMAC(CTRL, 7) SORF_DPP_FMAC(CTRL, 8)                  \
              SORF_DPP_FMAC(CTRL, 9) SORF_DPP_FMAC(CTRL, 10) SORF_DPP_FMAC(CTRL, 11)            \
                  SORF_DPP_FMAC(CTRL, 12) SORF_DPP_FMAC(CTRL, 13) SORF_DPP_FMAC(CTRL, 14)       \
                      SORF_DPP_FMAC(CTRL, 15)

template <int BIT>
__device__ __forceinline__ void dpp_fmac16(float* v, float m) {
  if constexpr (BIT == 0) {
    asm volatile(SORF_DPP_BLOCK16("quad_perm:[1,0,3,2]")
                 : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]),
                   "+v"(v[6]), "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]),
                   "+v"(v[12]), "+v"(v[13]), "+v"(v[14]), "+v"(v[15])
                 : "v"(m));
  } else {
    asm volatile(SORF_DPP_BLOCK16("quad_perm:[2,3,0,1]")
                 : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]),
                   "+v"(v[6]), "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]),
                   "+v"(v[12]), "+v"(v[13]), "+v"(v[14]), "+v"(v[15])
                 : "v"(m));
  }
}

template <int BIT, int LOGK, int EPL>
__device__ __forceinline__ void fwht_across_lanes(float (&v)[EPL], uint32_t q) {
  if constexpr (BIT < LOGK) {
    const float m = ((q >> BIT) & 1u) ? -1.0f : 1.0f;
    if constexpr (BIT <= 1 && EPL % 16 == 0) {
#pragma unroll
      for (int r = 0; r < EPL; r += 16) dpp_fmac16<BIT>(v + r, m);
    } else {
#pragma unroll
      for (int r = 0; r < EPL; ++r) v[r] = __builtin_fmaf(m, lane_xor<BIT>(v[r]), v[r]);
    }
    fwht_across_lanes<BIT + 1, LOGK, EPL>(v, q);
  }
}

template <int LOGK, int EPL>
__device__ __forceinline__ void fwht(float (&v)[EPL], uint32_t q) {
  fwht_in_lane<EPL>(v);
  fwht_across_lanes<0, LOGK, EPL>(v, q);
}

// Multiply entry r by -1 when bit r of the lane's sign words is set.
template <int EPL>
__device__ __forceinline__ void apply_signs(float (&v)[EPL], const uint32_t* w) {
#pragma unroll
  for (int r = 0; r < EPL; ++r) {
    // shift bit r to bit 31 and xor it into the sign (one shift + one v_bitop3)
    const uint32_t mask = (w[r >> 5] << (31 - (r & 31))) & 0x80000000u;
    v[r] = __uint_as_float(__float_as_uint(v[r]) ^ mask);
  }
}

// Sign words of one lane for one (element, transform, stack) vector.
// `vec` points at the W = ceil(d/32) words of the vector.
template <int EPL>
__device__ __forceinline__ void load_sign_words(uint32_t (&w)[EPL >= 32 ? EPL / 32 : 1],
                                                const uint32_t* __restrict__ vec, uint32_t q,
                                                uint32_t flip) {
  if constexpr (EPL >= 32) {
#pragma unroll
    for (int i = 0; i < EPL / 32; ++i) w[i] = vec[q * (EPL / 32) + i] ^ flip;
  } else {
    const uint32_t bit0 = q * EPL;
    w[0] = (vec[bit0 >> 5] >> (bit0 & 31)) ^ flip;
  }
}

template <int EPL>
__device__ __forceinline__ void load_vec(float (&v)[EPL], const float* __restrict__ p) {
  if constexpr (EPL % 4 == 0) {
#pragma unroll
    for (int i = 0; i < EPL / 4; ++i) {
      const float4 t = reinterpret_cast<const float4*>(p)[i];
      v[4 * i + 0] = t.x;
      v[4 * i + 1] = t.y;
      v[4 * i + 2] = t.z;
      v[4 * i + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPL; ++i) v[i] = p[i];
  }
}

template <int EPL>
__device__ __forceinline__ void store_vec(float* __restrict__ p, const float (&v)[EPL], float s) {
  if constexpr (EPL % 4 == 0) {
#pragma unroll
    for (int i = 0; i < EPL / 4; ++i) {
      reinterpret_cast<float4*>(p)[i] =
          make_float4(v[4 * i] * s, v[4 * i + 1] * s, v[4 * i + 2] * s, v[4 * i + 3] * s);
    }
  } else {
#pragma unroll
    for (int i = 0; i < EPL; ++i) p[i] = v[i] * s;
  }
}

__device__ __forceinline__ int64_t molecule_of(const int64_t* __restrict__ mol_ptr, int64_t n_mols,
                                               int64_t atom) {
  // largest m with mol_ptr[m] <= atom (skips empty molecules)
  int64_t lo = 0, hi = n_mols;  // invariant: mol_ptr[lo] <= atom < mol_ptr[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (mol_ptr[mid] <= atom) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace sorf

// ---------------------------------------------------------------------------
// Launchers (host side), implemented in the kernel translation units. Each
// returns a hipError_t from the launch.
// ---------------------------------------------------------------------------
struct SorfFeatureArgs {
  int32_t d, n_stacks, n_transforms, n_elements;
  float sigma;
  const uint32_t* signs;
  const float* bias;
  const float* x;
  const int32_t* element;
  const int64_t* mol_ptr;
  int64_t n_atoms, n_mols;
};

// Force contraction shape of a molecule of n atoms: its J block is
// [n d rows][3 n columns]; rows are cut into min(ceil(n d / 256), 32) chunks
// and columns into 64-column blocks. It depends on the molecule alone, so its
// forces are summed in the same order in any batch.
constexpr int64_t kForceRowChunk = 256;
constexpr int64_t kForceMaxChunks = 32;
struct ForceShape {
  int64_t nrc;    // row chunks
  int64_t ncb;    // 64-column blocks
  int64_t chunk;  // rows per chunk (last may be shorter)
};
__host__ __device__ inline ForceShape force_shape(int64_t n, int32_t d) {
  ForceShape f;
  const int64_t rows = n * d;
  const int64_t c = (rows + kForceRowChunk - 1) / kForceRowChunk;
  f.nrc = c < kForceMaxChunks ? c : kForceMaxChunks;
  f.chunk = f.nrc > 0 ? (rows + f.nrc - 1) / f.nrc : 0;
  f.ncb = (3 * n + 63) / 64;
  return f;
}

// Persistent serving kernel (energies and forces of batches of requests).
// The host publishes batches in a ring of descriptors in host-coherent
// memory and counts them in ServeControl::head; the kernel, resident on
// every compute unit, takes them in order, writes energies and forces into
// the batch's host-coherent result slot and counts finished batches in
// ServeControl::done.
constexpr int kServeMaxRequests = 64;
struct ServeDesc {
  int64_t atom0;        // pool index of the batch's first atom (its requests are contiguous)
  int64_t n_atoms;
  int64_t n_req;        // < 0: the kernel exits
  int64_t slot;         // result slot
  int64_t mol_ptr[kServeMaxRequests + 1];     // atom offsets relative to atom0
  int64_t j_ptr[kServeMaxRequests + 1];       // float offsets of the J blocks in the J pool
  int64_t tile_start[kServeMaxRequests + 1];  // force tiles of the requests before each
  int64_t part_start[kServeMaxRequests + 1];  // force partial floats before each
};
struct ServeControl {
  int64_t head;      // batches published (host)
  int64_t done;      // batches finished (device)
  int32_t stop;      // host: finish the published batches and exit
  int32_t state;     // device: 0 running, 1 exited on stop, 2 exited idle, 3 exited on a wait limit
};
struct ServeKernelArgs {
  int32_t d, n_stacks, n_transforms, n_waves;
  const uint32_t* signs;
  const float* bias;
  const float* alpha;
  const float* x_pool;
  const int32_t* element_pool;
  const float* J_pool;
  const ServeDesc* ring;          // host-coherent, ring_slots descriptors
  ServeControl* ctl;              // host-coherent
  float* results;                 // host-coherent, ring_slots x slot_floats
  int64_t ring_slots, slot_floats, max_atoms;
  ServeDesc* dev_desc;            // device scratch: the current batch
  unsigned long long* bar;        // device scratch: [0] arrivals, [1] release generation
  float* grad;                    // device scratch [max_atoms][d]
  float* e_atom;                  // device scratch [max_atoms]
  float* partial;                 // device scratch [kForceMaxChunks * 3 * max_atoms]
  float c_rev, g_scale, e_scale;
  int64_t idle_ticks, wait_ticks;   // limits on the constant-rate real-time counter
};
// Waves per atom of the energy + force adjoint and its scale factors (the
// serving kernel uses the same, so its results equal sorf_predict's).
int sorf_adjoint_waves(int32_t d, int32_t n_stacks);
void sorf_adjoint_scales(const SorfFeatureArgs& a, float* c_rev, float* g_scale, float* e_scale);
size_t sorf_serve_scratch_bytes(int32_t d, int64_t max_atoms);
// grid: resident workgroups (one per compute unit); cooperative launch
hipError_t sorf_launch_serve(const ServeKernelArgs& a, int grid, hipStream_t s);

hipError_t sorf_launch_forward(const SorfFeatureArgs& a, float* Z, hipStream_t s);
// E[m] = sum_f alpha_f Z[m][f] without storing Z; part: n_mols * n_stacks floats.
// Energies without forces: a molecule's atoms are taken kEnergyChunkAtoms at a
// time (chunk_ptr: [n_mols + 1] offsets of the molecules' chunks, formed on
// the device; part: [chunks][n_stacks] partial energies).
constexpr int64_t kEnergyChunkAtoms = 32;
__host__ __device__ inline int64_t energy_chunk_bound(int64_t n_atoms, int64_t n_mols) {
  return n_mols + (n_atoms + kEnergyChunkAtoms - 1) / kEnergyChunkAtoms;
}
hipError_t sorf_launch_energies(const SorfFeatureArgs& a, const float* alpha, int64_t* chunk_ptr,
                                float* part, float* E, hipStream_t st);
hipError_t sorf_launch_atom_adjoint(const SorfFeatureArgs& a, const float* alpha, const float* dE,
                                    float* grad_x, float* e_atom, hipStream_t s);
// Energies E [n_mols] and dE/dx [n_atoms][d] in one adjoint pass (one wave per
// atom); e_atom: [n_atoms] workspace of the atoms' energy shares.
hipError_t sorf_launch_energy_grad(const SorfFeatureArgs& a, const float* alpha, float* grad_x,
                                   float* e_atom, float* E, hipStream_t s);
// Workspace of the force contraction: tile and partial offsets per molecule
// plus at most 32 partial rows of 3 N_m floats per molecule.
size_t sorf_force_plan_bytes(int64_t n_atoms, int64_t n_mols);
hipError_t sorf_launch_molecule_reduce(const SorfFeatureArgs& a, const float* e_atom,
                                       const float* grad, const float* J, const int64_t* J_ptr,
                                       float* E, float* F, void* plan_ws, hipStream_t s);
// Derivative features dZ [3 n_atoms][D] (rows of the force-trained normal equation).
hipError_t sorf_launch_dz(const SorfFeatureArgs& a, const float* J, const int64_t* J_ptr,
                          float* dZ, hipStream_t s);
// Per-element projection x_i = rho_i^T U_{e_i}; workspace: bucket counts, offsets and list.
size_t sorf_project_ws_bytes(int64_t n_atoms, int32_t n_elements);
hipError_t sorf_launch_project(int64_t n_atoms, int32_t d_rep, const float* rho,
                               const int32_t* element, int32_t n_elements, const float* U,
                               int32_t d, float* x, void* ws, hipStream_t s);
// Fit of one element's projection: top n_pca eigenvectors of sum rho^T rho (FP64 Jacobi).
size_t sorf_fit_ws_bytes(int32_t d_rep);
hipError_t sorf_launch_projection_fit(int64_t n_samples, int32_t d_rep, const float* sample,
                                      int32_t n_pca, float* U, double* sv, void* ws, hipStream_t s);
// FCHL19 representation (parameters as in the paper's table).
struct FchlParamsHost {
  int32_t n2, n3;
  float eta2, eta3, N2, N3, c3, zeta, rcut;
};
int64_t sorf_fchl19_len(int32_t n_elements, int32_t n2, int32_t n3);
hipError_t sorf_launch_fchl19_forward(const float* R, const int32_t* element,
                                      const int64_t* mol_ptr, int64_t n_atoms, int64_t n_mols,
                                      int32_t n_elements, const FchlParamsHost& p, float* rho,
                                      hipStream_t s);
hipError_t sorf_launch_fchl19_backward(const float* R, const int32_t* element,
                                       const int64_t* mol_ptr, int64_t n_mols, int32_t n_elements,
                                       const FchlParamsHost& p, const float* g, float* dR,
                                       hipStream_t s);
hipError_t sorf_launch_validate(const SorfFeatureArgs& a, int32_t* result, hipStream_t s);
hipError_t sorf_launch_fill(float* p, int64_t n, float v, hipStream_t s);

size_t sorf_gram_ws_bytes(int64_t n_rows, int32_t D, int mode);
hipError_t sorf_launch_gram(int64_t n_rows, int32_t D, const float* Z, const float* y, int mode,
                            int32_t scale_exp, float* G, float* Zty, void* ws, hipStream_t s);
size_t sorf_gram_split_ws_bytes(int64_t n_rows, int32_t D);
hipError_t sorf_launch_gram_split(int64_t n_rows, int32_t D, const float* Z, const float* y,
                                  double* G, double* Zty, void* ws, hipStream_t s);
hipError_t sorf_launch_gram_f64(int64_t n_rows, int32_t D, const float* Z, const float* y,
                                double* G, double* Zty, hipStream_t s);

size_t sorf_solve_ws_bytes(int32_t D);
// side == nullptr: every launch on s; otherwise the lookahead runs on side,
// ordered with s through the two caller-owned events
hipError_t sorf_launch_solve(int32_t D, const float* G, const float* Zty, double lambda,
                             int32_t n_refine, double* alpha, int32_t* info, void* ws,
                             hipStream_t s, hipStream_t side, hipEvent_t ev_fork,
                             hipEvent_t ev_join);
hipError_t sorf_launch_solve_f64(int32_t D, const double* G, const double* Zty, double lambda,
                                 int32_t n_refine, double* alpha, int32_t* info, void* ws,
                                 hipStream_t s, hipStream_t side, hipEvent_t ev_fork,
                                 hipEvent_t ev_join);
