// FCHL19 atomic representation (arXiv 2206.01580, Theory section,
// Representation subsection; parameters from the Computational Details
// table): for every atom i,
//   rho_i = [G2_X for every element X] ++ [G3_XY for every element pair X <= Y],
//   G2_X[k]     = sum_{j in X} f_cut(r_ij) r_ij^-N2 LN(R_k; mu(r_ij), sigma(r_ij)),
//                 LN the log-normal density, mu = ln(r / sqrt(1 + eta2/r^2)),
//                 sigma^2 = ln(1 + eta2/r^2), R_k = r_cut (k + 1) / n2;
//   G3_XY[k][t] = sum over unordered neighbour pairs {j, k'} of elements {X, Y} of
//                 xi3 f_cut(r_ij) f_cut(r_jk') f_cut(r_ik') sqrt(eta3/pi)
//                 exp(-eta3 ((r_ij + r_ik')/2 - R_k)^2) A_t(theta),
//                 xi3 = c3 (1 + 3 cos_i cos_j cos_k') / (r_ij r_jk' r_ik')^N3 (Axilrod-Teller-Muto),
//                 A_cos = 2 e^(-zeta^2/2) cos(theta), A_sin = 2 e^(-zeta^2/2) sin(theta),
//                 theta the angle at i, R_k = r_cut k / (n3 - 1); f_cut(r) = (cos(pi r/r_cut) + 1)/2
//                 below r_cut and 0 beyond.
//
// Atoms of molecules of up to 64 atoms take one wave each (see
// fchl19_forward_small_kernel). Larger molecules: one workgroup (4 waves) per atom. The atom's neighbours (same molecule,
// closer than r_cut) are gathered into LDS grouped by element, in atom order
// inside each group (ballot compaction, no atomics), with their per-neighbour
// two-body factors. Two-body bins: one thread per (element, bin) sums its
// element's neighbours in order. Three-body: the unordered pairs are numbered
// by element pair (X <= Y), then by position; chunks of pairs get their
// radial-independent weight (xi3, cutoffs, angle) computed by all threads
// into LDS, and one thread per (element pair, radial bin) sums its pairs of
// the chunk in order. Every entry of rho is therefore summed in a fixed order.
#include <cmath>

#include "sorf_internal.h"

namespace sorf {

constexpr int kFchlMaxNb = 512;        // neighbours of one atom held in LDS
constexpr int kFchlPairChunk = 2048;   // three-body pairs per LDS chunk
constexpr int kFchlMaxElements = 16;
constexpr int kFchlSmallMol = 64;       // molecules up to this size take the wave-per-atom kernel

struct FchlParams {
  int32_t n2, n3;
  float eta2, eta3, N2, N3, c3, zeta, rcut;
};

// The argument of the cutoff's cosine, pi r / r_cut, lies in [0, pi) below
// r_cut, so the hardware sine and cosine (argument in revolutions, here in
// [0, 1/2)) serve without range reduction; f_cut is exactly 0 at and beyond r_cut.
__device__ __forceinline__ float fchl_fcut(float r, float rc) {
  return r < rc ? 0.5f * (__builtin_amdgcn_cosf(r * (0.5f / rc)) + 1.0f) : 0.0f;
}
// d f_cut / dr
__device__ __forceinline__ float fchl_dfcut(float r, float rc) {
  return r < rc ? -0.5f * (3.14159265358979f / rc) * __builtin_amdgcn_sinf(r * (0.5f / rc)) : 0.0f;
}

// Hardware exp2, log2 and reciprocal (about 1 ulp each) for the radial-bin
// loops, where the correctly rounded library sequences cost several times
// as many instructions; arguments there are at most a few tens in magnitude,
// so the results keep a relative accuracy of about 1e-6.
__device__ __forceinline__ float fchl_exp(float x) {
  return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
}
__device__ __forceinline__ float fchl_ln(float x) {
  return __builtin_amdgcn_logf(x) * 0.693147180559945309f;
}
__device__ __forceinline__ float fchl_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// element pair (a <= b) -> position in the lexicographic list of pairs
__device__ __forceinline__ int fchl_pair(int a, int b, int E) { return a * E - a * (a - 1) / 2 + (b - a); }

// Atom i of molecule m (atoms a0 .. a1 - 1).
__device__ __forceinline__ void fchl19_forward_atom(
    int64_t i, int64_t a0, int64_t a1, const float* __restrict__ R,
    const int32_t* __restrict__ element, int32_t E, const FchlParams& p, int64_t size,
    float* __restrict__ rho) {
  __shared__ float nx[kFchlMaxNb], ny[kFchlMaxNb], nz[kFchlMaxNb], nr[kFchlMaxNb];
  __shared__ float c2[kFchlMaxNb], mu2[kFchlMaxNb], inv2s2[kFchlMaxNb];
  __shared__ int32_t grp[kFchlMaxElements + 1];     // neighbour offsets per element
  __shared__ int32_t wcount[4];
  __shared__ int64_t seg[kFchlMaxElements * (kFchlMaxElements + 1) / 2 + 1];
  __shared__ float pw_c[kFchlPairChunk], pw_s[kFchlPairChunk], pmid[kFchlPairChunk];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const float rc = p.rcut;
  const float xi = R[3 * i], yi = R[3 * i + 1], zi = R[3 * i + 2];
  float* __restrict__ out = rho + i * size;

  // neighbours grouped by element, atom order inside a group
  int total = 0;
  bool overflow = false;
  for (int X = 0; X < E; ++X) {
    if (tid == 0) grp[X] = total;
    for (int64_t j0 = a0; j0 < a1; j0 += 256) {
      const int64_t j = j0 + tid;
      float dx = 0.f, dy = 0.f, dz = 0.f, r = 0.f;
      bool f = false;
      if (j < a1 && j != i && element[j] == X) {
        dx = R[3 * j] - xi;
        dy = R[3 * j + 1] - yi;
        dz = R[3 * j + 2] - zi;
        r = sqrtf(dx * dx + dy * dy + dz * dz);
        f = r < rc;
      }
      const uint64_t mask = __ballot(f);
      const int before = __popcll(mask & ((uint64_t(1) << lane) - 1));
      if (lane == 0) wcount[wv] = __popcll(mask);
      __syncthreads();
      int off = total;
      for (int w = 0; w < wv; ++w) off += wcount[w];
      const int chunk = wcount[0] + wcount[1] + wcount[2] + wcount[3];
      if (f) {
        const int slot = off + before;
        if (slot < kFchlMaxNb) {
          nx[slot] = dx;
          ny[slot] = dy;
          nz[slot] = dz;
          nr[slot] = r;
          // two-body factors: f_cut r^-N2 / (sigma sqrt(2 pi)), mu, 1 / (2 sigma^2)
          const float q = 1.0f + p.eta2 / (r * r);
          const float s2 = logf(q);
          c2[slot] = fchl_fcut(r, rc) * powf(r, -p.N2) / (sqrtf(s2) * 2.50662827463100f);
          mu2[slot] = logf(r / sqrtf(q));
          inv2s2[slot] = 0.5f / s2;
        }
      }
      total += chunk;
      __syncthreads();
    }
  }
  if (tid == 0) grp[E] = total;
  overflow = total > kFchlMaxNb;
  if (overflow) {   // more neighbours than the LDS list holds: mark the row, do not guess
    for (int64_t t = tid; t < size; t += 256) out[t] = __builtin_nanf("");
    return;
  }
  __syncthreads();

  // two-body bins
  for (int t = tid; t < E * p.n2; t += 256) {
    const int X = t / p.n2, k = t % p.n2;
    const float Rk = rc * float(k + 1) / float(p.n2);
    const float lnR = logf(Rk);
    float acc = 0.0f;
    for (int s = grp[X]; s < grp[X + 1]; ++s) {
      const float d = lnR - mu2[s];
      acc += c2[s] * fchl_exp(-d * d * inv2s2[s]);
    }
    out[t] = acc / Rk;
  }

  // three-body: pair numbering by element pair X <= Y
  const int NP = E * (E + 1) / 2;
  if (tid == 0) {
    int64_t o = 0;
    for (int X = 0; X < E; ++X)
      for (int Y = X; Y < E; ++Y) {
        seg[fchl_pair(X, Y, E)] = o;
        const int64_t cx = grp[X + 1] - grp[X], cy = grp[Y + 1] - grp[Y];
        o += X == Y ? cx * (cx - 1) / 2 : cx * cy;
      }
    seg[NP] = o;
  }
  __syncthreads();
  const int64_t n_pairs = seg[NP];
  const float angw = 2.0f * expf(-0.5f * p.zeta * p.zeta) * sqrtf(p.eta3 / 3.14159265358979f);
  const int nbins = NP * p.n3;
  // rounds of 512 (element pair, radial bin) outputs, two per thread
  for (int t0 = 0; t0 < nbins; t0 += 512) {
    float acc_c[2] = {0.f, 0.f}, acc_s[2] = {0.f, 0.f};
    for (int64_t q0 = 0; q0 < n_pairs; q0 += kFchlPairChunk) {
      const int64_t q1 = q0 + kFchlPairChunk < n_pairs ? q0 + kFchlPairChunk : n_pairs;
      for (int64_t q = q0 + tid; q < q1; q += 256) {
        // pair q -> element pair P (row X, column Y) -> neighbours (a, b)
        int P = 0;
        while (q >= seg[P + 1]) ++P;
        int X = 0;
        while (fchl_pair(X, X, E) + (E - X) <= P) ++X;
        const int Y = X + (P - fchl_pair(X, X, E));
        const int64_t loc = q - seg[P];
        int a, b;
        if (X != Y) {
          const int cy = grp[Y + 1] - grp[Y];
          a = grp[X] + int(loc / cy);
          b = grp[Y] + int(loc % cy);
        } else {
          // loc -> (u, v), u < v; row u starts at u (2 cx - u - 1) / 2
          const int cx = grp[X + 1] - grp[X];
          const double c2x = 2.0 * cx - 1.0;
          int u = int((c2x - sqrt(c2x * c2x - 8.0 * double(loc))) * 0.5);
          if (u < 0) u = 0;
          while (u > 0 && int64_t(u) * (2 * cx - u - 1) / 2 > loc) --u;
          while (int64_t(u + 1) * (2 * cx - u - 2) / 2 <= loc) ++u;
          a = grp[X] + u;
          b = grp[X] + u + 1 + int(loc - int64_t(u) * (2 * cx - u - 1) / 2);
        }
        const float rij = nr[a], rik = nr[b];
        const float jx = nx[b] - nx[a], jy = ny[b] - ny[a], jz = nz[b] - nz[a];
        const float rjk = sqrtf(jx * jx + jy * jy + jz * jz);
        const float cos_i = (nx[a] * nx[b] + ny[a] * ny[b] + nz[a] * nz[b]) / (rij * rik);
        const float cos_j = -(nx[a] * jx + ny[a] * jy + nz[a] * jz) / (rij * rjk);
        const float cos_k = (nx[b] * jx + ny[b] * jy + nz[b] * jz) / (rik * rjk);
        const float sin_i = sqrtf(fmaxf(0.0f, 1.0f - cos_i * cos_i));
        const float xi3 = p.c3 * (1.0f + 3.0f * cos_i * cos_j * cos_k) / powf(rij * rjk * rik, p.N3);
        const float w = xi3 * fchl_fcut(rij, rc) * fchl_fcut(rjk, rc) * fchl_fcut(rik, rc) * angw;
        const int sl = int(q - q0);
        pw_c[sl] = w * cos_i;
        pw_s[sl] = w * sin_i;
        pmid[sl] = 0.5f * (rij + rik);
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = t0 + tid + 256 * h;
        if (t < nbins) {
          const int P = t / p.n3, k = t % p.n3;
          const float Rk = rc * float(k) / float(p.n3 - 1);
          const int64_t lo = seg[P] > q0 ? seg[P] : q0;
          const int64_t hi = seg[P + 1] < q1 ? seg[P + 1] : q1;
          float c = acc_c[h], sn = acc_s[h];
          for (int64_t q = lo; q < hi; ++q) {
            const int sl = int(q - q0);
            const float d = pmid[sl] - Rk;
            const float g = fchl_exp(-p.eta3 * d * d);
            c += pw_c[sl] * g;
            sn += pw_s[sl] * g;
          }
          acc_c[h] = c;
          acc_s[h] = sn;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = t0 + tid + 256 * h;
      if (t < nbins) {
        float* o = out + int64_t(E) * p.n2 + 2 * int64_t(t);
        o[0] = acc_c[h];
        o[1] = acc_s[h];
      }
    }
  }
}

// Atoms of larger molecules: a persistent grid in which every workgroup reads
// the molecule sizes 256 at a time (coalesced), collects the molecules above
// kFchlSmallMol atoms with ballots, and gives a whole workgroup to atom j of
// such a molecule m when (m + j) mod grid is its own index, so that the atoms
// of one large molecule spread over consecutive workgroups.
__global__ __launch_bounds__(256) void fchl19_forward_kernel(
    const float* __restrict__ R, const int32_t* __restrict__ element,
    const int64_t* __restrict__ mol_ptr, int64_t n_mols, int32_t E, FchlParams p,
    int64_t size, float* __restrict__ rho) {
  __shared__ int32_t big[256];
  __shared__ int32_t wbig[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t G = gridDim.x, b = blockIdx.x;
  int64_t lo = 0, hi = 0;
  if (tid < n_mols) {
    lo = mol_ptr[tid];
    hi = mol_ptr[tid + 1];
  }
  for (int64_t m0 = 0; m0 < n_mols; m0 += 256) {
    const int64_t m = m0 + tid;
    const bool large = m < n_mols && hi - lo > kFchlSmallMol;
    // next group's sizes in flight while this group is processed
    if (m + 256 < n_mols) {
      lo = mol_ptr[m + 256];
      hi = mol_ptr[m + 257];
    }
    const uint64_t mask = __ballot(large);
    if (lane == 0) wbig[wv] = __popcll(mask);
    __syncthreads();
    int off = 0, nbig = 0;
    for (int w = 0; w < 4; ++w) {
      off += w < wv ? wbig[w] : 0;
      nbig += wbig[w];
    }
    if (large) big[off + __popcll(mask & ((uint64_t(1) << lane) - 1))] = tid;
    __syncthreads();
    for (int t = 0; t < nbig; ++t) {
      const int64_t mm = m0 + big[t];
      const int64_t a0 = mol_ptr[mm], a1 = mol_ptr[mm + 1];
      for (int64_t j = ((b - mm) % G + G) % G; j < a1 - a0; j += G) {
        fchl19_forward_atom(a0 + j, a0, a1, R, element, E, p, size, rho);
        __syncthreads();   // the next atom reuses the LDS
      }
    }
    __syncthreads();   // big[] and wbig[] are rewritten by the next group
  }
}

// Atoms of molecules of at most kFchlSmallMol atoms: one wave per atom, four
// atoms per workgroup, no workgroup barriers. The wave's lanes take the
// molecule's atoms, gather the neighbours by element with ballots into the
// wave's LDS, form the two-body bins (lanes over bins), then the three-body
// pair weights in chunks (lanes over pairs) and the three-body bins: lane
// groups of one lane per radial bin split each chunk's pairs into equal
// parts, so that no lane walks a whole large element pair (H-C, say) while
// the others idle. Every entry is summed in a fixed order (pairs in the
// workgroup-per-atom kernel's numbering, parts in group order, chunks in
// order), so results are deterministic.
constexpr int kFchlWavePairs = 384;   // covers the 378 pairs of a centre with 28 neighbours

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256) void fchl19_forward_small_kernel(
    const float* __restrict__ R, const int32_t* __restrict__ element,
    const int64_t* __restrict__ mol_ptr, int64_t atom0, int64_t n_atoms, int64_t n_mols,
    int32_t E, FchlParams p, int64_t size, float* __restrict__ rho) {
  __shared__ float nx[4][kFchlSmallMol], ny[4][kFchlSmallMol], nz[4][kFchlSmallMol];
  __shared__ float nr[4][kFchlSmallMol], c2[4][kFchlSmallMol], mu2[4][kFchlSmallMol],
      inv2s2[4][kFchlSmallMol];
  __shared__ int32_t grp[4][kFchlMaxElements + 1];
  __shared__ int32_t seg[4][kFchlMaxElements * (kFchlMaxElements + 1) / 2 + 1];
  __shared__ float pw_c[4][kFchlWavePairs], pw_s[4][kFchlWavePairs], pmid[4][kFchlWavePairs];
  __shared__ float tail[4][64][2];

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i = atom0 + int64_t(blockIdx.x) * 4 + wv;
  if (i >= n_atoms) return;                   // whole waves leave
  const int64_t m = molecule_of(mol_ptr, n_mols, i);
  const int64_t a0 = mol_ptr[m];
  const int N = int(mol_ptr[m + 1] - a0);
  if (N > kFchlSmallMol) return;              // fchl19_forward_kernel takes this atom
  const float rc = p.rcut;
  float* __restrict__ out = rho + i * size;

  // neighbours by element, atom order inside a group (lane = candidate atom)
  const int64_t j = a0 + lane;
  float dx = 0.f, dy = 0.f, dz = 0.f, r = 0.f;
  bool in = false;
  int ej = -1;
  if (lane < N && j != i) {
    dx = R[3 * j] - R[3 * i];
    dy = R[3 * j + 1] - R[3 * i + 1];
    dz = R[3 * j + 2] - R[3 * i + 2];
    r = sqrtf(dx * dx + dy * dy + dz * dz);
    in = r < rc;
    ej = element[j];
  }
  int n = 0;
  for (int X = 0; X < E; ++X) {
    if (lane == 0) grp[wv][X] = n;
    const bool f = in && ej == X;
    const uint64_t mask = __ballot(f);
    if (f) {
      const int sl = n + __popcll(mask & ((uint64_t(1) << lane) - 1));
      nx[wv][sl] = dx;
      ny[wv][sl] = dy;
      nz[wv][sl] = dz;
      nr[wv][sl] = r;
      const float q = 1.0f + p.eta2 / (r * r);
      const float s2 = logf(q);
      c2[wv][sl] = fchl_fcut(r, rc) * powf(r, -p.N2) / (sqrtf(s2) * 2.50662827463100f);
      mu2[wv][sl] = logf(r / sqrtf(q));
      inv2s2[wv][sl] = 0.5f / s2;
    }
    n += __popcll(mask);
  }
  if (lane == 0) grp[wv][E] = n;
  wave_sync_lds();

  // two-body bins
  for (int t = lane; t < E * p.n2; t += 64) {
    const int X = t / p.n2, k = t % p.n2;
    const float Rk = rc * float(k + 1) / float(p.n2);
    const float lnR = logf(Rk);
    float acc = 0.0f;
    for (int sl = grp[wv][X]; sl < grp[wv][X + 1]; ++sl) {
      const float d = lnR - mu2[wv][sl];
      acc += c2[wv][sl] * fchl_exp(-d * d * inv2s2[wv][sl]);
    }
    out[t] = acc / Rk;
  }

  // three-body: pairs numbered by element pair, then by position (the
  // workgroup-per-atom kernel's numbering)
  const int NP = E * (E + 1) / 2;
  if (lane == 0) {
    int32_t o = 0;
    for (int X = 0; X < E; ++X)
      for (int Y = X; Y < E; ++Y) {
        seg[wv][fchl_pair(X, Y, E)] = o;
        const int32_t cx = grp[wv][X + 1] - grp[wv][X], cy = grp[wv][Y + 1] - grp[wv][Y];
        o += X == Y ? cx * (cx - 1) / 2 : cx * cy;
      }
    seg[wv][NP] = o;
  }
  wave_sync_lds();
  const int32_t n_pairs = seg[wv][NP];
  const float angw = 2.0f * expf(-0.5f * p.zeta * p.zeta) * sqrtf(p.eta3 / 3.14159265358979f);
  // Bins: G groups of n3 lanes, one lane per radial bin; group g walks the
  // g-th of G equal parts of the chunk's pairs in order. An element pair
  // whose pairs fall in several parts is finished by the group where it ends,
  // which adds the partial sums of the earlier groups in group order. With
  // more than 64 radial bins one group's lanes loop over them.
  const int G = p.n3 <= 64 ? 64 / p.n3 : 1;
  const int g = p.n3 <= 64 ? lane / p.n3 : 0;
  const int kl = p.n3 <= 64 ? lane % p.n3 : lane;
  float* __restrict__ out3 = out + int64_t(E) * p.n2;
  int P = 0, X = 0;   // decode state: non-decreasing in q, kept across iterations
  for (int32_t q0 = 0; q0 < n_pairs || q0 == 0; q0 += kFchlWavePairs) {
    const int32_t q1 = q0 + kFchlWavePairs < n_pairs ? q0 + kFchlWavePairs : n_pairs;
    for (int32_t q = q0 + lane; q < q1; q += 64) {
      while (q >= seg[wv][P + 1]) ++P;
      while (fchl_pair(X, X, E) + (E - X) <= P) ++X;
      const int Y = X + (P - fchl_pair(X, X, E));
      const int32_t loc = q - seg[wv][P];
      int a, b;
      if (X != Y) {
        const int cy = grp[wv][Y + 1] - grp[wv][Y];
        a = grp[wv][X] + loc / cy;
        b = grp[wv][Y] + loc % cy;
      } else {
        const int cx = grp[wv][X + 1] - grp[wv][X];
        const float c2x = 2.0f * float(cx) - 1.0f;
        int u = int((c2x - sqrtf(c2x * c2x - 8.0f * float(loc))) * 0.5f);
        if (u < 0) u = 0;
        while (u > 0 && u * (2 * cx - u - 1) / 2 > loc) --u;
        while ((u + 1) * (2 * cx - u - 2) / 2 <= loc) ++u;
        a = grp[wv][X] + u;
        b = grp[wv][X] + u + 1 + (loc - u * (2 * cx - u - 1) / 2);
      }
      const float rij = nr[wv][a], rik = nr[wv][b];
      const float jx = nx[wv][b] - nx[wv][a], jy = ny[wv][b] - ny[wv][a], jz = nz[wv][b] - nz[wv][a];
      const float rjk = sqrtf(jx * jx + jy * jy + jz * jz);
      const float iij = fchl_rcp(rij), iik = fchl_rcp(rik), ijk = fchl_rcp(rjk);
      const float cos_i = (nx[wv][a] * nx[wv][b] + ny[wv][a] * ny[wv][b] + nz[wv][a] * nz[wv][b]) * (iij * iik);
      const float cos_j = -(nx[wv][a] * jx + ny[wv][a] * jy + nz[wv][a] * jz) * (iij * ijk);
      const float cos_k = (nx[wv][b] * jx + ny[wv][b] * jy + nz[wv][b] * jz) * (iik * ijk);
      const float sin_i = sqrtf(fmaxf(0.0f, 1.0f - cos_i * cos_i));
      const float xi3 = p.c3 * (1.0f + 3.0f * cos_i * cos_j * cos_k) *
                        __builtin_amdgcn_exp2f(-p.N3 * __builtin_amdgcn_logf(rij * rjk * rik));
      const float w = xi3 * fchl_fcut(rij, rc) * fchl_fcut(rjk, rc) * fchl_fcut(rik, rc) * angw;
      const int sl = q - q0;
      pw_c[wv][sl] = w * cos_i;
      pw_s[wv][sl] = w * sin_i;
      pmid[wv][sl] = 0.5f * (rij + rik);
    }
    // element pairs without pairs in the first chunk: their bins start at 0
    if (q0 == 0)
      for (int Q = 0; Q < NP; ++Q) {
        const int32_t s0 = seg[wv][Q], s1 = seg[wv][Q + 1] < q1 ? seg[wv][Q + 1] : q1;
        if (s1 <= s0)
          for (int k = lane; k < p.n3; k += 64) {
            out3[2 * (int64_t(Q) * p.n3 + k)] = 0.0f;
            out3[2 * (int64_t(Q) * p.n3 + k) + 1] = 0.0f;
          }
      }
    wave_sync_lds();
    const int32_t L = q1 - q0;
    int pend = -1;                      // element pair to finish after the tails are stored
    float pc = 0.f, ps = 0.f;
    for (int k = kl; k < p.n3 && g < G; k += 64) {
      const float Rk = rc * float(k) / float(p.n3 - 1);
      const int32_t lo = q0 + int32_t(int64_t(L) * g / G), hi = q0 + int32_t(int64_t(L) * (g + 1) / G);
      int Q = 0;
      while (Q < NP && seg[wv][Q + 1] <= lo) ++Q;
      bool started = Q < NP && (seg[wv][Q] > q0 ? seg[wv][Q] : q0) >= lo;
      int32_t segend = Q < NP && seg[wv][Q + 1] < q1 ? seg[wv][Q + 1] : q1;
      float c = 0.f, sn = 0.f;
      for (int32_t q = lo; q < hi; ++q) {
        const int sl = q - q0;
        const float d = pmid[wv][sl] - Rk;
        const float gk = fchl_exp(-p.eta3 * d * d);
        c += pw_c[wv][sl] * gk;
        sn += pw_s[wv][sl] * gk;
        if (q + 1 == segend) {          // element pair Q ends in this part
          if (started) {
            float* o = out3 + 2 * (int64_t(Q) * p.n3 + k);
            if (q0 == 0) {
              o[0] = c;
              o[1] = sn;
            } else {
              o[0] += c;
              o[1] += sn;
            }
          } else {
            pend = Q;
            pc = c;
            ps = sn;
          }
          c = 0.f;
          sn = 0.f;
          ++Q;
          while (Q < NP && seg[wv][Q + 1] <= q + 1) ++Q;
          started = true;
          segend = Q < NP && seg[wv][Q + 1] < q1 ? seg[wv][Q + 1] : q1;
        }
      }
      tail[wv][lane][0] = c;            // open partial at the end of the part (0 if none)
      tail[wv][lane][1] = sn;
    }
    wave_sync_lds();
    if (pend >= 0) {
      const int32_t st = seg[wv][pend] > q0 ? seg[wv][pend] : q0;
      int gs = 0;
      while (q0 + int32_t(int64_t(L) * (gs + 1) / G) <= st) ++gs;
      float sc = 0.f, ss = 0.f;
      for (int gg = gs; gg < g; ++gg) {
        sc += tail[wv][gg * p.n3 + kl][0];
        ss += tail[wv][gg * p.n3 + kl][1];
      }
      float* o = out3 + 2 * (int64_t(pend) * p.n3 + kl);
      if (q0 == 0) {
        o[0] = sc + pc;
        o[1] = ss + ps;
      } else {
        o[0] += sc + pc;
        o[1] += ss + ps;
      }
    }
    wave_sync_lds();   // weights and tails are reused, and the next chunk adds to these entries
    if (n_pairs == 0) break;
  }
}

// ---------------------------------------------------------------------------
// Coordinate gradient: dR = d(sum_i g_i . rho_i)/dR for an upstream g = dE/drho
// (the forces are -dR). Every three-body term of a centre i and its pair of
// neighbours (j, l) depends on the positions only through the three sides
// a = r_ij, b = r_il, c = r_jl (the cosines follow by the law of cosines), so
// its gradient is dL/da u_ij + dL/db u_il + dL/dc u_jl distributed to the
// three atoms; a two-body term gives dL/dr u_ij to j and minus that to i.
//
// Molecules of at most kFchlSmallAtoms atoms: one workgroup per molecule
// scatters each centre's contributions to its atoms inside LDS. Larger
// molecules: one workgroup per atom gathers the contributions that land on
// it from every centre, so a single large molecule spreads over the chip.
// Every gradient entry is summed in a fixed order (deterministic, no atomics).
// ---------------------------------------------------------------------------
// dL/da, dL/db, dL/dc for one centre i and neighbour pair (j, l) with sides
// a = r_ij, b = r_il, c = r_jl, where L is the pair's three-body terms
// contracted with the centre's upstream gradient gp (the 2 n3 entries of the
// pair's element pair, [radial bin][cos, sin]). The cosines are functions of
// the sides (law of cosines), so this is the whole positional dependence.
__device__ __forceinline__ void fchl_triple_grad(float a, float b, float c,
                                                 const float* __restrict__ gp,
                                                 const FchlParams& p, float angw, float (&dL)[3]) {
  const float rc = p.rcut;
  const float ia = fchl_rcp(a), ib = fchl_rcp(b), ic = fchl_rcp(c);
  const float a2 = a * a, b2 = b * b, c2 = c * c;
  const float ci_ = 0.5f * (a2 + b2 - c2) * ia * ib;
  const float cj_ = 0.5f * (a2 + c2 - b2) * ia * ic;
  const float cl_ = 0.5f * (b2 + c2 - a2) * ib * ic;
  const float dci[3] = {0.5f * (a2 - b2 + c2) * ia * ia * ib, 0.5f * (b2 - a2 + c2) * ia * ib * ib,
                        -c * ia * ib};
  const float dcj[3] = {0.5f * (a2 - c2 + b2) * ia * ia * ic, -b * ia * ic,
                        0.5f * (c2 - a2 + b2) * ia * ic * ic};
  const float dcl[3] = {-a * ib * ic, 0.5f * (b2 - c2 + a2) * ib * ib * ic,
                        0.5f * (c2 - b2 + a2) * ib * ic * ic};
  const float si = sqrtf(fmaxf(0.0f, 1.0f - ci_ * ci_));
  const float dsi_dc = si > 1e-12f ? -ci_ * fchl_rcp(si) : 0.0f;
  const float C = ci_ * cj_ * cl_;
  const float invP3 = __builtin_amdgcn_exp2f(-p.N3 * __builtin_amdgcn_logf(a * b * c));
  const float xi3 = p.c3 * (1.0f + 3.0f * C) * invP3;
  const float fa = fchl_fcut(a, rc), fb = fchl_fcut(b, rc), fcc = fchl_fcut(c, rc);
  const float dfa = fchl_dfcut(a, rc), dfb = fchl_dfcut(b, rc), dfcc = fchl_dfcut(c, rc);
  const float Fc = fa * fb * fcc;
  const float dF[3] = {dfa * fb * fcc, fa * dfb * fcc, fa * fb * dfcc};
  const float inv_side[3] = {ia, ib, ic};
  const float A = angw * xi3 * Fc;
  const float wc = A * ci_, ws = A * si;
  const float mid = 0.5f * (a + b);
  const float step = rc / float(p.n3 - 1);
  float Gc = 0.f, Gs = 0.f, Gcp = 0.f, Gsp = 0.f;
  for (int k = 0; k < p.n3; ++k) {
    const float d = mid - float(k) * step;
    const float rad = fchl_exp(-p.eta3 * d * d);
    const float drad = -2.0f * p.eta3 * d * rad;
    Gc += gp[2 * k] * rad;
    Gs += gp[2 * k + 1] * rad;
    Gcp += gp[2 * k] * drad;
    Gsp += gp[2 * k + 1] * drad;
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const float dC = dci[v] * cj_ * cl_ + ci_ * dcj[v] * cl_ + ci_ * cj_ * dcl[v];
    const float dxi = p.c3 * 3.0f * dC * invP3 - p.N3 * xi3 * inv_side[v];
    const float dA = angw * (dxi * Fc + xi3 * dF[v]);
    const float dwc = dA * ci_ + A * dci[v];
    const float dws = dA * si + A * dsi_dc * dci[v];
    const float dmid = v < 2 ? 0.5f : 0.0f;
    dL[v] = Gc * dwc + Gs * dws + (wc * Gcp + ws * Gsp) * dmid;
  }
}

// d/dr of the two-body terms of one neighbour at distance r, contracted with
// the centre's upstream gradient gX (the n2 bins of the neighbour's element),
// over the bins k0, k0 + kstep, ...
__device__ __forceinline__ float fchl_pair_grad(float r, const float* __restrict__ gX,
                                                const FchlParams& p, int k0 = 0, int kstep = 1) {
  const float rc = p.rcut;
  const float q = 1.0f + p.eta2 / (r * r);
  const float s2 = logf(q);
  const float ds2 = -2.0f * p.eta2 / (r * r * r * q);
  const float mu = logf(r / sqrtf(q));
  const float dmu = 1.0f / r + p.eta2 / (r * r * r * q);
  const float fcv = fchl_fcut(r, rc);
  const float dfc = fchl_dfcut(r, rc);
  const float pref = powf(r, -p.N2) / (sqrtf(s2) * 2.50662827463100f);
  const float is2 = 1.0f / s2;
  // D = D0 + Lk D1 + Lk^2 D2
  const float D0 = -p.N2 / r - 0.5f * ds2 * is2, D1 = dmu * is2, D2 = 0.5f * ds2 * is2 * is2;
  const float step = rc / float(p.n2);
  float dL = 0.0f;
  for (int k = k0; k < p.n2; k += kstep) {
    const float Rk = float(k + 1) * step;
    const float Lk = fchl_ln(Rk) - mu;
    const float B = pref * fchl_exp(-0.5f * Lk * Lk * is2) * fchl_rcp(Rk);
    const float D = D0 + Lk * (D1 + Lk * D2);
    dL += gX[k] * (dfc + fcv * D) * B;
  }
  return dL;
}

// Molecules of at most kFchlSmallAtoms atoms: one workgroup per molecule,
// its four waves take four centres at a time. For a centre with n
// neighbours, every unordered pair is evaluated once: lanes take the pairs
// (in chunks of kFchlBwdPairs) and store dL/da, dL/db, dL/dc in the wave's
// LDS. Then each neighbour s gets H lanes (H = 4, 2, 1 for at most 16, 32,
// 63 neighbours); lane h walks the partners t = h, h + H, ... in order (and
// the two-body bins h, h + H, ...) and sums T_s (dL/da where s is the pair's
// j, dL/db where it is l, plus its two-body term) and V_s = -sum dL/dc
// (x_t - x_s) / r_st; the H parts are combined by fixed shuffles. Neighbour s
// gets T_s u_s + V_s, the centre -sum_s T_s u_s (u_s the unit vector from the
// centre to s, summed by fixed shuffles), and the four centres' results are
// merged into the molecule's gradient in centre order.
// STAGED: the centre's upstream gradient row (at most kFchlStage entries) is
// copied into the wave's LDS first, so that the radial-bin loops read LDS.
constexpr int kFchlSmallAtoms = 64;
constexpr int kFchlStage = 1024;
constexpr int kFchlBwdPairs = 256;

template <bool STAGED>
__global__ __launch_bounds__(256) void fchl19_backward_small_kernel(
    const float* __restrict__ R, const int32_t* __restrict__ element,
    const int64_t* __restrict__ mol_ptr, int64_t m0, int64_t n_mols, int32_t E, FchlParams p,
    int64_t size, const float* __restrict__ g, float* __restrict__ dR) {
  __shared__ float ax[kFchlSmallAtoms], ay[kFchlSmallAtoms], az[kFchlSmallAtoms];
  __shared__ int32_t ael[kFchlSmallAtoms];
  __shared__ float gsum[3][kFchlSmallAtoms];
  __shared__ float res[4][3][kFchlSmallAtoms];
  __shared__ int32_t nid[4][kFchlSmallAtoms];
  __shared__ float dls[4][3][kFchlBwdPairs];
  __shared__ float gst[4][STAGED ? kFchlStage : 1];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t m = m0 + blockIdx.x;
  if (m >= n_mols) return;
  const int64_t a0 = mol_ptr[m];
  const int N = int(mol_ptr[m + 1] - a0);
  if (N <= 0 || N > kFchlSmallAtoms) return;   // larger molecules: fchl19_backward_gather_kernel
  const float rc = p.rcut;
  if (tid < N) {
    ax[tid] = R[3 * (a0 + tid)];
    ay[tid] = R[3 * (a0 + tid) + 1];
    az[tid] = R[3 * (a0 + tid) + 2];
    ael[tid] = element[a0 + tid];
    gsum[0][tid] = gsum[1][tid] = gsum[2][tid] = 0.0f;
  }
  __syncthreads();
  const float angw = 2.0f * expf(-0.5f * p.zeta * p.zeta) * sqrtf(p.eta3 / 3.14159265358979f);

  for (int c0 = 0; c0 < N; c0 += 4) {
    const int ci = c0 + wv;
    res[wv][0][lane] = res[wv][1][lane] = res[wv][2][lane] = 0.0f;
    if (ci < N) {   // wave-uniform
      const float* __restrict__ gi = g + (a0 + ci) * size;
      if (STAGED) {
        for (int64_t t = lane; t < size; t += 64) gst[wv][t] = gi[t];
        gi = &gst[wv][0];   // made visible by the wave barrier below
      }
      const float xi = ax[ci], yi = ay[ci], zi = az[ci];
      // this lane's candidate atom, then the neighbours in element order
      const int t = lane;
      bool in = false;
      if (t < N && t != ci) {
        const float dx = ax[t] - xi, dy = ay[t] - yi, dz = az[t] - zi;
        in = sqrtf(dx * dx + dy * dy + dz * dz) < rc;
      }
      int n = 0;
      for (int X = 0; X < E; ++X) {
        const bool f = in && ael[t < N ? t : 0] == X;
        const uint64_t mask = __ballot(f);
        if (f) nid[wv][n + __popcll(mask & ((uint64_t(1) << lane) - 1))] = t;
        n += __popcll(mask);
      }
      wave_sync_lds();
      // H lanes per neighbour slot when the neighbours are few: lane (sl, h)
      // takes the two-body bins and the partners h, h + H, ... of slot sl
      const int H = n <= 16 ? 4 : (n <= 32 ? 2 : 1);
      const int sl = lane / H, h = lane % H;
      int js = 0;
      float xs = 0.f, ys = 0.f, zs = 0.f, ux = 0.f, uy = 0.f, uz = 0.f;
      float T = 0.f, Vx = 0.f, Vy = 0.f, Vz = 0.f;
      if (sl < n) {
        js = nid[wv][sl];
        xs = ax[js];
        ys = ay[js];
        zs = az[js];
        const float vx = xs - xi, vy = ys - yi, vz = zs - zi;
        const float rs = sqrtf(vx * vx + vy * vy + vz * vz);
        ux = vx / rs;
        uy = vy / rs;
        uz = vz / rs;
        T = fchl_pair_grad(rs, gi + ael[js] * p.n2, p, h, H);
      }
      const int32_t n_pairs = n * (n - 1) / 2;
      for (int32_t q0 = 0; q0 < n_pairs; q0 += kFchlBwdPairs) {
        const int32_t q1 = q0 + kFchlBwdPairs < n_pairs ? q0 + kFchlBwdPairs : n_pairs;
        for (int32_t q = q0 + lane; q < q1; q += 64) {
          // q -> slots (s, t), s < t; row s starts at s (2n - s - 1) / 2
          const float c2n = 2.0f * float(n) - 1.0f;
          int s = int((c2n - sqrtf(c2n * c2n - 8.0f * float(q))) * 0.5f);
          s = s < 0 ? 0 : (s > n - 2 ? n - 2 : s);
          while (s > 0 && s * (2 * n - s - 1) / 2 > q) --s;
          while ((s + 1) * (2 * n - s - 2) / 2 <= q) ++s;
          const int tt = s + 1 + (q - s * (2 * n - s - 1) / 2);
          const int ja = nid[wv][s], jb = nid[wv][tt];
          const float vax = ax[ja] - xi, vay = ay[ja] - yi, vaz = az[ja] - zi;
          const float vbx = ax[jb] - xi, vby = ay[jb] - yi, vbz = az[jb] - zi;
          const float a = sqrtf(vax * vax + vay * vay + vaz * vaz);
          const float b = sqrtf(vbx * vbx + vby * vby + vbz * vbz);
          const float wx = vbx - vax, wy = vby - vay, wz = vbz - vaz;
          const float c = sqrtf(wx * wx + wy * wy + wz * wz);
          const int Xa = ael[ja], Xb = ael[jb];
          const int P = fchl_pair(Xa < Xb ? Xa : Xb, Xa < Xb ? Xb : Xa, E);
          float dL[3];
          fchl_triple_grad(a, b, c, gi + int64_t(E) * p.n2 + int64_t(P) * p.n3 * 2, p, angw, dL);
          const int sl = q - q0;
          dls[wv][0][sl] = dL[0];
          dls[wv][1][sl] = dL[1];
          dls[wv][2][sl] = dL[2];
        }
        wave_sync_lds();
        if (sl < n) {
          const int s = sl;
          for (int u = h; u < n; u += H) {
            if (u == s) continue;
            const int lo = s < u ? s : u, hi = s < u ? u : s;
            const int32_t q = lo * (2 * n - lo - 1) / 2 + (hi - lo - 1);
            if (q < q0 || q >= q1) continue;
            const int sl = q - q0;
            T += s < u ? dls[wv][0][sl] : dls[wv][1][sl];
            const int ju = nid[wv][u];
            const float wx = (ax[ju] - xi) - (xs - xi), wy = (ay[ju] - yi) - (ys - yi),
                        wz = (az[ju] - zi) - (zs - zi);
            const float f = dls[wv][2][sl] / sqrtf(wx * wx + wy * wy + wz * wz);
            Vx -= f * wx;
            Vy -= f * wy;
            Vz -= f * wz;
          }
        }
        wave_sync_lds();   // the chunk's derivatives are no longer read
      }
      // the H parts of a slot, combined in a fixed order (every lane of the
      // slot then holds the same sums)
      if (H >= 2) {
        T += __shfl_xor(T, 1);
        Vx += __shfl_xor(Vx, 1);
        Vy += __shfl_xor(Vy, 1);
        Vz += __shfl_xor(Vz, 1);
      }
      if (H >= 4) {
        T += __shfl_xor(T, 2);
        Vx += __shfl_xor(Vx, 2);
        Vy += __shfl_xor(Vy, 2);
        Vz += __shfl_xor(Vz, 2);
      }
      const bool owner = sl < n && h == 0;
      if (owner) {
        res[wv][0][js] = T * ux + Vx;
        res[wv][1][js] = T * uy + Vy;
        res[wv][2][js] = T * uz + Vz;
      }
      // the centre's total over the slots' owner lanes, in a fixed butterfly order
      float cx = owner ? -T * ux : 0.f, cy = owner ? -T * uy : 0.f, cz = owner ? -T * uz : 0.f;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        cx += __shfl_xor(cx, o);
        cy += __shfl_xor(cy, o);
        cz += __shfl_xor(cz, o);
      }
      if (lane == 0) {
        res[wv][0][ci] = cx;
        res[wv][1][ci] = cy;
        res[wv][2][ci] = cz;
      }
    }
    __syncthreads();
    if (tid < N) {
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        float acc = gsum[v][tid];
        acc += res[0][v][tid];
        acc += res[1][v][tid];
        acc += res[2][v][tid];
        acc += res[3][v][tid];
        gsum[v][tid] = acc;
      }
    }
    __syncthreads();
  }
  if (tid < N) {
    dR[3 * (a0 + tid)] = gsum[0][tid];
    dR[3 * (a0 + tid) + 1] = gsum[1][tid];
    dR[3 * (a0 + tid) + 2] = gsum[2][tid];
  }
}

// Molecules above kFchlSmallAtoms atoms (any size): one workgroup per atom
// t gathers the gradient at R_t from every centre whose representation
// depends on it, t itself and each neighbour c of t:
//   centre t: -dL/dr (R_s - R_t) / r_ts for the two-body term of every
//     neighbour s, and -(dL/da (R_j - R_t) / a + dL/db (R_l - R_t) / b) for
//     every unordered neighbour pair {j, l} (a = r_tj, b = r_tl);
//   centre c: dL/dr (R_t - R_c) / r_ct for t's two-body term, and for every
//     other neighbour l of c the pair {t, l}, with sides a = r_ct, b = r_cl,
//     c = r_tl: dL/da (R_t - R_c) / a + dL/dc (R_t - R_l) / c.
// The three-body terms are symmetric in the pair's two atoms (the mean
// distance, the centre's angle and the product of the three cosines do not
// change when j and l swap), so the pair's sides may be passed in either
// order. t's neighbours are gathered into LDS as in the forward kernel
// (kFchlMaxNb at most; more leave t's row NaN). A pair {t, l} of a centre c
// carries f_cut(r_tl), so l is itself a neighbour of t: the centre-c terms
// come from the pairs (c, l) of t's own list with r_cl < r_cut. Each thread
// sums a fixed subset of the terms and the threads' sums are added in thread
// order: the result is deterministic and does not depend on the rest of the
// batch; the sums are FP64, since an atom of a large molecule gathers
// thousands of terms. Every pair derivative of a centre is evaluated once for
// each of the pair's atoms (three times over), the price of needing no
// workspace and no bound on the molecule's size.
__device__ void fchl19_backward_atom(int64_t t, int64_t a0, int64_t a1,
                                     const float* __restrict__ R,
                                     const int32_t* __restrict__ element, int32_t E,
                                     const FchlParams& p, int64_t size,
                                     const float* __restrict__ g, float* __restrict__ dR) {
  __shared__ int32_t nidx[kFchlMaxNb];
  __shared__ float nx[kFchlMaxNb], ny[kFchlMaxNb], nz[kFchlMaxNb], nr[kFchlMaxNb];
  __shared__ int32_t grp[kFchlMaxElements + 1];
  __shared__ int32_t wcount[4];
  __shared__ int64_t seg[kFchlMaxElements * (kFchlMaxElements + 1) / 2 + 1];
  __shared__ double red[3][256];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const float rc = p.rcut;
  const float angw = 2.0f * expf(-0.5f * p.zeta * p.zeta) * sqrtf(p.eta3 / 3.14159265358979f);
  const int NP = E * (E + 1) / 2;
  const float xt = R[3 * t], yt = R[3 * t + 1], zt = R[3 * t + 2];
  const int et = element[t];

  // t's neighbours grouped by element, atom order inside a group
  int total = 0;
  for (int X = 0; X < E; ++X) {
    if (tid == 0) grp[X] = total;
    for (int64_t j0 = a0; j0 < a1; j0 += 256) {
      const int64_t j = j0 + tid;
      float dx = 0.f, dy = 0.f, dz = 0.f, r = 0.f;
      bool f = false;
      if (j < a1 && j != t && element[j] == X) {
        dx = R[3 * j] - xt;
        dy = R[3 * j + 1] - yt;
        dz = R[3 * j + 2] - zt;
        r = sqrtf(dx * dx + dy * dy + dz * dz);
        f = r < rc;
      }
      const uint64_t mask = __ballot(f);
      const int before = __popcll(mask & ((uint64_t(1) << lane) - 1));
      if (lane == 0) wcount[wv] = __popcll(mask);
      __syncthreads();
      int off = total;
      for (int w = 0; w < wv; ++w) off += wcount[w];
      const int chunk = wcount[0] + wcount[1] + wcount[2] + wcount[3];
      if (f && off + before < kFchlMaxNb) {
        const int sl = off + before;
        nidx[sl] = int32_t(j - a0);
        nx[sl] = dx;
        ny[sl] = dy;
        nz[sl] = dz;
        nr[sl] = r;
      }
      total += chunk;
      __syncthreads();
    }
  }
  const bool bad = total > kFchlMaxNb;   // uniform: every thread counted the same chunks
  double px = 0.0, py = 0.0, pz = 0.0;   // FP64 sums: a large centre adds thousands of terms
  if (!bad) {
    if (tid == 0) {
      grp[E] = total;
      int64_t o = 0;
      for (int X = 0; X < E; ++X)
        for (int Y = X; Y < E; ++Y) {
          seg[fchl_pair(X, Y, E)] = o;
          const int64_t cxn = grp[X + 1] - grp[X], cyn = grp[Y + 1] - grp[Y];
          o += X == Y ? cxn * (cxn - 1) / 2 : cxn * cyn;
        }
      seg[NP] = o;
    }
    __syncthreads();
    const float* __restrict__ gt = g + t * size;
    // centre t, two-body
    for (int sl = tid; sl < total; sl += 256) {
      int X = 0;
      while (sl >= grp[X + 1]) ++X;
      const float r = nr[sl];
      const float f = fchl_pair_grad(r, gt + X * p.n2, p) / r;
      px -= f * nx[sl];
      py -= f * ny[sl];
      pz -= f * nz[sl];
    }
    // centre t, three-body over its unordered neighbour pairs
    const int64_t n_pairs = seg[NP];
    for (int64_t q = tid; q < n_pairs; q += 256) {
      int P = 0;
      while (q >= seg[P + 1]) ++P;
      int X = 0;
      while (fchl_pair(X, X, E) + (E - X) <= P) ++X;
      const int Y = X + (P - fchl_pair(X, X, E));
      const int64_t loc = q - seg[P];
      int sa, sb;
      if (X != Y) {
        const int cyn = grp[Y + 1] - grp[Y];
        sa = grp[X] + int(loc / cyn);
        sb = grp[Y] + int(loc % cyn);
      } else {
        const int cxn = grp[X + 1] - grp[X];
        const double c2x = 2.0 * cxn - 1.0;
        int u = int((c2x - sqrt(c2x * c2x - 8.0 * double(loc))) * 0.5);
        if (u < 0) u = 0;
        while (u > 0 && int64_t(u) * (2 * cxn - u - 1) / 2 > loc) --u;
        while (int64_t(u + 1) * (2 * cxn - u - 2) / 2 <= loc) ++u;
        sa = grp[X] + u;
        sb = grp[X] + u + 1 + int(loc - int64_t(u) * (2 * cxn - u - 1) / 2);
      }
      const float a = nr[sa], b = nr[sb];
      const float wx = nx[sb] - nx[sa], wy = ny[sb] - ny[sa], wz = nz[sb] - nz[sa];
      const float c = sqrtf(wx * wx + wy * wy + wz * wz);
      if (!(c < rc)) continue;   // f_cut(r_jl) and its derivative vanish
      float dL[3];
      fchl_triple_grad(a, b, c, gt + int64_t(E) * p.n2 + int64_t(P) * p.n3 * 2, p, angw, dL);
      const float fa = dL[0] / a, fb = dL[1] / b;
      px -= fa * nx[sa] + fb * nx[sb];
      py -= fa * ny[sa] + fb * ny[sb];
      pz -= fa * nz[sa] + fb * nz[sb];
    }
    // each neighbour c of t as a centre: t's two-body term in c's row, and
    // the pairs {t, l} of c. A pair's terms carry f_cut(r_tl), so only the
    // neighbours l of t contribute, and those are in t's list: the pairs
    // (c, l) of t's list with r_cl < r_cut, flattened over the threads
    const int et = element[t];
    for (int cs = tid; cs < total; cs += 256) {
      const float* __restrict__ gc = g + (a0 + nidx[cs]) * size;
      const float rct = nr[cs];
      const float f = fchl_pair_grad(rct, gc + et * p.n2, p) / rct;
      px -= f * nx[cs];   // (R_t - R_c) = -(R_c - R_t)
      py -= f * ny[cs];
      pz -= f * nz[cs];
    }
    const int64_t n_cl = int64_t(total) * total;
    for (int64_t q = tid; q < n_cl; q += 256) {
      const int cs = int(q / total), ls = int(q - int64_t(cs) * total);
      if (ls == cs) continue;
      const float wx = nx[ls] - nx[cs], wy = ny[ls] - ny[cs], wz = nz[ls] - nz[cs];   // R_l - R_c
      const float rcl = sqrtf(wx * wx + wy * wy + wz * wz);
      if (!(rcl < rc)) continue;
      int Y = 0;
      while (ls >= grp[Y + 1]) ++Y;
      const int P = et <= Y ? fchl_pair(et, Y, E) : fchl_pair(Y, et, E);
      const float* __restrict__ gc = g + (a0 + nidx[cs]) * size;
      const float rct = nr[cs], rtl = nr[ls];
      float dL[3];
      fchl_triple_grad(rct, rcl, rtl, gc + int64_t(E) * p.n2 + int64_t(P) * p.n3 * 2, p, angw, dL);
      // dL/da (R_t - R_c) / a + dL/dc (R_t - R_l) / c, with R_x - R_t = n[x]
      const float fa = dL[0] / rct, fc = dL[2] / rtl;
      px -= fa * nx[cs] + fc * nx[ls];
      py -= fa * ny[cs] + fc * ny[ls];
      pz -= fa * nz[cs] + fc * nz[ls];
    }
  }
  red[0][tid] = px;
  red[1][tid] = py;
  red[2][tid] = pz;
  __syncthreads();
  if (tid < 3) {
    double sum = 0.0;
    for (int k = 0; k < 256; ++k) sum += red[tid][k];
    dR[3 * t + tid] = bad ? __builtin_nanf("") : float(sum);
  }
  __syncthreads();   // red[], the neighbour list and seg[] are rewritten for the next atom
}

// Molecules above kFchlSmallAtoms atoms: a resident grid (three workgroups
// per compute unit) deals their atoms out, atom j of molecule m to workgroup
// (m + j) mod G, as the forward kernel deals the atoms of large molecules.
__global__ __launch_bounds__(256) void fchl19_backward_gather_kernel(
    const float* __restrict__ R, const int32_t* __restrict__ element,
    const int64_t* __restrict__ mol_ptr, int64_t n_mols, int32_t E, FchlParams p, int64_t size,
    const float* __restrict__ g, float* __restrict__ dR) {
  __shared__ int32_t big[256];
  __shared__ int32_t wbig[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t G = gridDim.x, b = blockIdx.x;
  for (int64_t m0 = 0; m0 < n_mols; m0 += 256) {
    const int64_t m = m0 + tid;
    const bool large = m < n_mols && mol_ptr[m + 1] - mol_ptr[m] > kFchlSmallAtoms;
    const uint64_t mask = __ballot(large);
    if (lane == 0) wbig[wv] = __popcll(mask);
    __syncthreads();
    int off = 0, nbig = 0;
    for (int w = 0; w < 4; ++w) {
      off += w < wv ? wbig[w] : 0;
      nbig += wbig[w];
    }
    if (large) big[off + __popcll(mask & ((uint64_t(1) << lane) - 1))] = tid;
    __syncthreads();
    for (int k = 0; k < nbig; ++k) {
      const int64_t mm = m0 + big[k];
      const int64_t a0 = mol_ptr[mm], a1 = mol_ptr[mm + 1];
      for (int64_t j = ((b - mm) % G + G) % G; j < a1 - a0; j += G)
        fchl19_backward_atom(a0 + j, a0, a1, R, element, E, p, size, g, dR);
    }
    __syncthreads();   // big[] and wbig[] are rewritten by the next group of molecules
  }
}

}  // namespace sorf

using namespace sorf;

int64_t sorf_fchl19_len(int32_t E, int32_t n2, int32_t n3) {
  return int64_t(E) * n2 + int64_t(E) * (E + 1) / 2 * n3 * 2;
}

hipError_t sorf_launch_fchl19_forward(const float* R, const int32_t* element,
                                      const int64_t* mol_ptr, int64_t n_atoms, int64_t n_mols,
                                      int32_t E, const FchlParamsHost& ph, float* rho,
                                      hipStream_t st) {
  if (n_atoms == 0) return hipSuccess;
  const FchlParams p{ph.n2, ph.n3, ph.eta2, ph.eta3, ph.N2, ph.N3, ph.c3, ph.zeta, ph.rcut};
  const int64_t size = sorf_fchl19_len(E, ph.n2, ph.n3);
  constexpr int64_t kPerLaunch = int64_t(1) << 30;
  for (int64_t a0 = 0; a0 < n_atoms; a0 += kPerLaunch) {
    const int64_t cnt = n_atoms - a0 < kPerLaunch ? n_atoms - a0 : kPerLaunch;
    hipLaunchKernelGGL(fchl19_forward_small_kernel, dim3(unsigned((cnt + 3) / 4)), dim3(256), 0, st,
                       R, element, mol_ptr, a0, n_atoms, n_mols, E, p, size, rho);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_mols == 0) return hipSuccess;
  // three workgroups of this kernel fit a compute unit (LDS), 256 units: the
  // whole grid is resident, so the size scan runs once
  const int64_t grid = n_atoms < 768 ? n_atoms : 768;
  hipLaunchKernelGGL(fchl19_forward_kernel, dim3(unsigned(grid)), dim3(256), 0, st, R, element,
                     mol_ptr, n_mols, E, p, size, rho);
  return hipGetLastError();
}

hipError_t sorf_launch_fchl19_backward(const float* R, const int32_t* element,
                                       const int64_t* mol_ptr, int64_t n_mols, int32_t E,
                                       const FchlParamsHost& ph, const float* g, float* dR,
                                       hipStream_t st) {
  if (n_mols == 0) return hipSuccess;
  const FchlParams p{ph.n2, ph.n3, ph.eta2, ph.eta3, ph.N2, ph.N3, ph.c3, ph.zeta, ph.rcut};
  const int64_t size = sorf_fchl19_len(E, ph.n2, ph.n3);
  constexpr int64_t kPerLaunch = int64_t(1) << 30;
  for (int64_t m0 = 0; m0 < n_mols; m0 += kPerLaunch) {
    const int64_t cnt = n_mols - m0 < kPerLaunch ? n_mols - m0 : kPerLaunch;
    if (size <= kFchlStage)
      hipLaunchKernelGGL(fchl19_backward_small_kernel<true>, dim3(unsigned(cnt)), dim3(256), 0, st,
                         R, element, mol_ptr, m0, n_mols, E, p, size, g, dR);
    else
      hipLaunchKernelGGL(fchl19_backward_small_kernel<false>, dim3(unsigned(cnt)), dim3(256), 0,
                         st, R, element, mol_ptr, m0, n_mols, E, p, size, g, dR);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // molecules above kFchlSmallAtoms atoms: a resident grid, one workgroup per atom
  hipLaunchKernelGGL(fchl19_backward_gather_kernel, dim3(768u), dim3(256), 0, st, R, element,
                     mol_ptr, n_mols, E, p, size, g, dR);
  return hipGetLastError();
}
