// Per-element projection of the atomic representation to d = 2^n entries
// (arXiv 2206.01580, Theory section, SORF subsection): x_i = rho_i^T U_{e_i},
// where U_e holds the first d left singular vectors of element e's sampled
// representations. Every element has its own matrix, so the product is a
// grouped GEMM: the atoms are bucketed by element, and each bucket is
// multiplied by its element's d_rep x d matrix on the FP32 matrix cores.
//
// Launches:
//   count    per-element atom counts (LDS histogram per block, then one
//            integer atomic per element and block);
//   offsets  one block: bucket offsets, bucket cursors and tile offsets;
//   scatter  every atom takes a slot of its element's bucket (a block
//            reserves its atoms' ranges with one atomic per element); the
//            order inside a bucket varies between runs, but each output row
//            depends on its own input row only, so x does not;
//   gemm     one workgroup per 128 atoms of one bucket x 128 output columns.
//            rho rows are gathered through the bucket list into LDS as
//            [k][atom], U_e rows as [k][column], both double-buffered in
//            chunks of 16 k with the next chunk held in registers while the
//            current one is multiplied. Each wave owns 32 atoms x 128 columns
//            (4 blocks of v_mfma_f32_32x32x2f32) and writes its rows once.
#include "sorf_internal.h"

namespace sorf {

constexpr int kProjRows = 128;   // atoms per tile
constexpr int kProjCols = 128;   // output columns per tile
constexpr int kProjK = 16;       // k per LDS stage
constexpr int kProjMaxElements = 256;

typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void proj_count_kernel(const int32_t* __restrict__ element,
                                                         int64_t n, int32_t E,
                                                         unsigned long long* __restrict__ counts) {
  __shared__ unsigned int h[kProjMaxElements];
  for (int i = threadIdx.x; i < E; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  for (int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; a < n;
       a += int64_t(gridDim.x) * blockDim.x) {
    const int32_t e = element[a];
    if (e >= 0 && e < E) atomicAdd(&h[e], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < E; i += blockDim.x)
    if (h[i] != 0u) atomicAdd(&counts[i], static_cast<unsigned long long>(h[i]));
}

// off[e] = atoms of elements before e; cursor[e] = off[e]; tiles[e] = tiles of
// elements before e (tiles[E] = all tiles).
__global__ void proj_offsets_kernel(const unsigned long long* __restrict__ counts, int32_t E,
                                    int64_t* __restrict__ off,
                                    unsigned long long* __restrict__ cursor,
                                    int64_t* __restrict__ tiles) {
  if (threadIdx.x != 0) return;
  int64_t o = 0, t = 0;
  for (int32_t e = 0; e < E; ++e) {
    off[e] = o;
    cursor[e] = static_cast<unsigned long long>(o);
    tiles[e] = t;
    const int64_t c = int64_t(counts[e]);
    o += c;
    t += (c + kProjRows - 1) / kProjRows;
  }
  off[E] = o;
  tiles[E] = t;
}

// A block owns a contiguous run of atoms. It counts them per element in LDS,
// reserves each element's range in the bucket with one global atomic, and
// hands out the slots of that range with LDS atomics.
__global__ __launch_bounds__(256) void proj_scatter_kernel(const int32_t* __restrict__ element,
                                                           int64_t n, int32_t E,
                                                           unsigned long long* __restrict__ cursor,
                                                           int64_t* __restrict__ perm) {
  __shared__ unsigned int h[kProjMaxElements];
  __shared__ unsigned long long base[kProjMaxElements];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t a0 = int64_t(blockIdx.x) * per;
  const int64_t a1 = a0 + per < n ? a0 + per : n;
  for (int i = threadIdx.x; i < E; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  for (int64_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
    const int32_t e = element[a];
    if (e >= 0 && e < E) atomicAdd(&h[e], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < E; i += blockDim.x) {
    base[i] = h[i] != 0u ? atomicAdd(&cursor[i], static_cast<unsigned long long>(h[i])) : 0ull;
    h[i] = 0u;
  }
  __syncthreads();
  for (int64_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
    const int32_t e = element[a];
    if (e >= 0 && e < E) perm[int64_t(base[e] + atomicAdd(&h[e], 1u))] = a;
  }
}

template <bool VEC4>
__global__ __launch_bounds__(256) void proj_gemm_kernel(
    const float* __restrict__ rho, int32_t d_rep, const float* __restrict__ U, int32_t d,
    int32_t E, const int64_t* __restrict__ off, const int64_t* __restrict__ tiles,
    const int64_t* __restrict__ perm, float* __restrict__ x) {
  constexpr int LDA = kProjRows + 4, LDB = kProjCols + 4;
  __shared__ float sA[2][kProjK][LDA];
  __shared__ __attribute__((aligned(16))) float sB[2][kProjK][LDB];
  __shared__ int64_t sPerm[kProjRows];

  // tile -> (element, first bucket slot)
  const int64_t t = blockIdx.x;
  if (t >= tiles[E]) return;
  int32_t e = 0;
  while (t >= tiles[e + 1]) ++e;
  const int64_t r0 = off[e] + (t - tiles[e]) * kProjRows;
  const int nrows = int(off[e + 1] - r0 < kProjRows ? off[e + 1] - r0 : kProjRows);
  const int64_t c0 = int64_t(blockIdx.y) * kProjCols;
  const int ncols = int(d - c0 < kProjCols ? d - c0 : kProjCols);
  const float* __restrict__ Ue = U + int64_t(e) * d_rep * d;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  if (tid < kProjRows) sPerm[tid] = perm[r0 + (tid < nrows ? tid : nrows - 1)];
  __syncthreads();

  // A: thread -> atom tid / 2, k = 8 (tid % 2) .. + 7; B: k = tid / 16, columns 8 (tid % 16) .. + 7
  const int ar = tid >> 1, ak = (tid & 1) * 8;
  const int bk = tid >> 4, bc = (tid & 15) * 8;
  const float* __restrict__ arow = rho + sPerm[ar] * int64_t(d_rep);
  float pa[8], pb[8];
  auto load = [&](int k0) {
    const int ka = k0 + ak;
    if (VEC4 && ka + 8 <= d_rep) {
      const float4 u = *reinterpret_cast<const float4*>(arow + ka);
      const float4 w = *reinterpret_cast<const float4*>(arow + ka + 4);
      pa[0] = u.x; pa[1] = u.y; pa[2] = u.z; pa[3] = u.w;
      pa[4] = w.x; pa[5] = w.y; pa[6] = w.z; pa[7] = w.w;
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = ka + j;
        const float v = arow[k < d_rep ? k : d_rep - 1];
        pa[j] = k < d_rep ? v : 0.0f;
      }
    }
    const int kb = k0 + bk;
    const int64_t cb = c0 + bc;
    const int kbc = kb < d_rep ? kb : d_rep - 1;
    const float* __restrict__ brow = Ue + int64_t(kbc) * d;
    if (VEC4 && kb < d_rep && cb + 8 <= d) {
      const float4 u = *reinterpret_cast<const float4*>(brow + cb);
      const float4 w = *reinterpret_cast<const float4*>(brow + cb + 4);
      pb[0] = u.x; pb[1] = u.y; pb[2] = u.z; pb[3] = u.w;
      pb[4] = w.x; pb[5] = w.y; pb[6] = w.z; pb[7] = w.w;
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t c = cb + j;
        const float v = brow[c < d ? c : d - 1];
        pb[j] = (kb < d_rep && c < d) ? v : 0.0f;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 8; ++j) sA[buf][ak + j][ar] = pa[j];
    *reinterpret_cast<float4*>(&sB[buf][bk][bc]) = make_float4(pb[0], pb[1], pb[2], pb[3]);
    *reinterpret_cast<float4*>(&sB[buf][bk][bc + 4]) = make_float4(pb[4], pb[5], pb[6], pb[7]);
  };

  f32x16 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[b][r] = 0.0f;

  const int n_stages = (d_rep + kProjK - 1) / kProjK;
  load(0);
  store(0);
  __syncthreads();
  for (int s = 0; s < n_stages; ++s) {
    const int buf = s & 1;
    if (s + 1 < n_stages) load((s + 1) * kProjK);
#pragma unroll
    for (int kk = 0; kk < kProjK; kk += 2) {
      const int k = kk + (lane >> 5);
      const float a = sA[buf][k][wv * 32 + (lane & 31)];
      float bv[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sB[buf][k][b * 32 + (lane & 31)];
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv[b], acc[b], 0, 0, 0);
    }
    if (s + 1 < n_stages) store(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wv * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int col = b * 32 + (lane & 31);
      if (row < nrows && col < ncols) x[sPerm[row] * int64_t(d) + c0 + col] = acc[b][r];
    }
}

// ---------------------------------------------------------------------------
// Fit of one element's projection (SORF subsection: Z~_e = U_e S_e V_e^T over
// sampled representations, U_e^{N_PCA} its first N_PCA columns). The left
// singular vectors of Z~_e are the eigenvectors of G = Z~_e Z~_e^T = sum over
// the sampled rows of rho^T rho (d_rep x d_rep), and the singular values the
// square roots of its eigenvalues. G is formed in FP64 by the FP64 Gram kernel;
// its eigenvectors come from the cyclic Jacobi method in FP64 with the
// round-robin ordering, which rotates m / 2 disjoint index pairs at a time
// (m = d_rep rounded up to even; a padded zero row and column is never
// rotated). A step computes every pair's rotation from the diagonal 2 x 2
// blocks of A and applies all of them at once: the (a, b) block of the new
// A is R_a^T A_ab R_b, so one thread per block needs nothing from the others
// (A is double-buffered), and V = V R in place. After each sweep (m - 1 steps)
// one block sums the squared off-diagonal entries directly (not as a
// difference of totals, which cancels) and stops the iteration once they are
// below 1e-30 of the total, or after kFitMaxSweeps sweeps.
// ---------------------------------------------------------------------------
constexpr int kFitMaxSweeps = 15;

__device__ __forceinline__ void fit_pair(int a, int k, int m, int& p, int& q) {
  // slot 0 keeps player 0; the other players rotate by one slot per step
  auto player = [&](int slot) { return slot == 0 ? 0 : 1 + (slot - 1 + k) % (m - 1); };
  const int u = player(a), v = player(m - 1 - a);
  p = u < v ? u : v;
  q = u < v ? v : u;
}

// rotation (c, s) with J = [[c, s], [-s, c]] on (p, q) that zeroes (J^T A J)_pq
__device__ __forceinline__ void fit_rotation(const double* __restrict__ A, int m, int p, int q,
                                             double& c, double& s) {
  const double apq = A[int64_t(p) * m + q];
  if (apq == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double tau = (A[int64_t(q) * m + q] - A[int64_t(p) * m + p]) / (2.0 * apq);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// A (m x m) = the symmetric matrix whose lower triangle is G (n x n), zero-padded;
// V = I; done = 0
__global__ __launch_bounds__(256) void fit_init_kernel(const double* __restrict__ G, int n, int m,
                                                       double* __restrict__ A,
                                                       double* __restrict__ V,
                                                       int32_t* __restrict__ done) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(m) * m) return;
  const int i = int(t / m), j = int(t % m);
  double v = 0.0;
  if (i < n && j < n) v = i >= j ? G[int64_t(i) * n + j] : G[int64_t(j) * n + i];
  A[t] = v;
  V[t] = i == j ? 1.0 : 0.0;
  if (t == 0) *done = 0;
}

__global__ __launch_bounds__(256) void fit_step_kernel(const double* __restrict__ Ain,
                                                       double* __restrict__ Aout,
                                                       double* __restrict__ V, int m, int k,
                                                       const int32_t* __restrict__ done) {
  if (*done) return;
  const int h = m / 2;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nblk = int64_t(h) * h;
  if (t < nblk) {
    const int a = int(t / h), b = int(t % h);
    int pa, qa, pb, qb;
    fit_pair(a, k, m, pa, qa);
    fit_pair(b, k, m, pb, qb);
    double ca, sa, cb, sb;
    fit_rotation(Ain, m, pa, qa, ca, sa);
    fit_rotation(Ain, m, pb, qb, cb, sb);
    const double x = Ain[int64_t(pa) * m + pb], y = Ain[int64_t(pa) * m + qb];
    const double z = Ain[int64_t(qa) * m + pb], w = Ain[int64_t(qa) * m + qb];
    const double x1 = x * cb - y * sb, y1 = x * sb + y * cb;
    const double z1 = z * cb - w * sb, w1 = z * sb + w * cb;
    Aout[int64_t(pa) * m + pb] = ca * x1 - sa * z1;
    Aout[int64_t(pa) * m + qb] = ca * y1 - sa * w1;
    Aout[int64_t(qa) * m + pb] = sa * x1 + ca * z1;
    Aout[int64_t(qa) * m + qb] = sa * y1 + ca * w1;
  } else if (t < nblk + int64_t(m) * h) {
    const int64_t u = t - nblk;
    const int i = int(u / h), a = int(u % h);
    int p, q;
    fit_pair(a, k, m, p, q);
    double c, s;
    fit_rotation(Ain, m, p, q, c, s);
    const double vp = V[int64_t(i) * m + p], vq = V[int64_t(i) * m + q];
    V[int64_t(i) * m + p] = vp * c - vq * s;
    V[int64_t(i) * m + q] = vp * s + vq * c;
  }
}

// end of a sweep: stop when the off-diagonal mass is negligible (or on the last sweep)
__global__ __launch_bounds__(1024) void fit_check_kernel(const double* __restrict__ A, int m,
                                                         int last, int32_t* __restrict__ done,
                                                         double* __restrict__ lam) {
  __shared__ double so[1024], st[1024];
  if (*done) return;
  double off = 0.0, tot = 0.0;
  for (int64_t t = threadIdx.x; t < int64_t(m) * m; t += 1024) {
    const double v = A[t];
    tot += v * v;
    if (t / m != t % m) off += v * v;
  }
  so[threadIdx.x] = off;
  st[threadIdx.x] = tot;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      st[threadIdx.x] += st[threadIdx.x + w];
    }
    __syncthreads();
  }
  const bool stop = last || so[0] <= 1e-30 * st[0];
  if (stop) {
    for (int i = threadIdx.x; i < m; i += 1024) lam[i] = A[int64_t(i) * m + i];
  }
  __syncthreads();
  if (stop && threadIdx.x == 0) *done = 1;
}

// column r of U = eigenvector of the r-th largest eigenvalue (ties: lower index
// first), sign fixed by its largest-magnitude entry (ties: lower row first)
__global__ __launch_bounds__(256) void fit_select_kernel(const double* __restrict__ lam,
                                                         const double* __restrict__ V, int n,
                                                         int m, int n_pca, float* __restrict__ U,
                                                         double* __restrict__ sv) {
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double li = lam[i];
  int rank = 0;
  for (int j = 0; j < n; ++j) rank += (lam[j] > li || (lam[j] == li && j < i)) ? 1 : 0;
  if (rank >= n_pca) return;
  int piv = 0;
  double best = -1.0;
  for (int r = 0; r < n; ++r) {
    const double a = fabs(V[int64_t(r) * m + i]);
    if (a > best) {
      best = a;
      piv = r;
    }
  }
  const double sgn = V[int64_t(piv) * m + i] < 0.0 ? -1.0 : 1.0;
  for (int r = 0; r < n; ++r) U[int64_t(r) * n_pca + rank] = float(sgn * V[int64_t(r) * m + i]);
  if (sv != nullptr) sv[rank] = sqrt(li > 0.0 ? li : 0.0);
}

}  // namespace sorf

using namespace sorf;

size_t sorf_project_ws_bytes(int64_t n_atoms, int32_t n_elements) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t E = size_t(n_elements);
  return al(8 * E) + al(8 * (E + 1)) + al(8 * E) + al(8 * (E + 1)) + al(8 * size_t(n_atoms));
}

hipError_t sorf_launch_project(int64_t n_atoms, int32_t d_rep, const float* rho,
                               const int32_t* element, int32_t E, const float* U, int32_t d,
                               float* x, void* ws, hipStream_t st) {
  if (n_atoms == 0) return hipSuccess;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* p = static_cast<char*>(ws);
  auto* counts = reinterpret_cast<unsigned long long*>(p);
  p += al(8 * size_t(E));
  auto* off = reinterpret_cast<int64_t*>(p);
  p += al(8 * size_t(E + 1));
  auto* cursor = reinterpret_cast<unsigned long long*>(p);
  p += al(8 * size_t(E));
  auto* tiles = reinterpret_cast<int64_t*>(p);
  p += al(8 * size_t(E + 1));
  auto* perm = reinterpret_cast<int64_t*>(p);

  // counts start at zero: a fill kernel, not a memset, so the call can be captured
  hipError_t err = sorf_launch_fill(reinterpret_cast<float*>(counts), 2 * int64_t(E), 0.0f, st);
  if (err != hipSuccess) return err;
  int64_t blocks = (n_atoms + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(proj_count_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, element, n_atoms,
                     E, counts);
  hipLaunchKernelGGL(proj_offsets_kernel, dim3(1), dim3(64), 0, st, counts, E, off, cursor, tiles);
  hipLaunchKernelGGL(proj_scatter_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, element,
                     n_atoms, E, cursor, perm);
  // at most ceil(A / 128) + E tiles; blocks past the real count exit
  const int64_t max_tiles = (n_atoms + kProjRows - 1) / kProjRows + E;
  const dim3 grid(unsigned(max_tiles), unsigned((d + kProjCols - 1) / kProjCols));
  const bool vec4 = (d_rep % 4 == 0) && (d % 4 == 0) &&
                    (reinterpret_cast<uintptr_t>(rho) & 15u) == 0 &&
                    (reinterpret_cast<uintptr_t>(U) & 15u) == 0;
  if (vec4)
    hipLaunchKernelGGL(proj_gemm_kernel<true>, grid, dim3(256), 0, st, rho, d_rep, U, d, E, off,
                       tiles, perm, x);
  else
    hipLaunchKernelGGL(proj_gemm_kernel<false>, grid, dim3(256), 0, st, rho, d_rep, U, d, E, off,
                       tiles, perm, x);
  return hipGetLastError();
}

size_t sorf_fit_ws_bytes(int32_t d_rep) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t n = size_t(d_rep), m = n + (n & 1);
  return al(8 * n * n) + 3 * al(8 * m * m) + al(8 * m) + al(4);
}

hipError_t sorf_launch_projection_fit(int64_t n_samples, int32_t d_rep, const float* sample,
                                      int32_t n_pca, float* U, double* sv, void* ws,
                                      hipStream_t st) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const int n = d_rep, m = d_rep + (d_rep & 1);
  char* p = static_cast<char*>(ws);
  double* G = reinterpret_cast<double*>(p);
  p += al(8 * size_t(n) * n);
  double* A[2];
  A[0] = reinterpret_cast<double*>(p);
  p += al(8 * size_t(m) * m);
  A[1] = reinterpret_cast<double*>(p);
  p += al(8 * size_t(m) * m);
  double* V = reinterpret_cast<double*>(p);
  p += al(8 * size_t(m) * m);
  double* lam = reinterpret_cast<double*>(p);
  p += al(8 * size_t(m));
  int32_t* done = reinterpret_cast<int32_t*>(p);

  hipError_t err = sorf_launch_fill(reinterpret_cast<float*>(G), 2 * int64_t(n) * n, 0.0f, st);
  if (err != hipSuccess) return err;
  err = sorf_launch_gram_f64(n_samples, n, sample, nullptr, G, nullptr, st);
  if (err != hipSuccess) return err;
  const int64_t mm = int64_t(m) * m;
  hipLaunchKernelGGL(fit_init_kernel, dim3(unsigned((mm + 255) / 256)), dim3(256), 0, st, G, n,
                     m, A[0], V, done);
  const int h = m / 2;
  const int64_t threads = int64_t(h) * h + int64_t(m) * h;
  const dim3 sgrid(unsigned((threads + 255) / 256));
  int cur = 0;
  for (int sweep = 0; sweep < kFitMaxSweeps; ++sweep) {
    for (int k = 0; k < m - 1; ++k) {
      hipLaunchKernelGGL(fit_step_kernel, sgrid, dim3(256), 0, st, A[cur], A[cur ^ 1], V, m, k,
                         done);
      cur ^= 1;
    }
    hipLaunchKernelGGL(fit_check_kernel, dim3(1), dim3(1024), 0, st, A[cur], m,
                       int(sweep == kFitMaxSweeps - 1), done, lam);
  }
  hipLaunchKernelGGL(fit_select_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, lam, V,
                     n, m, n_pca, U, sv);
  return hipGetLastError();
}
