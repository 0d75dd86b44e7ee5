// Ridge solve (G + lambda I) alpha = Zty in FP64 on gfx950.
//
// Paper: arXiv 2206.01580, RFF subsection (regularised normal equation, solved
// by a matrix decomposition on the GPU; the matrix is symmetric positive
// definite for lambda > 0, so a Cholesky factorisation gives the paper's alpha)
// and the Training-time discussion (FP32 round-off in Z^T Z harms the
// conditioning; here the factorisation, the triangular solves and the residual
// of the iterative refinement are all FP64).
//
// Blocked right-looking Cholesky with panel width NB = 128:
//   1. factor the NB x NB diagonal block in LDS (right-looking, 512 threads)
//      and invert it in place (column sweep from the right),
//   2. panel below: L21 = A21 L11^{-T} = A21 (L11^{-1})^T as an FP64 MFMA GEMM,
//   3. trailing update A22 -= L21 L21^T on the lower triangle, 128 x 128
//      tiles of FP64 MFMA.
// Triangular solves use the inverted diagonal blocks: one launch per block
// row updates the remaining right-hand side with coalesced reads of L, and
// the workgroup that finishes the next block's rows also solves that block.
#include <cmath>

#include "sorf_internal.h"

namespace sorf {

constexpr int NB = 128;
typedef double f64x4 __attribute__((ext_vector_type(4)));

static __device__ __forceinline__ void tri_tile(int64_t t, int64_t& I, int64_t& J) {
  int64_t i = int64_t((std::sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

// v_mfma_f64_16x16x4f64 operands: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// the result D[l/16 + 4 r][l%16] sits in register r of lane l.
static __device__ __forceinline__ f64x4 mfma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct SolveWs {
  double* A;     // [D][D], lower triangle used
  double* Linv;  // [nblk][NB][NB] inverses of the diagonal blocks
  double* LinvT; // [nblk][NB][NB] their transposes (row access for the backward sweep)
  double* b;     // [D]
  double* y;     // [D]
  double* dx;    // [D]
  double* part;  // [nt][nt][64] partial sums of the symmetric product
};

static size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

static SolveWs carve(void* ws, int32_t D) {
  const size_t nblk = (size_t(D) + NB - 1) / NB;
  char* p = static_cast<char*>(ws);
  SolveWs w;
  w.A = reinterpret_cast<double*>(p);      p += align256(sizeof(double) * size_t(D) * D);
  w.Linv = reinterpret_cast<double*>(p);   p += align256(sizeof(double) * nblk * NB * NB);
  w.LinvT = reinterpret_cast<double*>(p);  p += align256(sizeof(double) * nblk * NB * NB);
  w.b = reinterpret_cast<double*>(p);      p += align256(sizeof(double) * D);
  w.y = reinterpret_cast<double*>(p);      p += align256(sizeof(double) * D);
  w.dx = reinterpret_cast<double*>(p);     p += align256(sizeof(double) * D);
  w.part = reinterpret_cast<double*>(p);
  return w;
}

// A = G + lambda I on the lower triangle, promoted to FP64; clears info.
template <typename TG>
__global__ __launch_bounds__(256) void promote_kernel(const TG* __restrict__ G, int32_t D,
                                                     double lambda, double* __restrict__ A,
                                                     int32_t* __restrict__ info) {
  const int64_t i = blockIdx.y;
  const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i == 0 && j == 0) *info = 0;
  if (j <= i && j < D) A[i * D + j] = double(G[i * D + j]) + (i == j ? lambda : 0.0);
}

// Factor the diagonal block at (k, k) in LDS, write L back into A and the
// inverse of L (and its transpose) into Linv / LinvT[k / NB].
// Both sweeps are right-looking: each step is one barrier-separated rank-1
// update spread over a 16 x 32 thread grid, with no dependent load chains.
__global__ __launch_bounds__(512) void potrf_diag_kernel(double* __restrict__ A, int32_t D, int32_t k,
                                                        int32_t* __restrict__ info,
                                                        double* __restrict__ Linv,
                                                        double* __restrict__ LinvT) {
  __shared__ double L[NB][NB + 1];
  __shared__ double col[NB];
  __shared__ double rowk[NB];
  __shared__ double sc[3];
  const int tid = threadIdx.x;
  const int ty = tid >> 5, tx = tid & 31;
  const int n = (D - k) < NB ? (D - k) : NB;
  for (int t = tid; t < NB * NB; t += 512) {
    const int i = t >> 7, j = t & (NB - 1);
    L[i][j] = (i < n && j <= i) ? A[int64_t(k + i) * D + (k + j)] : 0.0;
  }
  __syncthreads();
  // Cholesky: column j is scaled by 1/sqrt(d); the trailing update uses the
  // unscaled column and 1/d
  for (int j = 0; j < n; ++j) {
    if (tid < n - j) col[j + tid] = L[j + tid][j];
    if (tid == 0) {
      const double d = L[j][j];
      const bool bad = !(d > 0.0) || !std::isfinite(d);
      if (bad && *info == 0) *info = k + j + 1;
      const double piv = bad ? __builtin_nan("") : std::sqrt(d);
      sc[0] = piv;
      sc[1] = 1.0 / piv;
      sc[2] = 1.0 / d;
    }
    __syncthreads();
    const double rpiv = sc[1], rd = sc[2];
    if (tid < n - j) L[j + tid][j] = (tid == 0) ? sc[0] : col[j + tid] * rpiv;
    for (int i = j + 1 + ty; i < n; i += 16) {
      const double ci = col[i] * rd;
      for (int l = j + 1 + tx; l <= i; l += 32) L[i][l] -= ci * col[l];
    }
    __syncthreads();
  }
  for (int t = tid; t < NB * NB; t += 512) {
    const int i = t >> 7, j = t & (NB - 1);
    if (i < n && j <= i) A[int64_t(k + i) * D + (k + j)] = L[i][j];
  }
  __syncthreads();
  // in-place inverse by forward elimination of [L | I]: at step q row q is
  // divided by L[q][q] and subtracted from the rows below; the storage of
  // L[i][c] (c < i) is reused for X[i][c] once column c has been consumed
  for (int q = 0; q < n; ++q) {
    if (tid < n - q) col[q + tid] = L[q + tid][q];
    if (tid < q) rowk[tid] = L[q][tid];
    __syncthreads();
    const double inv = 1.0 / col[q];
    if (tid <= q) L[q][tid] = (tid == q) ? inv : rowk[tid] * inv;
    for (int i = q + 1 + ty; i < n; i += 16) {
      const double f = col[i] * inv;
      for (int c = tx; c <= q; c += 32) L[i][c] = (c == q) ? -f : L[i][c] - f * rowk[c];
    }
    __syncthreads();
  }
  double* out = Linv + int64_t(k / NB) * NB * NB;
  double* outT = LinvT + int64_t(k / NB) * NB * NB;
  for (int t = tid; t < NB * NB; t += 512) {
    const int i = t >> 7, j = t & (NB - 1);
    out[t] = (i < n && j <= i) ? L[i][j] : 0.0;
    outT[t] = (j < n && i <= j) ? L[j][i] : 0.0;
  }
}

// Panel below the diagonal block: L21 = A21 (L11^{-1})^T, in place.
// 64 rows x 128 columns per workgroup, K = 128 in chunks of 32 through LDS.
__global__ __launch_bounds__(256) void trsm_kernel(double* __restrict__ A, int32_t D, int32_t k,
                                                  const double* __restrict__ Linv) {
  constexpr int KC = 32;
  __shared__ double sP[64][KC + 1];
  __shared__ double sV[NB][KC + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;  // wave owns output columns [32 wv, 32 wv + 32)
  const int64_t r0 = int64_t(k) + NB + int64_t(blockIdx.x) * 64;
  const double* inv = Linv + int64_t(k / NB) * NB * NB;
  f64x4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < NB; c0 += KC) {
    for (int t = tid; t < 64 * KC; t += 256) {
      const int i = t / KC, p = t % KC;
      sP[i][p] = (r0 + i < D) ? A[(r0 + i) * D + k + c0 + p] : 0.0;
    }
    for (int t = tid; t < NB * KC; t += 256) {
      const int j = t / KC, p = t % KC;
      sV[j][p] = inv[j * NB + c0 + p];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int p = kk + (lane >> 4);
      double av[4], bv[2];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sP[a * 16 + (lane & 15)][p];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = sV[wv * 32 + b * 16 + (lane & 15)][p];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = r0 + a * 16 + (lane >> 4) + 4 * r;
        const int64_t gj = k + wv * 32 + b * 16 + (lane & 15);
        if (gi < D) A[gi * D + gj] = acc[a][b][r];
      }
}

// Trailing update A22 -= L21 L21^T on the lower triangle: 128 x 128 tiles,
// 8 waves of 32 x 64 (2 x 4 MFMA blocks), K = NB in chunks of 16 via LDS with
// a register double buffer. On a diagonal tile the waves whose block lies
// above the diagonal only help with the loads.
__global__ __launch_bounds__(512) void syrk_kernel(double* __restrict__ A, int32_t D, int32_t k) {
  constexpr int T = 128, KC = 16;
  __shared__ double sI[T][KC + 1];
  __shared__ double sJ[T][KC + 1];
  int64_t I, J;
  tri_tile(blockIdx.x, I, J);
  const bool diag = (I == J);
  const int64_t s0 = int64_t(k) + NB;
  const int64_t I0 = s0 + I * T, J0 = s0 + J * T;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv >> 1, wx = wv & 1;  // rows [32 wy, +32), columns [64 wx, +64)
  const bool idle = diag && (32 * wy + 31 < 64 * wx);
  f64x4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int lr = tid >> 2;          // row 0..127 of the slab
  const int lp = (tid & 3) * 4;     // 4 consecutive k
  const bool okI = I0 + lr < D, okJ = J0 + lr < D;
  const double* pI = A + (I0 + lr) * D + k + lp;
  const double* pJ = A + (J0 + lr) * D + k + lp;
  double rI[4], rJ[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    rI[q] = okI ? pI[q] : 0.0;
    rJ[q] = (!diag && okJ) ? pJ[q] : 0.0;
  }
  for (int c0 = 0; c0 < NB; c0 += KC) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sI[lr][lp + q] = rI[q];
      if (!diag) sJ[lr][lp + q] = rJ[q];
    }
    __syncthreads();
    if (c0 + KC < NB) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        rI[q] = okI ? pI[c0 + KC + q] : 0.0;
        rJ[q] = (!diag && okJ) ? pJ[c0 + KC + q] : 0.0;
      }
    }
    const double (*sb)[KC + 1] = diag ? sI : sJ;
    if (!idle) {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        const int p = kk + (lane >> 4);
        double av[2], bv[4];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = sI[wy * 32 + a * 16 + (lane & 15)][p];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = sb[wx * 64 + b * 16 + (lane & 15)][p];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = mfma64(av[a], bv[b], acc[a][b]);
      }
    }
    __syncthreads();
  }
  if (idle) return;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = I0 + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int64_t gj = J0 + wx * 64 + b * 16 + (lane & 15);
        if (gi < D && gj < D && gi >= gj) A[gi * D + gj] -= acc[a][b][r];
      }
}

// out[i] = sum_p M[i][p] v[p] for a 128 x 128 block M stored row-major (the
// zero half of a triangular block contributes nothing): one wave per row,
// lanes read the row as two coalesced 512-byte loads, wave-sum by xor shuffles.
static __device__ void block_mv(const double* __restrict__ M, const double* v, int n,
                                double* out_global, int tid, int nthreads) {
  const int lane = tid & 63, wv = tid >> 6, nw = nthreads >> 6;
  const double v0 = lane < n ? v[lane] : 0.0;
  const double v1 = lane + 64 < n ? v[lane + 64] : 0.0;
  for (int i = wv; i < n; i += nw) {
    const double* row = M + i * NB;
    double s = (lane < n ? row[lane] * v0 : 0.0) + (lane + 64 < n ? row[lane + 64] * v1 : 0.0);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) out_global[i] = s;
  }
}

// y_0 = L_00^{-1} b_0 (first block of the forward sweep)
__global__ __launch_bounds__(256) void trsv_fwd_first_kernel(const double* __restrict__ Linv,
                                                            int32_t D, const double* __restrict__ b,
                                                            double* __restrict__ y) {
  __shared__ double v[NB];
  const int n = D < NB ? D : NB;
  if (threadIdx.x < n) v[threadIdx.x] = b[threadIdx.x];
  __syncthreads();
  block_mv(Linv, v, n, y, threadIdx.x, 256);
}

// Forward sweep, block row k (y_k already in y): rows i >= k + n get
// b_i -= L_ik y_k. Each workgroup owns 128 rows (16 per wave, coalesced
// 512-byte row reads). Workgroup 0 owns exactly the next block, so after its
// update it solves that block: y_{k+n} = L^{-1} b_{k+n}.
__global__ __launch_bounds__(256) void trsv_fwd_kernel(const double* __restrict__ A,
                                                      const double* __restrict__ Linv, int32_t D,
                                                      int32_t k, double* __restrict__ b,
                                                      double* __restrict__ y) {
  __shared__ double vk[NB];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int n = (D - k) < NB ? (D - k) : NB;
  const double y0 = lane < n ? y[k + lane] : 0.0;
  const double y1 = lane + 64 < n ? y[k + 64 + lane] : 0.0;
  const int64_t r0 = int64_t(k) + n + int64_t(blockIdx.x) * 128;
  for (int r = 0; r < 32; ++r) {
    const int64_t i = r0 + wv * 32 + r;
    if (i >= D) break;
    const double* row = A + i * D + k;
    double s = (lane < n ? row[lane] * y0 : 0.0) + (lane + 64 < n ? row[lane + 64] * y1 : 0.0);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) b[i] -= s;
  }
  if (blockIdx.x != 0 || r0 >= D) return;
  __threadfence_block();
  __syncthreads();
  const int64_t kn = r0;  // next block start
  const int nn = (D - kn) < NB ? int(D - kn) : NB;
  if (tid < nn) vk[tid] = b[kn + tid];
  __syncthreads();
  block_mv(Linv + (kn / NB) * NB * NB, vk, nn, y + kn, tid, 256);
}

// x_last = L_last^{-T} c_last (first block of the backward sweep)
__global__ __launch_bounds__(256) void trsv_bwd_first_kernel(const double* __restrict__ LinvT,
                                                            int32_t D, const double* __restrict__ c,
                                                            double* __restrict__ x) {
  __shared__ double v[NB];
  const int k = ((D - 1) / NB) * NB;
  const int n = D - k;
  if (threadIdx.x < n) v[threadIdx.x] = c[k + threadIdx.x];
  __syncthreads();
  block_mv(LinvT + (k / NB) * NB * NB, v, n, x + k, threadIdx.x, 256);
}

// Backward sweep, block row k (x_k already in x): rows i < k get
// c_i -= sum_p L[k + p][i] x_k[p] (one thread per row, coalesced over i).
// The last workgroup owns exactly rows [k - NB, k), so after its update it
// solves that block: x_{k-NB} = L^{-T} c_{k-NB}.
__global__ __launch_bounds__(128) void trsv_bwd_kernel(const double* __restrict__ A,
                                                      const double* __restrict__ LinvT, int32_t D,
                                                      int32_t k, double* __restrict__ c,
                                                      double* __restrict__ x) {
  __shared__ double xk[NB];
  __shared__ double vk[NB];
  const int tid = threadIdx.x;
  const int n = (D - k) < NB ? (D - k) : NB;
  if (tid < n) xk[tid] = x[k + tid];
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * 128 + tid;
  if (i < k) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int p = 0;
    for (; p + 3 < n; p += 4) {
      s0 += A[int64_t(k + p) * D + i] * xk[p];
      s1 += A[int64_t(k + p + 1) * D + i] * xk[p + 1];
      s2 += A[int64_t(k + p + 2) * D + i] * xk[p + 2];
      s3 += A[int64_t(k + p + 3) * D + i] * xk[p + 3];
    }
    for (; p < n; ++p) s0 += A[int64_t(k + p) * D + i] * xk[p];
    c[i] -= (s0 + s1) + (s2 + s3);
  }
  if (int64_t(blockIdx.x) + 1 != int64_t(gridDim.x) || k == 0) return;
  __threadfence_block();
  __syncthreads();
  const int kp = k - NB;  // previous block start (full block)
  vk[tid] = c[kp + tid];
  __syncthreads();
  block_mv(LinvT + (kp / NB) * NB * NB, vk, NB, x + kp, tid, 128);
}

// Partial sums of (lower-stored symmetric G) x over 64 x 64 tiles:
// part[X][Y][.] = contribution to rows of block X from the tile pairing X and Y.
template <typename TG>
__global__ __launch_bounds__(256) void symv_tiles_kernel(const TG* __restrict__ G, int32_t D,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ part) {
  __shared__ double T[64][65];
  __shared__ double xi[64], xj[64];
  int64_t I, J;
  tri_tile(blockIdx.x, I, J);
  const int64_t nt = (int64_t(D) + 63) / 64;
  const int64_t I0 = I * 64, J0 = J * 64;
  const int tid = threadIdx.x;
  for (int t = tid; t < 64 * 64; t += 256) {
    const int i = t / 64, j = t % 64;
    const int64_t gi = I0 + i, gj = J0 + j;
    T[i][j] = (gi < D && gj < D && gj <= gi) ? double(G[gi * D + gj]) : 0.0;
  }
  if (tid < 64) {
    xi[tid] = (I0 + tid < D) ? x[I0 + tid] : 0.0;
    xj[tid] = (J0 + tid < D) ? x[J0 + tid] : 0.0;
  }
  __syncthreads();
  if (I != J) {
    if (tid < 64) {
      double s = 0.0;
      for (int j = 0; j < 64; ++j) s += T[tid][j] * xj[j];
      part[(I * nt + J) * 64 + tid] = s;
    } else if (tid < 128) {
      const int j = tid - 64;
      double s = 0.0;
      for (int i = 0; i < 64; ++i) s += T[i][j] * xi[i];
      part[(J * nt + I) * 64 + j] = s;
    }
  } else if (tid < 64) {
    const int i = tid;
    double s = 0.0;
    for (int j = 0; j <= i; ++j) s += T[i][j] * xi[j];
    for (int j = i + 1; j < 64; ++j) s += T[j][i] * xi[j];
    part[(I * nt + I) * 64 + i] = s;
  }
}

// r = Zty - lambda x - sum_Y part[X][Y] (fixed order)
template <typename TG>
__global__ __launch_bounds__(256) void residual_kernel(const double* __restrict__ part, int32_t D,
                                                      double lambda, const TG* __restrict__ rhs,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ r) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= D) return;
  const int64_t nt = (int64_t(D) + 63) / 64;
  const int64_t X = i / 64;
  double s = 0.0;
  for (int64_t Y = 0; Y < nt; ++Y) s += part[(X * nt + Y) * 64 + (i & 63)];
  r[i] = (double(rhs[i]) - lambda * x[i]) - s;
}

template <typename TG>
__global__ void to_double_kernel(const TG* __restrict__ a, double* __restrict__ b, int32_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) b[i] = double(a[i]);
}

__global__ void axpy_kernel(double* __restrict__ x, const double* __restrict__ d, int32_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) x[i] += d[i];
}

static hipError_t solve_triangular(const SolveWs& w, int32_t D, double* rhs, double* tmp,
                                   double* out, hipStream_t st) {
  // L tmp = rhs (rhs overwritten), then L^T out = tmp (tmp overwritten)
  hipLaunchKernelGGL(trsv_fwd_first_kernel, dim3(1), dim3(256), 0, st, w.Linv, D, rhs, tmp);
  for (int32_t k = 0; k + NB < D; k += NB) {
    const int64_t rest = int64_t(D) - k - NB;
    hipLaunchKernelGGL(trsv_fwd_kernel, dim3(unsigned((rest + 127) / 128)), dim3(256), 0, st,
                       w.A, w.Linv, D, k, rhs, tmp);
  }
  hipLaunchKernelGGL(trsv_bwd_first_kernel, dim3(1), dim3(256), 0, st, w.LinvT, D, tmp, out);
  const int32_t last = ((D - 1) / NB) * NB;
  for (int32_t k = last; k > 0; k -= NB) {
    hipLaunchKernelGGL(trsv_bwd_kernel, dim3(unsigned((int64_t(k) + 127) / 128)), dim3(128), 0,
                       st, w.A, w.LinvT, D, k, tmp, out);
  }
  return hipGetLastError();
}

template <typename TG>
static hipError_t launch_solve(int32_t D, const TG* G, const TG* Zty, double lambda,
                               int32_t n_refine, double* alpha, int32_t* info, void* ws,
                               hipStream_t st) {
  const SolveWs w = carve(ws, D);
  const unsigned vg = unsigned((D + 255) / 256);
  hipLaunchKernelGGL(promote_kernel<TG>, dim3(vg, unsigned(D)), dim3(256), 0, st, G, D, lambda,
                     w.A, info);
  for (int32_t k = 0; k < D; k += NB) {
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(512), 0, st, w.A, D, k, info, w.Linv,
                       w.LinvT);
    const int64_t rest = int64_t(D) - k - NB;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_kernel, dim3(unsigned((rest + 63) / 64)), dim3(256), 0, st, w.A, D,
                         k, w.Linv);
      const int64_t nt = (rest + 127) / 128;
      hipLaunchKernelGGL(syrk_kernel, dim3(unsigned(nt * (nt + 1) / 2)), dim3(512), 0, st, w.A,
                         D, k);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(to_double_kernel<TG>, dim3(vg), dim3(256), 0, st, Zty, w.b, D);
  e = solve_triangular(w, D, w.b, w.y, alpha, st);
  if (e != hipSuccess) return e;
  const int64_t nt = (int64_t(D) + 63) / 64;
  for (int32_t it = 0; it < n_refine; ++it) {
    hipLaunchKernelGGL(symv_tiles_kernel<TG>, dim3(unsigned(nt * (nt + 1) / 2)), dim3(256), 0, st,
                       G, D, alpha, w.part);
    hipLaunchKernelGGL(residual_kernel<TG>, dim3(vg), dim3(256), 0, st, w.part, D, lambda, Zty,
                       alpha, w.b);
    e = solve_triangular(w, D, w.b, w.y, w.dx, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(axpy_kernel, dim3(vg), dim3(256), 0, st, alpha, w.dx, D);
  }
  return hipGetLastError();
}

}  // namespace sorf

using namespace sorf;

size_t sorf_solve_ws_bytes(int32_t D) {
  const size_t nblk = (size_t(D) + NB - 1) / NB;
  const size_t nt = (size_t(D) + 63) / 64;
  return align256(sizeof(double) * size_t(D) * D) + 2 * align256(sizeof(double) * nblk * NB * NB) +
         3 * align256(sizeof(double) * D) + align256(sizeof(double) * nt * nt * 64);
}

hipError_t sorf_launch_solve(int32_t D, const float* G, const float* Zty, double lambda,
                             int32_t n_refine, double* alpha, int32_t* info, void* ws,
                             hipStream_t st) {
  return launch_solve<float>(D, G, Zty, lambda, n_refine, alpha, info, ws, st);
}

hipError_t sorf_launch_solve_f64(int32_t D, const double* G, const double* Zty, double lambda,
                                 int32_t n_refine, double* alpha, int32_t* info, void* ws,
                                 hipStream_t st) {
  return launch_solve<double>(D, G, Zty, lambda, n_refine, alpha, info, ws, st);
}
