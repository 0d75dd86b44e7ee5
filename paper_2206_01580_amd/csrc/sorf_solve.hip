// Ridge solve (G + lambda I) alpha = Zty in FP64 on gfx950.
//
// Paper: arXiv 2206.01580, RFF subsection (regularised normal equation, solved
// by a matrix decomposition on the GPU; the matrix is symmetric positive
// definite for lambda > 0, so a Cholesky factorisation gives the paper's alpha)
// and the Training-time discussion (FP32 round-off in Z^T Z harms the
// conditioning; here the factorisation, the triangular solves and the residual
// of the iterative refinement are all FP64).
//
// Blocked right-looking Cholesky with panel width NB = 64:
//   1. factor the NB x NB diagonal block in LDS and form its inverse,
//   2. panel below: L21 = A21 L11^{-T} = A21 (L11^{-1})^T,
//   3. trailing update A22 -= L21 L21^T on the lower triangle with FP64 MFMA.
// Triangular solves use the inverted diagonal blocks: one launch per block
// row, every workgroup recomputing the block's solution from the (unchanged)
// right-hand side and updating its share of the remaining rows.
#include <cmath>

#include "sorf_internal.h"

namespace sorf {

constexpr int NB = 64;
typedef double f64x4 __attribute__((ext_vector_type(4)));

static __device__ __forceinline__ void tri_tile(int64_t t, int64_t& I, int64_t& J) {
  int64_t i = int64_t((std::sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

struct SolveWs {
  double* A;     // [D][D], lower triangle used
  double* Linv;  // [nblk][NB][NB] inverses of the diagonal blocks
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

// Factor the diagonal block at (k, k) and write its inverse.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ A, int32_t D, int32_t k,
                                                        int32_t* __restrict__ info,
                                                        double* __restrict__ Linv) {
  __shared__ double L[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int tid = threadIdx.x;
  const int nbk = (D - k) < NB ? (D - k) : NB;
  for (int t = tid; t < NB * NB; t += 256) {
    const int i = t / NB, j = t % NB;
    L[i][j] = (i < nbk && j <= i) ? A[int64_t(k + i) * D + (k + j)] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nbk; ++j) {
    if (tid == 0) {
      double p = L[j][j];
      if (!(p > 0.0) || !std::isfinite(p)) {
        if (*info == 0) *info = k + j + 1;
        p = __builtin_nan("");
      }
      L[j][j] = std::sqrt(p);
    }
    __syncthreads();
    const double piv = L[j][j];
    for (int i = j + 1 + tid; i < nbk; i += 256) L[i][j] /= piv;
    __syncthreads();
    const int w = nbk - j - 1;
    for (int t = tid; t < w * w; t += 256) {
      const int i = j + 1 + t / w, l = j + 1 + t % w;
      if (l <= i) L[i][l] -= L[i][j] * L[l][j];
    }
    __syncthreads();
  }
  for (int t = tid; t < nbk * nbk; t += 256) {
    const int i = t / nbk, j = t % nbk;
    if (j <= i) A[int64_t(k + i) * D + (k + j)] = L[i][j];
  }
  // inverse of the lower-triangular block, one column per thread
  if (tid < NB) {
    const int c = tid;
    for (int i = 0; i < NB; ++i) X[i][c] = 0.0;
    if (c < nbk) {
      X[c][c] = 1.0 / L[c][c];
      for (int i = c + 1; i < nbk; ++i) {
        double s = 0.0;
        for (int p = c; p < i; ++p) s += L[i][p] * X[p][c];
        X[i][c] = -s / L[i][i];
      }
    }
  }
  __syncthreads();
  double* out = Linv + int64_t(k / NB) * NB * NB;
  for (int t = tid; t < NB * NB; t += 256) out[t] = X[t / NB][t % NB];
}

// Panel below the diagonal block: L21 = A21 (L11^{-1})^T, 64 rows per group.
__global__ __launch_bounds__(256) void trsm_kernel(double* __restrict__ A, int32_t D, int32_t k,
                                                  const double* __restrict__ Linv) {
  __shared__ double P[64][NB + 1];
  __shared__ double V[NB][NB + 1];
  const int tid = threadIdx.x;
  const int64_t r0 = int64_t(k) + NB + int64_t(blockIdx.x) * 64;
  const double* inv = Linv + int64_t(k / NB) * NB * NB;
  for (int t = tid; t < 64 * NB; t += 256) {
    const int i = t / NB, j = t % NB;
    P[i][j] = (r0 + i < D) ? A[(r0 + i) * D + k + j] : 0.0;
    V[i][j] = inv[t];
  }
  __syncthreads();
  const int row = tid >> 2;
  const int part = tid & 3;
  if (r0 + row < D) {
    for (int j = part; j < NB; j += 4) {
      double s = 0.0;
      for (int p = 0; p <= j; ++p) s += P[row][p] * V[j][p];
      A[(r0 + row) * D + k + j] = s;
    }
  }
}

// Trailing update A22 -= L21 L21^T on the lower triangle (64 x 64 tiles).
__global__ __launch_bounds__(256) void syrk_kernel(double* __restrict__ A, int32_t D, int32_t k) {
  __shared__ double LI[64][NB + 1];
  __shared__ double LJ[64][NB + 1];
  int64_t I, J;
  tri_tile(blockIdx.x, I, J);
  const int64_t s0 = int64_t(k) + NB;
  const int64_t I0 = s0 + I * 64, J0 = s0 + J * 64;
  const int tid = threadIdx.x;
  for (int t = tid; t < 64 * NB; t += 256) {
    const int i = t / NB, p = t % NB;
    LI[i][p] = (I0 + i < D) ? A[(I0 + i) * D + k + p] : 0.0;
    LJ[i][p] = (J0 + i < D) ? A[(J0 + i) * D + k + p] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv >> 1, wx = wv & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < NB; kk += 4) {
    const int p = kk + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      av[b] = LI[wy * 32 + b * 16 + (lane & 15)][p];
      bv[b] = LJ[wx * 32 + b * 16 + (lane & 15)][p];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
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
        if (gi < D && gj < D && gi >= gj) A[gi * D + gj] -= acc[a][b][r];
      }
}

// Forward substitution, block row k: y_k = L_kk^{-1} b_k; b_i -= L_ik y_k below.
__global__ __launch_bounds__(256) void trsv_fwd_kernel(const double* __restrict__ A,
                                                      const double* __restrict__ Linv, int32_t D,
                                                      int32_t k, double* __restrict__ b,
                                                      double* __restrict__ y) {
  __shared__ double yk[NB];
  const int tid = threadIdx.x;
  const int nbk = (D - k) < NB ? (D - k) : NB;
  const double* inv = Linv + int64_t(k / NB) * NB * NB;
  if (tid < nbk) {
    double s = 0.0;
    for (int p = 0; p <= tid; ++p) s += inv[tid * NB + p] * b[k + p];
    yk[tid] = s;
    if (blockIdx.x == 0) y[k + tid] = s;
  }
  __syncthreads();
  const int64_t i = int64_t(k) + nbk + int64_t(blockIdx.x) * 256 + tid;
  if (i < D) {
    const double* row = A + i * D + k;
    double s = 0.0;
    for (int p = 0; p < nbk; ++p) s += row[p] * yk[p];
    b[i] -= s;
  }
}

// Back substitution with L^T, block row k: x_k = L_kk^{-T} c_k; c_i -= L_ki^T x_k above.
__global__ __launch_bounds__(256) void trsv_bwd_kernel(const double* __restrict__ A,
                                                      const double* __restrict__ Linv, int32_t D,
                                                      int32_t k, double* __restrict__ c,
                                                      double* __restrict__ x) {
  __shared__ double xk[NB];
  const int tid = threadIdx.x;
  const int nbk = (D - k) < NB ? (D - k) : NB;
  const double* inv = Linv + int64_t(k / NB) * NB * NB;
  if (tid < nbk) {
    double s = 0.0;
    for (int p = tid; p < nbk; ++p) s += inv[p * NB + tid] * c[k + p];
    xk[tid] = s;
    if (blockIdx.x == 0) x[k + tid] = s;
  }
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * 256 + tid;
  if (i < k) {
    double s = 0.0;
    for (int p = 0; p < nbk; ++p) s += A[int64_t(k + p) * D + i] * xk[p];
    c[i] -= s;
  }
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
  for (int32_t k = 0; k < D; k += NB) {
    const int32_t nbk = (D - k) < NB ? (D - k) : NB;
    const int64_t rest = int64_t(D) - k - nbk;
    const unsigned g = unsigned(rest > 0 ? (rest + 255) / 256 : 1);
    hipLaunchKernelGGL(trsv_fwd_kernel, dim3(g), dim3(256), 0, st, w.A, w.Linv, D, k, rhs, tmp);
  }
  const int32_t last = ((D - 1) / NB) * NB;
  for (int32_t k = last; k >= 0; k -= NB) {
    const unsigned g = unsigned(k > 0 ? (int64_t(k) + 255) / 256 : 1);
    hipLaunchKernelGGL(trsv_bwd_kernel, dim3(g), dim3(256), 0, st, w.A, w.Linv, D, k, tmp, out);
  }
  return hipGetLastError();
}

}  // namespace sorf

using namespace sorf;

size_t sorf_solve_ws_bytes(int32_t D) {
  const size_t nblk = (size_t(D) + NB - 1) / NB;
  const size_t nt = (size_t(D) + 63) / 64;
  return align256(sizeof(double) * size_t(D) * D) + align256(sizeof(double) * nblk * NB * NB) +
         3 * align256(sizeof(double) * D) + align256(sizeof(double) * nt * nt * 64);
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
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, w.A, D, k, info, w.Linv);
    const int64_t rest = int64_t(D) - k - NB;
    if (rest > 0) {
      const int64_t nt = (rest + 63) / 64;
      hipLaunchKernelGGL(trsm_kernel, dim3(unsigned(nt)), dim3(256), 0, st, w.A, D, k, w.Linv);
      hipLaunchKernelGGL(syrk_kernel, dim3(unsigned(nt * (nt + 1) / 2)), dim3(256), 0, st, w.A, D, k);
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
