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
//   1. factor the NB x NB diagonal block in LDS and invert it (one workgroup;
//      the 64 x 64 halves are factored and inverted by one wave in registers),
//   2. panel below: L21 = A21 L11^{-T} = A21 (L11^{-1})^T as an FP64 MFMA GEMM,
//      fused with the update of the next diagonal tile,
//   3. trailing update A22 -= L21 L21^T on the rest of the lower triangle,
//      128 x 128 tiles of FP64 MFMA.
// Triangular solves use the inverted diagonal blocks: one launch per sweep,
// one workgroup per block row, each waiting for the solved values it needs.
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

// Values of the triangular sweeps' outputs are their own ready signals: a
// slot holds the signalling-NaN pattern kNotReady (never produced by
// arithmetic) until its value is stored; stores and polls are agent-scope
// atomics, so they are seen across the XCDs' L2 caches.
constexpr long long kNotReady = 0x7FF4534457454550ll;

static __device__ __forceinline__ double not_ready() { return __longlong_as_double(kNotReady); }
static __device__ __forceinline__ bool is_not_ready(double v) {
  return __double_as_longlong(v) == kNotReady;
}
static __device__ __forceinline__ double poll_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
static __device__ __forceinline__ void signal_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct SolveWs {
  double* A;     // [D][D], lower triangle used
  double* Linv;  // [nblk][NB][NB] inverses of the diagonal blocks
  double* LinvT; // [nblk][NB][NB] their transposes (row access in the forward sweep)
  double* b;     // [D]
  double* y;     // [D]
  double* dx;    // [D]
  double* part;  // [nt][nt][64] partial sums of the symmetric product
  int32_t* pflags;  // [8] strip flags of the panel kernel, then of syrk_next (epoch = block + 1)
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
  p += align256(sizeof(double) * ((size_t(D) + 63) / 64) * ((size_t(D) + 63) / 64) * 64);
  w.pflags = reinterpret_cast<int32_t*>(p);
  return w;
}

// A = G + lambda I on the lower triangle, promoted to FP64; clears info.
template <typename TG>
__global__ __launch_bounds__(256) void promote_kernel(const TG* __restrict__ G, int32_t D,
                                                     double lambda, double* __restrict__ A,
                                                     int32_t* __restrict__ info,
                                                     double* y, int32_t* __restrict__ pflags) {
  const int64_t i = blockIdx.y;
  const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i == 0 && j == 0) *info = 0;
  if (i == 0 && j < 8) pflags[j] = 0;
  if (i == 0 && j < D) signal_store(y + j, not_ready());   // output of the first forward sweep
  if (j <= i && j < D) A[i * D + j] = double(G[i * D + j]) + (i == j ? lambda : 0.0);
}

// ---------------------------------------------------------------------------
// Diagonal block: factor and invert a 128 x 128 block in LDS.
//
// The block is split into 64 x 64 halves. A single wave factors (and later
// inverts) a half with no workgroup barriers: the LDS operations of one wave
// execute in order, so between steps it only waits for its own LDS traffic
// (lgkmcnt(0)) and stops the compiler from moving memory operations across
// the step (wave barrier). The couplings between the halves are 64 x 64 x 64
// products spread over all four waves.
// ---------------------------------------------------------------------------
// Row stride NB + 8 doubles: the 8 x 8 lane grids of the one-wave steps
// (rows ly + 8a, columns lx + 8b) then fall on distinct LDS banks.
constexpr int LDL = NB + 8;
typedef double LdsBlock[LDL];

// 1 / d to full double precision: hardware reciprocal plus one Newton step
// (the exact IEEE division is a longer dependent chain on the critical path).
static __device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  const double e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}

static __device__ __forceinline__ void wave_step_fence() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS reads/writes are done
  __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no compiler motion of memory accesses across
  __builtin_amdgcn_wave_barrier();
}

// One wave factors (and later inverts) a 64 x 64 half with the matrix held in
// registers: lane (ly, lx) of an 8 x 8 grid owns the entries
// (ly + 8a, lx + 8b), a, b = 0..7, for the whole factorisation. A step only
// publishes one column (and, for the inverse, one row) through a 64-entry
// LDS buffer; since one wave issues its LDS operations in order, the reads
// that follow see the published values. Step J = 8 JB + jr runs with JB
// fixed at compile time, so every register index is static; the masks that
// select the updated entries split into a factor per row block and a
// factor per column block, so the update is one FMA per entry.

// Cholesky, unscaled right-looking form: at step J every entry (i, l) with
// i >= l > J loses A[i][J] A[l][J] / A[J][J]; the columns are scaled by
// 1/sqrt(A[J][J]) after the last step (piv[] keeps the square roots).
// Software-pipelined: a step first updates the block column that holds
// column J + 1, publishes that column and issues the reads the next step
// needs (fr, cr, dJ), and only then updates the remaining block columns, so
// the LDS round trip overlaps the bulk of the FMAs.
static __device__ __forceinline__ void order_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

template <int JB, int BC>
static __device__ __forceinline__ void rpotrf_col(double (&R)[8][8], const double (&f)[8],
                                                  const double (&c)[8], bool lower) {
#pragma unroll
  for (int a = BC; a < 8; ++a)
    R[a][BC] = __builtin_fma(-f[a], a == BC ? (lower ? c[BC] : 0.0) : c[BC], R[a][BC]);
}

template <int JB>
static __device__ __forceinline__ void rpotrf_block(double (&R)[8][8], double* col, double* piv,
                                                    double* dummy, int ly, int lx, int lane,
                                                    double (&fr)[8], double (&cr)[8],
                                                    double& dJ) {
  const bool lower = ly >= lx;
  for (int jr = 0; jr < 8; ++jr) {
    const int J = 8 * JB + jr;
    const double d = dJ;
    *(lane == 0 ? &piv[J] : &dummy[lane]) = d;   // checked and rooted after the last step
    const double rd = recip(d);
    double f[8], c[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) f[a] = a >= JB ? fr[a] * rd : 0.0;
#pragma unroll
    for (int b = 0; b < 8; ++b) c[b] = (b >= JB && lx + 8 * b > J) ? cr[b] : 0.0;
    // 1. the block column of column J + 1, then publish column J + 1
    if (jr < 7) {
      rpotrf_col<JB, JB>(R, f, c, lower);
#pragma unroll
      for (int a = JB; a < 8; ++a) *(lx == jr + 1 ? &col[ly + 8 * a] : &dummy[lane]) = R[a][JB];
    } else if constexpr (JB < 7) {
      rpotrf_col<JB, JB + 1>(R, f, c, lower);
#pragma unroll
      for (int a = JB + 1; a < 8; ++a) *(lx == 0 ? &col[ly + 8 * a] : &dummy[lane]) = R[a][JB + 1];
    }
    order_fence();
    // 2. the next step's reads
    if (J + 1 < 64) {
#pragma unroll
      for (int a = JB; a < 8; ++a) {
        fr[a] = col[ly + 8 * a];
        cr[a] = col[lx + 8 * a];
      }
      dJ = col[J + 1];
    }
    order_fence();
    // 3. the remaining block columns
#pragma unroll
    for (int b = JB; b < 8; ++b) {
      if (b == JB && jr < 7) continue;
      if (b == JB + 1 && jr == 7) continue;
#pragma unroll
      for (int a = b; a < 8; ++a)
        R[a][b] = __builtin_fma(-f[a], a == b ? (lower ? c[b] : 0.0) : c[b], R[a][b]);
    }
  }
}

static __device__ __forceinline__ void wave_potrf64(LdsBlock* L, int o, int ly, int lx, int lane,
                                                    double* piv, double* col, double* dummy,
                                                    int32_t* info, int gbase, int nvalid) {
  double R[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) R[a][b] = L[o + ly + 8 * a][o + lx + 8 * b];
  // publish column 0 and read it for the first step
#pragma unroll
  for (int a = 0; a < 8; ++a) *(lx == 0 ? &col[ly + 8 * a] : &dummy[lane]) = R[a][0];
  wave_step_fence();
  double fr[8], cr[8], dJ;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    fr[a] = col[ly + 8 * a];
    cr[a] = col[lx + 8 * a];
  }
  dJ = col[0];
  order_fence();
  rpotrf_block<0>(R, col, piv, dummy, ly, lx, lane, fr, cr, dJ);
  rpotrf_block<1>(R, col, piv, dummy, ly, lx, lane, fr, cr, dJ);
  rpotrf_block<2>(R, col, piv, dummy, ly, lx, lane, fr, cr, dJ);
  rpotrf_block<3>(R, col, piv, dummy, ly, lx, lane, fr, cr, dJ);
  rpotrf_block<4>(R, col, piv, dummy, ly, lx, lane, fr, cr, dJ);
  rpotrf_block<5>(R, col, piv, dummy, ly, lx, lane, fr, cr, dJ);
  rpotrf_block<6>(R, col, piv, dummy, ly, lx, lane, fr, cr, dJ);
  rpotrf_block<7>(R, col, piv, dummy, ly, lx, lane, fr, cr, dJ);
  wave_step_fence();
  // pivots: the first one that is not positive and finite sets info
  {
    const double d = piv[lane];
    const bool bad = !(d > 0.0) || !std::isfinite(d);
    const unsigned long long m = __ballot(bad && lane < nvalid);
    if (m != 0ull && lane == 0 && *info == 0) *info = gbase + __ffsll((long long)m);
    piv[lane] = bad ? __builtin_nan("") : std::sqrt(d);
  }
  wave_step_fence();
  // L[i][l] = A[i][l] / piv[l] below the diagonal, piv[l] on it, 0 above
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int l = lx + 8 * b;
    const double p = piv[l];
    const double rp = recip(p);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int i = ly + 8 * a;
      L[o + i][o + l] = i > l ? R[a][b] * rp : (i == l ? p : 0.0);
    }
  }
  wave_step_fence();
}

// Inverse of the lower-triangular 64 x 64 half by forward elimination of
// [L | I] in place: at step Q every row i > Q loses L[i][Q] / L[Q][Q] times
// the (still unscaled) row Q of X on the columns c < Q, and X[i][Q] becomes
// -L[i][Q] / L[Q][Q]. Row Q is final after step Q except for the scale
// 1/L[Q][Q], applied at the end (rinv[] holds the reciprocal pivots). The
// columns of L are read from the untouched LDS copy; a step first finishes
// row Q + 1, publishes it and issues the next step's reads, then updates the
// remaining block rows.
template <int QB, int BR>
static __device__ __forceinline__ void rtrtri_row(double (&R)[8][8], const double (&f)[8],
                                                  const double (&r)[8], bool colq) {
#pragma unroll
  for (int b = 0; b <= QB; ++b) R[BR][b] = __builtin_fma(-f[BR], r[b], R[BR][b]);
  R[BR][QB] = colq ? -f[BR] : R[BR][QB];
}

template <int QB>
static __device__ __forceinline__ void rtrtri_block(double (&R)[8][8], const LdsBlock* L, int o,
                                                    double* rowv, const double* rinv,
                                                    double* dummy, int ly, int lx, int lane,
                                                    double (&rowr)[8], double (&coll)[8],
                                                    double& inv) {
  for (int qr = 0; qr < 8; ++qr) {
    const int Q = 8 * QB + qr;
    double f[8], r[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) f[a] = (a >= QB && ly + 8 * a > Q) ? coll[a] * inv : 0.0;
#pragma unroll
    for (int b = 0; b < 8; ++b) r[b] = (b <= QB && lx + 8 * b < Q) ? rowr[b] : 0.0;
    const bool mine = lx == qr;   // this lane holds column Q in block column QB
    // 1. row Q + 1, then publish it (entries at columns <= Q)
    if (qr < 7) {
      rtrtri_row<QB, QB>(R, f, r, mine && ly + 8 * QB > Q);
#pragma unroll
      for (int b = 0; b <= QB; ++b) *(ly == qr + 1 ? &rowv[lx + 8 * b] : &dummy[lane]) = R[QB][b];
    } else if constexpr (QB < 7) {
      rtrtri_row<QB, QB + 1>(R, f, r, mine);
#pragma unroll
      for (int b = 0; b <= QB; ++b) *(ly == 0 ? &rowv[lx + 8 * b] : &dummy[lane]) = R[QB + 1][b];
    }
    order_fence();
    // 2. the next step's reads
    if (Q + 1 < 64) {
#pragma unroll
      for (int b = 0; b < 8; ++b) rowr[b] = rowv[min(lx + 8 * b, 63)];
#pragma unroll
      for (int a = 0; a < 8; ++a) coll[a] = L[o + ly + 8 * a][o + Q + 1];
      inv = rinv[Q + 1];
    }
    order_fence();
    // 3. the remaining block rows
#pragma unroll
    for (int a = QB; a < 8; ++a) {
      if (a == QB && qr < 7) continue;
      if (a == QB + 1 && qr == 7) continue;
#pragma unroll
      for (int b = 0; b <= QB; ++b) R[a][b] = __builtin_fma(-f[a], r[b], R[a][b]);
      R[a][QB] = (mine && ly + 8 * a > Q) ? -f[a] : R[a][QB];
    }
  }
}

static __device__ __forceinline__ void wave_trtri64(LdsBlock* L, int o, int ly, int lx, int lane,
                                                    double* rinv, double* colv, double* rowv,
                                                    double* dummy) {
  (void)colv;
  rinv[lane] = recip(L[o + lane][o + lane]);
  double R[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) R[a][b] = L[o + ly + 8 * a][o + lx + 8 * b];
  wave_step_fence();
  double rowr[8], coll[8], inv;
#pragma unroll
  for (int b = 0; b < 8; ++b) rowr[b] = 0.0;   // row 0 has no entries left of the diagonal
#pragma unroll
  for (int a = 0; a < 8; ++a) coll[a] = L[o + ly + 8 * a][o];
  inv = rinv[0];
  order_fence();
  rtrtri_block<0>(R, L, o, rowv, rinv, dummy, ly, lx, lane, rowr, coll, inv);
  rtrtri_block<1>(R, L, o, rowv, rinv, dummy, ly, lx, lane, rowr, coll, inv);
  rtrtri_block<2>(R, L, o, rowv, rinv, dummy, ly, lx, lane, rowr, coll, inv);
  rtrtri_block<3>(R, L, o, rowv, rinv, dummy, ly, lx, lane, rowr, coll, inv);
  rtrtri_block<4>(R, L, o, rowv, rinv, dummy, ly, lx, lane, rowr, coll, inv);
  rtrtri_block<5>(R, L, o, rowv, rinv, dummy, ly, lx, lane, rowr, coll, inv);
  rtrtri_block<6>(R, L, o, rowv, rinv, dummy, ly, lx, lane, rowr, coll, inv);
  rtrtri_block<7>(R, L, o, rowv, rinv, dummy, ly, lx, lane, rowr, coll, inv);
  wave_step_fence();
  // row i scaled by 1/L[i][i] below the diagonal; the diagonal becomes 1/L[i][i]
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int i = ly + 8 * a;
    const double ri = rinv[i];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int c = lx + 8 * b;
      L[o + i][o + c] = c < i ? R[a][b] * ri : (c == i ? ri : 0.0);
    }
  }
  wave_step_fence();
}

// C = A B for 64 x 64 operands held in the LDS block, on FP64 MFMA: wave
// (wy, wx) computes the 32 x 32 quadrant of C at (32 wy, 32 wx).
// A[i][p] = L[ar + i][ac + p]; B[p][j] = L[br + p][bc + j], or with BT the
// transposed access B[p][j] = L[br + j][bc + p].
template <bool BT>
static __device__ __forceinline__ void lds_mm64(LdsBlock* L, int ar, int ac, int br, int bc,
                                                int wy, int wx, int lane, f64x4 (&acc)[2][2]) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < 64; kk += 4) {
    const int p = kk + lk;
    double a[2], b[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) a[x] = L[ar + 32 * wy + 16 * x + li][ac + p];
#pragma unroll
    for (int y = 0; y < 2; ++y)
      b[y] = BT ? L[br + 32 * wx + 16 * y + li][bc + p] : L[br + p][bc + 32 * wx + 16 * y + li];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = mfma64(a[x], b[y], acc[x][y]);
  }
}

// Row / column of entry r of accumulator (x, y) in lane `lane` (see mfma64).
#define SORF_MM_ROW(wy, x, lane, r) (32 * (wy) + 16 * (x) + ((lane) >> 4) + 4 * (r))
#define SORF_MM_COL(wx, y, lane) (32 * (wx) + 16 * (y) + ((lane) & 15))

// Factor the diagonal block at (k, k) and write the inverse of
// L into Linv[k / NB] (the diagonal block of L itself is not needed again:
// the panel solve and the sweeps use the inverse). 256 threads.
//   L = [L11 0; L21 L22]:  L11 = chol(A11), L21 = A21 L11^{-T},
//   L22 = chol(A22 - L21 L21^T);  L^{-1} = [X11 0; -X22 L21 X11, X22].
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ A, int32_t D, int32_t k,
                                                        int32_t* __restrict__ info,
                                                        double* __restrict__ Linv,
                                                        double* __restrict__ LinvT) {
  __shared__ double L[NB][LDL];
  __shared__ double piv[64];
  __shared__ double dummy[64];
  __shared__ double colv[64], rowv[64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wy = wv >> 1, wx = wv & 1;
  const int ly = lane >> 3, lx = lane & 7;
  const int n = (D - k) < NB ? (D - k) : NB;
  // rows past the matrix are padded with the identity; every thread issues
  // its 64 loads (column lane, rows wv + 4 m) before it stores any
  {
    const int64_t gj0 = k + min(lane, n - 1), gj1 = k + min(lane + 64, n - 1);
#pragma unroll
    for (int m0 = 0; m0 < 32; m0 += 16) {
      double v0[16], v1[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int64_t gi = k + min(wv + 4 * (m0 + m), n - 1);
        v0[m] = A[gi * D + gj0];
        v1[m] = A[gi * D + gj1];
      }
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int i = wv + 4 * (m0 + m);
        L[i][lane] = (i < n && lane <= i) ? v0[m] : (i == lane ? 1.0 : 0.0);
        L[i][lane + 64] = (i < n && lane + 64 <= i) ? v1[m] : (i == lane + 64 ? 1.0 : 0.0);
      }
    }
  }
  __syncthreads();
  if (wv == 0) wave_potrf64(L, 0, ly, lx, lane, piv, colv, dummy, info, k, n);
  __syncthreads();
  if (wv == 0) wave_trtri64(L, 0, ly, lx, lane, piv, colv, rowv, dummy);   // X11 = L11^{-1} in place
  __syncthreads();
  f64x4 acc[2][2];
  // L21 = A21 X11^T
  lds_mm64<true>(L, 64, 0, 0, 0, wy, wx, lane, acc);
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        L[64 + SORF_MM_ROW(wy, x, lane, r)][SORF_MM_COL(wx, y, lane)] = acc[x][y][r];
  __syncthreads();
  // A22 -= L21 L21^T (lower part)
  lds_mm64<true>(L, 64, 0, 64, 0, wy, wx, lane, acc);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = SORF_MM_ROW(wy, x, lane, r), j = SORF_MM_COL(wx, y, lane);
        if (j <= i) L[64 + i][64 + j] -= acc[x][y][r];
      }
  __syncthreads();
  if (wv == 0) wave_potrf64(L, 64, ly, lx, lane, piv, colv, dummy, info, k + 64, n - 64);
  __syncthreads();
  if (wv == 0) wave_trtri64(L, 64, ly, lx, lane, piv, colv, rowv, dummy);   // X22 = L22^{-1} in place
  __syncthreads();
  // T = L21 X11, stored over L21
  lds_mm64<false>(L, 64, 0, 0, 0, wy, wx, lane, acc);
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        L[64 + SORF_MM_ROW(wy, x, lane, r)][SORF_MM_COL(wx, y, lane)] = acc[x][y][r];
  __syncthreads();
  // X21 = -X22 T, stored over T
  lds_mm64<false>(L, 64, 64, 64, 0, wy, wx, lane, acc);
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        L[64 + SORF_MM_ROW(wy, x, lane, r)][SORF_MM_COL(wx, y, lane)] = -acc[x][y][r];
  __syncthreads();
  double* out = Linv + int64_t(k / NB) * NB * NB;
  (void)LinvT;   // transposed by transpose_blocks_kernel after the factorisation
#pragma unroll 8
  for (int m = 0; m < 32; ++m) {
    const int i = wv + 4 * m;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = lane + 64 * h;
      out[i * NB + j] = (i < n && j <= i) ? L[i][j] : 0.0;
    }
  }
}

// LinvT[b] = Linv[b]^T for every diagonal block (the backward sweeps read
// rows of the transposed inverses). One workgroup per block, 32 x 32 tiles
// through LDS.
__global__ __launch_bounds__(256) void transpose_blocks_kernel(const double* __restrict__ Linv,
                                                              double* __restrict__ LinvT) {
  __shared__ double t[32][33];
  const double* src = Linv + int64_t(blockIdx.x) * NB * NB;
  double* dst = LinvT + int64_t(blockIdx.x) * NB * NB;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int bi = 0; bi < NB; bi += 32)
    for (int bj = 0; bj < NB; bj += 32) {
#pragma unroll
      for (int r = 0; r < 32; r += 8) t[ty + r][tx] = src[(bi + ty + r) * NB + bj + tx];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 32; r += 8) dst[(bj + ty + r) * NB + bi + tx] = t[tx][ty + r];
      __syncthreads();
    }
}

// Next block row of the panel, fused with the update of the next diagonal
// tile: workgroup b (0..3) computes the 32 rows
// L21 = A21 (L11^{-1})^T starting at k + NB + 32 b (8 waves of 16 x 32, 1 x 2 FP64 MFMA blocks; the inverse
// block sits in LDS; each lane loads its A operands for all of K at once,
// four consecutive k per row: the MFMA's k index t = lane / 16 stands for
// k = kb + 4 t + s in step s, and the B operands use the same order).
// (The panel rows below the next block row are formed by syrk_next.) Each
// workgroup publishes its rows (agent release, then flags[b] = epoch), waits for the lower-numbered ones (which
// are dispatched first, so the waits end), and then applies
//   A[r][c] -= sum_p L21[r][p] L21[c][p]
// to its 32 rows r of the next diagonal tile and the columns c <= r. The
// next diagonal block is therefore updated when the kernel ends, with the
// tile work spread over four compute units. A wait longer than
// kPanelWaitTicks (100 MHz counter) sets *info = -1 and stops waiting.
constexpr int PLD = NB + 4;   // LDS row stride of the panel kernel (doubles)
constexpr int kSyrkGrid = 248;   // 8 of the 256 compute units stay free for the chain
constexpr int PR = 32;        // rows per panel workgroup
constexpr uint64_t kPanelWaitTicks = uint64_t(1) << 28;   // about 2.7 s

__global__ __launch_bounds__(512) void panel_kernel(double* __restrict__ A, int32_t D, int32_t k,
                                                   const double* __restrict__ Linv,
                                                   int32_t* __restrict__ flags,
                                                   int32_t* __restrict__ info) {
  __shared__ double sL[NB][PLD];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wy = wv >> 2, wx = wv & 3;   // rows [16 wy, +16), columns [32 wx, +32)
  const int li = lane & 15, lt = lane >> 4;
  const int b = int(blockIdx.x);
  const int64_t r0 = int64_t(k) + NB + int64_t(b) * PR;
  const double* inv = Linv + int64_t(k / NB) * NB * NB;
  for (int t = tid; t < NB * NB / 2; t += 512) {
    const int j = t >> 6, p = (t & 63) * 2;
    const double2 v = *reinterpret_cast<const double2*>(inv + j * NB + p);
    sL[j][p] = v.x;
    sL[j][p + 1] = v.y;
  }
  double ar[8][4];
  {
    const int64_t row = r0 + 16 * wy + li;
    const bool ok = row < D;
    const double* src = A + (ok ? row : int64_t(D) - 1) * D + k + 4 * lt;
#pragma unroll
    for (int kb = 0; kb < 8; ++kb)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double v = src[16 * kb + s];   // rows of A need not be 16-byte aligned
        ar[kb][s] = ok ? v : 0.0;
      }
  }
  __syncthreads();
  f64x4 acc[2];
  acc[0] = acc[1] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kb = 0; kb < 8; ++kb) {
    double br[2][4];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int s = 0; s < 4; ++s) br[c][s] = sL[32 * wx + 16 * c + li][16 * kb + 4 * lt + s];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[c] = mfma64(ar[kb][s], br[c][s], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + 16 * wy + lt + 4 * r;
      if (row < D) A[row * D + k + 32 * wx + 16 * c + li] = acc[c][r];
    }
  // publish this strip of the next block row
  const int32_t epoch = k / NB + 1;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (tid == 0) __hip_atomic_store(flags + b, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  // wait for the strips above it
  if (tid == 0) {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (int q = 0; q < b; ++q) {
      while (__hip_atomic_load(flags + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
        if (__builtin_amdgcn_s_memrealtime() - t0 > kPanelWaitTicks) {
          int32_t expect = 0;
          __hip_atomic_compare_exchange_strong(info, &expect, -1, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  // rows 0 .. 32 (b + 1) - 1 of the next block row of L, into LDS
  const int nrow = PR * (b + 1);
  const int64_t rb = int64_t(k) + NB;
  for (int t = tid; t < nrow * (NB / 2); t += 512) {
    const int i = t >> 6, p = (t & 63) * 2;
    const int64_t row = rb + i;
    const bool ok = row < D;
    const double* src = A + (ok ? row : int64_t(D) - 1) * D + k + p;
    const double v0 = src[0], v1 = src[1];
    sL[i][p] = ok ? v0 : 0.0;
    sL[i][p + 1] = ok ? v1 : 0.0;
  }
  __syncthreads();
  // rows 32 b + 16 wy + [0, 16), columns 32 wx + [0, 32): only blocks that reach the lower part
  const int ib = PR * b + 16 * wy;
  if (32 * wx > ib + 15) return;
  f64x4 cc[2];
  cc[0] = cc[1] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
  for (int kb = 0; kb < 8; ++kb) {
    double pa[4], pb[2][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      pa[s] = sL[ib + li][16 * kb + 4 * lt + s];
#pragma unroll
      for (int c = 0; c < 2; ++c) pb[c][s] = sL[32 * wx + 16 * c + li][16 * kb + 4 * lt + s];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 2; ++c) cc[c] = mfma64(pa[s], pb[c][s], cc[c]);
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = ib + lt + 4 * r, j = 32 * wx + 16 * c + li;
      const int64_t gi = rb + i, gj = rb + j;
      if (gi < D && i >= j) A[gi * D + gj] -= cc[c][r];
    }
}

// Trailing update A22 -= L21 L21^T on the lower triangle: 128 x 128 tiles,
// 8 waves of 32 x 64 (2 x 4 MFMA blocks), K = NB in chunks of 32 via LDS with
// a register double buffer. Each wave loads its entries of the tile before
// the products, so the read of A22 overlaps them. On a diagonal tile the
// waves whose block lies above the diagonal only help with the loads.
// Tile (I, J) of the trailing matrix starts at block row/column k/NB + 1 + I/J.
constexpr int ST = 128, SKC = 32;
typedef double SyrkSlab[ST][SKC + 1];

static __device__ __forceinline__ void syrk_tile(double* __restrict__ A, int32_t D, int32_t k,
                                                 int64_t I, int64_t J, SyrkSlab& sI,
                                                 SyrkSlab& sJ) {
  constexpr int T = ST, KC = SKC;
  const bool diag = (I == J);
  const int64_t s0 = int64_t(k) + NB;
  const int64_t I0 = s0 + I * T, J0 = s0 + J * T;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv >> 1, wx = wv & 1;  // rows [32 wy, +32), columns [64 wx, +64)
  const bool idle = diag && (32 * wy + 31 < 64 * wx);
  const int lr = tid >> 2;          // row 0..127 of the slab
  const int lp = (tid & 3) * 8;     // 8 consecutive k
  const bool okI = I0 + lr < D, okJ = J0 + lr < D;
  const double* pI = A + min(I0 + lr, int64_t(D) - 1) * D + k + lp;
  const double* pJ = A + min(J0 + lr, int64_t(D) - 1) * D + k + lp;
  double rI[8], rJ[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double a = pI[q], b = pJ[q];
    rI[q] = okI ? a : 0.0;
    rJ[q] = okJ ? b : 0.0;
  }
  // this wave's entries of the tile (lower part inside the matrix)
  double c[2][4][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = I0 + wy * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int64_t gj = J0 + wx * 64 + b * 16 + (lane & 15);
        const bool ok = !idle && gi < D && gj < D && gi >= gj;
        c[a][b][r] = ok ? A[gi * D + gj] : 0.0;
      }
  f64x4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < NB; c0 += KC) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      sI[lr][lp + q] = rI[q];
      if (!diag) sJ[lr][lp + q] = rJ[q];
    }
    __syncthreads();
    if (c0 + KC < NB) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double a = pI[c0 + KC + q], b = pJ[c0 + KC + q];
        rI[q] = okI ? a : 0.0;
        rJ[q] = okJ ? b : 0.0;
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
        if (gi < D && gj < D && gi >= gj) A[gi * D + gj] = c[a][b][r] - acc[a][b][r];
      }
}

// Rows [RP h, RP h + RP) of tile (I, J), RP = 128 / NP: the same update as
// syrk_tile with the 8 waves on RP / 16 x 128 / (16 BB) blocks of 16 x 16 (BB
// MFMA blocks each), so that a tile takes NP workgroups. On a diagonal tile
// the rows are rows RP h .. of the J slab.
template <int NP>
static __device__ __forceinline__ void syrk_part_tile(double* __restrict__ A, int32_t D,
                                                      int32_t k, int64_t I, int64_t J, int h,
                                                      SyrkSlab& sI, SyrkSlab& sJ) {
  constexpr int KC = SKC;
  constexpr int RP = ST / NP;            // rows of the part
  constexpr int WYN = RP / 16;           // wave rows
  constexpr int WC = ST / (8 / WYN);     // columns per wave
  constexpr int BB = WC / 16;            // MFMA blocks per wave
  static_assert(WYN >= 1 && WYN <= 8 && BB >= 1, "part shape");
  const bool diag = (I == J);
  const int64_t s0 = int64_t(k) + NB;
  const int64_t J0 = s0 + J * ST, I0 = s0 + I * ST + RP * h;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wy = wv % WYN, wx = wv / WYN;   // rows [16 wy, +16) of the part, columns [WC wx, +WC)
  const bool idle = diag && (RP * h + 16 * wy + 15 < WC * wx);
  const int lr = tid >> 2;          // row 0..127 of the J slab (0..RP-1 of the I slab)
  const int lp = (tid & 3) * 8;     // 8 consecutive k
  const bool loadI = !diag && lr < RP;
  const bool okI = I0 + lr < D, okJ = J0 + lr < D;
  const double* pI = A + min(I0 + (lr % RP), int64_t(D) - 1) * D + k + lp;
  const double* pJ = A + min(J0 + lr, int64_t(D) - 1) * D + k + lp;
  double rI[8], rJ[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double a = pI[q], b = pJ[q];
    rI[q] = okI ? a : 0.0;
    rJ[q] = okJ ? b : 0.0;
  }
  double c[BB][4];
#pragma unroll
  for (int b = 0; b < BB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t gi = I0 + wy * 16 + (lane >> 4) + 4 * r;
      const int64_t gj = J0 + wx * WC + b * 16 + (lane & 15);
      const bool ok = !idle && gi < D && gj < D && gi >= gj;
      c[b][r] = ok ? A[gi * D + gj] : 0.0;
    }
  f64x4 acc[BB];
#pragma unroll
  for (int b = 0; b < BB; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // A operand: row 16 wy + (lane & 15) of the I slab, or row RP h + ... of the J slab
  const double (*sa)[KC + 1] = diag ? sJ : sI;
  const int ra = (diag ? RP * h : 0) + wy * 16 + (lane & 15);
  for (int c0 = 0; c0 < NB; c0 += KC) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (loadI) sI[lr][lp + q] = rI[q];
      sJ[lr][lp + q] = rJ[q];
    }
    __syncthreads();
    if (c0 + KC < NB) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double a = pI[c0 + KC + q], b = pJ[c0 + KC + q];
        rI[q] = okI ? a : 0.0;
        rJ[q] = okJ ? b : 0.0;
      }
    }
    if (!idle) {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        const int p = kk + (lane >> 4);
        const double av = sa[ra][p];
        double bv[BB];
#pragma unroll
        for (int b = 0; b < BB; ++b) bv[b] = sJ[wx * WC + b * 16 + (lane & 15)][p];
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[b] = mfma64(av, bv[b], acc[b]);
      }
    }
    __syncthreads();
  }
  if (idle) return;
#pragma unroll
  for (int b = 0; b < BB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t gi = I0 + wy * 16 + (lane >> 4) + 4 * r;
      const int64_t gj = J0 + wx * WC + b * 16 + (lane & 15);
      if (gi < D && gj < D && gi >= gj) A[gi * D + gj] = c[b][r] - acc[b][r];
    }
}

// The part of the trailing update that the next panel reads, fused with the
// panel rows it needs. Tiles of the trailing matrix's first block column
// below its diagonal, (I, 0) for I >= 1, each in kNextParts workgroups of
// RP = 32 rows: a workgroup first forms its 32 panel rows
// L_I = A_I (L_kk^{-1})^T (K = NB in chunks of 32 through LDS, the same
// products as the panel kernel), stores them in A and keeps them in LDS, then
// updates its rows of the tile with C -= L_I L_0^T, L_0 being the next block
// row that the chain's panel kernel wrote. The last kNextParts workgroups
// update the diagonal tile (1, 1) of the block after next (the tile (0, 0) is
// updated by the panel kernel) once the workgroups of tile (1, 0) have
// published L_1 (flags[4 + h] = epoch): those have lower indices and are
// dispatched first, so the wait ends; past kPanelWaitTicks it sets *info = -1.
// Splitting tiles into row parts keeps most compute units busy on these few
// tiles, and forming the panel rows here saves a launch and a pass over them.
constexpr int kNextParts = 4;
constexpr int kNextRows = ST / kNextParts;   // 32
__global__ __launch_bounds__(512) void syrk_next_kernel(double* __restrict__ A, int32_t D,
                                                       int32_t k, int32_t nt,
                                                       const double* __restrict__ Linv,
                                                       int32_t* __restrict__ flags,
                                                       int32_t* __restrict__ info) {
  __shared__ SyrkSlab sI, sJ;
  __shared__ double sP[kNextRows][NB + 1];
  constexpr int KC = SKC, RP = kNextRows, WC = 32, BB = 2;
  const int64_t t = blockIdx.x / kNextParts;
  const int h = int(blockIdx.x % kNextParts);
  const int32_t epoch = k / NB + 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (t + 1 >= nt) {   // diagonal tile (1, 1): wait for L_1
    if (tid == 0) {
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      for (int q = 0; q < kNextParts; ++q) {
        while (__hip_atomic_load(flags + 4 + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               epoch) {
          if (__builtin_amdgcn_s_memrealtime() - t0 > kPanelWaitTicks) {
            int32_t expect = 0;
            __hip_atomic_compare_exchange_strong(info, &expect, -1, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    syrk_part_tile<kNextParts>(A, D, k, 1, 1, h, sI, sJ);
    return;
  }
  const int64_t I = t + 1;
  const int64_t s0 = int64_t(k) + NB;
  const int64_t R0 = s0 + I * ST + RP * h;   // first row of this part
  const int wy = wv & 1, wx = wv >> 1;       // rows [16 wy, +16), columns [32 wx, +32)
  const int lr = tid >> 2;                   // row 0..127 of the J slab (0..31 of the I slab)
  const int lp = (tid & 3) * 8;              // 8 consecutive k
  // 1. panel rows: sI <- A rows R0 + lr (columns k ..), sJ <- rows of L_kk^{-1}
  {
    const bool okI = R0 + lr < D;
    const double* pI = A + min(R0 + (lr % RP), int64_t(D) - 1) * D + k + lp;
    const double* pJ = Linv + int64_t(k / NB) * NB * NB + lr * NB + lp;
    double rI[8], rJ[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double a = pI[q];
      rI[q] = okI ? a : 0.0;
      rJ[q] = pJ[q];
    }
    f64x4 acc[BB];
#pragma unroll
    for (int b = 0; b < BB; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int c0 = 0; c0 < NB; c0 += KC) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (lr < RP) sI[lr][lp + q] = rI[q];
        sJ[lr][lp + q] = rJ[q];
      }
      __syncthreads();
      if (c0 + KC < NB) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double a = pI[c0 + KC + q];
          rI[q] = okI ? a : 0.0;
          rJ[q] = pJ[c0 + KC + q];
        }
      }
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        const int p = kk + (lane >> 4);
        const double av = sI[wy * 16 + (lane & 15)][p];
        double bv[BB];
#pragma unroll
        for (int b = 0; b < BB; ++b) bv[b] = sJ[wx * WC + b * 16 + (lane & 15)][p];
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[b] = mfma64(av, bv[b], acc[b]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wy * 16 + (lane >> 4) + 4 * r, j = wx * WC + b * 16 + (lane & 15);
        sP[i][j] = acc[b][r];
        if (R0 + i < D) A[(R0 + i) * D + k + j] = acc[b][r];
      }
  }
  if (I == 1) {   // publish this part of L_1 for the diagonal tile's workgroups
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) __hip_atomic_store(flags + 4 + h, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (R0 >= D) return;
  // 2. C -= L_I L_0^T on rows R0 .., columns J0 .. of the tile (I, 0)
  const int64_t J0 = s0;
  const bool okJ = J0 + lr < D;
  const double* pJ = A + min(J0 + lr, int64_t(D) - 1) * D + k + lp;
  double rJ[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double b = pJ[q];
    rJ[q] = okJ ? b : 0.0;
  }
  double c[BB][4];
#pragma unroll
  for (int b = 0; b < BB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t gi = R0 + wy * 16 + (lane >> 4) + 4 * r;
      const int64_t gj = J0 + wx * WC + b * 16 + (lane & 15);
      c[b][r] = gi < D && gj < D ? A[gi * D + gj] : 0.0;
    }
  f64x4 acc[BB];
#pragma unroll
  for (int b = 0; b < BB; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < NB; c0 += KC) {
#pragma unroll
    for (int q = 0; q < 8; ++q) sJ[lr][lp + q] = rJ[q];
    __syncthreads();
    if (c0 + KC < NB) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double b = pJ[c0 + KC + q];
        rJ[q] = okJ ? b : 0.0;
      }
    }
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int p = kk + (lane >> 4);
      const double av = sP[wy * 16 + (lane & 15)][c0 + p];
      double bv[BB];
#pragma unroll
      for (int b = 0; b < BB; ++b) bv[b] = sJ[wx * WC + b * 16 + (lane & 15)][p];
#pragma unroll
      for (int b = 0; b < BB; ++b) acc[b] = mfma64(av, bv[b], acc[b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < BB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t gi = R0 + wy * 16 + (lane >> 4) + 4 * r;
      const int64_t gj = J0 + wx * WC + b * 16 + (lane & 15);
      if (gi < D && gj < D) A[gi * D + gj] = c[b][r] - acc[b][r];
    }
}

// The rest of the trailing update, tiles (I, J) with 1 <= J <= I other than
// (1, 1), in a persistent grid of at most kSyrkGrid workgroups: workgroup w
// takes the tiles w, w + G, ... of the sub-triangle's row-major order after
// (1, 1). The grid stays below the number of compute units so that the panel
// and diagonal kernels of the next steps find free units while it runs.
__global__ __launch_bounds__(512) void syrk_far_kernel(double* __restrict__ A, int32_t D,
                                                      int32_t k, int64_t n_sub) {
  __shared__ SyrkSlab sI, sJ;
  for (int64_t t = 1 + int64_t(blockIdx.x); t < n_sub; t += gridDim.x) {
    int64_t I, J;
    tri_tile(t, I, J);
    syrk_tile(A, D, k, I + 1, J + 1, sI, sJ);
    __syncthreads();   // the next tile reuses the LDS slabs
  }
}

// ---------------------------------------------------------------------------
// Triangular sweeps: one launch per sweep, one workgroup (512 threads) per
// block row, in dependency order: a workgroup only waits for blocks owned by
// workgroups with a lower index, which are dispatched before it, so the
// waits always end. Every solved value is its own ready signal: the output
// vectors hold a signalling-NaN pattern (kNotReady, which arithmetic never
// produces) until the value is stored, and consumers poll the values they
// need with agent-scope atomic loads, each wave on its own (no workgroup
// barrier and no separate flag round trip on the dependency chain). Loads of
// L that do not depend on the awaited block are issued before the wait. A
// wait that exceeds kSweepWaitTicks of the 100 MHz real-time counter sets
// *info = -1 (when it is still 0) and stops waiting in that wave, so every
// wave exits. The forward sweep marks its output of the backward sweep not
// ready; the backward sweep marks each block of its input not ready once it
// has read it, ready for the next forward sweep; the promote kernel marks
// the forward output not ready at the start of a solve.
constexpr uint64_t kSweepWaitTicks = uint64_t(1) << 28;   // about 2.7 s

// Re-polls until no lane of the wave holds a not-ready value (or the wait
// times out); v[] are the values at p[], reloaded where still not ready.
template <int N>
static __device__ __forceinline__ void wave_wait(const double* const (&p)[N], double (&v)[N],
                                                 int32_t* info, bool& failed) {
  bool pending = false;
#pragma unroll
  for (int t = 0; t < N; ++t) pending |= is_not_ready(v[t]);
  if (!__any(pending) || failed) return;
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  while (true) {
    __builtin_amdgcn_s_sleep(1);
    pending = false;
#pragma unroll
    for (int t = 0; t < N; ++t) {
      if (is_not_ready(v[t])) v[t] = poll_load(p[t]);
      pending |= is_not_ready(v[t]);
    }
    if (!__any(pending)) return;
    if (__builtin_amdgcn_s_memrealtime() - t0 > kSweepWaitTicks) {
      if ((threadIdx.x & 63) == 0) {
        int32_t expect = 0;
        __hip_atomic_compare_exchange_strong(info, &expect, -1, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      failed = true;
      return;
    }
  }
}

// Sums 16 per-lane partials over the 64 lanes of a wave: afterwards every
// lane with (lane >> 2) & 15 == r holds the full sum of partial r.
static __device__ __forceinline__ double wave_sum16(double (&p)[16], int lane) {
#pragma unroll
  for (int lvl = 0; lvl < 4; ++lvl) {
    const int mask = 32 >> lvl, half = 8 >> lvl;
    const bool upper = (lane & mask) != 0;
#pragma unroll
    for (int r = 0; r < half; ++r) {
      const double keep = upper ? p[r + half] : p[r];
      const double send = upper ? p[r] : p[r + half];
      p[r] = keep + __shfl_xor(send, mask);
    }
  }
  const double t = p[0] + __shfl_xor(p[0], 2);
  return t + __shfl_xor(t, 1);
}

// out[i] = sum_c M[c][i] v[c] for a 128 x 128 block stored row-major (c rows);
// thread (i, q) holds M[32 q + m][i], m < 32, and the four quarters are added
// in a fixed order. v and red are LDS; red holds 4 x 128 doubles. The results
// are stored as ready signals.
static __device__ __forceinline__ void block_mvT_load(const double* __restrict__ M, double (&a)[32],
                                                      int tid) {
  const int i = tid & 127, q = tid >> 7;
#pragma unroll
  for (int m = 0; m < 32; ++m) a[m] = M[(32 * q + m) * NB + i];
}
static __device__ __forceinline__ void block_mvT_finish(const double (&a)[32], const double* v,
                                                        int n, double* out, double (*red)[NB],
                                                        int tid) {
  const int i = tid & 127, q = tid >> 7;
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int m = 0; m < 32; m += 2) {
    s0 = __builtin_fma(a[m], v[32 * q + m], s0);
    s1 = __builtin_fma(a[m + 1], v[32 * q + m + 1], s1);
  }
  red[q][i] = s0 + s1;
  __syncthreads();
  if (q == 0 && i < n) signal_store(out + i, (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]));
}

// Forward sweep L y = b, left-looking by block rows:
//   y_k = L_kk^{-1} (b_k - sum_{j<k} L_kj y_j).
// Workgroup k: wave w owns rows 16 w .. 16 w + 15 of the block; lane l holds
// columns l and l + 64 of each block L_kj (coalesced 512-byte row reads) and
// keeps per-lane partial sums over all j, reduced across lanes once. y must
// be not ready on entry; x (the backward sweep's output) is marked not ready.
__global__ __launch_bounds__(512) void sweep_fwd_kernel(const double* __restrict__ A,
                                                       const double* __restrict__ LinvT, int32_t D,
                                                       const double* __restrict__ b, double* y,
                                                       double* x, int32_t* __restrict__ info) {
  __shared__ double rv[NB];
  __shared__ double red[4][NB];
  bool failed = false;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int k = blockIdx.x;
  const int64_t r0 = int64_t(k) * NB;
  const int n = (D - r0) < NB ? int(D - r0) : NB;
  if (tid < n) signal_store(x + r0 + tid, not_ready());
  double inv[32];
  block_mvT_load(LinvT + int64_t(k) * NB * NB, inv, tid);
  double acc[16][2];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r][0] = acc[r][1] = 0.0;
  for (int j = 0; j < k; ++j) {
    double lb[16][2];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = r0 + 16 * wv + r;
      const double* p = A + (row < D ? row : D - 1) * D + int64_t(j) * NB;
      lb[r][0] = p[lane];
      lb[r][1] = p[lane + 64];
    }
    const double* const yp[2] = {y + int64_t(j) * NB + lane, y + int64_t(j) * NB + 64 + lane};
    double yv[2] = {poll_load(yp[0]), poll_load(yp[1])};
    wave_wait<2>(yp, yv, info, failed);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      acc[r][0] = __builtin_fma(lb[r][0], yv[0], acc[r][0]);
      acc[r][1] = __builtin_fma(lb[r][1], yv[1], acc[r][1]);
    }
  }
  double ps[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) ps[r] = acc[r][0] + acc[r][1];
  const double s = wave_sum16(ps, lane);
  if ((lane & 3) == 0) {
    const int i = 16 * wv + ((lane >> 2) & 15);
    rv[i] = i < n ? b[r0 + i] - s : 0.0;
  }
  __syncthreads();
  block_mvT_finish(inv, rv, n, y + r0, red, tid);
}

// Backward sweep L^T x = y, by block rows of L^T from the last:
//   x_k = L_kk^{-T} (y_k - sum_{j>k} L_jk^T x_j).
// Workgroup g owns block k = nblk - 1 - g. Thread (c, q) holds column c of
// the block and rows 32 q .. 32 q + 31 of each block L_jk (coalesced over c),
// so the products need no cross-lane sums; the quarters are added once.
// Lane m < 32 of a wave polls x_j[32 q + m]; the values reach the other
// lanes by shuffles. x must be not ready on entry; y_k is marked not ready
// after it is read.
__global__ __launch_bounds__(512) void sweep_bwd_kernel(const double* __restrict__ A,
                                                       const double* __restrict__ Linv, int32_t D,
                                                       double* y, double* x,
                                                       int32_t* __restrict__ info) {
  __shared__ double rv[NB];
  __shared__ double red[4][NB];
  bool failed = false;
  const int tid = threadIdx.x, lane = tid & 63;
  const int c = tid & 127, q = tid >> 7;
  const int nblk = (D + NB - 1) / NB;
  const int k = nblk - 1 - int(blockIdx.x);
  const int64_t c0 = int64_t(k) * NB;
  const int n = (D - c0) < NB ? int(D - c0) : NB;
  double inv[32];
  block_mvT_load(Linv + int64_t(k) * NB * NB, inv, tid);
  const int64_t col = c0 + (c < n ? c : n - 1);
  double acc = 0.0;
  for (int j = nblk - 1; j > k; --j) {
    const int64_t rj = int64_t(j) * NB + 32 * q;
    double lb[32];
#pragma unroll
    for (int m = 0; m < 32; ++m) {
      const int64_t row = rj + m;
      lb[m] = row < D ? A[row * D + col] : 0.0;
    }
    const int64_t mine = rj + (lane & 31);
    const double* const xp[1] = {x + (mine < D ? mine : D - 1)};
    double xv[1] = {poll_load(xp[0])};
    wave_wait<1>(xp, xv, info, failed);
#pragma unroll
    for (int m = 0; m < 32; ++m) acc = __builtin_fma(lb[m], __shfl(xv[0], m), acc);
  }
  red[q][c] = acc;
  __syncthreads();
  if (q == 0 && c < n) {
    rv[c] = y[c0 + c] - ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c]));
    signal_store(y + c0 + c, not_ready());   // for the next forward sweep
  } else if (q == 0) {
    rv[c] = 0.0;
  }
  __syncthreads();
  block_mvT_finish(inv, rv, n, x + c0, red, tid);
}

// Partial sums of (lower-stored symmetric G) x over 64 x 64 tiles:
// part[X][Y][.] = contribution to rows of block X from the tile pairing X and Y.
// Thread t holds 4 x 4 entries of the tile (rows t / 16 + 16 m, columns
// 4 (t % 16) + c); row sums reduce over the 16 lanes of a row group, column
// sums over the 4 row groups of a wave and then the 4 waves, all in a fixed
// order.
template <typename TG>
__global__ __launch_bounds__(256) void symv_tiles_kernel(const TG* __restrict__ G, int32_t D,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ part) {
  __shared__ double csum[4][64];
  __shared__ double rsum[64];
  int64_t I, J;
  tri_tile(blockIdx.x, I, J);
  const int64_t nt = (int64_t(D) + 63) / 64;
  const int64_t I0 = I * 64, J0 = J * 64;
  const bool diag = I == J;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c0 = 4 * (tid & 15), r0 = tid >> 4;   // rows r0 + 16 m
  double g[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int64_t gi = I0 + r0 + 16 * m;
    const int64_t gic = gi < D ? gi : int64_t(D) - 1;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t gj = J0 + c0 + c;
      const TG v = G[gic * D + (gj < D ? gj : int64_t(D) - 1)];
      g[m][c] = (gi < D && gj < D && gj <= gi) ? double(v) : 0.0;
    }
  }
  double xj[4], xi[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) xj[c] = J0 + c0 + c < D ? x[J0 + c0 + c] : 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m) xi[m] = I0 + r0 + 16 * m < D ? x[I0 + r0 + 16 * m] : 0.0;
  // rows: G x over this tile's columns; columns: G^T x over its rows (strictly
  // below the diagonal on a diagonal tile, where the row sums already hold it)
  double rs[4], cs[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) rs[m] = ((g[m][0] * xj[0] + g[m][1] * xj[1]) + g[m][2] * xj[2]) + g[m][3] * xj[3];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cs[c] = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const bool strict = !diag || (r0 + 16 * m > c0 + c);
      cs[c] += strict ? g[m][c] * xi[m] : 0.0;
    }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) rs[m] += __shfl_xor(rs[m], o);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cs[c] += __shfl_xor(cs[c], 16);
    cs[c] += __shfl_xor(cs[c], 32);
  }
  if ((tid & 15) == 0) {
#pragma unroll
    for (int m = 0; m < 4; ++m) rsum[r0 + 16 * m] = rs[m];
  }
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 4; ++c) csum[wv][c0 + c] = cs[c];
  }
  __syncthreads();
  if (tid < 64) {
    const double col = (csum[0][tid] + csum[1][tid]) + (csum[2][tid] + csum[3][tid]);
    if (diag) {
      part[(I * nt + I) * 64 + tid] = rsum[tid] + col;
    } else {
      part[(I * nt + J) * 64 + tid] = rsum[tid];
      part[(J * nt + I) * 64 + tid] = col;
    }
  }
}

// r = Zty - lambda x - sum_Y part[X][Y]: one workgroup per 64-row block X;
// thread (i, q) sums Y in [q nt / 4, (q + 1) nt / 4) in order and the four
// quarters are added in a fixed order.
template <typename TG>
__global__ __launch_bounds__(256) void residual_kernel(const double* __restrict__ part, int32_t D,
                                                      double lambda, const TG* __restrict__ rhs,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ r) {
  __shared__ double qs[4][64];
  const int64_t nt = (int64_t(D) + 63) / 64;
  const int64_t X = blockIdx.x;
  const int i = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t y0 = nt * q / 4, y1 = nt * (q + 1) / 4;
  double s = 0.0;
  for (int64_t Y = y0; Y < y1; ++Y) s += part[(X * nt + Y) * 64 + i];
  qs[q][i] = s;
  __syncthreads();
  const int64_t gi = X * 64 + i;
  if (q == 0 && gi < D)
    r[gi] = (double(rhs[gi]) - lambda * x[gi]) - ((qs[0][i] + qs[1][i]) + (qs[2][i] + qs[3][i]));
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

static hipError_t solve_triangular(const SolveWs& w, int32_t D, const double* rhs, double* tmp,
                                   double* out, int32_t* info, hipStream_t st) {
  // L tmp = rhs, then L^T out = tmp: one launch per sweep, one workgroup per block
  const unsigned nblk = unsigned((D + NB - 1) / NB);
  hipLaunchKernelGGL(sweep_fwd_kernel, dim3(nblk), dim3(512), 0, st, w.A, w.LinvT, D, rhs, tmp,
                     out, info);
  hipLaunchKernelGGL(sweep_bwd_kernel, dim3(nblk), dim3(512), 0, st, w.A, w.Linv, D, tmp, out,
                     info);
  return hipGetLastError();
}

template <typename TG>
static hipError_t launch_solve(int32_t D, const TG* G, const TG* Zty, double lambda,
                               int32_t n_refine, double* alpha, int32_t* info, void* ws,
                               hipStream_t st, hipStream_t side, hipEvent_t ev_panel,
                               hipEvent_t ev_next) {
  const SolveWs w = carve(ws, D);
  const unsigned vg = unsigned((D + 255) / 256);
  hipLaunchKernelGGL(promote_kernel<TG>, dim3(vg, unsigned(D)), dim3(256), 0, st, G, D, lambda,
                     w.A, info, w.y, w.pflags);
  // Right-looking blocked Cholesky with lookahead over two streams. Caller's
  // stream (the chain of dependent steps): the panel rows of the next block
  // row, fused with the update of the next diagonal tile (4 workgroups), then
  // the factorisation of that block. Second stream: the other panel rows, the
  // trailing tiles the next panel reads (first block column and the next
  // diagonal tile but one), then the rest of the trailing update in a
  // persistent grid that leaves compute units free, so the chain's kernels of
  // the following steps run beside it. The chain waits for the next-panel
  // tiles through an event. Every tile is updated by the steps in order: the
  // second stream runs the far update of step k before the next-panel tiles
  // of step k + 1. Only stream events order kernels of different streams, so
  // the schedule stays correct when a tool serialises the launches.
  // The second stream and both events belong to the caller. Without them
  // (side == nullptr) every launch goes to the caller's stream in the same
  // order, which serialises the chain behind each trailing update but runs
  // the same kernels on the same data: the result is bitwise the same.
  const bool two = side != nullptr;
  if (!two) side = st;
  hipError_t e = hipSuccess;
  hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, w.A, D, 0, info, w.Linv,
                     w.LinvT);
  for (int32_t k = 0; k + NB < D; k += NB) {
    const int64_t rest = int64_t(D) - k - NB;
    const int64_t nt = (rest + 127) / 128;
    const int64_t nwg = (rest + PR - 1) / PR;
    const int64_t strips = nwg < NB / PR ? nwg : NB / PR;
    hipLaunchKernelGGL(panel_kernel, dim3(unsigned(strips)), dim3(512), 0, st, w.A, D, k, w.Linv,
                       w.pflags, info);
    // rows below the next block row (nt > 1): their panel rows are formed by
    // syrk_next together with the tiles that read them
    const bool side_work = nt > 1;
    if (side_work) {
      if (two) {
        if ((e = hipEventRecord(ev_panel, st)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(side, ev_panel, 0)) != hipSuccess) return e;
      }
      hipLaunchKernelGGL(syrk_next_kernel, dim3(unsigned(kNextParts * nt)), dim3(512), 0, side,
                         w.A, D, k, int32_t(nt), w.Linv, w.pflags, info);
      if (two && (e = hipEventRecord(ev_next, side)) != hipSuccess) return e;
      const int64_t n_sub = (nt - 1) * nt / 2;   // sub-triangle from (1, 1)
      if (n_sub > 1) {
        const int64_t g = n_sub - 1 < kSyrkGrid ? n_sub - 1 : kSyrkGrid;
        hipLaunchKernelGGL(syrk_far_kernel, dim3(unsigned(g)), dim3(512), 0, side, w.A, D, k,
                           n_sub);
      }
    }
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, w.A, D, k + NB, info,
                       w.Linv, w.LinvT);
    if (two && side_work && (e = hipStreamWaitEvent(st, ev_next, 0)) != hipSuccess) return e;
  }
  // the last far update (if any) before the sweeps read L
  if (two) {
    if ((e = hipEventRecord(ev_next, side)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(st, ev_next, 0)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(transpose_blocks_kernel, dim3(unsigned((D + NB - 1) / NB)), dim3(256), 0, st,
                     w.Linv, w.LinvT);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(to_double_kernel<TG>, dim3(vg), dim3(256), 0, st, Zty, w.b, D);
  e = solve_triangular(w, D, w.b, w.y, alpha, info, st);
  if (e != hipSuccess) return e;
  const int64_t nt = (int64_t(D) + 63) / 64;
  for (int32_t it = 0; it < n_refine; ++it) {
    hipLaunchKernelGGL(symv_tiles_kernel<TG>, dim3(unsigned(nt * (nt + 1) / 2)), dim3(256), 0, st,
                       G, D, alpha, w.part);
    hipLaunchKernelGGL(residual_kernel<TG>, dim3(unsigned(nt)), dim3(256), 0, st, w.part, D,
                       lambda, Zty, alpha, w.b);
    e = solve_triangular(w, D, w.b, w.y, w.dx, info, st);
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
         3 * align256(sizeof(double) * D) + align256(sizeof(double) * nt * nt * 64) + 256;
}

hipError_t sorf_launch_solve(int32_t D, const float* G, const float* Zty, double lambda,
                             int32_t n_refine, double* alpha, int32_t* info, void* ws,
                             hipStream_t st, hipStream_t side, hipEvent_t ev_fork,
                             hipEvent_t ev_join) {
  return launch_solve<float>(D, G, Zty, lambda, n_refine, alpha, info, ws, st, side, ev_fork,
                             ev_join);
}

hipError_t sorf_launch_solve_f64(int32_t D, const double* G, const double* Zty, double lambda,
                                 int32_t n_refine, double* alpha, int32_t* info, void* ws,
                                 hipStream_t st, hipStream_t side, hipEvent_t ev_fork,
                                 hipEvent_t ev_join) {
  return launch_solve<double>(D, G, Zty, lambda, n_refine, alpha, info, ws, st, side, ev_fork,
                              ev_join);
}
