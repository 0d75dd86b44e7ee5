/*
 * sorf.h -- C ABI of the MI355X (gfx950) SORF hot-path library.
 *
 * Structured orthogonal random features (arXiv 2206.01580, Theory section):
 *
 *   z(x_i)  = sqrt(2/D) * cos(c * H D_{T-1} ... H D_1 H D_0 x_i + b_e)     (RFF feature map;
 *             SORF approximation W ~ (sqrt(d)/sigma) [H_i D_i]_{N_transform}, stacked N_F/d times)
 *   Z_m     = sum_{i in molecule m} z(x_i)                                  (atomic energy decomposition)
 *   (Z^T Z + lambda I) alpha = Z^T y                                         (regularised normal equation)
 *   E_m     = Z_m alpha                                                       (prediction)
 *   F       = -dE/dr = -sum_i J_i^T dE/dx_i                                  (forces via derivative features)
 *
 * with H the +-1 Walsh-Hadamard matrix of order d (Sylvester recursion, natural
 * order: H[i][j] = (-1)^popcount(i & j)), D_t diagonal Rademacher sign matrices
 * that depend on the element e of the atom, the transform t and the stack s,
 * c = (sqrt(d)/sigma) * d^(-T/2), D = n_stacks * d features ordered f = s*d + j,
 * and b_e the per-element phase vector.
 *
 * Conventions shared by every call:
 *   - Pointers named in the structs and arguments are DEVICE pointers unless a
 *     comment says "host". All buffers are owned by the caller; the library
 *     keeps no state and never frees anything. The only HIP objects it creates
 *     are those sorf_solve_streams_create hands to the caller, who owns them.
 *     The one exception is sorf_predict_noalloc, whose workspace is a fixed
 *     device array of the library (see there).
 *   - Every compute call is asynchronous on `stream` (a hipStream_t; NULL means
 *     the default stream), returns a status immediately, never prints and never
 *     allocates device memory. Host-side validation of sizes, flags and null
 *     pointers happens before any HIP call and returns SORF_ERR_INVALID_ARG or
 *     SORF_ERR_UNSUPPORTED; a failed launch returns SORF_ERR_DEVICE.
 *   - Preconditions that live in device memory are NOT checked (CSR offsets
 *     non-decreasing with mol_ptr[0] = 0 and mol_ptr[n_mols] = n_atoms, element
 *     ids in [0, n_elements)); sorf_validate_batch checks them on request.
 *   - Float arrays (x, bias, alpha, Z, grad_x) must be 16-byte aligned, sign words
 *     4-byte aligned (any allocation from hipMalloc is); misaligned pointers are
 *     rejected with SORF_ERR_INVALID_ARG.
 *   - Results are deterministic: no floating-point atomics, fixed summation order.
 *   - Distinct streams may run calls concurrently; calls that write the same
 *     output buffer must be ordered by the caller.
 */
#ifndef SORF_H
#define SORF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SORF_ABI_VERSION 8

typedef void* sorf_stream_t; /* a hipStream_t */

typedef enum {
  SORF_OK = 0,
  SORF_ERR_INVALID_ARG = 1,  /* null pointer with non-zero size, bad size or flag */
  SORF_ERR_UNSUPPORTED = 2,  /* valid request outside what the kernels implement */
  SORF_ERR_DEVICE = 3,       /* a HIP launch or runtime call failed */
  SORF_ERR_WORKSPACE = 4,    /* workspace missing or smaller than the query returns */
  SORF_ERR_BUSY = 5          /* sorf_server_submit: every ring slot holds an unfinished batch */
} sorf_status;

typedef enum {
  SORF_GRAM_FP32 = 0,        /* FP32 operands, FP32 MFMA, FP32 accumulation */
  SORF_GRAM_BF16 = 1,        /* one bf16 product hi^T hi, FP32 accumulation */
  SORF_GRAM_FP16 = 2,        /* one fp16 product hi^T hi, FP32 accumulation */
  SORF_GRAM_BF16_HILO = 3,   /* (hi + lo)^T (hi + lo), four bf16 products, hi = bf16(z),
                                lo = bf16(z - hi); the Gram of hi + lo, so it stays PSD */
  SORF_GRAM_FP16_HILO = 4,   /* the same with fp16 parts of 2^scale_exp * z */
  SORF_GRAM_FP32_KAHAN = 5   /* FP32 as mode 0, with each 256-row block sum added into the
                                running FP32 sum by Kahan's compensated summation (the
                                paper's FP32 training mode, Timings subsection) */
} sorf_gram_precision;

/* Model parameters (host struct; the arrays it points to are device-resident).
 * SORF subsection: per-element sign diagonals and the stacking of N_F/d blocks;
 * RFF subsection: phases b in [0, 2 pi). */
typedef struct {
  int32_t d;             /* representation size, a power of two in [2, 1024]            */
  int32_t n_stacks;      /* S >= 1; D = S * d features (D <= 2^20)                      */
  int32_t n_transforms;  /* T in {1, 2, 3}: number of (sign, Hadamard) rounds           */
  int32_t n_elements;    /* E >= 1                                                      */
  float sigma;           /* kernel length scale, finite and > 0                         */
  const uint32_t* signs; /* [E][T][S][W] with W = ceil(d / 32) words per vector; bit j of
                            word j/32 set means entry j of D_t is -1. t = 0 is applied first. */
  const float* bias;     /* [E][D] phases in radians                                     */
} sorf_model;

/* A batch of molecules in CSR form (host struct, device arrays). */
typedef struct {
  const float* x;          /* [n_atoms][d] row-major projected representations          */
  const int32_t* element;  /* [n_atoms] element ids                                      */
  const int64_t* mol_ptr;  /* [n_mols + 1] atom offsets of each molecule                 */
  int64_t n_atoms;         /* >= 0; may be 0 (outputs are then zeroed)                   */
  int64_t n_mols;          /* >= 0; molecules with zero atoms give zero rows / energies  */
} sorf_batch;

/* FCHL19 representation parameters (Representation subsection and the parameter table
 * of Computational Details; the energy+force column is n2 = 24, n3 = 20, eta2 = 0.32,
 * eta3 = 2.7, N2 = 1.8, N3 = 0.57, c3 = 13.4, zeta = pi, rcut = 6.0 Angstrom). Host struct. */
typedef struct {
  int32_t n2;    /* two-body radial bins, centres rcut (k + 1) / n2                       */
  int32_t n3;    /* three-body radial bins (>= 2), centres rcut k / (n3 - 1)                */
  float eta2;    /* log-normal width parameter of the two-body term                         */
  float eta3;    /* width of the three-body radial Gaussians                                */
  float N2;      /* two-body distance exponent                                              */
  float N3;      /* three-body (Axilrod-Teller-Muto) distance exponent                      */
  float c3;      /* three-body weight                                                       */
  float zeta;    /* angular Gaussian width                                                  */
  float rcut;    /* cutoff radius                                                           */
} sorf_fchl19_params;

/* ABI version of the loaded library (compare with SORF_ABI_VERSION). */
int32_t sorf_abi_version(void);

/* Human-readable name of a status code (static storage, never NULL). */
const char* sorf_status_string(sorf_status s);

/* Feature matrix. RFF feature map summed over each molecule's atoms (atomic
 * energy decomposition); SORF operator applied with the fast Walsh-Hadamard
 * transform in O(T * D * log d) per atom (SORF subsection).
 *   Z: [n_mols][D] row-major FP32, overwritten (rows of empty molecules = 0). */
sorf_status sorf_forward(const sorf_model* model, const sorf_batch* batch, float* Z,
                         sorf_stream_t stream);

/* Adjoint of the energy E_m = Z_m alpha with respect to the inputs x (the
 * derivative features of the force-trained normal equation, contracted with
 * alpha): for atom i of molecule m,
 *   grad_x[i] = dE[m] * sum_s c * D_0 H D_1 ... D_{T-1} H g_{i,s},
 *   g_{i,f} = -sqrt(2/D) * alpha_f * sin(c * v_{i,f} + b_{e,f}).
 *   alpha:  [D] FP32;  dE: [n_mols] upstream weights or NULL for all ones;
 *   grad_x: [n_atoms][d] FP32, overwritten. */
sorf_status sorf_backward(const sorf_model* model, const sorf_batch* batch, const float* alpha,
                          const float* dE, float* grad_x, sorf_stream_t stream);

/* Bytes of workspace sorf_energy_grad needs for n_atoms atoms (host-only query,
 * nondecreasing). Returns 0 for negative sizes. */
size_t sorf_energy_grad_workspace_bytes(int64_t n_atoms);

/* Energies and their gradient with respect to the inputs in one pass over the features
 * (RFF subsection: E_m = Z_m alpha through the atomic energy decomposition, and its
 * derivative, the adjoint above with dE = 1): each atom's features are formed once and
 * give both its energy share alpha^T z(x_i) and its gradient row.
 *   alpha: [D] FP32.  E: [n_mols] FP32 out, each molecule's atom shares summed in atom
 *   order (as sorf_predict with J: equal to sorf_predict's energies without J to FP32
 *   rounding, not bitwise).  grad_x: [n_atoms][d] FP32 out, the same values as
 *   sorf_backward with dE = NULL.
 *   workspace: device memory of at least sorf_energy_grad_workspace_bytes(n_atoms),
 *   256-byte aligned (the atoms' energy shares). */
sorf_status sorf_energy_grad(const sorf_model* model, const sorf_batch* batch, const float* alpha,
                             float* E, float* grad_x, void* workspace, size_t workspace_bytes,
                             sorf_stream_t stream);

/* Derivative feature matrix of the force-trained normal equation (RFF subsection:
 * ((Z, dZ)^T (Z, dZ) + lambda I) alpha = (Z, dZ)^T (E, F), dZ with one row per atomic
 * coordinate). Row 3 a + k (atom a of molecule m, coordinate k in [0, 3)) is minus the
 * derivative of the molecule's feature row with respect to that coordinate:
 *   dZ[3 a + k][f] = sqrt(2/D) sum_{i in m} sin(u_{i,f}) (W_{e_i} J_i)[f][3 (a - a0) + k],
 *   u_i = W_{e_i} x_i + b_{e_i},  a0 = mol_ptr[m],
 * so that dZ alpha = F = -dE/dr. Accumulating (Z, E) and then (dZ, F) with
 * sorf_gram_accumulate into the same G and Zty forms the force-trained system.
 *   J, J_ptr: the per-molecule Jacobian blocks exactly as sorf_predict takes them
 *     (block m is [N_m][d][3 N_m] row-major at float offset J_ptr[m]; no alignment).
 *     One atom's part of a block, d * 3 N_m floats, must stay below 2^32 bytes
 *     (N_m < 2^30 / (3 d) atoms in one molecule; not checked, as N_m lives in device memory).
 *   dZ: [3 n_atoms][D] row-major FP32, 16-byte aligned, overwritten (molecules with no
 *     atoms own no rows). Each row is summed over its molecule's atoms in atom order,
 *     so a molecule's rows are bitwise the same in any batch.
 *   Required non-NULL when n_atoms > 0. Needs no workspace. */
sorf_status sorf_derivative_features(const sorf_model* model, const sorf_batch* batch,
                                     const float* J, const int64_t* J_ptr, float* dZ,
                                     sorf_stream_t stream);

/* Bytes of workspace sorf_projection_fit needs for representations of d_rep entries
 * (host-only query): about 4 d_rep^2 doubles. 0 unless 1 <= d_rep <= 4096. */
size_t sorf_projection_fit_workspace_bytes(int32_t d_rep);

/* Fit of one element's projection matrix (SORF subsection: the SVD Z~_e = U_e S_e V_e^T of
 * the matrix whose columns are sampled representations of element e; U_e^{N_PCA} is its
 * first N_PCA columns). Computed as the eigenvectors of Z~_e Z~_e^T = sum_rows rho^T rho,
 * formed in FP64, by the cyclic Jacobi method in FP64 (at most 15 sweeps).
 *   sample: [n_samples][d_rep] FP32 rows (any alignment).
 *   U: [d_rep][n_pca] row-major FP32 out; column r is the left singular vector of the
 *     r-th largest singular value (equal values: lower eigenvector index first), its sign
 *     chosen so that its entry of largest magnitude (ties: lowest row) is positive. Writing
 *     element e's result at U_all + e * d_rep * d with n_pca = d builds the [E][d_rep][d]
 *     array sorf_project takes.
 *   singular_values: [n_pca] FP64 out (sqrt of the eigenvalues, negatives clamped to 0), or NULL.
 *   1 <= n_pca <= d_rep <= 4096 (larger d_rep: SORF_ERR_UNSUPPORTED). The columns are
 *   determined only for distinct, nonzero singular values: the sample needs rank >= n_pca
 *   (columns past its rank are arbitrary unit vectors of the null space).
 *   workspace: at least sorf_projection_fit_workspace_bytes(d_rep), 256-byte aligned.
 *   About 15 (d_rep + 1) kernel launches; deterministic. */
sorf_status sorf_projection_fit(int64_t n_samples, int32_t d_rep, const float* sample,
                                int32_t n_pca, float* U, double* singular_values,
                                void* workspace, size_t workspace_bytes, sorf_stream_t stream);

/* Bytes of workspace sorf_project needs (host-only query; nondecreasing in n_atoms).
 * 0 for invalid sizes (n_atoms < 0, n_elements outside [1, 256]). */
size_t sorf_project_workspace_bytes(int64_t n_atoms, int32_t n_elements);

/* Per-element projection of the atomic representation to the transform size (SORF
 * subsection: rho_proj = rho^T U_e^{N_PCA}, U_e^{N_PCA} the first N_PCA left singular
 * vectors of element e's sampled representations, one matrix per element):
 *   x[i][j] = sum_k rho[i][k] U[e_i][k][j]   (FP32 matrix-core products and sums).
 *   rho: [n_atoms][d_rep] row-major FP32 (any alignment; 16-byte aligned rows with d_rep and
 *   d multiples of 4 take the vector path); element: [n_atoms] int32 in [0, n_elements)
 *   (atoms with other ids are skipped and their x rows left as they were);
 *   U: [n_elements][d_rep][d] row-major FP32; x: [n_atoms][d] FP32 out.
 *   1 <= n_elements <= 256 (else SORF_ERR_UNSUPPORTED), d_rep >= 1, 1 <= d <= 2^20.
 *   workspace: at least sorf_project_workspace_bytes(n_atoms, n_elements), 256-byte aligned.
 *   x is deterministic: every row depends on its own rho row only. */
sorf_status sorf_project(int64_t n_atoms, int32_t d_rep, const float* rho, const int32_t* element,
                         int32_t n_elements, const float* U, int32_t d, float* x,
                         void* workspace, size_t workspace_bytes, sorf_stream_t stream);

/* Length of the FCHL19 representation for n_elements elements:
 * n_elements n2 + n_elements (n_elements + 1) / 2 n3 2 (720 for five elements with the
 * energy+force parameters). Host-only; 0 for invalid arguments. */
int64_t sorf_fchl19_length(int32_t n_elements, const sorf_fchl19_params* params);

/* FCHL19 representation of every atom (Representation subsection):
 *   rho_i = [G2_X for each element X] ++ [G3_XY for each element pair X <= Y, lexicographic],
 *   G2_X[k] = sum_{j of element X} f_cut(r_ij) r_ij^-N2 LN(R_k; mu(r_ij), sigma(r_ij)),
 *     LN the log-normal density with mu = ln(r / sqrt(1 + eta2/r^2)), sigma^2 = ln(1 + eta2/r^2);
 *   G3_XY[k][t] = sum over unordered neighbour pairs {j, l} of elements {X, Y} of
 *     xi3 f_cut(r_ij) f_cut(r_jl) f_cut(r_il) sqrt(eta3/pi) exp(-eta3 ((r_ij + r_il)/2 - R_k)^2) A_t,
 *     xi3 = c3 (1 + 3 cos_i cos_j cos_l) / (r_ij r_jl r_il)^N3, A_cos = 2 e^(-zeta^2/2) cos(theta_i),
 *     A_sin = 2 e^(-zeta^2/2) sin(theta_i), theta_i the angle at i; f_cut(r) = (cos(pi r/rcut)+1)/2
 *     for r < rcut, else 0. Neighbours: other atoms of the same molecule closer than rcut.
 *   R: [n_atoms][3] FP32 coordinates (Angstrom); element: [n_atoms] int32 in [0, n_elements);
 *   mol_ptr: [n_mols + 1] CSR atom offsets; rho: [n_atoms][length] FP32 out.
 *   1 <= n_elements <= 16; at most 512 neighbours per atom (an atom with more gets a row of
 *   NaN). Each entry is summed in a fixed order (deterministic). No workspace. */
sorf_status sorf_fchl19_forward(const float* R, const int32_t* element, const int64_t* mol_ptr,
                                int64_t n_atoms, int64_t n_mols, int32_t n_elements,
                                const sorf_fchl19_params* params, float* rho,
                                sorf_stream_t stream);

/* Coordinate gradient of the FCHL19 representation contracted with an upstream gradient:
 *   dR[a] = d(sum_i g_i . rho_i) / dR_a,  so that for g = dE/drho the forces are -dR
 * (the representation's backward pass, GPU impl. of the Representation subsection).
 *   g: [n_atoms][length] FP32 (dE/drho); dR: [n_atoms][3] FP32 out; other arguments as
 *   sorf_fchl19_forward. Molecules of any size; an atom with more than 512 neighbours gets a
 *   NaN row. Every row is summed in an
 *   order fixed by its molecule alone (deterministic, the same alone as inside any batch).
 *   No workspace. */
sorf_status sorf_fchl19_backward(const float* R, const int32_t* element, const int64_t* mol_ptr,
                                 int64_t n_atoms, int64_t n_mols, int32_t n_elements,
                                 const sorf_fchl19_params* params, const float* g, float* dR,
                                 sorf_stream_t stream);

/* Bytes of workspace sorf_gram_accumulate needs for n_rows rows of D features in the given
 * precision (host-only query): the FP32 mode needs only the Z^T y partials (D * 8 bytes per
 * 1024 rows); the 16-bit modes also hold Z packed once in matrix-core fragment order
 * (2 bytes per entry per part, rows padded to 32 and columns to 256). 0 for invalid sizes. */
size_t sorf_gram_workspace_bytes(int64_t n_rows, int32_t D, sorf_gram_precision precision);

/* Normal-equation accumulation (RFF subsection, regularised normal equation):
 *   G[i][j] += sum_m Z[m][i] * Z[m][j]   for i >= j only (the strict upper triangle of G is
 *                                         neither read nor written),
 *   Zty[i]  += sum_m Z[m][i] * y[m]       (FP64 sums added to the FP32 Zty; skipped when y
 *                                         is NULL).
 *   Z: [n_rows][D] row-major, 16-byte aligned; G: [D][D] row-major.
 *   Every mode sums 256 rows at a time on the matrix cores and adds those partial sums in
 *   FP32 with round-to-nearest, so no long matrix-core accumulation drifts.
 *   scale_exp: the FP16 modes split 2^scale_exp * Z into parts and scale G back by
 *   2^(-2*scale_exp) exactly (keeps the low part out of the fp16 subnormal range); must be
 *   0 for the other modes, |scale_exp| <= 60.
 *   workspace: device memory of at least sorf_gram_workspace_bytes(n_rows, D, precision),
 *   256-byte aligned (may be NULL when that is 0). Results are deterministic. */
sorf_status sorf_gram_accumulate(int64_t n_rows, int32_t D, const float* Z, const float* y,
                                 sorf_gram_precision precision, int32_t scale_exp, float* G,
                                 float* Zty, void* workspace, size_t workspace_bytes,
                                 sorf_stream_t stream);

/* Double-precision normal equations (the paper's DP training mode; FP32 storage of
 * G cannot hold a ridge lambda far below 2^-24 * ||G|| -- e.g. lambda = 1e-6 on a
 * rank-deficient Gram -- because rounding G to FP32 already moves its eigenvalues
 * by more than lambda):
 *   G[i][j] += sum_m Z[m][i] Z[m][j] (i >= j, FP64 products and sums of the FP32 Z),
 *   Zty[i]  += sum_m Z[m][i] y[m] (FP64).   G: [D][D] FP64 row-major, Zty: [D] FP64. */
sorf_status sorf_gram_accumulate_f64(int64_t n_rows, int32_t D, const float* Z, const float* y,
                                     double* G, double* Zty, sorf_stream_t stream);

/* Bytes of workspace sorf_gram_accumulate_split needs (host-only query): Z^T y partials,
 * column maxima and exponents, and Z packed once as an int8 head (1 byte per entry) and
 * fp16 head and tail (2 bytes each), rows padded to 64 and columns to 256. 0 for invalid
 * sizes or n_rows = 0. */
size_t sorf_gram_split_workspace_bytes(int64_t n_rows, int32_t D);

/* Normal equations with an FP64 G from 8- and 16-bit matrix-core products (the RFF
 * subsection's regularised normal equation; Timings subsection: FP32 accumulation of
 * Z^T Z costs accuracy on ill-conditioned systems). Each column f of Z is scaled by
 * 2^e_f, e_f the largest exponent with max_m |Z[m][f]| 2^e_f <= 127, and split into an
 * integer head h = rint(Z 2^e_f) (|h| <= 127) and an fp16 tail t = fp16(Z 2^e_f - h):
 *   G[i][j] += 2^-(e_i + e_j) sum_m (h + t)[m][i] (h + t)[m][j]   for i >= j,
 * the Gram of the split representation, so G stays positive semidefinite. h^T h runs on
 * the int8 matrix cores with exact int32 sums (up to 131,072 rows per pass, more rows
 * take more passes); h^T t + t^T h + t^T t on the fp16 matrix cores, summed in FP32 over
 * 256-row blocks. |Z - 2^-e_f (h + t)| <= 2^-13 2^-e_f per entry, below 2^-19 of the
 * column's maximum (max 2^e_f > 63.5).
 *   Z^T y is summed in FP64 (skipped when y is NULL).
 *   Z: [n_rows][D] FP32 row-major, 16-byte aligned; G: [D][D] FP64 row-major (only the
 *   lower triangle is read and written); Zty: [D] FP64. workspace: at least
 *   sorf_gram_split_workspace_bytes(n_rows, D), 256-byte aligned. Deterministic. */
sorf_status sorf_gram_accumulate_split(int64_t n_rows, int32_t D, const float* Z, const float* y,
                                       double* G, double* Zty, void* workspace,
                                       size_t workspace_bytes, sorf_stream_t stream);

/* Bytes of workspace sorf_solve needs for a D x D system, 1 <= D <= 32768
 * (host-only query; returns 0 for an unsupported D). */
size_t sorf_solve_workspace_bytes(int32_t D);

/* Ridge solve of the regularised normal equation (LU in the paper; the matrix
 * is symmetric positive definite for lambda > 0, so Cholesky gives the same alpha):
 *   A = G + lambda I (G: lower triangle of an FP32 [D][D] row-major matrix, promoted to FP64),
 *   FP64 Cholesky A = L L^T, alpha = A^{-1} Zty, then n_refine steps of iterative
 *   refinement alpha += A^{-1} (Zty - A alpha) with the residual in FP64.
 *   alpha: [D] FP64 out. info: device int32, written 0 on success or k > 0 when the
 *   leading minor of order k is not positive definite (LAPACK convention; alpha is then
 *   undefined), or -1 if a triangular sweep gave up waiting for a block (an internal
 *   fault, reported instead of hanging; alpha is then undefined). workspace: device memory
 *   of at least sorf_solve_workspace_bytes(D), 256-byte aligned. 0 <= n_refine <= 16,
 *   lambda >= 0 and finite.
 *   Every launch goes to `stream`; the call uses no other stream or event. Calls on
 *   distinct streams with distinct workspaces and outputs are independent. */
sorf_status sorf_solve(int32_t D, const float* G, const float* Zty, double lambda,
                       int32_t n_refine, double* alpha, int32_t* info, void* workspace,
                       size_t workspace_bytes, sorf_stream_t stream);

/* sorf_solve for an FP64 lower-triangular G and FP64 Zty (from sorf_gram_accumulate_f64
 * or sorf_gram_accumulate_split); same workspace, outputs and error behaviour. */
sorf_status sorf_solve_f64(int32_t D, const double* G, const double* Zty, double lambda,
                           int32_t n_refine, double* alpha, int32_t* info, void* workspace,
                           size_t workspace_bytes, sorf_stream_t stream);

/* Caller-owned resources for the lookahead schedule of the factorisation: a second stream
 * on which the trailing updates run beside the chain of dependent diagonal steps, and two
 * events that order it with the call's stream. Host struct of HIP handles. */
typedef struct {
  sorf_stream_t side;  /* hipStream_t, must differ from the call's stream          */
  void* event_fork;    /* hipEvent_t                                              */
  void* event_join;    /* hipEvent_t, distinct from event_fork                    */
} sorf_solve_streams;

/* Create the resources of a sorf_solve_streams on the current device: a non-blocking
 * stream of default priority and two events without timing. Host call; returns
 * SORF_ERR_DEVICE (with every field NULL) if HIP refuses. The caller releases them with
 * sorf_solve_streams_destroy, which waits for the side stream first. */
sorf_status sorf_solve_streams_create(sorf_solve_streams* s);
sorf_status sorf_solve_streams_destroy(sorf_solve_streams* s);

/* sorf_solve / sorf_solve_f64 with the lookahead schedule: the trailing updates of step k
 * run on streams->side beside the diagonal factorisation of step k + 1 on `stream`. The
 * result is bitwise the one of sorf_solve (the same kernels in the same per-tile order);
 * the call returns with all its work ordered before later work on `stream`. The events
 * are recorded and waited for inside the call, so one sorf_solve_streams must not serve
 * two calls at once (calls from different host threads need one each); streams == NULL
 * is sorf_solve. Same arguments, outputs and errors otherwise; SORF_ERR_INVALID_ARG if a
 * handle is NULL, the side stream is `stream` or the two events are the same. */
sorf_status sorf_solve_streamed(int32_t D, const float* G, const float* Zty, double lambda,
                                int32_t n_refine, double* alpha, int32_t* info, void* workspace,
                                size_t workspace_bytes, const sorf_solve_streams* streams,
                                sorf_stream_t stream);
sorf_status sorf_solve_f64_streamed(int32_t D, const double* G, const double* Zty, double lambda,
                                    int32_t n_refine, double* alpha, int32_t* info,
                                    void* workspace, size_t workspace_bytes,
                                    const sorf_solve_streams* streams, sorf_stream_t stream);

/* Bytes of workspace sorf_predict needs for a batch of n_atoms atoms in n_mols molecules
 * (host-only query; nondecreasing in both, so a buffer sized for the largest batch serves
 * every smaller one). Returns 0 for an invalid model or negative sizes. */
size_t sorf_predict_workspace_bytes(const sorf_model* model, int64_t n_atoms, int64_t n_mols);

/* Prediction of energies (E = Z alpha, without forming Z) and, when J is given,
 * forces F = -sum_{i in m} J_i^T dE/dx_i (RFF subsection: the atomic energy
 * decomposition E = sum_I alpha^T z(rho_I) = Z alpha, and forces as minus the coordinate
 * derivative of the energy, taken through the representations' Jacobians; Timings
 * subsection: energies and forces of many configurations predicted in one call).
 *   alpha: [D] FP32.  E: [n_mols] FP32 out.
 *   J: concatenated per-molecule blocks, block m is [N_m][d][3 N_m] row-major
 *      (J_i = dx_i/dr_m, coordinates ordered [atom][xyz]) starting at float offset
 *      J_ptr[m]; J_ptr: [n_mols + 1] int64 device array. Blocks may sit anywhere in J
 *      (no order, gaps allowed; J_ptr[n_mols] is not read) and need no alignment.
 *      Both NULL for energies only.
 *   Each molecule's E and F are summed in an order fixed by its own atoms, so a
 *   molecule's results are bitwise the same in any batch. Without J, E is summed per
 *   (molecule, stack) over the atoms and then over the stacks; with J, per atom over the
 *   features and then over the atoms: the two E agree to FP32 rounding, not bitwise.
 *   F: [3 n_atoms] FP32 out ([atom][xyz]), required iff J is given.
 *   workspace: device memory of at least sorf_predict_workspace_bytes(), 256-byte aligned. */
sorf_status sorf_predict(const sorf_model* model, const sorf_batch* batch, const float* alpha,
                         const float* J, const int64_t* J_ptr, float* E, float* F,
                         void* workspace, size_t workspace_bytes, sorf_stream_t stream);

/* sorf_predict for callers that cannot allocate device memory or pass a workspace:
 * code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments (minus the workspace), kernels, results (bitwise) and error behaviour
 * as sorf_predict. The workspace is a file-scope device array of
 * SORF_PREDICT_NOALLOC_SCRATCH_BYTES per GPU, held from library load until the process
 * ends; its device address is looked up once per device on the first call made with that
 * device current. A batch whose sorf_predict_workspace_bytes() exceeds
 * SORF_PREDICT_NOALLOC_SCRATCH_BYTES is rejected with SORF_ERR_WORKSPACE before any
 * device work; SORF_ERR_DEVICE if the array's address cannot be obtained. Every kernel
 * writes the scratch it reads, so nothing needs clearing between calls. All calls on
 * one GPU share that GPU's array: calls that overlap on one GPU (different streams or
 * host threads without ordering) race and give undefined results; the caller must
 * serialise them. */
#define SORF_PREDICT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sorf_status sorf_predict_noalloc(const sorf_model* model, const sorf_batch* batch,
                                 const float* alpha, const float* J, const int64_t* J_ptr,
                                 float* E, float* F, sorf_stream_t stream);

/* Bytes of workspace sorf_forces needs for n_atoms atoms in n_mols molecules (host-only
 * query, nondecreasing in both). Returns 0 for negative sizes. */
size_t sorf_forces_workspace_bytes(int64_t n_atoms, int64_t n_mols);

/* Forces from a given gradient of the energy with respect to the atoms'
 * representations, dE/dx (Theory section: the forces are minus the derivative of
 * the energy with respect to the atomic coordinates, which the chain rule takes
 * through the representation's Jacobians):
 *   F[3 a + k] = -sum_{i in m} (J_i^T grad_x_i)[3 (a - a0) + k],  a0 = mol_ptr[m],
 * for atom a of molecule m and coordinate k. With grad_x from sorf_backward (dE = NULL)
 * this is the force part of sorf_predict, as a call of its own.
 *   d: length of each atom's gradient row, >= 1.  mol_ptr: [n_mols + 1] int64 CSR
 *     (same device-side preconditions as a batch).
 *   grad_x: [n_atoms][d] FP32.  J, J_ptr: the Jacobian blocks exactly as sorf_predict
 *     takes them.  F: [3 n_atoms] FP32 out ([atom][xyz]).
 *   Each force is summed in an order fixed by its own molecule (row chunks of the
 *   block, then chunks in order), so a molecule's forces are bitwise the same in any
 *   batch and equal to sorf_predict's for the same gradient.
 *   workspace: device memory of at least sorf_forces_workspace_bytes(), 256-byte
 *     aligned. grad_x, J, J_ptr, F and the workspace are required when n_atoms > 0. */
sorf_status sorf_forces(int32_t d, int64_t n_atoms, int64_t n_mols, const int64_t* mol_ptr,
                        const float* grad_x, const float* J, const int64_t* J_ptr, float* F,
                        void* workspace, size_t workspace_bytes, sorf_stream_t stream);

/* ---------------------------------------------------------------------------
 * Continuous-batching server for energy + force requests (Timings subsection:
 * predicting many configurations in one call rather than one small molecule at
 * a time). sorf_server_start launches one persistent kernel that stays resident
 * on every compute unit of the current device until sorf_server_stop. The host
 * then publishes batches of requests, each a contiguous run of molecules of a
 * device-resident request pool, with sorf_server_submit (a descriptor written into
 * a ring in host-coherent memory: no launch, copy or event per batch). The kernel
 * takes the batches in submission order and writes each one's energies and forces
 * into a host-coherent result slot; sorf_server_query reports completion. Every
 * result is summed in the order sorf_predict uses, so a request's energy and forces
 * are bitwise those of sorf_predict with its Jacobian on that request alone,
 * whatever batch it is served in.
 * Exceptions to the conventions above: sorf_server_start allocates the ring,
 * control word and result slots in pinned host memory (hipHostMalloc) and
 * sorf_server_stop frees them; while the kernel runs it holds nearly all the
 * vector registers of every compute unit, so other kernels on the device wait
 * until it exits (sorf_server_stop, or the idle timeout): a served device serves
 * only; sorf_server_stop blocks until the kernel has exited. A server is used
 * from one host thread at a time.
 * --------------------------------------------------------------------------- */
typedef struct sorf_server sorf_server;   /* opaque, owned by the caller between start and stop */
typedef struct {
  int64_t max_batch_atoms;   /* atoms of the largest batch, 1 .. 2^24 (sizes scratch and slots) */
  int32_t ring_slots;        /* batches published ahead of the kernel, 1 .. 64; a batch's result
                                slot is reused by the batch ring_slots later */
  double idle_timeout_s;     /* the kernel exits after this long without a batch, (0, 3600] */
} sorf_server_config;

/* Bytes of device workspace a server needs (host-only query): 0 for an invalid model or
 * configuration. */
size_t sorf_server_workspace_bytes(const sorf_model* model, const sorf_server_config* cfg);

/* Starts the server on `stream` (a stream of the current device that the caller does not
 * use otherwise until sorf_server_stop). alpha: [D] FP32; x_pool [A][d], element_pool [A]:
 * the request pool's atoms; J_pool: Jacobian blocks, block r at any float offset (as in
 * sorf_predict). All device arrays must stay valid and unchanged until the server stops.
 * workspace: device memory of at least sorf_server_workspace_bytes(), 256-byte aligned, kept
 * by the server until stop. On success *server is the handle; on failure it is NULL and no
 * kernel runs. */
sorf_status sorf_server_start(const sorf_model* model, const float* alpha, const float* x_pool,
                              const int32_t* element_pool, const float* J_pool,
                              const sorf_server_config* cfg, void* workspace,
                              size_t workspace_bytes, sorf_stream_t stream, sorf_server** server);

/* Publishes a batch of n_requests (1 .. 64) requests: request r has atoms
 * [atom_offsets[r], atom_offsets[r + 1]) of the pool (host array of n_requests + 1
 * nondecreasing offsets, at most max_batch_atoms atoms in all) and its Jacobian block at
 * float offset J_offsets[r] of J_pool (host array). *ticket receives the batch number
 * (0, 1, 2, ... in submission order). SORF_ERR_BUSY: ring_slots batches are unfinished;
 * SORF_ERR_DEVICE: the kernel has exited. */
sorf_status sorf_server_submit(sorf_server* server, int32_t n_requests, const int64_t* atom_offsets,
                               const int64_t* J_offsets, int64_t* ticket);

/* 1: batch `ticket` is finished and its results readable; 0: not yet; -1: the kernel has
 * exited without finishing it; -2: no such ticket. */
int32_t sorf_server_query(const sorf_server* server, int64_t ticket);

/* Host pointers into the result slot of a finished batch: energies [n_requests] and forces
 * [3 x atoms of the batch] ([atom][xyz], requests in order). Valid until the batch
 * ring_slots later is submitted or the server stops; NULL for an unknown ticket. */
const float* sorf_server_energies(const sorf_server* server, int64_t ticket);
const float* sorf_server_forces(const sorf_server* server, int64_t ticket);

/* Asks the kernel to finish the published batches and exit, waits for it and frees the
 * server. *state (may be NULL): 1 stopped on request, 2 had exited after idle_timeout_s,
 * 3 had exited on a wait limit (a fault of the server, reported rather than hung). */
sorf_status sorf_server_stop(sorf_server* server, int32_t* state);

/* Opt-in debug check of the device-side preconditions of a batch. Writes to
 * *result (device int32) a bit mask: 0 if mol_ptr is a valid CSR over n_atoms atoms
 * and every element id is in [0, n_elements); otherwise bit 0: mol_ptr[0] != 0,
 * bit 1: some offset decreases, bit 2: mol_ptr[n_mols] != n_atoms,
 * bit 3: an element id is out of range. */
sorf_status sorf_validate_batch(const sorf_batch* batch, int32_t n_elements, int32_t* result,
                                sorf_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SORF_H */
