"""FP64 CPU oracle for the SORF hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It shares no code with the HIP
library -- no kernels, headers, helpers, tables or pre/post-processing.

It computes the same estimator the GPU computes, but by the plain dense
route the paper describes before introducing the fast transform: it builds
the explicit matrix W = c * H D_{T-1} ... H D_0 for every element and stack,
multiplies, takes the cosine, sums per molecule, forms the normal equations
with a library matmul, and solves them with a library Cholesky. Everything is
float64.

Paper passages followed (arXiv 2206.01580, Theory section):

* RFF subsection, feature-map equation: z(rho) = sqrt(2/N_F) [cos(w_i^T rho + b_i)],
  b_i uniform on [0, 2 pi).
* RFF subsection, atomic energy decomposition: E = sum_I alpha^T z(rho_I) = Z alpha.
* RFF subsection, regularised normal equation: (Z^T Z + lambda I) alpha = Z^T E.
* RFF subsection, force derivatives dZ (derivative features); forces are the
  negative coordinate gradient of the energy.
* RFF subsection, force-trained normal equation:
  ((Z, dZ)^T (Z, dZ) + lambda I) alpha = (Z, dZ)^T (E, F), dZ with one row
  per atomic coordinate (3 N_atom rows).
* SORF subsection, W_ORF ~ (sqrt(d)/sigma) [H_i D_i]_{N_transform}; the
  Sylvester recursion for H; stacking of N_F/d independent blocks.
* SORF subsection, projection to 2^n dimensions: per element, the SVD
  Z~_e = U_e S_e V_e^T of sampled representations and rho_proj = rho^T U_e^{N_PCA}.

Readings taken where the paper is silent or ambiguous (all listed in the
design notes of the repository):

* Normalisation: the bracket [H_i D_i] stands for an orthogonal matrix, so H
  is used as H/sqrt(d); on the +-1 Sylvester matrix this gives the scalar
  c = (sqrt(d)/sigma) * d**(-T/2).
* Transform order: sign matrix t = 0 is applied first.
* Feature order: feature f = s*d + j (stack-major), j in natural Sylvester order.
* Per-element signs and per-element phases.
* Normaliser sqrt(2/D) with D = n_stacks * d the total number of features.
* No intercept; lambda is added to the diagonal unscaled.
* Forces F = -dE/dr; with Jacobian blocks J_i = dx_i/dr (d x 3N) this is
  F = -sum_i J_i^T (dE/dx_i).
* The rows of dZ hold the NEGATIVE coordinate derivatives of Z, so that
  dZ alpha = F and the stacked system pairs dZ with F as printed.
* Projection: the representations are the COLUMNS of Z~_e (so U_e acts on
  representation space), the SVD is of the raw matrix (no centring; the
  paper names an SVD, not a covariance), and each singular vector's sign is
  fixed by its largest-magnitude entry.

Pins: each function is checked in ``tests/test_oracle_pins.py`` against
closed forms, invariants, exact enumeration, brute force and independent
library routines.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

__all__ = [
    "hadamard", "sorf_scale", "dense_block", "dense_w", "phases", "atom_features",
    "molecule_features", "gram", "solve", "predict_energies", "grad_x", "forces",
    "derivative_features", "force_normal_equations", "projection_fit", "project",
    "round_bf16", "round_fp16", "split_hilo", "gram_emulated", "split_head_tail",
]


# --------------------------------------------------------------------------
# The structured operator (SORF subsection)
# --------------------------------------------------------------------------

def hadamard(d: int) -> np.ndarray:
    """Walsh-Hadamard matrix of order d by the Sylvester recursion
    H_1 = 1, H_{2n} = [[H_n, H_n], [H_n, -H_n]] (SORF subsection)."""
    if d < 1 or d & (d - 1):
        raise ValueError("d must be a power of two")
    H = np.ones((1, 1), dtype=np.float64)
    while H.shape[0] < d:
        H = np.block([[H, H], [H, -H]])
    return H


def sorf_scale(d: int, n_transforms: int, sigma: float) -> float:
    """Scalar in front of the product of +-1 Hadamard and sign matrices.

    The SORF approximation writes W ~ (sqrt(d)/sigma) Q with Q orthogonal and
    Q replaced by the product of N_transform factors H D. Each +-1 Hadamard
    factor is orthogonal only after division by sqrt(d), so
    c = (sqrt(d)/sigma) * d**(-N_transform/2)."""
    return math.sqrt(d) / sigma * d ** (-n_transforms / 2.0)


def dense_block(signs_ts: np.ndarray, sigma: float) -> np.ndarray:
    """One d x d block W_s = c * H D_{T-1} ... H D_1 H D_0 for one element and
    one stack. ``signs_ts`` is [T, d] with entries +-1, row t = D_t."""
    signs_ts = np.asarray(signs_ts, dtype=np.float64)
    T, d = signs_ts.shape
    H = hadamard(d)
    B = np.eye(d)
    for t in range(T):
        B = H @ np.diag(signs_ts[t]) @ B
    return sorf_scale(d, T, sigma) * B


def dense_w(signs_e: np.ndarray, sigma: float) -> np.ndarray:
    """Stacked W_e of shape [D, d] for one element: rows s*d .. s*d+d-1 come
    from stack s (stacking of N_F/d blocks, SORF subsection).
    ``signs_e`` is [T, S, d]."""
    T, S, d = signs_e.shape
    return np.concatenate([dense_block(signs_e[:, s, :], sigma) for s in range(S)], axis=0)


# --------------------------------------------------------------------------
# Feature map and per-molecule features (RFF subsection)
# --------------------------------------------------------------------------

def _molecule_index(mol_ptr: np.ndarray) -> np.ndarray:
    sizes = np.diff(np.asarray(mol_ptr, dtype=np.int64))
    return np.repeat(np.arange(len(sizes)), sizes)


def phases(x, element, signs, bias, sigma, atoms=None, cols=None) -> np.ndarray:
    """u_i = W_{e_i} x_i + b_{e_i} for the atoms listed (all by default),
    restricted to the feature columns ``cols`` (all by default); returns
    [len(atoms), len(cols)] float64."""
    x = np.asarray(x, dtype=np.float64)
    element = np.asarray(element)
    if atoms is None:
        atoms = np.arange(x.shape[0])
    atoms = np.asarray(atoms, dtype=np.int64)
    E = signs.shape[0]
    D = signs.shape[2] * signs.shape[3]
    cols = np.arange(D) if cols is None else np.asarray(cols, dtype=np.int64)
    u = np.empty((len(atoms), len(cols)), dtype=np.float64)
    for e in range(E):
        sel = np.nonzero(element[atoms] == e)[0]
        if len(sel) == 0:
            continue
        W = dense_w(signs[e], sigma)[cols]
        u[sel] = x[atoms[sel]] @ W.T + np.asarray(bias[e], dtype=np.float64)[cols]
    return u


def atom_features(x, element, signs, bias, sigma, atoms=None, cols=None) -> np.ndarray:
    """z(x_i) = sqrt(2/D) cos(W_{e_i} x_i + b_{e_i}) (feature-map equation),
    D being the total number of features even when only ``cols`` are formed."""
    D = signs.shape[2] * signs.shape[3]
    u = phases(x, element, signs, bias, sigma, atoms, cols)
    return math.sqrt(2.0 / D) * np.cos(u)


def molecule_features(x, element, mol_ptr, signs, bias, sigma, mols=None,
                      chunk_atoms: int = 4096, cols=None) -> np.ndarray:
    """Rows Z_m = sum over the atoms of molecule m of z(x_i) (atomic energy
    decomposition: E_m = sum_I alpha^T z(rho_I) = Z_m alpha).
    ``mols`` selects rows and ``cols`` feature columns (all by default);
    returns [len(mols), len(cols)]."""
    mol_ptr = np.asarray(mol_ptr, dtype=np.int64)
    M = len(mol_ptr) - 1
    if mols is None:
        mols = np.arange(M)
    mols = np.asarray(mols, dtype=np.int64)
    D = signs.shape[2] * signs.shape[3] if cols is None else len(cols)
    Z = np.zeros((len(mols), D), dtype=np.float64)
    # gather the atoms of the selected molecules, remember which row they feed
    atom_lists = [np.arange(mol_ptr[m], mol_ptr[m + 1]) for m in mols]
    rows = np.concatenate([np.full(len(a), r) for r, a in enumerate(atom_lists)]) \
        if len(mols) else np.zeros(0, np.int64)
    atoms = np.concatenate(atom_lists) if len(mols) else np.zeros(0, np.int64)
    for c0 in range(0, len(atoms), chunk_atoms):
        sl = slice(c0, c0 + chunk_atoms)
        z = atom_features(x, element, signs, bias, sigma, atoms[sl], cols)
        np.add.at(Z, rows[sl], z)
    return Z


# --------------------------------------------------------------------------
# Normal equations, solve, prediction (RFF subsection)
# --------------------------------------------------------------------------

def gram(Z, y=None):
    """G = Z^T Z and r = Z^T y in float64 (regularised normal equation)."""
    Z = np.asarray(Z, dtype=np.float64)
    G = Z.T @ Z
    r = None if y is None else Z.T @ np.asarray(y, dtype=np.float64)
    return G, r


def solve(G, rhs, lam: float) -> np.ndarray:
    """alpha = (G + lam I)^{-1} rhs by Cholesky (the matrix is symmetric
    positive definite for lam > 0; the paper's LU gives the same alpha)."""
    G = np.asarray(G, dtype=np.float64)
    A = G + lam * np.eye(G.shape[0])
    cf = scipy.linalg.cho_factor(A, lower=True)
    return scipy.linalg.cho_solve(cf, np.asarray(rhs, dtype=np.float64))


def predict_energies(Z, alpha) -> np.ndarray:
    """E = Z alpha."""
    return np.asarray(Z, dtype=np.float64) @ np.asarray(alpha, dtype=np.float64)


def grad_x(x, element, mol_ptr, signs, bias, sigma, alpha, dE=None,
           chunk_atoms: int = 4096) -> np.ndarray:
    """dL/dx_i for L = sum_m dE_m E_m (dE = upstream weights, default 1):
    dL/dx_i = dE_{m(i)} * W_{e_i}^T ( -sqrt(2/D) sin(u_i) * alpha )."""
    x = np.asarray(x, dtype=np.float64)
    A, d = x.shape
    D = signs.shape[2] * signs.shape[3]
    alpha = np.asarray(alpha, dtype=np.float64)
    mol_of = _molecule_index(mol_ptr)
    w = np.ones(len(mol_ptr) - 1) if dE is None else np.asarray(dE, dtype=np.float64)
    out = np.zeros((A, d), dtype=np.float64)
    Ws = [dense_w(signs[e], sigma) for e in range(signs.shape[0])]
    for c0 in range(0, A, chunk_atoms):
        idx = np.arange(c0, min(A, c0 + chunk_atoms))
        u = phases(x, element, signs, bias, sigma, idx)
        g = -math.sqrt(2.0 / D) * np.sin(u) * alpha[None, :] * w[mol_of[idx]][:, None]
        for e in range(signs.shape[0]):
            sel = np.nonzero(np.asarray(element)[idx] == e)[0]
            if len(sel):
                out[idx[sel]] = g[sel] @ Ws[e]
    return out


def forces(grad, J, J_ptr, mol_ptr) -> np.ndarray:
    """F_m = -sum_{i in m} J_i^T dE/dx_i with J_i = dx_i/dr_m of shape d x 3N_m,
    blocks stored [N_m, d, 3N_m] at J[J_ptr[m]:]. Returns [3 * n_atoms]
    ordered [atom][xyz] like the coordinates."""
    grad = np.asarray(grad, dtype=np.float64)
    mol_ptr = np.asarray(mol_ptr, dtype=np.int64)
    A, d = grad.shape
    F = np.zeros(3 * A, dtype=np.float64)
    for m in range(len(mol_ptr) - 1):
        a0, a1 = int(mol_ptr[m]), int(mol_ptr[m + 1])
        n = a1 - a0
        if n == 0:
            continue
        blk = np.asarray(J[J_ptr[m]:J_ptr[m + 1]], dtype=np.float64).reshape(n, d, 3 * n)
        F[3 * a0:3 * a1] = -np.einsum("ijk,ij->k", blk, grad[a0:a1])
    return F


def derivative_features(x, element, mol_ptr, signs, bias, sigma, J, J_ptr,
                        mols=None, cols=None) -> np.ndarray:
    """Derivative feature matrix dZ of the force-trained normal equation
    (RFF subsection): one row per atomic coordinate, rows ordered like the
    coordinates ([atom][xyz]), holding the negative derivative of the
    molecule's feature row with respect to that coordinate,

        dZ[3 a + k] = -dZ_m / dr_{a,k}
                    = sqrt(2/D) sum_{i in m} sin(u_i) * (W_{e_i} J_i)[:, 3 (a - a0) + k],

    so that dZ alpha = -dE/dr = F and (Z, dZ)^T (E, F) pairs energies with Z
    and forces with dZ. J_i = dx_i/dr_m (d x 3 N_m) is block m of J as in
    ``forces``. ``mols`` selects molecules (all by default; their rows are
    concatenated in the given order) and ``cols`` feature columns.
    Returns [3 * (atoms of mols), len(cols)] float64."""
    x = np.asarray(x, dtype=np.float64)
    element = np.asarray(element)
    mol_ptr = np.asarray(mol_ptr, dtype=np.int64)
    A, d = x.shape
    D = signs.shape[2] * signs.shape[3]
    cols = np.arange(D) if cols is None else np.asarray(cols, dtype=np.int64)
    if mols is None:
        mols = np.arange(len(mol_ptr) - 1)
    Ws = [dense_w(signs[e], sigma)[cols] for e in range(signs.shape[0])]
    blocks = []
    for m in np.asarray(mols, dtype=np.int64):
        a0, a1 = int(mol_ptr[m]), int(mol_ptr[m + 1])
        n = a1 - a0
        out = np.zeros((3 * n, len(cols)), dtype=np.float64)
        if n:
            blk = np.asarray(J[J_ptr[m]:J_ptr[m] + n * d * 3 * n],
                             dtype=np.float64).reshape(n, d, 3 * n)
            s = np.sin(phases(x, element, signs, bias, sigma, np.arange(a0, a1), cols))
            for i in range(n):
                WJ = Ws[element[a0 + i]] @ blk[i]          # [len(cols), 3 n]
                out += (s[i][:, None] * WJ).T
            out *= math.sqrt(2.0 / D)
        blocks.append(out)
    if not blocks:
        return np.zeros((0, len(cols)), dtype=np.float64)
    return np.concatenate(blocks, axis=0)


def force_normal_equations(Z, dZ, E, F):
    """(Z, dZ)^T (Z, dZ) and (Z, dZ)^T (E, F) of the force-trained normal
    equation: the energy rows and the coordinate rows stacked into one
    least-squares system. float64."""
    A = np.concatenate([np.asarray(Z, dtype=np.float64), np.asarray(dZ, dtype=np.float64)])
    b = np.concatenate([np.asarray(E, dtype=np.float64), np.asarray(F, dtype=np.float64)])
    return A.T @ A, A.T @ b


# --------------------------------------------------------------------------
# Per-element projection of the representation to d = 2^n (SORF subsection)
# --------------------------------------------------------------------------

def projection_fit(rho_sample, n_pca: int):
    """U_e^{N_PCA} of one element: the first ``n_pca`` left singular vectors of
    the matrix whose columns are the sampled representations of that element
    (Z~_e = U_e S_e V_e^T, SORF subsection), each column's sign fixed so that
    its entry of largest magnitude is positive (the SVD leaves the sign free).
    rho_sample: [n_samples, d_rep]. Returns (U [d_rep, n_pca], s [n_pca]) in
    float64; the singular values come in decreasing order. The columns are
    unique (up to the sign fixed here) only where the singular values are
    distinct and nonzero, so the sample needs at least n_pca rows of rank
    n_pca."""
    Zt = np.asarray(rho_sample, dtype=np.float64).T
    U, s, _ = np.linalg.svd(Zt, full_matrices=False)
    U = U[:, :n_pca].copy()
    piv = np.argmax(np.abs(U), axis=0)
    U *= np.sign(U[piv, np.arange(U.shape[1])])[None, :]
    return U, s[:n_pca]


def project(rho, element, U):
    """x_i = rho_i^T U_{e_i}: the projected representation of every atom with
    its own element's matrix. rho: [A, d_rep]; U: [E, d_rep, d]. float64."""
    rho = np.asarray(rho, dtype=np.float64)
    element = np.asarray(element)
    U = np.asarray(U, dtype=np.float64)
    x = np.zeros((rho.shape[0], U.shape[2]), dtype=np.float64)
    for e in range(U.shape[0]):
        sel = np.nonzero(element == e)[0]
        if len(sel):
            x[sel] = rho[sel] @ U[e]
    return x


# --------------------------------------------------------------------------
# Reduced-precision Gram emulation
# --------------------------------------------------------------------------

def round_bf16(a) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even);
    returned as float32 holding the rounded values. Finite inputs only."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def round_fp16(a) -> np.ndarray:
    """Round float32 values to IEEE binary16 (ties to even); returned as
    float32 holding the rounded values."""
    return np.asarray(a, dtype=np.float32).astype(np.float16).astype(np.float32)


def split_hilo(Z, kind: str, scale_exp: int = 0):
    """hi = round(s*z), lo = round(s*z - hi) with s = 2**scale_exp, the
    difference taken in float32 (exact). ``kind`` is 'bf16' or 'fp16'."""
    rnd = round_bf16 if kind == "bf16" else round_fp16
    z = np.asarray(Z, dtype=np.float32) * np.float32(2.0 ** scale_exp)
    hi = rnd(z)
    lo = rnd((z - hi).astype(np.float32))
    return hi, lo


def split_head_tail(Z):
    """Per-column integer head and fp16 tail of the split Gram mode.

    For column f, e_f is the largest integer with max_m |Z[m, f]| * 2**e_f <= 127
    (0 for an all-zero column); w = Z * 2**e_f (exact); h = round-half-even(w),
    an integer with |h| <= 127; t = fp16(w - h). Returns (h, t, e) with h and t
    float64 arrays holding the exact values and e int64 [D]. Found here by a
    search from a floating-point guess, checked against the defining inequality."""
    Z32 = np.asarray(Z, dtype=np.float32)
    m = np.abs(Z32).max(axis=0).astype(np.float64) if Z32.shape[0] else np.zeros(Z32.shape[1])
    e = np.zeros(m.shape, dtype=np.int64)
    for f in range(len(m)):
        if m[f] == 0.0:
            continue
        k = int(math.floor(math.log2(127.0 / m[f])))
        while math.ldexp(m[f], k) > 127.0:
            k -= 1
        while math.ldexp(m[f], k + 1) <= 127.0:
            k += 1
        e[f] = k
    w = Z32.astype(np.float64) * np.exp2(e.astype(np.float64))[None, :]   # exact
    h = np.rint(w)
    t = (w - h).astype(np.float32).astype(np.float16).astype(np.float64)
    return h, t, e


def gram_emulated(Z, mode: str, scale_exp: int = 0) -> np.ndarray:
    """The Gram matrix each reduced-precision mode must produce when its
    products are exact and accumulation error is ignored (float64 sums):

    * 'fp32', 'fp32_kahan'  Z^T Z of the float32 values (the modes differ
                   only in how their accumulation rounds)
    * 'bf16'/'fp16'      hi^T hi
    * 'bf16_hilo'/'fp16_hilo'  (hi + lo)^T (hi + lo), all four products

    * 'split'      (h + t)^T (h + t) scaled by 2**-(e_i + e_j), the head and
                   tail of ``split_head_tail`` (``scale_exp`` unused)

    scaled back by 2**(-2*scale_exp). The split modes keep lo^T lo so that
    the result is the Gram matrix of the two-term approximation hi + lo and
    stays positive semidefinite, as the normal equations require."""
    Z32 = np.asarray(Z, dtype=np.float32)
    if mode == "split":
        h, t, e = split_head_tail(Z32)
        v = (h + t) * np.exp2(-e.astype(np.float64))[None, :]    # exact in float64
        return v.T @ v
    if mode in ("fp32", "fp32_kahan"):
        Zd = Z32.astype(np.float64)
        return Zd.T @ Zd
    kind = mode.split("_")[0]
    hi, lo = split_hilo(Z32, kind, scale_exp)
    hi = hi.astype(np.float64)
    lo = lo.astype(np.float64)
    if mode.endswith("hilo"):
        z2 = hi + lo          # exact in float64
        G = z2.T @ z2
    else:
        G = hi.T @ hi
    return G * 2.0 ** (-2 * scale_exp)
