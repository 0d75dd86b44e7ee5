"""Seeded synthetic inputs for the SORF hot path.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no Hadamard transform, no cosine, no sums over atoms).
Both the HIP path and the FP64 oracle consume exactly the arrays it returns.

The random parameters the method itself draws -- the Rademacher sign
diagonals of the SORF operator (SORF subsection, the W_ORF approximation) and
the phases b ~ U[0, 2*pi) of the random-feature map (RFF subsection, feature
map equation) -- are drawn here and passed to both sides as inputs.

Array conventions (shared by both sides):

* ``x``        float32 [n_atoms, d]    per-atom projected representation
* ``element``  int32   [n_atoms]       element index in [0, n_elements)
* ``mol_ptr``  int64   [n_mols + 1]    CSR offsets, atoms of molecule m are
                                       mol_ptr[m] .. mol_ptr[m+1]-1
* ``signs``    int8    [n_elements, n_transforms, n_stacks, d]  entries +-1;
                                       transform index t = 0 is applied first
* ``bias``     float32 [n_elements, n_stacks * d]  phases in [0, 2*pi)
* ``y``        float32 [n_mols]        regression targets (energy workloads)
* ``alpha``    float32 [n_stacks * d]  model weights (differentiation/serving)
* ``J``        float32 concatenated per-molecule blocks [N_m, d, 3 N_m]
* ``J_ptr``    int64   [n_mols + 1]    float offsets of each block in ``J``

The workloads mirror the molecule-shaped inputs the paper trains and predicts
on (QM9-like and MD17-like sets, Results section); the datasets themselves are
not used -- only their sizes and element mixes are imitated with synthetic
numbers.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 220601580


@dataclasses.dataclass
class Problem:
    """One synthetic workload. All arrays are host numpy arrays."""

    name: str
    d: int
    n_stacks: int
    n_transforms: int
    sigma: float
    element_names: tuple
    x: np.ndarray
    element: np.ndarray
    mol_ptr: np.ndarray
    signs: np.ndarray
    bias: np.ndarray
    y: Optional[np.ndarray] = None
    alpha: Optional[np.ndarray] = None
    J: Optional[np.ndarray] = None
    J_ptr: Optional[np.ndarray] = None
    lam: float = 0.0
    seed: int = 0

    @property
    def n_features(self) -> int:
        return self.d * self.n_stacks

    @property
    def n_atoms(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_mols(self) -> int:
        return int(self.mol_ptr.shape[0] - 1)

    @property
    def n_elements(self) -> int:
        return int(self.signs.shape[0])

    def mol_sizes(self) -> np.ndarray:
        return np.diff(self.mol_ptr)

    def subset(self, mols) -> "Problem":
        """Molecules ``mols`` (in the order given) as a new Problem that shares
        the model parameters. J is sliced along with the atoms if present."""
        mols = np.asarray(mols, dtype=np.int64)
        sizes = self.mol_sizes()[mols]
        ptr = np.zeros(len(mols) + 1, dtype=np.int64)
        np.cumsum(sizes, out=ptr[1:])
        atoms = np.concatenate(
            [np.arange(self.mol_ptr[m], self.mol_ptr[m + 1]) for m in mols]
        ) if len(mols) else np.zeros(0, dtype=np.int64)
        J = J_ptr = None
        if self.J is not None:
            blocks = [self.J[self.J_ptr[m]:self.J_ptr[m + 1]] for m in mols]
            J = np.concatenate(blocks) if blocks else np.zeros(0, np.float32)
            J_ptr = np.zeros(len(mols) + 1, dtype=np.int64)
            np.cumsum([b.size for b in blocks], out=J_ptr[1:])
        return dataclasses.replace(
            self,
            x=np.ascontiguousarray(self.x[atoms]),
            element=np.ascontiguousarray(self.element[atoms]),
            mol_ptr=ptr,
            y=None if self.y is None else np.ascontiguousarray(self.y[mols]),
            J=J,
            J_ptr=J_ptr,
        )


def _jacobian_rng(seed: int):
    """Jacobians come from their own stream so that leaving them out does not
    change any other array of the workload."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1])))


def _ptr_from_sizes(sizes: np.ndarray) -> np.ndarray:
    ptr = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    return ptr


def draw_signs(rng, n_elements, n_transforms, n_stacks, d) -> np.ndarray:
    """Rademacher entries of the diagonal sign matrices, one set per element,
    transform and stack."""
    bits = rng.integers(0, 2, size=(n_elements, n_transforms, n_stacks, d), dtype=np.int8)
    return (1 - 2 * bits).astype(np.int8)


def draw_bias(rng, n_elements, n_features) -> np.ndarray:
    """Phases b ~ U[0, 2*pi), one per element and feature."""
    b = rng.uniform(0.0, 2.0 * math.pi, size=(n_elements, n_features))
    b = b.astype(np.float32)
    # float32 rounding may land exactly on 2*pi; keep the half-open interval.
    b[b >= np.float32(2.0 * math.pi)] = 0.0
    return b


def _linear_targets(rng, x, mol_ptr, noise_std=0.01):
    """y_m = sum over the atoms of a random linear functional a^T x_i, plus
    Gaussian noise. Targets only; this is not part of the SORF arithmetic."""
    d = x.shape[1]
    a = rng.normal(0.0, 1.0 / math.sqrt(d), size=d)
    per_atom = x.astype(np.float64) @ a
    csum = np.concatenate([[0.0], np.cumsum(per_atom)])
    y = csum[mol_ptr[1:]] - csum[mol_ptr[:-1]]
    y = y + rng.normal(0.0, noise_std, size=y.shape)
    return y.astype(np.float32)


def qm9_like_sizes(rng, n_mols):
    """QM9-like molecule sizes: 3 + Binomial(26, 15/26), support 3..29, mean 18."""
    return 3 + rng.binomial(26, 15.0 / 26.0, size=n_mols)


def small_energy_batch(seed_offset: int = 0) -> Problem:
    """Small energy model: 200 molecules of 3..20 atoms, d=64, 4 stacks."""
    seed = SEED_BASE + 1 + seed_offset
    rng = np.random.Generator(np.random.PCG64(seed))
    M, d, S, T = 200, 64, 4, 3
    names = ("H", "C", "N", "O")
    sizes = rng.integers(3, 21, size=M)
    ptr = _ptr_from_sizes(sizes)
    A = int(ptr[-1])
    element = rng.choice(len(names), size=A, p=[0.5, 0.3, 0.1, 0.1]).astype(np.int32)
    x = (0.5 * rng.standard_normal((A, d))).astype(np.float32)
    signs = draw_signs(rng, len(names), T, S, d)
    bias = draw_bias(rng, len(names), S * d)
    y = _linear_targets(rng, x, ptr)
    return Problem("small-energy-200", d, S, T, 2.0, names, x, element, ptr,
                   signs, bias, y=y, lam=1e-6, seed=seed)


def qm9_like(n_mols: int, n_stacks: int, seed: int, name: str, sigma=4.0, lam=0.0,
             d: int = 128) -> Problem:
    rng = np.random.Generator(np.random.PCG64(seed))
    T = 3
    names = ("H", "C", "N", "O", "F")
    sizes = qm9_like_sizes(rng, n_mols)
    ptr = _ptr_from_sizes(sizes)
    A = int(ptr[-1])
    element = rng.choice(len(names), size=A,
                         p=[0.51, 0.35, 0.06, 0.07, 0.01]).astype(np.int32)
    std = 1.0 / np.sqrt(1.0 + np.arange(d))
    x = (rng.standard_normal((A, d)) * std).astype(np.float32)
    signs = draw_signs(rng, len(names), T, n_stacks, d)
    bias = draw_bias(rng, len(names), n_stacks * d)
    y = _linear_targets(rng, x, ptr)
    return Problem(name, d, n_stacks, T, sigma, names, x, element, ptr, signs, bias,
                   y=y, lam=lam, seed=seed)


def qm9_batch(n_mols: int = 20000, seed_offset: int = 0) -> Problem:
    """QM9-like forward + Gram: 20k molecules, d=128, 64 stacks (D=8192), sigma=4."""
    return qm9_like(n_mols, 64, SEED_BASE + 2 + seed_offset,
                    "qm9like-20000", sigma=4.0, lam=1e-6)


def precision_batch(n_mols: int = 100000, seed_offset: int = 0) -> Problem:
    """Precision study: 100k QM9-like molecules, d=128, 128 stacks (D=16384)."""
    return qm9_like(n_mols, 128, SEED_BASE + 4 + seed_offset,
                    "qm9like-precision-100000", sigma=4.0, lam=1e-8)


def conformations(n_conf: int = 2000, seed_offset: int = 0, with_J: bool = True) -> Problem:
    """Differentiation: one 21-atom molecule (9 C, 8 H, 4 O) in ``n_conf``
    conformations; x = x0 + N(0, 0.05); Jacobians dx/dr of shape d x 63 per
    atom drawn N(0, 0.1); D = 8192, sigma = 8; alpha ~ N(0, 1)."""
    seed = SEED_BASE + 3 + seed_offset
    rng = np.random.Generator(np.random.PCG64(seed))
    d, S, T = 128, 64, 3
    names = ("H", "C", "O")
    n_at = 21
    sizes = np.full(n_conf, n_at)
    ptr = _ptr_from_sizes(sizes)
    one = np.array([1] * 9 + [0] * 8 + [2] * 4, dtype=np.int32)
    element = np.tile(one, n_conf)
    x0 = rng.standard_normal((n_at, d))
    x = (np.tile(x0, (n_conf, 1)) + 0.05 * rng.standard_normal((n_conf * n_at, d)))
    x = x.astype(np.float32)
    J = J_ptr = None
    if with_J:
        jrng = _jacobian_rng(seed)
        J = (0.1 * jrng.standard_normal(n_conf * n_at * d * 3 * n_at,
                                        dtype=np.float32)).astype(np.float32)
        J_ptr = np.arange(n_conf + 1, dtype=np.int64) * (n_at * d * 3 * n_at)
    signs = draw_signs(rng, len(names), T, S, d)
    bias = draw_bias(rng, len(names), S * d)
    alpha = rng.standard_normal(S * d).astype(np.float32)
    return Problem("conformations-21-atoms", d, S, T, 8.0, names, x, element, ptr,
                   signs, bias, alpha=alpha, J=J, J_ptr=J_ptr, seed=seed)


def with_transforms(p: Problem, T: int) -> Problem:
    """The same workload with N_transform = T: the first T sign diagonals of
    every element and stack (the paper's runs use T = 2; the studies compare
    T = 1, 2, 3 on otherwise identical inputs)."""
    if not 1 <= T <= p.signs.shape[1]:
        raise ValueError(f"T must be in [1, {p.signs.shape[1]}]")
    return dataclasses.replace(p, name=f"{p.name}-T{T}", n_transforms=T,
                               signs=np.ascontiguousarray(p.signs[:, :T]))


@dataclasses.dataclass
class ServingTrace:
    """Arrival trace of energy+force requests plus the resident model.

    Jacobian blocks (N x d x 3N floats each, N(0, 0.1)) are taken from one
    seeded random pool: request r uses the block starting at float offset
    J_off[r]. Their values only feed the force contraction, so a pool of
    bounded size stands in for per-request Jacobians (which would total about
    17 MB per mean request)."""

    model: Problem          # parameters (signs, bias, alpha, sigma)
    arrival_s: np.ndarray   # float64 [R] arrival times in seconds
    sizes: np.ndarray       # int64 [R] atoms per request
    x: np.ndarray           # float32 [sum(sizes), d]
    element: np.ndarray     # int32 [sum(sizes)]
    J_off: np.ndarray       # int64 [R] float offsets into the Jacobian pool
    J_pool_floats: int      # pool size in floats
    J_seed: int             # seed of the pool (device_normal / host_normal)

    def host_J_pool(self) -> np.ndarray:
        return host_normal(self.J_pool_floats, self.J_seed, 0.1)


# Representation vectors ahead of the projection. The FCHL19 representation
# with the energy+force parameters (n2 = 24 two-body bins per element, n3 = 20
# three-body radial bins times the cosine and sine terms per element pair)
# has 5 * 24 + 15 * 20 * 2 = 720 entries for five elements. Synthetic stand-in:
# per element a nonnegative mean plus a rank-256 Gaussian part with a decaying
# spectrum (scale 2^(-j/32) along direction j), so that a few hundred
# directions carry the variance, as in a real representation set.
FCHL19_EF_SIZE = 720


def representation_model(seed: int, n_elements: int, d_rep: int, rank: int = 256):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 2])))
    mu = np.abs(rng.standard_normal((n_elements, d_rep)))
    L = rng.standard_normal((n_elements, d_rep, rank)) / math.sqrt(rank)
    scale = 2.0 ** (-np.arange(rank) / 32.0)
    return mu, L, scale


def host_representations(element: np.ndarray, n_elements: int, d_rep: int, seed: int,
                         rank: int = 256) -> np.ndarray:
    """rho [A, d_rep] float32 for the atoms' elements (host, for tests)."""
    mu, L, scale = representation_model(seed, n_elements, d_rep, rank)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 3])))
    g = rng.standard_normal((len(element), rank)) * scale[None, :]
    rho = np.empty((len(element), d_rep), dtype=np.float64)
    for e in range(n_elements):
        sel = np.nonzero(np.asarray(element) == e)[0]
        rho[sel] = mu[e][None, :] + g[sel] @ L[e].T
    return rho.astype(np.float32)


def device_representations(element, n_elements: int, d_rep: int, seed: int, rank: int = 256,
                           device="cuda"):
    """The same distribution drawn on the device (for the benchmark's sizes)."""
    import torch
    mu, L, scale = representation_model(seed, n_elements, d_rep, rank)
    el = torch.as_tensor(np.asarray(element), device=device)
    g = device_normal(len(element) * rank, seed + 3, 1.0, device).view(len(element), rank)
    g.mul_(torch.as_tensor(scale, dtype=torch.float32, device=device))
    rho = torch.empty((len(element), d_rep), dtype=torch.float32, device=device)
    for e in range(n_elements):
        sel = torch.nonzero(el == e).flatten()
        Le = torch.as_tensor(L[e].T.copy(), dtype=torch.float32, device=device)
        rho[sel] = torch.as_tensor(mu[e], dtype=torch.float32, device=device) + g[sel] @ Le
    return rho


def random_projection(seed: int, n_elements: int, d_rep: int, d: int) -> np.ndarray:
    """U [E, d_rep, d] float32 with orthonormal columns (Q of a Gaussian matrix):
    a stand-in for fitted projections where only their shape matters."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 4])))
    U = np.empty((n_elements, d_rep, d), dtype=np.float32)
    for e in range(n_elements):
        q, _ = np.linalg.qr(rng.standard_normal((d_rep, d)))
        U[e] = q.astype(np.float32)
    return U


# FCHL19 parameters of the energy+force column of the paper's table (n2, n3,
# eta2, eta3, N2, N3, c3, zeta, r_cut in Angstrom), and an element list of
# nuclear charges in the order the representation's bins use.
FCHL19_EF = dict(n2=24, n3=20, eta2=0.32, eta3=2.7, N2=1.8, N3=0.57, c3=13.4,
                 zeta=math.pi, rcut=6.0)
QM9_CHARGES = (1, 6, 7, 8, 9)


def molecule_geometry(rng, n: int, bond=(1.0, 1.6), min_dist=0.95) -> np.ndarray:
    """Coordinates [n, 3] (Angstrom) of a molecule-like cluster: every atom
    after the first sits at a bond length U[1.0, 1.6] from a random earlier
    atom, in a random direction, and no two atoms come closer than 0.95."""
    R = np.zeros((n, 3))
    for a in range(1, n):
        for _ in range(1000):
            base = R[rng.integers(0, a)]
            v = rng.standard_normal(3)
            cand = base + rng.uniform(*bond) * v / np.linalg.norm(v)
            if np.min(np.linalg.norm(R[:a] - cand, axis=1)) >= min_dist:
                R[a] = cand
                break
        else:
            raise RuntimeError("could not place an atom")
    return R


def host_geometries(sizes, seed: int) -> np.ndarray:
    """Concatenated coordinates [sum(sizes), 3] float32 of molecules of the given sizes."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 5])))
    parts = [molecule_geometry(rng, int(n)) for n in sizes]
    return (np.concatenate(parts) if parts else np.zeros((0, 3))).astype(np.float32)


def host_normal(n: int, seed: int, std: float) -> np.ndarray:
    """n float32 draws of N(0, std^2) from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (std * rng.standard_normal(n, dtype=np.float32)).astype(np.float32)


def device_normal(n: int, seed: int, std: float, device="cuda"):
    """n float32 draws of N(0, std^2) generated on the device with a seeded
    torch generator (for large pools that only feed timing runs)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn(n, generator=g, device=device, dtype=torch.float32).mul_(std)


def serving_trace(rate_hz: float = 2000.0, duration_s: float = 20.0, seed_offset: int = 0,
            max_requests: Optional[int] = None, j_pool_floats: int = 1 << 27,
            d: int = 128, n_stacks: int = 128) -> ServingTrace:
    """Serving: Poisson arrivals at ``rate_hz``, sizes round(exp(U[ln 5, ln 300])),
    six elements uniform, x ~ N(0, 1), Jacobians N(0, 0.1) of shape d x 3N per
    atom, D = 16384 (d = 128, 128 stacks), sigma = 4, alpha ~ N(0, 1)."""
    seed = SEED_BASE + 5 + seed_offset
    rng = np.random.Generator(np.random.PCG64(seed))
    S, T = n_stacks, 3
    names = ("H", "C", "N", "O", "F", "S")
    gaps = rng.exponential(1.0 / rate_hz, size=int(rate_hz * duration_s * 1.2) + 16)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    if max_requests is not None:
        t = t[:max_requests]
    R = len(t)
    sizes = np.rint(np.exp(rng.uniform(math.log(5.0), math.log(300.0), size=R))).astype(np.int64)
    A = int(sizes.sum())
    element = rng.integers(0, len(names), size=A).astype(np.int32)
    x = rng.standard_normal((A, d), dtype=np.float32)
    block = sizes * d * 3 * sizes
    pool = max(int(j_pool_floats), int(block.max()) if R else 1)
    J_off = (rng.random(R) * (pool - block + 1)).astype(np.int64) if R else np.zeros(0, np.int64)
    signs = draw_signs(rng, len(names), T, S, d)
    bias = draw_bias(rng, len(names), S * d)
    alpha = rng.standard_normal(S * d).astype(np.float32)
    ptr = _ptr_from_sizes(sizes)
    model = Problem("serving-d16384", d, S, T, 4.0, names, x, element, ptr, signs, bias,
                    alpha=alpha, seed=seed)
    return ServingTrace(model, t, sizes, x, element, J_off, pool,
                        int(np.random.SeedSequence([seed, 1]).generate_state(1)[0]))


def random_problem(seed: int, d: int, n_stacks: int, n_transforms: int = 3,
                   n_elements: int = 3, n_mols: int = 7, max_atoms: int = 12,
                   min_atoms: int = 0, sigma: Optional[float] = None,
                   x_scale: float = 1.0, with_y: bool = True,
                   with_J: bool = False) -> Problem:
    """Small random problem for property and parity tests. Molecule sizes are
    uniform in [min_atoms, max_atoms] (zero-atom molecules allowed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(min_atoms, max_atoms + 1, size=n_mols)
    ptr = _ptr_from_sizes(sizes)
    A = int(ptr[-1])
    element = rng.integers(0, n_elements, size=A).astype(np.int32)
    x = (x_scale * rng.standard_normal((A, d))).astype(np.float32)
    J = J_ptr = None
    if with_J:
        jsz = sizes * d * 3 * sizes
        J_ptr = _ptr_from_sizes(jsz)
        J = (0.1 * _jacobian_rng(seed).standard_normal(int(J_ptr[-1]))).astype(np.float32)
    signs = draw_signs(rng, n_elements, n_transforms, n_stacks, d)
    bias = draw_bias(rng, n_elements, n_stacks * d)
    if sigma is None:
        sigma = float(rng.uniform(0.5, 4.0))
    y = _linear_targets(rng, x, ptr) if with_y else None
    alpha = rng.standard_normal(n_stacks * d).astype(np.float32)
    return Problem(f"random-d{d}-S{n_stacks}-T{n_transforms}", d, n_stacks, n_transforms,
                   sigma, tuple(f"E{i}" for i in range(n_elements)), x, element, ptr,
                   signs, bias, y=y, alpha=alpha, J=J, J_ptr=J_ptr, lam=1e-6, seed=seed)


WORKLOADS = {"small-energy": small_energy_batch, "qm9-like": qm9_batch,
             "conformations": conformations, "precision": precision_batch}
