"""FP64 CPU oracle of the FCHL19 representation and its coordinate gradient.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` legs of ``bench.py`` use it. It shares no code with the HIP
library. Plain PyTorch CPU operations in float64; the coordinate gradient is
PyTorch's reverse-mode differentiation of this forward (a library primitive),
pinned against central differences in the tests.

Paper passages followed (arXiv 2206.01580, Theory section, Representation
subsection, and the parameter table of Computational Details):

* rho_i = [G2_X for every element X] ++ [G3_XY for every element pair X <= Y].
* Two-body: G2 = f_cut(r) r^(-N2) / (R_s sigma(r) sqrt(2 pi)) *
  exp(-(ln R_s - mu(r))^2 / (2 sigma(r)^2)), mu(r) = ln(r / sqrt(1 + eta2 / r^2)),
  sigma(r)^2 = ln(1 + eta2 / r^2): a log-normal density in R_s whose mean is r.
* Cutoff: f_cut(r) = (cos(pi r / r_cut) + 1) / 2.
* Three-body: G3 = xi3 * G3_radial * G3_angular * f_cut(r_ij) f_cut(r_jk) f_cut(r_ik),
  G3_radial = sqrt(eta3 / pi) exp(-eta3 ((r_ij + r_ik) / 2 - R_s)^2),
  xi3 = c3 (1 + 3 cos(theta_kij) cos(theta_ijk) cos(theta_jki)) / (r_ij r_jk r_ki)^N3
  (Axilrod-Teller-Muto), angular Fourier terms of order n = 1 only.

Readings taken where the text is garbled or silent (all listed in the design
notes of the repository):

* The angular vector is [G^cos, G^sin] (printed as [G^cos, G^cos]); G^sin is
  exp(-(zeta n)^2 / 2) (sin(n theta) - sin(n (theta + pi))) (printed with a cos
  in the second term). For n = 1: G^cos = 2 e^(-zeta^2/2) cos(theta_kij),
  G^sin = 2 e^(-zeta^2/2) sin(theta_kij), theta_kij the angle at atom i.
* The ATM denominator is the product of the three distinct sides
  r_ij r_jk r_ki (printed as r_ik r_jk r_ki).
* f_cut is 0 at and beyond r_cut (the cosine formula is used below r_cut only);
  neighbours are the other atoms of the same molecule closer than r_cut to i.
  The three-body cutoff product includes f_cut(r_jk) as printed.
* Two-body grid: n2 centres R_s = r_cut (k + 1) / n2, k = 0 .. n2 - 1 ("linearly
  distributed between 0 and r_cut", excluding 0 where ln R_s is undefined).
  Three-body grid: n3 centres R_s = r_cut k / (n3 - 1), k = 0 .. n3 - 1.
* Each unordered neighbour pair {j, k} of atom i is counted once, in the bin of
  its element pair sorted (X <= Y); pairs (X, Y) are ordered lexicographically
  by element index. Within G3_XY the entries are [radial bin][cos, sin].
* With E elements the representation has E n2 + E (E + 1) / 2 n3 2 entries:
  720 for five elements with the energy+force parameters (n2 = 24, n3 = 20).
"""
from __future__ import annotations

import math

import numpy as np
import torch

__all__ = ["fchl19_size", "pair_index", "fchl19", "fchl19_grad"]


def fchl19_size(n_elements: int, n2: int, n3: int, **_) -> int:
    return n_elements * n2 + n_elements * (n_elements + 1) // 2 * n3 * 2


def pair_index(a: int, b: int, n_elements: int) -> int:
    """Position of the element pair (min, max) in the lexicographic list of pairs X <= Y."""
    a, b = min(a, b), max(a, b)
    return a * n_elements - a * (a - 1) // 2 + (b - a)


def _fcut(r, rcut):
    return torch.where(r < rcut, 0.5 * (torch.cos(math.pi * r / rcut) + 1.0), torch.zeros_like(r))


def _molecule(P, el, n_elements, prm):
    """rho of the atoms of one molecule: P [N, 3] (may require grad), in P's dtype."""
    N = P.shape[0]
    n2, n3 = prm["n2"], prm["n3"]
    rc = prm["rcut"]
    size = fchl19_size(n_elements, n2, n3)
    out = []
    Rs2 = torch.tensor([rc * (k + 1) / n2 for k in range(n2)], dtype=P.dtype)
    Rs3 = torch.tensor([rc * k / (n3 - 1) for k in range(n3)], dtype=P.dtype)
    angw = 2.0 * math.exp(-prm["zeta"] ** 2 / 2.0)
    for i in range(N):
        rho = torch.zeros(size, dtype=P.dtype)
        with torch.no_grad():
            dist = torch.sqrt(torch.sum((P - P[i]) ** 2, dim=1))
        near = [j for j in range(N) if j != i and float(dist[j]) < rc]
        if not near:
            out.append(rho)
            continue
        nb = torch.tensor(near, dtype=torch.long)
        v = P[nb] - P[i]                                  # [n, 3], from i to each neighbour
        r = torch.sqrt(torch.sum(v * v, dim=1))
        eln = torch.tensor([int(el[j]) for j in near], dtype=torch.long)
        # two-body: one log-normal profile per neighbour, in the bins of its element
        q = 1.0 + prm["eta2"] / (r * r)
        mu = torch.log(r / torch.sqrt(q))
        sig2 = torch.log(q)
        dens = torch.exp(-(torch.log(Rs2)[None, :] - mu[:, None]) ** 2 / (2.0 * sig2[:, None])) / (
            Rs2[None, :] * torch.sqrt(sig2)[:, None] * math.sqrt(2.0 * math.pi))
        val = (_fcut(r, rc) * r ** (-prm["N2"]))[:, None] * dens
        idx = eln[:, None] * n2 + torch.arange(n2)[None, :]
        rho = rho.index_add(0, idx.reshape(-1), val.reshape(-1))
        # three-body over unordered neighbour pairs {j, k}
        n = len(near)
        if n >= 2:
            ia, ib = torch.triu_indices(n, n, 1)
            vij, vik = v[ia], v[ib]
            rij, rik = r[ia], r[ib]
            vjk = vik - vij                               # from j to k
            rjk = torch.sqrt(torch.sum(vjk * vjk, dim=1))
            cos_i = torch.sum(vij * vik, dim=1) / (rij * rik)
            cos_j = torch.sum(-vij * vjk, dim=1) / (rij * rjk)
            cos_k = torch.sum(vik * vjk, dim=1) / (rik * rjk)
            xi = prm["c3"] * (1.0 + 3.0 * cos_i * cos_j * cos_k) / (rij * rjk * rik) ** prm["N3"]
            fc = _fcut(rij, rc) * _fcut(rjk, rc) * _fcut(rik, rc)
            rad = math.sqrt(prm["eta3"] / math.pi) * torch.exp(
                -prm["eta3"] * ((rij + rik)[:, None] / 2.0 - Rs3[None, :]) ** 2)
            sin_i = torch.sqrt(torch.clamp(1.0 - cos_i * cos_i,
                                            min=1e-300 if P.dtype == torch.float64
                                            else torch.finfo(P.dtype).tiny))
            w = xi * fc * angw
            vals = torch.stack([rad * (w * cos_i)[:, None], rad * (w * sin_i)[:, None]], dim=2)
            a_el, b_el = eln[ia], eln[ib]
            lo, hi = torch.minimum(a_el, b_el), torch.maximum(a_el, b_el)
            pidx = lo * n_elements - lo * (lo - 1) // 2 + (hi - lo)
            base = n_elements * n2 + pidx * (n3 * 2)
            idx = base[:, None] + torch.arange(2 * n3)[None, :]
            rho = rho.index_add(0, idx.reshape(-1), vals.reshape(-1))
        out.append(rho)
    return torch.stack(out) if out else torch.zeros((0, size), dtype=P.dtype)


def fchl19(R, element, mol_ptr, n_elements: int, prm: dict, requires_grad: bool = False,
           dtype=torch.float64):
    """rho [A, size] (float64 by default) for atoms at R [A, 3] (Angstrom) with element ids
    ``element`` in [0, n_elements), molecules in CSR form ``mol_ptr``.
    Returns (rho, R_tensor) so that a caller can differentiate. ``dtype``
    torch.float32 evaluates the same definition in FP32 arithmetic (the
    rounding floor a test of FP32 code can compare against)."""
    Rt = torch.tensor(np.asarray(R, dtype=np.float64), dtype=dtype, requires_grad=requires_grad)
    el = np.asarray(element)
    ptr = np.asarray(mol_ptr, dtype=np.int64)
    parts = [_molecule(Rt[ptr[m]:ptr[m + 1]], el[ptr[m]:ptr[m + 1]], n_elements, prm)
             for m in range(len(ptr) - 1)]
    size = fchl19_size(n_elements, prm["n2"], prm["n3"])
    rho = torch.cat(parts) if parts else torch.zeros((0, size), dtype=dtype)
    return rho, Rt


def fchl19_grad(R, element, mol_ptr, n_elements: int, prm: dict, g,
                dtype=torch.float64) -> np.ndarray:
    """d(sum_i g_i . rho_i)/dR [A, 3]: the coordinate gradient of an energy
    whose derivative with respect to the representation is g [A, size]
    (float64 arithmetic; ``dtype`` as in fchl19)."""
    rho, Rt = fchl19(R, element, mol_ptr, n_elements, prm, requires_grad=True, dtype=dtype)
    L = torch.sum(rho * torch.tensor(np.asarray(g, dtype=np.float64), dtype=dtype))
    (dR,) = torch.autograd.grad(L, Rt, allow_unused=True)
    return np.zeros(Rt.shape) if dR is None else dR.numpy()
