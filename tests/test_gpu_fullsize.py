"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times, on outputs the oracle can afford one by one.

* QM9-like training set (20,000 molecules, D = 8192): Z rows of 200 sampled
  molecules; energies Z alpha of 64 sampled molecules; G and Z^T y on a 48-column sample (every Gram mode) against the
  FP64 oracle's columns of Z; the ridge solve through its residual.
* Differentiation set (2000 conformations of a 21-atom molecule, D = 8192,
  1.36 GB of Jacobians): energies, dE/dx and forces of 8 sampled conformations.

Gram bound per entry (i, j): |dG_ij| <= (2 u + 1e-5) sum_m |Z_mi Z_mj|, with u
the unit roundoff of the operand format (each product of rounded operands is
within (2u + u^2) of the exact one; 1e-5 covers the FP32 features and the
FP32 sums): u = 0 for FP32, 2^-9 bf16, 2^-12 fp16, 2^-17 bf16 hi+lo,
2^-23 fp16 hi+lo.
"""
import math

import numpy as np
import pytest

from oracle import sorf_oracle as O
from paper_2206_01580_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

UNIT = {"fp32": 0.0, "fp32_kahan": 0.0, "bf16": 2.0 ** -9, "fp16": 2.0 ** -12, "bf16_hilo": 2.0 ** -17,
        "fp16_hilo": 2.0 ** -23}


def S():
    from paper_2206_01580_amd import sorf
    return sorf


@pytest.fixture(scope="module")
def qm9():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    p = W.qm9_batch()
    s = S()
    model, batch = s.Model.from_problem(p), s.Batch.from_problem(p)
    Z = s.forward(model, batch)
    torch.cuda.synchronize()
    D = p.n_features
    rng = np.random.default_rng(11)
    cols = np.unique(np.concatenate([[0, 1, 127, 128, 255, 256, 4095, 4096, D - 129, D - 128,
                                      D - 1], rng.choice(D, 37, replace=False)]))
    Zc = O.molecule_features(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, cols=cols,
                             chunk_atoms=1 << 20)
    return p, Z, cols, Zc


def test_qm9_forward_sampled_rows(qm9):
    p, Z, _, _ = qm9
    rng = np.random.default_rng(12)
    sizes = p.mol_sizes()
    mols = np.unique(np.concatenate([[0, p.n_mols - 1, int(np.argmax(sizes)), int(np.argmin(sizes))],
                                     rng.choice(p.n_mols, 196, replace=False)]))
    Zo = O.molecule_features(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, mols=mols)
    Zg = Z[torch.from_numpy(mols).cuda()].cpu().numpy().astype(np.float64)
    err = np.abs(Zg - Zo).max(axis=1) / np.abs(Zo).max(axis=1)
    assert err.max() <= 1e-5, err.max()


def test_qm9_energies_sampled(qm9):
    """Energies without forces over the whole training set (the launch the
    benchmark's energy phase times), sampled molecules against Z_oracle alpha."""
    p, _, _, _ = qm9
    s = S()
    model, batch = s.Model.from_problem(p), s.Batch.from_problem(p)
    rng = np.random.default_rng(13)
    alpha = rng.standard_normal(p.n_features).astype(np.float32)
    E = s.Predictor(model)(batch, torch.from_numpy(alpha).cuda())
    torch.cuda.synchronize()
    sizes = p.mol_sizes()
    mols = np.unique(np.concatenate([[0, p.n_mols - 1, int(np.argmax(sizes))],
                                     rng.choice(p.n_mols, 61, replace=False)]))
    Zo = O.molecule_features(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, mols=mols)
    Eo = Zo @ alpha.astype(np.float64)
    scale = np.abs(Zo * alpha[None, :]).sum(axis=1)
    err = np.abs(E.cpu().numpy()[mols].astype(np.float64) - Eo) / scale
    assert err.max() <= 1e-5, err.max()


def test_qm9_energy_grad_sampled(qm9):
    """Energies and dE/dx in one pass over the whole training set (the launch
    the benchmark's energy + gradient phase times): sampled molecules'
    energies and their atoms' gradient rows against the oracle."""
    p, _, _, _ = qm9
    s = S()
    model, batch = s.Model.from_problem(p), s.Batch.from_problem(p)
    rng = np.random.default_rng(14)
    alpha = rng.standard_normal(p.n_features).astype(np.float32)
    E, g = s.EnergyGrad(model)(batch, torch.from_numpy(alpha).cuda())
    torch.cuda.synchronize()
    E, g = E.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    sizes = p.mol_sizes()
    mols = np.unique(np.concatenate([[0, p.n_mols - 1, int(np.argmax(sizes))],
                                     rng.choice(p.n_mols, 29, replace=False)]))
    Zo = O.molecule_features(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, mols=mols)
    Eo = Zo @ alpha.astype(np.float64)
    scale = np.abs(Zo * alpha[None, :]).sum(axis=1)
    assert (np.abs(E[mols] - Eo) / scale).max() <= 1e-5
    # the sampled molecules' atoms as one small batch for the oracle
    atoms = np.concatenate([np.arange(p.mol_ptr[m], p.mol_ptr[m + 1]) for m in mols])
    ptr = np.concatenate([[0], np.cumsum(sizes[mols])]).astype(np.int64)
    go = O.grad_x(p.x[atoms], p.element[atoms], ptr, p.signs, p.bias, p.sigma, alpha)
    err = np.abs(g[atoms] - go).max(axis=1) / np.abs(go).max(axis=1)
    assert err.max() <= 1e-5, err.max()


def test_qm9_feature_columns(qm9):
    p, Z, cols, Zc = qm9
    Zg = Z[:, torch.from_numpy(cols).cuda()].cpu().numpy().astype(np.float64)
    row_scale = np.abs(Zc).max(axis=1, keepdims=True)
    # same normwise reading as the row test, with the sampled columns' own scale
    assert (np.abs(Zg - Zc) / row_scale).max() <= 1e-5


@pytest.mark.parametrize("mode", ["fp32", "fp32_kahan", "bf16", "fp16", "bf16_hilo", "fp16_hilo"])
def test_qm9_gram_sampled(qm9, mode):
    p, Z, cols, Zc = qm9
    s = S()
    D = p.n_features
    y = torch.from_numpy(p.y).cuda()
    G = torch.zeros(D, D, device="cuda")
    Zty = torch.zeros(D, device="cuda")
    k = s.fp16_scale_exp(29 * math.sqrt(2.0 / D)) if mode.startswith("fp16") else 0
    s.gram_accumulate(Z, G, y, Zty, precision=mode, scale_exp=k)
    torch.cuda.synchronize()
    ci = torch.from_numpy(cols).cuda()
    Gs = G[ci][:, ci].cpu().numpy().astype(np.float64)
    Go = Zc.T @ Zc
    bound = (2 * UNIT[mode] + 1e-5) * (np.abs(Zc).T @ np.abs(Zc))
    low = np.tril_indices(len(cols))
    assert np.all(np.abs(Gs - Go)[low] <= bound[low]), float(np.max((np.abs(Gs - Go) / bound)[low]))
    ro = Zc.T @ p.y.astype(np.float64)
    rb = 1e-5 * (np.abs(Zc).T @ np.abs(p.y.astype(np.float64)))
    assert np.all(np.abs(Zty[ci].cpu().numpy() - ro) <= rb)
    # the strict upper triangle is never written
    assert float(torch.triu(G, 1).abs().max()) == 0.0


def test_qm9_solve_residual():
    """Full-size ridge solve (D = 8192, lambda = 1e-6, 3 refinements) on the
    bf16 hi+lo Gram: the FP64 residual of the system it was given is small."""
    p = W.qm9_batch()
    s = S()
    model, batch = s.Model.from_problem(p), s.Batch.from_problem(p)
    Z = s.forward(model, batch)
    D = p.n_features
    G = torch.zeros(D, D, device="cuda")
    Zty = torch.zeros(D, device="cuda")
    s.gram_accumulate(Z, G, torch.from_numpy(p.y).cuda(), Zty, precision="bf16_hilo")
    solver = s.Solver(D, device="cuda")
    alpha = solver(G, Zty, 1e-6, 3)
    torch.cuda.synchronize()
    assert int(solver.info.item()) == 0
    A = torch.tril(G).double()
    A = A + A.T - torch.diag(torch.diag(A)) + 1e-6 * torch.eye(D, dtype=torch.float64, device="cuda")
    r = A @ alpha - Zty.double()
    # backward-error form: ||r|| <= c eps_64 (||A|| ||alpha|| + ||b||)
    scale = torch.linalg.norm(A) * torch.linalg.norm(alpha) + torch.linalg.norm(Zty.double())
    assert float(torch.linalg.norm(r) / scale) <= 1e-12


def test_differentiation_set_sampled_conformations():
    p = W.conformations()
    s = S()
    model, batch = s.Model.from_problem(p), s.Batch.from_problem(p)
    alpha = torch.from_numpy(p.alpha).cuda()
    J = torch.from_numpy(p.J).cuda()
    J_ptr = torch.from_numpy(p.J_ptr).cuda()
    E, F = s.predict(model, batch, alpha, J, J_ptr)
    grad = s.backward(model, batch, alpha)
    torch.cuda.synchronize()
    rng = np.random.default_rng(13)
    mols = np.unique(np.concatenate([[0, p.n_mols - 1], rng.choice(p.n_mols, 6, replace=False)]))
    q = p.subset(mols)
    Zo = O.molecule_features(q.x, q.element, q.mol_ptr, q.signs, q.bias, q.sigma)
    a64 = p.alpha.astype(np.float64)
    Eo = Zo @ a64
    Es = E.cpu().numpy()[mols]
    assert np.all(np.abs(Es - Eo) <= 1e-5 * np.abs(Zo * a64[None, :]).sum(axis=1))
    go = O.grad_x(q.x, q.element, q.mol_ptr, q.signs, q.bias, q.sigma, p.alpha)
    Fo = O.forces(go, q.J, q.J_ptr, q.mol_ptr)
    gg = grad.cpu().numpy()
    Fg = F.cpu().numpy()
    for r, m in enumerate(mols):
        a0, a1 = int(p.mol_ptr[m]), int(p.mol_ptr[m + 1])
        b0, b1 = int(q.mol_ptr[r]), int(q.mol_ptr[r + 1])
        ga, gb = gg[a0:a1].astype(np.float64), go[b0:b1]
        assert np.all(np.abs(ga - gb).max(axis=1) <= 1e-5 * np.abs(gb).max(axis=1))
        fa, fb = Fg[3 * a0:3 * a1], Fo[3 * b0:3 * b1]
        assert np.abs(fa - fb).max() <= 1e-5 * np.abs(fb).max()
