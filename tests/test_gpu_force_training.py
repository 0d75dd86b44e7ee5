"""GPU parity of the derivative features dZ and of the force-trained normal
equation ((Z, dZ)^T (Z, dZ) + lambda I) alpha = (Z, dZ)^T (E, F).

Tolerances (FP32 kernel vs FP64 oracle):
  dZ  per row (one atomic coordinate): max_f |d dZ| <= 1e-5 * s_row + p_row, with
      s_row = max_f sqrt(2/D) sum_i |(W_{e_i} J_i)[f, col]|, the size of the row's
      terms before the sin weights cancel them, and p_row the first-order effect of
      FP32 phase rounding, sqrt(2/D) sum_i eps (T log2 d + 3) max|u_i| max_f |(W J_i)[f, col]|
      (the reading used for Z, applied to each term of the sum).
  dZ alpha against the forces of sorf_predict: per molecule max |d| <= 1e-5 * max_r
      sum_f |dZ[r, f] alpha_f| (the size of the terms the force sums).
  Force-trained G and Zty (FP32 mode) against FP64 sums of the same FP32 rows:
      ||dG||_F <= 1e-6 ||G||_F.
"""
import math

import numpy as np
import pytest

from oracle import sorf_oracle as O
from paper_2206_01580_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2206_01580_amd import _lib
    _lib.load()  # fails loudly if the HIP library is not built
    yield


def S():
    from paper_2206_01580_amd import sorf
    return sorf


def device_inputs(p):
    s = S()
    return (s.Model.from_problem(p), s.Batch.from_problem(p), torch.from_numpy(p.J).cuda(),
            torch.from_numpy(p.J_ptr).cuda())


def gpu_dz(p):
    model, batch, J, J_ptr = device_inputs(p)
    dZ = S().derivative_features(model, batch, J, J_ptr)
    torch.cuda.synchronize()
    return dZ


def row_bounds(p, mols):
    """s_row and p_row of the module docstring for the rows of ``mols``."""
    D = p.n_features
    eps = 2.0 ** -24
    k = p.n_transforms * math.log2(p.d) + 3
    Ws = [O.dense_w(p.signs[e], p.sigma) for e in range(p.signs.shape[0])]
    s_rows, p_rows = [], []
    for m in mols:
        a0, a1 = int(p.mol_ptr[m]), int(p.mol_ptr[m + 1])
        n = a1 - a0
        if n == 0:
            continue
        blk = p.J[p.J_ptr[m]:p.J_ptr[m] + n * p.d * 3 * n].astype(np.float64).reshape(n, p.d, 3 * n)
        umax = np.abs(O.phases(p.x, p.element, p.signs, p.bias, p.sigma,
                               np.arange(a0, a1))).max(axis=1)
        tot = np.zeros((D, 3 * n))
        pb = np.zeros(3 * n)
        for i in range(n):
            WJ = np.abs(Ws[p.element[a0 + i]] @ blk[i])
            tot += WJ
            pb += eps * k * umax[i] * WJ.max(axis=0)
        s_rows.append(math.sqrt(2.0 / D) * tot.max(axis=0))
        p_rows.append(math.sqrt(2.0 / D) * pb)
    if not s_rows:
        return np.zeros(0), np.zeros(0)
    return np.concatenate(s_rows), np.concatenate(p_rows)


def check_dz(dz_gpu, p, mols=None):
    mols = np.arange(p.n_mols) if mols is None else np.asarray(mols)
    ref = O.derivative_features(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, p.J,
                                p.J_ptr, mols=mols)
    s_row, p_row = row_bounds(p, mols)
    got = np.asarray(dz_gpu, dtype=np.float64)
    assert got.shape == ref.shape
    err = np.abs(got - ref).max(axis=1) if len(ref) else np.zeros(0)
    allow = 1e-5 * s_row + p_row
    assert np.all(err <= allow), float(np.max(err / np.maximum(s_row, 1e-30)))
    return float(np.max(err / np.maximum(s_row, 1e-30))) if len(err) else 0.0


def rows_of(p, mols):
    return np.concatenate([np.arange(3 * p.mol_ptr[m], 3 * p.mol_ptr[m + 1]) for m in mols])


# (d, S, T, elements, molecules, min atoms, max atoms): every lane layout (d = 2 has
# 2 entries per lane, d >= 32 has 32), empty molecules, column groups that end
# inside a wave, and at d = 1024 molecules longer than one atom chunk (8 atoms)
@pytest.mark.parametrize("shape", [(2, 5, 3, 2, 6, 0, 5), (8, 3, 3, 2, 7, 0, 9),
                                   (32, 3, 2, 3, 5, 1, 12), (64, 4, 3, 3, 6, 0, 20),
                                   (128, 4, 3, 4, 7, 0, 29), (256, 3, 3, 2, 4, 1, 9),
                                   (1024, 2, 1, 2, 3, 1, 12)],
                         ids=lambda s: "d{}-S{}-T{}".format(*s[:3]))
def test_dz_random_shapes(shape):
    d, S_, T, E, M, lo, hi = shape
    p = W.random_problem(3000 + d + S_, d, S_, T, E, M, hi, lo, with_J=True)
    rel = check_dz(gpu_dz(p).cpu().numpy(), p)
    print(f"{p.name}: max row error / row scale {rel:.2e}")


def test_dz_molecules_longer_than_an_atom_chunk():
    """d = 128 keeps sin(u) of 64 atoms in LDS: 65..150 atoms take the chunked
    path, where the column groups of the four waves advance in lockstep."""
    p = W.random_problem(3101, 128, 2, 3, 3, 3, 150, 65, with_J=True)
    assert p.mol_sizes().min() > 64
    check_dz(gpu_dz(p).cpu().numpy(), p)


def test_dz_no_atoms_and_empty_molecules():
    p = W.random_problem(3102, 16, 2, 3, 2, 4, 0, 0, with_J=True)
    assert p.n_atoms == 0
    model, batch, J, J_ptr = device_inputs(p)
    out = torch.empty((0, p.n_features), dtype=torch.float32, device="cuda")
    S().derivative_features(model, batch, J, J_ptr, out)
    torch.cuda.synchronize()


def test_dz_rows_do_not_depend_on_the_batch():
    p = W.random_problem(3103, 64, 3, 3, 3, 9, 14, 0, with_J=True)
    full = gpu_dz(p).cpu().numpy()
    mols = [7, 2, 5]
    sub = p.subset(mols)
    part = gpu_dz(sub).cpu().numpy()
    assert np.array_equal(part, full[rows_of(p, mols)])


def test_dz_alpha_equals_predicted_forces():
    p = W.random_problem(3104, 128, 8, 3, 4, 12, 25, 1, with_J=True)
    model, batch, J, J_ptr = device_inputs(p)
    alpha = torch.from_numpy(p.alpha).cuda()
    dZ = S().derivative_features(model, batch, J, J_ptr)
    E, F = S().predict(model, batch, alpha, J, J_ptr)
    torch.cuda.synchronize()
    dz = dZ.double().cpu().numpy()
    a64 = p.alpha.astype(np.float64)
    Fd = dz @ a64
    scale = np.abs(dz) @ np.abs(a64)
    Fp = F.double().cpu().numpy()
    for m in range(p.n_mols):
        r = slice(3 * p.mol_ptr[m], 3 * p.mol_ptr[m + 1])
        if r.start == r.stop:
            continue
        assert np.abs(Fd[r] - Fp[r]).max() <= 1e-5 * scale[r].max()


def test_dz_conformations_sampled_molecules():
    """The full differentiation workload (2,000 conformations of a 21-atom
    molecule, D = 8192: dZ is 126,000 x 8192) in the launch configuration the
    benchmark times; sampled conformations against the oracle."""
    p = W.conformations()
    dZ = gpu_dz(p)
    mols = [0, 1, 997, 1998, 1999]
    rows = torch.from_numpy(rows_of(p, mols)).cuda()
    got = dZ.index_select(0, rows).cpu().numpy()
    rel = check_dz(got, p, mols)
    print(f"conformations dZ: max row error / row scale {rel:.2e}")
    # dZ alpha against the forces of the predict path on every conformation
    model, batch, J, J_ptr = device_inputs(p)
    alpha = torch.from_numpy(p.alpha).cuda()
    _, F = S().predict(model, batch, alpha, J, J_ptr)
    a64 = alpha.double()
    Fd = (dZ.double() @ a64).view(p.n_mols, -1)
    scale = (dZ.double().abs() @ a64.abs()).view(p.n_mols, -1).amax(dim=1)
    Fp = F.double().view(p.n_mols, -1)
    err = (Fd - Fp).abs().amax(dim=1)
    assert bool((err <= 1e-5 * scale).all()), float((err / scale).max())


def test_force_trained_normal_equations_fp32():
    """G = Z^T Z + dZ^T dZ and Zty = Z^T E + dZ^T F by two accumulations into
    the same buffers, then the FP64 solve: against FP64 sums of the same FP32
    rows, and the solution against the oracle's solve of that system."""
    p = W.random_problem(3105, 32, 4, 3, 3, 40, 8, 2, with_J=True)
    model, batch, J, J_ptr = device_inputs(p)
    s = S()
    Z = s.forward(model, batch)
    dZ = s.derivative_features(model, batch, J, J_ptr)
    rng = np.random.default_rng(5)
    E = torch.from_numpy(rng.standard_normal(p.n_mols).astype(np.float32)).cuda()
    F = torch.from_numpy(rng.standard_normal(3 * p.n_atoms).astype(np.float32)).cuda()
    D = p.n_features
    G = torch.zeros((D, D), dtype=torch.float32, device="cuda")
    r = torch.zeros(D, dtype=torch.float32, device="cuda")
    s.gram_accumulate(Z, G, E, r, precision="fp32")
    s.gram_accumulate(dZ, G, F, r, precision="fp32")
    lam = 1e-4
    alpha, info = s.solve(G, r, lam, n_refine=3)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Gr, rr = O.force_normal_equations(Z.cpu().numpy(), dZ.cpu().numpy(), E.cpu().numpy(),
                                      F.cpu().numpy())
    Gg = np.tril(G.double().cpu().numpy())
    assert np.linalg.norm(Gg - np.tril(Gr)) <= 1e-6 * np.linalg.norm(np.tril(Gr))
    assert np.abs(r.double().cpu().numpy() - rr).max() <= 1e-6 * np.abs(rr).max()
    Gs = Gg + np.tril(Gg, -1).T
    ref = O.solve(Gs, r.double().cpu().numpy(), lam)
    a = alpha.cpu().numpy()
    assert np.abs(a - ref).max() <= 1e-8 * np.abs(ref).max()
