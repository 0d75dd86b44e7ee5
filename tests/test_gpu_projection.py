"""GPU parity of the per-element projection x_i = rho_i^T U_{e_i}.

Tolerance (FP32 matrix-core sums vs the FP64 oracle): per entry
  |dx_ij| <= (d_rep 2^-24 + 2^-24) sum_k |rho_ik U_{e_i},kj|,
the worst-case bound of a length-d_rep FP32 dot product (products and sums
rounded once each). Features computed from the projected x are held to the
feature tolerance of the other tests (row max 1e-5 plus the phase bound).
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


def check_projection(x_gpu, rho, element, U, rows=None):
    rows = np.arange(len(element)) if rows is None else np.asarray(rows)
    ref = O.project(rho[rows], element[rows], U)
    mag = O.project(np.abs(rho[rows]), element[rows], np.abs(U))
    d_rep = rho.shape[1]
    allow = (d_rep + 1) * 2.0 ** -24 * mag
    err = np.abs(np.asarray(x_gpu, np.float64) - ref)
    assert np.all(err <= allow), float(np.max(err / np.maximum(mag, 1e-30)))
    return float(np.max(err / np.maximum(mag, 1e-30)))


def run(rho, element, U, out=None):
    x = S().project(torch.from_numpy(rho).cuda(), torch.from_numpy(element).cuda(),
                    torch.from_numpy(U).cuda(), out)
    torch.cuda.synchronize()
    return x


# (atoms, d_rep, d, elements): the FCHL19 size with d = 128 and 256, an odd
# d_rep (scalar loads), a d that is not a multiple of 128 (ragged column
# tile) and small sizes with tiles that are mostly empty
@pytest.mark.parametrize("shape", [(1000, 720, 128, 5), (777, 775, 256, 4), (300, 40, 8, 3),
                                   (3000, 33, 130, 2), (5, 720, 128, 5), (1, 16, 2, 1)],
                         ids=lambda s: "A{}-drep{}-d{}-E{}".format(*s))
def test_project_random_shapes(shape):
    A, d_rep, d, E = shape
    rng = np.random.default_rng(A + d_rep + d)
    element = rng.integers(0, E, size=A).astype(np.int32)
    rho = W.host_representations(element, E, d_rep, seed=A + d)
    U = rng.standard_normal((E, d_rep, d)).astype(np.float32) / math.sqrt(d_rep)
    x = run(rho, element, U)
    rel = check_projection(x.cpu().numpy(), rho, element, U)
    print(f"A={A} d_rep={d_rep} d={d}: max error / bound scale {rel:.2e}")


def test_project_unaligned_rows_take_the_scalar_path():
    rng = np.random.default_rng(3)
    A, d_rep, d, E = 400, 720, 128, 3
    element = rng.integers(0, E, size=A).astype(np.int32)
    rho = W.host_representations(element, E, d_rep, seed=4)
    U = W.random_projection(5, E, d_rep, d)
    buf = torch.empty(A * d_rep + 1, dtype=torch.float32, device="cuda")
    view = buf[1:].view(A, d_rep)               # 4-byte offset: not 16-byte aligned
    view.copy_(torch.from_numpy(rho))
    x = S().project(view, torch.from_numpy(element).cuda(), torch.from_numpy(U).cuda())
    torch.cuda.synchronize()
    check_projection(x.cpu().numpy(), rho, element, U)


def test_project_skips_invalid_elements_and_empty_batches():
    rng = np.random.default_rng(6)
    A, d_rep, d, E = 200, 64, 32, 2
    element = rng.integers(0, E, size=A).astype(np.int32)
    element[[3, 50, 199]] = [-1, 2, 7]
    rho = rng.standard_normal((A, d_rep)).astype(np.float32)
    U = rng.standard_normal((E, d_rep, d)).astype(np.float32)
    out = torch.full((A, d), 123.0, dtype=torch.float32, device="cuda")
    x = run(rho, element, U, out).cpu().numpy()
    bad = np.array([3, 50, 199])
    assert np.all(x[bad] == 123.0)
    good = np.setdiff1d(np.arange(A), bad)
    check_projection(x[good], rho, element, U, rows=good)
    # no atoms: nothing to do
    empty = torch.empty((0, d), dtype=torch.float32, device="cuda")
    S().project(torch.empty((0, d_rep), device="cuda"), torch.empty(0, dtype=torch.int32,
                device="cuda"), torch.from_numpy(U).cuda(), empty)
    torch.cuda.synchronize()


def test_project_deterministic():
    rng = np.random.default_rng(7)
    A, d_rep, d, E = 5000, 720, 128, 5
    element = rng.integers(0, E, size=A).astype(np.int32)
    rho = W.host_representations(element, E, d_rep, seed=8)
    U = W.random_projection(9, E, d_rep, d)
    a = run(rho, element, U).cpu().numpy()
    b = run(rho, element, U).cpu().numpy()
    assert np.array_equal(a, b)


def test_projected_features_match_the_oracle():
    """rho -> x (sorf_project) -> Z (sorf_forward) against the oracle's
    project -> molecule_features on a small QM9-like batch."""
    p = W.qm9_batch(n_mols=40)
    d_rep = W.FCHL19_EF_SIZE
    rho = W.host_representations(p.element, p.n_elements, d_rep, seed=10)
    U = W.random_projection(11, p.n_elements, d_rep, p.d)
    s = S()
    x = s.project(torch.from_numpy(rho).cuda(), torch.from_numpy(p.element).cuda(),
                  torch.from_numpy(U).cuda())
    model = s.Model.from_problem(p)
    batch = s.Batch(x, torch.from_numpy(p.element).cuda(), torch.from_numpy(p.mol_ptr).cuda())
    Z = s.forward(model, batch)
    torch.cuda.synchronize()
    x_ora = O.project(rho, p.element, U)
    Zo = O.molecule_features(x_ora, p.element, p.mol_ptr, p.signs, p.bias, p.sigma)
    scale = np.abs(Zo).max(axis=1)
    err = np.abs(Z.double().cpu().numpy() - Zo).max(axis=1)
    assert np.all(err <= 1e-5 * scale), float(np.max(err / scale))


def test_project_qm9_like_full_size_sampled_rows():
    """The benchmark's projection: every atom of the 20,000-molecule QM9-like
    batch (360,149 atoms, d_rep = 720 -> d = 128), sampled rows against the oracle."""
    p = W.qm9_batch()
    d_rep = W.FCHL19_EF_SIZE
    el = torch.from_numpy(p.element).cuda()
    rho = W.device_representations(p.element, p.n_elements, d_rep, seed=12)
    U = W.random_projection(13, p.n_elements, d_rep, p.d)
    x = S().project(rho, el, torch.from_numpy(U).cuda())
    torch.cuda.synchronize()
    rows = np.random.default_rng(14).choice(p.n_atoms, size=2000, replace=False)
    idx = torch.from_numpy(rows).cuda()
    rho_s = rho.index_select(0, idx).cpu().numpy()
    got = x.index_select(0, idx).cpu().numpy()
    ref = O.project(rho_s, p.element[rows], U)
    mag = O.project(np.abs(rho_s), p.element[rows], np.abs(U))
    assert np.all(np.abs(got - ref) <= (d_rep + 1) * 2.0 ** -24 * mag)


# ------------------------------------------------------------------ the fit
# Tolerances. Column r of U may differ from the oracle's by
#   1e-6 + 2 d_rep eps64 lambda_max / gap_r
# per entry: 1e-6 for the FP32 output, and the Davis-Kahan bound for a
# backward error d_rep eps64 ||G|| in each of the two FP64 routes (SVD of the
# sample, Jacobi on its Gram), gap_r being the distance from lambda_r = s_r^2
# to the nearest other eigenvalue. Squared singular values: within 1e-12 of
# the largest one.
def column_tolerance(s_all, n_pca, d_rep):
    lam = np.asarray(s_all, np.float64) ** 2
    gap = np.full(n_pca, np.inf)
    for r in range(n_pca):
        if r > 0:
            gap[r] = min(gap[r], lam[r - 1] - lam[r])
        if r + 1 < len(lam):
            gap[r] = min(gap[r], lam[r] - lam[r + 1])
    return 1e-6 + 2 * d_rep * 2.0 ** -52 * lam[0] / gap


def full_spectrum(sample):
    return np.linalg.svd(np.asarray(sample, np.float64), compute_uv=False)
@pytest.mark.parametrize("shape", [(2000, 720, 128), (1500, 775, 256), (300, 33, 8)],
                         ids=lambda s: "n{}-drep{}-npca{}".format(*s))
def test_projection_fit_matches_oracle(shape):
    n, d_rep, n_pca = shape
    element = np.zeros(n, dtype=np.int32)
    sample = W.host_representations(element, 1, d_rep, seed=n + d_rep)
    U, sv = S().projection_fit(torch.from_numpy(sample).cuda(), n_pca)
    torch.cuda.synchronize()
    Uo, so = O.projection_fit(sample, n_pca)
    tol = column_tolerance(full_spectrum(sample), n_pca, d_rep)
    diff = np.abs(U.double().cpu().numpy() - Uo).max(axis=0)
    assert np.all(diff <= tol), float(np.max(diff / tol))
    err = diff.max()
    s2 = sv.cpu().numpy() ** 2
    assert np.abs(s2 - so ** 2).max() <= 1e-12 * so[0] ** 2
    print(f"n={n} d_rep={d_rep} n_pca={n_pca}: max |dU| {err:.2e}")


def test_projection_fit_recovers_a_planted_subspace():
    rng = np.random.default_rng(21)
    B, _ = np.linalg.qr(rng.standard_normal((32, 8)))
    g = rng.standard_normal((500, 8)) * np.linspace(3.0, 1.0, 8)[None, :]
    sample = (g @ B.T).astype(np.float32)
    U, sv = S().projection_fit(torch.from_numpy(sample).cuda(), 8)
    torch.cuda.synchronize()
    U = U.double().cpu().numpy()
    assert np.abs(U @ U.T - B @ B.T).max() < 1e-6
    assert np.abs(U.T @ U - np.eye(8)).max() < 1e-6


def test_fitted_projection_feeds_the_projection():
    """Fit per element on a sample of a QM9-like batch, project every atom, and
    compare with the oracle's fit + projection."""
    p = W.qm9_batch(n_mols=2000)      # at least d atoms of every element, fluorine included
    d_rep = W.FCHL19_EF_SIZE
    assert np.bincount(p.element).min() >= p.d
    rho = W.host_representations(p.element, p.n_elements, d_rep, seed=22)
    s = S()
    Ug = torch.empty((p.n_elements, d_rep, p.d), dtype=torch.float32, device="cuda")
    Uo = np.empty((p.n_elements, d_rep, p.d))
    rng = np.random.default_rng(23)
    tol = np.empty((p.n_elements, p.d))
    for e in range(p.n_elements):
        rows = np.nonzero(p.element == e)[0]
        rows = rng.choice(rows, size=min(len(rows), 1000), replace=False)
        s.projection_fit(torch.from_numpy(rho[rows]).cuda(), p.d, out=Ug[e])
        Uo[e] = O.projection_fit(rho[rows], p.d)[0]
        tol[e] = column_tolerance(full_spectrum(rho[rows]), p.d, d_rep)
    x = s.project(torch.from_numpy(rho).cuda(), torch.from_numpy(p.element).cuda(), Ug)
    torch.cuda.synchronize()
    dU = np.abs(Ug.double().cpu().numpy() - Uo).max(axis=1)
    assert np.all(dU <= tol)
    xo = O.project(rho, p.element, Uo)
    mag = O.project(np.abs(rho), p.element, np.abs(Uo))
    # the fitted U differs from the oracle's by <= tol per column: add that to the bound
    allow = (d_rep + 1) * 2.0 ** -24 * mag + np.abs(rho).sum(axis=1, keepdims=True) * tol[p.element]
    assert np.all(np.abs(x.double().cpu().numpy() - xo) <= allow)
