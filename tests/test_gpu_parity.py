"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (FP32 kernels vs FP64 oracle):
  Z      per molecule row, max_f |dZ| <= 1e-5 * max_f |Z_ora| (rows of empty molecules exactly 0)
  grad   per atom, max_j |dg| <= 1e-5 * max_j |g_ora|
  E      |dE_m| <= 1e-5 * sum_f |alpha_f Z_ora[m, f]|
  F      per molecule, max |dF| <= 1e-5 * max |F_ora|
  G      ||dG||_F / ||G||_F <= 1e-6 against the oracle's emulation of the same precision mode
The normwise reading of the feature tolerance: FP32 cos near its zeros makes
elementwise relative error meaningless, while the row max sets the scale the
features are used at.
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


def dev_problem(p):
    s = S()
    return s.Model.from_problem(p), s.Batch.from_problem(p)


def check_rows(Zg, Zo, tol=1e-5, abs_bound=None):
    Zg = np.asarray(Zg, dtype=np.float64)
    scale = np.abs(Zo).max(axis=1)
    err = np.abs(Zg - Zo).max(axis=1) if Zo.shape[1] else np.zeros(len(Zo))
    empty = scale == 0
    assert np.all(Zg[empty] == 0.0)
    allow = tol * scale
    if abs_bound is not None:
        allow = np.maximum(allow, abs_bound)
    bad = err[~empty] > allow[~empty]
    assert not bad.any(), f"max rel row err {np.max(err[~empty] / scale[~empty]):.3e}"
    return float(np.max(err[~empty] / scale[~empty])) if (~empty).any() else 0.0


def phase_bound(p):
    """First-order FP32 error bound of a Z row when phases are large: each
    phase u = c v + b is formed with T log2(d) rounded butterfly stages plus
    the scale and the bias, so |du| <= eps (T log2 d + 3) |u| per entry, and
    the row sums sqrt(2/D) |du| over the molecule's atoms."""
    eps = 2.0 ** -24
    u = O.phases(p.x, p.element, p.signs, p.bias, p.sigma)
    per_atom = np.abs(u).max(axis=1) if u.size else np.zeros(0)
    k = p.n_transforms * math.log2(p.d) + 3
    out = np.zeros(p.n_mols)
    for m in range(p.n_mols):
        out[m] = eps * k * math.sqrt(2.0 / p.n_features) * per_atom[p.mol_ptr[m]:p.mol_ptr[m + 1]].sum()
    return out


def gpu_forward(p):
    model, batch = dev_problem(p)
    Z = S().forward(model, batch)
    torch.cuda.synchronize()
    return Z.cpu().numpy()


def oracle_forward(p, mols=None):
    return O.molecule_features(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, mols)


# ------------------------------------------------------------------ forward
def test_forward_small_energy_batch():
    p = W.small_energy_batch()
    rel = check_rows(gpu_forward(p), oracle_forward(p))
    print(f"small energy batch: forward max normwise row error {rel:.2e}")


SHAPES = [  # (d, n_stacks, T, n_elements, n_mols, min_atoms, max_atoms)
    (2, 3, 1, 2, 9, 0, 5), (4, 5, 2, 3, 11, 0, 7), (8, 7, 3, 2, 6, 1, 9), (16, 3, 3, 4, 13, 0, 6),
    (32, 9, 2, 3, 7, 0, 8), (64, 4, 3, 4, 10, 1, 12), (64, 33, 1, 2, 5, 0, 9),
    (128, 16, 3, 5, 9, 0, 14), (128, 21, 2, 3, 6, 1, 30), (256, 6, 3, 3, 5, 0, 9),
    (512, 3, 3, 2, 4, 1, 5), (1024, 2, 2, 2, 3, 1, 4),
    # stack counts that are multiples of the lane groups per wave (32 at d = 64,
    # 8 at d = 256): the wave-shared x-row form of the forward kernel
    (64, 32, 3, 3, 4, 0, 11), (256, 8, 3, 3, 5, 0, 10),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "d{}-S{}-T{}-E{}-M{}".format(*s[:5]))
def test_forward_random_shapes(shape):
    d, S_, T, E, M, lo, hi = shape
    p = W.random_problem(1000 + d + S_ + T, d, S_, T, E, M, hi, lo)
    check_rows(gpu_forward(p), oracle_forward(p), abs_bound=phase_bound(p))


def test_forward_all_empty_and_no_molecules():
    p = W.random_problem(5, 64, 2, 3, 2, 4, 0, 0)
    assert p.n_atoms == 0
    Z = gpu_forward(p)
    assert Z.shape == (4, 128) and np.all(Z == 0.0)
    q = p.subset([])
    assert gpu_forward(q).shape == (0, 128)


def test_forward_large_phases():
    # big |x| / small sigma: phases of many revolutions
    p = W.random_problem(77, 128, 4, 3, 3, 5, 6, 1, sigma=0.05, x_scale=3.0)
    check_rows(gpu_forward(p), oracle_forward(p), abs_bound=phase_bound(p))


def test_forward_deterministic():
    p = W.random_problem(8, 128, 8, 3, 3, 20, 12, 1)
    model, batch = dev_problem(p)
    a = S().forward(model, batch)
    b = S().forward(model, batch)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


# ------------------------------------------------------------------ backward
@pytest.mark.parametrize("shape", [(4, 3, 2, 2, 5, 0, 4), (32, 5, 3, 3, 6, 1, 6),
                                   (64, 7, 1, 2, 4, 1, 5), (128, 20, 3, 4, 5, 0, 7),
                                   (256, 4, 3, 2, 3, 1, 4), (1024, 2, 3, 2, 2, 1, 3)],
                         ids=lambda s: "d{}-S{}-T{}".format(*s[:3]))
def test_backward_random_shapes(shape):
    d, S_, T, E, M, lo, hi = shape
    p = W.random_problem(2000 + d + S_, d, S_, T, E, M, hi, lo)
    model, batch = dev_problem(p)
    alpha = torch.from_numpy(p.alpha).cuda()
    dE = np.random.default_rng(d).standard_normal(M).astype(np.float32)
    g = S().backward(model, batch, alpha, torch.from_numpy(dE).cuda())
    torch.cuda.synchronize()
    go = O.grad_x(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, p.alpha, dE)
    check_rows(g.cpu().numpy(), go)


def test_backward_conformations_subset():
    p = W.conformations(n_conf=24, with_J=False)
    model, batch = dev_problem(p)
    alpha = torch.from_numpy(p.alpha).cuda()
    g = S().backward(model, batch, alpha)
    torch.cuda.synchronize()
    go = O.grad_x(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, p.alpha)
    rel = check_rows(g.cpu().numpy(), go)
    print(f"conformations: grad max normwise atom error {rel:.2e}")


# ------------------------------------------------------------------ predict
def _check_energy(Eg, p, alpha):
    Zo = oracle_forward(p)
    Eo = Zo @ alpha.astype(np.float64)
    scale = np.abs(Zo * alpha[None, :]).sum(axis=1)
    err = np.abs(np.asarray(Eg, np.float64) - Eo)
    assert np.all(err <= 1e-5 * np.maximum(scale, 1e-30)), float(np.max(err / np.maximum(scale, 1e-30)))


@pytest.mark.parametrize("shape", [(8, 3, 3, 2, 7, 0, 5), (64, 4, 3, 3, 9, 1, 10),
                                   (128, 16, 3, 5, 6, 0, 9), (256, 3, 2, 2, 4, 1, 6),
                                   (64, 32, 3, 3, 4, 0, 8), (256, 8, 2, 2, 4, 1, 6),
                                   # the energy + force adjoint spreads an atom's stack
                                   # passes over up to 8 waves: 10 passes (waves 0, 1
                                   # take two), 2 passes at d = 1024
                                   (128, 160, 3, 3, 5, 0, 6), (1024, 3, 2, 2, 3, 1, 3)],
                         ids=lambda s: "d{}-S{}-T{}".format(*s[:3]))
def test_predict_energies_and_forces(shape):
    d, S_, T, E, M, lo, hi = shape
    # at d = 1024 a random sigma down to 0.5 gives phases of up to 160 radians,
    # whose FP32 rounding alone (eps (T log2 d + 3) |u|) exceeds the force bound
    # (the large-phase reading of the feature tolerance); sigma = 32 keeps them
    # below 10 radians, the bias's range
    p = W.random_problem(3000 + d, d, S_, T, E, M, hi, lo, with_J=True,
                         sigma=32.0 if d >= 1024 else None)
    model, batch = dev_problem(p)
    alpha = torch.from_numpy(p.alpha).cuda()
    En = S().predict(model, batch, alpha)
    Ef, F = S().predict(model, batch, alpha, torch.from_numpy(p.J).cuda(),
                        torch.from_numpy(p.J_ptr).cuda())
    torch.cuda.synchronize()
    # energies alone are summed per stack, with forces per atom: both within the bound
    _check_energy(En.cpu().numpy(), p, p.alpha)
    _check_energy(Ef.cpu().numpy(), p, p.alpha)
    go = O.grad_x(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, p.alpha)
    Fo = O.forces(go, p.J, p.J_ptr, p.mol_ptr)
    Fg = F.cpu().numpy().astype(np.float64)
    for m in range(p.n_mols):
        a0, a1 = 3 * p.mol_ptr[m], 3 * p.mol_ptr[m + 1]
        if a1 > a0:
            assert np.abs(Fg[a0:a1] - Fo[a0:a1]).max() <= 1e-5 * np.abs(Fo[a0:a1]).max()


@pytest.mark.parametrize("shape", [(8, 3, 3, 2, 7, 0, 5), (64, 4, 3, 3, 9, 1, 10),
                                   (128, 16, 3, 5, 6, 0, 9), (256, 3, 2, 2, 4, 1, 6),
                                   (1024, 3, 2, 2, 3, 1, 3),
                                   # molecules of up to 300 atoms (energy sums over many
                                   # groups of 16 atoms)
                                   (32, 4, 3, 3, 4, 40, 300)],
                         ids=lambda s: "d{}-S{}-T{}-N{}".format(s[0], s[1], s[2], s[6]))
def test_energy_grad_matches_oracle_and_separate_calls(shape):
    """sorf_energy_grad: energies within the energy bound of the oracle, dE/dx
    within the gradient bound and bitwise equal to sorf_backward (same kernel
    family and summation order), energies equal to sorf_predict's to FP32
    rounding. Includes empty molecules (lo = 0)."""
    d, S_, T, E, M, lo, hi = shape
    p = W.random_problem(3500 + d, d, S_, T, E, M, hi, lo, sigma=32.0 if d >= 1024 else None)
    model, batch = dev_problem(p)
    alpha = torch.from_numpy(p.alpha).cuda()
    eg = S().EnergyGrad(model)
    Eg, g = eg(batch, alpha)
    gb = S().backward(model, batch, alpha)
    En = S().predict(model, batch, alpha)
    torch.cuda.synchronize()
    _check_energy(Eg.cpu().numpy(), p, p.alpha)
    go = O.grad_x(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, p.alpha)
    check_rows(g.cpu().numpy(), go)
    assert torch.equal(g, gb)
    Zo = oracle_forward(p)
    scale = np.abs(Zo * p.alpha[None, :]).sum(axis=1)
    diff = np.abs(Eg.cpu().numpy().astype(np.float64) - En.cpu().numpy())
    assert np.all(diff <= 2e-5 * np.maximum(scale, 1e-30))


def test_energy_grad_empty_batch_gives_zero_energies():
    """No atoms, three (empty) molecules: E = 0 exactly, no workspace needed."""
    from paper_2206_01580_amd import _lib
    import ctypes
    p = W.random_problem(77, 16, 2, 2, 2, 3, 0, 0)
    assert p.x.shape[0] == 0
    model, batch = dev_problem(p)
    lib = _lib.load()
    E = torch.full((3,), 7.0, device="cuda")
    alpha = torch.from_numpy(p.alpha).cuda()
    m, b = model.c_struct(), batch.c_struct()
    st = lib.sorf_energy_grad(ctypes.byref(m), ctypes.byref(b), alpha.data_ptr(), E.data_ptr(),
                              None, None, 0, torch.cuda.current_stream().cuda_stream)
    assert st == _lib.SORF_OK
    torch.cuda.synchronize()
    assert torch.equal(E, torch.zeros(3, device="cuda"))


def test_predict_conformations_subset_with_jacobians():
    p = W.conformations(n_conf=6)
    model, batch = dev_problem(p)
    alpha = torch.from_numpy(p.alpha).cuda()
    E, F = S().predict(model, batch, alpha, torch.from_numpy(p.J).cuda(), torch.from_numpy(p.J_ptr).cuda())
    torch.cuda.synchronize()
    _check_energy(E.cpu().numpy(), p, p.alpha)
    go = O.grad_x(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, p.alpha)
    Fo = O.forces(go, p.J, p.J_ptr, p.mol_ptr)
    Fg = F.cpu().numpy()
    for m in range(p.n_mols):
        sl = slice(3 * p.mol_ptr[m], 3 * p.mol_ptr[m + 1])
        assert np.abs(Fg[sl] - Fo[sl]).max() <= 1e-5 * np.abs(Fo[sl]).max()


def test_predict_forces_large_and_empty_molecules():
    """Force contraction across every tiling regime: empty molecules, a 1-atom
    molecule (3 columns), one whose rows exceed the 32-chunk cap (257 atoms at
    d = 128: 32896 rows, 771 columns in 13 column blocks), and blocks placed out
    of order with gaps in the Jacobian buffer."""
    import dataclasses
    base = W.random_problem(3900, 128, 2, 3, 3, 1, 1, 1)
    sizes = np.array([0, 1, 257, 3, 0, 64])
    rng = np.random.default_rng(3901)
    A = int(sizes.sum())
    ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    blocks = sizes * 128 * 3 * sizes
    order = rng.permutation(len(sizes))
    J_off = np.zeros(len(sizes), np.int64)
    off = 7                                        # unaligned start, gaps between blocks
    for m in order:
        J_off[m] = off
        off += int(blocks[m]) + 13
    J = (0.1 * rng.standard_normal(off)).astype(np.float32)
    p = dataclasses.replace(base, x=rng.standard_normal((A, 128)).astype(np.float32),
                            element=rng.integers(0, 3, A).astype(np.int32), mol_ptr=ptr,
                            alpha=rng.standard_normal(256).astype(np.float32))
    model, batch = dev_problem(p)
    J_ptr = np.concatenate([J_off, [-1]]).astype(np.int64)   # J_ptr[n_mols] is not read
    E, F = S().predict(model, batch, torch.from_numpy(p.alpha).cuda(), torch.from_numpy(J).cuda(),
                       torch.from_numpy(J_ptr).cuda())
    En = S().predict(model, batch, torch.from_numpy(p.alpha).cuda())
    torch.cuda.synchronize()
    _check_energy(E.cpu().numpy(), p, p.alpha)
    _check_energy(En.cpu().numpy(), p, p.alpha)
    assert np.all(En.cpu().numpy()[sizes == 0] == 0.0) and np.all(E.cpu().numpy()[sizes == 0] == 0.0)
    go = O.grad_x(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma, p.alpha)
    Fg = F.cpu().numpy()
    for m in range(len(sizes)):
        n = int(sizes[m])
        if n == 0:
            continue
        blk = J[J_off[m]:J_off[m] + blocks[m]]
        Fo = O.forces(go[ptr[m]:ptr[m + 1]], blk, np.array([0, blocks[m]]), np.array([0, n]))
        sl = slice(3 * ptr[m], 3 * ptr[m + 1])
        assert np.abs(Fg[sl] - Fo).max() <= 1e-5 * np.abs(Fo).max(), m


def test_forces_call_matches_definition_and_predict():
    """sorf_forces: for an arbitrary gradient, F = -sum_i J_i^T g_i per molecule
    against the oracle's FP64 contraction (same per-molecule bound as predict),
    over empty, 1-atom and 257-atom molecules with out-of-order, gapped,
    unaligned Jacobian blocks; on sorf_backward's gradient it gives
    sorf_predict's forces; no atoms is a no-op."""
    sizes = np.array([0, 1, 257, 3, 0, 64])
    rng = np.random.default_rng(3911)
    A, d = int(sizes.sum()), 128
    ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    blocks = sizes * d * 3 * sizes
    J_off = np.zeros(len(sizes), np.int64)
    off = 5
    for m in rng.permutation(len(sizes)):
        J_off[m] = off
        off += int(blocks[m]) + 11
    J = (0.1 * rng.standard_normal(off)).astype(np.float32)
    J_ptr = np.concatenate([J_off, [-1]]).astype(np.int64)
    g = rng.standard_normal((A, d)).astype(np.float32)
    Jd, Jp, Pd = (torch.from_numpy(J).cuda(), torch.from_numpy(J_ptr).cuda(),
                  torch.from_numpy(ptr).cuda())
    F = S().forces(Pd, torch.from_numpy(g).cuda(), Jd, Jp).cpu().numpy()
    for m in range(len(sizes)):
        n = int(sizes[m])
        if n == 0:
            continue
        blk = J[J_off[m]:J_off[m] + blocks[m]]
        Fo = O.forces(g[ptr[m]:ptr[m + 1]], blk, np.array([0, blocks[m]]), np.array([0, n]))
        sl = slice(3 * ptr[m], 3 * ptr[m + 1])
        assert np.abs(F[sl] - Fo).max() <= 1e-5 * np.abs(Fo).max(), m
    # the force part of sorf_predict, as a call of its own
    import dataclasses
    base = W.random_problem(3910, d, 2, 3, 3, 1, 1, 1)
    p = dataclasses.replace(base, x=rng.standard_normal((A, d)).astype(np.float32),
                            element=rng.integers(0, 3, A).astype(np.int32), mol_ptr=ptr,
                            alpha=rng.standard_normal(2 * d).astype(np.float32))
    model, batch = dev_problem(p)
    alpha = torch.from_numpy(p.alpha).cuda()
    _, Fp = S().predict(model, batch, alpha, Jd, Jp)
    gx = S().backward(model, batch, alpha)
    Fs = S().forces(batch.mol_ptr, gx, Jd, Jp)
    torch.cuda.synchronize()
    Fp, Fs = Fp.cpu().numpy().astype(np.float64), Fs.cpu().numpy().astype(np.float64)
    for m in range(len(sizes)):
        sl = slice(3 * ptr[m], 3 * ptr[m + 1])
        if sizes[m]:
            assert np.abs(Fs[sl] - Fp[sl]).max() <= 1e-6 * np.abs(Fp[sl]).max(), m
    # no atoms
    out = torch.empty(0, device="cuda")
    S().forces(torch.zeros(3, dtype=torch.int64, device="cuda"), torch.empty((0, d), device="cuda"),
               Jd, torch.zeros(3, dtype=torch.int64, device="cuda"), out=out)
    torch.cuda.synchronize()


def test_autograd_function_matches_central_differences():
    """SorfEnergy backward vs FP64 central differences of the oracle energy."""
    p = W.random_problem(4242, 16, 3, 3, 2, 2, 3, 2)
    model, batch = dev_problem(p)
    alpha = torch.from_numpy(p.alpha).cuda()
    x = batch.x.clone().requires_grad_(True)
    w = torch.tensor([0.7, -1.3], device="cuda")
    E = S().energy(x, model, batch, alpha)
    (E * w).sum().backward()
    g = x.grad.cpu().numpy().astype(np.float64)
    h = 1e-4
    xs = p.x.astype(np.float64)
    fd = np.zeros_like(xs)
    for i in range(xs.shape[0]):
        for j in range(xs.shape[1]):
            for sgn in (1, -1):
                xx = xs.copy()
                xx[i, j] += sgn * h
                Z = O.molecule_features(xx, p.element, p.mol_ptr, p.signs, p.bias, p.sigma)
                fd[i, j] += sgn * float(np.array([0.7, -1.3]) @ (Z @ p.alpha.astype(np.float64))) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-5 * np.abs(fd).max()


# ------------------------------------------------------------------ Gram
@pytest.mark.parametrize("mode", ["fp32", "fp32_kahan", "bf16", "fp16", "bf16_hilo", "fp16_hilo"])
@pytest.mark.parametrize("MD", [(333, 300), (64, 128), (1000, 37), (5, 257), (600, 1100)], ids=lambda t: f"M{t[0]}-D{t[1]}")
def test_gram_against_emulated_modes(mode, MD):
    M, D = MD
    rng = np.random.default_rng(M + D)
    Z = (rng.standard_normal((M, D)) * 0.05).astype(np.float32)
    y = rng.standard_normal(M).astype(np.float32)
    k = S().fp16_scale_exp(float(np.abs(Z).max())) if mode.startswith("fp16") else 0
    G0 = rng.standard_normal((D, D)).astype(np.float32)  # accumulate onto existing values
    Zt, Gt = torch.from_numpy(Z).cuda(), torch.from_numpy(G0.copy()).cuda()
    Zty = torch.zeros(D, device="cuda")
    S().gram_accumulate(Zt, Gt, torch.from_numpy(y).cuda(), Zty, precision=mode, scale_exp=k)
    torch.cuda.synchronize()
    Gg = Gt.cpu().numpy().astype(np.float64)
    upper = np.triu_indices(D, 1)
    assert np.array_equal(Gg[upper], G0[upper].astype(np.float64)), "upper triangle touched"
    Ge = O.gram_emulated(Z, mode, k)
    low = np.tril_indices(D)
    diff = (Gg - G0.astype(np.float64))[low] - Ge[low]
    assert np.linalg.norm(diff) <= 1e-6 * np.linalg.norm(Ge[low]) + 1e-6 * np.linalg.norm(G0)
    _, r = O.gram(Z, y)
    assert np.abs(Zty.cpu().numpy() - r).max() <= 1e-6 * np.abs(Z).sum(axis=0).max() * np.abs(y).max()


def _split_cross_bound(Z):
    """Entry bound of the split mode against its exact emulation: the head is exact,
    the tail products are summed in FP32 over 256-row blocks and the block sums in FP32,
    so |dG_ij| <= (256 + ceil(M / 256) + 2) 2^-24 C_ij with C_ij the sum of the tail
    products' magnitudes, 2^-(e_i + e_j) sum_m (|h_i t_j| + |t_i h_j| + |t_i t_j|)."""
    h, t, e = O.split_head_tail(Z)
    sc = 2.0 ** -e.astype(np.float64)
    H, T = np.abs(h) * sc, np.abs(t) * sc
    C = H.T @ T + T.T @ H + T.T @ T
    return (256 + -(-len(Z) // 256) + 2) * 2.0 ** -24 * C


@pytest.mark.parametrize("MD", [(333, 300), (64, 128), (1000, 37), (5, 257), (600, 1100),
                                (3000, 1024), (1100, 5900)], ids=lambda t: f"M{t[0]}-D{t[1]}")
def test_gram_split_against_emulation(MD):
    """Split mode (FP64 G): every lower entry within the FP32 bound of the tail sums of
    the exact emulation, accumulated onto existing FP64 values; the strict upper triangle
    untouched; Z^T y in FP64. D = 5900 runs whole head tiles plus row-sliced tail tiles
    combined in int64."""
    M, D = MD
    rng = np.random.default_rng(M + D + 1)
    Z = (rng.standard_normal((M, D)) * 0.05 * np.exp(rng.uniform(-3, 3, D))[None, :]).astype(np.float32)
    y = rng.standard_normal(M).astype(np.float32)
    G0 = rng.standard_normal((D, D))
    Gt = torch.from_numpy(G0.copy()).cuda()
    Zty = torch.zeros(D, device="cuda", dtype=torch.float64)
    S().gram_accumulate(torch.from_numpy(Z).cuda(), Gt, torch.from_numpy(y).cuda(), Zty,
                        precision="split")
    torch.cuda.synchronize()
    Gg = Gt.cpu().numpy()
    upper = np.triu_indices(D, 1)
    assert np.array_equal(Gg[upper], G0[upper]), "upper triangle touched"
    Ge = O.gram_emulated(Z, "split")
    low = np.tril_indices(D)
    diff = np.abs((Gg - G0)[low] - Ge[low])
    bound = _split_cross_bound(Z)[low] + 4e-16 * (np.abs(G0[low]) + np.abs(Ge[low]))
    assert (diff <= bound).all(), float((diff / bound).max())
    _, r = O.gram(Z, y)
    assert np.abs(Zty.cpu().numpy() - r).max() <= 1e-12 * np.abs(Z).sum(axis=0).max() * np.abs(y).max()


def test_gram_split_head_is_exact():
    """Columns of integers times a power of two, each reaching 127 2^-k: the tail is zero,
    so the split mode's G is the int8 head alone and must equal the FP64 Gram exactly."""
    M, D = 2000, 300
    rng = np.random.default_rng(17)
    ints = rng.integers(-127, 128, size=(M, D))
    ints[rng.integers(0, M, D), np.arange(D)] = 127
    k = rng.integers(4, 12, size=D)
    Z = (ints * 2.0 ** -k[None, :]).astype(np.float32)
    G = torch.zeros(D, D, device="cuda", dtype=torch.float64)
    S().gram_accumulate(torch.from_numpy(Z).cuda(), G, precision="split")
    torch.cuda.synchronize()
    exact = Z.astype(np.float64).T @ Z.astype(np.float64)
    low = np.tril_indices(D)
    assert np.array_equal(G.cpu().numpy()[low], exact[low])


def test_gram_split_two_head_passes():
    """140,000 rows: more than one exact int32 pass of the head (131,072 rows each)."""
    M, D = 140000, 256
    rng = np.random.default_rng(18)
    Z = (rng.standard_normal((M, D)) * 0.05).astype(np.float32)
    G = torch.zeros(D, D, device="cuda", dtype=torch.float64)
    S().gram_accumulate(torch.from_numpy(Z).cuda(), G, precision="split")
    torch.cuda.synchronize()
    Ge = O.gram_emulated(Z, "split")
    low = np.tril_indices(D)
    diff = np.abs(G.cpu().numpy()[low] - Ge[low])
    assert (diff <= _split_cross_bound(Z)[low] + 4e-16 * np.abs(Ge[low])).all()


def test_gram_split_deterministic():
    rng = np.random.default_rng(19)
    Z = torch.from_numpy((rng.standard_normal((700, 640)) * 0.1).astype(np.float32)).cuda()
    outs = []
    for _ in range(2):
        G = torch.zeros(640, 640, device="cuda", dtype=torch.float64)
        S().gram_accumulate(Z, G, precision="split")
        outs.append(G)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("D", [64, 30], ids=["ring-D64", "slab-D30"])
def test_kahan_flush_beats_plain_fp32_on_a_long_sum(D):
    """131,072 rows of positive entries near 1 (both modes against FP64 sums of
    the same FP32 rows).

    slab kernel (D % 4 != 0, one pass over all rows): the running FP32 sum grows
    to 1.3e5 while each 256-row block adds ~256, so plain FP32 flushes lose low
    bits at every add; the compensated flush keeps them (5x smaller error).

    ring kernel (D % 4 == 0): the rows of a tile are split into 8 slices of
    16,384 rows whose sums are added in slice order, so the running sums stay
    8x shorter and plain FP32 already lands at the rounding floor of the result
    (about half an ulp, 6e-8 relative); both modes must stay within two ulps
    (2^-22 relative) and the compensated one no worse than the plain one."""
    M = 1 << 17
    rng = np.random.default_rng(D)
    Z = (1.0 + 0.01 * rng.standard_normal((M, D))).astype(np.float32)
    Zd = Z.astype(np.float64)
    Ge = Zd.T @ Zd
    low = np.tril_indices(D)
    errs = {}
    for mode in ("fp32", "fp32_kahan"):
        G = torch.zeros(D, D, device="cuda")
        S().gram_accumulate(torch.from_numpy(Z).cuda(), G, precision=mode)
        torch.cuda.synchronize()
        errs[mode] = float(np.linalg.norm(G.double().cpu().numpy()[low] - Ge[low]) /
                           np.linalg.norm(Ge[low]))
    print("relative Frobenius errors:", errs)
    if D % 4 != 0:
        assert errs["fp32_kahan"] <= 0.2 * errs["fp32"], errs
        assert errs["fp32_kahan"] <= 1e-6
    else:
        assert errs["fp32"] <= 2.0 ** -22 and errs["fp32_kahan"] <= 2.0 ** -22, errs
        assert errs["fp32_kahan"] <= 1.05 * errs["fp32"], errs


@pytest.mark.parametrize("MD", [(333, 300), (17, 64), (5, 129)], ids=lambda t: f"M{t[0]}-D{t[1]}")
def test_gram_fp64(MD):
    M, D = MD
    rng = np.random.default_rng(7 * M + D)
    Z = (rng.standard_normal((M, D)) * 0.05).astype(np.float32)
    y = rng.standard_normal(M).astype(np.float32)
    G = torch.zeros(D, D, device="cuda", dtype=torch.float64)
    Zty = torch.zeros(D, device="cuda", dtype=torch.float64)
    S().gram_accumulate(torch.from_numpy(Z).cuda(), G, torch.from_numpy(y).cuda(), Zty, "fp64")
    torch.cuda.synchronize()
    Go, ro = O.gram(Z, y)
    low = np.tril_indices(D)
    Gg = G.cpu().numpy()
    assert np.abs(Gg[low] - Go[low]).max() <= 1e-13 * np.abs(Go).max()
    assert np.all(Gg[np.triu_indices(D, 1)] == 0.0)
    assert np.abs(Zty.cpu().numpy() - ro).max() <= 1e-13 * np.abs(ro).max()


@pytest.mark.parametrize("mode", ["fp32", "fp32_kahan"])
@pytest.mark.parametrize("MD", [(20001, 256), (4100, 1000), (9000, 1536)],
                         ids=lambda t: f"M{t[0]}-D{t[1]}")
def test_gram_fp32_row_slices(mode, MD):
    """Row counts at which the FP32 tile kernel splits every tile's rows into
    slices (8 slices of 2560 rows with a last one of 2081; 2 with a ragged 1796;
    5 with a last one of 808; D = 1000 also ends in a partial tile): slice 0 adds
    into G, the others go through partial tiles combined in slice order. G
    accumulates onto existing values, the upper triangle stays untouched, and the
    result is within the FP32 bound of the FP64 Gram and bitwise repeatable."""
    M, D = MD
    rng = np.random.default_rng(3 * M + D)
    Z = (rng.standard_normal((M, D)) * 0.05).astype(np.float32)
    G0 = rng.standard_normal((D, D)).astype(np.float32)
    Zt = torch.from_numpy(Z).cuda()
    outs = []
    for _ in range(2):
        Gt = torch.from_numpy(G0.copy()).cuda()
        S().gram_accumulate(Zt, Gt, precision=mode)
        outs.append(Gt)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    Gg = outs[0].cpu().numpy().astype(np.float64)
    upper = np.triu_indices(D, 1)
    assert np.array_equal(Gg[upper], G0[upper].astype(np.float64)), "upper triangle touched"
    Ge = O.gram_emulated(Z, mode, 0)
    low = np.tril_indices(D)
    diff = (Gg - G0.astype(np.float64))[low] - Ge[low]
    assert np.linalg.norm(diff) <= 1e-6 * np.linalg.norm(Ge[low]) + 1e-6 * np.linalg.norm(G0)


@pytest.mark.parametrize("mode", ["bf16", "fp16"])
def test_gram_single_product_whole_and_sliced_tiles(mode):
    # D = 5900: 300 tiles of 256 x 256, so one whole round of 256 tiles plus
    # 44 tail tiles whose rows are split into slices and combined
    M, D = 1100, 5900
    rng = np.random.default_rng(5)
    Z = (rng.standard_normal((M, D)) * 0.05).astype(np.float32)
    k = S().fp16_scale_exp(float(np.abs(Z).max())) if mode == "fp16" else 0
    G = torch.zeros(D, D, device="cuda")
    S().gram_accumulate(torch.from_numpy(Z).cuda(), G, precision=mode, scale_exp=k)
    torch.cuda.synchronize()
    Gg = G.cpu().numpy().astype(np.float64)
    assert np.all(Gg[np.triu_indices(D, 1)] == 0.0)
    Ge = O.gram_emulated(Z, mode, k)
    low = np.tril_indices(D)
    assert np.linalg.norm(Gg[low] - Ge[low]) <= 1e-6 * np.linalg.norm(Ge[low])


@pytest.mark.parametrize("mode", ["bf16_hilo", "bf16"])
def test_gram_deterministic(mode):
    rng = np.random.default_rng(1)
    Z = torch.from_numpy((rng.standard_normal((700, 384)) * 0.1).astype(np.float32)).cuda()
    outs = []
    for _ in range(2):
        G = torch.zeros(384, 384, device="cuda")
        S().gram_accumulate(Z, G, precision=mode)
        outs.append(G)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


# ------------------------------------------------------------------ solve
@pytest.mark.parametrize("D", [1, 50, 64, 128, 200, 256, 513, 1000])
def test_solve_matches_oracle(D):
    rng = np.random.default_rng(D)
    Z = rng.standard_normal((2 * D + 10, D)).astype(np.float32)
    G = (Z.astype(np.float64).T @ Z.astype(np.float64)).astype(np.float32)
    rhs = rng.standard_normal(D).astype(np.float32)
    lam = 1e-3
    a, info = S().solve(torch.from_numpy(G).cuda(), torch.from_numpy(rhs).cuda(), lam, 3)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    ao = O.solve(np.tril(G) + np.tril(G, -1).T, rhs, lam)
    assert np.abs(a.cpu().numpy() - ao).max() <= 1e-10 * np.abs(ao).max()


def test_solve_reads_only_lower_triangle():
    D = 130
    rng = np.random.default_rng(3)
    Z = rng.standard_normal((300, D)).astype(np.float32)
    G = (Z.T.astype(np.float64) @ Z).astype(np.float32)
    junk = G.copy()
    junk[np.triu_indices(D, 1)] = np.nan
    rhs = rng.standard_normal(D).astype(np.float32)
    a1, i1 = S().solve(torch.from_numpy(G).cuda(), torch.from_numpy(rhs).cuda(), 1e-2, 2)
    a2, i2 = S().solve(torch.from_numpy(junk).cuda(), torch.from_numpy(rhs).cuda(), 1e-2, 2)
    torch.cuda.synchronize()
    assert int(i1.item()) == 0 and int(i2.item()) == 0
    assert torch.equal(a1, a2)


def test_solve_reports_non_spd():
    D = 100
    G = np.eye(D, dtype=np.float32)
    G[70, 70] = -5.0
    a, info = S().solve(torch.from_numpy(G).cuda(), torch.ones(D, device="cuda"), 0.0, 0)
    torch.cuda.synchronize()
    assert int(info.item()) == 71


def _spd_system(D, seed):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((2 * D + 10, D)).astype(np.float32)
    G = (Z.astype(np.float64).T @ Z.astype(np.float64)).astype(np.float32)
    rhs = rng.standard_normal(D).astype(np.float32)
    return torch.from_numpy(G).cuda(), torch.from_numpy(rhs).cuda()


@pytest.mark.parametrize("D", [100, 640, 1000])
def test_solve_one_stream_equals_lookahead(D):
    """sorf_solve (every launch on the caller's stream, no other HIP object) and
    sorf_solve_streamed (caller-owned side stream and events) run the same kernels
    on the same data: bitwise the same alpha."""
    sorf = S()
    G, r = _spd_system(D, 11 + D)
    a1 = sorf.Solver(D, lookahead=False)(G, r, 1e-3, 3)
    solver = sorf.Solver(D, lookahead=True)
    a2 = solver(G, r, 1e-3, 3)
    torch.cuda.synchronize()
    assert int(solver.info.item()) == 0
    assert torch.equal(a1, a2)
    solver.close()


def test_concurrent_solves_from_two_threads():
    """Two host threads, each with its own Solver (workspace and side stream) and its
    own torch stream, solve different systems at the same time, three times each:
    every result is bitwise the result of the same solve run alone. The library keeps
    no state that the two could share."""
    import threading
    sorf = S()
    systems = [_spd_system(1000, 21), _spd_system(1000, 22)]
    solo = []
    for G, r in systems:
        sv = sorf.Solver(1000)
        solo.append(sv(G, r, 1e-3, 3).clone())
        torch.cuda.synchronize()
        assert int(sv.info.item()) == 0
        sv.close()
    results = [[], []]
    errors = []
    barrier = threading.Barrier(2)

    def run(i):
        try:
            sv = sorf.Solver(1000)
            st = torch.cuda.Stream()
            G, r = systems[i]
            torch.cuda.synchronize()
            barrier.wait()
            with torch.cuda.stream(st):
                for _ in range(3):
                    results[i].append(sv(G, r, 1e-3, 3).clone())
            st.synchronize()
            if int(sv.info.item()) != 0:
                errors.append(f"thread {i}: info {int(sv.info.item())}")
            sv.close()
        except Exception as exc:  # reported below
            errors.append(f"thread {i}: {exc!r}")

    threads = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=60)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    for i in range(2):
        assert len(results[i]) == 3
        for a in results[i]:
            assert torch.equal(a, solo[i])


# ------------------------------------------------------------------ end to end
def test_end_to_end_small_energy_batch():
    """forward -> Gram (FP64, the paper's DP mode) -> FP64 solve -> predict,
    against the oracle pipeline; checked on energies (the 200-molecule batch is rank
    deficient: N=200 < D=256, and lambda = 1e-6 is below the FP32 rounding of G).

    Bound: the batch is interpolated (fewer molecules than features), so the fitted
    energies of the GPU's own features equal the targets to ~1e-11 relative whatever
    the features' FP32 error is (the oracle, refitting on features perturbed by 1e-6
    of each row's maximum, moves its fitted energies by 6e-12 relative). What is left is
    the difference between the FP32 features of sorf_predict and those of sorf_forward
    that the fit saw, weighted by the GPU's alpha: the condition-aware energy bound
    |dE_m| <= 1e-5 sum_f |alpha_f Z_mf| of the feature kernels."""
    p = W.small_energy_batch()
    s = S()
    model, batch = dev_problem(p)
    D = p.n_features
    Z = s.forward(model, batch)
    G = torch.zeros(D, D, device="cuda", dtype=torch.float64)
    Zty = torch.zeros(D, device="cuda", dtype=torch.float64)
    y = torch.from_numpy(p.y).cuda()
    s.gram_accumulate(Z, G, y, Zty, "fp64")
    a, info = s.solve(G, Zty, p.lam, 3)
    E = s.predict(model, batch, a.float())
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Zo = oracle_forward(p)
    Go, ro = O.gram(Zo, p.y)
    ao = O.solve(Go, ro, p.lam)
    Eo = Zo @ ao
    Eg = E.cpu().numpy().astype(np.float64)
    rel = np.abs(Eg - Eo).max() / np.abs(Eo).max()
    scale = (np.abs(a.cpu().numpy())[None, :] * np.abs(Zo)).sum(axis=1)
    print(f"small energy batch: end-to-end energy max rel error {rel:.2e}; "
          f"max |dE|/sum|aZ| {(np.abs(Eg - Eo) / scale).max():.2e}; "
          f"fit rmse {np.sqrt(np.mean((Eo - p.y) ** 2)):.3e}")
    assert (np.abs(Eg - Eo) <= 1e-5 * scale).all()


# ------------------------------------------------------------------ validation kernel
def test_validate_batch_flags():
    s = S()
    p = W.random_problem(9, 8, 2, 3, 3, 5, 4, 1)
    _, batch = dev_problem(p)
    assert s.validate_batch(batch, 3) == 0
    assert s.validate_batch(batch, 2) & 8 or (p.element < 2).all()
    bad_ptr = p.mol_ptr.copy()
    bad_ptr[2] = bad_ptr[3] + 1          # offsets decrease from index 2 to 3
    b2 = s.Batch.from_arrays(p.x, p.element, bad_ptr)
    assert s.validate_batch(b2, 3) & 2
    b3 = s.Batch.from_arrays(p.x, p.element, p.mol_ptr + 1)
    assert s.validate_batch(b3, 3) & 1
