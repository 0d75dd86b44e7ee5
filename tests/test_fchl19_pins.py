"""Pins of the FCHL19 oracle against what the paper's formulas and geometry
fix, independently of the oracle's own code: library densities (log-normal,
normal), closed forms on triangles of known angles, integrals of the two-body
profile, invariances, the cutoff, and central differences for the gradient."""
import math

import numpy as np
import pytest
import scipy.stats
import torch

from oracle import fchl19_oracle as F
from paper_2206_01580_amd import workloads as W

PRM = dict(W.FCHL19_EF)


def rho_of(R, el, n_el=3, prm=PRM):
    rho, _ = F.fchl19(np.asarray(R, float), np.asarray(el), [0, len(el)], n_el, prm)
    return rho.numpy()


def g3(rho, n_el, p, prm=PRM):
    base = n_el * prm["n2"] + p * prm["n3"] * 2
    return rho[base:base + 2 * prm["n3"]].reshape(prm["n3"], 2)


def fcut(r, rc=PRM["rcut"]):
    return 0.5 * (math.cos(math.pi * r / rc) + 1.0) if r < rc else 0.0


def test_size_and_pair_order():
    assert F.fchl19_size(5, 24, 20) == 720
    assert F.fchl19_size(5, 23, 22) == 5 * 23 + 15 * 22 * 2
    pairs = [(a, b) for a in range(5) for b in range(a, 5)]
    assert [F.pair_index(a, b, 5) for a, b in pairs] == list(range(15))
    assert F.pair_index(3, 1, 5) == F.pair_index(1, 3, 5)


def test_two_body_is_a_lognormal_density_with_mean_r():
    """Two atoms at distance r: the bins of the neighbour's element hold
    f_cut(r) r^-N2 times the log-normal density with the paper's mu, sigma
    (scipy), and with a fine grid that density integrates to 1 with mean r."""
    r = 1.7
    rho = rho_of([[0, 0, 0], [r, 0, 0]], [0, 2])[0]
    q = 1 + PRM["eta2"] / r ** 2
    mu, s = math.log(r / math.sqrt(q)), math.sqrt(math.log(q))
    Rs = PRM["rcut"] * (np.arange(PRM["n2"]) + 1) / PRM["n2"]
    ref = fcut(r) * r ** -PRM["N2"] * scipy.stats.lognorm.pdf(Rs, s=s, scale=math.exp(mu))
    assert np.allclose(rho[2 * 24:3 * 24], ref, rtol=1e-12, atol=1e-15)
    assert np.all(rho[:2 * 24] == 0) and np.all(rho[3 * 24:] == 0)
    fine = dict(PRM, n2=20000, rcut=40.0)
    prof = rho_of([[0, 0, 0], [r, 0, 0]], [0, 0], 1, fine)[0][:20000] / (fcut(r, 40.0) * r ** -PRM["N2"])
    dR = 40.0 / 20000
    grid = 40.0 * (np.arange(20000) + 1) / 20000
    assert abs(prof.sum() * dR - 1.0) < 1e-6
    assert abs((grid * prof).sum() * dR - r) < 1e-6


def test_equilateral_triangle_closed_form():
    """All angles 60 degrees: xi3 = c3 (1 + 3/8) / r^(3 N3); cos and sin terms
    2 e^(-zeta^2/2) (1/2, sqrt(3)/2); radial profile = normal density with
    mean r and variance 1 / (2 eta3) (scipy)."""
    r = 1.4
    R = [[0, 0, 0], [r, 0, 0], [r / 2, r * math.sqrt(3) / 2, 0]]
    rho = rho_of(R, [0, 1, 2], 3)
    Rs = PRM["rcut"] * np.arange(PRM["n3"]) / (PRM["n3"] - 1)
    radial = scipy.stats.norm.pdf(Rs, loc=r, scale=1 / math.sqrt(2 * PRM["eta3"]))
    xi = PRM["c3"] * (1 + 3 / 8) / r ** (3 * PRM["N3"])
    w = xi * fcut(r) ** 3 * 2 * math.exp(-PRM["zeta"] ** 2 / 2) * radial
    G = g3(rho[0], 3, F.pair_index(1, 2, 3))
    assert np.allclose(G[:, 0], w * 0.5, rtol=1e-10, atol=1e-300)
    assert np.allclose(G[:, 1], w * math.sqrt(3) / 2, rtol=1e-10, atol=1e-300)
    # atom 0 sees the pair (1, 2) only: every other three-body bin is empty
    other = rho[0][3 * 24:].copy()
    base = F.pair_index(1, 2, 3) * 40
    other[base:base + 40] = 0
    assert np.all(other == 0)


def test_right_angle_and_collinear_cases():
    """Right angle at i: cos term 0, ATM numerator 1 (cos_i = 0). i between j and
    k on a line: sin term 0, cos_i = -1, cos_j = cos_k = 1, numerator 1 - 3."""
    a, b = 1.2, 1.5
    rho = rho_of([[0, 0, 0], [a, 0, 0], [0, b, 0]], [0, 0, 0], 1)[0]
    G = g3(rho, 1, 0)
    c = math.hypot(a, b)
    Rs = PRM["rcut"] * np.arange(PRM["n3"]) / (PRM["n3"] - 1)
    radial = scipy.stats.norm.pdf(Rs, loc=(a + b) / 2, scale=1 / math.sqrt(2 * PRM["eta3"]))
    xi = PRM["c3"] * 1.0 / (a * b * c) ** PRM["N3"]
    w = xi * fcut(a) * fcut(b) * fcut(c) * 2 * math.exp(-PRM["zeta"] ** 2 / 2) * radial
    assert np.allclose(G[:, 0], 0.0, atol=1e-15 * w.max())
    assert np.allclose(G[:, 1], w, rtol=1e-10)
    rho = rho_of([[0, 0, 0], [-a, 0, 0], [b, 0, 0]], [0, 0, 0], 1)[0]
    G = g3(rho, 1, 0)
    xi = PRM["c3"] * (1 - 3) / (a * b * (a + b)) ** PRM["N3"]
    radial = scipy.stats.norm.pdf(Rs, loc=(a + b) / 2, scale=1 / math.sqrt(2 * PRM["eta3"]))
    w = xi * fcut(a) * fcut(b) * fcut(a + b) * 2 * math.exp(-PRM["zeta"] ** 2 / 2) * radial
    assert np.allclose(G[:, 0], -w, rtol=1e-10)
    assert np.abs(G[:, 1]).max() < 1e-6 * np.abs(w).max()


def test_invariances_rotation_translation_permutation():
    rng = np.random.default_rng(3)
    R = W.host_geometries([12], 4).astype(np.float64)
    el = rng.integers(0, 3, 12)
    rho = rho_of(R, el)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    assert np.abs(rho_of(R @ Q.T + np.array([3.0, -1.0, 2.0]), el) - rho).max() < 1e-10 * np.abs(rho).max()
    perm = rng.permutation(12)
    assert np.abs(rho_of(R[perm], el[perm]) - rho[perm]).max() < 1e-10 * np.abs(rho).max()


def test_cutoff():
    rc = PRM["rcut"]
    # a neighbour at or beyond the cutoff contributes nothing
    rho = rho_of([[0, 0, 0], [rc, 0, 0]], [0, 1])
    assert np.all(rho == 0)
    # contributions fade to zero as r -> r_cut
    near = rho_of([[0, 0, 0], [rc - 1e-3, 0, 0]], [0, 1])[0]
    mid = rho_of([[0, 0, 0], [rc - 1.0, 0, 0]], [0, 1])[0]
    assert np.abs(near).max() < 1e-5 * np.abs(mid).max()
    # a third atom beyond r_cut of the pair j-k but inside r_cut of i still cuts the triple
    rho = rho_of([[0, 0, 0], [-3.5, 0, 0], [3.5, 0, 0]], [0, 0, 0], 1)[0]
    assert np.all(rho[24:] == 0)


def test_gradient_central_differences():
    rng = np.random.default_rng(5)
    sizes = [7, 4]
    R = W.host_geometries(sizes, 6).astype(np.float64)
    el = rng.integers(0, 3, sum(sizes))
    ptr = np.r_[0, np.cumsum(sizes)]
    prm = PRM
    size = F.fchl19_size(3, prm["n2"], prm["n3"])
    g = rng.standard_normal((sum(sizes), size))
    dR = F.fchl19_grad(R, el, ptr, 3, prm, g)
    h = 1e-5

    def L(Rx):
        rho, _ = F.fchl19(Rx, el, ptr, 3, prm)
        return float(torch.sum(rho * torch.tensor(g)))
    for a in range(sum(sizes)):
        for c in range(3):
            Rp = R.copy(); Rp[a, c] += h
            Rm = R.copy(); Rm[a, c] -= h
            fd = (L(Rp) - L(Rm)) / (2 * h)
            assert abs(dR[a, c] - fd) <= 1e-6 * max(1.0, abs(fd)), (a, c, dR[a, c], fd)
    # no interaction across molecules: the gradient of molecule 1 ignores molecule 0's g
    g2 = g.copy(); g2[:7] = 0
    d2 = F.fchl19_grad(R, el, ptr, 3, prm, g2)
    assert np.all(d2[:7] == 0)
