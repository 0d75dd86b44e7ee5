"""Pin P10 at the size of the differentiation workload: the oracle's analytic
gradient (dense W^T route: grad_x, then forces F = -sum_i J_i^T grad_x_i) against
FP64 central differences of its own energy, on 16 conformations of the 21-atom
molecule (d = 128, D = 8192, sigma = 8, alpha ~ N(0, 1)).

Directions per conformation: all 63 Cartesian coordinates, through the Jacobian
columns (x(r + h e_k) = x + h J[:, :, k], the linearised representation of the
differentiation workload), and 8 random unit directions in x-space spread over
all 21 atoms. h = 1e-4.

Error budget of a central difference in FP64: truncation (h^2 / 6) |E'''| plus
rounding ~ 1e-16 |E| / h. Along a unit direction u the third derivative of
E = sum_f alpha_f sqrt(2/D) sum_i cos(u_i,f) is at most sqrt(2/D) sum_f |alpha_f|
sum_i |w_f . u_i|^3, which the test evaluates; the bound used is twice the sum
of the two terms. Theory section, RFF subsection (energies E = Z alpha and their
coordinate derivatives; forces are minus the coordinate gradient)."""
import math

import numpy as np
import pytest

from oracle import sorf_oracle as O
from paper_2206_01580_amd import workloads as W

N_CONF = 16
N_RANDOM = 8
H = 1e-4


@pytest.fixture(scope="module")
def problem():
    # the first 16 conformations of the 2000-conformation workload; its Jacobians
    # come from their own seeded stream, so the first blocks are those of the full run
    full = W.conformations(2000, with_J=False)
    n_at, d = 21, full.d
    jrng = W._jacobian_rng(full.seed)
    J = (0.1 * jrng.standard_normal(N_CONF * n_at * d * 3 * n_at, dtype=np.float32))
    return full, J.astype(np.float64).reshape(N_CONF, n_at, d, 3 * n_at)


def _energies(p, xs, alpha):
    """Energy of each x in xs (a list of [21, d] arrays) through the oracle's forward."""
    n = len(xs)
    X = np.concatenate(xs, axis=0)
    element = np.tile(p.element[:21], n)
    ptr = np.arange(n + 1, dtype=np.int64) * 21
    Z = O.molecule_features(X, element, ptr, p.signs, p.bias, p.sigma, chunk_atoms=1 << 14)
    return Z @ alpha


@pytest.mark.slow
def test_forces_and_random_directions_central_differences(problem):
    p, J = problem
    alpha = p.alpha.astype(np.float64)
    D = p.n_features
    rng = np.random.default_rng(20220603)
    Wd = {e: O.dense_w(p.signs[e], p.sigma) for e in range(p.signs.shape[0])}
    worst = 0.0
    for c in range(N_CONF):
        a0 = 21 * c
        x = p.x[a0:a0 + 21].astype(np.float64)
        el = p.element[a0:a0 + 21]
        ptr = np.array([0, 21], dtype=np.int64)
        g = O.grad_x(x, el, ptr, p.signs, p.bias, p.sigma, alpha)
        F = O.forces(g, J[c].ravel(), np.array([0, J[c].size], dtype=np.int64), ptr)
        dirs = [J[c][:, :, k] for k in range(63)]
        for _ in range(N_RANDOM):
            u = rng.standard_normal((21, p.d))
            dirs.append(u / np.linalg.norm(u))
        xs = [x + H * u for u in dirs] + [x - H * u for u in dirs]
        E = _energies(p, xs, alpha)
        n = len(dirs)
        fd = (E[:n] - E[n:]) / (2 * H)
        analytic = np.array([float(np.sum(g * u)) for u in dirs])
        # forces: F_k = -dE/dr_k, so along Jacobian column k the derivative is -F_k
        assert np.abs(-F - analytic[:63]).max() <= 1e-12 * max(1.0, np.abs(F).max())
        Eabs = np.abs(_energies(p, [x], np.abs(alpha)))[0]
        for k, u in enumerate(dirs):
            third = math.sqrt(2.0 / D) * sum(
                float(np.abs(alpha) @ np.abs(Wd[int(el[i])] @ u[i]) ** 3) for i in range(21))
            bound = 2.0 * (H * H / 6.0 * third + 1e-16 * Eabs / H)
            err = abs(fd[k] - analytic[k])
            worst = max(worst, err / bound)
            assert err <= bound, (c, k, err, bound)
    print(f"central differences: worst error / bound = {worst:.3f}")
