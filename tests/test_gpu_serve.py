"""GPU tests of the serving path (continuous batching of energy + force
requests over sorf_predict).

* batch invariance: every request served inside a multi-request batch gets
  the same energy and forces, bit for bit, as when it is launched alone;
* parity: sampled served requests match the FP64 oracle (energy bound
  1e-5 * sum_f |alpha_f Z_f|, forces 1e-5 * max |F|, as in the predict tests);
* the Jacobian blocks are read at arbitrary, non-contiguous offsets of one
  pool, as the serving trace places them.
"""
import numpy as np
import pytest

from oracle import sorf_oracle as O
from paper_2206_01580_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trace():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2206_01580_amd import _lib
    _lib.load()
    tr = W.serving_trace(rate_hz=20000.0, duration_s=1.0, max_requests=48, j_pool_floats=1 << 22,
                   d=32, n_stacks=8)
    Jh = tr.host_J_pool()
    return tr, Jh, torch.from_numpy(Jh).cuda()


def _serve(tr, Jd, n_slots, max_atoms, plain):
    from paper_2206_01580_amd import serve, sorf
    pool = serve.RequestPool(tr.x, tr.element, tr.sizes, Jd, tr.J_off)
    model = sorf.Model.from_problem(tr.model)
    alpha = torch.from_numpy(tr.model.alpha).cuda()
    ex = serve.GpuExecutor(model, alpha, pool, max_batch_atoms=max(max_atoms, int(tr.sizes.max())),
                           max_batch_reqs=len(tr.sizes), n_slots=n_slots)
    arrivals = np.zeros(len(tr.sizes))          # all requests queued at t = 0
    if plain:
        st = serve.PlainRunner(ex).run(arrivals, tr.sizes)
    else:
        st = serve.BatchingScheduler(ex, max_atoms, n_slots, 1 << 40).run(arrivals, tr.sizes)
    torch.cuda.synchronize()
    return st, serve.request_results(ex, tr.sizes)


def test_batched_requests_equal_solo_launches_bitwise(trace):
    tr, _, Jd = trace
    st_b, res_b = _serve(tr, Jd, n_slots=3, max_atoms=1024, plain=False)
    st_p, res_p = _serve(tr, Jd, n_slots=1, max_atoms=0, plain=True)
    assert any(b - a > 1 for a, b in st_b.batches), "no multi-request batch formed"
    assert len(st_p.batches) == len(tr.sizes)
    assert sorted(res_b) == sorted(res_p) == list(range(len(tr.sizes)))
    for r in range(len(tr.sizes)):
        Eb, Fb = res_b[r]
        Ep, Fp = res_p[r]
        assert np.float32(Eb).tobytes() == np.float32(Ep).tobytes(), r
        assert Fb.tobytes() == Fp.tobytes(), r


@pytest.mark.parametrize("which", ["smallest", "largest", "first"])
def test_served_requests_match_oracle(trace, which):
    tr, Jh, Jd = trace
    _, res = _serve(tr, Jd, n_slots=2, max_atoms=2048, plain=False)
    r = {"smallest": int(np.argmin(tr.sizes)), "largest": int(np.argmax(tr.sizes)), "first": 0}[which]
    m = tr.model
    a0 = int(np.sum(tr.sizes[:r]))
    n = int(tr.sizes[r])
    x, el = tr.x[a0:a0 + n], tr.element[a0:a0 + n]
    ptr = np.array([0, n], dtype=np.int64)
    alpha = m.alpha.astype(np.float64)
    za = O.atom_features(x, el, m.signs, m.bias, m.sigma)
    Eo = float((za @ alpha).sum())
    scale = float(np.abs(za * alpha[None, :]).sum())
    Eg, Fg = res[r]
    assert abs(Eg - Eo) <= 1e-5 * scale, (Eg, Eo, scale)
    g = O.grad_x(x, el, ptr, m.signs, m.bias, m.sigma, alpha)
    nJ = n * m.d * 3 * n
    blk = Jh[tr.J_off[r]:tr.J_off[r] + nJ]
    Fo = O.forces(g, blk, np.array([0, nJ]), ptr)
    assert np.abs(Fg.astype(np.float64) - Fo).max() <= 1e-5 * np.abs(Fo).max()
