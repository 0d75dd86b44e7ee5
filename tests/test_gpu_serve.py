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


def test_staggered_arrivals_at_the_serving_shape():
    """Requests of the serving workload's shape (d = 128, 128 stacks: D = 16384,
    5..300 atoms, Jacobian blocks at random offsets of a pool) arrive every
    ~50 us on the clock, so later requests are admitted while earlier batches
    are still on the device. Every request's energy and forces equal its solo
    launch bit for bit, and two requests match the FP64 oracle."""
    from paper_2206_01580_amd import serve, sorf
    tr = W.serving_trace(rate_hz=20000.0, duration_s=1.0, max_requests=64, j_pool_floats=1 << 25)
    Jd = W.device_normal(tr.J_pool_floats, tr.J_seed, 0.1)
    pool = serve.RequestPool(tr.x, tr.element, tr.sizes, Jd, tr.J_off)
    model = sorf.Model.from_problem(tr.model)
    alpha = torch.from_numpy(tr.model.alpha).cuda()
    R = len(tr.sizes)
    print(f"staggered serve: {R} requests, {int(tr.sizes.sum())} atoms, "
          f"last arrival {tr.arrival_s[-1] * 1e3:.2f} ms", flush=True)
    exb = serve.GpuExecutor(model, alpha, pool, max_batch_atoms=1024, max_batch_reqs=R, n_slots=3)
    exp = serve.GpuExecutor(model, alpha, pool, max_batch_atoms=int(tr.sizes.max()),
                            max_batch_reqs=1, n_slots=1)
    for ex in (exb, exp):        # load the kernels once before the clock starts
        h = ex.submit(0, 1)
        while not h.done():
            pass
        ex.results.clear()
    torch.cuda.synchronize()
    st_b = serve.BatchingScheduler(exb, 1024, 3, 1 << 40).run(tr.arrival_s, tr.sizes)
    st_p = serve.PlainRunner(exp).run(tr.arrival_s, tr.sizes)
    torch.cuda.synchronize()
    res_b = serve.request_results(exb, tr.sizes)
    res_p = serve.request_results(exp, tr.sizes)
    assert sorted(res_b) == sorted(res_p) == list(range(R))
    assert st_b.summary()["launches_beside_inflight"] > 0, "no launch overlapped a batch in flight"
    for r in range(R):
        assert np.float32(res_b[r][0]).tobytes() == np.float32(res_p[r][0]).tobytes(), r
        assert res_b[r][1].tobytes() == res_p[r][1].tobytes(), r
    m = tr.model
    alpha64 = m.alpha.astype(np.float64)
    for r in (int(np.argmax(tr.sizes)), R - 1):
        a0, n = int(np.sum(tr.sizes[:r])), int(tr.sizes[r])
        x, el = tr.x[a0:a0 + n], tr.element[a0:a0 + n]
        ptr = np.array([0, n], dtype=np.int64)
        za = O.atom_features(x, el, m.signs, m.bias, m.sigma)
        Eo = float((za @ alpha64).sum())
        assert abs(res_b[r][0] - Eo) <= 1e-5 * float(np.abs(za * alpha64[None, :]).sum())
        g = O.grad_x(x, el, ptr, m.signs, m.bias, m.sigma, alpha64)
        nJ = n * m.d * 3 * n
        blk = Jd[int(tr.J_off[r]):int(tr.J_off[r]) + nJ].cpu().numpy()
        Fo = O.forces(g, blk, np.array([0, nJ]), ptr)
        assert np.abs(res_b[r][1].astype(np.float64) - Fo).max() <= 1e-5 * np.abs(Fo).max()


def _predict_solo(tr, Jd, model, alpha, r):
    """sorf_predict on request r alone (its Jacobian block at its pool offset)."""
    from paper_2206_01580_amd import sorf
    a0, n = int(np.sum(tr.sizes[:r])), int(tr.sizes[r])
    batch = sorf.Batch(torch.from_numpy(np.ascontiguousarray(tr.x[a0:a0 + n])).cuda(),
                       torch.from_numpy(np.ascontiguousarray(tr.element[a0:a0 + n])).cuda(),
                       torch.tensor([0, n], dtype=torch.int64, device="cuda"))
    jp = torch.tensor([int(tr.J_off[r]), 0], dtype=torch.int64, device="cuda")
    E, F = sorf.Predictor(model)(batch, alpha, Jd, jp)
    torch.cuda.synchronize()
    return float(E.cpu().numpy()[0]), F.cpu().numpy()


@pytest.mark.parametrize("shape", [(128, 128, 20000.0, 48), (32, 8, 2.0e7, 300)],
                         ids=["d128-S128", "d32-S8-many"])
def test_native_server_equals_predict_bitwise(shape):
    """The persistent serving kernel (sorf_server_*): requests arrive on the
    clock while earlier batches are on the device (d = 128, D = 16384, 5..300
    atoms, about one every 50 us; and a burst of 300 small d = 32 requests
    within 15 us, so that batches reach the 64-request limit). Every request's energy and
    forces are bitwise those of sorf_predict on it alone; the kernel stops on
    request."""
    from paper_2206_01580_amd import serve, sorf
    d, S_, rate, R = shape
    tr = W.serving_trace(rate_hz=rate, duration_s=1.0, max_requests=R, j_pool_floats=1 << 24,
                         d=d, n_stacks=S_)
    Jd = W.device_normal(tr.J_pool_floats, tr.J_seed, 0.1)
    pool = serve.RequestPool(tr.x, tr.element, tr.sizes, Jd, tr.J_off)
    model = sorf.Model.from_problem(tr.model)
    alpha = torch.from_numpy(tr.model.alpha).cuda()
    R = len(tr.sizes)
    cap = 8192
    print(f"native server: d {d}, {S_} stacks, {R} requests, {int(tr.sizes.sum())} atoms", flush=True)
    srv = serve.NativeServer(model, alpha, pool, max_batch_atoms=cap, ring_slots=4, idle_timeout_s=5.0)
    try:
        st = serve.BatchingScheduler(srv, cap, 4, 1 << 40, max_batch_requests=64).run(tr.arrival_s, tr.sizes)
    finally:
        state = srv.stop()
    assert state == 1, state
    res = serve.request_results(srv, tr.sizes)
    assert sorted(res) == list(range(R))
    sizes = [b - a for a, b in st.batches]
    print("batches:", len(st.batches), "largest", max(sizes), "beside in-flight",
          st.summary()["launches_beside_inflight"])
    if d == 32:
        assert max(sizes) == 64           # the per-batch request limit is reached
    for r in range(R):
        E, F = _predict_solo(tr, Jd, model, alpha, r)
        assert np.float32(res[r][0]).tobytes() == np.float32(E).tobytes(), r
        assert res[r][1].tobytes() == F.tobytes(), r


def test_native_server_idle_exit_and_busy_ring():
    """A server with one ring slot: a second batch submitted before the first
    is done gets SORF_ERR_BUSY (or goes through if the first already finished);
    with no batches the kernel exits on its idle timeout and reports it."""
    import ctypes
    from paper_2206_01580_amd import _lib, serve, sorf
    tr = W.serving_trace(rate_hz=1000.0, duration_s=1.0, max_requests=4, j_pool_floats=1 << 22,
                         d=32, n_stacks=8)
    Jd = W.device_normal(tr.J_pool_floats, tr.J_seed, 0.1)
    pool = serve.RequestPool(tr.x, tr.element, tr.sizes, Jd, tr.J_off)
    model = sorf.Model.from_problem(tr.model)
    alpha = torch.from_numpy(tr.model.alpha).cuda()
    srv = serve.NativeServer(model, alpha, pool, max_batch_atoms=1024, ring_slots=1, idle_timeout_s=0.5)
    lib = srv.lib
    ao = np.ascontiguousarray(pool.atom_ptr[0:2], dtype=np.int64)
    jo = np.ascontiguousarray(pool.J_off[0:1], dtype=np.int64)
    t = ctypes.c_int64()
    assert lib.sorf_server_submit(srv.h, 1, ao.ctypes.data, jo.ctypes.data, ctypes.byref(t)) == 0
    rc = lib.sorf_server_submit(srv.h, 1, ao.ctypes.data, jo.ctypes.data, ctypes.byref(t))
    assert rc in (_lib.SORF_OK, _lib.SORF_ERR_BUSY)
    # invalid batches are refused before anything is published
    bad = np.array([0, 0], dtype=np.int64)
    assert lib.sorf_server_submit(srv.h, 1, bad.ctypes.data, jo.ctypes.data, ctypes.byref(t)) == \
        _lib.SORF_ERR_INVALID_ARG
    assert lib.sorf_server_submit(srv.h, 65, ao.ctypes.data, jo.ctypes.data, ctypes.byref(t)) == \
        _lib.SORF_ERR_INVALID_ARG
    import time
    t0 = time.perf_counter()
    while lib.sorf_server_query(srv.h, 0) == 0 and time.perf_counter() - t0 < 5.0:
        pass
    assert lib.sorf_server_query(srv.h, 0) == 1
    time.sleep(1.5)                      # longer than the idle timeout
    state = srv.stop()
    assert state == 2, state
