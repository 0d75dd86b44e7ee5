"""Host-side tests of the continuous-batching scheduler with a mock executor
and a simulated clock: FIFO contiguous batches, the atom cap, the in-flight
memory budget, rejection of requests that can never fit, and latency
accounting."""
import numpy as np
import pytest

from paper_2206_01580_amd.serve import BatchingScheduler, PlainRunner


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt=1e-5):
        self.t += dt


class MockExecutor:
    """Completes a batch `base + per_atom * atoms` seconds after submission;
    checks the memory budget is never exceeded and slots are never overused."""

    def __init__(self, clock, sizes, bytes_per_atom, budget, max_inflight, base=2e-4, per_atom=1e-6):
        self.clock, self.sizes = clock, np.asarray(sizes)
        self.bpa, self.budget, self.max_inflight = bytes_per_atom, budget, max_inflight
        self.base, self.per_atom = base, per_atom
        self.inflight = []
        self.used = 0
        self.max_used = 0
        self.submitted = []

    def bytes_for(self, first, last):
        return int(self.sizes[first:last].sum()) * self.bpa

    def submit(self, first, last):
        nbytes = self.bytes_for(first, last)
        self.used += nbytes
        assert self.used <= self.budget, "memory budget exceeded"
        self.max_used = max(self.max_used, self.used)
        self.submitted.append((first, last))
        ex = self
        t_done = self.clock() + self.base + self.per_atom * int(self.sizes[first:last].sum())

        class H:
            released = False

            def done(self_h):
                if ex.clock() >= t_done:
                    if not self_h.released:
                        self_h.released = True
                        ex.used -= nbytes
                        ex.inflight.remove(self_h)
                    return True
                return False

        h = H()
        self.inflight.append(h)
        assert len(self.inflight) <= self.max_inflight, "too many batches in flight"
        return h


def make_trace(seed, R=300, rate=4000.0, lo=5, hi=300):
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, R))
    sizes = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), R))).astype(np.int64)
    return arrivals, sizes


@pytest.mark.parametrize("max_atoms,budget,inflight", [(2048, 10 ** 9, 4), (512, 300_000, 2),
                                                        (100_000, 150_000, 3)])
def test_batches_are_fifo_contiguous_and_within_limits(max_atoms, budget, inflight):
    arrivals, sizes = make_trace(1)
    clock = FakeClock()
    ex = MockExecutor(clock, sizes, bytes_per_atom=500, budget=budget, max_inflight=inflight)
    sch = BatchingScheduler(ex, max_batch_atoms=max_atoms, max_inflight=inflight, mem_budget=budget,
                            clock=clock, idle=clock.advance)
    st = sch.run(arrivals, sizes)
    # every request served exactly once, in order, in contiguous runs
    covered = []
    for a, b in st.batches:
        assert b > a
        covered.extend(range(a, b))
    assert covered == list(range(len(sizes)))
    assert st.batches == ex.submitted
    for a, b in st.batches:
        if b - a > 1:
            assert sizes[a:b].sum() <= max_atoms
    assert ex.max_used <= budget
    assert np.all(st.latency_s >= 0) and np.all(np.isfinite(st.latency_s))
    assert st.atoms == int(sizes.sum())


def test_requests_larger_than_budget_are_rejected_not_stalled():
    arrivals = np.array([0.0, 1e-4, 2e-4, 3e-4])
    sizes = np.array([10, 5000, 10, 10])
    clock = FakeClock()
    ex = MockExecutor(clock, sizes, bytes_per_atom=100, budget=100_000, max_inflight=2)
    sch = BatchingScheduler(ex, max_batch_atoms=10_000, max_inflight=2, mem_budget=100_000,
                            clock=clock, idle=clock.advance)
    st = sch.run(arrivals, sizes)
    assert st.rejected == [1]
    assert np.isinf(st.completion_s[1])
    assert np.all(np.isfinite(st.completion_s[[0, 2, 3]]))


def test_batching_beats_serial_launches_under_load():
    # offered load above what one-request-per-launch sustains: batching must cut
    # the tail latency (launch overhead amortised over the batch)
    arrivals, sizes = make_trace(3, R=400, rate=8000.0)
    c1, c2 = FakeClock(), FakeClock()
    ex1 = MockExecutor(c1, sizes, 1, 10 ** 12, 4, base=3e-4, per_atom=2e-7)
    ex2 = MockExecutor(c2, sizes, 1, 10 ** 12, 1, base=3e-4, per_atom=2e-7)
    b = BatchingScheduler(ex1, 4096, 4, 10 ** 12, clock=c1, idle=c1.advance).run(arrivals, sizes)

    p = PlainRunner(ex2, clock=c2, idle=c2.advance).run(arrivals, sizes)
    sb, sp = b.summary(), p.summary()
    assert sb["p99_ms"] < sp["p99_ms"]
    assert sb["p50_ms"] < sp["p50_ms"]
    assert sb["launches"] < sp["launches"]


def test_summary_excludes_warmup():
    arrivals, sizes = make_trace(4, R=100)
    clock = FakeClock()
    ex = MockExecutor(clock, sizes, 1, 10 ** 9, 2)
    st = BatchingScheduler(ex, 1024, 2, 10 ** 9, clock=clock, idle=clock.advance).run(arrivals, sizes)
    s_all = st.summary()
    s_w = st.summary(warmup_s=arrivals[50], arrivals=arrivals)
    assert s_all["requests"] == 100 and s_w["requests"] == int((arrivals >= arrivals[50]).sum())
