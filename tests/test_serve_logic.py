"""Serving loop logic on the CPU (fake backend with a virtual clock):
admission by footprint, slot reuse, continuous batching, latency accounting
and isolation of a failing request."""
import pytest

from paper_1812_07993_amd.serve import FakeBackend, Request, Server, summarize


def reqs(spec):
    return [Request(i, t, p, s, n) for i, (t, p, s, n) in enumerate(spec)]


def test_fifo_admission_and_latency():
    be = FakeBackend(budget=10_000, max_slots=4, cost_per_atom_step=1e-6)
    srv = Server(be, chunk_steps=10, clock=be.clock, sleep=be.sleep)
    r = srv.run(reqs([(0.0, "mixed", 100, 5), (0.0, "mixed", 50, 5), (0.5, "fp64", 20, 5)]))
    assert [x.index for x in r] == [0, 1, 2]
    assert all(x.status == "ok" and x.output["steps"] == x.steps for x in r)
    # request 2 arrives later and runs in its own batch
    assert r[2].admitted >= 0.5
    assert all(x.finished >= x.admitted >= x.arrival for x in r)


def test_budget_gates_admission_and_slots_are_reused():
    # each request needs 6000 bytes; only one fits the 10000-byte budget
    be = FakeBackend(budget=10_000, max_slots=4, bytes_per_atom=1000, cost_per_atom_step=1e-6)
    srv = Server(be, chunk_steps=10, clock=be.clock, sleep=be.sleep)
    r = srv.run(reqs([(0.0, "mixed", 30, 6), (0.0, "mixed", 30, 6), (0.0, "mixed", 30, 6)]))
    assert be.peak_used <= 10_000
    # strictly one after another: each admitted when the previous finished
    assert r[1].admitted >= r[0].finished - 1e-12
    assert r[2].admitted >= r[1].finished - 1e-12
    s = summarize(r)
    assert s["requests"] == 3 and s["p99_s"] >= s["p50_s"]


def test_small_request_passes_a_blocked_large_one():
    be = FakeBackend(budget=10_000, max_slots=8, bytes_per_atom=1000, cost_per_atom_step=1e-6)
    srv = Server(be, chunk_steps=10, clock=be.clock, sleep=be.sleep)
    r = srv.run(reqs([(0.0, "mixed", 100, 6), (0.0, "mixed", 100, 6), (0.0, "mixed", 10, 2)]))
    # the 2-atom request fits beside the first and is not stuck behind the second
    assert r[2].admitted < r[0].finished
    assert r[1].admitted >= r[0].finished - 1e-12


def test_continuous_batching_overlaps_requests():
    be = FakeBackend(budget=100_000, max_slots=4, cost_per_atom_step=1e-6)
    srv = Server(be, chunk_steps=10, clock=be.clock, sleep=be.sleep)
    r = srv.run(reqs([(0.0, "mixed", 200, 10), (0.001, "mixed", 200, 10)]))
    # the second joins while the first runs: total time well below serial time
    serial = 2 * 200 * 10 * 1e-6
    assert max(x.finished for x in r) < 0.8 * serial


def test_failing_request_is_isolated():
    be = FakeBackend(budget=100_000, max_slots=4, fail_indices={1})
    srv = Server(be, chunk_steps=10, clock=be.clock, sleep=be.sleep)
    r = srv.run(reqs([(0.0, "mixed", 20, 5), (0.0, "mixed", 20, 5), (0.0, "fp64", 20, 5)]))
    assert [x.status for x in r] == ["ok", "error", "ok"]
    assert summarize(r)["errors"] == 1


def test_request_larger_than_budget_is_reported():
    be = FakeBackend(budget=1000, max_slots=4, bytes_per_atom=1000)
    srv = Server(be, chunk_steps=10, clock=be.clock, sleep=be.sleep)
    with pytest.raises(RuntimeError):
        srv.run(reqs([(0.0, "mixed", 10, 5)]))


def test_creation_on_worker_threads():
    """With creation on worker threads the same requests all complete, in the
    same admission order constraints."""
    be = FakeBackend(budget=100_000, max_slots=4, cost_per_atom_step=1e-6)
    srv = Server(be, chunk_steps=10, clock=be.clock, sleep=be.sleep, create_workers=2)
    r = srv.run(reqs([(0.0, "mixed", 100, 5), (0.0, "fp64", 50, 5), (0.01, "mixed", 30, 5)]))
    assert [x.status for x in r] == ["ok"] * 3
    assert all(x.output["steps"] == x.steps for x in r)
    assert all(x.finished >= x.admitted >= x.arrival for x in r)
