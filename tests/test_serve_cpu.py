"""Scheduling logic of the request loop, on the CPU with a test double that
simulates durations and allocation failures (it computes nothing)."""
import time

import numpy as np
import pytest

from paper_2302_00414_amd.serve import FakeExecutor, Server, ServerError


def _server(budget=10**9, slots=2, max_rhs=16, **kw):
    ex = FakeExecutor(**kw)
    srv = Server(budget, max_slots=slots, max_batch_rhs=max_rhs, executor=ex)
    return srv, ex


def _nodes(n):
    return np.zeros((n, 2))


def test_requests_complete_and_stats():
    srv, ex = _server()
    srv.register("a", _nodes(100), 8, 2.0, 4, None)
    srv.start()
    futs = [srv.submit("a", None, nrhs=2) for _ in range(5)]
    for f in futs:
        assert f.result(timeout=5)[0] == "result"
    srv.drain()
    st = srv.stats()
    assert st["requests"] == 5 and st["p99_ms"] >= st["p50_ms"] > 0
    assert st["points_per_s"] > 0
    srv.close()


def test_continuous_batching_groups_same_node_set():
    """Requests that arrive while a batch runs are fused into the next batch of
    their node set, up to the right-hand-side limit, oldest first."""
    srv, ex = _server(slots=1, max_rhs=8, duration=lambda N, r: 0.05)
    srv.register("a", _nodes(10), 8, 2.0, 4, None)
    srv.register("b", _nodes(10), 8, 2.0, 4, None)
    srv.start()
    f0 = srv.submit("a", None, nrhs=1)
    time.sleep(0.01)                       # the first batch is running
    fs = [srv.submit("a", None, nrhs=3), srv.submit("b", None, nrhs=1),
          srv.submit("a", None, nrhs=3), srv.submit("a", None, nrhs=3)]
    for f in [f0] + fs:
        f.result(timeout=5)
    srv.close()
    groups = [l["rids"] for l in ex.launched]
    assert groups[0] == [1]
    assert groups[1] == [2, 4]             # a: 3 + 3 <= 8; the third a (3) would exceed 8
    assert groups[2] == [3]                # then b (now the oldest)
    assert groups[3] == [5]
    assert all(l["nrhs"] <= 8 for l in ex.launched)


def test_slots_overlap():
    srv, ex = _server(slots=3, duration=lambda N, r: 0.05)
    for k in "abc":
        srv.register(k, _nodes(10), 8, 2.0, 4, None)
    srv.start()
    t0 = time.perf_counter()
    fs = [srv.submit(k, None, nrhs=1) for k in "abc"]
    for f in fs:
        f.result(timeout=5)
    assert time.perf_counter() - t0 < 0.12   # three batches ran concurrently
    assert len({l["slot"] for l in ex.launched}) == 3
    srv.close()


def test_admission_by_footprint_rejects_what_never_fits():
    # plan bytes 100*N = 1000; workspace 10^6 per rhs is over any budget left
    srv, ex = _server(budget=5000, ws_bytes=lambda N, r: 10**6)
    srv.register("a", _nodes(10), 8, 2.0, 4, None)
    srv.start()
    f = srv.submit("a", None, nrhs=1)
    with pytest.raises(ServerError):
        f.result(timeout=5)
    srv.close()
    assert srv.rejected == 1


def test_registration_over_budget_is_refused():
    srv, _ = _server(budget=500)
    with pytest.raises(ServerError):
        srv.register("a", _nodes(10), 8, 2.0, 4, None)


def test_allocation_failure_is_reported_not_fatal():
    fail = {"on": True}
    srv, ex = _server(fail_alloc=lambda nbytes: fail["on"])
    srv.register("a", _nodes(10), 8, 2.0, 4, None)
    srv.start()
    with pytest.raises(ServerError):
        srv.submit("a", None, nrhs=1).result(timeout=5)
    fail["on"] = False
    assert srv.submit("a", None, nrhs=1).result(timeout=5)[0] == "result"
    srv.close()


def test_memory_is_reused_across_node_sets():
    """With room for one workspace only, idle workspaces of other node sets are
    freed to admit the next batch instead of rejecting it."""
    srv, ex = _server(budget=2000 + 16 * 1000 + 200000, slots=1,
                      ws_bytes=lambda N, r: 1000 * r)
    srv.register("a", _nodes(10), 8, 2.0, 4, None)
    srv.register("b", _nodes(10), 8, 2.0, 4, None)
    srv.start()
    for k in "abab":
        srv.submit(k, None, nrhs=1).result(timeout=5)
    srv.close()
    assert srv.rejected == 0 and len(ex.launched) == 4


def test_cancel_pending():
    srv, ex = _server(slots=1, duration=lambda N, r: 0.1)
    srv.register("a", _nodes(10), 8, 2.0, 4, None)
    srv.register("b", _nodes(10), 8, 2.0, 4, None)
    srv.start()
    first = srv.submit("a", None, nrhs=1)
    time.sleep(0.02)
    later = [srv.submit("b", None, nrhs=1) for _ in range(3)]
    assert srv.cancel_pending() == 3
    assert all(f.cancelled() for f in later)
    first.result(timeout=5)
    srv.close()


def test_unknown_node_set_and_oversized_request():
    srv, _ = _server(max_rhs=4)
    srv.register("a", _nodes(10), 8, 2.0, 4, None)
    with pytest.raises(ServerError):
        srv.submit("zz", None, nrhs=1)
    with pytest.raises(ServerError):
        srv.submit("a", None, nrhs=5)


def test_no_batching_runs_each_request_alone():
    srv, ex = _server(slots=1, max_rhs=16, duration=lambda N, r: 0.02)
    srv = Server(10**9, max_slots=1, max_batch_rhs=16, executor=ex, batching=False)
    srv.register("a", _nodes(100), 8, 2.0, 4, None)
    srv.start()
    futs = [srv.submit("a", None, nrhs=2) for _ in range(6)]
    for fu in futs:
        fu.result(timeout=5)
    srv.drain()
    assert srv.batches == 6
    srv.close()


def test_finished_requests_release_their_data():
    """The server keeps statistics of finished requests, not their samples or
    results: once the caller drops a future, its result can be freed (a long
    request stream must not accumulate device memory)."""
    import gc
    import weakref

    class Res:
        pass

    class Ex(FakeExecutor):
        def results(self, token, reqs):
            return [Res() for _ in reqs]

    srv = Server(10**9, max_slots=2, max_batch_rhs=16, executor=Ex())
    srv.register("a", _nodes(10), 8, 2.0, 4, None)
    srv.start()
    sample = Res()
    fut = srv.submit("a", sample, nrhs=1)
    res_ref, sample_ref = weakref.ref(fut.result(timeout=5)), weakref.ref(sample)
    srv.drain()
    del fut, sample
    gc.collect()
    assert res_ref() is None and sample_ref() is None
    st = srv.stats()
    assert st["requests"] == 1 and st["p50_ms"] > 0
    srv.close()


def test_io_buffers_evict_idle_workspaces():
    """A batch whose input/output buffers fit only once idle workspaces are
    freed is admitted after freeing them, not left waiting forever."""
    # workspaces 100 * N * 16: a (N = 10) 16000, b (N = 5) 8000; plans 1000 + 500;
    # io (N + 64) * 8 * nrhs: a with 1 rhs 592, b with 16 rhs 8832.
    # a runs (1500 + 16000 + 592 <= 20000); b's io fits only without a's idle
    # workspace (1500 + 16000 + 8832 > 20000), and with b's own workspace it
    # does (1500 + 8832 + 8000 <= 20000)
    srv, ex = _server(budget=20000, slots=1, ws_bytes=lambda N, r: 100 * N * r)
    srv.register("a", _nodes(10), 8, 2.0, 4, None)
    srv.register("b", _nodes(5), 8, 2.0, 4, None)
    srv.start()
    srv.submit("a", None, nrhs=1).result(timeout=5)   # a's workspace is now idle
    srv.submit("b", None, nrhs=16).result(timeout=5)
    srv.drain(timeout=5)
    assert srv.rejected == 0 and len(ex.launched) == 2
    srv.close()


def test_io_alone_over_budget_is_rejected():
    """Input/output buffers larger than the whole budget: the request is
    rejected once nothing runs, and draining ends."""
    srv, ex = _server(budget=1000 + 500, ws_bytes=lambda N, r: 10)
    srv.register("a", _nodes(10), 8, 2.0, 4, None)   # plan 1000; io = 592 * 16 > 500
    srv.start()
    f = srv.submit("a", None, nrhs=16)
    with pytest.raises(ServerError):
        f.result(timeout=5)
    srv.drain(timeout=5)
    assert srv.rejected == 1
    srv.close()
