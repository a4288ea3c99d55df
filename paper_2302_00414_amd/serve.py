"""Request loop for weighted adjoint NFFT reconstructions (continuous batching).

Requests name a resident node set (plan + weights) and bring one or more
right-hand sides of samples. The scheduler

* keeps every registered node set resident on the device (its plan: sorted
  nodes, weights, tables);
* admits work by device-memory footprint: a batch runs only if its workspace
  (a clone of the plan with its own workspace) and its input/output buffers fit
  in the memory budget next to what is already resident and in flight;
* batches continuously: whenever a slot (a stream) is free it takes the
  oldest waiting request and every other waiting request of the same node
  set, up to a right-hand-side limit, and runs them as one fused multi-RHS
  adjoint on that slot's stream, so requests that arrive while others run are
  admitted as slots and memory free up and their work overlaps on the device;
* reports, per request, the latency from submission to the moment the result
  is known to be ready, and throughput in nonuniform points per second.

The device work goes through an executor. ``DeviceExecutor`` uses the HIP
library through :mod:`paper_2302_00414_amd.nfft` on PyTorch streams;
``FakeExecutor`` simulates durations and allocation failures on the CPU and
is only a test double for the scheduling logic (it computes nothing).

    python -m paper_2302_00414_amd.serve --qps 2000 --seconds 3
"""
from __future__ import annotations

import argparse
import collections
import concurrent.futures as cf
import json
import math
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional

import numpy as np


# ----------------------------------------------------------------- requests
@dataclass
class Request:
    rid: int
    key: Any
    f: Any                      # (nrhs, N) samples (device tensor for the device executor)
    nrhs: int
    t_submit: float
    future: cf.Future = field(default_factory=cf.Future)
    t_start: float = 0.0
    t_done: float = 0.0
    batch: int = -1             # index of the batch that ran it


@dataclass(frozen=True)
class Done:
    """What the statistics keep of a finished request (not its data or result,
    which belong to the caller once the future is resolved)."""
    key: Any
    nrhs: int
    t_submit: float
    t_done: float
    batch: int


@dataclass
class NodeSet:
    key: Any
    N: int
    M: int
    d: int
    handle: Any                 # executor plan handle
    bytes: int                  # resident bytes (plan + weights)
    idle: List[Any] = field(default_factory=list)   # idle workspaces: (ws, max_rhs, bytes)


@dataclass
class Batch:
    key: Any
    reqs: List[Request]
    ws: Any
    ws_rhs: int
    ws_bytes: int
    io_bytes: int
    slot: int
    token: Any                  # executor completion token


class ServerError(RuntimeError):
    pass


# ---------------------------------------------------------------- executors
class DeviceExecutor:
    """HIP library on one device; one PyTorch stream per slot."""

    def __init__(self, device: str = "cuda:0", precision: str = "f32", tuning=None):
        import torch
        from . import nfft as _nfft
        self.torch = torch
        self.nfft = _nfft
        self.device = torch.device(device)
        self.precision = precision
        self.tuning = tuning  # None (library defaults), a dict, or "auto" (timed per node set)
        self.cdtype = torch.complex64 if precision == "f32" else torch.complex128
        self.streams: Dict[int, Any] = {}

    def stream(self, slot: int):
        if slot not in self.streams:
            with self.torch.cuda.device(self.device):
                self.streams[slot] = self.torch.cuda.Stream(device=self.device)
        return self.streams[slot]

    def create(self, nodes, M, sigma, m, weights):
        plan = self.nfft.Plan(nodes, M, sigma, m, precision=self.precision, max_rhs=1,
                              device=self.device, tuning=self.tuning)
        plan.set_weights(weights)
        info = plan.info()
        return plan, info["bytes"]

    def workspace(self, plan, max_rhs: int):
        ws = plan.clone(max_rhs)
        return ws, ws.info()["workspace_bytes"]

    def io_bytes(self, N: int, M: int, d: int, nrhs: int) -> int:
        c = 8 if self.precision == "f32" else 16
        return (N + M ** d) * nrhs * c

    def launch(self, ws, reqs: List[Request], slot: int):
        torch = self.torch
        s = self.stream(slot)
        cur = torch.cuda.current_stream(self.device)
        s.wait_stream(cur)                       # the requests' inputs are ready on the current stream
        with torch.cuda.stream(s):
            f = reqs[0].f if len(reqs) == 1 else torch.cat([r.f for r in reqs], dim=0)
            nrhs = f.shape[0]
            out = torch.empty((nrhs, ws.M ** ws.d), dtype=self.cdtype, device=self.device)
            ws.adjoint(f, out=out, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        for r in reqs:
            r.f.record_stream(s)
        return (ev, out, f)

    def done(self, token) -> bool:
        return token[0].query()

    def results(self, token, reqs: List[Request]):
        out = token[1]
        res, o = [], 0
        for r in reqs:
            res.append(out[o:o + r.nrhs])
            o += r.nrhs
        return res

    def release(self, ws):
        ws.close()


class FakeExecutor:
    """CPU test double: simulated durations, optional allocation failures."""

    def __init__(self, duration: Callable[[int, int], float] = lambda N, nrhs: 1e-3,
                 fail_alloc: Callable[[int], bool] = lambda nbytes: False,
                 ws_bytes: Callable[[int, int], int] = lambda N, rhs: 1000 * rhs):
        self.duration = duration
        self.fail_alloc = fail_alloc
        self.ws_bytes = ws_bytes
        self.launched: List[dict] = []

    def create(self, nodes, M, sigma, m, weights):
        N = len(nodes)
        return dict(N=N, M=M, d=np.ndim(nodes[0]) if np.ndim(nodes) > 1 else 1), 100 * N

    def workspace(self, plan, max_rhs: int):
        nbytes = self.ws_bytes(plan["N"], max_rhs)
        if self.fail_alloc(nbytes):
            raise ServerError("simulated allocation failure")
        return dict(plan=plan, max_rhs=max_rhs), nbytes

    def io_bytes(self, N, M, d, nrhs):
        return (N + M ** d) * nrhs * 8

    def launch(self, ws, reqs, slot):
        nrhs = sum(r.nrhs for r in reqs)
        t_end = time.perf_counter() + self.duration(ws["plan"]["N"], nrhs)
        self.launched.append(dict(slot=slot, rids=[r.rid for r in reqs], nrhs=nrhs))
        return (t_end, reqs)

    def done(self, token) -> bool:
        return time.perf_counter() >= token[0]

    def results(self, token, reqs):
        return [("result", r.rid) for r in reqs]

    def release(self, ws):
        pass


# ------------------------------------------------------------------- server
class Server:
    """Continuous-batching server over one device.

    hbm_budget    bytes the server may keep allocated (resident plans, live
                  workspaces and in-flight input/output buffers)
    max_slots     concurrent batches (one stream each)
    max_batch_rhs right-hand sides fused into one call
    """

    def __init__(self, hbm_budget: int, max_slots: int = 4, max_batch_rhs: int = 16,
                 executor=None, poll_s: float = 20e-6, batching: bool = True):
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.max_batch_rhs = max_batch_rhs
        self.batching = batching  # False: every request is a batch of its own
        self.ex = executor if executor is not None else DeviceExecutor()
        self.poll_s = poll_s
        self.sets: Dict[Any, NodeSet] = {}
        self.queue: collections.deque = collections.deque()
        self.running: List[Batch] = []
        self.free_slots = list(range(max_slots))
        self.used = 0
        self.lock = threading.Condition()
        self.completed: List[Done] = []
        self.points = 0
        self.rejected = 0
        self.batches = 0
        self._rid = 0
        self._stop = False
        self._thread: Optional[threading.Thread] = None

    # ------------------------------------------------------------ set-up
    def register(self, key, nodes, M: int, sigma: float, m: int, weights) -> None:
        with self.lock:
            if key in self.sets:
                raise ServerError(f"node set {key!r} already registered")
        handle, nbytes = self.ex.create(nodes, M, sigma, m, weights)
        nodes_arr = np.asarray(nodes)
        d = 1 if nodes_arr.ndim == 1 else nodes_arr.shape[1]
        with self.lock:
            if self.used + nbytes > self.budget:
                raise ServerError(f"node set {key!r} needs {nbytes} bytes, "
                                  f"{self.budget - self.used} left in the budget")
            self.used += nbytes
            self.sets[key] = NodeSet(key, len(nodes_arr), M, d, handle, nbytes)

    def start(self) -> "Server":
        self._thread = threading.Thread(target=self._loop, name="nfft-server", daemon=True)
        self._thread.start()
        return self

    def close(self) -> None:
        with self.lock:
            self._stop = True
            self.lock.notify_all()
        if self._thread:
            self._thread.join()
        for ns in self.sets.values():
            for ws, _, _ in ns.idle:
                self.ex.release(ws)
            ns.idle.clear()

    # ----------------------------------------------------------- requests
    def submit(self, key, f, nrhs: Optional[int] = None) -> cf.Future:
        with self.lock:
            if key not in self.sets:
                raise ServerError(f"unknown node set {key!r}")
            self._rid += 1
            n = nrhs if nrhs is not None else (f.shape[0] if getattr(f, "ndim", 1) > 1 else 1)
            if n > self.max_batch_rhs:
                raise ServerError(f"request has {n} right-hand sides, limit {self.max_batch_rhs}")
            r = Request(self._rid, key, f, n, time.perf_counter())
            self.queue.append(r)
            self.lock.notify_all()
            return r.future

    def cancel_pending(self) -> int:
        """Drop every request that has not started; their futures are cancelled."""
        with self.lock:
            n = 0
            while self.queue:
                r = self.queue.popleft()
                r.future.cancel()
                n += 1
            return n

    # ---------------------------------------------------------- scheduler
    def _retire(self) -> bool:
        progressed = False
        for b in list(self.running):
            if not self.ex.done(b.token):
                continue
            t = time.perf_counter()
            res = self.ex.results(b.token, b.reqs)
            for r, v in zip(b.reqs, res):
                r.t_done = t
                self.points += self.sets[r.key].N * r.nrhs
                self.completed.append(Done(r.key, r.nrhs, r.t_submit, t, r.batch))
                r.f = None                     # the samples are the caller's again
                r.future.set_result(v)
            self.running.remove(b)
            self.free_slots.append(b.slot)
            self.used -= b.io_bytes
            self.sets[b.key].idle.append((b.ws, b.ws_rhs, b.ws_bytes))
            progressed = True
        return progressed

    def _take_workspace(self, ns: NodeSet, rhs: int):
        """An idle workspace of this node set with room for `rhs`, or a new
        one within the budget (idle workspaces of other node sets are freed
        first when memory is short). None if it cannot fit now."""
        for i, (ws, wr, wb) in enumerate(ns.idle):
            if wr >= rhs:
                return ns.idle.pop(i)
        want = self.max_batch_rhs
        while True:
            try:
                ws, wb = self.ex.workspace(ns.handle, want)
            except Exception:          # allocation failure: treat as "does not fit now"
                ws = None
            if ws is not None and self.used + wb <= self.budget:
                self.used += wb
                return (ws, want, wb)
            if ws is not None:
                self.ex.release(ws)
            # free idle workspaces elsewhere, largest first, then retry
            if not self._evict_one():
                return None

    def _evict_one(self) -> bool:
        """Free the largest idle workspace of any node set; False if none is idle."""
        victims = sorted(((wb2, k, i) for k, s2 in self.sets.items()
                          for i, (_, _, wb2) in enumerate(s2.idle)), reverse=True)
        if not victims:
            return False
        wb2, k, i = victims[0]
        w2, _, _ = self.sets[k].idle.pop(i)
        self.ex.release(w2)
        self.used -= wb2
        return True

    def _admit(self) -> bool:
        progressed = False
        while self.free_slots and self.queue:
            head = self.queue[0]
            ns = self.sets[head.key]
            # continuous batching: the oldest request and the next ones of the same node set
            group, rhs = [], 0
            for r in self.queue:
                if r.key == head.key and rhs + r.nrhs <= self.max_batch_rhs:
                    group.append(r)
                    rhs += r.nrhs
                    if not self.batching:
                        break
            io = self.ex.io_bytes(ns.N, ns.M, ns.d, rhs)
            # idle workspaces give way to the batch's input and output buffers
            while self.used + io > self.budget and self._evict_one():
                pass
            got = self._take_workspace(ns, rhs) if self.used + io <= self.budget else None
            if got is None:
                if not self.running:
                    # nothing will ever free memory: reject the head request
                    self.queue.popleft()
                    head.future.set_exception(ServerError("request does not fit the memory budget"))
                    self.rejected += 1
                    progressed = True
                    continue
                break
            ws, ws_rhs, ws_bytes = got
            for r in group:
                self.queue.remove(r)
            slot = self.free_slots.pop()
            t = time.perf_counter()
            for r in group:
                r.t_start = t
                r.batch = self.batches
            token = self.ex.launch(ws, group, slot)
            self.batches += 1
            self.used += io
            self.running.append(Batch(head.key, group, ws, ws_rhs, ws_bytes, io, slot, token))
            progressed = True
        return progressed

    def _loop(self) -> None:
        while True:
            with self.lock:
                if self._stop and not self.queue and not self.running:
                    return
                p1 = self._retire()
                p2 = self._admit()
                if not (p1 or p2):
                    if not self.running and not self.queue:
                        self.lock.wait(timeout=0.01)
                        continue
            if not (p1 or p2):
                time.sleep(self.poll_s)

    def drain(self, timeout: float = 60.0) -> None:
        t0 = time.perf_counter()
        while True:
            with self.lock:
                if not self.queue and not self.running:
                    return
            if time.perf_counter() - t0 > timeout:
                raise ServerError("drain timed out")
            time.sleep(1e-4)

    # -------------------------------------------------------------- stats
    def stats(self, since: int = 0) -> dict:
        done = self.completed[since:]
        lat = np.array([r.t_done - r.t_submit for r in done]) * 1e3
        if not len(lat):
            return dict(requests=0)
        span = max(r.t_done for r in done) - min(r.t_submit for r in done)
        pts = sum(self.sets[r.key].N * r.nrhs for r in done)
        return dict(requests=len(done), p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                    points_per_s=pts / span if span > 0 else float("nan"),
                    rejected=self.rejected, batches=len({r.batch for r in done}))


# -------------------------------------------------------------- workload
def make_served_stream(n_sets_per_M=2, Ms=(64, 128, 256, 512), seed=0):
    """Node sets of the served workload: d = 2, N = M^2 u with u ~ U(1, 4),
    uniform or polar nodes (polar: R = 2 ceil(sqrt(N)/2), T = 2 ceil(N/(2R)))."""
    from . import workloads as wl
    rng = np.random.default_rng(seed)
    sets = []
    for M in Ms:
        for s in range(n_sets_per_M):
            u = rng.uniform(1.0, 4.0)
            N = int(round(M * M * u))
            if rng.random() < 0.5:
                x = wl.uniform_nodes(N, 2, int(rng.integers(1 << 30)))
                kind = "uniform"
            else:
                R = 2 * math.ceil(math.sqrt(N) / 2)
                T = 2 * math.ceil(N / (2 * R))
                x = wl.polar_nodes(R, T)
                kind = "polar"
            w = np.full(x.shape[0], 1.0 / x.shape[0], dtype=np.complex128)
            sets.append(dict(key=(M, s), M=M, nodes=x, weights=w, kind=kind))
    return sets


def run_stream(srv: Server, keys, pools, qps: float, seconds: float, rng) -> int:
    """Submit a seeded Poisson stream of requests at `qps` for `seconds`
    (node set uniform over `keys`, 1-16 right-hand sides each, samples taken
    from `pools[key]`), then wait for all of them. Returns the index of the
    first completion record of this stream (for Server.stats)."""
    mark = len(srv.completed)
    n = int(qps * seconds)
    gaps = rng.exponential(1.0 / qps, size=n)
    t_next = time.perf_counter()
    for i in range(n):
        t_next += gaps[i]
        # sleep (releasing the interpreter lock for the scheduler thread)
        # until shortly before the arrival time, then spin
        while True:
            left = t_next - time.perf_counter()
            if left <= 0:
                break
            if left > 3e-4:
                time.sleep(left - 2e-4)
        key = keys[rng.integers(len(keys))]
        nrhs = int(rng.integers(1, 17))
        srv.submit(key, pools[key][:nrhs])
    srv.drain()
    return mark


def saturation_points_per_s(srv: Server, keys, pools, n: int, rng) -> float:
    """Points per second with `n` requests of the stream's mix submitted at
    once (the server's throughput with its queue never empty)."""
    mark = len(srv.completed)
    for _ in range(n):
        key = keys[rng.integers(len(keys))]
        srv.submit(key, pools[key][:int(rng.integers(1, 17))])
    srv.drain()
    return float(srv.stats(mark)["points_per_s"])


def served_setup(precision="f32", slots=4, max_batch_rhs=16, budget_gib=32.0, m=6,
                 sets_per_M=2, Ms=(64, 128, 256, 512), tuning=None, batching=True):
    """A started server with the served workload's node sets registered and
    a pool of device samples per set: (server, keys, pools, sets)."""
    import torch
    ex = DeviceExecutor(precision=precision, tuning=tuning)
    srv = Server(int(budget_gib * (1 << 30)), max_slots=slots, max_batch_rhs=max_batch_rhs,
                 executor=ex, batching=batching).start()
    sets = make_served_stream(sets_per_M, tuple(Ms))
    for s in sets:
        srv.register(s["key"], s["nodes"], s["M"], 2.0, m, s["weights"])
    dev = torch.device("cuda:0")
    cdt = torch.complex64 if precision == "f32" else torch.complex128
    pools = {s["key"]: torch.randn(16, s["nodes"].shape[0], dtype=cdt, device=dev)
             for s in sets}
    return srv, [s["key"] for s in sets], pools, sets


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--qps", type=float, nargs="+", default=[1000.0])
    ap.add_argument("--seconds", type=float, default=2.0)
    ap.add_argument("--warmup-seconds", type=float, default=1.0,
                    help="an untimed stream at the first rate first (first launches, "
                         "workspaces)")
    ap.add_argument("--sets-per-M", type=int, default=2)
    ap.add_argument("--Ms", type=int, nargs="+", default=[64, 128, 256, 512])
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=32.0)
    ap.add_argument("--m", type=int, default=6)
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32")
    ap.add_argument("--max-batch-rhs", type=int, default=16,
                    help="right-hand sides one batch may gather")
    ap.add_argument("--no-batching", action="store_true",
                    help="every request runs as a batch of its own")
    ap.add_argument("--tuning", choices=["default", "auto"], default="default",
                    help="auto: the library autotuner picks each node set's tuning")
    args = ap.parse_args()
    rng = np.random.default_rng(1)
    srv, keys, pools, _ = served_setup(args.precision, args.slots, args.max_batch_rhs,
                                       args.budget_gib, args.m, args.sets_per_M, args.Ms,
                                       "auto" if args.tuning == "auto" else None,
                                       not args.no_batching)
    out = []
    run_stream(srv, keys, pools, args.qps[0], args.warmup_seconds, rng)
    for qps in args.qps:
        mark = run_stream(srv, keys, pools, qps, args.seconds, rng)
        st = srv.stats(mark)
        st["qps"] = qps
        st["precision"] = args.precision
        st["max_batch_rhs"] = args.max_batch_rhs
        st["batching"] = not args.no_batching
        st["slots"] = args.slots
        out.append(st)
        print(json.dumps(st), flush=True)
    srv.close()
    return out


if __name__ == "__main__":
    main()
