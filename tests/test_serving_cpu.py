"""Serving scheduler on the CPU with a simulated engine: admission by HBM
footprint, continuous batching at iteration boundaries, plan residency and
eviction, per-request bookkeeping."""
import numpy as np
import pytest

from paper_2402_19364_amd.serve import Request, Server, latency_stats


class FakeDecomp:
    def __init__(self, n, nnz):
        self.n, self.nnz = n, nnz

    def info(self):
        return {"n": self.n, "nnz": self.nnz}


class FakeEvent:
    def __init__(self, t):
        self.t = t


class SimEngine:
    """Virtual clock; a step of a group costs a fixed time plus a share per
    member; results are a deterministic function of the request's own input."""

    def __init__(self, step_time=1.0, per_member=0.25):
        self.plan_fp = {}
        self.now = 0.0
        self.step_time = step_time
        self.per_member = per_member
        self.loaded, self.freed = [], []
        self.batches = []
        self.live_plans = set()

    def clock(self):
        return self.now

    def plan_footprint(self, d):
        return d.nnz * 10

    def load_plan(self, name, d):
        self.loaded.append(name)
        self.live_plans.add(name)
        self.plan_fp[name] = self.plan_footprint(d)
        return name

    def plan_bytes(self, handle):
        return self.plan_fp[handle]

    def free_plan(self, name):
        self.freed.append(name)
        self.live_plans.discard(name)

    def request_footprint(self, d, req):
        return d.n * req.k * 8

    def new_stream(self):
        return object()

    def start(self, plan, req, stream):
        assert plan in self.live_plans
        return {"acc": req.x0.astype(np.float64).copy()}

    def step(self, plan, states, steps, stream):
        assert plan in self.live_plans
        for st, t in zip(states, steps):
            st["acc"] = st["acc"] * 2.0 + t
        self.batches.append((plan, len(states), self.now))
        return FakeEvent(self.now + self.step_time + self.per_member * len(states))

    def query(self, ev):
        return self.now >= ev.t

    def wait_any(self, events):
        self.now = max(self.now, min(e.t for e in events))

    def wait_until(self, t, clock):
        self.now = max(self.now, t)

    def finish(self, plan, st, req, stream):
        req.result = st["acc"]


def expected(x0, iters):
    acc = x0.astype(np.float64)
    for t in range(iters):
        acc = acc * 2.0 + t
    return acc


def make_reqs(spec, rng):
    reqs = []
    for rid, (graph, k, iters, arrival) in enumerate(spec):
        x0 = rng.standard_normal((8, k)).astype(np.float32)
        reqs.append(Request(rid, graph, x0, iters, "f32", arrival))
    return reqs


def server(engine, budget, graphs):
    s = Server(engine, budget, clock=engine.clock)
    for name, d in graphs.items():
        s.register_graph(name, d)
    return s


def test_all_complete_with_own_results_and_batching():
    eng = SimEngine()
    s = server(eng, 10 ** 9, {"g1": FakeDecomp(8, 100), "g2": FakeDecomp(8, 50)})
    rng = np.random.default_rng(0)
    spec = [("g1", 16, 5, 0.0), ("g1", 32, 3, 0.5), ("g2", 16, 4, 0.0), ("g1", 16, 6, 2.2),
            ("g2", 64, 2, 3.0)]
    reqs = make_reqs(spec, rng)
    done = s.run(reqs)
    assert len(done) == len(reqs)
    for r in reqs:
        assert np.array_equal(r.result, expected(r.x0, r.iters))
        assert r.done >= r.admitted >= r.arrival
    # continuous batching: request 3 arrived while request 0 was mid-run and
    # joined its group (a batch of the g1 group had 2+ members)
    assert max(w for p, w, _ in eng.batches if p == "g1") >= 2
    assert reqs[3].admitted < reqs[0].done
    st = latency_stats(done)
    assert st["count"] == 5 and st["p99_ms"] >= st["p50_ms"]


def test_budget_is_never_exceeded_and_fifo_blocks():
    eng = SimEngine()
    d = FakeDecomp(100, 100)           # plan 1000 B; request 100*k*8 B
    s = server(eng, 1000 + 100 * 16 * 8 * 2, {"g": d})
    rng = np.random.default_rng(1)
    spec = [("g", 16, 4, 0.0), ("g", 16, 4, 0.0), ("g", 16, 4, 0.0), ("g", 16, 4, 0.0)]
    reqs = make_reqs(spec, rng)
    s.run(reqs)
    assert s.peak_used <= s.budget
    # only two fit at a time: the third starts after one of the first two ends
    first_done = min(reqs[0].done, reqs[1].done)
    assert reqs[2].admitted >= first_done
    for r in reqs:
        assert np.array_equal(r.result, expected(r.x0, r.iters))


def test_bypass_lets_small_requests_pass_a_blocked_large_one():
    eng = SimEngine()
    d = FakeDecomp(100, 100)
    budget = 1000 + 100 * 64 * 8 + 100 * 16 * 8
    rng = np.random.default_rng(2)
    spec = [("g", 64, 6, 0.0), ("g", 64, 2, 0.1), ("g", 16, 2, 0.2)]
    reqs = make_reqs(spec, rng)
    s = server(eng, budget, {"g": d})
    s.run(reqs, bypass=True)
    assert reqs[2].done < reqs[1].admitted      # the small one passed the blocked one
    reqs2 = make_reqs(spec, np.random.default_rng(2))
    eng2 = SimEngine()
    s2 = server(eng2, budget, {"g": d})
    s2.run(reqs2, bypass=False)
    assert reqs2[2].admitted >= reqs2[1].admitted  # strict arrival order


def test_idle_plans_are_evicted_lru():
    eng = SimEngine()
    graphs = {f"g{i}": FakeDecomp(10, 100) for i in range(3)}  # plan 1000 B each
    budget = 2000 + 10 * 16 * 8
    s = server(eng, budget, graphs)
    rng = np.random.default_rng(3)
    spec = [("g0", 16, 2, 0.0), ("g1", 16, 2, 10.0), ("g2", 16, 2, 20.0), ("g0", 16, 2, 30.0)]
    reqs = make_reqs(spec, rng)
    s.run(reqs)
    assert s.peak_used <= budget
    assert eng.freed[:2] == ["g0", "g1"]
    assert eng.loaded == ["g0", "g1", "g2", "g0"]


def test_request_that_can_never_fit_is_rejected():
    eng = SimEngine()
    s = server(eng, 500, {"g": FakeDecomp(100, 10)})
    with pytest.raises(ValueError):
        s.run(make_reqs([("g", 16, 2, 0.0)], np.random.default_rng(4)))
