"""Serving loop: continuous batching of iterated arrow-SpMM jobs on one GPU.

Requests name a registered graph, an FP32 X_0 (original vertex order), a
feature width k, a storage dtype and an iteration count T.  The server

* keeps decompositions on the host and plans resident on the device (evicting
  idle plans least-recently-used when memory is needed),
* admits waiting requests in arrival order whenever their HBM footprint
  (X/Y buffers, workspace, norm state and, if absent, the plan) fits the
  budget -- requests that arrive while others run join at the next iteration
  boundary of their group,
* batches all active requests of one (graph, dtype) into one product call per
  iteration (one operand per request) on that group's stream; the library runs
  the operands of one tile width as one launch sequence over all their column
  tiles, so the matrix is read once per iteration for the whole group (a wider
  effective k); different groups run on different streams, so their work
  overlaps on the device,
* finishes a request after its T products: X_T = Y_{T-1} / ||Y_{T-1}||_col is
  permuted back to the original order and copied to the host.

Every request's arithmetic depends only on its own operand (the library's work
partition is fixed by the plan and the operand's own k and dtype), so its
result is bitwise the same alone or in any mix.

The scheduling logic talks to an engine object; `GpuEngine` drives libarrow,
and tests can substitute a simulated engine.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    graph: str
    x0: Optional[np.ndarray]  # host FP32, n x k, original order (or None: use x0_seed)
    iters: int
    dtype: str = "f32"
    arrival: float = 0.0      # seconds on the server clock
    width: int = 0            # k when x0 is None
    x0_seed: int = 0          # X_0 ~ N(0, 1) drawn on the device from this seed
    keep_on_device: bool = False  # leave the result as a device tensor
    # filled in by the server
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Optional[object] = None     # X_T, original order (host array or device tensor)
    norms: Optional[np.ndarray] = None  # FP64 [iters, k]

    @property
    def k(self) -> int:
        return int(self.x0.shape[1]) if self.x0 is not None else int(self.width)

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


@dataclasses.dataclass
class _Active:
    req: Request
    state: object
    footprint: int
    step: int = 0


class _Group:
    def __init__(self, key, stream):
        self.key = key
        self.stream = stream
        self.active: List[_Active] = []
        self.inflight: Optional[object] = None   # engine event of the issued step
        self.inflight_members: List[_Active] = []


class Server:
    """Continuous-batching scheduler over an engine (see GpuEngine)."""

    def __init__(self, engine, hbm_budget: int, clock: Callable[[], float] = time.perf_counter):
        self.engine = engine
        self.budget = int(hbm_budget)
        self.clock = clock
        self.graphs: Dict[str, object] = {}
        self.plans: "collections.OrderedDict[str, tuple]" = collections.OrderedDict()
        self.used = 0
        self.groups: Dict[tuple, _Group] = {}
        self.finished: List[Request] = []
        self.peak_used = 0
        self.steps_issued = 0
        self.max_group_width = 0

    # -- registry -----------------------------------------------------------
    def register_graph(self, name: str, decomposition) -> None:
        self.graphs[name] = decomposition

    # -- memory accounting --------------------------------------------------
    def _plan_users(self, graph: str) -> int:
        return sum(len(g.active) for key, g in self.groups.items() if key[0] == graph)

    def _ensure_plan(self, graph: str, extra: int) -> bool:
        """Make the plan of `graph` resident with `extra` more bytes free."""
        if graph in self.plans:
            need = extra
        else:
            need = extra + self.engine.plan_footprint(self.graphs[graph])
        while self.used + need > self.budget:
            idle = [g for g in self.plans if g != graph and self._plan_users(g) == 0]
            if not idle:
                return False
            victim = idle[0]  # least recently used
            _, fp = self.plans.pop(victim)
            self.engine.free_plan(victim)
            self.used -= fp
        if graph not in self.plans:
            handle = self.engine.load_plan(graph, self.graphs[graph])
            # account the plan's actual device bytes (the estimate only gates
            # admission before the plan exists; it is an upper bound)
            fp = self.engine.plan_bytes(handle)
            self.plans[graph] = (handle, fp)
            self.used += fp
        self.plans.move_to_end(graph)
        return True

    def _try_admit(self, req: Request) -> bool:
        fp = self.engine.request_footprint(self.graphs[req.graph], req)
        if fp + (0 if req.graph in self.plans else
                 self.engine.plan_footprint(self.graphs[req.graph])) > self.budget:
            raise ValueError(f"request {req.rid} can never fit the HBM budget")
        if not self._ensure_plan(req.graph, fp):
            return False
        plan = self.plans[req.graph][0]
        key = (req.graph, req.dtype)
        g = self.groups.get(key)
        if g is None:
            g = _Group(key, self.engine.new_stream())
            self.groups[key] = g
        state = self.engine.start(plan, req, g.stream)
        self.used += fp
        self.peak_used = max(self.peak_used, self.used)
        req.admitted = self.clock()
        g.active.append(_Active(req, state, fp))
        return True

    # -- main loop ----------------------------------------------------------
    def run(self, requests: List[Request], bypass: bool = False) -> List[Request]:
        """Serve `requests` (arrival times on this server's clock, relative to
        the call).  Returns them in completion order."""
        t0 = self.clock()
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        for r in pending:
            r.arrival += t0
        waiting: collections.deque = collections.deque()
        done: List[Request] = []
        total = len(pending)
        while len(done) < total:
            progressed = False
            now = self.clock()
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # completions
            for g in self.groups.values():
                if g.inflight is not None and self.engine.query(g.inflight):
                    g.inflight = None
                    for a in g.inflight_members:
                        a.step += 1
                    finished = [a for a in g.inflight_members if a.step >= a.req.iters]
                    for a in finished:
                        g.active.remove(a)
                        self.engine.finish(self.plans[a.req.graph][0], a.state, a.req, g.stream)
                        a.req.done = self.clock()
                        self.used -= a.footprint
                        done.append(a.req)
                    g.inflight_members = []
                    progressed = True
            # admissions (arrival order; with bypass, later requests may pass a
            # blocked one)
            blocked = []
            while waiting:
                r = waiting.popleft()
                if self._try_admit(r):
                    progressed = True
                    continue
                blocked.append(r)
                if not bypass:
                    break
            waiting = collections.deque(blocked + list(waiting))
            # issue one product for every idle group with active requests
            for g in self.groups.values():
                if g.inflight is None and g.active:
                    members = list(g.active)
                    plan = self.plans[g.key[0]][0]
                    g.inflight = self.engine.step(plan, [a.state for a in members],
                                                  [a.step for a in members], g.stream)
                    g.inflight_members = members
                    self.steps_issued += 1
                    self.max_group_width = max(self.max_group_width, len(members))
                    progressed = True
            if not progressed:
                inflight = [g.inflight for g in self.groups.values() if g.inflight is not None]
                if inflight:
                    self.engine.wait_any(inflight)
                elif pending:
                    self.engine.wait_until(pending[0].arrival, self.clock)
                elif waiting:
                    raise RuntimeError("requests are waiting but nothing runs (budget too small)")
        self.finished.extend(done)
        return done


def latency_stats(reqs: List[Request]) -> dict:
    lat = np.array([r.latency for r in reqs if r.latency is not None])
    if lat.size == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "count": int(lat.size)}


# ---------------------------------------------------------------------------
# GPU engine
# ---------------------------------------------------------------------------

class GpuEngine:
    """Engine that runs the products with libarrow on one device."""

    def __init__(self, device: int = 0):
        import torch

        import paper_2402_19364_amd as arrow
        self.torch = torch
        self.arrow = arrow
        self.device = device
        self.dev = torch.device(f"cuda:{device}")
        self._plans: Dict[str, object] = {}
        self._fp: Dict[int, int] = {}
        # plan buffers come from PyTorch's caching allocator (process-wide
        # setting): evicting a plan returns its memory to the pool without a
        # device synchronisation
        arrow.use_torch_allocator()

    # plans
    def plan_footprint(self, decomposition) -> int:
        """Upper bound of a plan's device bytes, before it exists: per entry at
        most a 4-byte column or 2-byte code plus a 6-byte far-table slot and the
        4-byte value; per row the entry and list offsets, the permutation, the
        processing order and a listed partial row."""
        key = id(decomposition)
        if key not in self._fp:
            info = decomposition.info()
            self._fp[key] = int(info["nnz"] * 12 + info["n"] * 24 + (1 << 20))
        return self._fp[key]

    def plan_bytes(self, plan) -> int:
        return int(plan.footprint())

    def load_plan(self, name: str, decomposition):
        plan = self.arrow.Plan(decomposition, self.device)
        self._plans[name] = plan
        return plan

    def free_plan(self, name: str) -> None:
        # only idle plans are evicted: every product that used it has completed
        # (its group's event was observed), so no kernel still reads it
        plan = self._plans.pop(name, None)
        if plan is not None:
            plan.close()

    # requests
    def request_footprint(self, decomposition, req: Request) -> int:
        info = decomposition.info()
        n, k = info["n"], req.k
        es = self.arrow.ELEM_SIZE[self.arrow.DTYPES[req.dtype]]
        ws = n * k * 4  # partial rows + column partials (upper bound used for admission)
        return int(2 * n * k * es + n * k * 4 + ws + (1 << 16))

    def new_stream(self):
        return self.torch.cuda.Stream(device=self.dev)

    def start(self, plan, req: Request, stream):
        torch = self.torch
        arrow = self.arrow
        k = req.k
        scaled = req.dtype in ("f16", "f8e4m3")
        with torch.cuda.stream(stream):
            if req.x0 is not None:
                x0 = torch.from_numpy(np.ascontiguousarray(req.x0, dtype=np.float32)).to(
                    self.dev, non_blocking=False)
            else:
                gen = torch.Generator(device=self.dev)
                gen.manual_seed(int(req.x0_seed))
                x0 = torch.randn((plan.n, k), generator=gen, dtype=torch.float32,
                                 device=self.dev)
            st = {
                "x0": x0,
                "buf": [plan.empty(k, req.dtype) for _ in range(2)],
                "ws_bytes": plan.workspace_size(k, req.dtype),
                "inv": [torch.zeros(k, dtype=torch.float64, device=self.dev) for _ in range(2)],
                "mx": [torch.zeros(k, dtype=torch.float32, device=self.dev) for _ in range(2)],
                "sc": [torch.ones(k, dtype=torch.float32, device=self.dev) for _ in range(2)],
                "norms": torch.zeros((req.iters, k), dtype=torch.float64, device=self.dev),
                "dtype": req.dtype, "scaled": scaled, "iters": req.iters,
            }
            plan.permute_in(st["x0"], st["buf"][0], req.dtype,
                            x_scale=st["sc"][0] if scaled else None,
                            x_maxabs=st["mx"][0] if scaled else None, stream=stream)
            del st["x0"]
        return st

    def step(self, plan, states, steps, stream):
        """One product for every member of a group: one library call, one
        operand per request, on the group's stream."""
        torch = self.torch
        arrow = self.arrow
        ops = []
        total = 0
        for st, t in zip(states, steps):
            src, dst = t % 2, (t + 1) % 2  # ping-pong: input of step t, output of step t
            sc = st["scaled"]
            ops.append(arrow.operand(
                st["buf"][src], st["buf"][dst], st["dtype"],
                x_scale=st["sc"][src] if sc else None,
                x_inv_norm=st["inv"][(t - 1) % 2] if t > 0 else None,
                x_maxabs=st["mx"][src] if sc else None,
                y_scale=st["sc"][dst] if sc else None,
                y_maxabs=st["mx"][dst] if sc else None,
                y_norm=st["norms"][t], y_inv_norm=st["inv"][t % 2]))
            total += st["ws_bytes"]
        with torch.cuda.stream(stream):
            ws = torch.empty(max(total, 256), dtype=torch.uint8, device=self.dev)
            plan.spmm(ops, ws, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev

    def query(self, ev) -> bool:
        return ev.query()

    def wait_until(self, t: float, clock) -> None:
        delay = t - clock()
        if delay > 0:
            time.sleep(min(delay, 0.005))

    def wait_any(self, events) -> None:
        """Return as soon as any of the events has completed (polling, so a
        long step of one group does not hold up the others)."""
        while not any(ev.query() for ev in events):
            time.sleep(20e-6)

    def finish(self, plan, st, req: Request, stream):
        torch = self.torch
        k = req.k
        t = req.iters - 1
        last = st["buf"][(t + 1) % 2]
        out = torch.empty((plan.n, k), dtype=torch.float32, device=self.dev)
        with torch.cuda.stream(stream):
            plan.permute_out(last, out, st["dtype"],
                             x_scale=st["sc"][(t + 1) % 2] if st["scaled"] else None,
                             col_factor=st["inv"][t % 2], stream=stream)
            req.result = out if req.keep_on_device else out.cpu().numpy()
            req.norms = st["norms"].cpu().numpy()
        stream.synchronize()
        st.clear()
