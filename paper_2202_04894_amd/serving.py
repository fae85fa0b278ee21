"""Serving loop: continuous batching of matvec requests on one GPU.

A request is a geometry (points, kappa, L, leaf size) and a number of
matvecs with fresh charges, as a GMRES solve of a boundary integral equation
would issue them.  The scheduler:

  * keeps plans (tree, lists, spectra) resident per geometry id and reuses
    them (LRU eviction of plans no request is using);
  * admits arrived requests in arrival order while a slot is free and their
    HBM footprint (workspace, plus the plan when it is not cached) fits the
    budget; requests that arrive while others run are admitted as soon as
    slots and memory free up;
  * gives each admitted request its own workspace and stream, so the work of
    concurrent requests overlaps on the device;
  * isolates failures: a request whose plan cannot be built (bad input,
    out of memory) fails alone.

The scheduler knows nothing of the device: it drives an executor.
`DeviceExecutor` runs requests through the library; the tests also drive the
scheduler with a simulated executor on the CPU.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    geometry: str                         # plan-cache key: same key, same points and parameters
    make_points: Callable[[], np.ndarray]  # (n, 3) float64
    n_points: int
    kappa: float
    order_L: int = 5
    ncrit: int = 64
    n_matvecs: int = 20
    charges: Optional[Callable[[int], np.ndarray]] = None  # k -> (n,) complex charges of matvec k
    arrival: float = 0.0                  # seconds after the start of the run
    # a solve instead of a fixed number of matvecs: GMRES on alpha x + G (w x) = b
    # with keys alpha, weight (w, the same for every point), tol, restart,
    # maxiter, seed (of the complex N(0,1) right-hand side); the number of
    # matvecs is whatever the solve needs
    solve: Optional[dict] = None
    knobs: tuple = (1.0, 2.0, 0)          # (eta, hf_threshold, dir_refine) of the plan


@dataclasses.dataclass
class Outcome:
    rid: int
    ok: bool
    error: str = ""
    arrival: float = 0.0
    admitted: float = float("nan")
    done: float = float("nan")
    plan_cached: bool = False
    matvec_ms: list = dataclasses.field(default_factory=list)
    results: Optional[list] = None        # potentials per matvec (host), when kept; a solve: [x]
    info: dict = dataclasses.field(default_factory=dict)  # a solve: iterations, matvecs, residual, converged

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """Admission, plan cache and bookkeeping over an executor.

    executor interface:
      now() -> float                       seconds on the executor's clock
      idle(dt)                             wait up to dt seconds (no work to admit)
      estimate(req) -> (plan_bytes, ws_bytes)   before the plan exists
      build(req) -> (plan, plan_bytes, ws_bytes) may raise: the request fails
      start(req, plan) -> handle           enqueue the request's matvecs (reusing a
                                           workspace the plan's last request left)
      done(handle) -> bool
      finish(handle) -> (done_time, matvec_ms, results[, info]); the workspace is kept
      release_plan(plan)                   frees the plan and its kept workspaces
    """

    def __init__(self, executor, budget_bytes: int, max_slots: int = 8, keep_results: bool = False):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.keep_results = keep_results
        # geometry -> [plan, plan_bytes, ws_bytes, users, pooled]: a finished
        # request's workspace stays with its plan (pooled, still charged) and
        # serves the next request of that geometry; eviction frees both
        self.plans = collections.OrderedDict()
        self.used = 0
        self.stats = dict(builds=0, cache_hits=0, evictions=0, failed=0, max_running=0, peak_bytes=0)

    def _evict_for(self, need: int, keep: str) -> bool:
        for key in list(self.plans):
            if self.used + need <= self.budget:
                break
            ent = self.plans[key]
            if ent[3] == 0 and key != keep:
                self.ex.release_plan(ent[0])
                self.used -= ent[1] + ent[4] * ent[2]
                del self.plans[key]
                self.stats["evictions"] += 1
        return self.used + need <= self.budget

    def run(self, requests) -> list:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        running = {}  # rid -> (req, handle, ws_bytes, outcome)
        outcomes = {}
        t0 = self.ex.now()
        while pending or queue or running:
            now = self.ex.now() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            progressed = False
            for rid in list(running):
                req, h, wsb, oc = running[rid]
                if self.ex.done(h):
                    fin = self.ex.finish(h)
                    done, ms, res = fin[:3]
                    oc.done = done - t0
                    oc.matvec_ms = ms
                    oc.results = res if self.keep_results else None
                    if len(fin) > 3:
                        oc.info = fin[3]
                    ent = self.plans[req.geometry]
                    ent[3] -= 1
                    ent[4] += 1
                    outcomes[rid] = oc
                    del running[rid]
                    progressed = True
            while queue and len(running) < self.max_slots:
                req = queue[0]
                ent = self.plans.get(req.geometry)
                if ent is not None:
                    need = 0 if ent[4] > 0 else ent[2]
                else:
                    pb, wb = self.ex.estimate(req)
                    need = pb + wb
                if self.used + need > self.budget and not self._evict_for(need, req.geometry):
                    if running:
                        break  # wait for memory to free up
                    if ent is not None:
                        # nothing runs and every other plan is gone: can never fit
                        queue.popleft()
                        outcomes[req.rid] = Outcome(req.rid, False, "footprint exceeds the memory budget",
                                                    arrival=req.arrival)
                        self.stats["failed"] += 1
                        progressed = True
                        continue
                    # the device is idle: build, and let the real footprint decide
                queue.popleft()
                oc = Outcome(req.rid, True, arrival=req.arrival, admitted=self.ex.now() - t0)
                if ent is None:
                    try:
                        plan, pb, wb = self.ex.build(req)
                    except Exception as e:  # the request fails alone
                        oc.ok = False
                        oc.error = f"{type(e).__name__}: {e}"
                        outcomes[req.rid] = oc
                        self.stats["failed"] += 1
                        progressed = True
                        continue
                    ent = self.plans[req.geometry] = [plan, pb, wb, 0, 0]
                    self.used += pb
                    self.stats["builds"] += 1
                    if pb + wb > self.budget:
                        self.ex.release_plan(plan)
                        self.used -= pb
                        del self.plans[req.geometry]
                        oc.ok = False
                        oc.error = "footprint exceeds the memory budget"
                        outcomes[req.rid] = oc
                        self.stats["failed"] += 1
                        progressed = True
                        continue
                    if self.used + wb > self.budget and not self._evict_for(wb, req.geometry):
                        # the estimate was low: wait for memory, the plan stays cached
                        queue.appendleft(req)
                        progressed = True
                        break
                else:
                    self.plans.move_to_end(req.geometry)
                    oc.plan_cached = True
                    self.stats["cache_hits"] += 1
                ent[3] += 1
                pooled = ent[4] > 0
                if pooled:
                    ent[4] -= 1
                else:
                    self.used += ent[2]
                try:
                    h = self.ex.start(req, ent[0])
                except Exception as e:
                    ent[3] -= 1
                    if pooled:
                        ent[4] += 1
                    else:
                        self.used -= ent[2]
                    oc.ok = False
                    oc.error = f"{type(e).__name__}: {e}"
                    outcomes[req.rid] = oc
                    self.stats["failed"] += 1
                    progressed = True
                    continue
                running[req.rid] = (req, h, ent[2], oc)
                self.stats["max_running"] = max(self.stats["max_running"], len(running))
                self.stats["peak_bytes"] = max(self.stats["peak_bytes"], self.used)
                progressed = True
            if not progressed:
                nxt = pending[0].arrival - now if pending else 1e-3
                self.ex.idle(min(max(nxt, 0.0), 1e-3))
        for ent in self.plans.values():
            self.ex.release_plan(ent[0])
        self.plans.clear()
        self.used = 0
        return [outcomes[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


class DeviceExecutor:
    """Runs requests through the library, complex64, on the current GPU.

    Each started request gets a workspace (reused from the plan's pool when
    possible) and a stream (default priority).  Its matvecs are enqueued at
    once, with a HIP event pair around each, which give the per-matvec
    latencies (contention with other requests included) and the completion
    time on the host clock.
    """

    def __init__(self, plan_bytes_per_point: float = 1024.0, ws_bytes_per_point: float = 2048.0,
                 keep_results: bool = False, graphs: bool = False):
        import torch
        from . import defmm
        self.torch, self.defmm = torch, defmm
        # per-point footprint estimates for plans not built yet; raised to the
        # largest ratio seen on built plans (plan creation also needs
        # transient builder memory of the same order)
        self.plan_bpp = plan_bytes_per_point
        self.ws_bpp = ws_bytes_per_point
        self.keep_results = keep_results
        # Replaying each workspace's captured HIP graph on fixed buffers
        # (defmm_matvec_graph) inside this executor ended once in a host
        # segmentation fault whose cause is not known: the path stays closed.
        if graphs:
            raise NotImplementedError("graph replay in the serving executor is disabled: a run of it ended in "
                                      "a host segmentation fault whose cause has not been found")
        self.graphs = False
        self.pool = {}  # id(plan) -> idle (workspace, charge buffer, potential buffer) of that plan
        self.active_solves = 0
        self.build_stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record()
        self.ref.synchronize()
        self.t_ref = time.perf_counter()

    def now(self):
        return time.perf_counter()

    def idle(self, dt):
        # a running solve needs the host between its steps: poll more often
        time.sleep(min(dt, 5e-5) if self.active_solves else dt)

    def estimate(self, req):
        return int(self.plan_bpp * req.n_points), int(self.ws_bpp * req.n_points)

    def build(self, req):
        torch, defmm = self.torch, self.defmm
        X = torch.as_tensor(np.ascontiguousarray(req.make_points(), dtype=np.float64), device="cuda")
        eta, hf, e0 = req.knobs
        prm = defmm.Params(order_L=req.order_L, ncrit=req.ncrit, eta=eta, hf_threshold=hf, dir_refine=e0,
                           precision=defmm.C64)
        plan = defmm.Plan(X, None, req.kappa, prm, stream=self.build_stream)
        self.build_stream.synchronize()
        pb, wb = plan.footprint()
        wb += 8 * (plan.nx + plan.ny)  # the workspace's charge and potential buffers
        n = max(req.n_points, 1)
        self.plan_bpp = max(self.plan_bpp, pb / n)
        self.ws_bpp = max(self.ws_bpp, wb / n)
        return plan, pb, wb

    def start(self, req, plan):
        torch, defmm = self.torch, self.defmm
        s = torch.cuda.Stream()
        pool = self.pool.setdefault(id(plan), [])
        with torch.cuda.stream(s):
            if pool:
                ws, qbuf, pbuf = pool.pop()
            else:
                ws = defmm.Workspace(plan)
                qbuf = pbuf = None
                if self.graphs:
                    qbuf = torch.empty(plan.ny, dtype=torch.complex64, device="cuda")
                    pbuf = torch.empty(plan.nx, dtype=torch.complex64, device="cuda")
            if req.solve is not None:
                return self._start_solve(req, plan, s, ws, qbuf, pbuf)
            qs = []
            if req.charges is not None:
                for k in range(req.n_matvecs):
                    q = torch.from_numpy(np.ascontiguousarray(req.charges(k), dtype=np.complex64)).pin_memory()
                    qs.append(q.to("cuda", non_blocking=True))
            else:
                # seeded complex normal charges drawn on the device
                g = torch.Generator(device="cuda")
                g.manual_seed(1_000_003 * (req.rid + 1))
                for k in range(req.n_matvecs):
                    qs.append(torch.randn(req.n_points, dtype=torch.complex64, device="cuda", generator=g))
            ps, evs = [], []
            for k in range(req.n_matvecs):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s)
                if self.graphs:
                    # the workspace's captured matvec on its fixed buffers
                    qbuf.copy_(qs[k])
                    ws.matvec(qbuf, pbuf, stream=s, graph=True)
                    p = pbuf.clone() if self.keep_results else pbuf
                else:
                    p = ws.matvec(qs[k], stream=s)
                e1.record(s)
                if self.keep_results:
                    ps.append(p)
                evs.append((e0, e1))
        return dict(s=s, ws=ws, bufs=(qbuf, pbuf), qs=qs, ps=ps, evs=evs)

    def _start_solve(self, req, plan, s, ws, qbuf, pbuf):
        """A GMRES solve of alpha x + G (w x) = b on the request's stream: the
        stepper enqueues work and is advanced from done() whenever its last
        step has finished, so solves interleave with the other requests."""
        torch = self.torch
        from . import solve as SV
        sp = req.solve
        g = torch.Generator(device="cuda")
        g.manual_seed(int(sp.get("seed", 1_000_003 * (req.rid + 1))))
        b = torch.randn(req.n_points, dtype=torch.complex64, device="cuda", generator=g)
        op = SV.SecondKindOperator(ws, complex(sp.get("alpha", 0.5)),
                                   weights=np.full(req.n_points, float(sp.get("weight", 1.0))), stream=s)
        e0 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        st = SV.GmresStepper(op, b, tol=float(sp.get("tol", 1e-4)), restart=int(sp.get("restart", 30)),
                             maxiter=int(sp.get("maxiter", 100)), stream=s, timed=True)
        self.active_solves += 1
        return dict(s=s, ws=ws, bufs=(qbuf, pbuf), solve=st, op=op, b=b, e0=e0, evs=[])

    def done(self, h):
        st = h.get("solve")
        if st is not None:
            while not st.finished and st.ready():
                st.advance()
            return st.finished
        return h["evs"][-1][1].query() if h["evs"] else True

    def finish(self, h):
        st = h.get("solve")
        if st is not None:
            st.event.synchronize()
            done = self.t_ref + self.ref.elapsed_time(st.event) / 1e3
            r = st.result()
            info = dict(iterations=r.iterations, matvecs=h["op"].matvecs, converged=r.converged,
                        residual=float(r.residuals[-1]) if r.residuals else None,
                        solve_ms=h["e0"].elapsed_time(st.event))
            res = [r.x.cpu().numpy(), h["b"].cpu().numpy()] if self.keep_results else None
            self.pool.setdefault(id(h["ws"].plan), []).append((h["ws"], *h["bufs"]))
            h.clear()
            self.active_solves -= 1
            return done, [], res, info
        h["evs"][-1][1].synchronize() if h["evs"] else h["s"].synchronize()
        ms = [a.elapsed_time(b) for a, b in h["evs"]]
        done = self.t_ref + (self.ref.elapsed_time(h["evs"][-1][1]) / 1e3 if h["evs"] else 0.0)
        res = [p.cpu().numpy() for p in h["ps"]] if self.keep_results else None
        # keep the workspace (and its buffers and captured graph) for the
        # plan's next request: freeing device memory synchronises the whole
        # device, which would stall the other requests
        self.pool.setdefault(id(h["ws"].plan), []).append((h["ws"], *h["bufs"]))
        h.clear()
        return done, ms, res

    def release_plan(self, plan):
        for ws, _, _ in self.pool.pop(id(plan), []):
            ws.close()
        plan.close()


# Knob settings (eta, hf_threshold, dir_refine) per interpolation order and
# kappa*D band whose potentials came within 1e-4 of the FP64 direct sum in
# device and oracle sweeps: L = 5 on 1,048,576 sphere points at kappa*D = 256
# (8.4e-5 at eta = 0.35; 0.3 keeps a margin for the mix); L = 4 on 8,192
# sphere points at kappa*D = 32 (4.8e-5 at E0 = 1, run with one refinement
# more) and, for kappa*D >= 96, on the mix's L = 4 geometries at kappa*D
# 234-251, where eta = 0.15 left 6.8e-5 to 1.15e-4 and eta = 0.1 gives
# 2.9e-5 to 4.0e-5.  The paper-literal setting is (1, 2, 0).
ACCURATE_KNOBS = {4: (0.15, 0.75, 2), 5: (0.3, 0.75, 1)}
ACCURATE_KNOBS_HIGH_KD = {4: (0.1, 0.75, 2), 5: (0.3, 0.75, 1)}
HIGH_KD = 96.0


def accurate_knobs(L, kappa_d):
    """The per-request setting within 1e-4 of the direct sum for order L at kappa*D."""
    return (ACCURATE_KNOBS_HIGH_KD if kappa_d >= HIGH_KD else ACCURATE_KNOBS)[L]


LITERAL_KNOBS = (1.0, 2.0, 0)


def config_requests(n_requests=256, n_geometries=32, seed=7, n_min=10_000, n_max=500_000, kd=(16.0, 256.0),
                    orders=(4, 5), n_matvecs=20, rate=None, host_charges=False, accurate=True):
    """Requests with the shapes of the serving configuration: N log-uniform in
    [n_min, n_max] on the unit sphere or the cap-weighted ellipsoid (50/50),
    kappa*D uniform in kd, L drawn from orders, leaves <= 64, fresh complex
    N(0,1) charges per matvec; geometries drawn from a pool of n_geometries
    (a request reuses its geometry's plan when it is cached); Poisson arrivals
    at `rate` per second (None: all at time 0).  Charges come from numpy
    (host_charges) or are drawn on the device from a per-request seed."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    pool = []
    for g in range(n_geometries):
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        kind = "sphere" if rng.uniform() < 0.5 else "ellipsoid"
        kD = float(rng.uniform(*kd))
        L = int(rng.choice(orders))
        pool.append((n, kind, kD, L, 5000 + g))
    t = 0.0
    reqs = []
    for i in range(n_requests):
        n, kind, kD, L, gseed = pool[int(rng.integers(n_geometries))]
        if rate:
            t += float(rng.exponential(1.0 / rate))
        cseed = 9000 + 1000 * i

        def mk(n=n, kind=kind, gseed=gseed):
            return W.GENERATORS[kind](n, gseed)

        def ch(k, n=n, cseed=cseed):
            return W.charges(n, cseed + k, np.complex64)

        knobs = accurate_knobs(L, kD) if accurate else LITERAL_KNOBS
        reqs.append(Request(rid=i, geometry=f"{kind}-{n}-{kD:.3f}-{L}-{knobs}", make_points=mk, n_points=n,
                            kappa=kD / 2.0, order_L=L, ncrit=64, n_matvecs=n_matvecs,
                            charges=ch if host_charges else None, arrival=t, knobs=knobs))
    return reqs


# Surface areas of the two serving geometries (unit sphere; the (1, 0.5, 0.25)
# ellipsoid, by Thomsen's approximation), for equal-area quadrature weights.
SURFACE_AREA = {"sphere": 4.0 * np.pi, "ellipsoid": 3.975}


def solve_requests(n_requests=32, n_geometries=32, seed=7, rate=None, alpha=0.5, tol=1e-4, restart=30,
                   maxiter=100, **kw):
    """Solve requests on the geometries of config_requests (same pool, same
    seed): GMRES on alpha x + G (w x) = b with equal-area weights w and a
    seeded complex N(0,1) right-hand side, to a relative residual of tol; each
    needs a data-dependent number of matvecs."""
    reqs = config_requests(n_requests=n_requests, n_geometries=n_geometries, seed=seed, rate=rate, **kw)
    for r in reqs:
        kind = r.geometry.split("-")[0]
        r.solve = dict(alpha=alpha, weight=SURFACE_AREA[kind] / r.n_points, tol=tol, restart=restart,
                       maxiter=maxiter, seed=7_000_003 * (r.rid + 1))
        r.n_matvecs = 0
    return reqs


def summarize(outcomes, wall_s):
    ok = [o for o in outcomes if o.ok]
    mv = np.array([m for o in ok for m in o.matvec_ms]) if any(o.matvec_ms for o in ok) else np.zeros(1)
    lat = np.array([o.latency for o in ok]) if ok else np.zeros(1)
    return dict(requests=len(outcomes), completed=len(ok), failed=len(outcomes) - len(ok),
                wall_s=round(wall_s, 3),
                matvec_p50_ms=round(float(np.percentile(mv, 50)), 3),
                matvec_p99_ms=round(float(np.percentile(mv, 99)), 3),
                request_p50_s=round(float(np.percentile(lat, 50)), 4),
                request_p99_s=round(float(np.percentile(lat, 99)), 4))
