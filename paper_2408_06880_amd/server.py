"""Continuous-batching server for permeability solves.

Requests (a seeded sphere packing, its size, porosity and relaxation time)
arrive over time.  The server admits them while the device-memory budget
allows, keeps every admitted solve resident in HBM, and advances all active
solves together: one batched launch per AA half-step over the concatenated
fluid lists (`lbm_step_batch`), K steps per round, then one deterministic FP64
reduction per solve (`lbm_reduce_batch`).  A solve retires when its
mean-momentum residual r(n) = |J_x(n) - J_x(n-K)| / |J_x(n)| drops below the
tolerance (or it hits its step cap); its memory is freed and queued requests
are admitted at the next round boundary.  Rounds are K steps long with K even,
so every solve is at even parity when it joins or leaves the batch.

The permeability follows Darcy's law with a body force,
k = nu * <rho u_x> / F_x over the whole box (nu = (tau - 1/2)/3, lattice
units).

Backends: `GpuStepper` drives liblbm; `MockStepper` is a host-only stand-in
with a modelled cost and convergence for testing the scheduler without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the trace starts
    L: int                  # box edge (periodic cube)
    phi: float              # target porosity
    seed: int               # geometry seed
    tau: float              # relaxation time
    force: float = 1e-6     # body force along x


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    steps: int = 0
    n_fluid: int = 0
    permeability: float = math.nan
    residual: float = math.nan
    converged: bool = False
    refined_at: int = 0          # step at which the solve moved to finer storage
    error: str = ""

    @property
    def latency(self):
        return self.finished - self.arrival


def make_trace(n, rate_hz, seed=31, L_range=(64, 384), phi_range=(0.3, 0.9),
               tau_range=(0.6, 1.0), L_step=8):
    """Poisson arrivals (exponential gaps, mean 1/rate) and uniformly drawn
    request parameters, all from one seeded generator."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        L = int(rng.integers(L_range[0] // L_step, L_range[1] // L_step + 1)) * L_step
        out.append(Request(rid=i, arrival=t, L=L, phi=float(rng.uniform(*phi_range)),
                           seed=1000 + i, tau=float(rng.uniform(*tau_range))))
    return out


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return math.nan
    k = (len(xs) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


class Server:
    def __init__(self, stepper, budget_bytes, K=100, tol=1e-6, max_steps=200_000,
                 max_active=64, target_cells=None, clock=time.perf_counter, sleep=time.sleep,
                 on_finish=None, refine_tol=None):
        """target_cells: admit new solves only while the active fluid cells
        stay below this (one solve is always admitted).  Enough cells to
        saturate the GPU keep throughput, fewer concurrent solves finish
        sooner; None admits whatever the memory budget allows.  on_finish:
        called with each Result as its request retires.  refine_tol: once a
        solve's residual drops below it, the stepper's refine() may move the
        solve to finer storage (16-bit storage can stall near the steady
        state when per-step changes fall below its resolution); the residual
        history restarts and the solve then runs to tol."""
        if K <= 0 or K % 2:
            raise ValueError("K must be a positive even number of steps")
        self.stepper = stepper
        self.budget = int(budget_bytes)
        self.K = K
        self.tol = tol
        self.max_steps = max_steps
        self.max_active = max_active
        self.target_cells = target_cells
        self.clock = clock
        self.sleep = sleep
        self.on_finish = on_finish
        self.refine_tol = refine_tol

    def run(self, trace):
        """Serve `trace` (list of Request) in real time; returns (results,
        metrics)."""
        pending = collections.deque(sorted(trace, key=lambda r: r.arrival))
        queue = collections.deque()
        active = []       # dicts: req, res, handle, bytes, jx history
        results = {}
        used = 0
        flups = 0
        t0 = self.clock()
        busy = 0.0
        while pending or queue or active:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                queue.append(r)
                results[r.rid] = Result(rid=r.rid, arrival=r.arrival)
                self.stepper.prepare(r)   # host-side set-up may start now
            # admission: FIFO while the head fits the memory budget.  While
            # solves are active, a head whose host-side set-up is unfinished
            # waits (the GPU keeps stepping); admitted solves are built
            # during the next round's steps and join after it.
            admit = []
            cells = sum(a["res"].n_fluid for a in active)
            while queue and len(active) + len(admit) < self.max_active:
                r = queue[0]
                need = self.stepper.bytes_needed(r)
                # memory held only while the solve is built
                extra = getattr(self.stepper, "transient_bytes", lambda _r: 0)(r)
                if need + extra > self.budget:
                    queue.popleft()
                    results[r.rid].error = f"needs {need + extra} bytes > budget {self.budget}"
                    results[r.rid].finished = self.clock() - t0
                    continue
                if used + need + extra > self.budget:
                    break
                if (self.target_cells is not None and (active or admit) and
                        cells + self.stepper.cells_estimate(r) > self.target_cells):
                    break
                if (active or admit) and not getattr(self.stepper, "ready", lambda _r: True)(r):
                    break
                queue.popleft()
                results[r.rid].admitted = self.clock() - t0
                admit.append((r, need))
                used += need
                cells += self.stepper.cells_estimate(r)
            if not active and not admit:
                if pending:
                    wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(wait)
                continue

            def start(batch):
                """Build the admitted requests; one that cannot be built
                fails alone and gives its memory back."""
                nonlocal used
                out = []
                for r, need in batch:
                    res = results[r.rid]
                    try:
                        handle = self.stepper.build(r)
                    except Exception as e:   # noqa: BLE001 (reported per request)
                        res.error = f"build failed: {e}"
                        res.finished = self.clock() - t0
                        used -= need
                        continue
                    res.n_fluid = self.stepper.n_fluid(handle)
                    out.append({"req": r, "res": res, "handle": handle, "bytes": need,
                                "jx": [], "refined": False})
                return out

            if not active:   # nothing to overlap with: build, then step
                active = start(admit)
                admit = []
                if not active:
                    continue
            # one round: K lockstep steps for every active solve, with the
            # builds of newly admitted solves overlapping them
            tb = self.clock()
            self.stepper.step([a["handle"] for a in active], self.K)
            joined = start(admit)
            red = self.stepper.reduce([a["handle"] for a in active])
            busy += self.clock() - tb
            keep = []
            for a, (jx, finite) in zip(active, red):
                res = a["res"]
                res.steps += self.K
                flups += res.n_fluid * self.K
                a["jx"].append(jx)
                done = False
                if not finite:
                    res.error = "non-finite state"
                    done = True
                elif len(a["jx"]) >= 2 and abs(a["jx"][-1]) > 0:
                    res.residual = abs(a["jx"][-1] - a["jx"][-2]) / abs(a["jx"][-1])
                    refined_now = False
                    if (self.refine_tol is not None and not a["refined"] and
                            res.steps >= 2 * self.K and res.residual < self.refine_tol):
                        a["refined"] = True
                        refined_now = bool(self.stepper.refine(a["handle"]))
                        if refined_now:
                            a["jx"] = []
                            res.refined_at = res.steps
                    if not refined_now and res.steps >= 2 * self.K and res.residual < self.tol:
                        res.converged = True
                        done = True
                if res.steps >= self.max_steps:
                    done = True
                if done:
                    r = a["req"]
                    nu = (r.tau - 0.5) / 3.0
                    res.permeability = nu * (jx / float(r.L ** 3)) / r.force
                    res.finished = self.clock() - t0
                    self.stepper.free(a["handle"])
                    used -= a["bytes"]
                    if self.on_finish is not None:
                        self.on_finish(res)
                else:
                    keep.append(a)
            active = keep + joined
        makespan = self.clock() - t0
        done = [r for r in results.values() if not r.error]
        lat = [r.latency for r in done]
        metrics = {
            "requests": len(results),
            "completed": len(done),
            "converged": sum(r.converged for r in done),
            "rejected_or_failed": len(results) - len(done),
            "p50_latency_s": percentile(lat, 50),
            "p99_latency_s": percentile(lat, 99),
            "p50_queue_s": percentile([r.admitted - r.arrival for r in done], 50),
            "p99_queue_s": percentile([r.admitted - r.arrival for r in done], 99),
            "p50_service_s": percentile([r.finished - r.admitted for r in done], 50),
            "p99_service_s": percentile([r.finished - r.admitted for r in done], 99),
            "makespan_s": makespan,
            "aggregate_mflups": flups / makespan / 1e6 if makespan > 0 else 0.0,
            "busy_mflups": flups / busy / 1e6 if busy > 0 else 0.0,
            "fluid_cell_updates": flups,
        }
        return [results[k] for k in sorted(results)], metrics


class MockStepper:
    """Host-only backend: a solve of N_F = phi * L^3 cells costs N_F / rate
    seconds per step on a simulated clock and its momentum approaches a
    request-specific limit geometrically, so the scheduler can be tested
    deterministically without a GPU."""

    def __init__(self, rate_flups=1e9, bytes_per_cell=112, decay=0.9, fail_rid=None, prep_s=0.0):
        """refine() halves a solve's step rate (finer storage moves twice the
        bytes) and can be called once per solve.  prep_s: host set-up time
        of a request (its geometry is ready prep_s after prepare()); a build
        before that waits for it."""
        self.rate = rate_flups
        self.prep_s = prep_s
        self.prepared = {}
        self.waited = 0.0
        self.bpc = bytes_per_cell
        self.decay = decay
        self.fail_rid = fail_rid
        self.now = 0.0
        self.live = {}
        self.built = []

    def clock(self):
        return self.now

    def sleep(self, dt):
        self.now += dt

    def bytes_needed(self, r):
        return int(r.phi * r.L ** 3) * self.bpc

    def prepare(self, r):
        self.prepared.setdefault(r.rid, self.now)

    def ready(self, r):
        self.prepare(r)
        return self.now >= self.prepared[r.rid] + self.prep_s

    def cells_estimate(self, r):
        return int(r.phi * r.L ** 3)

    def build(self, r):
        self.prepare(r)
        t_ready = self.prepared[r.rid] + self.prep_s
        if self.now < t_ready:
            self.waited += t_ready - self.now
            self.now = t_ready
        h = {"req": r, "nf": int(r.phi * r.L ** 3), "t": 0}
        self.live[id(h)] = h
        self.built.append(r.rid)
        return h

    def n_fluid(self, h):
        return h["nf"]

    def step(self, hs, n):
        self.now += sum(h["nf"] * (2 if h.get("fine") else 1) for h in hs) * n / self.rate
        for h in hs:
            h["t"] += n

    def refine(self, h):
        if h.get("fine"):
            return False
        h["fine"] = True
        return True

    def reduce(self, hs):
        out = []
        for h in hs:
            r = h["req"]
            limit = r.L * r.phi
            jx = limit * (1.0 - self.decay ** (h["t"] / 100.0))
            out.append((jx, r.rid != self.fail_rid))
        return out

    def free(self, h):
        del self.live[id(h)]


class GpuStepper:
    """liblbm backend: seeded packing -> GPU builder -> resident solve."""

    def __init__(self, storage=None, q=19, dev_exp=14, order=None, index="runs", magic=3 / 16,
                 r_range=(4.0, 12.0), stream=None, refine_storage=None):
        """refine_storage: storage a solve moves to when the server asks
        (lbm_convert, exact from 16-bit deviations); default FP32 deviations
        for 16-bit storage, none otherwise."""
        from . import lbm
        self.lbm = lbm
        self.storage = lbm.STORE_F16DEV if storage is None else storage
        self.q = q
        self.dev_exp = dev_exp if self.storage == lbm.STORE_F16DEV else 0
        if refine_storage is None and self.storage in (lbm.STORE_F16DEV, lbm.STORE_BF16DEV):
            refine_storage = lbm.STORE_F32DEV
        self.refine_storage = refine_storage
        self.order = lbm.ORDER_BLOCKED if order is None else order
        if index not in ("runs", "16", "32"):
            raise ValueError(f"index form must be 'runs', '16' or '32' (got {index!r})")
        self.index = index
        self.magic = magic
        self.r_range = r_range
        self.stream = stream
        import concurrent.futures
        import torch
        self.torch = torch
        self._ws = None
        self._step_ws = None
        # the stream every step, reduction and conversion runs on
        self._step_stream = stream if stream is not None else torch.cuda.current_stream()
        # builds run on a stream of their own so they overlap the steps
        self._build_stream = torch.cuda.Stream()
        # Geometry generation runs on host threads while the GPU steps the
        # active solves (the blocking GPU calls release the interpreter lock).
        self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=2)
        self._labels = {}

    def _geometry(self, r):
        from .inputs import boolean_spheres
        lab, _ = boolean_spheres(r.L, self.r_range[0], self.r_range[1], r.phi, seed=r.seed)
        return lab

    def cells_estimate(self, r):
        return int(r.phi * r.L ** 3)

    def prepare(self, r):
        if r.rid not in self._labels:
            self._labels[r.rid] = self._pool.submit(self._geometry, r)

    def ready(self, r):
        """Whether the request's geometry has been generated."""
        self.prepare(r)
        return self._labels[r.rid].done()

    def _nf_bound(self, r):
        return int(math.ceil(r.phi * r.L ** 3 * 1.02)) + 64

    def bytes_needed(self, r):
        """Device bytes a solve holds while it runs, from the target
        porosity: PDF-list (plus the refine storage's, both held while
        converting), index-list forms, fluid list, a little slack for the
        reduction workspace.  The run form is sized for one run start in
        four entries (packings measure about one in twelve); the int32
        index-list is dropped once the run form is built."""
        nf = self._nf_bound(r)
        b = self.lbm.STORE_BYTES[self.storage]
        per_cell = self.q * b + 4
        if self.index == "16":
            per_cell += (self.q - 1) * (4 + 2)
        elif self.index == "runs":
            per_cell += (self.q - 1) * (8 / 64 + 4 / 4)
        else:
            per_cell += (self.q - 1) * 4
        if self.refine_storage is not None:
            per_cell += self.q * self.lbm.STORE_BYTES[self.refine_storage]
        return int(nf * per_cell) + (1 << 20)

    def transient_bytes(self, r):
        """Bytes held only while a solve is built: the labels and the
        builder's workspace (5 B per box cell) and, for the run form, the
        int32 index-list it is compressed from."""
        extra = 5 * r.L ** 3
        if self.index == "runs":
            extra += (self.q - 1) * 4 * self._nf_bound(r)
        return extra

    def build(self, r):
        """Builds on the side stream (every torch copy and allocation of the
        build is ordered there too) and returns once that stream is idle, so
        the solve's buffers are complete when it joins the step stream."""
        from .inputs import PERIODIC_ALL
        self.prepare(r)
        lab = self._labels.pop(r.rid).result()
        bs = self._build_stream
        with self.torch.cuda.stream(bs):
            dom = self.lbm.SparseDomain(lab, PERIODIC_ALL, self.q, self.order, 64, stream=bs)
            if self.index == "16":
                dom.compact(stream=bs)
            elif self.index == "runs":
                dom.compact_runs(stream=bs, drop_index=True)
            sol = self.lbm.Solver(dom, self.storage, self.dev_exp)
            sol.init(stream=bs)
        bs.synchronize()
        # The buffers come from the build stream's pool but are used on the
        # step stream from now on: when one is released (retirement, or the
        # old PDF-list after a refinement), the allocator must not hand it to
        # a later build before the step stream's queued work has read it.
        for t in (dom.cells, dom.index, dom.links, dom.index16, dom.runs, sol.pdf, sol._red_ws):
            if t is not None:
                t.record_stream(self._step_stream)
        coll = self.lbm.collision(self.lbm.COLL_TRT, tau=r.tau, magic=self.magic,
                                  force=(r.force, 0.0, 0.0))
        return {"req": r, "sol": sol, "coll": coll}

    def n_fluid(self, h):
        return h["sol"].domain.n_fluid

    def _by_storage(self, hs):
        groups = {}
        for j, h in enumerate(hs):
            groups.setdefault(h["sol"].storage, []).append(j)
        return groups.values()

    def step(self, hs, n):
        # one batch per storage format (refined solves run in finer storage);
        # the segment-table workspace is reused in stream order
        need = self.lbm.lbm_step_batch_workspace_bytes(len(hs))
        if self._step_ws is None or self._step_ws.numel() < need:
            self._step_ws = self.torch.empty(max(need, 1 << 16), dtype=self.torch.uint8,
                                             device="cuda")
        for idx in self._by_storage(hs):
            self.lbm.lbm_step_batch([hs[j]["sol"].state for j in idx],
                                    [hs[j]["coll"] for j in idx], None, n, self.stream,
                                    workspace=self._step_ws)

    def reduce(self, hs):
        need = sum(self.lbm.lbm_reduce_workspace_bytes(h["sol"].domain.layout) for h in hs)
        if self._ws is None or self._ws.numel() < need:
            self._ws = self.torch.empty(max(need, 1 << 16), dtype=self.torch.uint8, device="cuda")
        out = [None] * len(hs)
        for idx in self._by_storage(hs):
            red = self.lbm.lbm_reduce_batch([hs[j]["sol"].state for j in idx],
                                            [hs[j]["coll"] for j in idx], self._ws, self.stream,
                                            check=False)
            for j, r in zip(idx, red):
                out[j] = (r.mom[0], bool(r.finite))
        return out

    def refine(self, h):
        """Move a solve to the refine storage; False when it is there already."""
        if self.refine_storage is None or h["sol"].storage == self.refine_storage:
            return False
        h["sol"] = h["sol"].converted(self.refine_storage, 0, stream=self.stream)
        return True

    def free(self, h):
        h["sol"] = None
        h["coll"] = None


def run_sequential(stepper, trace, K=100, tol=1e-6, max_steps=200_000, refine_tol=None):
    """Baseline: the same trace served one solve at a time (no batching)."""
    srv = Server(stepper, budget_bytes=1 << 62, K=K, tol=tol, max_steps=max_steps, max_active=1,
                 refine_tol=refine_tol)
    return srv.run(trace)
