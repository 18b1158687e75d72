"""Host-only tests of the serving scheduler (mock backend) and the tuner's
selection and cache logic."""
import json

import pytest

from paper_2408_06880_amd import autotune, server


class BudgetCheckingStepper(server.MockStepper):
    def __init__(self, budget, **kw):
        super().__init__(**kw)
        self.budget = budget
        self.peak = 0

    def build(self, r):
        h = super().build(r)
        live = sum(self.bytes_needed(x["req"]) for x in self.live.values())
        self.peak = max(self.peak, live)
        assert live <= self.budget
        return h


def _run(trace, budget, **kw):
    st = BudgetCheckingStepper(budget, rate_flups=5e9)
    srv = server.Server(st, budget, K=100, tol=1e-6, clock=st.clock, sleep=st.sleep, **kw)
    res, met = srv.run(trace)
    return st, res, met


def test_trace_is_seeded_and_poisson_like():
    a = server.make_trace(200, 20.0, seed=31)
    b = server.make_trace(200, 20.0, seed=31)
    assert [(r.arrival, r.L, r.phi, r.tau) for r in a] == [(r.arrival, r.L, r.phi, r.tau) for r in b]
    gaps = [y.arrival - x.arrival for x, y in zip(a, a[1:])]
    assert 0.03 < sum(gaps) / len(gaps) < 0.07
    assert all(64 <= r.L <= 384 and 0.3 <= r.phi <= 0.9 and 0.6 <= r.tau <= 1.0 for r in a)


def test_all_requests_complete_within_budget_in_fifo_order():
    trace = server.make_trace(40, 50.0, seed=3, L_range=(32, 96))
    budget = 3 * 112 * 96 ** 3   # about three of the largest requests at a time
    st, res, met = _run(trace, budget)
    assert met["completed"] == 40 and met["converged"] == 40
    assert st.built == sorted(st.built)               # admitted in arrival order
    assert st.peak <= budget
    for r in res:
        assert r.arrival <= r.admitted <= r.finished
        assert r.steps % 100 == 0 and r.steps >= 200
    assert met["p50_latency_s"] <= met["p99_latency_s"]
    assert met["aggregate_mflups"] > 0


def test_oversized_request_rejected_others_served():
    trace = server.make_trace(6, 10.0, seed=4, L_range=(32, 48))
    big = server.Request(rid=99, arrival=0.01, L=400, phi=0.9, seed=1, tau=0.8)
    st, res, met = _run(trace + [big], budget=112 * 64 ** 3)
    err = [r for r in res if r.error]
    assert [r.rid for r in err] == [99]
    assert met["completed"] == 6


def test_failed_solve_does_not_stop_the_others():
    trace = server.make_trace(8, 20.0, seed=5, L_range=(32, 64))
    st = server.MockStepper(rate_flups=5e9, fail_rid=3)
    srv = server.Server(st, 1 << 40, K=100, clock=st.clock, sleep=st.sleep)
    res, met = srv.run(trace)
    assert [r.rid for r in res if r.error] == [3]
    assert met["completed"] == 7


def test_step_cap_and_even_rounds():
    with pytest.raises(ValueError):
        server.Server(server.MockStepper(), 1 << 30, K=99)
    st = server.MockStepper(rate_flups=5e9, decay=0.999999)
    srv = server.Server(st, 1 << 40, K=100, tol=1e-12, max_steps=1000, clock=st.clock,
                        sleep=st.sleep)
    res, met = srv.run(server.make_trace(3, 10.0, seed=6, L_range=(32, 40)))
    assert all(r.steps == 1000 and not r.converged for r in res)


def test_percentiles():
    assert server.percentile([1, 2, 3, 4], 50) == 2.5
    assert server.percentile([5], 99) == 5
    assert server.percentile(list(range(101)), 99) == 99


def test_tuner_choice_and_cache(tmp_path):
    t = {(64, 0): 3.0, (128, 1): 2.0, (256, 1): 2.0, (256, 0): 2.5}
    assert autotune.choose(t) == (256, 1)
    assert autotune.choose({(256, 1, 2): 1.0, (256, 1, 1): 1.0}) == (256, 1, 1)
    # ties keep the uncapped residency
    assert autotune.choose({(256, 1, 1, 3): 1.0, (256, 1, 1, 0): 1.0}) == (256, 1, 1, 0)
    res = autotune.tune(lambda k, b, x, c, g: 1.0 / b + (0.1 if x == 0 else 0.0) + k
                        - (0.01 if c == 2 else 0.0) - (0.001 if g == 3 else 0.0))
    # tile orders 1, 16 and 256 tie here: the largest value is kept
    assert res[0][0] == (256, 256, 1, 3) and res[1][0] == (256, 256, 2, 3)
    assert len(res[0][1]) == 48 and len(res[1][1]) == 96     # cells per thread: even only
    path = tmp_path / "launch.json"
    autotune.save(str(path), {autotune.cache_key("gfx950", 0, 19, 1, 23): {"block": 128,
                                                                            "xcd_remap": 1}})
    autotune.save(str(path), {autotune.cache_key("gfx950", 0, 19, 1, 15): {"block": 64,
                                                                            "xcd_remap": 0}})
    cache = json.load(open(path))
    assert len(cache) == 2
    e = autotune.lookup(cache, "gfx950", 0, 19, 1, n_fluid=10_000_000)   # bucket 23
    assert e["block"] == 128
    e = autotune.lookup(cache, "gfx950", 0, 19, 1, n_fluid=40_000)       # bucket 15
    assert e["block"] == 64
    assert autotune.lookup(cache, "gfx950", 1, 19, 1, 1000) is None


def test_target_cells_limits_concurrency_and_cuts_median_latency():
    trace = server.make_trace(30, 100.0, seed=8, L_range=(48, 96))
    lat = {}
    for tgt in (None, 2 * 96 ** 3):
        st = server.MockStepper(rate_flups=2e9)
        srv = server.Server(st, 1 << 40, K=100, target_cells=tgt, clock=st.clock, sleep=st.sleep)
        res, met = srv.run(trace)
        assert met["completed"] == 30
        lat[tgt] = met["p50_latency_s"]
    assert lat[2 * 96 ** 3] < lat[None]


def test_refinement_moves_solves_to_finer_storage_once():
    """With refine_tol, a solve whose residual drops below it is moved to
    finer storage once, its residual history restarts, and it then runs to
    tol; without refine_tol nothing is refined."""
    trace = server.make_trace(6, 50.0, seed=5, L_range=(16, 32))
    for tol_r in (None, 1e-3):
        st = server.MockStepper(rate_flups=1e8, decay=0.8)
        res, met = server.Server(st, 1 << 40, K=100, tol=1e-6, max_steps=100_000,
                                 clock=st.clock, sleep=st.sleep, refine_tol=tol_r).run(trace)
        assert met["completed"] == 6 and all(r.converged for r in res)
        for r in res:
            if tol_r is None:
                assert r.refined_at == 0
            else:
                # refined once, strictly before the end, and at least two more
                # rounds ran to rebuild the residual in the finer storage
                assert 0 < r.refined_at <= r.steps - 200


def test_refinement_falls_back_when_the_stepper_cannot_refine():
    class NoRefine(server.MockStepper):
        def refine(self, h):
            return False

    trace = server.make_trace(3, 50.0, seed=2, L_range=(16, 24))
    st = NoRefine(rate_flups=1e8, decay=0.8)
    res, met = server.Server(st, 1 << 40, K=100, tol=1e-6, max_steps=100_000, clock=st.clock,
                             sleep=st.sleep, refine_tol=1e-3).run(trace)
    assert all(r.converged and r.refined_at == 0 for r in res)


def test_builds_overlap_steps_and_never_wait_while_solves_are_active():
    """A request whose host-side set-up is unfinished is not admitted while
    other solves run (they keep stepping); admitted solves are built during
    the next round and join after it.  Ignoring readiness makes builds wait
    with solves active and stretches the run."""

    class Recording(server.MockStepper):
        def __init__(self, gate, **kw):
            super().__init__(**kw)
            self.gate = gate
            self.waits_while_busy = 0

        def ready(self, r):
            return super().ready(r) if self.gate else True

        def build(self, r):
            busy, before = bool(self.live), self.waited
            h = super().build(r)
            if self.waited > before and busy:
                self.waits_while_busy += 1
            return h

    trace = server.make_trace(12, 40.0, seed=12, L_range=(32, 64))
    out = {}
    for gate in (True, False):
        st = Recording(gate, rate_flups=2e8, prep_s=0.2)
        res, met = server.Server(st, 1 << 40, K=100, clock=st.clock, sleep=st.sleep).run(trace)
        assert met["completed"] == 12 and all(r.converged for r in res)
        assert st.built == sorted(st.built)
        out[gate] = (st.waits_while_busy, met["makespan_s"])
    assert out[True][0] == 0 and out[False][0] > 0
    assert out[True][1] < out[False][1]


def test_admission_counts_the_build_transient():
    """A request whose held bytes fit but whose build transient does not
    waits for memory (or is rejected when it can never fit)."""

    class Transient(server.MockStepper):
        def transient_bytes(self, r):
            return self.bytes_needed(r)          # the build needs as much again

    trace = [server.Request(rid=i, arrival=0.0, L=32, phi=0.5, seed=i, tau=0.8) for i in range(3)]
    one = int(0.5 * 32 ** 3) * 112
    st = Transient(rate_flups=5e9)
    srv = server.Server(st, 3 * one, K=100, clock=st.clock, sleep=st.sleep)
    res, met = srv.run(trace)
    assert met["completed"] == 3
    # 3 x held would fit, but each admission also needs a transient of one
    # solve: at most two solves are resident at a time
    peak = max(len([r for r in res if r.admitted <= t < r.finished]) for t in
               sorted({r.admitted for r in res}))
    assert peak <= 2
    st = Transient(rate_flups=5e9)
    res, met = server.Server(st, one + one // 2, K=100, clock=st.clock,
                             sleep=st.sleep).run(trace[:1])
    assert res[0].error and met["completed"] == 0


def test_failed_build_fails_only_that_request():
    """A request whose build raises (with or without other solves active)
    gets an error and its memory back; the others are served."""

    class BuildFails(server.MockStepper):
        def build(self, r):
            if r.rid in (0, 4):
                raise RuntimeError("cannot build")
            return super().build(r)

    trace = server.make_trace(8, 20.0, seed=9, L_range=(32, 48))
    st = BuildFails(rate_flups=5e9)
    budget = 1 << 40
    srv = server.Server(st, budget, K=100, clock=st.clock, sleep=st.sleep)
    res, met = srv.run(trace)
    assert sorted(r.rid for r in res if r.error) == [0, 4]
    assert all("build failed" in r.error for r in res if r.error)
    assert met["completed"] == 6 and met["converged"] == 6


def test_stepper_without_readiness_query_is_served():
    """ready() and transient_bytes() are optional parts of a stepper."""

    class Minimal:
        def __init__(self, inner):
            self._inner = inner

        def __getattr__(self, name):
            if name in ("ready", "transient_bytes"):
                raise AttributeError(name)
            return getattr(self._inner, name)

    st = server.MockStepper(rate_flups=5e9)
    wrapped = Minimal(st)
    assert not hasattr(wrapped, "ready") and not hasattr(wrapped, "transient_bytes")
    res, met = server.Server(wrapped, 1 << 40, K=100, clock=st.clock, sleep=st.sleep).run(
        server.make_trace(4, 20.0, seed=2, L_range=(32, 40)))
    assert met["completed"] == 4
