"""GPU tests of the continuous-batching server: every result is the same
alone and in the mix, and the 16-bit serving path meets the permeability
error target against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2408_06880_amd import inputs, server

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_06880_amd import lbm  # noqa: E402


def _trace():
    reqs = server.make_trace(5, 1000.0, seed=7, L_range=(24, 48), phi_range=(0.4, 0.8))
    for r in reqs:
        r.arrival = 0.0
        r.force = 1e-5
    return reqs


def test_batched_results_equal_alone():
    """R13: per-cell arithmetic does not depend on the batch, so steps,
    residuals and permeabilities are bitwise those of each solve alone."""
    trace = _trace()
    mixed, met = server.Server(server.GpuStepper(), 1 << 34, K=100, tol=1e-6,
                               max_steps=3000).run(trace)
    alone, _ = server.run_sequential(server.GpuStepper(), _trace(), K=100, tol=1e-6,
                                     max_steps=3000)
    assert met["completed"] == len(trace)
    for a, b in zip(mixed, alone):
        assert (a.rid, a.steps, a.n_fluid, a.converged) == (b.rid, b.steps, b.n_fluid, b.converged)
        assert a.permeability == b.permeability and a.residual == b.residual


@pytest.mark.parametrize("storage,limit", [(lbm.STORE_F32, 1e-5), (lbm.STORE_F16DEV, 1e-3),
                                           (lbm.STORE_BF16DEV, None)])
def test_serving_permeability_vs_oracle(storage, limit):
    """Steady-state permeability of a served request against the FP64 oracle
    run for the same number of steps (target < 1e-3 relative for 16-bit
    storage; bfloat16 is reported, not bounded)."""
    req = server.Request(rid=0, arrival=0.0, L=24, phi=0.55, seed=77, tau=0.8, force=1e-6)
    res, met = server.Server(server.GpuStepper(storage=storage), 1 << 34, K=100, tol=1e-6,
                             max_steps=6000).run([req])
    r = res[0]
    assert not r.error and r.steps > 0
    lab, info = inputs.boolean_spheres(24, 4.0, 12.0, 0.55, seed=77)
    p = oracle.params(q=19, kind=oracle.TRT, tau=0.8, magic=3 / 16, force=(1e-6, 0, 0))
    A = oracle.dense_run(p, lab, inputs.PERIODIC_ALL, r.steps, oracle.dense_init(19, lab))
    _, J, nf = oracle.dense_reduce(p, lab, A)
    k_ref = (0.8 - 0.5) / 3.0 * (J[0] / 24 ** 3) / 1e-6
    err = abs(r.permeability - k_ref) / abs(k_ref)
    print(f"[gpu-test] storage {storage}: steps {r.steps} converged {r.converged} "
          f"residual {r.residual:.2e} k {r.permeability:.6e} ref {k_ref:.6e} rel err {err:.2e}",
          flush=True)
    if limit is not None:
        assert err < limit


def test_tuner_installs_a_measured_configuration(tmp_path):
    """The tuner times every (block, XCD order, cells per thread, residency
    cap) candidate on a real solve, installs the fastest and caches it."""
    from paper_2408_06880_amd import autotune
    lab, per, info = inputs.workload_c1(0.6, L=96, seed=5)
    dom = lbm.SparseDomain(lab, per, 19, lbm.ORDER_BLOCKED)
    dom.compact()
    sol = lbm.Solver(dom, lbm.STORE_F32)
    sol.init()
    coll = lbm.collision(lbm.COLL_TRT, tau=0.8, force=(1e-6, 0, 0))
    old = [lbm.lbm_get_launch(k, 19, lbm.STORE_F32, full=True) for k in (0, 1)]
    try:
        path = str(tmp_path / "launch.json")
        res = autotune.tune_solver(sol, coll, cache_path=path, steps=3)
        for k, n in ((0, 48), (1, 96)):
            (b, x, c, g), timings = res[k]
            assert len(timings) == n and min(timings.values()) == timings[(b, x, c, g)]
            got = lbm.lbm_get_launch(k, 19, lbm.STORE_F32, full=True)
            assert (got[0], got[1], got[3], got[4]) == (b, x, c, g)
        assert autotune.apply(path, 19, lbm.STORE_F32, dom.n_fluid) == 2
    finally:
        for k, cfg in zip((0, 1), old):
            lbm.lbm_set_launch(k, 19, lbm.STORE_F32, *cfg)


def test_refinement_reaches_fp32_accuracy_and_stays_batch_independent():
    """FP16-deviation solves moved to FP32 deviations once their residual is
    below 1e-5 (lbm_convert, exact): the served permeability then has the
    FP32 error against the FP64 oracle, and batched results still equal the
    solves alone."""
    req = server.Request(rid=0, arrival=0.0, L=24, phi=0.55, seed=77, tau=0.8, force=1e-6)
    res, _ = server.Server(server.GpuStepper(storage=lbm.STORE_F16DEV), 1 << 34, K=100,
                           tol=1e-6, max_steps=8000, refine_tol=1e-5).run([req])
    r = res[0]
    assert r.converged and 0 < r.refined_at < r.steps
    lab, info = inputs.boolean_spheres(24, 4.0, 12.0, 0.55, seed=77)
    p = oracle.params(q=19, kind=oracle.TRT, tau=0.8, magic=3 / 16, force=(1e-6, 0, 0))
    A = oracle.dense_run(p, lab, inputs.PERIODIC_ALL, r.steps, oracle.dense_init(19, lab))
    _, J, nf = oracle.dense_reduce(p, lab, A)
    k_ref = (0.8 - 0.5) / 3.0 * (J[0] / 24 ** 3) / 1e-6
    err = abs(r.permeability - k_ref) / abs(k_ref)
    print(f"[gpu-test] refined at {r.refined_at}, steps {r.steps}, rel err {err:.2e}", flush=True)
    assert err < 5e-5
    trace = _trace()
    mixed, _ = server.Server(server.GpuStepper(storage=lbm.STORE_F16DEV), 1 << 34, K=100,
                             tol=1e-6, max_steps=3000, refine_tol=1e-4).run(trace)
    alone, _ = server.run_sequential(server.GpuStepper(storage=lbm.STORE_F16DEV), _trace(),
                                     K=100, tol=1e-6, max_steps=3000, refine_tol=1e-4)
    assert any(a.refined_at for a in mixed)
    for a, b in zip(mixed, alone):
        assert (a.steps, a.refined_at, a.converged) == (b.steps, b.refined_at, b.converged)
        assert a.permeability == b.permeability


class _SimClockStepper(server.GpuStepper):
    """GpuStepper on a simulated clock: a round of n steps advances the clock
    by a fixed amount per solve, and a request's geometry counts as ready
    once generated, so admissions happen at the same rounds in every run.
    Records, for each build, how many solves were being stepped."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.now = 0.0
        self.live = 0
        self.builds = []

    def clock(self):
        return self.now

    def sleep(self, dt):
        self.now += dt

    def ready(self, r):
        self.prepare(r)
        self._labels[r.rid].result()
        return True

    def step(self, hs, n):
        self.live = len(hs)
        super().step(hs, n)
        self.now += 0.01 * len(hs) * n / 100

    def build(self, r):
        self.builds.append((r.rid, self.live))
        return super().build(r)

    def free(self, h):
        self.live -= 1
        super().free(h)


def test_requests_joining_mid_flight_equal_alone():
    """Staggered arrivals on a simulated clock: later requests are admitted
    and built (on the side stream) while earlier ones are stepping, and
    16-bit solves are refined to FP32 deviations in the same rounds (their
    old PDF-lists released while builds run).  Every result -- step count,
    refinement step, permeability -- is bitwise that of the request served
    alone."""
    def trace():
        reqs = server.make_trace(6, 1000.0, seed=9, L_range=(24, 40), phi_range=(0.4, 0.8))
        for j, r in enumerate(reqs):
            r.arrival = 0.03 * j
            r.force = 1e-5
        return reqs

    st = _SimClockStepper(storage=lbm.STORE_F16DEV)
    mixed, met = server.Server(st, 1 << 34, K=100, tol=1e-6, max_steps=3000, refine_tol=1e-4,
                               clock=st.clock, sleep=st.sleep).run(trace())
    alone, _ = server.run_sequential(server.GpuStepper(storage=lbm.STORE_F16DEV), trace(),
                                     K=100, tol=1e-6, max_steps=3000, refine_tol=1e-4)
    print(f"[gpu-test] builds (rid, solves stepping): {st.builds}", flush=True)
    assert met["completed"] == 6
    assert any(live > 0 for _, live in st.builds[1:])     # joins during stepping
    assert any(a.refined_at for a in mixed)
    for a, b in zip(mixed, alone):
        assert (a.rid, a.steps, a.refined_at, a.converged) == (b.rid, b.steps, b.refined_at,
                                                                b.converged)
        assert a.permeability == b.permeability
