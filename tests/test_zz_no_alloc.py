"""The allocation-free batch entry point, lbm_step_batch_noalloc, against
lbm_step_batch (the same steps with the segment tables in a caller
workspace): bit-identical PDF-lists on two calls in a row, the second with
fewer and smaller solves, so that the library's device array holds the
first call's tables when the second one starts."""
import numpy as np
import pytest

from paper_2408_06880_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_06880_amd import lbm  # noqa: E402

W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
CLASSES = [(lbm.BC_UBB, (0.0, 0.0, 0.02), 1.0), (lbm.BC_PRESSURE, (0, 0, 0), 1.002)]


def _say(*a):
    print("[gpu-test]", *a, flush=True)


def _solves(labs, seed):
    """One FP32 solve per mask (every third one with boundary classes, the
    index form cycling through int32, compact and run-only), all slots set
    to seeded values near the rest weights."""
    sols = []
    for j, lab in enumerate(labs):
        dom = lbm.SparseDomain(lab, 3 if j % 3 == 0 else 7, 19, lbm.ORDER_BLOCKED)
        if j % 3 == 1:
            dom.compact()
        elif j % 3 == 2 and dom.n_fluid > 0:
            dom.compact_runs(drop_index=True)
        s = lbm.Solver(dom, lbm.STORE_F32)
        s.init()
        S = dom.stride
        if S > 0:
            rng = np.random.default_rng(seed + j)
            f = W19[:, None] * (1.0 + 0.01 * rng.standard_normal((19, S)))
            s.pdf.copy_(torch.from_numpy(f.astype(np.float32).reshape(-1)))
        sols.append(s)
    return sols


def _masks(n, edge, seed):
    return [inputs.random_mask((edge + j % 3, edge + 1, edge - 1 + j % 2), 0.3, seed=seed + j,
                               n_classes=2 if j % 3 == 0 else 0, class_fraction=0.5)
            for j in range(n)]


@pytest.mark.parametrize("steps", [5])
def test_noalloc_batch_equals_workspace_batch(steps):
    coll = lbm.collision(lbm.COLL_TRT, tau=0.7, force=(1e-5, 0.0, 0.0))
    bs = lbm.bspec(CLASSES)
    for call, (n, edge) in enumerate(((40, 11), (6, 7))):
        _say("no-alloc batch call", call, "solves", n, "edge", edge, "steps", steps)
        labs = _masks(n, edge, 500 + 100 * call)
        ref = _solves(labs, 900 + call)
        got = _solves(labs, 900 + call)
        ws = torch.empty(lbm.lbm_step_batch_workspace_bytes(n), dtype=torch.uint8, device="cuda")
        lbm.lbm_step_batch([s.state for s in ref], [coll] * n, [bs] * n, steps, workspace=ws)
        lbm.lbm_step_batch_noalloc([s.state for s in got], [coll] * n, [bs] * n, steps)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert a.t == b.t == steps
            assert torch.equal(a.pdf, b.pdf)


def test_noalloc_single_state_and_zero_steps():
    """One state needs no table; zero steps change nothing."""
    coll = lbm.collision(lbm.COLL_TRT, tau=0.8)
    labs = _masks(1, 9, 77)
    ref = _solves(labs, 5)
    got = _solves(labs, 5)
    _say("no-alloc batch: one state, 3 steps")
    ref[0].step(3, coll, lbm.bspec(CLASSES))
    lbm.lbm_step_batch_noalloc([got[0].state], [coll], [lbm.bspec(CLASSES)], 3)
    before = got[0].pdf.clone()
    lbm.lbm_step_batch_noalloc([got[0].state], [coll], None, 0)
    torch.cuda.synchronize()
    assert torch.equal(ref[0].pdf, got[0].pdf) and torch.equal(before, got[0].pdf)
    assert got[0].t == 3
