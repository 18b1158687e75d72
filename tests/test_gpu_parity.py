"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Lists and index tables: bit-exact.  PDFs: FP64 storage within 1e-12
relative, FP32 storage within 1e-5 relative after 100 steps (elementwise,
|f_gpu - f_ref| / |f_ref|; f >= w_min * rho > 0).  16-bit deviation storage:
one step from an exactly known state lands within one unit in the last
place of the stored code (plus FP32 arithmetic slack) at both parities.
"""
import numpy as np
import pytest

import oracle
from paper_2408_06880_amd import inputs
from tests import lbm_host_codec as codec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_06880_amd import lbm  # noqa: E402

KIND = {lbm.COLL_NONE: oracle.NONE, lbm.COLL_SRT: oracle.SRT, lbm.COLL_TRT: oracle.TRT,
        lbm.COLL_CUMULANT: oracle.CUMULANT, lbm.COLL_MRT: oracle.MRT, lbm.COLL_CM: oracle.CM}
BC = {lbm.BC_NOSLIP: oracle.BC_NOSLIP, lbm.BC_UBB: oracle.BC_UBB,
      lbm.BC_PRESSURE: oracle.BC_PRESSURE}


def _say(*a):
    print("[gpu-test]", *a, flush=True)


def _check_index(dom):
    """Host check before any step kernel: every pull position is in bounds
    and the table is a permutation of the slots (race-free AA)."""
    q, S, nf = dom.q, dom.stride, dom.n_fluid
    idx = dom.index[:(q - 1) * S].cpu().numpy().astype(np.int64)
    assert idx.min() >= 0 and idx.max() < q * S
    used = np.concatenate([idx[(i - 1) * S:(i - 1) * S + nf] for i in range(1, q)])
    expect = np.concatenate([i * S + np.arange(nf) for i in range(1, q)])
    assert np.array_equal(np.sort(used), expect)
    if dom.n_links:
        ln = dom.links[:2 * dom.n_links].cpu().numpy()
        assert ln[0::2].min() >= 0 and ln[0::2].max() < q * S


def _params(q, kind, tau, force, classes, magic=3.0 / 16.0, omega_bulk=1.0,
            rates=(1.3, 1.5, 1.2, 1.7)):
    """Collision (library), boundary spec and oracle parameters of one case;
    `rates` are the MRT group rates or the central-moment order rates."""
    coll = lbm.collision(kind, tau=tau, magic=magic, omega_bulk=omega_bulk, force=force,
                         rates=rates)
    bs = lbm.bspec(classes)
    op = oracle.params(q=q, kind=KIND[kind], tau=tau, magic=magic, omega_bulk=omega_bulk,
                       force=force, classes=[(BC[t], u, r) for t, u, r in classes],
                       rates=rates)
    return coll, bs, op


def _upload(sol, f_list, dev_exp):
    """f_list: FP64 [q, nf] in list order -> device PDF-list; returns the
    FP64 values the device sees."""
    dom = sol.domain
    q, S, nf = dom.q, dom.stride, dom.n_fluid
    raw, seen = codec.encode(sol.storage, f_list, q, dev_exp)
    _, w, _ = oracle.stencil(q)
    pad_raw, _ = codec.encode(sol.storage, np.repeat(w[:, None], max(S - nf, 1), 1), q, dev_exp)
    full = np.zeros((q, S), raw.dtype)
    full[:, :nf] = raw
    if S > nf:
        full[:, nf:] = pad_raw[:, :S - nf]
    sol.pdf.copy_(torch.from_numpy(full.reshape(-1)))
    sol.state.t = 0
    sol.state.link_vel_t = -1
    return seen


def _download(sol, dev_exp):
    """Post-collision FP64 populations [q, nf] in natural order at sol.t."""
    dom = sol.domain
    q, S, nf = dom.q, dom.stride, dom.n_fluid
    raw = sol.pdf[:q * S].cpu().numpy()
    f = codec.decode(sol.storage, raw.reshape(q, S), q, dev_exp).reshape(-1)
    if sol.t % 2 == 0:
        return f.reshape(q, S)[:, :nf]
    _, _, opp = oracle.stencil(q)
    idx = dom.index[:(q - 1) * S].cpu().numpy().astype(np.int64)
    out = np.empty((q, nf))
    out[0] = f[:nf]
    for j in range(1, q):
        out[j] = f[idx[(opp[j] - 1) * S:(opp[j] - 1) * S + nf]]
    return out


def _dense_from_list(f_list, cells, shape, q):
    _, w, _ = oracle.stencil(q)
    A = np.repeat(w[:, None], int(np.prod(shape)), 1)
    A[:, cells] = f_list
    return A.reshape((q,) + tuple(shape))


def _random_state(q, nf, seed, amp=1e-2):
    rng = np.random.default_rng(seed)
    c, w, _ = oracle.stencil(q)
    rho = 1 + 0.01 * rng.standard_normal(nf)
    u = 0.02 * rng.standard_normal((3, nf))
    cu = c.astype(float) @ u
    feq = w[:, None] * rho[None] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * np.sum(u * u, 0)[None])
    return feq * (1 + amp * rng.standard_normal((q, nf)))


CLASSES = [(lbm.BC_UBB, (0.0, 0.0, 0.02), 1.0), (lbm.BC_PRESSURE, (0, 0, 0), 1.002),
           (lbm.BC_UBB, (0.01, -0.01, 0.005), 1.0)]


# --------------------------------------------------------------- builder
BUILD_CASES = [((20, 18, 17), 0.4, 7, 19, 0, 64), ((33, 9, 21), 0.3, 5, 27, 0, 1),
               ((16, 16, 16), 0.5, 0, 19, 1, 8), ((40, 3, 7), 0.2, 2, 27, 1, 64),
               ((1, 1, 1), 0.0, 7, 19, 0, 64), ((5, 6, 7), 1.0, 7, 19, 0, 64),
               ((21, 35, 19), 0.35, 7, 19, 2, 64), ((7, 9, 40), 0.3, 4, 27, 2, 1),
               ((1, 1, 1), 0.0, 7, 27, 2, 64)]


@pytest.mark.parametrize("shape,solid,periodic,q,order,align", BUILD_CASES)
def test_builder_bit_exact(shape, solid, periodic, q, order, align):
    _say("builder", shape, solid, periodic, q, order, align)
    lab = inputs.random_mask(shape[::-1], solid, seed=sum(shape), n_classes=3,
                             class_fraction=0.5)
    ref = oracle.sparse_build(lab, periodic, q, order=order, align=align)
    dom = lbm.SparseDomain(lab, periodic, q, order, align)
    torch.cuda.synchronize()
    assert (dom.n_fluid, dom.stride, dom.n_links) == (ref.n_fluid, ref.stride, ref.n_links)
    nf, S = ref.n_fluid, ref.stride
    assert np.array_equal(dom.cells[:nf].cpu().numpy(), ref.cells)
    got = dom.index[:(q - 1) * S].cpu().numpy()
    for i in range(1, q):
        sl = slice((i - 1) * S, (i - 1) * S + nf)
        assert np.array_equal(got[sl], ref.index[sl]), i
    if ref.n_links:
        assert np.array_equal(dom.links[:2 * ref.n_links].cpu().numpy(), ref.links)
    if nf:
        _check_index(dom)


@pytest.fixture(scope="module")
def packing256():
    """The benchmark geometry and the oracle's lists for it."""
    lab, per, info = inputs.workload_c1(0.6)
    _say("oracle build 256^3", info["n_fluid"])
    return lab, per, info, oracle.sparse_build(lab, per, 19, order=0, align=64)


def test_builder_full_size_packing(packing256):
    """256^3 sphere packing at porosity 0.6 (the benchmark geometry):
    fluid list and index-list bit-exact against the oracle's builder."""
    lab, per, info, ref = packing256
    dom = lbm.SparseDomain(lab, per, 19, lbm.ORDER_MORTON, 64)
    torch.cuda.synchronize()
    assert dom.n_fluid == ref.n_fluid == info["n_fluid"]
    assert dom.stride == ref.stride
    assert torch.equal(dom.cells[:ref.n_fluid].cpu(), torch.from_numpy(ref.cells))
    nf, S = ref.n_fluid, ref.stride
    got = dom.index[:18 * S].cpu().numpy().reshape(18, S)[:, :nf]
    assert np.array_equal(got, ref.index.reshape(18, S)[:, :nf])


# ------------------------------------------------------ AA vs oracle
AA_CASES = [
    (19, lbm.COLL_SRT, lbm.STORE_F64), (19, lbm.COLL_TRT, lbm.STORE_F64),
    (19, lbm.COLL_NONE, lbm.STORE_F64), (27, lbm.COLL_CUMULANT, lbm.STORE_F64),
    (27, lbm.COLL_TRT, lbm.STORE_F64), (27, lbm.COLL_SRT, lbm.STORE_F64),
    (19, lbm.COLL_SRT, lbm.STORE_F32), (19, lbm.COLL_TRT, lbm.STORE_F32),
    (19, lbm.COLL_TRT, lbm.STORE_F32DEV), (27, lbm.COLL_CUMULANT, lbm.STORE_F32),
    (27, lbm.COLL_CUMULANT, lbm.STORE_F32DEV), (27, lbm.COLL_TRT, lbm.STORE_F32),
    (19, lbm.COLL_MRT, lbm.STORE_F64), (19, lbm.COLL_MRT, lbm.STORE_F32),
    (19, lbm.COLL_MRT, lbm.STORE_F32DEV), (27, lbm.COLL_CM, lbm.STORE_F64),
    (27, lbm.COLL_CM, lbm.STORE_F32),
]


@pytest.mark.parametrize("q,kind,storage", AA_CASES)
def test_aa_steps_match_oracle(q, kind, storage):
    """Random packing with inlet/outlet classes, partly periodic, a ragged
    last tile; compared after 1, 2, 4, 10 and 100 steps."""
    _say("aa", q, kind, storage)
    lab = inputs.random_mask((13, 15, 17), 0.3, seed=q + 10 * kind, n_classes=3,
                             class_fraction=0.5)
    per = 5
    force = (2e-5, -1e-5, 5e-6)
    coll, bs, op = _params(q, kind, 0.7, force, CLASSES, omega_bulk=1.2)
    dom = lbm.SparseDomain(lab, per, q)
    torch.cuda.synchronize()
    _check_index(dom)
    sol = lbm.Solver(dom, storage)
    f0 = _random_state(q, dom.n_fluid, seed=q + kind)
    seen = _upload(sol, f0, 0)
    cells = dom.cells[:dom.n_fluid].cpu().numpy()
    A = _dense_from_list(seen, cells, lab.shape, q)
    tol = 1e-12 if storage == lbm.STORE_F64 else 1e-5
    _, w, _ = oracle.stencil(q)
    t = 0
    for n in (1, 1, 2, 6, 90):
        sol.step(n, coll, bs)
        A = oracle.dense_run(op, lab, per, n, A)
        t += n
        torch.cuda.synchronize()
        got = _download(sol, 0)
        ref = A.reshape(q, -1)[:, cells]
        # Relative to |f|; the floor w_i/2 only matters for the collision-free
        # kind, whose populations drift through zero at moving walls.
        err = np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 0.5 * w[:, None]))
        assert err <= tol, (t, err)


@pytest.mark.parametrize("q,kind", [(19, lbm.COLL_TRT), (19, lbm.COLL_SRT),
                                    (27, lbm.COLL_CUMULANT), (19, lbm.COLL_MRT),
                                    (27, lbm.COLL_CM)])
@pytest.mark.parametrize("storage,dev_exp", [(lbm.STORE_F16DEV, 14), (lbm.STORE_F16DEV, 10),
                                             (lbm.STORE_BF16DEV, 0)])
def test_16bit_one_step_bounds(q, kind, storage, dev_exp):
    """16-bit deviation storage: starting from an exactly representable
    state, one odd and then one even step match the FP64 oracle within one
    unit in the last place of the stored code.  Cells with inlet/outlet
    links get the rounding of the link update on top: the library stores
    the updated boundary population in 16 bits before the collision reads
    it, and the collision carries that error to every population of the
    cell with a gain below 1 + 2 omega <= 5."""
    _say("16bit", q, kind, storage, dev_exp)
    lab = inputs.random_mask((12, 11, 10), 0.3, seed=5 + q, n_classes=2, class_fraction=0.5)
    per = 7
    coll, bs, op = _params(q, kind, 0.8, (1e-5, 0, 0), CLASSES[:2])
    dom = lbm.SparseDomain(lab, per, q)
    torch.cuda.synchronize()
    _check_index(dom)
    sol = lbm.Solver(dom, storage, dev_exp)
    f0 = _random_state(q, dom.n_fluid, seed=9, amp=2e-3)
    seen = _upload(sol, f0, dev_exp)
    link_pos = dom.links[:2 * dom.n_links].cpu().numpy()[0::2].astype(np.int64)
    assert dom.n_links > 0
    cells = dom.cells[:dom.n_fluid].cpu().numpy()
    A = _dense_from_list(seen, cells, lab.shape, q)
    for _ in range(2):
        sol.step(1, coll, bs)
        torch.cuda.synchronize()
        A = oracle.dense_run(op, lab, per, 1, A)
        ref = A.reshape(q, -1)[:, cells]
        got = _download(sol, dev_exp)
        ulp = codec.ulp_bound(storage, ref, q, dev_exp)
        bound = ulp + 2e-9
        link_cells = np.unique(link_pos % dom.stride)
        bound[:, link_cells] += 5.0 * np.max(ulp[:, link_cells], axis=0)
        assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)
        A = _dense_from_list(got, cells, lab.shape, q)  # continue from the device state


def test_rest_state_bitwise_fixed_point_in_deviation_storage():
    lab, per, _ = inputs.workload_c0()
    for storage in (lbm.STORE_F16DEV, lbm.STORE_BF16DEV, lbm.STORE_F32DEV):
        dom = lbm.SparseDomain(lab, per, 19)
        sol = lbm.Solver(dom, storage, 14 if storage == lbm.STORE_F16DEV else 0)
        sol.init()
        sol.step(10, lbm.collision(lbm.COLL_TRT, tau=0.8))
        torch.cuda.synchronize()
        assert int(torch.count_nonzero(sol.pdf)) == 0


# ------------------------------------------------------------ config 0
def test_config0_fp64_srt_200_steps():
    """32^3 periodic packing (~20k fluid cells), D3Q19 SRT tau = 0.8, FP64,
    F = 1e-6 x, rest start: PDFs within 1e-12 of the oracle at 100 and 200
    steps, mass drift at rounding level, mean velocity of the forced flow."""
    lab, per, info = inputs.workload_c0()
    _say("config0", info)
    coll, bs, op = _params(19, lbm.COLL_SRT, 0.8, (1e-6, 0, 0), [])
    dom = lbm.SparseDomain(lab, per, 19)
    torch.cuda.synchronize()
    _check_index(dom)
    sol = lbm.Solver(dom, lbm.STORE_F64)
    sol.init()
    m0 = sol.reduce(coll).mass
    A = oracle.dense_init(19, lab)
    cells = dom.cells[:dom.n_fluid].cpu().numpy()
    for n in (100, 100):
        sol.step(n, coll)
        A = oracle.dense_run(op, lab, per, n, A)
        torch.cuda.synchronize()
        got = _download(sol, 0)
        ref = A.reshape(19, -1)[:, cells]
        assert np.max(np.abs(got - ref) / ref) <= 1e-12
    r = sol.reduce(coll)
    assert abs(r.mass - m0) / m0 < 1e-13
    mref, Jref, nf = oracle.dense_reduce(op, lab, A)
    assert abs(r.mass - mref) / mref < 1e-13
    assert abs(r.mom[0] - Jref[0]) / abs(Jref[0]) < 1e-10
    assert 0 < r.mom[0] / nf < 200 * 1e-6


# -------------------------------------------------- moments, reductions
@pytest.mark.parametrize("storage", [lbm.STORE_F64, lbm.STORE_F32])
def test_moments_and_reduce_both_parities(storage):
    lab = inputs.random_mask((14, 13, 12), 0.35, seed=3)
    per = 7
    q = 19
    coll, bs, op = _params(q, lbm.COLL_TRT, 0.75, (1e-5, 2e-6, 0), [])
    dom = lbm.SparseDomain(lab, per, q)
    torch.cuda.synchronize()
    _check_index(dom)
    sol = lbm.Solver(dom, storage)
    seen = _upload(sol, _random_state(q, dom.n_fluid, seed=4), 0)
    cells = dom.cells[:dom.n_fluid].cpu().numpy()
    A = _dense_from_list(seen, cells, lab.shape, q)
    tol = 1e-12 if storage == lbm.STORE_F64 else 2e-6
    for n in (1, 1, 3):
        sol.step(n, coll)
        A = oracle.dense_run(op, lab, per, n, A)
        torch.cuda.synchronize()
        rho, u = sol.moments(coll, f64=True)
        rref, uref = oracle.dense_moments(op, lab, A)
        nf = dom.n_fluid
        rr = rref.reshape(-1)[cells]
        assert np.max(np.abs(rho[:nf].cpu().numpy() - rr)) <= tol
        for a in range(3):
            ua = uref[a].reshape(-1)[cells]
            assert np.max(np.abs(u[a, :nf].cpu().numpy() - ua)) <= tol
        red = sol.reduce(coll)
        m, J, nfr = oracle.dense_reduce(op, lab, A)
        assert red.n_fluid == nfr == nf and red.finite == 1
        assert abs(red.mass - m) / m <= tol
        assert np.max(np.abs(np.array(red.mom[:]) - J)) <= tol * nf * 0.05


def test_reduce_flags_non_finite():
    lab = inputs.random_mask((8, 8, 8), 0.2, seed=1)
    dom = lbm.SparseDomain(lab, 7, 19)
    sol = lbm.Solver(dom, lbm.STORE_F32)
    sol.init()
    sol.pdf[5] = float("nan")
    red = sol.reduce(lbm.collision(), check=False)
    assert red.finite == 0
    with pytest.raises(lbm.LbmError) as e:
        sol.reduce(lbm.collision())
    assert e.value.code == lbm.LBM_EUNSTABLE


# --------------------------------------------------------- batching
def test_batch_is_bitwise_identical_to_alone():
    """Three solves of different geometry, size and tau advanced together in
    one launch per step give bit-identical PDFs and reductions to each solve
    advanced alone."""
    geoms = [inputs.random_mask((10 + 3 * j, 12, 9 + j), 0.3 + 0.1 * j, seed=20 + j)
             for j in range(3)]
    taus = [0.6, 0.8, 1.0]
    storage = lbm.STORE_F16DEV
    alone, mixed, colls = [], [], []
    for lab, tau in zip(geoms, taus):
        coll = lbm.collision(lbm.COLL_TRT, tau=tau, force=(1e-5, 0, 0))
        colls.append(coll)
        for lst in (alone, mixed):
            dom = lbm.SparseDomain(lab, 7, 19)
            s = lbm.Solver(dom, storage, 14)
            s.init()
            lst.append(s)
    torch.cuda.synchronize()
    for s, c in zip(alone, colls):
        s.step(12, c)
    lbm.lbm_step_batch([s.state for s in mixed], colls, None, 12)
    torch.cuda.synchronize()
    for a, b in zip(alone, mixed):
        assert a.t == b.t == 12
        assert torch.equal(a.pdf, b.pdf)
    ws = torch.empty(sum(lbm.lbm_reduce_workspace_bytes(s.domain.layout) for s in mixed),
                     dtype=torch.uint8, device="cuda")
    rb = lbm.lbm_reduce_batch([s.state for s in mixed], colls, ws)
    for s, c, r in zip(alone, colls, rb):
        ra = s.reduce(c)
        assert (ra.mass, tuple(ra.mom)) == (r.mass, tuple(r.mom))


# ------------------------------------------------------------ dense
@pytest.mark.parametrize("storage,kind", [(lbm.STORE_F64, lbm.COLL_TRT),
                                          (lbm.STORE_F32, lbm.COLL_TRT),
                                          (lbm.STORE_F64, lbm.COLL_MRT),
                                          (lbm.STORE_F64, lbm.COLL_CM)])
def test_dense_comparator_matches_oracle(storage, kind):
    lab = inputs.random_mask((15, 14, 13), 0.35, seed=8)
    per = 6
    q = 27 if kind == lbm.COLL_CM else 19
    coll, _, op = _params(q, kind, 0.8, (1e-5, 0, 0), [])
    ds = lbm.DenseSolver(lab, per, q, storage)
    ds.init()
    ds.step(20, coll)
    torch.cuda.synchronize()
    A = oracle.dense_run(op, lab, per, 20, oracle.dense_init(q, lab))
    fl = (lab.reshape(-1) == 0)
    raw = ds.pdf.cpu().numpy().reshape(q, -1)
    got = codec.decode(storage, raw, q)[:, fl]
    ref = A.reshape(q, -1)[:, fl]
    tol = 1e-12 if storage == lbm.STORE_F64 else 1e-5
    assert np.max(np.abs(got - ref) / ref) <= tol


# -------------------------------------------------- full-size parity
@pytest.mark.parametrize("order,form", [(lbm.ORDER_MORTON, "int32"), (lbm.ORDER_BLOCKED, "runs")])
def test_full_size_packing_two_steps_fp32(packing256, order, form):
    """256^3 packing at porosity 0.6, D3Q19 TRT FP32: one odd and one even
    step from a perturbed state match the oracle's sparse AA scheme on every
    fluid cell -- in the benchmark's configuration (blocked order,
    run-compressed index, default launch table) and with Morton order and
    the int32 index."""
    lab, per, info, ref_lay = packing256
    _say("full size two steps", info["n_fluid"], order, form)
    q = 19
    if order != lbm.ORDER_MORTON:
        ref_lay = oracle.sparse_build(lab, per, q, order=order, align=64)
    coll, _, op = _params(q, lbm.COLL_TRT, 0.8, (1e-6, 0, 0), [])
    dom = lbm.SparseDomain(lab, per, q, order)
    if form == "runs":
        dom.compact_runs()
    torch.cuda.synchronize()
    sol = lbm.Solver(dom, lbm.STORE_F32)
    f0 = _random_state(q, dom.n_fluid, seed=1, amp=1e-3)
    seen = _upload(sol, f0, 0)
    assert np.array_equal(ref_lay.cells, dom.cells[:dom.n_fluid].cpu().numpy())
    pdf = np.zeros(q * ref_lay.stride)
    for i in range(q):
        pdf[i * ref_lay.stride:i * ref_lay.stride + dom.n_fluid] = seen[i]
    for t in range(2):
        sol.step(1, coll)
        pdf = oracle.sparse_run(op, ref_lay, pdf, t, 1)
        torch.cuda.synchronize()
        got = _download(sol, 0)
        ref = oracle.sparse_gather(ref_lay, pdf, t + 1)
        assert np.max(np.abs(got - ref) / ref) <= 1e-5


def test_full_size_packing_d3q27_cumulant_two_steps(packing256):
    """The D3Q27 cumulant kernels on the 256^3 packing at porosity 0.6
    (10.06 M fluid cells, FP32, blocked order, run-compressed index, default
    launch table; the configuration of the D3Q27 profile): one odd and one
    even step from a perturbed state match the oracle's sparse AA scheme on
    every fluid cell."""
    lab, per, info, _ = packing256
    q = 27
    _say("full size D3Q27 cumulant two steps", info["n_fluid"])
    ref_lay = oracle.sparse_build(lab, per, q, order=lbm.ORDER_BLOCKED, align=64)
    coll, _, op = _params(q, lbm.COLL_CUMULANT, 0.8, (1e-6, 0, 0), [])
    dom = lbm.SparseDomain(lab, per, q, lbm.ORDER_BLOCKED)
    dom.compact_runs()
    torch.cuda.synchronize()
    assert np.array_equal(ref_lay.cells, dom.cells[:dom.n_fluid].cpu().numpy())
    sol = lbm.Solver(dom, lbm.STORE_F32)
    seen = _upload(sol, _random_state(q, dom.n_fluid, seed=23, amp=1e-3), 0)
    S, nf = ref_lay.stride, dom.n_fluid
    pdf = np.zeros(q * S)
    for i in range(q):
        pdf[i * S:i * S + nf] = seen[i]
    del seen
    for t in range(2):
        sol.step(1, coll)
        pdf = oracle.sparse_run(op, ref_lay, pdf, t, 1)
        torch.cuda.synchronize()
        got = _download(sol, 0)
        ref = oracle.sparse_gather(ref_lay, pdf, t + 1)
        err = float(np.max(np.abs(got - ref) / np.abs(ref)))
        _say("full size D3Q27 step", t + 1, "max rel err", err)
        assert err <= 1e-5


@pytest.mark.parametrize("storage", [lbm.STORE_F64, lbm.STORE_F16DEV])
def test_full_size_tile_orders_bitwise(packing256, storage):
    """On the 256^3 benchmark packing (about 39 000 odd-step tiles, so
    every chunk size has full rounds and a partial last round) the odd and
    even steps give
    the same bits in dispatch order, one eighth per XCD, and chunks of 16
    and 256 tiles: each order assigns every tile to exactly one
    workgroup."""
    lab, per, info, _ = packing256
    _say("full size tile orders", storage)
    coll = lbm.collision(lbm.COLL_TRT, tau=0.8, force=(1e-6, 0, 0))
    dev_exp = 14 if storage == lbm.STORE_F16DEV else 0
    dom = lbm.SparseDomain(lab, per, 19, lbm.ORDER_BLOCKED)
    dom.compact_runs()
    f0 = _random_state(19, dom.n_fluid, seed=29, amp=1e-3)
    old = [lbm.lbm_get_launch(k, 19, storage, full=True) for k in (0, 1)]
    ref = None
    try:
        for x in (0, 1, 16, 256):
            for k in (0, 1):
                b0, _, p0, c0, g0 = old[k]
                lbm.lbm_set_launch(k, 19, storage, b0, x, p0, c0, g0)
            s = lbm.Solver(dom, storage, dev_exp)
            _upload(s, f0, dev_exp)
            s.step(2, coll)
            torch.cuda.synchronize()
            if ref is None:
                ref = s.pdf.clone()
            else:
                assert torch.equal(ref, s.pdf), x
            del s
    finally:
        for k in (0, 1):
            lbm.lbm_set_launch(k, 19, storage, *old[k])


def test_full_size_packing_fp64_100_steps(packing256):
    """The benchmark's headline configuration, exactly as bench.py times it:
    256^3 packing at porosity 0.6 (10.06 M fluid cells), D3Q19 TRT FP64,
    blocked order, run-compressed index-list only (int32 list dropped),
    default launch table.  100 AA steps from a perturbed state match the
    oracle's sparse AA scheme within 1e-12 relative on every fluid cell."""
    lab, per, info, _ = packing256
    q = 19
    _say("full size FP64 100 steps", info["n_fluid"])
    ref_lay = oracle.sparse_build(lab, per, q, order=lbm.ORDER_BLOCKED, align=64)
    coll, _, op = _params(q, lbm.COLL_TRT, 0.8, (1e-6, 0, 0), [])
    dom = lbm.SparseDomain(lab, per, q, lbm.ORDER_BLOCKED)
    dom.compact_runs(drop_index=True)
    torch.cuda.synchronize()
    assert dom.n_fluid == ref_lay.n_fluid and dom.stride == ref_lay.stride
    assert np.array_equal(ref_lay.cells, dom.cells[:dom.n_fluid].cpu().numpy())
    sol = lbm.Solver(dom, lbm.STORE_F64)
    f0 = _random_state(q, dom.n_fluid, seed=17, amp=1e-3)
    seen = _upload(sol, f0, 0)
    del f0
    S, nf = ref_lay.stride, dom.n_fluid
    pdf = np.zeros(q * S)
    for i in range(q):
        pdf[i * S:i * S + nf] = seen[i]
    del seen
    sol.step(100, coll)
    pdf = oracle.sparse_run(op, ref_lay, pdf, 0, 100)
    torch.cuda.synchronize()
    assert sol.t == 100
    got = sol.pdf[:q * S].cpu().numpy().reshape(q, S)[:, :nf]
    ref = pdf.reshape(q, S)[:, :nf]
    err = float(np.max(np.abs(got - ref) / np.abs(ref)))
    _say("full size FP64 max rel err", err)
    assert err <= 1e-12


@pytest.mark.parametrize("phi", [0.4, 0.95])
def test_full_size_packing_other_porosities(phi):
    """The benchmark's other 256^3 porosities (6.7 M and 15.9 M fluid cells)
    in its configuration (blocked order, run-compressed index): one odd and
    one even FP32 TRT step match the oracle's sparse AA scheme."""
    lab, per, info = inputs.workload_c1(phi)
    _say("full size", phi, info["n_fluid"])
    q = 19
    ref_lay = oracle.sparse_build(lab, per, q, order=lbm.ORDER_BLOCKED, align=64)
    coll, _, op = _params(q, lbm.COLL_TRT, 0.8, (1e-6, 0, 0), [])
    dom = lbm.SparseDomain(lab, per, q, lbm.ORDER_BLOCKED)
    dom.compact_runs()
    torch.cuda.synchronize()
    assert dom.n_fluid == ref_lay.n_fluid == info["n_fluid"]
    sol = lbm.Solver(dom, lbm.STORE_F32)
    seen = _upload(sol, _random_state(q, dom.n_fluid, seed=3, amp=1e-3), 0)
    pdf = np.zeros(q * ref_lay.stride)
    for i in range(q):
        pdf[i * ref_lay.stride:i * ref_lay.stride + dom.n_fluid] = seen[i]
    for t in range(2):
        sol.step(1, coll)
        pdf = oracle.sparse_run(op, ref_lay, pdf, t, 1)
        torch.cuda.synchronize()
        got = _download(sol, 0)
        ref = oracle.sparse_gather(ref_lay, pdf, t + 1)
        assert np.max(np.abs(got - ref) / ref) <= 1e-5


def test_full_size_384_packing_two_steps():
    """The 384^3 mixed-precision geometry (34 M fluid cells, the largest
    configuration) in the benchmark's configuration: one odd and one even
    FP32 TRT step against the oracle's sparse AA scheme, every fluid cell."""
    lab, info = inputs.boolean_spheres(384, 4.0, 12.0, 0.6, seed=21)
    per = inputs.PERIODIC_ALL
    _say("full size 384", info["n_fluid"])
    q = 19
    ref_lay = oracle.sparse_build(lab, per, q, order=lbm.ORDER_BLOCKED, align=64)
    coll, _, op = _params(q, lbm.COLL_TRT, 0.8, (1e-6, 0, 0), [])
    dom = lbm.SparseDomain(lab, per, q, lbm.ORDER_BLOCKED)
    dom.compact_runs()
    torch.cuda.synchronize()
    assert dom.n_fluid == ref_lay.n_fluid == info["n_fluid"]
    sol = lbm.Solver(dom, lbm.STORE_F32)
    seen = _upload(sol, _random_state(q, dom.n_fluid, seed=4, amp=1e-3), 0)
    pdf = np.zeros(q * ref_lay.stride)
    for i in range(q):
        pdf[i * ref_lay.stride:i * ref_lay.stride + dom.n_fluid] = seen[i]
    del seen
    for t in range(2):
        sol.step(1, coll)
        pdf = oracle.sparse_run(op, ref_lay, pdf, t, 1)
        torch.cuda.synchronize()
        got = _download(sol, 0)
        ref = oracle.sparse_gather(ref_lay, pdf, t + 1)
        assert np.max(np.abs(got - ref) / ref) <= 1e-5
        del got, ref


def test_empty_and_single_cell_domains():
    lab = np.ones((4, 4, 4), np.uint8)
    dom = lbm.SparseDomain(lab, 7, 19)
    assert dom.n_fluid == 0 and dom.stride == 0
    sol = lbm.Solver(dom, lbm.STORE_F32)
    sol.init()
    sol.step(3, lbm.collision())
    r = sol.reduce(lbm.collision())
    assert r.n_fluid == 0 and r.mass == 0.0
    lab[1, 2, 3] = 0
    dom = lbm.SparseDomain(lab, 7, 19)
    torch.cuda.synchronize()
    _check_index(dom)
    sol = lbm.Solver(dom, lbm.STORE_F64)
    sol.init()
    sol.step(4, lbm.collision(lbm.COLL_SRT, tau=0.9, force=(1e-3, 0, 0)))
    r = sol.reduce(lbm.collision(lbm.COLL_SRT, tau=0.9, force=(1e-3, 0, 0)))
    assert abs(r.mass - 1.0) < 1e-15


# -------------------------------------------------- compact index-list
def _decode_index16(dom):
    """Host decode of the compact index-list (layout documented in lbm.h);
    escaped entries are read from the int32 list."""
    q, S, nf = dom.q, dom.stride, dom.n_fluid
    raw = dom.index16.cpu().numpy()
    idx32 = dom.index[:(q - 1) * S].cpu().numpy().reshape(q - 1, S).astype(np.int64)
    a256 = lambda v: (v + 255) // 256 * 256
    ntiles = (S + 255) // 256
    off = raw[:2 * (q - 1) * S].view(np.uint16).reshape(q - 1, S).astype(np.int64)
    b0 = a256(2 * (q - 1) * S)
    base = raw[b0:b0 + 4 * (q - 1) * ntiles].view(np.int32).reshape(ntiles, q - 1).T.astype(
        np.int64)
    _, _, opp = oracle.stencil(q)
    k = np.arange(nf)
    out = np.empty((q - 1, nf), np.int64)
    n_esc = 0
    for i in range(1, q):
        o = off[i - 1, :nf]
        fl = i * S + k + base[i - 1, k // 256] + o
        out[i - 1] = np.where(o == 0xFFFF, opp[i] * S + k,
                              np.where(o == 0xFFFE, idx32[i - 1, :nf], fl))
        n_esc += int(np.count_nonzero(o == 0xFFFE))
        # entries stored as offsets lie in the fluid block of direction i
        assert np.all((fl[o < 0xFFFE] >= i * S) & (fl[o < 0xFFFE] < (i + 1) * S))
    return out, n_esc


@pytest.mark.parametrize("order", [lbm.ORDER_BLOCKED, lbm.ORDER_LEX, lbm.ORDER_MORTON])
@pytest.mark.parametrize("q", [19, 27])
def test_index16_decodes_to_int32_table(order, q):
    lab = inputs.random_mask((40, 33, 29), 0.35, seed=q + order, n_classes=2, class_fraction=0.3)
    dom = lbm.SparseDomain(lab, 5, q, order)
    dom.compact()
    torch.cuda.synchronize()
    S, nf = dom.stride, dom.n_fluid
    ref = dom.index[:(q - 1) * S].cpu().numpy().reshape(q - 1, S)[:, :nf].astype(np.int64)
    got, n_esc = _decode_index16(dom)
    assert np.array_equal(got, ref)
    assert n_esc == dom.escaped


def test_index16_steps_bitwise_equal_to_int32():
    """The compact index-list changes how positions are stored, not which:
    PDFs, moments and reductions are bitwise those of the int32 path."""
    lab = inputs.random_mask((30, 28, 26), 0.3, seed=4, n_classes=3, class_fraction=0.5)
    coll, bs, _ = _params(27, lbm.COLL_CUMULANT, 0.7, (1e-5, 0, 0), CLASSES)
    d32 = lbm.SparseDomain(lab, 3, 27, lbm.ORDER_BLOCKED)
    d16 = lbm.SparseDomain(lab, 3, 27, lbm.ORDER_BLOCKED)
    d16.compact()
    torch.cuda.synchronize()
    a = lbm.Solver(d32, lbm.STORE_F32)
    b = lbm.Solver(d16, lbm.STORE_F32)
    f0 = _random_state(27, d32.n_fluid, seed=3)
    _upload(a, f0, 0)
    _upload(b, f0, 0)
    a.step(11, coll, bs)
    b.step(11, coll, bs)
    torch.cuda.synchronize()
    assert torch.equal(a.pdf, b.pdf)
    nf = d32.n_fluid
    ra, ua = a.moments(coll)
    rb, ub = b.moments(coll)
    assert torch.equal(ra[:nf], rb[:nf]) and torch.equal(ua[:, :nf], ub[:, :nf])
    xa, xb = a.reduce(coll), b.reduce(coll)
    assert (xa.mass, tuple(xa.mom)) == (xb.mass, tuple(xb.mom))


@pytest.mark.parametrize("order", [2, 1])
def test_index16_full_size_packing(packing256, order):
    """The benchmark geometry: the compact list decodes to the oracle's
    int32 index-list, with escapes only where a tile's offsets form two
    clusters (block borders, the periodic wrap)."""
    lab, per, info, _ = packing256
    ref = oracle.sparse_build(lab, per, 19, order=order, align=64)
    dom = lbm.SparseDomain(lab, per, 19, order)
    frac = dom.compact()
    torch.cuda.synchronize()
    _say("escaped fraction", order, frac)
    nf, S = ref.n_fluid, ref.stride
    assert dom.n_fluid == nf and dom.stride == S
    got, n_esc = _decode_index16(dom)
    assert np.array_equal(got, ref.index.reshape(18, S)[:, :nf])
    assert frac < 0.2


# --------------------------------------------- run-compressed index-list
def _decode_runs(dom):
    """Host decode of the run-compressed index-list (layout documented in
    lbm.h): entries of every list position k < S, shape (q-1, S)."""
    q, S = dom.q, dom.stride
    raw = dom.runs.cpu().numpy()
    a256 = lambda v: (v + 255) // 256 * 256
    nw = (S + 63) // 64
    voff = raw[:4 * (nw + 1)].view(np.uint32).astype(np.int64)
    m0 = a256(4 * (nw + 1))
    mask = raw[m0:m0 + 8 * nw * (q - 1)].view(np.uint64).reshape(nw, q - 1)
    v0 = m0 + a256(8 * nw * (q - 1))
    val = raw[v0:v0 + 4 * int(voff[nw])].view(np.int32).astype(np.int64)
    assert dom.runs_bytes == v0 + 4 * int(voff[nw])
    bits = np.unpackbits(mask.view(np.uint8).reshape(nw, q - 1, 8), axis=2,
                         bitorder="little").astype(bool)            # [w][dir][lane]
    assert bits[:, :, 0].all()                                     # lane 0 starts a run
    counts = bits.sum(axis=2)                                      # runs per wave, direction
    first = voff[:nw, None] + np.concatenate(
        [np.zeros((nw, 1), np.int64), np.cumsum(counts, axis=1)[:, :-1]], axis=1)
    run = np.cumsum(bits, axis=2) - 1                              # run of each lane
    lane = np.arange(64)
    ent = val[first[:, :, None] + run] + lane                     # [w][dir][lane]
    assert int(voff[nw]) == int(counts.sum())
    return ent.transpose(1, 0, 2).reshape(q - 1, nw * 64)[:, :S]


@pytest.mark.parametrize("order", [lbm.ORDER_BLOCKED, lbm.ORDER_LEX, lbm.ORDER_MORTON])
@pytest.mark.parametrize("q", [19, 27])
def test_runs_decode_to_int32_table(order, q):
    """Every entry, padding included, decodes to the int32 index-list; the
    stride is not a multiple of 64 here (align 8), so the last wave is
    partial."""
    for seed in range(2 * q + order, 2 * q + order + 64):
        lab = inputs.random_mask((37, 30, 27), 0.35, seed=seed, n_classes=2,
                                 class_fraction=0.3)
        dom = lbm.SparseDomain(lab, 5, q, order, align=8)
        if dom.stride % 64 != 0:
            break
    bpc = dom.compact_runs()
    torch.cuda.synchronize()
    S = dom.stride
    assert S % 64 != 0
    ref = dom.index[:(q - 1) * S].cpu().numpy().reshape(q - 1, S).astype(np.int64)
    got = _decode_runs(dom)
    assert np.array_equal(got, ref)
    assert bpc < 4 * (q - 1)


def test_runs_capacity_protocol():
    """A header-sized buffer gets the size of the whole form and LBM_ENOMEM;
    a buffer of that size gets the form."""
    lab = inputs.random_mask((20, 18, 16), 0.3, seed=9)
    dom = lbm.SparseDomain(lab, 7, 19, lbm.ORDER_BLOCKED)
    hdr = lbm.lbm_runs_header_bytes(dom.layout)
    buf = torch.zeros(hdr, dtype=torch.uint8, device="cuda")
    rc, need = lbm.lbm_compress_runs(dom.layout, dom.index, buf, hdr)
    assert rc == lbm.LBM_ENOMEM and need > hdr
    buf = torch.zeros(need, dtype=torch.uint8, device="cuda")
    rc, need2 = lbm.lbm_compress_runs(dom.layout, dom.index, buf, need)
    assert rc == lbm.LBM_OK and need2 == need


@pytest.mark.parametrize("q,kind,storage", [(27, lbm.COLL_CUMULANT, lbm.STORE_F32),
                                            (19, lbm.COLL_TRT, lbm.STORE_F64),
                                            (19, lbm.COLL_SRT, lbm.STORE_F16DEV)])
def test_runs_steps_bitwise_equal_to_int32(q, kind, storage):
    """The run form changes how positions are stored, not which: PDFs,
    moments (also at odd t) and reductions are bitwise those of the int32
    path, with boundary links."""
    lab = inputs.random_mask((30, 28, 26), 0.3, seed=5, n_classes=3, class_fraction=0.5)
    coll, bs, _ = _params(q, kind, 0.7, (1e-5, 0, 0), CLASSES)
    d32 = lbm.SparseDomain(lab, 3, q, lbm.ORDER_BLOCKED)
    dr = lbm.SparseDomain(lab, 3, q, lbm.ORDER_BLOCKED)
    dr.compact_runs()
    torch.cuda.synchronize()
    dev_exp = 14 if storage == lbm.STORE_F16DEV else 0
    a = lbm.Solver(d32, storage, dev_exp)
    b = lbm.Solver(dr, storage, dev_exp)
    a.init()
    b.init()
    nf = d32.n_fluid
    for n in (1, 10):
        a.step(n, coll, bs)
        b.step(n, coll, bs)
        torch.cuda.synchronize()
        assert torch.equal(a.pdf, b.pdf)
        ra, ua = a.moments(coll)
        rb, ub = b.moments(coll)
        assert torch.equal(ra[:nf], rb[:nf]) and torch.equal(ua[:, :nf], ub[:, :nf])
        xa, xb = a.reduce(coll), b.reduce(coll)
        assert (xa.mass, tuple(xa.mom)) == (xb.mass, tuple(xb.mom))


@pytest.mark.parametrize("q,kind,storage,align", [(19, lbm.COLL_TRT, lbm.STORE_F32, 8),
                                                  (27, lbm.COLL_CUMULANT, lbm.STORE_F64, 64),
                                                  (19, lbm.COLL_MRT, lbm.STORE_BF16DEV, 1)])
def test_runs_without_int32_index(q, kind, storage, align):
    """With the int32 index-list freed after the run form is built, steps,
    moments at odd and even t (decoded one thread at a time) and reductions
    are bitwise those of the int32 path; strides that are not multiples of
    64 leave a partial last wave.  Pull steps and the compact form refuse
    the state."""
    lab = inputs.random_mask((29, 27, 25), 0.3, seed=11, n_classes=3, class_fraction=0.5)
    coll, bs, _ = _params(q, kind, 0.7, (1e-5, 0, 0), CLASSES)
    d32 = lbm.SparseDomain(lab, 3, q, lbm.ORDER_BLOCKED, align=align)
    dr = lbm.SparseDomain(lab, 3, q, lbm.ORDER_BLOCKED, align=align)
    held = dr.device_bytes()
    dr.compact_runs(drop_index=True)
    torch.cuda.synchronize()
    assert dr.index is None
    assert dr.device_bytes() == held - d32.index.numel() * 4 + dr.runs.numel()
    dev_exp = 14 if storage == lbm.STORE_F16DEV else 0
    a = lbm.Solver(d32, storage, dev_exp)
    b = lbm.Solver(dr, storage, dev_exp)
    assert b.state.index is None
    a.init()
    b.init()
    nf = d32.n_fluid
    for n in (1, 1, 7, 1):
        a.step(n, coll, bs)
        b.step(n, coll, bs)
        torch.cuda.synchronize()
        assert torch.equal(a.pdf, b.pdf)
        for f64 in (True, False):
            ra, ua = a.moments(coll, f64)
            rb, ub = b.moments(coll, f64)
            assert torch.equal(ra[:nf], rb[:nf]) and torch.equal(ua[:, :nf], ub[:, :nf])
        xa, xb = a.reduce(coll), b.reduce(coll)
        assert (xa.mass, tuple(xa.mom)) == (xb.mass, tuple(xb.mom))
    with pytest.raises(lbm.LbmError):
        b.step_pull(2, coll, bs)
    with pytest.raises(ValueError):
        dr.compact()
    # the pull error left the state as it was
    a.step(1, coll, bs)
    b.step(1, coll, bs)
    torch.cuda.synchronize()
    assert torch.equal(a.pdf, b.pdf)


def test_runs_batch_mixes_index_forms():
    """One batch holding int32, compact and run-form solves (one launch per
    form on odd steps) gives each solve the PDFs it gets alone."""
    labs = [inputs.workload_c1(0.6, L=L, seed=L + 1)[0] for L in (40, 48, 56)]
    coll = lbm.collision(lbm.COLL_TRT, tau=0.7, force=(1e-5, 0, 0))
    out = []
    for batched in (False, True):
        sols = []
        for j, lab in enumerate(labs):
            dom = lbm.SparseDomain(lab, 7, 19, lbm.ORDER_BLOCKED)
            if j == 1:
                dom.compact()
            elif j == 2:
                dom.compact_runs()
            s = lbm.Solver(dom, lbm.STORE_F32)
            _upload(s, _random_state(19, dom.n_fluid, seed=j + 1), 0)
            sols.append(s)
        if batched:
            lbm.lbm_step_batch([s.state for s in sols], [coll] * 3, None, 5)
        else:
            for s in sols:
                s.step(5, coll)
        torch.cuda.synchronize()
        out.append([s.pdf.clone() for s in sols])
    for x, y in zip(*out):
        assert torch.equal(x, y)


def test_batch_of_many_solves_matches_each_alone():
    """150 small solves of different sizes, index forms and boundary classes
    (one with no fluid cell), more than a kernel-argument table could hold:
    one launch per step and form reads the segment table from the batch
    workspace; batched steps and batched FP64 reductions equal each solve
    stepped and reduced alone, bit for bit."""
    n = 150
    coll, bs, _ = _params(19, lbm.COLL_TRT, 0.7, (1e-5, 0, 0), CLASSES)
    labs = [inputs.random_mask((6 + j % 5, 7 + j % 3, 5 + j % 4), 0.3, seed=200 + j,
                               n_classes=3 if j % 3 == 0 else 0, class_fraction=0.5)
            for j in range(n)]
    labs[7] = np.ones_like(labs[7])
    _say("batch of", n, "solves")
    out = []
    for batched in (False, True):
        sols = []
        for j, lab in enumerate(labs):
            dom = lbm.SparseDomain(lab, 3 if j % 3 == 0 else 7, 19, lbm.ORDER_BLOCKED)
            if j % 4 == 1:
                dom.compact()
            elif j % 4 == 2 and dom.n_fluid > 0:
                dom.compact_runs(drop_index=True)
            s = lbm.Solver(dom, lbm.STORE_F32)
            if dom.n_fluid > 0:
                _upload(s, _random_state(19, dom.n_fluid, seed=j + 50), 0)
            else:
                s.init()
            sols.append(s)
        if batched:
            ws = torch.empty(lbm.lbm_step_batch_workspace_bytes(n), dtype=torch.uint8,
                             device="cuda")
            lbm.lbm_step_batch([s.state for s in sols], [coll] * n, [bs] * n, 5, workspace=ws)
            ws = torch.empty(sum(lbm.lbm_reduce_workspace_bytes(s.domain.layout) for s in sols),
                             dtype=torch.uint8, device="cuda")
            red = lbm.lbm_reduce_batch([s.state for s in sols], [coll] * n, ws)
        else:
            for s in sols:
                s.step(5, coll, bs)
            red = [s.reduce(coll) for s in sols]
        torch.cuda.synchronize()
        out.append(([s.pdf.clone() for s in sols],
                    [(r.mass, tuple(r.mom), r.n_fluid) for r in red]))
    for a, b in zip(out[0][0], out[1][0]):
        assert torch.equal(a, b)
    assert out[0][1] == out[1][1]


def test_runs_empty_and_single_cell():
    lab = np.ones((4, 4, 4), np.uint8)
    dom = lbm.SparseDomain(lab, 7, 19)
    assert dom.compact_runs() > 0            # the header alone
    sol = lbm.Solver(dom, lbm.STORE_F32)
    sol.init()
    sol.step(3, lbm.collision())
    lab[1, 2, 3] = 0
    dom = lbm.SparseDomain(lab, 7, 19)
    dom.compact_runs()
    torch.cuda.synchronize()
    assert np.array_equal(_decode_runs(dom),
                          dom.index[:18 * dom.stride].cpu().numpy().reshape(18, -1))
    c = lbm.collision(lbm.COLL_SRT, tau=0.9, force=(1e-3, 0, 0))
    sol = lbm.Solver(dom, lbm.STORE_F64)
    sol.init()
    sol.step(4, c)
    assert abs(sol.reduce(c).mass - 1.0) < 1e-15


@pytest.mark.parametrize("order", [2, 1])
def test_runs_full_size_packing(packing256, order):
    """The benchmark geometry: the run form decodes to the oracle's int32
    index-list and needs under 10 bytes per fluid cell (36 for 16-bit
    offsets, 72 for int32)."""
    lab, per, info, _ = packing256
    ref = oracle.sparse_build(lab, per, 19, order=order, align=64)
    dom = lbm.SparseDomain(lab, per, 19, order)
    bpc = dom.compact_runs()
    torch.cuda.synchronize()
    _say("run form bytes per cell", order, bpc)
    nf, S = ref.n_fluid, ref.stride
    assert dom.n_fluid == nf and dom.stride == S
    got = _decode_runs(dom)
    assert np.array_equal(got[:, :nf], ref.index.reshape(18, S)[:, :nf])
    if order == 2:
        assert bpc < 10


def test_runs_without_int32_full_size_packing(packing256):
    """The benchmark geometry with only the run form: after an odd and an
    even step count, moments (decoded one thread at a time at odd t) and
    the FP64 reduction equal those of the int32 path bitwise."""
    lab, per, _, _ = packing256
    coll = lbm.collision(lbm.COLL_TRT, tau=0.8, force=(1e-6, 0, 0))
    a = lbm.Solver(lbm.SparseDomain(lab, per, 19, lbm.ORDER_BLOCKED), lbm.STORE_F32)
    dr = lbm.SparseDomain(lab, per, 19, lbm.ORDER_BLOCKED)
    dr.compact_runs(drop_index=True)
    b = lbm.Solver(dr, lbm.STORE_F32)
    nf = dr.n_fluid
    _upload(a, _random_state(19, nf, seed=3, amp=1e-3), 0)
    b.pdf.copy_(a.pdf)
    for n in (3, 1):
        a.step(n, coll)
        b.step(n, coll)
        ra, ua = a.moments(coll, False)
        rb, ub = b.moments(coll, False)
        torch.cuda.synchronize()
        assert torch.equal(ra[:nf], rb[:nf]) and torch.equal(ua[:, :nf], ub[:, :nf])
        xa, xb = a.reduce(coll), b.reduce(coll)
        assert (xa.mass, tuple(xa.mom)) == (xb.mass, tuple(xb.mom))
    assert torch.equal(a.pdf, b.pdf)


@pytest.mark.parametrize("storage", [lbm.STORE_F64, lbm.STORE_F16DEV])
def test_checkpoint_resume_is_bitwise(tmp_path, storage):
    """A solve written at odd or even t and restored into a solver on a
    rebuilt domain continues bit for bit like the uninterrupted one (links
    and body force included); a different storage or geometry is refused."""
    lab = inputs.random_mask((27, 25, 23), 0.3, seed=41, n_classes=3, class_fraction=0.5)
    coll, bs, _ = _params(19, lbm.COLL_TRT, 0.7, (1e-5, 0, 0), CLASSES)
    dev_exp = 14 if storage == lbm.STORE_F16DEV else 0

    def domain(mask):
        d = lbm.SparseDomain(mask, 3, 19, lbm.ORDER_BLOCKED)
        d.compact_runs(drop_index=True)
        return d

    a = lbm.Solver(domain(lab), storage, dev_exp)
    _upload(a, _random_state(19, a.domain.n_fluid, seed=5), dev_exp)
    paths = {}
    for t in (5, 8):
        a.step(t - a.t, coll, bs)
        paths[t] = str(tmp_path / f"t{t}.npz")
        a.checkpoint(paths[t])
    a.step(13 - a.t, coll, bs)
    torch.cuda.synchronize()
    for t in (5, 8):
        b = lbm.Solver(domain(lab), storage, dev_exp)
        b.init()
        b.restore(paths[t])
        assert b.t == t
        b.step(13 - t, coll, bs)
        torch.cuda.synchronize()
        assert torch.equal(a.pdf, b.pdf)
    other = lbm.STORE_F32 if storage == lbm.STORE_F64 else lbm.STORE_BF16DEV
    with pytest.raises(ValueError):
        lbm.Solver(a.domain, other, dev_exp).restore(paths[5])
    moved = lab.copy()
    fl = np.flatnonzero(moved == 0)
    moved.flat[fl[0]], moved.flat[fl[-1]] = 1, 1
    moved.flat[np.flatnonzero(lab == 1)[:2]] = 0      # same fluid count, other cells
    d2 = domain(moved)
    if d2.n_fluid == a.domain.n_fluid and d2.stride == a.domain.stride:
        with pytest.raises(ValueError):
            lbm.Solver(d2, storage, dev_exp).restore(paths[5])


def test_large_solve_with_positions_beyond_2_31():
    """A fully fluid periodic 600^3 box (216 M cells, 16.4 GB of FP32 PDFs):
    its positions run past 2^31 (q*S = 4.1e9 < 2^32, unsigned 32-bit).  One
    odd step on a random state through the run form, checked on sampled
    cells (including the last list positions, whose slots in the last
    direction blocks lie above 2^31) against the oracle's collision of the
    pulled populations.  A 610^3 box needs q*S >= 2^32 and is refused with
    LBM_ERANGE."""
    n, q = 600, 19
    lab = np.zeros((n, n, n), np.uint8)
    dom = lbm.SparseDomain(lab, 7, q, lbm.ORDER_BLOCKED)
    S, nf = dom.stride, dom.n_fluid
    assert nf == n ** 3 and 2 ** 31 < q * S < 2 ** 32
    dom.compact_runs()
    sol = lbm.Solver(dom, lbm.STORE_F32)
    _, w, _ = oracle.stencil(q)
    gen = torch.Generator(device="cuda").manual_seed(7)
    pdf = sol.pdf.view(q, S)
    for i in range(q):
        pdf[i].copy_(float(w[i]) * (1 + 0.05 * torch.rand(S, generator=gen, device="cuda")))
    rng = np.random.default_rng(3)
    ks = np.concatenate([rng.integers(0, nf, 48), np.arange(nf - 16, nf)])
    kt = torch.from_numpy(ks).cuda()
    lin = dom.cells[kt].long().cpu().numpy()
    inv = torch.empty(nf, dtype=torch.int64, device="cuda")
    inv[dom.cells[:nf].long()] = torch.arange(nf, device="cuda")
    c, _, opp = oracle.stencil(q)
    x, y, z = lin % n, (lin // n) % n, lin // (n * n)
    pulled = np.empty((len(ks), q))
    for i in range(q):
        up = ((x - c[i, 0]) % n) + n * (((y - c[i, 1]) % n) + n * ((z - c[i, 2]) % n))
        m = inv[torch.from_numpy(up).cuda()]
        pulled[:, i] = pdf[i, m].double().cpu().numpy()
    coll = lbm.collision(lbm.COLL_TRT, tau=0.8, force=(1e-5, 0, 0))
    p = oracle.params(q=q, kind=oracle.TRT, tau=0.8, magic=3 / 16, force=(1e-5, 0, 0))
    want = oracle.collide(p, pulled)
    del inv
    sol.step(1, coll)
    got = np.empty_like(want)
    idx = dom.index.view(q - 1, S)
    above = 0
    for j in range(q):
        pos = kt if j == 0 else idx[opp[j] - 1, kt].long() & 0xFFFFFFFF
        above += int((pos >= 2 ** 31).sum())
        got[:, j] = sol.pdf[pos].double().cpu().numpy()
    assert above > 0
    _say("large solve: max abs diff", np.max(np.abs(got - want)), "positions above 2^31:", above)
    assert np.max(np.abs(got - want)) < 1e-6
    del sol, dom, pdf, idx
    torch.cuda.empty_cache()
    with pytest.raises(lbm.LbmError) as e:
        lbm.SparseDomain(np.zeros((610, 610, 610), np.uint8), 7, q, lbm.ORDER_BLOCKED)
    assert e.value.code == lbm.LBM_ERANGE


# ------------------------------------------------------------ pull scheme
@pytest.mark.parametrize("compact,kind", [(False, lbm.COLL_TRT), (True, lbm.COLL_TRT),
                                          (False, lbm.COLL_MRT)])
def test_pull_scheme_bitwise_equals_aa(compact, kind):
    """An AA odd+even pair performs the same collisions on the same inputs
    as two pull steps (Section "In-place Streaming: AA Pattern"), so after
    every even step count the two schemes agree bit for bit (links too)."""
    lab = inputs.random_mask((22, 19, 17), 0.3, seed=6, n_classes=3, class_fraction=0.5)
    coll, bs, op = _params(19, kind, 0.75, (1e-5, 0, 0), CLASSES)
    doms = [lbm.SparseDomain(lab, 5, 19, lbm.ORDER_BLOCKED) for _ in range(2)]
    if compact:
        for d in doms:
            d.compact()
    torch.cuda.synchronize()
    _check_index(doms[0])
    a, b = lbm.Solver(doms[0], lbm.STORE_F32), lbm.Solver(doms[1], lbm.STORE_F32)
    f0 = _random_state(19, doms[0].n_fluid, seed=8)
    _upload(a, f0, 0)
    _upload(b, f0, 0)
    a.step(10, coll, bs)
    b.step_pull(10, coll, bs)
    torch.cuda.synchronize()
    assert a.t == b.t == 10
    S, nf = doms[0].stride, doms[0].n_fluid
    pa = a.pdf.view(19, S)[:, :nf]
    pb = b.pdf.view(19, S)[:, :nf]
    assert torch.equal(pa, pb)
    b.step(2, coll, bs)          # continues with AA steps from the pull state
    a.step(2, coll, bs)
    torch.cuda.synchronize()
    assert torch.equal(a.pdf.view(19, S)[:, :nf], b.pdf.view(19, S)[:, :nf])


@pytest.mark.parametrize("storage,compact,kind", [(lbm.STORE_F64, False, lbm.COLL_TRT),
                                                  (lbm.STORE_F32, False, lbm.COLL_TRT),
                                                  (lbm.STORE_F64, True, lbm.COLL_MRT),
                                                  (lbm.STORE_F32DEV, True, lbm.COLL_SRT)])
def test_pull_scheme_matches_dense_oracle(storage, compact, kind):
    """The two-array pull kernel against the oracle's dense pull scheme (the
    same scheme, written independently): 10 steps with inlet (UBB) and
    outlet (pressure) links on a partly periodic random packing, within
    1e-12 relative in FP64 and 1e-5 in FP32 storage on every fluid cell."""
    _say("pull vs oracle", storage, compact, kind)
    q = 19
    lab = inputs.random_mask((21, 17, 19), 0.3, seed=31 + kind, n_classes=3,
                             class_fraction=0.5)
    per = 5
    coll, bs, op = _params(q, kind, 0.7, (2e-5, -1e-5, 5e-6), CLASSES)
    dom = lbm.SparseDomain(lab, per, q, lbm.ORDER_BLOCKED)
    if compact:
        dom.compact()
    torch.cuda.synchronize()
    _check_index(dom)
    assert dom.n_links > 0
    sol = lbm.Solver(dom, storage)
    seen = _upload(sol, _random_state(q, dom.n_fluid, seed=5 + kind), 0)
    cells = dom.cells[:dom.n_fluid].cpu().numpy()
    A = _dense_from_list(seen, cells, lab.shape, q)
    tol = 1e-12 if storage == lbm.STORE_F64 else 1e-5
    for n in (2, 8):
        sol.step_pull(n, coll, bs)
        A = oracle.dense_run(op, lab, per, n, A)
        torch.cuda.synchronize()
        got = _download(sol, 0)
        ref = A.reshape(q, -1)[:, cells]
        err = float(np.max(np.abs(got - ref) / np.abs(ref)))
        assert err <= tol, (sol.t, err)
    assert sol.t == 10


# ------------------------------------------------------------ vessel tree
def _vessel_params():
    classes = [(lbm.BC_UBB, (0.0, 0.0, 0.02), 1.0), (lbm.BC_PRESSURE, (0, 0, 0), 1.0)]
    return _params(27, lbm.COLL_CUMULANT, 0.6, (0.0, 0.0, 0.0), classes)


def test_vessel_tree_small_matches_dense_oracle():
    """A 48^3 tree with the benchmark's branching rules: D3Q27 cumulant FP32
    with the UBB inlet and pressure outlets, 100 steps, against the dense
    FP64 oracle."""
    lab, per, info = inputs.vessel_tree(n=48, r0=5.0, k_len=5.0, r_min=1.5, seed=3)
    assert info["n_fluid"] > 1000 and (lab == 2).any() and (lab == 3).any()
    coll, bs, op = _vessel_params()
    dom = lbm.SparseDomain(lab, per, 27, lbm.ORDER_BLOCKED)
    dom.compact()
    torch.cuda.synchronize()
    _check_index(dom)
    sol = lbm.Solver(dom, lbm.STORE_F32)
    sol.init()
    sol.step(100, coll, bs)
    A = oracle.dense_run(op, lab, per, 100, oracle.dense_init(27, lab))
    torch.cuda.synchronize()
    cells = dom.cells[:dom.n_fluid].cpu().numpy()
    got = _download(sol, 0)
    ref = A.reshape(27, -1)[:, cells]
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-5


def test_vessel_tree_full_size_two_steps():
    """The 512^3 benchmark tree in the benchmark's launch configuration: one
    odd and one even step from a perturbed state against the oracle's sparse
    AA scheme (links included), every fluid cell."""
    lab, per, info = inputs.workload_vessel()
    _say("vessel full size", info["n_fluid"], info["n_outlets"])
    coll, bs, op = _vessel_params()
    dom = lbm.SparseDomain(lab, per, 27, lbm.ORDER_BLOCKED)
    dom.compact_runs()            # the benchmark's index form
    torch.cuda.synchronize()
    sol = lbm.Solver(dom, lbm.STORE_F32)
    seen = _upload(sol, _random_state(27, dom.n_fluid, seed=2, amp=1e-3), 0)
    ref_lay = oracle.sparse_build(lab, per, 27, order=2, align=64)
    assert np.array_equal(ref_lay.cells, dom.cells[:dom.n_fluid].cpu().numpy())
    assert ref_lay.n_links == dom.n_links
    pdf = np.zeros(27 * ref_lay.stride)
    for i in range(27):
        pdf[i * ref_lay.stride:i * ref_lay.stride + dom.n_fluid] = seen[i]
    for t in range(2):
        sol.step(1, coll, bs)
        pdf = oracle.sparse_run(op, ref_lay, pdf, t, 1)
        torch.cuda.synchronize()
        got = _download(sol, 0)
        ref = oracle.sparse_gather(ref_lay, pdf, t + 1)
        assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-5


def test_pipelined_odd_kernel_is_bitwise_identical():
    """The persistent, pipelined odd kernel performs the same per-cell
    arithmetic: identical PDFs to the one-tile-per-workgroup kernel, also
    for a batch of solves (tiles of several segments in one launch)."""
    labs = [inputs.workload_c1(0.6, L=L, seed=L)[0] for L in (64, 72, 96)]
    coll = lbm.collision(lbm.COLL_TRT, tau=0.7, force=(1e-5, 0, 0))
    runs = []
    old = lbm.lbm_get_launch(lbm.KERNEL_ODD, 19, lbm.STORE_F32, full=True)
    try:
        for pipelined in (0, 1):
            lbm.lbm_set_launch(lbm.KERNEL_ODD, 19, lbm.STORE_F32, 256, 1, pipelined)
            sols = []
            for lab in labs:
                dom = lbm.SparseDomain(lab, 7, 19, lbm.ORDER_BLOCKED)
                assert dom.compact() > 0          # some escaped entries
                s = lbm.Solver(dom, lbm.STORE_F32)
                _upload(s, _random_state(19, dom.n_fluid, seed=dom.n_fluid), 0)
                sols.append(s)
            sols[2].step(6, coll)
            lbm.lbm_step_batch([s.state for s in sols[:2]], [coll, coll], None, 6)
            torch.cuda.synchronize()
            runs.append([s.pdf.clone() for s in sols])
    finally:
        lbm.lbm_set_launch(lbm.KERNEL_ODD, 19, lbm.STORE_F32, *old)
    for a, b in zip(*runs):
        assert torch.equal(a, b)


@pytest.mark.parametrize("storage", [lbm.STORE_F64, lbm.STORE_F32, lbm.STORE_F16DEV])
def test_default_launch_odd_and_even_strides_agree(storage):
    """With the library's default launch table, an even stride (two cells
    per thread where the table says so) and an odd one (the one-cell
    fallback, without the two-cell kernel's residency cap) give the same
    PDFs on the fluid cells, bit for bit."""
    lab = inputs.random_mask((25, 23, 21), 0.3, seed=61, n_classes=3, class_fraction=0.5)
    if np.count_nonzero(lab == 0) % 2 == 0:       # odd fluid count: odd stride at align 1
        lab[np.unravel_index(np.flatnonzero(lab == 1)[0], lab.shape)] = 0
    coll, bs, _ = _params(19, lbm.COLL_TRT, 0.7, (1e-5, 0, 0), CLASSES)
    dev_exp = 14 if storage == lbm.STORE_F16DEV else 0
    out = []
    for align in (64, 1):
        dom = lbm.SparseDomain(lab, 3, 19, lbm.ORDER_BLOCKED, align=align)
        assert (dom.stride % 2 == 1) == (align == 1)
        dom.compact_runs()
        s = lbm.Solver(dom, storage, dev_exp)
        _upload(s, _random_state(19, dom.n_fluid, seed=8), dev_exp)
        s.step(6, coll, bs)
        torch.cuda.synchronize()
        out.append(s.pdf.view(19, -1)[:, :dom.n_fluid].clone())
    assert torch.equal(out[0], out[1])


@pytest.mark.parametrize("q,kind,storage", [(19, lbm.COLL_TRT, lbm.STORE_F32),
                                            (19, lbm.COLL_TRT, lbm.STORE_F64),
                                            (27, lbm.COLL_CM, lbm.STORE_F16DEV)])
def test_residency_caps_are_bitwise_identical(q, kind, storage):
    """Capping the resident workgroups per CU (reserved LDS) and the tile
    order over the XCDs change where and when tiles run, not the
    arithmetic: PDFs after odd and even step counts are identical for every
    cap, block size and tile order (dispatch order, one eighth per XCD,
    chunks of 3 and 16 tiles, whose last partial round maps to itself),
    alone and batched."""
    lab = inputs.random_mask((26, 22, 20), 0.3, seed=21, n_classes=3, class_fraction=0.5)
    coll, bs, _ = _params(q, kind, 0.7, (1e-5, 0, 0), CLASSES)
    dev_exp = 14 if storage == lbm.STORE_F16DEV else 0
    old = [lbm.lbm_get_launch(k, q, storage, full=True) for k in (0, 1)]
    out = []
    try:
        for block, g, x in ((256, 0, None), (256, 2, 0), (256, 4, 1), (128, 3, 3),
                            (64, 16, 16), (64, 0, 3)):
            for k in (0, 1):
                b0, x0, _, c0, _ = old[k]
                lbm.lbm_set_launch(k, q, storage, block, x0 if x is None else x, 0, c0, g)
            sols = []
            for j, sub in enumerate((lab, lab[:, 1:, :])):
                d = lbm.SparseDomain(sub, 3, q, lbm.ORDER_BLOCKED)
                d.compact_runs()
                s = lbm.Solver(d, storage, dev_exp)
                _upload(s, _random_state(q, d.n_fluid, seed=j + 31), dev_exp)
                sols.append(s)
            sols[0].step(4, coll, bs)
            lbm.lbm_step_batch([s.state for s in sols], [coll, coll], [bs, bs], 5)
            torch.cuda.synchronize()
            out.append([s.pdf.clone() for s in sols])
    finally:
        for k in (0, 1):
            lbm.lbm_set_launch(k, q, storage, *old[k])
    for run in out[1:]:
        for a, b in zip(out[0], run):
            assert torch.equal(a, b)


@pytest.mark.parametrize("q,kind,storage", [(19, lbm.COLL_TRT, lbm.STORE_F32),
                                            (19, lbm.COLL_SRT, lbm.STORE_F16DEV),
                                            (19, lbm.COLL_TRT, lbm.STORE_F64),
                                            (27, lbm.COLL_CUMULANT, lbm.STORE_BF16DEV)])
def test_even_kernel_two_cells_per_thread_is_bitwise_identical(q, kind, storage):
    """The even kernel with two cells per thread performs each cell's
    arithmetic unchanged: identical PDFs to one cell per thread, alone and
    in a batch, with boundary links and an odd fluid-cell count (the last
    pair ends in a padding slot)."""
    lab = inputs.random_mask((23, 21, 19), 0.3, seed=12, n_classes=3, class_fraction=0.5)
    if np.count_nonzero(lab == 0) % 2 == 0:       # make the fluid-cell count odd
        lab[np.unravel_index(np.flatnonzero(lab == 1)[0], lab.shape)] = 0
    coll, bs, _ = _params(q, kind, 0.7, (1e-5, 0, 0), CLASSES)
    dev_exp = 14 if storage == lbm.STORE_F16DEV else 0
    old = lbm.lbm_get_launch(lbm.KERNEL_EVEN, q, storage, full=True)
    out = []
    try:
        for cpt in (1, 2):
            lbm.lbm_set_launch(lbm.KERNEL_EVEN, q, storage, 256, 0, 0, cpt)
            doms = [lbm.SparseDomain(lab, 3, q, lbm.ORDER_BLOCKED),
                    lbm.SparseDomain(lab[:, :, 1:], 3, q, lbm.ORDER_BLOCKED)]
            # an unpadded list with an odd stride falls back to one cell per
            # thread (stepped alone below)
            odd = lbm.SparseDomain(lab, 3, q, lbm.ORDER_BLOCKED, align=1)
            assert odd.stride == odd.n_fluid and odd.stride % 2 == 1
            so = lbm.Solver(odd, storage, dev_exp)
            _upload(so, _random_state(q, odd.n_fluid, seed=9), dev_exp)
            so.step(5, coll, bs)
            sols = []
            for j, d in enumerate(doms):
                d.compact_runs()
                s = lbm.Solver(d, storage, dev_exp)
                _upload(s, _random_state(q, d.n_fluid, seed=j + 4), dev_exp)
                sols.append(s)
            assert doms[0].n_fluid % 2 == 1
            sols[0].step(6, coll, bs)
            lbm.lbm_step_batch([s.state for s in sols], [coll, coll], [bs, bs], 5)
            torch.cuda.synchronize()
            out.append([s.pdf[:q * s.domain.stride].view(q, -1)[:, :s.domain.n_fluid].clone()
                        for s in sols + [so]])
    finally:
        lbm.lbm_set_launch(lbm.KERNEL_EVEN, q, storage, *old)
    for a, b in zip(*out):
        d = (a.double() - b.double()).abs()
        bad = torch.nonzero(d)
        assert torch.equal(a, b), (float(d.max()), bad.shape[0], bad[:5].tolist())


def test_convert_storage_formats():
    """lbm_convert: FP16 deviations convert to FP32 deviations and FP64
    exactly (value for value, at an odd step count, so in swapped slots),
    FP64 -> FP16 gives back the same codes, the step count is kept, and the
    converted state steps on (the serving tests check the accuracy of a
    solve continued after conversion)."""
    lab = inputs.random_mask((20, 17, 15), 0.3, seed=21)
    dom = lbm.SparseDomain(lab, 7, 19, lbm.ORDER_BLOCKED)
    q, S, nf = 19, dom.stride, dom.n_fluid
    coll = lbm.collision(lbm.COLL_TRT, tau=0.8, force=(1e-5, 0, 0))
    a = lbm.Solver(dom, lbm.STORE_F16DEV, 14)
    _upload(a, _random_state(q, nf, seed=5, amp=1e-2), 14)
    a.step(3, coll)                                   # odd t: swapped slots
    b = a.converted(lbm.STORE_F32DEV)
    c = a.converted(lbm.STORE_F64)
    torch.cuda.synchronize()
    assert b.t == c.t == a.t == 3
    da = _download(a, 14)
    assert np.array_equal(_download(b, 0), da) and np.array_equal(_download(c, 0), da)
    # FP64 -> FP16 rounds to the nearest code, as the host codec does
    d = c.converted(lbm.STORE_F16DEV, 14)
    torch.cuda.synchronize()
    assert torch.equal(d.pdf[:q * S].view(q, S)[:, :nf], a.pdf[:q * S].view(q, S)[:, :nf])
    b.step(1, coll)
    r = b.reduce(coll)
    assert b.t == 4 and r.finite and abs(r.mass - a.reduce(coll).mass) < 1e-5 * r.mass
    # layouts must match
    other = lbm.SparseDomain(lab[:, :, 1:], 7, 19, lbm.ORDER_BLOCKED)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_convert(a.state, lbm.Solver(other, lbm.STORE_F32).state)


# ------------------------------------------------- link-velocity buffer
def _link_vel_host(sol):
    """(marked cells, sums (rho - 1, j)) held by a solve's link-velocity
    buffer."""
    dom = sol.domain
    q, S = dom.q, dom.stride
    W = (S + 63) // 64
    a256 = lambda v: (v + 255) // 256 * 256  # noqa: E731
    raw = sol.link_vel.cpu().numpy()
    mask = raw[:8 * W].view(np.uint64)
    woff = raw[a256(8 * W):a256(8 * W) + 4 * (W + 1)].view(np.uint32)
    bits = np.unpackbits(mask.view(np.uint8), bitorder="little").reshape(W, 64)
    cells = np.nonzero(bits.reshape(-1))[0]
    assert woff[W] == len(cells)
    assert np.array_equal(woff[:W], np.concatenate([[0], np.cumsum(bits.sum(1))[:-1]]))
    dt = np.float64 if sol.storage == lbm.STORE_F64 else np.float32
    base = a256(8 * W) + a256(4 * (W + 1))
    sums = raw[base:base + 4 * len(cells) * np.dtype(dt).itemsize].view(dt).reshape(-1, 4)
    return cells, sums


LINK_VEL_CASES = [(19, lbm.COLL_TRT, lbm.STORE_F64, "runs", 64),
                  (19, lbm.COLL_TRT, lbm.STORE_F64, "runs", 1),
                  (19, lbm.COLL_TRT, lbm.STORE_F32, "i32", 64),
                  (19, lbm.COLL_TRT, lbm.STORE_F16DEV, "runs", 64),
                  (19, lbm.COLL_TRT, lbm.STORE_F16DEV, "i32", 1),
                  (19, lbm.COLL_MRT, lbm.STORE_F32DEV, "i16", 64),
                  (27, lbm.COLL_CUMULANT, lbm.STORE_F32, "runs", 64),
                  (27, lbm.COLL_CUMULANT, lbm.STORE_BF16DEV, "i32", 64),
                  (27, lbm.COLL_CM, lbm.STORE_F64, "i16", 64)]


@pytest.mark.parametrize("q,kind,storage,form,align", LINK_VEL_CASES)
def test_link_velocity_buffer_is_bitwise_identical(q, kind, storage, form, align):
    """With the link-velocity buffer the step kernels hand the boundary
    cells' density and momentum to the next link update; the PDFs stay bit
    for bit those of the gathering link update, over calls of 1 and several
    steps ending at both parities, a force that changes between calls and a
    PDF-list written from outside, and the buffer holds the sums of exactly
    the cells that have links."""
    _say("link vel", q, kind, storage, form, align)
    lab = inputs.random_mask((19, 14, 23), 0.3, seed=5 * q + kind, n_classes=3,
                             class_fraction=0.5)
    coll, bs, _ = _params(q, kind, 0.7, (2e-5, -1e-5, 5e-6), CLASSES, omega_bulk=1.2)
    coll2, _, _ = _params(q, kind, 0.7, (-3e-5, 2e-5, 1e-5), CLASSES, omega_bulk=1.2)
    dev_exp = 10 if storage in (lbm.STORE_F16DEV, lbm.STORE_BF16DEV) else 0
    sols = []
    for use in (False, True):
        dom = lbm.SparseDomain(lab, 5, q, lbm.ORDER_BLOCKED, align=align)
        if form == "runs":
            dom.compact_runs()
        elif form == "i16":
            dom.compact()
        torch.cuda.synchronize()
        if not use:
            _check_index(dom)
        s = lbm.Solver(dom, storage, dev_exp, link_vel=use)
        assert (s.link_vel is not None) == use and dom.n_links > 0
        _upload(s, _random_state(q, dom.n_fluid, seed=q + kind, amp=1e-3), dev_exp)
        sols.append(s)
    ln = sols[1].domain.links[:2 * sols[1].domain.n_links].cpu().numpy().astype(np.int64)
    _, _, opp = oracle.stencil(q)
    S = sols[1].domain.stride
    link_cells = np.unique(ln[0::2] - opp[ln[1::2] & 0xff] * S)
    c, _, _ = oracle.stencil(q)
    for n, cl in ((1, coll), (5, coll), (2, coll2), (9, coll)):
        for s in sols:
            s.step(n, cl, bs)
        torch.cuda.synchronize()
        assert torch.equal(sols[0].pdf, sols[1].pdf), (sols[1].t, n)
        cells, sums = _link_vel_host(sols[1])
        assert np.array_equal(cells, link_cells)
        # written by the call's last step kernel: the sums at sol.t
        f = _download(sols[1], dev_exp)[:, cells]
        ref = np.vstack([f.sum(0) - 1.0, c.T.astype(float) @ f])
        tol = 1e-12 if storage == lbm.STORE_F64 else 1e-5
        assert np.max(np.abs(sums.T - ref)) <= tol * max(np.max(np.abs(ref)), 1e-3)
    # a PDF-list written from outside clears the stamp: the next step gathers
    for s in sols:
        _upload(s, _random_state(q, s.domain.n_fluid, seed=7 * q + kind, amp=1e-3), dev_exp)
        s.step(3, coll, bs)
    torch.cuda.synchronize()
    assert torch.equal(sols[0].pdf, sols[1].pdf)


def test_link_velocity_buffer_batch_and_pull():
    """Two vessel-tree solves advanced in one batch, each with its own
    link-velocity buffer, and a pull-scheme solve: the same bits as without
    the buffers."""
    lab, per, _ = inputs.vessel_tree(n=40, r0=4.0, k_len=5.0, r_min=1.5, seed=4)
    coll, bs, _ = _vessel_params()
    out = []
    for use in (False, True):
        sols = []
        for j in range(2):
            dom = lbm.SparseDomain(lab, per, 27, lbm.ORDER_BLOCKED)
            dom.compact_runs()
            s = lbm.Solver(dom, lbm.STORE_F32, link_vel=use)
            _upload(s, _random_state(27, dom.n_fluid, seed=40 + j, amp=1e-3), 0)
            sols.append(s)
        lbm.lbm_step_batch([s.state for s in sols], [coll, coll], [bs, bs], 7)
        dom = lbm.SparseDomain(lab, per, 27, lbm.ORDER_BLOCKED)
        p = lbm.Solver(dom, lbm.STORE_F32, link_vel=use)
        _upload(p, _random_state(27, dom.n_fluid, seed=42, amp=1e-3), 0)
        p.step_pull(8, coll, bs)
        torch.cuda.synchronize()
        out.append([s.pdf.clone() for s in sols] + [p.pdf.clone()])
    for a, b in zip(*out):
        assert torch.equal(a, b)
