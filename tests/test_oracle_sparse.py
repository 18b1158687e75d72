"""Pins of the oracle's sparse variant: the list builder (brute force on tiny
masks, the permutation invariant, the paper's worked example, Morton order)
and the in-place AA scheme against the dense pull scheme."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_2408_06880_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_force_tables(lab, periodic, q, order, align):
    """Direct, coordinate-by-coordinate restatement of the index rule of
    Section 'Sparse Data Structure' / 'Sparse Boundary Conditions'."""
    c, _, opp = oracle.stencil(q)
    nz, ny, nx = lab.shape
    fluid = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx) if lab[z, y, x] == 0]

    def key(p):
        if order == 1:
            return p[0] + nx * (p[1] + ny * p[2])
        if order == 2:
            ty, tz = p[1] // 8, p[2] // 8
            t = 0
            for b in range(8):
                t |= ((ty >> b) & 1) << (2 * b)
                t |= ((tz >> b) & 1) << (2 * b + 1)
            return (t, p[2] % 8, p[1] % 8, p[0])
        k = 0
        for b in range(10):
            for a in range(3):
                k |= ((p[a] >> b) & 1) << (3 * b + a)
        return k

    fluid.sort(key=key)
    nf = len(fluid)
    S = -(-nf // align) * align
    pos_of = {p: k for k, p in enumerate(fluid)}
    index = np.full((q - 1) * S, -1, np.int64)
    links = []
    dims = (nx, ny, nz)
    for k, p in enumerate(fluid):
        for i in range(1, q):
            yv = [p[a] - c[i, a] for a in range(3)]
            outside = False
            for a in range(3):
                if yv[a] < 0 or yv[a] >= dims[a]:
                    if (periodic >> a) & 1:
                        yv[a] %= dims[a]
                    else:
                        outside = True
            lab_y = 1 if outside else int(lab[yv[2], yv[1], yv[0]])
            if lab_y == 0:
                index[(i - 1) * S + k] = i * S + pos_of[tuple(yv)]
            else:
                index[(i - 1) * S + k] = opp[i] * S + k
            if lab_y >= 2:
                links += [opp[i] * S + k, i | ((lab_y - 2) << 8)]
    cells = np.array([p[0] + nx * (p[1] + ny * p[2]) for p in fluid], np.int64)
    return nf, S, cells, index, np.array(links, np.int64)


CASES = [((5, 4, 3), 0.3, 7, 19, 0, 1), ((6, 6, 6), 0.5, 0, 19, 0, 64),
         ((4, 7, 5), 0.2, 5, 27, 0, 8), ((8, 3, 5), 0.4, 3, 27, 1, 1),
         ((3, 3, 3), 0.0, 7, 19, 1, 4), ((7, 5, 6), 0.6, 2, 19, 0, 16),
         ((9, 19, 17), 0.3, 7, 19, 2, 64), ((5, 20, 9), 0.4, 3, 27, 2, 1)]


@pytest.mark.parametrize("shape,solid,periodic,q,order,align", CASES)
def test_builder_brute_force(shape, solid, periodic, q, order, align):
    lab = inputs.random_mask(shape[::-1], solid, seed=sum(shape) + q, n_classes=3,
                             class_fraction=0.4)
    lay = oracle.sparse_build(lab, periodic, q, order=order, align=align)
    nf, S, cells, index, links = brute_force_tables(lab, periodic, q, order, align)
    assert lay.n_fluid == nf == int(np.count_nonzero(lab == 0))
    assert lay.stride == S and S % align == 0 and S - nf < align
    assert np.array_equal(lay.cells, cells)
    got = lay.index.astype(np.int64)
    for i in range(1, q):
        blk = slice((i - 1) * S, (i - 1) * S + nf)
        assert np.array_equal(got[blk], index[blk])
    assert np.array_equal(lay.links.astype(np.int64), links)


@pytest.mark.parametrize("shape,solid,periodic,q,order,align", CASES)
def test_index_table_is_a_permutation(shape, solid, periodic, q, order, align):
    """Each slot i*S + m (i >= 1, m < N_F) is pulled by exactly one (cell,
    direction): the property that makes the in-place AA update race-free."""
    lab = inputs.random_mask(shape[::-1], solid, seed=100 + sum(shape), n_classes=2,
                             class_fraction=0.5)
    lay = oracle.sparse_build(lab, periodic, q, order=order, align=align)
    S, nf = lay.stride, lay.n_fluid
    used = np.concatenate([lay.index[(i - 1) * S:(i - 1) * S + nf] for i in range(1, q)])
    expect = np.concatenate([i * S + np.arange(nf) for i in range(1, q)])
    assert np.array_equal(np.sort(used), np.sort(expect))


def test_fully_fluid_periodic_and_isolated_cell():
    q = 19
    c, _, opp = oracle.stencil(q)
    lab, per = inputs.periodic_box(4, 4, 4)
    lay = oracle.sparse_build(lab, per, q, order=1, align=1)
    S = lay.stride
    for i in range(1, q):
        for k in range(lay.n_fluid):
            x, y, z = k % 4, (k // 4) % 4, k // 16
            m = ((x - c[i, 0]) % 4) + 4 * (((y - c[i, 1]) % 4) + 4 * ((z - c[i, 2]) % 4))
            assert lay.index[(i - 1) * S + k] == i * S + m
    lab = np.ones((3, 3, 3), np.uint8)
    lab[1, 1, 1] = 0
    lay = oracle.sparse_build(lab, 7, q, order=0, align=1)
    assert lay.n_fluid == 1
    for i in range(1, q):
        assert lay.index[i - 1] == opp[i]


def test_worked_example_of_the_paper():
    """The paper's printed positions (10 fluid cells, west block at 40, east
    block at 20): the west population of cell 0 (position 40) pulls position
    41 (cell 1's west population, the right neighbour), and the west
    population of cell 1 (position 41), whose right neighbour is no-slip,
    pulls its own east population at 21.  We build a row of 10 fluid cells
    where cell 1's right neighbour is solid and map the oracle's direction
    blocks onto the paper's block bases."""
    g = json.load(open(os.path.join(GOLDEN, "sparse_worked_example.json")))
    q = 19
    c, _, opp = oracle.stencil(q)
    west = [i for i in range(q) if tuple(c[i]) == (-1, 0, 0)][0]
    east = opp[west]
    # 2-D arrangement: cells 0,1 in a row with solid to the right of cell 1,
    # the other 8 cells elsewhere in lexicographic order after them.
    lab = np.ones((1, 3, 12), np.uint8)
    lab[0, 0, 0:2] = 0          # cells 0, 1 ; (2,0) solid
    lab[0, 2, 1:9] = 0          # cells 2..9
    lay = oracle.sparse_build(lab, 0, q, order=1, align=1)
    S = lay.stride
    assert lay.n_fluid == S == g["n_fluid"]
    # translate oracle positions d*S + k into the paper's numbering, where
    # the west block starts at 40 and the east block at 20
    paper_base = {west: g["west_block_base"], east: g["east_block_base"]}

    def to_paper(pos):
        d, k = divmod(int(pos), S)
        return paper_base[d] + k

    assert to_paper(west * S + 0) == g["west_pdf_of_cell0"]
    assert to_paper(lay.index[(west - 1) * S + 0]) == g["west_pull_of_cell0"]
    assert to_paper(west * S + 1) == g["west_pdf_of_cell1"]
    assert to_paper(lay.index[(west - 1) * S + 1]) == \
        g["west_pull_of_cell1_when_east_neighbour_is_noslip"]
    assert to_paper(west * S + 9) == g["west_pdf_of_cell9"]


def test_morton_keys():
    """Bit interleave with x in the lowest bit; the builder's fluid list is
    in strictly increasing key order."""
    assert oracle.morton_key(1, 0, 0) == 1
    assert oracle.morton_key(0, 1, 0) == 2
    assert oracle.morton_key(0, 0, 1) == 4
    # x = 3 = 011b, y = 5 = 101b, z = 6 = 110b; bit triple b holds (z_b y_b x_b):
    # b0 -> 011, b1 -> 101, b2 -> 110
    assert oracle.morton_key(3, 5, 6) == 0b110_101_011
    assert oracle.morton_key(1023, 1023, 1023) == (1 << 30) - 1
    lab = inputs.random_mask((9, 10, 11), 0.3, seed=1)
    lay = oracle.sparse_build(lab, 7, 19, order=0)
    xs = lay.cells % 11
    ys = (lay.cells // 11) % 10
    zs = lay.cells // 110
    keys = [oracle.morton_key(int(x), int(y), int(z)) for x, y, z in zip(xs, ys, zs)]
    assert all(a < b for a, b in zip(keys, keys[1:]))


def _classes():
    return [(oracle.BC_UBB, (0.0, 0.0, 0.02), 1.0), (oracle.BC_PRESSURE, (0, 0, 0), 1.001),
            (oracle.BC_UBB, (0.01, -0.01, 0.0), 1.0)]


SPARSE_CASES = [(19, oracle.SRT, 7), (19, oracle.TRT, 0), (19, oracle.NONE, 5),
                (27, oracle.CUMULANT, 3), (27, oracle.TRT, 7)]


@pytest.mark.parametrize("q,kind,periodic", SPARSE_CASES)
def test_sparse_aa_equals_dense_pull(q, kind, periodic):
    """One AA odd+even pair equals two pull steps (Section 'In-place
    Streaming: AA Pattern'): after every even step count the sparse state
    equals the dense one, including boundary links of every class; after
    odd counts the parity-aware gather recovers it."""
    lab = inputs.random_mask((6, 7, 8), 0.35, seed=q + kind, n_classes=3, class_fraction=0.5)
    p = oracle.params(q=q, kind=kind, tau=0.7, magic=3 / 16, force=(2e-5, -1e-5, 5e-6),
                      classes=_classes())
    rng = np.random.default_rng(1)
    A0 = oracle.dense_init(q, lab) * (1 + 0.01 * rng.standard_normal((q,) + lab.shape))
    lay = oracle.sparse_build(lab, periodic, q, order=0, align=8)
    pdf = oracle.sparse_init(lay, A0)
    t = 0
    A = A0
    for n in (1, 1, 2, 4):
        pdf = oracle.sparse_run(p, lay, pdf, t, n)
        A = oracle.dense_run(p, lab, periodic, n, A)
        t += n
        got = oracle.sparse_gather(lay, pdf, t)
        ref = A.reshape(q, -1)[:, lay.cells]
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)), t


def test_sparse_aa_matches_dense_on_packing():
    """Sphere packing, D3Q19 SRT, FP64, 100 steps: sparse AA == dense pull."""
    lab, info = inputs.rsa_spheres(16, 2.0, 3.0, 0.6, seed=2, max_rejects=3000)
    p = oracle.params(q=19, kind=oracle.SRT, tau=0.8, force=(1e-6, 0, 0))
    A0 = oracle.dense_init(19, lab)
    lay = oracle.sparse_build(lab, 7, 19)
    pdf = oracle.sparse_run(p, lay, oracle.sparse_init(lay, A0), 0, 100)
    A = oracle.dense_run(p, lab, 7, 100, A0)
    got = oracle.sparse_gather(lay, pdf, 100)
    ref = A.reshape(19, -1)[:, lay.cells]
    assert np.max(np.abs(got - ref) / ref) < 1e-14


def test_vessel_tree_generator_is_seeded_and_labelled():
    a, per, ia = inputs.vessel_tree(n=40, r0=4.0, k_len=5.0, r_min=1.5, seed=9)
    b, _, ib = inputs.vessel_tree(n=40, r0=4.0, k_len=5.0, r_min=1.5, seed=9)
    assert np.array_equal(a, b) and per == 0
    assert set(np.unique(a)) <= {0, 1, 2, 3}
    assert ia["n_fluid"] == int(np.count_nonzero(a == 0)) > 0
    assert np.all(a[0][a[0] != 1] == 2)            # the z = 0 layer is tissue or inlet
    lay = oracle.sparse_build(a, per, 27, order=2, align=8)
    cls = (lay.links[1::2] >> 8) & 0xff
    assert set(np.unique(cls)) == {0, 1}          # inlet and outlet links both present
