"""Seeded synthetic geometries (label masks) for the sparse LBM path.

This module generates *inputs only*: uint8 label arrays of shape (nz, ny, nx),
x fastest (linear id = x + nx*(y + ny*z)), with

    0 = fluid, 1 = solid (no-slip), 2 + c = boundary class c (inlet/outlet),

and a 3-bit periodicity mask (bit 0 = x, bit 1 = y, bit 2 = z).  It holds none
of the method's arithmetic and is shared by the HIP path, the oracle tests and
the benchmark.  All randomness comes from ``numpy.random.default_rng(seed)``.

The paper's own workloads (artificial porosity domains, a particle bed, a
patient coronary artery) are not available; these generators stand in for
them: sphere packings for the porous media runs, a body-forced channel for the
Poiseuille check, a periodic box for shear waves, and a bifurcating vessel
tree with a velocity inlet and pressure outlets for the artery-like run.

Sphere voxelisation: voxel centres sit at integer coordinates; a voxel is
solid iff its periodic minimum-image squared distance to a sphere centre is
<= r^2.  Spheres are added until the voxel porosity drops to the target (the
last sphere may overshoot; the achieved porosity is returned).
"""
from __future__ import annotations

import collections
import math

import numpy as np

FLUID, SOLID = 0, 1
PERIODIC_X, PERIODIC_Y, PERIODIC_Z = 1, 2, 4
PERIODIC_ALL = 7


def _stamp_indices(L, c, r):
    """Box index arrays (wrapped) and squared distances of the voxels near a sphere."""
    axes = []
    d2 = None
    for a in range(3):  # a = x, y, z
        lo = int(math.floor(c[a] - r))
        hi = int(math.ceil(c[a] + r))
        coords = np.arange(lo, hi + 1)
        diff = (coords - c[a]) ** 2
        axes.append(np.mod(coords, L[a]))
        shape = [1, 1, 1]
        shape[2 - a] = len(coords)  # array order is (z, y, x)
        term = diff.reshape(shape)
        d2 = term if d2 is None else d2 + term
    return axes, d2


def _stamp(mask, c, r):
    """Mark the voxels of sphere (c, r) solid; return how many became solid."""
    nz, ny, nx = mask.shape
    (ix, iy, iz), d2 = _stamp_indices((nx, ny, nz), c, r)
    inside = d2 <= r * r
    sub = mask[np.ix_(iz, iy, ix)]
    newly = int(np.count_nonzero(inside & (sub == FLUID)))
    sub[inside] = SOLID
    mask[np.ix_(iz, iy, ix)] = sub
    return newly


def boolean_spheres(L, r_min, r_max, target_phi, seed):
    """Overlapping (Boolean-model) spheres in a periodic box of edge L.

    Centres uniform in [0, L)^3, radii uniform in [r_min, r_max]; spheres are
    added until porosity <= target_phi.  Returns (labels, info)."""
    rng = np.random.default_rng(seed)
    mask = np.zeros((L, L, L), np.uint8)
    total = L ** 3
    solid = 0
    n = 0
    while (total - solid) / total > target_phi:
        c = rng.uniform(0.0, L, size=3)
        r = rng.uniform(r_min, r_max)
        solid += _stamp(mask, c, r)
        n += 1
    info = {"kind": "boolean_spheres", "L": L, "r": [r_min, r_max], "target_phi": target_phi,
            "seed": seed, "n_spheres": n, "phi": (total - solid) / total,
            "n_fluid": total - solid}
    return mask, info


def rsa_spheres(L, r_min, r_max, target_phi, seed, max_rejects=100_000, batch=512,
                window=1 << 18, min_accept=1e-4):
    """Non-overlapping spheres by random sequential addition (periodic box).

    A candidate (centre uniform in [0, L)^3, radius uniform in [r_min, r_max])
    is accepted iff its periodic centre distance to every accepted sphere is
    >= r1 + r2.  Stops when porosity <= target_phi, after `max_rejects`
    consecutive rejections, or when fewer than `min_accept` of the last
    `window` candidates were accepted (approaching the jamming limit; this
    test does not depend on the box volume).  Candidates are drawn in
    batches but accepted strictly in draw order, so the result depends only
    on the seed."""
    assert 2 * r_max + 2 < L
    rng = np.random.default_rng(seed)
    mask = np.zeros((L, L, L), np.uint8)
    total = L ** 3
    solid = 0
    nb = max(1, int(L // (2.0 * r_max)))
    bin_w = L / nb
    cap = 8
    table = np.full((nb, nb, nb, cap), -1, np.int64)
    fill = np.zeros((nb, nb, nb), np.int64)
    centres = np.zeros((1024, 3))
    radii = np.zeros(1024)
    n = 0
    rejects = 0
    drawn = 0                       # candidates drawn so far
    acc_hist = collections.deque()  # (drawn, accepted) at batch ends
    jammed_rate = False
    if nb >= 3:
        offs = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
    else:
        offs = np.array([(a, b, c) for a in range(nb) for b in range(nb) for c in range(nb)])

    def min_image_d2(p, q):
        d = np.abs(p - q)
        d = np.minimum(d, L - d)
        return np.sum(d * d, axis=-1)

    while (total - solid) / total > target_phi and rejects < max_rejects and not jammed_rate:
        acc_hist.append((drawn, n))
        while acc_hist and acc_hist[0][0] < drawn - window:
            acc_hist.popleft()
        if drawn >= window and acc_hist and (n - acc_hist[0][1]) < min_accept * (drawn - acc_hist[0][0]):
            jammed_rate = True
            break
        drawn += batch
        cs = rng.uniform(0.0, L, size=(batch, 3))
        rs = rng.uniform(r_min, r_max, size=batch)
        b = np.floor(cs / bin_w).astype(np.int64) % nb
        nbins = (b[:, None, :] + offs[None, :, :]) % nb if nb >= 3 else np.broadcast_to(
            offs[None], (batch,) + offs.shape)
        ids = table[nbins[..., 0], nbins[..., 1], nbins[..., 2]].reshape(batch, -1)
        valid = ids >= 0
        idc = np.where(valid, ids, 0)
        d2 = min_image_d2(cs[:, None, :], centres[idc])
        clash = np.any(valid & (d2 < (rs[:, None] + radii[idc]) ** 2), axis=1)
        fresh = []  # accepted in this batch
        for j in range(batch):
            if (total - solid) / total <= target_phi or rejects >= max_rejects:
                break
            c, r = cs[j], rs[j]
            bad = bool(clash[j])
            if not bad:
                for m in fresh:
                    if min_image_d2(c, centres[m]) < (r + radii[m]) ** 2:
                        bad = True
                        break
            if bad:
                rejects += 1
                continue
            rejects = 0
            if n == len(radii):
                centres = np.concatenate([centres, np.zeros_like(centres)])
                radii = np.concatenate([radii, np.zeros_like(radii)])
            centres[n] = c
            radii[n] = r
            key = tuple(int(v) for v in (np.floor(c / bin_w).astype(np.int64) % nb))
            if fill[key] == cap:
                table = np.concatenate([table, np.full(table.shape[:3] + (cap,), -1, np.int64)],
                                       axis=3)
                cap *= 2
            table[key + (int(fill[key]),)] = n
            fill[key] += 1
            fresh.append(n)
            n += 1
            solid += _stamp(mask, c, r)
    info = {"kind": "rsa_spheres", "L": L, "r": [r_min, r_max], "target_phi": target_phi,
            "seed": seed, "n_spheres": n, "phi": (total - solid) / total,
            "n_fluid": total - solid, "jammed": rejects >= max_rejects or jammed_rate}
    return mask, info


def channel(nx, ny, nz):
    """Plane channel: all cells fluid; walls are the two non-periodic y faces
    (halfway between the first/last fluid layer and the outside).
    Returns (labels, periodic)."""
    return np.zeros((nz, ny, nx), np.uint8), PERIODIC_X | PERIODIC_Z


def periodic_box(nx, ny, nz):
    """Fully periodic all-fluid box (shear waves, uniform flow)."""
    return np.zeros((nz, ny, nx), np.uint8), PERIODIC_ALL


def random_mask(shape, solid_fraction, seed, n_classes=0, class_fraction=0.0):
    """Uncorrelated random labels for brute-force builder tests."""
    rng = np.random.default_rng(seed)
    u = rng.random(shape)
    lab = np.where(u < solid_fraction, SOLID, FLUID).astype(np.uint8)
    if n_classes:
        v = rng.random(shape)
        cls = rng.integers(0, n_classes, size=shape)
        lab = np.where((lab == SOLID) & (v < class_fraction), 2 + cls, lab).astype(np.uint8)
    return lab


def _capsule_stamp(mask, value, p0, p1, r, only_where=None, flat_end=False, flat_start=False):
    """Set voxels within distance r of segment p0-p1 (non-periodic box).
    flat_end / flat_start: cut the tube by the plane through p1 / p0
    normal to the axis instead of rounding it (a cylinder end)."""
    nz, ny, nx = mask.shape
    lo = np.floor(np.minimum(p0, p1) - r).astype(int)
    hi = np.ceil(np.maximum(p0, p1) + r).astype(int)
    lo = np.maximum(lo, 0)
    hi = np.minimum(hi, np.array([nx - 1, ny - 1, nz - 1]))
    if np.any(hi < lo):
        return
    xs = np.arange(lo[0], hi[0] + 1)
    ys = np.arange(lo[1], hi[1] + 1)
    zs = np.arange(lo[2], hi[2] + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1).astype(np.float64)
    d = p1 - p0
    dd = float(d @ d)
    tr = ((P - p0) @ d) / dd if dd > 0 else np.zeros(P.shape[:-1])
    t = np.clip(tr, 0.0, 1.0)
    Q = p0 + t[..., None] * d
    inside = np.sum((P - Q) ** 2, axis=-1) <= r * r
    if flat_end:
        inside &= tr <= 1.0
    if flat_start:
        inside &= tr > 0.0
    sub = mask[zs[0]:zs[-1] + 1, ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1]
    if only_where is not None:
        inside &= sub == only_where
    sub[inside] = value


def vessel_tree(n=512, r0=24.0, ratio=0.79, k_len=6.0, seed=7, angle_deg=(20.0, 60.0),
                r_min=2.0, inlet_u=0.02, n_azimuth=24, max_depth=16):
    """Synthetic bifurcating vessel tree in a closed box (no periodicity).

    Root tube from the inlet disk at z = 0, centred in x-y, along +z, radius
    r0.  Each segment has length k_len * r; its end spawns two daughters of
    radius ratio*r with polar angles drawn uniformly from `angle_deg`
    (measured from the parent axis) and azimuths psi and psi + pi.  psi is
    the first of `n_azimuth` seeded candidates for which both daughter
    segments stay inside the box margin (r + 2 cells); if only one daughter
    fits any candidate it grows alone.  A branch ends (outlet) when the
    daughter radius would drop below r_min or no daughter fits.  Tubes are
    capsules (their union is the lumen), except that a terminal segment ends
    flat (cut by the plane normal to its axis through its end point).
    Labels: fluid 0, tissue 1, inlet class 0 (label 2) = the z = 0 disk,
    outlet class 1 (label 3) = the tissue cells of the slab just past each
    flat end (axial distance in (0, 2], radial distance <= r), so that every
    fluid cell of the end face has its axial neighbours in the outlet.
    Returns (labels, periodic=0, info)."""
    rng = np.random.default_rng(seed)
    mask = np.ones((n, n, n), np.uint8)  # tissue everywhere
    segs = []
    ends = []

    def inside(p, r):
        return bool(np.all(p >= r + 2) and np.all(p <= n - r - 2))

    stack = [(np.array([n / 2.0, n / 2.0, 0.0]), np.array([0.0, 0.0, 1.0]), r0, 0)]
    while stack:
        p0, axis, r, depth = stack.pop()
        p1 = p0 + axis * k_len * r
        segs.append([p0, p1, r, False])
        rd = ratio * r
        if rd < r_min or depth >= max_depth:
            segs[-1][3] = True
            ends.append((p1, axis, r))
            continue
        tmp = np.array([1.0, 0.0, 0.0]) if abs(axis[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(axis, tmp)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(axis, e1)
        th = np.deg2rad(rng.uniform(*angle_deg, size=2))
        psi0 = rng.uniform(0.0, 2.0 * np.pi)
        best = None
        for c in range(n_azimuth):
            psi = psi0 + 2.0 * np.pi * c / n_azimuth
            dirs = []
            for t, ps in ((th[0], psi), (th[1], psi + np.pi)):
                d = np.cos(t) * axis + np.sin(t) * (np.cos(ps) * e1 + np.sin(ps) * e2)
                dirs.append(d / np.linalg.norm(d))
            fits = [inside(p1 + d * k_len * rd, rd) for d in dirs]
            if all(fits):
                best = dirs
                break
            if best is None and any(fits):
                best = [d for d, f in zip(dirs, fits) if f]
        if not best:
            segs[-1][3] = True
            ends.append((p1, axis, r))
            continue
        for d in best:
            stack.append((p1.copy(), d, rd, depth + 1))
    for p0, p1, r, terminal in segs:
        _capsule_stamp(mask, 0, p0, p1, r, flat_end=terminal)
    # outlets: the slab just past each flat end, on tissue only
    for p1, axis, r in ends:
        _capsule_stamp(mask, 3, p1, p1 + axis * 2.0, r, only_where=1, flat_end=True,
                       flat_start=True)
    # inlet: the z = 0 layer inside the root disk becomes the inlet class
    yy, xx = np.mgrid[0:n, 0:n]
    disk = (xx - n / 2.0) ** 2 + (yy - n / 2.0) ** 2 <= r0 * r0
    layer = mask[0]
    layer[disk] = 2
    mask[0] = layer
    nf = int(np.count_nonzero(mask == 0))
    info = {"kind": "vessel_tree", "n": n, "r0": r0, "ratio": ratio, "k_len": k_len,
            "seed": seed, "n_segments": len(segs), "n_outlets": len(ends),
            "phi": nf / float(n ** 3), "n_fluid": nf, "inlet_u": inlet_u}
    return mask, 0, info


def hybrid_bed(L=256, phi_bed=0.4, r_min=4.0, r_max=12.0, seed=15, batch=16):
    """Particle bed under free flow (the scenario that motivates a block-wise
    choice between sparse and dense storage): a periodic box of edge L whose
    lower half (z < L/2) holds overlapping spheres (centres uniform in that
    half, radii uniform in [r_min, r_max]) added in batches until the lower
    half's porosity is <= phi_bed, and whose upper half is fluid (spheres
    reaching into it are cut off there).  Returns (labels, periodic, info)."""
    rng = np.random.default_rng(seed)
    mask = np.zeros((L, L, L), np.uint8)
    half = L // 2
    lower = half * L * L
    n = 0
    while True:
        solid = int(np.count_nonzero(mask[:half]))
        if (lower - solid) / lower <= phi_bed:
            break
        for _ in range(batch):
            c = np.array([rng.uniform(0.0, L), rng.uniform(0.0, L), rng.uniform(0.0, half)])
            _stamp(mask, c, rng.uniform(r_min, r_max))
            n += 1
    mask[half:] = 0
    nf = int(np.count_nonzero(mask == 0))
    info = {"kind": "hybrid_bed", "L": L, "phi_bed_target": phi_bed,
            "phi_bed": 1.0 - np.count_nonzero(mask[:half]) / lower, "phi": nf / L ** 3,
            "n_fluid": nf, "n_fluid_free": L * L * (L - half), "seed": seed, "n_spheres": n,
            "r": [r_min, r_max]}
    return mask, PERIODIC_ALL, info


def workload_c0():
    """32^3 periodic box, non-overlapping spheres r in [3, 5], porosity ~0.6, seed 1."""
    lab, info = rsa_spheres(32, 3.0, 5.0, 0.6, seed=1)
    return lab, PERIODIC_ALL, info


def workload_vessel(n=512):
    """512^3 vessel tree (root radius 24, ratio 0.79, branch angles 20-60 deg),
    velocity inlet 0.02 along +z at z = 0, pressure outlets (rho = 1)."""
    return vessel_tree(n=n)


def workload_c1(phi=0.6, L=256, seed=None):
    """256^3 periodic box, overlapping spheres r in [4, 12] at porosity phi."""
    seeds = {0.4: 11, 0.6: 12, 0.8: 13, 0.95: 14}
    if seed is None:
        seed = seeds.get(phi, 12)
    lab, info = boolean_spheres(L, 4.0, 12.0, phi, seed=seed)
    return lab, PERIODIC_ALL, info
