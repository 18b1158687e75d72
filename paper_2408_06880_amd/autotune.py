"""Launch-configuration tuner for the AA step kernels.

For each kernel kind (odd step, even step, dense comparator) of a given
(stencil, storage) pair, time every candidate (workgroup size x XCD-aware tile
order x cap on resident workgroups per CU, and for the even step one or two
cells per thread) on a representative solve and keep the fastest.  Results go to a JSON cache keyed by device,
kernel, stencil, storage and a fluid-cell size bucket; `apply()` loads a cache
and installs the entries through `lbm_set_launch`.  The arithmetic does not
depend on the launch configuration (every candidate performs each cell's
update with the same instructions), so tuning changes speed only.
"""
from __future__ import annotations

import json
import math
import os

BLOCKS = (64, 128, 256)
XCD = (0, 1, 16, 256)   # dispatch order, one eighth per XCD, chunks of 16 / 256 tiles
CELLS = (1, 2)          # cells per thread, even-step kernel only
GROUPS = (0, 2, 3, 4)   # resident workgroups per CU (0: as registers allow)
KERNEL_NAMES = {0: "odd", 1: "even", 2: "dense"}


def size_bucket(n_fluid: int) -> int:
    """log2 bucket of the fluid-cell count (configurations are tuned per bucket)."""
    return int(math.floor(math.log2(max(n_fluid, 1))))


def cache_key(device: str, kernel: int, q: int, storage: int, bucket: int) -> str:
    return f"{device}|{KERNEL_NAMES[kernel]}|q{q}|s{storage}|b{bucket}"


def choose(timings: dict) -> tuple:
    """timings: {(block, xcd[, cells[, groups]]): seconds} -> the fastest
    configuration; ties keep the larger block (fewer workgroups), then the
    larger XCD order value, then fewer cells per thread, then no residency
    cap."""
    best = None
    for cfg, t in timings.items():
        key = (t, -cfg[0], -cfg[1], *cfg[2:3], *(g if g else -1 for g in cfg[3:]))
        if best is None or key < best[0]:
            best = (key, cfg)
    return best[1]


def candidates(kernel, blocks=BLOCKS, xcds=XCD, cells=CELLS, groups=GROUPS):
    """(block, xcd, cells per thread, groups per CU) candidates of one kernel
    kind."""
    cs = cells if kernel == 1 else (1,)
    return [(b, x, c, g) for b in blocks for x in xcds for c in cs for g in groups]


def tune(measure, kernels=(0, 1), blocks=BLOCKS, xcds=XCD, cells=CELLS, groups=GROUPS):
    """measure(kernel, block, xcd, cells, groups) -> seconds per launch.
    Returns {kernel: ((block, xcd, cells, groups), {cfg: seconds})}."""
    out = {}
    for k in kernels:
        timings = {cfg: float(measure(k, *cfg))
                   for cfg in candidates(k, blocks, xcds, cells, groups)}
        out[k] = (choose(timings), timings)
    return out


def gpu_measure(solver, coll, steps=8):
    """measure() for a real solve: per-kernel HIP-event times of `steps`
    launches of each parity on the solver's current stream."""
    import torch

    from . import lbm

    def measure(kernel, block, xcd, cells=1, groups=0):
        q, st = solver.domain.q, solver.storage
        lbm.lbm_set_launch(kernel, q, st, block, xcd, 0, cells, groups)
        solver.step(2, coll)
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps + 1)]
        p0 = solver.t & 1
        evs[0].record()
        for i in range(2 * steps):
            solver.step(1, coll)
            evs[i + 1].record()
        torch.cuda.synchronize()
        d = [evs[i].elapsed_time(evs[i + 1]) / 1e3 for i in range(2 * steps)]
        want = 0 if kernel == lbm.KERNEL_ODD else 1
        sel = [x for i, x in enumerate(d) if ((p0 + i) & 1) == want]
        return sum(sel) / len(sel)

    return measure


def device_name() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name)


def tune_solver(solver, coll, cache_path=None, steps=8):
    """Tune odd and even kernels on `solver`, install the winners, and store
    them in `cache_path` (JSON) if given.  Returns the result dict."""
    from . import lbm
    res = tune(gpu_measure(solver, coll, steps))
    dev = device_name()
    q, st, nf = solver.domain.q, solver.storage, solver.domain.n_fluid
    entries = {}
    for k, ((b, x, c, g), timings) in res.items():
        lbm.lbm_set_launch(k, q, st, b, x, 0, c, g)
        entries[cache_key(dev, k, q, st, size_bucket(nf))] = {
            "block": b, "xcd_remap": x, "cells_per_thread": c, "max_groups_per_cu": g,
            "timings_us": {"/".join(map(str, cfg)): round(t * 1e6, 2)
                           for cfg, t in timings.items()}}
    if cache_path:
        save(cache_path, entries)
    return res


def load(path) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(path, entries: dict):
    data = load(path)
    data.update(entries)
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(cache: dict, device: str, kernel: int, q: int, storage: int, n_fluid: int):
    """Entry for the nearest tuned size bucket of this (device, kernel, q,
    storage), or None."""
    want = size_bucket(n_fluid)
    best = None
    prefix = f"{device}|{KERNEL_NAMES[kernel]}|q{q}|s{storage}|b"
    for key, val in cache.items():
        if key.startswith(prefix):
            b = int(key[len(prefix):])
            d = abs(b - want)
            if best is None or d < best[0]:
                best = (d, val)
    return None if best is None else best[1]


def apply(cache_path, q, storage, n_fluid, device=None):
    """Install cached configurations for (q, storage) at this size; returns
    the number of kernels configured."""
    from . import lbm
    cache = load(cache_path)
    device = device or device_name()
    n = 0
    for k in (lbm.KERNEL_ODD, lbm.KERNEL_EVEN, lbm.KERNEL_DENSE):
        e = lookup(cache, device, k, q, storage, n_fluid)
        if e is not None:
            lbm.lbm_set_launch(k, q, storage, e["block"], e["xcd_remap"], 0,
                               e.get("cells_per_thread", 1), e.get("max_groups_per_cu", 0))
            n += 1
    return n
