"""Benchmark of the sparse AA lattice Boltzmann step on one MI355X.

Workload (default): D3Q19 TRT (Lambda = 3/16, tau = 0.8), AA in-place
streaming, body force F = 1e-6 x, on a 256^3 periodic box filled with seeded
overlapping spheres (radius uniform 4-12) at porosity 0.6 (synthetic
stand-in for the paper's artificial porosity domains).  The headline line is
FP64 storage (the paper's single-GPU benchmark counts 8-byte PDFs); FP32 and
FP16-deviation storage of the same solve are reported beside it as
sub-records with their own rooflines.

One step = one AA half-step (odd or even kernel) over every fluid cell.
`value` = fluid-cell updates per second (MFLUPS) over K timed steps with all
data resident in HBM.  Per-kernel durations come from HIP events recorded on
the launch stream between the launches of the timed region, and from the
committed rocprofv3 summaries in profiles/ while they match the kernel
sources and launch configuration.

Prints one JSON line.  `python bench.py --gpus N` with N > 1 exits: the
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MFLUPS + % HBM BW, sparse D3Q19 TRT 256^3 packing; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
# serving: 16-bit solves finish in FP32 deviations once their residual is
# below this (16-bit storage can stall near the steady state)
REFINE_TOL = 1e-5


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def copy_bandwidth(lbm, torch, nbytes=2 << 30, reps=10):
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        lbm.lbm_copy(dst, src, nbytes)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lbm.lbm_copy(dst, src, nbytes)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2 * nbytes / s / 1e9


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(lab, per, q, tau, magic, force, n_fluid, budget_s):
    """The FP64 oracle (dense two-array pull, OpenMP over z-planes) on the
    same geometry: one untimed step (first touch of the second array), then
    whole-grid steps until `budget_s` seconds have passed on all threads,
    then the same on one thread for a third of the budget."""
    import ctypes

    import numpy as np

    import oracle
    p = oracle.params(q=q, kind=oracle.TRT, tau=tau, magic=magic, force=force)
    lib = oracle._load()
    lab = np.ascontiguousarray(lab, np.uint8)
    nz, ny, nx = lab.shape
    A = oracle.dense_init(q, lab)
    B = np.empty_like(A)

    def step(a, b):
        rc = lib.orc_dense_step(ctypes.byref(p), oracle._ptr(lab), nx, ny, nz, per,
                                oracle._ptr(a), oracle._ptr(b))
        if rc:
            raise RuntimeError("oracle step failed")

    step(A, B)
    A, B = B, A

    def timed(budget):
        nonlocal A, B
        steps = 0
        t0 = time.perf_counter()
        while True:
            step(A, B)
            A, B = B, A
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return steps, el

    threads = oracle.num_threads()
    steps, el = timed(budget_s)
    oracle.set_num_threads(1)
    try:
        steps1, el1 = timed(budget_s / 3)
    finally:
        oracle.set_num_threads(threads)
    return {"value": round(n_fluid * steps / el / 1e6, 3), "unit": "MFLUPS",
            "cores": threads, "kind": "oracle",
            "sample": f"{steps} dense FP64 pull TRT step(s) of the full {nx}x{ny}x{nz} geometry "
                      f"({n_fluid} fluid cells) after one untimed step, {el:.1f} s",
            "single_thread_value": round(n_fluid * steps1 / el1 / 1e6, 3),
            "single_thread_sample": f"{steps1} step(s), {el1:.1f} s",
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}


def recorded_profile(workload_key, launch_odd):
    """Figures of the committed rocprofv3 summary in profiles/ taken on this
    workload with the current kernel sources and the odd kernel's current
    launch configuration, else None: HBM bytes per launch of the odd
    (dominant) and even kernels from the counters, and their average
    durations from the kernel trace."""
    import glob

    from paper_2408_06880_amd import kernel_source_hash
    h = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        kv = {}
        for line in open(path):
            if line.startswith("traffic_") and ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if (kv.get("traffic_workload") == workload_key and kv.get("traffic_source_hash") == h
                and kv.get("traffic_launch") == "/".join(map(str, launch_odd))):
            def num(key):
                return float(kv[key]) if kv.get(key) else None
            return {"odd_bytes": num("traffic_bytes_per_launch"),
                    "even_bytes": num("traffic_even_bytes_per_launch"),
                    "odd_avg_us": num("traffic_odd_avg_us"),
                    "even_avg_us": num("traffic_even_avg_us"),
                    "source": os.path.relpath(path, ROOT)}
    return None


def _device_used(torch):
    """Device bytes in use (hipMemGetInfo), after returning cached blocks."""
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    return total - free


def memory_study(L=256, phis=(0.2, 0.4, 0.6, 0.8, 0.95), storages=("f64", "f32", "f16dev")):
    """Device memory of one D3Q19 solve against porosity: sparse AA with the
    int32 index-list, sparse AA with only the run form, and the dense AA
    comparator, each with density and velocity output fields.  Measured as
    the drop of free device memory, next to the paper's memory model
    (in-place AA on both sides, five other fields) and to the exact sum of
    the buffers this library allocates."""
    import torch

    from paper_2408_06880_amd import costmodel, inputs, lbm
    q = 19
    rows = []
    for phi in phis:
        lab, per, info = inputs.workload_c1(phi, L=L)
        lab_dev = torch.from_numpy(lab).cuda()
        N = lab.size
        for name in storages:
            storage = {"f64": lbm.STORE_F64, "f32": lbm.STORE_F32,
                       "f16dev": lbm.STORE_F16DEV}[name]
            b = lbm.STORE_BYTES[storage]
            fdt = torch.float64 if storage == lbm.STORE_F64 else torch.float32
            bf = 8 if storage == lbm.STORE_F64 else 4
            row = {"phi": round(info["phi"], 4), "storage": name}
            for form in ("int32", "runs", "dense"):
                base = _device_used(torch)
                torch.cuda.reset_peak_memory_stats()
                a0 = torch.cuda.memory_allocated()
                if form == "dense":
                    obj = lbm.DenseSolver(lab_dev, per, q, storage)
                    n = N
                    exact = obj.pdf.numel() * b + obj.mask.numel() * 4
                else:
                    dom = lbm.SparseDomain(lab_dev, per, q, lbm.ORDER_BLOCKED, 64)
                    if form == "runs":
                        dom.compact_runs(drop_index=True)
                        # hand the int32 list's segment back to the device;
                        # otherwise torch's cache carves the later buffers
                        # out of it and holds the rest
                        torch.cuda.synchronize()
                        torch.cuda.empty_cache()
                    obj = lbm.Solver(dom, storage, 14 if storage == lbm.STORE_F16DEV else 0)
                    n = dom.stride
                    nf = dom.n_fluid
                    exact = dom.device_bytes() + obj.device_bytes()
                fields = (torch.empty(n, dtype=fdt, device="cuda"),
                          torch.empty(3 * n, dtype=fdt, device="cuda"))
                exact += 4 * n * bf
                peak = torch.cuda.max_memory_allocated() - a0
                used = _device_used(torch) - base
                row[form] = {"measured_bytes": used, "exact_bytes": exact,
                             "build_peak_bytes": peak,
                             "measured_per_fluid_cell": round(used / nf, 2)}
                if form == "runs":
                    row[form]["index_bytes_per_fluid_cell"] = round(dom.runs_bytes / nf, 3)
                del obj, fields
                if form != "dense":
                    del dom
            row["n_fluid"] = nf
            row["model_sparse_aa"] = costmodel.memory(N, nf / N, q, b, 4, "aa", True)
            row["model_dense_aa"] = costmodel.memory(N, nf / N, q, b, 4, "aa", False)
            d = row["dense"]["measured_bytes"]
            for form in ("int32", "runs"):
                m = row[form]["measured_bytes"]
                row[form]["vs_dense"] = round(m / d, 4)
                # porosity at which this structure would match the dense one
                row[form]["break_even_phi"] = round(d / (N * m / nf), 4)
            row["int32_vs_model"] = round(row["int32"]["measured_bytes"] / row["model_sparse_aa"], 4)
            row["dense_vs_model"] = round(d / row["model_dense_aa"], 4)
            log(f"memory phi={row['phi']} {name}: int32 {row['int32']['measured_bytes'] / 2**20:.0f} "
                f"MiB, runs {row['runs']['measured_bytes'] / 2**20:.0f} MiB, dense "
                f"{d / 2**20:.0f} MiB")
            rows.append(row)
        del lab_dev
    return rows


SERVING_L = (64, 384)
SERVING_TARGET_CELLS = 32_000_000


def _converged_percentiles(res):
    """p50/p99 time to steady state over the requests that reached the
    residual tolerance, and the same over every completed request."""
    from paper_2408_06880_amd import server
    conv = [r.latency for r in res if r.converged and not r.error]
    done = [r.latency for r in res if not r.error]
    return {"p50_converged_latency_s": server.percentile(conv, 50),
            "p99_converged_latency_s": server.percentile(conv, 99),
            "p50_all_latency_s": server.percentile(done, 50),
            "p99_all_latency_s": server.percentile(done, 99)}


def serving_leg(n_requests, max_steps, target_cells=SERVING_TARGET_CELLS):
    """Continuous batching (FP16 deviation storage, refined to FP32
    deviations near the steady state) against one-at-a-time FP32 solves of
    the same Poisson trace at the serving configuration's sizes (edge
    U{64..384}); time to steady state per request, converged requests and
    capped ones reported apart."""
    from paper_2408_06880_amd import lbm, server
    budget = 288 * (1 << 30) - 8 * (1 << 30)
    kw = dict(L_range=SERVING_L, phi_range=(0.3, 0.9), tau_range=(0.6, 1.0))

    def retired(tag):
        def f(r):
            log(f"serving {tag}: request {r.rid} retired, {r.n_fluid} cells, {r.steps} steps, "
                f"converged {r.converged}, latency {r.latency:.2f} s")
        return f

    trace = server.make_trace(n_requests, 20.0, seed=31, **kw)
    res, met = server.Server(server.GpuStepper(storage=lbm.STORE_F16DEV), budget, K=100,
                             tol=1e-6, max_steps=max_steps, target_cells=target_cells,
                             refine_tol=REFINE_TOL, on_finish=retired("f16dev batched")).run(trace)
    log(f"serving (batched f16dev): p50 {met['p50_latency_s']:.3f} s p99 "
        f"{met['p99_latency_s']:.3f} s, {met['aggregate_mflups']:.0f} MFLUPS")
    # the same continuous batching in FP32 storage: separates what batching
    # gains from what 16-bit storage gains
    resb32, metb32 = server.Server(server.GpuStepper(storage=lbm.STORE_F32), budget, K=100,
                                   tol=1e-6, max_steps=max_steps, target_cells=target_cells,
                                   on_finish=retired("f32 batched")).run(
        server.make_trace(n_requests, 20.0, seed=31, **kw))
    log(f"serving (batched f32): p50 {metb32['p50_latency_s']:.3f} s p99 "
        f"{metb32['p99_latency_s']:.3f} s, {metb32['aggregate_mflups']:.0f} MFLUPS")
    res32, met32 = server.run_sequential(server.GpuStepper(storage=lbm.STORE_F32),
                                         server.make_trace(n_requests, 20.0, seed=31, **kw),
                                         K=100, tol=1e-6, max_steps=max_steps)
    log(f"serving (sequential f32): p50 {met32['p50_latency_s']:.3f} s p99 "
        f"{met32['p99_latency_s']:.3f} s, {met32['aggregate_mflups']:.0f} MFLUPS")
    res = sorted(res, key=lambda r: r.rid)
    resb32 = sorted(resb32, key=lambda r: r.rid)
    res32 = sorted(res32, key=lambda r: r.rid)
    per = []
    for t, a, b in zip(trace, res, res32):
        d = abs(a.permeability - b.permeability) / abs(b.permeability) if b.permeability else None
        per.append({"rid": t.rid, "arrival_s": round(t.arrival, 3), "L": t.L,
                    "phi": round(t.phi, 3), "tau": round(t.tau, 3), "n_fluid": a.n_fluid,
                    "f16_steps": a.steps, "f16_converged": a.converged,
                    "f16_refined_at": a.refined_at, "f16_latency_s": round(a.latency, 3),
                    "f32_steps": b.steps, "f32_converged": b.converged,
                    "f32_latency_s": round(b.latency, 3),
                    "permeability_rel_diff": d})
    both = [p["permeability_rel_diff"] for p in per
            if p["f16_converged"] and p["f32_converged"] and p["permeability_rel_diff"] is not None]
    keys = ("p50_latency_s", "p99_latency_s", "p50_queue_s", "p99_queue_s", "p50_service_s",
            "p99_service_s", "aggregate_mflups", "busy_mflups", "makespan_s", "completed",
            "converged")
    out = {}
    for tag, r, m in (("batched_f16dev", res, met), ("batched_f32", resb32, metb32),
                      ("sequential_f32", res32, met32)):
        rec = {k: m[k] for k in keys}
        rec.update(_converged_percentiles(r))
        rec["capped"] = sum(1 for x in r if not x.converged and not x.error)
        # offered load: the trace's work at this run's busy throughput over
        # the span of its arrivals
        work = sum(x.n_fluid * x.steps for x in r)
        rec["offered_load_factor"] = (work / (m["busy_mflups"] * 1e6) / trace[-1].arrival
                                      if m["busy_mflups"] else None)
        out[tag] = rec
    # share of the batched 16-bit run's fluid-cell updates done in FP16
    # storage (the rest ran in FP32 deviations after refinement)
    f16_updates = sum(x.n_fluid * (x.refined_at if x.refined_at else x.steps) for x in res)
    all_updates = sum(x.n_fluid * x.steps for x in res)
    out["batched_f16dev"]["f16_update_fraction"] = (f16_updates / all_updates
                                                    if all_updates else None)
    return {"trace": f"{n_requests} requests, Poisson 20/s, seed 31, L U{{{SERVING_L[0]}.."
                     f"{SERVING_L[1]}}} (steps of 8), phi U[0.3,0.9], tau U[0.6,1.0], D3Q19 TRT, "
                     f"residual < 1e-6 (K = 100) or the cap of {max_steps} steps; batched FP16 "
                     f"deviations move to FP32 deviations below residual {REFINE_TOL}; admission "
                     f"while active fluid cells < {target_cells}",
            **out,
            "permeability_rel_diff_f16_vs_f32_max_both_converged": max(both) if both else None,
            "requests": per}


def _steady_run(lbm, torch, dom, storage, dev_exp, coll, K, tol, cap, L):
    """Advance a fresh solve in rounds of K steps until the mean-momentum
    residual drops below tol (or cap); returns its figures."""
    sol = lbm.Solver(dom, storage, dev_exp)
    sol.init()
    jx, res, t_gpu = [], float("nan"), 0.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    while sol.t < cap:
        e0.record()
        sol.step(K, coll)
        e1.record()
        r = sol.reduce(coll)
        t_gpu += e0.elapsed_time(e1) / 1e3
        jx.append(r.mom[0])
        if len(jx) >= 2 and jx[-1] != 0:
            res = abs(jx[-1] - jx[-2]) / abs(jx[-1])
            if sol.t >= 2 * K and res < tol:
                break
    rho, u = sol.moments(coll, f64=True)
    nf = dom.n_fluid
    umax = float(torch.sqrt((u[:, :nf] ** 2).sum(0)).max())
    nu = (coll.tau - 0.5) / 3.0
    k = nu * (jx[-1] / float(L ** 3)) / coll.force[0]
    return {"steps": sol.t, "residual": res, "converged": res < tol, "permeability": k,
            "max_speed": umax, "mflups": nf * sol.t / t_gpu / 1e6}


def mixed_precision_study(L=384, oracle_L=64, K=100, tol=1e-6, cap=20000):
    """Config 3: the benchmark's packing geometry (overlapping spheres, r 4-12,
    porosity 0.6) at 384^3 run to steady state with every storage format; permeability and maximum speed
    against FP64 storage on the GPU at full size and against the FP64 oracle
    at a reduced size the oracle can converge."""
    import torch

    import oracle
    from paper_2408_06880_amd import inputs, lbm
    fmts = [("f64", lbm.STORE_F64, 0), ("f32", lbm.STORE_F32, 0), ("f32dev", lbm.STORE_F32DEV, 0),
            ("f16dev", lbm.STORE_F16DEV, 14), ("bf16dev", lbm.STORE_BF16DEV, 0)]
    coll = lbm.collision(lbm.COLL_TRT, tau=0.8, magic=3 / 16, force=(1e-6, 0.0, 0.0))
    out = {}
    for size, tag in ((oracle_L, "oracle_size"), (L, "full_size")):
        t0 = time.perf_counter()
        lab, info = inputs.boolean_spheres(size, 4.0, 12.0, 0.6, seed=21)
        log(f"mixed precision {size}^3: phi {info['phi']:.4f}, n_fluid {info['n_fluid']}, "
            f"{info['n_spheres']} spheres ({time.perf_counter() - t0:.1f} s)")
        dom = lbm.SparseDomain(lab, inputs.PERIODIC_ALL, 19, lbm.ORDER_BLOCKED)
        dom.compact_runs()
        runs = {}
        for name, st, e in fmts:
            runs[name] = _steady_run(lbm, torch, dom, st, e, coll, K, tol, cap, size)
            log(f"  {name}: {runs[name]}")
        ref = {"permeability": runs["f64"]["permeability"], "max_speed": runs["f64"]["max_speed"],
               "source": "FP64 storage on the GPU (itself within 1e-12 of the oracle per step)"}
        if tag == "oracle_size":
            p = oracle.params(q=19, kind=oracle.TRT, tau=0.8, magic=3 / 16, force=(1e-6, 0, 0))
            A = oracle.dense_init(19, lab)
            jx, steps, res = [], 0, float("nan")
            while steps < cap:
                A = oracle.dense_run(p, lab, inputs.PERIODIC_ALL, K, A)
                steps += K
                _, J, _ = oracle.dense_reduce(p, lab, A)
                jx.append(J[0])
                if len(jx) >= 2:
                    res = abs(jx[-1] - jx[-2]) / abs(jx[-1])
                    if steps >= 2 * K and res < tol:
                        break
            rho, u = oracle.dense_moments(p, lab, A)
            fl = lab == 0
            ref = {"permeability": (0.8 - 0.5) / 3.0 * (jx[-1] / size ** 3) / 1e-6,
                   "max_speed": float(np.sqrt((u[:, fl] ** 2).sum(0)).max()),
                   "steps": steps, "residual": res, "source": "FP64 CPU oracle (dense pull)"}
        for name in runs:
            runs[name]["permeability_rel_err"] = abs(runs[name]["permeability"] -
                                                     ref["permeability"]) / abs(ref["permeability"])
            runs[name]["max_speed_rel_err"] = abs(runs[name]["max_speed"] -
                                                  ref["max_speed"]) / ref["max_speed"]
        out[tag] = {"L": size, "phi": info["phi"], "n_fluid": info["n_fluid"], "reference": ref,
                    "runs": runs}
        del dom
        torch.cuda.empty_cache()
    return out


def _timed_steps(torch, step, K):
    """Seconds per step of `step(n)` over K steps (HIP events on the current
    stream around the whole run, after two untimed steps)."""
    step(2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    step(K)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / K


def hybrid_study(L=256, phi_bed=0.4, K=200, storages=("f64", "f32")):
    """The paper's hybrid motivation (free flow over a particle bed): a 256^3
    periodic box, lower half a porosity-0.4 packing, upper half fluid.
    Measured per storage: the sparse run-form solve of the whole box, the
    dense AA comparator of the whole box, and the time a block hybrid could
    reach at best -- the dense kernel on the fluid half plus the sparse
    kernel on the bed half, each timed as a solve of its own (no interface
    exchange counted), which is a lower bound on any hybrid's step time."""
    import torch

    from paper_2408_06880_amd import inputs, lbm
    lab, per, info = inputs.hybrid_bed(L, phi_bed)
    half = L // 2
    bed = np.ascontiguousarray(lab[:half])
    free = np.zeros_like(bed)
    q = 19
    coll = lbm.collision(lbm.COLL_TRT, tau=0.8, magic=3 / 16, force=(1e-6, 0.0, 0.0))
    nf = info["n_fluid"]
    nf_bed = int(np.count_nonzero(bed == 0))
    nf_free = free.size
    out = {"workload": f"{L}^3 periodic box, lower half overlapping spheres r 4-12 at porosity "
                       f"{info['phi_bed']:.3f} (seed {info['seed']}), upper half fluid; D3Q19 TRT "
                       "tau 0.8",
           "n_fluid": nf, "n_fluid_bed_half": nf_bed, "n_fluid_free_half": nf_free,
           "steps": K}

    def sparse_t(mask, storage):
        dom = lbm.SparseDomain(mask, per, q, lbm.ORDER_BLOCKED, 64)
        bpc = dom.compact_runs(drop_index=True)
        sol = lbm.Solver(dom, storage, 14 if storage == lbm.STORE_F16DEV else 0)
        sol.init()
        t = _timed_steps(torch, lambda n: sol.step(n, coll), K)
        del sol, dom
        torch.cuda.empty_cache()
        return t, bpc

    def dense_t(mask, storage):
        ds = lbm.DenseSolver(mask, per, q, storage, 14 if storage == lbm.STORE_F16DEV else 0)
        ds.init()
        t = _timed_steps(torch, lambda n: ds.step(n, coll), K)
        del ds
        torch.cuda.empty_cache()
        return t

    for name in storages:
        st = STORAGES[name]
        t_sp, bpc = sparse_t(lab, st)
        t_de = dense_t(lab, st)
        t_bed, _ = sparse_t(bed, st)
        t_free_dense = dense_t(free, st)
        t_free_sparse, bpc_free = sparse_t(free, st)
        t_hyb = t_bed + t_free_dense
        rec = {"sparse_runs_mflups": nf / t_sp / 1e6, "sparse_index_bytes_per_cell": bpc,
               "dense_mflups_fluid": nf / t_de / 1e6,
               "hybrid_bound_mflups": nf / t_hyb / 1e6,
               "bed_half_sparse_us": t_bed * 1e6, "free_half_dense_us": t_free_dense * 1e6,
               "free_half_sparse_us": t_free_sparse * 1e6,
               "free_half_sparse_index_bytes_per_cell": bpc_free,
               "whole_sparse_us": t_sp * 1e6, "whole_dense_us": t_de * 1e6}
        log(f"hybrid {name}: sparse {rec['sparse_runs_mflups']:.0f}, dense "
            f"{rec['dense_mflups_fluid']:.0f}, hybrid bound {rec['hybrid_bound_mflups']:.0f} MFLUPS; "
            f"free half dense {t_free_dense * 1e6:.1f} us vs sparse {t_free_sparse * 1e6:.1f} us")
        out[name] = rec
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="packing",
                    choices=["packing", "vessel", "mixed", "serving", "memory", "hybrid"],
                    help="packing: D3Q19 TRT 256^3 sphere packing (the metric's workload); "
                         "vessel: D3Q27 cumulant 512^3 vessel tree with inlet/outlets")
    ap.add_argument("--phi", type=float, default=0.6)
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--tau", type=float, default=None,
                    help="relaxation time (default 0.8 for the packing, 0.6 for the vessel tree)")
    ap.add_argument("--storage", default=None, choices=list(STORAGE_NAMES),
                    help="storage of the headline record (default: FP64, the paper's 8-byte "
                         "PDFs; FP32 for the vessel tree)")
    ap.add_argument("--sub", default=None,
                    help="comma-separated storages timed on the same solve as sub-records "
                         "(default f32,f16dev for the packing, none for the vessel tree)")
    ap.add_argument("--order", default="blocked", choices=["morton", "lex", "blocked"])
    ap.add_argument("--index", default="run", choices=["16", "32", "run"],
                    help="index-list form: 16 = compact (2 B/entry), 32 = int32, "
                         "run = run-compressed")
    ap.add_argument("--dense-steps", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--pipelined", type=int, default=0, choices=[0, 1],
                    help="odd kernel as persistent workgroups prefetching the next tile")
    ap.add_argument("--coll", default="trt", choices=["trt", "srt", "mrt", "cumulant", "cm"],
                    help="packing workload: collision operator (D3Q19; cumulant and "
                         "central moments on D3Q27)")
    ap.add_argument("--even-cells", type=int, default=0, choices=[0, 1, 2],
                    help="cells per thread of the even-step kernel (0: the library's "
                         "default, two for 16-bit storage)")
    ap.add_argument("--tune", action="store_true",
                    help="run the launch tuner on this solve first (untimed) and keep the "
                         "fastest configurations")
    ap.add_argument("--odd-block", type=int, default=None, choices=[64, 128, 256],
                    help="workgroup size of the odd-step kernel (default: the library's table)")
    ap.add_argument("--even-block", type=int, default=None, choices=[64, 128, 256],
                    help="the same for the even-step kernel")
    ap.add_argument("--odd-xcd", type=int, default=None,
                    help="tile order of the odd-step kernel over the XCDs: 0 dispatch order, "
                         "1 one eighth per XCD, m >= 2 chunks of m tiles (default: the "
                         "library's table)")
    ap.add_argument("--even-xcd", type=int, default=None,
                    help="the same for the even-step kernel")
    ap.add_argument("--odd-groups", type=int, default=None,
                    help="resident workgroups per CU of the odd-step kernel (0: uncapped; "
                         "default: the library's table)")
    ap.add_argument("--even-groups", type=int, default=None,
                    help="the same for the even-step kernel")
    ap.add_argument("--scheme", default="aa", choices=["aa", "pull"],
                    help="aa: in-place AA steps; pull: two-array pull steps (comparison)")
    ap.add_argument("--requests", type=int, default=48,
                    help="--workload serving: requests in the trace")
    ap.add_argument("--max-steps", type=int, default=8000,
                    help="--workload serving: step cap per request")
    ap.add_argument("--target-cells", type=int, default=32_000_000,
                    help="--workload serving: admit while active fluid cells stay below this")
    ap.add_argument("--serving", type=int, default=16,
                    help="requests in the serving trace (0: skip the serving leg)")
    ap.add_argument("--serving-cap", type=int, default=30000,
                    help="step cap per request in the serving leg")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; multi-GPU runs are not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2408_06880_amd import costmodel, inputs, lbm
    STORAGES.update({"f64": lbm.STORE_F64, "f32": lbm.STORE_F32, "f16dev": lbm.STORE_F16DEV,
                     "bf16dev": lbm.STORE_BF16DEV, "f32dev": lbm.STORE_F32DEV})

    if args.workload == "memory":
        print(json.dumps({"metric": "device memory per solve vs porosity, sparse AA (int32 "
                                    "index-list or run form only) vs dense AA, D3Q19",
                          "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": f"{args.L}^3 overlapping-sphere packings "
                                                 "(r 4-12), density and velocity fields included"},
                          "memory": memory_study(L=args.L)}), flush=True)
        return

    if args.workload == "serving":
        from paper_2408_06880_amd import server
        budget = 288 * (1 << 30) - 8 * (1 << 30)
        trace = server.make_trace(args.requests, 20.0, seed=31)
        def retired(r):
            log(f"request {r.rid} retired: {r.n_fluid} cells, {r.steps} steps, "
                f"converged {r.converged}, latency {r.latency:.1f} s")

        res, met = server.Server(server.GpuStepper(storage=lbm.STORE_F16DEV), budget, K=100,
                                 tol=1e-6, max_steps=args.max_steps,
                                 target_cells=args.target_cells, on_finish=retired,
                                 refine_tol=REFINE_TOL).run(trace)
        work = sum(r.n_fluid * r.steps for r in res)
        capacity_s = work / (met["busy_mflups"] * 1e6) if met["busy_mflups"] else None
        print(json.dumps({
            "metric": "p50/p99 time to steady state and aggregate MFLUPS, continuous batching",
            "value": round(met["aggregate_mflups"], 1), "unit": "MFLUPS", "n_gpus": 1,
            "data": "synthetic",
            "config": {"workload": f"{args.requests} permeability requests, Poisson 20/s (seed 31), "
                                   "edge U{64..384}, porosity U[0.3,0.9], tau U[0.6,1.0], "
                                   "D3Q19 TRT FP16-deviation storage (FP32 deviations below "
                                   f"residual {REFINE_TOL}), residual < 1e-6, "
                                   f"cap {args.max_steps} steps, 280 GB admission budget, "
                                   f"admission while active fluid cells < {args.target_cells}"},
            "serving": met,
            "offered_load_factor": (capacity_s / trace[-1].arrival) if capacity_s else None,
            "requests": [{"rid": r.rid, "L": t.L, "phi": round(t.phi, 3), "n_fluid": r.n_fluid,
                          "steps": r.steps, "converged": r.converged, "refined_at": r.refined_at,
                          "latency_s": round(r.latency, 3), "permeability": r.permeability}
                         for r, t in zip(res, trace)]}), flush=True)
        return

    if args.workload == "hybrid":
        print(json.dumps({"metric": "MFLUPS of sparse (run form), dense and the best block "
                                    "hybrid on a particle bed under free flow",
                          "n_gpus": 1, "data": "synthetic",
                          "hybrid": hybrid_study(K=args.steps if args.steps != 1000 else 200)}),
              flush=True)
        return

    if args.workload == "mixed":
        study = mixed_precision_study()
        print(json.dumps({"metric": "steady-state permeability / max-speed error by storage "
                                    "format (D3Q19 TRT, overlapping-sphere packing r 4-12, porosity 0.6)",
                          "n_gpus": 1, "data": "synthetic", "mixed_precision": study}), flush=True)
        return

    q, magic, force = 19, 3.0 / 16.0, (1e-6, 0.0, 0.0)
    if args.tau is None:
        args.tau = 0.6 if args.workload == "vessel" else 0.8
    if args.coll in ("cumulant", "cm"):
        q = 27
    if args.storage is None:
        args.storage = "f32" if args.workload == "vessel" else "f64"
    if args.sub is None:
        args.sub = "" if args.workload == "vessel" else "f32,f16dev"
    order = {"morton": lbm.ORDER_MORTON, "lex": lbm.ORDER_LEX,
             "blocked": lbm.ORDER_BLOCKED}[args.order]
    torch.cuda.set_device(0)
    vessel = args.workload == "vessel"
    bs = None

    t0 = time.perf_counter()
    if vessel:
        q, force = 27, (0.0, 0.0, 0.0)
        lab, per, info = inputs.workload_vessel()
        args.L = lab.shape[0]
        bs = lbm.bspec([(lbm.BC_UBB, (0.0, 0.0, info["inlet_u"]), 1.0),
                        (lbm.BC_PRESSURE, (0.0, 0.0, 0.0), 1.0)])
    else:
        lab, per, info = inputs.workload_c1(args.phi, L=args.L)
    log(f"geometry {args.L}^3 phi={info['phi']:.4f} n_fluid={info['n_fluid']} "
        f"({time.perf_counter() - t0:.1f} s)")
    lab_dev = torch.from_numpy(lab).cuda()
    torch.cuda.synchronize()
    if vessel:
        coll = lbm.collision(lbm.COLL_CUMULANT, tau=args.tau, omega_bulk=1.0, force=force)
    else:
        kind = {"trt": lbm.COLL_TRT, "srt": lbm.COLL_SRT, "mrt": lbm.COLL_MRT,
                "cumulant": lbm.COLL_CUMULANT, "cm": lbm.COLL_CM}[args.coll]
        coll = lbm.collision(kind, tau=args.tau, magic=magic, force=force, omega_bulk=1.19)
    workload = (f"sparse D3Q{q} {args.coll.upper()} AA, {args.L}^3 periodic overlapping-sphere packing "
                f"phi={info['phi']:.3f} (r 4-12, seed {info['seed']})")
    if vessel:
        workload = (f"sparse D3Q27 cumulant AA (tau {args.tau}), {args.L}^3 vessel tree "
                    f"(root r 24, ratio 0.79, seed {info['seed']}, {info['n_outlets']} outlets, "
                    f"phi={info['phi']:.4f}), UBB inlet u_z={info['inlet_u']}, pressure outlets")

    main_rec, dom_info = packing_record(lbm, torch, costmodel, lab_dev, per, q, order, args,
                                        args.storage, coll, bs, workload)
    nf = dom_info["n_fluid"]
    subs = {}
    for name in [x for x in args.sub.split(",") if x and x != args.storage]:
        subs[name], _ = packing_record(lbm, torch, costmodel, lab_dev, per, q, order, args, name,
                                       coll, bs, workload)

    copy_gbs = None if args.no_copy else copy_bandwidth(lbm, torch)
    if copy_gbs:
        log(f"copy kernel {copy_gbs:.0f} GB/s")
        for rec in [main_rec] + list(subs.values()):
            rec["pct_copy_bw"] = round(100.0 * rec["value"] * 1e6 * rec["bytes_per_flup_alg"] /
                                       (copy_gbs * 1e9), 2)

    storage = STORAGES[args.storage]
    dev_exp = 14 if storage == lbm.STORE_F16DEV else 0
    dense = None
    if args.dense_steps > 0 and not vessel:
        torch.cuda.empty_cache()
        ds = lbm.DenseSolver(lab_dev, per, q, storage, dev_exp)
        ds.init()
        ds.step(10, coll)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ds.step(args.dense_steps, coll)
        e1.record()
        torch.cuda.synchronize()
        sd = e0.elapsed_time(e1) / 1e3
        dense = {"kernel": "dense direct-addressing AA over all cells", "storage": args.storage,
                 "mflups_fluid": nf * args.dense_steps / sd / 1e6,
                 "mlups_all_cells": lab.size * args.dense_steps / sd / 1e6,
                 "steps": args.dense_steps}
        log(f"dense comparator {dense['mflups_fluid']:.0f} MFLUPS (fluid cells)")
        del ds
        torch.cuda.empty_cache()

    serving = None
    if args.serving > 0 and not vessel:
        serving = serving_leg(args.serving, args.serving_cap)

    cpu = None
    if not args.no_cpu and not vessel:
        cpu = cpu_baseline(lab, per, q, args.tau, magic, force, nf, args.cpu_seconds)
        log(f"cpu oracle {cpu['value']:.1f} MFLUPS on {cpu['cores']} threads")

    out = {
        "metric": METRIC if not vessel else
        "MFLUPS + % HBM BW, sparse D3Q27 cumulant 512^3 vessel tree",
        "value": main_rec.pop("value"),
        "unit": "MFLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_rec.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_rec.pop("dtype"),
        "data": "synthetic",
        "config": {"workload": workload, "n_fluid": nf, "tau": args.tau, "magic": magic,
                   "force": list(force), "order": args.order, "scheme": args.scheme,
                   "stride": dom_info["stride"], **main_rec.pop("config")},
    }
    out.update(main_rec)
    out.update({"builder_ms": dom_info["builder_ms"],
                "copy_kernel_gbs": round(copy_gbs, 1) if copy_gbs else None,
                "sub_records": subs,
                "dense_comparator": dense,
                "serving": serving,
                "cpu_baseline": cpu})
    print(json.dumps(out), flush=True)


STORAGE_NAMES = ("f64", "f32", "f16dev", "bf16dev", "f32dev")
STORAGES = {}


def packing_record(lbm, torch, costmodel, lab_dev, per, q, order, args, name, coll, bs, workload):
    """Build the solve in storage `name`, warm up, time args.steps AA steps
    (one lbm_step call per step, HIP events between the launches on the
    launch stream) and return its record: MFLUPS, per-kernel durations,
    rooflines of the odd (dominant) and even kernels, and the solve's size."""
    storage = STORAGES[name]
    dev_exp = 14 if storage == lbm.STORE_F16DEV else 0
    torch.cuda.synchronize()
    tb = time.perf_counter()
    dom = lbm.SparseDomain(lab_dev, per, q, order, 64)
    index_form = "int32"
    escaped = None
    if args.index == "16":
        escaped = dom.compact()
        index_form = "compact16"
        log(f"compact index-list: {100 * escaped:.2f}% of entries escape to int32")
    elif args.index == "run":
        if args.scheme == "pull":
            raise SystemExit("--scheme pull reads the int32 or 16-bit index-list, not runs")
        # AA steps, moments and reductions need only the run form
        runs_bpc = dom.compact_runs(drop_index=True)
        index_form = "runs"
        log(f"run-compressed index-list: {runs_bpc:.2f} bytes per fluid cell")
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb) * 1e3
    nf = dom.n_fluid
    if args.pipelined:
        b, x = lbm.lbm_get_launch(lbm.KERNEL_ODD, q, storage)
        lbm.lbm_set_launch(lbm.KERNEL_ODD, q, storage, 256, x, 1)
    if args.even_cells:
        cfg = list(lbm.lbm_get_launch(lbm.KERNEL_EVEN, q, storage, full=True))
        cfg[3] = args.even_cells
        lbm.lbm_set_launch(lbm.KERNEL_EVEN, q, storage, *cfg)
    for kern, blk, g, x in ((lbm.KERNEL_ODD, args.odd_block, args.odd_groups, args.odd_xcd),
                            (lbm.KERNEL_EVEN, args.even_block, args.even_groups, args.even_xcd)):
        cfg = list(lbm.lbm_get_launch(kern, q, storage, full=True))
        if blk is not None:
            cfg[0] = blk
        if g is not None:
            cfg[4] = g
        if x is not None:
            cfg[1] = x
        lbm.lbm_set_launch(kern, q, storage, *cfg)
    sol = lbm.Solver(dom, storage, dev_exp)
    solve_bytes = dom.device_bytes() + sol.device_bytes()
    if args.tune:
        from paper_2408_06880_amd import autotune
        sol.init()
        tuned = autotune.tune_solver(sol, coll, steps=8)
        log("tuned launch (block, xcd, cells, groups): " +
            ", ".join(f"{'odd' if k == 0 else 'even'} {v[0]}" for k, v in tuned.items()))
    sol.init()
    sol.step(args.warmup, coll, bs)
    torch.cuda.synchronize()
    log(f"{name}: built lists in {build_ms:.1f} ms; warmup {args.warmup} steps done")

    K = args.steps
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    parity0 = sol.t & 1
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    if args.scheme == "pull":
        if K % 2 or sol.t % 2:
            raise SystemExit("the pull scheme needs an even number of steps and warm-up steps")
        sol.step_pull(2, coll)
        torch.cuda.synchronize()
        evs = evs[:K // 2 + 1]
        w0 = time.perf_counter()
        evs[0].record(stream)
        for s in range(K // 2):
            sol.step_pull(2, coll, None, stream)
            evs[s + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        t_odd = t_even = sum(evs[s].elapsed_time(evs[s + 1]) / 2e3 for s in range(K // 2)) / (K // 2)
    else:
        evs[0].record(stream)
        for s in range(K):
            lbm.lbm_step(sol.state, 1, coll, bs, stream)
            evs[s + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        durs = [evs[s].elapsed_time(evs[s + 1]) / 1e3 for s in range(K)]
        odd_d = [d for s, d in enumerate(durs) if ((parity0 + s) & 1) == 0]
        even_d = [d for s, d in enumerate(durs) if ((parity0 + s) & 1) == 1]
        t_odd = sum(odd_d) / max(len(odd_d), 1)
        t_even = sum(even_d) / max(len(even_d), 1)
    mflups = nf * K / wall / 1e6
    b_pdf = lbm.STORE_BYTES[storage]
    # The paper's byte model (int32 index-list, Section "Single Node
    # Results" access table): the figures its bandwidth percentages use.
    b_odd_m, b_even_m, b_alg_m = costmodel.aa_step_bytes(q, b_pdf, 4)
    if args.scheme == "pull":
        b_even_m = b_alg_m = b_odd_m
    # Algorithmic bytes of the kernels as built: the same PDF traffic plus
    # the bytes the index form in use needs (fewer for compressed forms).
    b_idx = 2 if index_form == "compact16" else 4
    b_odd, b_even, b_alg = costmodel.aa_step_bytes(q, b_pdf, b_idx)
    if index_form == "compact16":
        # one int32 base per direction per 256 cells; escaped entries also
        # read their int32 position
        b_odd += (q - 1) * 4 / 256 + (q - 1) * 4 * escaped
        b_alg = 0.5 * (b_odd + b_even)
    elif index_form == "runs":
        # the whole run form (offsets, masks, values) is read once per odd step
        b_odd = 2 * q * b_pdf + dom.runs_bytes / nf
        b_alg = 0.5 * (b_odd + b_even)
    if args.scheme == "pull":   # every step gathers through the index-list
        b_even = b_odd
        b_alg = b_odd
    log(f"{name}: timed {K} steps: {wall * 1e3:.2f} ms, {mflups:.0f} MFLUPS; "
        f"odd {t_odd * 1e6:.1f} us, even {t_even * 1e6:.1f} us")
    red = sol.reduce(coll)
    if not red.finite:
        raise RuntimeError("non-finite state after the timed steps")
    launch_odd = lbm.lbm_get_launch(lbm.KERNEL_ODD, q, storage, full=True)
    launch_even = lbm.lbm_get_launch(lbm.KERNEL_EVEN, q, storage, full=True)
    prof = recorded_profile(f"{workload}; storage={name}; order={args.order}; index={index_form}"
                            + ("; scheme=pull" if args.scheme == "pull" else ""), launch_odd)
    # kernel duration: the rocprofv3 kernel trace of the committed summary
    # while it matches these kernels, else the HIP events of this run
    t_odd_prof = prof["odd_avg_us"] * 1e-6 if prof and prof.get("odd_avg_us") else None
    t_even_prof = prof["even_avg_us"] * 1e-6 if prof and prof.get("even_avg_us") else None
    t_use = t_odd_prof or t_odd
    traffic = prof["odd_bytes"] if prof else None
    achieved = nf * b_odd / t_use / 1e9
    del sol
    keep_dom = {"n_fluid": nf, "stride": dom.stride, "builder_ms": round(build_ms, 2)}
    del dom
    torch.cuda.empty_cache()
    rec = {
        "value": round(mflups, 1),
        "ms_per_step": round(wall / K * 1e3, 5),
        "dtype": {"f64": "f64", "f32": "f32", "f16dev": "f32 (f16 storage)",
                  "bf16dev": "f32 (bf16 storage)", "f32dev": "f32"}[name],
        "config": {"storage": name, "index": index_form, "pipelined_odd": args.pipelined,
                   "tuned": args.tune, "launch_odd": launch_odd, "launch_even": launch_even,
                   "index_escaped_fraction": escaped},
        # percentages of 8 TB/s on the paper's byte model per update (int32
        # index-list) and on the bytes the kernels as built need
        "pct_hbm_peak": round(100.0 * mflups * 1e6 * b_alg_m / (HBM_PEAK_GBS * 1e9), 2),
        "bytes_per_flup_alg": b_alg_m,
        "pct_hbm_peak_index_form": round(100.0 * mflups * 1e6 * b_alg / (HBM_PEAK_GBS * 1e9), 2),
        "bytes_per_flup_index_form": b_alg,
        # HBM bytes per update from the counter summary (odd + even launch)
        "bytes_per_flup_measured": (round((prof["odd_bytes"] + prof["even_bytes"]) / (2 * nf), 2)
                                    if prof and prof.get("even_bytes") and args.scheme == "aa"
                                    else None),
        "roofline": {
            "bound": "hbm",
            "kernel": ("AA odd step (index gather + collide + scatter)"
                       if args.scheme == "aa" else "pull step (gather + collide + store)"),
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_source": prof["source"] if prof else None,
            "bytes_per_launch": round(nf * b_odd),
            "bytes_model": (f"{2 * q} x {b_pdf} B PDFs + the {index_form} index-list "
                            f"({b_odd - 2 * q * b_pdf:.2f} B) per fluid cell"),
            "avg_launch_us": round(t_use * 1e6, 2),
            "timing_source": ("rocprofv3 kernel trace in " + prof["source"]) if t_odd_prof else
                             "HIP events between the launches of the timed region",
            "avg_launch_us_events": round(t_odd * 1e6, 2),
            "frac_events": round(nf * b_odd / t_odd / 1e9 / HBM_PEAK_GBS, 4),
            "achieved_counted": round(traffic / t_use / 1e9, 1) if traffic else None,
            # the same launch priced at the paper's int32 byte model
            "bytes_per_launch_model_equiv": nf * b_odd_m,
            "achieved_model_equiv": round(nf * b_odd_m / t_use / 1e9, 1),
            "frac_model_equiv": round(nf * b_odd_m / t_use / 1e9 / HBM_PEAK_GBS, 4)},
        "even_kernel": {"achieved_gbs": round(nf * b_even / (t_even_prof or t_even) / 1e9, 1),
                        "avg_launch_us": round((t_even_prof or t_even) * 1e6, 2),
                        "avg_launch_us_events": round(t_even * 1e6, 2),
                        "bytes_per_launch": nf * b_even,
                        "traffic": prof["even_bytes"] if prof else None},
        # device buffers of the solve: lists, PDF-list, reduction workspace
        "solve_device_bytes": solve_bytes,
        "solve_bytes_per_fluid_cell": round(solve_bytes / nf, 2),
    }
    return rec, keep_dom


if __name__ == "__main__":
    main()
