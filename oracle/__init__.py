"""Plain FP64 CPU oracle for the sparse AA lattice Boltzmann path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_2408_06880_amd``) never imports it, and it never imports the product
path.  It shares no code, table or constant with the HIP library.

The numerics live in ``lbm_oracle.c`` (compiled with gcc, no FMA contraction,
FP64 throughout).  This module is argument marshalling over ctypes plus the
Python-side loops that drive whole runs.  Every C function cites the passage
of the paper (arXiv 2408.06880) it follows.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, brute force or the paper's worked example,
except the cumulant at general relaxation rates with a body force, which is
pinned only by invariants (conservation, vanishing higher cumulants at F = 0,
the omega = 1 closed form, shear-wave viscosity).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lock = threading.Lock()
_lib = None

NONE, SRT, TRT, CUMULANT, MRT, CM = 0, 1, 2, 3, 4, 5
BC_NOSLIP, BC_UBB, BC_PRESSURE = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE FP64, OpenMP over planes)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int32),
        ("kind", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("magic", ctypes.c_double),
        ("omega_bulk", ctypes.c_double),
        ("rates", ctypes.c_double * 4),
        ("force", ctypes.c_double * 3),
        ("n_classes", ctypes.c_int32),
        ("cls_type", ctypes.c_int32 * 8),
        ("cls_u", (ctypes.c_double * 3) * 8),
        ("cls_rho", ctypes.c_double * 8),
    ]


MRT_RATES = (1.4, 1.4, 1.2, 1.98)   # epsilon, pi, q, m (d'Humieres et al. 2002)
CM_RATES = (1.0, 1.0, 1.0, 1.0)     # central moments of order 3, 4, 5, 6


def params(q=19, kind=SRT, tau=0.8, magic=3.0 / 16.0, omega_bulk=1.0, force=(0.0, 0.0, 0.0),
           classes=(), rates=None):
    """classes: sequence of (type, (ux, uy, uz), rho) for labels 2, 3, ...;
    rates: MRT relaxation rates of the epsilon, pi, q and m moments, or
    central-moment rates of orders 3-6 (default per kind)."""
    if rates is None:
        rates = CM_RATES if kind == CM else MRT_RATES
    p = Params()
    p.q = q
    p.kind = kind
    p.tau = tau
    p.magic = magic
    p.omega_bulk = omega_bulk
    for a in range(4):
        p.rates[a] = float(rates[a])
    for a in range(3):
        p.force[a] = float(force[a])
    p.n_classes = len(classes)
    for c, (typ, u, rho) in enumerate(classes):
        p.cls_type[c] = typ
        for a in range(3):
            p.cls_u[c][a] = float(u[a])
        p.cls_rho[c] = float(rho)
    return p


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(Params)
        vp = ctypes.c_void_p
        i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        lib.orc_stencil_tables.argtypes = [i32, vp, vp, vp]
        lib.orc_collide_cells.argtypes = [P, i64, vp, vp]
        lib.orc_mrt_matrix.argtypes = [vp]
        lib.orc_dense_step.argtypes = [P, vp, i32, i32, i32, u32, vp, vp]
        lib.orc_dense_run.argtypes = [P, vp, i32, i32, i32, u32, i64, vp, vp]
        lib.orc_dense_init.argtypes = [i32, vp, i64, ctypes.c_double, vp, vp]
        lib.orc_dense_moments.argtypes = [P, vp, i64, vp, vp, vp]
        lib.orc_dense_reduce.argtypes = [P, vp, i64, vp, vp]
        lib.orc_morton_key.argtypes = [u32, u32, u32]
        lib.orc_morton_key.restype = ctypes.c_uint64
        lib.orc_sparse_build.argtypes = [vp, i32, i32, i32, u32, i32, i32, i32,
                                         ctypes.POINTER(i64), ctypes.POINTER(i64),
                                         ctypes.POINTER(i64), vp, vp, vp]
        lib.orc_sparse_step.argtypes = [P, i64, i64, vp, i64, vp, i64, vp]
        lib.orc_sparse_gather.argtypes = [i32, i64, i64, vp, i64, vp, vp]
        _lib = lib
        return lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's later parallel loops (for timings)."""
    _load().orc_set_num_threads(int(n))


def stencil(q):
    """(c [q,3] int32, w [q] float64, opp [q] int32) of the oracle's velocity set."""
    lib = _load()
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q, np.float64)
    opp = np.zeros(q, np.int32)
    _check(lib.orc_stencil_tables(q, _ptr(c), _ptr(w), _ptr(opp)), "stencil")
    return c, w, opp


def collide(p: Params, f: np.ndarray) -> np.ndarray:
    """Collide cells f[n, q] (pre-collision) -> f*[n, q]."""
    lib = _load()
    f = np.ascontiguousarray(f, np.float64)
    out = np.empty_like(f)
    _check(lib.orc_collide_cells(ctypes.byref(p), f.shape[0], _ptr(f), _ptr(out)), "collide")
    return out


def mrt_matrix() -> np.ndarray:
    """The D3Q19 MRT moment matrix M[k, i] (moment k of direction i)."""
    M = np.empty((19, 19), np.float64)
    _check(_load().orc_mrt_matrix(_ptr(M)), "mrt_matrix")
    return M


def _dims(labels):
    nz, ny, nx = labels.shape
    return nx, ny, nz


def dense_init(q, labels, rho0=1.0, u0=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Equilibrium state A[q, nz, ny, nx] (x fastest)."""
    lib = _load()
    labels = np.ascontiguousarray(labels, np.uint8)
    A = np.empty((q,) + labels.shape, np.float64)
    u = np.asarray(u0, np.float64)
    _check(lib.orc_dense_init(q, _ptr(labels), labels.size, float(rho0), _ptr(u), _ptr(A)),
           "dense_init")
    return A


def dense_run(p: Params, labels, periodic: int, n_steps: int, A: np.ndarray) -> np.ndarray:
    """Advance the dense pull scheme n_steps from post-collision state A (copied)."""
    lib = _load()
    labels = np.ascontiguousarray(labels, np.uint8)
    nx, ny, nz = _dims(labels)
    A = np.ascontiguousarray(A, np.float64).copy()
    B = np.empty_like(A)
    _check(lib.orc_dense_run(ctypes.byref(p), _ptr(labels), nx, ny, nz, periodic, n_steps,
                             _ptr(A), _ptr(B)), "dense_run")
    return A


def dense_moments(p: Params, labels, A):
    lib = _load()
    labels = np.ascontiguousarray(labels, np.uint8)
    rho = np.empty(labels.shape, np.float64)
    u = np.empty((3,) + labels.shape, np.float64)
    _check(lib.orc_dense_moments(ctypes.byref(p), _ptr(labels), labels.size, _ptr(A), _ptr(rho),
                                 _ptr(u)), "dense_moments")
    return rho, u


def dense_reduce(p: Params, labels, A):
    """(mass, momentum[3], n_fluid) with Kahan sums over fluid cells."""
    lib = _load()
    labels = np.ascontiguousarray(labels, np.uint8)
    out = np.empty(5, np.float64)
    _check(lib.orc_dense_reduce(ctypes.byref(p), _ptr(labels), labels.size, _ptr(A), _ptr(out)),
           "dense_reduce")
    return float(out[0]), out[1:4].copy(), int(out[4])


def morton_key(x, y, z) -> int:
    return int(_load().orc_morton_key(x, y, z))


class SparseLayout:
    def __init__(self, n_fluid, stride, n_links, cells, index, links, q, shape, periodic):
        self.n_fluid, self.stride, self.n_links = n_fluid, stride, n_links
        self.cells, self.index, self.links = cells, index, links
        self.q, self.shape, self.periodic = q, shape, periodic


def sparse_build(labels, periodic: int, q: int, order: int = 0, align: int = 64) -> SparseLayout:
    lib = _load()
    labels = np.ascontiguousarray(labels, np.uint8)
    nx, ny, nz = _dims(labels)
    nf, S, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.orc_sparse_build(_ptr(labels), nx, ny, nz, periodic, q, order, align,
                                ctypes.byref(nf), ctypes.byref(S), ctypes.byref(nl),
                                None, None, None), "sparse_build(plan)")
    cells = np.empty(max(nf.value, 1), np.int32)
    index = np.empty(max((q - 1) * S.value, 1), np.int32)
    links = np.empty(max(2 * nl.value, 2), np.int32)
    _check(lib.orc_sparse_build(_ptr(labels), nx, ny, nz, periodic, q, order, align,
                                ctypes.byref(nf), ctypes.byref(S), ctypes.byref(nl),
                                _ptr(cells), _ptr(index), _ptr(links)), "sparse_build")
    return SparseLayout(nf.value, S.value, nl.value, cells[:nf.value], index[:(q - 1) * S.value],
                        links[:2 * nl.value], q, labels.shape, periodic)


def sparse_init(lay: SparseLayout, A_dense: np.ndarray) -> np.ndarray:
    """Scatter a dense post-collision state into the natural slots pdf[i*S + k]."""
    q, S = lay.q, lay.stride
    pdf = np.zeros(q * S, np.float64)
    Af = A_dense.reshape(q, -1)
    for i in range(q):
        pdf[i * S:i * S + lay.n_fluid] = Af[i, lay.cells]
    return pdf


def sparse_run(p: Params, lay: SparseLayout, pdf: np.ndarray, t0: int, n_steps: int) -> np.ndarray:
    lib = _load()
    pdf = np.ascontiguousarray(pdf, np.float64).copy()
    links = np.ascontiguousarray(lay.links if lay.n_links else np.zeros(2, np.int32))
    for t in range(t0, t0 + n_steps):
        _check(lib.orc_sparse_step(ctypes.byref(p), lay.n_fluid, lay.stride, _ptr(lay.index),
                                   lay.n_links, _ptr(links), t, _ptr(pdf)), "sparse_step")
    return pdf


def sparse_gather(lay: SparseLayout, pdf: np.ndarray, t: int) -> np.ndarray:
    """Post-collision PDFs [q, n_fluid] in natural order at time t (either parity)."""
    lib = _load()
    out = np.empty((lay.q, lay.n_fluid), np.float64)
    _check(lib.orc_sparse_gather(lay.q, lay.n_fluid, lay.stride, _ptr(lay.index), t,
                                 _ptr(np.ascontiguousarray(pdf)), _ptr(out)), "sparse_gather")
    return out


def sparse_to_dense(lay: SparseLayout, fk: np.ndarray, fill=np.nan) -> np.ndarray:
    """[q, n_fluid] in list order -> [q, nz, ny, nx] (non-fluid cells = fill)."""
    q = fk.shape[0]
    out = np.full((q, int(np.prod(lay.shape))), fill, np.float64)
    out[:, lay.cells] = fk
    return out.reshape((q,) + tuple(lay.shape))
