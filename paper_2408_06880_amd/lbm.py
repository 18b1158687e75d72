"""Thin Python binding of liblbm.so (the C-ABI declared in include/lbm.h).

The functions named ``lbm_*`` marshal arguments onto the C entry points of
the same name and raise ``LbmError`` on a non-zero status.  Every step of the
sparse AA path runs in the library's HIP kernels; PyTorch only provides
device memory (``tensor.data_ptr()``) and the stream
(``torch.cuda.current_stream().cuda_stream``).  There is no CPU fallback: if
the library is missing or cannot be loaded, importing this module raises.

The helper classes ``SparseDomain``/``Solver`` and ``DenseSolver`` allocate
the device buffers a caller needs and drive the entry points.
"""
from __future__ import annotations

import ctypes
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY may point at another build of the same sources (launch-bound
# variants compared by the tuner); default: the in-tree library.
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(_PKG, "liblbm.so")

# ----------------------------------------------------------------- constants
LBM_OK, LBM_EINVAL, LBM_ERANGE, LBM_ENOMEM = 0, -1, -2, -3
LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = -4, -5, -6
D3Q19, D3Q27 = 19, 27
COLL_NONE, COLL_SRT, COLL_TRT, COLL_CUMULANT, COLL_MRT, COLL_CM = 0, 1, 2, 3, 4, 5
# MRT rates of the epsilon, pi, q and m moments suggested by d'Humieres et al. (2002)
MRT_RATES = (1.4, 1.4, 1.2, 1.98)
# central-moment rates of orders 3-6: all one (higher moments at equilibrium)
CM_RATES = (1.0, 1.0, 1.0, 1.0)
STORE_F64, STORE_F32, STORE_F16DEV, STORE_BF16DEV, STORE_F32DEV = 0, 1, 2, 3, 4
ORDER_MORTON, ORDER_LEX, ORDER_BLOCKED = 0, 1, 2
BC_NOSLIP, BC_UBB, BC_PRESSURE = 0, 1, 2
KERNEL_ODD, KERNEL_EVEN, KERNEL_DENSE = 0, 1, 2

STORE_BYTES = {STORE_F64: 8, STORE_F32: 4, STORE_F16DEV: 2, STORE_BF16DEV: 2, STORE_F32DEV: 4}
STORE_NAMES = {STORE_F64: "f64", STORE_F32: "f32", STORE_F16DEV: "f16dev",
               STORE_BF16DEV: "bf16dev", STORE_F32DEV: "f32dev"}

_i32, _i64, _u32, _u64, _f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                ctypes.c_uint64, ctypes.c_double)
_vp = ctypes.c_void_p


class lbm_layout(ctypes.Structure):
    _fields_ = [("nx", _i32), ("ny", _i32), ("nz", _i32), ("periodic", _u32), ("q", _i32),
                ("order", _i32), ("align", _i32), ("reserved", _i32), ("n_fluid", _i64),
                ("stride", _i64), ("n_links", _i64)]


class lbm_state(ctypes.Structure):
    _fields_ = [("layout", lbm_layout), ("storage", _i32), ("dev_exp", _i32), ("pdf", _vp),
                ("index", _vp), ("index16", _vp), ("runs", _vp), ("links", _vp), ("t", _i64),
                ("link_vel", _vp), ("link_vel_t", _i64)]


class lbm_collision(ctypes.Structure):
    _fields_ = [("kind", _i32), ("reserved", _i32), ("tau", _f64), ("magic", _f64),
                ("omega_bulk", _f64), ("force", _f64 * 3), ("rates", _f64 * 4)]


class lbm_bclass(ctypes.Structure):
    _fields_ = [("type", _i32), ("reserved", _i32), ("u", _f64 * 3), ("rho", _f64)]


class lbm_bspec(ctypes.Structure):
    _fields_ = [("n_classes", _i32), ("reserved", _i32), ("cls", lbm_bclass * 8)]


class lbm_reduction(ctypes.Structure):
    _fields_ = [("mass", _f64), ("mom", _f64 * 3), ("n_fluid", _i64), ("finite", _i32),
                ("reserved", _i32)]


class lbm_dense_state(ctypes.Structure):
    _fields_ = [("nx", _i32), ("ny", _i32), ("nz", _i32), ("periodic", _u32), ("q", _i32),
                ("storage", _i32), ("dev_exp", _i32), ("reserved", _i32), ("pdf", _vp),
                ("mask", _vp), ("t", _i64)]


class lbm_launch(ctypes.Structure):
    _fields_ = [("block", _i32), ("xcd_remap", _i32), ("pipelined", _i32),
                ("cells_per_thread", _i32), ("max_groups_per_cu", _i32)]


class LbmError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


_lock = threading.Lock()
_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "lbm_abi_version": (_i32, []),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_build_workspace_bytes": (_u64, [_i32, _i32, _i32, _i32]),
    "lbm_build_sparse": (_i32, [_vp, _i32, _i32, _i32, _u32, _i32, _i32, _i32, _vp,
                                ctypes.POINTER(lbm_layout), _vp, _vp, _vp, _vp]),
    "lbm_index16_bytes": (_u64, [ctypes.POINTER(lbm_layout)]),
    "lbm_compress_index": (_i32, [ctypes.POINTER(lbm_layout), _vp, _vp,
                                  ctypes.POINTER(_u64), _vp]),
    "lbm_runs_header_bytes": (_u64, [ctypes.POINTER(lbm_layout)]),
    "lbm_link_vel_bytes": (_u64, [ctypes.POINTER(lbm_layout)]),
    "lbm_link_vel_prepare": (_i32, [ctypes.POINTER(lbm_layout), _vp, _vp, _vp]),
    "lbm_compress_runs": (_i32, [ctypes.POINTER(lbm_layout), _vp, _vp, _u64,
                                 ctypes.POINTER(_u64), _vp]),
    "lbm_convert": (_i32, [ctypes.POINTER(lbm_state), ctypes.POINTER(lbm_state), _vp]),
    "lbm_init_equilibrium": (_i32, [ctypes.POINTER(lbm_state), _f64, ctypes.POINTER(_f64), _vp]),
    "lbm_step": (_i32, [ctypes.POINTER(lbm_state), _i32, ctypes.POINTER(lbm_collision),
                        ctypes.POINTER(lbm_bspec), _vp]),
    "lbm_step_pull": (_i32, [ctypes.POINTER(lbm_state), ctypes.POINTER(_vp), _i32,
                             ctypes.POINTER(lbm_collision), ctypes.POINTER(lbm_bspec), _vp]),
    "lbm_moments": (_i32, [ctypes.POINTER(lbm_state), ctypes.POINTER(lbm_collision), _i32, _vp,
                           _vp, _vp]),
    "lbm_reduce_workspace_bytes": (_u64, [ctypes.POINTER(lbm_layout)]),
    "lbm_reduce": (_i32, [ctypes.POINTER(lbm_state), ctypes.POINTER(lbm_collision), _vp,
                          ctypes.POINTER(lbm_reduction), _vp]),
    "lbm_step_batch_workspace_bytes": (_u64, [_i32]),
    "lbm_step_batch": (_i32, [ctypes.POINTER(ctypes.POINTER(lbm_state)),
                              ctypes.POINTER(ctypes.POINTER(lbm_collision)),
                              ctypes.POINTER(ctypes.POINTER(lbm_bspec)), _i32, _i32, _vp, _u64,
                              _vp]),
    "lbm_step_batch_noalloc": (_i32, [ctypes.POINTER(ctypes.POINTER(lbm_state)),
                                      ctypes.POINTER(ctypes.POINTER(lbm_collision)),
                                      ctypes.POINTER(ctypes.POINTER(lbm_bspec)), _i32, _i32,
                                      _vp]),
    "lbm_reduce_batch": (_i32, [ctypes.POINTER(ctypes.POINTER(lbm_state)),
                                ctypes.POINTER(ctypes.POINTER(lbm_collision)), _i32, _vp,
                                ctypes.POINTER(lbm_reduction), _vp]),
    "lbm_dense_build_mask": (_i32, [_vp, _i32, _i32, _i32, _u32, _i32, _vp, _vp]),
    "lbm_dense_init_equilibrium": (_i32, [ctypes.POINTER(lbm_dense_state), _f64,
                                          ctypes.POINTER(_f64), _vp]),
    "lbm_dense_step": (_i32, [ctypes.POINTER(lbm_dense_state), _i32,
                              ctypes.POINTER(lbm_collision), _vp]),
    "lbm_set_launch": (_i32, [_i32, _i32, _i32, ctypes.POINTER(lbm_launch)]),
    "lbm_get_launch": (_i32, [_i32, _i32, _i32, ctypes.POINTER(lbm_launch)]),
    "lbm_copy": (_i32, [_vp, _vp, _u64, _vp]),
}

EXPORTED = tuple(_SIGS)


def load():
    """Load liblbm.so (raises if it is missing: there is no fallback path)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -m paper_2408_06880_amd.build` (hipcc, gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _call(name, *args):
    lib = load()
    rc = getattr(lib, name)(*args)
    if rc != 0:
        msg = lib.lbm_last_error()
        raise LbmError(name, rc, msg.decode() if msg else "")
    return rc


def _stream(stream):
    if stream is None:
        import torch
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _vp(stream)
    return _vp(stream.cuda_stream)


def _ptr(t):
    """Device pointer of a tensor (or a raw address given as int)."""
    if t is None:
        return None
    return _vp(t) if isinstance(t, int) else _vp(t.data_ptr())


# ------------------------------------------------------ C entry points
def lbm_abi_version():
    return load().lbm_abi_version()


def lbm_last_error():
    m = load().lbm_last_error()
    return m.decode() if m else ""


def lbm_build_workspace_bytes(nx, ny, nz, order=ORDER_MORTON):
    return int(load().lbm_build_workspace_bytes(nx, ny, nz, order))


def lbm_build_sparse(labels, nx, ny, nz, periodic, q, order, align, workspace, layout=None,
                     cells=None, index=None, links=None, stream=None):
    """Plan (cells None: returns a new lbm_layout) or fill (writes cells/index/links)."""
    lay = layout if layout is not None else lbm_layout()
    _call("lbm_build_sparse", _ptr(labels), nx, ny, nz, periodic, q, order, align,
          _ptr(workspace), ctypes.byref(lay), _ptr(cells), _ptr(index), _ptr(links),
          _stream(stream))
    return lay


def lbm_index16_bytes(layout):
    return int(load().lbm_index16_bytes(ctypes.byref(layout)))


def lbm_compress_index(layout, index, index16, stream=None):
    """Returns the number of escaped entries."""
    n = _u64(0)
    _call("lbm_compress_index", ctypes.byref(layout), _ptr(index), _ptr(index16),
          ctypes.byref(n), _stream(stream))
    return int(n.value)


def lbm_runs_header_bytes(layout):
    return int(load().lbm_runs_header_bytes(ctypes.byref(layout)))


def lbm_link_vel_bytes(layout):
    return int(load().lbm_link_vel_bytes(ctypes.byref(layout)))


def lbm_link_vel_prepare(layout, links, link_vel, stream=None):
    _call("lbm_link_vel_prepare", ctypes.byref(layout), _ptr(links), _ptr(link_vel),
          _stream(stream))


def lbm_compress_runs(layout, index, runs, capacity, stream=None):
    """Returns (status, needed bytes): status 0 when the whole form was
    written, LBM_ENOMEM when only the header fitted in `capacity`; raises
    for any other error, including a capacity below the header size."""
    lib = load()
    need = _u64(0)
    rc = lib.lbm_compress_runs(ctypes.byref(layout), _ptr(index), _ptr(runs), int(capacity),
                               ctypes.byref(need), _stream(stream))
    if rc != LBM_OK and (rc != LBM_ENOMEM or int(capacity) < lbm_runs_header_bytes(layout)):
        msg = lib.lbm_last_error()
        raise LbmError("lbm_compress_runs", rc, msg.decode() if msg else "")
    return int(rc), int(need.value)


def lbm_convert(src, dst, stream=None):
    _call("lbm_convert", ctypes.byref(src), ctypes.byref(dst), _stream(stream))


def lbm_init_equilibrium(state, rho0=1.0, u0=(0.0, 0.0, 0.0), stream=None):
    u = (_f64 * 3)(*u0)
    _call("lbm_init_equilibrium", ctypes.byref(state), float(rho0), u, _stream(stream))


def lbm_step(state, n_steps, coll, bspec=None, stream=None):
    _call("lbm_step", ctypes.byref(state), int(n_steps), ctypes.byref(coll),
          ctypes.byref(bspec) if bspec is not None else None, _stream(stream))


def lbm_step_pull(state, spare_ptr, n_steps, coll, bspec=None, stream=None):
    """spare_ptr: device address of the second PDF-list; returns the address
    now holding the other buffer."""
    sp = _vp(spare_ptr)
    _call("lbm_step_pull", ctypes.byref(state), ctypes.byref(sp), int(n_steps),
          ctypes.byref(coll), ctypes.byref(bspec) if bspec is not None else None,
          _stream(stream))
    return sp.value


def lbm_moments(state, coll, out_f64, rho, u, stream=None):
    _call("lbm_moments", ctypes.byref(state), ctypes.byref(coll), 1 if out_f64 else 0,
          _ptr(rho), _ptr(u), _stream(stream))


def lbm_reduce_workspace_bytes(layout):
    return int(load().lbm_reduce_workspace_bytes(ctypes.byref(layout)))


def lbm_reduce(state, coll, workspace, stream=None, check=True):
    out = lbm_reduction()
    rc = load().lbm_reduce(ctypes.byref(state), ctypes.byref(coll), _ptr(workspace),
                           ctypes.byref(out), _stream(stream))
    if rc != 0 and (check or rc != LBM_EUNSTABLE):
        raise LbmError("lbm_reduce", rc, lbm_last_error())
    return out


def lbm_step_batch_workspace_bytes(n_states):
    return int(load().lbm_step_batch_workspace_bytes(int(n_states)))


def lbm_step_batch(states, colls, bspecs, n_steps, stream=None, workspace=None,
                   workspace_bytes=None):
    """workspace: device tensor of at least lbm_step_batch_workspace_bytes(n)
    bytes (or a raw device address with workspace_bytes); None allocates one
    for this call (its memory is kept from reuse until the call's launches on
    `stream` have run)."""
    n = len(states)
    sp = (ctypes.POINTER(lbm_state) * n)(*[ctypes.pointer(s) for s in states])
    cp = (ctypes.POINTER(lbm_collision) * n)(*[ctypes.pointer(c) for c in colls])
    bp = None
    if bspecs is not None:
        bp = (ctypes.POINTER(lbm_bspec) * n)(
            *[ctypes.pointer(b) if b is not None else ctypes.POINTER(lbm_bspec)() for b in bspecs])
    need = lbm_step_batch_workspace_bytes(n)
    if workspace is None and n > 1:
        import torch
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
        st = stream if stream is not None else torch.cuda.current_stream()
        if isinstance(st, int):
            st = torch.cuda.ExternalStream(st)
        workspace.record_stream(st)
    if workspace_bytes is not None:
        nbytes = int(workspace_bytes)
    elif workspace is not None and not isinstance(workspace, int):
        nbytes = workspace.numel() * workspace.element_size()
    else:
        nbytes = 0
    _call("lbm_step_batch", sp, cp, bp, n, int(n_steps), _ptr(workspace), nbytes,
          _stream(stream))


LBM_STEP_BATCH_NOALLOC_MAX = 1024


def lbm_step_batch_noalloc(states, colls, bspecs, n_steps, stream=None):
    """lbm_step_batch with the segment tables in the library's own device
    array (no workspace, nothing allocated)."""
    n = len(states)
    sp = (ctypes.POINTER(lbm_state) * n)(*[ctypes.pointer(s) for s in states])
    cp = (ctypes.POINTER(lbm_collision) * n)(*[ctypes.pointer(c) for c in colls])
    bp = None
    if bspecs is not None:
        bp = (ctypes.POINTER(lbm_bspec) * n)(
            *[ctypes.pointer(b) if b is not None else ctypes.POINTER(lbm_bspec)() for b in bspecs])
    _call("lbm_step_batch_noalloc", sp, cp, bp, n, int(n_steps), _stream(stream))


def lbm_reduce_batch(states, colls, workspace, stream=None, check=True):
    n = len(states)
    sp = (ctypes.POINTER(lbm_state) * n)(*[ctypes.pointer(s) for s in states])
    cp = (ctypes.POINTER(lbm_collision) * n)(*[ctypes.pointer(c) for c in colls])
    out = (lbm_reduction * n)()
    rc = load().lbm_reduce_batch(sp, cp, n, _ptr(workspace), out, _stream(stream))
    if rc != 0 and (check or rc != LBM_EUNSTABLE):
        raise LbmError("lbm_reduce_batch", rc, lbm_last_error())
    return list(out)


def lbm_dense_build_mask(labels, nx, ny, nz, periodic, q, mask, stream=None):
    _call("lbm_dense_build_mask", _ptr(labels), nx, ny, nz, periodic, q, _ptr(mask),
          _stream(stream))


def lbm_dense_init_equilibrium(state, rho0=1.0, u0=(0.0, 0.0, 0.0), stream=None):
    u = (_f64 * 3)(*u0)
    _call("lbm_dense_init_equilibrium", ctypes.byref(state), float(rho0), u, _stream(stream))


def lbm_dense_step(state, n_steps, coll, stream=None):
    _call("lbm_dense_step", ctypes.byref(state), int(n_steps), ctypes.byref(coll),
          _stream(stream))


def lbm_set_launch(kernel, q, storage, block=256, xcd_remap=16, pipelined=0, cells_per_thread=1,
                   max_groups_per_cu=0):
    cfg = lbm_launch(block, xcd_remap, pipelined, cells_per_thread, max_groups_per_cu)
    _call("lbm_set_launch", kernel, q, storage, ctypes.byref(cfg))


def lbm_get_launch(kernel, q, storage, full=False):
    """(block, xcd_remap), or with full=True (block, xcd_remap, pipelined,
    cells_per_thread, max_groups_per_cu): the argument order of
    lbm_set_launch."""
    cfg = lbm_launch()
    _call("lbm_get_launch", kernel, q, storage, ctypes.byref(cfg))
    if full:
        return (cfg.block, cfg.xcd_remap, cfg.pipelined, cfg.cells_per_thread,
                cfg.max_groups_per_cu)
    return (cfg.block, cfg.xcd_remap)


def lbm_copy(dst, src, nbytes, stream=None):
    _call("lbm_copy", _ptr(dst), _ptr(src), int(nbytes), _stream(stream))


# ------------------------------------------------------- conveniences
def collision(kind=COLL_TRT, tau=0.8, magic=3.0 / 16.0, omega_bulk=1.0, force=(0.0, 0.0, 0.0),
              rates=None):
    """rates: MRT epsilon, pi, q, m groups, or central-moment orders 3-6
    (default per kind)."""
    if rates is None:
        rates = CM_RATES if kind == COLL_CM else MRT_RATES
    c = lbm_collision()
    c.kind, c.tau, c.magic, c.omega_bulk = kind, tau, magic, omega_bulk
    for a in range(3):
        c.force[a] = float(force[a])
    for a in range(4):
        c.rates[a] = float(rates[a])
    return c


def bspec(classes=()):
    """classes: sequence of (type, (ux, uy, uz), rho) for labels 2, 3, ..."""
    b = lbm_bspec()
    b.n_classes = len(classes)
    for i, (typ, u, rho) in enumerate(classes):
        b.cls[i].type = typ
        for a in range(3):
            b.cls[i].u[a] = float(u[a])
        b.cls[i].rho = float(rho)
    return b


def _torch_storage_dtype(storage):
    import torch
    return {STORE_F64: torch.float64, STORE_F32: torch.float32, STORE_F16DEV: torch.int16,
            STORE_BF16DEV: torch.int16, STORE_F32DEV: torch.float32}[storage]


class SparseDomain:
    """Fluid list, index-list and boundary links of one geometry (device)."""

    def __init__(self, labels, periodic, q=19, order=ORDER_MORTON, align=64, stream=None,
                 device="cuda"):
        import numpy as np
        import torch
        lab = labels
        if isinstance(lab, np.ndarray):
            lab = torch.from_numpy(np.ascontiguousarray(lab, dtype=np.uint8))
        lab = lab.to(device=device, dtype=torch.uint8).contiguous()
        nz, ny, nx = lab.shape
        ws = torch.empty(lbm_build_workspace_bytes(nx, ny, nz, order), dtype=torch.uint8,
                         device=device)
        lay = lbm_build_sparse(lab, nx, ny, nz, periodic, q, order, align, ws, stream=stream)
        self.cells = torch.empty(max(lay.n_fluid, 1), dtype=torch.int32, device=device)
        self.index = torch.empty(max((q - 1) * lay.stride, 1), dtype=torch.int32, device=device)
        self.links = torch.empty(max(2 * lay.n_links, 2), dtype=torch.int32, device=device)
        lbm_build_sparse(lab, nx, ny, nz, periodic, q, order, align, ws, layout=lay,
                         cells=self.cells, index=self.index,
                         links=self.links if lay.n_links else None, stream=stream)
        self.layout = lay
        self.shape = (nz, ny, nx)
        self.q = q
        self.periodic = periodic
        self.index16 = None
        self.runs = None
        del ws

    def compact(self, stream=None):
        """Build the compact (16-bit) index-list next to the int32 one;
        returns the fraction of entries that escape to the int32 form."""
        import torch
        if self.index is None:
            raise ValueError("the int32 index-list was dropped; the compact form needs it")
        buf = torch.empty(max(lbm_index16_bytes(self.layout), 1), dtype=torch.uint8,
                          device=self.index.device)
        n_esc = lbm_compress_index(self.layout, self.index, buf, stream)
        self.index16 = buf
        self.escaped = n_esc
        return n_esc / max((self.q - 1) * self.n_fluid, 1)

    def compact_runs(self, stream=None, drop_index=False):
        """Build the run-compressed index-list next to the int32 one (odd
        steps then read it); returns its size in bytes per fluid cell.

        drop_index frees the int32 index-list afterwards: AA steps, moments
        and reductions need only the run form, pull steps and the compact
        16-bit form need the int32 one.  The freed buffer goes back to
        torch's caching allocator (torch.cuda.empty_cache() hands it back
        to the device)."""
        import torch
        if self.index is None:
            raise ValueError("the int32 index-list was dropped already")
        if drop_index and self.index16 is not None:
            raise ValueError("the compact index-list needs the int32 one; cannot drop it")
        dev = self.index.device
        hdr = lbm_runs_header_bytes(self.layout)
        buf = torch.empty(max(hdr, 1), dtype=torch.uint8, device=dev)
        rc, need = lbm_compress_runs(self.layout, self.index, buf, hdr, stream)
        if rc != LBM_OK:
            buf = torch.empty(need, dtype=torch.uint8, device=dev)
            rc, need2 = lbm_compress_runs(self.layout, self.index, buf, need, stream)
            if rc != LBM_OK or need2 != need:
                raise LbmError("lbm_compress_runs", rc, "size changed between calls")
        self.runs = buf
        self.runs_bytes = need
        if drop_index:
            self.index = None   # lbm_compress_runs returned after its kernels ended
        return need / max(self.n_fluid, 1)

    def device_bytes(self):
        """Bytes of the device buffers this domain holds."""
        bufs = (self.cells, self.index, self.links, self.index16, self.runs)
        return sum(b.numel() * b.element_size() for b in bufs if b is not None)

    @property
    def n_fluid(self):
        return int(self.layout.n_fluid)

    @property
    def stride(self):
        return int(self.layout.stride)

    @property
    def n_links(self):
        return int(self.layout.n_links)


class Solver:
    """One sparse AA solve: PDF-list on the device plus its lbm_state."""

    def __init__(self, domain: SparseDomain, storage=STORE_F32, dev_exp=0, device="cuda",
                 link_vel=True):
        """link_vel: give a solve with boundary links its link-velocity
        buffer (the step kernels then hand the outlet cells' velocity to
        the next link update; same results, fewer gathers)."""
        import torch
        self.domain = domain
        n = domain.q * domain.stride
        self.pdf = torch.empty(max(n, 1), dtype=_torch_storage_dtype(storage), device=device)
        st = lbm_state()
        st.layout = domain.layout
        st.storage = storage
        st.dev_exp = dev_exp
        st.pdf = self.pdf.data_ptr()
        st.index = domain.index.data_ptr() if domain.index is not None else None
        st.index16 = domain.index16.data_ptr() if domain.index16 is not None else None
        st.runs = domain.runs.data_ptr() if domain.runs is not None else None
        st.links = domain.links.data_ptr() if domain.n_links else None
        st.t = 0
        st.link_vel_t = -1
        self.link_vel = None
        nb = lbm_link_vel_bytes(domain.layout) if (link_vel and domain.n_links) else 0
        if nb:
            self.link_vel = torch.empty(nb, dtype=torch.uint8, device=device)
            lbm_link_vel_prepare(domain.layout, domain.links, self.link_vel)
            st.link_vel = self.link_vel.data_ptr()
        self.state = st
        self.storage = storage
        self._red_ws = torch.empty(lbm_reduce_workspace_bytes(domain.layout), dtype=torch.uint8,
                                   device=device)

    @property
    def t(self):
        return int(self.state.t)

    def init(self, rho0=1.0, u0=(0.0, 0.0, 0.0), stream=None):
        lbm_init_equilibrium(self.state, rho0, u0, stream)

    def step(self, n, coll, bs=None, stream=None):
        lbm_step(self.state, n, coll, bs, stream)

    def converted(self, storage, dev_exp=0, stream=None):
        """A new Solver on the same domain holding this state in `storage`
        (same step count); this one is left unchanged."""
        other = Solver(self.domain, storage, dev_exp, device=self.pdf.device,
                       link_vel=self.link_vel is not None)
        lbm_convert(self.state, other.state, stream)
        return other

    def step_pull(self, n, coll, bs=None, stream=None):
        """n (even) two-array pull steps; allocates the second array once."""
        import torch
        if getattr(self, "_spare", None) is None:
            self._spare = torch.empty_like(self.pdf)
        bufs = {self.pdf.data_ptr(): self.pdf, self._spare.data_ptr(): self._spare}
        other = lbm_step_pull(self.state, self._spare.data_ptr(), n, coll, bs, stream)
        self.pdf, self._spare = bufs[self.state.pdf], bufs[other]

    def moments(self, coll, f64=True, stream=None):
        import torch
        dt = torch.float64 if f64 else torch.float32
        S = max(self.domain.stride, 1)
        rho = torch.empty(S, dtype=dt, device=self.pdf.device)
        u = torch.empty(3 * S, dtype=dt, device=self.pdf.device)
        lbm_moments(self.state, coll, f64, rho, u, stream)
        return rho, u.view(3, S)

    def reduce(self, coll, stream=None, check=True):
        return lbm_reduce(self.state, coll, self._red_ws, stream, check)

    _CKPT_LAYOUT = ("nx", "ny", "nz", "periodic", "q", "order", "align", "n_fluid", "stride",
                    "n_links")

    def checkpoint(self, path, stream=None):
        """Write the solve to `path` (.npz, no pickled objects): layout,
        storage, scale exponent, step count and the raw PDF-list bytes, plus
        a digest of the fluid list that identifies the geometry.  Waits for
        `stream` (default: the current one)."""
        import hashlib

        import numpy as np
        import torch
        (stream or torch.cuda.current_stream()).synchronize()
        lay = self.state.layout
        meta = np.array([getattr(lay, f) for f in self._CKPT_LAYOUT] +
                        [self.storage, int(self.state.dev_exp), self.t], dtype=np.int64)
        cells = self.domain.cells[:self.domain.n_fluid].cpu().numpy()
        digest = np.frombuffer(hashlib.sha256(cells.tobytes()).digest(), dtype=np.uint8)
        raw = self.pdf.view(torch.uint8).cpu().numpy()
        with open(path, "wb") as f:
            np.savez(f, meta=meta, cells_sha256=digest, pdf=raw)

    def restore(self, path):
        """Load a checkpoint written by checkpoint() for the same geometry
        and storage: the PDF-list and the step count are replaced, so the
        solve continues bit for bit where it was saved (either parity)."""
        import hashlib

        import numpy as np
        import torch
        with np.load(path, allow_pickle=False) as z:
            meta, digest, raw = z["meta"], z["cells_sha256"], z["pdf"]
        lay = self.state.layout
        want = [getattr(lay, f) for f in self._CKPT_LAYOUT] + [self.storage,
                                                                  int(self.state.dev_exp)]
        if meta.shape != (len(want) + 1,) or [int(v) for v in meta[:-1]] != want:
            raise ValueError("checkpoint layout, storage or scale differs from this solve")
        cells = self.domain.cells[:self.domain.n_fluid].cpu().numpy()
        if hashlib.sha256(cells.tobytes()).digest() != digest.tobytes():
            raise ValueError("checkpoint was taken on a different geometry")
        dst = self.pdf.view(torch.uint8)
        if raw.shape != (dst.numel(),):
            raise ValueError("checkpoint PDF-list size differs from this solve")
        dst.copy_(torch.from_numpy(raw))
        torch.cuda.current_stream().synchronize()
        self.state.t = int(meta[-1])
        self.state.link_vel_t = -1   # the PDF-list was written from the file

    def device_bytes(self):
        """Bytes of the device buffers this solver holds (not the domain's)."""
        bufs = (self.pdf, self._red_ws, getattr(self, "_spare", None), self.link_vel)
        return sum(b.numel() * b.element_size() for b in bufs if b is not None)


class DenseSolver:
    """Dense direct-addressing AA comparator over every box cell."""

    def __init__(self, labels, periodic, q=19, storage=STORE_F32, dev_exp=0, device="cuda",
                 stream=None):
        import numpy as np
        import torch
        lab = labels
        if isinstance(lab, np.ndarray):
            lab = torch.from_numpy(np.ascontiguousarray(lab, dtype=np.uint8))
        lab = lab.to(device=device, dtype=torch.uint8).contiguous()
        nz, ny, nx = lab.shape
        N = nx * ny * nz
        self.mask = torch.empty(N, dtype=torch.int32, device=device)
        lbm_dense_build_mask(lab, nx, ny, nz, periodic, q, self.mask, stream)
        self.pdf = torch.empty(q * N, dtype=_torch_storage_dtype(storage), device=device)
        st = lbm_dense_state()
        st.nx, st.ny, st.nz, st.periodic, st.q = nx, ny, nz, periodic, q
        st.storage, st.dev_exp = storage, dev_exp
        st.pdf = self.pdf.data_ptr()
        st.mask = self.mask.data_ptr()
        st.t = 0
        self.state = st
        self.shape = (nz, ny, nx)
        self.q = q

    def init(self, rho0=1.0, u0=(0.0, 0.0, 0.0), stream=None):
        lbm_dense_init_equilibrium(self.state, rho0, u0, stream)

    def step(self, n, coll, stream=None):
        lbm_dense_step(self.state, n, coll, stream)
