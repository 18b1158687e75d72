"""CPU-side checks of the C-ABI library: it loads, exports every function
include/lbm.h declares, and rejects invalid arguments before touching the
GPU (host-only paths; no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_2408_06880_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(lbm.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = lbm.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lbm.lbm_abi_version() == 7


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(lbm.lbm_layout) == 56
    assert ctypes.sizeof(lbm.lbm_state) == 56 + 8 + 40 + 8 + 16
    assert ctypes.sizeof(lbm.lbm_collision) == 8 + 8 * 6 + 8 * 4
    assert ctypes.sizeof(lbm.lbm_bspec) == 8 + 8 * 40
    assert ctypes.sizeof(lbm.lbm_reduction) == 48
    assert ctypes.sizeof(lbm.lbm_dense_state) == 32 + 16 + 8
    assert ctypes.sizeof(lbm.lbm_launch) == 5 * 4


def test_workspace_queries():
    assert lbm.lbm_build_workspace_bytes(0, 4, 4) == 0
    assert lbm.lbm_build_workspace_bytes(2000, 4, 4) == 0
    n = lbm.lbm_build_workspace_bytes(32, 32, 32, lbm.ORDER_MORTON)
    assert n >= 4 * 32 ** 3
    lay = lbm.lbm_layout()
    lay.n_fluid = 1000
    assert lbm.lbm_reduce_workspace_bytes(lay) >= 4 * 5 * 8
    lay.q, lay.stride = 19, 1024
    assert lbm.lbm_index16_bytes(lay) >= 18 * 1024 * 2 + 18 * 4 * 4
    # run form header: uint32 per wave (+1) and uint64 per wave and direction
    a256 = lambda v: (v + 255) // 256 * 256
    assert lbm.lbm_runs_header_bytes(lay) == a256(4 * 17) + a256(8 * 16 * 18)
    lay.q, lay.stride = 27, 1000
    assert lbm.lbm_runs_header_bytes(lay) == a256(4 * 17) + a256(8 * 16 * 26)
    # link-velocity buffer: mask word per wave, offsets (+1), 4 values of
    # 8 bytes per link (an upper bound on the cells with links)
    assert lbm.lbm_link_vel_bytes(lay) == 0
    lay.n_links = 37
    assert lbm.lbm_link_vel_bytes(lay) == a256(8 * 16) + a256(4 * 17) + a256(32 * 37)
    # preparing the buffer checks its arguments before any device work; a
    # layout without links needs no buffer
    expect(lbm.LBM_EINVAL, lbm.lbm_link_vel_prepare, lay, None, 16, 0)
    expect(lbm.LBM_EINVAL, lbm.lbm_link_vel_prepare, lay, 16, None, 0)
    lay.q = 20
    expect(lbm.LBM_EINVAL, lbm.lbm_link_vel_prepare, lay, 16, 16, 0)
    lay.q, lay.n_links = 27, 0
    lbm.lbm_link_vel_prepare(lay, None, None, 0)


def _fake_state(q=19, nf=100, S=128, storage=lbm.STORE_F32):
    st = lbm.lbm_state()
    st.layout.q = q
    st.layout.n_fluid = nf
    st.layout.stride = S
    st.storage = storage
    st.pdf = 16   # never dereferenced: validation fails first
    st.index = 16
    return st


def expect(code, fn, *args, **kw):
    with pytest.raises(lbm.LbmError) as e:
        fn(*args, **kw)
    assert e.value.code == code


def test_invalid_arguments_rejected_on_host():
    coll_bad = lbm.collision(lbm.COLL_SRT, tau=0.5)
    expect(lbm.LBM_EINVAL, lbm.lbm_step, _fake_state(), 1, coll_bad, None, 0)
    expect(lbm.LBM_EINVAL, lbm.lbm_step, _fake_state(q=19), 1,
           lbm.collision(lbm.COLL_CUMULANT, tau=0.8), None, 0)
    expect(lbm.LBM_EINVAL, lbm.lbm_step, _fake_state(storage=9), 1, lbm.collision(), None, 0)
    # MRT: D3Q19 only, every rate in (0, 2)
    expect(lbm.LBM_EINVAL, lbm.lbm_step, _fake_state(q=27), 1,
           lbm.collision(lbm.COLL_MRT, tau=0.8), None, 0)
    expect(lbm.LBM_EINVAL, lbm.lbm_step, _fake_state(), 1,
           lbm.collision(lbm.COLL_MRT, tau=0.8, rates=(1.4, 1.4, 2.0, 1.0)), None, 0)
    expect(lbm.LBM_EINVAL, lbm.lbm_step, _fake_state(), 1,
           lbm.collision(lbm.COLL_MRT, tau=0.8, omega_bulk=0.0), None, 0)
    # central moments: D3Q27 only
    expect(lbm.LBM_EINVAL, lbm.lbm_step, _fake_state(q=19), 1,
           lbm.collision(lbm.COLL_CM, tau=0.8), None, 0)
    expect(lbm.LBM_EINVAL, lbm.lbm_step, _fake_state(q=27), 1,
           lbm.collision(lbm.COLL_CM, tau=0.8, rates=(1, 1, 0, 1)), None, 0)
    st = _fake_state(storage=lbm.STORE_F16DEV)
    st.dev_exp = 30
    expect(lbm.LBM_EINVAL, lbm.lbm_step, st, 1, lbm.collision(), None, 0)
    # positions are unsigned 32-bit: 19 * S between 2^31 and 2^32 is accepted
    # (the size query below gets past validation), from 2^32 on it is not
    need = ctypes.c_uint64(0)
    mid = _fake_state(nf=200_000_000, S=200_000_000).layout
    rc = lbm.load().lbm_compress_runs(ctypes.byref(mid), ctypes.c_void_p(16),
                                      ctypes.c_void_p(16), 0, ctypes.byref(need), None)
    assert rc == lbm.LBM_ENOMEM and need.value == lbm.lbm_runs_header_bytes(mid)
    big = _fake_state(nf=230_000_000, S=230_000_000)   # 19 * S >= 2^32
    rc = lbm.load().lbm_compress_runs(ctypes.byref(big.layout), ctypes.c_void_p(16),
                                      ctypes.c_void_p(16), 0, ctypes.byref(need), None)
    assert rc == lbm.LBM_ERANGE
    expect(lbm.LBM_ERANGE, lbm.lbm_step, big, 1, lbm.collision(), None, 0)
    expect(lbm.LBM_EINVAL, lbm.lbm_step, _fake_state(), -1, lbm.collision(), None, 0)
    expect(lbm.LBM_EINVAL, lbm.lbm_set_launch, lbm.KERNEL_ODD, 19, lbm.STORE_F32, 100, 1)
    expect(lbm.LBM_EINVAL, lbm.lbm_set_launch, 7, 19, lbm.STORE_F32, 256, 1)
    lay = _fake_state().layout
    expect(lbm.LBM_EINVAL, lbm.lbm_compress_runs, lay, None, 16, 1 << 20, 0)
    # a buffer below the header size is refused before any device work
    expect(lbm.LBM_ENOMEM, lbm.lbm_compress_runs, lay, 16, 16,
           lbm.lbm_runs_header_bytes(lay) - 1, 0)
    # an index-list is required: int32 or runs; the compact form needs int32
    st = _fake_state()
    st.index = None
    expect(lbm.LBM_EINVAL, lbm.lbm_step, st, 1, lbm.collision(), None, 0)
    st.index16 = 16
    st.runs = 16
    expect(lbm.LBM_EINVAL, lbm.lbm_step, st, 1, lbm.collision(), None, 0)
    # runs without int32: AA steps may run, pull steps may not
    st.index16 = None
    spare = ctypes.c_void_p(32)
    rc = lbm.load().lbm_step_pull(ctypes.byref(st), ctypes.byref(spare), 2,
                                  ctypes.byref(lbm.collision()), None, None)
    assert rc == lbm.LBM_EINVAL and b"int32" in lbm.load().lbm_last_error()
    need = ctypes.c_uint64(0)
    rc = lbm.load().lbm_compress_runs(ctypes.byref(lay), ctypes.c_void_p(16),
                                      ctypes.c_void_p(16), 0, ctypes.byref(need), None)
    assert rc == lbm.LBM_ENOMEM and need.value == lbm.lbm_runs_header_bytes(lay)


def test_batch_mismatch_rejected_on_host():
    a = _fake_state(storage=lbm.STORE_F32)
    b = _fake_state(storage=lbm.STORE_F64)
    c = lbm.collision()
    ws = dict(workspace=16, workspace_bytes=1 << 20)
    expect(lbm.LBM_ESTATE, lbm.lbm_step_batch, [a, b], [c, c], None, 1, 0, **ws)
    b = _fake_state(storage=lbm.STORE_F32)
    b.t = 1
    expect(lbm.LBM_ESTATE, lbm.lbm_step_batch, [a, b], [c, c], None, 1, 0, **ws)


def test_batch_workspace_checked_on_host():
    """Several states need a workspace of the queried size (their segment
    table); the size check comes before any device work."""
    assert lbm.lbm_step_batch_workspace_bytes(0) == 0
    one = lbm.lbm_step_batch_workspace_bytes(1)
    assert one >= 2 * 128 and one % 256 == 0
    n = 100
    need = lbm.lbm_step_batch_workspace_bytes(n)
    assert need >= 2 * n * 128 and need % 256 == 0 and need > one
    states = [_fake_state() for _ in range(n)]
    c = lbm.collision()
    expect(lbm.LBM_EINVAL, lbm.lbm_step_batch, states, [c] * n, None, 1, 0, workspace=0,
           workspace_bytes=0)
    expect(lbm.LBM_ENOMEM, lbm.lbm_step_batch, states, [c] * n, None, 1, 0, workspace=16,
           workspace_bytes=need - 1)


def test_noalloc_batch_checked_on_host():
    """The allocation-free batch refuses more states than its device array
    holds, and mismatched states, before any device work."""
    n = lbm.LBM_STEP_BATCH_NOALLOC_MAX + 1
    states = [_fake_state() for _ in range(n)]
    c = lbm.collision()
    expect(lbm.LBM_ENOMEM, lbm.lbm_step_batch_noalloc, states, [c] * n, None, 1, 0)
    assert b"at most 1024" in lbm.load().lbm_last_error()
    a = _fake_state(storage=lbm.STORE_F32)
    b = _fake_state(storage=lbm.STORE_F64)
    expect(lbm.LBM_ESTATE, lbm.lbm_step_batch_noalloc, [a, b], [c, c], None, 1, 0)


def test_launch_table_roundtrip():
    old = lbm.lbm_get_launch(lbm.KERNEL_EVEN, 27, lbm.STORE_F16DEV, full=True)
    assert old == (256, 0, 0, 2, 0)       # 16-bit storage: two cells per thread
    assert lbm.lbm_get_launch(lbm.KERNEL_EVEN, 27, lbm.STORE_F32, full=True) == (256, 0, 0, 1, 0)
    # measured residency caps: D3Q19 FP32 and FP32-dev odd 4 and even 3; FP64
    # even step 64-thread workgroups, two cells per thread, 2 per CU
    assert lbm.lbm_get_launch(lbm.KERNEL_ODD, 19, lbm.STORE_F32, full=True) == (256, 16, 0, 1, 4)
    assert lbm.lbm_get_launch(lbm.KERNEL_EVEN, 19, lbm.STORE_F32, full=True) == (256, 0, 0, 1, 3)
    assert lbm.lbm_get_launch(lbm.KERNEL_EVEN, 19, lbm.STORE_F64, full=True) == (64, 0, 0, 2, 2)
    assert lbm.lbm_get_launch(lbm.KERNEL_ODD, 19, lbm.STORE_F64, full=True) == (256, 16, 0, 1, 0)
    assert lbm.lbm_get_launch(lbm.KERNEL_EVEN, 19, lbm.STORE_F32DEV, full=True) == (256, 0, 0, 1, 3)
    assert lbm.lbm_get_launch(lbm.KERNEL_ODD, 27, lbm.STORE_F32, full=True) == (256, 16, 0, 1, 3)
    # D3Q19 16-bit storage: the odd step's tiles in chunks of 256
    assert lbm.lbm_get_launch(lbm.KERNEL_ODD, 19, lbm.STORE_F16DEV, full=True) == (256, 256, 0, 1, 0)
    assert lbm.lbm_get_launch(lbm.KERNEL_ODD, 27, lbm.STORE_F16DEV, full=True) == (256, 16, 0, 1, 0)
    assert lbm.lbm_get_launch(lbm.KERNEL_DENSE, 19, lbm.STORE_F32, full=True)[4] == 0
    lbm.lbm_set_launch(lbm.KERNEL_EVEN, 27, lbm.STORE_F16DEV, 128, 0)
    assert lbm.lbm_get_launch(lbm.KERNEL_EVEN, 27, lbm.STORE_F16DEV) == (128, 0)
    lbm.lbm_set_launch(lbm.KERNEL_EVEN, 27, lbm.STORE_F16DEV, *old)
    assert lbm.lbm_get_launch(lbm.KERNEL_EVEN, 27, lbm.STORE_F16DEV, full=True) == old
    # two cells per thread exist for the even kernel only
    expect(lbm.LBM_EINVAL, lbm.lbm_set_launch, lbm.KERNEL_ODD, 19, lbm.STORE_F32, 256, 1, 0, 2)
    expect(lbm.LBM_EINVAL, lbm.lbm_set_launch, lbm.KERNEL_EVEN, 19, lbm.STORE_F32, 256, 0, 0, 3)
    # tile order: 0, 1 or a chunk of 2..65536 tiles
    for bad in (-1, 65537):
        expect(lbm.LBM_EINVAL, lbm.lbm_set_launch, lbm.KERNEL_ODD, 19, lbm.STORE_F32, 256, bad)
    # residency caps: 0 or 2..16, AA kernels only, not with the pipelined odd kernel
    for bad in (1, 17, -1):
        expect(lbm.LBM_EINVAL, lbm.lbm_set_launch, lbm.KERNEL_ODD, 19, lbm.STORE_F32, 256, 1, 0,
               1, bad)
    expect(lbm.LBM_EINVAL, lbm.lbm_set_launch, lbm.KERNEL_DENSE, 19, lbm.STORE_F32, 256, 0, 0,
           1, 2)
    expect(lbm.LBM_EINVAL, lbm.lbm_set_launch, lbm.KERNEL_ODD, 19, lbm.STORE_F32, 256, 1, 1,
           1, 4)


def test_header_compiles_as_c_and_cxx(tmp_path):
    """include/lbm.h is self-contained C and C++ (no HIP types)."""
    import subprocess
    src = tmp_path / "use.c"
    src.write_text('#include "lbm.h"\nint main(void) { lbm_state s; (void)s; return 0; }\n')
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", f"-I{inc}", str(src)],
                   check=True)
    subprocess.run(["g++", "-std=c++11", "-Wall", "-Werror", "-fsyntax-only", "-x", "c++",
                    f"-I{inc}", str(src)], check=True)
