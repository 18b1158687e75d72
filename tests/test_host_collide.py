"""The library's collision headers compiled for the host and compared with
the oracle's independent FP64 operators on random near-equilibrium cells.
The GPU kernels run exactly this arithmetic; here it is checked on the CPU
(FP64 to ~1e-15, FP32 to a few ulp of the deviations)."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CXX = shutil.which("clang++", path="/opt/rocm/llvm/bin") or shutil.which("clang++")


@pytest.fixture(scope="module")
def hostlib(tmp_path_factory):
    if CXX is None:
        pytest.skip("no clang++ for the host build")
    out = tmp_path_factory.mktemp("hostemu") / "libcollide_host.so"
    subprocess.run([CXX, "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                    f"-I{os.path.join(HERE, 'hostemu')}",
                    f"-I{os.path.join(ROOT, 'paper_2408_06880_amd', 'csrc')}",
                    os.path.join(HERE, "hostemu", "collide_host.cpp"), "-o", str(out)],
                   check=True)
    lib = ctypes.CDLL(str(out))
    lib.host_collide.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_long,
                                                      ctypes.c_void_p, ctypes.c_void_p]
    return lib


def _states(q, n, seed):
    rng = np.random.default_rng(seed)
    c, w, _ = oracle.stencil(q)
    out = []
    for _ in range(n):
        rho = 1 + 0.02 * rng.standard_normal()
        u = 0.03 * rng.standard_normal(3)
        cu = c @ u
        out.append(w * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u) *
                   (1 + 0.01 * rng.standard_normal(q)))
    return np.ascontiguousarray(out)


CASES = [(19, 1, 0.8, 0.0, 1.0), (19, 2, 0.7, 3 / 16, 1.0), (27, 1, 0.9, 0.0, 1.0),
         (27, 2, 0.6, 3 / 16, 1.0), (27, 3, 0.62, 0.0, 1.0), (27, 3, 0.8, 0.0, 1.3),
         (27, 3, 1.0, 0.0, 1.0), (19, 4, 0.8, 0.0, 1.19), (19, 4, 0.55, 0.0, 1.6),
         (27, 5, 0.7, 0.0, 1.2), (27, 5, 0.9, 0.0, 1.0)]
RATES = {(4, 0.8): (1.4, 1.4, 1.2, 1.98), (4, 0.55): (1.1, 1.7, 0.6, 1.3),
         (5, 0.7): (1.2, 0.8, 1.5, 1.9), (5, 0.9): (1.0, 1.0, 1.0, 1.0)}


@pytest.mark.parametrize("q,kind,tau,magic,wb", CASES)
def test_device_collision_matches_oracle(hostlib, q, kind, tau, magic, wb):
    F = (1e-5, -2e-6, 3e-6)
    rates = RATES.get((kind, tau), oracle.MRT_RATES)
    p = oracle.params(q=q, kind=kind, tau=tau, magic=magic, omega_bulk=wb, force=F,
                      rates=rates)
    om1 = 1 / tau
    om2 = om1 if kind == 1 else (1 / (0.5 + magic / (tau - 0.5)) if kind == 2 else wb)
    P = np.array((om1, om2) + F + tuple(rates))
    f = _states(q, 200, seed=q + kind)
    ref = oracle.collide(p, f)
    _, w, _ = oracle.stencil(q)
    for f64, tol in ((1, 4e-15), (0, 3e-7)):
        out = np.empty_like(f)
        assert hostlib.host_collide(q, kind, f64, P.ctypes.data, f.shape[0], f.ctypes.data,
                                    out.ctypes.data) == 0
        err = np.max(np.abs(out - ref) / np.abs(ref))
        assert err < tol, (f64, err)
