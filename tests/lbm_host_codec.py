"""Host-side encode/decode of the library's PDF storage formats, for tests.

These mirror the storage formats documented in include/lbm.h (FP64/FP32
populations, FP32/FP16/BF16 deviations f - w with a 2^dev_exp scale) so that
a test can hand the GPU an exactly known state and hand the oracle the very
same values in FP64.  No method arithmetic lives here.
"""
import numpy as np

import oracle

F64, F32, F16DEV, BF16DEV, F32DEV = 0, 1, 2, 3, 4


def _bf16_bits(x32: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit pattern, round to nearest even."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def _bf16_value(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def encode(storage, f, q, dev_exp=0):
    """f: FP64 [q, n].  Returns (raw array for the device, FP64 values the
    device will see)."""
    _, w, _ = oracle.stencil(q)
    w = w[:, None]
    sc = 2.0 ** dev_exp
    if storage == F64:
        return f.astype(np.float64), f.astype(np.float64)
    if storage == F32:
        a = f.astype(np.float32)
        return a, a.astype(np.float64)
    if storage == F32DEV:
        a = (f - w).astype(np.float32)
        return a, w + a.astype(np.float64)
    if storage == F16DEV:
        a = ((f - w) * sc).astype(np.float16)
        return a.view(np.int16), w + a.astype(np.float64) / sc
    if storage == BF16DEV:
        bits = _bf16_bits(((f - w) * sc).astype(np.float32))
        return bits.view(np.int16), w + _bf16_value(bits) / sc
    raise ValueError(storage)


def decode(storage, raw, q, dev_exp=0):
    _, w, _ = oracle.stencil(q)
    w = w[:, None]
    sc = 2.0 ** dev_exp
    if storage in (F64, F32):
        return raw.astype(np.float64)
    if storage == F32DEV:
        return w + raw.astype(np.float64)
    if storage == F16DEV:
        return w + raw.view(np.float16).astype(np.float64) / sc
    if storage == BF16DEV:
        return w + _bf16_value(raw.view(np.uint16)) / sc
    raise ValueError(storage)


def ulp_bound(storage, f_ref, q, dev_exp=0):
    """One unit in the last place of the 16-bit code of f_ref - w, in f units."""
    _, w, _ = oracle.stencil(q)
    x = np.abs((f_ref - w[:, None]) * 2.0 ** dev_exp)
    m, e = np.frexp(np.maximum(x, 1e-300))
    if storage == F16DEV:
        ulp = np.maximum(2.0 ** (e - 11), 2.0 ** -24)
    elif storage == BF16DEV:
        ulp = 2.0 ** (e - 8)
    else:
        raise ValueError(storage)
    return ulp / 2.0 ** dev_exp
