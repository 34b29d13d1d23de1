"""Helpers shared by the GPU tests (not collected by pytest)."""
import numpy as np


def e4m3(d):
    """OCP E4M3 byte of a small integer |d| <= 16 (independent host encoder)."""
    d = int(d)
    if d == 0:
        return 0
    s = 0x80 if d < 0 else 0
    a = abs(d)
    e = a.bit_length() - 1
    mant = ((a << 3) >> e) - 8
    assert ((mant + 8) << e) >> 3 == a
    return s | ((e + 7) << 3) | mant


def to_torch(x, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(device)


def rel_l2(a, b_hi, b_lo=None):
    a = np.asarray(a, dtype=np.complex128)
    d = (a - b_hi) if b_lo is None else ((a - b_hi) - b_lo)
    return float(np.sqrt(np.sum(np.abs(d) ** 2)) / np.sqrt(np.sum(np.abs(b_hi) ** 2)))


def words_to_int(ws, signed=False):
    v = 0
    for i, w in enumerate(ws):
        v |= (int(w) & 0xFFFFFFFF) << (32 * i)
    if signed and len(ws) and (int(ws[-1]) & 0x80000000):
        v -= 1 << (32 * len(ws))
    return v
