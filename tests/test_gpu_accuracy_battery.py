"""The accuracy battery on the GPU (the paper's input classes, Sec. 9 item
(1a)): impulses, single frequencies, cancellation-heavy and signed data and
a wide exponent range, each transformed forward and back.

For every class: the forward output equals the exact-pipeline oracle bit for
bit; its normwise error against the double-double DFT is <= 1e-14, as is the
native FP64 transform's (both printed); Parseval's identity and the inverse
residual hold to 1e-14; and a second run gives the same bits (deterministic
replay: an LDS or scheduling race would break it).  Closed forms are checked
exactly where the quantised method reproduces them exactly: an impulse at the
origin transforms to exactly all ones.
"""
import numpy as np
import pytest

from gpu_util import rel_l2
from oracle import exact as ox

pytestmark = pytest.mark.gpu

SHAPE = (16, 24, 32)


def _classes():
    rng = np.random.default_rng(90)
    n1, n2, n3 = SHAPE
    out = {}
    x = np.zeros(SHAPE, np.complex128)
    x[0, 0, 0] = 1.0
    out["impulse_origin"] = x
    x = np.zeros(SHAPE, np.complex128)
    x[3, 7, 11] = 1.0 - 0.5j
    out["impulse_offset"] = x
    j = np.indices(SHAPE)
    out["single_tone"] = np.exp(2j * np.pi * (2 * j[0] / n1 + 5 * j[1] / n2 + 9 * j[2] / n3))
    base = rng.uniform(-1, 1, SHAPE) + 1j * rng.uniform(-1, 1, SHAPE)
    # cancellation: pairs of nearly opposite large values plus small ones
    c = base.copy()
    c[:, :, 1::2] = -c[:, :, 0::2] * (1 + 2.0 ** -40)
    out["cancellation"] = c
    out["signed"] = np.sign(rng.uniform(-1, 1, SHAPE)) + 1j * np.sign(rng.uniform(-1, 1, SHAPE))
    u = rng.uniform(-30, 30, SHAPE)
    out["wide_exponent"] = np.exp2(u) * np.exp(2j * np.pi * rng.uniform(0, 1, SHAPE))
    return {k: np.ascontiguousarray(v.astype(np.complex128)) for k, v in out.items()}


CLASSES = _classes()


@pytest.mark.parametrize("kind", list(CLASSES))
def test_accuracy_battery(gpu, kind):
    import torch
    from paper_2606_23698_amd import api
    x = CLASSES[kind]
    plan = api.Plan(SHAPE)
    info = plan.info()
    pq = tuple(zip(info["p"], info["q"]))
    xt = torch.from_numpy(x).to(gpu)
    y = plan.forward(xt)
    y2 = plan.forward(xt)
    yn = plan.native_forward(xt)
    back = plan.inverse(y)
    torch.cuda.synchronize()
    yh, y2h, ynh, bh = y.cpu().numpy(), y2.cpu().numpy(), yn.cpu().numpy(), back.cpu().numpy()
    assert np.array_equal(yh.view(np.uint64), y2h.view(np.uint64))   # deterministic replay
    assert np.count_nonzero(yh != ox.fft3_exact(x, pq)) == 0
    hi, lo = ox.fft3_dd(x)
    e_emu, e_nat = rel_l2(yh, hi, lo), rel_l2(ynh, hi, lo)
    print(f"\n[battery] {kind}: emulated {e_emu:.3e}, native FP64 {e_nat:.3e}", flush=True)
    assert e_emu <= 1e-14 and e_nat <= 1e-14
    n = np.prod(SHAPE)
    px, py = float(np.sum(np.abs(x) ** 2)), float(np.sum(np.abs(yh) ** 2))
    assert abs(py / (n * px) - 1.0) <= 1e-14
    assert rel_l2(bh, x) <= 1e-14
    if kind == "impulse_origin":
        assert np.all(yh == 1.0 + 0.0j)
