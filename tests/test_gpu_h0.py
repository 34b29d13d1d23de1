"""GPU parity of the H0 fold-and-add residue reduction (Sec. 2, the
reduction-friendly moduli; Sec. 8.3, rung H0).

The fold changes how the stage kernels reduce the GEMM sums of the seven
friendly moduli, not what they compute: residues are unique, so every output
must equal the default (reciprocal) reduction's and the exact-pipeline
oracle's bit for bit, and the residue tap must equal the oracle's exact
integers mod m_i.  Shapes cover every contraction class (K = 2 .. 32,
including the full-length K = 8, 12, 16 and 32 kernels) and inputs at the
magnitude extreme, where the GEMM sums come closest to 2^24.
"""
import numpy as np
import pytest
import torch

from oracle import constants as K
from oracle import exact as ox
from paper_2606_23698_amd import inputs

pytestmark = pytest.mark.gpu


def _api():
    from paper_2606_23698_amd import api
    return api


def _pq(plan):
    info = plan.info()
    return tuple(zip(info["p"], info["q"]))


def _extreme(shape, seed):
    a = 1.0 - 2.0 ** -53
    rng = np.random.default_rng(seed)
    return a * rng.choice([-1.0, 1.0], size=shape) + 1j * a * rng.choice([-1.0, 1.0], size=shape)


def test_h0_forward_32cubed_equals_oracle(gpu):
    api = _api()
    x = inputs.uniform((32, 32, 32), 0)
    plan = api.Plan((32, 32, 32), reduction="h0")
    xt = torch.from_numpy(x).to(gpu)
    y = plan.forward(xt)
    torch.cuda.synchronize()
    ref = ox.fft3_exact(x, _pq(plan))
    assert np.count_nonzero(y.cpu().numpy() != ref) == 0


@pytest.mark.parametrize("shape,kind", [
    ((96, 16, 1024), "uniform"),    # K = 8 / 12, 4 / 4, 32 / 32
    ((256, 6, 64), "uniform"),      # K = 16 / 16, 2 / 3, 8 / 8
    ((12, 4, 1024), "extreme"),     # sums near the FP32 exactness bound
    ((32, 16, 64), "extreme"),
])
def test_h0_bit_identical_to_default(gpu, shape, kind):
    api = _api()
    x = inputs.uniform(shape, 5) if kind == "uniform" else _extreme(shape, 6)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(gpu)
    ref_plan = api.Plan(shape)
    h0_plan = api.Plan(shape, reduction="h0")
    for kind_fn in ("forward", "inverse"):
        a = getattr(ref_plan, kind_fn)(xt)
        b = getattr(h0_plan, kind_fn)(xt)
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(a), torch.view_as_real(b)), kind_fn


def test_h0_residue_tap_matches_oracle_integers(gpu):
    """K = 32 stages (the full-length kernel): the canonical residues of every
    stage output equal the oracle's exact integers mod m_i."""
    api = _api()
    shape = (2, 2, 1024)
    x = _extreme(shape, 7)
    plan = api.Plan(shape, reduction="h0")
    p, q = plan.info()["p"][2], plan.info()["q"][2]
    assert (p, q) == (32, 32)
    xt = torch.from_numpy(x).to(gpu)
    r = 12
    taps = torch.zeros((x.size, 2, r), dtype=torch.int16, device=gpu)
    y1 = plan.stage(2, 1, xt, residues=taps)
    taps2 = torch.zeros((x.size, 2, r), dtype=torch.int16, device=gpu)
    y2 = plan.stage(2, 2, y1, residues=taps2)
    torch.cuda.synchronize()
    N = 1024
    t1 = taps.cpu().numpy().reshape(-1, N, 2, r)
    t2 = taps2.cpu().numpy().reshape(-1, N, 2, r)
    y1h = y1.cpu().numpy().reshape(-1, N)
    y2h = y2.cpu().numpy().reshape(-1, N)
    for line in (0, 3):
        s1 = ox.line_stage(x.reshape(-1, N)[line], N, p, q, 1)
        assert np.array_equal(y1h[line], s1["out"])
        s2 = ox.line_stage(s1["out"], N, p, q, 2)
        assert np.array_equal(y2h[line], s2["out"])
        for k, m in enumerate(K.MODULI_FP64):
            assert np.array_equal(t1[line, :, 0, k], np.array([v % m for v in s1["re"]]))
            assert np.array_equal(t1[line, :, 1, k], np.array([v % m for v in s1["im"]]))
            assert np.array_equal(t2[line, :, 0, k], np.array([v % m for v in s2["re"]]))
            assert np.array_equal(t2[line, :, 1, k], np.array([v % m for v in s2["im"]]))
