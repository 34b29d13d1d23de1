"""The autotuner: admissible factorisations (host) and a tuned plan's parity (GPU)."""
import os

import numpy as np
import pytest

from paper_2606_23698_amd import inputs


def test_admissible_splits():
    from paper_2606_23698_amd.autotune import splits
    assert splits(1024) == [(32, 32)]
    assert splits(512) == [(16, 32), (32, 16)]
    assert splits(96) == [(3, 32), (4, 24), (6, 16), (8, 12), (12, 8), (16, 6), (24, 4), (32, 3)]
    assert splits(1) == [(1, 1)]
    assert splits(37) == []
    for n in (1, 9, 32, 64, 96, 128, 192, 256, 384, 768):
        for p, q in splits(n):
            assert p * q == n and 1 <= p <= 32 and 1 <= q <= 32


@pytest.mark.gpu
def test_tuned_plan_is_bit_exact(gpu, tmp_path):
    import torch
    from oracle import exact as ox
    from paper_2606_23698_amd import autotune
    os.environ["OBFFT_AUTOTUNE_CACHE"] = str(tmp_path / "tune.json")
    shape = (16, 96, 64)
    best = autotune.tune(shape, reps=1)
    assert best["substrate"] in ("fp16", "int8", "fp8")
    assert best["group_block"] in (0, 4, 16, 32)
    again = autotune.tune(shape, reps=1)          # served from the cache
    assert again == best
    plan = autotune.tuned_plan(shape, reps=1)
    x = inputs.uniform(shape, 21)
    y = plan.forward(torch.from_numpy(x).to(gpu)).cpu().numpy()
    pq = tuple(tuple(v) for v in best["pq"])
    ref = ox.fft3_exact(x, pq)
    assert np.count_nonzero(y != ref) == 0


@pytest.mark.gpu
def test_group_block_changes_no_bits(gpu):
    """The stage-2 tile order of the contiguous axis is a speed knob only."""
    import torch
    from paper_2606_23698_amd import api
    # contiguous axis 512 = 16 x 32 (q = 32); 384 and 512 columns per group give
    # 6 and 8 tiles per group, the two grid shapes of the group-block order
    for shape in ((16, 24, 512), (32, 16, 512)):
        x = torch.from_numpy(inputs.uniform(shape, 22)).to(gpu)
        ref = api.Plan(shape).forward(x)
        for gb in (1, 2, 4, 16, 32):
            y = api.Plan(shape, group_block=gb).forward(x)
            torch.cuda.synchronize()
            assert torch.equal(torch.view_as_real(y), torch.view_as_real(ref)), (shape, gb)
