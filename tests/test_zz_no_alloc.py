"""The allocation-free forward transform (fft3d_z2z_forward_noalloc).

It runs the same kernels as fft3d_z2z_forward with the library's fixed
scratch array as the Y' workspace, so its output must equal the forward
transform's bit for bit.  Two calls in a row, the second on a smaller
input (the scratch keeps the first call's contents, which the second must
not see), then the first shape again; a plan whose workspace exceeds the
scratch is rejected before anything runs, and the output is left untouched.
"""
import pytest
import torch

from paper_2606_23698_amd import inputs

pytestmark = pytest.mark.gpu

SCRATCH_EXCEEDED = 10


def _api():
    from paper_2606_23698_amd import api
    return api


def test_noalloc_forward_equals_forward(gpu):
    api = _api()
    for shape, seed in (((64, 96, 128), 50), ((16, 8, 32), 51), ((64, 96, 128), 52)):
        plan = api.get_plan(shape)
        x = torch.from_numpy(inputs.uniform(shape, seed)).to(gpu)
        ref = plan.forward(x)
        out = torch.full_like(x, complex(float("nan"), float("nan")))
        plan.forward_noalloc(x, out)
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref)), shape
        assert plan.last_error() == 0


def test_noalloc_rejects_a_transform_beyond_the_scratch(gpu):
    api = _api()
    from paper_2606_23698_amd import _lib as L
    cap = int(L.lib().obfft_noalloc_scratch_bytes())
    assert cap == 256 << 20
    shape = (512, 256, 256)            # 2^25 complex128 elements: 512 MiB of workspace
    plan = api.Plan(shape)
    assert plan.info()["workspace_bytes"] > cap
    x = torch.zeros(shape, dtype=torch.complex128, device=gpu)
    out = torch.full_like(x, 7.0)
    with pytest.raises(L.ObfftError) as ei:
        plan.forward_noalloc(x, out)
    assert ei.value.status == SCRATCH_EXCEEDED
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    plan.clear_error()
