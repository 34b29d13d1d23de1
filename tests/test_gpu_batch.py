"""Batched uneven transforms: one launch per Bailey pass and contraction
class (the default) or one persistent launch over every pass of every
member, replayed from a hipGraph.

Every member's output must be bit-identical to the single-transform path
(the same plan, factorisation and axis order), in both modes, on several
graph replays with eager work and synchronisation in between, and with the
graph switched off.  At the full 64-transform workload, the smallest members
are also checked against the oracle's exact pipeline.  The persistent
launch's bounded dependency wait is exercised by a poll limit of zero set
from the host: the kernel then gives up, every workgroup leaves, and the
plan reports OBFFT_BATCH_ABORTED.
"""
import numpy as np
import pytest
import torch

from paper_2606_23698_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["persistent", "passes"])
def test_batch_matches_single_transforms(gpu, mode):
    from paper_2606_23698_amd import api
    shapes, rng = inputs.batch_shapes(seed=3, count=64)
    shapes = [tuple(max(e // 4, 16) if e in (64, 128, 256) else e // 2 for e in s) for s in shapes[:10]]
    shapes += [(32, 64, 96), (64, 64, 64)]
    xs = [torch.from_numpy(inputs.uniform(s, 10 + i)).to(gpu) for i, s in enumerate(shapes)]
    bp = api.BatchPlan(shapes)
    bp.set_mode(mode)
    ref = [api.get_plan(s).forward(x) for s, x in zip(shapes, xs)]
    torch.cuda.synchronize()
    for rep in range(3):
        outs = bp.forward(xs)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            assert torch.equal(o, r), (rep, i, shapes[i])
        _ = torch.randn(1000, device=gpu).sum()   # eager work between replays
    bp.set_graph(False)
    outs = bp.forward(xs)
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)


@pytest.mark.parametrize("mode", ["persistent", "passes"])
def test_batch_on_the_two_m_tile_shape(gpu, mode):
    """Members with length-32 contractions, ragged K (5, 9, 14, 20) and length-1
    axes: every tile variant of the persistent launch."""
    from paper_2606_23698_amd import api
    shapes = [(8, 16, 512), (16, 16, 16), (12, 8, 32), (4, 1024, 4), (25, 81, 196), (1, 45, 400), (3, 2, 7)]
    xs = [torch.from_numpy(inputs.uniform(s, 20 + i)).to(gpu) for i, s in enumerate(shapes)]
    bp = api.BatchPlan(shapes)
    bp.set_mode(mode)
    ref = [api.get_plan(s).forward(x) for s, x in zip(shapes, xs)]
    outs = bp.forward(xs)
    torch.cuda.synchronize()
    for o, r, s in zip(outs, ref, shapes):
        assert torch.equal(o, r), s


def test_batch_64_uneven_workload(gpu):
    """The full 64-transform workload (extents from {64, 96, 128, 192, 256} per
    axis, seed 3): every member equals its single-transform output bit for bit,
    and the three smallest members equal the oracle's exact pipeline."""
    from oracle import exact as ox
    from paper_2606_23698_amd import api
    shapes, xs = inputs.batch_to_device(3, 64, device=gpu)
    bp = api.BatchPlan(shapes)
    outs = bp.forward(xs)
    torch.cuda.synchronize()
    for i, (s, x, o) in enumerate(zip(shapes, xs, outs)):
        assert torch.equal(o, api.get_plan(s).forward(x)), (i, s)
    bp.set_mode("persistent")
    outp = bp.forward(xs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(outp, outs)):
        assert torch.equal(a, b), (i, shapes[i])
    smallest = sorted(range(len(shapes)), key=lambda i: int(np.prod(shapes[i])))[:3]
    for i in smallest:
        plan = api.get_plan(shapes[i])
        pq = tuple(zip(plan.info()["p"], plan.info()["q"]))
        ref = ox.fft3_exact(xs[i].cpu().numpy(), pq)
        assert np.count_nonzero(outs[i].cpu().numpy() != ref) == 0, (i, shapes[i])


def test_persistent_batch_gives_up_when_told(gpu):
    """Poll limit 0: the first unmet dependency makes the persistent launch give
    up; the kernel ends, the plan reports OBFFT_BATCH_ABORTED, and with the
    limit restored the next call is complete and bit-exact again."""
    from paper_2606_23698_amd import api
    shapes = [(128, 128, 128), (64, 96, 64)]
    xs = [torch.from_numpy(inputs.uniform(s, 40 + i)).to(gpu) for i, s in enumerate(shapes)]
    ref = [api.get_plan(s).forward(x) for s, x in zip(shapes, xs)]
    bp = api.BatchPlan(shapes)
    bp.set_mode("persistent")
    bp.set_poll_limit(0)
    bp.forward(xs)
    torch.cuda.synchronize()
    assert bp.last_error() == 9
    bp.clear_error()
    assert bp.last_error() == 0
    bp.set_poll_limit(1 << 21)
    outs = bp.forward(xs)
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)


def test_batch_with_tuned_member_options(gpu, tmp_path, monkeypatch):
    """Per-member options (the autotuner's factorisation and tile order per
    shape): each member equals fft3d_z2z_forward on a single plan made with
    its own options, bit for bit, in both modes; and one member's options
    change only that member's bits."""
    from paper_2606_23698_amd import api, autotune
    monkeypatch.setenv("OBFFT_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    shapes = [(16, 96, 64), (32, 48, 24), (16, 96, 64), (12, 40, 8)]
    mo = autotune.tune_batch(shapes, reps=1)
    assert mo[0] == mo[2]
    # a forced, unbalanced split of the second member (K = 3 and 16 on its n3 axis)
    mo[1] = {"pq": [(4, 8), (3, 16), (3, 8)], "group_block": 0}
    xs = [torch.from_numpy(inputs.uniform(s, 60 + i)).to(gpu) for i, s in enumerate(shapes)]
    refs = [api.Plan(s, substrate="fp16", pq=m["pq"], group_block=m["group_block"]).forward(x)
            for s, m, x in zip(shapes, mo, xs)]
    for mode in ("persistent", "passes"):
        bp = api.BatchPlan(shapes, substrate="fp16", member_options=mo)
        bp.set_mode(mode)
        outs = bp.forward(xs)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert torch.equal(o, r), (mode, i, shapes[i], mo[i])
    default = api.get_plan(shapes[1]).forward(xs[1])
    torch.cuda.synchronize()
    assert not torch.equal(default, refs[1])   # another split rounds elsewhere


def test_persistent_claim_sizes(gpu):
    """Every claim size of the persistent launch (tiles a workgroup takes and
    publishes together) gives the single transforms' bits, on members whose
    passes span one to hundreds of tiles."""
    from paper_2606_23698_amd import api
    shapes = [(64, 96, 128), (16, 16, 16), (96, 64, 32), (8, 256, 8), (32, 32, 32)]
    xs = [torch.from_numpy(inputs.uniform(s, 70 + i)).to(gpu) for i, s in enumerate(shapes)]
    ref = [api.get_plan(s).forward(x) for s, x in zip(shapes, xs)]
    bp = api.BatchPlan(shapes)
    assert 1 <= bp.claim() <= 64
    for c in (1, 2, 3, 7, 64, 256):
        bp.set_claim(c)
        assert bp.claim() == c
        for rep in range(2):
            outs = bp.forward(xs)
            torch.cuda.synchronize()
            for i, (o, r) in enumerate(zip(outs, ref)):
                assert torch.equal(o, r), (c, rep, i, shapes[i])


def test_fp8_batch_class_with_mixed_lengths(gpu):
    """FP8 batch whose K = 32 stage shares a launch with a K = 24 stage (768 =
    24 x 32): the class runs the general tile, which reads the general plane
    layout of the K = 32 member (its plan also holds the full-length tile's);
    outputs equal the single FP8 plans, which take the full-length tile."""
    from paper_2606_23698_amd import api
    shapes = [(2, 2, 1024), (2, 2, 768)]
    xs = [torch.from_numpy(inputs.uniform(s, 90 + i)).to(gpu) for i, s in enumerate(shapes)]
    ref = [api.Plan(s, substrate="fp8").forward(x) for s, x in zip(shapes, xs)]
    bp = api.BatchPlan(shapes, substrate="fp8")
    outs = bp.forward(xs)
    torch.cuda.synchronize()
    for o, r, s in zip(outs, ref, shapes):
        assert torch.equal(o, r), s


def test_fp8_batch_with_full_length_members(gpu):
    """FP8 batches (one launch per pass and class): a class of K = 32 stages
    takes the full-length FP8 tile; outputs equal the single FP8 plans."""
    from paper_2606_23698_amd import api
    shapes = [(2, 4, 1024), (4, 4, 32), (3, 1024, 2)]
    xs = [torch.from_numpy(inputs.uniform(s, 80 + i)).to(gpu) for i, s in enumerate(shapes)]
    ref = [api.Plan(s, substrate="fp8").forward(x) for s, x in zip(shapes, xs)]
    bp = api.BatchPlan(shapes, substrate="fp8")
    outs = bp.forward(xs)
    torch.cuda.synchronize()
    for o, r, s in zip(outs, ref, shapes):
        assert torch.equal(o, r), s
