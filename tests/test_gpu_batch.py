"""Batched uneven transforms: one persistent launch per Bailey pass, replayed from a hipGraph.

Every member's output must be bit-identical to the single-transform path
(the same plan, factorisation and axis order), on several graph replays with
eager work and synchronisation in between, and with the graph switched off.
At the full 64-transform workload, the smallest members are also checked
against the oracle's exact pipeline.
"""
import numpy as np
import pytest
import torch

from paper_2606_23698_amd import inputs

pytestmark = pytest.mark.gpu


def test_batch_matches_single_transforms(gpu):
    from paper_2606_23698_amd import api
    shapes, rng = inputs.batch_shapes(seed=3, count=64)
    shapes = [tuple(max(e // 4, 16) if e in (64, 128, 256) else e // 2 for e in s) for s in shapes[:10]]
    shapes += [(32, 64, 96), (64, 64, 64)]
    xs = [torch.from_numpy(inputs.uniform(s, 10 + i)).to(gpu) for i, s in enumerate(shapes)]
    bp = api.BatchPlan(shapes)
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


def test_batch_on_the_two_m_tile_shape(gpu):
    """A member with a length-32 contraction puts the whole batch on the K = 32 shape."""
    from paper_2606_23698_amd import api
    shapes = [(8, 16, 512), (16, 16, 16), (12, 8, 32), (4, 1024, 4)]
    xs = [torch.from_numpy(inputs.uniform(s, 20 + i)).to(gpu) for i, s in enumerate(shapes)]
    bp = api.BatchPlan(shapes)
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
    smallest = sorted(range(len(shapes)), key=lambda i: int(np.prod(shapes[i])))[:3]
    for i in smallest:
        plan = api.get_plan(shapes[i])
        pq = tuple(zip(plan.info()["p"], plan.info()["q"]))
        ref = ox.fft3_exact(xs[i].cpu().numpy(), pq)
        assert np.count_nonzero(outs[i].cpu().numpy() != ref) == 0, (i, shapes[i])
