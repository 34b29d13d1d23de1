"""Autotuner: per shape, the six-step factorisation, the MFMA substrate and
the tile order of the contiguous axis's second stage.

Candidates per axis are the admissible splits N = p q (both <= 32;
p <= q and p > q are different plans with different output bits, as the
factorisation fixes which roundings happen where); candidates for the
substrate are FP16, INT8 and FP8 (bit-identical outputs for one
factorisation); candidates for the tile order are the group blocks 4, 8,
16 and 32 that divide q of the contiguous axis (how many twiddle groups
run back to back on one XCD; results never depend on it).  Every candidate plan is
timed on the device with HIP events (median of `reps` forward transforms on
a seeded input) and the fastest is cached in a JSON file keyed by shape,
precision and device name ($OBFFT_AUTOTUNE_CACHE, default
~/.cache/obfft/autotune.json).
"""
import itertools
import json
import os

import torch

from . import api, inputs

MAX_K = 32


def splits(N):
    out = []
    for p in range(1, MAX_K + 1):
        if N % p == 0:
            q = N // p
            if 1 <= q <= MAX_K:
                out.append((p, q))
    return out


def _cache_path():
    return os.environ.get("OBFFT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "obfft", "autotune.json"))


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    path = _cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_plan(plan, x, reps):
    y = torch.empty_like(x)
    plan.forward(x, y)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.forward(x, y)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def _try_time(shape, precision, sub, pq, x, reps, group_block=0):
    from ._lib import ObfftError
    try:
        plan = api.Plan(shape, precision=precision, substrate=sub, pq=pq, group_block=group_block)
    except ObfftError:
        return None  # e.g. FP16 with a modulus set it cannot host
    try:
        return _time_plan(plan, x, reps)
    finally:
        plan.close()


def tune(shape, precision="fp64", substrates=("fp16", "int8", "fp8"), reps=3, max_splits=2,
         use_cache=True):
    """Returns {"substrate", "pq", "group_block", "ms"} for the fastest candidate plan of `shape`.

    Phase 1 times every combination of the `max_splits` most balanced splits
    per axis on the first substrate; phase 2 times the other substrates on the
    winning factorisation; phase 3 the group blocks of the winner.
    """
    shape = tuple(int(n) for n in shape)
    dev = torch.cuda.get_device_name(0)
    key = f"{shape[0]}x{shape[1]}x{shape[2]}/{precision}/{dev}"
    cache = _load() if use_cache else {}
    if key in cache:
        return cache[key]
    per_axis = [splits(n) for n in shape]
    if any(not s for s in per_axis):
        raise ValueError(f"no admissible factorisation for {shape}")
    per_axis = [sorted(s, key=lambda pq: (abs(pq[0] - pq[1]), pq[0]))[:max_splits] for s in per_axis]
    dtype = torch.complex128 if precision == "fp64" else torch.complex64
    x = inputs.device_uniform(shape, 0, dtype=dtype)
    best = None
    for pq in itertools.product(*per_axis):
        for sub in substrates:
            ms = _try_time(shape, precision, sub, pq, x, reps)
            if ms is not None:
                break
        if ms is not None and (best is None or ms < best["ms"]):
            best = {"substrate": sub, "pq": [list(v) for v in pq], "ms": ms}
    if best is None:
        raise ValueError(f"no plan could be built for {shape}")
    pq = tuple(tuple(v) for v in best["pq"])
    for sub in substrates:
        if sub == best["substrate"]:
            continue
        ms = _try_time(shape, precision, sub, pq, x, reps)
        if ms is not None and ms < best["ms"]:
            best = {"substrate": sub, "pq": [list(v) for v in pq], "ms": ms}
    best["group_block"] = 0
    q3 = pq[2][1]
    for gb in (4, 8, 16, 32):
        if q3 % gb or gb == 8:  # 8 is the default order just timed
            continue
        ms = _try_time(shape, precision, best["substrate"], pq, x, reps, gb)
        if ms is not None and ms < best["ms"]:
            best = dict(best, group_block=gb, ms=ms)
    if use_cache:
        cache = _load()
        cache[key] = best
        _store(cache)
    return best


def tuned_plan(shape, precision="fp64", **kw):
    t = tune(shape, precision, **kw)
    return api.Plan(shape, precision=precision, substrate=t["substrate"], pq=[tuple(v) for v in t["pq"]],
                    group_block=t.get("group_block", 0))


def tune_batch(shapes, reps=3, max_splits=2, use_cache=True):
    """Per-member choices for a batched plan: every distinct shape is tuned on
    the FP16 substrate (the persistent batch kernel's) over its factorisation
    (which fixes the tile variant of each stage: the packed four- and
    two-column tiles for K <= 4 and K <= 8, the full-length tiles at K = 12,
    16 and 32, the general ones otherwise) and the stage-2 tile order.
    Returns one options dict per member, for api.BatchPlan(member_options=...)."""
    per_shape = {}
    for s in shapes:
        s = tuple(int(n) for n in s)
        if s not in per_shape:
            t = tune(s, substrates=("fp16",), reps=reps, max_splits=max_splits, use_cache=use_cache)
            per_shape[s] = {"pq": [tuple(v) for v in t["pq"]], "group_block": t.get("group_block", 0)}
    return [dict(per_shape[tuple(int(n) for n in s)]) for s in shapes]


def tuned_batch_plan(shapes, **kw):
    return api.BatchPlan(shapes, substrate="fp16", member_options=tune_batch(shapes, **kw))
