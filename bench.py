"""Benchmark: ms per 1024^3 complex FP64 3-D FFT, emulated (Ozaki-Bailey) vs native FP64.

One step = one forward transform of the whole 1024^3 array (all six Bailey
stage launches: three axes x two stages).  Input: uniform[-1, 1) real and
imaginary parts from the PCG64 stream of seed 2 (all real parts, then all
imaginary parts, C order), resident in HBM before the timed region.  Prints
one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--size N]
                    [--substrate auto|fp8|int8] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per 1024^3 Z2Z FFT, emulated vs native FP64, HBM-roof fraction @≤1e-14"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
VALU_PEAK_TOPS = 39.3216       # 256 CU x 64 lane-ops/clk x 2.4 GHz
C_EPI_MIN = 203                # the paper's integer-epilogue ledger, low end, instructions / output
XGMI_LINK_GBS = 153.0          # one xGMI link of MI355X, per direction
SUB_NAME = {0: "fp8", 1: "int8", 2: "fp16"}
# HBM bytes per stage launch at 1024^3 on the FP16 substrate, from the
# FETCH_SIZE (x2.0) and WRITE_SIZE (x1.0) counters in
# profiles/ob_stage_kernel_fp16_1024cubed_counters.md; valid only for the
# kernel sources they were taken with (fingerprint below), else null.
TRAFFIC_MEASURED = {"bytes": 34.610e9, "sources_sha256_16": "74bd6d6a25ee0a68"}
KERNEL_SOURCES = ["paper_2606_23698_amd/csrc/ob_kernels.hip", "paper_2606_23698_amd/csrc/ob_stage.h",
                  "paper_2606_23698_amd/csrc/ob_device.h", "paper_2606_23698_amd/csrc/ob_recon.h",
                  "paper_2606_23698_amd/csrc/obfft_internal.h"]


def measured_traffic(N, substrate):
    import hashlib
    if N != 1024 or substrate != 2:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC_MEASURED["bytes"] if h.hexdigest()[:16] == TRAFFIC_MEASURED["sources_sha256_16"] else None
SUB_DTYPE = {0: "fp8", 1: "i8", 2: "f16"}


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _events()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return e0.elapsed_time(e1) / steps, wall


def stage_durations(plan, x, y, ws_a, reps):
    """Durations of the six stage launches of a transform (the same kernels
    forward runs, launched through the stage entry point), with events between
    consecutive launches on the launch stream and one synchronisation at the end."""
    import torch
    evs = []
    for _ in range(reps):
        cur = x
        for axis in (2, 1, 0):
            for stage, src, dst in ((1, cur, ws_a), (2, ws_a, y)):
                e0, e1 = _events()
                e0.record()
                plan.stage(axis, stage, src, dst)
                e1.record()
                evs.append((e0, e1))
            cur = y
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in evs[-6:]]


def sampled_line_errors(x_host, outs, samples):
    """Normwise relative error of each output against the double-double DFT on
    sampled final-axis lines (the oracle evaluates each line's cost cone)."""
    from oracle import exact as ox
    t0 = time.perf_counter()
    ref = ox.dd_cone_lines(x_host, samples)
    res = {}
    for name, got in outs.items():
        num = den = 0.0
        for s, (hi, lo) in ref.items():
            d = (np.asarray(got[s], dtype=np.complex128) - hi) - lo
            num += float(np.sum(np.abs(d) ** 2))
            den += float(np.sum(np.abs(hi) ** 2))
        res[name] = math.sqrt(num / den)
    res["oracle_s"] = round(time.perf_counter() - t0, 1)
    return res


def precision_sweep(api, x, y_ref, steps, samples=(), lines_out=None):
    """The other substrates and the H0 fold reduction (bit-identical outputs) and
    the FP32 target at the same size (its sampled lines go to lines_out)."""
    import torch
    out = {}
    for sub in ("fp8", "int8"):
        plan = api.Plan(tuple(x.shape), substrate=sub)
        y = torch.empty_like(x)
        ms, _ = time_steps(lambda: plan.forward(x, y), steps, 1)
        same = bool(torch.equal(torch.view_as_real(y), torch.view_as_real(y_ref)))
        out[sub] = {"ms": round(ms, 3), "bit_identical_to_default": same}
        print(f"[bench] {sub}: {ms:.2f} ms, identical={same}", file=sys.stderr, flush=True)
        del y, plan
        torch.cuda.empty_cache()
    # H0 ablation: fold-and-add reduction of the seven friendly moduli
    plan = api.Plan(tuple(x.shape), reduction="h0")
    y = torch.empty_like(x)
    ms, _ = time_steps(lambda: plan.forward(x, y), steps, 1)
    same = bool(torch.equal(torch.view_as_real(y), torch.view_as_real(y_ref)))
    out["h0_fold_reduction"] = {"ms": round(ms, 3), "bit_identical_to_default": same}
    print(f"[bench] h0 fold reduction: {ms:.2f} ms, identical={same}", file=sys.stderr, flush=True)
    del y, plan
    torch.cuda.empty_cache()
    x32 = x.to(torch.complex64)
    plan = api.Plan(tuple(x.shape), precision="fp32")
    y32 = torch.empty_like(x32)
    ms, _ = time_steps(lambda: plan.forward(x32, y32), steps, 1)
    if lines_out is not None:
        lines_out.update({s: y32[:, s[0], s[1]].cpu().numpy() for s in samples})
    out["fp32_target"] = {"ms": round(ms, 3),
                          "hbm_roof_ms": round(48.0 * x.numel() / (HBM_PEAK_GBS * 1e9) * 1e3, 3)}
    print(f"[bench] fp32 target: {ms:.2f} ms", file=sys.stderr, flush=True)
    del x32, y32, plan
    torch.cuda.empty_cache()
    return out


def batch_throughput(api, inputs, steps):
    """64 uneven transforms under a hipGraph: one launch per Bailey pass and
    contraction class (the default), one persistent launch over every pass,
    and the same with the autotuner's factorisation per member shape, against
    loops of single-transform plans."""
    import torch
    from paper_2606_23698_amd import autotune
    shapes, xs = inputs.batch_to_device(3, 64)
    ys = [torch.empty_like(x) for x in xs]
    bp = api.BatchPlan(shapes)
    ms_b, _ = time_steps(lambda: bp.forward(xs, ys), steps, 1)
    bp.set_mode("persistent")
    ysp = [torch.empty_like(x) for x in xs]
    ms_p, _ = time_steps(lambda: bp.forward(xs, ysp), steps, 1)
    claim = bp.claim()
    # the claim size of the persistent launch: fewer releases (each an L2
    # write-back) against a coarser dependency grain
    sweep = {}
    for c in (32, 128, 256):
        bp.set_claim(c)
        sweep[c] = round(time_steps(lambda: bp.forward(xs, ysp), steps, 1)[0], 3)
    sweep[claim] = round(ms_p, 3)
    bp.set_claim(claim)
    plans = [api.get_plan(s) for s in shapes]
    ys2 = [torch.empty_like(x) for x in xs]

    def loop():
        for pl, x, o in zip(plans, xs, ys2):
            pl.forward(x, o)
    ms_l, _ = time_steps(loop, steps, 1)
    same = all(torch.equal(torch.view_as_real(a), torch.view_as_real(b)) for a, b in zip(ys, ys2))
    same_p = all(torch.equal(torch.view_as_real(a), torch.view_as_real(b)) for a, b in zip(ysp, ys2))
    del ysp, bp
    # per-member tuned options (factorisation and tile order per distinct shape)
    t0 = time.perf_counter()
    mo = autotune.tune_batch(shapes, reps=2)
    tune_s = time.perf_counter() - t0
    bt = api.BatchPlan(shapes, substrate="fp16", member_options=mo)
    ms_t, _ = time_steps(lambda: bt.forward(xs, ys), steps, 1)
    tplans = {}
    for s, m in zip(shapes, mo):
        key = (s, tuple(m["pq"]), m["group_block"])
        if key not in tplans:
            tplans[key] = api.Plan(s, substrate="fp16", pq=m["pq"], group_block=m["group_block"])

    def tloop():
        for s, m, x, o in zip(shapes, mo, xs, ys2):
            tplans[(s, tuple(m["pq"]), m["group_block"])].forward(x, o)
    ms_tl, _ = time_steps(tloop, steps, 1)
    same_t = all(torch.equal(torch.view_as_real(a), torch.view_as_real(b)) for a, b in zip(ys, ys2))
    elems = sum(int(np.prod(s)) for s in shapes)
    print(f"[bench] batch64: {ms_b:.2f} ms per-pass graph, {ms_p:.2f} ms persistent (claim {claim}), "
          f"{ms_l:.2f} ms loop; tuned {ms_t:.2f} ms vs tuned loop {ms_tl:.2f} ms", file=sys.stderr, flush=True)
    return {"transforms": len(shapes), "elements": elems, "ms": round(ms_b, 3), "loop_ms": round(ms_l, 3),
            "speedup_vs_loop": round(ms_l / ms_b, 3), "bit_identical_to_loop": same,
            "persistent_ms": round(ms_p, 3), "persistent_claim": claim,
            "persistent_ms_by_claim": {str(k): sweep[k] for k in sorted(sweep)},
            "persistent_bit_identical_to_loop": same_p,
            "tuned": {"ms": round(ms_t, 3), "loop_ms": round(ms_tl, 3), "speedup_vs_loop": round(ms_tl / ms_t, 3),
                      "bit_identical_to_tuned_loop": same_t, "tune_s": round(tune_s, 1),
                      "distinct_shapes": len({tuple(s) for s in shapes})},
            "workload": "64 complex FP64 3-D FFTs, extents from {64,96,128,192,256} per axis, "
                        "uniform[-1,1) (PCG64 seed 3: shapes, then each member's data)"}


def crt_methods(api, inputs, steps):
    """The reconstruction ablations on the residues of one real stage: the
    Kulisch route with Phase A on FP16 and on INT8 MFMA and with 16-bit
    accumulator words, recursive Garner and the plain FP64 sum, each a standalone kernel that reads the residues from
    HBM."""
    import torch
    shape = (256, 256, 256)
    # the standalone reconstruction kernels take residues of the library's CRT
    # modulus set (the paper's), so the stage tap runs on a plan with that set
    # (INT8 substrate; the residues do not depend on the substrate)
    plan = api.Plan(shape, moduli=api.crt_constants("fp64")["moduli"])
    x = inputs.device_uniform(shape, 4)
    taps = torch.empty((x.numel(), 2, 12), dtype=torch.int16, device=x.device)
    plan.stage(2, 1, x, residues=taps)
    res = taps.view(-1, 12)
    n = res.shape[0]
    exps = torch.zeros(n, dtype=torch.int32, device=x.device)
    del x
    line = {"workload": "canonical residues of the 2^25 scalar outputs of stage 1 of the n3 axis of a "
                        "256^3 forward FFT (uniform[-1,1) seed 4), exponent 0",
            "n": n, "hbm_floor_ms": round(n * (24 + 4 + 8) / (HBM_PEAK_GBS * 1e9) * 1e3, 4)}
    outs = {}
    for m in ("kulisch", "kulisch_int8", "kulisch_int16", "garner", "slice_fp64"):
        o = torch.empty(n, dtype=torch.float64, device=res.device)
        ms, _ = time_steps(lambda m=m, o=o: api.crt_reconstruct_method(res, exps, m, out=o), steps, 2)
        outs[m] = o
        line[m] = {"ms": round(ms, 4), "ns_per_output": round(ms * 1e6 / n, 5)}
    exact = outs["kulisch"]
    for m in ("kulisch_int8", "kulisch_int16", "garner"):
        line[m]["bit_identical_to_kulisch"] = bool(torch.equal(outs[m].view(torch.int64), exact.view(torch.int64)))
    d = outs["slice_fp64"] - exact
    nz = exact != 0
    line["slice_fp64"]["rel_l2_vs_exact"] = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(exact))
    line["slice_fp64"]["max_rel_vs_exact"] = float((d[nz].abs() / exact[nz].abs()).max())
    print("[bench] crt methods (ms): " + " ".join(f"{m} {line[m]['ms']:.3f}" for m in outs) +
          f"; fp64-sum rel err {line['slice_fp64']['rel_l2_vs_exact']:.2e}", file=sys.stderr, flush=True)
    del outs, exact, d, res, taps, plan
    torch.cuda.empty_cache()
    return line


def slab_share(api, inputs, steps, P=8, N=1024):
    """One GPU's share of the N^3 transform on P GPUs under the slab
    decomposition: the n3 and n2 passes on its (N/P) x N x N slab, then the
    n1 pass on the transposed slab N x (N/P) x N.  The all-to-all between
    them needs P GPUs and is not run; its time is estimated from the link
    rate."""
    import torch

    def passes(plan, x, y, ws, axes):
        cur = x
        for axis in axes:
            plan.stage(axis, 1, cur, ws)
            plan.stage(axis, 2, ws, y)
            cur = y

    out = {}
    for name, shape, axes in (("local_axes", (N // P, N, N), (2, 1)), ("third_axis", (N, N // P, N), (0,))):
        plan = api.Plan(shape)
        x = inputs.device_uniform(shape, 5)
        y, ws = torch.empty_like(x), torch.empty_like(x)
        ms, _ = time_steps(lambda: passes(plan, x, y, ws, axes), steps, 1)
        out[name + "_ms"] = round(ms, 3)
        del plan, x, y, ws
        torch.cuda.empty_cache()
    slab_bytes = 16 * N ** 3 // P
    out["alltoall_estimate_ms"] = round(slab_bytes / P / (XGMI_LINK_GBS * 1e9) * 1e3, 3)
    out["per_gpu_ms"] = round(out["local_axes_ms"] + out["third_axis_ms"] + out["alltoall_estimate_ms"], 3)
    out["workload"] = (f"one GPU's share of {N}^3 on {P} GPUs: n3, n2 passes on {N // P}x{N}x{N}, n1 pass on "
                       f"{N}x{N // P}x{N} (uniform[-1,1) seed 5); all-to-all estimated at {XGMI_LINK_GBS} GB/s per "
                       f"link, one {slab_bytes // P >> 20} MiB message per peer")
    print(f"[bench] slab share P={P}: local {out['local_axes_ms']:.2f} ms, third {out['third_axis_ms']:.2f} ms",
          file=sys.stderr, flush=True)
    return out


def copy_bandwidth(x, reps=5):
    """Device-to-device copy rate of the transform's array (read + write bytes / time)."""
    import torch
    y = torch.empty_like(x)
    ms, _ = time_steps(lambda: y.copy_(x), reps, 1)
    del y
    torch.cuda.empty_cache()
    return 2 * x.numel() * x.element_size() / (ms * 1e-3) / 1e9


def cpu_baseline(N, pq, target_s=12.0):
    """The exact-pipeline oracle on a bounded sample of axis passes, scaled to one transform.

    The sample is a block of length-N lines of the same distribution (seed 2),
    transformed repeatedly (both Bailey stages, exact int128 products) until
    about `target_s` seconds of CPU time have been spent.
    """
    from oracle import exact as ox
    from paper_2606_23698_amd import inputs
    p, q = pq
    threads = len(os.sched_getaffinity(0))
    nl = max(1, min(32768, (1 << 25) // N))
    x = inputs.uniform((nl, N), 2).reshape(nl, N)
    done, t0 = 0, time.perf_counter()
    while True:
        ox.lines(x, N, p, q, nthreads=threads)
        done += nl
        dt = time.perf_counter() - t0
        if dt >= target_s:
            break
    total_lines = 3 * N * N
    ms = dt * 1e3 * total_lines / done
    return {"value": round(ms, 1), "unit": "ms per transform (extrapolated)", "cores": threads,
            "host_cpu_count": os.cpu_count(), "kind": "oracle",
            "sample": f"{done} length-{N} line passes (both Bailey stages, exact int128 pipeline) "
                      f"in {dt:.1f} s, scaled x{total_lines / done:.2f} to the 3 N^2 line passes of "
                      f"one {N}^3 transform"}


def wide_range_256(api, inputs, steps):
    """The 256^3 wide-dynamic-range workload (magnitudes 2^u, u uniform in
    [-20, 20], random signs and phases, seed 1): emulated forward and inverse,
    the native FP64 forward on the same data, and the round-trip error."""
    import torch
    shape = (256, 256, 256)
    x = torch.from_numpy(inputs.wide_range(shape, 1)).to("cuda:0")
    plan = api.Plan(shape)
    y, back, yn = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
    ms_f, _ = time_steps(lambda: plan.forward(x, y), steps, 2)
    ms_i, _ = time_steps(lambda: plan.inverse(y, back), steps, 2)
    ms_n, _ = time_steps(lambda: plan.native_forward(x, yn), steps, 2)
    rt = float(torch.linalg.vector_norm(back - x) / torch.linalg.vector_norm(x))
    diff = float(torch.linalg.vector_norm(y - yn) / torch.linalg.vector_norm(yn))
    print(f"[bench] wide-range 256^3: forward {ms_f:.3f} ms, inverse {ms_i:.3f} ms, native {ms_n:.3f} ms, "
          f"round trip {rt:.2e}", file=sys.stderr, flush=True)
    out = {"workload": "forward + inverse complex FP64 3-D FFT 256^3, magnitudes 2^u (u uniform[-20,20]), "
                       "random signs and phases (seed 1)",
           "forward_ms": round(ms_f, 4), "inverse_ms": round(ms_i, 4), "native_forward_ms": round(ms_n, 4),
           "hbm_roof_ms": round(96.0 * x.numel() / (HBM_PEAK_GBS * 1e9) * 1e3, 4),
           "rel_l2_round_trip": rt, "rel_l2_emulated_vs_native": diff}
    del x, y, back, yn
    torch.cuda.empty_cache()
    return out


def spectral_loss_512(api, inputs, steps):
    """The differentiable spectral loss L(x) = sum |w_k FFT3(x)|^2, w_k =
    1 / (1 + |k|^2), at 512^3 (uniform[-1, 1), seed 4): one forward and
    backward through the autograd function (emulated forward, hand-written
    adjoint), beside the same gradient from two native FP64 transforms."""
    import torch
    from paper_2606_23698_amd import autograd as ag
    shape = (512, 512, 512)
    x = inputs.uniform_to_device(shape, 4, device="cuda:0").requires_grad_(True)
    w = ag.spectral_weights(shape, x.device)
    plan = api.get_plan(shape, "fp64", "auto", 0)

    def emulated():
        x.grad = None
        ag.spectral_loss(x, w).backward()

    def native():
        with torch.no_grad():
            yn = plan.native_forward(x.detach())
            yn.mul_(w * w)
            return torch.conj(plan.native_forward(torch.conj(yn).resolve_conj())).resolve_conj().mul_(2.0)

    ms_e, _ = time_steps(emulated, steps, 1)
    ms_n, _ = time_steps(native, steps, 1)
    ref = native()
    err = float(torch.linalg.vector_norm(x.grad - ref) / torch.linalg.vector_norm(ref))
    print(f"[bench] spectral loss 512^3: forward+backward {ms_e:.2f} ms (native gradient {ms_n:.2f} ms), "
          f"gradient vs native {err:.2e}", file=sys.stderr, flush=True)
    out = {"workload": "L(x) = sum |w_k FFT3(x)|^2, w_k = 1/(1+|k|^2), complex FP64 512^3 uniform[-1,1) "
                       "(seed 4): loss and gradient through the autograd function",
           "forward_backward_ms": round(ms_e, 3), "native_gradient_ms": round(ms_n, 3),
           "rel_l2_gradient_vs_native": err}
    del x, w, ref
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--substrate", default="auto")
    ap.add_argument("--reduction", default="reciprocal", choices=["reciprocal", "h0"],
                    help="residue reduction of the stage kernels (h0: fold-and-add ablation)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--stage-reps", type=int, default=2)
    ap.add_argument("--no-native", action="store_true", help="skip the native FP64 comparator")
    ap.add_argument("--no-sweep", action="store_true", help="skip the FP8 / INT8 / FP32-target sweep")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-transform batched measurement")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 256^3 wide-range round trip and the 512^3 spectral-loss gradient")
    ap.add_argument("--no-crt", action="store_true", help="skip the reconstruction-method comparison")
    ap.add_argument("--no-slab", action="store_true", help="skip the one-GPU share of the 8-GPU slab decomposition")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the error against the double-double oracle on sampled lines")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run one plain device copy of the input (a known-size reference "
                         "for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU slab "
              "decomposition is not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2606_23698_amd import api, inputs
    dev = torch.device("cuda:0")
    N = args.size
    shape = (N, N, N)
    plan = api.Plan(shape, substrate=args.substrate, reduction=args.reduction)
    info = plan.info()
    x = inputs.uniform_to_device(shape, 2, device=dev)
    y = torch.empty_like(x)
    print(f"[bench] {N}^3 plan ready: p={info['p']} q={info['q']} substrate={info['substrate']}",
          file=sys.stderr, flush=True)

    ms, wall = time_steps(lambda: plan.forward(x, y), args.steps, args.warmup)
    print(f"[bench] emulated forward: {ms:.2f} ms/step", file=sys.stderr, flush=True)
    if args.copy_ref:
        xc = x.clone()
        torch.cuda.synchronize()
        del xc
    # sampled output lines (k2, k3) of the final axis for the accuracy check
    samples = [(k2 % N, 5 % N) for k2 in (0, 17, 511, 1023, 256, 900)]
    got = {"emulated": {s: y[:, s[0], s[1]].cpu().numpy() for s in samples}}
    ms_nat, diff = float("nan"), float("nan")
    if not args.no_native:
        yn = torch.empty_like(x)
        ms_nat, _ = time_steps(lambda: plan.native_forward(x, yn), args.steps, args.warmup)
        print(f"[bench] native forward: {ms_nat:.3f} ms/step", file=sys.stderr, flush=True)
        diff = float(torch.linalg.vector_norm(y - yn) / torch.linalg.vector_norm(yn))
        got["native_fp64"] = {s: yn[:, s[0], s[1]].cpu().numpy() for s in samples}
        del yn

    # the average launch of the dominant kernel over the timed region: the six
    # stage launches are the whole step
    stage_ms = ms / 6.0
    durs = []
    if args.stage_reps > 0:
        ws_a = torch.empty_like(x)
        durs = stage_durations(plan, x, y, ws_a, args.stage_reps)
        print("[bench] stage launches (ms): " + " ".join(f"{d:.2f}" for d in durs), file=sys.stderr, flush=True)
        del ws_a
    torch.cuda.synchronize()

    copy_gbs = copy_bandwidth(x)
    print(f"[bench] device copy: {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    elems = N ** 3
    roof_ms = 96.0 * elems / (HBM_PEAK_GBS * 1e9) * 1e3
    copy_roof_ms = 96.0 * elems / (copy_gbs * 1e9) * 1e3
    n_out_launch = 2 * elems
    achieved = C_EPI_MIN * n_out_launch / (stage_ms * 1e-3) / 1e12
    traffic = measured_traffic(N, info["substrate"]) if args.reduction == "reciprocal" else None
    alg_bytes_launch = 16 * elems      # 96 B per element per transform over six launches
    line = {
        "metric": METRIC,
        "value": round(ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": SUB_DTYPE[info["substrate"]],
        "data": "synthetic",
        "config": {"workload": f"forward complex FP64 3-D FFT {N}x{N}x{N}, Re/Im uniform[-1,1) (PCG64 seed 2)",
                   "n": shape, "p": info["p"], "q": info["q"], "moduli": info["r"],
                   "substrate": SUB_NAME[info["substrate"]], "reduction": args.reduction},
        "native_fp64_ms": round(ms_nat, 3) if ms_nat == ms_nat else None,
        "emulated_over_native": round(ms / ms_nat, 2) if ms_nat == ms_nat else None,
        "hbm_roof_ms": round(roof_ms, 3),
        "hbm_roof_frac": round(roof_ms / ms, 4),
        "native_hbm_roof_frac": round(roof_ms / ms_nat, 4) if ms_nat == ms_nat else None,
        # the roof at the bytes the two-launch axis passes move (Y' leaves the
        # chip between the stages: 192 B per element per transform)
        "hbm_roof_moved_ms": round(2.0 * roof_ms, 3),
        "hbm_roof_moved_frac": round(2.0 * roof_ms / ms, 4),
        "copy_GBs": round(copy_gbs, 1),
        "copy_roof_ms": round(copy_roof_ms, 3),
        "copy_roof_frac": round(copy_roof_ms / ms, 4),
        "native_copy_roof_frac": round(copy_roof_ms / ms_nat, 4) if ms_nat == ms_nat else None,
        "rel_l2_emulated_vs_native": diff if diff == diff else None,
        "wall_ms_per_step": round(wall, 3),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                     "traffic": traffic,
                     "kernel": "ob_stage_kernel", "avg_launch_ms": round(stage_ms, 3),
                     "avg_launch_source": "ms_per_step / 6 (the six stage launches are the timed step)",
                     "algorithmic_per_launch": f"{C_EPI_MIN} integer ops x {n_out_launch} outputs",
                     "stage_launch_ms": [round(d, 3) for d in durs],
                     "hbm_view": {"algorithmic_bytes_per_launch": alg_bytes_launch,
                                  "achieved_GBs": round(alg_bytes_launch / (stage_ms * 1e-3) / 1e9, 1),
                                  "peak_GBs": HBM_PEAK_GBS,
                                  "frac": round(alg_bytes_launch / (stage_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "traffic_over_algorithmic": round(traffic / alg_bytes_launch, 3) if traffic else None}},
    }
    lines32 = {}
    if not args.no_sweep:
        line["precision_sweep"] = precision_sweep(api, x, y, max(2, min(args.steps, 3)), samples, lines32)
    if not args.no_accuracy:
        x_host = x.cpu().numpy()
        err = sampled_line_errors(x_host, got, samples)
        acc = {"rel_l2_emulated": err["emulated"], "rel_l2_native_fp64": err.get("native_fp64"),
               "emulated_within_1e-14": bool(err["emulated"] <= 1e-14),
               "lines": f"{len(samples)} sampled final-axis lines (k2, k3) = {samples}; the FP8 and INT8 "
                        "substrates give the default's bits (precision_sweep), hence its error",
               "oracle_s": err["oracle_s"]}
        if lines32:
            e32 = sampled_line_errors(x_host.astype(np.complex64), {"fp32": lines32}, samples)
            acc["rel_l2_fp32_target"] = e32["fp32"]
            acc["fp32_reference"] = "double-double DFT of the binary32-rounded input"
            acc["oracle_s"] += e32["oracle_s"]
        del x_host
        line["accuracy_vs_double_double"] = acc
        print(f"[bench] error vs double-double on {len(samples)} lines: emulated {err['emulated']:.3e}, "
              f"native {err.get('native_fp64', float('nan')):.3e}, fp32 target "
              f"{acc.get('rel_l2_fp32_target', float('nan')):.3e}", file=sys.stderr, flush=True)
    # the 1024^3 arrays are not needed after this point
    del x, y
    torch.cuda.empty_cache()
    if not args.no_batch:
        line["batch64"] = batch_throughput(api, inputs, max(2, min(args.steps, 5)))
    if not args.no_configs:
        line["wide_range_256"] = wide_range_256(api, inputs, max(3, min(args.steps, 10)))
        line["spectral_loss_512"] = spectral_loss_512(api, inputs, max(2, min(args.steps, 3)))
    if not args.no_crt:
        line["crt_methods"] = crt_methods(api, inputs, max(5, min(args.steps, 10)))
    if not args.no_slab and N == 1024:
        line["slab_share_p8"] = slab_share(api, inputs, max(2, min(args.steps, 3)))
    if not args.no_cpu:
        try:
            line["cpu_baseline"] = cpu_baseline(N, (info["p"][2], info["q"][2]))
        except Exception as exc:  # the oracle is optional for the timing itself
            line["cpu_baseline"] = {"error": str(exc)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
