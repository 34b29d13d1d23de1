"""PyTorch-facing binding of libobfft: argument marshalling only.

Every step of the transform runs in the HIP kernels of libobfft.so; this
module checks tensors, passes device pointers and the current HIP stream,
and raises ObfftError on a failed status.  There is no CPU fallback.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L

SUBSTRATES = {"fp8": 0, "int8": 1, "fp16": 2, "auto": 3}
PRECISIONS = {"fp64": 0, "fp32": 1}
# residue reduction of the stage kernels: FP32 reciprocal (default) or the
# fold-and-add form of the friendly moduli (H0 ablation)
REDUCTIONS = {"reciprocal": 0, "h0": 1}


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _materialise(t):
    """Resolve torch's lazy conjugate / negative views: the kernels read raw memory."""
    if isinstance(t, torch.Tensor):
        if t.is_conj():
            t = t.resolve_conj()
        if t.is_neg():
            t = t.resolve_neg()
    return t


def _check_dev(t, dtype, numel=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def options(precision="fp64", substrate="auto", pq=None, moduli=None, reduction="reciprocal", group_block=0,
            axis_order=None):
    opt = L.Options()
    L.lib().obfft_options_default(ctypes.byref(opt))
    opt.precision = PRECISIONS[precision]
    opt.substrate = SUBSTRATES[substrate]
    opt.reduction = REDUCTIONS[reduction]
    opt.group_block = int(group_block)
    if axis_order is not None:
        for k, a in enumerate(axis_order):
            opt.axis_order[k] = int(a)
    if pq is not None:
        for a, (p, q) in enumerate(pq):
            opt.p[a] = int(p)
            opt.q[a] = int(q)
    keep = None
    if moduli is not None:
        keep = (ctypes.c_int32 * len(moduli))(*moduli)
        opt.n_moduli_override = len(moduli)
        opt.moduli_override = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int32))
    return opt, keep


class Plan:
    """An Ozaki-Bailey 3-D FFT plan for one shape on the current device."""

    def __init__(self, shape, precision="fp64", substrate="auto", pq=None, moduli=None, reduction="reciprocal",
                 group_block=0, axis_order=None):
        self.shape = tuple(int(n) for n in shape)
        if len(self.shape) != 3:
            raise ValueError("shape must have three extents")
        self.precision = precision
        opt, keep = options(precision, substrate, pq, moduli, reduction, group_block, axis_order)
        h = ctypes.c_void_p()
        L.check(L.lib().obfft_plan_create(ctypes.byref(h), *self.shape, ctypes.byref(opt)),
                "obfft_plan_create")
        self._h = h
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().obfft_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        inf = L.PlanInfo()
        L.check(L.lib().obfft_plan_info(self._h, ctypes.byref(inf)), "obfft_plan_info")
        return {"precision": inf.precision, "substrate": inf.substrate, "r": inf.r,
                "moduli": list(inf.moduli[:inf.r]), "log2M": inf.log2M,
                "budget_bits": inf.budget_bits, "p": list(inf.p), "q": list(inf.q),
                "S": inf.S, "S_frac": inf.S_frac, "n": list(inf.n),
                "workspace_bytes": inf.workspace_bytes}

    def roots(self, axis):
        N = self.shape[axis]
        out = np.zeros((N, 2), dtype=np.int64)
        L.check(L.lib().obfft_plan_roots(self._h, axis, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
                "obfft_plan_roots")
        return out

    def set_workspace(self, ws):
        L.check(L.lib().obfft_set_workspace(self._h, _ptr(ws), ws.numel() * ws.element_size()),
                "obfft_set_workspace")
        self._ws = ws

    def _run(self, fname, x, out, stream):
        x = _materialise(x)
        _check_dev(x, self.cdtype, name="input")
        if tuple(x.shape) != self.shape:
            raise ValueError(f"input shape {tuple(x.shape)} != plan shape {self.shape}")
        if out is None:
            out = torch.empty_like(x)
        _check_dev(out, self.cdtype, x.numel(), name="output")
        L.check(getattr(L.lib(), fname)(self._h, _ptr(x), _ptr(out), _stream(stream)), fname)
        return out

    def forward(self, x, out=None, stream=None):
        return self._run("fft3d_z2z_forward" if self.precision == "fp64" else "fft3d_c2c_forward",
                         x, out, stream)

    def forward_noalloc(self, x, out, stream=None):
        """Forward transform through the allocation-free entry point (FP64
        plans): the library's fixed scratch array replaces the plan's
        workspace, and `out` must be supplied."""
        if out is None:
            raise ValueError("forward_noalloc writes into a caller-supplied output")
        return self._run("fft3d_z2z_forward_noalloc", x, out, stream)

    def inverse(self, x, out=None, stream=None):
        return self._run("fft3d_z2z_inverse" if self.precision == "fp64" else "fft3d_c2c_inverse",
                         x, out, stream)

    def adjoint(self, x, out=None, stream=None):
        return self._run("fft3d_z2z_adjoint", x, out, stream)

    def native_forward(self, x, out=None, stream=None):
        return self._run("fft3d_z2z_native_forward", x, out, stream)

    def native_inverse(self, x, out=None, stream=None):
        return self._run("fft3d_z2z_native_inverse", x, out, stream)

    def stage(self, axis, stage, x, out=None, direction=0, residues=None, stream=None):
        """One Bailey stage of one axis; residues (int16 [numel, 2, r]) receives the tap."""
        x = _materialise(x)
        _check_dev(x, self.cdtype, name="input")
        if tuple(x.shape) != self.shape:
            raise ValueError(f"input shape {tuple(x.shape)} != plan shape {self.shape}")
        if out is None:
            out = torch.empty_like(x)
        _check_dev(out, self.cdtype, x.numel(), name="output")
        rp = ctypes.c_void_p(0)
        if residues is not None:
            r = 12 if self.cdtype == torch.complex128 else 6
            _check_dev(residues, torch.int16, x.numel() * 2 * r, name="residues")
            rp = _ptr(residues)
        L.check(L.lib().obfft_stage(self._h, axis, stage, direction, _ptr(x), _ptr(out), rp,
                                    _stream(stream)), "obfft_stage")
        return out

    def debug_tap(self, axis, stage, line, x, out=None, direction=0, stream=None):
        """Epilogue records of one line of one stage (see obfft_debug_tap):
        returns (stage output, uint32 array [n_axis, 2, 64])."""
        x = _materialise(x)
        _check_dev(x, self.cdtype, name="input")
        if tuple(x.shape) != self.shape:
            raise ValueError(f"input shape {tuple(x.shape)} != plan shape {self.shape}")
        if out is None:
            out = torch.empty_like(x)
        _check_dev(out, self.cdtype, x.numel(), name="output")
        dump = np.zeros((self.shape[axis], 2, 64), dtype=np.uint32)
        L.check(L.lib().obfft_debug_tap(self._h, axis, stage, direction, int(line), _ptr(x), _ptr(out),
                                        ctypes.c_void_p(dump.ctypes.data), _stream(stream)), "obfft_debug_tap")
        return out, dump

    def last_error(self):
        """The plan's status: the last failed call, or OBFFT_NONFINITE_INPUT when a
        kernel read an Inf or NaN (synchronise the stream first)."""
        return int(L.lib().obfft_last_error(self._h))

    def clear_error(self):
        L.check(L.lib().obfft_clear_error(self._h), "obfft_clear_error")


class BatchPlan:
    """Several independent FP64 transforms of (possibly) different shapes."""

    def __init__(self, shapes, substrate="auto", member_options=None):
        """member_options: None (library defaults for every member) or one dict
        per member with any of "pq", "group_block", "axis_order" (for example
        an autotuner's choice per shape)."""
        self.shapes = [tuple(int(n) for n in s) for s in shapes]
        arr = np.ascontiguousarray(np.array(self.shapes, dtype=np.int64).reshape(-1))
        h = ctypes.c_void_p()
        shp = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        if member_options is None:
            opt, _ = options("fp64", substrate)
            L.check(L.lib().obfft_batch_plan_create(ctypes.byref(h), len(self.shapes), shp, ctypes.byref(opt)),
                    "obfft_batch_plan_create")
        else:
            if len(member_options) != len(self.shapes):
                raise ValueError("one options dict per member")
            opts = (L.Options * len(self.shapes))()
            for i, mo in enumerate(member_options):
                opts[i], _ = options("fp64", substrate, pq=mo.get("pq"), group_block=mo.get("group_block", 0),
                                     axis_order=mo.get("axis_order"))
            L.check(L.lib().obfft_batch_plan_create_each(ctypes.byref(h), len(self.shapes), shp, opts),
                    "obfft_batch_plan_create_each")
        self._h = h

    def last_error(self):
        return int(L.lib().obfft_last_error(self._h))

    def clear_error(self):
        L.check(L.lib().obfft_clear_error(self._h), "obfft_clear_error")

    def set_graph(self, use_graph):
        L.check(L.lib().obfft_batch_set_graph(self._h, int(bool(use_graph))), "obfft_batch_set_graph")

    BATCH_MODES = {"passes": 0, "persistent": 1}

    def set_mode(self, mode):
        """'persistent': one persistent launch over every pass (FP16 substrate);
        'passes': one launch per Bailey pass and contraction class."""
        L.check(L.lib().obfft_batch_set_mode(self._h, self.BATCH_MODES[mode]), "obfft_batch_set_mode")

    def set_poll_limit(self, polls):
        L.check(L.lib().obfft_batch_set_poll_limit(self._h, int(polls)), "obfft_batch_set_poll_limit")

    def set_claim(self, items):
        """Tiles a workgroup of the persistent launch claims at once (1..256)."""
        L.check(L.lib().obfft_batch_set_claim(self._h, int(items)), "obfft_batch_set_claim")

    def claim(self):
        return int(L.lib().obfft_batch_get_claim(self._h))

    def forward(self, xs, outs=None, stream=None):
        if len(xs) != len(self.shapes):
            raise ValueError("wrong number of inputs")
        xs = [_materialise(x) for x in xs]
        if outs is None:
            outs = [torch.empty_like(x) for x in xs]
        for x, o, s in zip(xs, outs, self.shapes):
            _check_dev(x, torch.complex128, name="input")
            _check_dev(o, torch.complex128, x.numel(), name="output")
            if tuple(x.shape) != s:
                raise ValueError("input shape mismatch")
        ins = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        ous = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        L.check(L.lib().obfft_batch_forward(self._h, ins, ous, _stream(stream)), "obfft_batch_forward")
        return outs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().obfft_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_plans = {}


def get_plan(shape, precision="fp64", substrate="auto", device=None):
    dev = torch.cuda.current_device() if device is None else device
    key = (tuple(shape), precision, substrate, dev)
    if key not in _plans:
        with torch.cuda.device(dev):
            _plans[key] = Plan(shape, precision, substrate)
    return _plans[key]


def fft3(x, substrate="auto", out=None):
    prec = "fp64" if x.dtype == torch.complex128 else "fp32"
    return get_plan(x.shape, prec, substrate, x.device.index).forward(x, out)


def ifft3(x, substrate="auto", out=None):
    prec = "fp64" if x.dtype == torch.complex128 else "fp32"
    return get_plan(x.shape, prec, substrate, x.device.index).inverse(x, out)


def adjoint3(x, substrate="auto", out=None):
    return get_plan(x.shape, "fp64", substrate, x.device.index).adjoint(x, out)


def native_fft3(x, out=None):
    return get_plan(x.shape, "fp64", "auto", x.device.index).native_forward(x, out)


def native_ifft3(x, out=None):
    return get_plan(x.shape, "fp64", "auto", x.device.index).native_inverse(x, out)


def _check_residues(residues, precision):
    r = 12 if precision == "fp64" else 6
    _check_dev(residues, torch.int16, name="residues")
    if residues.dim() != 2 or residues.shape[1] != r:
        raise ValueError(f"residues must have shape [n, {r}] for {precision}, got {tuple(residues.shape)}")


def crt_reconstruct(residues, exps, precision="fp64", taps=False, stream=None):
    """Phase A + Kulisch Phase B of n scalars: residues int16 [n, r] (canonical), exps int32 [n]."""
    _check_residues(residues, precision)
    n = residues.shape[0]
    _check_dev(exps, torch.int32, n, name="exps")
    out = torch.empty(n, dtype=torch.float64 if precision == "fp64" else torch.float32,
                      device=residues.device)
    tp = None
    tptr = ctypes.c_void_p(0)
    if taps:
        lay = taps_layout()
        tp = torch.zeros((n, lay["stride"]), dtype=torch.int32, device=residues.device)
        tptr = _ptr(tp)
    L.check(L.lib().obfft_crt_reconstruct(PRECISIONS[precision], n, _ptr(residues), _ptr(exps),
                                          _ptr(out), tptr, _stream(stream)), "obfft_crt_reconstruct")
    return out, tp


CRT_METHODS = {"kulisch": 0, "garner": 1, "slice_fp64": 2, "kulisch_int8": 3, "kulisch_int16": 4}


def crt_reconstruct_method(residues, exps, method, precision="fp64", out=None, stream=None):
    """One of the reconstruction methods (kulisch, garner, slice_fp64, kulisch_int8,
    kulisch_int16) of n scalars:
    residues int16 [n, r] (canonical), exps int32 [n]."""
    _check_residues(residues, precision)
    n = residues.shape[0]
    _check_dev(exps, torch.int32, n, name="exps")
    dt = torch.float64 if precision == "fp64" else torch.float32
    if out is None:
        out = torch.empty(n, dtype=dt, device=residues.device)
    _check_dev(out, dt, n, name="out")
    L.check(L.lib().obfft_crt_reconstruct_method(PRECISIONS[precision], CRT_METHODS[method], n,
                                                 _ptr(residues), _ptr(exps), _ptr(out), _stream(stream)),
            "obfft_crt_reconstruct_method")
    return out


def taps_layout():
    t = L.TapsLayout()
    L.lib().obfft_taps_layout(ctypes.byref(t))
    return {n: getattr(t, n) for n, _ in L.TapsLayout._fields_}


# bytes of (a and b, d) of each probe kind (one register set per lane, 64 lanes)
_PROBE_BYTES = {0: (512, 1024), 1: (1024, 1024), 2: (1024, 4096), 3: (256, 512), 4: (256, 64),
                5: (1024, 1024), 6: (1024, 4096), 7: (2048, 1024)}


def mfma_probe(kind, a, b, d, stream=None):
    need_ab, need_d = _PROBE_BYTES[kind]
    need_a = need_ab + (256 if kind == 7 else 0)  # kind 7: 64 scales after the operands
    for name, t, need in (("a", a, need_a), ("b", b, need_ab if kind != 4 else 0), ("d", d, need_d)):
        if t is None and need == 0:
            continue
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or \
                t.numel() * t.element_size() < need:
            raise ValueError(f"probe {kind}: {name} must be a contiguous device tensor of >= {need} bytes")
    bp = _ptr(b) if b is not None else ctypes.c_void_p(0)
    L.check(L.lib().obfft_mfma_probe(kind, _ptr(a), bp, _ptr(d), _stream(stream)), "obfft_mfma_probe")
    return d


def quantised_roots(N, bits=52):
    out = np.zeros((N, 2), dtype=np.int64)
    L.check(L.lib().obfft_quantised_roots(N, bits, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
            "obfft_quantised_roots")
    return out


def crt_constants(precision="fp64"):
    c = L.CrtConstants()
    L.check(L.lib().obfft_crt_constants(PRECISIONS[precision], ctypes.byref(c)), "obfft_crt_constants")
    r = c.r

    def words(ws):
        return sum(int(w) << (32 * i) for i, w in enumerate(ws))

    return {"r": r, "S": c.S, "S_frac": c.S_frac, "log2M": c.log2M,
            "moduli": list(c.moduli[:r]), "M": words(c.M),
            "u": [words(c.u[k]) for k in range(r)], "w": [int(c.w[k]) for k in range(r)]}
