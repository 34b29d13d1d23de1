"""Parity of the full Ozaki-Bailey transform with the exact-pipeline oracle.

Bit-exact: every FP64 output of the GPU transform equals the oracle's (the
emulated transform has exactly one correct result per plan and input: the
quantised integer products are exact, and the only rounding is the single
correctly rounded pack, Sec. 5.1).  Accuracy: normwise relative L2 error
against the double-double DFT <= 1e-14 (the target of the method).
"""
import numpy as np
import pytest
import torch

from gpu_util import rel_l2
from oracle import exact as ox
from paper_2606_23698_amd import inputs

pytestmark = pytest.mark.gpu


def _api():
    from paper_2606_23698_amd import api
    return api


def _run(plan, x, gpu, kind="forward"):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(gpu)
    y = getattr(plan, kind)(xt)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _pq(plan):
    info = plan.info()
    return tuple(zip(info["p"], info["q"]))


@pytest.mark.parametrize("substrate", ["fp8", "int8", "fp16"])
def test_forward_32cubed_bit_exact(gpu, substrate):
    api = _api()
    x = inputs.uniform((32, 32, 32), 0)
    plan = api.Plan((32, 32, 32), substrate=substrate)
    assert _pq(plan) == ((4, 8),) * 3
    y = _run(plan, x, gpu)
    ref = ox.fft3_exact(x, _pq(plan))
    mism = np.count_nonzero(y != ref)
    assert mism == 0, f"{mism} mismatches"
    hi, lo = ox.fft3_dd(x)
    assert rel_l2(y, hi, lo) <= 1e-14


@pytest.mark.parametrize("shape,pq", [
    ((8, 12, 16), None),
    ((16, 8, 32), ((4, 4), (2, 4), (8, 4))),
    ((4, 64, 24), None),
    ((32, 16, 64), ((8, 4), (4, 4), (8, 8))),
    ((1, 9, 32), None),                       # length-1 axis, odd 3 x 3
    ((15, 1, 25), None),                      # 3 x 5 and 5 x 5
    ((3, 5, 7), None),                        # 1 x 3, 1 x 5, 1 x 7
    ((1, 1, 1), None),                        # the identity
    ((18, 4, 2), ((3, 6), (1, 4), (2, 1))),   # forced odd / unit factors
    ((96, 4, 48), ((8, 12), (2, 2), (4, 12))),  # full-length K = 12 and K = 8 launches
])
@pytest.mark.parametrize("substrate", ["fp8", "int8", "fp16"])
def test_forward_small_shapes_bit_exact(gpu, shape, pq, substrate):
    api = _api()
    x = inputs.uniform(shape, 7)
    plan = api.Plan(shape, substrate=substrate, pq=pq)
    y = _run(plan, x, gpu)
    ref = ox.fft3_exact(x, _pq(plan))
    assert np.count_nonzero(y != ref) == 0


@pytest.mark.parametrize("substrate", ["fp8", "fp16"])
def test_stage_residue_tap_matches_oracle_integers(gpu, substrate):
    """The canonical residues R_i, I_i of every stage output equal (exact integer) mod m_i."""
    api = _api()
    shape = (4, 4, 32)
    x = inputs.uniform(shape, 3)
    plan = api.Plan(shape, substrate=substrate)
    p, q = plan.info()["p"][2], plan.info()["q"][2]
    mods = plan.info()["moduli"]
    xt = torch.from_numpy(x).to(gpu)
    r = 12
    assert len(mods) == r
    taps = torch.zeros((x.size, 2, r), dtype=torch.int16, device=gpu)
    y1 = plan.stage(2, 1, xt, residues=taps)
    taps2 = torch.zeros((x.size, 2, r), dtype=torch.int16, device=gpu)
    y2 = plan.stage(2, 2, y1, residues=taps2)
    torch.cuda.synchronize()
    t1 = taps.cpu().numpy().reshape(-1, 32, 2, r)
    t2 = taps2.cpu().numpy().reshape(-1, 32, 2, r)
    y1h = y1.cpu().numpy().reshape(-1, 32)
    y2h = y2.cpu().numpy().reshape(-1, 32)
    for line in (0, 5, 15):
        xl = x.reshape(-1, 32)[line]
        s1 = ox.line_stage(xl, 32, p, q, 1)
        assert np.array_equal(y1h[line], s1["out"])
        s2 = ox.line_stage(s1["out"], 32, p, q, 2)
        assert np.array_equal(y2h[line], s2["out"])
        for slot in range(32):
            for k, m in enumerate(mods):
                assert t1[line, slot, 0, k] == s1["re"][slot] % m
                assert t1[line, slot, 1, k] == s1["im"][slot] % m
                assert t2[line, slot, 0, k] == s2["re"][slot] % m
                assert t2[line, slot, 1, k] == s2["im"][slot] % m


@pytest.mark.parametrize("kind", ["max_corners", "max_tone"])
def test_extreme_magnitudes_bit_exact(gpu, kind):
    """Every column quantised to its largest magnitudes, so stage outputs
    reach the capacity extreme (|C| near 2^109 .. 2^111: coherent sums of K
    products of 53-bit data and 53-bit roots, Eq. capacity) where the lift
    must still pick the right multiple of M."""
    api = _api()
    shape = (32, 16, 64)
    a = 1.0 - 2.0 ** -53
    if kind == "max_corners":
        rng = np.random.default_rng(17)
        x = (a * rng.choice([-1.0, 1.0], size=shape) + 1j * a * rng.choice([-1.0, 1.0], size=shape))
    else:
        n = [np.arange(m) for m in shape]
        ph = (3 * n[0][:, None, None] / shape[0] + 5 * n[1][None, :, None] / shape[1]
              + 7 * n[2][None, None, :] / shape[2])
        x = a * np.exp(2j * np.pi * ph)
    x = np.ascontiguousarray(x.astype(np.complex128))
    plan = api.Plan(shape)
    y = _run(plan, x, gpu)
    ref = ox.fft3_exact(x, _pq(plan))
    assert np.count_nonzero(y != ref) == 0
    hi, lo = ox.fft3_dd(x)
    assert rel_l2(y, hi, lo) <= 1e-14


def test_default_modulus_sets(gpu):
    """Transform plans default to the sets of moduli at most 1024; the H0
    reduction, which needs reduction-friendly moduli, to the paper's set."""
    from oracle import constants as K
    api = _api()
    shape = (8, 8, 16)
    info = api.Plan(shape).info()
    assert info["moduli"] == [1024, 1023, 1021, 1019, 1013, 1009, 997, 991, 983, 977, 971, 967]
    assert info["S"] == 15 and info["S_frac"] == 6 and info["log2M"] > info["budget_bits"]
    assert info["substrate"] == 2   # FP16 under substrate auto
    info32 = api.Plan(shape, precision="fp32").info()
    assert info32["moduli"] == [1024, 1023, 1021, 1019, 1013, 1009] and info32["S"] == 8
    assert api.Plan(shape, reduction="h0").info()["moduli"] == list(K.MODULI_FP64)
    # the paper's set on substrate auto runs on INT8 (it exceeds the FP16 single-slot bound)
    assert api.Plan(shape, moduli=list(K.MODULI_FP64)).info()["substrate"] == 1


@pytest.mark.parametrize("substrate", ["fp16", "int8", "fp8"])
def test_permuted_modulus_set_gives_identical_bits(gpu, substrate):
    """The reconstructed integers do not depend on the modulus set (any
    admissible set has the capacity, Eq. capacity), so another set must
    reproduce the default plan's output bit for bit: on INT8 and FP8 the
    paper's set, permuted (three-digit FP8 moduli, so the general FP8 tile);
    on FP16, whose single-slot residue GEMM takes moduli up to 1024, the
    default set reversed."""
    api = _api()
    shape = (8, 24, 32)
    x = inputs.uniform(shape, 12)
    if substrate == "fp16":
        mods = [967, 971, 977, 983, 991, 997, 1009, 1013, 1019, 1021, 1023, 1024]
    else:
        mods = [2039, 2029, 2027, 1089, 1024, 487, 491, 511, 529, 625, 841, 961]
    y0 = _run(api.Plan(shape), x, gpu)
    y1 = _run(api.Plan(shape, substrate=substrate, moduli=mods), x, gpu)
    assert np.array_equal(y0, y1)


def test_inverse_and_adjoint(gpu):
    api = _api()
    shape = (16, 32, 8)
    x = inputs.uniform(shape, 9)
    plan = api.Plan(shape)
    pq = _pq(plan)
    xinv = _run(plan, x, gpu, "inverse")
    ref = ox.fft3_exact(x, pq, inverse=True, final_shift=-12)
    assert np.count_nonzero(xinv != ref) == 0
    xadj = _run(plan, x, gpu, "adjoint")
    # adjoint = conj o forward o conj, bit for bit (conjugated roots are exact)
    fwd_conj = np.conj(_run(plan, np.conj(x), gpu, "forward"))
    assert np.array_equal(xadj, fwd_conj)
    # round trip
    y = _run(plan, x, gpu, "forward")
    back = _run(plan, y, gpu, "inverse")
    assert rel_l2(back, x) <= 1e-14


@pytest.mark.parametrize("substrate", ["fp8", "fp16"])
def test_fp32_target_bit_exact(gpu, substrate):
    api = _api()
    shape = (16, 32, 32)
    x = inputs.uniform(shape, 4).astype(np.complex64)
    plan = api.Plan(shape, precision="fp32", substrate=substrate)
    y = _run(plan, x, gpu)
    ref = ox.fft3_exact(x, _pq(plan), precision=1)
    assert y.dtype == np.complex64
    assert np.count_nonzero(y != ref) == 0


def test_native_fp64_fft_accuracy(gpu):
    api = _api()
    for shape in [(32, 32, 32), (8, 12, 16), (4, 64, 24), (64, 16, 96)]:
        x = inputs.uniform(shape, 1)
        plan = api.Plan(shape)
        y = _run(plan, x, gpu, "native_forward")
        hi, lo = ox.fft3_dd(x)
        assert rel_l2(y, hi, lo) <= 1e-14, shape
        back = _run(plan, y, gpu, "native_inverse")
        assert rel_l2(back, x) <= 1e-14


def test_native_streaming_shape_sampled_lines(gpu):
    """1024 x 512 x 512 (4 GiB, which the native kernels read and write with
    nontemporal accesses): four output lines along axis 0 against the
    double-double DFT of their cost cones, and the inverse returns the input."""
    api = _api()
    shape = (1024, 512, 512)
    x = inputs.uniform(shape, 6)
    xt = torch.from_numpy(x).to(gpu)
    plan = api.Plan(shape)
    y = plan.native_forward(xt)
    torch.cuda.synchronize()
    samples = [(0, 3), (100, 3), (257, 3), (511, 3)]
    got = {s: y[:, s[0], s[1]].cpu().numpy() for s in samples}
    back = plan.native_inverse(y)
    err_back = (torch.linalg.vector_norm(back - xt) / torch.linalg.vector_norm(xt)).item()
    del y, back, xt
    torch.cuda.empty_cache()
    dd = ox.dd_cone_lines(x, samples)
    for s in samples:
        hi, lo = dd[s]
        assert rel_l2(got[s], hi, lo) <= 1e-14, s
    assert err_back <= 1e-14


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fp8_full_length_tile_bit_exact(gpu, precision):
    """Stages of contraction length 32 on the FP8 substrate (the full-length
    tile with three digits per residue before the split and two after it)
    against the oracle, with a ragged third axis for the general tile."""
    api = _api()
    shape = (3, 32, 1024)
    pq = ((1, 3), (1, 32), (32, 32))
    dt = np.complex128 if precision == "fp64" else np.complex64
    x = inputs.uniform(shape, 13).astype(dt)
    plan = api.Plan(shape, precision=precision, substrate="fp8", pq=pq)
    y = _run(plan, x, gpu)
    ref = ox.fft3_exact(x, _pq(plan), precision=0 if precision == "fp64" else 1)
    assert np.count_nonzero(y != ref) == 0


def test_fp8_general_tile_at_k32(gpu):
    """A modulus set outside the full-length tile's digit rule (the paper's
    set reordered: its moduli above 1052 take three FP8 digits) runs the
    general FP8 tile at K = 32: the same bits as the default plan."""
    api = _api()
    shape = (2, 8, 1024)
    x = inputs.uniform(shape, 14)
    mods = [2039, 2029, 2027, 1024, 1089, 961, 841, 625, 529, 511, 491, 487]
    y0 = _run(api.Plan(shape), x, gpu)
    y1 = _run(api.Plan(shape, substrate="fp8", moduli=mods), x, gpu)
    assert np.array_equal(y0, y1)
