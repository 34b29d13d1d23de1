"""The C-ABI library on the CPU: exports, plan-time mathematics, host-side errors.

No compute call runs here (there is no GPU); plan creation fails on the host
checks (capacity budget, factorisation) before it touches a device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import constants as K
from oracle import roots

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2606_23698_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol():
    L = _lib()
    L.lib()
    header = open(os.path.join(ROOT, "include", "obfft.h")).read()
    decl = set(re.findall(r"^\s*(?:obfft_status_t|size_t|void|const char\*)\s+(\w+)\s*\(", header, re.M))
    assert len(decl) >= 25
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name
    assert decl <= set(L.EXPORTED) | {"obfft_options_default"}


@pytest.mark.parametrize("N", [4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 512, 1024])
def test_plan_roots_equal_oracle_roots(N):
    from paper_2606_23698_amd import api
    for bits in (52, 23):
        assert np.array_equal(api.quantised_roots(N, bits), roots.quantised_roots(N, bits))


@pytest.mark.parametrize("precision,mods", [("fp64", K.MODULI_FP64), ("fp32", K.MODULI_FP32)])
def test_plan_crt_constants_equal_oracle(precision, mods):
    from paper_2606_23698_amd import api
    c = api.crt_constants(precision)
    assert c["moduli"] == list(mods)
    assert c["M"] == K.modulus_product(mods)
    assert c["u"] == K.idempotents(mods)
    assert c["w"] == K.lift_weights(mods)
    assert c["S"] == K.n_slices(mods) and c["S_frac"] == K.n_frac_slices(mods)


# The transform plans' default modulus sets (every modulus at most 1024).
STAGE_FP64 = [1024, 1023, 1021, 1019, 1013, 1009, 997, 991, 983, 977, 971, 967]
STAGE_FP32 = [1024, 1023, 1021, 1019, 1013, 1009]


@pytest.mark.parametrize("mods,k", [(STAGE_FP64, 53), (STAGE_FP32, 24)])
def test_default_stage_sets_are_admissible(mods, k):
    """The default sets of the transform plans, checked by the oracle's own
    definitions: pairwise coprime, the capacity of Eq. capacity at the
    longest contraction (K = 32), every modulus inside the FP16 single-slot
    bound 64 h (h + e) <= 2^24, and the epilogue shape of the paper's sets
    (15 / 8 byte slices of u_k, 6 of w_k), which the kernels compile in."""
    assert K.pairwise_coprime(mods)
    assert K.capacity_ok(mods, 32, k)
    for m in mods:
        h = m // 2
        e = 0 if m & (m - 1) == 0 else 2
        assert 64 * h * (h + e) <= 2 ** 24, m
    paper = K.MODULI_FP64 if k == 53 else K.MODULI_FP32
    assert K.n_slices(mods) == K.n_slices(paper)
    assert K.n_frac_slices(mods) == K.n_frac_slices(paper) == 6


def test_capacity_budget_rejects_rev33():
    from paper_2606_23698_amd import api
    from paper_2606_23698_amd._lib import ObfftError
    with pytest.raises(ObfftError) as e:
        api.Plan((32, 32, 32), moduli=K.MODULI_REV33)
    assert e.value.status == 3   # OBFFT_CAPACITY_EXCEEDED


def test_unsupported_and_invalid_sizes():
    from paper_2606_23698_amd import api
    from paper_2606_23698_amd._lib import ObfftError
    for shape, status in [((37, 32, 32), 2), ((1030, 32, 32), 2), ((32, 32, 74), 2), ((32, 0, 32), 1)]:
        with pytest.raises(ObfftError) as e:
            api.Plan(shape)
        assert e.value.status == status, shape
    with pytest.raises(ObfftError) as e:
        api.Plan((32, 32, 32), pq=((4, 8), (4, 8), (4, 4)))   # p*q != n
    assert e.value.status == 1
    with pytest.raises(ObfftError) as e:
        api.Plan((32, 32, 32), moduli=[2039, 2039, 1024])      # not coprime
    assert e.value.status == 1
    # 4096 has no split p x q with both factors at most 32 (the longest contraction)
    with pytest.raises(ObfftError) as e:
        api.Plan((4096, 4096, 4096))
    assert e.value.status == 2


def test_h0_reduction_option_is_validated():
    """The fold-and-add reduction is an FP16-substrate, FP64-target ablation of
    single transforms; anything else is rejected before any device work."""
    import ctypes
    from paper_2606_23698_amd import api, _lib
    from paper_2606_23698_amd._lib import ObfftError
    for kw in ({"substrate": "int8"}, {"substrate": "fp8"}, {"precision": "fp32"}):
        with pytest.raises(ObfftError) as e:
            api.Plan((32, 32, 32), reduction="h0", **kw)
        assert e.value.status == 1, kw
    opt, _ = api.options()
    opt.reduction = 2
    h = ctypes.c_void_p()
    assert _lib.lib().obfft_plan_create(ctypes.byref(h), 32, 32, 32, ctypes.byref(opt)) == 1
    opt.reduction = 1
    shapes = (ctypes.c_int64 * 3)(32, 32, 32)
    assert _lib.lib().obfft_batch_plan_create(ctypes.byref(h), 1, shapes, ctypes.byref(opt)) == 1


def test_group_block_option_is_validated():
    from paper_2606_23698_amd import api
    from paper_2606_23698_amd._lib import ObfftError
    for gb in (-1, 3, 12, 64):
        with pytest.raises(ObfftError) as e:
            api.Plan((32, 32, 32), group_block=gb)
        assert e.value.status == 1, gb


def test_fp16_substrate_rejects_a_modulus_above_the_single_slot_bound():
    """With the reciprocal reduction FP16 takes one slot per index for every
    modulus of a set, which is exact only when 64 h (h + e) <= 2^24 (h =
    floor(m/2); e = 0 for a power of two, whose residues are exact, else 2):
    1023 and 1024 pass, 1089 does not, nor do the paper's moduli above 2000."""
    from paper_2606_23698_amd import api
    from paper_2606_23698_amd._lib import ObfftError
    h = 1089 // 2
    assert 64 * h * (h + 2) > 2 ** 24
    h = 1023 // 2
    assert 64 * h * (h + 2) <= 2 ** 24
    assert 64 * 512 * 512 == 2 ** 24          # m = 1024: exactly at the bound
    for mods in ([1024, 1089, 1021, 1019, 1013, 1009, 997, 991, 983, 977, 971, 967], list(K.MODULI_FP64)):
        with pytest.raises(ObfftError) as e:
            api.Plan((32, 32, 32), substrate="fp16", moduli=mods)
        assert e.value.status == 2, mods   # OBFFT_UNSUPPORTED_SIZE


def test_status_strings_and_taps_layout():
    from paper_2606_23698_amd import api
    from paper_2606_23698_amd._lib import status_string
    assert status_string(0) == "OBFFT_SUCCESS"
    assert status_string(3) == "OBFFT_CAPACITY_EXCEEDED"
    lay = api.taps_layout()
    assert lay["stride"] >= lay["R"] + lay["n_R"] + 1
    assert lay["Z"] >= lay["P"] + 15 and lay["E"] >= lay["Z"] + 6


def test_oracle_cone_matches_full_lines():
    from oracle import exact as ox
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, (40, 96)) + 1j * rng.uniform(-1, 1, (40, 96))
    full = ox.lines(x, 96, 8, 12)
    for k in (0, 5, 95, 50):
        assert np.array_equal(ox.lines_at(x, 96, 8, 12, k), full[:, k])
    y = ox.fft3_exact(x.reshape(1, 40, 96)[:, :32, :], ((1, 1), (4, 8), (8, 12)))
    assert y.shape == (1, 32, 96)


def test_axis_order_option_is_validated():
    """The axis order must be a permutation of (0, 1, 2) (all zero = default)."""
    from paper_2606_23698_amd import api
    from paper_2606_23698_amd._lib import ObfftError
    for order in ((0, 0, 1), (3, 1, 0), (-1, 1, 2), (1, 1, 1)):
        with pytest.raises(ObfftError) as e:
            api.Plan((32, 32, 32), axis_order=order)
        assert e.value.status == 1, order
