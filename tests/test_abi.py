"""The C-ABI library loads on the CPU and exports every symbol of
include/crsolve.h; plan creation and argument validation are host-only."""
import os
import re

import pytest

from paper_1807_00370_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "crsolve.h")).read()
    return sorted(set(re.findall(r"\b(crsolve_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    lib = _lib.load()
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_plan_validation_host_only():
    p = _lib.Plan([65536], [32], [16])
    assert p.ws_bytes > 65536 * 32 * 32 * 16 * 3
    for bad in (([0], [4], [1]), ([4], [0], [1]), ([4], [4], [0])):
        with pytest.raises(_lib.CrsolveError) as e:
            _lib.Plan(*bad)
        assert e.value.code == _lib.EINVAL
    with pytest.raises(_lib.CrsolveError) as e:
        _lib.Plan([8], [257], [1])
    assert e.value.code == _lib.EUNSUPPORTED
    with pytest.raises(_lib.CrsolveError) as e:
        _lib.Plan([8], [4], [1], dtype=_lib.C64, schedule=_lib.SCHED_PCR)
    assert e.value.code == _lib.EUNSUPPORTED
    assert _lib.error_string(_lib.EWORKSPACE) == "workspace too small"


def test_null_pointers_rejected_without_device_work():
    import ctypes
    p = _lib.Plan([8], [4], [1])
    lib = _lib.load()
    assert lib.crsolve_factor(p._h, None, None, None, p.ws_bytes, None, None) == _lib.EINVAL
    assert lib.crsolve_solve(p._h, None, p.ws_bytes, None, None, None, None, None, None) == \
        _lib.EINVAL
    fake = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced: size check fails first
    assert lib.crsolve_factor(p._h, fake, fake, fake, p.ws_bytes - 1, None, None) == \
        _lib.EWORKSPACE
    assert lib.crsolve_factor(None, fake, fake, fake, p.ws_bytes, None, None) == _lib.EINVAL


def test_solve_before_factor_is_a_state_error():
    """crsolve_solve / crsolve_backward on a workspace the plan never factored
    return CRSOLVE_ESTATE before any device work (the pointers are aligned
    and never dereferenced)."""
    import ctypes
    lib = _lib.load()
    fake = ctypes.c_void_p(1 << 20)
    for prec in (_lib.PREC_NATIVE, _lib.PREC_FP32_REFINE):
        p = _lib.Plan([16], [8], [2], precision=prec)
        assert lib.crsolve_solve(p._h, fake, p.ws_bytes, fake, fake, fake, fake, None,
                                 None) == _lib.ESTATE
    p = _lib.Plan([16], [8], [2])
    assert lib.crsolve_backward(p._h, fake, p.ws_bytes, fake, fake, fake, fake, fake,
                                None) == _lib.ESTATE
    # the size check still comes first
    assert lib.crsolve_solve(p._h, fake, p.ws_bytes - 1, None, None, fake, fake, None,
                             None) == _lib.EWORKSPACE


def test_block_size_limits_match_header():
    """1 <= m <= 256; N <= 2^24 when m > 64 (host-only plan creation)."""
    _lib.Plan([4], [256], [1])
    _lib.Plan([1 << 24], [65], [1])
    with pytest.raises(_lib.CrsolveError) as e:
        _lib.Plan([(1 << 24) + 1], [65], [1])
    assert e.value.code == _lib.EUNSUPPORTED
    hdr = open(os.path.join(ROOT, "include", "crsolve.h")).read()
    assert "1 <= m <= 256" in hdr and "m <= 64" not in hdr


def test_refine_fallback_region_is_one_system():
    """The mixed form reserves an FP64 fallback region for its largest
    system, not a second plan over the whole batch."""
    shapes = [(2048, 32, 4)] + [(256, 8, 1)] * 40
    Ns, ms, ks = zip(*shapes)
    mixed = _lib.Plan(Ns, ms, ks, precision=_lib.PREC_FP32_REFINE).ws_bytes
    big64 = _lib.Plan([2048], [32], [4]).ws_bytes
    whole64 = _lib.Plan(Ns, ms, ks).ws_bytes
    assert mixed < whole64 + big64
    assert mixed >= big64


def test_pcr_tail_validation():
    """The Algorithm 1 tail of the one-sided schedule: native plans only."""
    p = _lib.Plan([1000], [16], [4], pcr_tail_blocks=256)
    q = _lib.Plan([1000], [16], [4])
    assert p.ws_bytes > 0 and q.ws_bytes > 0
    with pytest.raises(_lib.CrsolveError) as e:
        _lib.Plan([1000], [16], [4], precision=_lib.PREC_FP32_REFINE, pcr_tail_blocks=64)
    assert e.value.code == _lib.EUNSUPPORTED
    with pytest.raises(_lib.CrsolveError) as e:
        _lib.Plan([1000], [16], [4], pcr_tail_blocks=-1)
    assert e.value.code == _lib.EINVAL


def test_noalloc_limits_checked_before_device_work():
    """crsolve_factor_solve_noalloc rejects a plan whose workspace exceeds the
    256 MiB scratch array, and non-native plans, before touching a GPU."""
    import ctypes
    lib = _lib.load()
    fake = ctypes.c_void_p(1 << 20)
    big = _lib.Plan([65536], [32], [16])
    assert big.ws_bytes > (256 << 20)
    assert lib.crsolve_factor_solve_noalloc(big._h, fake, fake, fake, fake, None, None) == \
        _lib.EWORKSPACE
    mixed = _lib.Plan([64], [4], [1], precision=_lib.PREC_FP32_REFINE)
    assert lib.crsolve_factor_solve_noalloc(mixed._h, fake, fake, fake, fake, None, None) == \
        _lib.EUNSUPPORTED
    small = _lib.Plan([2048], [16], [4])
    assert small.ws_bytes <= (256 << 20)
    hdr = open(os.path.join(ROOT, "include", "crsolve.h")).read()
    assert "256 MiB" in hdr


def test_pcr_tail_default_by_block_size():
    """The binding's default switch to Algorithm 1 follows the plan's largest
    block: 64 blocks up to m = 32, 16 up to m = 64, 8 above."""
    from paper_1807_00370_amd.solver import pcr_tail_default
    assert pcr_tail_default([1]) == 64 and pcr_tail_default([32]) == 64
    assert pcr_tail_default([33]) == 16 and pcr_tail_default([64]) == 16
    assert pcr_tail_default([65]) == 8 and pcr_tail_default([256]) == 8
    assert pcr_tail_default([8, 16, 100, 32]) == 8
    assert pcr_tail_default([8, 40]) == 16
