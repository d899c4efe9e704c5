"""Host-side checks of the C-ABI library: it loads, exports every entry point
declared in include/hd.h, and rejects invalid parameters before touching a
device (no compute calls are made here)."""
import ctypes as C
import os
import re

import pytest

from paper_1508_02892_amd import hd, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    if not os.path.exists(hd.LIB_PATH):
        from paper_1508_02892_amd import build
        build.build()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hd_[a-z_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert declared_symbols() == sorted(hd.SYMBOLS)


def test_library_exports_every_declared_symbol():
    _ensure_built()
    L = C.CDLL(hd.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(L, s), s


def test_abi_version():
    _ensure_built()
    assert hd.lib().hd_abi_version() == hd.HD_ABI_VERSION


def test_required_bytes_scales_with_particles():
    _ensure_built()
    small = hd.required_bytes(W.c0())
    big = hd.required_bytes(W.c1())
    assert 0 < small < big
    # FP32 particle state: 2 buffers x 24 B plus 20 B staging per slot at least
    assert big > W.c1()["capacity"] * 68


@pytest.mark.parametrize("bad", [dict(n_cells=1), dict(precision=7), dict(ion_model=5),
                                 dict(dt_s=0.0), dict(load_lo=0.9, load_hi=0.1),
                                 dict(n_macro=100, capacity=50), dict(sort_every=0)])
def test_invalid_params_rejected_without_device(bad):
    _ensure_built()
    p = W.c0(**bad)
    assert hd.required_bytes(p) == 0
    with pytest.raises(hd.HdError) as e:
        hd.Discharge(p)
    assert e.value.code == -1


def test_negative_cross_section_rejected():
    _ensure_built()
    p = W.c0()
    p["channels"] = [dict(p["channels"][0])]
    p["channels"][0]["sigma_m2"] = -p["channels"][0]["sigma_m2"]
    with pytest.raises(hd.HdError):
        hd.Discharge(p)
