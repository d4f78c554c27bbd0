"""CPU-side checks of the C ABI library: it loads and exports every entry
point that include/ecc_mi.h declares (no compute call is made without a GPU)."""

import ctypes
import os
import re

import pytest

from tests.common import ROOT

HEADER = os.path.join(ROOT, "include", "ecc_mi.h")
LIB = os.path.join(ROOT, "paper_2501_03245_amd", "libecc_mi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    # a name followed by "(" declares a function; "ecc_status (*f)(...)" is a
    # function-pointer member, not a declaration of ecc_status
    names = re.findall(r"\b(ecc_[a-z0-9_]+)\s*\((?!\s*\*)", text)
    return sorted(set(names))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("ecc_msm", "ecc_ctx_create", "ecc_ctx_destroy", "ecc_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_every_declared_symbol():
    import paper_2501_03245_amd as eccmi
    eccmi.library()
    assert sorted(eccmi.EXPORTED) == declared_functions()


def test_bucket_geometry_matches_digit_definition():
    """The binding's window count is the smallest W whose signed digits cover
    every scalar below 2^bits."""
    from oracle import ref
    bits_by_curve = {1: 254, 2: 255}
    for curve, bits in bits_by_curve.items():
        for c in (2, 5, 13, 16, 20):
            W = (bits + 1 + c - 1) // c
            ref.signed_digits((1 << bits) - 1, c, W)
            ref.signed_digits(int("10" * (bits // 2), 2), c, W)
            if W > 1 and c * (W - 1) >= bits + 1:
                pytest.fail("more windows than needed")
