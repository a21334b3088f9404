"""CPU checks of the C ABI: the built library loads and exports every entry
point that include/lensed.h declares; host-only calls behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lensed.h")
LIB = os.path.join(ROOT, "paper_1505_07674_amd", "liblensed_hip.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lensed_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblensed_hip.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["lensed_create", "lensed_destroy", "lensed_render", "lensed_loglike",
                     "lensed_loglike_batch", "lensed_loglike_grad", "lensed_param_count",
                     "lensed_status_string", "lensed_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in lensed.h but not exported"


def test_host_only_calls(lib):
    lib.lensed_param_count.restype = ctypes.c_int
    assert lib.lensed_param_count() == 17
    lib.lensed_status_string.restype = ctypes.c_char_p
    lib.lensed_status_string.argtypes = [ctypes.c_int]
    assert lib.lensed_status_string(0) == b"ok"
    assert lib.lensed_status_string(1) == b"invalid argument"
    lib.lensed_create.restype = ctypes.c_int
    lib.lensed_create.argtypes = [ctypes.c_void_p, ctypes.c_int]
    assert lib.lensed_create(None, 0) == 1          # NULL out-pointer is rejected before any HIP call


def test_binding_mirrors_the_struct_layout():
    from paper_1505_07674_amd.binding import LensedSystemC
    # int32 H, W; float pixscale, cx, cy; int32 nsub, ph, pw; three pointers; int32 rule, amplitude;
    # float zero_point; int32 source_position
    assert LensedSystemC.psf.offset == 32
    assert LensedSystemC.rule.offset == 8 * 4 + 3 * 8
    assert LensedSystemC.amplitude.offset == 8 * 4 + 3 * 8 + 4
    assert LensedSystemC.zero_point.offset == 8 * 4 + 3 * 8 + 8
    assert LensedSystemC.source_position.offset == 8 * 4 + 3 * 8 + 12
    assert ctypes.sizeof(LensedSystemC) == 8 * 4 + 3 * 8 + 16
