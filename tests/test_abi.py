"""CPU checks of the C ABI: the built library loads and exports every entry
point that include/lensed.h declares; host-only calls behave as documented."""
import ctypes
import os
import re

import numpy as np
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


def test_model_struct_layout_and_host_validation():
    """lensed_model: 4 + 8 int32, n_planes, 8 sie_plane, reserved, then 8 x 8 float64
    ratios. lensed_model_nparams validates the model's shape on the host."""
    from paper_1505_07674_amd.binding import LensedModelC, Model
    assert LensedModelC.n_planes.offset == 48
    assert LensedModelC.sie_plane.offset == 52
    assert LensedModelC.beta.offset == 88
    assert ctypes.sizeof(LensedModelC) == 600
    assert Model(2, ["foreground", "lensed"]).n_params == 5 * 2 + 2 + 7 * 2
    three = np.zeros((3, 3))
    three[0, 1], three[0, 2], three[1, 2] = 0.5, 0.7, 0.3
    m = Model(3, ["foreground", 1, 2, "lensed"], sie_planes=[0, 1, 2], beta=three)
    assert m.n_params == 5 * 3 + 2 + 7 * 4 and m.c_struct.plane[3] == 3
    bad = [dict(sie_planes=[0, 3, 1]),                          # SIE beyond the lens planes
           dict(sie_planes=[0, 1, 2], planes=["foreground", 4]),  # light beyond the source plane
           dict(sie_planes=[0, 1, 2], beta=three * 2)]          # a ratio above 1
    for kw in bad:
        args = dict(planes=["lensed"], beta=three)
        args.update(kw)
        with pytest.raises(ValueError):
            Model(3, args.pop("planes"), **args)
