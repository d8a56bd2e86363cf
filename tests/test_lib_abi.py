"""CPU checks of the boundary: the C-ABI library loads and exports every function that
include/conegauss.h declares, and the Python binding declares the same set."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "conegauss.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("cg_render_forward", "cg_render_backward", "cg_camera_unproject"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2609_13397_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    from paper_2609_13397_amd import serving
    assert set(declared_functions()) == set(_lib.SIGNATURES) | set(serving.SERVER_SIGNATURES)
    assert L.cg_version() == 1


def test_default_opts_and_errors_without_gpu():
    """Host-side validation runs before any device work, so it is testable here."""
    import ctypes as C

    from paper_2609_13397_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    L = _lib.lib()
    o = _lib.CgOpts()
    L.cg_default_opts(_lib.byref(o))
    assert o.filter_mode == 1 and abs(o.alpha_min - 1 / 255) < 1e-9 and abs(o.alpha_max - 0.99) < 1e-7
    assert abs(o.T_min - 1e-4) < 1e-9 and abs(o.t_near - 0.2) < 1e-7 and o.footprint_scale == 1.0
    assert o.count_pairs == 0 and o.order_mode == 0
    # an invalid camera is rejected with CG_ERR_INVALID_ARG and a message
    cam = _lib.CgCamera()
    cam.model = 7
    cam.full_w = cam.full_h = 4
    st = L.cg_camera_unproject(_lib.byref(cam), 0, None, None, None, None)
    assert st == -1
    assert b"model" in L.cg_last_error()
    # a non-monotone Kannala-Brandt polynomial is rejected
    cam.model = 1
    cam.fx = cam.fy = 10.0
    cam.cx = cam.cy = 2.0
    cam.theta_max = 1.6
    cam.k[:] = [-0.3, 0.0, 0.0, 0.0]
    cam.R_c2w[:] = [1, 0, 0, 0, 1, 0, 0, 0, 1]
    cam.crop_w = cam.crop_h = 4
    st = L.cg_camera_unproject(_lib.byref(cam), 0, None, None, None, None)
    assert st == -1 and b"increasing" in L.cg_last_error()
    # a crop outside the image
    cam.k[:] = [0, 0, 0, 0]
    cam.crop_x0 = 2
    st = L.cg_camera_unproject(_lib.byref(cam), 0, None, None, None, None)
    assert st == -1 and b"crop" in L.cg_last_error()
    # bad options are rejected before touching the device
    g = _lib.CgGaussians()
    g.n = 0
    g.color_mode = 0
    cam.crop_x0 = 0
    o.alpha_min = 0.0
    st = L.cg_render_forward(_lib.byref(g), _lib.byref(cam), 1, _lib.byref(o), None, None, None, None, None)
    assert st == -1 and b"alpha_min" in L.cg_last_error()


def test_order_mode_validation_without_gpu():
    """order_mode is 0 or 1, and the per-ray order (1) is forward-only: asking it for a
    backward state is refused before any device work."""
    import ctypes as C

    from paper_2609_13397_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    L = _lib.lib()
    o = _lib.CgOpts()
    L.cg_default_opts(_lib.byref(o))
    g = _lib.CgGaussians()
    g.n = 0
    g.color_mode = 0
    cam = _lib.CgCamera()
    o.order_mode = 2
    st = L.cg_render_forward(_lib.byref(g), _lib.byref(cam), 1, _lib.byref(o), None, None, None, None, None)
    assert st == -1 and b"order_mode" in L.cg_last_error()
    o.order_mode = 1
    state = C.c_void_p(0)
    st = L.cg_render_forward(_lib.byref(g), _lib.byref(cam), 1, _lib.byref(o), None, None, _lib.byref(state),
                             None, None)
    assert st == -2 and b"forward-only" in L.cg_last_error()
