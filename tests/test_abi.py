"""Host-side checks of the C ABI (no GPU): the built library loads and exports
every function that include/upslam.h declares, and the Python structs have
the header's sizes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "upslam.h")
SO = os.path.join(ROOT, "paper_2101_00585_amd",
                  "libupslam_san.so" if os.environ.get("UPS_SANITIZE") == "1" else "libupslam.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ups_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(SO):
        from paper_2101_00585_amd import build
        build.build(sanitize=os.environ.get("UPS_SANITIZE") == "1")
    return ctypes.CDLL(SO)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "ups_register_scan" in names and "ups_fuse_scan" in names and "ups_panorama_normals" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_sizes_match_header():
    import paper_2101_00585_amd as ups
    # ups_pose: 12 doubles; ups_geom: 2 ints + 4 doubles; result layout fixed by the header
    assert ctypes.sizeof(ups.ups_pose) == 96
    assert ctypes.sizeof(ups.ups_geom) == 40
    assert ctypes.sizeof(ups.ups_icp_params) == 4 + 16 + 16 + 4 + 8 + 4 + 4 + 4 + 4  # irls_delta + padding
    assert ups.ups_icp_params.irls_delta.offset == 56
    assert ups.RESULT_BYTES == 96 + 24 + 16 + 8 + 16 + 21 * 8 + 6 * 8 + 8
    assert ups.NEQ_BYTES == 21 * 8 + 6 * 8 + 8 + 16
    assert ctypes.sizeof(ups.ups_grid_params) == 6 * 4
    assert ctypes.sizeof(ups.ups_range_image) == 8 + 3 * 4 + 2 * 4 + 4  # pointer, 3 ints, 2 floats, padding
    assert ctypes.sizeof(ups.ups_consistency_params) == 3 * 4
    assert (ups.LOOP_NONE, ups.LOOP_WEAK, ups.LOOP_STRONG) == (0, 1, 2)


def test_last_error_without_gpu(lib):
    lib.ups_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.ups_last_error(), bytes)


def test_invalid_arguments_rejected_on_host(lib):
    """Null context / pointers are rejected before any device work."""
    import paper_2101_00585_amd as ups
    L = ups.load()
    g = ups.ups_geom(64, 512, 0.3, 0.01, 0.0, 50.0)
    p = ups.IcpParams().c()
    rc = L.ups_register_scan(None, ctypes.byref(g), None, ctypes.byref(g), None, None, ctypes.byref(p), None, None)
    assert rc == -1
    np_ = ups.NormalParams().c()
    rc = L.ups_panorama_normals(None, ctypes.byref(g), None, None, ctypes.byref(np_), None)
    assert rc == -1
    out = ctypes.c_void_p()
    rc = L.ups_context_create(ctypes.byref(out), 0, 10, 0, 0)
    assert rc == -1 and not out.value
    cp = ups.ConsistencyParams().c()
    rc = L.ups_keyframe_consistency(None, ctypes.byref(g), None, None, ctypes.byref(g), None, None, None,
                                    ctypes.byref(cp), None, None, None, None)
    assert rc == -1
    rc = L.ups_classify_loop_closures(None, 4, None, 0.5, None, None, None)
    assert rc == -1
    assert L.ups_batch_set_pyramid_mode(None, 1) == -1


def test_conv_arguments_rejected_on_host(lib):
    """Convolution shapes and pointer alignment are checked before any device
    work: cin above 65536, and a weight pointer that is not 8-byte aligned
    (the forward pass loads four weights at a time)."""
    import paper_2101_00585_amd as ups
    L = ups.load()
    L.ups_last_error.restype = ctypes.c_char_p
    P = ctypes.c_void_p
    args = (P(0x1000), P(0x2000), P(0x3000), P(0x4000), None)
    fwd = L.ups_conv3x3_forward
    fwd.argtypes = [ctypes.c_int32] * 6 + [P] * 5
    assert fwd(1, 4, 8, 65537, 4, 1, *args) == -1
    assert b"cin" in L.ups_last_error()
    assert fwd(1, 4, 8, 4, 4, 1, P(0x1000), P(0x2002), P(0x3000), P(0x4000), None) == -1
    assert b"w is not 8-byte aligned" in L.ups_last_error()
    assert fwd(0, 4, 8, 4, 4, 1, *args) == 0  # empty batch: nothing to do


def test_noalloc_limits_rejected_on_host(lib):
    """The entry point without a context rejects panoramas above its static
    scratch (262144 pixels) and invalid parameters before any device work."""
    import paper_2101_00585_amd as ups
    L = ups.load()
    L.ups_last_error.restype = ctypes.c_char_p
    P = ctypes.c_void_p
    small = ups.ups_geom(128, 2048, 0.39, 0.0062, 0.0, 50.0)
    big = ups.ups_geom(256, 2048, 0.39, 0.0031, 0.0, 50.0)
    p = ups.IcpParams(levels=3, iters=(10, 10, 10)).c()
    bufs = (P(0x10000), P(0x20000), P(0x30000), P(0x40000))
    rc = L.ups_register_scan_noalloc(ctypes.byref(big), bufs[0], ctypes.byref(small), bufs[1], bufs[2],
                                     ctypes.byref(p), bufs[3], None)
    assert rc == -4 and b"262144 pixels" in L.ups_last_error()
    rc = L.ups_register_scan_noalloc(ctypes.byref(small), bufs[0], ctypes.byref(big), bufs[1], bufs[2],
                                     ctypes.byref(p), bufs[3], None)
    assert rc == -4
    bad = ups.IcpParams(levels=5).c()
    rc = L.ups_register_scan_noalloc(ctypes.byref(small), bufs[0], ctypes.byref(small), bufs[1], bufs[2],
                                     ctypes.byref(bad), bufs[3], None)
    assert rc == -1
    rc = L.ups_register_scan_noalloc(ctypes.byref(small), P(0x10004), ctypes.byref(small), bufs[1], bufs[2],
                                     ctypes.byref(p), bufs[3], None)
    assert rc == -1 and b"aligned" in L.ups_last_error()
