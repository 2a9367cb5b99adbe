"""C-ABI contract checks that need no GPU.

* libsparsect.so loads and exports every function include/sparsect.h declares;
* the binding's signature table covers exactly those functions;
* argument validation happens before any HIP call and returns the documented
  status with a message.
"""
import ctypes
import os
import re

import pytest

import paper_1705_07497_amd as sct

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sparsect.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 12, names
    L = sct.lib()
    for name in names:
        assert hasattr(L, name), name
    assert sorted(sct.SIGNATURES) == names


def test_header_constants_match_binding():
    text = open(HEADER).read()
    consts = dict(re.findall(r"#define\s+(\w+)\s+(-?\d+)", text))
    assert int(consts["SPARSECT_F32"]) == sct.F32 and int(consts["SPARSECT_F64"]) == sct.F64
    assert int(consts["RADON_WS_SB"]) == sct.WS_SB and int(consts["RADON_SB_RESUME"]) == sct.SB_RESUME
    # struct sizes the binding assumes
    assert ctypes.sizeof(sct.CgInfo) == 24
    assert ctypes.sizeof(sct.SbParams) == 40
    assert ctypes.sizeof(sct.SbInfo) == 32
    assert ctypes.sizeof(sct._Info) == 104
    assert ctypes.sizeof(sct.PdParams) == 40
    assert int(consts["RADON_WS_PD"]) == sct.WS_PD
    assert int(consts["RADON_WS_TUNE"]) == sct.WS_TUNE
    assert int(consts["RADON_WS_ADJ"]) == sct.WS_ADJ
    assert int(consts["RADON_LAYOUT_IMAGE"]) == sct.LAYOUT_IMAGE
    assert int(consts["RADON_LAYOUT_PIXEL"]) == sct.LAYOUT_PIXEL
    hexes = dict(re.findall(r"#define\s+(\w+)\s+0x([0-9a-fA-F]+)", text))
    assert int(hexes["RADON_WS_PIXEL_LAYOUT"], 16) == sct.WS_PIXEL_LAYOUT
    assert ctypes.sizeof(sct._Geom) == 40
    assert ctypes.sizeof(sct.RadonSizes) == 72
    assert ctypes.sizeof(sct.RadonBuffers) == 80
    assert ctypes.sizeof(sct.Tuning) == 32


def _build(n, na, nb, dtype=0, measured=None, bundle=0, angles=0, compact=0, symmetric=0):
    L = sct.lib()
    m = None
    if measured is not None:
        arr = (ctypes.c_uint8 * len(measured))(*measured)
        m = ctypes.cast(arr, ctypes.POINTER(ctypes.c_uint8))
    g = sct._Geom(n, na, nb, dtype, m, bundle, angles, compact, symmetric)
    h = ctypes.c_void_p()
    rc = L.build_radon_csr(ctypes.byref(g), None, ctypes.byref(h))
    return rc, L.radon_last_error().decode()


@pytest.mark.parametrize("args,code,frag", [
    ((0, 4, 5), -1, "n must be"),
    ((40000, 4, 5), -1, "n must be"),
    ((8, 0, 5), -1, "n_angles"),
    ((8, 4, 0), -1, "n_bins"),
    ((8, 4, 70000), -1, "n_bins"),
    ((8, 4, 13, 7), -1, "dtype"),
])
def test_build_rejects_bad_geometry(args, code, frag):
    rc, msg = _build(*args)
    assert rc == code and frag in msg


@pytest.mark.parametrize("bundle,angles,frag", [
    (48, 0, "fwd_bundle"),
    (16, 2, "fwd_angles"),     # 8 bins per angle
    (32, 4, "fwd_angles"),
    (64, 3, "fwd_angles"),
    (64, -1, "fwd_angles"),
])
def test_build_rejects_bad_bundle_layout(bundle, angles, frag):
    rc, msg = _build(8, 4, 13, 0, None, bundle, angles)
    assert rc == -1 and frag in msg


def test_build_rejects_bad_compact_and_symmetric_flags():
    rc, msg = _build(8, 4, 13, 0, None, 0, 0, 2)
    assert rc == -1 and "fwd_compact" in msg
    rc, msg = _build(8, 4, 13, 0, None, 0, 0, 0, 5)
    assert rc == -1 and "fwd_symmetric" in msg
    rc, msg = _build(1, 4, 13, 0, None, 0, 0, 0, 1)
    assert rc == -1 and "n >= 2" in msg


@pytest.mark.parametrize("na,measured,frag", [
    (7, None, "even number"),               # pi/2 - theta is not an angle
    (8, [1, 0, 1, 1, 1, 1, 1, 1], "not covered"),   # pi/8 unmeasured: 3, 5 and 7 pi/8 have no stored image
])
def test_build_rejects_asymmetric_angle_sets(na, measured, frag):
    """The symmetry map is host logic, checked before any device work."""
    rc, msg = _build(16, na, 25, 0, measured, 0, 0, 0, 1)
    assert rc == -6 and frag in msg, msg


def test_build_rejects_no_measured_angle():
    rc, msg = _build(8, 4, 13, 0, [0, 0, 0, 0])
    assert rc == -1 and "no measured angle" in msg


def test_build_rejects_overflowing_geometry():
    # 32767^2 pixels x 40000 measured angles overflows the adjoint layout
    rc, msg = _build(32767, 40000, 46341)
    assert rc == -2, msg


def test_null_handles_are_rejected():
    L = sct.lib()
    assert L.build_radon_csr(None, None, None) == -1
    h = ctypes.c_void_p()
    assert L.build_radon_csr(None, None, ctypes.byref(h)) == -1
    assert L.radon_fwd(None, None, None, 1, 0, None, 0, None) == -1
    assert "NULL" in L.radon_last_error().decode()
    assert L.radon_adj(None, None, None, 1, 0, None, 0, None) == -1
    assert L.normal_apply(None, 1.0, 1.0, 0.0, None, None, None, 1, 0, None, 0, None) == -1
    assert L.cg_solve(None, 1.0, 1.0, 0.0, None, None, 0, 1, 0, 5, 0.0, None, 0, None, None) == -1
    assert L.split_bregman_tv(None, None, None, None, 1, 0, None, 0, None, None) == -1
    assert L.radon_workspace_bytes(None, 0, 1) == -1
    info = sct._Info()
    assert L.radon_op_info(None, ctypes.byref(info)) == -1
    assert L.radon_export_csr(None, None, None, None) == -1
    L.radon_op_destroy(None)   # no-op


def test_binding_refuses_without_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(sct.SparsectError):
        sct.RadonOp(8, 4, 13)


def test_group_and_graph_entry_points_validate_without_gpu():
    L = sct.lib()
    h = ctypes.c_void_p()
    assert L.radon_multi_create(None, 1, None, None, None, ctypes.byref(h)) == -1
    assert "ops is NULL" in L.radon_last_error().decode()
    arr = (ctypes.c_void_p * 1)(None)
    assert L.radon_multi_create(arr, 0, None, None, None, ctypes.byref(h)) == -1
    assert "count" in L.radon_last_error().decode()
    assert L.radon_multi_create(arr, 1, None, None, None, ctypes.byref(h)) == -1
    assert L.radon_multi_create(arr, 1, None, None, None, None) == -1
    assert L.radon_multi_info(None, None, None, None, None, None, None) == -1
    assert L.radon_multi_apply(None, 0, None, None, None, 0, None) == -1
    assert L.radon_multi_cg(None, None, None, 1, 0.0, None, 0, None, None) == -1
    assert L.radon_multi_cg_graph(None, None, None, 1, 0.0, None, 0, None, ctypes.byref(h)) == -1
    assert L.radon_graph_launch(None, None) == -1
    L.radon_graph_destroy(None)
    L.radon_multi_destroy(None)
    t, wf, wv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert L.radon_unrolled_sizes(None, 10, 5, 1, ctypes.byref(t), ctypes.byref(wf),
                                  ctypes.byref(wv)) == -1
    assert L.cg_unrolled(None, 1.0, 0.0, 1.0, None, None, 1, 10, 5, None, 0, None, 0, None) == -1
    assert L.cg_unrolled_vjp(None, 1.0, 0.0, 1.0, None, 0, None, None, 1, 10, 5, None, 0,
                             None) == -1


def test_fourier_entry_points_validate_without_gpu():
    L = sct.lib()
    text = open(HEADER).read()
    consts = dict(re.findall(r"#define\s+(\w+)\s+(-?\d+)", text))
    assert int(consts["RADON_FOURIER_FUSED"]) == sct.FOURIER_FUSED
    assert int(consts["RADON_FOURIER_NUFFT"]) == sct.FOURIER_NUFFT
    assert int(consts["RADON_FWS_SB"]) == sct.FWS_SB
    assert ctypes.sizeof(sct.FourierInfo) == 56
    h = ctypes.c_void_p()
    assert L.radon_fourier_create(None, 6, 0.0, 0, None, ctypes.byref(h)) == -1
    assert L.radon_fourier_create(None, 6, 0.0, 0, None, None) == -1
    assert "out is NULL" in L.radon_last_error().decode()
    assert L.radon_fourier_get_info(None, None) == -1
    assert L.radon_fourier_workspace_bytes(None, 0, 1) == -1
    assert L.fourier_fwd(None, None, None, 1, None, 0, None) == -1
    assert L.fourier_adj(None, None, None, 1.0, 1, None, 0, None) == -1
    assert L.fourier_normal(None, 0, 1.0, 0.0, 0.0, None, None, None, 1, None, 0, None) == -1
    assert "Fourier operator is NULL" in L.radon_last_error().decode()
    assert L.split_bregman_tv_fourier(None, 0, None, None, None, 1, None, 0, None, None) == -1
    L.radon_fourier_destroy(None)


def test_sb_graph_entry_point_validates_without_gpu():
    L = sct.lib()
    h = ctypes.c_void_p()
    assert L.split_bregman_tv_graph(None, None, None, None, 1, None, 0, None, ctypes.byref(h)) == -1
    assert L.split_bregman_tv_graph(None, None, None, None, 1, None, 0, None, None) == -1
    assert "out is NULL" in L.radon_last_error().decode()


def test_caller_storage_and_tuner_entry_points_validate_without_gpu():
    L = sct.lib()
    sz = sct.RadonSizes()
    assert L.radon_csr_sizes(None, None, 0, None, ctypes.byref(sz)) == -1
    g = sct._Geom(8, 4, 13, 0, None)
    assert L.radon_csr_sizes(ctypes.byref(g), None, 0, None, None) == -1
    assert "out is NULL" in L.radon_last_error().decode()
    bad = sct._Geom(8, 4, 13, 0, None, 24, 0)   # not a supported bundle width
    assert L.radon_csr_sizes(ctypes.byref(bad), None, 0, None, ctypes.byref(sz)) == -1
    assert "fwd_bundle" in L.radon_last_error().decode()
    h = ctypes.c_void_p()
    assert L.build_radon_csr(ctypes.byref(bad), None, ctypes.byref(h)) == -1
    assert L.build_radon_csr_into(ctypes.byref(g), None, None, ctypes.byref(h)) == -1
    assert "buffers are NULL" in L.radon_last_error().decode()
    b = sct.RadonBuffers()
    assert L.build_radon_csr_into(ctypes.byref(g), ctypes.byref(b), None, None) == -1
    src = ctypes.c_int32(7)
    assert L.radon_autotune(None, 1, None, 0, None, 0, None, ctypes.byref(src)) == -1
    assert L.normal_apply_noalloc(None, 1.0, 1.0, 0.0, None, None, None, 1, None) == -1
