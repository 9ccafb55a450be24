"""Host-side validation of scene blobs through the C ABI (no GPU needed: the blob is checked
completely before any device call).  Every malformed input returns PPT_EINVAL / PPT_EUNSUPPORTED
with a message; a valid blob only fails later, at the device step, on a machine without a GPU."""
import ctypes
import struct

import numpy as np
import pytest

import scenegen as sg


def _create(blob):
    from paper_2607_13265_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(blob, len(blob))
    rc = L.ppt_scene_create(buf, len(blob), ctypes.byref(h))
    msg = L.ppt_last_error().decode()
    if rc == 0:
        L.ppt_scene_destroy(h)
    return rc, msg


@pytest.fixture(scope="module")
def blob():
    from paper_2607_13265_amd import _lib
    import os
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("HIP library not built")
    return sg.config1().scene.to_blob()


def test_valid_blob_passes_host_validation(blob):
    rc, msg = _create(blob)
    assert rc == 0 or (rc == -3 and "device" in msg)  # no GPU here: fails only at the device step


@pytest.mark.parametrize("mutate,code", [
    (lambda b: b[:10], -1),                                            # truncated header
    (lambda b: struct.pack("<I", 0x12345678) + b[4:], -1),            # bad magic
    (lambda b: b[:-5], -1),                                            # truncated world data
    (lambda b: b + b"\0\0\0\0", -1),                                   # trailing bytes
    (lambda b: b[:8] + struct.pack("<I", 65) + b[12:], -4),            # too many slots
    (lambda b: b[:12] + struct.pack("<I", 0) + b[16:], -1),            # no world
])
def test_malformed_blobs_are_rejected(blob, mutate, code):
    rc, msg = _create(mutate(blob))
    assert rc == code and msg


def _scene_with(mat_kw):
    sc = sg.Scene()
    s = sc.add_slot("p", [0.5, 0.5, 0.5])
    w = sc.add_world()
    m = w.add_material(**mat_kw)
    w.add_quad((0, 0, 0), (1, 0, 0), (0, 1, 0), m)
    return sc.to_blob()


@pytest.mark.parametrize("kw", [
    dict(type=sg.MAT_LAMBERT, albedo_slot=5),                           # slot out of range
    dict(type=sg.MAT_LAMBERT, albedo_slot=0, albedo_off=1),            # 3 values past the end
    dict(type=sg.MAT_LAMBERT, albedo_slot=0, albedo_tw=4, albedo_th=4),  # texture larger than slot
    dict(type=sg.MAT_DIELECTRIC, eta_slot=-1),                           # missing IOR
    dict(type=sg.MAT_GGX_CONDUCTOR, alpha_slot=0, eta_slot=0),          # missing kappa
    dict(type=99),                                                       # unknown material type
    dict(type=sg.MAT_SHEET, axis=(0.0, 0.0, 0.0)),                      # degenerate polarizer axis
    dict(type=sg.MAT_EMITTER),                                           # emitter without radiance
    dict(type=sg.MAT_EMITTER, emit_slot=0, emit_circ=1.5),              # |circular degree| > 1
    dict(type=sg.MAT_LAMBERT, albedo_slot=0, spec_slot=0),              # specular map on a Lambertian
    dict(type=sg.MAT_GGX_DIELECTRIC, alpha_slot=0, eta_slot=0, spec_slot=0, spec_tw=2, spec_th=2),  # map past the slot
    dict(type=sg.MAT_LAMBERT, albedo_slot=0, normal_slot=0, normal_off=1),  # 3 normal components past the end
    dict(type=sg.MAT_LAMBERT, albedo_slot=0, normal_slot=0, normal_tw=1, normal_th=0),  # texture without height
    dict(type=sg.MAT_SHEET, axis=(1.0, 0.0, 0.0), normal_slot=0),       # normal map on a polarizer sheet
])
def test_bad_material_references(blob, kw):
    rc, msg = _create(_scene_with(kw))
    assert rc == -1 and "material" in msg


def test_bad_triangle_material_index(blob):
    sc = sg.Scene()
    sc.add_slot("p", [0.5, 0.5, 0.5])
    w = sc.add_world()
    w.add_material(type=sg.MAT_LAMBERT, albedo_slot=0)
    w.add_tris(np.zeros((1, 3, 3)), None, 7)
    rc, msg = _create(sc.to_blob())
    assert rc == -1 and "material" in msg


def test_non_finite_geometry(blob):
    sc = sg.Scene()
    sc.add_slot("p", [0.5, 0.5, 0.5])
    w = sc.add_world()
    m = w.add_material(type=sg.MAT_LAMBERT, albedo_slot=0)
    w.add_tris(np.array([[[0, 0, 0], [1, 0, 0], [0, np.nan, 0]]]), None, m)
    rc, msg = _create(sc.to_blob())
    assert rc == -1 and "finite" in msg


def test_light_circular_degree_out_of_range(blob):
    sc = sg.Scene()
    s_le = sc.add_slot("le", [1.0, 1.0, 1.0])
    w = sc.add_world()
    w.add_light((0, 0, 0), (1, 0, 0), (0, 1, 0), s_le, circ=-1.25)
    w.materials[-1]["emit_circ"] = 0.0  # only the light record is out of range
    rc, msg = _create(sc.to_blob())
    assert rc == -1 and "circular" in msg


def test_valid_light_stage_blob_passes_host_validation(blob):
    # circular lights, the light-stage analyzers' scene with normal and specular maps
    rc, msg = _create(sg.lightstage(res=16, spp=1).scene.to_blob())
    assert rc == 0 or (rc == -3 and "device" in msg)
