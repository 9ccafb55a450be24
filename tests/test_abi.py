"""CPU-side checks of the C ABI: the HIP library loads and exports every symbol that
include/ppt.h declares, and the Python binding names the same entry points."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ppt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(ppt_[a-z0-9_]+)\s*\(", src, re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("ppt_scene_create", "ppt_plan_create", "ppt_render", "ppt_backward", "ppt_last_error"):
        assert n in names
    assert len(names) >= 15


def test_library_exports_every_declared_symbol():
    import ctypes

    from paper_2607_13265_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("HIP library not built")
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2607_13265_amd import _lib
    assert sorted(_lib.SIGNATURES) == _declared()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2607_13265_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(_lib.PPTError):
        _lib.lib()


def test_view_layout_matches_generators():
    import scenegen as sg
    from paper_2607_13265_amd.core import VIEW_DTYPE
    assert VIEW_DTYPE == sg.VIEW_DTYPE and VIEW_DTYPE.itemsize == 88


C_PROGRAM = os.path.join(ROOT, "tests", "c", "abi_render.c")


def build_c_program(out_dir):
    """Compiles the plain-C user of the ABI (tests/c/abi_render.c) against the built library."""
    import shutil
    import subprocess

    from paper_2607_13265_amd import _lib
    if not os.path.exists(_lib.LIB_PATH) or not shutil.which("gcc"):
        pytest.skip("HIP library not built or no C compiler")
    exe = os.path.join(str(out_dir), "abi_render")
    libdir = os.path.dirname(_lib.LIB_PATH)
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", C_PROGRAM, "-L", libdir, "-lppt", "-L", "/opt/rocm/lib", "-lamdhip64",
           f"-Wl,-rpath,{libdir}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_program_builds_against_the_abi(tmp_path):
    # the ABI is usable from C alone: the header compiles as C99 and the library links
    assert os.path.exists(build_c_program(tmp_path))
