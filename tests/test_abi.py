"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every function the public header declares."""
import ctypes
import os
import subprocess

import pytest

from paper_2201_00701_amd import esom

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_path():
    if not os.path.exists(esom.LIB_PATH):
        from paper_2201_00701_amd import build
        build.build()
    return esom.LIB_PATH


def test_header_declares_the_entry_points():
    names = esom.header_functions()
    for required in ("esom_create", "esom_destroy", "esom_last_error", "esom_embed",
                     "esom_landmark_update", "esom_sync", "esom_get_stats",
                     "esom_default_params", "esom_set_timing", "esom_serve_create",
                     "esom_serve_destroy", "esom_serve_dataset_put", "esom_serve_dataset_drop",
                     "esom_serve_submit", "esom_serve_wait", "esom_serve_get_stats"):
        assert required in names


def test_library_exports_every_header_symbol():
    path = _lib_path()
    lib = ctypes.CDLL(path)
    missing = [n for n in esom.header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(esom.header_functions()) <= exported


def test_param_struct_matches_header_defaults():
    esom.load(_lib_path())
    p = esom.esom_default_params()
    assert (p.k, p.boost, p.adjust, p.cutoff, p.mode, p.candidates) == (16, 1.0, 1.0, 10.0, 0, 0)
    assert abs(p.gravity - 1e-5) < 1e-12
    assert ctypes.sizeof(esom.esom_params) == 28
    assert ctypes.sizeof(esom.esom_stats) == 96
    assert ctypes.sizeof(esom.esom_request_info) == 48
    assert ctypes.sizeof(esom.esom_serve_stats) == 128


def test_binding_never_imports_the_oracle():
    src = open(os.path.join(ROOT, "paper_2201_00701_amd", "esom.py")).read()
    assert "oracle" not in src.replace("No oracle", "")
    for f in os.listdir(os.path.join(ROOT, "paper_2201_00701_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2201_00701_amd", "csrc", f)).read()
