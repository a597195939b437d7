"""Host-side checks of the C-ABI library: it loads and exports every declared symbol,
and the Python binding declares exactly those entry points."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "yqbx.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(yq_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ["yq_create", "yq_set_particles", "yq_apply_operator", "yq_apply_far", "yq_solve",
                 "yq_forces", "yq_surface_gradient", "yq_eval_potential", "yq_get_nodes",
                 "yq_get_near", "yq_boundary_label", "yq_bessel"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1810_04131_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libyqbx.so not built")
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.SIGNATURES), "binding and header disagree"


def test_default_params_and_error_strings():
    from paper_1810_04131_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libyqbx.so not built")
    import paper_1810_04131_amd as yq
    p = yq.default_params()
    assert p.panels_per_particle == 32 and p.qbx_order == 10 and p.qbx_window == 2
    assert abs(p.qbx_radius - 0.25) < 1e-15 and p.qbx_oversample == 4
    lib = _lib.load()
    assert lib.yq_error_string(_lib.YQ_EGEOM).decode() == "geometry rejected"
    # parameter validation runs on the host (no device call)
    import ctypes
    bad = yq.default_params(qbx_order=0)
    h = ctypes.c_void_p()
    assert lib.yq_create(ctypes.byref(bad), ctypes.byref(h)) == _lib.YQ_EINVAL
    bad = yq.default_params(panels_per_particle=4)
    assert lib.yq_create(ctypes.byref(bad), ctypes.byref(h)) == _lib.YQ_EINVAL
    assert p.fmm_resid_order == 40 and p.fmm_m2l == yq.YQ_M2L_MFMA
    bad = yq.default_params(fmm_m2l=7)
    assert lib.yq_create(ctypes.byref(bad), ctypes.byref(h)) == _lib.YQ_EINVAL


def test_gauss_tables_generator_matches_header():
    # the committed coefficient header is what the generator writes
    import subprocess
    import sys
    gen = os.path.join(ROOT, "paper_1810_04131_amd", "csrc", "gen_bessel_tables.py")
    out = subprocess.run([sys.executable, gen], capture_output=True, text=True, check=True).stdout
    hdr = open(os.path.join(ROOT, "paper_1810_04131_amd", "csrc", "bessel_tables.h")).read()
    assert out.strip() == hdr.strip()


def test_library_shares_torch_hip_runtime():
    # loading the library before torch must not map a second HIP runtime
    import subprocess
    import sys
    from paper_1810_04131_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libyqbx.so not built")
    code = ("import paper_1810_04131_amd._lib as L; L.load(); import torch; "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True,
                         cwd=ROOT).stdout
    assert out.count("libamdhip64") == 1, out
