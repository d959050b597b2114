"""The C ABI library loads on any host and exports every entry point that
include/vls.h declares; the Python binding wraps each of them.  No compute
call is made (no GPU needed)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vls.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vls_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("vls_context_create", "vls_mesh_create", "vls_run", "vls_result_loop",
              "vls_result_reeb", "vls_result_field", "vls_result_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2105_13168_amd", "libvls.so"))
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    import paper_2105_13168_amd as vls
    assert sorted(vls.EXPORTED) == _declared()


def test_status_strings_and_defaults():
    import ctypes
    import paper_2105_13168_amd as vls
    assert vls.vls_status_string(0) == b"VLS_OK"
    assert vls.vls_status_string(-7) == b"VLS_E_STALLED"
    p = vls.default_params()
    assert p.struct_size == ctypes.sizeof(vls.vls_params)
    assert (p.tau, p.mu, p.a, p.w, p.e) == (0.5, 0.25, 1 / 25, (1 / 25) / 5, 1 / 30)
    assert p.seed_radius == 2 and p.dt_mode == 0
