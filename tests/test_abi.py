"""The C-ABI library loads and exports every entry point its header declares (CPU only)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "recon.h")
LIB = os.path.join(ROOT, "paper_1209_3332_amd", "librecon.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(recon_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("recon_dilate", "recon_fill_holes", "recon_batch", "recon_submit", "recon_poll",
                     "recon_wait", "recon_create", "recon_destroy", "recon_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "librecon.so not built; run __graft_entry__.build()"
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), "missing export %s" % name


def test_binding_names_match_header():
    import paper_1209_3332_amd as p
    assert sorted(p.EXPORTED) == declared_functions()
    for name in declared_functions():
        assert callable(getattr(p, name)), name


def test_struct_layouts():
    import paper_1209_3332_amd as p
    assert ctypes.sizeof(p.recon_image) == 24
    assert ctypes.sizeof(p.recon_task) == 64
    assert ctypes.sizeof(p.recon_config) == 48


def test_last_error_is_a_string():
    import paper_1209_3332_amd as p
    assert isinstance(p.recon_last_error(), str)
