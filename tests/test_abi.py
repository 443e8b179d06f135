"""The C-ABI library builds, loads and exports every symbol include/kbisim.h
declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "kbisim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kbisim_[a-z_]+)\s*\(", text)))


def test_header_declares_core_entry_points():
    names = declared_functions()
    for need in ["kbisim_create", "kbisim_refine", "kbisim_result", "kbisim_destroy",
                 "kbisim_status_str"]:
        assert need in names


def test_library_exports_all_declared():
    import paper_1210_0748_amd as kb
    if not os.path.exists(kb.lib_path()):
        pytest.skip("library not built")
    lib = ctypes.CDLL(kb.lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_null_handles():
    import paper_1210_0748_amd as kb
    if not os.path.exists(kb.lib_path()):
        pytest.skip("library not built")
    lib = kb.load_library()
    assert kb.kbisim_status_str(0) == "ok"
    assert kb.kbisim_status_str(-1) == "invalid argument"
    # argument checks that return before touching a device
    assert lib.kbisim_refine(None, 1, None) == -1
    assert lib.kbisim_result(None, None, 0, None, None, 0) == -1
    lib.kbisim_destroy(None)


def test_options_defaults_and_rejections_before_device_work():
    """kbisim_options_default and the option checks of kbisim_create, which
    reject out-of-range values before any device call."""
    import paper_1210_0748_amd as kb
    from paper_1210_0748_amd import _binding as B
    if not os.path.exists(kb.lib_path()):
        pytest.skip("library not built")
    lib = kb.load_library()
    opt = B.Options()
    lib.kbisim_options_default(ctypes.byref(opt))
    assert (opt.early_stop, opt.profile, opt.history, opt.update_mode, opt.radix_tile, opt.edge_window_bytes) == \
        (1, 0, 0, 0, 0, 0)
    assert opt.medium_cap == 4096
    desc = B.GraphDesc(0, 0, None, None, None, None, B.KBISIM_MEM_HOST, None)
    h = ctypes.c_void_p()
    for field, bad in (("radix_tile", 1000), ("radix_tile", 3000), ("radix_tile", -2048), ("medium_cap", 5000),
                       ("update_mode", 3), ("edge_window_bytes", -1)):
        o = B.Options()
        lib.kbisim_options_default(ctypes.byref(o))
        setattr(o, field, bad)
        assert lib.kbisim_create(ctypes.byref(desc), ctypes.byref(o), ctypes.byref(h)) == -1, (field, bad)
        assert field.split("_")[0] in lib.kbisim_last_error().decode(), field
