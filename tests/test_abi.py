"""CPU-side checks of the C ABI: the library loads and exports every declared entry point."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:tp_status|int|const char\*)\s+(tp_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["tp_symbol_build", "tp_apply", "tp_truncate", "tp_pcg_solve", "tp_inner", "tp_dst",
                     "tp_create", "tp_destroy", "tp_eval_grid", "tp_from_cp"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1809_01971_amd import _tp
    lib_path = _tp.library_path()
    if not os.path.exists(lib_path):
        pytest.skip("libtp.so not built")
    lib = _tp.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(_tp.exported_symbols())
    assert lib.tp_version() >= 100


def test_invalid_arguments_are_rejected_without_a_gpu():
    """tp_create on a machine without a device fails cleanly with a message."""
    from paper_1809_01971_amd import _tp
    import ctypes as C
    if not os.path.exists(_tp.library_path()):
        pytest.skip("libtp.so not built")
    lib = _tp.load_library()
    h = C.c_void_p()
    st = lib.tp_create(-1, None, 0, C.byref(h))
    assert st != 0
    assert len(lib.tp_last_error()) > 0
    # NULL out pointer
    assert lib.tp_create(0, None, 0, None) == _tp.TP_EINVAL
