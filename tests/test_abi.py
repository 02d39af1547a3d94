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
                     "tp_create", "tp_destroy", "tp_eval_grid", "tp_from_cp", "tp_pcg_solve_batched",
                     "tp_state_symbol_build", "tp_inner_sym", "tp_apply_sum", "tp_symbol_eval",
                     "tp_workspace_query", "tp_workspace_peak", "tp_profile", "tp_profile_read"]:
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


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's field offsets and size (gcc compiles a
    probe against include/tp.h; the binding's ctypes layout must agree field by field)."""
    import ctypes as C
    import shutil
    import subprocess
    from paper_1809_01971_amd import _tp
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = [_tp.tp_tensor, _tp.tp_cp, _tp.tp_sketch, _tp.tp_symbol_desc, _tp.tp_pcg_opts, _tp.tp_pcg_info]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tp.h"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append('  printf("%s sizeof %%zu\\n", sizeof(%s));' % (name, name))
        for f in st._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f[0], name, f[0]))
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for st in structs:
        name = st.__name__
        assert got[(name, "sizeof")] == C.sizeof(st), name
        for f in st._fields_:
            assert got[(name, f[0])] == getattr(st, f[0]).offset, (name, f[0])
