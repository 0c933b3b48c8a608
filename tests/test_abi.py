"""The C-ABI library loads and exports every entry point include/nnqp.h declares
(no GPU needed: nothing here launches device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nnqp.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nn_[a-z_]+)\s*\(", txt)))


def test_header_declares_expected_entry_points():
    from paper_1506_08435_amd import nnqp
    assert _declared() == sorted(nnqp.SYMBOLS)


def test_library_exports_every_declared_symbol():
    from paper_1506_08435_amd import nnqp
    lib = nnqp.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_opts_host_only():
    from paper_1506_08435_amd import nnqp
    o = nnqp.default_opts()
    assert o.tol == 1e-8 and o.inner_rtol == 0.1 and o.c0_value == 1e-8
    assert o.precision == nnqp.NN_FP64 and o.c0_mode == 0 and o.cg_chunk == 16
    with pytest.raises(KeyError):
        nnqp.default_opts(bogus=1)


def test_null_arguments_rejected_without_device_work():
    from paper_1506_08435_amd import nnqp
    lib = nnqp.load_library()
    b = ctypes.c_size_t()
    assert lib.nn_matrix_bytes(None, 0, ctypes.byref(b)) == nnqp.NN_EINVAL
    assert lib.nn_default_opts(None) == nnqp.NN_EINVAL
    assert lib.nn_matrix_info(None, None, None, None) == nnqp.NN_EINVAL
    assert lib.nn_last_error(None) == b"null context"
    assert lib.nn_solve_nonneg(None, None, None, None, None, None, None) == nnqp.NN_EINVAL
    # nn_create_ex needs both allocator hooks; it refuses before touching a device
    h = ctypes.c_void_p(1234)
    keep = nnqp.ALLOC_FN(lambda n, u: None)
    assert lib.nn_create_ex(ctypes.byref(h), 0, None, keep, nnqp.FREE_FN(), None) == nnqp.NN_EINVAL
    assert h.value is None


def test_struct_layouts_match_header(tmp_path):
    """Size and every field offset of the ctypes mirrors equal what the C
    compiler lays out for the declarations in include/nnqp.h."""
    import shutil
    import subprocess
    from paper_1506_08435_amd import nnqp
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"nn_opts": nnqp.Opts, "nn_stats": nnqp.Stats, "nn_mesh": nnqp.Mesh}
    lines = ['#include <stdio.h>', '#include "nnqp.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1506_08435_amd import nnqp
    saved = nnqp._lib
    nnqp._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            nnqp.load_library(str(tmp_path / "missing.so"))
    finally:
        nnqp._lib = saved
