"""The C-ABI library loads and exports every function that include/ddqmc.h
declares, and the Python structs match the C layouts (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddqmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ddqmc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1802_05931_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1802_05931_amd import build
        build.build()
    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_1802_05931_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Size and every field offset of the ctypes mirrors equal gcc's for the header."""
    import subprocess
    from paper_1802_05931_amd import _lib
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ddqmc.h"', "int main(void){"]
    for cname, cls in (("ddqmc_params", _lib.Params), ("ddqmc_obs", _lib.Obs)):
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = []
    for cls in (_lib.Params, _lib.Obs):
        want.append(ctypes.sizeof(cls))
        want.extend(getattr(cls, f).offset for f, _ in cls._fields_)
    assert got == want


def test_strerror_and_invalid_params_without_device(lib):
    from paper_1802_05931_amd import _lib
    assert lib.ddqmc_strerror(_lib.EOVERFLOW) == b"walker count left the int32 range"
    p = _lib.make_params(Lx=1)
    n = ctypes.c_size_t()
    assert lib.ddqmc_workspace_query(ctypes.byref(p), 0, ctypes.byref(n)) == _lib.EINVAL
    p = _lib.make_params(Lx=4, Ly=4)
    assert lib.ddqmc_workspace_query(ctypes.byref(p), 1 << 20, ctypes.byref(n)) == _lib.OK
    assert n.value > (1 << 20) * 24
    p.struct_size = 7
    assert lib.ddqmc_workspace_query(ctypes.byref(p), 0, ctypes.byref(n)) == _lib.EINVAL


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1802_05931_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.replace("Oracle", ""), f
