"""The C ABI: the header is plain C, the built library exports every symbol it
declares, the Python binding declares the same set, and the host-side
validation answers without a GPU."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dlmi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(dl_[a-z0-9_]+)\s*\(", text))


def test_header_is_plain_c():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    for lang, std in (("c", "-std=c99"), ("c++", "-std=c++11")):
        subprocess.run([gcc, "-fsyntax-only", "-Wall", "-Werror", "-x", lang, std, HEADER], check=True)


def test_binding_covers_header():
    from paper_1812_07607_amd import _lib
    assert set(_lib.SIGNATURES) == declared_functions()


def test_library_exports_declared_symbols():
    from paper_1812_07607_amd import _lib
    L = _lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(dl_[a-z0-9_]+)\b", out))
    assert declared_functions() <= exported


def test_host_validation_without_gpu():
    from paper_1812_07607_amd import _lib
    L = _lib.load()
    assert L.dl_version().startswith(b"dlmi")
    # null context and null arguments are rejected before any GPU work
    assert L.dl_featurize_rgb8(None, None, 0, 32, 32, 8, None, None) == _lib.DL_ERR_INVALID
    m = _lib.dl_mat(None, 0, 8, 8)
    pr = _lib.dl_pairs(None, None, None, 0, 0, 0, 0)
    assert L.dl_join_eps(None, m, m, 1, 1.0, 0, None, 0, ctypes.byref(pr), None) == _lib.DL_ERR_INVALID
    assert L.dl_join_topk(None, m, m, 1, 1, 0, 0, 0, None, 0, None, None, None, None) == _lib.DL_ERR_INVALID
    assert L.dl_create(0, None) == _lib.DL_ERR_INVALID
    h = ctypes.c_void_p()
    st = L.dl_create(0, ctypes.byref(h))
    if st == _lib.DL_OK:  # a GPU is present: the context must work and be destroyable
        assert L.dl_last_error(h) == b""
        L.dl_destroy(h)
    else:
        assert st == _lib.DL_ERR_DEVICE
    assert L.dl_last_error(None) == b"null context"


def test_workspace_queries():
    from paper_1812_07607_amd import _lib
    L = _lib.load()
    assert L.dl_join_eps_workspace(-1, 10, 8, 0, 0, 10) == 0
    assert L.dl_join_eps_workspace(10, 10, 0, 0, 0, 10) == 0
    assert L.dl_join_eps_workspace(10, 10, 8, 9, 0, 10) == 0
    a = L.dl_join_eps_workspace(1000, 2000, 64, 1, 0, 1000)
    b = L.dl_join_eps_workspace(1000, 2000, 64, 1, 0, 100000)
    assert 0 < a < b
    # a self-join needs one set of operand copies only
    assert L.dl_join_eps_workspace(1000, 1000, 64, 1, 1, 1000) < L.dl_join_eps_workspace(1000, 1000, 64, 1, 0, 1000)
    assert L.dl_join_topk_workspace(1000, 5000, 128, 1, 0, 10, 0) > 0
    assert L.dl_join_topk_workspace(1000, 5000, 128, 1, 0, 0, 0) == 0


def test_product_path_does_not_touch_oracle():
    """The library and its binding never import or link the oracle."""
    pkg = os.path.join(ROOT, "paper_1812_07607_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "dl_oracle" not in text and "liboracle" not in text, f


def test_struct_layouts_match_the_header(tmp_path):
    """Every public struct of the header has the size and field offsets of
    its ctypes declaration in the binding (a C program compiled against the
    header prints them)."""
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    from paper_1812_07607_amd import _lib
    structs = [getattr(_lib, n) for n in dir(_lib)
               if n.startswith("dl_") and isinstance(getattr(_lib, n), type)
               and issubclass(getattr(_lib, n), ctypes.Structure)]
    assert len(structs) >= 10
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dlmi.h"', "int main(void) {"]
    for s in structs:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (s.__name__, s.__name__))
        for f in s._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (s.__name__, f[0], s.__name__, f[0]))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               check=True).stdout.splitlines())
    for s in structs:
        assert int(got[s.__name__ + " size"]) == ctypes.sizeof(s), s.__name__
        for f in s._fields_:
            assert int(got["%s.%s" % (s.__name__, f[0])]) == getattr(s, f[0]).offset, (s.__name__, f[0])
