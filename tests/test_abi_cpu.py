"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/*.h declares, and the binding rejects malformed
arguments before anything reaches a kernel."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2210_01465_amd", "libfl.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        for m in re.finditer(r"\b(fl_[a-z_0-9]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fl_create", "fl_destroy", "fl_last_error", "fl_plan_create", "fl_execute",
                 "fl_plan_export", "fl_plan_destroy", "fl_analyze"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        import paper_2210_01465_amd.build as b
        b.build()
    import torch  # noqa: F401  (same runtime the binding uses)
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_prototypes_cover_the_header():
    from paper_2210_01465_amd import _abi
    assert set(_abi.PROTOTYPES) == declared_functions()


def _c_layout(struct: str, fields) -> list:
    """sizeof and field offsets of a struct of include/fl.h, as a C compiler
    lays it out."""
    import subprocess
    import tempfile
    body = [f'printf("%zu\\n", sizeof({struct}));']
    body += [f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"fl.h\"\nint main(void) {\n"
           + "\n".join(body) + "\nreturn 0;\n}\n")
    with tempfile.TemporaryDirectory() as tmp:
        c, exe = os.path.join(tmp, "l.c"), os.path.join(tmp, "l")
        with open(c, "w") as f:
            f.write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return [int(x) for x in out.split()]


@pytest.mark.parametrize("name", ["fl_params", "fl_summary", "fl_timing", "fl_space"])
def test_struct_layouts_match_header(name):
    from paper_2210_01465_amd import _abi
    cls = getattr(_abi, name)
    fields = [f for f, _ in cls._fields_]
    size, *offsets = _c_layout(name, fields)
    assert ctypes.sizeof(cls) == size
    assert [getattr(cls, f).offset for f in fields] == offsets


def test_null_context_is_rejected():
    from paper_2210_01465_amd import _abi
    lib = _abi.load()
    assert lib.fl_destroy(None) == _abi.FL_EINVAL
    assert lib.fl_last_error(None) == b"null context"
    assert lib.fl_plan_create(None, None, None, 0, None, None) == _abi.FL_EINVAL


def test_binding_checks_fitness_shape_on_host():
    from paper_2210_01465_amd import api

    class FakeCtx:
        device = 0
    with pytest.raises(TypeError):
        api._check_fitness(FakeCtx(), (2, 2), np.ones(4, np.float32))
