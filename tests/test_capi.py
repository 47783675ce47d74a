"""The C-ABI library loads and exports every entry point include/fil.h declares;
host-side argument validation rejects bad calls before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1903_12609_amd import build, _native
    srcs = build.sources() + [os.path.join(ROOT, "include", "fil.h")]
    srcs += [os.path.join(build.HERE, "csrc", f) for f in os.listdir(os.path.join(build.HERE, "csrc"))]
    if not os.path.exists(build.LIB) or os.path.getmtime(build.LIB) < max(os.path.getmtime(s) for s in srcs):
        build.build()
    return _native.lib()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fil.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(fil_[a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    L = _lib()
    names = declared_functions()
    assert "fil_rpy_mobility_apply" in names and len(names) >= 4
    for n in names:
        assert hasattr(L, n), n


def test_argument_validation_without_gpu():
    from paper_1903_12609_amd import _native
    L = _lib()
    p = ctypes.c_void_p(16)
    rc = L.fil_rpy_mobility_apply(10, p, p, p, -1.0, 1.0, 0, p, p, None, 0, None)
    assert rc == -1 and b"a and eta" in L.fil_last_error()
    rc = L.fil_rpy_mobility_apply(-3, p, p, p, 1.0, 1.0, 0, p, p, None, 0, None)
    assert rc == -1
    rc = L.fil_rpy_mobility_apply(10, p, p, p, 1.0, 1.0, 7, p, p, None, 0, None)
    assert rc == -1
    rc = L.fil_rpy_mobility_apply(10, None, p, p, 1.0, 1.0, 0, p, ctypes.c_void_p(32), None, 0, None)
    assert rc == -1 and b"null" in L.fil_last_error()
    assert L.fil_rpy_mobility_apply(0, None, None, None, 1.0, 1.0, 0, None, None, None, 0, None) == 0
    assert L.fil_rpy_workspace_bytes(1000, 0) > 0
    assert L.fil_rpy_workspace_bytes(-1, 0) == -1
    rc = L.fil_filament_internal_forces(3, 2, p, p, p, None, 2.2, 1.0, 1.0, p, p, None)
    assert rc == -1
