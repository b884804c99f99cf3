"""The C-ABI library loads and exports every symbol include/*.h declares
(CPU only: no compute call is made)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlh.h")
LIB = os.path.join(ROOT, "paper_1410_5003_amd", "libmlh.so")


def declared_functions():
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(mlh_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mlh_ctx_create", "mlh_stack_create", "mlh_solve", "mlh_stack_destroy",
                     "mlh_last_error", "mlh_stack_info", "mlh_stack_refill", "mlh_stack_set_flux_tolerance"):
        assert required in names
    # the inspection calls live in their own header
    src = open(HEADER).read()
    assert "mlh_debug_" not in re.sub(r"/\*.*?\*/", "", src, flags=re.S)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmlh.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmlh.so not built")
def test_binding_signatures_cover_the_header():
    from paper_1410_5003_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared_functions())


def test_no_oracle_import_in_product():
    pkg = os.path.join(ROOT, "paper_1410_5003_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f


def _header_struct_fields(name):
    """Field names, in order, of `typedef struct { ... } name;` in mlh.h."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", src)
    assert m, name
    fields = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if decl:
            fields += [v.strip().lstrip("*") for v in decl.split(None, 1)[1].split(",")]
    return fields


@pytest.mark.parametrize("struct", ["mlh_tuning", "mlh_profile"])
def test_binding_structs_follow_the_header(struct):
    """ctypes mirrors of the header's structs: same fields in the same order
    (a swapped pair would silently exchange two values across the boundary)."""
    from paper_1410_5003_amd import _lib
    assert [f for f, _ in getattr(_lib, struct)._fields_] == _header_struct_fields(struct)


def test_tuning_struct_is_five_int32():
    from paper_1410_5003_amd import _lib
    assert ctypes.sizeof(_lib.mlh_tuning) == 20
