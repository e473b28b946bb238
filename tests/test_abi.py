"""The C-ABI library loads and exports every entry point include/sphx.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sphx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sphx_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sphx_create", "sphx_set_fluid", "sphx_set_walls", "sphx_build_neighbors",
                     "sphx_get_neighbors", "sphx_advance", "sphx_get_field", "sphx_compute_rates"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2010_12375_amd import sphx
    lib = ctypes.CDLL(sphx.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []
    assert sorted(sphx.EXPORTED) == declared_functions()


def test_binding_layout_matches_header_structs():
    """sphx_params / sphx_diag field order and sizes as in the header."""
    from paper_2010_12375_amd import sphx
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} sphx_params;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(" ", 1)[1].split(","):
            names.append(re.sub(r"\[.*\]", "", part).strip())
    assert names == [f[0] for f in sphx.sphx_params._fields_]
    assert ctypes.sizeof(sphx.sphx_params) == 4 * 8 + 8 * (7 + 9 + 3)
    assert ctypes.sizeof(sphx.sphx_diag) == 8 * 12
    body = re.search(r"typedef struct \{([^{}]*?)\} sphx_wall_motion;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = [re.sub(r"\[.*\]", "", d.strip().split(" ", 1)[1]).strip() for d in body.split(";") if d.strip()]
    assert names == [f[0] for f in sphx.sphx_wall_motion._fields_]
    assert ctypes.sizeof(sphx.sphx_wall_motion) == 8 * 8


def test_missing_library_fails_loudly(tmp_path):
    from paper_2010_12375_amd import sphx
    with pytest.raises(ImportError):
        sphx.load(str(tmp_path / "nope.so"))


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2010_12375_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "sphx_oracle" not in src, f
