"""The C-ABI library loads and exports every entry point the header declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

from conftest import ROOT


def _declared():
    txt = open(os.path.join(ROOT, "include", "qp_pt2.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qp_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = _declared()
    for fn in ("qp_create", "qp_destroy", "qp_last_error", "qp_set_integrals", "qp_pt2",
               "qp_pt2_backward", "qp_energy"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    from paper_1902_08154_amd import _lib
    assert os.path.exists(_lib.LIB_PATH), "build the library first"
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for fn in _declared():
        assert hasattr(lib, fn), fn
    assert set(_lib.EXPORTS) == set(_declared())


def test_binding_refuses_to_run_without_library(tmp_path, monkeypatch):
    from paper_1902_08154_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    import pytest
    with pytest.raises(ImportError):
        _lib.load()


def test_stats_struct_layout():
    from paper_1902_08154_amd import _lib
    assert ctypes.sizeof(_lib.Stats) == 8 * 8 + 8 * (4 + 1 + 4 + 4) + 2 * 8


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a header struct, from a C program built with gcc."""
    import subprocess
    body = "".join(f'    printf(" %zu", offsetof({struct}, {f}));\n' for f in fields)
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "qp_pt2.h"\nint main(void)\n{\n'
                   f'    printf("%zu", sizeof({struct}));\n{body}    return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


def test_ctypes_structs_match_the_header(tmp_path):
    from paper_1902_08154_amd import _lib
    for cls, name in ((_lib.Stats, "qp_pt2_stats"), (_lib.System, "qp_system")):
        fields = [f for f, _ in cls._fields_]
        size, offs = _c_layout(tmp_path, name, fields)
        assert size == ctypes.sizeof(cls), name
        assert offs == [getattr(cls, f).offset for f in fields], name


def test_binding_constants_match_the_header():
    """Every QP_* integer macro of the header has the same value in the binding."""
    from paper_1902_08154_amd import _lib
    txt = open(os.path.join(ROOT, "include", "qp_pt2.h")).read()
    macros = dict((k, int(v)) for k, v in re.findall(r"#define\s+(QP_[A-Z0-9_]+)\s+(-?\d+)\b", txt))
    assert "QP_SIGMA_REUSE" in macros and "QP_E_NOCONV" in macros
    for k, v in macros.items():
        if hasattr(_lib, k):
            assert getattr(_lib, k) == v, k
    for k in ("QP_OK", "QP_FLAG_FINGERPRINT", "QP_FLAG_NOCHECK", "QP_FLAG_REUSE_INTEGRALS", "QP_SIGMA_S2",
              "QP_SIGMA_REUSE", "QP_MAX_STATES", "QP_MAX_SYSTEMS"):
        assert k in macros and getattr(_lib, k) == macros[k], k
