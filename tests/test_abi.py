"""The C-ABI library loads and exports every function include/nlte3d.h declares (no GPU)."""
import ctypes
import os
import re

import pytest

from paper_1701_01607_amd import nlte

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nlte3d.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nlte_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    assert set(declared_functions()) == set(nlte.SYMBOLS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(nlte.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(nlte.LIB_PATH)
    missing = [s for s in declared_functions() if not hasattr(lib, s)]
    assert not missing, missing
    lib.nlte_version.restype = ctypes.c_char_p
    assert lib.nlte_version().startswith(b"nlte3d")


def test_struct_layouts_match_header_field_order():
    # every field of the ctypes mirrors appears in the header struct, in order
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for cls, cname in ((nlte.AtomDesc, "nlte_atom_desc"), (nlte.AtmosDesc, "nlte_atmos_desc"),
                       (nlte.Params, "nlte_params"), (nlte.Result, "nlte_result")):
        chunk = [c for c in text.split("typedef struct {") if re.search(r"\}\s*" + cname + ";", c)][0]
        body = chunk[: chunk.index("}")]
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = re.findall(r"\**\s*([A-Za-z_][A-Za-z_0-9]*)\s*(?:\[\d+\])?\s*[,;]", body)
        assert [f[0] for f in cls._fields_] == names, cname


def test_load_fails_loudly_without_library(tmp_path):
    with pytest.raises(FileNotFoundError):
        nlte._lib = None
        try:
            nlte.load(str(tmp_path / "missing.so"))
        finally:
            nlte._lib = None
