"""The C-ABI library loads and exports every entry point include/mcrt.h declares
(no device calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcrt.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcrt_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("mcrt_setup", "mcrt_trace", "mcrt_update_T", "mcrt_pda_solve", "mcrt_sed",
              "mcrt_locate", "mcrt_get", "mcrt_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_0902_3092_amd import mcrt
    L = mcrt.lib()
    for n in declared():
        assert hasattr(L, n), n
    assert set(mcrt.EXPORTS) <= set(declared())


def test_default_options_and_errors_without_device():
    from paper_0902_3092_amd import mcrt
    o = mcrt.default_options()
    assert o.n_T == 256 and o.n_inc == 10 and o.gamma == 3.0 and o.precision == mcrt.FP64
    L = mcrt.lib()
    assert L.mcrt_strerror(mcrt.E_ARG) == b"invalid argument"
    # argument checks happen before any device call
    assert L.mcrt_setup(None, None, None, None, None, None) == mcrt.E_ARG
    assert L.mcrt_trace(None, 1, 1, 0, 0, None, None, 0, None) == mcrt.E_ARG
    assert b"null" in L.mcrt_last_error()


def test_options_struct_matches_header():
    """The ctypes mirror has the field order and types of mcrt_options."""
    from paper_0902_3092_amd import mcrt
    text = open(HEADER).read()
    end = text.index("} mcrt_options;")
    body = text[text.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, names = decl.split(None, 1)
        fields += [(n.strip(), typ) for n in names.split(",")]
    assert [f for f, _ in fields] == [f for f, _ in mcrt.Options._fields_]


def test_header_constants_match_the_binding():
    """Every #define of include/mcrt.h that the binding mirrors has the same
    value there: error codes, precisions, what mcrt_get returns, and the
    hand-off buffer size."""
    from paper_0902_3092_amd import mcrt
    text = open(HEADER).read()
    defs = {m.group(1): int(m.group(2)) for m in
            re.finditer(r"^#define MCRT_([A-Z0-9_]+)\s+\(?(-?\d+)\)?", text, flags=re.M)}
    mirrored = 0
    for name, value in defs.items():
        if hasattr(mcrt, name):
            assert getattr(mcrt, name) == value, name
            mirrored += 1
    for name in ("OK", "E_ARG", "E_STUCK", "E_SINGULAR_REGION", "FP32", "TAIL_CAP", "GET_E_ABS",
                 "GET_RHO", "GET_TABLES", "GET_MRW_PATH"):
        assert name in defs and hasattr(mcrt, name), name
    assert mirrored >= 20
