"""The C-ABI library loads on the host and exports every function that
include/rs.h declares (no compute call: no GPU needed)."""
import ctypes
import os
import re

from paper_1510_03110_amd import rs

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "rs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rs_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("rs_plan_create", "rs_plan_workspace_size", "rs_plan_destroy", "rs_batch_solve",
              "rs_factor", "rs_solve", "rs_plan_query", "rs_plan_export", "rs_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = rs.library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_options_struct_matches_header_size():
    # int32 precision, Ns, branch, max_refine; double tol; int32 flags, reserved
    assert ctypes.sizeof(rs.rs_options) == 32


def test_binding_constants_match_header():
    """Every #define and enum value of include/rs.h that the binding mirrors
    has the header's value (flags, status codes, precisions, sizes)."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    values = {}
    for name, expr in re.findall(r"#define\s+(RS_[A-Z0-9_]+)\s+(.+)", text):
        expr = expr.replace("(size_t)", "").strip()
        m = re.fullmatch(r"\(*\s*(\d+)\s*\)*(?:\s*<<\s*(\d+)\s*\)*)?", expr)
        if m:
            values[name] = int(m.group(1)) << int(m.group(2) or 0)
    for name, val in re.findall(r"\b(RS_[A-Z0-9_]+)\s*=\s*(\d+)", text):
        values[name] = int(val)
    checked = 0
    for name, val in values.items():
        if hasattr(rs, name):
            assert getattr(rs, name) == val, (name, getattr(rs, name), val)
            checked += 1
    assert checked >= 15
