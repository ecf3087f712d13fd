"""C interface checks that need no GPU: the built library loads, exports every
entry point include/tcplb.h declares, its parameter structs match the
header's layout, and invalid parameters are rejected before any device work."""
from __future__ import annotations

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tcplb.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(tcp_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2401_03041_amd import tcplb
    lib = tcplb.load()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
        # the binding declares every entry point's argument types
        assert getattr(lib, n).argtypes is not None, n
    assert sorted(tcplb.EXPORTS) == names


def test_params_layout_matches_header():
    """Field order of tcp_params in the header equals the ctypes mirror."""
    from paper_2401_03041_amd import tcplb
    text = open(HEADER).read()
    body = text[text.index("typedef struct {\n    int32_t nx"):]
    body = body[:body.index("} tcp_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names, count = [], 0
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl or decl.startswith("typedef"):
            decl = decl.replace("typedef struct {", "").strip()
        if not decl:
            continue
        parts = decl.split(None, 1)
        width = 4 if parts[0] == "int32_t" else 8
        for v in parts[1].split(","):
            v = v.strip()
            names.append(v.split("[")[0])
            count += width * (int(v.split("[")[1].rstrip("]")) if "[" in v else 1)
    assert names == [f for f, _ in tcplb.Params._fields_]
    assert C.sizeof(tcplb.Params) == count


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("q_pf", 19), ("q_thermal", 9), ("thermal", 3), ("precision", 3), ("nu_l", 0.0),
    ("mobility", -1.0), ("xi", 0.0), ("kappa_h", float("nan")), ("omega_bulk", 2.0)])
def test_invalid_parameters_rejected_without_gpu(field, value):
    from paper_2401_03041_amd import tcplb
    lib = tcplb.load()
    p = tcplb.Params()
    assert lib.tcp_params_default(C.byref(p)) == 0
    setattr(p, field, value)
    h = C.c_void_p()
    rc = lib.tcp_create(C.byref(p), None, None, C.byref(h))
    assert rc == -1
    assert not h.value
    assert lib.tcp_last_error(None)


def test_rk_stability_bound_rejected_without_gpu():
    from paper_2401_03041_amd import tcplb
    lib = tcplb.load()
    p = tcplb.Params()
    lib.tcp_params_default(C.byref(p))
    p.thermal = 1
    p.kappa_h = p.kappa_l = 0.4  # above 2/5.78 for RK2
    h = C.c_void_p()
    assert lib.tcp_create(C.byref(p), None, None, C.byref(h)) == -1
    assert b"stability" in lib.tcp_last_error(None)
    p.kappa_h = p.kappa_l = 2.25  # the capture channel's diffusivity needs the LB thermal solver
    p.thermal = 2
    assert lib.tcp_create(C.byref(p), None, None, C.byref(h)) == -1


@pytest.mark.parametrize("shape,precision,expect", [
    ((1024, 1024, 1024), 1, -2),   # one FP32 field of exactly 4 GiB: beyond 32-bit field offsets
    ((1024, 1024, 512), 0, -2),    # FP64, 4 GiB
    ((0, 8, 8), 1, -1),            # empty grid
    ((8, 1, 8), 1, -1)])           # walls need two rows
def test_grid_limits_rejected_without_gpu(shape, precision, expect):
    """Grids whose field arrays reach 4 GiB are refused (TCP_ERR_UNSUPPORTED)
    before any device work, as are empty grids (TCP_ERR_ARG)."""
    from paper_2401_03041_amd import tcplb
    lib = tcplb.load()
    p = tcplb.Params()
    lib.tcp_params_default(C.byref(p))
    p.nx, p.ny, p.nz = shape
    p.precision = precision
    p.walls_y = 1
    h = C.c_void_p()
    assert lib.tcp_create(C.byref(p), None, None, C.byref(h)) == expect
    assert not h.value


def test_error_strings():
    from paper_2401_03041_amd import tcplb
    lib = tcplb.load()
    for code in range(-6, 1):
        assert lib.tcp_error_string(code)


def test_warm_temperature_rejects_bad_arguments_without_a_domain():
    """A null domain is refused before anything touches the device."""
    from paper_2401_03041_amd import tcplb
    lib = tcplb.load()
    n, ch = C.c_int64(), C.c_double()
    assert lib.tcp_warm_temperature(None, 10, 0.0, 1, C.byref(n), C.byref(ch)) == -1  # TCP_ERR_ARG


def test_field_calls_reject_a_null_domain():
    """The field entry points, FP64 and FP32, refuse a null domain (TCP_ERR_ARG)
    before anything touches the device."""
    from paper_2401_03041_amd import tcplb
    lib = tcplb.load()
    buf = (C.c_double * 4)()
    fbuf = (C.c_float * 4)()
    assert lib.tcp_set_field(None, 0, buf, None) == -1
    assert lib.tcp_get_field(None, 0, buf, None) == -1
    assert lib.tcp_set_field_f32(None, 0, C.cast(fbuf, C.c_void_p)) == -1
    assert lib.tcp_get_field_f32(None, 0, C.cast(fbuf, C.c_void_p)) == -1
    assert lib.tcp_get_field_noalloc(None, 0, buf) == -1


def _declaration_comments():
    """(name, comment block directly above the declaration) for every entry point."""
    text = open(HEADER).read()
    out = []
    for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\*?\s*(tcp_\w+)\s*\(", text, flags=re.M):
        head = text[:m.start()].rstrip()
        # declarations directly after another one share the comment above the first
        while head.endswith(";") and "\n" in head:
            head = head[:head.rindex("\n")].rstrip()
        block = head[head.rindex("/*"):] if head.endswith("*/") else ""
        out.append((m.group(1), block))
    return out


# calls that carry the paper's problem statement: each must cite a section,
# equation, algorithm or appendix of the paper
PAPER_CALLS = ("tcp_params_default", "tcp_create", "tcp_set_field", "tcp_set_droplets", "tcp_set_heat_sources",
               "tcp_set_wall_temperature", "tcp_initialize", "tcp_step", "tcp_warm_temperature",
               "tcp_thermal_adjoint", "tcp_get_field", "tcp_get_pdfs", "tcp_reduce")


def test_every_declaration_names_its_passage():
    """Each entry point's comment opens with 'Passage:' and either cites the
    paper (Sec./Eq./Algorithm/App.) or says 'none' for a pure library utility;
    the calls of the problem statement always cite.  The allocation-free
    read-back names its callers instead."""
    cite = re.compile(r"Sec\. \d|Eq\. \w|Algorithm \d|App\. [A-C]")
    seen = set()
    for name, block in _declaration_comments():
        if name == "tcp_get_field_noalloc":
            # the allocation-free variant names the callers it exists for instead
            assert "callers that cannot allocate" in block, name
            seen.add(name)
            continue
        assert "Passage:" in block, f"{name}: no 'Passage:' line"
        passage = block[block.index("Passage:"):].split(".  ", 1)[0]
        assert cite.search(block) or "none" in passage, f"{name}: neither a citation nor 'none'"
        if name in PAPER_CALLS:
            assert cite.search(block), f"{name}: must cite the paper"
        seen.add(name)
    assert set(PAPER_CALLS) <= seen
