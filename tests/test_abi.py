"""The C ABI library loads, exports every symbol include/ctpd.h declares, and
rejects bad arguments before touching the GPU (no compute calls here)."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_1609_06041_amd import ctpd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctpd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctpd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ctpd_project", "ctpd_backproject", "ctpd_ramp_filter", "ctpd_pd_lowdose_solve",
                     "ctpd_pd_fewview_solve", "ctpd_op_create", "ctpd_op_destroy", "ctpd_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol(libctpd):
    for name in declared_functions():
        assert hasattr(libctpd, name), name
        assert name in ctpd._SIGNATURES, f"binding lacks a signature for {name}"


# the binding's ctypes mirrors and the header's structs they stand for
MIRRORS = [(ctpd.Geometry, "ctpd_geometry"), (ctpd.Params, "ctpd_params"), (ctpd.State, "ctpd_state"),
           (ctpd.Report, "ctpd_report"), (ctpd.BatchTiles, "ctpd_batch_tiles")]


def test_binding_struct_layouts_match_header(tmp_path):
    # the C compiler's sizeof / offsetof of every field against the ctypes mirrors
    gcc = shutil.which("gcc") or shutil.which("cc")
    if gcc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "ctpd.h"', "int main(void) {"]
    for cls, cname in MIRRORS:
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["    return 0;", "}"]
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([gcc, "-std=c99", "-Wall", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                          check=True).stdout.splitlines())
    for cls, cname in MIRRORS:
        assert int(got[f"{cname} size"]) == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert int(got[f"{cname} {field}"]) == getattr(cls, field).offset, (cname, field)
    text = open(HEADER).read()
    assert f"#define CTPD_MAX_BINS {ctpd.MAX_BINS}" in text


@pytest.mark.parametrize("n,m,nb", [(0, 10, 10), (10, 0, 10), (10, 10, 0), (-3, 1, 1), (8, 8, 4097)])
def test_op_create_rejects_bad_geometry(libctpd, n, m, nb):
    h = ctypes.c_void_p()
    g = ctpd.Geometry(n, m, nb)
    assert libctpd.ctpd_op_create(ctypes.byref(g), None, ctypes.byref(h)) == ctpd.CTPD_EINVAL
    assert not h.value
    assert b"invalid argument" in libctpd.ctpd_strerror(ctpd.CTPD_EINVAL)


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_op_create_rejects_non_finite_angles(libctpd, bad):
    h = ctypes.c_void_p()
    angles = np.array([0.0, 0.5, bad, 2.0])
    g, keep = ctpd._geometry(8, 4, 12, angles)
    assert libctpd.ctpd_op_create(ctypes.byref(g), None, ctypes.byref(h)) == ctpd.CTPD_EINVAL
    assert not h.value
    with pytest.raises(ValueError):
        ctpd._geometry(8, 5, 12, angles)


def test_null_arguments_are_rejected(libctpd):
    assert libctpd.ctpd_op_create(None, None, None) == ctpd.CTPD_EINVAL
    assert libctpd.ctpd_project(None, None, None) == ctpd.CTPD_EINVAL
    assert libctpd.ctpd_backproject(None, None, None) == ctpd.CTPD_EINVAL
    assert libctpd.ctpd_ramp_filter(None, 1.0, 0.0, None, None) == ctpd.CTPD_EINVAL
    assert libctpd.ctpd_filter_taps(None, 1.0, 0.0, None) == ctpd.CTPD_EINVAL
    assert libctpd.ctpd_ramp_filter_f64(None, 1.0, 0.0, None, None) == ctpd.CTPD_EINVAL
    assert libctpd.ctpd_tv_prox(None, None, 0.1, 1, 0.125, None, None) == ctpd.CTPD_EINVAL
    assert libctpd.ctpd_pd_lowdose_solve(None, None, None, 0.1, 1, None, None, None) == ctpd.CTPD_EINVAL
    assert libctpd.ctpd_pd_fewview_solve(None, None, 1, None, None, None) == ctpd.CTPD_EINVAL
    assert libctpd.ctpd_pd_fewview_eps_solve(None, None, ctypes.c_double(0.5), 1, None, None,
                                             None) == ctpd.CTPD_EINVAL
    libctpd.ctpd_op_destroy(None)   # no-op


def test_error_strings(libctpd):
    for code in (0, -1, -2, -3, -4, -99):
        assert libctpd.ctpd_strerror(code)
