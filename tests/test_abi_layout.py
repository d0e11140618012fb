"""The ctypes binding against the C ABI it marshals for: every struct the binding builds or
reads has the size and field offsets the header gives it, and every enum value the
binding passes or decodes equals the header's.  A small C program compiled with gcc from
include/gft.h prints the header's figures (host only; no GPU, no library call)."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_1907_07875_amd as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "gft_graph": G._Graph,
    "gft_pairing": G._Pairing,
    "gft_options": G._Options,
    "gft_tuning": G.Tuning,
    "gft_plan_stats": G.PlanStats,
}

ENUMS = {
    **{name: value for name, value in (("GFT_FP32", G.GFT_FP32), ("GFT_BF16", G.GFT_BF16),
                                       ("GFT_FP16", G.GFT_FP16), ("GFT_SPLIT_BF16", G.GFT_SPLIT_BF16))},
    "GFT_ORDER_EIGENVALUE": G.ORDER_EIGENVALUE, "GFT_ORDER_BLOCK": G.ORDER_BLOCK,
    "GFT_ENGINE_AUTO": G.ENGINES["auto"], "GFT_ENGINE_GENERIC": G.ENGINES["generic"],
    "GFT_ENGINE_BUTTERFLY": G.ENGINES["butterfly"], "GFT_ENGINE_LARGE": G.ENGINES["large"],
    "GFT_ENGINE_PRODUCT": G.ENGINES["product"],
    "GFT_DTYPE_FP32": G.DTYPES["fp32"], "GFT_DTYPE_BF16": G.DTYPES["bf16"],
    "GFT_LAPLACIAN_COMBINATORIAL": G.LAPLACIANS["combinatorial"],
    "GFT_LAPLACIAN_NORMALIZED": G.LAPLACIANS["normalized"],
    **{name: code for code, name in G.STATUS.items()},
}


def _header_figures(tmp_path):
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "gft.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("size {cname} %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("off {cname}.{field} %zu\\n", offsetof({cname}, {field}));')
    for name in ENUMS:
        lines.append(f'  printf("enum {name} %d\\n", (int){name});')
    # the binding's option and tuning encodings
    lines += ['  printf("enum GFT_RIGHT_HAAR_AUTO %d\\n", (int)GFT_RIGHT_HAAR_AUTO);',
              '  printf("enum GFT_RIGHT_HAAR_OFF %d\\n", (int)GFT_RIGHT_HAAR_OFF);',
              '  printf("enum GFT_AUTOTUNE_ON %d\\n", (int)GFT_AUTOTUNE_ON);',
              '  printf("enum GFT_AUTOTUNE_OFF %d\\n", (int)GFT_AUTOTUNE_OFF);',
              '  printf("enum GFT_TUNE_BUILTIN %d\\n", (int)GFT_TUNE_BUILTIN);',
              '  printf("enum GFT_TUNE_TIMED %d\\n", (int)GFT_TUNE_TIMED);',
              '  printf("enum GFT_TUNE_CACHED %d\\n", (int)GFT_TUNE_CACHED);',
              "  return 0;", "}"]
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([shutil.which("gcc"), "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True, capture_output=True, text=True, timeout=120)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout
    figures = {}
    for line in out.splitlines():
        kind, key, value = line.split()
        figures[(kind, key)] = int(value)
    return figures


@pytest.fixture(scope="module")
def header(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.fail("gcc is needed to read the header's layout")
    return _header_figures(tmp_path_factory.mktemp("abi"))


@pytest.mark.parametrize("cname", list(STRUCTS))
def test_struct_layout_matches_header(header, cname):
    cls = STRUCTS[cname]
    assert ctypes.sizeof(cls) == header[("size", cname)], cname
    for field, _ in cls._fields_:
        assert getattr(cls, field).offset == header[("off", f"{cname}.{field}")], f"{cname}.{field}"


def test_enum_values_match_header(header):
    for name, value in ENUMS.items():
        assert header[("enum", name)] == value, name
    # _options passes right_haar=True as AUTO and autotune=True as ON
    o = G._options(right_haar=True, autotune=True)
    assert o.right_haar == header[("enum", "GFT_RIGHT_HAAR_AUTO")]
    assert o.autotune == header[("enum", "GFT_AUTOTUNE_ON")]
    o = G._options(right_haar=False, autotune=False)
    assert o.right_haar == header[("enum", "GFT_RIGHT_HAAR_OFF")]
    assert o.autotune == header[("enum", "GFT_AUTOTUNE_OFF")]
    # Tuning.as_dict decodes the tune source and engine with the header's values
    t = G.Tuning()
    for enum, label in (("GFT_TUNE_BUILTIN", "builtin"), ("GFT_TUNE_TIMED", "timed"), ("GFT_TUNE_CACHED", "cached")):
        t.source = header[("enum", enum)]
        assert t.as_dict()["source"] == label
    for label in ("generic", "butterfly", "large", "product"):
        t.engine = header[("enum", f"GFT_ENGINE_{label.upper()}")]
        assert t.as_dict()["engine"] == label
