"""The C-ABI library loads and exports every entry point its header declares.
CPU only: no call here reaches the GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "drgraph.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(drg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2008_07799_amd import drgraph
    if not os.path.exists(drgraph.LIB_PATH):
        from paper_2008_07799_amd import build
        build.build()
    return drgraph.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("drg_build_similarity", "drg_coarsen", "drg_layout_step", "drg_layout"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_defaults_and_argument_errors(lib):
    from paper_2008_07799_amd import drgraph as d
    p = d.layout_params()
    assert (p.k, p.M, p.T, p.max_levels) == (1, 5, 400, 64)
    assert abs(p.gamma - 0.1) < 1e-7 and abs(p.rho - 0.8) < 1e-12
    assert lib.drg_layout_params_default(None) == d.DRG_E_INVALID
    assert b"NULL" in lib.drg_last_error()
    assert lib.drg_sim_info(None, None, None, None, None, None) == d.DRG_E_INVALID
    assert lib.drg_hier_info(None, None, None) == d.DRG_E_INVALID
    assert lib.drg_layout_step(None, None, None, None, None) == d.DRG_E_INVALID
    assert lib.drg_ctx_create(0, None, None, None) == d.DRG_E_INVALID
    # destroy calls are NULL-safe
    lib.drg_sim_destroy(None)
    lib.drg_hier_destroy(None)
    lib.drg_ctx_destroy(None)
    assert lib.drg_version().startswith(b"drgraph")


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structures have the size and field offsets that
    a C compiler gives the header's structures."""
    import subprocess
    from paper_2008_07799_amd import drgraph as d
    structs = {"drg_csr": d.Csr, "drg_step_params": d.StepParams,
               "drg_layout_params": d.LayoutParams, "drg_obj_params": d.ObjParams,
               "drg_allocator": d.Allocator}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "drgraph.h"',
             "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, key, val = line.split()
        got[(cname, key)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2008_07799_amd import drgraph as d
    monkeypatch.setattr(d, "_lib", None)
    monkeypatch.setattr(d, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        d.lib()


def test_shape_parameter_split():
    """b crosses the ABI as its whole part plus a half flag (1, 1.5, 2, 2.5,
    3); other values are refused before any call."""
    from paper_2008_07799_amd import drgraph as d
    assert [d._shape(b) for b in (1, 1.5, 2, 2.5, 3)] == [(1, 0), (1, 1), (2, 0), (2, 1), (3, 0)]
    for bad in (0.5, 1.25, 3.5, 4, 0):
        with pytest.raises(ValueError):
            d._shape(bad)
    p = d.StepParams(5, *d._shape(2.5)[:1], 0.1, 1.0, 4.0, 0, 0, 2, 0, 0, d._shape(2.5)[1])
    assert (p.b, p.b_half) == (2, 1)


def test_layout_params_variants(lib):
    """Defaults leave the variants off (whole b, one global sigma); keyword
    overrides set them."""
    from paper_2008_07799_amd import drgraph as d
    p = d.layout_params()
    assert (p.b_half, p.perplexity, p.dim) == (0, 0.0, 0)
    q = d.layout_params(b=1.5, perplexity=30.0, dim=3)
    assert (q.b, q.b_half, q.perplexity, q.dim) == (1, 1, 30.0, 3)
