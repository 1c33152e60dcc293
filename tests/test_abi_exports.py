"""The C-ABI library loads and exports every symbol include/abm.h declares.
No compute calls: these run without a GPU."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\**(abm_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libabm():
    from paper_2301_06984_amd import abm
    if not os.path.exists(abm.LIB_PATH):
        pytest.skip("libabm.so not built (run __graft_entry__.build())")
    return abm


def test_header_declares_expected_api():
    names = declared_functions()
    for n in ("abm_init", "abm_step", "abm_query", "abm_init_batched", "abm_backward", "abm_graph_capture"):
        assert n in names
    assert len(names) >= 20


def test_every_declared_symbol_is_exported(libabm):
    L = libabm.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(libabm.EXPORTS) == declared_functions()


def test_version_and_defaults(libabm):
    L = libabm.lib()
    assert L.abm_abi_version() == libabm.ABI_VERSION == 6
    p = libabm.default_params()
    assert p.order == libabm.ABM_ORDER_MORTON and libabm.default_params(order="hilbert").order == 1
    assert (p.k, p.gamma, p.mu, p.f_adh, p.delta_max) == (2.0, 1.0, 0.1, 0.0, 3.0)
    assert p.cell_factor == 1.0 and p.sort_every == 1 and p.block_size == 256 and p.super_fraction == 0.0


def test_struct_sizes_match_header(libabm):
    assert C.sizeof(libabm.abm_params) == 7 * 8 + 8 * 4 + 8   # seven doubles, eight ints, a double
    assert C.sizeof(libabm.abm_extent) == 2 * 8 + 7 * 8
    assert C.sizeof(libabm.abm_stats) == 3 * 8 + 2 * 4 + 5 * 8


def test_workspace_bytes_validation(libabm):
    L = libabm.lib()
    p = libabm.default_params()
    nb = C.c_int64()
    offs = (C.c_int64 * 2)(0, 1000)
    caps = (C.c_int64 * 1)(5000)
    assert L.abm_workspace_bytes(1, offs, caps, C.byref(p), C.byref(nb)) == 0
    small = nb.value
    p64 = libabm.default_params(precision="f64", keep_forces=True)
    assert L.abm_workspace_bytes(1, offs, caps, C.byref(p64), C.byref(nb)) == 0
    assert nb.value > small
    bad = libabm.default_params(cell_factor=0.5)
    assert L.abm_workspace_bytes(1, offs, caps, C.byref(bad), C.byref(nb)) == libabm.ABM_E_INVAL
    assert b"cell_factor" in L.abm_last_error()
    bad = libabm.default_params(block_size=100)
    assert L.abm_workspace_bytes(1, offs, caps, C.byref(bad), C.byref(nb)) == libabm.ABM_E_INVAL
    huge = (C.c_int64 * 1)(2 ** 33)
    assert L.abm_workspace_bytes(1, offs, huge, C.byref(p), C.byref(nb)) == libabm.ABM_E_GRID
    offs_bad = (C.c_int64 * 2)(5, 1000)
    assert L.abm_workspace_bytes(1, offs_bad, caps, C.byref(p), C.byref(nb)) == libabm.ABM_E_INVAL


def test_super_fraction_sizes_the_table(libabm):
    # the per-super-box tables (48 B per entry): ceil((cap + 1) / 2) entries
    # by default, min(that, ceil(f cap) + 64) with super_fraction f
    L = libabm.lib()
    nb = C.c_int64()
    cap = 8_000_000
    sizes = {}
    for f in (0.0, 0.15, 1.0):
        p = libabm.default_params(super_fraction=f)
        assert L.abm_workspace_bytes_capacity(10 ** 6, cap, C.byref(p), C.byref(nb)) == 0
        sizes[f] = nb.value
    assert sizes[1.0] == sizes[0.0]                  # capped at the any-grid size
    saved = sizes[0.0] - sizes[0.15]
    assert abs(saved - 48 * ((cap + 2) // 2 - (math.ceil(0.15 * cap) + 64))) <= 48 * 1024
    for f in (-0.1, 1.5, float("nan")):
        bad = libabm.default_params(super_fraction=f)
        assert L.abm_workspace_bytes_capacity(10 ** 6, cap, C.byref(bad), C.byref(nb)) == libabm.ABM_E_INVAL
        assert b"super_fraction" in L.abm_last_error()


def test_null_context_is_rejected(libabm):
    L = libabm.lib()
    assert L.abm_step(None, 1) == libabm.ABM_E_INVAL
    assert L.abm_sync(None) == libabm.ABM_E_INVAL
    L.abm_destroy(None)   # no-op


def test_product_path_does_not_touch_oracle():
    # the product package must not import, load or name the oracle
    pkg = os.path.join(ROOT, "paper_2301_06984_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f
