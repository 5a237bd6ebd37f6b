"""CPU checks of the C ABI: the library loads without a GPU and exports every
function include/tc.h declares; the binding's signatures cover the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")
LIB = os.path.join(ROOT, "paper_1706_05151_amd", "libtc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(tc_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tc_build_csr", "tc_count", "tc_count_per_node", "tc_clustering", "tc_list",
                     "tc_sparsify_count", "tc_graph_free", "tc_status_str", "tc_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtc.so not built")
def test_library_exports_every_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtc.so not built")
def test_binding_covers_header():
    from paper_1706_05151_amd import tc

    assert set(declared_functions()) == set(tc.SIGNATURES)
    L = tc.lib()
    assert L.tc_status_str(tc.TC_E_RANGE) == b"TC_E_RANGE"
    assert L.tc_status_str(tc.TC_E_TRUNC) == b"TC_E_TRUNC"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtc.so not built")
def test_options_roundtrip_on_host():
    from paper_1706_05151_amd import tc

    old = tc.get_option(tc.OPT_ITEM_WORK)
    tc.set_option(tc.OPT_ITEM_WORK, 1234)
    assert tc.get_option(tc.OPT_ITEM_WORK) == 1234
    tc.set_option(tc.OPT_ITEM_WORK, old)
    with pytest.raises(tc.TCError):
        tc.set_option(tc.OPT_KERNEL, 9)
    with pytest.raises(tc.TCError):
        tc.set_option(tc.OPT_ITEM_WORK, -1)
