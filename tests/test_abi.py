"""The C-ABI library loads and exports every call include/mcd.h declares."""

import ctypes

import paper_2309_15417_amd as mcd


def test_library_exports_header():
    decl = mcd.header_symbols()
    assert len(decl) >= 17
    assert mcd.exported_symbols() == decl


def test_abi_version_and_struct_sizes():
    L = mcd.load_library()
    assert L.mcd_abi_version() == 1
    assert mcd.PAIR_RESULT_DT.itemsize == 80
    assert mcd.CONTACT_DT.itemsize == 72
    assert mcd.STATS_DT.itemsize == 176
    # error string of a failed create is reachable without a context
    assert isinstance(L.mcd_last_error(None), bytes)
