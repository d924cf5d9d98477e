"""The C-ABI library loads and exports every call include/mcd.h declares."""

import ctypes

import paper_2309_15417_amd as mcd


def test_library_exports_header():
    decl = mcd.header_symbols()
    assert len(decl) >= 17
    assert mcd.exported_symbols() == decl


def test_abi_version_and_struct_sizes():
    L = mcd.load_library()
    assert L.mcd_abi_version() == 2
    assert mcd.PAIR_RESULT_DT.itemsize == 80
    assert mcd.CONTACT_DT.itemsize == 80
    assert mcd.STATS_DT.itemsize == 240
    # error string of a failed create is reachable without a context
    assert isinstance(L.mcd_last_error(None), bytes)


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a header struct, from a C program built with gcc."""
    import subprocess
    root = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mcd.h"', 'int main(void) {',
             '  printf("%%zu\\n", sizeof(%s));' % struct]
    lines += ['  printf("%%zu\\n", offsetof(%s, %s));' % (struct, f) for f in fields]
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", root + "/include", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


def test_record_layouts_match_header(tmp_path):
    """The binding's record dtypes and ctypes structs have the header's sizes
    and field offsets, as a C compiler lays them out."""
    for struct, dt in (("mcd_pair_result", mcd.PAIR_RESULT_DT), ("mcd_contact", mcd.CONTACT_DT),
                       ("mcd_stats", mcd.STATS_DT)):
        size, offs = _c_layout(tmp_path, struct, dt.names)
        assert size == dt.itemsize, struct
        assert offs == [dt.fields[n][1] for n in dt.names], struct
    from paper_2309_15417_amd import mcd as m
    for struct, cs in (("mcd_config", m._Config), ("mcd_qopts", m._QOpts), ("mcd_impulse_opts", m._ImpulseOpts)):
        names = [f[0] for f in cs._fields_]
        size, offs = _c_layout(tmp_path, struct, names)
        assert size == ctypes.sizeof(cs), struct
        assert offs == [getattr(cs, n).offset for n in names], struct
    size, offs = _c_layout(tmp_path, "mcd_state", ["x", "q", "v", "w"])
    assert (size, offs) == (104, [0, 24, 56, 80])
