"""CPU checks of the C-ABI library: it loads and exports every entry point
that include/lsms_tau.h declares, and the binding's structs match the header."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsms_tau.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*int\s+(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_header_symbols():
    import paper_2308_16317_amd as P

    L = P.lib()
    names = _declared()
    assert {"build_kkr", "tau00_batched", "tau00_solve", "lsms_build_liz"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(P.lsms.SYMBOLS)


def test_struct_layouts():
    from paper_2308_16317_amd import lsms

    assert ctypes.sizeof(lsms._Problem) == 6 * 4 + 6 * 8
    assert ctypes.sizeof(lsms.Opts) == 4 * 4
    assert [f[0] for f in lsms.Opts._fields_] == ["precision", "nb", "chunk", "flags"]


def test_null_handle_rejected_without_gpu():
    import paper_2308_16317_amd as P

    L = P.lib()
    assert L.lsms_destroy(None) == -1
    assert L.tau00_solve(None, None, None, None, None, None, 0, None) == -1
