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
    assert ctypes.sizeof(lsms.Opts) == 6 * 4 + 8
    assert [f[0] for f in lsms.Opts._fields_] == ["precision", "nb", "chunk", "flags", "max_refine", "reserved",
                                                  "tol"]


def test_header_constants_match_binding():
    from paper_2308_16317_amd import lsms

    src = open(HEADER).read()
    defs = {}
    for k, v in re.findall(r"#define\s+(LSMS_\w+)\s+([-()<\d\s]+?)\s*(?:/\*|$)", src, flags=re.M):
        defs[k] = eval(v)  # integer constants and shifts only (the pattern admits nothing else)
    assert int(defs["LSMS_PREC_FP64"]) == lsms.PREC_FP64
    assert int(defs["LSMS_PREC_FP32_IR"]) == lsms.PREC_FP32_IR
    assert int(defs["LSMS_INFO_FP64_FALLBACK"]) == lsms.INFO_FP64_FALLBACK
    assert int(defs["LSMS_PERSISTENT"]) == lsms.PERSISTENT
    assert int(defs["LSMS_GRAPH"]) == lsms.GRAPH
    assert int(defs["LSMS_INFO_LU_FALLBACK"]) == lsms.INFO_LU_FALLBACK
    assert int(defs["LSMS_INFO_PIVOT_MASK"]) == lsms.INFO_PIVOT_MASK
    assert int(defs["LSMS_MLP_PARAMS"]) == lsms.MLP_PARAMS
    assert int(defs["LSMS_MLP_ACT"]) == lsms.MLP_ACT


def test_network_size_matches_reference():
    from oracle import mlp

    from paper_2308_16317_amd import lsms

    assert mlp.param_count() == lsms.MLP_PARAMS
    # activations kept per sample: Z and H of three hidden layers, then the output
    assert lsms.MLP_ACT == 6 * 256 + 1024


def test_null_handle_rejected_without_gpu():
    import paper_2308_16317_amd as P

    L = P.lib()
    assert L.lsms_destroy(None) == -1
    assert L.tau00_solve(None, None, None, None, None, None, 0, None) == -1


def test_info_flags_above_every_pivot_step():
    # a zero pivot reports its elimination step k <= N in the low bits; the
    # fallback flags sit above every step and decode apart from it
    from paper_2308_16317_amd import lsms

    for flag in (lsms.INFO_FP64_FALLBACK, lsms.INFO_LU_FALLBACK):
        assert flag & lsms.INFO_PIVOT_MASK == 0 and flag & (flag - 1) == 0
        assert flag > 25 * 1024  # kk * max_liz, the largest N the ABI admits
    assert lsms.INFO_FP64_FALLBACK != lsms.INFO_LU_FALLBACK
    for k in (1, 256, 512, 4096):
        info = lsms.INFO_FP64_FALLBACK | k
        assert info & lsms.INFO_PIVOT_MASK == k and info & lsms.INFO_FP64_FALLBACK
