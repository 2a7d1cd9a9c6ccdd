"""The C-ABI library loads without a GPU and exports every declared entry point."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "irismpc.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(imc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("imc_create", "imc_destroy", "imc_share_db", "imc_share_query", "imc_dot_shares", "imc_reshare",
              "imc_compare_threshold", "imc_or_tree", "imc_open", "imc_append_db"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2405_04463_amd as imc

    if not os.path.exists(imc.LIB_PATH):
        pytest.fail("libirismpc.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(imc.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(imc.EXPORTS) == declared()


def test_host_side_helpers_without_gpu():
    import paper_2405_04463_amd as imc

    L = imc.lib()
    assert L.imc_strerror(0) == b"ok" and L.imc_strerror(-5).startswith(b"components")
    assert imc.db_bytes(1) == 32 * 102400 and imc.db_bytes(33) == 2 * 32 * 102400
    assert imc.query_op_bytes(3) == 3 * 102400 and imc.query_raw_bytes(2) == 2 * 2 * 2 * 12800 * 2
    # message buffers: planes x 64 words per group of 64 match words (31 rows x 5 words = 155 -> 3 groups)
    assert imc.compare_msg_bytes(0, 31, 300) == 406 * 64 * 3 * 8
    assert imc.compare_msg_bytes(imc.CMP_PLAIN_MASK, 31, 300) == 87 * 64 * 3 * 8
    assert imc.compare_msg_bytes(imc.CMP_LIFT18, 1, 1) == 210 * 64 * 8
    assert imc.compare_msg_bytes(imc.CMP_CONST32, 64, 64) == 183 * 64 * 8
    assert imc.compare_msg_bytes(9, 64, 64) == 0
    # a null parameter block is rejected before any device call
    h = ctypes.c_void_p()
    assert L.imc_create(None, 0, ctypes.byref(h)) == imc.IMC_EINVAL
    p = imc.imc_params()
    p.code_bits = 2048
    p.thr_a = 16384
    p.max_rows = 1
    assert L.imc_create(ctypes.byref(p), 0, ctypes.byref(h)) == imc.IMC_EUNSUPPORTED
