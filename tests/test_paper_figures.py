"""The oracle's circuit accounting against the figures the paper prints
(fixture: tests/golden/paper_figures.json, each entry cited)."""
import json
import os

import numpy as np

import oracle as orc

FIX = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_figures.json")))


def test_msb_counts_match_sec_4_and_5():
    f = FIX["msb16"]
    _, _, ands, depth = orc.t_bit_extract(16, 15, 40000, 30000, 20000, 1)
    assert ands == f["and_gates"] and depth[15] == f["rounds"]
    for k in (8, 18, 32):
        _, _, ands, depth = orc.t_bit_extract(k, k - 1, 5, 6, 7, 2)
        assert ands == 2 * k - 3 and depth[k - 1] == k - 1


def test_table3_bits_per_comparison():
    t = FIX["table3_comm_kB_per_party_per_100k"]
    bits = {k: v * 1000 * 8 / 100_000 for k, v in t.items() if k != "cite"}
    # Plain Mask = one MSB over Z_2^16 (29 AND), ConstLift / NoLift = one MSB
    # over Z_2^32 (61 AND), Or Tree = one AND per element: 1 bit each.
    assert round(bits["Plain Mask"]) == 29
    assert round(bits["ConstLift"]) == 61 and round(bits["NoLift"]) == 61
    assert round(bits["Or Tree"]) == 1
    # MPCLift: the paper's 171 bits are not re-derived here; the oracle's
    # count per party (excluding resharing) is reported beside it.
    m, _, _, counts, _ = orc.t_compare_one(np.array([1, 2, 3], np.uint16), np.array([4, 5, 6], np.uint16), 3)
    assert counts[1] == 94 + 62 and counts[2] == counts[3] == 94 + 31
    assert abs(bits["MPCLift"] - 171) < 0.1


def test_or_tree_one_gate_per_element(keys):
    _, party = keys
    nq, r, n = 1, 4, 64 * 8
    comps = np.zeros((3, nq * r, n // 64), dtype=np.uint64)
    _, nwords = orc.or_tree(party, comps, nq, r, 0)
    # word-level: (32 words -> 1) = 31 word gates, then 6 in-word levels;
    # 31*64 + 32+16+8+4+2+1 = 2047 = (r*n) - 1 meaningful bit gates
    assert nwords == 31 + 6
    assert 31 * 64 + (32 + 16 + 8 + 4 + 2 + 1) == r * n - 1


def test_limb_gemm_counts():
    # byte limbs i, j of a k-bit ring product survive mod 2^k iff i + j <= k/8 - 1
    f = FIX["int8_gemms"]
    for k, want in ((16, f["Z_2^16"]), (32, f["Z_2^32"])):
        nl = k // 8
        assert sum(1 for i in range(nl) for j in range(nl) if i + j <= nl - 1) == want


def test_dot_product_communication():
    f = FIX["dot_comm"]
    # one reshared Z_2^16 value per dot product per party
    assert f["db_size"] * 2 / 1e6 == f["MB"] and f["ring"] == 1 << 16
