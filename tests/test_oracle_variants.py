"""Pins of the oracle's comparison variants (masks in plain, Lift to Z_2^18,
ml over Z_2^32) and of its Z_2^32 dot products.

Each check ties the oracle to something it does not compute itself: the
threshold reductions written out exhaustively in numpy (Lemma 2 at the rings
the variants use; the floor reading of Lemma 1's rounding, by brute force),
the AND-gate counts and communication of the comparison benchmark (Sec. 6.2,
Table 3: Plain Mask 362 kB and ConstLift 763 kB per party for 100k
comparisons), the opened values of random sharings, and the plaintext
decision of the whole protocol.
"""
import numpy as np
import pytest

import oracle as orc
import workload as wl

L = 12800


# --------------------------------------------------------------------------
# threshold reductions, exhaustive (Sec. 4.3.1 Lemma 1; Sec. 5 Lemma 2)
# --------------------------------------------------------------------------
def _domain():
    ml = np.arange(0, L + 1, dtype=np.int64)
    for dot0 in range(-L, L + 1, 97):
        dot = np.arange(dot0, min(dot0 + 97, L + 1), dtype=np.int64)[:, None]
        ok = (np.abs(dot) <= ml) & (((dot - ml) & 1) == 0)
        yield ml, dot, ok


def test_plain_mask_threshold_exhaustive():
    # Masks public: MSB_16(floor(ml/4) - dot) == (4 dot > ml) for every valid
    # (ml, dot); Lemma 1's conditions l < t/4 and l < t - 2^(log t - 1) hold at t = 2^16.
    assert L < (1 << 16) // 4 and L < (1 << 16) - (1 << 15)
    for ml, dot, ok in _domain():
        y = (ml // 4 - dot) & 0xFFFF
        assert np.array_equal(((y >> 15) & 1 == 1) & ok, (4 * dot > ml) & ok)


def test_lift18_threshold_exhaustive():
    # a = 1, b = 4 = 2^m with m = 2: Lemma 2 needs b l < t/4 and
    # b l < t - 2^(log t - 1) at t = 2^18; then MSB_18(ml - 4 dot) decides.
    t = 1 << 18
    assert 4 * L < t // 4 and 4 * L < t - (1 << 17)
    for ml, dot, ok in _domain():
        y = (ml - 4 * dot) & (t - 1)
        assert np.array_equal(((y >> 17) & 1 == 1) & ok, (4 * dot > ml) & ok)


def test_lemma1_rounding_reading():
    # Lemma 1 states MSB(ceil(f ml) - hd) for hd > f ml; with non-integral
    # f ml the ceiling is off by one and the floor is exact (brute force at
    # f = 0.3 over ml < 40).  The oracle's PLAIN variant uses the floor.
    f = 0.3
    bad_ceil = bad_floor = 0
    for ml in range(40):
        for hd in range(ml + 1):
            want = hd > f * ml
            bad_ceil += (np.ceil(f * ml) - hd < 0) != want
            bad_floor += (np.floor(f * ml) - hd < 0) != want
    assert bad_floor == 0 and bad_ceil > 0


# --------------------------------------------------------------------------
# one comparison per variant on random sharings
# --------------------------------------------------------------------------
def _cases(rng, k=1500):
    cases = []
    for _ in range(k):
        ml = int(rng.integers(0, L + 1))
        dot = int(rng.integers(-ml, ml + 1))
        if (dot - ml) % 2:
            dot += 1 if dot < ml else -1
        cases.append((ml, dot))
    for ml in (0, 8, 800, 10368, 12800):
        for hd8 in (3 * ml, 3 * ml - 1, 3 * ml + 1):
            if hd8 >= 0 and hd8 % 8 == 0:
                cases.append((ml, ml - 2 * (hd8 // 8)))
    cases += [(12800, 12800), (12800, -12800), (1, 1), (1, -1), (3, 1), (4, 2), (5, 1), (5, 3)]
    return cases


def _split(rng, v, bits):
    mod = 1 << bits
    c = rng.integers(0, mod, 3, dtype=np.uint64)
    c[2] = (v - int(c[0]) - int(c[1])) % mod
    return c.astype(np.uint32)


@pytest.mark.parametrize("variant", [orc.CMPV_PLAIN, orc.CMPV_LIFT18, orc.CMPV_CONST32])
def test_compare_variant_random_and_boundaries(variant):
    rng = np.random.default_rng(40 + variant)
    want_counts = {
        # AND gates, then bits sent by parties 0, 1, 2 per comparison:
        # PLAIN: MSB over 16 bits, 2*16 - 3 = 29 gates.
        orc.CMPV_PLAIN: [29, 29, 29, 29],
        # LIFT18: Lift 33 + MSB over 18 bits 33; 3OT of the two injections
        # (k = 1, 2): party 0 sends 2k each, parties 1 and 2 k each.
        orc.CMPV_LIFT18: [66, 66 + 6, 66 + 3, 66 + 3],
        # CONST32: MSB over 32 bits, 61 gates, nothing else.
        orc.CMPV_CONST32: [61, 61, 61, 61],
    }[variant]
    want_depth = {orc.CMPV_PLAIN: 15, orc.CMPV_LIFT18: 17 + 2 + 17, orc.CMPV_CONST32: 31}[variant]
    for ml, dot in _cases(rng):
        d_bits = 32 if (variant == orc.CMPV_CONST32 and rng.integers(2)) else 16
        d = _split(rng, dot, d_bits)
        x = _split(rng, ml, 32 if variant == orc.CMPV_CONST32 else 16)
        m, yo, counts, depth = orc.t_compare_variant(variant, d, x, ml, int(rng.integers(1 << 62)))
        if variant == orc.CMPV_PLAIN:
            want_y = (ml // 4 - dot) % (1 << 16)
        elif variant == orc.CMPV_LIFT18:
            want_y = (ml - 4 * dot) % (1 << 18)
        else:
            want_y = ((1 << 14) * ml - (1 << 16) * dot) % (1 << 32)
        assert yo == want_y, (variant, ml, dot)
        assert m == int(4 * dot > ml), (variant, ml, dot)
        assert list(counts) == want_counts
        assert depth == want_depth


def test_table3_communication():
    # Sec. 6.2, Table 3: kB sent per party for 100k comparisons.
    per = {}
    for v in (orc.CMPV_PLAIN, orc.CMPV_CONST32):
        _, _, counts, _ = orc.t_compare_variant(v, [0, 0, 0], [0, 0, 0], 0, 1)
        per[v] = int(counts[1])
    # 29 and 61 bits give 362.5 and 762.5 kB; the table prints 362 and 763.
    assert abs(per[orc.CMPV_PLAIN] * 100_000 / 8 / 1000 - 362) <= 0.5     # Plain Mask
    assert abs(per[orc.CMPV_CONST32] * 100_000 / 8 / 1000 - 763) <= 0.5   # ConstLift / NoLift


def test_lift18_lifted_value_is_exact():
    # Lift with m = 2 on every ml: the value whose MSB is taken is ml - 4 dot
    # mod 2^18 for shares whose integer sum spans 0 .. 3 (2^16 - 1).
    rng = np.random.default_rng(7)
    for ml in range(0, L + 1, 37):
        for _ in range(3):
            x = _split(rng, ml, 16)
            d = _split(rng, 0, 16)
            _, yo, _, _ = orc.t_compare_variant(orc.CMPV_LIFT18, d, x, 0, int(rng.integers(1 << 62)))
            assert yo == ml


# --------------------------------------------------------------------------
# dot products over Z_2^32
# --------------------------------------------------------------------------
def test_share32_and_local_dot32(keys):
    dealer, party = keys
    dc, dm = wl.gen_codes(31, 0, 6)
    qc, qm = wl.gen_codes(31, 0, 2, query=True)
    rot = [-3, 0, 7]
    dsh = orc.share32(dealer, orc.DOM_SHARE32_DB, dc, dm, 0)
    qsh = orc.share32(dealer, orc.DOM_SHARE32_QUERY, qc, qm, 0)
    # components sum to the masked-bit encoding mod 2^32 (numpy, from the bits)
    bits = lambda w: ((w[:, :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).reshape(w.shape[0], -1)
    c, m = bits(dc).astype(np.int64), bits(dm).astype(np.int64)
    enc = np.stack([m - 2 * (c & m), m], axis=1) % (1 << 32)
    assert np.array_equal(dsh.astype(np.uint64).sum(axis=2) % (1 << 32), enc)
    assert not np.array_equal(dsh[:, :, 0], dsh[:, :, 1])
    # party dots sum to <c', C'> = ml - 2 hd and to ml, mod 2^32
    hd, ml, _, _ = orc.plain(qc, qm, rot, dc, dm)
    zc = np.zeros(ml.shape, dtype=np.uint64)
    zm = np.zeros(ml.shape, dtype=np.uint64)
    zs = []
    for p in range(3):
        a, b = orc.local_dot32(p, qsh, rot, dsh)
        zc += a
        zm += b
        zs.append((a, b))
    assert np.array_equal(zc % (1 << 32), (ml - 2 * hd).astype(np.int64) % (1 << 32))
    assert np.array_equal(zm % (1 << 32), ml.astype(np.uint64))
    # resharing keeps the sum and re-randomises
    zc3 = np.stack([z[0] for z in zs])
    zm3 = np.stack([z[1] for z in zs])
    rc, rm = orc.reshare32(party, zc3, zm3, 2, rot, 5, 0)
    assert np.array_equal(rc.astype(np.uint64).sum(axis=0) % (1 << 32), zc % (1 << 32))
    assert np.array_equal(rm.astype(np.uint64).sum(axis=0) % (1 << 32), zm % (1 << 32))
    assert not np.array_equal(rc, zc3)
    only_mask = orc.reshare32(party, None, zm3, 2, rot, 5, 0)
    assert only_mask[0] is None and np.array_equal(only_mask[1], rm)


# --------------------------------------------------------------------------
# whole protocol per comparison setting vs the plaintext decision
# --------------------------------------------------------------------------
def _case(seed=23, n=70):
    dc, dm = wl.gen_codes(seed, 0, n)
    qc, qm = wl.gen_codes(seed, 0, 4, query=True)
    rot = [-1, 0, 2]
    qc[0], qm[0] = wl.plant(seed, 0, dc[7], dm[7], 2, h=0.2)
    qc[1], qm[1] = wl.plant(seed, 1, dc[33], dm[33], -1, exact="eq")
    qc[2], qm[2] = wl.plant(seed, 2, dc[65], dm[65], 0, exact="lt")
    return qc, qm, rot, dc, dm


@pytest.mark.parametrize("setting", ["plain", "lift18", "constlift", "nolift"])
def test_protocol_settings_match_plaintext(keys, setting):
    dealer, party = keys
    qc, qm, rot, dc, dm = _case()
    hd, ml, match, dup = orc.plain(qc, qm, rot, dc, dm)
    res = orc.protocol(dealer, party, qc, qm, rot, dc, dm, qid_base=100, first_entry=0, compare_setting=setting)
    n = dc.shape[0]
    mw = orc.open_xor(res["match"])
    got = np.array([[(int(mw[r_, j // 64]) >> (j % 64)) & 1 for j in range(n)] for r_ in range(mw.shape[0])])
    assert np.array_equal(got, match)
    assert match.sum() == 2
    assert np.array_equal(orc.open_xor(res["dup"]), dup)
    dot = (ml - 2 * hd).astype(np.int64)
    mlv = ml.astype(np.int64)
    if setting == "plain":
        want_y = (mlv // 4 - dot) % (1 << 16)
    elif setting == "lift18":
        want_y = (mlv - 4 * dot) % (1 << 18)
    else:
        want_y = ((1 << 14) * mlv - (1 << 16) * dot) % (1 << 32)
    bits = {"plain": 16, "lift18": 18}.get(setting, 32)
    y = res["y"].astype(np.uint64).sum(axis=0) % (1 << bits)
    assert np.array_equal(y, want_y.astype(np.uint64))
