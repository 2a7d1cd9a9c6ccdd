"""Pins of the CPU oracle against facts fixed outside it.

Each check ties an oracle function to something it does not compute itself:
a library implementation (OpenSSL ChaCha20), closed forms and identities the
paper states (App. B masked-bit identities, Eq. (1), Lemma 2, the AND-gate
and round counts of Sec. 4.3.1 / Sec. 5.2), brute force over tiny rings, and
inputs whose answer is known by construction (identical, complementary,
disjoint and planted codes).  The full shared protocol is then pinned to the
plaintext decision.
"""
import ctypes
import ctypes.util
import itertools

import numpy as np
import pytest

import oracle as orc
import workload as wl

L = 12800


# --------------------------------------------------------------------------
# PRF: ChaCha block function vs OpenSSL's ChaCha20
# --------------------------------------------------------------------------
def _openssl_chacha20_block(key: bytes, counter: int, nonce: bytes) -> bytes:
    name = ctypes.util.find_library("crypto") or "libcrypto.so.3"
    c = ctypes.CDLL(name)
    c.EVP_chacha20.restype = ctypes.c_void_p
    c.EVP_CIPHER_CTX_new.restype = ctypes.c_void_p
    ctx = c.EVP_CIPHER_CTX_new()
    iv = counter.to_bytes(4, "little") + nonce
    assert c.EVP_EncryptInit_ex(ctypes.c_void_p(ctx), ctypes.c_void_p(c.EVP_chacha20()), None, key, iv) == 1
    out = ctypes.create_string_buffer(80)
    outl = ctypes.c_int(0)
    assert c.EVP_EncryptUpdate(ctypes.c_void_p(ctx), out, ctypes.byref(outl), bytes(64), 64) == 1
    c.EVP_CIPHER_CTX_free(ctypes.c_void_p(ctx))
    return out.raw[:64]


def test_chacha20_matches_openssl():
    rng = np.random.default_rng(1)
    for _ in range(20):
        key = rng.integers(0, 256, 32, dtype=np.uint8).tobytes()
        counter = int(rng.integers(0, 2**32))
        nonce = rng.integers(0, 256, 12, dtype=np.uint8).tobytes()
        words = [counter] + [int.from_bytes(nonce[4 * i:4 * i + 4], "little") for i in range(3)]
        mine = orc.chacha_block(key, 20, words).astype("<u4").tobytes()
        assert mine == _openssl_chacha20_block(key, counter, nonce)


def test_chacha_zero_rounds_is_doubled_state():
    # With no rounds the feed-forward adds the input state to itself.
    key = bytes(range(32))
    out = orc.chacha_block(key, 0, [5, 6, 7, 8])
    const = [0x61707865, 0x3320646E, 0x79622D32, 0x6B206574]
    kw = [int.from_bytes(key[4 * i:4 * i + 4], "little") for i in range(8)]
    state = np.array(const + kw + [5, 6, 7, 8], dtype=np.uint64)
    assert np.array_equal(out.astype(np.uint64), (2 * state) & 0xFFFFFFFF)


def test_prf_stream_addressing():
    key = bytes(range(1, 33))
    st = (3 << 56) | (77 << 8) | 16
    b = orc.prf_block(key, st, 9)
    ref = orc.chacha_block(key, 12, [9, 0, st & 0xFFFFFFFF, st >> 32])
    assert np.array_equal(b, ref)
    # u16 i of a stream: block i>>5, word (i>>1)&15, half i&1
    for i in (0, 1, 31, 32, 300, 12799):
        blk = orc.prf_block(key, st, i >> 5)
        w = int(blk[(i >> 1) & 15])
        assert orc.lib().orc_prf_u16(key, ctypes.c_uint64(st), ctypes.c_uint64(i)) == ((w >> 16) if i & 1 else (w & 0xFFFF))


# --------------------------------------------------------------------------
# O1 plaintext decision (Alg. 1)
# --------------------------------------------------------------------------
def _db(seed, n):
    return wl.gen_codes(seed, 0, n)


def test_plain_special_cases():
    dc, dm = _db(11, 4)
    full = np.full((1, 200), np.uint64(2**64 - 1))
    zero = np.zeros((1, 200), dtype=np.uint64)
    # identical code, query mask all ones: hd = 0, ml = |M|; match iff ml > 0
    hd, ml, m, _ = orc.plain(dc[:1], full, [0], dc[:1], dm[:1])
    assert hd[0, 0] == 0 and m[0, 0] == 1 and ml[0, 0] > 10000
    # complement: hd = ml, never a match
    hd, ml, m, _ = orc.plain(~dc[:1], full, [0], dc[:1], dm[:1])
    assert hd[0, 0] == ml[0, 0] and m[0, 0] == 0
    # all-ones masks on both sides: ml = l exactly
    hd, ml, m, _ = orc.plain(dc[:1], full, [0], dc[1:2], full)
    assert ml[0, 0] == L
    # disjoint masks: ml = 0 -> no match (0/0 read as "not similar")
    hd, ml, m, d = orc.plain(dc[:1], zero, [0], dc[:1], dm[:1])
    assert ml[0, 0] == 0 and hd[0, 0] == 0 and m[0, 0] == 0 and d[0] == 0


def test_plain_unmasked_matches_eq1():
    # Eq. (1): with full masks hd(a,b) = |a| + |b| - 2<a,b>.
    dc, _ = _db(12, 6)
    full = np.full((6, 200), np.uint64(2**64 - 1))
    hd, _, _, _ = orc.plain(dc[:3], full[:3], [0], dc[3:], full[3:])
    a = wl.unpack(dc).astype(np.int64)
    for i in range(3):
        for j in range(3):
            assert hd[i, j] == a[i].sum() + a[3 + j].sum() - 2 * int(a[i] @ a[3 + j])


def test_plain_random_pairs_statistics():
    dc, dm = _db(13, 200)
    qc, qm = wl.gen_codes(13, 0, 4, query=True)
    hd, ml, m, d = orc.plain(qc, qm, [0], dc, dm)
    frac = hd / ml
    assert abs(frac.mean() - 0.5) < 0.002          # independent Bernoulli(1/2) bits
    assert abs(ml.mean() / L - 0.81) < 0.003        # Bernoulli(0.9) AND Bernoulli(0.9)
    assert m.sum() == 0 and d.sum() == 0            # HD 0.5 is ~25 sigma above 0.375


@pytest.mark.parametrize("s", [-15, -4, 0, 1, 15])
def test_plain_planted_exact_hd_and_rotation(s):
    dc, dm = _db(14, 8)
    e = 5
    qc, qm = wl.plant(14, 3, dc[e], dm[e], s, h=0.2)
    hd, ml, m, d = orc.plain(qc[None], qm[None], list(range(-15, 16)), dc, dm)
    row = s + 15
    # the planted rotation has exactly round(0.2*ml) flips inside the combined mask
    assert hd[row, e] == int(np.floor(0.2 * ml[row, e] + 0.5))
    assert m[row, e] == 1 and d[0] == 1
    assert m.sum() == 1


def test_plain_rotation_is_relabelling():
    # querying rot_s(q) at rotation 0 equals querying q at rotation s
    dc, dm = _db(15, 5)
    qc, qm = wl.gen_codes(15, 0, 1, query=True)
    for s in (-7, 3, 15):
        rc = wl.pack(wl.rotate_bits(wl.unpack(qc[0]), s))[None]
        rm = wl.pack(wl.rotate_bits(wl.unpack(qm[0]), s))[None]
        a = orc.plain(rc, rm, [0], dc, dm)
        b = orc.plain(qc, qm, [s], dc, dm)
        for x, y in zip(a[:3], b[:3]):
            assert np.array_equal(x, y)
    # a full turn of 200 columns is the identity
    a = orc.plain(qc, qm, [0], dc, dm)
    rc = wl.pack(wl.rotate_bits(wl.unpack(qc[0]), 200))[None]
    rm = wl.pack(wl.rotate_bits(wl.unpack(qm[0]), 200))[None]
    b = orc.plain(rc, rm, [0], dc, dm)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_plain_threshold_boundaries():
    dc, dm = _db(16, 3)
    qe, me = wl.plant(16, 1, dc[0], dm[0], 2, exact="eq")
    ql, ml_ = wl.plant(16, 2, dc[1], dm[1], -3, exact="lt")
    hd, ml, m, _ = orc.plain(np.stack([qe, ql]), np.stack([me, ml_]), [2, -3], dc, dm)
    # row 0 = query 0 at rotation 2 vs entry 0: 8 hd == 3 ml -> not a match (strict <)
    assert 8 * hd[0, 0] == 3 * ml[0, 0] and m[0, 0] == 0
    # row 3 = query 1 at rotation -3 vs entry 1: 8 hd == 3 ml - 1 -> match
    assert 8 * hd[3, 1] == 3 * ml[3, 1] - 1 and m[3, 1] == 1


# --------------------------------------------------------------------------
# masked bit encoding (Sec. 4.1.1, App. B)
# --------------------------------------------------------------------------
def _signed(u):
    u = np.asarray(u, dtype=np.int64)
    return np.where(u >= 32768, u - 65536, u)


def test_masked_bit_truth_table():
    for a, ma, b, mb in itertools.product((0, 1), repeat=4):
        ca = np.zeros(200, np.uint64)
        cm = np.zeros(200, np.uint64)
        ca[0] = a
        cm[0] = ma
        xa, xma = orc.encode(ca, cm)
        ca[0] = b
        cm[0] = mb
        xb, _ = orc.encode(ca, cm)
        sa, sb = int(_signed(xa[0])), int(_signed(xb[0]))
        # (T,U,F) = (-1,0,1)
        assert sa == (0 if not ma else (-1 if a else 1))
        assert xma[0] == ma
        # a' b' is +1 (agree), -1 (differ) under both masks, 0 otherwise
        assert sa * sb == ma * mb * (1 - 2 * (a ^ b))
        # a'^2 extracts the mask; CountOnes(a') = (a'a' - a')/2
        assert sa * sa == ma and (sa * sa - sa) // 2 == (a & ma)


def test_encoded_dot_is_ml_minus_2hd():
    dc, dm = _db(17, 3)
    qc, qm = wl.gen_codes(17, 0, 2, query=True)
    hd, ml, _, _ = orc.plain(qc, qm, [0], dc, dm)
    for i in range(2):
        xq, _ = orc.encode(qc[i], qm[i])
        for j in range(3):
            xd, _ = orc.encode(dc[j], dm[j])
            dot = int((_signed(xq) * _signed(xd)).sum())
            assert dot == ml[i, j] - 2 * hd[i, j]           # App. B
            assert (hd[i, j] < 0.375 * ml[i, j]) == (dot > 0.25 * ml[i, j])


# --------------------------------------------------------------------------
# threshold reduction (Sec. 5, Lemma 2)
# --------------------------------------------------------------------------
def test_lemma2_exhaustive():
    # For every ml in [0, 12800] and dot in [-ml, ml] with dot = ml (mod 2):
    # MSB_32(2^14 ml - 2^16 dot) == (4 dot > ml) == (8 hd < 3 ml).
    assert (1 << 16) * L < (1 << 32) // 4
    ml = np.arange(0, L + 1, dtype=np.int64)
    for dot0 in range(-L, L + 1, 97):
        dot = np.arange(dot0, min(dot0 + 97, L + 1), dtype=np.int64)[:, None]
        ok = (np.abs(dot) <= ml) & (((dot - ml) & 1) == 0)
        y = ((1 << 14) * ml - (1 << 16) * dot) & 0xFFFFFFFF
        msb = (y >> 31) & 1
        hd = (ml - dot) // 2
        want = (4 * dot > ml) & ok
        assert np.array_equal((msb == 1) & ok, want)
        assert np.array_equal((8 * hd < 3 * ml) & ok, want)


# --------------------------------------------------------------------------
# sharing, local dot, reshare (App. C)
# --------------------------------------------------------------------------
def test_share_reconstructs_and_local_dots_sum(keys):
    dealer, party = keys
    dc, dm = _db(18, 5)
    qc, qm = wl.gen_codes(18, 0, 2, query=True)
    dsh = orc.share(dealer, orc.DOM_SHARE_DB, dc, dm, 0)
    qsh = orc.share(dealer, orc.DOM_SHARE_QUERY, qc, qm, 0)
    for e in range(5):
        xc, xm = orc.encode(dc[e], dm[e])
        assert np.array_equal(orc.open_add(dsh[e, 0], 16), xc)
        assert np.array_equal(orc.open_add(dsh[e, 1], 16), xm)
    # the components are uniform-looking, not the secret
    assert abs(dsh[:, :, 0].mean() - 32767.5) < 200
    rot = [-2, 0, 9]
    hd, ml, _, _ = orc.plain(qc, qm, rot, dc, dm)
    z = [orc.local_dot(p, qsh, rot, dsh) for p in range(3)]
    zc = np.stack([a for a, _ in z])
    zm = np.stack([b for _, b in z])
    assert np.array_equal(orc.open_add(zc, 16), ((ml - 2 * hd) & 0xFFFF).astype(np.uint16))
    assert np.array_equal(orc.open_add(zm, 16), ml.astype(np.uint16))
    rc, rm = orc.reshare(party, zc, zm, 2, rot, 0, 0)
    assert np.array_equal(orc.open_add(rc, 16), orc.open_add(zc, 16))
    assert np.array_equal(orc.open_add(rm, 16), orc.open_add(zm, 16))
    assert (rc != zc).mean() > 0.99     # re-randomised


# --------------------------------------------------------------------------
# boolean sub-protocols (App. D) by brute force on tiny rings
# --------------------------------------------------------------------------
def test_and_gate_exhaustive():
    for x in itertools.product((0, 1), repeat=3):
        for y in itertools.product((0, 1), repeat=3):
            for f in itertools.product((0, 1), repeat=3):
                z = orc.t_and(x, y, f)
                assert (z[0] ^ z[1] ^ z[2]) == ((x[0] ^ x[1] ^ x[2]) & (y[0] ^ y[1] ^ y[2]))


def test_full_adder_exhaustive():
    for a, b, c in itertools.product(itertools.product((0, 1), repeat=3), repeat=3):
        for f in ((0, 0, 0), (1, 0, 1), (1, 1, 1)):
            s, o = orc.t_fa(a, b, c, f)
            A, B, C = (v[0] ^ v[1] ^ v[2] for v in (a, b, c))
            assert (s[0] ^ s[1] ^ s[2]) == A ^ B ^ C
            assert (o[0] ^ o[1] ^ o[2]) == int(A + B + C >= 2)


@pytest.mark.parametrize("k", [4, 6])
def test_bit_extract_exhaustive_toy_ring(k):
    m = k - 1
    rng = np.random.default_rng(k)
    for x0 in range(1 << k):
        for x1 in range(1 << k):
            for x2 in range(0, 1 << k, 1 if k == 4 else 7):
                bits, _, ands, depth = orc.t_bit_extract(k, m, x0, x1, x2, int(rng.integers(1 << 62)))
                s = x0 + x1 + x2
                assert all(int(bits[i]) == (s >> i) & 1 for i in range(m + 1))
                assert ands == 2 * k - 3 and depth[m] == k - 1


def test_bit_extract_gate_and_round_counts():
    # Sec. 4.3.1: MSB of a 16-bit ring with a ripple-carry adder takes 29 AND
    # gates in 15 rounds; Sec. 5.2: 2k-3 gates and k-1 rounds for k bits.
    for k, want in ((16, 29), (32, 61)):
        bits, _, ands, depth = orc.t_bit_extract(k, k - 1, 12345, 54321, 999, 7)
        assert ands == want == 2 * k - 3
        assert depth[k - 1] == k - 1
        s = (12345 + 54321 + 999) & ((1 << k) - 1)
        assert int(bits[k - 1]) == (s >> (k - 1)) & 1


def test_bit_inject_exhaustive():
    rng = np.random.default_rng(3)
    for k in (1, 2, 15, 16):
        for x in itertools.product((0, 1), repeat=3):
            for _ in range(8):
                c0, c2, w0, w1 = (int(v) for v in rng.integers(0, 2**32, 4))
                out, bits = orc.t_bit_inject(x, k, c0, c2, w0, w1)
                assert int(out.astype(np.uint64).sum()) % (1 << k) == x[0] ^ x[1] ^ x[2]
                assert list(bits) == [2 * k, k, k]


def test_compare_one_random_and_boundaries():
    rng = np.random.default_rng(4)
    cases = []
    for _ in range(3000):
        ml = int(rng.integers(0, L + 1))
        dot = int(rng.integers(-ml, ml + 1))
        if (dot - ml) % 2:
            dot += 1 if dot < ml else -1
        cases.append((ml, dot))
    for ml in (0, 8, 800, 10368, 12800):     # 8 hd = 3 ml and 8 hd = 3 ml - 1 (when integral)
        for hd8 in (3 * ml, 3 * ml - 1):
            if hd8 >= 0 and hd8 % 8 == 0:
                cases.append((ml, ml - 2 * (hd8 // 8)))
    cases += [(12800, 12800), (12800, -12800), (1, 1), (1, -1), (3, 1)]
    for ml, dot in cases:
        x = rng.integers(0, 65536, 3).astype(np.uint16)
        x[2] = (ml - int(x[0]) - int(x[1])) & 0xFFFF
        d = rng.integers(0, 65536, 3).astype(np.uint16)
        d[2] = (dot - int(d[0]) - int(d[1])) & 0xFFFF
        m, mlo, yo, counts, depth = orc.t_compare_one(d, x, int(rng.integers(1 << 62)))
        assert mlo == ml                                    # Lift is exact
        assert yo == ((1 << 14) * ml - (1 << 16) * dot) & 0xFFFFFFFF
        assert m == int(4 * dot > ml)
        assert counts[0] == 33 + 61
        assert list(counts[1:]) == [94 + 62, 94 + 31, 94 + 31]
        assert depth == 17 + 2 + 31


# --------------------------------------------------------------------------
# OR-tree (Sec. 4.2) and the whole protocol vs the plaintext decision
# --------------------------------------------------------------------------
@pytest.mark.parametrize("nq,r,n", [(1, 1, 1), (2, 3, 64), (3, 2, 130), (2, 5, 700)])
def test_or_tree_opens_to_or(keys, nq, r, n):
    _, party = keys
    rng = np.random.default_rng(n)
    nw = (n + 63) // 64
    bits = (rng.random((nq * r, n)) < 1.5 / (r * n)).astype(np.uint8)
    words = np.zeros((nq * r, nw), dtype=np.uint64)
    for w in range(nw):
        chunk = bits[:, 64 * w:64 * w + 64]
        for o in range(chunk.shape[1]):
            words[:, w] |= chunk[:, o].astype(np.uint64) << np.uint64(o)
    c0 = rng.integers(0, 2**63, words.shape, dtype=np.uint64)
    c1 = rng.integers(0, 2**63, words.shape, dtype=np.uint64)
    tail = np.uint64((1 << (n % 64)) - 1) if n % 64 else np.uint64(2**64 - 1)
    c0[:, -1] &= tail
    c1[:, -1] &= tail
    comps = np.stack([c0, c1, words ^ c0 ^ c1])
    dup, nand = orc.or_tree(party, comps, nq, r, 0)
    want = bits.reshape(nq, r * n).max(axis=1)
    assert np.array_equal(dup[0] ^ dup[1] ^ dup[2], want)


def _small_case(seed=21, n=40):
    dc, dm = wl.gen_codes(seed, 0, n)
    qc, qm = wl.gen_codes(seed, 0, 4, query=True)
    rot = [-1, 0, 2]
    qc[0], qm[0] = wl.plant(seed, 0, dc[7], dm[7], 2, h=0.2)
    qc[1], qm[1] = wl.plant(seed, 1, dc[33], dm[33], -1, exact="eq")
    qc[2], qm[2] = wl.plant(seed, 2, dc[12], dm[12], 0, exact="lt")
    return qc, qm, rot, dc, dm


def test_protocol_matches_plaintext(keys):
    dealer, party = keys
    qc, qm, rot, dc, dm = _small_case()
    hd, ml, match, dup = orc.plain(qc, qm, rot, dc, dm)
    res = orc.protocol(dealer, party, qc, qm, rot, dc, dm, qid_base=100, first_entry=0)
    n = dc.shape[0]
    mw = orc.open_xor(res["match"])
    got = np.array([[(int(mw[r_, j // 64]) >> (j % 64)) & 1 for j in range(n)] for r_ in range(mw.shape[0])])
    assert np.array_equal(got, match)
    assert match.sum() == 2 and match[0 * 3 + 2, 7] == 1 and match[2 * 3 + 1, 12] == 1
    assert np.array_equal(orc.open_xor(res["dup"]), dup)
    assert list(dup) == [1, 0, 1, 0]
    # lifted ml opens to ml; y opens to 2^14 ml - 2^16 dot
    assert np.array_equal(orc.open_add(res["ml_lift"], 32), ml.astype(np.uint32))
    want_y = (((1 << 14) * ml.astype(np.int64) - (1 << 16) * (ml - 2 * hd)) & 0xFFFFFFFF).astype(np.uint32)
    assert np.array_equal(orc.open_add(res["y"], 32), want_y)
    # replicated consistency is structural; counts per comparison
    ncmp = match.size
    assert res["counts"][0] == 94 * ncmp
    assert list(res["counts"][1:]) == [156 * ncmp, 125 * ncmp, 125 * ncmp]


def test_protocol_is_batch_independent(keys):
    # Randomness is addressed by (query id, rotation, entry, gate): evaluating a
    # subset of queries / a 64-aligned entry range gives the same components.
    dealer, party = keys
    qc, qm, rot, dc, dm = _small_case(seed=22, n=130)
    full = orc.protocol(dealer, party, qc, qm, rot, dc, dm, qid_base=10, first_entry=0)
    part = orc.protocol(dealer, party, qc[2:3], qm[2:3], rot, dc[64:], dm[64:], qid_base=12, first_entry=64)
    assert np.array_equal(part["match"], full["match"][:, 6:9, 1:])
    assert np.array_equal(part["rep_code"], full["rep_code"][:, 6:9, 64:])


def test_protocol_is_thread_count_independent(keys):
    # The oracle's loops are split over host threads only by output element:
    # one thread gives the same components as all of them.
    dealer, party = keys
    qc, qm, rot, dc, dm = _small_case(seed=23, n=70)
    many = orc.protocol(dealer, party, qc, qm, rot, dc, dm, qid_base=10, first_entry=0)
    old = orc.set_threads(1)
    try:
        assert orc.threads() == 1
        one = orc.protocol(dealer, party, qc, qm, rot, dc, dm, qid_base=10, first_entry=0)
    finally:
        orc.set_threads(old)
    assert orc.threads() == old
    for k in ("match", "rep_code", "rep_mask", "dup"):
        assert np.array_equal(one[k], many[k]), k
