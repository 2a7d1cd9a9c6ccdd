"""Pins of the oracle's Shamir sharing over the Galois ring Z_2^16[X]/(X^2-X-1)
(Sec. 4.3.2) against facts fixed outside it.

* The ring product is pinned by the structure that defines the quotient ring:
  it is bilinear over Z_2^16, 1 is its identity, X * X = X + 1, and it is
  commutative and associative.  A bilinear map is fixed by its values on the
  basis {1, X}, so these checks pin every term.
* The paper's observation that the constant term of (c0 + c1 X)(d0 + d1 X) is
  the dot product c0 d0 + c1 d1.
* Inverses and the exceptional sequence: u * u^-1 = 1, non-units (both
  coefficients even) have none, and all pairwise differences of
  {0, alpha_0, alpha_1, alpha_2} are units.
* Lagrange coefficients: interpolating random degree-2 polynomials over the
  ring at 0 from the three parties' points returns their constant term.
* Shares: any two parties' shares of a pair interpolate (degree 1) to the
  encoded bits; the three lie on one line.
* End to end: the three parties' local dot shares sum to the plaintext
  <c', C'> = ml - 2 hd and ml (popcounts of the packed codes), over several
  rotations, and the shared protocol on Galois shares opens the plaintext
  match bits.
"""
import numpy as np

import oracle as orc
import workload as wl

M16 = 0xFFFF
rng = np.random.default_rng(20240507)


def mul(a, b):
    return tuple(int(v) for v in orc.t_gr_mul(a, b))


def add(a, b):
    return ((a[0] + b[0]) & M16, (a[1] + b[1]) & M16)


def sub(a, b):
    return ((a[0] - b[0]) & M16, (a[1] - b[1]) & M16)


def scal(k, a):
    return ((k * a[0]) & M16, (k * a[1]) & M16)


def rand_el():
    return tuple(int(v) for v in rng.integers(0, 1 << 16, 2))


ONE, X = (1, 0), (0, 1)


def test_product_is_the_quotient_ring_product():
    assert mul(ONE, ONE) == ONE
    assert mul(ONE, X) == X and mul(X, ONE) == X
    assert mul(X, X) == (1, 1)                      # X^2 = X + 1
    for _ in range(200):
        a, b, c = rand_el(), rand_el(), rand_el()
        k = int(rng.integers(0, 1 << 16))
        assert mul(add(a, b), c) == add(mul(a, c), mul(b, c))      # additive in each argument
        assert mul(a, add(b, c)) == add(mul(a, b), mul(a, c))
        assert mul(scal(k, a), b) == scal(k, mul(a, b))            # Z_2^16-linear
        assert mul(a, b) == mul(b, a)
        assert mul(mul(a, b), c) == mul(a, mul(b, c))


def test_constant_term_is_the_dot_product():
    for _ in range(200):
        a, b = rand_el(), rand_el()
        assert mul(a, b)[0] == (a[0] * b[0] + a[1] * b[1]) & M16


def test_inverses_and_exceptional_sequence():
    for _ in range(200):
        a = rand_el()
        inv = orc.t_gr_inv(a)
        if a[0] % 2 == 0 and a[1] % 2 == 0:
            assert inv is None
        else:
            assert mul(a, tuple(int(v) for v in inv)) == ONE
    alpha, _ = orc.galois_points()
    pts = [(0, 0)] + [tuple(int(v) for v in alpha[p]) for p in range(3)]
    for i in range(4):
        for j in range(i + 1, 4):
            assert orc.t_gr_inv(sub(pts[i], pts[j])) is not None, (pts[i], pts[j])


def test_lagrange_coefficients_interpolate_degree_two_at_zero():
    alpha, lam = orc.galois_points()
    alpha = [tuple(int(v) for v in a) for a in alpha]
    lam = [tuple(int(v) for v in l) for l in lam]
    for _ in range(100):
        f = [rand_el() for _ in range(3)]
        acc = (0, 0)
        for p in range(3):
            y = add(f[0], add(mul(f[1], alpha[p]), mul(f[2], mul(alpha[p], alpha[p]))))
            acc = add(acc, mul(lam[p], y))
        assert acc == f[0]


def test_shares_interpolate_to_the_encoded_pairs():
    dealer = bytes(range(32))
    codes, masks = wl.gen_codes(11, 0, 3)
    sh = orc.galois_share(dealer, orc.DOM_GALOIS_DB, codes, masks, 40)
    alpha, _ = orc.galois_points()
    alpha = [tuple(int(v) for v in a) for a in alpha]
    for e in range(3):
        xc, xm = orc.encode(codes[e], masks[e])
        for vec, x in ((0, xc), (1, xm)):
            for i in rng.integers(0, 6400, 40):
                s = [(int(sh[e, vec, p, 2 * i]), int(sh[e, vec, p, 2 * i + 1])) for p in range(3)]
                for p, q in ((0, 1), (1, 2), (0, 2)):
                    # g = (alpha_q s_p - alpha_p s_q) / (alpha_q - alpha_p)
                    inv = tuple(int(v) for v in orc.t_gr_inv(sub(alpha[q], alpha[p])))
                    g = mul(sub(mul(alpha[q], s[p]), mul(alpha[p], s[q])), inv)
                    assert g == (int(x[2 * i]), int(x[2 * i + 1]))
    # different ids draw different randomness: shares differ, secrets agree
    sh2 = orc.galois_share(dealer, orc.DOM_GALOIS_DB, codes, masks, 41)
    assert not np.array_equal(sh, sh2)


def test_local_dot_shares_sum_to_plaintext_dots():
    dealer = bytes(range(1, 33))
    rot = [-3, 0, 2, 15]
    dc, dm = wl.gen_codes(12, 0, 6)
    qc, qm = wl.gen_codes(12, 0, 2, query=True)
    qc[1], qm[1] = wl.plant(12, 1, dc[4], dm[4], 2, h=0.2)
    qsh = orc.galois_share(dealer, orc.DOM_GALOIS_QUERY, qc, qm, 7)
    dsh = orc.galois_share(dealer, orc.DOM_GALOIS_DB, dc, dm, 0)
    zc = np.zeros((8, 6), dtype=np.uint16)
    zm = np.zeros((8, 6), dtype=np.uint16)
    parts = []
    for p in range(3):
        c, m = orc.galois_local_dot(p, qsh, rot, dsh)
        parts.append(c)
        zc += c
        zm += m
    hd, ml, match, _ = orc.plain(qc, qm, rot, dc, dm)
    assert np.array_equal(zm, ml.astype(np.uint16))
    assert np.array_equal(zc, (ml.astype(np.int64) - 2 * hd.astype(np.int64)).astype(np.uint16))
    assert match[1 * 4 + 2, 4]                      # the planted pair
    # each party's share alone is not the dot
    assert not np.array_equal(parts[0], zc)


def test_galois_protocol_opens_plaintext_matches(keys):
    dealer, party = keys
    rot = [-1, 0, 1]
    dc, dm = wl.gen_codes(13, 0, 70)
    qc, qm = wl.gen_codes(13, 0, 3, query=True)
    qc[0], qm[0] = wl.plant(13, 0, dc[66], dm[66], 1, h=0.3)
    qc[2], qm[2] = wl.plant(13, 2, dc[5], dm[5], -1, exact="eq")    # 8 hd = 3 ml: not a match
    res = orc.protocol(dealer, party, qc, qm, rot, dc, dm, qid_base=0, first_entry=0, scheme="galois")
    _, _, match, dup = orc.plain(qc, qm, rot, dc, dm)
    nw = (70 + 63) // 64
    bits = np.unpackbits(orc.open_xor(res["match"]).view(np.uint8), bitorder="little").reshape(9, nw * 64)[:, :70]
    assert np.array_equal(bits.astype(bool), match)
    assert np.array_equal(orc.open_xor(res["dup"]).astype(bool), dup)
    assert dup[0] and not dup[2]
