"""Pins of the oracle's in-batch matching and decision combining (Sec. 6.4:
the queries of a batch are matched with each other as well as with the
database; a person's query covers both eyes).

* The OR gate on shared bits opens to the OR of the opened inputs, for every
  combination of component bits (brute force).
* The in-batch mask keeps exactly the columns j < qi of each row.
* End to end: with the batch part, a query's opened result equals the
  plaintext decision against the database plus the batch's earlier queries
  (O1 on the concatenated entries); later queries never count.
* Both eyes: with groups of two queries (a person's eyes), the mask keeps
  exactly the columns of earlier persons; the pair OR opens to the OR of
  each person's two eyes (brute force over all component bits); end to end,
  a person's opened decision is the plaintext OR over both eyes of (database
  + the eyes of earlier persons), and a right eye made from the same
  person's left eye does not count.
"""
import itertools

import numpy as np

import oracle as orc
import workload as wl


def _open_bits(c):
    return c[0] ^ c[1] ^ c[2]


def test_or_bits_truth_table(keys):
    _, party = keys
    combos = list(itertools.product([0, 1], repeat=6))     # components of a and b
    a = np.array([[c[0] for c in combos], [c[1] for c in combos], [c[2] for c in combos]], dtype=np.uint8)
    b = np.array([[c[3] for c in combos], [c[4] for c in combos], [c[5] for c in combos]], dtype=np.uint8)
    out = orc.or_bits(party, a, b, 77)
    assert np.array_equal(_open_bits(out), _open_bits(a) | _open_bits(b))
    # different ids draw different randomness (the components differ, the opening does not)
    out2 = orc.or_bits(party, a, b, 78)
    assert not np.array_equal(out, out2) and np.array_equal(_open_bits(out2), _open_bits(out))


def test_mask_in_batch_keeps_earlier_columns():
    q, r = 5, 3
    rng = np.random.default_rng(3)
    m = rng.integers(0, 1 << 63, size=(3, q * r, 2), dtype=np.uint64)
    out = orc.mask_in_batch(m, q, r, 1)
    assert np.array_equal(out[:, :, 0], m[:, :, 0])         # other words untouched
    for row in range(q * r):
        qi = row // r
        keep = np.uint64((1 << qi) - 1)
        assert np.array_equal(out[:, row, 1], m[:, row, 1] & keep)


def test_in_batch_protocol_matches_plaintext(keys):
    dealer, party = keys
    rot = [-1, 0, 2]
    dc, dm = wl.gen_codes(81, 0, 40)
    qc, qm = wl.gen_codes(81, 0, 5, query=True)
    # query 3 is a near-duplicate of query 1 (both unseen in the database);
    # query 0 is a near-duplicate of query 4 (later: must not count for query 0)
    qc[3], qm[3] = wl.plant(81, 3, qc[1], qm[1], 2, h=0.2)
    qc[0], qm[0] = wl.plant(81, 0, qc[4], qm[4], 0, h=0.2)
    qc[2], qm[2] = wl.plant(81, 2, dc[7], dm[7], -1, h=0.25)   # database duplicate
    res = orc.protocol_in_batch(dealer, party, qc, qm, rot, dc, dm, qid_base=10)
    got = _open_bits(res["dup"]).astype(bool)
    want = np.zeros(5, dtype=bool)
    for i in range(5):
        ec = np.concatenate([dc, qc[:i]]) if i else dc
        em = np.concatenate([dm, qm[:i]]) if i else dm
        want[i] = orc.plain(qc[i:i + 1], qm[i:i + 1], rot, ec, em)[3][0]
    assert np.array_equal(got, want)
    assert list(want) == [False, False, True, True, True]   # query 4 matches query 0 (earlier) by symmetry
    # the database-only decision misses the in-batch duplicates
    assert list(_open_bits(res["dup_db"]).astype(bool)) == [False, False, True, False, False]


def test_in_batch_protocol_galois(keys):
    dealer, party = keys
    rot = [0, 1]
    dc, dm = wl.gen_codes(82, 0, 20)
    qc, qm = wl.gen_codes(82, 0, 3, query=True)
    qc[2], qm[2] = wl.plant(82, 2, qc[0], qm[0], 1, h=0.3)
    res = orc.protocol_in_batch(dealer, party, qc, qm, rot, dc, dm, qid_base=0, scheme="galois")
    assert list(_open_bits(res["dup"]).astype(bool)) == [False, False, True]


def test_mask_in_batch_groups_of_two():
    q, r = 7, 2          # odd q: the last query's group is incomplete but masked the same way
    rng = np.random.default_rng(4)
    m = rng.integers(0, 1 << 63, size=(3, q * r, 1), dtype=np.uint64) | np.uint64(1 << 63)
    out = orc.mask_in_batch(m, q, r, 0, group=2)
    for row in range(q * r):
        qi = row // r
        kept = [j for j in range(64) if (int(out[0, row, 0]) >> j) & 1 or (int(out[1, row, 0]) >> j) & 1
                or (int(out[2, row, 0]) >> j) & 1]
        assert all(j < 2 * (qi // 2) for j in kept)
        keep = np.uint64((1 << (2 * (qi // 2))) - 1)
        assert np.array_equal(out[:, row, 0], m[:, row, 0] & keep)
    # group 1 is the plain triangle
    assert np.array_equal(orc.mask_in_batch(m, q, r, 0, group=1), orc.mask_in_batch(m, q, r, 0))


def test_or_pairs_truth_table(keys):
    _, party = keys
    combos = list(itertools.product([0, 1], repeat=6))     # components of both eyes
    x = np.zeros((3, 2 * len(combos)), dtype=np.uint8)
    for i, c in enumerate(combos):
        x[:, 2 * i] = c[:3]
        x[:, 2 * i + 1] = c[3:]
    out = orc.or_pairs(party, x, 91)
    assert out.shape == (3, len(combos))
    opened = _open_bits(x)
    assert np.array_equal(_open_bits(out), opened[0::2] | opened[1::2])


def test_two_eye_protocol_matches_plaintext(keys):
    dealer, party = keys
    rot = [-1, 0, 2]
    dc, dm = wl.gen_codes(83, 0, 30)
    qc, qm = wl.gen_codes(83, 0, 8, query=True)        # persons 0..3, eyes 2k (left), 2k+1 (right)
    qc[1], qm[1] = wl.plant(83, 1, dc[4], dm[4], 2, h=0.2)      # person 0: right eye in the database
    qc[4], qm[4] = wl.plant(83, 4, qc[0], qm[0], -1, h=0.25)    # person 2: left eye from person 0's left
    qc[7], qm[7] = wl.plant(83, 7, qc[6], qm[6], 0, h=0.1)      # person 3: right eye from its own left eye
    qc[2], qm[2] = wl.plant(83, 2, qc[5], qm[5], 1, h=0.2)      # person 1 left from person 2 right (later)
    res = orc.protocol_in_batch(dealer, party, qc, qm, rot, dc, dm, qid_base=3, group=2)
    eyes = np.zeros(8, dtype=bool)
    for i in range(8):
        k = 2 * (i // 2)                                # eyes of earlier persons
        eyes[i] = orc.plain(qc[i:i + 1], qm[i:i + 1], rot, np.concatenate([dc, qc[:k]]),
                            np.concatenate([dm, qm[:k]]))[3][0]
    assert np.array_equal(_open_bits(res["dup"]).astype(bool), eyes)
    persons = eyes[0::2] | eyes[1::2]
    assert np.array_equal(_open_bits(res["person"]).astype(bool), persons)
    assert list(persons) == [True, False, True, False]
    # with groups of one, person 3's right eye would match its own left eye
    one = orc.protocol_in_batch(dealer, party, qc, qm, rot, dc, dm, qid_base=3, group=1)
    assert bool(_open_bits(one["dup"])[7]) and not eyes[7]
