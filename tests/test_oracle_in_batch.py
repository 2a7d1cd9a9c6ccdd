"""Pins of the oracle's in-batch matching and decision combining (Sec. 6.4:
the queries of a batch are matched with each other as well as with the
database; a person's query covers both eyes).

* The OR gate on shared bits opens to the OR of the opened inputs, for every
  combination of component bits (brute force).
* The in-batch mask keeps exactly the columns j < qi of each row.
* End to end: with the batch part, a query's opened result equals the
  plaintext decision against the database plus the batch's earlier queries
  (O1 on the concatenated entries); later queries never count.
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
