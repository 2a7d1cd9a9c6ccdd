"""Checks of every opened value of a full-size run (a helper of the GPU tests,
not a test module): the opened match matrix and duplicate bits against the
plaintext decision of Alg. 1, and the duplicate-bit components against the
oracle's OR-tree (Sec. 4.2) run on the GPU's own match-bit components.

Why every opened bit is covered: an opened one is re-decided by the
plaintext check on its pair and must be a match; the opened ones must be
exactly the plaintext matches among the planted pairs (at every rotation);
and every other pair of the workload is a random code against a random
entry, whose fractional HD sits about 25 standard deviations above the
threshold (pinned by test_plain_random_pairs_statistics), so its plaintext
decision is 0."""
import numpy as np

import oracle as orc
import workload as wl


def opened_ones(mo):
    """(row, column) of every set bit of opened match words mo [rows, nw]."""
    out = []
    rows, words = np.nonzero(mo)
    for row, word in zip(rows.tolist(), words.tolist()):
        v = int(mo[row, word])
        while v:
            low = v & -v
            out.append((row, 64 * word + low.bit_length() - 1))
            v ^= low
    return out


def entries(seed, ents):
    dc = np.empty((len(ents), 200), np.uint64)
    dm = np.empty_like(dc)
    for i, e in enumerate(ents):
        c, m = wl.gen_codes(seed, e, 1)
        dc[i], dm[i] = c[0], m[0]
    return dc, dm


def check_every_opened_bit(mo, dup, w, qc, qm, n):
    """mo: opened match words [rows, nw] (uint64); dup: opened duplicate bits
    [n_q].  Returns (opened ones, duplicates)."""
    r = len(w.rot)
    ones = opened_ones(np.asarray(mo, dtype=np.uint64))
    assert all(c < n for _, c in ones), "an opened one beyond the last entry"
    ents = sorted({c for _, c in ones} | {e for _, e, _, _ in w.planted})
    dc, dm = entries(w.seed, ents)
    _, _, match, _ = orc.plain(qc, qm, w.rot, dc, dm)
    col = {e: i for i, e in enumerate(ents)}
    rejected = [(row, c) for row, c in ones if not match[row, col[c]]]
    assert not rejected, f"opened ones the plaintext check rejects: {rejected[:8]}"
    want = {(qi * r + ri, e) for qi, e, _, _ in w.planted for ri in range(r) if match[qi * r + ri, col[e]]}
    assert set(ones) == want, (sorted(set(ones) - want)[:8], sorted(want - set(ones))[:8])
    want_dup = np.zeros(w.n_q, np.uint8)
    for row, _ in want:
        want_dup[row // r] = 1
    assert np.array_equal(np.asarray(dup).astype(np.uint8), want_dup)
    return len(ones), int(want_dup.sum())


def check_or_tree_components(party_keys, match_comps, dup_planes, nq, r, qid_base=0):
    """match_comps [3, rows, nw]: component p of every match word (party p's
    own plane); dup_planes: per party the [2, nq] duplicate-bit planes the GPU
    wrote (own component, component p-1).  The oracle's OR-tree on the same
    components must give the same components."""
    ref, _ = orc.or_tree(party_keys, match_comps, nq, r, qid_base)
    for p in range(3):
        pm = (p + 2) % 3
        assert np.array_equal(dup_planes[p][0], ref[p]), p
        assert np.array_equal(dup_planes[p][1], ref[pm]), p
