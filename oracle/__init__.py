"""ctypes front-end of the plain CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product path.  It shares
no code with the GPU library; see ``oracle.c`` for what each function computes
and which part of the paper it follows.

Array conventions (numpy, C-contiguous):
  packed codes/masks  uint64 [n, 200]
  shares              uint16 [n, 2 (code, mask), 3 (component), 12800]
  per-party outputs   [3, rows, n]
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

L = 12800
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

DOM_SHARE_DB, DOM_SHARE_QUERY = 1, 2
DOM_GALOIS_DB, DOM_GALOIS_QUERY = 6, 7
DOM_SHARE32_DB, DOM_SHARE32_QUERY = 12, 13
N_GATES = 94   # AND gates per comparison: 33 (Lift) + 61 (MSB)
# comparison variants (oracle.c, "Comparison variants")
CMPV_PLAIN, CMPV_LIFT18, CMPV_CONST32 = 1, 2, 3
COMPARE_SETTINGS = ("mpclift", "plain", "lift18", "constlift", "nolift")


def build_lib() -> str:
    subprocess.check_call(
        ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB, os.path.join(_HERE, "oracle.c")]
    )
    return _LIB


def _p(a):
    # data_as keeps a reference to the array, so a temporary (a contiguous
    # copy made in the argument list) lives until the call returns
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        _lib = ctypes.CDLL(_LIB)
        _lib.orc_test_bit_extract.restype = ctypes.c_long
        _lib.orc_test_compare_one.restype = ctypes.c_int
        _lib.orc_prf_u16.restype = ctypes.c_uint16
        _lib.orc_prf_u64.restype = ctypes.c_uint64
        _lib.orc_threads.restype = ctypes.c_int
        _lib.orc_set_threads.restype = ctypes.c_int
        _lib.orc_compare.restype = ctypes.c_int
        _lib.orc_test_gr_inv.restype = ctypes.c_int
        _lib.orc_compare_variant.restype = ctypes.c_int
        _lib.orc_test_compare_variant.restype = ctypes.c_int
        _lib.orc_msg_count.restype = ctypes.c_int
    return _lib


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> int:
    """Thread count of later oracle calls; returns the previous count."""
    return lib().orc_set_threads(ctypes.c_int(n))


def chacha_block(key: bytes, rounds: int, words12_15) -> np.ndarray:
    out = np.zeros(16, dtype=np.uint32)
    inp = np.asarray(words12_15, dtype=np.uint32)
    lib().orc_chacha_block(ctypes.c_char_p(bytes(key)), ctypes.c_int(rounds), _p(inp), _p(out))
    return out


def prf_block(key: bytes, stream: int, pos: int) -> np.ndarray:
    out = np.zeros(16, dtype=np.uint32)
    lib().orc_prf_block(ctypes.c_char_p(bytes(key)), ctypes.c_uint64(stream), ctypes.c_uint64(pos), _p(out))
    return out


def _rot(rot):
    return np.ascontiguousarray(np.asarray(rot, dtype=np.int32))


def plain(qc, qm, rot, dc, dm):
    """O1: (hd, ml, match) [rows, n] and dup [nq] for packed inputs."""
    nq, n, r = qc.shape[0], dc.shape[0], len(rot)
    rows = nq * r
    hd = np.zeros((rows, n), dtype=np.int32)
    ml = np.zeros((rows, n), dtype=np.int32)
    match = np.zeros((rows, n), dtype=np.uint8)
    dup = np.zeros(nq, dtype=np.uint8)
    rr = _rot(rot)
    lib().orc_plain(_p(np.ascontiguousarray(qc)), _p(np.ascontiguousarray(qm)), ctypes.c_int(nq), _p(rr),
                    ctypes.c_int(r), _p(np.ascontiguousarray(dc)), _p(np.ascontiguousarray(dm)), ctypes.c_long(n),
                    _p(hd), _p(ml), _p(match), _p(dup))
    return hd, ml, match, dup


def encode(code, mask):
    xc = np.zeros(L, dtype=np.uint16)
    xm = np.zeros(L, dtype=np.uint16)
    lib().orc_encode(_p(np.ascontiguousarray(code)), _p(np.ascontiguousarray(mask)), _p(xc), _p(xm))
    return xc, xm


def share(dealer_key: bytes, dom: int, codes, masks, first_id: int):
    n = codes.shape[0]
    out = np.zeros((n, 2, 3, L), dtype=np.uint16)
    lib().orc_share(ctypes.c_char_p(bytes(dealer_key)), ctypes.c_int(dom), _p(np.ascontiguousarray(codes)),
                    _p(np.ascontiguousarray(masks)), ctypes.c_long(n), ctypes.c_uint64(first_id), _p(out))
    return out


def local_dot(p: int, qsh, rot, dsh):
    nq, n, r = qsh.shape[0], dsh.shape[0], len(rot)
    oc = np.zeros((nq * r, n), dtype=np.uint16)
    om = np.zeros((nq * r, n), dtype=np.uint16)
    lib().orc_local_dot(ctypes.c_int(p), _p(np.ascontiguousarray(qsh)), ctypes.c_int(nq), _p(_rot(rot)),
                        ctypes.c_int(r), _p(np.ascontiguousarray(dsh)), ctypes.c_long(n), _p(oc), _p(om))
    return oc, om


def reshare(keys: bytes, z_code, z_mask, nq, rot, qid_base, first_entry):
    """z_*: [3, rows, n] additive shares -> [3, rows, n] re-randomised components."""
    _, rows, n = z_code.shape
    oc = np.zeros_like(z_code)
    om = np.zeros_like(z_mask)
    lib().orc_reshare(ctypes.c_char_p(bytes(keys)), _p(np.ascontiguousarray(z_code)),
                      _p(np.ascontiguousarray(z_mask)), ctypes.c_int(nq), _p(_rot(rot)), ctypes.c_int(len(rot)),
                      ctypes.c_long(n), ctypes.c_uint64(qid_base), ctypes.c_uint64(first_entry), _p(oc), _p(om))
    return oc, om


def msg_count(variant: int = 0) -> int:
    """Messages (bits sent by the three parties) per comparison of a setting:
    0 = MPCLift, else CMPV_*."""
    return lib().orc_msg_count(ctypes.c_int(variant))


def compare(keys: bytes, d_comp, x_comp, nq, rot, qid_base, first_entry, want_aux=False, want_msg=False):
    """Components of the match bits [3, rows, nw] (u64) from components of the
    code dot and ml [3, rows, n].  With want_aux also returns lifted-ml and y
    components [3, rows, n] (u32) and counts (AND gates, bits sent by 0,1,2).
    With want_msg the last item returned is the message log
    [msg_count(0), rows, nw] (u64, bit o of word w = column 64 w + o)."""
    _, rows, n = d_comp.shape
    nw = (n + 63) // 64
    match = np.zeros((3, rows, nw), dtype=np.uint64)
    ml = np.zeros((3, rows, n), dtype=np.uint32) if want_aux else None
    y = np.zeros((3, rows, n), dtype=np.uint32) if want_aux else None
    msg = np.zeros((msg_count(0), rows, nw), dtype=np.uint64) if want_msg else None
    counts = np.zeros(4, dtype=np.int64)
    rc = lib().orc_compare(ctypes.c_char_p(bytes(keys)), _p(np.ascontiguousarray(d_comp)),
                           _p(np.ascontiguousarray(x_comp)), ctypes.c_int(nq), _p(_rot(rot)),
                           ctypes.c_int(len(rot)), ctypes.c_long(n), ctypes.c_uint64(qid_base),
                           ctypes.c_uint64(first_entry), _p(match), _p(ml), _p(y), _p(counts), _p(msg))
    if rc != 0:
        raise ValueError("first_entry must be a multiple of 64")
    out = (match, ml, y, counts) if want_aux else (match,)
    if want_msg:
        out = out + (msg,)
    return out if len(out) > 1 else match


def compare_variant(keys: bytes, variant: int, d_comp, x_comp, ml_pub, nq, rot, qid_base, first_entry,
                    want_aux=False, want_msg=False):
    """Comparison variant (CMPV_*) over [3, rows, n] components: d_comp the
    code dot (u16 or u32), x_comp ml (u16 for LIFT18, u32 for CONST32, None
    for PLAIN), ml_pub [rows, n] the public ml (PLAIN).  Returns the match
    components [3, rows, nw]; with want_aux also y components and counts;
    with want_msg the message log [msg_count(variant), rows, nw] last."""
    _, rows, n = d_comp.shape
    nw = (n + 63) // 64
    d32 = np.ascontiguousarray(d_comp.astype(np.uint32))
    x32 = None if x_comp is None else np.ascontiguousarray(x_comp.astype(np.uint32))
    mlp = None if ml_pub is None else np.ascontiguousarray(np.asarray(ml_pub, dtype=np.int32))
    match = np.zeros((3, rows, nw), dtype=np.uint64)
    y = np.zeros((3, rows, n), dtype=np.uint32) if want_aux else None
    msg = np.zeros((msg_count(variant), rows, nw), dtype=np.uint64) if want_msg else None
    counts = np.zeros(4, dtype=np.int64)
    rc = lib().orc_compare_variant(ctypes.c_int(variant), ctypes.c_char_p(bytes(keys)), _p(d32), _p(x32), _p(mlp),
                                   ctypes.c_int(nq), _p(_rot(rot)), ctypes.c_int(len(rot)), ctypes.c_long(n),
                                   ctypes.c_uint64(qid_base), ctypes.c_uint64(first_entry), _p(match), _p(y),
                                   _p(counts), _p(msg))
    if rc != 0:
        raise ValueError("bad variant or first_entry not a multiple of 64")
    out = (match, y, counts) if want_aux else (match,)
    if want_msg:
        out = out + (msg,)
    return out if len(out) > 1 else match


def share32(dealer_key: bytes, dom: int, codes, masks, first_id: int):
    """Shares over Z_2^32: uint32 [n, 2, 3, L]."""
    n = codes.shape[0]
    out = np.zeros((n, 2, 3, L), dtype=np.uint32)
    lib().orc_share32(ctypes.c_char_p(bytes(dealer_key)), ctypes.c_int(dom), _p(np.ascontiguousarray(codes)),
                      _p(np.ascontiguousarray(masks)), ctypes.c_long(n), ctypes.c_uint64(first_id), _p(out))
    return out


def local_dot32(p: int, qsh, rot, dsh):
    """Party p's additive shares over Z_2^32: (code, mask) uint32 [rows, n]."""
    nq, n = qsh.shape[0], dsh.shape[0]
    rows = nq * len(rot)
    oc = np.zeros((rows, n), dtype=np.uint32)
    om = np.zeros((rows, n), dtype=np.uint32)
    lib().orc_local_dot32(ctypes.c_int(p), _p(np.ascontiguousarray(qsh)), ctypes.c_int(nq), _p(_rot(rot)),
                          ctypes.c_int(len(rot)), _p(np.ascontiguousarray(dsh)), ctypes.c_long(n), _p(oc), _p(om))
    return oc, om


def reshare32(keys: bytes, z_code, z_mask, nq, rot, qid_base, first_entry):
    """Resharing over Z_2^32 of [3, rows, n] u32 additive shares (either may
    be None): re-randomised components."""
    ref = z_code if z_code is not None else z_mask
    _, rows, n = ref.shape
    oc = np.zeros_like(ref) if z_code is not None else None
    om = np.zeros_like(ref) if z_mask is not None else None
    zc = None if z_code is None else np.ascontiguousarray(z_code)
    zm = None if z_mask is None else np.ascontiguousarray(z_mask)
    lib().orc_reshare32(ctypes.c_char_p(bytes(keys)), _p(zc), _p(zm), ctypes.c_int(nq), _p(_rot(rot)),
                        ctypes.c_int(len(rot)), ctypes.c_long(n), ctypes.c_uint64(qid_base),
                        ctypes.c_uint64(first_entry), _p(oc), _p(om))
    return oc, om


def or_tree(keys: bytes, match, nq, r, qid_base):
    """match [3, nq*r, nw] -> dup components [3, nq] (0/1) and the number of
    word-wide AND gates."""
    _, rows, nw = match.shape
    dup = np.zeros((3, nq), dtype=np.uint8)
    cnt = ctypes.c_long(0)
    lib().orc_or_tree(ctypes.c_char_p(bytes(keys)), _p(np.ascontiguousarray(match)), ctypes.c_int(nq),
                      ctypes.c_int(r), ctypes.c_long(nw), ctypes.c_uint64(qid_base), _p(dup), ctypes.byref(cnt))
    return dup, cnt.value


def open_add(comps, bits: int):
    """Reconstruct arithmetic components [3, ...] mod 2^bits."""
    s = comps.astype(np.uint64).sum(axis=0)
    return (s & np.uint64((1 << bits) - 1)).astype(np.uint32 if bits > 16 else np.uint16)


def open_xor(comps):
    return comps[0] ^ comps[1] ^ comps[2]


# ---- sub-protocol hooks on explicit or seeded randomness (for pinning) ----
def t_bit_extract(k, m, x0, x1, x2, seed):
    bits = np.zeros(m + 1, dtype=np.uint8)
    comp = np.zeros(3 * (m + 1), dtype=np.uint8)
    depth = np.zeros(m + 1, dtype=np.int32)
    ands = lib().orc_test_bit_extract(ctypes.c_int(k), ctypes.c_int(m), ctypes.c_uint32(x0), ctypes.c_uint32(x1),
                                      ctypes.c_uint32(x2), ctypes.c_uint64(seed), _p(bits), _p(comp), _p(depth))
    return bits, comp.reshape(m + 1, 3), ands, depth


def t_and(x, y, f):
    x, y, f = (np.asarray(v, dtype=np.uint8) for v in (x, y, f))
    z = np.zeros(3, dtype=np.uint8)
    lib().orc_test_and(_p(x), _p(y), _p(f), _p(z))
    return z


def t_fa(a, b, c, f):
    a, b, c, f = (np.asarray(v, dtype=np.uint8) for v in (a, b, c, f))
    s = np.zeros(3, dtype=np.uint8)
    o = np.zeros(3, dtype=np.uint8)
    lib().orc_test_fa(_p(a), _p(b), _p(c), _p(f), _p(s), _p(o))
    return s, o


def t_bit_inject(x, k, c0, c2, w0, w1):
    x = np.asarray(x, dtype=np.uint8)
    out = np.zeros(3, dtype=np.uint32)
    bits = np.zeros(3, dtype=np.int64)
    lib().orc_test_bit_inject(_p(x), ctypes.c_int(k), ctypes.c_uint32(c0), ctypes.c_uint32(c2),
                              ctypes.c_uint32(w0), ctypes.c_uint32(w1), _p(out), _p(bits))
    return out, bits


def t_compare_one(d, x, seed):
    d = np.asarray(d, dtype=np.uint16)
    x = np.asarray(x, dtype=np.uint16)
    mlo = ctypes.c_uint32(0)
    yo = ctypes.c_uint32(0)
    counts = np.zeros(4, dtype=np.int64)
    depth = ctypes.c_int(0)
    m = lib().orc_test_compare_one(_p(d), _p(x), ctypes.c_uint64(seed), ctypes.byref(mlo), ctypes.byref(yo),
                                   _p(counts), ctypes.byref(depth))
    return m, mlo.value, yo.value, counts, depth.value


def t_compare_variant(variant, d, x, ml_pub, seed):
    """One comparison of a variant on explicit components (u32) with seeded
    randomness: (opened bit, opened y, counts, depth)."""
    d = np.asarray(d, dtype=np.uint32)
    x = np.asarray(x, dtype=np.uint32)
    yo = ctypes.c_uint32(0)
    counts = np.zeros(4, dtype=np.int64)
    depth = ctypes.c_int(0)
    m = lib().orc_test_compare_variant(ctypes.c_int(variant), _p(d), _p(x), ctypes.c_uint32(ml_pub),
                                       ctypes.c_uint64(seed), ctypes.byref(yo), _p(counts), ctypes.byref(depth))
    return m, yo.value, counts, depth.value


def galois_share(dealer_key: bytes, dom: int, codes, masks, first_id: int):
    """Shamir shares over Z_2^16[X]/(X^2-X-1): [n, 2 (code, mask), 3 (party), L],
    party p's share of pair i at positions (2i, 2i+1)."""
    n = codes.shape[0]
    out = np.zeros((n, 2, 3, L), dtype=np.uint16)
    lib().orc_galois_share(ctypes.c_char_p(bytes(dealer_key)), ctypes.c_int(dom), _p(np.ascontiguousarray(codes)),
                           _p(np.ascontiguousarray(masks)), ctypes.c_long(n), ctypes.c_uint64(first_id), _p(out))
    return out


def galois_local_dot(p: int, qsh, rot, dsh):
    """Party p's additive shares of the code and mask dots from Galois shares."""
    nq, n, r = qsh.shape[0], dsh.shape[0], len(rot)
    oc = np.zeros((nq * r, n), dtype=np.uint16)
    om = np.zeros((nq * r, n), dtype=np.uint16)
    lib().orc_galois_local_dot(ctypes.c_int(p), _p(np.ascontiguousarray(qsh)), ctypes.c_int(nq), _p(_rot(rot)),
                               ctypes.c_int(r), _p(np.ascontiguousarray(dsh)), ctypes.c_long(n), _p(oc), _p(om))
    return oc, om


def galois_points():
    """(alpha [3, 2], lambda [3, 2]) as (c0, c1) coefficient pairs."""
    a = np.zeros(6, dtype=np.uint16)
    lam = np.zeros(6, dtype=np.uint16)
    lib().orc_galois_points(_p(a), _p(lam))
    return a.reshape(3, 2), lam.reshape(3, 2)


def t_gr_mul(a, b):
    a = np.asarray(a, dtype=np.uint16)
    b = np.asarray(b, dtype=np.uint16)
    out = np.zeros(2, dtype=np.uint16)
    lib().orc_test_gr_mul(_p(a), _p(b), _p(out))
    return out


def t_gr_inv(a):
    a = np.asarray(a, dtype=np.uint16)
    out = np.zeros(2, dtype=np.uint16)
    ok = lib().orc_test_gr_inv(_p(a), _p(out))
    return out if ok else None


def mask_in_batch(match, q: int, r: int, word: int, group: int = 1):
    """Clear shared match bits of columns j with j//group >= qi//group in
    `word` of rows qi*r+ri (copy): a query meets only earlier groups."""
    out = np.ascontiguousarray(match, dtype=np.uint64).copy()
    lib().orc_mask_in_batch(_p(out), ctypes.c_int(q), ctypes.c_int(r), ctypes.c_long(out.shape[-1]),
                            ctypes.c_long(word), ctypes.c_int(group))
    return out


def or_bits(keys: bytes, a, b, id_: int):
    """Shared OR of two bit sharings [3, count] (0/1 bytes)."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    out = np.zeros_like(a)
    lib().orc_or_bits(ctypes.c_char_p(bytes(keys)), _p(a), _p(b), ctypes.c_long(a.shape[1]), ctypes.c_uint64(id_),
                      _p(out))
    return out


def or_pairs(keys: bytes, x, id_: int):
    """A person's decision from its eyes' decisions [Sec. 6.4]: element i of
    the result is element 2i OR element 2i+1 of x ([3, 2*count])."""
    x = np.asarray(x, dtype=np.uint8)
    return or_bits(keys, x[:, 0::2], x[:, 1::2], id_)


BATCH_ENTRY_BASE = 1 << 47    # entry ids of in-batch columns (distinct randomness from database entries)
PERSON_OR_BASE = 1 << 47      # OR-gate stream ids of the per-person combination


def protocol_in_batch(dealer_key: bytes, keys: bytes, qc, qm, rot, dc, dm, qid_base=0, scheme="aby3", group=1):
    """Protocol run where each query is also compared with the earlier queries
    of its batch: database part as `protocol`; batch part with the queries'
    own shares as entries (ids BATCH_ENTRY_BASE + j), the columns of its own
    and later groups cleared (group=2: a person's two eyes never meet), its
    OR-tree, then one OR gate per query combining both decisions."""
    q, r = qc.shape[0], len(rot)
    res = protocol(dealer_key, keys, qc, qm, rot, dc, dm, qid_base=qid_base, first_entry=0, scheme=scheme)
    qsh = res["qsh"]
    dot = galois_local_dot if scheme == "galois" else local_dot
    zc, zm = [], []
    for p in range(3):
        c, m = dot(p, qsh, rot, qsh)
        zc.append(c)
        zm.append(m)
    rc, rm = reshare(keys, np.stack(zc), np.stack(zm), q, rot, qid_base, BATCH_ENTRY_BASE)
    bm = compare(keys, rc, rm, q, rot, qid_base, BATCH_ENTRY_BASE)
    bm = mask_in_batch(bm, q, r, 0, group)
    dup_b, _ = or_tree(keys, bm, q, r, qid_base + (1 << 46))
    dup = or_bits(keys, res["dup"], dup_b, qid_base)
    res.update(batch_match=bm, dup_db=res["dup"], dup_batch=dup_b, dup=dup)
    if group == 2:     # person k = eyes 2k, 2k+1: duplicate if either eye is
        res["person"] = or_pairs(keys, dup, PERSON_OR_BASE | qid_base)
    return res


def protocol(dealer_key: bytes, keys: bytes, qc, qm, rot, dc, dm, qid_base=0, first_entry=0, scheme="aby3",
             compare_setting="mpclift"):
    """The whole shared protocol on the CPU: share, per-party local dots,
    reshare, compare, OR-tree.  Returns a dict of every intermediate.

    compare_setting: "mpclift" (ml and dot over Z_2^16, ml lifted to
    Z_2^32); "plain" (masks public, Alg. 2: ml in plain, code dot only);
    "lift18" (ml lifted to Z_2^18 only); "constlift" (ml by a dot product
    over Z_2^32, code dot over Z_2^16); "nolift" (both dots over Z_2^32)."""
    if compare_setting not in COMPARE_SETTINGS:
        raise ValueError(compare_setting)
    nq, r = qc.shape[0], len(rot)
    if scheme == "galois":
        qsh = galois_share(dealer_key, DOM_GALOIS_QUERY, qc, qm, qid_base)
        dsh = galois_share(dealer_key, DOM_GALOIS_DB, dc, dm, first_entry)
        dot = galois_local_dot
    else:
        qsh = share(dealer_key, DOM_SHARE_QUERY, qc, qm, qid_base)
        dsh = share(dealer_key, DOM_SHARE_DB, dc, dm, first_entry)
        dot = local_dot
    zc, zm = [], []
    for p in range(3):
        c, m = dot(p, qsh, rot, dsh)
        zc.append(c)
        zm.append(m)
    zc = np.stack(zc)
    zm = np.stack(zm)
    rc, rm = reshare(keys, zc, zm, nq, rot, qid_base, first_entry)
    out = dict(qsh=qsh, dsh=dsh, z_code=zc, z_mask=zm, rep_code=rc, rep_mask=rm)
    if compare_setting == "mpclift":
        match, ml, y, counts = compare(keys, rc, rm, nq, rot, qid_base, first_entry, want_aux=True)
        out.update(ml_lift=ml)
    elif compare_setting == "plain":
        _, ml_pub, _, _ = plain(qc, qm, rot, dc, dm)
        match, y, counts = compare_variant(keys, CMPV_PLAIN, rc, None, ml_pub, nq, rot, qid_base, first_entry,
                                           want_aux=True)
        out.update(ml_pub=ml_pub)
    elif compare_setting == "lift18":
        match, y, counts = compare_variant(keys, CMPV_LIFT18, rc, rm, None, nq, rot, qid_base, first_entry,
                                           want_aux=True)
    else:
        q32 = share32(dealer_key, DOM_SHARE32_QUERY, qc, qm, qid_base)
        d32 = share32(dealer_key, DOM_SHARE32_DB, dc, dm, first_entry)
        zc32, zm32 = [], []
        for p in range(3):
            c, m = local_dot32(p, q32, rot, d32)
            zc32.append(c)
            zm32.append(m)
        zc32, zm32 = np.stack(zc32), np.stack(zm32)
        rc32, rm32 = reshare32(keys, zc32 if compare_setting == "nolift" else None, zm32, nq, rot, qid_base,
                               first_entry)
        dcomp = rc32 if compare_setting == "nolift" else rc
        match, y, counts = compare_variant(keys, CMPV_CONST32, dcomp, rm32, None, nq, rot, qid_base, first_entry,
                                           want_aux=True)
        out.update(qsh32=q32, dsh32=d32, z_code32=zc32, z_mask32=zm32, rep_mask32=rm32,
                   rep_code32=rc32)
    dup, or_words = or_tree(keys, match, nq, r, qid_base)
    out.update(match=match, y=y, counts=counts, dup=dup, or_words=or_words)
    return out
