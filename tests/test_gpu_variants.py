"""GPU comparison settings (masks in plain, Lift to Z_2^18, ml over Z_2^32)
through the C ABI against the CPU oracle, bit-exact on every component.

The comparison kernels are fed (a) the outputs of the GPU's own dot products
and resharing in a full protocol run, compared step by step with the
oracle's run, and (b) random replicated components uploaded from the host,
which covers the Z_2^32 inputs, the vector and element-wise load paths
(ld a multiple of 8 or not) and ragged 64-entry words.
"""
import numpy as np
import pytest

import oracle as orc
import workload as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def imc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_04463_amd as imc_mod

    imc_mod.lib()
    return imc_mod


@pytest.fixture(scope="module")
def ctx(imc, keys):
    dealer, party = keys
    c = imc.Context(imc.Keys(dealer, party), max_rows=512)
    yield c
    c.close()


def dev64(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def u16(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint16)


def _rep_dev(comps: np.ndarray, ld: int, dtype):
    """[3, rows, n] components -> per party device [2, rows, ld] (own, previous)."""
    _, rows, n = comps.shape
    out = []
    for p in range(3):
        pm = (p + 2) % 3
        h = np.zeros((2, rows, ld), dtype=dtype)
        h[0, :, :n] = comps[p]
        h[1, :, :n] = comps[pm]
        t = torch.from_numpy(h.view(np.int16 if dtype == np.uint16 else np.int32)).cuda()
        out.append(t)
    return out


def _match_host(match, nw):
    return [m.cpu().numpy().view(np.uint64)[:, :, :nw] for m in match]


@pytest.mark.parametrize("variant", ["plain", "lift18", "const32", "nolift"])
@pytest.mark.parametrize("rows_r,n,ld,first", [
    ((3, [-2, 0, 5]), 200, 256, 64),      # vector loads, ragged last word
    ((2, [1, 4]), 130, 130, 0),           # ld not a multiple of 8: element-wise loads
    ((1, [0]), 1, 8, 0),                  # a single comparison
    ((5, [3]), 64, 64, 128),              # exactly one word
])
def test_compare_variant_on_random_components(ctx, imc, keys, variant, rows_r, n, ld, first):
    _, party = keys
    nq, rot = rows_r
    rows = nq * len(rot)
    rng = np.random.default_rng(sum(map(ord, variant)) * 1000 + n + ld)
    ml = rng.integers(0, 12801, (rows, n)).astype(np.int64)
    dot = np.array([[int(rng.integers(-m, m + 1)) for m in r_] for r_ in ml], dtype=np.int64).reshape(rows, n)
    dot += ((dot - ml) % 2) * np.where(dot < ml, 1, -1)
    # a few exact boundaries 8 hd = 3 ml (no match) and 8 hd = 3 ml - 8 (match)
    k = min(4, ml.size)
    ml.flat[:k] = [800, 800, 8, 0][:k]
    dot.flat[:k] = [800 - 2 * 300, 800 - 2 * 299, 8 - 2 * 3, 0][:k]
    code_bits = 32 if variant == "nolift" else 16
    mask_bits = 32 if variant in ("const32", "nolift") else 16

    def split(v, bits):
        mod = 1 << bits
        c = rng.integers(0, mod, (3,) + v.shape, dtype=np.uint64)
        c[2] = (v - c[0].astype(np.int64) - c[1].astype(np.int64)) % mod
        return c.astype(np.uint32 if bits == 32 else np.uint16)

    d = split(dot, code_bits)
    x = split(ml, mask_bits)
    v = {"plain": orc.CMPV_PLAIN, "lift18": orc.CMPV_LIFT18}.get(variant, orc.CMPV_CONST32)
    want = orc.compare_variant(party, v, d, None if variant == "plain" else x, ml if variant == "plain" else None,
                               nq, rot, 7, first)
    nw = (n + 63) // 64
    mw_ld = nw + 1
    rep_code = _rep_dev(d, ld, np.uint32 if code_bits == 32 else np.uint16)
    rep_mask = None if variant == "plain" else _rep_dev(x, ld, np.uint32 if mask_bits == 32 else np.uint16)
    ml_pub = None
    if variant == "plain":
        h = np.zeros((rows, ld), dtype=np.uint16)
        h[:, :n] = ml
        ml_pub = torch.from_numpy(h.view(np.int16)).cuda()
    match = [torch.full((2, rows, mw_ld), -1, dtype=torch.int64, device="cuda") for _ in range(3)]
    ids = imc.make_ids(7, rot, first)
    cv = {"plain": imc.CMP_PLAIN_MASK, "lift18": imc.CMP_LIFT18}.get(variant, imc.CMP_CONST32)
    ctx.compare_variant(cv, rep_code, code_bits, rep_mask, ml_pub, rows, n, ld, ids, match, mw_ld)
    torch.cuda.synchronize()
    got = _match_host(match, nw)
    for p in range(3):
        pm = (p + 2) % 3
        assert np.array_equal(got[p][0], want[p]), (variant, p)
        assert np.array_equal(got[p][1], want[pm]), (variant, p)
    opened = got[0][0] ^ got[1][0] ^ got[2][0]
    bits = np.array([[(int(opened[r_, j // 64]) >> (j % 64)) & 1 for j in range(n)] for r_ in range(rows)])
    assert np.array_equal(bits, (4 * dot > ml).astype(int))


@pytest.mark.parametrize("q,rot,n,first,pad", [
    (3, list(range(-15, 16)), 130, 64, 4),     # 93 rows: one row tile, ragged; three entry tiles, ragged
    (10, list(range(-15, 16)), 300, 0, 4),     # 310 rows: three row tiles of the rotation-aware kernel
    (9, list(range(-7, 8)), 257, 128, 3),      # 15 rotations (its larger query staging); row stride not 16-B aligned
    (5, [-3, 0, 9], 64, 0, 4),                 # one entry tile exactly
    (1, [7], 1, 0, 1),                         # a single comparison
    (2, list(range(-15, 16)), 1, 192, 2),      # one entry against the rotation-aware kernel's tiles
])
def test_dot32_and_reshare32_match_oracle(ctx, imc, keys, q, rot, n, first, pad):
    dealer, party = keys
    dc, dm = wl.gen_codes(72, first, n)
    qc, qm = wl.gen_codes(72, 0, q, query=True)
    dsh = orc.share32(dealer, orc.DOM_SHARE32_DB, dc, dm, first)
    qsh = orc.share32(dealer, orc.DOM_SHARE32_QUERY, qc, qm, 50)
    rows, ld = q * len(rot), ((n + 63) // 64) * 64 + pad
    ids = imc.make_ids(50, rot, first)
    z = [orc.local_dot32(p, qsh, rot, dsh) for p in range(3)]
    for vec in (0, 1):
        regions = [torch.empty(imc.db32_bytes(first + n), dtype=torch.uint8, device="cuda") for _ in range(3)]
        ops = [torch.empty(imc.query32_op_bytes(q), dtype=torch.uint8, device="cuda") for _ in range(3)]
        ctx.share32_db(vec, dev64(dc), dev64(dm), n, first, regions, first + n)
        ctx.share32_query(vec, dev64(qc), dev64(qm), q, 50, ops)
        dots = [torch.full((rows, ld), -1, dtype=torch.int32, device="cuda") for _ in range(3)]
        for p in range(3):
            ctx.dot32_shares(p, ops[p], q, ids, regions[p], first + n, n, dots[p], ld)
        msg = [torch.empty(rows, ld, dtype=torch.int32, device="cuda") for _ in range(3)]
        rep = [torch.empty(2, rows, ld, dtype=torch.int32, device="cuda") for _ in range(3)]
        ctx.reshare32(vec, dots, rows, n, ld, ids, msg, rep)
        torch.cuda.synchronize()
        zs = np.stack([z[p][vec] for p in range(3)])
        rc, rm = orc.reshare32(party, zs if vec == 0 else None, zs if vec == 1 else None, q, rot, 50, first)
        want = rc if vec == 0 else rm
        for p in range(3):
            pm = (p + 2) % 3
            got = dots[p].cpu().numpy().view(np.uint32)
            assert np.array_equal(got[:, :n], z[p][vec]), (vec, p)
            assert np.all(got[:, n:] == 0xFFFFFFFF)
            r_ = rep[p].cpu().numpy().view(np.uint32)
            assert np.array_equal(r_[0, :, :n], want[p]) and np.array_equal(r_[1, :, :n], want[pm])
            assert np.array_equal(msg[p].cpu().numpy().view(np.uint32)[:, :n], want[p])


@pytest.mark.parametrize("setting", ["plain", "lift18", "constlift", "nolift"])
def test_protocol_setting_matches_oracle(ctx, imc, keys, setting):
    """Every step on the GPU vs the oracle's protocol run in the same setting."""
    from paper_2405_04463_amd.pipeline import (VECS32, SharedDB, SharedDB32, SharedQueries, SharedQueries32,
                                               alloc_check, open_dup, open_match, run_check)

    dealer, party = keys
    n, q, rot, first = 200, 4, [-2, 0, 1, 5, 15], 64
    dc, dm = wl.gen_codes(43, first, n)
    qc, qm = wl.gen_codes(43, 0, q, query=True)
    qc[0], qm[0] = wl.plant(43, 0, dc[17], dm[17], 1, h=0.2)
    qc[1], qm[1] = wl.plant(43, 1, dc[150], dm[150], 5, exact="eq")
    qc[2], qm[2] = wl.plant(43, 2, dc[199], dm[199], -2, exact="lt")
    db = SharedDB(ctx, first + n)
    db.enroll(dev64(dc), dev64(dm), first)
    qs = SharedQueries(ctx, dev64(qc), dev64(qm), 100)
    buf = alloc_check(q, len(rot), n, compare=setting)
    db_masks = torch.zeros(first + n, 200, dtype=torch.int64, device="cuda")
    db_masks[first:] = dev64(dm)
    qs32 = db32 = None
    if setting in VECS32:
        db32 = SharedDB32(ctx, first + n, vecs=VECS32[setting])
        db32.enroll(dev64(dc), dev64(dm), first)
        qs32 = SharedQueries32(ctx, dev64(qc), dev64(qm), 100, vecs=VECS32[setting])
    run_check(ctx, qs, rot, db, first, n, buf, query_masks=dev64(qm), db_masks=db_masks, qs32=qs32, db32=db32)
    torch.cuda.synchronize()

    ref = orc.protocol(dealer, party, qc, qm, rot, dc, dm, qid_base=100, first_entry=first, compare_setting=setting)
    hd, ml, match, dup = orc.plain(qc, qm, rot, dc, dm)
    nw = (n + 63) // 64
    if setting == "plain":
        assert np.array_equal(u16(buf.ml_pub)[:, :n], ml.astype(np.uint16))
    for p in range(3):
        pm = (p + 2) % 3
        if setting != "nolift":
            assert np.array_equal(u16(buf.rep_code[p])[0, :, :n], ref["rep_code"][p])
            assert np.array_equal(u16(buf.rep_code[p])[1, :, :n], ref["rep_code"][pm])
        if setting in ("mpclift", "lift18"):
            assert np.array_equal(u16(buf.rep_mask[p])[0, :, :n], ref["rep_mask"][p])
        if setting in VECS32:
            u32 = lambda t: t.cpu().numpy().view(np.uint32)  # noqa: E731
            assert np.array_equal(u32(buf.rep32[1][p])[0, :, :n], ref["rep_mask32"][p])
            assert np.array_equal(u32(buf.rep32[1][p])[1, :, :n], ref["rep_mask32"][pm])
            if setting == "nolift":
                assert np.array_equal(u32(buf.rep32[0][p])[0, :, :n], ref["rep_code32"][p])
        mh = buf.match[p].cpu().numpy().view(np.uint64)
        assert np.array_equal(mh[0, :, :nw], ref["match"][p]), f"match component {p}"
        assert np.array_equal(mh[1, :, :nw], ref["match"][pm])
        dh = buf.dup[p].cpu().numpy()
        assert np.array_equal(dh[0], ref["dup"][p]) and np.array_equal(dh[1], ref["dup"][pm])
    mo, s = open_match(ctx, buf)
    assert s == imc.IMC_OK
    mo = mo.cpu().numpy().view(np.uint64)
    bits = np.array([[(int(mo[r_, j // 64]) >> (j % 64)) & 1 for j in range(n)] for r_ in range(len(rot) * q)])
    assert np.array_equal(bits, match)
    do, s = open_dup(ctx, buf, q)
    assert s == imc.IMC_OK and np.array_equal(do.cpu().numpy(), dup)


@pytest.mark.parametrize("rot", [list(range(-7, 8)), [0, 3]])   # rotation-aware and expanded dot kernels
def test_code_only_dot_and_reshare(ctx, imc, keys, rot):
    """mask_dot NULL computes the code dot alone; reshare with no mask vector
    leaves the mask plane of the message untouched."""
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries

    dealer, party = keys
    n, q = 70, 2
    dc, dm = wl.gen_codes(44, 0, n)
    qc, qm = wl.gen_codes(44, 0, q, query=True)
    db = SharedDB(ctx, n)
    db.enroll(dev64(dc), dev64(dm), 0)
    qs = SharedQueries(ctx, dev64(qc), dev64(qm), 9)
    rows, ld = q * len(rot), 128
    ids = imc.make_ids(9, rot, 0)
    dots = []
    for p in range(3):
        code = torch.zeros(rows, ld, dtype=torch.int16, device="cuda")
        ctx.dot_shares(p, qs.op[p], q, ids, db.regions[p], n, n, code, None, ld)
        dots.append(code)
    msg = [torch.full((2, rows, ld), 77, dtype=torch.int16, device="cuda") for _ in range(3)]
    rep = [torch.zeros(2, rows, ld, dtype=torch.int16, device="cuda") for _ in range(3)]
    ctx.reshare(dots, None, rows, n, ld, ids, msg, rep, None)
    torch.cuda.synchronize()
    qsh = orc.share(dealer, orc.DOM_SHARE_QUERY, qc, qm, 9)
    dsh = orc.share(dealer, orc.DOM_SHARE_DB, dc, dm, 0)
    zc = np.stack([orc.local_dot(p, qsh, rot, dsh)[0] for p in range(3)])
    rc, _ = orc.reshare(party, zc, zc, q, rot, 9, 0)
    for p in range(3):
        assert np.array_equal(u16(dots[p])[:, :n], zc[p])
        assert np.array_equal(u16(rep[p])[0, :, :n], rc[p])
        assert np.all(u16(msg[p])[1] == 77)


def test_variant_argument_errors(ctx, imc):
    z = torch.zeros(2, 4, 64, dtype=torch.int16, device="cuda")
    m = torch.zeros(2, 4, 1, dtype=torch.int64, device="cuda")
    ml = torch.zeros(4, 64, dtype=torch.int16, device="cuda")
    ids = imc.make_ids(0, [0], 0)
    bad = [
        (dict(variant=9), imc.IMC_EINVAL),
        (dict(variant=imc.CMP_PLAIN_MASK, code_bits=32), imc.IMC_EINVAL),
        (dict(variant=imc.CMP_LIFT18, rep_mask=None), imc.IMC_EINVAL),
        (dict(variant=imc.CMP_PLAIN_MASK, ml_pub=None), imc.IMC_EINVAL),
        (dict(variant=imc.CMP_LIFT18, ld=32), imc.IMC_ESHAPE),
    ]
    for kw, status in bad:
        a = dict(variant=imc.CMP_LIFT18, rep_code=[z] * 3, code_bits=16, rep_mask=[z] * 3, ml_pub=ml, rows=4, n=64,
                 ld=64, ids=ids, match=[m] * 3, mw_ld=1)
        a.update(kw)
        with pytest.raises(imc.IMCError) as e:
            ctx.compare_variant(a["variant"], a["rep_code"], a["code_bits"], a["rep_mask"], a["ml_pub"], a["rows"],
                                a["n"], a["ld"], a["ids"], a["match"], a["mw_ld"])
        assert e.value.status == status, kw
    with pytest.raises(imc.IMCError) as e:
        ctx.plain_ml(m, 1, m, 64, ml, 32)
    assert e.value.status == imc.IMC_ESHAPE
