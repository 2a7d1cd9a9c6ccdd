"""GPU Galois-ring Shamir path (Sec. 4.3.2) through the C ABI against the
oracle, bit-exact: share layouts, premultiplied query operands, the
party-local dot shares over several tiles and tile configurations, row-table
dots and appends, and the full protocol on Galois shares."""
import numpy as np
import pytest

import oracle as orc
import workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GBLOCK = 4 * 800 * 32 * 16          # bytes per 32-entry block of a Galois region


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


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def u16(t):
    return t.cpu().numpy().view(np.uint16)


def limbs_to_u16(lo, hi):
    return ((lo.astype(np.int32) + 256 * hi.astype(np.int32)) & 0xFFFF).astype(np.uint16)


def decode_region(region, e):
    blk = region[(e // 32) * GBLOCK:(e // 32 + 1) * GBLOCK].reshape(4, 800, 32, 16)
    planes = blk[:, :, e % 32, :].reshape(4, 12800).view(np.int8)
    return limbs_to_u16(planes[0], planes[1]), limbs_to_u16(planes[2], planes[3])


def decode_qop(op, qi):
    row = op[qi * 51200:(qi + 1) * 51200].view(np.int8).reshape(4, 12800)
    return limbs_to_u16(row[0], row[1]), limbs_to_u16(row[2], row[3])


def test_sizes(imc):
    assert imc.galois_db_bytes(33) == 2 * GBLOCK
    assert imc.galois_db_bytes(32) * 2 == imc.db_bytes(32)
    assert imc.galois_query_op_bytes(3) == 3 * 51200
    assert imc.galois_query_raw_bytes(3) == 3 * 2 * 12800 * 2


def test_share_db_layout_and_values(ctx, imc, keys):
    dealer, _ = keys
    n, first, cap = 70, 5, 96
    dc, dm = wl.gen_codes(71, first, n)
    ref = orc.galois_share(dealer, orc.DOM_GALOIS_DB, dc, dm, first)
    regions = [torch.zeros(imc.galois_db_bytes(cap), dtype=torch.uint8, device="cuda") for _ in range(3)]
    ctx.share_db(dev64(dc), dev64(dm), n, first, regions, cap, galois=True)
    torch.cuda.synchronize()
    host = [r.cpu().numpy() for r in regions]
    for p in range(3):
        for j in (0, 1, 26, 27, 69):
            code, mask = decode_region(host[p], first + j)
            assert np.array_equal(code, ref[j, 0, p]) and np.array_equal(mask, ref[j, 1, p]), (p, j)


def test_share_query_is_lagrange_premultiplied(ctx, imc, keys):
    dealer, _ = keys
    q = 3
    qc, qm = wl.gen_codes(72, 0, q, query=True)
    ref = orc.galois_share(dealer, orc.DOM_GALOIS_QUERY, qc, qm, 40)
    _, lam = orc.galois_points()
    op = [torch.empty(imc.galois_query_op_bytes(q), dtype=torch.uint8, device="cuda") for _ in range(3)]
    raw = [torch.empty(imc.galois_query_raw_bytes(q) // 2, dtype=torch.int16, device="cuda") for _ in range(3)]
    ctx.share_query(dev64(qc), dev64(qm), q, 40, op, raw, galois=True)
    torch.cuda.synchronize()
    for p in range(3):
        oh = op[p].cpu().numpy()
        rh = u16(raw[p]).reshape(q, 2, 12800)
        for qi in range(q):
            got = decode_qop(oh, qi)
            for vec in range(2):
                sh = ref[qi, vec, p]
                assert np.array_equal(rh[qi, vec], sh)
                want = np.empty(12800, dtype=np.uint16)
                for i in range(0, 6400, 97):      # a spread of pairs through the oracle's ring product
                    want[2 * i:2 * i + 2] = orc.t_gr_mul(lam[p], sh[2 * i:2 * i + 2])
                    assert np.array_equal(got[vec][2 * i:2 * i + 2], want[2 * i:2 * i + 2]), (p, qi, vec, i)


def _setup(ctx, seed, n, q, first=0):
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries

    dc, dm = wl.gen_codes(seed, first, n)
    qc, qm = wl.gen_codes(seed, 0, q, query=True)
    db = SharedDB(ctx, first + n, galois=True)
    db.enroll(dev64(dc), dev64(dm), first)
    qs = SharedQueries(ctx, dev64(qc), dev64(qm), 100, galois=True)
    return dc, dm, qc, qm, db, qs


@pytest.mark.parametrize("tiles", [0, 1, 2, 6, 7])
@pytest.mark.parametrize("q,rot,n,first", [
    (9, list(range(-15, 16)), 300, 64),   # 279 rows: 2 row tiles, ragged; 3 column tiles, ragged
    (2, [-3, 7], 129, 0),                  # expanded path, one past a column tile
    (12, list(range(-12, 12)), 200, 0),    # r = 24: rotation-aware tiles, queries straddle row tiles
])
def test_galois_dot_matches_oracle(imc, keys, q, rot, n, first, tiles):
    from paper_2405_04463_amd.pipeline import alloc_check

    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=512, dot_tiles=tiles)
    dc, dm, qc, qm, db, qs = _setup(ctx, 73 + n, n, q, first)
    qsh = orc.galois_share(dealer, orc.DOM_GALOIS_QUERY, qc, qm, 100)
    dsh = orc.galois_share(dealer, orc.DOM_GALOIS_DB, dc, dm, first)
    buf = alloc_check(q, len(rot), n)
    ids = imc.make_ids(100, rot, first)
    for p in range(3):
        ctx.dot_shares(p, qs.op[p], q, ids, db.regions[p], db.capacity, n, buf.dot_code[p], buf.dot_mask[p], buf.ld,
                       galois=True)
    torch.cuda.synchronize()
    tot_c = np.zeros((q * len(rot), n), dtype=np.uint16)
    for p in range(3):
        rc, rm = orc.galois_local_dot(p, qsh, rot, dsh)
        assert np.array_equal(u16(buf.dot_code[p])[:, :n], rc), f"party {p} code"
        assert np.array_equal(u16(buf.dot_mask[p])[:, :n], rm), f"party {p} mask"
        tot_c += u16(buf.dot_code[p])[:, :n]
    hd, ml, _, _ = orc.plain(qc, qm, rot, dc, dm)
    assert np.array_equal(tot_c, (ml.astype(np.int64) - 2 * hd).astype(np.uint16))
    ctx.close()


def test_galois_rows_and_append(ctx, imc, keys):
    dealer, _ = keys
    n, q = 130, 3
    dc, dm, qc, qm, db, qs = _setup(ctx, 74, n, q)
    table = [(2, -15), (0, 0), (1, 7), (2, 3), (0, 0)]
    rows = torch.tensor(table, dtype=torch.int32, device="cuda")
    ld = 192
    code = torch.empty(len(table), ld, dtype=torch.int16, device="cuda")
    mask = torch.empty_like(code)
    qsh = orc.galois_share(dealer, orc.DOM_GALOIS_QUERY, qc, qm, 100)
    dsh = orc.galois_share(dealer, orc.DOM_GALOIS_DB, dc, dm, 0)
    for p in range(3):
        ctx.dot_shares_rows(p, qs.op[p], q, rows, len(table), db.regions[p], db.capacity, 0, n, code, mask, ld,
                            galois=True)
        torch.cuda.synchronize()
        for i, (qi, s) in enumerate(table):
            rc, rm = orc.galois_local_dot(p, qsh[qi:qi + 1], [s], dsh)
            assert np.array_equal(u16(code)[i, :n], rc[0]) and np.array_equal(u16(mask)[i, :n], rm[0]), (p, i)
    # append query 1's shares as a new entry: its region slots equal the query's plain shares
    from paper_2405_04463_amd.pipeline import SharedDB

    db2 = SharedDB(ctx, n + 1, galois=True)
    db2.enroll(dev64(dc), dev64(dm), 0)
    e = db2.append(qs, 1)
    torch.cuda.synchronize()
    assert e == n
    for p in range(3):
        code_e, mask_e = decode_region(db2.regions[p].cpu().numpy(), e)
        assert np.array_equal(code_e, qsh[1, 0, p]) and np.array_equal(mask_e, qsh[1, 1, p])


def test_galois_full_protocol_matches_oracle(ctx, imc, keys):
    from paper_2405_04463_amd.pipeline import alloc_check, open_dup, open_match, run_check

    dealer, party = keys
    n, q, rot, first = 200, 4, [-2, 0, 1, 5, 15], 64
    dc, dm = wl.gen_codes(75, first, n)
    qc, qm = wl.gen_codes(75, 0, q, query=True)
    qc[0], qm[0] = wl.plant(75, 0, dc[17], dm[17], 1, h=0.2)
    qc[1], qm[1] = wl.plant(75, 1, dc[150], dm[150], 5, exact="eq")
    qc[2], qm[2] = wl.plant(75, 2, dc[199], dm[199], -2, exact="lt")
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries

    db = SharedDB(ctx, first + n, galois=True)
    db.enroll(dev64(dc), dev64(dm), first)
    qs = SharedQueries(ctx, dev64(qc), dev64(qm), 100, galois=True)
    buf = alloc_check(q, len(rot), n)
    run_check(ctx, qs, rot, db, first, n, buf)
    torch.cuda.synchronize()
    ref = orc.protocol(dealer, party, qc, qm, rot, dc, dm, qid_base=100, first_entry=first, scheme="galois")
    _, _, match, dup = orc.plain(qc, qm, rot, dc, dm)
    nw = (n + 63) // 64
    for p in range(3):
        pm = (p + 2) % 3
        assert np.array_equal(u16(buf.rep_code[p])[0, :, :n], ref["rep_code"][p])
        assert np.array_equal(u16(buf.rep_mask[p])[1, :, :n], ref["rep_mask"][pm])
        mh = buf.match[p].cpu().numpy().view(np.uint64)
        assert np.array_equal(mh[0, :, :nw], ref["match"][p]) and np.array_equal(mh[1, :, :nw], ref["match"][pm])
    mo, s = open_match(ctx, buf)
    assert s == imc.IMC_OK
    mo = mo.cpu().numpy().view(np.uint64)
    bits = np.array([[(int(mo[r_, j // 64]) >> (j % 64)) & 1 for j in range(n)] for r_ in range(len(rot) * q)])
    assert np.array_equal(bits, match)
    do, s = open_dup(ctx, buf, q)
    assert s == imc.IMC_OK
    assert np.array_equal(do.cpu().numpy(), dup) and list(dup) == [1, 0, 1, 0]
