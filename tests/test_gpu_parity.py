"""GPU path (through the C ABI) against the CPU oracle, bit-exact.

Sizes span several dot tiles (128 rows x 128 entries) and several 64-entry
comparison words with ragged tails; every value compared is an integer and
must match exactly.
"""
import numpy as np
import pytest

import oracle as orc
import workload as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def imc():
    _need_gpu()
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


def decode_db(region: np.ndarray, e: int):
    """Own/prev components (code, mask) of entry e from a tiled party region."""
    blk = region[(e // 32) * 3276800:(e // 32 + 1) * 3276800].reshape(4, 1600, 32, 16)
    planes = blk[:, :, e % 32, :].reshape(4, 25600).view(np.int8).astype(np.int32)
    code = (planes[0] + 256 * planes[1]) & 0xFFFF
    mask = (planes[2] + 256 * planes[3]) & 0xFFFF
    return code.astype(np.uint16), mask.astype(np.uint16)


def decode_qop(op: np.ndarray, qi: int):
    row = op[qi * 102400:(qi + 1) * 102400].view(np.int8).astype(np.int32).reshape(4, 25600)
    code = ((row[0] + 256 * row[1]) & 0xFFFF).astype(np.uint16)
    mask = ((row[2] + 256 * row[3]) & 0xFFFF).astype(np.uint16)
    return code, mask


def test_share_db_layout_and_values(ctx, imc, keys):
    dealer, _ = keys
    n, first, cap = 70, 5, 96
    dc, dm = wl.gen_codes(31, first, n)
    ref = orc.share(dealer, orc.DOM_SHARE_DB, dc, dm, first)
    regions = [torch.zeros(imc.db_bytes(cap), dtype=torch.uint8, device="cuda") for _ in range(3)]
    ctx.share_db(dev64(dc), dev64(dm), n, first, regions, cap)
    torch.cuda.synchronize()
    host = [r.cpu().numpy() for r in regions]
    for p in range(3):
        pm = (p + 2) % 3
        for j in (0, 1, 26, 27, 69):
            code, mask = decode_db(host[p], first + j)
            assert np.array_equal(code[:12800], ref[j, 0, p]) and np.array_equal(code[12800:], ref[j, 0, pm])
            assert np.array_equal(mask[:12800], ref[j, 1, p]) and np.array_equal(mask[12800:], ref[j, 1, pm])


def test_share_query_operand_and_raw(ctx, imc, keys):
    dealer, _ = keys
    q = 3
    qc, qm = wl.gen_codes(32, 0, q, query=True)
    ref = orc.share(dealer, orc.DOM_SHARE_QUERY, qc, qm, 40)
    op = [torch.empty(imc.query_op_bytes(q), dtype=torch.uint8, device="cuda") for _ in range(3)]
    raw = [torch.empty(imc.query_raw_bytes(q) // 2, dtype=torch.int16, device="cuda") for _ in range(3)]
    ctx.share_query(dev64(qc), dev64(qm), q, 40, op, raw)
    torch.cuda.synchronize()
    for p in range(3):
        pm = (p + 2) % 3
        oh = op[p].cpu().numpy()
        rh = u16(raw[p]).reshape(q, 2, 2, 12800)
        for qi in range(q):
            code, mask = decode_qop(oh, qi)
            for vec, got in ((0, code), (1, mask)):
                assert np.array_equal(got[:12800], (ref[qi, vec, p] + ref[qi, vec, pm]).astype(np.uint16))
                assert np.array_equal(got[12800:], ref[qi, vec, p])
                assert np.array_equal(rh[qi, vec, 0], ref[qi, vec, p])
                assert np.array_equal(rh[qi, vec, 1], ref[qi, vec, pm])


def _setup(imc, ctx, seed, n, q, first=0, cap=None):
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries

    cap = cap or (first + n)
    dc, dm = wl.gen_codes(seed, first, n)
    qc, qm = wl.gen_codes(seed, 0, q, query=True)
    db = SharedDB(ctx, cap)
    db.enroll(dev64(dc), dev64(dm), first)
    qs = SharedQueries(ctx, dev64(qc), dev64(qm), 100)
    return dc, dm, qc, qm, db, qs


@pytest.mark.parametrize("tiles", [0, 1, 2, 3, 6, 7])
@pytest.mark.parametrize("q,rot,n,first", [
    (9, list(range(-15, 16)), 300, 64),   # 279 rows: 2 row tiles of 256, ragged; 3 column tiles, ragged
    (1, [0], 1, 0),                        # a single comparison
    (2, [-3, 7], 129, 0),                  # one past a column tile
    (12, list(range(-12, 12)), 200, 0),    # r = 24: rotation-aware tiles, queries straddle row tiles
    (20, list(range(-7, 8)), 130, 64),     # r = 15: 22 query slots per 256-row tile (5 staging chunks)
    (18, list(range(-6, 7)), 70, 0),       # r = 13: the smallest rotation count of the rotation-aware path
])
def test_dot_shares_matches_oracle(imc, keys, q, rot, n, first, tiles):
    from paper_2405_04463_amd.pipeline import alloc_check

    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=512, dot_tiles=tiles)
    dc, dm, qc, qm, db, qs = _setup(imc, ctx, 33 + n, n, q, first)
    qsh = orc.share(dealer, orc.DOM_SHARE_QUERY, qc, qm, 100)
    dsh = orc.share(dealer, orc.DOM_SHARE_DB, dc, dm, first)
    buf = alloc_check(q, len(rot), n)
    ids = imc.make_ids(100, rot, first)
    for p in range(3):
        ctx.dot_shares(p, qs.op[p], q, ids, db.regions[p], db.capacity, n, buf.dot_code[p], buf.dot_mask[p], buf.ld)
    torch.cuda.synchronize()
    for p in range(3):
        rc, rm = orc.local_dot(p, qsh, rot, dsh)
        assert np.array_equal(u16(buf.dot_code[p])[:, :n], rc), f"party {p} code"
        assert np.array_equal(u16(buf.dot_mask[p])[:, :n], rm), f"party {p} mask"
    ctx.close()


@pytest.mark.parametrize("rot", [list(range(-15, 16)), [-1, 2]])
def test_dot_shares_gather_matches_oracle(imc, keys, rot):
    """Gathered queries (repeated, out of order) at uniform rotations: the
    rotation-aware kernel for 31 rotations, the expanded path for 2."""
    from paper_2405_04463_amd.pipeline import alloc_check

    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=512)
    n, first = 150, 64
    dc, dm, qc, qm, db, qs = _setup(imc, ctx, 44, n, 6, first)
    qsh = orc.share(dealer, orc.DOM_SHARE_QUERY, qc, qm, 100)
    dsh = orc.share(dealer, orc.DOM_SHARE_DB, dc, dm, first)
    order = [5, 0, 3, 3, 1, 4, 2, 0, 5, 1]
    qidx = torch.tensor(order, dtype=torch.int32, device="cuda")
    buf = alloc_check(len(order), len(rot), n)
    ids = imc.make_ids(0, rot, first)
    for p in (0, 2):
        ctx.dot_shares_gather(p, qs.op[p], qidx, len(order), ids, db.regions[p], db.capacity, n, buf.dot_code[p],
                              buf.dot_mask[p], buf.ld)
    torch.cuda.synchronize()
    for p in (0, 2):
        rc, rm = orc.local_dot(p, qsh[order], rot, dsh)
        assert np.array_equal(u16(buf.dot_code[p])[:, :n], rc), p
        assert np.array_equal(u16(buf.dot_mask[p])[:, :n], rm), p
    ctx.close()


def test_full_protocol_matches_oracle(ctx, imc, keys):
    """All steps on the GPU vs the oracle's protocol run: every component."""
    from paper_2405_04463_amd.pipeline import alloc_check, open_dup, open_match, run_check

    dealer, party = keys
    n, q, rot, first = 200, 4, [-2, 0, 1, 5, 15], 64
    dc, dm = wl.gen_codes(41, first, n)
    qc, qm = wl.gen_codes(41, 0, q, query=True)
    qc[0], qm[0] = wl.plant(41, 0, dc[17], dm[17], 1, h=0.2)
    qc[1], qm[1] = wl.plant(41, 1, dc[150], dm[150], 5, exact="eq")
    qc[2], qm[2] = wl.plant(41, 2, dc[199], dm[199], -2, exact="lt")
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries

    db = SharedDB(ctx, first + n)
    db.enroll(dev64(dc), dev64(dm), first)
    qs = SharedQueries(ctx, dev64(qc), dev64(qm), 100)
    buf = alloc_check(q, len(rot), n)
    run_check(ctx, qs, rot, db, first, n, buf)
    torch.cuda.synchronize()

    ref = orc.protocol(dealer, party, qc, qm, rot, dc, dm, qid_base=100, first_entry=first)
    hd, ml, match, dup = orc.plain(qc, qm, rot, dc, dm)
    nw = (n + 63) // 64
    for p in range(3):
        pm = (p + 2) % 3
        # resharing: own component, received component and the message
        assert np.array_equal(u16(buf.rep_code[p])[0, :, :n], ref["rep_code"][p])
        assert np.array_equal(u16(buf.rep_code[p])[1, :, :n], ref["rep_code"][pm])
        assert np.array_equal(u16(buf.rep_mask[p])[0, :, :n], ref["rep_mask"][p])
        assert np.array_equal(u16(buf.msg[p])[0, :, :n], ref["rep_code"][p])
        assert np.array_equal(u16(buf.msg[p])[1, :, :n], ref["rep_mask"][p])
        # comparison: components of the shared match bits
        mh = buf.match[p].cpu().numpy().view(np.uint64)
        assert np.array_equal(mh[0, :, :nw], ref["match"][p]), f"match component {p}"
        assert np.array_equal(mh[1, :, :nw], ref["match"][pm])
        # OR-tree
        dh = buf.dup[p].cpu().numpy()
        assert np.array_equal(dh[0], ref["dup"][p]) and np.array_equal(dh[1], ref["dup"][pm])
    # opened values against the plaintext decision
    mo, s = open_match(ctx, buf)
    assert s == imc.IMC_OK
    mo = mo.cpu().numpy().view(np.uint64)
    bits = np.array([[(int(mo[r_, j // 64]) >> (j % 64)) & 1 for j in range(n)] for r_ in range(len(rot) * q)])
    assert np.array_equal(bits, match)
    do, s = open_dup(ctx, buf, q)
    assert s == imc.IMC_OK
    assert np.array_equal(do.cpu().numpy(), dup) and list(dup) == [1, 0, 1, 0]


def test_open_check_detects_corruption(ctx, imc, keys):
    from paper_2405_04463_amd.pipeline import alloc_check, open_dots, run_check

    n, q, rot = 64, 1, [0]
    dc, dm, qc, qm, db, qs = _setup(imc, ctx, 51, n, q)
    buf = alloc_check(q, len(rot), n)
    run_check(ctx, qs, rot, db, 0, n, buf)
    _, _, st = open_dots(ctx, buf)
    assert st == (imc.IMC_OK, imc.IMC_OK)
    buf.rep_code[1][1, 0, 5] ^= 1          # party 1's copy of component 0 is altered in transit
    _, _, st = open_dots(ctx, buf)
    assert st[0] == imc.IMC_ECORRUPT and st[1] == imc.IMC_OK


def test_argument_errors(ctx, imc):
    from paper_2405_04463_amd.pipeline import alloc_check

    buf = alloc_check(1, 1, 64)
    op = torch.empty(imc.query_op_bytes(1), dtype=torch.uint8, device="cuda")
    region = torch.empty(imc.db_bytes(64), dtype=torch.uint8, device="cuda")
    with pytest.raises(imc.IMCError) as e:
        ctx.dot_shares(3, op, 1, imc.make_ids(0, [0]), region, 64, 64, buf.dot_code[0], buf.dot_mask[0], buf.ld)
    assert e.value.status == imc.IMC_EINVAL
    with pytest.raises(imc.IMCError) as e:        # first entry not a multiple of 64
        ctx.dot_shares(0, op, 1, imc.make_ids(0, [0], 32), region, 128, 64, buf.dot_code[0], buf.dot_mask[0], buf.ld)
    assert e.value.status == imc.IMC_EINVAL
    with pytest.raises(imc.IMCError) as e:        # rotation out of range
        ctx.dot_shares(0, op, 1, imc.make_ids(0, [16]), region, 64, 64, buf.dot_code[0], buf.dot_mask[0], buf.ld)
    assert e.value.status == imc.IMC_EINVAL
    with pytest.raises(imc.IMCError) as e:        # more entries than the region holds
        ctx.dot_shares(0, op, 1, imc.make_ids(0, [0]), region, 64, 65, buf.dot_code[0], buf.dot_mask[0], 128)
    assert e.value.status == imc.IMC_ESHAPE
    with pytest.raises(imc.IMCError) as e:        # more rows than the context was created for
        ctx.dot_shares(0, op, 600, imc.make_ids(0, [0]), region, 64, 64, buf.dot_code[0], buf.dot_mask[0], buf.ld)
    assert e.value.status == imc.IMC_ESHAPE
    # empty work is a no-op
    ctx.dot_shares(0, op, 0, imc.make_ids(0, [0]), region, 64, 64, buf.dot_code[0], buf.dot_mask[0], buf.ld)
    # tile configurations outside the supported set
    for bad in (5, 8, 0x20):
        with pytest.raises(imc.IMCError) as e:
            ctx.set_dot_tiles(bad)
        assert e.value.status == imc.IMC_EUNSUPPORTED


def test_small_unrotated_configuration_all_components(ctx, imc, keys):
    """1,000 entries, 16 queries, no rotation, 4 queries planted at HD 0.20:
    every component of every step bit-exact against the oracle's protocol run,
    and the opened duplicate flags are exactly the planted queries."""
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries, alloc_check, open_dup, open_match, run_check

    dealer, party = keys
    w = wl.small_plain()
    dc, dm = wl.gen_codes(w.seed, 0, w.n_db)
    qc, qm = wl.make_queries(w)
    db = SharedDB(ctx, w.n_db)
    db.enroll(dev64(dc), dev64(dm), 0)
    qs = SharedQueries(ctx, dev64(qc), dev64(qm), 500)
    buf = alloc_check(w.n_q, len(w.rot), w.n_db)
    run_check(ctx, qs, w.rot, db, 0, w.n_db, buf)
    torch.cuda.synchronize()
    ref = orc.protocol(dealer, party, qc, qm, w.rot, dc, dm, qid_base=500, first_entry=0)
    _, _, match, dup = orc.plain(qc, qm, w.rot, dc, dm)
    n, nw = w.n_db, (w.n_db + 63) // 64
    for p in range(3):
        pm = (p + 2) % 3
        assert np.array_equal(u16(buf.dot_code[p])[:, :n], ref["z_code"][p])
        assert np.array_equal(u16(buf.dot_mask[p])[:, :n], ref["z_mask"][p])
        assert np.array_equal(u16(buf.rep_code[p])[0, :, :n], ref["rep_code"][p])
        assert np.array_equal(u16(buf.rep_mask[p])[1, :, :n], ref["rep_mask"][pm])
        mh = buf.match[p].cpu().numpy().view(np.uint64)
        assert np.array_equal(mh[0, :, :nw], ref["match"][p]) and np.array_equal(mh[1, :, :nw], ref["match"][pm])
        dh = buf.dup[p].cpu().numpy()
        assert np.array_equal(dh[0], ref["dup"][p]) and np.array_equal(dh[1], ref["dup"][pm])
    mo, s = open_match(ctx, buf)
    assert s == imc.IMC_OK
    mo = mo.cpu().numpy().view(np.uint64)
    bits = np.array([[(int(mo[r_, j // 64]) >> (j % 64)) & 1 for j in range(n)] for r_ in range(w.rows)])
    assert np.array_equal(bits, match)
    do, s = open_dup(ctx, buf, w.n_q)
    assert s == imc.IMC_OK
    assert sorted(np.nonzero(do.cpu().numpy())[0].tolist()) == sorted(qi for qi, _, _, _ in w.planted) == [1, 5, 9, 13]
    assert np.array_equal(do.cpu().numpy(), dup)
