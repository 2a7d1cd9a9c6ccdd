"""Edge cases of the GPU path through the C ABI: degenerate codes and masks
(the identical code, the complement, empty masks, a rotated copy), the
largest row count a context admits, a database filled to its capacity, and
calls with nothing to do.  Every result is compared with the oracle."""
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


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def _full_check(imc, ctx, keys, qc, qm, rot, dc, dm, first, capacity, qid=300):
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries, alloc_check, open_dup, open_match, run_check

    dealer, party = keys
    n, q = dc.shape[0], qc.shape[0]
    db = SharedDB(ctx, capacity)
    db.enroll(dev64(dc), dev64(dm), first)
    qs = SharedQueries(ctx, dev64(qc), dev64(qm), qid)
    buf = alloc_check(q, len(rot), n)
    run_check(ctx, qs, rot, db, first, n, buf)
    mo, s1 = open_match(ctx, buf)
    do, s2 = open_dup(ctx, buf, q)
    torch.cuda.synchronize()
    assert s1 == imc.IMC_OK and s2 == imc.IMC_OK
    ref = orc.protocol(dealer, party, qc, qm, rot, dc, dm, qid_base=qid, first_entry=first)
    nw = (n + 63) // 64
    for p in range(3):
        pm = (p + 2) % 3
        mh = buf.match[p].cpu().numpy().view(np.uint64)
        assert np.array_equal(mh[0, :, :nw], ref["match"][p]) and np.array_equal(mh[1, :, :nw], ref["match"][pm])
    mo = mo.cpu().numpy().view(np.uint64)
    bits = np.array([[(int(mo[r_, j // 64]) >> (j % 64)) & 1 for j in range(n)] for r_ in range(q * len(rot))])
    return bits, do.cpu().numpy()


def test_degenerate_codes_and_masks(imc, keys):
    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=64)
    rot = [-5, 0, 5]
    dc, dm = wl.gen_codes(81, 0, 70)
    qc, qm = wl.gen_codes(81, 0, 4, query=True)
    full = np.full(200, np.uint64(2**64 - 1), dtype=np.uint64)
    qm[0] = full                                   # query 0: every bit valid
    dc[0], dm[0] = qc[0], full                     # identical code, full masks: hd = 0
    dc[1], dm[1] = ~qc[0], full                    # complement: hd = ml, never a match
    dm[2] = 0                                      # empty entry mask: ml = 0
    qm[2] = 0                                      # query 2: empty mask, matches nothing
    b = wl.unpack(qc[1:2])[0]                      # entry 3: query 1 rotated by 5 columns
    mb = wl.unpack(qm[1:2])[0]
    dc[3] = wl.pack(wl.rotate_bits(b, 5)[None])[0]
    dm[3] = wl.pack(wl.rotate_bits(mb, 5)[None])[0]
    hd, ml, match, dup = orc.plain(qc, qm, rot, dc, dm)
    r0 = rot.index(0)
    assert match[0 * 3 + r0, 0] == 1 and hd[0 * 3 + r0, 0] == 0
    assert match[:, 1].sum() == 0 and match[:, 2].sum() == 0 and (ml[:, 2] == 0).all()
    assert match[2 * 3:3 * 3].sum() == 0 and (ml[2 * 3:3 * 3] == 0).all()
    assert match[3:6, 3].sum() == 1                # the rotated copy matches at one rotation only
    bits, d = _full_check(imc, ctx, keys, qc, qm, rot, dc, dm, 0, 70)
    assert np.array_equal(bits, match) and np.array_equal(d, dup)
    assert list(d[:3]) == [1, 1, 0]
    ctx.close()


def test_largest_row_count_and_full_capacity(imc, keys):
    dealer, party = keys
    rot = list(range(-15, 16)) + [0]               # 32 rotations (the maximum), one repeated
    q = 4
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=q * len(rot))
    first, n = 64, 57                              # entries 64..120 fill a capacity of 121
    dc, dm = wl.gen_codes(82, first, n)
    qc, qm = wl.gen_codes(82, 0, q, query=True)
    qc[3], qm[3] = wl.plant(82, 3, dc[56], dm[56], -15, h=0.1)
    _, _, match, dup = orc.plain(qc, qm, rot, dc, dm)
    bits, d = _full_check(imc, ctx, keys, qc, qm, rot, dc, dm, first, first + n)
    assert np.array_equal(bits, match) and np.array_equal(d, dup) and d[3] == 1
    # one row more than the context admits
    from paper_2405_04463_amd.pipeline import alloc_check

    buf = alloc_check(q + 1, len(rot), 64)
    op = torch.empty(imc.query_op_bytes(q + 1), dtype=torch.uint8, device="cuda")
    region = torch.empty(imc.db_bytes(64), dtype=torch.uint8, device="cuda")
    with pytest.raises(imc.IMCError) as e:
        ctx.dot_shares(0, op, q + 1, imc.make_ids(0, rot), region, 64, 64, buf.dot_code[0], buf.dot_mask[0], buf.ld)
    assert e.value.status == imc.IMC_ESHAPE
    ctx.close()


def test_calls_with_nothing_to_do(imc, keys):
    from paper_2405_04463_amd.pipeline import alloc_check

    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=8)
    buf = alloc_check(1, 1, 64)
    ids = imc.make_ids(0, [0], 0)
    sentinel = [m.clone() for m in buf.match]
    ctx.reshare(buf.dot_code, buf.dot_mask, 1, 0, buf.ld, ids, buf.msg, buf.rep_code, buf.rep_mask)
    ctx.compare_threshold(buf.rep_code, buf.rep_mask, 0, 64, buf.ld, ids, buf.match, buf.nw)
    ctx.compare_variant(imc.CMP_LIFT18, buf.rep_code, 16, buf.rep_mask, None, 1, 0, buf.ld, ids, buf.match, buf.nw)
    ctx.or_tree(buf.match, 0, 1, buf.nw, ids, buf.ws, buf.ws.numel(), buf.dup)
    ctx.plain_ml(buf.match[0], 0, buf.match[0], 64, buf.dot_code[0], buf.ld)
    assert ctx.open(imc.OPEN_U16_ADD, buf.rep_code, 0, buf.dot_code[0], 1) == imc.IMC_OK
    torch.cuda.synchronize()
    for a, b in zip(buf.match, sentinel):
        assert torch.equal(a, b)
    ctx.close()
