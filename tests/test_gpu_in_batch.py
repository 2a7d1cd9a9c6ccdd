"""In-batch matching and the OR of two decisions on the GPU against the
oracle (components bit-exact) and the plaintext decision over the database
plus the batch's earlier queries; both eyes: persons of two queries, the
in-batch mask over earlier persons and the OR of each person's two eyes,
against the oracle and the plaintext OR over both eyes."""
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


@pytest.mark.parametrize("galois", [False, True])
def test_in_batch_matches_oracle_and_plaintext(imc, keys, galois):
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries, alloc_check, run_check, run_in_batch

    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=256)
    rot = [-1, 0, 2]
    n = 130
    dc, dm = wl.gen_codes(91, 0, n)
    qc, qm = wl.gen_codes(91, 0, 6, query=True)
    qc[3], qm[3] = wl.plant(91, 3, qc[1], qm[1], 2, h=0.2)      # duplicate of an earlier batch query
    qc[0], qm[0] = wl.plant(91, 0, qc[5], qm[5], 0, h=0.2)      # duplicate of a later one (counts for 5 only)
    qc[2], qm[2] = wl.plant(91, 2, dc[129], dm[129], -1, h=0.25)
    db = SharedDB(ctx, n, galois=galois)
    db.enroll(dev64(dc), dev64(dm), 0)
    qs = SharedQueries(ctx, dev64(qc), dev64(qm), 10, galois=galois)
    buf = alloc_check(6, len(rot), n)
    run_check(ctx, qs, rot, db, 0, n, buf)
    bb = run_in_batch(ctx, qs, rot, buf)
    torch.cuda.synchronize()
    ref = orc.protocol_in_batch(dealer, party, qc, qm, rot, dc, dm, qid_base=10,
                                scheme="galois" if galois else "aby3")
    for p in range(3):
        pm = (p + 2) % 3
        mh = bb.match[p].cpu().numpy().view(np.uint64)
        assert np.array_equal(mh[0, :, :1], ref["batch_match"][p]) and np.array_equal(mh[1, :, :1],
                                                                                   ref["batch_match"][pm])
        for name, got in (("dup_batch", bb.dup[p]), ("dup", bb.final[p])):
            g = got.cpu().numpy()
            assert np.array_equal(g[0], ref[name][p]) and np.array_equal(g[1], ref[name][pm]), (name, p)
    # a second run on the same buffers (nothing allocated) gives the same components
    first = [t.clone() for t in bb.final]
    again = run_in_batch(ctx, qs, rot, buf, reuse=bb)
    torch.cuda.synchronize()
    assert again is bb and all(torch.equal(a, b) for a, b in zip(first, bb.final))
    opened = np.bitwise_xor.reduce(np.stack([bb.final[p][0].cpu().numpy() for p in range(3)]), axis=0)
    want = [bool(orc.plain(qc[i:i + 1], qm[i:i + 1], rot, np.concatenate([dc, qc[:i]]),
                           np.concatenate([dm, qm[:i]]))[3][0]) for i in range(6)]
    assert list(opened.astype(bool)) == want == [False, False, True, True, False, True]
    ctx.close()


@pytest.mark.parametrize("galois", [False, True])
def test_two_eyes_matches_oracle_and_plaintext(imc, keys, galois):
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries, alloc_check, run_check, run_in_batch

    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=256)
    rot = [-2, 0, 1]
    n = 97                                         # two groups of entries, the second ragged
    dc, dm = wl.gen_codes(93, 0, n)
    qc, qm = wl.gen_codes(93, 0, 12, query=True)   # persons 0..5: eyes 2k (left), 2k+1 (right)
    qc[1], qm[1] = wl.plant(93, 1, dc[96], dm[96], -2, h=0.2)     # person 0: right eye in the database
    qc[4], qm[4] = wl.plant(93, 4, dc[3], dm[3], 0, h=0.22)       # person 2: both eyes in the database
    qc[5], qm[5] = wl.plant(93, 5, dc[70], dm[70], 1, h=0.3)
    # person 1 left from person 3 right: counts for person 3 (rotation -2 of eye 7 meets eye 2)
    qc[2], qm[2] = wl.plant(93, 2, qc[7], qm[7], 2, h=0.2)
    qc[9], qm[9] = wl.plant(93, 9, qc[8], qm[8], 0, h=0.1)        # person 4 right from its own left eye
    qc[10], qm[10] = wl.plant(93, 10, qc[1], qm[1], 1, h=0.25)    # person 5 left from person 0 right
    db = SharedDB(ctx, n, galois=galois)
    db.enroll(dev64(dc), dev64(dm), 0)
    qs = SharedQueries(ctx, dev64(qc), dev64(qm), 20, galois=galois)
    buf = alloc_check(12, len(rot), n)
    run_check(ctx, qs, rot, db, 0, n, buf)
    bb = run_in_batch(ctx, qs, rot, buf, group=2)
    torch.cuda.synchronize()
    ref = orc.protocol_in_batch(dealer, party, qc, qm, rot, dc, dm, qid_base=20,
                                scheme="galois" if galois else "aby3", group=2)
    for p in range(3):
        pm = (p + 2) % 3
        mh = bb.match[p].cpu().numpy().view(np.uint64)
        assert np.array_equal(mh[0, :, :1], ref["batch_match"][p]) and np.array_equal(mh[1, :, :1],
                                                                                   ref["batch_match"][pm])
        for name, got in (("dup_db", buf.dup[p]), ("dup_batch", bb.dup[p]), ("dup", bb.final[p]),
                          ("person", bb.person[p])):
            g = got.cpu().numpy()
            assert np.array_equal(g[0], ref[name][p]) and np.array_equal(g[1], ref[name][pm]), (name, p)
    opened = torch.empty(6, dtype=torch.uint8, device="cuda")
    assert ctx.open(imc.OPEN_U8_XOR, bb.person, 6, opened, 1) == imc.IMC_OK
    eyes = [bool(orc.plain(qc[i:i + 1], qm[i:i + 1], rot, np.concatenate([dc, qc[:2 * (i // 2)]]),
                           np.concatenate([dm, qm[:2 * (i // 2)]]))[3][0]) for i in range(12)]
    want = [eyes[2 * k] or eyes[2 * k + 1] for k in range(6)]
    assert list(opened.cpu().numpy().astype(bool)) == want == [True, False, True, True, False, True]
    # a second run on the same buffers (nothing allocated) gives the same components
    first = [t.clone() for t in bb.person]
    again = run_in_batch(ctx, qs, rot, buf, reuse=bb, group=2)
    torch.cuda.synchronize()
    assert again is bb and all(torch.equal(a, b) for a, b in zip(first, bb.person))
    ctx.close()


def test_or_pairs_matches_oracle(imc, keys):
    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=64)
    count = 333                                     # several words of randomness, ragged
    x = [torch.randint(0, 2, (2, 2 * count), dtype=torch.uint8, device="cuda") for _ in range(3)]
    out = [torch.empty(2, count, dtype=torch.uint8, device="cuda") for _ in range(3)]
    ctx.or_pairs(x, count, (1 << 47) | 9, out)
    torch.cuda.synchronize()
    xh = np.stack([t[0].cpu().numpy() for t in x])
    ref = orc.or_pairs(party, xh, (1 << 47) | 9)
    for p in range(3):
        assert np.array_equal(out[p][0].cpu().numpy(), ref[p]), p
        assert np.array_equal(out[p][1].cpu().numpy(), ref[(p + 2) % 3]), p
    m = [torch.zeros(2, 4, 1, dtype=torch.int64, device="cuda") for _ in range(3)]
    with pytest.raises(imc.IMCError) as e:
        ctx.mask_in_batch(m, 4, 1, 1, 0, group=0)  # a group of no queries
    assert e.value.status == imc.IMC_EINVAL
    ctx.close()


def test_or_bits_and_mask_errors(imc, keys):
    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=64)
    m = [torch.zeros(2, 65, 1, dtype=torch.int64, device="cuda") for _ in range(3)]
    with pytest.raises(imc.IMCError) as e:
        ctx.mask_in_batch(m, 65, 1, 1, 0)          # more than one word of columns
    assert e.value.status == imc.IMC_EINVAL
    with pytest.raises(imc.IMCError) as e:
        ctx.mask_in_batch(m, 4, 1, 1, 1)           # word outside the row
    assert e.value.status == imc.IMC_ESHAPE
    a = [torch.randint(0, 2, (2, 300), dtype=torch.uint8, device="cuda") for _ in range(3)]
    b = [torch.randint(0, 2, (2, 300), dtype=torch.uint8, device="cuda") for _ in range(3)]
    out = [torch.empty(2, 300, dtype=torch.uint8, device="cuda") for _ in range(3)]
    ctx.or_bits(a, b, 300, 5, out)
    torch.cuda.synchronize()
    ah = np.stack([x[0].cpu().numpy() for x in a])
    bh = np.stack([x[0].cpu().numpy() for x in b])
    ref = orc.or_bits(party, ah, bh, 5)
    for p in range(3):
        assert np.array_equal(out[p][0].cpu().numpy(), ref[p])
    ctx.close()
