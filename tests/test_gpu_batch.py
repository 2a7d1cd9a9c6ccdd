"""Batched uneven steps (one dot launch over the rows of many batches) against
per-batch launches, the oracle, and HIP-graph replays; bit-exact.  The fused
launch of several rotation lists (imc_dot_shares_groups), one tile per
workgroup and as a persistent grid walking several tiles per workgroup,
against one imc_dot_shares launch per group and the oracle on sampled
entries."""
import numpy as np
import pytest

import oracle as orc
import workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env(keys):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_04463_amd as imc
    from paper_2405_04463_amd.batch import Batch, BatchSet
    from paper_2405_04463_amd.pipeline import SharedDB

    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=1024)
    n, first = 200, 64
    dc, dm = wl.gen_codes(61, first, n)
    db = SharedDB(ctx, first + n)
    d64 = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()  # noqa: E731
    db.enroll(d64(dc), d64(dm), first)
    batches = [Batch(3, wl.rotations(31), 500), Batch(2, [0], 510), Batch(4, wl.rotations(15), 520),
               Batch(1, wl.rotations(31), 530), Batch(5, [0], 540), Batch(19, wl.rotations(15), 550)]
    qc, qm = wl.gen_codes(61, 0, sum(b.q for b in batches), query=True)
    qc[1], qm[1] = wl.plant(61, 1, dc[7], dm[7], 4, h=0.2)       # batch 0, query 1 at rotation 4
    qc[3], qm[3] = wl.plant(61, 3, dc[150], dm[150], 0, h=0.3)   # batch 1, query 0 (R = 1)
    bs = BatchSet(ctx, batches, d64(qc), d64(qm))
    torch.cuda.synchronize()
    yield dict(imc=imc, ctx=ctx, db=db, bs=bs, batches=batches, qc=qc, qm=qm, dc=dc, dm=dm, n=n, first=first,
               dealer=dealer, party=party)
    ctx.close()


def _u16(t):
    return t.cpu().numpy().view(np.uint16)


@pytest.mark.parametrize("mode,tiles", [("grouped", 0), ("rows", 0), ("fused", 4), ("fused", 0x14)])
def test_batched_equals_plain_and_oracle(env, mode, tiles):
    from paper_2405_04463_amd.batch import BatchedStep

    e = env
    e["ctx"].set_dot_tiles(tiles)
    st = BatchedStep(e["ctx"], e["bs"], e["db"], e["first"], e["n"], parties=(0, 1, 2), compare=True, mode=mode)
    st.run()
    torch.cuda.synchronize()
    e["ctx"].set_dot_tiles(0)
    got = {p: (_u16(st.dot_code[p]).copy(), _u16(st.dot_mask[p]).copy()) for p in range(3)}
    dup_b = [[pb["dup"][p].cpu().numpy().copy() for p in range(3)] for pb in st.per_batch]
    match_b = [[pb["match"][p].cpu().numpy().copy() for p in range(3)] for pb in st.per_batch]
    st.run_plain()
    torch.cuda.synchronize()
    for p in range(3):
        assert np.array_equal(_u16(st.dot_code[p]), got[p][0]) and np.array_equal(_u16(st.dot_mask[p]), got[p][1])
    # the comparison of each rotation list in one call gives every component of
    # the per-batch calls of the plain form
    for bi, pb in enumerate(st.per_batch):
        for p in range(3):
            assert np.array_equal(pb["match"][p].cpu().numpy(), match_b[bi][p]), (bi, p)
            assert np.array_equal(pb["dup"][p].cpu().numpy(), dup_b[bi][p]), (bi, p)
    # party 0 and 2 dot shares vs the oracle, batch by batch
    dsh = orc.share(e["dealer"], orc.DOM_SHARE_DB, e["dc"], e["dm"], e["first"])
    q0 = 0
    for bi, b in enumerate(e["batches"]):
        qsh = orc.share(e["dealer"], orc.DOM_SHARE_QUERY, e["qc"][q0:q0 + b.q], e["qm"][q0:q0 + b.q], b.qid_base)
        r0 = e["bs"].rbase[bi]
        for p in (0, 2):
            rc, rm = orc.local_dot(p, qsh, b.rot, dsh)
            assert np.array_equal(got[p][0][r0:r0 + b.rows, :e["n"]], rc), (bi, p)
            assert np.array_equal(got[p][1][r0:r0 + b.rows, :e["n"]], rm), (bi, p)
        # opened per-batch decision vs the plaintext oracle
        _, _, _, dup = orc.plain(e["qc"][q0:q0 + b.q], e["qm"][q0:q0 + b.q], b.rot, e["dc"], e["dm"])
        opened = dup_b[bi][0][0] ^ dup_b[bi][1][0] ^ dup_b[bi][2][0]
        assert np.array_equal(opened, dup), bi
        q0 += b.q
    assert dup_b[0][0][0][1] ^ dup_b[0][1][0][1] ^ dup_b[0][2][0][1] == 1
    assert dup_b[1][0][0][0] ^ dup_b[1][1][0][0] ^ dup_b[1][2][0][0] == 1


def test_chunked_db_walk_equals_one_pass(env):
    from paper_2405_04463_amd.batch import BatchedStep

    e = env
    one = BatchedStep(e["ctx"], e["bs"], e["db"], e["first"], e["n"], parties=(1,))
    one.run()
    torch.cuda.synchronize()
    ref = _u16(one.dot_code[1]).copy()
    ch = BatchedStep(e["ctx"], e["bs"], e["db"], e["first"], e["n"], chunk=64, parties=(1,))
    outs = []
    for c0, m in ch._chunks():
        e["ctx"].dot_shares_rows(1, e["bs"].op[1], e["bs"].q, e["bs"].rows, e["bs"].nrows, e["db"].regions[1],
                                 e["db"].capacity, e["first"] + c0, m, ch.dot_code[1], ch.dot_mask[1], ch.ld)
        torch.cuda.synchronize()
        outs.append(_u16(ch.dot_code[1])[:, :m].copy())
    assert np.array_equal(np.concatenate(outs, axis=1), ref[:, :e["n"]])


@pytest.mark.parametrize("mode,tiles", [("rows", 1), ("rows", 0x11), ("grouped", 0), ("fused", 0x14)])
def test_graph_replay_matches_eager(env, mode, tiles):
    from paper_2405_04463_amd.batch import BatchedStep

    e = env
    imc = e["imc"]
    e["ctx"].set_dot_tiles(tiles)
    st = BatchedStep(e["ctx"], e["bs"], e["db"], e["first"], e["n"], parties=(0,), mode=mode)
    n = e["n"]
    st.run()
    torch.cuda.synchronize()
    ref = (_u16(st.dot_code[0])[:, :n].copy(), _u16(st.dot_mask[0])[:, :n].copy())
    st.capture()
    for i in range(3):
        st.dot_code[0].zero_()
        st.dot_mask[0].zero_()
        st.replay()
        torch.cuda.synchronize()
        got = (_u16(st.dot_code[0])[:, :n], _u16(st.dot_mask[0])[:, :n])
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), i
        st.run_plain()           # eager work between replays
        torch.cuda.synchronize()
    e["ctx"].set_dot_tiles(imc.DOT_TILES_AUTO)


def test_graph_replay_of_the_three_party_step(env):
    """A captured step with every party's dots, the resharing and comparison
    of each rotation list in one call, and the per-batch OR-trees: every
    replay gives the eager step's match and decision components."""
    from paper_2405_04463_amd.batch import BatchedStep

    e = env
    st = BatchedStep(e["ctx"], e["bs"], e["db"], e["first"], e["n"], parties=(0, 1, 2), compare=True,
                     mode="grouped")
    st.run()
    torch.cuda.synchronize()
    ref = [[(pb["match"][p].cpu().numpy().copy(), pb["dup"][p].cpu().numpy().copy()) for p in range(3)]
           for pb in st.per_batch]
    st.capture()
    for i in range(3):
        for pb in st.per_batch:
            for p in range(3):
                pb["match"][p].zero_()
                pb["dup"][p].zero_()
        st.replay()
        torch.cuda.synchronize()
        for bi, pb in enumerate(st.per_batch):
            for p in range(3):
                assert np.array_equal(pb["match"][p].cpu().numpy(), ref[bi][p][0]), (i, bi, p)
                assert np.array_equal(pb["dup"][p].cpu().numpy(), ref[bi][p][1]), (i, bi, p)
        st.run_plain()           # eager work between replays
        torch.cuda.synchronize()


def test_autotune_keeps_the_fastest_and_outputs_are_unchanged(env):
    """The autotuner times every (mode, tile configuration) candidate on a
    probe slice and keeps the fastest; whichever it keeps, the outputs are the
    ones of the default configuration."""
    from paper_2405_04463_amd.batch import BatchedStep
    from paper_2405_04463_amd.tune import CANDIDATES_FUSED, CANDIDATES_ROWS, CANDIDATES_UNIFORM

    e = env
    imc = e["imc"]
    n = e["n"]
    e["ctx"].set_dot_tiles(imc.DOT_TILES_AUTO)
    ref = BatchedStep(e["ctx"], e["bs"], e["db"], e["first"], n, parties=(0,))
    ref.run()
    torch.cuda.synchronize()
    want = (_u16(ref.dot_code[0])[:, :n].copy(), _u16(ref.dot_mask[0])[:, :n].copy())
    st = BatchedStep(e["ctx"], e["bs"], e["db"], e["first"], n, parties=(0,))
    mode, flags, times = st.autotune(probe_n=128, reps=1)
    assert set(times) == ({("rows", c) for c in CANDIDATES_ROWS} | {("grouped", c) for c in CANDIDATES_UNIFORM}
                          | {("fused", c) for c in CANDIDATES_FUSED})
    assert times[(mode, flags)] == min(times.values()) and st.mode == mode
    st.run()
    torch.cuda.synchronize()
    assert np.array_equal(_u16(st.dot_code[0])[:, :n], want[0]) and np.array_equal(_u16(st.dot_mask[0])[:, :n], want[1])
    e["ctx"].set_dot_tiles(imc.DOT_TILES_AUTO)


@pytest.mark.parametrize("persistent,galois", [(False, False), (True, False), (True, True)])
def test_dot_groups_equal_per_group_launches_and_oracle(env, persistent, galois):
    """Two rotation lists (31 and 15) over 16,480 entries in one launch: 640
    tiles, so the persistent grid walks two or three tiles per workgroup; the
    outputs equal one imc_dot_shares launch per group bit for bit, and the
    oracle's local dot on the first 64 and the last 96 entries (a ragged
    column tile).  galois: the same on Galois-ring Shamir operands (K =
    12,800)."""
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries

    e = env
    imc, ctx = e["imc"], e["ctx"]
    n = 16384 + 96
    d64 = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()  # noqa: E731
    dc, dm = wl.gen_codes(62, 0, n)
    db = SharedDB(ctx, n, galois=galois)
    for s0 in range(0, n, 8192):
        db.enroll(d64(dc[s0:s0 + 8192]), d64(dm[s0:s0 + 8192]), s0)
    qc, qm = wl.gen_codes(62, 0, 50, query=True)
    qc[3], qm[3] = wl.plant(62, 3, dc[n - 5], dm[n - 5], -7, h=0.2)
    groups = [(SharedQueries(ctx, d64(qc[:20]), d64(qm[:20]), 700, galois=galois), wl.rotations(31)),
              (SharedQueries(ctx, d64(qc[20:]), d64(qm[20:]), 720, galois=galois), wl.rotations(15))]
    ld = n + 64
    outs = [[torch.zeros(qs.q * len(rot), ld, dtype=torch.int16, device="cuda") for _ in range(4)]
            for qs, rot in groups]
    ctx.set_dot_tiles(imc.DOT_TILES_ROTATION | (imc.DOT_PERSISTENT if persistent else 0))
    try:
        for p in (0, 2):
            desc = [(qs.op[p], qs.q, rot, o[0], o[1]) for (qs, rot), o in zip(groups, outs)]
            desc.insert(1, (groups[0][0].op[p], 0, wl.rotations(31), outs[0][0], outs[0][1]))   # empty: skipped
            ctx.dot_shares_groups(p, desc, db.regions[p], db.capacity, 0, n, ld, galois=galois)
            for (qs, rot), o in zip(groups, outs):
                ctx.dot_shares(p, qs.op[p], qs.q, imc.make_ids(0, rot, 0), db.regions[p], db.capacity, n, o[2], o[3],
                               ld, galois=galois)
            torch.cuda.synchronize()
            for gi, o in enumerate(outs):
                assert torch.equal(o[0][:, :n], o[2][:, :n]) and torch.equal(o[1][:, :n], o[3][:, :n]), (p, gi)
                assert not o[0][:, n:].any(), (p, gi)          # nothing written past the last entry
            # the oracle on sampled entries (party 0)
            for a, b in ((0, 64), (n - 96, n)) if p == 0 else ():
                share, dot = ((orc.galois_share, orc.galois_local_dot) if galois else (orc.share, orc.local_dot))
                dom_db, dom_q = ((orc.DOM_GALOIS_DB, orc.DOM_GALOIS_QUERY) if galois
                                 else (orc.DOM_SHARE_DB, orc.DOM_SHARE_QUERY))
                dsh = share(e["dealer"], dom_db, dc[a:b], dm[a:b], a)
                for (qs, rot), o, (q0, q1) in zip(groups, outs, ((0, 20), (20, 50))):
                    qsh = share(e["dealer"], dom_q, qc[q0:q1], qm[q0:q1], qs.qid_base)
                    rc, rm = dot(p, qsh, rot, dsh)
                    assert np.array_equal(_u16(o[0])[:, a:b], rc) and np.array_equal(_u16(o[1])[:, a:b], rm), (p, a)
    finally:
        ctx.set_dot_tiles(imc.DOT_TILES_AUTO)
        del db
        torch.cuda.empty_cache()


def test_dot_groups_argument_errors(env):
    e = env
    imc, ctx, bs = e["imc"], e["ctx"], e["bs"]
    out = torch.zeros(64 * 31, 256, dtype=torch.int16, device="cuda")
    g31 = (bs.op[0], 1, wl.rotations(31), out, out)
    cases = [([(bs.op[0], 1, [0], out, out)], 0),                    # fewer than 13 rotations
             ([g31, (bs.op[0], 1, wl.rotations(15), out, None)], 0),  # mask output in one group only
             ([g31] * 9, 0),                                          # more groups than the launch takes
             ([g31], 32)]                                             # first entry not a multiple of 64
    for desc, first in cases:
        with pytest.raises(imc.IMCError) as err:
            ctx.dot_shares_groups(0, desc, e["db"].regions[0], e["db"].capacity, first, 64, 256)
        assert err.value.status == imc.IMC_EINVAL
    with pytest.raises(imc.IMCError) as err:                                # ld < n
        ctx.dot_shares_groups(0, [g31], e["db"].regions[0], e["db"].capacity, 0, 200, 128)
    assert err.value.status == imc.IMC_ESHAPE
    with pytest.raises(imc.IMCError) as err:                                # past the region's capacity
        ctx.dot_shares_groups(0, [g31], e["db"].regions[0], e["db"].capacity, 64, e["db"].capacity, 1 << 20)
    assert err.value.status == imc.IMC_ESHAPE
