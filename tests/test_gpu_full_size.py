"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times, on outputs the oracle computes one by one.

* One party's dot products, 32 queries x 31 rotations (992 rows) against
  1,000,000 entries (102.4 GB of shares): every row against every planted
  entry, the first and last entries and 200 random ones, code and mask,
  against the oracle's local dot of party 0.
* The three-party protocol, 64 queries x 31 rotations against 300,000
  entries per party: the resharing components and the shared match bits of
  four 64-entry groups (the first, two random ones and the ragged last group
  of 32 entries) against the oracle's protocol run on those entries; the
  match-bit components of 32 more groups against the oracle's comparison of
  the GPU's reshared components, and for 8 of them every word of the message
  buffer (406 planes, every row) against the oracle's message log; the
  duplicate-bit components of every query
  against the oracle's OR-tree over the GPU's match-bit components of the
  whole database; every opened one re-decided by the plaintext check, the
  opened ones equal to the plaintext matches of the planted pairs and every
  opened duplicate bit equal to the plaintext one (tests/fullcheck.py).
* Both eyes at the deployed batch: 32 persons x 2 eyes x 31 rotations
  against 300,000 entries, with in-batch matching over the eyes of earlier
  persons: the database part as above (every opened bit, the OR-tree
  components), the batch part's match, duplicate, combined and person
  components against the oracle, and every opened person decision against
  the plaintext OR over its two eyes.
* The batched step of 200 uneven batches against 1,000,000 entries.
* Party-local serving over 1,500,000 entries of a 2,000,000-entry region.
* Three-party serving on Galois-ring shares of 1,500,000 entries.
* The comparison settings (public masks, Lift to Z_2^18, ConstLift, NoLift)
  at 64 queries x 31 rotations against 300,000 entries, with the same
  OR-tree and opened-bit checks.
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


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def enroll(db, seed, n, chunk=65536):
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        c, k = wl.gen_codes(seed, s, m)
        db.enroll(dev64(c), dev64(k), s)
    torch.cuda.synchronize()


def free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_party_dot_at_one_million_entries(imc, keys):
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries

    dealer, party = keys
    w = wl.party_local()
    assert (w.n_db, w.n_q, len(w.rot)) == (1_000_000, 32, 31)
    qc, qm = wl.make_queries(w)
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=w.rows)
    try:
        db = SharedDB(ctx, w.n_db, parties=(0,))
        enroll(db, w.seed, w.n_db)
        qs = SharedQueries(ctx, dev64(qc), dev64(qm), 0)
        ld = ((w.n_db + 63) // 64) * 64
        code = torch.empty(w.rows, ld, dtype=torch.int16, device="cuda")
        mask = torch.empty_like(code)
        ids = imc.make_ids(0, w.rot, 0)
        ctx.dot_shares(0, qs.op[0], qs.q, ids, db.regions[0], db.capacity, w.n_db, code, mask, ld)
        torch.cuda.synchronize()

        rng = np.random.default_rng(11)
        ents = sorted({0, w.n_db - 1} | {e for _, e, _, _ in w.planted} |
                      set(int(x) for x in rng.choice(w.n_db, 200, replace=False)))
        idx = torch.tensor(ents, dtype=torch.int64, device="cuda")
        got_c = code.index_select(1, idx).cpu().numpy().view(np.uint16)
        got_m = mask.index_select(1, idx).cpu().numpy().view(np.uint16)
        del code, mask, db, qs
        free()

        qsh = orc.share(dealer, orc.DOM_SHARE_QUERY, qc, qm, 0)
        dsh = []
        for e in ents:
            c, k = wl.gen_codes(w.seed, e, 1)
            dsh.append(orc.share(dealer, orc.DOM_SHARE_DB, c, k, e))
        want_c, want_m = orc.local_dot(0, qsh, w.rot, np.concatenate(dsh))
        assert np.array_equal(got_c, want_c)
        assert np.array_equal(got_m, want_m)
    finally:
        ctx.close()
        free()


@pytest.mark.parametrize("galois", [False, True])
def test_three_party_protocol_at_300k_entries(imc, keys, galois):
    """galois: the dot products on Galois-ring Shamir shares (the rest of the
    protocol unchanged).  Share-level parity on four groups from sharing on;
    the comparison on the GPU's own reshared components of 32 more groups,
    with every message word of 8 of them against the oracle's message log;
    every opened bit and duplicate against the plaintext decision; the
    duplicate-bit components against the oracle's OR-tree on the GPU's
    match-bit components of the whole database."""
    from fullcheck import check_every_opened_bit, check_or_tree_components
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries, alloc_check, open_dup, open_match, run_check

    dealer, party = keys
    w = wl.full_protocol()
    assert (w.n_db, w.n_q, len(w.rot)) == (300_000, 64, 31)
    n, r = w.n_db, len(w.rot)
    qc, qm = wl.make_queries(w)
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=w.rows)
    try:
        db = SharedDB(ctx, n, galois=galois)
        enroll(db, w.seed, n)
        qs = SharedQueries(ctx, dev64(qc), dev64(qm), 0, galois=galois)
        buf = alloc_check(w.n_q, r, n)
        run_check(ctx, qs, w.rot, db, 0, n, buf)
        mo, s1 = open_match(ctx, buf, check=1)
        do, s2 = open_dup(ctx, buf, w.n_q, check=1)
        torch.cuda.synchronize()
        assert s1 == imc.IMC_OK and s2 == imc.IMC_OK

        ngroups = (n + 63) // 64
        assert n % 64 == 32                                   # the last group is ragged
        rng = np.random.default_rng(12)
        groups = sorted({0, ngroups - 1} | set(int(x) for x in rng.choice(ngroups - 1, 2, replace=False)))
        more = sorted(set(int(x) for x in rng.choice(ngroups - 1, 40, replace=False)) - set(groups))[:32]
        u16 = lambda t: t.cpu().numpy().view(np.uint16)   # noqa: E731
        got = {}
        for g in groups + more:
            a, b = 64 * g, min(64 * g + 64, n)
            got[g] = [(u16(buf.rep_code[p][:, :, a:b]), u16(buf.rep_mask[p][:, :, a:b])) for p in range(3)]
        match_own = np.stack([buf.match[p][0].cpu().numpy().view(np.uint64) for p in range(3)])
        match_prev = [buf.match[p][1].cpu().numpy().view(np.uint64) for p in range(3)]
        dup_planes = [buf.dup[p].cpu().numpy() for p in range(3)]
        mo = mo.cpu().numpy().view(np.uint64)
        dup = do.cpu().numpy()
        # the message words of 8 of those groups, every row and all 406 planes,
        # gathered from the buffer's per-workgroup blocks (word t = row * nw + w
        # is lane t % 64 of block t // 64)
        nw = buf.nw
        msg_groups = more[:8]
        t = torch.arange(w.rows, dtype=torch.int64, device="cuda")[None, :] * nw
        planes = torch.arange(406, dtype=torch.int64, device="cuda")[:, None]
        msgs = {}
        for g in msg_groups:
            tg = t + g
            idx = ((tg // 64) * 406 + planes) * 64 + tg % 64
            msgs[g] = torch.take(buf.net, idx).cpu().numpy().view(np.uint64)     # [406][rows]
        del buf, db, qs
        free()
        for p in range(3):   # replicated: party p's second plane is component p-1
            assert np.array_equal(match_prev[p], match_own[(p + 2) % 3]), p

        # share level from the dealer's sharing on
        for g in groups:
            a, b = 64 * g, min(64 * g + 64, n)
            dc, dm = wl.gen_codes(w.seed, a, b - a)
            ref = orc.protocol(dealer, party, qc, qm, w.rot, dc, dm, qid_base=0, first_entry=a,
                               **({"scheme": "galois"} if galois else {}))
            for p in range(3):
                pm = (p + 2) % 3
                rc, rmk = got[g][p]
                assert np.array_equal(rc[0], ref["rep_code"][p]) and np.array_equal(rc[1], ref["rep_code"][pm]), g
                assert np.array_equal(rmk[0], ref["rep_mask"][p]) and np.array_equal(rmk[1], ref["rep_mask"][pm]), g
                assert np.array_equal(match_own[p][:, g], ref["match"][p][:, 0]), g
            _, _, match, _ = orc.plain(qc, qm, w.rot, dc, dm)
            bits = (mo[:, g][:, None] >> np.arange(b - a, dtype=np.uint64)) & np.uint64(1)
            assert np.array_equal(bits.astype(np.uint8), match), g

        # the comparison on the GPU's reshared components, 32 more groups
        for g in more:
            a = 64 * g
            d = np.stack([got[g][p][0][0] for p in range(3)])
            x = np.stack([got[g][p][1][0] for p in range(3)])
            for p in range(3):
                pm = (p + 2) % 3
                assert np.array_equal(got[g][p][0][1], d[pm]) and np.array_equal(got[g][p][1][1], x[pm]), g
            if g in msgs:      # and every message of the three parties, against the oracle's log
                ref, log = orc.compare(party, d, x, w.n_q, w.rot, 0, a, want_msg=True)
                assert np.array_equal(msgs[g], log[:, :, 0]), g
            else:
                ref = orc.compare(party, d, x, w.n_q, w.rot, 0, a)
            for p in range(3):
                assert np.array_equal(match_own[p][:, g], ref[p][:, 0]), (g, p)

        check_or_tree_components(party, match_own, dup_planes, w.n_q, r)
        nones, ndup = check_every_opened_bit(mo, dup, w, qc, qm, n)
        assert nones > 0 and ndup > 0
    finally:
        ctx.close()
        free()


def test_two_eyes_at_300k_entries(imc, keys):
    """The deployed batch shape (Sec. 6.4): the person decisions of 32
    persons, each eye checked against the database and the eyes of earlier
    persons, in the configuration of the benchmark's two-eye step."""
    from fullcheck import check_every_opened_bit, check_or_tree_components
    from paper_2405_04463_amd.pipeline import (PERSON_OR_BASE, SharedDB, SharedQueries, alloc_check, open_dup,
                                               open_match, run_check, run_in_batch)

    dealer, party = keys
    w = wl.two_eyes()
    assert (w.n_db, w.n_q, len(w.rot), w.group) == (300_000, 64, 31, 2)
    n, r = w.n_db, len(w.rot)
    qc, qm = wl.make_queries(w)
    wl.plant_in_batch(w, qc, qm, w.batch_pairs)
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=w.rows)
    try:
        db = SharedDB(ctx, n)
        enroll(db, w.seed, n)
        qs = SharedQueries(ctx, dev64(qc), dev64(qm), 0)
        buf = alloc_check(w.n_q, r, n)
        run_check(ctx, qs, w.rot, db, 0, n, buf)
        bb = run_in_batch(ctx, qs, w.rot, buf, group=2)
        mo, s1 = open_match(ctx, buf, check=1)
        do, s2 = open_dup(ctx, buf, w.n_q, check=1)
        persons = torch.empty(w.n_q // 2, dtype=torch.uint8, device="cuda")
        s3 = ctx.open(imc.OPEN_U8_XOR, bb.person, w.n_q // 2, persons, 1)
        torch.cuda.synchronize()
        assert s1 == imc.IMC_OK and s2 == imc.IMC_OK and s3 == imc.IMC_OK
        match_own = np.stack([buf.match[p][0].cpu().numpy().view(np.uint64) for p in range(3)])
        dup_planes = [buf.dup[p].cpu().numpy() for p in range(3)]
        host = lambda ts: [t.cpu().numpy() for t in ts]     # noqa: E731
        bmatch = [m.view(np.uint64) for m in host(bb.match)]
        bdup, bfinal, bperson = host(bb.dup), host(bb.final), host(bb.person)
        mo = mo.cpu().numpy().view(np.uint64)
        dup = do.cpu().numpy()
        persons = persons.cpu().numpy()
        del buf, bb, db, qs
        free()

        # the database part
        check_or_tree_components(party, match_own, dup_planes, w.n_q, r)
        nones, ndup = check_every_opened_bit(mo, dup, w, qc, qm, n)
        assert nones > 0 and ndup > 0
        # the batch part depends on the queries' shares alone: the oracle's run
        # over a one-entry database gives its components
        dc1, dm1 = wl.gen_codes(w.seed, 0, 1)
        ref = orc.protocol_in_batch(dealer, party, qc, qm, w.rot, dc1, dm1, qid_base=0, group=2)
        dup_db = np.stack([dup_planes[p][0] for p in range(3)])
        final = orc.or_bits(party, dup_db, ref["dup_batch"], 0)
        person = orc.or_pairs(party, final, PERSON_OR_BASE)
        for p in range(3):
            pm = (p + 2) % 3
            assert np.array_equal(bmatch[p][0, :, :1], ref["batch_match"][p]), p
            assert np.array_equal(bmatch[p][1, :, :1], ref["batch_match"][pm]), p
            for name, got, want in (("dup_batch", bdup, ref["dup_batch"]), ("dup", bfinal, final),
                                    ("person", bperson, person)):
                assert np.array_equal(got[p][0], want[p]) and np.array_equal(got[p][1], want[pm]), (name, p)
        # every opened person decision against the plaintext over both eyes
        batch = np.zeros(w.n_q, dtype=np.uint8)
        for i in range(2, w.n_q):
            k = 2 * (i // 2)
            batch[i] = orc.plain(qc[i:i + 1], qm[i:i + 1], w.rot, qc[:k], qm[:k])[3][0]
        eyes = dup.astype(np.uint8) | batch
        assert np.array_equal(persons, eyes[0::2] | eyes[1::2])
        assert batch[[22, 39, 55]].all() and batch.sum() == 3       # the in-batch pairs that count
        assert not batch[31] and not batch[62]                       # own left eye; exactly at the threshold
    finally:
        ctx.close()
        free()


def test_batched_step_at_one_million_entries(imc, keys):
    """200 uneven batches (1..64 queries, 1/15/31 rotations) against one
    party's 1,000,000 entries in 65,536-entry chunks, the tile choice made by
    the autotuner as in the benchmark: every row of every batch against 16
    entries of the last (ragged) chunk, including its first and last."""
    from paper_2405_04463_amd.batch import BatchedStep, BatchSet, uneven_batches
    from paper_2405_04463_amd.pipeline import SharedDB

    dealer, party = keys
    seed, n, chunk = 0x1A150004, 1_000_000, 65536
    batches = uneven_batches(200, seed=seed)
    nq = sum(b.q for b in batches)
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=sum(b.rows for b in batches))
    try:
        db = SharedDB(ctx, n, parties=(0,))
        enroll(db, seed, n)
        qc, qm = wl.gen_codes(seed, 0, nq, query=True)
        bs = BatchSet(ctx, batches, dev64(qc), dev64(qm))
        st = BatchedStep(ctx, bs, db, 0, n, chunk=chunk, parties=(0,))
        st.autotune(probe_n=16384)
        st.run()
        torch.cuda.synchronize()
        c0 = (n - 1) // chunk * chunk                         # first entry of the last chunk
        rng = np.random.default_rng(13)
        cols = sorted({0, n - 1 - c0} | set(int(x) for x in rng.choice(n - c0, 14, replace=False)))
        idx = torch.tensor(cols, dtype=torch.int64, device="cuda")
        got_c = st.dot_code[0].index_select(1, idx).cpu().numpy().view(np.uint16)
        got_m = st.dot_mask[0].index_select(1, idx).cpu().numpy().view(np.uint16)
        rbase = list(bs.rbase)
        del st, bs, db
        free()

        dsh = []
        for j in cols:
            c, k = wl.gen_codes(seed, c0 + j, 1)
            dsh.append(orc.share(dealer, orc.DOM_SHARE_DB, c, k, c0 + j))
        dsh = np.concatenate(dsh)
        q0 = 0
        for bi, b in enumerate(batches):
            qsh = orc.share(dealer, orc.DOM_SHARE_QUERY, qc[q0:q0 + b.q], qm[q0:q0 + b.q], b.qid_base)
            rc, rm = orc.local_dot(0, qsh, b.rot, dsh)
            r0 = rbase[bi]
            assert np.array_equal(got_c[r0:r0 + b.rows], rc), bi
            assert np.array_equal(got_m[r0:r0 + b.rows], rm), bi
            q0 += b.q
    finally:
        ctx.close()
        free()


def _drive(srv, reqs_at_tick):
    """Submit requests at given ticks and tick until all are done."""
    total = len(srv.done) + sum(len(v) for v in reqs_at_tick.values())
    t = 0
    while len(srv.done) < total:
        for r in reqs_at_tick.get(t, []):
            srv.submit(r)
        if not srv.tick():
            torch.cuda.synchronize()
        t += 1
        assert t < 5000, srv.state()
    torch.cuda.synchronize()
    return {r.rid: r for r in srv.done}


def test_party_local_serving_at_1_5M_entries(imc, keys):
    """One party's share of the service over a region of 2,000,000 entries
    holding 1,500,000 (204.8 GB allocated), 31 rotations, 65,536-entry chunks
    (the last one ragged): each request's dot outputs over the whole
    database, on the planted, first, last and 100 random entries, equal the
    oracle's party-0 local dots; a request gives the same outputs alone and
    joining a mix mid-cycle; the decided uniques are appended."""
    from paper_2405_04463_amd.pipeline import SharedDB
    from paper_2405_04463_amd.serve import Request, Server

    dealer, party = keys
    seed, n0, cap, chunk = 0x1A150005, 1_500_000, 2_000_000, 65536
    assert n0 % chunk != 0
    rot = wl.ROT31
    qc, qm = wl.gen_codes(seed, 0, 4, query=True)
    planted = {0: (1_234_567, 5, 0.20), 1: (n0 - 1, -9, 0.25)}
    for qi, (e, s, h) in planted.items():
        ec, em = wl.gen_codes(seed, e, 1)
        qc[qi], qm[qi] = wl.plant(seed, qi, ec[0], em[0], s, h=h)
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=64 * len(rot))
    try:
        db = SharedDB(ctx, cap, parties=(0,))
        enroll(db, seed, n0)
        req = lambda i: Request(rid=i, qid=7000 + i, code=qc[i].copy(), mask=qm[i].copy())   # noqa: E731
        decide = lambda r: 1 if r.rid in planted else 0                                        # noqa: E731
        alone = _drive(Server(ctx, db, rot, chunk=chunk, slots=64, append=False, keep_shares=True, decide=decide),
                       {0: [req(0)]})[0]
        srv = Server(ctx, db, rot, chunk=chunk, slots=64, append=True, keep_shares=True, decide=decide)
        done = _drive(srv, {0: [req(1), req(2)], 3: [req(0)], 7: [req(3)]})
        assert torch.equal(alone.dots[0][0], done[0].dots[0][0]) and torch.equal(alone.dots[0][1], done[0].dots[0][1])
        rng = np.random.default_rng(14)
        ents = sorted({0, n0 - 1} | {e for e, _, _ in planted.values()} |
                      set(int(x) for x in rng.choice(n0, 100, replace=False)))
        idx = torch.tensor(ents, dtype=torch.int64, device="cuda")
        got = {}
        for rid, r in done.items():
            assert r.snapshot == n0, rid
            got[rid] = (r.dots[0][0].index_select(1, idx).cpu().numpy().view(np.uint16),
                        r.dots[0][1].index_select(1, idx).cpu().numpy().view(np.uint16))
        assert db.n == n0 + sum(1 for r in done.values() if r.dup == 0)
        assert sorted(r.dup for r in done.values()) == [0, 0, 1, 1]
        del alone, srv, done, db
        free()

        qsh = orc.share(dealer, orc.DOM_SHARE_QUERY, qc, qm, 7000)
        dsh = []
        for e in ents:
            c, k = wl.gen_codes(seed, e, 1)
            dsh.append(orc.share(dealer, orc.DOM_SHARE_DB, c, k, e))
        dsh = np.concatenate(dsh)
        for rid, (gc, gm) in got.items():
            want_c, want_m = orc.local_dot(0, qsh[rid:rid + 1], rot, dsh)
            assert np.array_equal(gc, want_c), rid
            assert np.array_equal(gm, want_m), rid
    finally:
        ctx.close()
        free()


def test_three_party_galois_serving_at_1_5M_entries(imc, keys):
    """The three-party service on Galois-ring shares of 1,500,000 entries
    (230 GB), 31 rotations, 65,536-entry chunks (the last one ragged), one
    resharing and one comparison call per tick: two requests planted as
    near-duplicates of database entries are decided duplicates and two
    random ones unique (and appended); a request's match components over
    the database are the same alone and joining a mix mid-cycle; every
    opened match bit of every request is re-decided by the plaintext check
    on its pair and the planted pairs are among them."""
    from paper_2405_04463_amd.pipeline import SharedDB
    from paper_2405_04463_amd.serve import Request, Server

    dealer, party = keys
    seed, n0, chunk = 0x1A150005, 1_500_000, 65536
    assert n0 % chunk != 0 and n0 % 64 != 0
    rot = wl.ROT31
    qc, qm = wl.gen_codes(seed ^ 0x3E, 0, 4, query=True)
    planted = {0: (987_654, -4), 2: (n0 - 1, 11)}
    for qi, (e, s) in planted.items():
        ec, em = wl.gen_codes(seed, e, 1)
        qc[qi], qm[qi] = wl.plant(seed, 9000 + qi, ec[0], em[0], s, h=0.2)
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=64 * len(rot))
    try:
        db = SharedDB(ctx, n0 + 64, galois=True)
        enroll(db, seed, n0)
        req = lambda i: Request(rid=i, qid=9000 + i, code=qc[i].copy(), mask=qm[i].copy())   # noqa: E731
        alone = _drive(Server(ctx, db, rot, chunk=chunk, slots=64, append=False, keep_shares=True),
                       {0: [req(0)]})[0]
        free()
        srv = Server(ctx, db, rot, chunk=chunk, slots=64, append=True, keep_shares=True)
        done = _drive(srv, {0: [req(1), req(2)], 3: [req(0)], 7: [req(3)]})
        assert {rid: r.dup for rid, r in done.items()} == {0: 1, 1: 0, 2: 1, 3: 0}
        assert alone.dup == 1 and db.n == n0 + 2
        # whole words below the snapshot, and the snapshot's word up to it (past it
        # the mix also compared the entry appended meanwhile, serial order)
        full, keep = n0 // 64, np.int64((1 << (n0 % 64)) - 1)
        for p in range(3):
            assert np.array_equal(alone.match[p][:, :, :full], done[0].match[p][:, :, :full]), p
            assert np.array_equal(alone.match[p][:, :, full] & keep, done[0].match[p][:, :, full] & keep), p
        del srv
        free()
        for rid, r in done.items():
            assert r.snapshot == n0 and r.checked >= n0, rid
            opened = r.match[0][0] ^ r.match[1][0] ^ r.match[2][0]      # [rows][words], plane 0 of each party
            ones = [(row, 64 * w + b) for row, w in zip(*np.nonzero(opened))
                    for b in range(64) if (int(opened[row, w]) >> b) & 1]
            assert all(e < r.checked for _, e in ones), rid
            for row, e in ones:
                if e < n0:
                    ec, em = wl.gen_codes(seed, e, 1)
                else:                                   # an appended request's code
                    j = e - n0
                    ec, em = qc[[1, 3][j]:[1, 3][j] + 1], qm[[1, 3][j]:[1, 3][j] + 1]
                assert orc.plain(qc[rid:rid + 1], qm[rid:rid + 1], rot, ec, em)[2][row, 0], (rid, row, e)
            if rid in planted:
                assert any(e == planted[rid][0] for _, e in ones), rid
            else:
                assert not ones, rid
    finally:
        ctx.close()
        free()


@pytest.mark.parametrize("setting", ["plain", "lift18", "constlift", "nolift"])
def test_comparison_settings_at_300k_entries(imc, keys, setting):
    """The other comparison settings of the full protocol at 64 queries x 31
    rotations against 300,000 entries per party, as the benchmark runs them:
    the components of the compared values (public ml, reshared Z_2^16 or
    Z_2^32 shares) and of the match bits on four sampled 64-entry groups
    (the ragged last one among them) against the oracle's protocol in the
    same setting, the opened bits of those groups against the plaintext
    decision, the duplicate-bit components against the oracle's OR-tree over
    the GPU's match-bit components, and every opened bit and duplicate bit
    against the plaintext decision."""
    from fullcheck import check_every_opened_bit, check_or_tree_components
    from paper_2405_04463_amd.pipeline import (VECS32, SharedDB, SharedDB32, SharedQueries, SharedQueries32,
                                               alloc_check, open_dup, open_match, run_check)

    dealer, party = keys
    w = wl.full_protocol()
    n, r = w.n_db, len(w.rot)
    qc, qm = wl.make_queries(w)
    v32 = VECS32.get(setting, ())
    code16, plain = 0 not in v32, setting == "plain"
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=w.rows)
    try:
        db = SharedDB(ctx, n) if code16 else None
        db32 = SharedDB32(ctx, n, vecs=v32) if v32 else None
        db_masks = torch.empty(n, 200, dtype=torch.int64, device="cuda") if plain else None
        for s in range(0, n, 65536):
            m = min(65536, n - s)
            c, k = wl.gen_codes(w.seed, s, m)
            cd, kd = dev64(c), dev64(k)
            if db is not None:
                db.enroll(cd, kd, s)
            if db32 is not None:
                db32.enroll(cd, kd, s)
            if db_masks is not None:
                db_masks[s:s + m] = kd
        q_codes, q_masks = dev64(qc), dev64(qm)
        qs = SharedQueries(ctx, q_codes, q_masks, 0) if code16 else None
        qs32 = SharedQueries32(ctx, q_codes, q_masks, 0, vecs=v32) if v32 else None
        buf = alloc_check(w.n_q, r, n, compare=setting)
        run_check(ctx, qs, w.rot, db, 0, n, buf, query_masks=q_masks, db_masks=db_masks, qs32=qs32, db32=db32)
        mo, s1 = open_match(ctx, buf, check=1)
        do, s2 = open_dup(ctx, buf, w.n_q, check=1)
        torch.cuda.synchronize()
        assert s1 == imc.IMC_OK and s2 == imc.IMC_OK

        ngroups = (n + 63) // 64
        rng = np.random.default_rng(15)
        groups = sorted({0, ngroups - 1} | set(int(x) for x in rng.choice(ngroups - 1, 2, replace=False)))
        u16 = lambda t: t.cpu().numpy().view(np.uint16)   # noqa: E731
        u32 = lambda t: t.cpu().numpy().view(np.uint32)   # noqa: E731
        got = {}
        for g in groups:
            a, b = 64 * g, min(64 * g + 64, n)
            got[g] = {"match": [buf.match[p][:, :, g].cpu().numpy().view(np.uint64) for p in range(3)]}
            if code16:
                got[g]["rep_code"] = [u16(buf.rep_code[p][:, :, a:b]) for p in range(3)]
            if setting == "lift18":
                got[g]["rep_mask"] = [u16(buf.rep_mask[p][:, :, a:b]) for p in range(3)]
            if plain:
                got[g]["ml_pub"] = u16(buf.ml_pub[:, a:b])
            for v in v32:
                got[g]["rep32_%d" % v] = [u32(buf.rep32[v][p][:, :, a:b]) for p in range(3)]
        match_own = np.stack([buf.match[p][0].cpu().numpy().view(np.uint64) for p in range(3)])
        dup_planes = [buf.dup[p].cpu().numpy() for p in range(3)]
        mo = mo.cpu().numpy().view(np.uint64)
        dup = do.cpu().numpy()
        del buf, db, db32, db_masks, qs, qs32
        free()

        for g in groups:
            a, b = 64 * g, min(64 * g + 64, n)
            dc, dm = wl.gen_codes(w.seed, a, b - a)
            ref = orc.protocol(dealer, party, qc, qm, w.rot, dc, dm, qid_base=0, first_entry=a,
                               compare_setting=setting)
            _, ml, match, _ = orc.plain(qc, qm, w.rot, dc, dm)
            if plain:
                assert np.array_equal(got[g]["ml_pub"], ml.astype(np.uint16)), g
            for p in range(3):
                pm = (p + 2) % 3
                mt = got[g]["match"][p]
                assert np.array_equal(mt[0], ref["match"][p][:, 0]) and np.array_equal(mt[1], ref["match"][pm][:, 0])
                pairs = []
                if code16:
                    pairs.append(("rep_code", "rep_code"))
                if setting == "lift18":
                    pairs.append(("rep_mask", "rep_mask"))
                if 1 in v32:
                    pairs.append(("rep32_1", "rep_mask32"))
                if 0 in v32:
                    pairs.append(("rep32_0", "rep_code32"))
                for gk, rk in pairs:
                    x = got[g][gk][p]
                    assert np.array_equal(x[0], ref[rk][p]) and np.array_equal(x[1], ref[rk][pm]), (g, gk, p)
            bits = (mo[:, g][:, None] >> np.arange(b - a, dtype=np.uint64)) & np.uint64(1)
            assert np.array_equal(bits.astype(np.uint8), match), g

        check_or_tree_components(party, match_own, dup_planes, w.n_q, r)
        nones, ndup = check_every_opened_bit(mo, dup, w, qc, qm, n)
        assert nones > 0 and ndup > 0
    finally:
        ctx.close()
        free()
