"""Continuous-batching service: results are the same alone, in a mix (joining
mid-cycle at another chunk) and on the plain per-query path; opened results
agree with the oracle; unique requests are appended; every (request,
rotation, entry) is compared once, so each gate's randomness is used once."""
import numpy as np
import pytest

import oracle as orc
import workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROT = [-2, 0, 3]
N0, CHUNK = 600, 128          # 5 chunks, the last one ragged


@pytest.fixture(scope="module")
def env(keys):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_04463_amd as imc

    dealer, party = keys
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=16 * len(ROT))
    dc, dm = wl.gen_codes(71, 0, N0)
    qc, qm = wl.gen_codes(71, 0, 8, query=True)
    qc[0], qm[0] = wl.plant(71, 0, dc[300], dm[300], 3, h=0.2)     # X: matches entry 300
    qc[1], qm[1] = wl.plant(71, 1, dc[599], dm[599], -2, h=0.3)    # matches the ragged last chunk
    yield dict(imc=imc, ctx=ctx, dc=dc, dm=dm, qc=qc, qm=qm, dealer=dealer, party=party)
    ctx.close()


def _db(e, capacity=N0 + 16, galois=False):
    from paper_2405_04463_amd.pipeline import SharedDB

    db = SharedDB(e["ctx"], capacity, galois=galois)
    d64 = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()  # noqa: E731
    db.enroll(d64(e["dc"]), d64(e["dm"]), 0)
    torch.cuda.synchronize()
    return db


def _req(e, i, qid):
    from paper_2405_04463_amd.serve import Request

    return Request(rid=i, qid=qid, code=e["qc"][i].copy(), mask=e["qm"][i].copy())


def _drive(srv, reqs_at_tick):
    """Submit requests at given tick numbers and tick until all are done."""
    total = len(srv.done) + sum(len(v) for v in reqs_at_tick.values())
    t = 0
    while len(srv.done) < total:
        for r in reqs_at_tick.get(t, []):
            srv.submit(r)
        if not srv.tick():
            torch.cuda.synchronize()
        t += 1
        assert t < 1000, srv.state()
    torch.cuda.synchronize()
    return {r.rid: r for r in srv.done}


@pytest.mark.parametrize("galois,gather", [(False, True), (True, True), (False, False)])
def test_same_alone_in_mix_and_plain(env, galois, gather):
    from paper_2405_04463_amd.serve import Server, plain_check

    e = env
    db = _db(e, galois=galois)
    alone = _drive(Server(e["ctx"], db, ROT, chunk=CHUNK, slots=8, append=False, keep_shares=True, gather=gather),
                   {0: [_req(e, 0, 1000)]})[0]
    db2 = _db(e, galois=galois)
    srv = Server(e["ctx"], db2, ROT, chunk=CHUNK, slots=8, append=False, keep_shares=True, gather=gather)
    mixed = _drive(srv, {0: [_req(e, i, 1000 + i) for i in (1, 2, 3)], 2: [_req(e, 0, 1000)], 3: [_req(e, 4, 1004)]})
    # every (request, rotation, entry) compared exactly once: the chunk passes
    # stop at the last whole word below the snapshot, finalisation does the rest
    assert srv.cmps == len(ROT) * sum(r.checked for r in mixed.values()) == len(ROT) * N0 * 5
    x = mixed[0]
    assert alone.dup == x.dup == 1
    assert np.array_equal(alone.dup_shares, x.dup_shares)
    for p in range(3):
        assert np.array_equal(alone.match[p], x.match[p])
    # the plain per-query path: one request, whole database, one pass
    qs, out = plain_check(e["ctx"], db2, _req(e, 0, 1000), ROT, {})
    torch.cuda.synchronize()
    assert int(out.cpu()[0]) == 1
    # every opened result against the plaintext decision on the admitted snapshot
    for rid, r in mixed.items():
        _, _, _, dup = orc.plain(e["qc"][rid:rid + 1], e["qm"][rid:rid + 1], ROT, e["dc"], e["dm"])
        assert r.dup == int(dup[0]), rid
    assert mixed[1].dup == 1


def test_admission_waits_for_free_hbm(env):
    """Admission needs free HBM above the reserve: with the whole device
    reserved nothing is admitted and the queue waits; once memory is
    available again the queued requests run and give the plaintext decisions."""
    from paper_2405_04463_amd.serve import Server

    e = env
    db = _db(e)
    srv = Server(e["ctx"], db, ROT, chunk=CHUNK, slots=8, append=False, hbm_reserve=1.0)
    for i in (0, 2):
        srv.submit(_req(e, i, 4000 + i))
    for _ in range(3):
        assert srv.tick() is False
    st = srv.state()
    assert st["queued"] == 2 and st["active"] == 0 and st["done"] == 0
    srv.hbm_reserve = 0
    t = 0
    while len(srv.done) < 2:
        if not srv.tick():
            torch.cuda.synchronize()
        t += 1
        assert t < 1000, srv.state()
    torch.cuda.synchronize()
    for r in srv.done:
        _, _, _, dup = orc.plain(e["qc"][r.rid:r.rid + 1], e["qm"][r.rid:r.rid + 1], ROT, e["dc"], e["dm"])
        assert r.dup == int(dup[0]), r.rid
    assert sorted(r.dup for r in srv.done) == [0, 1]


@pytest.mark.parametrize("galois", [False, True])
def test_unique_requests_are_appended(env, galois):
    from paper_2405_04463_amd.serve import Request, Server

    e = env
    db = _db(e, galois=galois)
    srv = Server(e["ctx"], db, ROT, chunk=CHUNK, slots=8, append=True)
    done = _drive(srv, {0: [_req(e, 5, 2005)]})
    y = done[5]
    assert y.dup == 0 and y.entry == N0 and db.n == N0 + 1
    # a later request carrying the same code and mask now matches the appended entry
    z = Request(rid=9, qid=2009, code=e["qc"][5].copy(), mask=e["qm"][5].copy())
    done = _drive(srv, {0: [z]})
    assert done[9].dup == 1 and done[9].snapshot == N0 + 1 and db.n == N0 + 1


def test_party_local_serving(env):
    """One party's share of the work (its database region only): each
    request's dot outputs over the whole database equal the oracle's party-0
    local dots, alone and in a mix; the supplied decision drives appends."""
    from paper_2405_04463_amd.pipeline import SharedDB
    from paper_2405_04463_amd.serve import Server

    e = env
    db = SharedDB(e["ctx"], N0 + 16, parties=(0,))
    d64 = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()  # noqa: E731
    db.enroll(d64(e["dc"]), d64(e["dm"]), 0)
    torch.cuda.synchronize()
    decide = lambda r: 1 if r.rid in (0, 1) else 0   # noqa: E731  (planted: 0 and 1)
    alone = _drive(Server(e["ctx"], db, ROT, chunk=CHUNK, slots=8, append=False, keep_shares=True, decide=decide),
                   {0: [_req(e, 0, 3000)]})[0]
    srv = Server(e["ctx"], db, ROT, chunk=CHUNK, slots=8, append=True, keep_shares=True, decide=decide)
    done = _drive(srv, {0: [_req(e, i, 3000 + i) for i in (1, 2)], 2: [_req(e, 0, 3000)], 3: [_req(e, 6, 3006)]})
    qsh = orc.share(e["dealer"], orc.DOM_SHARE_QUERY, e["qc"], e["qm"], 3000)
    dsh = orc.share(e["dealer"], orc.DOM_SHARE_DB, e["dc"], e["dm"], 0)
    for rid, r in done.items():
        assert r.snapshot == N0 or rid == 6
        n = r.snapshot
        want_c, want_m = orc.local_dot(0, qsh[rid:rid + 1], ROT, dsh[:n]) if n == N0 else (None, None)
        if want_c is None:
            continue
        assert np.array_equal(r.dots[0][0].cpu().numpy().view(np.uint16), want_c), rid
        assert np.array_equal(r.dots[0][1].cpu().numpy().view(np.uint16), want_m), rid
    assert np.array_equal(alone.dots[0][0].cpu().numpy(), done[0].dots[0][0].cpu().numpy())
    # uniques (by the decision) were appended to the held region only
    assert db.n == N0 + sum(1 for r in done.values() if r.dup == 0)
    assert {r.dup for r in done.values()} == {0, 1}
    assert db.regions[1] is None and db.regions[2] is None


@pytest.mark.parametrize("galois", [False, True])
def test_serial_uniqueness_of_requests_in_flight(env, galois):
    """Two requests carrying the same iris, the second admitted while the
    first is still in flight: the first is unique and appended, the second
    is a duplicate of it (serial order), and its shares equal a plain check
    against the database as it stood after the first request."""
    from paper_2405_04463_amd.pipeline import SharedQueries, alloc_check, run_check
    from paper_2405_04463_amd.serve import Request, Server

    e = env
    db = _db(e, galois=galois)
    srv = Server(e["ctx"], db, ROT, chunk=CHUNK, slots=8, append=True, keep_shares=True)
    a = _req(e, 5, 4005)
    b = Request(rid=15, qid=4015, code=e["qc"][5].copy(), mask=e["qm"][5].copy())
    c = _req(e, 6, 4006)
    done = _drive(srv, {0: [a], 1: [b], 2: [c]})
    assert done[5].dup == 0 and done[5].entry == N0 and done[5].checked == N0
    assert done[15].snapshot == N0 and done[15].checked == N0 + 1
    assert done[15].dup == 1 and done[15].entry == -1
    assert done[6].dup == 0 and done[6].checked == N0 + 1 and done[6].entry == N0 + 1
    assert db.n == N0 + 2
    assert srv.cmps == len(ROT) * sum(r.checked for r in done.values())   # no entry compared twice
    # b against the database after a's append, checked plainly
    d64 = lambda x: torch.from_numpy(np.ascontiguousarray(x).view(np.int64).reshape(1, 200)).cuda()  # noqa: E731
    qs = SharedQueries(e["ctx"], d64(e["qc"][5]), d64(e["qm"][5]), 4015, galois=galois)
    buf = alloc_check(1, len(ROT), N0 + 1)
    run_check(e["ctx"], qs, ROT, db, 0, N0 + 1, buf)
    torch.cuda.synchronize()
    nw = (N0 + 1 + 63) // 64
    for p in range(3):
        assert np.array_equal(done[15].match[p][:, :, :nw], buf.match[p].cpu().numpy()[:, :, :nw]), p
        assert int(done[15].dup_shares[p]) == int(buf.dup[p].cpu().numpy()[0, 0]), p
