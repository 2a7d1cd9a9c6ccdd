"""imc_dot_shares_rows_noalloc (expanded rows in the library's static device
array) against imc_dot_shares_rows (context scratch) and the oracle: two calls
in a row, the second smaller, bit for bit."""
import numpy as np
import pytest

import oracle as orc
import workload as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _u16(t):
    return t.cpu().numpy().view(np.uint16)


def _rows_table(spec):
    """spec: list of (query_index, rotation) -> device int32 [nrows, 2]."""
    return torch.tensor(np.array(spec, dtype=np.int32).reshape(-1, 2)).cuda()


def test_noalloc_rows_equal_context_scratch_rows(keys):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_04463_amd as imc
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries

    dealer, party = keys
    rng = np.random.default_rng(7)
    first, n = 64, 300                      # three 128-column tiles, the last ragged
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=imc.NOALLOC_MAX_ROWS)
    dc, dm = wl.gen_codes(71, first, n)
    db = SharedDB(ctx, first + n)
    d64 = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()  # noqa: E731
    db.enroll(d64(dc), d64(dm), first)
    nq = 12
    qc, qm = wl.gen_codes(71, 0, nq, query=True)
    qc[2], qm[2] = wl.plant(71, 2, dc[40], dm[40], -6, h=0.2)
    qs = SharedQueries(ctx, d64(qc), d64(qm), 900)
    qsh = orc.share(dealer, orc.DOM_SHARE_QUERY, qc, qm, 900)
    dsh = orc.share(dealer, orc.DOM_SHARE_DB, dc, dm, first)

    # first call: every row the static array holds, uneven (query, rotation) pairs,
    # query index nq (out of range) gives zero rows
    big = [(int(rng.integers(0, nq + 1)), int(rng.integers(-15, 16))) for _ in range(imc.NOALLOC_MAX_ROWS)]
    # second call: fewer rows (a ragged 32-row block) over fewer entries
    small = [(int(rng.integers(0, nq)), int(rng.integers(-15, 16))) for _ in range(45)]
    for call, (spec, m, party_) in enumerate([(big, n, 0), (small, 130, 2)]):
        rows = _rows_table(spec)
        nrows, ld = len(spec), 320
        outs = []
        for fn in (ctx.dot_shares_rows, ctx.dot_shares_rows_noalloc):
            code = torch.full((nrows, ld), 0x5A5A, dtype=torch.int16, device="cuda")
            mask = torch.full((nrows, ld), 0x5A5A, dtype=torch.int16, device="cuda")
            fn(party_, qs.op[party_], nq, rows, nrows, db.regions[party_], db.capacity, first, m, code, mask, ld)
            torch.cuda.synchronize()
            outs.append((_u16(code).copy(), _u16(mask).copy()))
        (c_ref, m_ref), (c_got, m_got) = outs
        assert np.array_equal(c_got, c_ref), call
        assert np.array_equal(m_got, m_ref), call
        assert np.all(c_got[:, m:] == 0x5A5A) and np.all(m_got[:, m:] == 0x5A5A), call   # columns >= n untouched
        # oracle: party's additive shares of every valid row, by (query, rotation)
        for qi in sorted({qi for qi, _ in spec if qi < nq})[:4]:
            rots = sorted({s for q_, s in spec if q_ == qi})
            rc, rm = orc.local_dot(party_, qsh[qi:qi + 1], rots, dsh[:m])
            for i, (q_, s) in enumerate(spec):
                if q_ != qi:
                    continue
                j = rots.index(s)
                assert np.array_equal(c_got[i, :m], rc[j]) and np.array_equal(m_got[i, :m], rm[j]), (call, i)
        zero = [i for i, (q_, _) in enumerate(spec) if q_ >= nq]
        if zero:
            assert not c_got[zero, :m].any() and not m_got[zero, :m].any()

    # more rows than the static array holds is an argument error, nothing enqueued
    too_many = _rows_table([(0, 0)] * (imc.NOALLOC_MAX_ROWS + 1))
    code = torch.zeros((imc.NOALLOC_MAX_ROWS + 1, 128), dtype=torch.int16, device="cuda")
    with pytest.raises(imc.IMCError) as ei:
        ctx.dot_shares_rows_noalloc(0, qs.op[0], nq, too_many, imc.NOALLOC_MAX_ROWS + 1, db.regions[0], db.capacity,
                                    first, 128, code, code, 128)
    assert ei.value.status == imc.IMC_ESHAPE
    ctx.close()
