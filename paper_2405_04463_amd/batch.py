"""Batching of uneven query batches (buffers and call sequence only).

A *batch* is q queries checked at one rotation list (R = len(rot)) with
consecutive query ids.  A step over many batches puts all their rows, batch
after batch, into one row table (query operand index, rotation) and computes
every party's dot products for all rows with ONE launch per database chunk
(`imc_dot_shares_rows`), so the database streams from HBM once per chunk for
all batches instead of once per batch.  Resharing, comparison and the OR-tree
are elementwise per comparison and run per batch on the batch's row range.

`BatchedStep.capture()` records a whole step in a HIP graph (through torch's
graph API); `replay()` re-runs it.  Per-batch plain launches (`run_plain`) are
the comparison point.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import Context, galois_query_op_bytes, make_ids, or_tree_ws_bytes, query_op_bytes


@dataclass
class Batch:
    q: int
    rot: list
    qid_base: int

    @property
    def rows(self) -> int:
        return self.q * len(self.rot)


def _dev(device):
    return torch.device("cuda", device) if isinstance(device, int) else torch.device(device)


class BatchSet:
    """Shared queries of several batches and their row table."""

    def __init__(self, ctx: Context, batches: list, codes, masks, device=0, stream=None, galois: bool = False):
        """codes/masks: device int64 [sum q_b, 200], batch after batch.
        galois: share the queries as Galois-ring Shamir operands."""
        self.batches = batches
        self.galois = galois
        self.q = sum(b.q for b in batches)
        assert codes.shape[0] == self.q
        d = _dev(device)
        self.row_bytes = galois_query_op_bytes(1) if galois else query_op_bytes(1)
        self.op = [torch.empty(max(1, self.q * self.row_bytes), dtype=torch.uint8, device=d) for _ in range(3)]
        self.qbase, self.rbase = [], []
        qi = ri = 0
        table = []
        for b in batches:
            self.qbase.append(qi)
            self.rbase.append(ri)
            off = qi * self.row_bytes
            # each batch has its own id range: share it into its slice of the operand
            ctx.share_query(codes[qi:qi + b.q], masks[qi:qi + b.q], b.q, b.qid_base,
                            [o.data_ptr() + off for o in self.op], None, stream, galois=galois)
            for j in range(b.q):
                for s in b.rot:
                    table.append((qi + j, int(s)))
            qi += b.q
            ri += b.rows
        self.nrows = ri
        self.rows = torch.tensor(np.array(table, dtype=np.int32).reshape(-1, 2), device=d)


class BatchedStep:
    """Dot products of all batches against one database range, one launch per
    party per chunk of `chunk` entries, plus optionally the 3-party
    comparison per batch."""

    def __init__(self, ctx: Context, bs: BatchSet, db, first_entry: int, n: int, chunk: int | None = None,
                 parties=(0,), compare: bool = False, device=0):
        assert first_entry % 64 == 0
        assert bs.galois == bool(getattr(db, "galois", False)), "query and database sharing differ"
        self.ctx, self.bs, self.db = ctx, bs, db
        self.first, self.n = first_entry, n
        self.chunk = min(n, chunk or n)
        self.chunk = ((self.chunk + 63) // 64) * 64 if self.chunk < n else self.chunk
        self.parties = tuple(parties)
        self.compare = compare
        d = _dev(device)
        self.ld = ((self.chunk + 63) // 64) * 64
        self.nw = self.ld // 64
        R = bs.nrows
        i16 = lambda *s: torch.empty(*s, dtype=torch.int16, device=d)  # noqa: E731
        self.dot_code = {p: i16(R, self.ld) for p in self.parties}
        self.dot_mask = {p: i16(R, self.ld) for p in self.parties}
        if compare:
            assert self.parties == (0, 1, 2) and self.chunk == n, "the comparison needs all parties, one chunk"
            self.per_batch = []
            for b in bs.batches:
                rb, nw = b.rows, self.nw
                self.per_batch.append(dict(
                    msg=[i16(2, rb, self.ld) for _ in range(3)],
                    rep_code=[i16(2, rb, self.ld) for _ in range(3)],
                    rep_mask=[i16(2, rb, self.ld) for _ in range(3)],
                    match=[torch.empty(2, rb, nw, dtype=torch.int64, device=d) for _ in range(3)],
                    dup=[torch.empty(2, b.q, dtype=torch.uint8, device=d) for _ in range(3)],
                    ws=torch.empty(max(8, or_tree_ws_bytes(b.q, len(b.rot), nw)), dtype=torch.uint8, device=d),
                ))
        self.graph = None

    def _chunks(self):
        c0 = 0
        while c0 < self.n:
            yield c0, min(self.chunk, self.n - c0)
            c0 += self.chunk

    def run(self, stream=None):
        """Batched form: one dot launch per party per chunk over all rows."""
        ctx, bs, db = self.ctx, self.bs, self.db
        for c0, m in self._chunks():
            for p in self.parties:
                ctx.dot_shares_rows(p, bs.op[p], bs.q, bs.rows, bs.nrows, db.regions[p], db.capacity,
                                    self.first + c0, m, self.dot_code[p], self.dot_mask[p], self.ld, stream,
                                    galois=bs.galois)
        if self.compare:
            self._compare_all(stream)

    def run_plain(self, stream=None):
        """Plain form: one dot launch per batch per party per chunk."""
        ctx, bs, db = self.ctx, self.bs, self.db
        for c0, m in self._chunks():
            for bi, b in enumerate(bs.batches):
                ids = make_ids(b.qid_base, b.rot, self.first + c0)
                off = bs.qbase[bi] * bs.row_bytes
                r0 = bs.rbase[bi]
                for p in self.parties:
                    ctx.dot_shares(p, bs.op[p].data_ptr() + off, b.q, ids, db.regions[p], db.capacity, m,
                                   self.dot_code[p].data_ptr() + 2 * r0 * self.ld,
                                   self.dot_mask[p].data_ptr() + 2 * r0 * self.ld, self.ld, stream,
                                   galois=bs.galois)
        if self.compare:
            self._compare_all(stream)

    def _compare_all(self, stream=None):
        ctx, bs = self.ctx, self.bs
        for bi, b in enumerate(bs.batches):
            ids = make_ids(b.qid_base, b.rot, self.first)
            r0 = bs.rbase[bi]
            pb = self.per_batch[bi]
            add_c = [self.dot_code[p].data_ptr() + 2 * r0 * self.ld for p in range(3)]
            add_m = [self.dot_mask[p].data_ptr() + 2 * r0 * self.ld for p in range(3)]
            ctx.reshare(add_c, add_m, b.rows, self.n, self.ld, ids, pb["msg"], pb["rep_code"], pb["rep_mask"], stream)
            ctx.compare_threshold(pb["rep_code"], pb["rep_mask"], b.rows, self.n, self.ld, ids, pb["match"], self.nw,
                                  stream)
            ctx.or_tree(pb["match"], b.q, (self.n + 63) // 64, self.nw, ids, pb["ws"], pb["ws"].numel(), pb["dup"],
                        stream)

    def capture(self, plain: bool = False):
        """Record one step (batched or plain) in a HIP graph."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            (self.run_plain if plain else self.run)(torch.cuda.current_stream())
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()


def uneven_batches(n_batches: int, seed: int, qmax: int = 64, rot_counts=(1, 15, 31), qid0: int = 0):
    """Batch sizes uniform in 1..qmax, rotation counts drawn from rot_counts
    (centred offsets), consecutive query ids."""
    from workload import rotations

    rng = np.random.default_rng(seed)
    out, qid = [], qid0
    for _ in range(n_batches):
        q = int(rng.integers(1, qmax + 1))
        r = int(rng.choice(rot_counts))
        out.append(Batch(q, rotations(r), qid))
        qid += q
    return out
