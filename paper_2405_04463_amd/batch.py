"""Batching of uneven query batches (buffers and call sequence only).

A *batch* is q queries checked at one rotation list (R = len(rot)) with
consecutive query ids.  A step over many batches computes every party's dot
products for all their rows with one launch per database chunk per rotation
list ("grouped": the batches of one list are contiguous, so the launch is a
uniform `imc_dot_shares` and lists of 13 or more rotations get the
rotation-aware kernel), with ONE rotation-aware launch per chunk over every
list of 13 or more rotations ("fused": `imc_dot_shares_groups`, optionally
a persistent grid, plus one launch per shorter list), or with ONE launch per
chunk over a row table of all rows ("rows": `imc_dot_shares_rows`).  Either
way the database streams from HBM once per chunk (per launch) for all
batches instead of once per batch.
Resharing and comparison are elementwise per comparison: the batched form
runs them once per rotation list over the rows of all its batches
(`imc_reshare_queries`, `imc_compare_threshold_queries`, with a device table
giving every query its id and its place in its batch's match buffer); the
OR-tree runs per batch.  The comparisons pass their messages through one
shared device buffer, as the single check does.  The plain form reshares and
compares batch by batch.

`BatchedStep.capture()` records a whole step in a HIP graph (through torch's
graph API); `replay()` re-runs it.  Per-batch plain launches (`run_plain`) are
the comparison point.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import (MAX_DOT_GROUPS, Context, compare_msg_bytes, galois_query_op_bytes, make_ids, or_tree_ws_bytes,
               query_op_bytes, query_table)


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
    """Shared queries of several batches and their row table.

    The operand (and the row ranges of the outputs) is laid out grouped by
    rotation list, batch order kept within a group, so the batches of one
    rotation list are contiguous: a group can then run as one uniform
    `imc_dot_shares` call.  qbase[b] / rbase[b] are batch b's first operand row
    and output row; groups[i] = (rotation list, first batch slot, queries,
    first output row)."""

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
        src = np.cumsum([0] + [b.q for b in batches])[:-1]          # batch b's first row of codes
        order = sorted(range(len(batches)), key=lambda b: (-len(batches[b].rot), tuple(batches[b].rot), b))
        self.qbase, self.rbase = [0] * len(batches), [0] * len(batches)
        self.groups = []
        qi = ri = 0
        table = []
        for b in order:
            bt = batches[b]
            key = tuple(int(v) for v in bt.rot)
            if not self.groups or self.groups[-1][0] != key:
                self.groups.append([key, qi, 0, ri])
            self.groups[-1][2] += bt.q
            self.qbase[b], self.rbase[b] = qi, ri
            off = qi * self.row_bytes
            # each batch has its own id range: share it into its slice of the operand
            ctx.share_query(codes[src[b]:src[b] + bt.q], masks[src[b]:src[b] + bt.q], bt.q, bt.qid_base,
                            [o.data_ptr() + off for o in self.op], None, stream, galois=galois)
            for j in range(bt.q):
                for sft in bt.rot:
                    table.append((qi + j, int(sft)))
            qi += bt.q
            ri += bt.rows
        self.nrows = ri
        self.rows = torch.tensor(np.array(table, dtype=np.int32).reshape(-1, 2), device=d)


class BatchedStep:
    """Dot products of all batches against one database range, one launch per
    party per chunk of `chunk` entries, plus optionally the 3-party
    comparison per batch."""

    def __init__(self, ctx: Context, bs: BatchSet, db, first_entry: int, n: int, chunk: int | None = None,
                 parties=(0,), compare: bool = False, device=0, mode: str = "grouped"):
        assert first_entry % 64 == 0
        assert bs.galois == bool(getattr(db, "galois", False)), "query and database sharing differ"
        self.ctx, self.bs, self.db = ctx, bs, db
        self.first, self.n = first_entry, n
        self.chunk = min(n, chunk or n)
        self.chunk = ((self.chunk + 63) // 64) * 64 if self.chunk < n else self.chunk
        self.parties = tuple(parties)
        self.compare = compare
        self.mode = mode
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
                    match=[torch.empty(2, rb, nw, dtype=torch.int64, device=d) for _ in range(3)],
                    dup=[torch.empty(2, b.q, dtype=torch.uint8, device=d) for _ in range(3)],
                    ws=torch.empty(max(8, or_tree_ws_bytes(b.q, len(b.rot), nw)), dtype=torch.uint8, device=d),
                ))
            # resharing outputs of one rotation list's rows (the largest list);
            # every list, and every batch of the plain form, reuses them in
            # stream order
            gmax = max(qn * len(rot) for rot, _, qn, _ in bs.groups)
            self.msg = [i16(2, gmax, self.ld) for _ in range(3)]
            self.rep_code = [i16(2, gmax, self.ld) for _ in range(3)]
            self.rep_mask = [i16(2, gmax, self.ld) for _ in range(3)]
            # per rotation list, its queries in layout order: id, columns and
            # rows of its batch's match buffer (the table never changes, so a
            # captured step reads it as it is)
            self.tables = []
            order = sorted(range(len(bs.batches)), key=lambda i: bs.rbase[i])
            for rot, _, qn, r0 in bs.groups:
                entries = []
                for bi in order:
                    b = bs.batches[bi]
                    if not (r0 <= bs.rbase[bi] < r0 + qn * len(rot)):
                        continue
                    m = self.per_batch[bi]["match"]
                    for i in range(b.q):
                        entries.append((b.qid_base + i, n, [t.data_ptr() + 8 * i * len(rot) * nw for t in m],
                                        b.rows * nw))
                assert len(entries) == qn
                self.tables.append(query_table(entries).to(d))
            # the comparisons' network: one message buffer for the largest batch,
            # shared by the comparisons (they run in stream order; a rotation
            # list's call runs in launches of as many queries as it holds)
            rmax = max(b.rows for b in bs.batches)
            self.net = torch.empty(compare_msg_bytes(0, rmax, n) // 8, dtype=torch.int64, device=d)
        self.graph = None

    def _chunks(self):
        c0 = 0
        while c0 < self.n:
            yield c0, min(self.chunk, self.n - c0)
            c0 += self.chunk

    def run(self, stream=None):
        """Batched form.  mode "rows": one dot launch per party per chunk over
        the row table of all batches; mode "grouped": one launch per rotation
        list per party per chunk (uniform rotations, so the rotation-aware
        kernel serves every list of 13 or more rotations); mode "fused": the
        lists of 13 or more rotations in one rotation-aware launch per party
        per chunk (a persistent grid when the context's tiles carry
        DOT_PERSISTENT), each shorter list as in "grouped"."""
        ctx, bs, db = self.ctx, self.bs, self.db
        for c0, m in self._chunks():
            for p in self.parties:
                if self.mode == "rows":
                    ctx.dot_shares_rows(p, bs.op[p], bs.q, bs.rows, bs.nrows, db.regions[p], db.capacity,
                                        self.first + c0, m, self.dot_code[p], self.dot_mask[p], self.ld, stream,
                                        galois=bs.galois)
                    continue
                rest = bs.groups
                if self.mode == "fused":
                    rest = [g for g in bs.groups if len(g[0]) < 13]
                    big = [g for g in bs.groups if len(g[0]) >= 13]
                    for i in range(0, len(big), MAX_DOT_GROUPS):
                        desc = [(bs.op[p].data_ptr() + q0 * bs.row_bytes, qn, rot,
                                 self.dot_code[p].data_ptr() + 2 * r0 * self.ld,
                                 self.dot_mask[p].data_ptr() + 2 * r0 * self.ld)
                                for rot, q0, qn, r0 in big[i:i + MAX_DOT_GROUPS]]
                        ctx.dot_shares_groups(p, desc, db.regions[p], db.capacity, self.first + c0, m, self.ld,
                                              stream, galois=bs.galois)
                for rot, q0, qn, r0 in rest:
                    ids = make_ids(0, rot, self.first + c0)
                    ctx.dot_shares(p, bs.op[p].data_ptr() + q0 * bs.row_bytes, qn, ids, db.regions[p], db.capacity,
                                   m, self.dot_code[p].data_ptr() + 2 * r0 * self.ld,
                                   self.dot_mask[p].data_ptr() + 2 * r0 * self.ld, self.ld, stream, galois=bs.galois)
        if self.compare:
            self._compare_grouped(stream)

    def autotune(self, probe_n: int = 16384, reps: int = 2):
        """Time every (mode, tile configuration) on a probe slice of the
        database and keep the fastest; returns (mode, flags, {(mode, flags): ms})."""
        from .tune import CANDIDATES_FUSED, CANDIDATES_ROWS, CANDIDATES_UNIFORM

        probe = BatchedStep(self.ctx, self.bs, self.db, self.first, min(self.n, probe_n), parties=self.parties[:1])
        times = {}
        modes = [("rows", CANDIDATES_ROWS), ("grouped", CANDIDATES_UNIFORM)]
        if any(len(g[0]) >= 13 for g in self.bs.groups):
            modes.append(("fused", CANDIDATES_FUSED))
        for mode, cands in modes:
            probe.mode = mode
            for c in cands:
                self.ctx.set_dot_tiles(c)
                probe.run()
                torch.cuda.synchronize()
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
                for a, b in ev:
                    a.record()
                    probe.run()
                    b.record()
                torch.cuda.synchronize()
                times[(mode, c)] = min(a.elapsed_time(b) for a, b in ev)
        mode, flags = min(times, key=times.get)
        self.mode = mode
        self.ctx.set_dot_tiles(flags)
        del probe
        return mode, flags, times

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

    def _or_trees(self, stream=None):
        ctx, bs = self.ctx, self.bs
        for bi, b in enumerate(bs.batches):
            pb = self.per_batch[bi]
            ids = make_ids(b.qid_base, b.rot, self.first)
            ctx.or_tree(pb["match"], b.q, (self.n + 63) // 64, self.nw, ids, pb["ws"], pb["ws"].numel(), pb["dup"],
                        stream)

    def _compare_grouped(self, stream=None):
        """One resharing and one comparison call per rotation list."""
        ctx, bs = self.ctx, self.bs
        for (rot, _, qn, r0), table in zip(bs.groups, self.tables):
            ids = make_ids(0, rot, self.first)
            add_c = [self.dot_code[p].data_ptr() + 2 * r0 * self.ld for p in range(3)]
            add_m = [self.dot_mask[p].data_ptr() + 2 * r0 * self.ld for p in range(3)]
            ctx.reshare_queries(add_c, add_m, qn, self.n, self.ld, ids, table, self.msg, self.rep_code,
                                self.rep_mask, stream)
            ctx.compare_threshold_queries(self.rep_code, self.rep_mask, qn, self.n, self.ld, ids, table, self.nw,
                                          stream, msg_ws=self.net)
        self._or_trees(stream)

    def _compare_all(self, stream=None):
        """Batch by batch (the plain form)."""
        ctx, bs = self.ctx, self.bs
        for bi, b in enumerate(bs.batches):
            ids = make_ids(b.qid_base, b.rot, self.first)
            r0 = bs.rbase[bi]
            pb = self.per_batch[bi]
            add_c = [self.dot_code[p].data_ptr() + 2 * r0 * self.ld for p in range(3)]
            add_m = [self.dot_mask[p].data_ptr() + 2 * r0 * self.ld for p in range(3)]
            ctx.reshare(add_c, add_m, b.rows, self.n, self.ld, ids, self.msg, self.rep_code, self.rep_mask, stream)
            ctx.compare_threshold(self.rep_code, self.rep_mask, b.rows, self.n, self.ld, ids, pb["match"], self.nw,
                                  stream, msg_ws=self.net)
        self._or_trees(stream)

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


def centred_rotations(r: int) -> list[int]:
    """The r rotation offsets of a query (Sec. 3: small circular shifts of the
    angular axis), centred on 0: 1 -> [0], 15 -> [-7..7], 31 -> [-15..15]."""
    if r < 1 or r > 31 or r % 2 == 0:
        raise ValueError(f"rotation count {r}: an odd number in 1..31 is centred")
    h = (r - 1) // 2
    return list(range(-h, h + 1))


def uneven_batches(n_batches: int, seed: int, qmax: int = 64, rot_counts=(1, 15, 31), qid0: int = 0):
    """Batch sizes uniform in 1..qmax, rotation counts drawn from rot_counts
    (centred offsets), consecutive query ids."""
    rng = np.random.default_rng(seed)
    out, qid = [], qid0
    for _ in range(n_batches):
        q = int(rng.integers(1, qmax + 1))
        r = int(rng.choice(rot_counts))
        out.append(Batch(q, centred_rotations(r), qid))
        qid += q
    return out
