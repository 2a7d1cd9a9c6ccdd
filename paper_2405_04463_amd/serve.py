"""Continuous-batching uniqueness service, three parties simulated on one GPU.

Requests (one iris code + mask, checked at R rotations) arrive over time.
The database shares stay resident in HBM, split into fixed chunks of `chunk`
entries (a multiple of 64).  A cursor walks the chunks cyclically; on each
tick every admitted request that still needs the cursor's chunk contributes
its R rows to ONE batched dot launch per party (`imc_dot_shares_gather` over
the active slots, or `imc_dot_shares_rows` over a row table), then ONE
resharing and ONE comparison call over all of those rows
(`imc_reshare_queries`, `imc_compare_threshold_queries`: a device table
gives each request's query id, its columns in this chunk and its own
full-database match buffer, where its match words land at the chunk's word
offset).  A
request admitted while others are in flight joins at the current chunk (its
work overlaps theirs on the device) and completes after one full cycle; its
OR-tree then runs once over its whole match buffer and the result is opened.
Unique requests (dup = 0) are appended to the database.

Because every random value is addressed by (query id, rotation, entry, gate)
and the OR-tree runs over the request's complete buffer, a request's shares
and result are the same alone and in any mix, whatever chunk it starts at.
Each gate's correlated randomness is used once (App. C): the chunk passes
compare whole 64-entry words below the request's snapshot only, and the
word holding the snapshot -- whose lanes past the snapshot would otherwise
run the gates first on padding and later on appended entries under the
same randomness -- is compared exactly once, when the request is finalised,
together with any entries appended since.
Serial uniqueness (Sec. 6.4: a batch is also matched against itself): a
request must also match the unique requests admitted before it that were
still in flight at its admission.  With `serial=True` (the default) a request
whose pass over its snapshot is complete is finalised only after every
earlier-admitted request has been decided and, if unique, appended; it is
then compared with the entries appended since its admission (a short tail
pass over [64-aligned snapshot, current size) into the same match buffer)
before its OR-tree runs over the whole buffer.  Its shares and result then equal a plain check against the
database as it stands after every earlier request, i.e. the serial order.
(The tail pass starts at the 64-aligned snapshot: entries below it in that
word are reshared and compared there for the first time, so no gate runs
twice.)

Admission: a request needs a free slot (slots bound the rows of a tick) and
its per-request buffers must fit in free HBM above a reserve.

Party-local serving: when the database object holds one party's region
only (the other regions None), the server does that party's share of the
work -- its dot products over every chunk, with the same continuous batching,
admission and appends -- and nothing that needs the other parties.  The
uniqueness decision then comes from a caller-supplied `decide(request)`
(a deployment receives it from the interactive part of the protocol).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import OPEN_U8_XOR, QUERY_ENTRY_WORDS, Context, compare_msg_bytes, make_ids, or_tree_ws_bytes, query_table

ROW = 102400                 # query operand bytes per query (replicated form)
RAW = 2 * 2 * 12800 * 2      # raw query share bytes per query (replicated form)
GALOIS_ROW = 51200           # the same for Galois-ring Shamir shares
GALOIS_RAW = 2 * 12800 * 2


@dataclass
class Request:
    rid: int
    qid: int
    code: np.ndarray          # packed u64 [200]
    mask: np.ndarray
    arrival: float = 0.0      # seconds from the start of the run
    # filled by the server
    slot: int = -1
    snapshot: int = 0         # database entries this request is checked against
    remaining: set = field(default_factory=set)
    admitted_at: float = -1.0
    done_at: float = -1.0
    dup: int = -1
    entry: int = -1           # database slot when appended
    dup_shares: np.ndarray | None = None   # [3] components of the result
    dots: dict | None = None  # party-local serving with keep_shares: party -> (code, mask) [R, entries]
    seq: int = -1             # admission order
    checked: int = 0          # entries the final decision covers


class Server:
    def __init__(self, ctx: Context, db, rot, chunk: int = 65536, slots: int = 64, max_entries: int | None = None,
                 hbm_reserve: float = 0.01, append: bool = True, keep_shares: bool = False, device=0,
                 gather: bool = True, decide=None, serial: bool = True, net: str = "buffers"):
        """hbm_reserve: fraction of the device's memory kept free by admission.
        gather: run each tick's dot products as one gathered uniform launch
        (`imc_dot_shares_gather`); otherwise through a row table
        (`imc_dot_shares_rows`).  decide: request -> 0/1, the uniqueness
        decision in party-local serving (required there, unused otherwise).
        serial: also match requests against earlier-admitted requests that were
        in flight at their admission (see the module notes).  net: "buffers"
        runs each comparison with the parties apart and its messages through
        a device buffer (one, sized for 16 requests' rows of a chunk; a tick
        with more requests runs its comparison in launches of 16, which reuse
        it in stream order); "registers" holds them in registers."""
        self.gather = gather
        self.parties = [p for p in range(3) if db.regions[p] is not None]
        self.local = len(self.parties) < 3
        if self.local and decide is None:
            raise ValueError("party-local serving needs a decide(request) callback")
        self.decide = decide
        self.serial = serial and not self.local
        self.pending: list = []         # pass complete, waiting for every earlier request (serial)
        self.seq = 0
        assert chunk % 64 == 0
        self.ctx, self.db, self.rot = ctx, db, list(rot)
        self.galois = bool(getattr(db, "galois", False))
        self.row_bytes = GALOIS_ROW if self.galois else ROW
        self.raw_bytes = GALOIS_RAW if self.galois else RAW
        self.R = len(self.rot)
        self.chunk, self.slots = chunk, slots
        self.append_uniques, self.keep_shares = append, keep_shares
        self.hbm_reserve = int(hbm_reserve * torch.cuda.mem_get_info(device)[1])
        self.max_entries = max_entries or db.capacity
        d = torch.device("cuda", device)
        self.dev = d
        self.nw_full = (self.max_entries + 63) // 64
        rows = slots * self.R
        self.ld = chunk
        i16 = lambda *s: torch.empty(*s, dtype=torch.int16, device=d)  # noqa: E731
        # slot-indexed query shares (operand row = slot)
        self.op = [torch.empty(slots * self.row_bytes, dtype=torch.uint8, device=d) for _ in range(3)]
        self.raw = [torch.empty(slots * self.raw_bytes // 2, dtype=torch.int16, device=d) for _ in range(3)]
        # tick buffers: dot outputs of all slots' rows for one chunk (held parties)
        self.dot_code = [i16(rows, self.ld) if p in self.parties else None for p in range(3)]
        self.dot_mask = [i16(rows, self.ld) if p in self.parties else None for p in range(3)]
        # a small ring of row tables: the host fills one while earlier copies may
        # still be reading the others; a table is reused only after its copy ended
        self.ring = 4
        self.rows_host = [torch.empty(rows, 2, dtype=torch.int32).pin_memory() for _ in range(self.ring)]
        self.rows_dev = [torch.empty(rows, 2, dtype=torch.int32, device=d) for _ in range(self.ring)]
        self.rows_ev = [None] * self.ring
        # the same ring for the tick's query tables (query id, columns, match buffers)
        self.qtab_host = [torch.empty(slots, QUERY_ENTRY_WORDS, dtype=torch.int64).pin_memory()
                          for _ in range(self.ring)]
        self.qtab_dev = [torch.empty(slots, QUERY_ENTRY_WORDS, dtype=torch.int64, device=d) for _ in range(self.ring)]
        self.qtab_ev = [None] * self.ring
        self.tick_ev = deque()          # the host runs at most two ticks ahead of the GPU
        # the interactive steps' buffers (none in party-local serving): a tick's
        # resharing of all its rows, and one request's tail pass
        tr = 0 if self.local else rows
        self.t_msg = [i16(2, tr, self.ld) for _ in range(3)]
        self.t_rep_code = [i16(2, tr, self.ld) for _ in range(3)]
        self.t_rep_mask = [i16(2, tr, self.ld) for _ in range(3)]
        tl = 0 if self.local else self.R
        self.msg = [i16(2, tl, self.ld) for _ in range(3)]
        self.rep_code = [i16(2, tl, self.ld) for _ in range(3)]
        self.rep_mask = [i16(2, tl, self.ld) for _ in range(3)]
        self.match = [None] * slots     # [3] x [2, R, nw_full] int64, allocated on admission
        self.dup = [[torch.empty(2, 1, dtype=torch.uint8, device=d) for _ in range(3)] for _ in range(slots)]
        self.ws = torch.empty(max(8, or_tree_ws_bytes(1, self.R, self.nw_full)), dtype=torch.uint8, device=d)
        assert net in ("buffers", "registers")
        self.net = None
        if net == "buffers" and not self.local:
            self.net = torch.empty(compare_msg_bytes(0, min(slots, 16) * self.R, chunk) // 8, dtype=torch.int64,
                                   device=d)
        self.open_dev = torch.empty(slots, dtype=torch.uint8, device=d)
        self.open_host = torch.empty(slots, dtype=torch.uint8).pin_memory()
        self.free = list(range(slots))[::-1]
        self.active: dict[int, Request] = {}
        self.finishing: list = []       # (request, event)
        self.queue: deque = deque()
        self.cursor = 0
        self.done: list = []
        self.t0 = time.perf_counter()
        self.ticks = 0
        self.cmps = 0

    # ---------------------------------------------------------------- helpers
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def request_bytes(self) -> int:
        return 0 if self.local else 3 * 2 * self.R * self.nw_full * 8

    def n_chunks(self) -> int:
        return (self.db.n + self.chunk - 1) // self.chunk

    def submit(self, req: Request):
        self.queue.append(req)

    def state(self) -> dict:
        free_b, total_b = self.free_hbm(), torch.cuda.mem_get_info(self.dev)[1]
        return {"queued": len(self.queue), "active": len(self.active), "finishing": len(self.finishing),
                "done": len(self.done), "free_slots": len(self.free), "cursor": self.cursor, "ticks": self.ticks,
                "db_n": self.db.n, "hbm_free": free_b, "hbm_total": total_b, "reserve": self.hbm_reserve,
                "next_arrival": self.queue[0].arrival if self.queue else None, "now": self.now()}

    # -------------------------------------------------------------- admission
    def free_hbm(self) -> int:
        """Device memory a new request can still get: what the driver has free
        plus what torch's caching allocator holds unused (buffers of finished
        requests stay there and are handed out again)."""
        free_b, _ = torch.cuda.mem_get_info(self.dev)
        return free_b + torch.cuda.memory_reserved(self.dev) - torch.cuda.memory_allocated(self.dev)

    def _admit(self):
        now = self.now()
        while self.queue and self.free and self.queue[0].arrival <= now:
            if self.free_hbm() - self.request_bytes() < self.hbm_reserve:
                break
            req = self.queue.popleft()
            slot = self.free.pop()
            req.slot = slot
            req.seq = self.seq
            self.seq += 1
            req.snapshot = self.db.n
            req.remaining = set(range((req.snapshot + self.chunk - 1) // self.chunk))
            req.admitted_at = now
            c = torch.from_numpy(np.ascontiguousarray(req.code).view(np.int64).reshape(1, 200)).to(self.dev)
            m = torch.from_numpy(np.ascontiguousarray(req.mask).view(np.int64).reshape(1, 200)).to(self.dev)
            self.ctx.share_query(c, m, 1, req.qid, [o.data_ptr() + slot * self.row_bytes for o in self.op],
                                 [r.data_ptr() + slot * self.raw_bytes for r in self.raw], galois=self.galois)
            if not self.local:
                self.match[slot] = [torch.zeros(2, self.R, self.nw_full, dtype=torch.int64, device=self.dev)
                                    for _ in range(3)]
            elif self.keep_shares:   # test aid: the request's dot outputs over the whole database
                req.dots = {p: [torch.zeros(self.R, req.snapshot, dtype=torch.int16, device=self.dev)
                                for _ in range(2)] for p in self.parties}
            self.active[slot] = req

    # ------------------------------------------------------------------ tick
    def tick(self) -> bool:
        """Admit, then process the cursor's chunk for every request needing it.
        Returns False when nothing was launched (the caller then waits for the
        device or for the next arrival; finished requests are collected by the
        next tick)."""
        self._admit()
        self._poll()
        self._finalize_ready()
        if not self.active:
            return False
        nch = self.n_chunks()
        # advance the cursor to the next chunk some active request still needs
        for _ in range(nch):
            if any(self.cursor in r.remaining for r in self.active.values()):
                break
            self.cursor = (self.cursor + 1) % nch
        j = self.cursor
        reqs = [r for r in self.active.values() if j in r.remaining]
        first = j * self.chunk
        n_max = max(min(self.chunk, r.snapshot - first) for r in reqs)
        while len(self.tick_ev) >= 2:
            self.tick_ev.popleft().synchronize()
        # one batched dot launch per party over every participating request's rows
        b = self.ticks % self.ring
        if self.rows_ev[b] is not None:
            self.rows_ev[b].synchronize()
        if self.gather:
            # the participating slots as a gather list: every request has the same
            # rotations, so this is one uniform launch (rotation-aware kernel)
            table = np.array([r.slot for r in reqs], dtype=np.int32)
            k = table.shape[0]
            self.rows_host[b].view(-1)[:k].copy_(torch.from_numpy(table))
            self.rows_dev[b].view(-1)[:k].copy_(self.rows_host[b].view(-1)[:k], non_blocking=True)
        else:
            table = np.array([(r.slot, int(sft)) for r in reqs for sft in self.rot], dtype=np.int32)
            k = table.shape[0]
            self.rows_host[b][:k].copy_(torch.from_numpy(table))
            self.rows_dev[b][:k].copy_(self.rows_host[b][:k], non_blocking=True)
        self.rows_ev[b] = torch.cuda.Event()
        self.rows_ev[b].record()
        ids_t = make_ids(0, self.rot, first)
        for p in self.parties:
            if self.gather:
                self.ctx.dot_shares_gather(p, self.op[p], self.rows_dev[b], k, ids_t, self.db.regions[p],
                                           self.db.capacity, n_max, self.dot_code[p], self.dot_mask[p], self.ld,
                                           galois=self.galois)
            else:
                self.ctx.dot_shares_rows(p, self.op[p], self.slots, self.rows_dev[b], k, self.db.regions[p],
                                         self.db.capacity, first, n_max, self.dot_code[p], self.dot_mask[p], self.ld,
                                         galois=self.galois)
        # every request's rows: reshared and compared in one call each, the
        # match words going to the request's own buffer
        finished = []
        entries = []
        for i, r in enumerate(reqs):
            n_j = min(self.chunk, r.snapshot - first)
            r.remaining.discard(j)
            if not r.remaining:
                finished.append(r)
            if self.local:          # the party's share of the work ends with its dot products
                if self.keep_shares:
                    for p in self.parties:
                        for v, src in enumerate((self.dot_code[p], self.dot_mask[p])):
                            r.dots[p][v][:, first:first + n_j].copy_(src[i * self.R:(i + 1) * self.R, :n_j])
                self.cmps += self.R * n_j
                continue
            # whole words only: the word holding the snapshot waits for finalisation
            n_w = max(0, min(self.chunk, (r.snapshot // 64) * 64 - first))
            entries.append((r.qid, n_w, [m.data_ptr() + 8 * (first // 64) for m in self.match[r.slot]],
                            self.R * self.nw_full))
            self.cmps += self.R * n_w
        n_t = max((e[1] for e in entries), default=0)
        if n_t:
            k = len(entries)
            if self.qtab_ev[b] is not None:
                self.qtab_ev[b].synchronize()
            query_table(entries, out=self.qtab_host[b])
            self.qtab_dev[b][:k].copy_(self.qtab_host[b][:k], non_blocking=True)
            self.qtab_ev[b] = torch.cuda.Event()
            self.qtab_ev[b].record()
            self.ctx.reshare_queries(self.dot_code, self.dot_mask, k, n_t, self.ld, ids_t, self.qtab_dev[b],
                                     self.t_msg, self.t_rep_code, self.t_rep_mask)
            self.ctx.compare_threshold_queries(self.t_rep_code, self.t_rep_mask, k, n_t, self.ld, ids_t,
                                               self.qtab_dev[b], self.nw_full, msg_ws=self.net)
        # in stream order after every request of the tick has consumed its rows
        # of the shared dot buffers (a tail pass reuses them)
        for r in finished:
            self._finish(r)
        self.cursor = (j + 1) % max(1, self.n_chunks())
        self.ticks += 1
        ev = torch.cuda.Event()
        ev.record()
        self.tick_ev.append(ev)
        return True

    def _finish(self, r: Request):
        s = r.slot
        if self.local:
            ev = torch.cuda.Event()
            ev.record()
            del self.active[s]
            self.finishing.append((r, ev))
            return
        if self.serial:
            del self.active[s]
            self.pending.append(r)
            self._finalize_ready()
            return
        if r.snapshot % 64:
            self._tail_pass(r, r.snapshot)      # the word holding the snapshot, once
        self._finalize(r, r.snapshot)

    def _finalize_ready(self):
        """Finalise pending requests in admission order once every earlier
        request has been decided (and appended if unique)."""
        while self.pending:
            r = min(self.pending, key=lambda x: x.seq)
            if any(a.seq < r.seq for a in self.active.values()):
                return
            if self.finishing:
                # earlier requests' results are on their way: wait for them now
                # rather than a tick later, so a burst of finishing requests is
                # decided in one go
                for _, ev in self.finishing:
                    ev.synchronize()
                self._poll()
                continue
            self.pending.remove(r)
            n_now = self.db.n
            if n_now > (r.snapshot // 64) * 64:
                self._tail_pass(r, n_now)
            self._finalize(r, n_now)

    def _tail_pass(self, r: Request, n_now: int):
        """Compare r with entries [64-aligned snapshot, n_now) into its match
        buffer: the word holding the snapshot (not compared by the chunk
        passes) and the entries appended since admission, each gate once."""
        first = (r.snapshot // 64) * 64
        s = r.slot
        b = self.ticks % self.ring
        if self.rows_ev[b] is not None:
            self.rows_ev[b].synchronize()
        self.rows_host[b].view(-1)[:1].fill_(s)
        self.rows_dev[b].view(-1)[:1].copy_(self.rows_host[b].view(-1)[:1], non_blocking=True)
        self.rows_ev[b] = torch.cuda.Event()
        self.rows_ev[b].record()
        self.ticks += 1
        for f in range(first, n_now, self.chunk):
            n_j = min(self.chunk, n_now - f)
            ids = make_ids(r.qid, self.rot, f)
            for p in range(3):
                self.ctx.dot_shares_gather(p, self.op[p], self.rows_dev[b], 1, make_ids(0, self.rot, f),
                                           self.db.regions[p], self.db.capacity, n_j, self.dot_code[p],
                                           self.dot_mask[p], self.ld, galois=self.galois)
            self.ctx.reshare(self.dot_code, self.dot_mask, self.R, n_j, self.ld, ids, self.msg, self.rep_code,
                             self.rep_mask)
            mw = [m.data_ptr() + 8 * (f // 64) for m in self.match[s]]
            self.ctx.compare_threshold(self.rep_code, self.rep_mask, self.R, n_j, self.ld, ids, mw,
                                       self.nw_full, msg_ws=self.net)
            self.cmps += self.R * n_j

    def _finalize(self, r: Request, n_checked: int):
        s = r.slot
        r.checked = n_checked
        ids = make_ids(r.qid, self.rot, 0)
        nw = (n_checked + 63) // 64
        self.ctx.or_tree(self.match[s], 1, nw, self.nw_full, ids, self.ws, self.ws.numel(), self.dup[s])
        self.ctx.open(OPEN_U8_XOR, self.dup[s], 1, self.open_dev.data_ptr() + s, 0)
        self.open_host[s:s + 1].copy_(self.open_dev[s:s + 1], non_blocking=True)
        if self.keep_shares:
            r.dup_shares = torch.stack([d[0, 0] for d in self.dup[s]])
        ev = torch.cuda.Event()
        ev.record()
        self.active.pop(s, None)
        self.finishing.append((r, ev))

    def _poll(self):
        keep = []
        for r, ev in self.finishing:
            if not ev.query():
                keep.append((r, ev))
                continue
            r.dup = int(self.decide(r)) if self.local else int(self.open_host[r.slot].item())
            r.done_at = self.now()
            if self.keep_shares and not self.local:
                r.dup_shares = r.dup_shares.cpu().numpy()
                r.match = [m.cpu().numpy() for m in self.match[r.slot]]
            if r.dup == 0 and self.append_uniques and self.db.n < self.max_entries:
                raw = [x.data_ptr() + r.slot * self.raw_bytes for x in self.raw]
                r.entry = self.db.n
                self.ctx.append_db(raw, 0, self.db.regions, self.db.capacity, r.entry, galois=self.galois)
                self.db.n += 1
            self.match[r.slot] = None
            self.free.append(r.slot)
            self.done.append(r)
        self.finishing = keep

    # ------------------------------------------------------------------- run
    def run(self, requests, until_idle: bool = True, timeout: float = 600.0):
        """Feed requests (sorted by arrival) and tick until all are done."""
        for r in sorted(requests, key=lambda x: x.arrival):
            self.submit(r)
        self.t0 = time.perf_counter()
        total = len(self.queue)
        while len(self.done) < total:
            if self.now() > timeout:
                raise TimeoutError("serving run exceeded its time limit")
            busy = self.tick()
            if not busy:
                if self.finishing or self.pending:
                    torch.cuda.synchronize()
                elif self.queue:
                    wait = self.queue[0].arrival - self.now()
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
        torch.cuda.synchronize()
        return self.done


def plain_check(ctx: Context, db, req: Request, rot, buf_cache: dict):
    """The per-query path: one request checked alone against the whole
    database in one pass (its own dot launches, no batching)."""
    from .pipeline import SharedQueries, alloc_check, open_dup, run_check

    n = db.n
    key = (len(rot), n)
    if key not in buf_cache:
        buf_cache.clear()
        buf_cache[key] = alloc_check(1, len(rot), n)
    buf = buf_cache[key]
    c = torch.from_numpy(np.ascontiguousarray(req.code).view(np.int64).reshape(1, 200)).cuda()
    m = torch.from_numpy(np.ascontiguousarray(req.mask).view(np.int64).reshape(1, 200)).cuda()
    qs = SharedQueries(ctx, c, m, req.qid, galois=bool(getattr(db, "galois", False)))
    run_check(ctx, qs, rot, db, 0, n, buf)
    out, _ = open_dup(ctx, buf, 1, check=0)
    return qs, out
