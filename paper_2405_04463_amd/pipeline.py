"""Buffers and the call sequence of one uniqueness check (Alg. 3) on one GPU.

Allocation and sequencing only; all arithmetic is in the library's kernels:
  share_db / share_query -> dot_shares (each party) -> reshare ->
  compare_threshold (messages through a device buffer) -> or_tree -> open

Comparison settings (Sec. 6.2): "mpclift" (default, Alg. 3 with ml lifted to
Z_2^32), "lift18" (ml lifted to Z_2^18 only), "plain" (Alg. 2: masks public,
ml computed in plain by every party, only the code dot is shared),
"constlift" (ml by a dot product over Z_2^32, no Lift) and "nolift" (both dot
products over Z_2^32).
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import (CMP_CONST32, CMP_LIFT18, CMP_PLAIN_MASK, OPEN_U8_XOR, OPEN_U16_ADD, OPEN_U64_XOR, Context,
               compare_msg_bytes, db32_bytes, db_bytes, galois_db_bytes, galois_query_op_bytes, galois_query_raw_bytes,
               make_ids, or_tree_ws_bytes, query32_op_bytes, query_op_bytes, query_raw_bytes)

COMPARE_SETTINGS = ("mpclift", "lift18", "plain", "constlift", "nolift")
VECS32 = {"constlift": (1,), "nolift": (0, 1)}   # vectors whose dot products run over Z_2^32


def _dev(device):
    if isinstance(device, torch.device):
        return device
    return torch.device("cuda", device) if isinstance(device, int) else torch.device(device)


class SharedDB:
    """The three parties' database regions (one device buffer each).
    galois=True holds Shamir shares over the Galois ring (half the bytes)."""

    def __init__(self, ctx: Context, capacity: int, device=0, parties=(0, 1, 2), galois: bool = False):
        self.ctx = ctx
        self.capacity = capacity
        self.galois = galois
        self.n = 0
        nb = galois_db_bytes(capacity) if galois else db_bytes(capacity)
        self.regions = [torch.empty(nb, dtype=torch.uint8, device=_dev(device)) if p in parties else None
                        for p in range(3)]

    def enroll(self, codes, masks, first: int | None = None, stream=None):
        """Share packed device codes/masks [n, 200] (uint64 as int64) into slots first.."""
        n = codes.shape[0]
        first = self.n if first is None else first
        self.ctx.share_db(codes, masks, n, first, self.regions, self.capacity, stream, galois=self.galois)
        self.n = max(self.n, first + n)
        return first

    def append(self, qs: "SharedQueries", qi: int, stream=None) -> int:
        assert qs.galois == self.galois
        e = self.n
        self.ctx.append_db(qs.raw, qi, self.regions, self.capacity, e, stream, galois=self.galois)
        self.n += 1
        return e


class SharedQueries:
    """Shares of q queries: each party's dot operand and raw shares."""

    def __init__(self, ctx: Context, codes, masks, query_id_base: int, device=0, keep_raw: bool = True, stream=None,
                 galois: bool = False):
        self.q = codes.shape[0]
        self.qid_base = query_id_base
        self.galois = galois
        d = _dev(device)
        ob = galois_query_op_bytes(self.q) if galois else query_op_bytes(self.q)
        rb = galois_query_raw_bytes(self.q) if galois else query_raw_bytes(self.q)
        self.op = [torch.empty(max(1, ob), dtype=torch.uint8, device=d) for _ in range(3)]
        self.raw = ([torch.empty(max(2, rb) // 2, dtype=torch.int16, device=d) for _ in range(3)]
                    if keep_raw else None)
        ctx.share_query(codes, masks, self.q, query_id_base, self.op, self.raw, stream, galois=galois)


class SharedDB32:
    """Z_2^32 regions of the given vectors (0 code, 1 mask) for the three
    parties: regions[vec][p]."""

    def __init__(self, ctx: Context, capacity: int, vecs=(1,), device=0):
        self.ctx = ctx
        self.capacity = capacity
        self.vecs = tuple(vecs)
        self.regions = {v: [torch.empty(db32_bytes(capacity), dtype=torch.uint8, device=_dev(device))
                            for _ in range(3)] for v in self.vecs}

    def enroll(self, codes, masks, first: int, stream=None):
        for v in self.vecs:
            self.ctx.share32_db(v, codes, masks, codes.shape[0], first, self.regions[v], self.capacity, stream)


class SharedQueries32:
    """Z_2^32 query operands of the given vectors: op[vec][p]."""

    def __init__(self, ctx: Context, codes, masks, query_id_base: int, vecs=(1,), device=0, stream=None):
        self.q = codes.shape[0]
        self.qid_base = query_id_base
        self.vecs = tuple(vecs)
        self.op = {v: [torch.empty(max(16, query32_op_bytes(self.q)), dtype=torch.uint8, device=_dev(device))
                       for _ in range(3)] for v in self.vecs}
        for v in self.vecs:
            ctx.share32_query(v, codes, masks, self.q, query_id_base, self.op[v], stream)


@dataclass
class CheckBuffers:
    rows: int
    n: int
    ld: int
    nw: int
    dot_code: list
    dot_mask: list
    msg: list
    rep_code: list
    rep_mask: list
    match: list
    dup: list
    ws: torch.Tensor
    compare: str = "mpclift"
    ml_pub: torch.Tensor | None = None       # "plain": public ml [rows, ld]
    row_masks: torch.Tensor | None = None    # "plain": rotated query masks [rows, 200]
    dot32: dict | None = None                # Z_2^32 settings: vec -> 3 x u32 [rows, ld]
    msg32: dict | None = None                # vec -> 3 x u32 [rows, ld]
    rep32: dict | None = None                # vec -> 3 x u32 [2, rows, ld]
    net: torch.Tensor | None = None          # the comparison's message buffer (None: messages in registers)
    group: int = 1                           # in-batch part: queries per person
    person: list | None = None               # in-batch part, 2 eyes: 3 x u8 [2, q/2] person decisions


# Message-buffer layout of each comparison setting (imc_compare_msg_bytes's variant).
NET_VARIANT = {"mpclift": 0, "plain": CMP_PLAIN_MASK, "lift18": CMP_LIFT18, "constlift": CMP_CONST32,
               "nolift": CMP_CONST32}


def alloc_check(q: int, r: int, n: int, device=0, compare: str = "mpclift", net: str = "buffers") -> CheckBuffers:
    """Buffers of one check.  net = "buffers": the comparison's parties run
    apart and pass every message through a device buffer (406 bits per
    comparison for MPCLift); "registers": the faster simulation that holds
    all three parties of a comparison in one lane."""
    if compare not in COMPARE_SETTINGS:
        raise ValueError(compare)
    if net not in ("buffers", "registers"):
        raise ValueError(net)
    d = _dev(device)
    rows = q * r
    ld = ((n + 63) // 64) * 64
    nw = ld // 64
    plain = compare == "plain"
    v32 = VECS32.get(compare, ())
    u16 = lambda *s: torch.empty(*s, dtype=torch.int16, device=d)  # noqa: E731
    u32 = lambda *s: torch.empty(*s, dtype=torch.int32, device=d)  # noqa: E731
    code16 = 0 not in v32
    mask16 = not plain and 1 not in v32
    return CheckBuffers(
        rows=rows, n=n, ld=ld, nw=nw,
        dot_code=[u16(rows, ld) for _ in range(3)] if code16 else None,
        dot_mask=[u16(rows, ld) for _ in range(3)] if mask16 else None,
        msg=[u16(2, rows, ld) for _ in range(3)] if code16 else None,
        rep_code=[u16(2, rows, ld) for _ in range(3)] if code16 else None,
        rep_mask=[u16(2, rows, ld) for _ in range(3)] if mask16 else None,
        dot32={v: [u32(rows, ld) for _ in range(3)] for v in v32} if v32 else None,
        msg32={v: [u32(rows, ld) for _ in range(3)] for v in v32} if v32 else None,
        rep32={v: [u32(2, rows, ld) for _ in range(3)] for v in v32} if v32 else None,
        match=[torch.empty(2, rows, nw, dtype=torch.int64, device=d) for _ in range(3)],
        dup=[torch.empty(2, q, dtype=torch.uint8, device=d) for _ in range(3)],
        ws=torch.empty(max(8, or_tree_ws_bytes(q, r, nw)), dtype=torch.uint8, device=d),
        compare=compare,
        ml_pub=u16(rows, ld) if plain else None,
        row_masks=torch.empty(rows, 200, dtype=torch.int64, device=d) if plain else None,
        net=(torch.empty(compare_msg_bytes(NET_VARIANT[compare], rows, n) // 8, dtype=torch.int64, device=d)
             if net == "buffers" else None),
    )


def run_check(ctx: Context, qs: SharedQueries, rot, db: SharedDB, first_entry: int, n: int, buf: CheckBuffers,
              or_tree: bool = True, stream=None, query_masks=None, db_masks=None, qs32=None, db32=None):
    """Alg. 3 (Alg. 2 for buf.compare == "plain") for queries qs at rotations
    rot against entries first_entry..+n.  "plain" needs the public masks:
    query_masks [q, 200] and db_masks [>= first_entry + n, 200] (device int64);
    "constlift" / "nolift" the Z_2^32 operands and regions qs32, db32 of their
    vectors (qs and db then serve the code dot of "constlift" only)."""
    ids = make_ids(qs.qid_base if qs is not None else qs32.qid_base, rot, first_entry)
    plain = buf.compare == "plain"
    if buf.dot_code is not None:
        assert qs.galois == db.galois
        for p in range(3):
            ctx.dot_shares(p, qs.op[p], qs.q, ids, db.regions[p], db.capacity, n, buf.dot_code[p],
                           buf.dot_mask[p] if buf.dot_mask is not None else None, buf.ld, stream, galois=db.galois)
    if buf.dot32:
        for v, outs in buf.dot32.items():
            for p in range(3):
                ctx.dot32_shares(p, qs32.op[v][p], qs32.q, ids, db32.regions[v][p], db32.capacity, n, outs[p],
                                 buf.ld, stream)
    if plain:
        assert query_masks is not None and db_masks is not None and db_masks.shape[0] >= first_entry + n
        ctx.rotate_masks(query_masks, qs.q, ids, buf.row_masks, stream)
        ctx.plain_ml(buf.row_masks, buf.rows, db_masks[first_entry:], n, buf.ml_pub, buf.ld, stream)
    if buf.dot_code is not None:
        ctx.reshare(buf.dot_code, buf.dot_mask, buf.rows, n, buf.ld, ids, buf.msg, buf.rep_code, buf.rep_mask, stream)
    if buf.dot32:
        for v in buf.dot32:
            ctx.reshare32(v, buf.dot32[v], buf.rows, n, buf.ld, ids, buf.msg32[v], buf.rep32[v], stream)
    if buf.compare in VECS32:
        code, bits = (buf.rep32[0], 32) if 0 in buf.rep32 else (buf.rep_code, 16)
        ctx.compare_variant(CMP_CONST32, code, bits, buf.rep32[1], None, buf.rows, n, buf.ld, ids, buf.match, buf.nw,
                            stream, msg_ws=buf.net)
    elif plain:
        ctx.compare_variant(CMP_PLAIN_MASK, buf.rep_code, 16, None, buf.ml_pub, buf.rows, n, buf.ld, ids, buf.match,
                            buf.nw, stream, msg_ws=buf.net)
    elif buf.compare == "lift18":
        ctx.compare_variant(CMP_LIFT18, buf.rep_code, 16, buf.rep_mask, None, buf.rows, n, buf.ld, ids, buf.match,
                            buf.nw, stream, msg_ws=buf.net)
    else:
        ctx.compare_threshold(buf.rep_code, buf.rep_mask, buf.rows, n, buf.ld, ids, buf.match, buf.nw, stream,
                              msg_ws=buf.net)
    if or_tree:
        nw = (n + 63) // 64
        q = qs.q if qs is not None else qs32.q
        ctx.or_tree(buf.match, q, nw, buf.nw, ids, buf.ws, buf.ws.numel(), buf.dup, stream)
    return ids


def open_dup(ctx: Context, buf: CheckBuffers, q: int, check: int = 1, stream=None):
    out = torch.empty(q, dtype=torch.uint8, device=buf.dup[0].device)
    s = ctx.open(OPEN_U8_XOR, buf.dup, q, out, check, stream)
    return out, s


def open_match(ctx: Context, buf: CheckBuffers, check: int = 1, stream=None):
    out = torch.empty(buf.rows, buf.nw, dtype=torch.int64, device=buf.match[0].device)
    s = ctx.open(OPEN_U64_XOR, buf.match, buf.rows * buf.nw, out, check, stream)
    return out, s


def open_dots(ctx: Context, buf: CheckBuffers, check: int = 1, stream=None):
    outc = torch.empty(buf.rows, buf.ld, dtype=torch.int16, device=buf.rep_code[0].device)
    outm = torch.empty_like(outc)
    s1 = ctx.open(OPEN_U16_ADD, buf.rep_code, buf.rows * buf.ld, outc, check, stream)
    s2 = ctx.open(OPEN_U16_ADD, buf.rep_mask, buf.rows * buf.ld, outm, check, stream)
    return outc, outm, (s1, s2)


# In-batch matching (Sec. 6.4): the batch's queries are compared with each
# other as entries, under entry ids distinct from the database's and an
# OR-tree query-id offset distinct from the database tree's.
BATCH_ENTRY_BASE = 1 << 47
BATCH_OR_QID_OFFSET = 1 << 46
# Both eyes (Sec. 6.4): queries 2k and 2k+1 are person k's left and right
# eye; the person's decision is one more OR gate, under its own stream id.
PERSON_OR_BASE = 1 << 47


def run_in_batch(ctx: Context, qs: SharedQueries, rot, buf_db: CheckBuffers, stream=None, reuse=None,
                 group: int = 1):
    """Query qi of the batch is also compared with the queries of earlier
    groups (group=1: queries j < qi; group=2: the eyes of earlier persons).
    buf_db holds the database check of the same queries (its dup); returns
    the buffers of the batch part, whose `final` holds dup_db OR dup_batch
    per query and, for group=2, `person` the OR of each person's two eyes.
    reuse: the buffers a previous call on a batch of the same shape returned
    (nothing is allocated then)."""
    assert qs.raw is not None and 0 < qs.q <= 64 and group in (1, 2) and qs.q % group == 0
    q, r = qs.q, len(rot)
    dev = buf_db.dup[0].device
    if reuse is not None:
        assert reuse.rows == q * r and reuse.region.galois == qs.galois and reuse.group == group
        region, buf, final = reuse.region, reuse, reuse.final
    else:
        region = SharedDB(ctx, 64, galois=qs.galois, device=dev)
        buf = alloc_check(q, r, q, device=dev)
        final = [torch.empty(2, q, dtype=torch.uint8, device=dev) for _ in range(3)]
        buf.group = group
        buf.person = [torch.empty(2, q // 2, dtype=torch.uint8, device=dev) for _ in range(3)] if group == 2 else None
    for j in range(q):
        ctx.append_db(qs.raw, j, region.regions, region.capacity, j, stream, galois=qs.galois)
    region.n = q
    ids0 = make_ids(qs.qid_base, rot, 0)
    for p in range(3):
        ctx.dot_shares(p, qs.op[p], q, ids0, region.regions[p], region.capacity, q, buf.dot_code[p],
                       buf.dot_mask[p], buf.ld, stream, galois=qs.galois)
    ids = make_ids(qs.qid_base, rot, BATCH_ENTRY_BASE)
    ctx.reshare(buf.dot_code, buf.dot_mask, buf.rows, q, buf.ld, ids, buf.msg, buf.rep_code, buf.rep_mask, stream)
    ctx.compare_threshold(buf.rep_code, buf.rep_mask, buf.rows, q, buf.ld, ids, buf.match, buf.nw, stream,
                          msg_ws=buf.net)
    ctx.mask_in_batch(buf.match, q, r, buf.nw, 0, stream, group=group)
    ids_or = make_ids(qs.qid_base + BATCH_OR_QID_OFFSET, rot, BATCH_ENTRY_BASE)
    ctx.or_tree(buf.match, q, 1, buf.nw, ids_or, buf.ws, buf.ws.numel(), buf.dup, stream)
    ctx.or_bits(buf_db.dup, buf.dup, q, qs.qid_base, final, stream)
    if group == 2:
        ctx.or_pairs(final, q // 2, PERSON_OR_BASE | qs.qid_base, buf.person, stream)
    buf.final = final
    buf.region = region
    return buf
