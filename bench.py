"""Benchmark: shared iris comparisons per second on one MI355X.

Default workload: the full 3-party protocol (all parties simulated on one
GPU) for 64 queries x 31 rotations (1,984 rows) against a database of
300,000 entries per party, inputs resident in HBM.  One step = every party's
dot products, resharing, the MPCLift comparison, the OR-tree and opening the
per-query result.  `--workload party` times one party's dot products for 32
queries x 31 rotations against 1,000,000 entries instead; `batched` and
`serve` run uneven batches and the continuous-batching service; `compare`
times the comparison settings of Sec. 6.2 side by side.  `--compare` picks
the comparison setting of the full workload (MPCLift, Lift to Z_2^18 only, or
masks in plain).

Prints one JSON line (see the keys below).  Only N = 1 GPU is supported.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_I8_PEAK_TOPS = 5000.0      # MI355X dense int8, tera-ops/s (MAC = 2 ops)
# HBM traffic of one launch of the rotation-aware dot kernel (one party, 1,984
# rows x 300,000 entries) from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch, mean of 6 dispatches), each scaled by what the
# same counter reads for a 1 GiB device-to-device copy (FETCH_SIZE 524,302 KiB,
# WRITE_SIZE 1,048,580 KiB).  Valid only for the kernel sources it was taken on.
DOT_TRAFFIC = {
    "sources": {"paper_2405_04463_amd/csrc/rot_dot.hip":
                "a9592bebea11d7be944f6ee6108420874e50f6ff51af5bcf44a651a8a84dd862",
                "paper_2405_04463_amd/csrc/device.h":
                "4c1a3b4ab4b31d959d8bad5a27477516a04872568ad8d0abc29b0de3c59b9f10"},
    "rows": 1984, "n_db": 300_000,
    "fetch_kib": 16_900_882.0, "write_kib": 2_329_442.0,
    "fetch_scale": 1_048_576 / 524_303.0, "write_scale": 1_048_576 / 1_048_580.0,
}

HBM_PEAK_GBS = 8000.0
OPS_PER_CMP_PARTY = 2 * 2 * 12800 * 3 * 2   # (code, mask) x K=25,600 x 3 limb products x 2 ops = 307,200
DB_BYTES_PER_ENTRY_PARTY = 4 * 2 * 12800      # 4 limb planes x K=25,600 bytes = 102,400


def dot_traffic(rows, n_db, dot_tiles):
    """HBM bytes per dot launch from the stored counter passes, or None when
    the workload, the kernel configuration or its sources differ."""
    t = DOT_TRAFFIC
    if rows != t["rows"] or n_db != t["n_db"] or dot_tiles not in (0, 4):
        return None
    for rel, digest in t["sources"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def keys():
    dealer = hashlib.sha256(b"bench-dealer").digest()
    party = b"".join(hashlib.sha256(b"bench-party%d" % i).digest() for i in range(3))
    return dealer, party


def enroll_db(ctx, db, seed, n, chunk=32768, keep_masks=False, db32=None):
    """Share entries 0..n-1 into db (and into the Z_2^32 regions db32); with
    keep_masks also return the packed masks on the device ([n, 200] int64:
    the public masks of the setting with masks in plain)."""
    import torch

    import workload as wl

    masks = torch.empty(n, 200, dtype=torch.int64, device="cuda") if keep_masks else None
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        c, k = wl.gen_codes(seed, s, m)
        cd = torch.from_numpy(c.view(np.int64)).cuda()
        kd = torch.from_numpy(k.view(np.int64)).cuda()
        if db is not None:
            db.enroll(cd, kd, s)
        if db32 is not None:
            db32.enroll(cd, kd, s)
        if masks is not None:
            masks[s:s + m] = kd
    torch.cuda.synchronize()
    return masks


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, qc, qm, sample_q=4, sample_n=40960, galois=False, compare="mpclift"):
    """The oracle's step (local dots of all parties, reshare, compare, OR-tree)
    on a bounded sample of the same workload on all host threads, plus the
    same step and the plaintext check (popcounts) on one thread; shares are
    made before timing."""
    import oracle as orc
    import workload as wl

    dealer, party = keys()
    dc, dm = wl.gen_codes(w.seed, 0, sample_n)

    def shares(nq, n):
        if galois:
            qsh = orc.galois_share(dealer, orc.DOM_GALOIS_QUERY, qc[:nq], qm[:nq], 0)
            dsh = orc.galois_share(dealer, orc.DOM_GALOIS_DB, dc[:n], dm[:n], 0)
        else:
            qsh = orc.share(dealer, orc.DOM_SHARE_QUERY, qc[:nq], qm[:nq], 0)
            dsh = orc.share(dealer, orc.DOM_SHARE_DB, dc[:n], dm[:n], 0)
        q32 = d32 = None
        if compare in ("constlift", "nolift"):
            q32 = orc.share32(dealer, orc.DOM_SHARE32_QUERY, qc[:nq], qm[:nq], 0)
            d32 = orc.share32(dealer, orc.DOM_SHARE32_DB, dc[:n], dm[:n], 0)
        return qsh, dsh, q32, d32

    def step(nq, n, sh):
        qsh, dsh, q32, d32 = sh
        local_dot = orc.galois_local_dot if galois else orc.local_dot
        t0 = time.perf_counter()
        zc, zm = [], []
        for p in range(3):
            c, m = local_dot(p, qsh, w.rot, dsh)
            zc.append(c)
            zm.append(m)
        rc, rm = orc.reshare(party, np.stack(zc), np.stack(zm), nq, w.rot, 0, 0)
        if q32 is not None:
            z32 = [orc.local_dot32(p, q32, w.rot, d32) for p in range(3)]
            rc32, rm32 = orc.reshare32(party, np.stack([z[0] for z in z32]) if compare == "nolift" else None,
                                       np.stack([z[1] for z in z32]), nq, w.rot, 0, 0)
            match = orc.compare_variant(party, orc.CMPV_CONST32, rc32 if compare == "nolift" else rc, rm32, None,
                                        nq, w.rot, 0, 0)
        elif compare == "plain":
            _, ml, _, _ = orc.plain(qc[:nq], qm[:nq], w.rot, dc[:n], dm[:n])   # public ml
            match = orc.compare_variant(party, orc.CMPV_PLAIN, rc, None, ml, nq, w.rot, 0, 0)
        elif compare == "lift18":
            match = orc.compare_variant(party, orc.CMPV_LIFT18, rc, rm, None, nq, w.rot, 0, 0)
        else:
            match = orc.compare(party, rc, rm, nq, w.rot, 0, 0)
        orc.or_tree(party, match, nq, len(w.rot), 0)
        return time.perf_counter() - t0

    def plain_rate(nq, n):
        t0 = time.perf_counter()
        orc.plain(qc[:nq], qm[:nq], w.rot, dc[:n], dm[:n])
        return nq * len(w.rot) * n / (time.perf_counter() - t0)

    dt = step(sample_q, sample_n, shares(sample_q, sample_n))
    ncmp = sample_q * len(w.rot) * sample_n
    cores = orc.threads()
    o1_all = plain_rate(sample_q, sample_n)
    # one thread: one query of the sample against 1,024 entries
    one_n = min(1024, sample_n)
    sh1 = shares(1, one_n)
    old = orc.set_threads(1)
    try:
        dt1 = step(1, one_n, sh1)
        o1_one = plain_rate(1, one_n)
    finally:
        orc.set_threads(old)
    n1 = len(w.rot) * one_n
    return {"value": ncmp / dt, "unit": "comparisons/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle step (3 parties' local dots, reshare, {compare} compare, OR-tree) on {sample_q} "
                      f"queries x {len(w.rot)} rotations x {sample_n} entries = {ncmp} comparisons, {dt:.1f} s",
            "cpu_model": _cpu_model(),
            "single_core": {"value": n1 / dt1, "sample": f"the same step on 1 query x {len(w.rot)} rotations x "
                                                         f"{one_n} entries, one thread, {dt1:.1f} s"},
            "plaintext_check": {"all_cores": o1_all, "single_core": o1_one, "unit": "comparisons/s",
                                "note": "the oracle's plaintext definition (popcounts of masked XOR and AND)"}}


def verify(ctx, buf, w, qc, qm, party_keys):
    """Every opened value of the step against the plaintext oracle (Alg. 1)
    and the duplicate-bit components against the oracle's OR-tree (Sec. 4.2)
    over the GPU's own match-bit components: each opened one is re-decided
    on its pair and must be a match; the opened ones must be exactly the
    plaintext matches of the planted pairs (all rotations), every other pair
    being a random code ~25 standard deviations above the threshold; and
    every opened duplicate bit must equal the plaintext one (0 for a query
    without a planted match)."""
    import oracle as orc
    import workload as wl
    from paper_2405_04463_amd.pipeline import open_dup, open_match

    mo, s1 = open_match(ctx, buf, check=1)
    do, s2 = open_dup(ctx, buf, w.n_q, check=1)
    mo = mo.cpu().numpy().view(np.uint64)
    dup = do.cpu().numpy()
    r, n = len(w.rot), buf.n
    ones = []
    for row, word in zip(*[x.tolist() for x in np.nonzero(mo)]):
        v = int(mo[row, word])
        while v:
            low = v & -v
            ones.append((row, 64 * word + low.bit_length() - 1))
            v ^= low
    ents = sorted({c for _, c in ones if c < n} | {e for _, e, _, _ in w.planted})
    dc = np.empty((len(ents), 200), np.uint64)
    dm = np.empty_like(dc)
    for i, e in enumerate(ents):
        c, m = wl.gen_codes(w.seed, e, 1)
        dc[i], dm[i] = c[0], m[0]
    _, _, match, _ = orc.plain(qc, qm, w.rot, dc, dm)
    col = {e: i for i, e in enumerate(ents)}
    want = {(qi * r + ri, e) for qi, e, _, _ in w.planted for ri in range(r) if match[qi * r + ri, col[e]]}
    rejected = sum(1 for row, c in ones if c >= n or not match[row, col[c]])
    want_dup = np.zeros(w.n_q, np.uint8)
    for row, _ in want:
        want_dup[row // r] = 1
    comps = np.stack([buf.match[p][0].cpu().numpy().view(np.uint64)[:, :(n + 63) // 64] for p in range(3)])
    ref, _ = orc.or_tree(party_keys, comps, w.n_q, r, 0)
    or_ok = all(np.array_equal(buf.dup[p][0].cpu().numpy(), ref[p]) for p in range(3))
    ok = (rejected == 0 and set(ones) == want and np.array_equal(dup, want_dup) and or_ok
          and s1 == 0 and s2 == 0)
    return {"bit_exact": bool(ok), "opened_bits": int(mo.shape[0]) * n,
            "opened_ones": len(ones), "ones_rejected_by_plaintext": rejected, "planted_matches": len(want),
            "dup_true": int(dup.sum()), "dup_expected": int(want_dup.sum()), "or_tree_components_equal": or_ok}


def verify_in_batch(ctx, buf, bb, w, qc, qm):
    """The opened final decision of every query against the opened database
    decision OR the plaintext decision over the queries of earlier groups
    (w.group = 2: the eyes of earlier persons); with two eyes, also every
    opened person decision against the OR of its eyes' expected decisions."""
    import torch

    import oracle as orc
    import paper_2405_04463_amd as imc
    from paper_2405_04463_amd.pipeline import open_dup

    g = w.group
    db_dup, s1 = open_dup(ctx, buf, w.n_q, check=1)
    final = torch.empty(w.n_q, dtype=torch.uint8, device="cuda")
    s2 = ctx.open(imc.OPEN_U8_XOR, bb.final, w.n_q, final, 1)
    torch.cuda.synchronize()
    batch = np.zeros(w.n_q, dtype=np.uint8)
    for i in range(g, w.n_q):
        k = g * (i // g)
        batch[i] = orc.plain(qc[i:i + 1], qm[i:i + 1], w.rot, qc[:k], qm[:k])[3][0]
    want = db_dup.cpu().numpy() | batch
    got = final.cpu().numpy()
    res = {"bit_exact": bool(np.array_equal(got, want)) and s1 == 0 and s2 == 0,
           "batch_duplicates": int(batch.sum()), "final_true": int(got.sum())}
    if g == 2:
        persons = torch.empty(w.n_q // 2, dtype=torch.uint8, device="cuda")
        s3 = ctx.open(imc.OPEN_U8_XOR, bb.person, w.n_q // 2, persons, 1)
        torch.cuda.synchronize()
        pw = want[0::2] | want[1::2]
        pg = persons.cpu().numpy()
        res["persons_bit_exact"] = bool(np.array_equal(pg, pw)) and s3 == 0
        res["bit_exact"] = res["bit_exact"] and res["persons_bit_exact"]
        res["persons"] = int(pg.size)
        res["persons_duplicate"] = int(pg.sum())
        # the patterns of the workload: eyes the database holds, eyes that
        # only in-batch matching finds, and a person's own eyes never meeting
        res["persons_by_left_eye_only"] = int(((want[0::2] == 1) & (want[1::2] == 0)).sum())
        res["persons_by_right_eye_only"] = int(((want[0::2] == 0) & (want[1::2] == 1)).sum())
        res["persons_by_both_eyes"] = int(((want[0::2] == 1) & (want[1::2] == 1)).sum())
    return res


# ChaCha12 blocks per 64 comparisons of each comparison circuit (their PRF tapes)
# and int32 ops per block (12 rounds x 4 quarter-rounds x 12 ops + 16 adds).
CMP_BLOCKS_PER_64 = {"mpclift": 55, "lift18": 34, "plain": 12, "constlift": 24, "nolift": 24}
CHACHA12_OPS = 12 * 4 * 12 + 16
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12     # int32 lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz


# Bits each party sends per comparison, per setting (the oracle's message
# counts): AND-gate messages plus the 3OT roles of the BitInjects.
MSG_BITS = {"mpclift": (156, 125, 125), "lift18": (72, 69, 69), "plain": (29, 29, 29), "constlift": (61, 61, 61),
            "nolift": (61, 61, 61)}


def circuit_report(compare, ncmp, reshare_ms, compare_ms, plain, v32, net="registers", other_ms=None,
                   msgs_only=False):
    """The interactive steps of one batch: resharing against the HBM roof
    (algorithmic bytes) and the comparison against the VALU roof (its PRF
    work alone, a lower bound on its ops).  net: how the step's comparison
    passed its messages ("buffers": parties apart, every message stored and
    loaded through device memory; "registers": the three parties of a
    comparison in one lane); other_ms: the comparison in the other mode;
    msgs_only: the resharing wrote its messages only (the comparison reads
    the replicated components in place from them)."""
    n16 = 0 if 0 in v32 else 1
    n16 += 0 if (plain or 1 in v32) else 1                 # Z_2^16 vectors reshared
    # per vector and comparison, 3 parties: read the additive share, write the
    # message and both planes of the replicated share: 3 x (1 + 1 + 2) elements;
    # messages only: 3 x (1 + 1)
    per = 2 if msgs_only else 4
    per_vec16, per_vec32 = 3 * per * 2, 3 * per * 4
    rb = ncmp * (n16 * per_vec16 + len(v32) * per_vec32)
    ops = ncmp * CMP_BLOCKS_PER_64[compare] * CHACHA12_OPS / 64
    bits = MSG_BITS[compare]
    # the buffered network runs each party's two keys: 2 of the 3 PRF blocks
    # per tape position per party, i.e. twice the register simulation's PRF work
    ops_net = ops * (2 if net == "buffers" else 1)
    r = {"reshare_writes": "messages" if msgs_only else "messages and replicated planes",
         "reshare_ms": reshare_ms, "reshare_bytes": rb, "reshare_gbs": rb / (reshare_ms / 1e3) / 1e9,
         "reshare_hbm_frac": rb / (reshare_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
         "compare_net": net, "compare_ms": compare_ms, "compare_prf_ops": ops_net,
         "compare_valu_tops": ops_net / (compare_ms / 1e3) / 1e12,
         "compare_valu_frac": ops_net / (compare_ms / 1e3) / 1e12 / VALU_PEAK_TOPS,
         "message_bits_per_comparison": {"party0": bits[0], "party1": bits[1], "party2": bits[2]}}
    if net == "buffers":
        mb = ncmp * sum(bits) / 8
        r["message_bytes"] = mb
        r["message_gbs"] = 2 * mb / (compare_ms / 1e3) / 1e9      # each message stored once and loaded once
    if other_ms is not None:
        r["compare_ms_" + ("registers" if net == "buffers" else "buffers")] = other_ms
    return r


def run_full(args):
    import torch

    import paper_2405_04463_amd as imc
    import workload as wl
    from paper_2405_04463_amd.pipeline import (VECS32, SharedDB, SharedDB32, SharedQueries, SharedQueries32,
                                               alloc_check, open_dup, run_check, run_in_batch)

    if args.two_eyes:
        w = wl.two_eyes(n_db=args.n_db, persons=(args.n_q or 64) // 2)
    else:
        w = wl.full_protocol(n_db=args.n_db, n_q=args.n_q)
    in_batch = args.in_batch or args.two_eyes
    if in_batch and (args.compare != "mpclift" or w.n_q < 16):
        raise SystemExit("--in-batch and --two-eyes run with the MPCLift comparison and at least 16 queries")
    dealer, party = keys()
    galois = args.scheme == "galois"
    plain = args.compare == "plain"
    v32 = VECS32.get(args.compare, ())
    code16 = 0 not in v32
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=w.rows, dot_tiles=args.dot_tiles)
    nbytes = (imc.galois_db_bytes(w.n_db) if galois else imc.db_bytes(w.n_db)) if code16 else 0
    nbytes += len(v32) * imc.db32_bytes(w.n_db)
    log(f"enrolling {w.n_db} entries x 3 parties ({3 * nbytes / 1e9:.1f} GB, {args.scheme} shares"
        + (f", Z_2^32 vectors {v32}" if v32 else "") + ")")
    probe = serve_probe_applies(args)
    # room for the served-latency probe's appended uniques
    db = SharedDB(ctx, (w.n_db + (SERVE_PROBE_REQUESTS if probe else 0)) if code16 else 32, galois=galois)
    db32 = SharedDB32(ctx, w.n_db, vecs=v32) if v32 else None
    db_masks = enroll_db(ctx, db if code16 else None, w.seed, w.n_db, keep_masks=plain, db32=db32)
    qc, qm = wl.make_queries(w)
    if args.two_eyes:
        wl.plant_in_batch(w, qc, qm, w.batch_pairs)
    elif in_batch:
        wl.plant_in_batch(w, qc, qm)
    q_codes = torch.from_numpy(qc.view(np.int64)).cuda()
    q_masks = torch.from_numpy(qm.view(np.int64)).cuda()
    qs = SharedQueries(ctx, q_codes, q_masks, 0, galois=galois)
    qs32 = SharedQueries32(ctx, q_codes, q_masks, 0, vecs=v32) if v32 else None
    buf = alloc_check(w.n_q, len(w.rot), w.n_db, compare=args.compare, net=args.net)
    torch.cuda.synchronize()
    log(f"first step + verification against the oracle ({args.compare} comparison)")
    run_check(ctx, qs, w.rot, db, 0, w.n_db, buf, query_masks=q_masks, db_masks=db_masks, qs32=qs32, db32=db32)
    torch.cuda.synchronize()
    ver = verify(ctx, buf, w, qc, qm, party)
    log(f"verification: {ver}")
    # the verified step's match and duplicate components, to check the timed
    # steps (which may take another route, e.g. the messages-only resharing)
    ref_match = [m.clone() for m in buf.match]
    ref_dup = [d.clone() for d in buf.dup]
    bb = None
    if in_batch:
        bb = run_in_batch(ctx, qs, w.rot, buf, group=w.group)
        ver["in_batch"] = verify_in_batch(ctx, buf, bb, w, qc, qm)
        log(f"in-batch verification: {ver['in_batch']}")
    final_out = torch.empty(w.n_q, dtype=torch.uint8, device="cuda")

    stream = torch.cuda.current_stream()
    ids = imc.make_ids(0, w.rot, 0)
    # MPCLift: the resharing writes its messages only and the comparison reads
    # each party's components in place (own message, the one received)
    msgs_only = args.compare == "mpclift"

    def compare(net):
        """The step's comparison; net: its message buffer (None: messages in registers)."""
        if plain:
            ctx.compare_variant(imc.CMP_PLAIN_MASK, buf.rep_code, 16, None, buf.ml_pub, buf.rows, w.n_db, buf.ld,
                                ids, buf.match, buf.nw, stream, msg_ws=net)
        elif args.compare == "lift18":
            ctx.compare_variant(imc.CMP_LIFT18, buf.rep_code, 16, buf.rep_mask, None, buf.rows, w.n_db, buf.ld,
                                ids, buf.match, buf.nw, stream, msg_ws=net)
        elif v32:
            code, bits = (buf.rep32[0], 32) if 0 in v32 else (buf.rep_code, 16)
            ctx.compare_variant(imc.CMP_CONST32, code, bits, buf.rep32[1], None, buf.rows, w.n_db, buf.ld, ids,
                                buf.match, buf.nw, stream, msg_ws=net)
        else:
            # the replicated components read in place from the resharing's messages
            ctx.compare_threshold_msgs(buf.msg, buf.rows, w.n_db, buf.ld, ids, buf.match, buf.nw, stream, msg_ws=net)

    def step(events=None):
        for p in range(3):
            if events is not None:
                events[p][0].record(stream)
            if code16:
                ctx.dot_shares(p, qs.op[p], qs.q, ids, db.regions[p], db.capacity, w.n_db, buf.dot_code[p],
                               buf.dot_mask[p] if buf.dot_mask is not None else None, buf.ld, stream, galois=galois)
            for v in v32:
                ctx.dot32_shares(p, qs32.op[v][p], qs.q, ids, db32.regions[v][p], db32.capacity, w.n_db,
                                 buf.dot32[v][p], buf.ld, stream)
            if events is not None:
                events[p][1].record(stream)
        if plain:   # masks public: every party computes ml itself
            ctx.rotate_masks(q_masks, qs.q, ids, buf.row_masks, stream)
            ctx.plain_ml(buf.row_masks, buf.rows, db_masks, w.n_db, buf.ml_pub, buf.ld, stream)
        if events is not None:
            events[3][0].record(stream)
        if code16 and msgs_only:
            ctx.reshare(buf.dot_code, buf.dot_mask, buf.rows, w.n_db, buf.ld, ids, buf.msg, None, None, stream)
        elif code16:
            ctx.reshare(buf.dot_code, buf.dot_mask, buf.rows, w.n_db, buf.ld, ids, buf.msg, buf.rep_code,
                        buf.rep_mask, stream)
        for v in v32:
            ctx.reshare32(v, buf.dot32[v], buf.rows, w.n_db, buf.ld, ids, buf.msg32[v], buf.rep32[v], stream)
        if events is not None:
            events[3][1].record(stream)
            events[4][0].record(stream)
        compare(buf.net)
        if events is not None:
            events[4][1].record(stream)
        ctx.or_tree(buf.match, qs.q, buf.nw, buf.nw, ids, buf.ws, buf.ws.numel(), buf.dup, stream)
        if in_batch:
            if events is not None:
                events[5][0].record(stream)
            run_in_batch(ctx, qs, w.rot, buf, stream, reuse=bb, group=w.group)
            if events is not None:
                events[5][1].record(stream)
            if w.group == 2:
                ctx.open(imc.OPEN_U8_XOR, bb.person, qs.q // 2, final_out, 0, stream)
            else:
                ctx.open(imc.OPEN_U8_XOR, bb.final, qs.q, final_out, 0, stream)
        else:
            open_dup(ctx, buf, qs.q, check=0, stream=stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup}")
    evs = []
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(6)]
        step(ev)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        evs.append(ev)
        log(f"step {i + 1}/{args.steps}: {lat[-1] * 1e3:.1f} ms")
    total = time.perf_counter() - t0
    ver["timed_steps_equal_verified_step"] = bool(
        all(torch.equal(a, b) for a, b in zip(ref_match, buf.match)) and
        all(torch.equal(a, b) for a, b in zip(ref_dup, buf.dup)))
    del ref_match, ref_dup
    # the comparison in the other network mode, outside the timed steps (the
    # register simulation when the step passes messages through the buffer)
    other_ms = None
    if buf.net is not None:
        ts = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            compare(None)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        other_ms = float(np.mean(ts))     # (the same match components as the step's)
    dot_ms = [a.elapsed_time(b) for ev in evs for a, b in ev[:3]]
    reshare_ms = float(np.mean([ev[3][0].elapsed_time(ev[3][1]) for ev in evs]))
    compare_ms = float(np.mean([ev[4][0].elapsed_time(ev[4][1]) for ev in evs]))
    ncmp = w.rows * w.n_db
    ms = total / args.steps * 1e3
    dot_avg_s = float(np.mean(dot_ms)) / 1e3
    # per party: 3 limb products per Z_2^16 vector, 10 per Z_2^32 vector (a
    # vector is 25,600 k x 2 ops per product); masks in plain: code dot only
    n16 = 0 if not code16 else (1 if (plain or v32) else 2)
    prods = 3 * n16 + 10 * len(v32)
    vec_frac = prods / 6.0
    ops = int(ncmp * (OPS_PER_CMP_PARTY // 2 if galois else OPS_PER_CMP_PARTY) * vec_frac)
    achieved = ops / dot_avg_s / 1e12
    traffic = None if (galois or plain or v32) else dot_traffic(w.rows, w.n_db, args.dot_tiles)
    entry_bytes = int((DB_BYTES_PER_ENTRY_PARTY // 2 if galois else DB_BYTES_PER_ENTRY_PARTY) * (n16 + 2 * len(v32)) / 2)
    alg_bytes = w.n_db * entry_bytes + 2 * 2 * w.rows * w.n_db   # DB region read + u16 outputs
    res = {
        "metric": "shared iris comparisons/sec on 1 MI355X (bit-exact); p50/p99 query latency",
        "value": ncmp / (total / args.steps),
        "unit": "comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16", "data": "synthetic",
        "config": {"workload": f"3-party protocol on one GPU: DB {w.n_db} entries per party, {w.n_q} queries x "
                               f"{len(w.rot)} rotations ({w.rows} rows)"
                               + (", dot products on Galois-ring Shamir shares" if galois else "")
                               + {"mpclift": "", "lift18": ", ml lifted to Z_2^18 only",
                                  "plain": ", masks in plain (public ml, code dot only)",
                                  "constlift": ", ml by a dot product over Z_2^32 (ConstLift)",
                                  "nolift": ", both dot products over Z_2^32 (NoLift)"}[args.compare],
                   "rows": w.rows, "db_entries": w.n_db, "parties": 3, "sharing": args.scheme,
                   "comparison": args.compare},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                       "note": "one batch of all queries per step; per-query latency = step latency"},
        "roofline": {"bound": "mfma", "kernel": "dot_shares (one party, i8 MFMA over byte limbs)",
                     "achieved": achieved, "peak": MFMA_I8_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / MFMA_I8_PEAK_TOPS, "traffic": traffic,
                     "ops_per_launch": ops, "avg_launch_ms": dot_avg_s * 1e3,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "hbm_gbs": None if traffic is None else traffic / dot_avg_s / 1e9},
        "circuit": circuit_report(args.compare, w.rows * w.n_db, reshare_ms, compare_ms, plain, v32, args.net,
                                  other_ms, msgs_only),
        "verification": ver,
    }
    if args.two_eyes:
        res["config"]["workload"] = (f"3-party protocol on one GPU: DB {w.n_db} entries per party, "
                                     f"{w.n_q // 2} persons x 2 eyes x {len(w.rot)} rotations ({w.rows} rows), "
                                     f"in-batch matching of each eye against the eyes of earlier persons "
                                     f"({w.rows} x {w.n_q} more comparisons), a person a duplicate if "
                                     f"either eye is")
        res["config"]["persons"] = w.n_q // 2
    elif in_batch:
        res["config"]["workload"] += (f", plus in-batch matching (each query against the batch's earlier "
                                      f"queries: {w.rows} x {w.n_q} more comparisons)")
    if probe:
        # per-query latency: the continuous-batching service on the same
        # resident database (the step's buffers are released first)
        del step, compare, buf, bb
        torch.cuda.empty_cache()
        db.n = w.n_db
        served = serve_probe(ctx, db, w)
        res["step_latency_ms"] = res["latency_ms"]
        res["latency_ms"] = {"p50": served["p50_ms"], "p99": served["p99_ms"],
                             "note": "per query, from arrival to opened decision, in the continuous-batching "
                                     "service on the same database (see served)"}
        res["served"] = served
    if in_batch:
        res["config"]["in_batch"] = True
        res["in_batch"] = {"ms_per_step": float(np.mean([ev[5][0].elapsed_time(ev[5][1]) for ev in evs])),
                           "comparisons": w.rows * w.n_q,
                           "note": "batch appended as entries, dots, reshare, compare, triangle mask, OR-tree, "
                                   "OR with the database decision"
                                   + (", OR of each person's two eyes" if w.group == 2 else "")
                                   + "; inside the timed step"}
    return res, (w, qc, qm)


SERVE_PROBE_RATE = 50.0        # requests per second
SERVE_PROBE_REQUESTS = 100     # two seconds of arrivals


def serve_probe_applies(args) -> bool:
    return (args.workload == "full" and args.compare == "mpclift" and not args.in_batch and not args.two_eyes
            and not args.no_serve_probe)


def serve_probe(ctx, db, w):
    """Poisson arrivals of single-iris requests (31 rotations) at 50/s into
    the continuous-batching service over the step's resident database:
    p50/p99 from arrival to opened decision, two requests planted as
    near-duplicates of database entries (their decisions re-decided on the
    plaintext pair), the rest random codes, which are appended as unique
    entries in serial order; then the plain per-query path on the grown
    database for comparison."""
    import torch

    import oracle as orc
    import workload as wl
    from paper_2405_04463_amd.serve import Request, Server, plain_check

    rot = w.rot
    n_req = SERVE_PROBE_REQUESTS
    qid0 = 1 << 32                                    # ids apart from the step's queries
    rng = np.random.default_rng(0x5E57E)
    arr = np.cumsum(rng.exponential(1.0 / SERVE_PROBE_RATE, n_req))
    qc, qm = wl.gen_codes(w.seed ^ 0x5E57E, qid0, n_req, query=True)
    planted = {17: (int(w.n_db * 0.3), 5), 71: (w.n_db - 1, -9)}   # request -> (entry, rotation)
    for i, (e, sft) in planted.items():
        ec, em = wl.gen_codes(w.seed, e, 1)
        qc[i], qm[i] = wl.plant(w.seed, qid0 + i, ec[0], em[0], sft, h=0.2)
    reqs = [Request(rid=i, qid=qid0 + i, code=qc[i], mask=qm[i], arrival=float(arr[i])) for i in range(n_req)]
    srv = Server(ctx, db, rot, chunk=65536, slots=64, serial=True, net="buffers")
    n0 = db.n
    log(f"served-latency probe: {n_req} requests at {SERVE_PROBE_RATE:.0f}/s, DB {n0} entries")
    t0 = time.perf_counter()
    done = srv.run(reqs, timeout=120)
    wall = time.perf_counter() - t0
    lat = np.array([r.done_at - r.arrival for r in done])
    dups = sorted(r.rid for r in done if r.dup)
    want = []
    for i, (e, _) in planted.items():
        ec, em = wl.gen_codes(w.seed, e, 1)
        if orc.plain(qc[i:i + 1], qm[i:i + 1], rot, ec, em)[3][0]:
            want.append(i)
    ts, cache = [], {}
    for i in range(4):
        q = Request(rid=i, qid=qid0 + n_req + i, code=qc[i], mask=qm[i])
        t1 = time.perf_counter()
        plain_check(ctx, db, q, rot, cache)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t1)
    del srv, cache
    torch.cuda.empty_cache()
    t_plain = float(np.median(ts[1:]))
    out = {"lambda_per_s": SERVE_PROBE_RATE, "requests": n_req, "wall_s": wall,
           "comparisons_per_s": srv_cmps(done, rot, n0), "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "db_entries_at_start": n0,
           "appended": db.n - n0, "duplicates": dups, "duplicates_expected": sorted(want),
           "decisions_ok": dups == sorted(want) and db.n - n0 == n_req - len(want),
           "plain_per_query_ms": t_plain * 1e3,
           "workload": f"continuous-batching service, 3 parties on one GPU, Poisson arrivals at "
                       f"{SERVE_PROBE_RATE:.0f}/s of one iris at {len(rot)} rotations, chunks of 65,536 entries, "
                       f"64 slots, serial uniqueness, uniques appended, comparison messages through the device "
                       f"buffer"}
    log(f"served: p50 {out['p50_ms']:.1f} ms, p99 {out['p99_ms']:.1f} ms, plain per query {t_plain * 1e3:.1f} ms, "
        f"decisions ok: {out['decisions_ok']}")
    return out


def srv_cmps(done, rot, n0):
    """Comparisons per second the probe's requests received over its run
    (each request against the database it was checked against)."""
    if not done:
        return 0.0
    t = max(r.done_at for r in done) - min(r.arrival for r in done)
    return sum(len(rot) * r.checked for r in done) / t if t > 0 else 0.0


# AND gates and bits sent by party 0 per comparison, per setting (Sec. 6.2).
COMPARE_COUNTS = {"mpclift": (94, 156), "lift18": (66, 72), "plain": (29, 29), "constlift": (61, 61),
                  "nolift": (61, 61)}


def run_compare(args):
    """The comparison settings side by side (Sec. 6.2, Table 3): each setting's
    comparison kernel over the same rows x entries of replicated components
    resident in HBM, then the OR-tree over one setting's output.  Component
    values are random (the kernels' work does not depend on them; their
    results are checked against the oracle by the test-suite)."""
    import torch

    import paper_2405_04463_amd as imc

    dealer, party = keys()
    rot = list(range(-15, 16))
    q, n = args.n_q, args.n_db
    rows = q * len(rot)
    ld = ((n + 63) // 64) * 64
    nw = ld // 64
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=rows)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)

    def rnd(dtype, lo, hi, shape):
        return torch.randint(lo, hi, shape, dtype=dtype, device="cuda", generator=g)

    log(f"components for {rows} rows x {n} entries")
    code = [rnd(torch.int16, -32768, 32768, (2, rows, ld)) for _ in range(3)]
    mask = [rnd(torch.int16, -32768, 32768, (2, rows, ld)) for _ in range(3)]
    code32 = [rnd(torch.int32, -2**31, 2**31 - 1, (2, rows, ld)) for _ in range(3)]
    mask32 = [rnd(torch.int32, -2**31, 2**31 - 1, (2, rows, ld)) for _ in range(3)]
    ml_pub = rnd(torch.int16, 0, 12801, (rows, ld))
    match = [torch.empty(2, rows, nw, dtype=torch.int64, device="cuda") for _ in range(3)]
    dup = [torch.empty(2, q, dtype=torch.uint8, device="cuda") for _ in range(3)]
    ws = torch.empty(max(8, imc.or_tree_ws_bytes(q, len(rot), nw)), dtype=torch.uint8, device="cuda")
    ids = imc.make_ids(0, rot, 0)
    stream = torch.cuda.current_stream()
    calls = {
        "mpclift": lambda: ctx.compare_threshold(code, mask, rows, n, ld, ids, match, nw, stream),
        "lift18": lambda: ctx.compare_variant(imc.CMP_LIFT18, code, 16, mask, None, rows, n, ld, ids, match, nw,
                                              stream),
        "plain": lambda: ctx.compare_variant(imc.CMP_PLAIN_MASK, code, 16, None, ml_pub, rows, n, ld, ids, match, nw,
                                             stream),
        "constlift": lambda: ctx.compare_variant(imc.CMP_CONST32, code, 16, mask32, None, rows, n, ld, ids, match,
                                                 nw, stream),
        "nolift": lambda: ctx.compare_variant(imc.CMP_CONST32, code32, 32, mask32, None, rows, n, ld, ids, match,
                                              nw, stream),
        "or_tree": lambda: ctx.or_tree(match, q, nw, nw, ids, ws, ws.numel(), dup, stream),
    }
    # the same settings with the parties apart and their messages through a device buffer
    net = torch.empty(imc.compare_msg_bytes(0, rows, n) // 8, dtype=torch.int64, device="cuda")
    calls.update({
        "mpclift_buffers": lambda: ctx.compare_threshold(code, mask, rows, n, ld, ids, match, nw, stream, msg_ws=net),
        "lift18_buffers": lambda: ctx.compare_variant(imc.CMP_LIFT18, code, 16, mask, None, rows, n, ld, ids, match,
                                                      nw, stream, msg_ws=net),
        "plain_buffers": lambda: ctx.compare_variant(imc.CMP_PLAIN_MASK, code, 16, None, ml_pub, rows, n, ld, ids,
                                                     match, nw, stream, msg_ws=net),
        "constlift_buffers": lambda: ctx.compare_variant(imc.CMP_CONST32, code, 16, mask32, None, rows, n, ld, ids,
                                                         match, nw, stream, msg_ws=net),
        "nolift_buffers": lambda: ctx.compare_variant(imc.CMP_CONST32, code32, 32, mask32, None, rows, n, ld, ids,
                                                      match, nw, stream, msg_ws=net),
    })
    out = {}
    ncmp = rows * n
    for name, fn in calls.items():
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        out[name] = {"ms": ms, "elements_per_s": ncmp / (ms / 1e3)}
        setting = name.split("_")[0]
        if setting in COMPARE_COUNTS:
            ands, bits = COMPARE_COUNTS[setting]
            out[name].update(and_gates=ands, bits_sent_party0=bits, kb_per_party_per_100k=bits * 100_000 / 8e3,
                             messages="device buffer, parties apart" if name.endswith("_buffers")
                             else "registers, three parties per lane")
        log(f"{name}: {ms:.3f} ms per call, {ncmp / (ms / 1e3):.3e} elements/s")
    res = {
        "metric": "shared iris comparisons/sec on 1 MI355X (bit-exact); p50/p99 query latency",
        "value": out["mpclift_buffers"]["elements_per_s"], "unit": "comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": out["mpclift_buffers"]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16", "data": "synthetic",
        "config": {"workload": f"comparison kernels alone (3 parties on one GPU, messages through a device "
                               f"buffer): {q} queries x {len(rot)} rotations ({rows} rows) x {n} entries of "
                               f"reshared components per call",
                   "rows": rows, "db_entries": n},
        "settings": out,
    }
    return res, (None, None, None)


def run_party(args):
    import torch

    import paper_2405_04463_amd as imc
    import workload as wl
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries

    w = wl.party_local(n_db=args.n_db, n_q=args.n_q)
    dealer, party = keys()
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=w.rows, dot_tiles=args.dot_tiles)
    db = SharedDB(ctx, w.n_db, parties=(0,))
    log(f"enrolling {w.n_db} entries ({imc.db_bytes(w.n_db) / 1e9:.1f} GB, party 0's region)")
    enroll_db(ctx, db, w.seed, w.n_db)
    qc, qm = wl.make_queries(w)
    qs = SharedQueries(ctx, torch.from_numpy(qc.view(np.int64)).cuda(), torch.from_numpy(qm.view(np.int64)).cuda(), 0)
    ld = ((w.n_db + 63) // 64) * 64
    code = torch.empty(w.rows, ld, dtype=torch.int16, device="cuda")
    mask = torch.empty_like(code)
    ids = imc.make_ids(0, w.rot, 0)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ctx.dot_shares(0, qs.op[0], qs.q, ids, db.regions[0], db.capacity, w.n_db, code, mask, ld, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        ctx.dot_shares(0, qs.op[0], qs.q, ids, db.regions[0], db.capacity, w.n_db, code, mask, ld, stream)
        b.record(stream)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    dot_avg_s = float(np.mean([a.elapsed_time(b) for a, b in ev])) / 1e3
    ncmp = w.rows * w.n_db
    ops = ncmp * OPS_PER_CMP_PARTY
    achieved = ops / dot_avg_s / 1e12
    return {
        "metric": "shared iris comparisons/sec on 1 MI355X (bit-exact); p50/p99 query latency",
        "value": ncmp / (total / args.steps), "unit": "comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16", "data": "synthetic",
        "config": {"workload": f"one party's dot products: DB {w.n_db} entries, {w.n_q} queries x {len(w.rot)} "
                               f"rotations ({w.rows} rows)", "rows": w.rows, "db_entries": w.n_db, "parties": 1},
        "roofline": {"bound": "mfma", "kernel": "dot_shares", "achieved": achieved, "peak": MFMA_I8_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / MFMA_I8_PEAK_TOPS, "traffic": None,
                     "ops_per_launch": ops, "avg_launch_ms": dot_avg_s * 1e3},
    }, (w, qc, qm)


def run_batched(args):
    """Uneven batches (sizes 1..64, 1/15/31 rotations) against a party-local
    database: one graph-captured step of batched launches (one dot launch
    per database chunk over all batches' rows) vs per-batch plain launches."""
    import torch

    import paper_2405_04463_amd as imc
    import workload as wl
    from paper_2405_04463_amd.batch import BatchedStep, BatchSet, uneven_batches
    from paper_2405_04463_amd.pipeline import SharedDB

    dealer, party = keys()
    batches = uneven_batches(args.n_batches, seed=0x1A150004)
    nq = sum(b.q for b in batches)
    nrows = sum(b.rows for b in batches)
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=nrows)
    galois = args.scheme == "galois"
    db = SharedDB(ctx, args.n_db, parties=(0,), galois=galois)
    nbytes = imc.galois_db_bytes(args.n_db) if galois else imc.db_bytes(args.n_db)
    log(f"enrolling {args.n_db} entries (party 0, {nbytes / 1e9:.1f} GB, {args.scheme} shares); "
        f"{len(batches)} batches, {nq} queries, {nrows} rows")
    enroll_db(ctx, db, 0x1A150004, args.n_db)
    qc, qm = wl.gen_codes(0x1A150004, 0, nq, query=True)
    bs = BatchSet(ctx, batches, torch.from_numpy(qc.view(np.int64)).cuda(), torch.from_numpy(qm.view(np.int64)).cuda(),
                  galois=galois)
    st = BatchedStep(ctx, bs, db, 0, args.n_db, chunk=args.chunk, parties=(0,))
    if args.batched_mode == "auto":
        mode, best, times = st.autotune(probe_n=16384)
        log(f"autotuned: mode {mode}, dot configuration {best}; probe ms {times}")
    else:
        mode, best = args.batched_mode, args.dot_tiles
        st.mode = mode
        ctx.set_dot_tiles(best)
        log(f"mode {mode}, dot configuration {best} (no autotuning)")
    torch.cuda.empty_cache()
    st.run()
    torch.cuda.synchronize()
    st.capture()
    ncmp = nrows * args.n_db

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k):
            fn()
            torch.cuda.synchronize()
            log(f"  step {i + 1}/{k}: {time.perf_counter() - t0:.2f} s")
        return (time.perf_counter() - t0) / k

    log("batched, graph-captured")
    t_b = timed(st.replay, args.steps)
    ref = st.dot_code[0][:, :min(args.n_db, st.ld)].clone()
    log("plain per-batch launches")
    ctx.set_dot_tiles(imc.DOT_TILES_AUTO)
    t_p = timed(st.run_plain, max(1, args.steps // 2))
    same = bool(torch.equal(ref, st.dot_code[0][:, :ref.shape[1]]))
    return {
        "metric": "shared iris comparisons/sec on 1 MI355X (bit-exact); p50/p99 query latency",
        "value": ncmp / t_b, "unit": "comparisons/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": t_b * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u16", "data": "synthetic",
        "config": {"workload": f"{len(batches)} uneven batches (1..64 queries, 1/15/31 rotations, {nrows} rows) vs "
                               f"party-local DB {args.n_db} entries, dot products only",
                   "chunk": args.chunk, "batched_mode": mode, "dot_config": int(best), "sharing": args.scheme},
        "plain": {"value": ncmp / t_p, "ms_per_step": t_p * 1e3, "same_outputs": same},
        "speedup_vs_plain": t_p / t_b,
    }, (None, None, None)


def run_serve(args):
    """Poisson arrivals into the continuous-batching service (3 parties on one
    GPU, database resident, uniques appended) vs the plain per-query path.
    With --party-local: one party's share of the service (its region of a
    database growing from n_db towards 2,000,000 entries, its dot products),
    the uniqueness decision for appends taken from the workload's planted
    flags (the interactive part needs the other parties' GPUs)."""
    import torch

    import paper_2405_04463_amd as imc
    import workload as wl
    from paper_2405_04463_amd.pipeline import SharedDB
    from paper_2405_04463_amd.serve import Request, Server, plain_check

    dealer, party = keys()
    rot = wl.ROT31
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=args.slots * len(rot))
    galois = args.scheme == "galois"
    local = args.party_local
    cap = max(2_000_000, args.n_db) if local else args.n_db + 20000
    parties = (0,) if local else (0, 1, 2)
    db = SharedDB(ctx, cap, galois=galois, parties=parties)
    nbytes = imc.galois_db_bytes(cap) if galois else imc.db_bytes(cap)
    log(f"enrolling {args.n_db} entries x {len(parties)} part{'y' if local else 'ies'} "
        f"({len(parties) * nbytes / 1e9:.1f} GB reserved, {args.scheme} shares)")
    enroll_db(ctx, db, 0x1A150005, args.n_db)
    db.n = args.n_db
    planted_qids = set()
    rng = np.random.default_rng(5)
    out = {"lambda": {}}
    qid = 0
    for lam in args.rates:
        n_req = max(1, int(lam * args.duration))
        arr = np.cumsum(rng.exponential(1.0 / lam, n_req))
        qc, qm = wl.gen_codes(0x1A150005 + int(lam), qid, n_req, query=True)
        for i in range(n_req):                       # 1% planted near-duplicates
            if rng.random() < 0.01:
                e = int(rng.integers(0, args.n_db))
                ec, em = wl.gen_codes(0x1A150005, e, 1)
                qc[i], qm[i] = wl.plant(0x1A150005, qid + i, ec[0], em[0], int(rng.integers(-15, 16)), h=0.2)
                planted_qids.add(qid + i)
        reqs = [Request(rid=i, qid=qid + i, code=qc[i], mask=qm[i], arrival=float(arr[i])) for i in range(n_req)]
        qid += n_req
        decide = (lambda r: int(r.qid in planted_qids)) if local else None
        srv = Server(ctx, db, rot, chunk=args.chunk, slots=args.slots, decide=decide, serial=not args.no_serial,
                     net=args.net)
        n0 = db.n
        log(f"serving lambda={lam}/s: {n_req} requests over {args.duration:.1f} s, DB {n0} entries")
        t0 = time.perf_counter()
        done = srv.run(reqs, timeout=600)
        wall = time.perf_counter() - t0
        lat = np.array([r.done_at - r.arrival for r in done])
        out["lambda"][str(lam)] = {
            "requests": n_req, "wall_s": wall, "comparisons_per_s": srv.cmps / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "dups": int(sum(r.dup for r in done)), "appended": db.n - n0, "ticks": srv.ticks,
        }
        log(f"  {out['lambda'][str(lam)]}")
        del srv
        torch.cuda.empty_cache()
    # plain per-query path: requests one after another, each a full pass
    cache = {}
    qc, qm = wl.gen_codes(0x1A150006, qid, 4, query=True)
    ts = []
    for i in range(4):
        t0 = time.perf_counter()
        if local:
            plain_local_check(ctx, db, qc[i:i + 1], qm[i:i + 1], qid + i, rot, cache)
        else:
            plain_check(ctx, db, Request(rid=i, qid=qid + i, code=qc[i], mask=qm[i]), rot, cache)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t_plain = float(np.median(ts[1:]))
    out["plain_per_query"] = {"latency_ms": t_plain * 1e3, "comparisons_per_s": len(rot) * db.n / t_plain,
                              "requests_per_s": 1.0 / t_plain}
    best = max(v["comparisons_per_s"] for v in out["lambda"].values())
    top = max(out["lambda"], key=lambda k: out["lambda"][k]["comparisons_per_s"])
    return {
        "metric": "shared iris comparisons/sec on 1 MI355X (bit-exact); p50/p99 query latency",
        "value": best, "unit": "comparisons/s", "n_gpus": 1, "steps": len(args.rates), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": (f"continuous-batching service, party 0's share (its dot products) of a DB of "
                                f"{args.n_db} entries (+ appends, capacity {cap}), appends decided by the planted "
                                f"flags" if local else
                                f"continuous-batching service, 3 parties on one GPU, DB {args.n_db} entries per party "
                                f"(+ appends)") + f", 31 rotations, Poisson arrivals {args.rates}/s for "
                                                  f"{args.duration} s",
                   "chunk": args.chunk, "slots": args.slots, "sharing": args.scheme,
                   "parties": len(parties), "serial_uniqueness": not (args.no_serial or local),
                   "compare_net": None if local else args.net},
        "latency_ms": {"p50": out["lambda"][top]["p50_ms"], "p99": out["lambda"][top]["p99_ms"], "at_lambda": top},
        "serve": out,
    }, (None, None, None)


def plain_local_check(ctx, db, qc, qm, qid, rot, cache):
    """Party 0's plain per-query work: one query's dot products over the whole
    database in one launch (no batching)."""
    import torch

    import paper_2405_04463_amd as imc
    from paper_2405_04463_amd.pipeline import SharedQueries

    n = db.n
    ld = ((n + 63) // 64) * 64
    if cache.get("ld") != ld:
        cache.clear()
        cache["ld"] = ld
        cache["out"] = [torch.empty(len(rot), ld, dtype=torch.int16, device="cuda") for _ in range(2)]
    qs = SharedQueries(ctx, torch.from_numpy(qc.view(np.int64)).cuda(), torch.from_numpy(qm.view(np.int64)).cuda(),
                       qid, galois=db.galois)
    ids = imc.make_ids(qid, rot, 0)
    ctx.dot_shares(0, qs.op[0], 1, ids, db.regions[0], db.capacity, n, cache["out"][0], cache["out"][1], ld,
                   galois=db.galois)


def run_copy_probe(args):
    """A plain device-to-device copy of a known size (calibrates the HBM
    byte counters): 1 GiB read and 1 GiB written per copy."""
    import torch

    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 1 << 30, "copies": 3}), flush=True)


def run_gemm_probe(args):
    """Reference point for the dot kernel's MFMA fraction: the vendor
    library's plain int8 GEMM (torch._int_mm, i8 x i8 -> i32, which ROCm
    serves with hipBLASLt) on one limb product of the dot's shape (M = 1,984
    rows, K = 25,600, N = 300,000 entries, the database operand stored
    entry-major as the library's column-major B) and on square shapes.  One
    rot_dot_kernel launch does six such products (3 limb products x code and
    mask) plus the mod 2^16 fold and the rotations.  Not part of the path."""
    import torch

    out = []
    for m, k, n in ((8192, 8192, 8192), (4096, 16384, 16384), (1984, 25600, 300000)):
        a = torch.randint(-128, 128, (m, k), dtype=torch.int8, device="cuda")
        b = torch.randint(-128, 128, (n, k), dtype=torch.int8, device="cuda").t()
        torch._int_mm(a, b)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            torch._int_mm(a, b)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        t = float(np.median(ts))
        tops = 2 * m * n * k / t / 1e9
        out.append({"m": m, "k": k, "n": n, "ms": t, "tops": tops, "frac": tops / MFMA_I8_PEAK_TOPS})
        log(f"int8 GEMM {m} x {k} x {n}: {t:.2f} ms, {tops:.0f} TOP/s = {tops / MFMA_I8_PEAK_TOPS:.3f} of peak")
        del a, b
        torch.cuda.empty_cache()
    print(json.dumps({"gemm_probe": out, "peak_tops": MFMA_I8_PEAK_TOPS}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["full", "party", "batched", "serve", "compare", "copy-probe",
                                           "gemm-probe"],
                    default="full")
    ap.add_argument("--n-batches", type=int, default=200)
    ap.add_argument("--chunk", type=int, default=65536)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--rates", type=lambda x: [float(v) for v in x.split(",")], default=[50.0, 200.0, 1000.0])
    ap.add_argument("--duration", type=float, default=4.0)
    ap.add_argument("--n-db", type=int, default=None)
    ap.add_argument("--n-q", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve-probe", action="store_true",
                    help="full workload: skip the served-latency probe after the timed steps")
    ap.add_argument("--dot-tiles", type=int, default=0, help="dot kernel tile configuration (IMC_DOT_TILES_*)")
    ap.add_argument("--scheme", choices=["replicated", "galois"], default="replicated",
                    help="sharing of the dot-product operands (full, batched and serve workloads)")
    ap.add_argument("--no-serial", action="store_true",
                    help="serve workload: do not match requests with earlier requests still in flight")
    ap.add_argument("--party-local", action="store_true",
                    help="serve workload: one party's share of the service (its DB region and dot products)")
    ap.add_argument("--compare", choices=["mpclift", "lift18", "plain", "constlift", "nolift"], default="mpclift",
                    help="comparison setting of the full workload (Sec. 6.2)")
    ap.add_argument("--net", choices=["buffers", "registers"], default="buffers",
                    help="comparison messages: through a device buffer with the parties apart (default), or held "
                         "in registers with the three parties of a comparison in one lane")
    ap.add_argument("--batched-mode", choices=["auto", "grouped", "fused", "rows"], default="auto",
                    help="batched workload: the autotuner's choice, or one mode with the --dot-tiles configuration")
    ap.add_argument("--two-eyes", action="store_true",
                    help="full workload as persons of two eyes (queries 2k, 2k+1), with in-batch matching over "
                         "earlier persons and one decision per person")
    ap.add_argument("--in-batch", action="store_true",
                    help="full workload: also match each query against the batch's earlier queries (Sec. 6.4)")
    args = ap.parse_args()
    if args.workload == "copy-probe":
        run_copy_probe(args)
        return
    if args.workload == "gemm-probe":
        run_gemm_probe(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the protocol's three parties are simulated on it "
              "(multi-GPU party transport is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "full":
        args.n_db = args.n_db or 300_000
        args.n_q = args.n_q or 64
        res, (w, qc, qm) = run_full(args)
    elif args.workload == "party":
        args.n_db = args.n_db or 1_000_000
        args.n_q = args.n_q or 32
        res, (w, qc, qm) = run_party(args)
    elif args.workload == "batched":
        args.n_db = args.n_db or 1_000_000
        res, (w, qc, qm) = run_batched(args)
    elif args.workload == "compare":
        args.n_db = args.n_db or 300_000
        args.n_q = args.n_q or 64
        res, (w, qc, qm) = run_compare(args)
    else:
        args.n_db = args.n_db or (1_500_000 if args.party_local else 600_000)
        res, (w, qc, qm) = run_serve(args)
    if not args.no_cpu_baseline and w is not None:
        log("timing the oracle on a bounded sample")
        full = args.workload == "full"
        res["cpu_baseline"] = cpu_baseline(w, qc, qm, galois=full and args.scheme == "galois",
                                           compare=args.compare if full else "mpclift")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
