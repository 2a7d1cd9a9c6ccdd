"""Benchmark: shared iris comparisons per second on one MI355X.

Default workload: the full 3-party protocol (all parties simulated on one
GPU) for 64 queries x 31 rotations (1,984 rows) against a database of
300,000 entries per party, inputs resident in HBM.  One step = every party's
dot products, resharing, the MPCLift comparison, the OR-tree and opening the
per-query result.  `--workload party` times one party's dot products for 32
queries x 31 rotations against 1,000,000 entries instead.

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
HBM_PEAK_GBS = 8000.0
OPS_PER_CMP_PARTY = 2 * 2 * 12800 * 3 * 2   # (code, mask) x K=25,600 x 3 limb products x 2 ops = 307,200


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def keys():
    dealer = hashlib.sha256(b"bench-dealer").digest()
    party = b"".join(hashlib.sha256(b"bench-party%d" % i).digest() for i in range(3))
    return dealer, party


def enroll_db(ctx, db, seed, n, chunk=32768):
    import torch

    import workload as wl

    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        c, k = wl.gen_codes(seed, s, m)
        db.enroll(torch.from_numpy(c.view(np.int64)).cuda(), torch.from_numpy(k.view(np.int64)).cuda(), s)
    torch.cuda.synchronize()


def cpu_baseline(w, qc, qm, sample_q=4, sample_n=8192):
    """The oracle's step (local dots of all parties, reshare, compare, OR-tree)
    on a bounded sample of the same workload; shares made before timing."""
    import oracle as orc
    import workload as wl

    dealer, party = keys()
    dc, dm = wl.gen_codes(w.seed, 0, sample_n)
    qsh = orc.share(dealer, orc.DOM_SHARE_QUERY, qc[:sample_q], qm[:sample_q], 0)
    dsh = orc.share(dealer, orc.DOM_SHARE_DB, dc, dm, 0)
    t0 = time.perf_counter()
    zc, zm = [], []
    for p in range(3):
        c, m = orc.local_dot(p, qsh, w.rot, dsh)
        zc.append(c)
        zm.append(m)
    rc, rm = orc.reshare(party, np.stack(zc), np.stack(zm), sample_q, w.rot, 0, 0)
    match = orc.compare(party, rc, rm, sample_q, w.rot, 0, 0)
    orc.or_tree(party, match, sample_q, len(w.rot), 0)
    dt = time.perf_counter() - t0
    ncmp = sample_q * len(w.rot) * sample_n
    return {"value": ncmp / dt, "unit": "comparisons/s", "cores": orc.threads(), "kind": "oracle",
            "sample": f"oracle step (3 parties' local dots, reshare, compare, OR-tree) on {sample_q} queries x "
                      f"{len(w.rot)} rotations x {sample_n} entries = {ncmp} comparisons, {dt:.1f} s"}


def verify(ctx, buf, w, qc, qm, n_sample=1024):
    """Opened match bits vs the plaintext oracle on every planted entry plus a
    random sample of entries (all rows)."""
    import oracle as orc
    import workload as wl
    from paper_2405_04463_amd.pipeline import open_dup, open_match

    mo, s1 = open_match(ctx, buf, check=1)
    do, s2 = open_dup(ctx, buf, w.n_q, check=1)
    mo = mo.cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(5)
    ents = sorted(set([e for _, e, _, _ in w.planted] + list(rng.choice(w.n_db, n_sample, replace=False))))
    dc = np.empty((len(ents), 200), np.uint64)
    dm = np.empty_like(dc)
    for i, e in enumerate(ents):
        c, m = wl.gen_codes(w.seed, e, 1)
        dc[i], dm[i] = c[0], m[0]
    _, _, match, _ = orc.plain(qc, qm, w.rot, dc, dm)
    got = np.stack([(mo[:, e // 64] >> np.uint64(e % 64)) & np.uint64(1) for e in ents], axis=1).astype(np.uint8)
    ok = bool(np.array_equal(got, match)) and s1 == 0 and s2 == 0
    # every planted query that matches its entry must open dup = 1
    dup = do.cpu().numpy()
    planted_rows = {(qi, e): (match[qi * len(w.rot) + w.rot.index(s), ents.index(e)]) for qi, e, s, _ in w.planted}
    for (qi, e), m in planted_rows.items():
        if m:
            ok = ok and bool(dup[qi] == 1)
    return {"bit_exact": bool(ok), "pairs_checked": int(match.size), "matches_in_sample": int(match.sum()),
            "dup_true": int(dup.sum())}


def run_full(args):
    import torch

    import paper_2405_04463_amd as imc
    import workload as wl
    from paper_2405_04463_amd.pipeline import SharedDB, SharedQueries, alloc_check, open_dup, run_check

    w = wl.full_protocol(n_db=args.n_db, n_q=args.n_q)
    dealer, party = keys()
    ctx = imc.Context(imc.Keys(dealer, party), max_rows=w.rows, dot_tiles=args.dot_tiles)
    log(f"enrolling {w.n_db} entries x 3 parties ({3 * imc.db_bytes(w.n_db) / 1e9:.1f} GB)")
    db = SharedDB(ctx, w.n_db)
    enroll_db(ctx, db, w.seed, w.n_db)
    qc, qm = wl.make_queries(w)
    qs = SharedQueries(ctx, torch.from_numpy(qc.view(np.int64)).cuda(), torch.from_numpy(qm.view(np.int64)).cuda(), 0)
    buf = alloc_check(w.n_q, len(w.rot), w.n_db)
    torch.cuda.synchronize()
    log("first step + verification against the oracle")
    run_check(ctx, qs, w.rot, db, 0, w.n_db, buf)
    torch.cuda.synchronize()
    ver = verify(ctx, buf, w, qc, qm)
    log(f"verification: {ver}")

    stream = torch.cuda.current_stream()
    ids = imc.make_ids(0, w.rot, 0)

    def step(events=None):
        for p in range(3):
            if events is not None:
                events[p][0].record(stream)
            ctx.dot_shares(p, qs.op[p], qs.q, ids, db.regions[p], db.capacity, w.n_db, buf.dot_code[p],
                           buf.dot_mask[p], buf.ld, stream)
            if events is not None:
                events[p][1].record(stream)
        ctx.reshare(buf.dot_code, buf.dot_mask, buf.rows, w.n_db, buf.ld, ids, buf.msg, buf.rep_code, buf.rep_mask,
                    stream)
        ctx.compare_threshold(buf.rep_code, buf.rep_mask, buf.rows, w.n_db, buf.ld, ids, buf.match, buf.nw, stream)
        ctx.or_tree(buf.match, qs.q, buf.nw, buf.nw, ids, buf.ws, buf.ws.numel(), buf.dup, stream)
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
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        step(ev)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        evs.append(ev)
        log(f"step {i + 1}/{args.steps}: {lat[-1] * 1e3:.1f} ms")
    total = time.perf_counter() - t0
    dot_ms = [a.elapsed_time(b) for ev in evs for a, b in ev]
    ncmp = w.rows * w.n_db
    ms = total / args.steps * 1e3
    dot_avg_s = float(np.mean(dot_ms)) / 1e3
    ops = ncmp * OPS_PER_CMP_PARTY
    achieved = ops / dot_avg_s / 1e12
    res = {
        "metric": "shared iris comparisons/sec on 1 MI355X (bit-exact); p50/p99 query latency",
        "value": ncmp / (total / args.steps),
        "unit": "comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16", "data": "synthetic",
        "config": {"workload": f"3-party protocol on one GPU: DB {w.n_db} entries per party, {w.n_q} queries x "
                               f"{len(w.rot)} rotations ({w.rows} rows)",
                   "rows": w.rows, "db_entries": w.n_db, "parties": 3},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                       "note": "one batch of all queries per step; per-query latency = step latency"},
        "roofline": {"bound": "mfma", "kernel": "dot_shares (one party: rotation expand + i8 MFMA dot)",
                     "achieved": achieved, "peak": MFMA_I8_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / MFMA_I8_PEAK_TOPS, "traffic": None,
                     "ops_per_launch": ops, "avg_launch_ms": dot_avg_s * 1e3},
        "verification": ver,
    }
    return res, (w, qc, qm)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["full", "party"], default="full")
    ap.add_argument("--n-db", type=int, default=None)
    ap.add_argument("--n-q", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dot-tiles", type=int, default=0, help="dot kernel tile configuration (IMC_DOT_TILES_*)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the protocol's three parties are simulated on it "
              "(multi-GPU party transport is not part of this build)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "full":
        args.n_db = args.n_db or 300_000
        args.n_q = args.n_q or 64
        res, (w, qc, qm) = run_full(args)
    else:
        args.n_db = args.n_db or 1_000_000
        args.n_q = args.n_q or 32
        res, (w, qc, qm) = run_party(args)
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(w, qc, qm)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
