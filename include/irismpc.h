/*
 * irismpc.h -- C ABI of the MI355X (gfx950) library for the secret-shared
 * masked Hamming-distance uniqueness check of arxiv 2405.04463
 * ("Large-Scale MPC: Scaling Private Iris Code Uniqueness Checks to Millions
 * of Users"), protocol of Alg. 3 (codes and masks shared) in 3-party
 * replicated sharing over Z_2^16 with the MPCLift threshold comparison.
 *
 * All three parties are simulated on one GPU.  Party p (0-based; the paper's
 * parties are 1..3) holds components (x_p, x_{p-1 mod 3}) of every replicated
 * sharing (App. C) and key_p, key_{p-1} of the correlated randomness (App. D).
 * Calls that need an exchange between parties (reshare, compare_threshold,
 * or_tree, open) take all three parties' buffers; what party p sends to
 * party p+1 passes through caller-visible device memory.
 *
 * Conventions
 *   - Every large buffer is caller-owned DEVICE memory on the context's
 *     device; pointers are plain addresses, sizes are element counts.
 *   - Work is enqueued on the caller's stream and is asynchronous, except
 *     where a call says it synchronises.
 *   - Argument errors are reported before anything is enqueued; the library
 *     never throws across this boundary.  A failed launch returns
 *     IMC_EDEVICE; a fault inside a kernel surfaces at the caller's next
 *     synchronisation.
 *   - A context is used by one host thread at a time.  Calls that share a
 *     context's internal scratch (dot_shares, open with check) must not
 *     overlap on different streams.
 *   - Identifiers: query qi of a call has id ids->query_id_base + qi (< 2^48),
 *     result row qi*r + ri is that query at rotation ids->rot[ri]; result
 *     column j is database entry ids->first_entry_id + j.  Every random value
 *     the protocol draws is addressed by (query id, rotation, entry id, gate),
 *     never by batch position, so results do not depend on batching.
 *
 * Code layout: 12,800 bits, bit i in u64 word i>>6 at bit i&63, with
 * i = ((row*200 + col)*2 + f)*2 + j (16 rows x 200 columns x 4 bits).  A
 * rotation by s moves column col to col + s (mod 200) within each row.
 */
#ifndef IRISMPC_H
#define IRISMPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int imc_status;
#define IMC_OK 0
#define IMC_EINVAL (-1)        /* null/misaligned pointer, bad party, rotation or id */
#define IMC_ESHAPE (-2)        /* sizes inconsistent (ld < n, capacity exceeded, rows > max_rows) */
#define IMC_ENOMEM (-3)        /* the context could not allocate its own scratch */
#define IMC_EDEVICE (-4)       /* a HIP call or launch failed */
#define IMC_ECORRUPT (-5)      /* open with check: the two holders of a component disagree */
#define IMC_EUNSUPPORTED (-6)  /* a parameter outside what the library implements */

#define IMC_CODE_BITS 12800
#define IMC_CODE_WORDS 200
#define IMC_MAX_ROT 32         /* rotations per query in one call */
#define IMC_ENTRY_BYTES 102400 /* one party's database bytes per entry */

/* Dot-product kernel configurations (imc_params.flags bits 0-3).  All give
 * identical results; they differ in tiling and in how rotations are formed. */
#define IMC_DOT_TILES_AUTO 0             /* ROTATION when r >= 13, else EXPANDED_256x128 */
#define IMC_DOT_TILES_EXPANDED_256x128 1 /* rotated rows expanded into scratch; 256 x 128 tiles,
                                            8 waves of 64 x 64, global loads 4 K-steps ahead */
#define IMC_DOT_TILES_EXPANDED_128x128 2 /* as 1 with 128 x 128 tiles, 4 waves */
#define IMC_DOT_TILES_EXPANDED_SHALLOW 3 /* as 1 with global loads 3 K-steps ahead */
#define IMC_DOT_TILES_ROTATION 4         /* 256 x 128 tiles; each tile's queries staged unrotated in
                                            LDS per 800-byte segment, rotations read in place
                                            (used when r >= 13, else as AUTO) */
                                         /* 5: not used */
#define IMC_DOT_TILES_ROTATION_LDSCOPY 6 /* as 4 with both operands copied from HBM straight into
                                            LDS (8 database stages, no staging registers);
                                            used when r >= 22, else as AUTO */
#define IMC_DOT_TILES_ROTATION_DIRECT 7  /* as 4 with each wave loading its database fragments
                                            straight into registers (only the query segments
                                            pass through LDS; two barriers per 25 K-steps);
                                            used when r >= 22, else as AUTO */
#define IMC_DOT_TILES_MAX 7
#define IMC_DOT_PERSISTENT 0x10          /* bit 4: expanded tilings and imc_dot_shares_groups run a
                                            persistent grid (one workgroup per CU walking its
                                            XCD's tile sequence) */

/* Stream handle: a hipStream_t (NULL = the default stream). */
typedef struct ihipStream_t* imc_stream;

typedef struct imc_ctx imc_ctx;

typedef struct imc_params {
  uint32_t code_bits;          /* l; must be 12800 (Sec. 3) */
  uint32_t thr_a;              /* threshold a with b = 2^16, 1 - 2*MATCH_RATIO = a/b (Sec. 5);
                                  must be 16384 (MATCH_RATIO = 3/8) */
  uint32_t max_rows;           /* largest q*r any dot_shares call uses (sizes internal scratch) */
  uint32_t flags;              /* bits 0-3: dot-product tile configuration (IMC_DOT_TILES_*);
                                  bit 4: IMC_DOT_PERSISTENT; other bits reserved, must be 0 */
  uint8_t dealer_key[32];      /* key of the input dealer's sharing PRF */
  uint8_t party_key[3][32];    /* key_p of party p; the paper's seed_{p+1} (App. D) */
} imc_params;

/* One result row of a batched dot product: which query operand row to use,
 * at which rotation.  Rows of several uneven batches (different query counts
 * and rotation counts) go through one launch with a table of these. */
typedef struct imc_row {
  uint32_t query_index;        /* row of the query operand (< q; otherwise the row is zero) */
  int32_t rot;                 /* rotation offset in [-15, 15] */
} imc_row;

typedef struct imc_ids {
  uint64_t query_id_base;      /* id of the call's query 0 */
  uint64_t first_entry_id;     /* entry id of result column 0; multiple of 64 */
  int32_t r;                   /* rotations per query, 1..32 */
  int8_t rot[IMC_MAX_ROT];     /* rotation offsets, each in [-15, 15] */
} imc_ids;

/* Create a context on HIP device `device`.  Copies the keys, allocates the
 * internal scratch (rotated query operands for params->max_rows rows, about
 * 102,400 B per row, and a few counters) and, the first time on a device,
 * looks up the device address of the static array that
 * imc_dot_shares_rows_noalloc uses.  Errors: IMC_EINVAL (null),
 * IMC_EUNSUPPORTED (code_bits, thr_a, flags; device index >= 64),
 * IMC_ENOMEM, IMC_EDEVICE. */
imc_status imc_create(const imc_params* params, int device, imc_ctx** out);

/* Release the context and its scratch (synchronises the device).  NULL is a no-op. */
void imc_destroy(imc_ctx* ctx);

/* Static text for a status code. */
const char* imc_strerror(imc_status s);

/* Bytes of one party's database region for `capacity` entries (entries are
 * stored in blocks of 32; see imc_share_db). */
size_t imc_db_bytes(size_t capacity);
/* Bytes of one party's query operand / raw query shares for q queries. */
size_t imc_query_op_bytes(size_t q);
size_t imc_query_raw_bytes(size_t q);
/* Bytes of the OR-tree workspace for q queries with r rotations and nw words per row. */
size_t imc_or_tree_ws_bytes(size_t q, size_t r, size_t nw);

/* Enrolment (Sec. 4.3, "the orb secret shares each bit"; App. C sharing).
 * codes, masks: device u64 [n][200] packed bits of entries first_entry_id ..
 * first_entry_id + n - 1.  Each bit becomes the masked bit c' = m - 2 (c AND m)
 * in Z_2^16 (Sec. 4.1.1) and each mask bit m in Z_2^16; the dealer splits
 * x = x_0 + x_1 + x_2 with x_0, x_1 from its PRF; party p's region db[p]
 * receives (x_p, x_{p-1}) of code and mask for every entry.
 * db[p]: device region of imc_db_bytes(db_capacity) bytes (alignment 256), or
 * NULL for a party whose region is not held on this device (at least one set).
 * Layout: entry e lives in block e/32 at slot e%32; a block is
 * [plane 4][k-chunk 1600][slot 32][16 B] with planes (code lo, code hi,
 * mask lo, mask hi) of the balanced byte limbs v = lo + 256 hi (lo, hi signed
 * bytes), k < 12800 holding x_p and k >= 12800 holding x_{p-1}.
 * Errors: IMC_EINVAL (null, unaligned), IMC_ESHAPE (first+n > capacity). */
imc_status imc_share_db(imc_ctx* ctx, const uint64_t* codes, const uint64_t* masks, size_t n,
                        uint64_t first_entry_id, void* const db[3], size_t db_capacity,
                        imc_stream stream);

/* Query sharing (same dealer sharing, its own PRF domain, keyed by query id).
 * qop[p]: party p's dot-product operand, device i8 [q][plane 4][25600] with
 * k < 12800 holding x_p + x_{p-1} and k >= 12800 holding x_p (the
 * preprocessed share of App. C on the query side), balanced byte limbs.
 * qraw[p] (optional, may be NULL): device u16 [q][vec 2][comp 2][12800],
 * vec 0 code / 1 mask, comp 0 = x_p, comp 1 = x_{p-1}; imc_append_db copies
 * it into a database region. */
imc_status imc_share_query(imc_ctx* ctx, const uint64_t* codes, const uint64_t* masks, size_t q,
                           uint64_t query_id_base, void* const qop[3], void* const qraw[3],
                           imc_stream stream);

/* Party-local dot products (Alg. 3, the two inner products; App. C):
 * for every row (query qi at rotation rot[ri]) and entry e,
 *   code_dot = sum_k (x_p + x_{p-1})_k y_{p,k} + (x_p)_k y_{p-1,k}  mod 2^16
 * over the rotated code shares x and entry shares y, and mask_dot likewise:
 * party p's additive share of <c', C'_e> and of ml before re-randomisation.
 * Rotating shares rotates the secret (sharing is elementwise, Sec. 3).
 * qop: party p's operand from imc_share_query; db: party p's region;
 * code_dot, mask_dot: device u16 [q*ids->r][ld], ld >= n.  mask_dot may be
 * NULL: then only the code dot is computed (the setting with masks in plain,
 * Sec. 4.3 Alg. 2, where ml is public; see imc_plain_ml).
 * Errors: IMC_EINVAL (party, rotation, first_entry_id % 64), IMC_ESHAPE
 * (q*r > max_rows, ld < n, first+n > capacity). */
imc_status imc_dot_shares(imc_ctx* ctx, int party, const void* qop, size_t q, const imc_ids* ids,
                          const void* db, size_t db_capacity, size_t n, uint16_t* code_dot,
                          uint16_t* mask_dot, size_t ld, imc_stream stream);

/* Batched party-local dot products (the same arithmetic as imc_dot_shares)
 * for an arbitrary list of (query, rotation) rows: rows[i] (DEVICE array of
 * nrows imc_row) selects query operand row rows[i].query_index of qop (q
 * rows) at rotation rows[i].rot; output row i of code_dot / mask_dot holds its
 * products with entries first_entry_id .. first_entry_id + n - 1.  Used to
 * run many small uneven batches as one launch over one pass of the database.
 * The rows' rotated operands are expanded into context scratch (nrows <=
 * max_rows).  Errors as imc_dot_shares; first_entry_id % 64 != 0 -> EINVAL. */
imc_status imc_dot_shares_rows(imc_ctx* ctx, int party, const void* qop, size_t q, const imc_row* rows,
                               size_t nrows, const void* db, size_t db_capacity, uint64_t first_entry_id,
                               size_t n, uint16_t* code_dot, uint16_t* mask_dot, size_t ld, imc_stream stream);

/* Largest nrows of imc_dot_shares_rows_noalloc. */
#define IMC_NOALLOC_MAX_ROWS 512

/* For callers that cannot allocate device memory when they call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * imc_dot_shares_rows with the expanded rotated rows kept in a device array
 * that the library holds statically (IMC_NOALLOC_MAX_ROWS rows, 52,428,800 B,
 * on every GPU the library runs on, until the process ends) instead of the
 * context's scratch.  The call allocates nothing; every byte of the array
 * that the dot kernel reads is written by the same call first.  Arguments,
 * results and errors are those of imc_dot_shares_rows, except that nrows is
 * limited by IMC_NOALLOC_MAX_ROWS instead of the context's max_rows (more:
 * IMC_ESHAPE).  All calls on one GPU share that GPU's array: calls that may
 * overlap on one GPU (different streams, host threads or contexts) race and
 * must be serialised by the caller. */
imc_status imc_dot_shares_rows_noalloc(imc_ctx* ctx, int party, const void* qop, size_t q, const imc_row* rows,
                                       size_t nrows, const void* db, size_t db_capacity, uint64_t first_entry_id,
                                       size_t n, uint16_t* code_dot, uint16_t* mask_dot, size_t ld,
                                       imc_stream stream);

/* imc_dot_shares over gathered queries: query i of the call (i < q) is row
 * qidx[i] of qop (qidx: DEVICE array of q u32; rows may repeat or come in any
 * order), every query at the rotations of ids; output row i*r + ri.  Lets a
 * serving loop run the queries of its active slots as one uniform launch
 * (the rotation-aware kernel when ids->r >= 13).  The caller guarantees every
 * qidx[i] is a row of qop.  Errors as imc_dot_shares; null qidx -> EINVAL. */
imc_status imc_dot_shares_gather(imc_ctx* ctx, int party, const void* qop, const uint32_t* qidx, size_t q,
                                 const imc_ids* ids, const void* db, size_t db_capacity, size_t n,
                                 uint16_t* code_dot, uint16_t* mask_dot, size_t ld, imc_stream stream);

/* Query groups of one fused dot launch (imc_dot_shares_groups). */
#define IMC_MAX_DOT_GROUPS 8

typedef struct imc_dot_group {
  const void* qop;             /* the group's unrotated query operand: q rows as written by
                                  imc_share_query (16-byte aligned) */
  uint64_t q;                  /* queries of the group (0: the group is skipped) */
  int32_t r;                   /* rotations per query, 13..32 */
  int8_t rot[IMC_MAX_ROT];     /* rotation offsets, each in [-15, 15] */
  uint16_t* code_dot;          /* device u16 [q*r][ld]: row qi*r + ri, column e - first_entry_id */
  uint16_t* mask_dot;          /* the same for the mask vector; NULL in every group or in none */
} imc_dot_group;

/* imc_dot_shares for several query groups at once (Alg. 3's inner products
 * of uneven batches, Sec. 6.4: many queries per pass over the database):
 * group g's queries at g's rotations against entries first_entry_id ..
 * first_entry_id + n - 1, written to g's outputs, all groups in ONE launch of
 * the rotation-aware kernel (each group keeps its own row tiles; a tile never
 * mixes groups).  With IMC_DOT_PERSISTENT set on the context the launch is a
 * persistent grid (a multiple of 8 workgroups, at most one per CU) walking
 * every group's tiles.  groups: HOST array of n_groups (<= IMC_MAX_DOT_GROUPS)
 * descriptors, read during the call.  The same products as one
 * imc_dot_shares call per group.  Errors: IMC_EINVAL (party, null or
 * unaligned pointers, r outside 13..32, a rotation outside [-15, 15],
 * first_entry_id % 64, mask_dot NULL in some groups only, n_groups >
 * IMC_MAX_DOT_GROUPS), IMC_ESHAPE (ld < n, first+n > capacity, q*r >= 2^31). */
imc_status imc_dot_shares_groups(imc_ctx* ctx, int party, const imc_dot_group* groups, size_t n_groups,
                                 const void* db, size_t db_capacity, uint64_t first_entry_id, size_t n, size_t ld,
                                 imc_stream stream);

/* Select the dot-product configuration of an existing context (same values as
 * imc_params.flags bits 0-4).  Errors: IMC_EUNSUPPORTED. */
imc_status imc_set_dot_tiles(imc_ctx* ctx, uint32_t flags);

/* Resharing of the dot products (App. C: add a zero share, send to the next
 * party).  add_code[p], add_mask[p]: party p's additive shares, u16
 * [rows][ld].  Party p adds F(key_p) - F(key_{p-1}) (ChaCha12 at (query id,
 * rotation, entry)) and sends the result to party p+1: msg[p] is device u16
 * [2][rows][ld] (code, mask).  rep_code[p], rep_mask[p]: device u16
 * [2][rows][ld]: plane 0 = own re-randomised share, plane 1 = the one
 * received from party p-1.  rows must equal q * ids->r for some q.
 * add_mask may be NULL (masks in plain: no mask dot); then only the code
 * shares are reshared, rep_mask is ignored and the mask plane of msg[p] is
 * left untouched.  rep_code may be NULL: then only the messages are written
 * (rep_mask is ignored), and party p's replicated components are msg[p]
 * (its own) and msg[p-1] (the one it received), which
 * imc_compare_threshold_msgs reads in place.  When ld % 8 == 0 every plane
 * must be 16-byte aligned. */
imc_status imc_reshare(imc_ctx* ctx, const uint16_t* const add_code[3], const uint16_t* const add_mask[3],
                       size_t rows, size_t n, size_t ld, const imc_ids* ids, uint16_t* const msg[3],
                       uint16_t* const rep_code[3], uint16_t* const rep_mask[3], imc_stream stream);

/* Threshold comparison, MPCLift variant (Alg. 3, its lift and MSB steps; Sec. 5.1,
 * Sec. 5.2; App. D Lift, BitExtract, BitInject, 3OT, ConstLift):
 *   [ml'] = Lift([ml]_{2^16}) to Z_2^32, y = 2^14 [ml'] - ConstLift([dot], 2^16),
 *   [match] = MSB(y)   (match <=> hd/ml < 3/8 <=> 4 dot > ml).
 * rep_code[p], rep_mask[p]: as produced by imc_reshare ([2][rows][ld]; all
 * 16-byte aligned when ld % 8 == 0).
 * match[p]: device u64 [2][rows][mw_ld] (mw_ld >= ceil(n/64)): plane 0 = party
 * p's own component, plane 1 = component p-1; bit o of word w is column
 * 64w + o; bits at columns >= n are public zeros.  All 3 x 94 AND gates per
 * comparison and both BitInjects run, 64 comparisons bit-sliced per lane.
 * ids->first_entry_id must be a multiple of 64.
 * msg_ws: the network between the parties (Sec. 6.4 keeps it on the GPU):
 * msg_ws_bytes >= imc_compare_msg_bytes(0, rows, n), alignment 8.  Then the
 * three parties run as three waves of a workgroup, each holding its own
 * view only (components p and p-1, keys p and p-1), and every message is
 * stored by its sender into its plane and loaded by its receiver after a
 * workgroup barrier, one barrier per round (50 rounds).  Layout: the match
 * words are numbered t = row * nw + w (nw = ceil(n/64)) and taken 64 at a
 * time; plane m of word t is the u64 at index
 * (floor(t/64) * planes + m) * 64 + t % 64 (planes = 406 here), so the
 * messages of one group of 64 words are contiguous.  Plane order (the
 * oracle's message log): AND gate g
 * (numbered bit by bit, a bit's FA-layer gate before its ripple gate; gates
 * 0..32 the Lift, 33..93 the MSB) sent by party p at plane 3g + p; then
 * the BitInject of bit 17 (Z_2^15) at planes 282.. and of bit 16 (Z_2^16)
 * at 342..: k0, k1 (party 0 -> 1), w_c (party 2 -> 1), c1 (party 1 -> 2),
 * k planes each.  Column bits >= n of a plane are unspecified.  On return
 * the buffer holds every message of the call (406 bits per comparison:
 * 156 sent by party 0, 125 by party 1, 125 by party 2).
 * msg_ws NULL: the same arithmetic with the three parties of a comparison in
 * one lane, messages held in registers (a faster simulation; identical
 * outputs).
 * Errors: IMC_EINVAL (null, unaligned), IMC_ESHAPE (sizes, msg_ws_bytes). */
imc_status imc_compare_threshold(imc_ctx* ctx, const uint16_t* const rep_code[3],
                                 const uint16_t* const rep_mask[3], size_t rows, size_t n, size_t ld,
                                 const imc_ids* ids, void* msg_ws, size_t msg_ws_bytes,
                                 uint64_t* const match[3], size_t mw_ld, imc_stream stream);

/* One query of a reshare or comparison call whose queries are not
 * consecutive: the requests of one serving tick (Sec. 1: sign-ups checked
 * as they arrive against the database of the moment), each with its own id,
 * its own database snapshot and its own match buffer.  A call reads a table
 * of q of these from device memory; the caller owns it and keeps it
 * unchanged until the call has completed on its stream. */
typedef struct imc_query_entry {
  uint64_t query_id;     /* keys the randomness of the query's rows, as ids->query_id_base + i
                            does for query i of imc_reshare / imc_compare_threshold; must be
                            < 2^48 like every query id (the kernels keep its low 48 bits, so a
                            larger id would reuse another query's randomness) */
  uint64_t n;            /* columns of its rows taken part: [0, min(n, call's n)) */
  uint64_t* match[3];    /* imc_compare_threshold_queries: party p's match words of this query's
                            first row in plane 0 (its r rows mw_ld u64 apart), 8-byte aligned;
                            ignored by imc_reshare_queries */
  uint64_t match_plane;  /* u64 from a word of plane 0 to the same word of plane 1
                            (r * mw_ld for a [2][r][mw_ld] buffer of the query alone) */
} imc_query_entry;

/* imc_reshare over the rows of q queries that each carry their own id and
 * column count (table: device, q entries): rows i*r .. i*r + r - 1 of every
 * plane belong to table[i], and the call writes exactly what imc_reshare
 * writes for those rows with query_id_base = table[i].query_id and
 * n = min(table[i].n, n) (columns past that are left untouched).  ids gives
 * r, the rotations and first_entry_id; its query_id_base is ignored.
 * Planes as in imc_reshare, with rows = q * r.  One launch for all q queries.
 * Errors: as imc_reshare, plus IMC_EINVAL for a NULL or unaligned table. */
imc_status imc_reshare_queries(imc_ctx* ctx, const uint16_t* const add_code[3], const uint16_t* const add_mask[3],
                               size_t q, size_t n, size_t ld, const imc_ids* ids, const imc_query_entry* table,
                               uint16_t* const msg[3], uint16_t* const rep_code[3], uint16_t* const rep_mask[3],
                               imc_stream stream);

/* imc_compare_threshold over the rows of q queries that each carry their own
 * id, column count and match buffer (table: device, q entries): query i's
 * rows i*r .. of rep_code / rep_mask are compared exactly as a call of
 * imc_compare_threshold with query_id_base = table[i].query_id,
 * n = min(table[i].n, n) and match = table[i].match would, and its match
 * words are written there, plane 1 at table[i].match_plane words from plane
 * 0 (words past ceil(n_i/64) are left untouched, the last one masked to
 * n_i).  rep_code / rep_mask: [2][q*r][ld] as written by
 * imc_reshare_queries.  msg_ws: NULL (register simulation) or a message
 * buffer holding at least one query's messages,
 * imc_compare_msg_bytes(0, r, n); the call then runs as few launches as the
 * buffer allows, each over as many whole queries as fit in it (every launch
 * reuses the buffer; on return it holds the last launch's messages).
 * Errors: as imc_compare_threshold, plus IMC_EINVAL for a NULL or unaligned
 * table and IMC_ESHAPE for a buffer smaller than one query's messages. */
imc_status imc_compare_threshold_queries(imc_ctx* ctx, const uint16_t* const rep_code[3],
                                         const uint16_t* const rep_mask[3], size_t q, size_t n, size_t ld,
                                         const imc_ids* ids, const imc_query_entry* table, void* msg_ws,
                                         size_t msg_ws_bytes, size_t mw_ld, imc_stream stream);

/* imc_compare_threshold with the replicated components read in place from
 * the resharing's messages (App. C: after the resharing party p holds its
 * own re-randomised share and the one party p-1 sent it): party p's own
 * code and mask dot components are planes 0 and 1 of msgs[p], its second
 * ones planes 0 and 1 of msgs[p-1] (msgs[p]: u16 [2][rows][ld] as
 * imc_reshare writes msg[p]; 16-byte aligned when ld % 8 == 0).  Outputs,
 * msg_ws and errors as imc_compare_threshold; identical match components. */
imc_status imc_compare_threshold_msgs(imc_ctx* ctx, const uint16_t* const msgs[3], size_t rows, size_t n, size_t ld,
                                      const imc_ids* ids, void* msg_ws, size_t msg_ws_bytes,
                                      uint64_t* const match[3], size_t mw_ld, imc_stream stream);

/* Bytes of the message buffer of a comparison call over rows x n
 * comparisons: planes x 64 x ceil(rows * ceil(n/64) / 64) u64, with
 * variant 0 = MPCLift (imc_compare_threshold) 406 planes,
 * IMC_CMP_PLAIN_MASK 87, IMC_CMP_LIFT18 210, IMC_CMP_CONST32 183; 0 for an
 * unknown variant. */
size_t imc_compare_msg_bytes(int variant, size_t rows, size_t n);

/* Other settings of the threshold comparison (Sec. 4.3 Alg. 2 and Sec. 4.3.1;
 * Sec. 5.1-5.2; the settings compared in Sec. 6.2).  The threshold 1 - 2*3/8
 * is 1/4 exactly, so every setting decides match <=> 4 dot > ml.
 *   IMC_CMP_PLAIN_MASK  masks public: ml_pub (device u16 [rows][ld], from
 *                       imc_plain_ml) is a public integer, the code dot is
 *                       shared over Z_2^16; [match] = MSB_16(floor(ml/4) -
 *                       [dot]), 29 AND gates.  rep_mask is ignored.
 *   IMC_CMP_LIFT18      ml shared over Z_2^16 (rep_mask u16 as from
 *                       imc_reshare) and lifted to Z_2^18 only (the Lift of
 *                       App. D with m = 2), the dot ConstLifted by b = 4,
 *                       a = 1: [match] = MSB_18([ml'] - 4 [dot]), 66 AND gates.
 *   IMC_CMP_CONST32     ml shared over Z_2^32 (rep_mask device u32
 *                       [2][rows][ld], from a dot product over Z_2^32), so no
 *                       Lift: [match] = MSB_32(2^14 [ml] - 2^16 [dot]), 61 AND
 *                       gates.  The code dot may be over Z_2^16 (ConstLift)
 *                       or Z_2^32 (code_bits = 32: NoLift); both give the same
 *                       bit, 2^16 dot mod 2^32 depending on dot mod 2^16 only.
 * rep_code[p]: [2][rows][ld] components as from imc_reshare, u16 (code_bits
 * 16) or u32 (code_bits 32, IMC_CMP_CONST32 only).  match[p], ids, the output
 * layout and the first_entry_id alignment are as imc_compare_threshold.  Each
 * setting draws its randomness from its own PRF domain.
 * msg_ws, msg_ws_bytes: as imc_compare_threshold (NULL: messages held in
 * registers), imc_compare_msg_bytes(variant, rows, n) bytes in the same
 * layout with the setting's planes: Plain AND
 * gates 0..28 (87 planes); Lift18 gates 0..32 (Lift) and 33..65 (MSB), then
 * the BitInjects of bit 17 (Z_2^1) at planes 198.. and bit 16 (Z_2^2) at
 * 202.. (210 planes); Const32 gates 0..60 (183 planes).
 * Errors: IMC_EINVAL (null, unaligned, unknown variant, code_bits), IMC_ESHAPE. */
#define IMC_CMP_PLAIN_MASK 1
#define IMC_CMP_LIFT18 2
#define IMC_CMP_CONST32 3
imc_status imc_compare_variant(imc_ctx* ctx, int variant, const void* const rep_code[3], int code_bits,
                               const void* const rep_mask[3], const uint16_t* ml_pub, size_t rows, size_t n,
                               size_t ld, const imc_ids* ids, void* msg_ws, size_t msg_ws_bytes,
                               uint64_t* const match[3], size_t mw_ld, imc_stream stream);

/* Public mask overlap for the setting with masks in plain (Sec. 4.3 Alg. 2:
 * the masks travel in plain, so every party computes ml = |m' AND M| for
 * itself; Sec. 3 for m' and ml).  Two steps:
 * imc_rotate_masks: masks device u64 [q][200] (packed query masks) ->
 *   out device u64 [q*ids->r][200], row qi*r + ri = the mask at rotation
 *   ids->rot[ri].  Errors: IMC_EINVAL (null, unaligned, rotations).
 * imc_plain_ml: row_masks device u64 [rows][200] (rotated query masks),
 *   db_masks device u64 [n][200] (entry masks) -> ml device u16 [rows][ld]
 *   (ld >= n), ml[row][e] = popcount(row_masks[row] AND db_masks[e]).
 *   Errors: IMC_EINVAL (null, unaligned), IMC_ESHAPE (ld < n). */
imc_status imc_rotate_masks(imc_ctx* ctx, const uint64_t* masks, size_t q, const imc_ids* ids, uint64_t* out,
                            imc_stream stream);
imc_status imc_plain_ml(imc_ctx* ctx, const uint64_t* row_masks, size_t rows, const uint64_t* db_masks, size_t n,
                        uint16_t* ml, size_t ld, imc_stream stream);

/* OR-tree (Sec. 4.2; Alg. 3 return): dup[q] = OR over rotations and entries
 * of the shared match bits, as a binary tree of x OR y = x ^ y ^ (x AND y):
 * words 2i, 2i+1 of each level pair up (rotation-major order, a public zero
 * word appended to odd levels), then six in-word levels fold 64 bits to 1.
 * match[p]: [2][q*r][mw_ld] from imc_compare_threshold; nw = words per row.
 * ws: device workspace of imc_or_tree_ws_bytes(q, r, nw) bytes.
 * dup[p]: device u8 [2][q] (0/1), own component then component p-1. */
imc_status imc_or_tree(imc_ctx* ctx, const uint64_t* const match[3], size_t q, size_t nw, size_t mw_ld,
                       const imc_ids* ids, void* ws, size_t ws_bytes, uint8_t* const dup[3],
                       imc_stream stream);

#define IMC_OPEN_U8_XOR 0      /* bits stored one per byte, reconstructed by XOR */
#define IMC_OPEN_U64_XOR 1     /* bit-sliced words, XOR */
#define IMC_OPEN_U16_ADD 2     /* Z_2^16 values, sum */
#define IMC_OPEN_U32_ADD 3     /* Z_2^32 values, sum */

/* Opening: each party sends its own component to the party that lacks it;
 * out = x_0 op x_1 op x_2.  rep[p]: device [2][count] elements of the kind's
 * type (plane 0 own component, plane 1 component p-1); out: device [count].
 * check != 0 additionally compares every component's two holders and
 * SYNCHRONISES the stream; a disagreement returns IMC_ECORRUPT (out is still
 * written). */
imc_status imc_open(imc_ctx* ctx, int kind, const void* const rep[3], size_t count, void* out, int check,
                    imc_stream stream);

/* Append: copy query qi's raw shares (qraw[p] from imc_share_query) into
 * database slot entry_id of every party's region (Sec. 1: a unique query is
 * enrolled); a NULL db[p] skips that party.  Errors: IMC_EINVAL (no region,
 * or a held region without its qraw), IMC_ESHAPE (entry_id >= capacity). */
imc_status imc_append_db(imc_ctx* ctx, const void* const qraw[3], size_t qi, void* const db[3],
                         size_t db_capacity, uint64_t entry_id, imc_stream stream);

/* In-batch matching (Sec. 6.4: the queries of a batch are also matched with
 * each other).  The batch's queries are compared as entries (their raw
 * shares appended to a region with imc_append_db, compared under entry ids
 * distinct from the database's) and query qi may only match the queries of
 * earlier groups, a group being `group` consecutive queries (1: each query
 * alone; 2: a person's two eyes, Sec. 6.4 / Table 4): this call turns the
 * shared match bits of columns j >= group * floor(qi / group) in word `word`
 * of every row qi*r + ri into public zeros (all components of both planes of
 * match[p], [2][q*r][mw_ld], are cleared).  q <= 64 (one word of columns).
 * Errors: IMC_EINVAL (null, unaligned, q > 64, r outside 1..32, group 0),
 * IMC_ESHAPE (word >= mw_ld). */
imc_status imc_mask_in_batch(imc_ctx* ctx, uint64_t* const match[3], size_t q, size_t r, size_t mw_ld, size_t word,
                             size_t group, imc_stream stream);

/* Shared OR of two bit sharings (Sec. 4.2's x OR y = x ^ y ^ (x AND y), one
 * AND gate per element): combines two decisions, e.g. a query's database and
 * in-batch results, or the two eyes of a person.  a[p], b[p], out[p]: device
 * u8 [2][count] (own component, then component p-1; 0/1).  The gate of
 * element i draws bit i%64 of word i/64 of the PRF stream (8 << 56 | id); use
 * a distinct id per combination.  Errors: IMC_EINVAL (null). */
imc_status imc_or_bits(imc_ctx* ctx, const uint8_t* const a[3], const uint8_t* const b[3], size_t count,
                       uint64_t id, uint8_t* const out[3], imc_stream stream);

/* A person's decision from the decisions of its two eyes (Sec. 6.4: a
 * person is a duplicate if either eye is): out element i = in element 2i OR
 * in element 2i+1, one AND gate per person, with the randomness and results
 * of imc_or_bits on a = the even elements, b = the odd ones.  in[p]: device
 * u8 [2][2*count] (own component, then component p-1; 0/1), out[p]: device
 * u8 [2][count].  Errors: IMC_EINVAL (null). */
imc_status imc_or_pairs(imc_ctx* ctx, const uint8_t* const in[3], size_t count, uint64_t id, uint8_t* const out[3],
                        imc_stream stream);

/* ---------------------------------------------------------------------------
 * Galois-ring Shamir form of the dot products (Sec. 4.3.2, "Optimized
 * 3-party Shamir over Galois Rings" and "Iris Membership using Shamir
 * Sharing over Galois Rings").  Two consecutive elements of the encoded
 * vector (masked code bits or mask bits in Z_2^16) form one element
 * g = x_2i + x_2i+1 X of GR = Z_2^16[X]/(X^2 - X - 1); the dealer shares it
 * with a degree-1 polynomial g + r Y and party p (p = 0, 1, 2) holds its value
 * at alpha_p = 1, X, 1 + X.  The query side stores lambda_p times the share,
 * lambda_p being party p's Lagrange coefficient for interpolation at 0, so the
 * constant term of the ring product with the entry's share, summed over the
 * 6,400 pairs, is party p's 3-party additive share of the dot product: the
 * same kind of output as imc_dot_shares, consumed by imc_reshare,
 * imc_compare_threshold and the rest unchanged.  A party stores one share
 * instead of two (51,200 B per entry instead of 102,400) and computes one
 * length-12,800 dot per vector instead of one of length 25,600.
 * Rotations move whole 4-element columns, so pairs stay pairs and rotating a
 * party's share vector rotates the secret.
 * ------------------------------------------------------------------------- */

/* Bytes of one party's Galois-form region for `capacity` entries: blocks of
 * 32 entries [plane 4][k-chunk 800][slot 32][16 B] (planes as in
 * imc_share_db). */
size_t imc_galois_db_bytes(size_t capacity);
/* Bytes of one party's Galois query operand / plain query shares for q queries. */
size_t imc_galois_query_op_bytes(size_t q);
size_t imc_galois_query_raw_bytes(size_t q);

/* Enrolment in the Galois form: entry e's code and mask pairs are shared with
 * dealer randomness r (ChaCha12, its own PRF domain, keyed by entry id) and
 * party p's region db[p] (imc_galois_db_bytes(db_capacity) bytes, alignment
 * 256, or NULL when not held here) receives its share coefficients, element
 * 2i = constant coefficient and 2i+1 = X coefficient of pair i, as balanced
 * byte limbs.  Errors as imc_share_db. */
imc_status imc_galois_share_db(imc_ctx* ctx, const uint64_t* codes, const uint64_t* masks, size_t n,
                               uint64_t first_entry_id, void* const db[3], size_t db_capacity,
                               imc_stream stream);

/* Query sharing in the Galois form.  qop[p]: device i8 [q][plane 4][12800],
 * lambda_p times party p's share (coefficients as above).  qraw[p] (optional):
 * device u16 [q][vec 2][12800], the plain share, for imc_galois_append_db.
 * Errors as imc_share_query. */
imc_status imc_galois_share_query(imc_ctx* ctx, const uint64_t* codes, const uint64_t* masks, size_t q,
                                  uint64_t query_id_base, void* const qop[3], void* const qraw[3],
                                  imc_stream stream);

/* Party-local dot products in the Galois form: for every row (query qi at
 * rotation rot[ri]) and entry e, code_dot = sum_k a_k b_k mod 2^16 over the
 * 12,800 coefficients of party p's premultiplied rotated query share a and
 * entry share b (the constant terms of the ring products), and mask_dot
 * likewise.  Arguments, layouts, tile configurations and errors as
 * imc_dot_shares, with Galois-form operand and region. */
imc_status imc_galois_dot_shares(imc_ctx* ctx, int party, const void* qop, size_t q, const imc_ids* ids,
                                 const void* db, size_t db_capacity, size_t n, uint16_t* code_dot,
                                 uint16_t* mask_dot, size_t ld, imc_stream stream);

/* imc_dot_shares_groups for Galois-form operands and regions. */
imc_status imc_galois_dot_shares_groups(imc_ctx* ctx, int party, const imc_dot_group* groups, size_t n_groups,
                                        const void* db, size_t db_capacity, uint64_t first_entry_id, size_t n,
                                        size_t ld, imc_stream stream);

/* imc_dot_shares_gather for Galois-form operands and regions. */
imc_status imc_galois_dot_shares_gather(imc_ctx* ctx, int party, const void* qop, const uint32_t* qidx, size_t q,
                                        const imc_ids* ids, const void* db, size_t db_capacity, size_t n,
                                        uint16_t* code_dot, uint16_t* mask_dot, size_t ld, imc_stream stream);

/* imc_dot_shares_rows for Galois-form operands and regions. */
imc_status imc_galois_dot_shares_rows(imc_ctx* ctx, int party, const void* qop, size_t q, const imc_row* rows,
                                      size_t nrows, const void* db, size_t db_capacity, uint64_t first_entry_id,
                                      size_t n, uint16_t* code_dot, uint16_t* mask_dot, size_t ld,
                                      imc_stream stream);

/* imc_append_db for Galois-form plain query shares and regions. */
imc_status imc_galois_append_db(imc_ctx* ctx, const void* const qraw[3], size_t qi, void* const db[3],
                                size_t db_capacity, uint64_t entry_id, imc_stream stream);

/* ---------------------------------------------------------------------------
 * Dot products over Z_2^32 (Sec. 5.1, "Lifting vs. Larger Dot-Product"): the
 * ConstLift setting computes ml in the larger ring (no Lift in MPC), NoLift
 * also the code dot; the comparison is then imc_compare_variant with
 * IMC_CMP_CONST32.  One vector (vec 0 = masked code bits, 1 = mask bits) per
 * region and operand.  A Z_2^32 value is stored as four balanced byte limbs
 * v = b0 + 2^8 b1 + 2^16 b2 + 2^24 b3 (b_i signed bytes); a dot product takes
 * the 10 limb products with i + j <= 3 (Sec. 6.1), accumulated exactly in
 * i32 and combined mod 2^32.
 * ------------------------------------------------------------------------- */

/* Bytes of one party's Z_2^32 region of one vector for `capacity` entries
 * (blocks of 32: [limb 4][k-chunk 1600][slot 32][16 B], k < 12800 holding
 * x_p and k >= 12800 holding x_{p-1}; 102,400 B per entry), and of one
 * party's Z_2^32 query operand of one vector for q queries ([q][limb 4][25600],
 * k < 12800 holding x_p + x_{p-1}, k >= 12800 holding x_p). */
size_t imc_db32_bytes(size_t capacity);
size_t imc_query32_op_bytes(size_t q);

/* Dealer sharing over Z_2^32 of vector vec of entries first_entry_id ..
 * first_entry_id + n - 1 (codes, masks: device u64 [n][200]): x_0, x_1 from
 * the dealer's PRF (ChaCha12, its own domain, keyed by vector, component and
 * entry id; one block per 16 elements), x_2 = x - x_0 - x_1.  db[p]: region of
 * imc_db32_bytes(db_capacity) bytes (alignment 256), NULL when not held.
 * Errors: IMC_EINVAL (vec, null, unaligned), IMC_ESHAPE (first+n > capacity). */
imc_status imc_share32_db(imc_ctx* ctx, int vec, const uint64_t* codes, const uint64_t* masks, size_t n,
                          uint64_t first_entry_id, void* const db[3], size_t db_capacity, imc_stream stream);

/* Query sharing over Z_2^32 of vector vec (own PRF domain, keyed by query
 * id): qop[p] receives party p's operand of imc_query32_op_bytes(q) bytes
 * (alignment 16).  Errors: IMC_EINVAL. */
imc_status imc_share32_query(imc_ctx* ctx, int vec, const uint64_t* codes, const uint64_t* masks, size_t q,
                             uint64_t query_id_base, void* const qop[3], imc_stream stream);

/* Party-local dot products over Z_2^32 of one vector: for every row (query
 * qi at rotation rot[ri]) and entry e,
 *   dot = sum_k (x_p + x_{p-1})_k y_{p,k} + (x_p)_k y_{p-1,k}  mod 2^32,
 * party p's additive share (before re-randomisation).  qop, db: party p's
 * operand and region of the same vector; dot: device u32 [q*ids->r][ld].
 * Errors: IMC_EINVAL (party, rotations, first_entry_id % 64, null,
 * unaligned), IMC_ESHAPE (ld < n, first+n > capacity). */
imc_status imc_dot32_shares(imc_ctx* ctx, int party, const void* qop, size_t q, const imc_ids* ids, const void* db,
                            size_t db_capacity, size_t n, uint32_t* dot, size_t ld, imc_stream stream);

/* Resharing over Z_2^32 of one vector (App. C): party p adds F(key_p) -
 * F(key_{p-1}) (ChaCha12 at (query id, rotation), block entry/8, word
 * 2 (entry % 8) + vec) and sends the result to party p+1.  add[p]: u32
 * [rows][ld] additive shares; msg[p]: device u32 [rows][ld] (party p's
 * message); rep[p]: device u32 [2][rows][ld] (own share, the one received
 * from party p-1).  Errors as imc_reshare, IMC_EINVAL for vec. */
imc_status imc_reshare32(imc_ctx* ctx, int vec, const uint32_t* const add[3], size_t rows, size_t n, size_t ld,
                         const imc_ids* ids, uint32_t* const msg[3], uint32_t* const rep[3], imc_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* IRISMPC_H */
