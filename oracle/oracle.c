/*
 * oracle.c -- plain CPU reference for the secret-shared masked Hamming
 * distance check (3-party replicated sharing over Z_2^16, MPCLift threshold
 * comparison, OR-tree).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU library: every step below is written out from the
 * paper, scalar, one comparison (one bit) at a time, with no blocking,
 * packing or reordering beyond what the definitions state.
 *
 * What is computed (paper sections in brackets):
 *   O1  plaintext decision [Alg. 1, Sec. 3]: for every query rotation and
 *       database entry, ml = |m & M|, hd = |(c ^ C) & m & M|, and
 *       match = hd / ml < MATCH_RATIO with MATCH_RATIO = 3/8, i.e.
 *       8 hd < 3 ml in integers (ml = 0 is no match); dup[q] = OR over all
 *       rotations and entries.
 *   O2  the shared protocol [Alg. 3, Sec. 5; App. C; App. D]:
 *       masked-bit encoding [Sec. 4.1.1], dealer sharing, party-local
 *       dot products [App. C], resharing with zero shares [App. C],
 *       Lift of ml to Z_2^32 [App. D "Lift"], ConstLift of the code dot
 *       [App. D "ConstLift", Sec. 5.1], MSB by BitExtract [App. D, Sec. 5.2],
 *       OR-tree [Sec. 4.2], opening.
 *   O3  the dot product on Shamir shares over the Galois ring
 *       Z_2^16[X]/(X^2 - X - 1) [Sec. 4.3.2]: dealer sharing of packed
 *       bit pairs with degree-1 polynomials at the points 1, X, 1 + X,
 *       Lagrange-premultiplied query shares, constant terms of the ring
 *       products summed into additive shares; resharing, comparison and
 *       OR-tree then run as in O2.
 *   O4  comparison variants [Sec. 4.3 Alg. 2; Sec. 5.1-5.2; Sec. 6.2]:
 *       masks in plain (public ml, MSB over Z_2^16), Lift of ml to Z_2^18
 *       only, and ml computed by a dot product over Z_2^32 (ConstLift;
 *       NoLift when the code dot is also over Z_2^32), with the sharing,
 *       local dot and resharing over Z_2^32 they need.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   - parties are 0-based: party p holds components (x_p, x_{p-1 mod 3})
 *     [App. C], sends to p+1; the paper's parties 1,2,3 are p = 0,1,2 and
 *     its seed_i is key_{i-1}; party p holds key_p and key_{p-1}.
 *   - FA returns (sum, carry); BinAdd is the standard ripple-carry adder
 *     (its printed pseudo-code mislabels the carry), BitExtract feeds the
 *     carry vector shifted up by one bit [App. D].
 *   - AND-gate count of BitExtract with top index m: m gates in the FA layer
 *     (the carry out of bit m is not needed) plus m-1 in the ripple chain
 *     (the shifted carry vector has a public zero at bit 0), i.e. 2m-1;
 *     for an MSB over a k-bit ring this is the paper's 2k-3 [Sec. 4.3.1,
 *     Sec. 5.2].  Lift extracts bits {17,16}: m = 17, 33 gates.
 *   - threshold a/b = 2^14 / 2^16 = 1 - 2*3/8 exactly [Sec. 5]; with masks
 *     in plain the public term is floor(ml / 4): Lemma 1's ceiling is off by
 *     one whenever f ml is not an integer [Sec. 4.3.1].
 *   - the PRF "RNG.Gen" [App. D] is ChaCha with 12 rounds (block function
 *     of Bernstein's ChaCha, state layout as in RFC 8439), addressed by a
 *     64-bit stream id and a 64-bit position; the addressing of every
 *     random value is fixed below so that results never depend on batching.
 *   - OR-tree [Sec. 4.2]: pairwise over 64-bit words of match bits (rotation
 *     major), a public zero word appended at odd levels, then six in-word
 *     halving levels.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_L 12800          /* iris code length in bits [Sec. 3] */
#define ORC_W 200            /* u64 words per packed code */
#define ORC_ROWLEN 800       /* elements per angular row: 200 columns x 4 bits */

/* PRF domains (high byte of the 64-bit stream id). */
#define DOM_SHARE_DB 1u
#define DOM_SHARE_QUERY 2u
#define DOM_RESHARE 3u
#define DOM_CMP 4u
#define DOM_OR 5u
#define DOM_GALOIS_DB 6u
#define DOM_GALOIS_QUERY 7u
#define DOM_OR_PAIRS 8u

/* Circuit layout of one comparison (gate numbers index the PRF tape). */
#define LIFT_M 17            /* Lift extracts bits {17,16}: 33 AND gates */
#define LIFT_W0 0            /* tape words 0..33 */
#define MSB_M 31             /* MSB of the 32-bit comparison ring: 61 AND gates */
#define MSB_W0 40            /* tape words 40..101 */
#define N_GATE_WORDS 102
#define INJ_A_K 15           /* bit 17 is injected into Z_2^15 */
#define INJ_B_K 16           /* bit 16 is injected into Z_2^16 */
/* Per 64-entry group each key has a tape of u64 words (8 per ChaCha block).
 * AND gates of a BitExtract with word base w0: the FA-layer gate of bit i
 * uses word w0 + 2i, the ripple gate producing the carry into bit i+1 uses
 * word w0 + 2i + 1 (so word w0 + 1 is unused).
 *   words   0..33   Lift (w0 = 0)                          blocks 0..4
 *   words  40..101  MSB  (w0 = 40)                         blocks 5..12
 *   BitInject values, bit j of a k-bit value in word base + j:
 *     key_0: c0 of inject A at 104, of inject B at 120     blocks 13..16
 *     key_2: c2, w0, w1 of inject A at 104, 120, 136;
 *            c2, w0, w1 of inject B at 152, 168, 184      blocks 13..24 */
#define TAPE_C0_A 104
#define TAPE_C0_B 120
#define TAPE_C2_A 104
#define TAPE_W0_A 120
#define TAPE_W1_A 136
#define TAPE_C2_B 152
#define TAPE_W0_B 168
#define TAPE_W1_B 184
#define TAPE_WORDS 200       /* 25 ChaCha blocks per key per 64-entry group */
/* Message log of one MPCLift comparison (see ccount): 94 AND gates x 3
 * senders, then the two BitInjects (4 x 15 and 4 x 16 bits): 406 messages,
 * the bits the three parties send (156 + 125 + 125). */
#define MSG_INJ_A (3 * (2 * LIFT_M - 1 + 2 * MSB_M - 1))   /* 282 */
#define MSG_INJ_B (MSG_INJ_A + 4 * INJ_A_K)                   /* 342 */
#define MSG_MPCLIFT (MSG_INJ_B + 4 * INJ_B_K)                 /* 406 */
#define TAPE_BLOCKS_PER_GROUP 32

/* ------------------------------------------------------------------ */
/* ChaCha block function (Bernstein; RFC 8439 state layout).           */
/* ------------------------------------------------------------------ */
static uint32_t rotl32(uint32_t v, int c) { return (v << c) | (v >> (32 - c)); }

static void quarter(uint32_t* x, int a, int b, int c, int d) {
  x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 16);
  x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 12);
  x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 8);
  x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 7);
}

/* key: 32 bytes, read as 8 little-endian words; in: state words 12..15. */
void orc_chacha_block(const uint8_t* key, int rounds, const uint32_t* in, uint32_t* out) {
  uint32_t s[16], x[16];
  s[0] = 0x61707865u; s[1] = 0x3320646eu; s[2] = 0x79622d32u; s[3] = 0x6b206574u;
  for (int i = 0; i < 8; ++i)
    s[4 + i] = (uint32_t)key[4 * i] | ((uint32_t)key[4 * i + 1] << 8) |
               ((uint32_t)key[4 * i + 2] << 16) | ((uint32_t)key[4 * i + 3] << 24);
  for (int i = 0; i < 4; ++i) s[12 + i] = in[i];
  memcpy(x, s, sizeof s);
  for (int r = 0; r < rounds; r += 2) {
    quarter(x, 0, 4, 8, 12); quarter(x, 1, 5, 9, 13);
    quarter(x, 2, 6, 10, 14); quarter(x, 3, 7, 11, 15);
    quarter(x, 0, 5, 10, 15); quarter(x, 1, 6, 11, 12);
    quarter(x, 2, 7, 8, 13); quarter(x, 3, 4, 9, 14);
  }
  for (int i = 0; i < 16; ++i) out[i] = x[i] + s[i];
}

/* The PRF: ChaCha12 with words 12..15 = (pos lo, pos hi, stream lo, stream hi). */
static void prf_block(const uint8_t* key, uint64_t stream, uint64_t pos, uint32_t* out) {
  uint32_t in[4] = {(uint32_t)pos, (uint32_t)(pos >> 32), (uint32_t)stream, (uint32_t)(stream >> 32)};
  orc_chacha_block(key, 12, in, out);
}

/* u16 number i of a stream read as consecutive little-endian u16s. */
static uint16_t prf_u16_at(const uint8_t* key, uint64_t stream, uint64_t i) {
  uint32_t b[16];
  prf_block(key, stream, i >> 5, b);
  uint32_t w = b[(i >> 1) & 15];
  return (uint16_t)((i & 1) ? (w >> 16) : (w & 0xFFFF));
}

/* u64 word t of a stream whose block index is base + t/8. */
static uint64_t prf_u64_at(const uint8_t* key, uint64_t stream, uint64_t base, uint64_t t) {
  uint32_t b[16];
  prf_block(key, stream, base + (t >> 3), b);
  return (uint64_t)b[2 * (t & 7)] | ((uint64_t)b[2 * (t & 7) + 1] << 32);
}

static uint64_t row_stream(uint32_t dom, uint64_t qid, int rot) {
  return ((uint64_t)dom << 56) | ((qid & 0xFFFFFFFFFFFFull) << 8) | (uint64_t)(uint8_t)(rot + 16);
}

/* ------------------------------------------------------------------ */
/* Bits, rotation, O1 plaintext decision [Alg. 1].                     */
/* ------------------------------------------------------------------ */
static int getbit(const uint64_t* v, int i) { return (int)((v[i >> 6] >> (i & 63)) & 1u); }

/* Bit index i = ((row*200 + col)*2 + f)*2 + j.  A rotation by s moves column
 * col to col + s (mod 200) inside its row: rot_s(v)[row][col] = v[row][col - s]. */
static int rot_src(int i, int s) {
  int row = i / ORC_ROWLEN, w = i % ORC_ROWLEN;
  int src = ((w - 4 * s) % ORC_ROWLEN + ORC_ROWLEN) % ORC_ROWLEN;
  return row * ORC_ROWLEN + src;
}

/* O1.  Query row qi*r + ri is query qi at rotation rot[ri].  Outputs are
 * [rows][n]; dup is [nq].  Any output pointer may be NULL. */
void orc_plain(const uint64_t* qc, const uint64_t* qm, int nq, const int* rot, int r,
               const uint64_t* dc, const uint64_t* dm, long n,
               int32_t* hd_out, int32_t* ml_out, uint8_t* match_out, uint8_t* dup_out) {
  long rows = (long)nq * r;
  if (dup_out) memset(dup_out, 0, (size_t)nq);
#pragma omp parallel for schedule(dynamic, 1)
  for (long row = 0; row < rows; ++row) {
    int qi = (int)(row / r), s = rot[row % r];
    uint8_t c[ORC_L], m[ORC_L];
    for (int i = 0; i < ORC_L; ++i) {
      int j = rot_src(i, s);
      c[i] = (uint8_t)getbit(qc + (size_t)qi * ORC_W, j);
      m[i] = (uint8_t)getbit(qm + (size_t)qi * ORC_W, j);
    }
    int any = 0;
    for (long e = 0; e < n; ++e) {
      const uint64_t* C = dc + (size_t)e * ORC_W;
      const uint64_t* M = dm + (size_t)e * ORC_W;
      int ml = 0, hd = 0;
      for (int i = 0; i < ORC_L; ++i) {
        int mm = m[i] & getbit(M, i);               /* m' = m AND M[i] */
        ml += mm;                                    /* ml = CountOnes(m') */
        hd += (c[i] ^ getbit(C, i)) & mm;            /* hd = CountOnes((c XOR C) AND m') */
      }
      int match = (ml > 0) && (8 * hd < 3 * ml);     /* hd/ml < 3/8 */
      size_t o = (size_t)row * n + e;
      if (hd_out) hd_out[o] = hd;
      if (ml_out) ml_out[o] = ml;
      if (match_out) match_out[o] = (uint8_t)match;
      any |= match;
    }
    if (dup_out && any) {
#pragma omp atomic write
      dup_out[qi] = 1;
    }
  }
}

/* ------------------------------------------------------------------ */
/* Encoding and dealer sharing [Sec. 4.1.1, App. B, App. C].           */
/* ------------------------------------------------------------------ */

/* Masked bit a' = m_a - 2 (a AND m_a) in Z_2^16 (T,U,F = -1,0,1). */
static uint16_t masked_bit(int a, int ma) { return (uint16_t)(ma - 2 * (a & ma)); }

void orc_encode(const uint64_t* code, const uint64_t* mask, uint16_t* xc, uint16_t* xm) {
  for (int i = 0; i < ORC_L; ++i) {
    int a = getbit(code, i), ma = getbit(mask, i);
    xc[i] = masked_bit(a, ma);
    xm[i] = (uint16_t)ma;
  }
}

/* Share n vectors: out is [n][vec 2][comp 3][L] u16, vec 0 = code, 1 = mask.
 * comp0, comp1 are dealer-PRF streams, comp2 = x - comp0 - comp1 (mod 2^16).
 * Stream of (vec, comp, id): (dom<<56) | (vec<<52) | (comp<<48) | id. */
void orc_share(const uint8_t* dealer_key, int dom, const uint64_t* codes, const uint64_t* masks,
               long n, uint64_t first_id, uint16_t* out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (long e = 0; e < n; ++e) {
    uint16_t x[2][ORC_L];
    orc_encode(codes + (size_t)e * ORC_W, masks + (size_t)e * ORC_W, x[0], x[1]);
    uint64_t id = (first_id + (uint64_t)e) & 0xFFFFFFFFFFFFull;
    for (int vec = 0; vec < 2; ++vec) {
      uint16_t* o = out + ((size_t)e * 2 + vec) * 3 * ORC_L;
      uint64_t s0 = ((uint64_t)dom << 56) | ((uint64_t)vec << 52) | (0ull << 48) | id;
      uint64_t s1 = ((uint64_t)dom << 56) | ((uint64_t)vec << 52) | (1ull << 48) | id;
      uint32_t b0[16], b1[16];
      for (int i = 0; i < ORC_L; ++i) {
        if ((i & 31) == 0) {   /* one block serves 32 consecutive u16s */
          prf_block(dealer_key, s0, (uint64_t)(i >> 5), b0);
          prf_block(dealer_key, s1, (uint64_t)(i >> 5), b1);
        }
        uint32_t w0 = b0[(i >> 1) & 15], w1 = b1[(i >> 1) & 15];
        uint16_t c0 = (uint16_t)((i & 1) ? (w0 >> 16) : (w0 & 0xFFFF));
        uint16_t c1 = (uint16_t)((i & 1) ? (w1 >> 16) : (w1 & 0xFFFF));
        o[i] = c0;
        o[ORC_L + i] = c1;
        o[2 * ORC_L + i] = (uint16_t)(x[vec][i] - c0 - c1);
      }
    }
  }
}

/* ------------------------------------------------------------------ */
/* Party-local dot product [Alg. 3; App. C].                           */
/* ------------------------------------------------------------------ */

/* Party p's additive share of <x, y> for every query row and entry:
 *   z_p = sum_k x_p y_p + x_{p-1} y_p + x_p y_{p-1}   (mod 2^16)
 * (the ABY3 product without its zero share, which resharing adds).
 * qsh: [nq][2][3][L] comps of the unrotated queries; the query row
 * qi*r + ri uses rotation rot[ri], applied to the party's shares (sharing is
 * elementwise, so rotating shares rotates the secret).
 * dsh: [n][2][3][L].  out_code/out_mask: [rows][n]. */
void orc_local_dot(int p, const uint16_t* qsh, int nq, const int* rot, int r,
                   const uint16_t* dsh, long n, uint16_t* out_code, uint16_t* out_mask) {
  int pm = (p + 2) % 3;
  long rows = (long)nq * r;
#pragma omp parallel for schedule(dynamic, 1)
  for (long row = 0; row < rows; ++row) {
    int qi = (int)(row / r), s = rot[row % r];
    static __thread uint16_t xr[2][2][ORC_L];   /* [vec][own, prev] rotated */
    for (int vec = 0; vec < 2; ++vec) {
      const uint16_t* q = qsh + ((size_t)qi * 2 + vec) * 3 * ORC_L;
      for (int i = 0; i < ORC_L; ++i) {
        int j = rot_src(i, s);
        xr[vec][0][i] = q[p * ORC_L + j];
        xr[vec][1][i] = q[pm * ORC_L + j];
      }
    }
    for (long e = 0; e < n; ++e) {
      for (int vec = 0; vec < 2; ++vec) {
        const uint16_t* d = dsh + ((size_t)e * 2 + vec) * 3 * ORC_L;
        const uint16_t* yp = d + p * ORC_L;
        const uint16_t* ypm = d + pm * ORC_L;
        uint32_t z = 0;
        for (int i = 0; i < ORC_L; ++i)
          z += (uint32_t)xr[vec][0][i] * yp[i] + (uint32_t)xr[vec][1][i] * yp[i] +
               (uint32_t)xr[vec][0][i] * ypm[i];
        uint16_t* o = vec ? out_mask : out_code;
        o[(size_t)row * n + e] = (uint16_t)z;
      }
    }
  }
}

/* ------------------------------------------------------------------ */
/* Resharing [App. C]: z_p + (F(key_p) - F(key_{p-1})), sent to p+1.   */
/* ------------------------------------------------------------------ */

/* z_code/z_mask: [3][rows][n] additive shares (party p's is plane p).
 * out_code/out_mask: [3][rows][n] re-randomised components; party p then
 * holds (out[p], out[p-1]) and out[p] is its message to p+1.
 * Randomness: stream (DOM_RESHARE, qid, rot), position entry>>4, u32 word
 * entry&15; low half for the code, high half for the mask. */
void orc_reshare(const uint8_t* keys, const uint16_t* z_code, const uint16_t* z_mask,
                 int nq, const int* rot, int r, long n, uint64_t qid_base, uint64_t first_entry,
                 uint16_t* out_code, uint16_t* out_mask) {
  long rows = (long)nq * r;
#pragma omp parallel for schedule(dynamic, 1)
  for (long row = 0; row < rows; ++row) {
    uint64_t qid = qid_base + (uint64_t)(row / r);
    uint64_t st = row_stream(DOM_RESHARE, qid, rot[row % r]);
    uint32_t blk[3][16];
    uint64_t have = ~0ull;
    for (long j = 0; j < n; ++j) {
      uint64_t e = first_entry + (uint64_t)j;
      if ((e >> 4) != have) {   /* one block serves 16 consecutive entries */
        for (int k = 0; k < 3; ++k) prf_block(keys + 32 * k, st, e >> 4, blk[k]);
        have = e >> 4;
      }
      uint32_t F[3] = {blk[0][e & 15], blk[1][e & 15], blk[2][e & 15]};
      for (int p = 0; p < 3; ++p) {
        int pm = (p + 2) % 3;
        uint16_t ac = (uint16_t)((F[p] & 0xFFFF) - (F[pm] & 0xFFFF));
        uint16_t am = (uint16_t)((F[p] >> 16) - (F[pm] >> 16));
        size_t o = ((size_t)p * rows + row) * n + j;
        out_code[o] = (uint16_t)(z_code[o] + ac);
        out_mask[o] = (uint16_t)(z_mask[o] + am);
      }
    }
  }
}

/* ------------------------------------------------------------------ */
/* Boolean replicated gates and the sub-protocols of App. D, one bit   */
/* per comparison.  A sharing holds all three components; party p's   */
/* view is (c[p], c[p-1]).                                              */
/* ------------------------------------------------------------------ */
typedef struct { uint8_t c[3]; int depth; } bsh;   /* depth: AND rounds behind this value */

/* Randomness of one comparison: one bit per key per AND gate, and the
 * BitInject values (c0 from key_0; c2, w0, w1 from key_2). */
typedef struct {
  uint8_t g[N_GATE_WORDS][3];   /* indexed by tape word */
  uint32_t c0[2], c2[2], w0[2], w1[2];   /* [0] = inject A (Z_2^15), [1] = inject B (Z_2^16) */
} crand;

/* Communication and gate accounting.  msg (optional) logs every message of
 * one comparison, one bit per message, in the order the protocol sends them:
 * AND gate g (numbered in evaluation order) from party p at msg[3 g + p];
 * then, per BitInject (first the one of the higher bit), the 3OT messages
 * k0 and k1 (party 0 -> 1), w_c (party 2 -> 1) and c1 (party 1 -> 2), k bits
 * each, bit j of k0 at base + j, of k1 at base + k + j, of w_c at
 * base + 2k + j, of c1 at base + 3k + j.  The log changes no arithmetic. */
typedef struct { long and_gates; long bits_sent[3]; uint8_t* msg; } ccount;

static bsh bxor(bsh a, bsh b) {
  bsh z;
  for (int p = 0; p < 3; ++p) z.c[p] = a.c[p] ^ b.c[p];
  z.depth = a.depth > b.depth ? a.depth : b.depth;
  return z;
}
static bsh bsh_zero(void) { bsh z = {{0, 0, 0}, 0}; return z; }

/* ABY3 AND [App. C]: z_p = x_p y_p ^ x_{p-1} y_p ^ x_p y_{p-1} ^ r_p with the
 * zero share r_p = F(key_p) ^ F(key_{p-1}); z_p is sent to party p+1.  g is
 * the gate's number in evaluation order (its messages' place in the log). */
static bsh band(bsh x, bsh y, const uint8_t* f, int g, ccount* cnt) {
  bsh z;
  for (int p = 0; p < 3; ++p) {
    int pm = (p + 2) % 3;
    z.c[p] = (uint8_t)((x.c[p] & y.c[p]) ^ (x.c[pm] & y.c[p]) ^ (x.c[p] & y.c[pm]) ^ f[p] ^ f[pm]);
  }
  z.depth = (x.depth > y.depth ? x.depth : y.depth) + 1;
  if (cnt) {
    cnt->and_gates++;
    for (int p = 0; p < 3; ++p) cnt->bits_sent[p]++;
    if (cnt->msg) for (int p = 0; p < 3; ++p) cnt->msg[3 * g + p] = z.c[p];
  }
  return z;
}

/* FA [App. D]: t1 = a^c, t2 = b^c, s = t1^b, o = t1 t2 ^ c.  Returns s; o via out. */
static bsh full_adder(bsh a, bsh b, bsh c, const uint8_t* f, int g, bsh* carry, ccount* cnt) {
  bsh t1 = bxor(a, c), t2 = bxor(b, c);
  bsh s = bxor(t1, b);
  if (carry) *carry = bxor(band(t1, t2, f, g, cnt), c);
  return s;
}

/* BitExtract [App. D] of bits 0..m of x0 + x1 + x2 (integers, no reduction
 * beyond bit m).  ShareSplit: bit i of component j becomes the trivial
 * sharing InpLocal(x_j[i], j) (component j set, others zero).  FA layer on
 * bits 0..m (carry of bit m unused), then BinAdd((c[m-1..0], 0), s[m..0]).
 * Randomness: the FA-layer gate of bit i (i < m) uses tape word w0 + 2i, the
 * ripple gate producing the carry into bit i+1 (1 <= i < m) word w0 + 2i + 1.
 * Gate numbers (message log order) run bit by bit, a bit's FA-layer gate
 * before its ripple gate: the FA gate of bit i is g0 + 2i - 1 (g0 for
 * i = 0), the ripple gate of bit i is g0 + 2i; 2m - 1 gates in all.
 * Returns r[0..m]. */
static void bit_extract(const uint32_t x[3], int m, int w0, int g0, int d0, const crand* rnd, bsh* r,
                        ccount* cnt) {
  bsh s[33], c[33];
  for (int i = 0; i < 33; ++i) s[i] = c[i] = bsh_zero();
  for (int i = 0; i <= m; ++i) {
    bsh a = bsh_zero(), b = bsh_zero(), cc = bsh_zero();
    a.depth = b.depth = cc.depth = d0;     /* inputs available after d0 rounds */
    a.c[0] = (uint8_t)((x[0] >> i) & 1u);   /* InpLocal(x_1[i], party 1) */
    b.c[1] = (uint8_t)((x[1] >> i) & 1u);   /* InpLocal(x_2[i], party 2) */
    cc.c[2] = (uint8_t)((x[2] >> i) & 1u);  /* InpLocal(x_3[i], party 3) */
    s[i] = full_adder(a, b, cc, rnd->g[w0 + 2 * i], g0 + (i == 0 ? 0 : 2 * i - 1), i < m ? &c[i] : NULL, cnt);
  }
  /* BinAdd: A[0] = 0 (public), A[i] = c[i-1]; B[i] = s[i]. */
  bsh carry = bsh_zero();   /* carry into bit 1 is A[0] AND B[0] = 0 (public) */
  r[0] = s[0];
  for (int i = 1; i <= m; ++i) {
    bsh A = c[i - 1], B = s[i];
    r[i] = bxor(bxor(A, B), carry);
    if (i < m) {
      bsh t1 = bxor(A, carry), t2 = bxor(B, carry);
      carry = bxor(band(t1, t2, rnd->g[w0 + 2 * i + 1], g0 + 2 * i, cnt), carry);
    }
  }
}

/* 3OT [App. D]: sender party 0 holds (m0, m1), receiver party 1 and helper
 * party 2 hold the choice bit ch; pads w0, w1 come from key_2 (held by
 * parties 0 and 2).  Returns m_ch at the receiver. */
static uint32_t three_ot(uint32_t m0, uint32_t m1, int ch, uint32_t w0, uint32_t w1, int k, int mbase,
                         ccount* cnt) {
  uint32_t mask = (k == 32) ? 0xFFFFFFFFu : ((1u << k) - 1u);
  uint32_t k0 = (w0 ^ m0) & mask, k1 = (w1 ^ m1) & mask;   /* party 0 -> party 1 */
  uint32_t wc = (ch ? w1 : w0) & mask;                      /* party 2 -> party 1 */
  if (cnt) {
    cnt->bits_sent[0] += 2 * k;
    cnt->bits_sent[2] += k;
    if (cnt->msg)
      for (int j = 0; j < k; ++j) {
        cnt->msg[mbase + j] = (uint8_t)((k0 >> j) & 1u);
        cnt->msg[mbase + k + j] = (uint8_t)((k1 >> j) & 1u);
        cnt->msg[mbase + 2 * k + j] = (uint8_t)((wc >> j) & 1u);
      }
  }
  return (wc ^ (ch ? k1 : k0)) & mask;
}

/* BitInject [App. D]: [x]_2 -> [x]_{2^k}.  c0 (key_0, parties 0,1) and c2
 * (key_2, parties 0,2) are random; party 0 forms m_t = (t ^ x0 ^ x2) - c0 - c2
 * for t in {0,1}; the 3OT with choice x1 gives party 1 c1 = m_{x1}, which it
 * sends to party 2.  Output components (c0, c1, c2) mod 2^k. */
static void bit_inject(bsh x, int k, uint32_t c0, uint32_t c2, uint32_t w0, uint32_t w1, int mbase,
                       uint32_t out[3], ccount* cnt) {
  uint32_t mask = (k == 32) ? 0xFFFFFFFFu : ((1u << k) - 1u);
  c0 &= mask; c2 &= mask;
  uint32_t m[2];
  for (int t = 0; t < 2; ++t) m[t] = ((uint32_t)(t ^ x.c[0] ^ x.c[2]) - c0 - c2) & mask;
  uint32_t c1 = three_ot(m[0], m[1], x.c[1], w0, w1, k, mbase, cnt);
  if (cnt) {
    cnt->bits_sent[1] += k;   /* party 1 -> party 2 */
    if (cnt->msg)
      for (int j = 0; j < k; ++j) cnt->msg[mbase + 3 * k + j] = (uint8_t)((c1 >> j) & 1u);
  }
  out[0] = c0; out[1] = c1; out[2] = c2;
}

/* One comparison of the MPCLift protocol [Alg. 3, Sec. 5.1, App. D].
 * d[3]: components of the code dot over Z_2^16; x[3]: components of ml over
 * Z_2^16.  Returns the shared match bit = MSB(a [ml'] - ConstLift([dot], b))
 * with a = 2^14, b = 2^16; optional: components of ml' and of y. */
static bsh compare_one(const uint16_t d[3], const uint16_t x[3], const crand* rnd,
                       uint32_t* ml_lift, uint32_t* y_out, ccount* cnt) {
  /* Lift [App. D]: InpLocal each component into Z_2^32 and add. */
  uint32_t S[3] = {x[0], x[1], x[2]};
  bsh r[33];
  bit_extract(S, LIFT_M, LIFT_W0, 0, 0, rnd, r, cnt);
  bsh a = r[17], b = r[16];
  int d_inj = (a.depth > b.depth ? a.depth : b.depth) + 2;   /* 3OT round + c1 forwarding round */
  uint32_t A[3], B[3];
  bit_inject(a, INJ_A_K, rnd->c0[0], rnd->c2[0], rnd->w0[0], rnd->w1[0], MSG_INJ_A, A, cnt);
  bit_inject(b, INJ_B_K, rnd->c0[1], rnd->c2[1], rnd->w0[1], rnd->w1[1], MSG_INJ_B, B, cnt);
  uint32_t ml[3], y[3];
  for (int p = 0; p < 3; ++p) {
    uint32_t a17 = A[p] << 17;        /* ConstLift([a]_{2^15}, 2^17) */
    uint32_t b16 = B[p] << 16;        /* ConstLift([b]_{2^16}, 2^16) */
    ml[p] = S[p] - a17 - b16;         /* [ml]_{2^32} */
    uint32_t hd_lift = (uint32_t)d[p] << 16;   /* ConstLift([dot]_{2^16}, 2^16) = b [dot] */
    y[p] = (ml[p] << 14) - hd_lift;   /* a [ml'] - b [dot'], a = 2^14 */
    if (ml_lift) ml_lift[p] = ml[p];
    if (y_out) y_out[p] = y[p];
  }
  bit_extract(y, MSB_M, MSB_W0, 2 * LIFT_M - 1, d_inj, rnd, r, cnt);
  return r[31];
}

/* Gather one comparison's randomness from its group's tapes.  tape[k] holds
 * TAPE_WORDS u64 words of key k for the comparison's 64-entry group; bit o of
 * a word belongs to the comparison at offset o in the group.  A k-bit value
 * takes its bit j from word (base + j). */
static void gather_rand(const uint64_t tape[3][TAPE_WORDS], int o, crand* rnd) {
  for (int w = 0; w < N_GATE_WORDS; ++w)
    for (int k = 0; k < 3; ++k) rnd->g[w][k] = (uint8_t)((tape[k][w] >> o) & 1u);
  const int kk[2] = {INJ_A_K, INJ_B_K};
  const int bc0[2] = {TAPE_C0_A, TAPE_C0_B}, bc2[2] = {TAPE_C2_A, TAPE_C2_B};
  const int bw0[2] = {TAPE_W0_A, TAPE_W0_B}, bw1[2] = {TAPE_W1_A, TAPE_W1_B};
  for (int v = 0; v < 2; ++v) {
    uint32_t c0 = 0, c2 = 0, w0 = 0, w1 = 0;
    for (int j = 0; j < kk[v]; ++j) {
      c0 |= (uint32_t)((tape[0][bc0[v] + j] >> o) & 1u) << j;
      c2 |= (uint32_t)((tape[2][bc2[v] + j] >> o) & 1u) << j;
      w0 |= (uint32_t)((tape[2][bw0[v] + j] >> o) & 1u) << j;
      w1 |= (uint32_t)((tape[2][bw1[v] + j] >> o) & 1u) << j;
    }
    rnd->c0[v] = c0; rnd->c2[v] = c2; rnd->w0[v] = w0; rnd->w1[v] = w1;
  }
}

/* compare_threshold over rows x n comparisons.
 * d_comp/x_comp: [3][rows][n] components (after resharing) of the code dot
 * and of ml.  match: [3][rows][nw] u64 components of the match bits, bit o of
 * word w = entry column 64w + o; bits at columns >= n are public zeros.
 * Optional (NULL to skip): ml_out [3][rows][n] u32 components of lifted ml;
 * y_out likewise; counts[4] = {AND gates, bits sent by party 0, 1, 2};
 * msg_out [406][rows][nw] u64: every message of every comparison (the log
 * order of ccount), bit o of word w = the comparison at column 64w + o.
 * Randomness: stream (DOM_CMP, qid, rot), group G = entry>>6 at block
 * position G*32 + t/8.  first_entry must be a multiple of 64. */
int orc_compare(const uint8_t* keys, const uint16_t* d_comp, const uint16_t* x_comp,
                int nq, const int* rot, int r, long n, uint64_t qid_base, uint64_t first_entry,
                uint64_t* match, uint32_t* ml_out, uint32_t* y_out, long* counts, uint64_t* msg_out) {
  if (first_entry % 64) return -1;
  long rows = (long)nq * r;
  long nw = (n + 63) / 64;
  long tot_and = 0, tot_bits[3] = {0, 0, 0};
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tot_and)
  for (long row = 0; row < rows; ++row) {
    uint64_t qid = qid_base + (uint64_t)(row / r);
    uint64_t st = row_stream(DOM_CMP, qid, rot[row % r]);
    ccount cnt = {0, {0, 0, 0}, NULL};
    static __thread uint64_t tape[3][TAPE_WORDS];
    for (long w = 0; w < nw; ++w) {
      uint64_t G = (first_entry >> 6) + (uint64_t)w;
      for (int k = 0; k < 3; ++k)
        for (int blk = 0; blk < TAPE_WORDS / 8; ++blk) {
          uint32_t b[16];
          prf_block(keys + 32 * k, st, G * TAPE_BLOCKS_PER_GROUP + (uint64_t)blk, b);
          for (int u = 0; u < 8; ++u)
            tape[k][8 * blk + u] = (uint64_t)b[2 * u] | ((uint64_t)b[2 * u + 1] << 32);
        }
      uint64_t mw[3] = {0, 0, 0};
      for (int o = 0; o < 64; ++o) {
        long j = w * 64 + o;
        if (j >= n) break;
        uint16_t d[3], x[3];
        for (int p = 0; p < 3; ++p) {
          d[p] = d_comp[((size_t)p * rows + row) * n + j];
          x[p] = x_comp[((size_t)p * rows + row) * n + j];
        }
        crand rnd;
        gather_rand(tape, o, &rnd);
        uint32_t mlv[3], yv[3];
        uint8_t msg[MSG_MPCLIFT];
        cnt.msg = msg_out ? msg : NULL;
        bsh mb = compare_one(d, x, &rnd, mlv, yv, &cnt);
        for (int p = 0; p < 3; ++p) {
          mw[p] |= (uint64_t)mb.c[p] << o;
          if (ml_out) ml_out[((size_t)p * rows + row) * n + j] = mlv[p];
          if (y_out) y_out[((size_t)p * rows + row) * n + j] = yv[p];
        }
        if (msg_out)
          for (int m = 0; m < MSG_MPCLIFT; ++m) msg_out[((size_t)m * rows + row) * nw + w] |= (uint64_t)msg[m] << o;
      }
      for (int p = 0; p < 3; ++p) match[((size_t)p * rows + row) * nw + w] = mw[p];
    }
    tot_and += cnt.and_gates;
#pragma omp critical
    { for (int p = 0; p < 3; ++p) tot_bits[p] += cnt.bits_sent[p]; }
  }
  if (counts) { counts[0] = tot_and; counts[1] = tot_bits[0]; counts[2] = tot_bits[1]; counts[3] = tot_bits[2]; }
  return 0;
}

/* ------------------------------------------------------------------ */
/* OR-tree [Sec. 4.2]: x OR y = x ^ y ^ (x AND y), evaluated as a       */
/* binary tree.                                                         */
/* ------------------------------------------------------------------ */

/* Word-wide AND of replicated u64 sharings: the bit gate above applied to
 * all 64 positions of a word; randomness one u64 per key. */
static void wand(const uint64_t x[3], const uint64_t y[3], const uint64_t f[3], uint64_t z[3]) {
  for (int p = 0; p < 3; ++p) {
    int pm = (p + 2) % 3;
    z[p] = (x[p] & y[p]) ^ (x[pm] & y[p]) ^ (x[p] & y[pm]) ^ f[p] ^ f[pm];
  }
}

static void wor(const uint8_t* keys, uint64_t st, int level, uint64_t idx,
                const uint64_t x[3], const uint64_t y[3], uint64_t z[3]) {
  uint64_t f[3], a[3];
  for (int k = 0; k < 3; ++k) f[k] = prf_u64_at(keys + 32 * k, st, (uint64_t)level << 40, idx);
  wand(x, y, f, a);
  for (int p = 0; p < 3; ++p) z[p] = x[p] ^ y[p] ^ a[p];
}

/* match: [3][nq*r][nw] components; per query the words are taken rotation
 * major (ri*nw + w).  Levels 0.. pair words 2i, 2i+1 (a public zero word is
 * appended when a level has odd length); then six in-word levels OR each
 * word with itself shifted right by 32,16,8,4,2,1.  Gate i at level L uses
 * stream (DOM_OR<<56 | qid) position (L<<40) + i/8, word i%8.
 * dup: [3][nq] components (bit 0 of the final word), as 0/1 bytes. */
void orc_or_tree(const uint8_t* keys, const uint64_t* match, int nq, int r, long nw,
                 uint64_t qid_base, uint8_t* dup, long* and_words) {
  long rows = (long)nq * r;
  long tot = 0;
  /* queries are independent trees: one per thread */
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tot)
  for (int qi = 0; qi < nq; ++qi) {
    uint64_t st = ((uint64_t)DOM_OR << 56) | ((qid_base + (uint64_t)qi) & 0xFFFFFFFFFFFFull);
    long len = (long)r * nw;
    uint64_t* cur = (uint64_t*)calloc((size_t)(len + 1) * 3, sizeof(uint64_t));
    for (int ri = 0; ri < r; ++ri)
      for (long w = 0; w < nw; ++w)
        for (int p = 0; p < 3; ++p)
          cur[((size_t)ri * nw + w) * 3 + p] = match[((size_t)p * rows + (size_t)qi * r + ri) * nw + w];
    int level = 0;
    while (len > 1) {
      if (len & 1) { for (int p = 0; p < 3; ++p) cur[(size_t)len * 3 + p] = 0; len++; }
      long half = len / 2;
      for (long i = 0; i < half; ++i) {
        uint64_t z[3];
        wor(keys, st, level, (uint64_t)i, cur + (size_t)(2 * i) * 3, cur + (size_t)(2 * i + 1) * 3, z);
        for (int p = 0; p < 3; ++p) cur[(size_t)i * 3 + p] = z[p];
        tot++;
      }
      len = half;
      level++;
    }
    uint64_t w[3] = {len ? cur[0] : 0, len ? cur[1] : 0, len ? cur[2] : 0};
    for (int sh = 32; sh >= 1; sh /= 2) {
      uint64_t y[3] = {w[0] >> sh, w[1] >> sh, w[2] >> sh}, z[3];
      wor(keys, st, level, 0, w, y, z);
      for (int p = 0; p < 3; ++p) w[p] = z[p];
      tot++;
      level++;
    }
    for (int p = 0; p < 3; ++p) dup[(size_t)p * nq + qi] = (uint8_t)(w[p] & 1u);
    free(cur);
  }
  if (and_words) *and_words = tot;
}

/* ------------------------------------------------------------------ */
/* In-batch matching and combining decisions [Sec. 6.4: the queries of a */
/* batch are also matched with each other; a person's query covers both  */
/* eyes].  Query i of a batch is compared with the queries of earlier     */
/* groups only (a group: one query, or the two eyes of one person): the   */
/* other shared match bits are replaced by public zeros (every component  */
/* cleared).  Two shared decisions are combined with one OR gate,        */
/* x OR y = x ^ y ^ (x AND y).                                            */
/* ------------------------------------------------------------------ */

/* match: [3][q*r][nw] components.  Queries come in groups of `group`
 * consecutive queries (1: every query alone; 2: the two eyes of a person);
 * query qi is compared with the queries of earlier groups only, so bit j of
 * word `word` in every row qi*r + ri survives iff j/group < qi/group. */
void orc_mask_in_batch(uint64_t* match, int q, int r, long nw, long word, int group) {
  long rows = (long)q * r;
  for (int p = 0; p < 3; ++p)
    for (long row = 0; row < rows; ++row) {
      int qi = (int)(row / r);
      for (int j = 0; j < 64; ++j)
        if (j / group >= qi / group) match[((size_t)p * rows + row) * nw + word] &= ~(1ull << j);
    }
}

/* a, b, out: [3][count] bit components (0/1 bytes).  AND randomness of
 * element i: bit i%64 of u64 word i/64 of stream (DOM_OR_PAIRS<<56)|id. */
void orc_or_bits(const uint8_t* keys, const uint8_t* a, const uint8_t* b, long count, uint64_t id, uint8_t* out) {
  uint64_t st = ((uint64_t)DOM_OR_PAIRS << 56) | (id & 0xFFFFFFFFFFFFull);
  for (long i = 0; i < count; ++i) {
    uint8_t f[3];
    for (int k = 0; k < 3; ++k) f[k] = (uint8_t)((prf_u64_at(keys + 32 * k, st, 0, (uint64_t)(i >> 6)) >> (i & 63)) & 1u);
    bsh x, y;
    for (int p = 0; p < 3; ++p) {
      x.c[p] = a[(size_t)p * count + i];
      y.c[p] = b[(size_t)p * count + i];
    }
    x.depth = y.depth = 0;
    bsh z = band(x, y, f, 0, NULL);
    for (int p = 0; p < 3; ++p) out[(size_t)p * count + i] = (uint8_t)(x.c[p] ^ y.c[p] ^ z.c[p]);
  }
}

/* ------------------------------------------------------------------ */
/* Shamir sharing over the Galois ring GR = Z_2^16[X]/(X^2 - X - 1)    */
/* [Sec. 4.3.2, "Optimized 3-party Shamir over Galois Rings" and       */
/* "Iris Membership using Shamir Sharing over Galois Rings"].          */
/*                                                                      */
/* Two consecutive elements of the encoded vector form one ring element */
/* g = x[2i] + x[2i+1] X.  The dealer shares g with a degree-1          */
/* polynomial f(Y) = g + r Y (r uniform in GR) and gives party p the    */
/* evaluation f(alpha_p); the secret sits at Y = 0.  Party p multiplies */
/* its query share by its Lagrange coefficient lambda_p (interpolation  */
/* at 0 from alpha_0..alpha_2); the constant term of lambda_p g_p h_p,  */
/* summed over the packed pairs, is party p's additive share of the     */
/* dot product, because the three products are points of a degree-2     */
/* polynomial whose value at 0 is g h.                                  */
/* ------------------------------------------------------------------ */
typedef struct { uint16_t c0, c1; } gr;   /* c0 + c1 X */

static gr gr_make(uint16_t c0, uint16_t c1) { gr a = {c0, c1}; return a; }
static gr gr_add(gr a, gr b) { return gr_make((uint16_t)(a.c0 + b.c0), (uint16_t)(a.c1 + b.c1)); }
static gr gr_sub(gr a, gr b) { return gr_make((uint16_t)(a.c0 - b.c0), (uint16_t)(a.c1 - b.c1)); }

/* (a0 + a1 X)(b0 + b1 X) = a0 b0 + (a0 b1 + a1 b0) X + a1 b1 X^2, and
 * X^2 = X + 1 in the quotient ring. */
static gr gr_mul(gr a, gr b) {
  uint32_t x0 = (uint32_t)a.c0 * b.c0, x1 = (uint32_t)a.c0 * b.c1 + (uint32_t)a.c1 * b.c0;
  uint32_t x2 = (uint32_t)a.c1 * b.c1;
  return gr_make((uint16_t)(x0 + x2), (uint16_t)(x1 + x2));
}

/* Inverse: (a0 + a1 X)(c0 + c1 X) = 1 is the linear system
 *   a0 c0 + a1 c1 = 1,   a1 c0 + (a0 + a1) c1 = 0,
 * solvable iff its determinant a0 (a0 + a1) - a1^2 is odd (a unit of
 * Z_2^16).  Returns 0 if a is not a unit. */
static int gr_inv(gr a, gr* out) {
  uint16_t det = (uint16_t)((uint32_t)a.c0 * (uint16_t)(a.c0 + a.c1) - (uint32_t)a.c1 * a.c1);
  if (!(det & 1u)) return 0;
  uint16_t y = 1;   /* Newton iteration for 1/det mod 2^16: each step doubles the correct bits */
  for (int it = 0; it < 5; ++it) y = (uint16_t)(y * (uint16_t)(2u - (uint32_t)det * y));
  *out = gr_make((uint16_t)((uint32_t)(uint16_t)(a.c0 + a.c1) * y), (uint16_t)(-(uint32_t)a.c1 * y));
  return 1;
}

/* Evaluation points: an exceptional sequence {0, 1, X, 1 + X} (pairwise
 * differences are units); 0 carries the secret, party p uses alpha_p. */
static gr gr_alpha(int p) {
  return p == 0 ? gr_make(1, 0) : p == 1 ? gr_make(0, 1) : gr_make(1, 1);
}

/* Lagrange coefficient of party p for interpolation at 0 from alpha_0..2:
 * lambda_p = prod_{j != p} alpha_j / (alpha_j - alpha_p). */
static gr gr_lambda(int p) {
  gr l = gr_make(1, 0);
  for (int j = 0; j < 3; ++j) {
    if (j == p) continue;
    gr inv;
    if (!gr_inv(gr_sub(gr_alpha(j), gr_alpha(p)), &inv)) abort();   /* cannot happen: exceptional sequence */
    l = gr_mul(l, gr_mul(gr_alpha(j), inv));
  }
  return l;
}

/* Share n vectors: out is [n][vec 2][party 3][L] u16; party p's share of
 * pair i is (out[2i], out[2i+1]) = g_i + r_i alpha_p.  r_i = (u16 number 2i,
 * u16 number 2i+1) of the dealer stream (dom<<56)|(vec<<52)|id. */
void orc_galois_share(const uint8_t* dealer_key, int dom, const uint64_t* codes, const uint64_t* masks,
                      long n, uint64_t first_id, uint16_t* out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (long e = 0; e < n; ++e) {
    uint16_t x[2][ORC_L];
    orc_encode(codes + (size_t)e * ORC_W, masks + (size_t)e * ORC_W, x[0], x[1]);
    uint64_t id = (first_id + (uint64_t)e) & 0xFFFFFFFFFFFFull;
    for (int vec = 0; vec < 2; ++vec) {
      uint16_t* o = out + ((size_t)e * 2 + vec) * 3 * ORC_L;
      uint64_t st = ((uint64_t)dom << 56) | ((uint64_t)vec << 52) | id;
      uint32_t b[16];
      for (int i = 0; i < ORC_L / 2; ++i) {
        if ((i & 15) == 0) prf_block(dealer_key, st, (uint64_t)(i >> 4), b);   /* 16 pairs per block */
        uint32_t w = b[i & 15];
        gr r = gr_make((uint16_t)(w & 0xFFFF), (uint16_t)(w >> 16));
        gr g = gr_make(x[vec][2 * i], x[vec][2 * i + 1]);
        for (int p = 0; p < 3; ++p) {
          gr sh = gr_add(g, gr_mul(r, gr_alpha(p)));
          o[(size_t)p * ORC_L + 2 * i] = sh.c0;
          o[(size_t)p * ORC_L + 2 * i + 1] = sh.c1;
        }
      }
    }
  }
}

/* Party p's additive share of <x, y> for every query row and entry:
 *   z_p = sum_i const( (lambda_p g_i) h_i )   (mod 2^16)
 * with g_i the party's share of query pair i (after rotating the share
 * vector: rotations move whole 4-element columns, so pairs stay pairs) and
 * h_i its share of the entry's pair i.  qsh: [nq][2][3][L], dsh: [n][2][3][L]
 * as written by orc_galois_share.  out_code/out_mask: [rows][n]. */
void orc_galois_local_dot(int p, const uint16_t* qsh, int nq, const int* rot, int r,
                          const uint16_t* dsh, long n, uint16_t* out_code, uint16_t* out_mask) {
  long rows = (long)nq * r;
  gr lam = gr_lambda(p);
#pragma omp parallel for schedule(dynamic, 1)
  for (long row = 0; row < rows; ++row) {
    int qi = (int)(row / r), s = rot[row % r];
    static __thread gr g[2][ORC_L / 2];   /* lambda_p times the rotated share */
    for (int vec = 0; vec < 2; ++vec) {
      const uint16_t* q = qsh + (((size_t)qi * 2 + vec) * 3 + p) * ORC_L;
      for (int i = 0; i < ORC_L / 2; ++i)
        g[vec][i] = gr_mul(lam, gr_make(q[rot_src(2 * i, s)], q[rot_src(2 * i + 1, s)]));
    }
    for (long e = 0; e < n; ++e) {
      for (int vec = 0; vec < 2; ++vec) {
        const uint16_t* d = dsh + (((size_t)e * 2 + vec) * 3 + p) * ORC_L;
        uint16_t z = 0;
        for (int i = 0; i < ORC_L / 2; ++i) z = (uint16_t)(z + gr_mul(g[vec][i], gr_make(d[2 * i], d[2 * i + 1])).c0);
        uint16_t* o = vec ? out_mask : out_code;
        o[(size_t)row * n + e] = z;
      }
    }
  }
}

/* Test hooks for the ring arithmetic. */
void orc_test_gr_mul(const uint16_t* a, const uint16_t* b, uint16_t* out) {
  gr z = gr_mul(gr_make(a[0], a[1]), gr_make(b[0], b[1]));
  out[0] = z.c0;
  out[1] = z.c1;
}
int orc_test_gr_inv(const uint16_t* a, uint16_t* out) {
  gr z;
  if (!gr_inv(gr_make(a[0], a[1]), &z)) return 0;
  out[0] = z.c0;
  out[1] = z.c1;
  return 1;
}
void orc_galois_points(uint16_t* alpha, uint16_t* lambda) {
  for (int p = 0; p < 3; ++p) {
    gr a = gr_alpha(p), l = gr_lambda(p);
    alpha[2 * p] = a.c0;
    alpha[2 * p + 1] = a.c1;
    lambda[2 * p] = l.c0;
    lambda[2 * p + 1] = l.c1;
  }
}

/* ------------------------------------------------------------------ */
/* Comparison variants [Sec. 4.3 Alg. 2 and Sec. 4.3.1 (masks in       */
/* plain); Sec. 5.1-5.2 (lifting versus a larger dot-product ring); the */
/* comparison benchmark of Sec. 6.2, Table 3].  The threshold 1 - 2*3/8 is 1/4   */
/* exactly, so every variant decides 4 dot > ml (with ml = 0 no match).  */
/*                                                                      */
/*   PLAIN    masks public: ml is a public integer, the code dot stays   */
/*            in Z_2^16 and the bit is MSB_16(floor(ml / 4) - dot),      */
/*            BitExtract with m = 15: 29 AND gates.                      */
/*   LIFT18   masks shared: ml is lifted from Z_2^16 to Z_2^18 (the      */
/*            Lift of App. D with m = 2: bits 17 and 16 injected into    */
/*            Z_2^1 and Z_2^2), the dot is ConstLifted by b = 4 and      */
/*            a = 1; MSB over 18 bits.  33 + 33 AND gates.                */
/*   CONST32  ml is computed over Z_2^32 by a dot product in the larger  */
/*            ring, so only the code dot is lifted (ConstLift by 2^16,   */
/*            free); MSB over 32 bits: 61 AND gates.  The same circuit   */
/*            serves the NoLift setting (code dot also over Z_2^32),     */
/*            since 2^16 dot mod 2^32 depends only on dot mod 2^16.      */
/*                                                                      */
/* Randomness: stream (domain of the variant, qid, rot), the per-group  */
/* tape of MPCLift (32 blocks per 64-entry group), laid out as          */
/*   PLAIN    MSB (m = 15)  words 0..29                                  */
/*   LIFT18   Lift (m = 17) words 0..33, MSB (m = 17) words 40..73,      */
/*            inject A (bit 17 -> Z_2^1): key_0 c0 word 80; key_2 c2 80,  */
/*            w0 81, w1 82; inject B (bit 16 -> Z_2^2): key_0 c0 words    */
/*            88..89; key_2 c2 88..89, w0 90..91, w1 92..93               */
/*   CONST32  MSB (m = 31)  words 0..61                                  */
/* ------------------------------------------------------------------ */
#define CMPV_PLAIN 1
#define CMPV_LIFT18 2
#define CMPV_CONST32 3
#define DOM_CMP_PLAIN 9u
#define DOM_CMP_LIFT18 10u
#define DOM_CMP_CONST32 11u

static uint32_t cmpv_dom(int v) {
  return v == CMPV_PLAIN ? DOM_CMP_PLAIN : v == CMPV_LIFT18 ? DOM_CMP_LIFT18 : DOM_CMP_CONST32;
}

/* Tape blocks per key a variant reads. */
static int cmpv_blocks(int v) { return v == CMPV_PLAIN ? 4 : v == CMPV_LIFT18 ? 12 : 8; }

/* Messages per comparison (the bits the three parties send, in the log
 * order of ccount): MPCLift (v = 0) 406; PLAIN 29 AND gates = 87; LIFT18
 * 33 + 33 AND gates and BitInjects of 1 and 2 bits = 198 + 12; CONST32 61
 * AND gates = 183.  LIFT18 logs its injects after all 66 gates. */
int orc_msg_count(int v) {
  return v == 0 ? MSG_MPCLIFT : v == CMPV_PLAIN ? 87 : v == CMPV_LIFT18 ? 210 : v == CMPV_CONST32 ? 183 : -1;
}

/* One comparison.  d: code-dot components (Z_2^16 for PLAIN and LIFT18;
 * Z_2^16 or Z_2^32 for CONST32); x: ml components (Z_2^16 for LIFT18,
 * Z_2^32 for CONST32; unused for PLAIN); ml_pub: public ml (PLAIN).
 * Returns the shared match bit; y_out: components of the value whose MSB
 * is taken. */
static bsh compare_variant_one(int v, const uint32_t d[3], const uint32_t x[3], uint32_t ml_pub,
                               const crand* rnd, uint32_t* y_out, ccount* cnt) {
  bsh r[33];
  uint32_t y[3];
  if (v == CMPV_PLAIN) {
    /* public minus shared: the constant enters component 0 only */
    uint32_t t = ml_pub / 4u;
    for (int p = 0; p < 3; ++p) y[p] = ((p == 0 ? t : 0u) - d[p]) & 0xFFFFu;
    bit_extract(y, 15, 0, 0, 0, rnd, r, cnt);
    if (y_out) for (int p = 0; p < 3; ++p) y_out[p] = y[p];
    return r[15];
  }
  if (v == CMPV_LIFT18) {
    uint32_t S[3] = {x[0] & 0xFFFFu, x[1] & 0xFFFFu, x[2] & 0xFFFFu};
    bit_extract(S, 17, 0, 0, 0, rnd, r, cnt);
    bsh hi = r[17], lo = r[16];
    int d_inj = (hi.depth > lo.depth ? hi.depth : lo.depth) + 2;
    uint32_t A[3], B[3];
    bit_inject(hi, 1, rnd->c0[0], rnd->c2[0], rnd->w0[0], rnd->w1[0], 3 * 66, A, cnt);
    bit_inject(lo, 2, rnd->c0[1], rnd->c2[1], rnd->w0[1], rnd->w1[1], 3 * 66 + 4, B, cnt);
    for (int p = 0; p < 3; ++p) {
      uint32_t ml = S[p] - (A[p] << 17) - (B[p] << 16);     /* [ml]_{2^18} */
      y[p] = (ml - ((d[p] & 0xFFFFu) << 2)) & 0x3FFFFu;     /* a [ml] - b [dot], a = 1, b = 4 */
    }
    bit_extract(y, 17, 40, 33, d_inj, rnd, r, cnt);
    if (y_out) for (int p = 0; p < 3; ++p) y_out[p] = y[p];
    return r[17];
  }
  for (int p = 0; p < 3; ++p) y[p] = (x[p] << 14) - (d[p] << 16);   /* a = 2^14, b = 2^16 over Z_2^32 */
  bit_extract(y, 31, 0, 0, 0, rnd, r, cnt);
  if (y_out) for (int p = 0; p < 3; ++p) y_out[p] = y[p];
  return r[31];
}

static void gather_rand_variant(int v, const uint64_t tape[3][TAPE_WORDS], int o, crand* rnd) {
  memset(rnd, 0, sizeof(*rnd));
  int words = 8 * cmpv_blocks(v);
  for (int w = 0; w < N_GATE_WORDS && w < words; ++w)
    for (int k = 0; k < 3; ++k) rnd->g[w][k] = (uint8_t)((tape[k][w] >> o) & 1u);
  if (v != CMPV_LIFT18) return;
  const int kk[2] = {1, 2}, bc0[2] = {80, 88}, bc2[2] = {80, 88}, bw0[2] = {81, 90}, bw1[2] = {82, 92};
  for (int i = 0; i < 2; ++i) {
    uint32_t c0 = 0, c2 = 0, w0 = 0, w1 = 0;
    for (int j = 0; j < kk[i]; ++j) {
      c0 |= (uint32_t)((tape[0][bc0[i] + j] >> o) & 1u) << j;
      c2 |= (uint32_t)((tape[2][bc2[i] + j] >> o) & 1u) << j;
      w0 |= (uint32_t)((tape[2][bw0[i] + j] >> o) & 1u) << j;
      w1 |= (uint32_t)((tape[2][bw1[i] + j] >> o) & 1u) << j;
    }
    rnd->c0[i] = c0; rnd->c2[i] = c2; rnd->w0[i] = w0; rnd->w1[i] = w1;
  }
}

/* rows x n comparisons of variant v.  d_comp, x_comp: [3][rows][n] u32
 * components (x_comp unused for PLAIN); ml_pub: [rows][n] public ml (PLAIN
 * only).  match: [3][rows][nw] u64 components as in orc_compare; y_out
 * (optional) [3][rows][n] u32; counts[4] = {AND gates, bits sent by party
 * 0, 1, 2}; msg_out (optional) [orc_msg_count(v)][rows][nw] u64, the
 * message log as in orc_compare.  first_entry must be a multiple of 64. */
int orc_compare_variant(int v, const uint8_t* keys, const uint32_t* d_comp, const uint32_t* x_comp,
                        const int32_t* ml_pub, int nq, const int* rot, int r, long n, uint64_t qid_base,
                        uint64_t first_entry, uint64_t* match, uint32_t* y_out, long* counts,
                        uint64_t* msg_out) {
  if (first_entry % 64) return -1;
  if (v < CMPV_PLAIN || v > CMPV_CONST32) return -2;
  long rows = (long)nq * r;
  long nw = (n + 63) / 64;
  int nblk = cmpv_blocks(v);
  const int nmsg = orc_msg_count(v);
  long tot_and = 0, tot_bits[3] = {0, 0, 0};
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tot_and)
  for (long row = 0; row < rows; ++row) {
    uint64_t qid = qid_base + (uint64_t)(row / r);
    uint64_t st = row_stream(cmpv_dom(v), qid, rot[row % r]);
    ccount cnt = {0, {0, 0, 0}, NULL};
    static __thread uint64_t tape[3][TAPE_WORDS];
    for (long w = 0; w < nw; ++w) {
      uint64_t G = (first_entry >> 6) + (uint64_t)w;
      for (int k = 0; k < 3; ++k)
        for (int blk = 0; blk < nblk; ++blk) {
          uint32_t b[16];
          prf_block(keys + 32 * k, st, G * TAPE_BLOCKS_PER_GROUP + (uint64_t)blk, b);
          for (int u = 0; u < 8; ++u)
            tape[k][8 * blk + u] = (uint64_t)b[2 * u] | ((uint64_t)b[2 * u + 1] << 32);
        }
      uint64_t mw[3] = {0, 0, 0};
      for (int o = 0; o < 64; ++o) {
        long j = w * 64 + o;
        if (j >= n) break;
        uint32_t d[3], x[3] = {0, 0, 0};
        for (int p = 0; p < 3; ++p) {
          size_t idx = ((size_t)p * rows + row) * n + j;
          d[p] = d_comp[idx];
          if (x_comp) x[p] = x_comp[idx];
        }
        uint32_t mlp = ml_pub ? (uint32_t)ml_pub[(size_t)row * n + j] : 0u;
        crand rnd;
        gather_rand_variant(v, tape, o, &rnd);
        uint32_t yv[3];
        uint8_t msg[MSG_MPCLIFT];
        cnt.msg = msg_out ? msg : NULL;
        bsh mb = compare_variant_one(v, d, x, mlp, &rnd, yv, &cnt);
        for (int p = 0; p < 3; ++p) {
          mw[p] |= (uint64_t)mb.c[p] << o;
          if (y_out) y_out[((size_t)p * rows + row) * n + j] = yv[p];
        }
        if (msg_out)
          for (int m = 0; m < nmsg; ++m) msg_out[((size_t)m * rows + row) * nw + w] |= (uint64_t)msg[m] << o;
      }
      for (int p = 0; p < 3; ++p) match[((size_t)p * rows + row) * nw + w] = mw[p];
    }
    tot_and += cnt.and_gates;
#pragma omp critical
    { for (int p = 0; p < 3; ++p) tot_bits[p] += cnt.bits_sent[p]; }
  }
  if (counts) { counts[0] = tot_and; counts[1] = tot_bits[0]; counts[2] = tot_bits[1]; counts[3] = tot_bits[2]; }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Dot products over Z_2^32 [Sec. 5.1, "Lifting vs. Larger             */
/* Dot-Product": computing ml (ConstLift) or both values (NoLift) in    */
/* the larger ring removes the Lift at the price of a wider dot].       */
/* Same steps as the Z_2^16 versions with 32-bit components.            */
/* ------------------------------------------------------------------ */
#define DOM_SHARE32_DB 12u
#define DOM_SHARE32_QUERY 13u
#define DOM_RESHARE32 14u

/* out: [n][vec 2][comp 3][L] u32.  comp0, comp1 are dealer-PRF streams
 * (stream (dom<<56)|(vec<<52)|(comp<<48)|id, one block per 16 elements),
 * comp2 = x - comp0 - comp1 (mod 2^32); x is the masked-bit encoding of the
 * code (vec 0) or the mask bit (vec 1). */
void orc_share32(const uint8_t* dealer_key, int dom, const uint64_t* codes, const uint64_t* masks,
                 long n, uint64_t first_id, uint32_t* out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (long e = 0; e < n; ++e) {
    const uint64_t* code = codes + (size_t)e * ORC_W;
    const uint64_t* mask = masks + (size_t)e * ORC_W;
    uint64_t id = (first_id + (uint64_t)e) & 0xFFFFFFFFFFFFull;
    for (int vec = 0; vec < 2; ++vec) {
      uint32_t* o = out + ((size_t)e * 2 + vec) * 3 * ORC_L;
      uint64_t s0 = ((uint64_t)dom << 56) | ((uint64_t)vec << 52) | (0ull << 48) | id;
      uint64_t s1 = ((uint64_t)dom << 56) | ((uint64_t)vec << 52) | (1ull << 48) | id;
      uint32_t b0[16], b1[16];
      for (int i = 0; i < ORC_L; ++i) {
        if ((i & 15) == 0) {
          prf_block(dealer_key, s0, (uint64_t)(i >> 4), b0);
          prf_block(dealer_key, s1, (uint64_t)(i >> 4), b1);
        }
        int a = getbit(code, i), ma = getbit(mask, i);
        uint32_t x = vec ? (uint32_t)ma : (uint32_t)(ma - 2 * (a & ma));
        uint32_t c0 = b0[i & 15], c1 = b1[i & 15];
        o[i] = c0;
        o[ORC_L + i] = c1;
        o[2 * ORC_L + i] = x - c0 - c1;
      }
    }
  }
}

/* As orc_local_dot over Z_2^32: qsh [nq][2][3][L], dsh [n][2][3][L] u32;
 * out_code/out_mask [rows][n] u32 (either may be NULL to skip). */
void orc_local_dot32(int p, const uint32_t* qsh, int nq, const int* rot, int r,
                     const uint32_t* dsh, long n, uint32_t* out_code, uint32_t* out_mask) {
  int pm = (p + 2) % 3;
  long rows = (long)nq * r;
#pragma omp parallel for schedule(dynamic, 1)
  for (long row = 0; row < rows; ++row) {
    int qi = (int)(row / r), s = rot[row % r];
    static __thread uint32_t xr[2][2][ORC_L];
    for (int vec = 0; vec < 2; ++vec) {
      const uint32_t* q = qsh + ((size_t)qi * 2 + vec) * 3 * ORC_L;
      for (int i = 0; i < ORC_L; ++i) {
        int j = rot_src(i, s);
        xr[vec][0][i] = q[p * ORC_L + j];
        xr[vec][1][i] = q[pm * ORC_L + j];
      }
    }
    for (long e = 0; e < n; ++e)
      for (int vec = 0; vec < 2; ++vec) {
        uint32_t* o = vec ? out_mask : out_code;
        if (!o) continue;
        const uint32_t* d = dsh + ((size_t)e * 2 + vec) * 3 * ORC_L;
        const uint32_t* yp = d + p * ORC_L;
        const uint32_t* ypm = d + pm * ORC_L;
        uint32_t z = 0;
        for (int i = 0; i < ORC_L; ++i)
          z += xr[vec][0][i] * yp[i] + xr[vec][1][i] * yp[i] + xr[vec][0][i] * ypm[i];
        o[(size_t)row * n + e] = z;
      }
  }
}

/* Resharing over Z_2^32: z_p + F(key_p) - F(key_{p-1}).  Randomness: stream
 * (DOM_RESHARE32, qid, rot), position entry>>3, u32 word 2*(entry&7) for the
 * code and 2*(entry&7)+1 for the mask.  z/out: [3][rows][n] u32; a NULL
 * vector is skipped. */
void orc_reshare32(const uint8_t* keys, const uint32_t* z_code, const uint32_t* z_mask,
                   int nq, const int* rot, int r, long n, uint64_t qid_base, uint64_t first_entry,
                   uint32_t* out_code, uint32_t* out_mask) {
  long rows = (long)nq * r;
#pragma omp parallel for schedule(dynamic, 1)
  for (long row = 0; row < rows; ++row) {
    uint64_t qid = qid_base + (uint64_t)(row / r);
    uint64_t st = row_stream(DOM_RESHARE32, qid, rot[row % r]);
    uint32_t blk[3][16];
    uint64_t have = ~0ull;
    for (long j = 0; j < n; ++j) {
      uint64_t e = first_entry + (uint64_t)j;
      if ((e >> 3) != have) {
        for (int k = 0; k < 3; ++k) prf_block(keys + 32 * k, st, e >> 3, blk[k]);
        have = e >> 3;
      }
      for (int p = 0; p < 3; ++p) {
        int pm = (p + 2) % 3;
        size_t o = ((size_t)p * rows + row) * n + j;
        if (z_code) out_code[o] = z_code[o] + blk[p][2 * (e & 7)] - blk[pm][2 * (e & 7)];
        if (z_mask) out_mask[o] = z_mask[o] + blk[p][2 * (e & 7) + 1] - blk[pm][2 * (e & 7) + 1];
      }
    }
  }
}

/* ------------------------------------------------------------------ */
/* Test hooks: the sub-protocols on explicit randomness, for pinning.   */
/* ------------------------------------------------------------------ */

/* Deterministic test randomness (SplitMix64). */
static uint64_t sm64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static void random_crand(uint64_t* s, crand* rnd) {
  for (int w = 0; w < N_GATE_WORDS; ++w)
    for (int k = 0; k < 3; ++k) rnd->g[w][k] = (uint8_t)(sm64(s) & 1u);
  for (int v = 0; v < 2; ++v) {
    rnd->c0[v] = (uint32_t)sm64(s); rnd->c2[v] = (uint32_t)sm64(s);
    rnd->w0[v] = (uint32_t)sm64(s); rnd->w1[v] = (uint32_t)sm64(s);
  }
}

/* BitExtract of x0+x1+x2 (components masked to k bits), bits 0..m.
 * out_bits[i] = opened bit i; out_comp[3*(m+1)] the bit components;
 * returns the AND-gate count. */
long orc_test_bit_extract(int k, int m, uint32_t x0, uint32_t x1, uint32_t x2, uint64_t seed,
                          uint8_t* out_bits, uint8_t* out_comp, int* out_depth) {
  uint32_t mask = (k == 32) ? 0xFFFFFFFFu : ((1u << k) - 1u);
  uint32_t x[3] = {x0 & mask, x1 & mask, x2 & mask};
  crand rnd; uint64_t s = seed; random_crand(&s, &rnd);
  ccount cnt = {0, {0, 0, 0}, NULL};
  bsh r[33];
  bit_extract(x, m, 0, 0, 0, &rnd, r, &cnt);
  for (int i = 0; i <= m; ++i) {
    out_bits[i] = r[i].c[0] ^ r[i].c[1] ^ r[i].c[2];
    if (out_depth) out_depth[i] = r[i].depth;
    if (out_comp) for (int p = 0; p < 3; ++p) out_comp[3 * i + p] = r[i].c[p];
  }
  return cnt.and_gates;
}

/* AND gate on bits given as components. */
void orc_test_and(const uint8_t* x, const uint8_t* y, const uint8_t* f, uint8_t* z) {
  bsh a = bsh_zero(), b = bsh_zero();
  for (int p = 0; p < 3; ++p) { a.c[p] = x[p]; b.c[p] = y[p]; }
  bsh c = band(a, b, f, 0, NULL);
  for (int p = 0; p < 3; ++p) z[p] = c.c[p];
}

/* Full adder on bits given as components; s[3], o[3] components out. */
void orc_test_fa(const uint8_t* a, const uint8_t* b, const uint8_t* c, const uint8_t* f,
                 uint8_t* s, uint8_t* o) {
  bsh A = bsh_zero(), B = bsh_zero(), C = bsh_zero(), O = bsh_zero();
  for (int p = 0; p < 3; ++p) { A.c[p] = a[p]; B.c[p] = b[p]; C.c[p] = c[p]; }
  bsh S = full_adder(A, B, C, f, 0, &O, NULL);
  for (int p = 0; p < 3; ++p) { s[p] = S.c[p]; o[p] = O.c[p]; }
}

/* BitInject of a bit given as components; returns components in Z_2^k and
 * the bits each party sent. */
void orc_test_bit_inject(const uint8_t* x, int k, uint32_t c0, uint32_t c2, uint32_t w0, uint32_t w1,
                         uint32_t* out, long* bits_sent) {
  bsh b = bsh_zero();
  for (int p = 0; p < 3; ++p) b.c[p] = x[p];
  ccount cnt = {0, {0, 0, 0}, NULL};
  bit_inject(b, k, c0, c2, w0, w1, 0, out, &cnt);
  if (bits_sent) for (int p = 0; p < 3; ++p) bits_sent[p] = cnt.bits_sent[p];
}

/* One comparison on explicit components with seeded randomness; returns the
 * opened match bit and (optionally) opened ml' and y, and the gate count. */
int orc_test_compare_one(const uint16_t* d, const uint16_t* x, uint64_t seed,
                         uint32_t* ml_open, uint32_t* y_open, long* counts, int* depth) {
  crand rnd; uint64_t s = seed; random_crand(&s, &rnd);
  ccount cnt = {0, {0, 0, 0}, NULL};
  uint32_t ml[3], y[3];
  bsh mb = compare_one(d, x, &rnd, ml, y, &cnt);
  if (depth) *depth = mb.depth;
  if (ml_open) *ml_open = ml[0] + ml[1] + ml[2];
  if (y_open) *y_open = y[0] + y[1] + y[2];
  if (counts) { counts[0] = cnt.and_gates; for (int p = 0; p < 3; ++p) counts[1 + p] = cnt.bits_sent[p]; }
  return mb.c[0] ^ mb.c[1] ^ mb.c[2];
}

/* One comparison of variant v on explicit components with seeded
 * randomness; returns the opened match bit, optionally the opened value
 * whose MSB is taken (mod the variant's ring), the counts and the depth. */
int orc_test_compare_variant(int v, const uint32_t* d, const uint32_t* x, uint32_t ml_pub, uint64_t seed,
                             uint32_t* y_open, long* counts, int* depth) {
  crand rnd; uint64_t s = seed; random_crand(&s, &rnd);
  ccount cnt = {0, {0, 0, 0}, NULL};
  uint32_t y[3];
  bsh mb = compare_variant_one(v, d, x, ml_pub, &rnd, y, &cnt);
  if (depth) *depth = mb.depth;
  if (y_open) {
    uint32_t ring = v == CMPV_PLAIN ? 0xFFFFu : v == CMPV_LIFT18 ? 0x3FFFFu : 0xFFFFFFFFu;
    *y_open = (y[0] + y[1] + y[2]) & ring;
  }
  if (counts) { counts[0] = cnt.and_gates; for (int p = 0; p < 3; ++p) counts[1 + p] = cnt.bits_sent[p]; }
  return mb.c[0] ^ mb.c[1] ^ mb.c[2];
}

/* Exposed PRF helpers for cross-checks of the stream addressing. */
uint16_t orc_prf_u16(const uint8_t* key, uint64_t stream, uint64_t i) { return prf_u16_at(key, stream, i); }
uint64_t orc_prf_u64(const uint8_t* key, uint64_t stream, uint64_t base, uint64_t t) {
  return prf_u64_at(key, stream, base, t);
}
void orc_prf_block(const uint8_t* key, uint64_t stream, uint64_t pos, uint32_t* out) {
  prf_block(key, stream, pos, out);
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Thread count of later calls (for timing on one core); returns the old one. */
int orc_set_threads(int n) {
#ifdef _OPENMP
  const int old = omp_get_max_threads();
  if (n > 0) omp_set_num_threads(n);
  return old;
#else
  (void)n;
  return 1;
#endif
}
