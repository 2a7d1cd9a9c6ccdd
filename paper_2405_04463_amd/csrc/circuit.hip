// circuit.hip -- the interactive part of the protocol, all three parties
// simulated on one GPU: resharing of the dot products (App. C), the MPCLift
// threshold comparison (Sec. 5.1-5.2; App. D Lift, BitExtract, BitInject,
// 3OT, ConstLift), the OR-tree (Sec. 4.2) and opening.
//
// Comparison layout: one lane evaluates 64 comparisons (one row, 64
// consecutive entries) bit-sliced: bit o of every u64 word belongs to entry
// 64w + o.  A replicated boolean sharing is held as its three components
// (party p's view is components p and p-1).  Gates are evaluated in bit
// order, so the lane streams through its ChaCha12 tape one block at a time.
#include "bits.h"
#include "device.h"
#include "launch.h"

namespace imc {

// ---------------------------------------------------------------------------
// Replicated boolean sharing of 64 bits.
// ---------------------------------------------------------------------------
struct B3 {
  uint64_t c[3];
};

__device__ __forceinline__ B3 bx(const B3& a, const B3& b) {
  return B3{{a.c[0] ^ b.c[0], a.c[1] ^ b.c[1], a.c[2] ^ b.c[2]}};
}

// ABY3 AND (App. C): z_p = x_p y_p ^ x_{p-1} y_p ^ x_p y_{p-1} ^ F_p ^ F_{p-1};
// party p sends z_p to party p+1.
__device__ __forceinline__ B3 band(const B3& x, const B3& y, uint64_t f0, uint64_t f1, uint64_t f2) {
  const uint64_t f[3] = {f0, f1, f2};
  B3 z;
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
    z.c[p] = (x.c[p] & y.c[p]) ^ (x.c[pm] & y.c[p]) ^ (x.c[p] & y.c[pm]) ^ f[p] ^ f[pm];
  }
  return z;
}

// Three keys' ChaCha12 blocks of one tape position (8 u64 words each).
struct Blk3 {
  uint32_t w[3][16];
};

__device__ __forceinline__ void gen3(Blk3& b, const Keys3& keys, uint64_t stream, uint64_t pos) {
  const Key* const ks[3] = {&keys.k[0], &keys.k[1], &keys.k[2]};
  const uint64_t st[3] = {stream, stream, stream}, ps[3] = {pos, pos, pos};
  chacha12_n<3>(ks, st, ps, b.w);
}

// ---------------------------------------------------------------------------
// BitExtract streaming step for bit i (inputs y_p = bit i of component p).
// The FA-layer gate of bit i uses tape word w0 + 2i, the ripple gate (carry
// into bit i+1) word w0 + 2i + 1; both sit in block (w0 + 2i) / 8, whose
// words are passed in `b` (u = (w0 + 2i) % 8).  State: c_prev (FA carry of
// bit i-1) and the running carry.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bx_step(const Blk3& b, int u, int i, int m, uint64_t y0, uint64_t y1, uint64_t y2,
                                        B3& c_prev, B3& carry, B3& r) {
  const B3 s{{y0, y1, y2}};                   // t1 ^ b with t1 = (y0,0,y2), b = (0,y1,0)
  B3 c_i{{0, 0, 0}};
  if (i < m) {
    const B3 t1{{y0, 0, y2}}, t2{{0, y1, y2}}, cc{{0, 0, y2}};
    c_i = bx(band(t1, t2, word64(b.w[0], u), word64(b.w[1], u), word64(b.w[2], u)), cc);
  }
  if (i == 0) {
    r = s;
  } else {
    const B3 A = c_prev;
    r = bx(bx(A, s), carry);
    if (i < m)
      carry = bx(band(bx(A, carry), bx(s, carry), word64(b.w[0], u + 1), word64(b.w[1], u + 1),
                      word64(b.w[2], u + 1)),
                 carry);
  }
  c_prev = c_i;
}

// ---------------------------------------------------------------------------
// BitInject (App. D) bit-sliced over k planes: [x]_2 -> [x]_{2^k}.
// Party 0 forms m_t = (t ^ x0 ^ x2) - c0 - c2 (mod 2^k); 3OT: k_t = w_t ^ m_t
// to party 1, w_{x1} from party 2 to party 1, c1 = w_{x1} ^ k_{x1}; party 1
// sends c1 to party 2.  Only the low `keep` planes of the result are
// returned (the comparison uses bit 0 of the Z_2^15 value and bits 0..1 of
// the Z_2^16 value: higher bits vanish under the 2^14 multiplier mod 2^32).
// ---------------------------------------------------------------------------
template <int K, int KEEP>
__device__ __forceinline__ void bit_inject(const Keys3& keys, uint64_t stream, uint64_t base, int c0w, int c2w,
                                           int w0w, int w1w, const B3& x, uint64_t out[3][KEEP]) {
  const uint64_t u = x.c[0] ^ x.c[2];
  uint64_t bA0 = 0, bA1 = 0, bB0 = 0, bB1 = 0;   // borrows of (V - c0) and (. - c2) for t = 0, 1
#pragma unroll
  for (int g = 0; g < (K + 7) / 8; ++g) {          // 8 bits per ChaCha block
    uint32_t blk[4][16];
    const uint64_t dep = bA0 ^ bB1;
    {
      const Key* const ks[4] = {&keys.k[0], &keys.k[2], &keys.k[2], &keys.k[2]};
      const uint64_t st[4] = {stream, stream, stream, stream};
      const uint64_t ps[4] = {after(base + uint64_t(c0w / 8 + g), dep), after(base + uint64_t(c2w / 8 + g), dep),
                              after(base + uint64_t(w0w / 8 + g), dep), after(base + uint64_t(w1w / 8 + g), dep)};
      chacha12_n<4>(ks, st, ps, blk);
    }
    const uint32_t* C0 = blk[0];
    const uint32_t* C2 = blk[1];
    const uint32_t* W0 = blk[2];
    const uint32_t* W1 = blk[3];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int j = 8 * g + jj;
      if (j >= K) break;
      const uint64_t c0 = word64(C0, jj), c2 = word64(C2, jj), w0 = word64(W0, jj), w1 = word64(W1, jj);
      const uint64_t v0 = (j == 0) ? u : 0, v1 = (j == 0) ? ~u : 0;
      // party 0: m_0 = v0 - c0 - c2, m_1 = v1 - c0 - c2 (mod 2^K)
      const uint64_t d0 = v0 ^ c0 ^ bA0;
      bA0 = (~v0 & c0) | (~(v0 ^ c0) & bA0);
      const uint64_t m0 = d0 ^ c2 ^ bB0;
      bB0 = (~d0 & c2) | (~(d0 ^ c2) & bB0);
      const uint64_t d1 = v1 ^ c0 ^ bA1;
      bA1 = (~v1 & c0) | (~(v1 ^ c0) & bA1);
      const uint64_t m1 = d1 ^ c2 ^ bB1;
      bB1 = (~d1 & c2) | (~(d1 ^ c2) & bB1);
      const uint64_t k0 = w0 ^ m0, k1 = w1 ^ m1;            // party 0 -> party 1
      const uint64_t ch = x.c[1];
      const uint64_t wc = (ch & w1) | (~ch & w0);           // party 2 -> party 1
      const uint64_t c1 = wc ^ ((ch & k1) | (~ch & k0));    // party 1, sent to party 2
      if (j < KEEP) {
        out[0][j] = c0;
        out[1][j] = c1;
        out[2][j] = c2;
      }
    }
  }
}

struct CmpArgs {
  Keys3 keys;
  const uint16_t* code[3];   // rep_code[p] plane 0 (party p's own component)
  const uint16_t* mask[3];
  uint64_t* match[3];        // [2][rows][mw_ld]
  const imc_query_entry* tab;  // optional: per-query id, column count and match planes
  uint64_t ld, mw_ld, n, nw, rows, plane_elems, match_plane;
  uint64_t qid_base, first_entry;
  int32_t r;
  int8_t rot[IMC_MAX_ROT_DEV];
};

__global__ void __launch_bounds__(256) compare_kernel(CmpArgs a) {
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.rows * a.nw) return;
  const uint64_t row = t / a.nw, w = t % a.nw;
  const uint64_t col0 = w * 64;
  const uint64_t qi = row / uint64_t(a.r);
  uint64_t qid = a.qid_base + qi, n = a.n;
  if (a.tab) {
    qid = a.tab[qi].query_id;
    n = min<uint64_t>(n, a.tab[qi].n);
    if (col0 >= n) return;
  }
  const int nval = int(min<uint64_t>(64, n - col0));
  const bool vec_ok = (a.ld % 8) == 0;
  const int rot = a.rot[row % uint64_t(a.r)];
  const uint64_t stream = row_stream(kDomCmp, qid, rot);
  const uint64_t base = ((a.first_entry >> 6) + w) * kTapeBlocksPerGroup;

  // ml components -> planes
  uint64_t x[3][16];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    uint32_t W[32];
    load64(a.mask[p] + row * a.ld, col0, nval, vec_ok, W);
    to_planes(W, x[p]);
  }

  // Lift (App. D): bits 16, 17 of S = x0 + x1 + x2 by BitExtract (m = 17),
  // tape words 0..33 (blocks 0..4).
  B3 cprev{{0, 0, 0}}, carry{{0, 0, 0}}, r{{0, 0, 0}}, bit16{{0, 0, 0}}, bit17{{0, 0, 0}};
#pragma unroll
  for (int blk = 0; blk < 5; ++blk) {
    Blk3 b;
    gen3(b, a.keys, stream, after(base + blk, carry.c[0] ^ cprev.c[1]));
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int i = 4 * blk + ii;
      const uint64_t y0 = i < 16 ? x[0][i] : 0, y1 = i < 16 ? x[1][i] : 0, y2 = i < 16 ? x[2][i] : 0;
      if (i > 17) break;
      bx_step(b, 2 * ii, i, 17, y0, y1, y2, cprev, carry, r);
      if (i == 16) bit16 = r;
      if (i == 17) bit17 = r;   // bit 17 has no gates (its carry out is not needed)
    }
  }

  // BitInject bit 17 into Z_2^15 and bit 16 into Z_2^16 (tape blocks 13..24).
  uint64_t A[3][1], B[3][2];
  bit_inject<15, 1>(a.keys, stream, base, 104, 104, 120, 136, bit17, A);
  bit_inject<16, 2>(a.keys, stream, base, 120, 152, 168, 184, bit16, B);

  // y_p = 2^14 (x_p - 2^17 A_p - 2^16 B_p) - 2^16 d_p  (mod 2^32):
  // bits 0..13 zero, bits 14,15 = x_p bits 0,1, bits 16..31 =
  // U_p = (x_p >> 2) - d_p - (B_p mod 4) 2^14 - (A_p mod 2) 2^15  (mod 2^16).
  // The ml planes were consumed by the Lift; reload them with the dot planes.
  uint64_t U[3][16], xlo[3][2];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    uint32_t W[32];
    uint64_t xm[16], d[16];
    load64(a.mask[p] + row * a.ld, col0, nval, vec_ok, W);
    to_planes(W, xm);
    load64(a.code[p] + row * a.ld, col0, nval, vec_ok, W);
    to_planes(W, d);
    xlo[p][0] = xm[0];
    xlo[p][1] = xm[1];
    uint64_t br = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint64_t X = j < 14 ? xm[j + 2] : 0;
      U[p][j] = X ^ d[j] ^ br;
      br = (~X & d[j]) | (~(X ^ d[j]) & br);
    }
    const uint64_t u14 = U[p][14];
    U[p][14] = u14 ^ B[p][0];
    const uint64_t b2 = ~u14 & B[p][0];
    U[p][15] = U[p][15] ^ B[p][1] ^ b2 ^ A[p][0];
  }

  // MSB of y by BitExtract (m = 31), tape words 40..101 (blocks 5..12).
  cprev = B3{{0, 0, 0}};
  carry = B3{{0, 0, 0}};
#pragma unroll
  for (int blk = 0; blk < 8; ++blk) {
    Blk3 b;
    gen3(b, a.keys, stream, after(base + 5 + blk, carry.c[0] ^ cprev.c[1]));
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int i = 4 * blk + ii;
      uint64_t y0 = 0, y1 = 0, y2 = 0;
      if (i == 14 || i == 15) { y0 = xlo[0][i - 14]; y1 = xlo[1][i - 14]; y2 = xlo[2][i - 14]; }
      if (i >= 16) { y0 = U[0][i - 16]; y1 = U[1][i - 16]; y2 = U[2][i - 16]; }
      bx_step(b, 2 * ii, i, 31, y0, y1, y2, cprev, carry, r);
    }
  }

  const uint64_t keep = nval == 64 ? ~0ull : ((1ull << nval) - 1ull);
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
    uint64_t* m = a.tab ? a.tab[qi].match[p] + (row % uint64_t(a.r)) * a.mw_ld : a.match[p] + row * a.mw_ld;
    const uint64_t plane = a.tab ? a.tab[qi].match_plane : a.match_plane;
    m[w] = r.c[p] & keep;
    m[plane + w] = r.c[pm] & keep;
  }
}

// ---------------------------------------------------------------------------
// Comparison variants (Sec. 4.3 Alg. 2 and Sec. 4.3.1: masks in plain;
// Sec. 5.1-5.2: lifting versus a dot product in the larger ring; the
// settings of the comparison benchmark, Sec. 6.2).  The threshold 1 - 2*3/8
// is 1/4 exactly; every variant decides 4 dot > ml.
//
//   kCmpPlain    ml public (u16 per comparison), code dot over Z_2^16:
//                MSB_16(floor(ml/4) - dot), BitExtract m = 15 on tape
//                words 0..29 (blocks 0..3): 29 AND gates.
//   kCmpLift18   ml shared over Z_2^16 and lifted to Z_2^18 (bits 17 and
//                16 of x0 + x1 + x2 by BitExtract m = 17 on words 0..33,
//                injected into Z_2^1 and Z_2^2); y = ml - 4 dot over Z_2^18,
//                MSB by BitExtract m = 17 on words 40..73 (blocks 5..9).
//                Inject values: key_0 c0 word 80 (A), words 88..89 (B);
//                key_2 c2 80, w0 81, w1 82 (A), c2 88..89, w0 90..91,
//                w1 92..93 (B) -- blocks 10 and 11.  66 AND gates.
//   kCmpConst32  ml shared over Z_2^32 (a dot product in the larger ring),
//                the code dot over Z_2^16 or Z_2^32: y = 2^14 ml - 2^16 dot
//                over Z_2^32, MSB by BitExtract m = 31 on words 0..61
//                (blocks 0..7): 61 AND gates.
// ---------------------------------------------------------------------------
constexpr int kCmpPlain = 1, kCmpLift18 = 2, kCmpConst32 = 3;

struct CmpVArgs {
  Keys3 keys;
  const void* code[3];        // rep_code[p] plane 0: u16, or u32 when code32
  const void* mask[3];        // rep_mask[p] plane 0: u16 (Lift18) or u32 (Const32)
  const uint16_t* ml_pub;     // [rows][ld] public ml (Plain)
  uint64_t* match[3];         // [2][rows][mw_ld]
  uint64_t ld, mw_ld, n, nw, rows, match_plane;
  uint64_t qid_base, first_entry;
  int32_t r;
  int32_t vec;                // 16-byte loads allowed (ld % 8 == 0, 16-byte aligned rows)
  int8_t rot[IMC_MAX_ROT_DEV];
};

// BitExtract over bits 0..M of y0 + y1 + y2 given as NB planes per component
// (higher planes are zero); FA gate of bit i on tape word W0 + 2i, ripple
// gate on W0 + 2i + 1 (W0 a multiple of 8).  Returns the sharing of bit M.
template <int M, int W0, int NB>
__device__ __forceinline__ B3 bit_extract_msb(const Keys3& keys, uint64_t stream, uint64_t base,
                                              const uint64_t (&y)[3][NB]) {
  static_assert(W0 % 8 == 0, "gate words start a block");
  B3 cprev{{0, 0, 0}}, carry{{0, 0, 0}}, r{{0, 0, 0}};
#pragma unroll
  for (int blk = 0; blk < (M + 4) / 4; ++blk) {
    Blk3 b;
    gen3(b, keys, stream, after(base + W0 / 8 + blk, carry.c[0] ^ cprev.c[1]));
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int i = 4 * blk + ii;
      if (i > M) break;
      const uint64_t y0 = i < NB ? y[0][i] : 0, y1 = i < NB ? y[1][i] : 0, y2 = i < NB ? y[2][i] : 0;
      bx_step(b, 2 * ii, i, M, y0, y1, y2, cprev, carry, r);
    }
  }
  return r;
}

// BitInject of x into Z_2^K from tape words given per bit (see bit_inject).
template <int K>
__device__ __forceinline__ void inject_words(const B3& x, const uint64_t (&c0)[K], const uint64_t (&c2)[K],
                                             const uint64_t (&w0)[K], const uint64_t (&w1)[K], uint64_t out[3][K]) {
  const uint64_t u = x.c[0] ^ x.c[2], ch = x.c[1];
  uint64_t bA0 = 0, bA1 = 0, bB0 = 0, bB1 = 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint64_t v0 = (j == 0) ? u : 0, v1 = (j == 0) ? ~u : 0;
    const uint64_t d0 = v0 ^ c0[j] ^ bA0;
    bA0 = (~v0 & c0[j]) | (~(v0 ^ c0[j]) & bA0);
    const uint64_t m0 = d0 ^ c2[j] ^ bB0;
    bB0 = (~d0 & c2[j]) | (~(d0 ^ c2[j]) & bB0);
    const uint64_t d1 = v1 ^ c0[j] ^ bA1;
    bA1 = (~v1 & c0[j]) | (~(v1 ^ c0[j]) & bA1);
    const uint64_t m1 = d1 ^ c2[j] ^ bB1;
    bB1 = (~d1 & c2[j]) | (~(d1 ^ c2[j]) & bB1);
    const uint64_t k0 = w0[j] ^ m0, k1 = w1[j] ^ m1;          // party 0 -> party 1
    const uint64_t wc = (ch & w1[j]) | (~ch & w0[j]);         // party 2 -> party 1
    out[0][j] = c0[j];
    out[1][j] = wc ^ ((ch & k1) | (~ch & k0));                // party 1 -> party 2
    out[2][j] = c2[j];
  }
}

template <int V, bool C32>
__global__ void __launch_bounds__(256) compare_variant_kernel(CmpVArgs a) {
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.rows * a.nw) return;
  const uint64_t row = t / a.nw, w = t % a.nw;
  const uint64_t col0 = w * 64;
  const int nval = int(min<uint64_t>(64, a.n - col0));
  const bool vec_ok = a.vec != 0;
  const uint64_t qid = a.qid_base + row / uint64_t(a.r);
  const int rot = a.rot[row % uint64_t(a.r)];
  const uint32_t dom = V == kCmpPlain ? kDomCmpPlain : V == kCmpLift18 ? kDomCmpLift18 : kDomCmpConst32;
  const uint64_t stream = row_stream(dom, qid, rot);
  const uint64_t base = ((a.first_entry >> 6) + w) * kTapeBlocksPerGroup;
  B3 r;

  if constexpr (V == kCmpPlain) {
    // y_0 = floor(ml/4) - d_0, y_p = -d_p (mod 2^16): the public term enters component 0
    uint32_t M[32];
    load64(a.ml_pub + row * a.ld, col0, nval, vec_ok, M);
    uint64_t y[3][16];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      uint32_t W[32];
      load64(static_cast<const uint16_t*>(a.code[p]) + row * a.ld, col0, nval, vec_ok, W);
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        const uint32_t tl = p == 0 ? ((M[i] & 0xFFFFu) >> 2) : 0u, th = p == 0 ? (M[i] >> 18) : 0u;
        const uint32_t lo = (tl - (W[i] & 0xFFFFu)) & 0xFFFFu, hi = (th - (W[i] >> 16)) & 0xFFFFu;
        W[i] = lo | (hi << 16);
      }
      to_planes(W, y[p]);
    }
    r = bit_extract_msb<15, 0, 16>(a.keys, stream, base, y);
  } else if constexpr (V == kCmpLift18) {
    uint64_t x[3][16];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      uint32_t W[32];
      load64(static_cast<const uint16_t*>(a.mask[p]) + row * a.ld, col0, nval, vec_ok, W);
      to_planes(W, x[p]);
    }
    // Lift: bits 16 and 17 of S = x0 + x1 + x2 (BitExtract m = 17, words 0..33)
    B3 bit16{{0, 0, 0}}, bit17{{0, 0, 0}};
    {
      B3 cprev{{0, 0, 0}}, carry{{0, 0, 0}}, rr{{0, 0, 0}};
#pragma unroll
      for (int blk = 0; blk < 5; ++blk) {
        Blk3 b;
        gen3(b, a.keys, stream, after(base + blk, carry.c[0] ^ cprev.c[1]));
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int i = 4 * blk + ii;
          if (i > 17) break;
          const uint64_t y0 = i < 16 ? x[0][i] : 0, y1 = i < 16 ? x[1][i] : 0, y2 = i < 16 ? x[2][i] : 0;
          bx_step(b, 2 * ii, i, 17, y0, y1, y2, cprev, carry, rr);
          if (i == 16) bit16 = rr;
          if (i == 17) bit17 = rr;
        }
      }
    }
    // Inject bit 17 into Z_2^1 and bit 16 into Z_2^2 (blocks 10, 11)
    uint64_t A[3][1], B[3][2];
    {
      uint32_t blk[4][16];
      const Key* const ks[4] = {&a.keys.k[0], &a.keys.k[0], &a.keys.k[2], &a.keys.k[2]};
      const uint64_t st[4] = {stream, stream, stream, stream};
      const uint64_t dep = bit16.c[0] ^ bit17.c[1];
      const uint64_t ps[4] = {after(base + 10, dep), after(base + 11, dep), after(base + 10, dep),
                              after(base + 11, dep)};
      chacha12_n<4>(ks, st, ps, blk);
      const uint64_t c0a[1] = {word64(blk[0], 0)}, c2a[1] = {word64(blk[2], 0)};
      const uint64_t w0a[1] = {word64(blk[2], 1)}, w1a[1] = {word64(blk[2], 2)};
      const uint64_t c0b[2] = {word64(blk[1], 0), word64(blk[1], 1)};
      const uint64_t c2b[2] = {word64(blk[3], 0), word64(blk[3], 1)};
      const uint64_t w0b[2] = {word64(blk[3], 2), word64(blk[3], 3)};
      const uint64_t w1b[2] = {word64(blk[3], 4), word64(blk[3], 5)};
      inject_words<1>(bit17, c0a, c2a, w0a, w1a, A);
      inject_words<2>(bit16, c0b, c2b, w0b, w1b, B);
    }
    // y_p = x_p - 2^17 A_p - 2^16 B_p - 4 d_p (mod 2^18)
    uint64_t y[3][18];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      uint32_t W[32];
      uint64_t d[16];
      load64(static_cast<const uint16_t*>(a.code[p]) + row * a.ld, col0, nval, vec_ok, W);
      to_planes(W, d);
      uint64_t s[18];
#pragma unroll
      for (int j = 0; j < 18; ++j) {
        y[p][j] = j < 16 ? x[p][j] : 0;
        s[j] = j >= 2 ? d[j - 2] : 0;
      }
      sub_planes<18>(y[p], s);
#pragma unroll
      for (int j = 0; j < 18; ++j) s[j] = j == 16 ? B[p][0] : j == 17 ? (B[p][1] ^ A[p][0]) : 0;
      // 2^16 B + 2^17 A has bit 16 = B0 and bit 17 = B1 ^ A0 (mod 2^18)
      sub_planes<18>(y[p], s);
    }
    r = bit_extract_msb<17, 40, 18>(a.keys, stream, base, y);
  } else {
    // y_p = 2^14 x_p - 2^16 d_p = (x_p - 4 d_p) 2^14 (mod 2^32): bits 0..13
    // are zero, bits 14..31 are t = (x_p - 4 d_p) mod 2^18.  Four columns at
    // a time: t's low 16 bits packed for the transpose, bits 16, 17 gathered
    // into their planes directly.
    uint64_t y[3][32];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const uint32_t* xr = static_cast<const uint32_t*>(a.mask[p]) + row * a.ld + col0;
      const uint32_t* dr32 = static_cast<const uint32_t*>(a.code[p]) + row * a.ld + col0;
      const uint16_t* dr16 = static_cast<const uint16_t*>(a.code[p]) + row * a.ld + col0;
      uint32_t Wl[32];
      uint64_t h16 = 0, h17 = 0;
      auto put = [&](int g, const uint32_t (&xv)[4], const uint32_t (&dv)[4]) {
        uint32_t tv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          tv[k] = xv[k] - (dv[k] << 2);
          h16 |= uint64_t((tv[k] >> 16) & 1u) << (4 * g + k);
          h17 |= uint64_t((tv[k] >> 17) & 1u) << (4 * g + k);
        }
        Wl[2 * g] = (tv[0] & 0xFFFFu) | (tv[1] << 16);
        Wl[2 * g + 1] = (tv[2] & 0xFFFFu) | (tv[3] << 16);
      };
      if (vec_ok && nval == 64) {
#pragma unroll
        for (int g = 0; g < 16; ++g) {
          const uint4 v = reinterpret_cast<const uint4*>(xr)[g];
          const uint32_t xv[4] = {v.x, v.y, v.z, v.w};
          uint32_t dv[4];
          if constexpr (C32) {
            const uint4 d = reinterpret_cast<const uint4*>(dr32)[g];
            dv[0] = d.x; dv[1] = d.y; dv[2] = d.z; dv[3] = d.w;
          } else {
            const uint2 d = reinterpret_cast<const uint2*>(dr16)[g];
            dv[0] = d.x & 0xFFFFu; dv[1] = d.x >> 16; dv[2] = d.y & 0xFFFFu; dv[3] = d.y >> 16;
          }
          put(g, xv, dv);
        }
      } else {
#pragma unroll
        for (int g = 0; g < 16; ++g) {
          uint32_t xv[4], dv[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int c = 4 * g + k;
            xv[k] = c < nval ? xr[c] : 0u;
            if constexpr (C32) dv[k] = c < nval ? dr32[c] : 0u;
            else dv[k] = c < nval ? uint32_t(dr16[c]) : 0u;
          }
          put(g, xv, dv);
        }
      }
      uint64_t tp[16];
      to_planes(Wl, tp);
#pragma unroll
      for (int j = 0; j < 32; ++j) y[p][j] = j < 14 ? 0 : j < 30 ? tp[j - 14] : j == 30 ? h16 : h17;
    }
    r = bit_extract_msb<31, 0, 32>(a.keys, stream, base, y);
  }

  const uint64_t keep = nval == 64 ? ~0ull : ((1ull << nval) - 1ull);
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
    a.match[p][row * a.mw_ld + w] = r.c[p] & keep;
    a.match[p][a.match_plane + row * a.mw_ld + w] = r.c[pm] & keep;
  }
}

// ---------------------------------------------------------------------------
// Reshare (App. C): z'_p = z_p + F(key_p) - F(key_{p-1}); party p sends z'_p
// to p+1.  One thread: 16 consecutive entries of one row (one block per key).
// ---------------------------------------------------------------------------
struct ReshareArgs {
  Keys3 keys;
  const uint16_t* add_code[3];
  const uint16_t* add_mask[3];
  uint16_t* msg[3];          // [2][rows][ld]
  uint16_t* rep_code[3];     // [2][rows][ld]
  uint16_t* rep_mask[3];
  const imc_query_entry* tab;  // optional: per-query id and column count
  uint64_t ld, n, rows, plane;
  uint64_t qid_base, first_entry;
  int32_t r;
  int8_t rot[IMC_MAX_ROT_DEV];
};

__device__ __forceinline__ void ld16(const uint16_t* p, int nval, bool vec, uint16_t v[16]) {
  if (vec && nval == 16) {
    const uint4 a = reinterpret_cast<const uint4*>(p)[0], b = reinterpret_cast<const uint4*>(p)[1];
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = uint16_t((j & 1) ? (w[j >> 1] >> 16) : (w[j >> 1] & 0xFFFF));
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = j < nval ? p[j] : 0;
  }
}

__device__ __forceinline__ void st16(uint16_t* p, int nval, bool vec, const uint16_t v[16]) {
  if (vec && nval == 16) {
    uint32_t w[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) w[j] = uint32_t(v[2 * j]) | (uint32_t(v[2 * j + 1]) << 16);
    reinterpret_cast<uint4*>(p)[0] = make_uint4(w[0], w[1], w[2], w[3]);
    reinterpret_cast<uint4*>(p)[1] = make_uint4(w[4], w[5], w[6], w[7]);
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (j < nval) p[j] = v[j];
  }
}

__global__ void __launch_bounds__(256) reshare_kernel(ReshareArgs a) {
  const uint64_t nc = (a.n + 15) / 16;
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.rows * nc) return;
  const uint64_t row = t / nc, c = t % nc;
  const uint64_t qi = row / uint64_t(a.r);
  uint64_t qid = a.qid_base + qi, n = a.n;
  const uint64_t col0 = 16 * c;
  if (a.tab) {
    qid = a.tab[qi].query_id;
    n = min<uint64_t>(n, a.tab[qi].n);
    if (col0 >= n) return;
  }
  const int rot = a.rot[row % uint64_t(a.r)];
  const uint64_t stream = row_stream(kDomReshare, qid, rot);
  const uint64_t e0 = a.first_entry + 16 * c;
  const int nval = int(min<uint64_t>(16, n - col0));
  const uint64_t off = row * a.ld + col0;
  const bool vec = (a.ld % 8) == 0;
  const bool with_mask = a.add_mask[0] != nullptr;   // no mask dot when masks are public
  const bool with_rep = a.rep_code[0] != nullptr;     // otherwise the messages alone
  uint16_t zc[3][16], zm[3][16];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    ld16(a.add_code[p] + off, nval, vec, zc[p]);
    if (with_mask) ld16(a.add_mask[p] + off, nval, vec, zm[p]);
  }
  uint32_t F[3][16];
  {
    const Key* const ks[3] = {&a.keys.k[0], &a.keys.k[1], &a.keys.k[2]};
    const uint64_t st[3] = {stream, stream, stream}, ps[3] = {e0 >> 4, e0 >> 4, e0 >> 4};
    chacha12_n<3>(ks, st, ps, F);
  }
  uint16_t oc[3][16], om[3][16];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      oc[p][j] = uint16_t(zc[p][j] + uint16_t((F[p][j] & 0xFFFFu) - (F[pm][j] & 0xFFFFu)));
      om[p][j] = uint16_t(zm[p][j] + uint16_t((F[p][j] >> 16) - (F[pm][j] >> 16)));
    }
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
    st16(a.msg[p] + off, nval, vec, oc[p]);              // party p -> party p+1
    if (with_rep) {
      st16(a.rep_code[p] + off, nval, vec, oc[p]);
      st16(a.rep_code[p] + a.plane + off, nval, vec, oc[pm]);   // received from party p-1
    }
    if (!with_mask) continue;
    st16(a.msg[p] + a.plane + off, nval, vec, om[p]);
    if (with_rep) {
      st16(a.rep_mask[p] + off, nval, vec, om[p]);
      st16(a.rep_mask[p] + a.plane + off, nval, vec, om[pm]);
    }
  }
}

// ---------------------------------------------------------------------------
// OR-tree (Sec. 4.2): x OR y = x ^ y ^ AND(x, y), gate i of level L uses
// stream (DOM_OR, qid) at position (L << 40) + i/8, word i%8.
// ---------------------------------------------------------------------------
struct OrArgs {
  Keys3 keys;
  const uint64_t* in0[3];    // level 0: match[p] plane 0, [rows][mw_ld]
  const uint64_t* in;        // levels > 0: [q][len][3]
  uint64_t* out;             // [q][(len+1)/2][3]
  uint64_t q, len, nw, mw_ld, in_stride, out_stride;
  uint64_t qid_base;
  int32_t r, level, first;
};

__global__ void __launch_bounds__(256) or_level_kernel(OrArgs a) {
  const uint64_t half = (a.len + 1) / 2;
  const uint64_t ng = (half + 7) / 8;
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.q * ng) return;
  const uint64_t qi = t / ng, g = t % ng;
  const uint64_t stream = (uint64_t(kDomOr) << 56) | ((a.qid_base + qi) & 0xFFFFFFFFFFFFull);
  uint32_t F[3][16];
#pragma unroll
  for (int k = 0; k < 3; ++k) chacha12(a.keys.k[k], stream, (uint64_t(a.level) << 40) + g, F[k]);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const uint64_t i = 8 * g + u;
    if (i >= half) break;
    B3 x, y;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const uint64_t i0 = 2 * i, i1 = 2 * i + 1;
      if (a.first) {
        const uint64_t r0 = i0 / a.nw, w0 = i0 % a.nw;
        x.c[p] = a.in0[p][(qi * a.r + r0) * a.mw_ld + w0];
        if (i1 < a.len) {
          const uint64_t r1 = i1 / a.nw, w1 = i1 % a.nw;
          y.c[p] = a.in0[p][(qi * a.r + r1) * a.mw_ld + w1];
        } else {
          y.c[p] = 0;
        }
      } else {
        x.c[p] = a.in[(qi * a.in_stride + i0) * 3 + p];
        y.c[p] = i1 < a.len ? a.in[(qi * a.in_stride + i1) * 3 + p] : 0;
      }
    }
    const uint64_t f0 = uint64_t(F[0][2 * u]) | (uint64_t(F[0][2 * u + 1]) << 32);
    const uint64_t f1 = uint64_t(F[1][2 * u]) | (uint64_t(F[1][2 * u + 1]) << 32);
    const uint64_t f2 = uint64_t(F[2][2 * u]) | (uint64_t(F[2][2 * u + 1]) << 32);
    const B3 z = bx(bx(x, y), band(x, y, f0, f1, f2));
#pragma unroll
    for (int p = 0; p < 3; ++p) a.out[(qi * a.out_stride + i) * 3 + p] = z.c[p];
  }
}

struct OrFinalArgs {
  Keys3 keys;
  const uint64_t* in0[3];    // used when the tree had a single word per query
  const uint64_t* in;        // [q][stride][3]
  uint8_t* dup[3];           // [2][q]
  uint64_t q, stride, mw_ld;
  uint64_t qid_base;
  int32_t r, level, first;
};

__global__ void __launch_bounds__(64) or_final_kernel(OrFinalArgs a) {
  const uint64_t qi = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (qi >= a.q) return;
  const uint64_t stream = (uint64_t(kDomOr) << 56) | ((a.qid_base + qi) & 0xFFFFFFFFFFFFull);
  B3 w;
#pragma unroll
  for (int p = 0; p < 3; ++p)
    w.c[p] = a.first ? a.in0[p][(qi * a.r) * a.mw_ld] : a.in[(qi * a.stride) * 3 + p];
#pragma unroll
  for (int lv = 0; lv < 6; ++lv) {
    const int sh = 32 >> lv;
    const int level = a.level + lv;
    uint32_t F[3][16];
#pragma unroll
    for (int k = 0; k < 3; ++k) chacha12(a.keys.k[k], stream, uint64_t(level) << 40, F[k]);
    const B3 y{{w.c[0] >> sh, w.c[1] >> sh, w.c[2] >> sh}};
    w = bx(bx(w, y), band(w, y, uint64_t(F[0][0]) | (uint64_t(F[0][1]) << 32),
                          uint64_t(F[1][0]) | (uint64_t(F[1][1]) << 32),
                          uint64_t(F[2][0]) | (uint64_t(F[2][1]) << 32)));
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
    a.dup[p][qi] = uint8_t(w.c[p] & 1u);
    a.dup[p][a.q + qi] = uint8_t(w.c[pm] & 1u);
  }
}

// ---------------------------------------------------------------------------
// In-batch matching (Sec. 6.4): query qi of a batch is compared with the
// queries of earlier groups only (groups of `group` consecutive queries, e.g.
// a person's two eyes): the shared match bits of columns
// j >= group * floor(qi / group) in word `word` of every row qi*r + ri become
// public zeros (every component of both planes is cleared).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) mask_in_batch_kernel(uint64_t* m0, uint64_t* m1, uint64_t* m2, uint64_t q,
                                                            uint32_t r, uint64_t mw_ld, uint64_t word, uint64_t group) {
  const uint64_t rows = q * r;
  const uint64_t row = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  const uint64_t cut = (row / r) / group * group;   // first query of this query's group
  const uint64_t keep = cut >= 64 ? ~0ull : ((1ull << cut) - 1);
  uint64_t* m[3] = {m0, m1, m2};
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int plane = 0; plane < 2; ++plane) m[p][(plane * rows + row) * mw_ld + word] &= keep;
}

// Shared OR of two bit sharings, one AND gate per element: z = x ^ y ^ (x AND y).
// The gate of element i takes bit i%64 of u64 word i/64 of stream
// (kDomOrPairs << 56 | id) from every key.  a, b, out: u8 [2][count].
struct OrBitsArgs {
  Keys3 keys;
  const uint8_t* a[3];       // element i at a[p][i * stride]
  const uint8_t* b[3];
  uint8_t* out[3];
  uint64_t count, id, stride;
};

__global__ void __launch_bounds__(256) or_bits_kernel(OrBitsArgs a) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.count) return;
  const uint64_t stream = (uint64_t(kDomOrPairs) << 56) | (a.id & 0xFFFFFFFFFFFFull);
  const uint64_t t = i >> 6;
  uint64_t f[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint32_t F[16];
    chacha12(a.keys.k[k], stream, t >> 3, F);
    const int u = int(t & 7);
    f[k] = ((uint64_t(F[2 * u]) | (uint64_t(F[2 * u + 1]) << 32)) >> (i & 63)) & 1u;
  }
  B3 x, y;
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    x.c[p] = a.a[p][i * a.stride] & 1u;
    y.c[p] = a.b[p][i * a.stride] & 1u;
  }
  const B3 z = bx(bx(x, y), band(x, y, f[0], f[1], f[2]));
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
    a.out[p][i] = uint8_t(z.c[p] & 1u);
    a.out[p][a.count + i] = uint8_t(z.c[pm] & 1u);
  }
}

// ---------------------------------------------------------------------------
// Open: out = x_0 op x_1 op x_2 from each party's own component; with check,
// count positions where party p's copy of x_{p-1} differs from party p-1's.
// ---------------------------------------------------------------------------
template <typename T, bool XOR>
__global__ void __launch_bounds__(256) open_kernel(const T* r0, const T* r1, const T* r2, uint64_t count, T* out,
                                                   int check, unsigned long long* bad) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const T a = r0[i], b = r1[i], c = r2[i];
  out[i] = XOR ? T(a ^ b ^ c) : T(a + b + c);
  if (check) {
    const bool ok = (r1[count + i] == a) && (r2[count + i] == b) && (r0[count + i] == c);
    if (!ok) atomicAdd(bad, 1ull);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static void fill_rot(int8_t* dst, const imc_ids_dev& ids) {
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) dst[i] = i < ids.r ? ids.rot[i] : 0;
}

hipError_t launch_reshare(const Keys3& keys, const uint16_t* const add_code[3], const uint16_t* const add_mask[3],
                          uint64_t rows, uint64_t n, uint64_t ld, const imc_ids_dev& ids, uint16_t* const msg[3],
                          uint16_t* const rep_code[3], uint16_t* const rep_mask[3], hipStream_t s,
                          const QueryTab& qt) {
  if (rows == 0 || n == 0) return hipSuccess;
  ReshareArgs a;
  a.tab = qt.tab;
  a.keys = keys;
  for (int p = 0; p < 3; ++p) {
    a.add_code[p] = add_code[p];
    a.add_mask[p] = add_mask ? add_mask[p] : nullptr;
    a.msg[p] = msg[p];
    a.rep_code[p] = rep_code ? rep_code[p] : nullptr;
    a.rep_mask[p] = (add_mask && rep_code) ? rep_mask[p] : nullptr;
  }
  a.ld = ld;
  a.n = n;
  a.rows = rows;
  a.plane = (qt.plane_rows ? qt.plane_rows : rows) * ld;
  a.qid_base = ids.query_id_base;
  a.first_entry = ids.first_entry_id;
  a.r = ids.r;
  fill_rot(a.rot, ids);
  const uint64_t threads = rows * ((n + 15) / 16);
  if (!fits_grid(threads, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reshare_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_compare(const Keys3& keys, const uint16_t* const rep_code[3], const uint16_t* const rep_mask[3],
                          uint64_t rows, uint64_t n, uint64_t ld, const imc_ids_dev& ids, uint64_t* const match[3],
                          uint64_t mw_ld, hipStream_t s, const QueryTab& qt) {
  if (rows == 0 || n == 0) return hipSuccess;
  CmpArgs a;
  a.tab = qt.tab;
  a.keys = keys;
  for (int p = 0; p < 3; ++p) {
    a.code[p] = rep_code[p];
    a.mask[p] = rep_mask[p];
    a.match[p] = match[p];
  }
  a.ld = ld;
  a.mw_ld = mw_ld;
  a.n = n;
  a.nw = (n + 63) / 64;
  a.rows = rows;
  a.plane_elems = (qt.plane_rows ? qt.plane_rows : rows) * ld;
  a.match_plane = rows * mw_ld;
  a.qid_base = ids.query_id_base;
  a.first_entry = ids.first_entry_id;
  a.r = ids.r;
  fill_rot(a.rot, ids);
  const uint64_t threads = rows * a.nw;
  if (!fits_grid(threads, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(compare_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_compare_variant(int variant, const Keys3& keys, const void* const rep_code[3], bool code32,
                                  const void* const rep_mask[3], const uint16_t* ml_pub, uint64_t rows, uint64_t n,
                                  uint64_t ld, const imc_ids_dev& ids, uint64_t* const match[3], uint64_t mw_ld,
                                  hipStream_t s) {
  if (rows == 0 || n == 0) return hipSuccess;
  CmpVArgs a;
  a.keys = keys;
  for (int p = 0; p < 3; ++p) {
    a.code[p] = rep_code[p];
    a.mask[p] = rep_mask ? rep_mask[p] : nullptr;
    a.match[p] = match[p];
  }
  a.ml_pub = ml_pub;
  a.ld = ld;
  a.mw_ld = mw_ld;
  a.n = n;
  a.nw = (n + 63) / 64;
  a.rows = rows;
  a.match_plane = rows * mw_ld;
  a.qid_base = ids.query_id_base;
  a.first_entry = ids.first_entry_id;
  a.r = ids.r;
  bool vec = (ld % 8) == 0 && (reinterpret_cast<uintptr_t>(ml_pub) % 16) == 0;
  for (int p = 0; p < 3; ++p)
    vec = vec && (reinterpret_cast<uintptr_t>(a.code[p]) % 16) == 0 && (reinterpret_cast<uintptr_t>(a.mask[p]) % 16) == 0;
  a.vec = vec ? 1 : 0;
  fill_rot(a.rot, ids);
  if (!fits_grid(rows * a.nw, 256)) return hipErrorInvalidValue;
  const dim3 grid(unsigned((rows * a.nw + 255) / 256)), block(256);
  switch (variant) {
    case kCmpPlain: hipLaunchKernelGGL((compare_variant_kernel<kCmpPlain, false>), grid, block, 0, s, a); break;
    case kCmpLift18: hipLaunchKernelGGL((compare_variant_kernel<kCmpLift18, false>), grid, block, 0, s, a); break;
    case kCmpConst32:
      if (code32) hipLaunchKernelGGL((compare_variant_kernel<kCmpConst32, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((compare_variant_kernel<kCmpConst32, false>), grid, block, 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t or_tree_ws_bytes(uint64_t q, uint64_t r, uint64_t nw) {
  const uint64_t len = r * nw;
  const uint64_t half = (len + 1) / 2;
  return size_t(2 * q * half * 3 * sizeof(uint64_t));
}

hipError_t launch_or_tree(const Keys3& keys, const uint64_t* const match[3], uint64_t q, uint64_t nw, uint64_t mw_ld,
                          const imc_ids_dev& ids, void* ws, uint8_t* const dup[3], hipStream_t s) {
  if (q == 0) return hipSuccess;
  const uint64_t len0 = uint64_t(ids.r) * nw;
  const uint64_t stride = (len0 + 1) / 2;
  uint64_t* buf[2] = {reinterpret_cast<uint64_t*>(ws), reinterpret_cast<uint64_t*>(ws) + q * stride * 3};
  uint64_t len = len0;
  int level = 0, cur = -1;
  while (len > 1) {
    OrArgs a;
    a.keys = keys;
    for (int p = 0; p < 3; ++p) a.in0[p] = match[p];
    a.in = cur >= 0 ? buf[cur] : nullptr;
    a.out = buf[cur >= 0 ? 1 - cur : 0];
    a.q = q;
    a.len = len;
    a.nw = nw;
    a.mw_ld = mw_ld;
    a.in_stride = stride;
    a.out_stride = stride;
    a.qid_base = ids.query_id_base;
    a.r = ids.r;
    a.level = level;
    a.first = cur < 0;
    const uint64_t half = (len + 1) / 2;
    const uint64_t threads = q * ((half + 7) / 8);
    if (!fits_grid(threads, 256)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(or_level_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur = cur >= 0 ? 1 - cur : 0;
    len = half;
    ++level;
  }
  OrFinalArgs f;
  f.keys = keys;
  for (int p = 0; p < 3; ++p) {
    f.in0[p] = match[p];
    f.dup[p] = dup[p];
  }
  f.in = cur >= 0 ? buf[cur] : nullptr;
  f.q = q;
  f.stride = stride;
  f.mw_ld = mw_ld;
  f.qid_base = ids.query_id_base;
  f.r = ids.r;
  f.level = level;
  f.first = cur < 0;
  if (!fits_grid(q, 64)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(or_final_kernel, dim3(unsigned((q + 63) / 64)), dim3(64), 0, s, f);
  return hipGetLastError();
}

__global__ void zero_counter_kernel(unsigned long long* c) { *c = 0ull; }

hipError_t launch_open(int kind, const void* const rep[3], uint64_t count, void* out, int check,
                       unsigned long long* bad, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (!fits_grid(count, 256)) return hipErrorInvalidValue;
  if (check) hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, bad);
  const dim3 grid(unsigned((count + 255) / 256)), block(256);
  switch (kind) {
    case 0:
      hipLaunchKernelGGL((open_kernel<uint8_t, true>), grid, block, 0, s, (const uint8_t*)rep[0],
                         (const uint8_t*)rep[1], (const uint8_t*)rep[2], count, (uint8_t*)out, check, bad);
      break;
    case 1:
      hipLaunchKernelGGL((open_kernel<uint64_t, true>), grid, block, 0, s, (const uint64_t*)rep[0],
                         (const uint64_t*)rep[1], (const uint64_t*)rep[2], count, (uint64_t*)out, check, bad);
      break;
    case 2:
      hipLaunchKernelGGL((open_kernel<uint16_t, false>), grid, block, 0, s, (const uint16_t*)rep[0],
                         (const uint16_t*)rep[1], (const uint16_t*)rep[2], count, (uint16_t*)out, check, bad);
      break;
    default:
      hipLaunchKernelGGL((open_kernel<uint32_t, false>), grid, block, 0, s, (const uint32_t*)rep[0],
                         (const uint32_t*)rep[1], (const uint32_t*)rep[2], count, (uint32_t*)out, check, bad);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_mask_in_batch(uint64_t* const match[3], uint64_t q, uint32_t r, uint64_t mw_ld, uint64_t word,
                                uint64_t group, hipStream_t s) {
  const uint64_t rows = q * r;
  if (rows == 0) return hipSuccess;
  if (!fits_grid(rows, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mask_in_batch_kernel, dim3(unsigned((rows + 255) / 256)), dim3(256), 0, s, match[0], match[1],
                     match[2], q, r, mw_ld, word, group);
  return hipGetLastError();
}

hipError_t launch_or_bits(const Keys3& keys, const uint8_t* const x[3], const uint8_t* const y[3], uint64_t count,
                          uint64_t id, uint8_t* const out[3], hipStream_t s) {
  if (count == 0) return hipSuccess;
  OrBitsArgs a;
  a.keys = keys;
  for (int p = 0; p < 3; ++p) {
    a.a[p] = x[p];
    a.b[p] = y[p];
    a.out[p] = out[p];
  }
  a.count = count;
  a.id = id;
  a.stride = 1;
  if (!fits_grid(count, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(or_bits_kernel, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_or_pairs(const Keys3& keys, const uint8_t* const in[3], uint64_t count, uint64_t id,
                           uint8_t* const out[3], hipStream_t s) {
  if (count == 0) return hipSuccess;
  OrBitsArgs a;
  a.keys = keys;
  for (int p = 0; p < 3; ++p) {
    a.a[p] = in[p];        // elements 2i
    a.b[p] = in[p] + 1;    // elements 2i + 1
    a.out[p] = out[p];
  }
  a.count = count;
  a.id = id;
  a.stride = 2;
  if (!fits_grid(count, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(or_bits_kernel, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace imc
