// circuit_msg.hip -- the threshold comparison with the three parties kept
// apart and every message between them passed through a device buffer (the
// AND gates of App. C, BitExtract / BitInject / 3OT of App. D; Sec. 6.4 keeps
// all of the deployment's communication on the GPU).
//
// A workgroup is three waves, one per party; lane l of each wave works on the
// same 64 comparisons (one row, 64 consecutive entries, bit-sliced).  Wave p
// holds party p's view only -- components p and p-1 of every sharing, keys p
// and p-1 of the correlated randomness -- and learns components p-1 of gate
// outputs by reading what party p-1 stored in its plane of the message
// buffer.  Each round of the circuit is: every party stores its messages,
// workgroup barrier, every party loads what was sent to it.
//
// Message planes (bit o of match word w = column 64w+o), in the order of the
// oracle's message log, stored per workgroup: the 64 words of workgroup b
// keep plane m at u64 (b * planes + m) * 64 + lane, so a workgroup's
// messages are one contiguous block (a few pages instead of one page per
// plane: 8 % faster than planes of rows x mw_ld words on the full
// comparison).  Order: AND gate g (numbered bit by bit,
// the FA-layer gate of a bit before its ripple gate) sent by party p at plane
// 3g + p; then, per BitInject of k bits, k0 and k1 (party 0 to 1), w_c
// (party 2 to 1) and c1 (party 1 to 2), k planes each.
#include "bits.h"
#include "device.h"
#include "launch.h"

namespace imc {

// Party p's view of a bit-sliced boolean sharing: own component p and
// component p-1.
struct PV {
  uint64_t o, v;
};
__device__ __forceinline__ PV pvx(PV a, PV b) { return PV{a.o ^ b.o, a.v ^ b.v}; }

// InpLocal (App. D) of bit i of component j, seen by party p, from party p's
// bit planes yo (component p) and yv (component p-1): component j is the bit,
// the others are zero.
__device__ __forceinline__ PV inp(int j, int p, uint64_t yo, uint64_t yv) {
  return PV{j == p ? yo : 0ull, j == (p + 2) % 3 ? yv : 0ull};
}

// ABY3 AND, party p's local share: z_p = x_p y_p ^ x_{p-1} y_p ^ x_p y_{p-1}
// ^ F(key_p) ^ F(key_{p-1}); z_p goes to party p+1.
__device__ __forceinline__ uint64_t and_local(PV x, PV y, uint64_t fo, uint64_t fv) {
  return (x.o & y.o) ^ (x.v & y.o) ^ (x.o & y.v) ^ fo ^ fv;
}

// The message buffer as seen by one lane: plane m of its workgroup's block
// starts at the wave-uniform address msg + 64 m, the lane's word is lane
// words in.
struct Net {
  uint64_t* msg;     // the workgroup's block: [planes][64]
  uint32_t lane;
  bool active;       // lanes past the last word store and load nothing
  __device__ __forceinline__ void send(int m, uint64_t v) const {
    if (active) msg[uint32_t(m) * 64u + lane] = v;
  }
  __device__ __forceinline__ uint64_t recv(int m) const {
    return active ? msg[uint32_t(m) * 64u + lane] : 0ull;
  }
};
__device__ __forceinline__ Net net_of(uint64_t* msg, int planes, bool active) {
  return Net{msg + uint64_t(blockIdx.x) * uint64_t(planes) * 64u, uint32_t(threadIdx.x & 63), active};
}

// Tape words of one key, visited in increasing order: the ChaCha12 block of a
// word is generated when the walk enters it (word / 8 changes).
struct Tape {
  uint32_t b[16];
  int cur = -1;
  __device__ __forceinline__ uint64_t word(const Key& k, uint64_t stream, uint64_t base, int wd) {
    if ((wd >> 3) != cur) {
      chacha12(k, stream, base + uint64_t(wd >> 3), b);
      cur = wd >> 3;
    }
    return word64(b, wd & 7);
  }
};

// Bit planes of party p's two components of an arithmetic sharing, read one
// bit at a time by the bit-serial circuits: planes 0..NREG-1 of each
// component in registers, planes NREG..NB-1 in the wave's slice of LDS
// (slots 0.. own component, then previous), planes >= NB zero.  The bit loop
// indexes planes at run time; held in a register array they would go to
// per-lane scratch, whose round trips through L2 cost a third of the kernel
// (measured).  Up to kPlaneSlots LDS slots of 64 u64 per wave: 39 KB per
// workgroup of three waves, so four workgroups (12 waves) share a CU, as many
// as the registers allow.
constexpr int kPlaneSlots = 26;
__shared__ uint64_t lds_planes[3][kPlaneSlots][64];

template <int NB, int NREG>
struct SplitPlanes {
  static constexpr int kLds = NB - NREG;
  static_assert(NREG >= 1 && 2 * kLds <= kPlaneSlots, "planes exceed the LDS slots");
  uint64_t ro[NREG], rv[NREG];
  uint64_t* L;   // this lane's word of slot 0 of its wave
  __device__ __forceinline__ SplitPlanes() : L(&lds_planes[threadIdx.x >> 6][0][threadIdx.x & 63]) {}
  // component c (0: own, 1: previous)
  __device__ __forceinline__ void put(int c, const uint64_t (&x)[NB]) {
#pragma unroll
    for (int j = 0; j < NREG; ++j) (c ? rv : ro)[j] = x[j];
#pragma unroll
    for (int j = NREG; j < NB; ++j) L[(c * kLds + j - NREG) * 64] = x[j];
  }
  // plane k (compile-time, < NB) of component c
  __device__ __forceinline__ uint64_t plane(int c, int k) const {
    return k < NREG ? (c ? rv : ro)[k < NREG ? k : 0] : L[(c * kLds + (k < NREG ? 0 : k - NREG)) * 64];
  }
  __device__ __forceinline__ void get(int k, uint64_t& bo, uint64_t& bv) const {
    const int slot = k < NREG ? 0 : k < NB ? k - NREG : kLds - 1;
    uint64_t a = L[slot * 64], b = L[(kLds + slot) * 64];
    a = k < NB ? a : 0ull;
    b = k < NB ? b : 0ull;
#pragma unroll
    for (int j = 0; j < NREG; ++j) {
      a = k == j ? ro[j] : a;
      b = k == j ? rv[j] : b;
    }
    bo = a;
    bv = b;
  }
  __device__ __forceinline__ void at(int i, uint64_t, uint64_t& bo, uint64_t& bv) const { get(i, bo, bv); }
};

// BitExtract (App. D) of bits 0..M of y_0 + y_1 + y_2; y.at(i, dep, bo, bv)
// gives party p's bit-i planes of its two components when bit i is reached
// (dep: a value of the circuit's state at that point).  The FA-layer gate of
// bit i takes tape word W0 + 2i and is message gate G0 + 2i - 1 (G0 for
// i = 0); the ripple gate of bit i (carry into bit i+1) takes word
// W0 + 2i + 1 and is gate G0 + 2i.  Both gates of a bit go out in one round.
// Returns bit M of the sum; bit M - 1 in *rm1 if given.
template <int M, int W0, int G0, typename Y>
__device__ __forceinline__ PV msg_bit_extract(int p, const Key& ko, const Key& kv, uint64_t stream, uint64_t base,
                                              Y& y, const Net& net, PV* rm1) {
  static_assert(W0 % 8 == 0, "gate words start a block");
  const int pm = (p + 2) % 3;
  PV cprev{0, 0}, carry{0, 0}, r{0, 0};
  // Kept rolled (the bit index is wave-uniform): one block's code instead of
  // (M + 4) / 4 copies and live ranges that end with the block.  The planes
  // are then indexed at run time, which the compiler serves from per-lane
  // scratch; measured on the full comparison, this (about 150 registers,
  // three waves per SIMD) beats every unrolled form (210-330 registers, one
  // or two waves per SIMD; 34 ms against 44-59 ms per 1,984 x 300,000 call).
#pragma unroll 1
  for (int blk = 0; blk < (M + 4) / 4; ++blk) {   // 4 bits (8 tape words) per block
    uint32_t F[2][16];
    {
      const Key* const ks[2] = {&ko, &kv};
      const uint64_t pos = after(base + W0 / 8 + blk, carry.o ^ cprev.v);
      const uint64_t st[2] = {stream, stream}, ps[2] = {pos, pos};
      chacha12_n<2>(ks, st, ps, F);
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int i = 4 * blk + ii;
      if (i > M) continue;   // (no early exit: the four bits unroll)
      uint64_t bo, bv;
      y.at(i, carry.o ^ cprev.v, bo, bv);
      const PV a = inp(0, p, bo, bv), b = inp(1, p, bo, bv), c = inp(2, p, bo, bv);
      const PV t1 = pvx(a, c), t2 = pvx(b, c), s = pvx(t1, b);
      const PV A = cprev;
      const bool fa = i < M, rip = i >= 1 && i < M;
      const int gfa = G0 + (i == 0 ? 0 : 2 * i - 1), grip = G0 + 2 * i;
      PV zf{0, 0}, zr{0, 0};
      if (fa) {
        zf.o = and_local(t1, t2, word64(F[0], 2 * ii), word64(F[1], 2 * ii));
        net.send(3 * gfa + p, zf.o);
      }
      if (rip) {
        zr.o = and_local(pvx(A, carry), pvx(s, carry), word64(F[0], 2 * ii + 1), word64(F[1], 2 * ii + 1));
        net.send(3 * grip + p, zr.o);
      }
      if (fa || rip) __syncthreads();   // the round's messages are in the buffer
      PV ci{0, 0};
      if (fa) {
        zf.v = net.recv(3 * gfa + pm);
        ci = pvx(zf, c);                // FA carry: t1 t2 ^ c
      }
      if (i == 0) {
        r = s;
      } else {
        r = pvx(pvx(A, s), carry);
        if (rip) {
          zr.v = net.recv(3 * grip + pm);
          carry = pvx(zr, carry);
        }
      }
      if (rm1 && i == M - 1) *rm1 = r;
      cprev = ci;
    }
  }
  return r;
}

// BitInject (App. D) of a bit x into Z_2^K, first round: party 0 (sender,
// holding components 0 and 2 of x) forms m_t = (t ^ x0 ^ x2) - c0 - c2 and
// sends k_t = w_t ^ m_t to party 1; party 2 (helper, holding component 1)
// sends w_{x1}.  c0 comes from key_0 (words C0W..), c2, w0, w1 from key_2
// (words C2W.., WAW.., WBW..).  Messages at planes mb + j (k0), mb + K + j
// (k1), mb + 2K + j (w_c).  Party 0 keeps the low KEEP planes of c0 and c2.
template <int K, int KEEP, int C0W, int C2W, int WAW, int WBW>
__device__ __forceinline__ void inject_send(int p, const Keys3& keys, uint64_t stream, uint64_t base, PV x,
                                            const Net& net, int mb, uint64_t (&c0k)[KEEP], uint64_t (&c2k)[KEEP]) {
  if (p == 0) {
    const uint64_t u = x.o ^ x.v;
    Tape t0, tc, ta, tb;
    uint64_t bA0 = 0, bA1 = 0, bB0 = 0, bB1 = 0;   // borrows of (V - c0) and (. - c2) for t = 0, 1
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const uint64_t c0 = t0.word(keys.k[0], stream, base, C0W + j);
      const uint64_t c2 = tc.word(keys.k[2], stream, base, C2W + j);
      const uint64_t w0 = ta.word(keys.k[2], stream, base, WAW + j);
      const uint64_t w1 = tb.word(keys.k[2], stream, base, WBW + j);
      const uint64_t v0 = (j == 0) ? u : 0, v1 = (j == 0) ? ~u : 0;
      const uint64_t d0 = v0 ^ c0 ^ bA0;
      bA0 = (~v0 & c0) | (~(v0 ^ c0) & bA0);
      const uint64_t m0 = d0 ^ c2 ^ bB0;
      bB0 = (~d0 & c2) | (~(d0 ^ c2) & bB0);
      const uint64_t d1 = v1 ^ c0 ^ bA1;
      bA1 = (~v1 & c0) | (~(v1 ^ c0) & bA1);
      const uint64_t m1 = d1 ^ c2 ^ bB1;
      bB1 = (~d1 & c2) | (~(d1 ^ c2) & bB1);
      net.send(mb + j, w0 ^ m0);
      net.send(mb + K + j, w1 ^ m1);
      if (j < KEEP) {
        c0k[j] = c0;
        c2k[j] = c2;
      }
    }
  } else if (p == 2) {
    const uint64_t ch = x.v;                       // component 1
    Tape ta, tb;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const uint64_t w0 = ta.word(keys.k[2], stream, base, WAW + j);
      const uint64_t w1 = tb.word(keys.k[2], stream, base, WBW + j);
      net.send(mb + 2 * K + j, (ch & w1) | (~ch & w0));
    }
  }
}

// Second round: party 1 (receiver, choice bit = its component 1) takes
// c1 = w_c ^ k_{x1} and forwards it to party 2 (planes mb + 3K + j).
template <int K, int KEEP>
__device__ __forceinline__ void inject_forward(int p, PV x, const Net& net, int mb, uint64_t (&c1k)[KEEP]) {
  if (p != 1) return;
  const uint64_t ch = x.o;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint64_t k0 = net.recv(mb + j), k1 = net.recv(mb + K + j), wc = net.recv(mb + 2 * K + j);
    const uint64_t c1 = wc ^ ((ch & k1) | (~ch & k0));
    net.send(mb + 3 * K + j, c1);
    if (j < KEEP) c1k[j] = c1;
  }
}

// After the second round: party p's view of the low KEEP planes of the
// injected value, components (c0, c1, c2): party 0 holds (c0, c2), party 1
// (c1, c0), party 2 (c2, c1), c1 received from party 1.
template <int K, int KEEP, int C0W, int C2W>
__device__ __forceinline__ void inject_view(int p, const Keys3& keys, uint64_t stream, uint64_t base, const Net& net,
                                            int mb, const uint64_t (&c0k)[KEEP], const uint64_t (&c2k)[KEEP],
                                            const uint64_t (&c1k)[KEEP], uint64_t (&vo)[KEEP],
                                            uint64_t (&vv)[KEEP]) {
  if (p == 0) {
#pragma unroll
    for (int j = 0; j < KEEP; ++j) {
      vo[j] = c0k[j];
      vv[j] = c2k[j];
    }
  } else if (p == 1) {
    Tape t0;
#pragma unroll
    for (int j = 0; j < KEEP; ++j) {
      vo[j] = c1k[j];
      vv[j] = t0.word(keys.k[0], stream, base, C0W + j);
    }
  } else {
    Tape tc;
#pragma unroll
    for (int j = 0; j < KEEP; ++j) {
      vo[j] = tc.word(keys.k[2], stream, base, C2W + j);
      vv[j] = net.recv(mb + 3 * K + j);
    }
  }
}

struct CmpMsgArgs {
  Keys3 keys;
  const void* code[3];       // rep_code[p] plane 0 (own component); plane 1 at + plane_elems
  const uint16_t* prev_code[3];  // MPCLift: party p's second component (party p-1's share) of the
  const uint16_t* prev_mask[3];  // code and mask dots: plane 1 of rep_*, or party p-1's message
  const void* mask[3];       // rep_mask[p] likewise (MPCLift, Lift18, Const32)
  const uint16_t* ml_pub;    // [rows][ld] public ml (Plain)
  uint64_t* match[3];        // [2][rows][mw_ld]
  const imc_query_entry* tab;  // optional: per-query id, column count and match planes
  uint64_t* msg;             // [workgroup][planes][64]
  uint64_t ld, mw_ld, n, nw, rows, plane_elems, match_plane;
  uint64_t qid_base, first_entry;
  int32_t r;
  int32_t vec;               // 16-byte loads allowed
  int8_t rot[IMC_MAX_ROT_DEV];
};

// Bits 16..31 of one component of the MPCLift y from that component of ml
// (xm planes), of the code dot (d planes) and of the two injected values:
// y = 2^14 (x - 2^17 A - 2^16 B) - 2^16 d (mod 2^32) has bits 0..13 zero,
// bits 14, 15 = x bits 0, 1, and bits 16..31 =
// (x >> 2) - d - (B mod 4) 2^14 - (A mod 2) 2^15 (mod 2^16).
__device__ __forceinline__ void mpclift_u(const uint64_t (&xm)[16], const uint64_t (&d)[16], uint64_t a0, uint64_t b0,
                                          uint64_t b1, uint64_t (&u)[16]) {
  uint64_t br = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint64_t X = j < 14 ? xm[j + 2] : 0;
    u[j] = X ^ d[j] ^ br;
    br = (~X & d[j]) | (~(X ^ d[j]) & br);
  }
  const uint64_t u14 = u[14];
  u[14] = u14 ^ b0;
  const uint64_t b2 = ~u14 & b0;
  u[15] = u[15] ^ b1 ^ b2 ^ a0;
}

// Party p's planes of the MPCLift y: bits 0..13 zero, bits 14 and 15 the ml
// planes 0 and 1, bits 16..31 formed before the MSB circuit starts from the
// ml planes the Lift read (in `hi` until then) and the transposed code dot,
// one component at a time.
struct MpcliftY {
  uint64_t lo[2][2];            // [own / prev][ml planes 0, 1]
  SplitPlanes<16, 3> hi;        // the Lift's ml planes, then bits 16..31
  __device__ __forceinline__ void at(int i, uint64_t, uint64_t& bo, uint64_t& bv) const {
    if (i < 14) {
      bo = bv = 0;
    } else if (i < 16) {
      bo = i == 14 ? lo[0][0] : lo[0][1];
      bv = i == 14 ? lo[1][0] : lo[1][1];
    } else {
      hi.get(i - 16, bo, bv);
    }
  }
};

// The party a wave simulates: its wave index, made wave-uniform (a scalar
// register) so that every party-dependent choice is a scalar branch.
__device__ __forceinline__ int party_of_wave() { return __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)); }

// Lanes past the last word work on word 0 (in bounds) and store nothing.
// A lane's match word: row, word, its query's id and columns.  With a query
// table, a word at or past its query's column count is inactive (it still
// reads in-range inputs and takes part in every barrier).
struct Lane {
  bool active;
  uint64_t row, w, col0, qid;
  int nval;
};
__device__ __forceinline__ Lane lane_of(const CmpMsgArgs& a) {
  const uint64_t t = uint64_t(blockIdx.x) * 64 + (threadIdx.x & 63);
  Lane l;
  l.active = t < a.rows * a.nw;
  const uint64_t tt = l.active ? t : 0;
  l.row = tt / a.nw;
  l.w = tt % a.nw;
  l.col0 = l.w * 64;
  const uint64_t qi = l.row / uint64_t(a.r);
  uint64_t n = a.n;
  l.qid = a.qid_base + qi;
  if (a.tab) {
    l.qid = a.tab[qi].query_id;
    const uint64_t nq = min<uint64_t>(n, a.tab[qi].n);
    if (l.col0 < nq) n = nq;
    else l.active = false;
  }
  l.nval = int(min<uint64_t>(64, n - l.col0));
  return l;
}

__device__ __forceinline__ void store_match(const CmpMsgArgs& a, int p, const Lane& l, PV r) {
  if (!l.active) return;
  const uint64_t keep = l.nval == 64 ? ~0ull : ((1ull << l.nval) - 1ull);
  uint64_t* m;
  uint64_t plane;
  if (a.tab) {
    const imc_query_entry& e = a.tab[l.row / uint64_t(a.r)];
    m = e.match[p] + (l.row % uint64_t(a.r)) * a.mw_ld;
    plane = e.match_plane;
  } else {
    m = a.match[p] + l.row * a.mw_ld;
    plane = a.match_plane;
  }
  m[l.w] = r.o & keep;
  m[plane + l.w] = r.v & keep;
}

// MPCLift (Sec. 5.1-5.2): Lift ml to Z_2^32 (BitExtract m = 17 on words
// 0..33, gates 0..32; BitInject of bit 17 into Z_2^15 and of bit 16 into
// Z_2^16 on words 104.. of key_0 and 104.. / 152.. of key_2, messages at
// planes 282 and 342), y = 2^14 ml' - 2^16 dot, MSB by BitExtract m = 31 on
// words 40..101, gates 33..93.  406 message planes.
__global__ void __launch_bounds__(192) compare_msg_kernel(CmpMsgArgs a) {
  constexpr int kPlanes = 406;
  const int p = party_of_wave(), pm = (p + 2) % 3;
  const Lane l = lane_of(a);
  const bool vec_ok = (a.ld % 8) == 0;
  const uint64_t stream = row_stream(kDomCmp, l.qid, a.rot[l.row % uint64_t(a.r)]);
  const uint64_t base = ((a.first_entry >> 6) + l.w) * kTapeBlocksPerGroup;
  const Key& ko = a.keys.k[p];
  const Key& kv = a.keys.k[pm];
  const Net net = net_of(a.msg, kPlanes, l.active);
  const uint16_t* const mrow[2] = {static_cast<const uint16_t*>(a.mask[p]) + l.row * a.ld,
                                   a.prev_mask[p] + l.row * a.ld};
  const uint16_t* const drow[2] = {static_cast<const uint16_t*>(a.code[p]) + l.row * a.ld,
                                   a.prev_code[p] + l.row * a.ld};

  // Lift: bits 16 and 17 of ml_0 + ml_1 + ml_2
  PV bit16{0, 0}, bit17{0, 0};
  MpcliftY y;   // ml planes 0, 1 of both components: bits 14, 15 of y
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    uint64_t xc[16];
    uint32_t W[32];
    load64(mrow[c], l.col0, l.nval, vec_ok, W);
    to_planes(W, xc);
    y.hi.put(c, xc);
    y.lo[c][0] = xc[0];
    y.lo[c][1] = xc[1];
  }
  bit17 = msg_bit_extract<17, 0, 0>(p, ko, kv, stream, base, y.hi, net, &bit16);

  // BitInject bit 17 into Z_2^15 (A) and bit 16 into Z_2^16 (B): two rounds
  uint64_t c0A[1] = {0}, c2A[1] = {0}, c1A[1] = {0}, c0B[2] = {0, 0}, c2B[2] = {0, 0}, c1B[2] = {0, 0};
  inject_send<15, 1, 104, 104, 120, 136>(p, a.keys, stream, base, bit17, net, 282, c0A, c2A);
  inject_send<16, 2, 120, 152, 168, 184>(p, a.keys, stream, base, bit16, net, 342, c0B, c2B);
  __syncthreads();
  inject_forward<15, 1>(p, bit17, net, 282, c1A);
  inject_forward<16, 2>(p, bit16, net, 342, c1B);
  __syncthreads();
  uint64_t Ao[1], Av[1], Bo[2], Bv[2];
  inject_view<15, 1, 104, 104>(p, a.keys, stream, base, net, 282, c0A, c2A, c1A, Ao, Av);
  inject_view<16, 2, 120, 152>(p, a.keys, stream, base, net, 342, c0B, c2B, c1B, Bo, Bv);

  // bits 16..31 of y, one component at a time: component c's ml planes are
  // read back before its y planes take their place; then the MSB of y
  {
    const uint64_t a0[2] = {Ao[0], Av[0]}, b0[2] = {Bo[0], Bv[0]}, b1[2] = {Bo[1], Bv[1]};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint64_t xm[16], d[16], u[16];
      uint32_t W[32];
#pragma unroll
      for (int j = 0; j < 16; ++j) xm[j] = y.hi.plane(c, j);
      load64(drow[c], l.col0, l.nval, vec_ok, W);
      to_planes(W, d);
      mpclift_u(xm, d, a0[c], b0[c], b1[c], u);
      y.hi.put(c, u);
    }
  }
  const PV r = msg_bit_extract<31, 40, 33>(p, ko, kv, stream, base, y, net, nullptr);
  store_match(a, p, l, r);
}

// Plain Mask (Sec. 4.3 Alg. 2): component j of y is (j == 0 ? floor(ml/4) : 0)
// minus component j of the code dot over Z_2^16.
__device__ __forceinline__ void plain_y(const CmpMsgArgs& a, const Lane& l, bool vec_ok, int comp, const uint16_t* drow,
                                        uint64_t (&y)[16]) {
  uint32_t M[32], W[32];
  load64(a.ml_pub + l.row * a.ld, l.col0, l.nval, vec_ok, M);
  load64(drow, l.col0, l.nval, vec_ok, W);
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const uint32_t tl = comp == 0 ? ((M[i] & 0xFFFFu) >> 2) : 0u, th = comp == 0 ? (M[i] >> 18) : 0u;
    const uint32_t lo = (tl - (W[i] & 0xFFFFu)) & 0xFFFFu, hi = (th - (W[i] >> 16)) & 0xFFFFu;
    W[i] = lo | (hi << 16);
  }
  to_planes(W, y);
}

// Lift18: y = x - 2^17 A - 2^16 B - 4 d (mod 2^18) for one component.
__device__ __forceinline__ void lift18_y(const uint64_t (&x)[16], const uint64_t (&d)[16], uint64_t a0, uint64_t b0,
                                         uint64_t b1, uint64_t (&y)[18]) {
  uint64_t s[18];
#pragma unroll
  for (int j = 0; j < 18; ++j) {
    y[j] = j < 16 ? x[j] : 0;
    s[j] = j >= 2 ? d[j - 2] : 0;
  }
  sub_planes<18>(y, s);
#pragma unroll
  for (int j = 0; j < 18; ++j) s[j] = j == 16 ? b0 : j == 17 ? (b1 ^ a0) : 0;
  sub_planes<18>(y, s);
}

// Const32 / NoLift: y = 2^14 x - 2^16 d (mod 2^32) for one component, x over
// Z_2^32 and d over Z_2^16 or Z_2^32: bits 0..13 zero, bits 14..31 =
// t = (x - 4 d) mod 2^18, returned as the 18 planes of t.
template <bool C32>
__device__ __forceinline__ void const32_y(const uint32_t* xr, const void* drow, const Lane& l, bool vec_ok,
                                          uint64_t (&y)[18]) {
  uint32_t Wl[32];
  uint64_t h16 = 0, h17 = 0;
  const bool vec = vec_ok && l.nval == 64;
#pragma unroll
  for (int q = 0; q < 4; ++q) {   // 16 columns at a time (bounded live registers)
    uint32_t xv[16], dv[16];
    if (vec) {
      const uint4* px = reinterpret_cast<const uint4*>(xr + l.col0 + 16 * q);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint4 v = px[i];
        xv[4 * i] = v.x; xv[4 * i + 1] = v.y; xv[4 * i + 2] = v.z; xv[4 * i + 3] = v.w;
      }
      if constexpr (C32) {
        const uint4* pd = reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(drow) + l.col0 + 16 * q);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint4 v = pd[i];
          dv[4 * i] = v.x; dv[4 * i + 1] = v.y; dv[4 * i + 2] = v.z; dv[4 * i + 3] = v.w;
        }
      } else {
        const uint4* pd = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(drow) + l.col0 + 16 * q);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const uint4 v = pd[i];
          const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            dv[8 * i + 2 * j] = w[j] & 0xFFFFu;
            dv[8 * i + 2 * j + 1] = w[j] >> 16;
          }
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int c = 16 * q + k;
        xv[k] = c < l.nval ? xr[l.col0 + c] : 0u;
        dv[k] = 0;
        if (c < l.nval) {
          if constexpr (C32) dv[k] = static_cast<const uint32_t*>(drow)[l.col0 + c];
          else dv[k] = static_cast<const uint16_t*>(drow)[l.col0 + c];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 16; k += 2) {
      const int c = 16 * q + k;
      const uint32_t t0 = xv[k] - (dv[k] << 2), t1 = xv[k + 1] - (dv[k + 1] << 2);
      h16 |= (uint64_t((t0 >> 16) & 1u) << c) | (uint64_t((t1 >> 16) & 1u) << (c + 1));
      h17 |= (uint64_t((t0 >> 17) & 1u) << c) | (uint64_t((t1 >> 17) & 1u) << (c + 1));
      Wl[c >> 1] = (t0 & 0xFFFFu) | (t1 << 16);
    }
  }
  uint64_t tp[16];
  to_planes(Wl, tp);
#pragma unroll
  for (int j = 0; j < 18; ++j) y[j] = j < 16 ? tp[j] : j == 16 ? h16 : h17;
}

// The Const32 y seen from the MSB circuit: bits 0..13 zero, bits 14..31 the
// 18 planes of t.
struct Const32Y {
  SplitPlanes<18, 5> t;
  __device__ __forceinline__ void at(int i, uint64_t, uint64_t& bo, uint64_t& bv) const {
    if (i < 14) {
      bo = bv = 0;
    } else {
      t.get(i - 14, bo, bv);
    }
  }
};

// The other comparison settings (Sec. 4.3 Alg. 2, Sec. 5.1-5.2), with the
// tape words and AND-gate order of their register-mode kernels:
//   Plain    MSB m = 15 on words 0..29, gates 0..28 (87 planes)
//   Lift18   Lift m = 17 on words 0..33 (gates 0..32), BitInject of bit 17
//            into Z_2^1 (key_0 c0 word 80; key_2 c2 80, w0 81, w1 82;
//            planes 198..201) and of bit 16 into Z_2^2 (key_0 c0 88..89;
//            key_2 c2 88..89, w0 90..91, w1 92..93; planes 202..209), MSB
//            m = 17 on words 40..73 (gates 33..65) (210 planes)
//   Const32  MSB m = 31 on words 0..61, gates 0..60 (183 planes)
// Held to 168 registers (three waves per SIMD) so that four workgroups share
// a CU, as many as their LDS allows: the Const32 instances would otherwise
// take about 184 and fit two; the few registers they then spill cost less
// than the halved occupancy.
template <int V, bool C32>
__global__ void __launch_bounds__(192) __attribute__((amdgpu_waves_per_eu(3)))
compare_msg_variant_kernel(CmpMsgArgs a) {
  constexpr int kPlanes = V == 1 ? 87 : V == 2 ? 210 : 183;
  const int p = party_of_wave(), pm = (p + 2) % 3;
  const Lane l = lane_of(a);
  const bool vec_ok = a.vec != 0;
  const uint32_t dom = V == 1 ? kDomCmpPlain : V == 2 ? kDomCmpLift18 : kDomCmpConst32;
  const uint64_t stream = row_stream(dom, l.qid, a.rot[l.row % uint64_t(a.r)]);
  const uint64_t base = ((a.first_entry >> 6) + l.w) * kTapeBlocksPerGroup;
  const Key& ko = a.keys.k[p];
  const Key& kv = a.keys.k[pm];
  const Net net = net_of(a.msg, kPlanes, l.active);
  PV r;
  if constexpr (V == 1) {
    const uint16_t* drow = static_cast<const uint16_t*>(a.code[p]) + l.row * a.ld;
    SplitPlanes<16, 3> y;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint64_t yc[16];
      plain_y(a, l, vec_ok, c ? pm : p, drow + c * a.plane_elems, yc);
      y.put(c, yc);
    }
    r = msg_bit_extract<15, 0, 0>(p, ko, kv, stream, base, y, net, nullptr);
  } else if constexpr (V == 2) {
    const uint16_t* mrow = static_cast<const uint16_t*>(a.mask[p]) + l.row * a.ld;
    const uint16_t* drow = static_cast<const uint16_t*>(a.code[p]) + l.row * a.ld;
    PV bit16{0, 0}, bit17{0, 0};
    SplitPlanes<16, 3> xs;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint64_t xc[16];
      uint32_t W[32];
      load64(mrow + c * a.plane_elems, l.col0, l.nval, vec_ok, W);
      to_planes(W, xc);
      xs.put(c, xc);
    }
    bit17 = msg_bit_extract<17, 0, 0>(p, ko, kv, stream, base, xs, net, &bit16);
    uint64_t c0A[1] = {0}, c2A[1] = {0}, c1A[1] = {0}, c0B[2] = {0, 0}, c2B[2] = {0, 0}, c1B[2] = {0, 0};
    inject_send<1, 1, 80, 80, 81, 82>(p, a.keys, stream, base, bit17, net, 198, c0A, c2A);
    inject_send<2, 2, 88, 88, 90, 92>(p, a.keys, stream, base, bit16, net, 202, c0B, c2B);
    __syncthreads();
    inject_forward<1, 1>(p, bit17, net, 198, c1A);
    inject_forward<2, 2>(p, bit16, net, 202, c1B);
    __syncthreads();
    uint64_t Ao[1], Av[1], Bo[2], Bv[2];
    inject_view<1, 1, 80, 80>(p, a.keys, stream, base, net, 198, c0A, c2A, c1A, Ao, Av);
    inject_view<2, 2, 88, 88>(p, a.keys, stream, base, net, 202, c0B, c2B, c1B, Bo, Bv);
    // y over Z_2^18, one component at a time: component c's ml planes are
    // read back before its y planes take their LDS slots
    SplitPlanes<18, 5> y;
    const uint64_t a0[2] = {Ao[0], Av[0]}, b0[2] = {Bo[0], Bv[0]}, b1[2] = {Bo[1], Bv[1]};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint64_t x[16], d[16], yc[18];
      uint32_t W[32];
#pragma unroll
      for (int j = 0; j < 16; ++j) x[j] = xs.plane(c, j);
      load64(drow + c * a.plane_elems, l.col0, l.nval, vec_ok, W);
      to_planes(W, d);
      lift18_y(x, d, a0[c], b0[c], b1[c], yc);
      y.put(c, yc);
    }
    r = msg_bit_extract<17, 40, 33>(p, ko, kv, stream, base, y, net, nullptr);
  } else {
    const uint32_t* xr = static_cast<const uint32_t*>(a.mask[p]) + l.row * a.ld;
    const size_t dw = C32 ? 4 : 2;
    const uint8_t* dr = static_cast<const uint8_t*>(a.code[p]) + l.row * a.ld * dw;
    Const32Y y;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint64_t tc[18];
      const32_y<C32>(xr + c * a.plane_elems, dr + c * a.plane_elems * dw, l, vec_ok, tc);
      y.t.put(c, tc);
    }
    r = msg_bit_extract<31, 0, 0>(p, ko, kv, stream, base, y, net, nullptr);
  }
  store_match(a, p, l, r);
}

size_t compare_msg_planes(int variant) {
  switch (variant) {
    case 0: return 406;
    case 1: return 87;
    case 2: return 210;
    case 3: return 183;
    default: return 0;
  }
}

static hipError_t run_compare_msg(int variant, CmpMsgArgs& a, bool code32, hipStream_t s);

hipError_t launch_compare_msg(int variant, const Keys3& keys, const void* const rep_code[3], bool code32,
                              const void* const rep_mask[3], const uint16_t* ml_pub, uint64_t rows, uint64_t n,
                              uint64_t ld, const imc_ids_dev& ids, uint64_t* const match[3], uint64_t mw_ld,
                              uint64_t* msg, hipStream_t s, const QueryTab& qt) {
  if (rows == 0 || n == 0) return hipSuccess;
  CmpMsgArgs a;
  a.tab = qt.tab;
  a.keys = keys;
  for (int p = 0; p < 3; ++p) {
    a.code[p] = rep_code[p];
    a.mask[p] = rep_mask ? rep_mask[p] : nullptr;
    a.match[p] = match[p];
  }
  a.ml_pub = ml_pub;
  a.msg = msg;
  a.ld = ld;
  a.mw_ld = mw_ld;
  a.n = n;
  a.nw = (n + 63) / 64;
  a.rows = rows;
  a.plane_elems = (qt.plane_rows ? qt.plane_rows : rows) * ld;
  for (int p = 0; p < 3; ++p) {
    a.prev_code[p] = static_cast<const uint16_t*>(a.code[p]) + a.plane_elems;
    a.prev_mask[p] = a.mask[p] ? static_cast<const uint16_t*>(a.mask[p]) + a.plane_elems : nullptr;
  }
  a.match_plane = rows * mw_ld;
  a.qid_base = ids.query_id_base;
  a.first_entry = ids.first_entry_id;
  a.r = ids.r;
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) a.rot[i] = i < ids.r ? ids.rot[i] : 0;
  return run_compare_msg(variant, a, code32, s);
}

hipError_t launch_compare_msgs(const Keys3& keys, const uint16_t* const msgs[3], uint64_t rows, uint64_t n,
                               uint64_t ld, const imc_ids_dev& ids, uint64_t* const match[3], uint64_t mw_ld,
                               uint64_t* msg, hipStream_t s) {
  if (rows == 0 || n == 0) return hipSuccess;
  CmpMsgArgs a;
  a.tab = nullptr;
  a.keys = keys;
  const uint64_t plane = rows * ld;       // msgs[p]: [code, mask][rows][ld]
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
    a.code[p] = msgs[p];
    a.mask[p] = msgs[p] + plane;
    a.prev_code[p] = msgs[pm];
    a.prev_mask[p] = msgs[pm] + plane;
    a.match[p] = match[p];
  }
  a.ml_pub = nullptr;
  a.msg = msg;
  a.ld = ld;
  a.mw_ld = mw_ld;
  a.n = n;
  a.nw = (n + 63) / 64;
  a.rows = rows;
  a.plane_elems = plane;
  a.match_plane = rows * mw_ld;
  a.qid_base = ids.query_id_base;
  a.first_entry = ids.first_entry_id;
  a.r = ids.r;
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) a.rot[i] = i < ids.r ? ids.rot[i] : 0;
  return run_compare_msg(0, a, false, s);
}

static hipError_t run_compare_msg(int variant, CmpMsgArgs& a, bool code32, hipStream_t s) {
  const uint64_t ld = a.ld, rows = a.rows;
  const uint16_t* ml_pub = a.ml_pub;
  bool vec = (ld % 8) == 0 && (reinterpret_cast<uintptr_t>(ml_pub) % 16) == 0;
  for (int p = 0; p < 3; ++p)
    vec = vec && (reinterpret_cast<uintptr_t>(a.code[p]) % 16) == 0 && (reinterpret_cast<uintptr_t>(a.mask[p]) % 16) == 0;
  a.vec = vec ? 1 : 0;
  const uint64_t groups = (rows * a.nw + 63) / 64;
  if (groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid{unsigned(groups), 1, 1}, block{192, 1, 1};
  switch (variant) {
    case 0: hipLaunchKernelGGL(compare_msg_kernel, grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((compare_msg_variant_kernel<1, false>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((compare_msg_variant_kernel<2, false>), grid, block, 0, s, a); break;
    case 3:
      if (code32) hipLaunchKernelGGL((compare_msg_variant_kernel<3, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((compare_msg_variant_kernel<3, false>), grid, block, 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace imc
