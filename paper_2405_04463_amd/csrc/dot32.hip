// dot32.hip -- sharing and party-local dot products over Z_2^32 for the
// settings that compute ml (ConstLift) or both values (NoLift) in the larger
// ring instead of lifting them in MPC (Sec. 5.1, "Lifting vs. Larger
// Dot-Product"; Sec. 6.1: 10 i8 products instead of 3).
//
// A Z_2^32 value is four balanced byte limbs, v = b0 + 2^8 b1 + 2^16 b2 +
// 2^24 b3 (mod 2^32), b_i in [-128, 127].  Mod 2^32 only the limb products
// with i + j <= 3 survive, so an output needs four accumulators
//   acc_s = sum over i + j = s of sum_k a_i b_j      (s = 0..3, 10 products)
// and z = acc0 + 2^8 acc1 + 2^16 acc2 + 2^24 acc3.  |acc3| <= 4 * 25600 *
// 2^14 < 2^31, so no accumulator wraps.  One vector (code or mask) per region.
#include "device.h"
#include "launch.h"

namespace imc {

constexpr int kLimbs32 = 4;
constexpr size_t kPlane32Bytes = size_t(kChunks) * 32 * 16;        // one limb plane of a 32-entry block
constexpr size_t kBlock32Bytes = kLimbs32 * kPlane32Bytes;         // 3,276,800: 102,400 B per entry
constexpr size_t kQop32RowBytes = size_t(kLimbs32) * kK;           // 102,400 per query

__device__ __forceinline__ void limbs32(uint32_t v, int8_t b[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int l = int(int8_t(v & 0xFFu));
    b[i] = int8_t(l);
    v = (v - uint32_t(l)) >> 8;
  }
}

// Encoded element i of a vector: the masked bit m - 2 (c AND m) (code) or
// the mask bit (mask), as a Z_2^32 value.
__device__ __forceinline__ uint32_t encode32(const uint64_t* code, const uint64_t* mask, int vec, int i) {
  const uint32_t c = uint32_t(code[i >> 6] >> (i & 63)) & 1u, m = uint32_t(mask[i >> 6] >> (i & 63)) & 1u;
  return vec ? m : m - 2u * (c & m);
}

// Dealer components of 16 consecutive elements 16g..16g+15 of vector vec of
// the item with id `id`: comp0, comp1 from the PRF (one block each), comp2 =
// x - comp0 - comp1.
__device__ __forceinline__ void share16x32(const Key& dk, uint32_t dom, int vec, uint64_t id, const uint64_t* code,
                                           const uint64_t* mask, int g, uint32_t c[3][16]) {
  chacha12(dk, share_stream(dom, vec, 0, id), uint64_t(g), c[0]);
  chacha12(dk, share_stream(dom, vec, 1, id), uint64_t(g), c[1]);
#pragma unroll
  for (int j = 0; j < 16; ++j) c[2][j] = encode32(code, mask, vec, 16 * g + j) - c[0][j] - c[1][j];
}

// 16 values -> 16 bytes of each of the four limb planes.
__device__ __forceinline__ void limb_rows(const uint32_t v[16], uint4 out[4]) {
  uint32_t w[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int l = 0; l < 4; ++l) w[l][q] = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    int8_t b[4];
    limbs32(v[j], b);
#pragma unroll
    for (int l = 0; l < 4; ++l) w[l][j >> 2] |= uint32_t(uint8_t(b[l])) << (8 * (j & 3));
  }
#pragma unroll
  for (int l = 0; l < 4; ++l) out[l] = make_uint4(w[l][0], w[l][1], w[l][2], w[l][3]);
}

// Database: party p's region of vector vec, entry e in block e/32 slot e%32,
// k-chunk g holds x_p[16g..], k-chunk 800 + g holds x_{p-1}[16g..].  Thread
// layout: 32 consecutive entries (one block) per 32 lanes, then g, so that a
// wave's stores of one limb plane and k-chunk are 512 contiguous bytes.
__global__ void __launch_bounds__(256) share32_db_kernel(Key dk, int vec, const uint64_t* codes, const uint64_t* masks,
                                                         uint64_t n, uint64_t first, uint8_t* d0, uint8_t* d1,
                                                         uint8_t* d2) {
  constexpr uint32_t kGroups = kCodeBits / 16;   // 800
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint64_t chunk = t / (32 * kGroups);
  const uint32_t within = uint32_t(t % (32 * kGroups));
  const int g = int(within / 32);
  const uint64_t j = chunk * 32 + within % 32;
  if (j >= n) return;
  const uint64_t e = first + j;
  uint32_t c[3][16];
  share16x32(dk, kDomShare32Db, vec, e, codes + j * kWords, masks + j * kWords, g, c);
  uint4 lr[3][4];
#pragma unroll
  for (int p = 0; p < 3; ++p) limb_rows(c[p], lr[p]);
  uint8_t* const d[3] = {d0, d1, d2};
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    if (!d[p]) continue;
    const int pm = (p + 2) % 3;
    uint8_t* blk = d[p] + (e / 32) * kBlock32Bytes + (e % 32) * 16;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      *reinterpret_cast<uint4*>(blk + l * kPlane32Bytes + size_t(g) * 512) = lr[p][l];
      *reinterpret_cast<uint4*>(blk + l * kPlane32Bytes + size_t(kCodeBits / 16 + g) * 512) = lr[pm][l];
    }
  }
}

// Query operand: party p's row [limb 4][25600], k < 12800 holding x_p + x_{p-1},
// k >= 12800 holding x_p (the query-side preprocessing of the replicated dot).
__global__ void __launch_bounds__(256) share32_query_kernel(Key dk, int vec, const uint64_t* codes,
                                                            const uint64_t* masks, uint64_t q, uint64_t qid_base,
                                                            int8_t* o0, int8_t* o1, int8_t* o2) {
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= q * (kCodeBits / 16)) return;
  const uint64_t qi = t / (kCodeBits / 16);
  const int g = int(t % (kCodeBits / 16));
  uint32_t c[3][16];
  share16x32(dk, kDomShare32Query, vec, qid_base + qi, codes + qi * kWords, masks + qi * kWords, g, c);
  int8_t* const o[3] = {o0, o1, o2};
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
    uint32_t sum[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) sum[j] = c[p][j] + c[pm][j];
    uint4 ls[4], lo[4];
    limb_rows(sum, ls);
    limb_rows(c[p], lo);
    int8_t* row = o[p] + qi * kQop32RowBytes;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      *reinterpret_cast<uint4*>(row + l * kK + 16 * g) = ls[l];
      *reinterpret_cast<uint4*>(row + l * kK + kCodeBits + 16 * g) = lo[l];
    }
  }
}

// ---------------------------------------------------------------------------
// Dot kernel over Z_2^32.  Workgroup: 4 waves, tile 128 rows x 64 entries;
// wave w owns rows 32w..32w+31 and both 32-entry blocks.  Operands go from
// global memory straight to registers, one K-step (32 k) ahead: the query
// fragment of a lane is 16 consecutive elements of its rotated row, read as
// four dwords at rotated offsets (a rotation by s moves 4s elements inside
// an 800-element angular row), the database fragment one 16-byte chunk of
// the tiled region per limb.
// ---------------------------------------------------------------------------
struct Dot32Args {
  const int8_t* qop;
  const int8_t* b;
  uint32_t* out;
  uint64_t ld;
  uint32_t rows, r;
  uint64_t b_block0, b_blocks, n;
  uint32_t mt, nt;
  int8_t rot[IMC_MAX_ROT_DEV];
};

struct Frag32 {
  v4i a[4];        // query limbs
  v4i b[2][4];     // entry blocks x limbs
};

__device__ __forceinline__ void load_frag32(Frag32& f, const int8_t* qrow, int s, bool row_ok, const int8_t* const bsrc[2],
                                            int kt, int lane) {
  const int k0 = 32 * kt + 16 * (lane >> 5);
  const int h = k0 >= kCodeBits ? 1 : 0;
  const int i0 = k0 - h * kCodeBits;
  const int arow = i0 / kRowLen, w0 = i0 - arow * kRowLen;
  const int8_t* base = qrow + h * kCodeBits + arow * kRowLen;
  int off[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int w = w0 + 4 * j - 4 * s;
    w += w < 0 ? kRowLen : 0;
    w -= w >= kRowLen ? kRowLen : 0;
    off[j] = w;
  }
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    if (row_ok) {
      const int8_t* p = base + l * kK;
      f.a[l] = v4i{*reinterpret_cast<const int*>(p + off[0]), *reinterpret_cast<const int*>(p + off[1]),
                   *reinterpret_cast<const int*>(p + off[2]), *reinterpret_cast<const int*>(p + off[3])};
    } else {
      f.a[l] = v4i{0, 0, 0, 0};
    }
  }
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int l = 0; l < 4; ++l)
      f.b[y][l] = *reinterpret_cast<const v4i*>(bsrc[y] + l * kPlane32Bytes + size_t(2 * kt) * 512);
}

__device__ __forceinline__ void mfma32(v16i (&acc)[4][2], const Frag32& f) {
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j + i < 4; ++j)
        acc[i + j][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[i], f.b[y][j], acc[i + j][y], 0, 0, 0);
}

__global__ void __launch_bounds__(256) dot32_kernel(Dot32Args args) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t i = blockIdx.x, xcd = i & 7, s8 = i >> 3;
  const uint32_t u = s8 % args.mt, t = (s8 / args.mt) * 8 + xcd;
  if (t >= args.nt) return;
  const uint32_t row = u * 128 + wave * 32 + (lane & 31);
  const bool row_ok = row < args.rows;
  const int8_t* qrow = args.qop;
  int s = 0;
  if (row_ok) {
    qrow = args.qop + size_t(row / args.r) * kQop32RowBytes;
    s = args.rot[row % args.r];
  }
  const int8_t* bsrc[2];
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    uint64_t cb = uint64_t(t) * 2 + y;
    cb = cb < args.b_blocks ? cb : args.b_blocks - 1;
    bsrc[y] = args.b + size_t(args.b_block0 + cb) * kBlock32Bytes + size_t(lane >> 5) * 512 + (lane & 31) * 16;
  }
  v16i acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][y][e] = 0;

  constexpr int kSteps = kChunks / 2;   // 800 steps of 32 k
  Frag32 f0, f1;
  load_frag32(f0, qrow, s, row_ok, bsrc, 0, lane);
  for (int kt = 0; kt < kSteps; kt += 2) {
    load_frag32(f1, qrow, s, row_ok, bsrc, kt + 1, lane);
    mfma32(acc, f0);
    if (kt + 2 < kSteps) load_frag32(f0, qrow, s, row_ok, bsrc, kt + 2, lane);
    mfma32(acc, f1);
  }

  // lane l holds column l%32, register e row 8(e/4) + 4(l/32) + e%4 of a block
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const uint64_t col = uint64_t(t) * 64 + 32 * y + (lane & 31);
    if (col >= args.n) continue;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const uint32_t rr = u * 128 + wave * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      if (rr < args.rows) {
        const uint32_t z = uint32_t(acc[0][y][e]) + (uint32_t(acc[1][y][e]) << 8) + (uint32_t(acc[2][y][e]) << 16) +
                           (uint32_t(acc[3][y][e]) << 24);
        args.out[uint64_t(rr) * args.ld + col] = z;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Rotation-aware dot kernel over Z_2^32 (r >= 13 rotations per query).  A
// row tile of kBM (query, rotation) rows holds only ceil(kBM / r) + 1
// distinct queries, so the workgroup keeps each tile query's bytes of the
// current 800-byte angular-row segment in LDS (four limb planes, circular
// padding as in the Z_2^16 kernel) and every lane reads its rotated fragment
// in place; the database tile streams through three LDS stages, one K-step
// per stage.  Database data is loaded NSETS steps ahead into registers; the
// next query segment is loaded during the current one and stored half-way
// through it into the other of two A buffers.  A wave's tile of WM x WN
// 32 x 32 blocks needs 64 WM WN accumulator registers (four limb sums), so
// tiles stay small: two waves per SIMD at 32 x 64.
// ---------------------------------------------------------------------------
struct RotDot32Args {
  const int8_t* qop;     // [q][limb 4][25600]
  const int8_t* b;       // party's Z_2^32 region of the vector
  uint32_t* out;
  uint64_t ld;
  uint32_t rows, q, r;
  uint64_t b_block0, b_blocks, n;
  uint32_t mt, nt;
  uint32_t max_q;        // query slots per tile (LDS sizing)
  int8_t rot[IMC_MAX_ROT_DEV];
};

template <int WM, int WN, int WAVES_M, int WAVES_N, int NSETS, int ACH>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N) rot_dot32_kernel(RotDot32Args args) {
  constexpr int kBM = 32 * WM * WAVES_M, kBN = 32 * WN * WAVES_N;
  constexpr int kThreads = 64 * WAVES_M * WAVES_N;
  constexpr int kBBlk = kBN / 32;
  constexpr int kBChunks = kBBlk * kLimbs32 * 2 * 32;          // 16-byte chunks per K-step
  constexpr int kBPerThread = kBChunks / kThreads;
  constexpr int kBStage = kBChunks * 16;
  constexpr int kSlotBytes = kLimbs32 * kSegBytes;              // one query's segment, four limbs
  static_assert(kBChunks % kThreads == 0, "B chunks must divide evenly");
  extern __shared__ __align__(16) int8_t lds[];
  int8_t* bst = lds;                                            // 3 B stages
  int8_t* ast = lds + 3 * kBStage;                              // 2 A segment buffers
  const uint32_t abuf = args.max_q * kSlotBytes;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  const uint32_t i = blockIdx.x, xcd = i & 7, s8 = i >> 3;
  const uint32_t u = s8 % args.mt, t = (s8 / args.mt) * 8 + xcd;
  if (t >= args.nt) return;

  const uint32_t m0 = u * kBM;
  const uint32_t q_lo = m0 / args.r;
  const uint32_t last_row = min(m0 + kBM, args.rows) - 1;
  const uint32_t nq = last_row / args.r - q_lo + 1;             // <= max_q

  // byte offset of this lane's rotated fragment (limb 0) in an A buffer
  int a_off[WM];
#pragma unroll
  for (int x = 0; x < WM; ++x) {
    const uint32_t row = m0 + (wm * WM + x) * 32 + (lane & 31);
    int slot = 0, sft = 0;
    if (row < args.rows) {
      slot = int(row / args.r - q_lo);
      sft = 4 * args.rot[row % args.r];
    }
    a_off[x] = slot * kSlotBytes + kSegPad - sft + 16 * (lane >> 5);
  }

  // B chunk c of a stage = (block, limb, k-chunk of the step, slot) at byte 16 c
  const int8_t* bsrc[kBPerThread];
#pragma unroll
  for (int j = 0; j < kBPerThread; ++j) {
    const int c = tid + j * kThreads;
    const int blk = c >> 8, rem = c & 255;
    const int limb = rem >> 6, kcl = (rem >> 5) & 1, slot = rem & 31;
    uint64_t cb = uint64_t(t) * kBBlk + blk;
    cb = cb < args.b_blocks ? cb : args.b_blocks - 1;
    bsrc[j] = args.b + size_t(args.b_block0 + cb) * kBlock32Bytes + size_t(limb) * kPlane32Bytes + size_t(kcl) * 512 +
              slot * 16;
  }
  // A chunk c of a segment buffer = (query slot, limb, 16-byte piece)
  const int a_chunks = int(nq) * kLimbs32 * kSegChunks;
  const int8_t* asrc[ACH];
  int adst[ACH];
#pragma unroll
  for (int j = 0; j < ACH; ++j) {
    int c = tid + j * kThreads;
    const bool ok = c < a_chunks;
    c = ok ? c : 0;
    const int qs = c / (kLimbs32 * kSegChunks), rem = c % (kLimbs32 * kSegChunks);
    const int limb = rem / kSegChunks, piece = rem % kSegChunks;
    const int src_off = ((piece * 16 - kSegPad) % kRowLen + kRowLen) % kRowLen;   // circular
    asrc[j] = args.qop + size_t(q_lo + qs) * kQop32RowBytes + size_t(limb) * kK + src_off;
    adst[j] = ok ? (qs * kSlotBytes + limb * kSegBytes + piece * 16) : -1;
  }

  v16i acc[4][WM][WN];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int x = 0; x < WM; ++x)
#pragma unroll
      for (int y = 0; y < WN; ++y)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[a][x][y][e] = 0;

  constexpr int kSteps = kChunks / 2;         // 800 steps of 32 k
  constexpr int kSegSteps = kRowLen / 32;     // 25 per segment
  constexpr int kSegs = kSteps / kSegSteps;   // 32
  static_assert(kSteps % NSETS == 0, "the K loop is unrolled by NSETS");
  v4i rs[NSETS][kBPerThread];
  v4i ra[ACH];

#define IMC_BLOAD(R, KS)                                                              \
  _Pragma("unroll") for (int c_ = 0; c_ < kBPerThread; ++c_)                          \
      R[c_] = *reinterpret_cast<const v4i*>(bsrc[c_] + size_t(2 * (KS)) * 512);
#define IMC_BSTORE(R, STAGE)                                                          \
  _Pragma("unroll") for (int c_ = 0; c_ < kBPerThread; ++c_)                          \
      *reinterpret_cast<v4i*>(bst + (STAGE) * kBStage + (tid + c_ * kThreads) * 16) = R[c_];
#define IMC_ALOAD(SEG)                                                                \
  _Pragma("unroll") for (int c_ = 0; c_ < ACH; ++c_)                                  \
      ra[c_] = *reinterpret_cast<const v4i*>(asrc[c_] + size_t(SEG) * kRowLen);
#define IMC_ASTORE(BUF)                                                               \
  _Pragma("unroll") for (int c_ = 0; c_ < ACH; ++c_)                                  \
      if (adst[c_] >= 0) *reinterpret_cast<v4i*>(ast + (BUF) * abuf + adst[c_]) = ra[c_];
#define IMC_AFRAGS(FA, K)                                                             \
  {                                                                                   \
    const int kk_ = (K);                                                              \
    const int seg_ = kk_ / kSegSteps, ts_ = kk_ - seg_ * kSegSteps;                   \
    const int8_t* sa_ = ast + (seg_ & 1) * abuf + 32 * ts_;                           \
    _Pragma("unroll") for (int x_ = 0; x_ < WM; ++x_)                                 \
    _Pragma("unroll") for (int l_ = 0; l_ < kLimbs32; ++l_) {                         \
      const int32_t* pa_ = reinterpret_cast<const int32_t*>(sa_ + a_off[x_] + l_ * kSegBytes); \
      FA[x_][l_] = v4i{pa_[0], pa_[1], pa_[2], pa_[3]};                               \
    }                                                                                 \
  }
#define IMC_BFRAGS(FB, Y, K)                                                          \
  _Pragma("unroll") for (int l_ = 0; l_ < kLimbs32; ++l_)                             \
    FB[l_] = *reinterpret_cast<const v4i*>(bst + ((K) % 3) * kBStage +                \
                                           ((wn * WN + (Y)) * kLimbs32 + l_) * 1024 + lane * 16);

  // prologue: A segment 0; B steps 0 and 1 in stages 0 and 1; steps 2.. in registers
  IMC_ALOAD(0)
  IMC_ASTORE(0)
  {
    v4i r0[kBPerThread];
    IMC_BLOAD(r0, 0)
    IMC_BSTORE(r0, 0)
    IMC_BLOAD(r0, 1)
    IMC_BSTORE(r0, 1)
  }
#pragma unroll
  for (int set = 0; set < NSETS; ++set) { IMC_BLOAD(rs[set], set + 2) }
  IMC_ALOAD(1)
  __syncthreads();
  // Query fragments are double-buffered (read one step ahead); database
  // fragments of column block y are re-read for the next step right after
  // the MFMAs of block y have been issued.
  v4i fa[WM][kLimbs32], na[WM][kLimbs32], fb[WN][kLimbs32];
  IMC_AFRAGS(fa, 0)
#pragma unroll
  for (int y = 0; y < WN; ++y) { IMC_BFRAGS(fb[y], y, 0) }

  // Stage (k+2)%3 is overwritten at step k: it held step k-1, whose
  // fragments were read during step k-2 and consumed before the barrier that
  // ends step k-1.
  for (int k0 = 0; k0 < kSteps; k0 += NSETS) {
#pragma unroll
    for (int uu = 0; uu < NSETS; ++uu) {
      const int k = k0 + uu;
      const int seg = k / kSegSteps, ts = k - seg * kSegSteps;
      const int kn = min(k + 1, kSteps - 1);
      IMC_AFRAGS(na, kn)
#pragma unroll
      for (int y = 0; y < WN; ++y) {
#pragma unroll
        for (int x = 0; x < WM; ++x)
#pragma unroll
          for (int ia = 0; ia < kLimbs32; ++ia)
#pragma unroll
            for (int jb = 0; ia + jb < kLimbs32; ++jb)
              acc[ia + jb][x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[x][ia], fb[y][jb], acc[ia + jb][x][y],
                                                                         0, 0, 0);
        IMC_BFRAGS(fb[y], y, kn)
      }
      IMC_BSTORE(rs[uu], (k + 2) % 3)
      if (ts == kSegSteps / 2 && seg + 1 < kSegs) {
        IMC_ASTORE((seg + 1) & 1)
        IMC_ALOAD(min(seg + 2, kSegs - 1))
      }
      __syncthreads();
      IMC_BLOAD(rs[uu], min(k + 2 + NSETS, kSteps - 1))
#pragma unroll
      for (int x = 0; x < WM; ++x)
#pragma unroll
        for (int l = 0; l < kLimbs32; ++l) fa[x][l] = na[x][l];
    }
  }
#undef IMC_AFRAGS
#undef IMC_BFRAGS
#undef IMC_BLOAD
#undef IMC_BSTORE
#undef IMC_ALOAD
#undef IMC_ASTORE

#pragma unroll
  for (int x = 0; x < WM; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y) {
      const uint64_t col = uint64_t(t) * kBN + (wn * WN + y) * 32 + (lane & 31);
      if (col >= args.n) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const uint32_t row = m0 + (wm * WM + x) * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (row < args.rows) {
          const uint32_t z = uint32_t(acc[0][x][y][e]) + (uint32_t(acc[1][x][y][e]) << 8) +
                             (uint32_t(acc[2][x][y][e]) << 16) + (uint32_t(acc[3][x][y][e]) << 24);
          args.out[uint64_t(row) * args.ld + col] = z;
        }
      }
    }
}

template <int WM, int WN, int WAVES_M, int WAVES_N, int NSETS, int ACH>
static hipError_t launch_rot_dot32(const int8_t* qop, uint32_t q, uint32_t r, const int8_t* rot, const int8_t* b,
                                   uint64_t first_entry, uint64_t n, uint32_t* out, uint64_t ld, hipStream_t s) {
  constexpr int kBM = 32 * WM * WAVES_M, kBN = 32 * WN * WAVES_N, kThreads = 64 * WAVES_M * WAVES_N;
  RotDot32Args d;
  d.qop = qop;
  d.b = b;
  d.out = out;
  d.ld = ld;
  d.rows = q * r;
  d.q = q;
  d.r = r;
  d.b_block0 = first_entry / 32;
  d.b_blocks = (n + 31) / 32;
  d.n = n;
  d.mt = (d.rows + kBM - 1) / kBM;
  d.nt = uint32_t((n + kBN - 1) / kBN);
  d.max_q = (kBM + r - 1) / r + 1;
  if (int(d.max_q) * kLimbs32 * kSegChunks > ACH * kThreads) return hipErrorInvalidValue;
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) d.rot[i] = i < int(r) ? rot[i] : 0;
  const uint64_t groups = uint64_t((d.nt + 7) / 8) * 8 * d.mt;
  if (groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const size_t lds = 3 * size_t(kBN / 32) * kLimbs32 * 2 * 32 * 16 + 2 * size_t(d.max_q) * kLimbs32 * kSegBytes;
  auto kern = rot_dot32_kernel<WM, WN, WAVES_M, WAVES_N, NSETS, ACH>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(unsigned(groups)), dim3(kThreads), lds, s, d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Resharing over Z_2^32 (App. C): z_p + F(key_p) - F(key_{p-1}), stream
// (DOM_RESHARE32, qid, rot), block entry >> 3, word 2 (entry & 7) + vec.
// One thread: 8 consecutive entries of one row.
// ---------------------------------------------------------------------------
struct Reshare32Args {
  Keys3 keys;
  const uint32_t* add[3];
  uint32_t* msg[3];     // [rows][ld]
  uint32_t* rep[3];     // [2][rows][ld]
  uint64_t ld, n, rows, plane, qid_base, first_entry;
  int32_t r, vec;
  int32_t wide;         // every row offset 16-byte aligned: 8 values move as two 16-byte accesses
  int8_t rot[IMC_MAX_ROT_DEV];
};

__device__ __forceinline__ void ld8u32(const uint32_t* p, int nval, bool wide, uint32_t v[8]) {
  if (wide && nval == 8) {
    const uint4 x = reinterpret_cast<const uint4*>(p)[0], y = reinterpret_cast<const uint4*>(p)[1];
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = j < nval ? p[j] : 0u;
  }
}

__device__ __forceinline__ void st8u32(uint32_t* p, int nval, bool wide, const uint32_t v[8]) {
  if (wide && nval == 8) {
    reinterpret_cast<uint4*>(p)[0] = make_uint4(v[0], v[1], v[2], v[3]);
    reinterpret_cast<uint4*>(p)[1] = make_uint4(v[4], v[5], v[6], v[7]);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < nval) p[j] = v[j];
  }
}

__global__ void __launch_bounds__(256) reshare32_kernel(Reshare32Args a) {
  const uint64_t nc = (a.n + 7) / 8;
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.rows * nc) return;
  const uint64_t row = t / nc, c = t % nc;
  const uint64_t qid = a.qid_base + row / uint64_t(a.r);
  const uint64_t stream = row_stream(kDomReshare32, qid, a.rot[row % uint64_t(a.r)]);
  const uint64_t e0 = a.first_entry + 8 * c;
  uint32_t F[3][16];
  {
    const Key* const ks[3] = {&a.keys.k[0], &a.keys.k[1], &a.keys.k[2]};
    const uint64_t st[3] = {stream, stream, stream}, ps[3] = {e0 >> 3, e0 >> 3, e0 >> 3};
    chacha12_n<3>(ks, st, ps, F);
  }
  const int nval = int(min<uint64_t>(8, a.n - 8 * c));
  const uint64_t off = row * a.ld + 8 * c;
  const bool wide = a.wide != 0;
  uint32_t z[3][8], G[3][8];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    ld8u32(a.add[p] + off, nval, wide, z[p]);
#pragma unroll
    for (int j = 0; j < 8; ++j) G[p][j] = a.vec ? F[p][2 * j + 1] : F[p][2 * j];
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
    uint32_t own[8], prev[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      own[j] = z[p][j] + G[p][j] - G[pm][j];
      prev[j] = z[pm][j] + G[pm][j] - G[(pm + 2) % 3][j];
    }
    st8u32(a.msg[p] + off, nval, wide, own);                  // party p -> party p+1
    st8u32(a.rep[p] + off, nval, wide, own);
    st8u32(a.rep[p] + a.plane + off, nval, wide, prev);      // received from party p-1
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_share32_db(const Key& dk, int vec, const uint64_t* codes, const uint64_t* masks, uint64_t n,
                             uint64_t first, uint8_t* const db[3], hipStream_t s) {
  const uint64_t threads = (n + 31) / 32 * 32 * (kCodeBits / 16);
  if (threads == 0) return hipSuccess;
  if ((threads + 255) / 256 > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(share32_db_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, dk, vec, codes, masks,
                     n, first, db[0], db[1], db[2]);
  return hipGetLastError();
}

hipError_t launch_share32_query(const Key& dk, int vec, const uint64_t* codes, const uint64_t* masks, uint64_t q,
                                uint64_t qid_base, int8_t* const op[3], hipStream_t s) {
  const uint64_t threads = q * (kCodeBits / 16);
  if (threads == 0) return hipSuccess;
  if ((threads + 255) / 256 > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(share32_query_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, dk, vec, codes,
                     masks, q, qid_base, op[0], op[1], op[2]);
  return hipGetLastError();
}

hipError_t launch_dot32(const int8_t* qop, uint32_t q, uint32_t r, const int8_t* rot, const int8_t* b,
                        uint64_t first_entry, uint64_t n, uint32_t* out, uint64_t ld, hipStream_t s) {
  const uint32_t rows = q * r;
  if (rows == 0 || n == 0) return hipSuccess;
  // rotation-aware tiles of 128 x 128 (8 waves of 32 x 64) when the tile's
  // queries fit the A staging (3 chunks per thread: r >= 26; 5: r >= 13)
  if (r >= 26) return launch_rot_dot32<1, 2, 4, 2, 2, 3>(qop, q, r, rot, b, first_entry, n, out, ld, s);
  if (r >= 13) return launch_rot_dot32<1, 2, 4, 2, 2, 5>(qop, q, r, rot, b, first_entry, n, out, ld, s);
  Dot32Args d;
  d.qop = qop;
  d.b = b;
  d.out = out;
  d.ld = ld;
  d.rows = rows;
  d.r = r;
  d.b_block0 = first_entry / 32;
  d.b_blocks = (n + 31) / 32;
  d.n = n;
  d.mt = (rows + 127) / 128;
  d.nt = uint32_t((n + 63) / 64);
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) d.rot[i] = i < int(r) ? rot[i] : 0;
  const uint64_t groups = uint64_t((d.nt + 7) / 8) * 8 * d.mt;
  if (groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dot32_kernel, dim3(unsigned(groups)), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_reshare32(const Keys3& keys, int vec, const uint32_t* const add[3], uint64_t rows, uint64_t n,
                            uint64_t ld, const imc_ids_dev& ids, uint32_t* const msg[3], uint32_t* const rep[3],
                            hipStream_t s) {
  if (rows == 0 || n == 0) return hipSuccess;
  Reshare32Args a;
  a.keys = keys;
  for (int p = 0; p < 3; ++p) {
    a.add[p] = add[p];
    a.msg[p] = msg[p];
    a.rep[p] = rep[p];
  }
  a.ld = ld;
  a.n = n;
  a.rows = rows;
  a.plane = rows * ld;
  a.qid_base = ids.query_id_base;
  a.first_entry = ids.first_entry_id;
  a.r = ids.r;
  a.vec = vec;
  bool wide = ld % 4 == 0;
  for (int p = 0; p < 3; ++p)
    wide = wide && (reinterpret_cast<uintptr_t>(add[p]) | reinterpret_cast<uintptr_t>(msg[p]) |
                    reinterpret_cast<uintptr_t>(rep[p])) % 16 == 0;
  a.wide = wide ? 1 : 0;
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) a.rot[i] = i < ids.r ? ids.rot[i] : 0;
  const uint64_t threads = rows * ((n + 7) / 8);
  if ((threads + 255) / 256 > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reshare32_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

size_t db32_bytes(uint64_t capacity) { return size_t((capacity + 31) / 32) * kBlock32Bytes; }
size_t query32_op_bytes(uint64_t q) { return size_t(q) * kQop32RowBytes; }

}  // namespace imc
