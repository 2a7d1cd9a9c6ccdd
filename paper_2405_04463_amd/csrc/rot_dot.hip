// rot_dot.hip -- rotation-aware variant of the party-local dot products
// (Alg. 3; App. C).  Same arithmetic as the expanded kernel (balanced byte
// limbs, i8 MFMA with i32 accumulation, three products into two
// accumulators); the query rotations (Sec. 3: circular shifts of the
// angular axis, party-local because sharing is elementwise) are applied
// while reading the query operand from LDS instead of being materialised.
#include <algorithm>

#include "device.h"
#include "launch.h"

namespace imc {

// ---------------------------------------------------------------------------
// Rotation-aware dot kernel.  Rows are (query, rotation) pairs, so a 256-row
// tile holds only ceil(256/R) + 1 distinct queries.  The K loop walks the 32
// angular-row segments of 800 bytes (16 rows x 2 halves); for each segment the
// workgroup keeps every tile query's bytes of that segment in LDS with 64
// bytes of circular padding on both sides (928 B per plane), and a lane reads
// its rotated fragment directly: rotation s shifts the segment by 4s bytes,
// so the 16 bytes at (32t + 16g - 4s) are four aligned dword reads.  Only the
// database operand streams through LDS per K-step.  Query segments are loaded
// into registers one segment ahead and written into the other of two LDS
// buffers half-way through the current segment.
// ---------------------------------------------------------------------------
struct RotDotArgs {
  const int8_t* qop;     // unrotated query operand, row-major [q][plane 4][K]
  const uint32_t* qidx;  // optional: query i of the call is operand row qidx[i]
  const int8_t* b;       // party's database region
  uint16_t* out[2];
  uint64_t ld;
  uint32_t rows, q, r;
  uint64_t b_block0, b_blocks, n;
  uint32_t mt, nt;
  uint32_t max_q;        // query slots per tile (LDS sizing)
  int8_t rot[IMC_MAX_ROT_DEV];
};

// Waits and barriers with explicit counts (the kernels below keep copies and
// reads in flight across them).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  // gfx9 s_waitcnt: vmcnt bits 3:0 and 15:14, expcnt 6:4 (7 = no wait), lgkmcnt 11:8 (15 = no wait)
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Wait for every outstanding LDS read (and nothing else).
__device__ __forceinline__ void wait_lds() {
  __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4) | (0 << 8));
}

__device__ __forceinline__ void bar() {
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ void copy16(const int8_t* g, int8_t* l) {
  __builtin_amdgcn_global_load_lds(static_cast<const void*>(g), (__attribute__((address_space(3))) void*)(l), 16, 0,
                                   0);
}

// What one output tile of the rotation-aware kernel reads and writes: the
// call's (or group's) unrotated query operand, its rotation list, the
// database region and the output plane of vector `vec`.
struct RotTile {
  const int8_t* qop;
  const uint32_t* qidx;
  const int8_t* b;
  uint16_t* out;
  const int8_t* rot;
  uint64_t ld, b_block0, b_blocks, n;
  uint32_t rows, r, max_q;
};

// One 256 x 128 output tile (row tile u, column tile t) of vector `vec`,
// the whole K loop and the epilogue.  LDS: 3 database stages, then the two
// query segment buffers of max_q slots.
template <int K, int WM, int WN, int WAVES_M, int WAVES_N, int NSETS, int ACH>
__device__ __forceinline__ void rot_dot_tile(const RotTile& args, uint32_t u, uint32_t t, int vec, int8_t* lds) {
  using G = Geo<K>;
  constexpr int kBM = 32 * WM * WAVES_M, kBN = 32 * WN * WAVES_N;
  constexpr int kThreads = 64 * WAVES_M * WAVES_N;
  constexpr int kBBlk = kBN / 32;
  constexpr int kBChunks = kBBlk * 2 * 2 * 32;                 // per K-step
  constexpr int kBPerThread = kBChunks / kThreads;
  constexpr int kBStage = kBChunks * 16;
  static_assert(kBChunks % kThreads == 0, "B chunks must divide evenly");
  int8_t* bst = lds;                                           // 3 B stages
  int8_t* ast = lds + 3 * kBStage;                             // 2 A segment buffers
  const uint32_t abuf = args.max_q * 2 * kSegBytes;            // bytes per A buffer

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;

  const uint32_t m0 = u * kBM;
  const uint32_t q_lo = m0 / args.r;
  const uint32_t last_row = min(m0 + kBM, args.rows) - 1;
  const uint32_t nq = last_row / args.r - q_lo + 1;            // <= max_q

  // Per-lane A fragment offsets (bytes into an A buffer) for its row-blocks.
  int a_off[WM];
#pragma unroll
  for (int x = 0; x < WM; ++x) {
    const uint32_t row = m0 + (wm * WM + x) * 32 + (lane & 31);
    int slot = 0, sft = 0;
    if (row < args.rows) {
      slot = int(row / args.r - q_lo);
      sft = 4 * args.rot[row % args.r];
    }
    a_off[x] = slot * 2 * kSegBytes + kSegPad - sft + 16 * (lane >> 5);
  }

  // B staging sources (database tile), as in dot_kernel.
  const int8_t* bsrc[kBPerThread];
#pragma unroll
  for (int j = 0; j < kBPerThread; ++j) {
    const int c = tid + j * kThreads;
    const int blk = c >> 7, rem = c & 127;
    const int plane = rem >> 6, kcl = (rem >> 5) & 1, slot = rem & 31;
    uint64_t cb = uint64_t(t) * kBBlk + blk;
    cb = cb < args.b_blocks ? cb : args.b_blocks - 1;
    bsrc[j] = args.b + size_t(args.b_block0 + cb) * G::kBlockBytes + size_t(2 * vec + plane) * G::kPlaneBlockBytes +
              size_t(kcl) * 512 + slot * 16;
  }
  // A staging: chunk c of a segment buffer = (query slot, plane, 16-byte piece).
  const int a_chunks = int(nq) * 2 * kSegChunks;
  const int8_t* asrc[ACH];
  int adst[ACH];
#pragma unroll
  for (int j = 0; j < ACH; ++j) {
    int c = tid + j * kThreads;
    const bool ok = c < a_chunks;
    c = ok ? c : 0;
    const int qs = c / (2 * kSegChunks), rem = c % (2 * kSegChunks);
    const int pl = rem / kSegChunks, piece = rem % kSegChunks;
    const int src_off = ((piece * 16 - kSegPad) % kRowLen + kRowLen) % kRowLen;   // circular
    const uint32_t qrow = args.qidx ? args.qidx[q_lo + qs] : q_lo + qs;
    asrc[j] = args.qop + size_t(qrow) * G::kQopRowBytes + size_t(2 * vec + pl) * G::kK + src_off;
    adst[j] = ok ? (qs * 2 * kSegBytes + pl * kSegBytes + piece * 16) : -1;
  }

  v16i acc0[WM][WN], acc1[WM][WN];
#pragma unroll
  for (int x = 0; x < WM; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) { acc0[x][y][e] = 0; acc1[x][y][e] = 0; }

  constexpr int kSteps = G::kChunks / 2;        // 800 or 400
  constexpr int kSegSteps = kRowLen / 32;    // 25 K-steps per segment
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

  // Pipeline: B data for step j is global-loaded NSETS iterations ahead into
  // register set (j - 2) % NSETS, written to LDS stage j % 3 two iterations
  // ahead, and its fragments are read one iteration ahead (while the MFMAs
  // of the current step run).  Stage (k+2)%3 is overwritten at iteration k;
  // it was last read at iteration k-2.
  v4i falo[WM], fahi[WM], fblo[WN], fbhi[WN];     // fragments of the current step
  v4i nalo[WM], nahi[WM], nblo[WN], nbhi[WN];     // fragments of the next step
#define IMC_FRAGS(ALO, AHI, BLO, BHI, K)                                              \
  {                                                                                   \
    const int kk_ = (K);                                                              \
    const int seg_ = kk_ / kSegSteps, ts_ = kk_ - seg_ * kSegSteps;                   \
    const int8_t* sb_ = bst + (kk_ % 3) * kBStage;                                    \
    const int8_t* sa_ = ast + (seg_ & 1) * abuf + 32 * ts_;                           \
    _Pragma("unroll") for (int x_ = 0; x_ < WM; ++x_) {                               \
      const int32_t* pa_ = reinterpret_cast<const int32_t*>(sa_ + a_off[x_]);         \
      const int32_t* ph_ = reinterpret_cast<const int32_t*>(sa_ + a_off[x_] + kSegBytes); \
      ALO[x_] = v4i{pa_[0], pa_[1], pa_[2], pa_[3]};                                  \
      AHI[x_] = v4i{ph_[0], ph_[1], ph_[2], ph_[3]};                                  \
    }                                                                                 \
    _Pragma("unroll") for (int y_ = 0; y_ < WN; ++y_) {                               \
      const int8_t* pb_ = sb_ + (wn * WN + y_) * 2048 + lane * 16;                    \
      BLO[y_] = *reinterpret_cast<const v4i*>(pb_);                                   \
      BHI[y_] = *reinterpret_cast<const v4i*>(pb_ + 1024);                            \
    }                                                                                 \
  }

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
  // a wave whose rows are all past the last row (the partial last row tile)
  // only stages operands for the others: no fragment reads, no MFMAs
  const bool live = m0 + uint32_t(wm * WM * 32) < args.rows;
  if (!live) {
    for (int k0 = 0; k0 < kSteps; k0 += NSETS) {
#pragma unroll
      for (int uu = 0; uu < NSETS; ++uu) {
        const int k = k0 + uu;
        const int seg = k / kSegSteps, ts = k - seg * kSegSteps;
        IMC_BSTORE(rs[uu], (k + 2) % 3)
        if (ts == kSegSteps / 2 && seg + 1 < kSteps / kSegSteps) {
          IMC_ASTORE((seg + 1) & 1)
          IMC_ALOAD(min(seg + 2, kSteps / kSegSteps - 1))
        }
        __syncthreads();
        IMC_BLOAD(rs[uu], min(k + 2 + NSETS, kSteps - 1))
      }
    }
  } else {
    IMC_FRAGS(falo, fahi, fblo, fbhi, 0)

    for (int k0 = 0; k0 < kSteps; k0 += NSETS) {
#pragma unroll
      for (int uu = 0; uu < NSETS; ++uu) {
        const int k = k0 + uu;
        const int seg = k / kSegSteps, ts = k - seg * kSegSteps;
        // interleave the next step's fragment reads with this step's MFMAs
        // (the compiler's single-wave small-GEMM schedule; ~1.5 % faster here)
        __builtin_amdgcn_iglp_opt(1);
        IMC_FRAGS(nalo, nahi, nblo, nbhi, min(k + 1, kSteps - 1))
#pragma unroll
        for (int x = 0; x < WM; ++x)
#pragma unroll
          for (int y = 0; y < WN; ++y) {
            acc0[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(falo[x], fblo[y], acc0[x][y], 0, 0, 0);
            acc1[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(falo[x], fbhi[y], acc1[x][y], 0, 0, 0);
            acc1[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fahi[x], fblo[y], acc1[x][y], 0, 0, 0);
          }
        IMC_BSTORE(rs[uu], (k + 2) % 3)             // step k + 2
        // mid-segment: the next segment's query bytes go to the other A buffer
        // (last read during the previous segment), then its loads are issued
        // for the segment after it.
        if (ts == kSegSteps / 2 && seg + 1 < kSteps / kSegSteps) {
          IMC_ASTORE((seg + 1) & 1)
          IMC_ALOAD(min(seg + 2, kSteps / kSegSteps - 1))
        }
        __syncthreads();
        IMC_BLOAD(rs[uu], min(k + 2 + NSETS, kSteps - 1))
#pragma unroll
        for (int x = 0; x < WM; ++x) { falo[x] = nalo[x]; fahi[x] = nahi[x]; }
#pragma unroll
        for (int y = 0; y < WN; ++y) { fblo[y] = nblo[y]; fbhi[y] = nbhi[y]; }
      }
    }
  }
#undef IMC_FRAGS
#undef IMC_BLOAD
#undef IMC_BSTORE
#undef IMC_ALOAD
#undef IMC_ASTORE

  uint16_t* out = args.out;
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
          const uint32_t z = uint32_t(acc0[x][y][e]) + (uint32_t(acc1[x][y][e]) << 8);
          out[uint64_t(row) * args.ld + col] = uint16_t(z);
        }
      }
    }
}

// One launch per call: workgroup i is output tile (u, t) in an XCD-aware
// order (consecutive workgroups go to the 8 XCDs in turn; each XCD walks
// every row tile of its column tiles, so a column tile's database bytes are
// read into one XCD's L2).
template <int K, int WM, int WN, int WAVES_M, int WAVES_N, int NSETS, int ACH>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N) rot_dot_kernel(RotDotArgs args) {
  extern __shared__ __align__(16) int8_t lds[];
  const int vec = blockIdx.z;
  const uint32_t i = blockIdx.x;
  const uint32_t xcd = i & 7, s8 = i >> 3;
  const uint32_t u = s8 % args.mt, tg = s8 / args.mt;
  const uint32_t t = tg * 8 + xcd;
  if (t >= args.nt) return;
  const RotTile tile{args.qop, args.qidx, args.b, args.out[vec], args.rot, args.ld, args.b_block0, args.b_blocks,
                     args.n, args.rows, args.r, args.max_q};
  rot_dot_tile<K, WM, WN, WAVES_M, WAVES_N, NSETS, ACH>(tile, u, t, vec, lds);
}

// ---------------------------------------------------------------------------
// Several query groups in one launch (uneven batches: each group is the
// queries of one rotation list, e.g. the batches checked at 31 rotations and
// those at 15).  Group g owns global tiles [tile0, tile0 + 8 * ntg * mt) and
// maps them to its (row tile, column tile) pairs exactly as one launch of
// rot_dot_kernel would, so every group keeps the XCD-aware order.  With a
// persistent grid (a multiple of 8 workgroups, fewer than the tiles) each
// workgroup walks tiles i, i + grid, ...: the same residue mod 8, so the
// same XCD, as a one-tile-per-workgroup launch would give them.
// ---------------------------------------------------------------------------
constexpr int kMaxDotGroups = IMC_MAX_DOT_GROUPS;
struct RotGroup {
  const int8_t* qop;
  uint16_t* out[2];
  uint32_t rows, r, mt, tile0;
  int8_t rot[IMC_MAX_ROT_DEV];
};
struct RotGroupsArgs {
  const int8_t* b;
  uint64_t ld, b_block0, b_blocks, n;
  uint32_t nt, ntiles, ngroups, max_q;
  RotGroup g[kMaxDotGroups];
};

template <int K, int WM, int WN, int WAVES_M, int WAVES_N, int NSETS, int ACH>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N) rot_dot_groups_kernel(RotGroupsArgs args) {
  extern __shared__ __align__(16) int8_t lds[];
  const int vec = blockIdx.z;
  bool first = true;
  for (uint32_t i = blockIdx.x; i < args.ntiles; i += gridDim.x) {
    uint32_t gi = 0;
    while (gi + 1 < args.ngroups && i >= args.g[gi + 1].tile0) ++gi;
    const RotGroup& grp = args.g[gi];
    const uint32_t li = i - grp.tile0;
    const uint32_t xcd = li & 7, s8 = li >> 3;
    const uint32_t u = s8 % grp.mt, tg = s8 / grp.mt;
    const uint32_t t = tg * 8 + xcd;
    if (t >= args.nt) continue;
    // the previous tile's last fragment reads end before this tile's prologue
    // overwrites the LDS stages
    if (!first) __syncthreads();
    first = false;
    const RotTile tile{grp.qop, nullptr, args.b, grp.out[vec], grp.rot, args.ld, args.b_block0, args.b_blocks,
                       args.n, grp.rows, grp.r, args.max_q};
    rot_dot_tile<K, WM, WN, WAVES_M, WAVES_N, NSETS, ACH>(tile, u, t, vec, lds);
  }
}

// The query slots of a 256-row tile (ceil(256 / r) + 1 of them) must fit the
// A staging of the configuration: 3 chunks per thread up to 13 queries (r >= 22),
// 5 up to 22 queries (r >= 13, default configuration only).
bool rot_dot_applies(uint32_t r, int kind) { return kind == 0 ? r >= 13 : r >= 22; }

// ---------------------------------------------------------------------------
// The same rotation-aware tiling with the database fragments loaded by every
// wave straight from HBM (through its L1/L2) into registers D K-steps ahead:
// a fragment is 1 KB contiguous in the tiled layout, and the WAVES_M waves
// that share a column block hit the same lines.  Only the query segments go
// through LDS, so there is no per-step barrier: two per 25-step segment,
// around the store of the next segment into the other A buffer.
// ---------------------------------------------------------------------------
template <int K, int WM, int WN, int WAVES_M, int WAVES_N, int D, int ACH>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N) rot_dot_gb_kernel(RotDotArgs args) {
  using G = Geo<K>;
  constexpr int kBM = 32 * WM * WAVES_M, kBN = 32 * WN * WAVES_N;
  constexpr int kThreads = 64 * WAVES_M * WAVES_N;
  constexpr int kBBlk = kBN / 32;
  extern __shared__ __align__(16) int8_t lds[];
  int8_t* ast = lds;                                           // 2 A segment buffers
  const uint32_t abuf = args.max_q * 2 * kSegBytes;            // bytes per A buffer

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  const int vec = blockIdx.z;
  const uint32_t i = blockIdx.x;
  const uint32_t xcd = i & 7, s8 = i >> 3;
  const uint32_t u = s8 % args.mt, tg = s8 / args.mt;
  const uint32_t t = tg * 8 + xcd;
  if (t >= args.nt) return;

  const uint32_t m0 = u * kBM;
  const uint32_t q_lo = m0 / args.r;
  const uint32_t last_row = min(m0 + kBM, args.rows) - 1;
  const uint32_t nq = last_row / args.r - q_lo + 1;            // <= max_q

  int a_off[WM];
#pragma unroll
  for (int x = 0; x < WM; ++x) {
    const uint32_t row = m0 + (wm * WM + x) * 32 + (lane & 31);
    int slot = 0, sft = 0;
    if (row < args.rows) {
      slot = int(row / args.r - q_lo);
      sft = 4 * args.rot[row % args.r];
    }
    a_off[x] = slot * 2 * kSegBytes + kSegPad - sft + 16 * (lane >> 5);
  }

  // This lane's 16 bytes of the lo-plane fragment of each of the wave's column
  // blocks at K-step 0; step k adds 1 KB, the hi plane one plane block.
  const int8_t* bfr[WN];
#pragma unroll
  for (int y = 0; y < WN; ++y) {
    uint64_t cb = uint64_t(t) * kBBlk + wn * WN + y;
    cb = cb < args.b_blocks ? cb : args.b_blocks - 1;
    bfr[y] = args.b + size_t(args.b_block0 + cb) * G::kBlockBytes + size_t(2 * vec) * G::kPlaneBlockBytes + lane * 16;
  }
  const int a_chunks = int(nq) * 2 * kSegChunks;
  const int8_t* asrc[ACH];
  int adst[ACH];
#pragma unroll
  for (int j = 0; j < ACH; ++j) {
    int c = tid + j * kThreads;
    const bool ok = c < a_chunks;
    c = ok ? c : 0;
    const int qs = c / (2 * kSegChunks), rem = c % (2 * kSegChunks);
    const int pl = rem / kSegChunks, piece = rem % kSegChunks;
    const int src_off = ((piece * 16 - kSegPad) % kRowLen + kRowLen) % kRowLen;   // circular
    const uint32_t qrow = args.qidx ? args.qidx[q_lo + qs] : q_lo + qs;
    asrc[j] = args.qop + size_t(qrow) * G::kQopRowBytes + size_t(2 * vec + pl) * G::kK + src_off;
    adst[j] = ok ? (qs * 2 * kSegBytes + pl * kSegBytes + piece * 16) : -1;
  }

  v16i acc0[WM][WN], acc1[WM][WN];
#pragma unroll
  for (int x = 0; x < WM; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) { acc0[x][y][e] = 0; acc1[x][y][e] = 0; }

  constexpr int kSteps = G::kChunks / 2;        // 800 or 400
  constexpr int kSegSteps = kRowLen / 32;       // 25 K-steps per segment
  static_assert(kSteps % D == 0, "the K loop is unrolled by D");
  v4i bl[D][WN], bh[D][WN];                     // database fragments, set = step % D
  v4i ra[ACH];

#define IMC_BLOAD(SET, KS)                                                            \
  _Pragma("unroll") for (int y_ = 0; y_ < WN; ++y_) {                                 \
    const int8_t* p_ = bfr[y_] + size_t(KS) * 1024;                                   \
    bl[SET][y_] = *reinterpret_cast<const v4i*>(p_);                                  \
    bh[SET][y_] = *reinterpret_cast<const v4i*>(p_ + G::kPlaneBlockBytes);            \
  }
#define IMC_ALOAD(SEG)                                                                \
  _Pragma("unroll") for (int c_ = 0; c_ < ACH; ++c_)                                  \
      ra[c_] = *reinterpret_cast<const v4i*>(asrc[c_] + size_t(SEG) * kRowLen);
#define IMC_ASTORE(BUF)                                                               \
  _Pragma("unroll") for (int c_ = 0; c_ < ACH; ++c_)                                  \
      if (adst[c_] >= 0) *reinterpret_cast<v4i*>(ast + (BUF) * abuf + adst[c_]) = ra[c_];
#define IMC_AFRAGS(ALO, AHI, K)                                                       \
  {                                                                                   \
    const int kk_ = (K);                                                              \
    const int seg_ = kk_ / kSegSteps, ts_ = kk_ - seg_ * kSegSteps;                   \
    const int8_t* sa_ = ast + (seg_ & 1) * abuf + 32 * ts_;                           \
    _Pragma("unroll") for (int x_ = 0; x_ < WM; ++x_) {                               \
      const int32_t* pa_ = reinterpret_cast<const int32_t*>(sa_ + a_off[x_]);         \
      const int32_t* ph_ = reinterpret_cast<const int32_t*>(sa_ + a_off[x_] + kSegBytes); \
      ALO[x_] = v4i{pa_[0], pa_[1], pa_[2], pa_[3]};                                  \
      AHI[x_] = v4i{ph_[0], ph_[1], ph_[2], ph_[3]};                                  \
    }                                                                                 \
  }

  // prologue: A segment 0 in buffer 0, segment 1 in registers; database
  // fragments of steps 0 .. D-1 in flight
  IMC_ALOAD(0)
  IMC_ASTORE(0)
  IMC_ALOAD(1)
#pragma unroll
  for (int set = 0; set < D; ++set) { IMC_BLOAD(set, set) }
  __syncthreads();
  v4i falo[WM], fahi[WM], nalo[WM], nahi[WM];
  IMC_AFRAGS(falo, fahi, 0)

  // One K-step: the next step's A fragments are read first (pinned ahead of
  // the MFMAs, so they complete under them), then the MFMAs of this step,
  // then the database fragments of step k + D are requested into the set
  // this step consumed.  Two A register sets alternate (the loop is unrolled
  // by D, which is even).
#define IMC_GSTEP(CUR, NXT, UU)                                                       \
  {                                                                                   \
    const int k_ = k0 + (UU);                                                         \
    const int seg_ = k_ / kSegSteps, ts_ = k_ - seg_ * kSegSteps;                     \
    wait_lds(); /* this step's A fragments, read during the previous step */          \
    if (ts_ == kSegSteps / 2 && seg_ + 1 < kSteps / kSegSteps) {                      \
      /* every wave is past its last read of the other A buffer (segment seg-1): */   \
      /* store segment seg+1 there and make it visible before the segment ends */     \
      __syncthreads();                                                                \
      IMC_ASTORE((seg_ + 1) & 1)                                                      \
      __syncthreads();                                                                \
      IMC_ALOAD(min(seg_ + 2, kSteps / kSegSteps - 1))                                \
    }                                                                                 \
    IMC_AFRAGS(NXT##alo, NXT##ahi, min(k_ + 1, kSteps - 1))                            \
    __builtin_amdgcn_sched_barrier(0);                                                \
    _Pragma("unroll") for (int x = 0; x < WM; ++x)                                    \
    _Pragma("unroll") for (int y = 0; y < WN; ++y) {                                  \
      acc0[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(CUR##alo[x], bl[UU][y], acc0[x][y], 0, 0, 0); \
      acc1[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(CUR##alo[x], bh[UU][y], acc1[x][y], 0, 0, 0); \
      acc1[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(CUR##ahi[x], bl[UU][y], acc1[x][y], 0, 0, 0); \
    }                                                                                 \
    IMC_BLOAD(UU, min(k_ + D, kSteps - 1))                                            \
  }
  static_assert(D % 2 == 0, "A register sets alternate");
  for (int k0 = 0; k0 < kSteps; k0 += D) {
#pragma unroll
    for (int h = 0; h < D; h += 2) {
      IMC_GSTEP(f, n, h)
      IMC_GSTEP(n, f, h + 1)
    }
  }
#undef IMC_GSTEP
#undef IMC_AFRAGS
#undef IMC_BLOAD
#undef IMC_ALOAD
#undef IMC_ASTORE

  uint16_t* out = args.out[vec];
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
          const uint32_t z = uint32_t(acc0[x][y][e]) + (uint32_t(acc1[x][y][e]) << 8);
          out[uint64_t(row) * args.ld + col] = uint16_t(z);
        }
      }
    }
}

// ---------------------------------------------------------------------------
// The same rotation-aware tiling with the operands copied HBM -> LDS by the
// load units themselves (global_load_lds_dwordx4): no staging registers and
// no LDS store instructions, so the database stream can run S - 3 K-steps
// ahead through S LDS stages.  Each wave issues an identical sequence of
// copies (one per K-step for the database, ACH per query segment, inactive
// lanes copying a valid source into the buffer's unused tail), so a per-wave
// vmcnt wait of S - 3 guarantees that the copy of step k + 2 has landed
// before the barrier that precedes its fragment reads.  The barriers are
// bare s_barrier instructions: a workgroup fence would wait for every
// outstanding copy.
// ---------------------------------------------------------------------------

template <int K, int WM, int WN, int WAVES_M, int WAVES_N, int S, int ACH>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N) rot_dot_dma_kernel(RotDotArgs args) {
  using G = Geo<K>;
  constexpr int kBM = 32 * WM * WAVES_M, kBN = 32 * WN * WAVES_N;
  constexpr int kThreads = 64 * WAVES_M * WAVES_N;
  constexpr int kBBlk = kBN / 32;
  constexpr int kBChunks = kBBlk * 2 * 2 * 32;                 // per K-step
  constexpr int kBPerThread = kBChunks / kThreads;
  constexpr int kBStage = kBChunks * 16;
  constexpr int kABuf = ACH * kThreads * 16;                   // A buffer incl. the unused tail
  static_assert(kBChunks % kThreads == 0, "B chunks must divide evenly");
  static_assert(S >= 4, "at least one copy in flight beyond the two read-ahead stages");
  // the wait for step k + 2 must also cover the query segment copied at mid-segment
  static_assert(S <= 12, "query segment copy must precede the copy waited for at the segment end");
  extern __shared__ __align__(16) int8_t lds[];
  int8_t* bst = lds;                                           // S B stages
  int8_t* ast = lds + S * kBStage;                             // 2 A segment buffers

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  const int vec = blockIdx.z;
  const uint32_t i = blockIdx.x;
  const uint32_t xcd = i & 7, s8 = i >> 3;
  const uint32_t u = s8 % args.mt, tg = s8 / args.mt;
  const uint32_t t = tg * 8 + xcd;
  if (t >= args.nt) return;

  const uint32_t m0 = u * kBM;
  const uint32_t q_lo = m0 / args.r;
  const uint32_t last_row = min(m0 + kBM, args.rows) - 1;
  const uint32_t nq = last_row / args.r - q_lo + 1;            // <= max_q

  int a_off[WM];
#pragma unroll
  for (int x = 0; x < WM; ++x) {
    const uint32_t row = m0 + (wm * WM + x) * 32 + (lane & 31);
    int slot = 0, sft = 0;
    if (row < args.rows) {
      slot = int(row / args.r - q_lo);
      sft = 4 * args.rot[row % args.r];
    }
    a_off[x] = slot * 2 * kSegBytes + kSegPad - sft + 16 * (lane >> 5);
  }

  const int8_t* bsrc[kBPerThread];
#pragma unroll
  for (int j = 0; j < kBPerThread; ++j) {
    const int c = tid + j * kThreads;
    const int blk = c >> 7, rem = c & 127;
    const int plane = rem >> 6, kcl = (rem >> 5) & 1, slot = rem & 31;
    uint64_t cb = uint64_t(t) * kBBlk + blk;
    cb = cb < args.b_blocks ? cb : args.b_blocks - 1;
    bsrc[j] = args.b + size_t(args.b_block0 + cb) * G::kBlockBytes + size_t(2 * vec + plane) * G::kPlaneBlockBytes +
              size_t(kcl) * 512 + slot * 16;
  }
  // A chunk c of a segment buffer = (query slot, plane, 16-byte piece) lands at
  // byte 16 c; chunks past the tile's queries copy piece 0 of slot 0.
  const int a_chunks = int(nq) * 2 * kSegChunks;
  const int8_t* asrc[ACH];
#pragma unroll
  for (int j = 0; j < ACH; ++j) {
    int c = tid + j * kThreads;
    c = c < a_chunks ? c : 0;
    const int qs = c / (2 * kSegChunks), rem = c % (2 * kSegChunks);
    const int pl = rem / kSegChunks, piece = rem % kSegChunks;
    const int src_off = ((piece * 16 - kSegPad) % kRowLen + kRowLen) % kRowLen;   // circular
    const uint32_t qrow = args.qidx ? args.qidx[q_lo + qs] : q_lo + qs;
    asrc[j] = args.qop + size_t(qrow) * G::kQopRowBytes + size_t(2 * vec + pl) * G::kK + src_off;
  }

  v16i acc0[WM][WN], acc1[WM][WN];
#pragma unroll
  for (int x = 0; x < WM; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) { acc0[x][y][e] = 0; acc1[x][y][e] = 0; }

  constexpr int kSteps = G::kChunks / 2;        // 800 or 400
  constexpr int kSegSteps = kRowLen / 32;    // 25 K-steps per segment
  constexpr int kSegs = kSteps / kSegSteps;  // 32 or 16

  // wave-uniform LDS bases of this wave's copies
  const int wbase = wave * 64 * 16;
#define IMC_BCOPY(KS)                                                                 \
  {                                                                                   \
    const int ks_ = (KS);                                                             \
    _Pragma("unroll") for (int c_ = 0; c_ < kBPerThread; ++c_)                        \
      copy16(bsrc[c_] + size_t(2 * ks_) * 512,                                        \
             bst + (ks_ % S) * kBStage + c_ * kThreads * 16 + wbase);                 \
  }
#define IMC_ACOPY(SEG, BUF)                                                           \
  _Pragma("unroll") for (int c_ = 0; c_ < ACH; ++c_)                                  \
    copy16(asrc[c_] + size_t(SEG) * kRowLen, ast + (BUF) * kABuf + c_ * kThreads * 16 + wbase);

  v4i falo[WM], fahi[WM], fblo[WN], fbhi[WN];
  v4i nalo[WM], nahi[WM], nblo[WN], nbhi[WN];
#define IMC_FRAGS(ALO, AHI, BLO, BHI, K)                                              \
  {                                                                                   \
    const int kk_ = (K);                                                              \
    const int seg_ = kk_ / kSegSteps, ts_ = kk_ - seg_ * kSegSteps;                   \
    const int8_t* sb_ = bst + (kk_ % S) * kBStage;                                    \
    const int8_t* sa_ = ast + (seg_ & 1) * kABuf + 32 * ts_;                          \
    _Pragma("unroll") for (int x_ = 0; x_ < WM; ++x_) {                               \
      const int32_t* pa_ = reinterpret_cast<const int32_t*>(sa_ + a_off[x_]);         \
      const int32_t* ph_ = reinterpret_cast<const int32_t*>(sa_ + a_off[x_] + kSegBytes); \
      ALO[x_] = v4i{pa_[0], pa_[1], pa_[2], pa_[3]};                                  \
      AHI[x_] = v4i{ph_[0], ph_[1], ph_[2], ph_[3]};                                  \
    }                                                                                 \
    _Pragma("unroll") for (int y_ = 0; y_ < WN; ++y_) {                               \
      const int8_t* pb_ = sb_ + (wn * WN + y_) * 2048 + lane * 16;                    \
      BLO[y_] = *reinterpret_cast<const v4i*>(pb_);                                   \
      BHI[y_] = *reinterpret_cast<const v4i*>(pb_ + 1024);                            \
    }                                                                                 \
  }

  // prologue: A segment 0, B steps 0 .. S - 2; all landed before the first reads
  IMC_ACOPY(0, 0)
#pragma unroll
  for (int j = 0; j < S - 1; ++j) IMC_BCOPY(j)
  wait_vm<0>();
  bar();
  IMC_FRAGS(falo, fahi, fblo, fbhi, 0)

  // One K-step: copies for later steps, the next step's fragment reads (issued
  // before the MFMAs so that they complete under them), the MFMAs, then the
  // wait for the copy of step k + 2 and the barrier.  Unrolled by two so the
  // current / next fragment registers alternate without moves.
#define IMC_STEP(CUR, NXT, K)                                                         \
  {                                                                                   \
    const int k_ = (K);                                                               \
    const int seg_ = k_ / kSegSteps, ts_ = k_ - seg_ * kSegSteps;                     \
    wait_lds(); /* this step's fragments, read during the previous step */            \
    if (ts_ == kSegSteps / 2 && seg_ + 1 < kSegs) IMC_ACOPY(seg_ + 1, (seg_ + 1) & 1) \
    const bool more_ = k_ + S - 1 < kSteps;                                           \
    if (more_) IMC_BCOPY(k_ + S - 1)                                                  \
    IMC_FRAGS(NXT##alo, NXT##ahi, NXT##blo, NXT##bhi, min(k_ + 1, kSteps - 1))         \
    __builtin_amdgcn_sched_barrier(0);                                                \
    _Pragma("unroll") for (int x = 0; x < WM; ++x)                                    \
    _Pragma("unroll") for (int y = 0; y < WN; ++y) {                                  \
      acc0[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(CUR##alo[x], CUR##blo[y], acc0[x][y], 0, 0, 0); \
      acc1[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(CUR##alo[x], CUR##bhi[y], acc1[x][y], 0, 0, 0); \
      acc1[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(CUR##ahi[x], CUR##blo[y], acc1[x][y], 0, 0, 0); \
    }                                                                                 \
    if (more_)                                                                        \
      wait_vm<S - 3>();                                                               \
    else                                                                              \
      wait_vm<0>();                                                                   \
    bar();                                                                            \
  }
  static_assert(kSteps % 2 == 0, "the K loop is unrolled by two");
  for (int k = 0; k < kSteps; k += 2) {
    IMC_STEP(f, n, k)
    IMC_STEP(n, f, k + 1)
  }
#undef IMC_STEP
  wait_vm<0>();
#undef IMC_FRAGS
#undef IMC_BCOPY
#undef IMC_ACOPY

  uint16_t* out = args.out[vec];
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
          const uint32_t z = uint32_t(acc0[x][y][e]) + (uint32_t(acc1[x][y][e]) << 8);
          out[uint64_t(row) * args.ld + col] = uint16_t(z);
        }
      }
    }
}

template <int K, int WM, int WN, int WAVES_M, int WAVES_N, int NSETS, int ACH>
static hipError_t launch_rot_cfg(const int8_t* qop, const uint32_t* qidx, uint32_t q, uint32_t r, const int8_t* rot,
                                 const int8_t* b,
                                 uint64_t first_entry, uint64_t n, uint16_t* code, uint16_t* mask, uint64_t ld,
                                 hipStream_t s) {
  constexpr int kBM = 32 * WM * WAVES_M, kBN = 32 * WN * WAVES_N, kThreads = 64 * WAVES_M * WAVES_N;
  const uint32_t rows = q * r;
  if (rows == 0 || n == 0) return hipSuccess;
  if (r < 13) return hipErrorInvalidValue;
  RotDotArgs d;
  d.qop = qop;
  d.qidx = qidx;
  d.b = b;
  d.out[0] = code;
  d.out[1] = mask;
  d.ld = ld;
  d.rows = rows;
  d.q = q;
  d.r = r;
  d.b_block0 = first_entry / 32;
  d.b_blocks = (n + 31) / 32;
  d.n = n;
  d.mt = (rows + kBM - 1) / kBM;
  d.nt = uint32_t((n + kBN - 1) / kBN);
  d.max_q = (kBM + r - 1) / r + 1;
  if (int(d.max_q) * 2 * kSegChunks > ACH * kThreads) return hipErrorInvalidValue;
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) d.rot[i] = i < int(r) ? rot[i] : 0;
  const uint32_t ntg = (d.nt + 7) / 8;
  if (uint64_t(ntg) * 8 * d.mt > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid(ntg * 8 * d.mt, 1, mask ? 2 : 1);   // z: code, mask
  const size_t lds = 3 * size_t(kBN / 32) * 2 * 2 * 32 * 16 + 2 * size_t(d.max_q) * 2 * kSegBytes;
  auto kern = rot_dot_kernel<K, WM, WN, WAVES_M, WAVES_N, NSETS, ACH>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, d);
  return hipGetLastError();
}

template <int K>
static hipError_t launch_rot_dma(const int8_t* qop, const uint32_t* qidx, uint32_t q, uint32_t r, const int8_t* rot,
                                 const int8_t* b,
                                 uint64_t first_entry, uint64_t n, uint16_t* code, uint16_t* mask, uint64_t ld,
                                 hipStream_t s) {
  constexpr int WM = 2, WN = 2, WAVES_M = 4, WAVES_N = 2, S = 8, ACH = 3;
  constexpr int kBM = 32 * WM * WAVES_M, kBN = 32 * WN * WAVES_N, kThreads = 64 * WAVES_M * WAVES_N;
  const uint32_t rows = q * r;
  if (rows == 0 || n == 0) return hipSuccess;
  if (r < 13) return hipErrorInvalidValue;
  RotDotArgs d;
  d.qop = qop;
  d.qidx = qidx;
  d.b = b;
  d.out[0] = code;
  d.out[1] = mask;
  d.ld = ld;
  d.rows = rows;
  d.q = q;
  d.r = r;
  d.b_block0 = first_entry / 32;
  d.b_blocks = (n + 31) / 32;
  d.n = n;
  d.mt = (rows + kBM - 1) / kBM;
  d.nt = uint32_t((n + kBN - 1) / kBN);
  d.max_q = (kBM + r - 1) / r + 1;
  if (int(d.max_q) * 2 * kSegChunks > ACH * kThreads) return hipErrorInvalidValue;
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) d.rot[i] = i < int(r) ? rot[i] : 0;
  const uint32_t ntg = (d.nt + 7) / 8;
  if (uint64_t(ntg) * 8 * d.mt > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid(ntg * 8 * d.mt, 1, mask ? 2 : 1);   // z: code, mask
  const size_t lds = size_t(S) * (kBN / 32) * 2 * 2 * 32 * 16 + 2 * size_t(ACH) * kThreads * 16;
  auto kern = rot_dot_dma_kernel<K, WM, WN, WAVES_M, WAVES_N, S, ACH>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, d);
  return hipGetLastError();
}

template <int K, int WM, int WN, int WAVES_M, int WAVES_N, int D, int ACH>
static hipError_t launch_rot_gb(const int8_t* qop, const uint32_t* qidx, uint32_t q, uint32_t r, const int8_t* rot,
                                 const int8_t* b,
                                uint64_t first_entry, uint64_t n, uint16_t* code, uint16_t* mask, uint64_t ld,
                                hipStream_t s) {
  constexpr int kBM = 32 * WM * WAVES_M, kBN = 32 * WN * WAVES_N, kThreads = 64 * WAVES_M * WAVES_N;
  const uint32_t rows = q * r;
  if (rows == 0 || n == 0) return hipSuccess;
  if (r < 13) return hipErrorInvalidValue;
  RotDotArgs d;
  d.qop = qop;
  d.qidx = qidx;
  d.b = b;
  d.out[0] = code;
  d.out[1] = mask;
  d.ld = ld;
  d.rows = rows;
  d.q = q;
  d.r = r;
  d.b_block0 = first_entry / 32;
  d.b_blocks = (n + 31) / 32;
  d.n = n;
  d.mt = (rows + kBM - 1) / kBM;
  d.nt = uint32_t((n + kBN - 1) / kBN);
  d.max_q = (kBM + r - 1) / r + 1;
  if (int(d.max_q) * 2 * kSegChunks > ACH * kThreads) return hipErrorInvalidValue;
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) d.rot[i] = i < int(r) ? rot[i] : 0;
  const uint32_t ntg = (d.nt + 7) / 8;
  if (uint64_t(ntg) * 8 * d.mt > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid(ntg * 8 * d.mt, 1, mask ? 2 : 1);   // z: code, mask
  const size_t lds = 2 * size_t(d.max_q) * 2 * kSegBytes;
  auto kern = rot_dot_gb_kernel<K, WM, WN, WAVES_M, WAVES_N, D, ACH>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, d);
  return hipGetLastError();
}

template <int K, int ACH>
static hipError_t launch_rot_groups_cfg(const DotGroup* groups, uint32_t ngroups, const int8_t* b,
                                        uint64_t first_entry, uint64_t n, uint64_t ld, bool persistent,
                                        hipStream_t s) {
  constexpr int WM = 2, WN = 2, WAVES_M = 4, WAVES_N = 2, NSETS = 4;
  constexpr int kBM = 32 * WM * WAVES_M, kBN = 32 * WN * WAVES_N, kThreads = 64 * WAVES_M * WAVES_N;
  RotGroupsArgs d;
  d.b = b;
  d.ld = ld;
  d.b_block0 = first_entry / 32;
  d.b_blocks = (n + 31) / 32;
  d.n = n;
  d.nt = uint32_t((n + kBN - 1) / kBN);
  const uint64_t ntg = (d.nt + 7) / 8;
  uint64_t tiles = 0;
  uint32_t max_q = 0, used = 0;
  bool mask = false;
  for (uint32_t gi = 0; gi < ngroups; ++gi) {
    const DotGroup& g = groups[gi];
    const uint32_t rows = g.q * g.r;
    if (rows == 0) continue;
    RotGroup& o = d.g[used++];
    o.qop = g.qop;
    o.out[0] = g.code;
    o.out[1] = g.mask;
    mask = g.mask != nullptr;
    o.rows = rows;
    o.r = g.r;
    o.mt = (rows + kBM - 1) / kBM;
    o.tile0 = uint32_t(tiles);
    for (int j = 0; j < IMC_MAX_ROT_DEV; ++j) o.rot[j] = j < int(g.r) ? g.rot[j] : 0;
    max_q = std::max(max_q, (kBM + g.r - 1) / g.r + 1);
    tiles += ntg * 8 * o.mt;
    if (tiles > 0x7FFFFFFFull) return hipErrorInvalidValue;
  }
  if (used == 0 || n == 0) return hipSuccess;
  if (int(max_q) * 2 * kSegChunks > ACH * kThreads) return hipErrorInvalidValue;
  d.ngroups = used;
  d.ntiles = uint32_t(tiles);
  d.max_q = max_q;
  const size_t lds = 3 * size_t(kBN / 32) * 2 * 2 * 32 * 16 + 2 * size_t(max_q) * 2 * kSegBytes;
  auto kern = rot_dot_groups_kernel<K, WM, WN, WAVES_M, WAVES_N, NSETS, ACH>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  uint32_t grid = d.ntiles;
  if (persistent) {
    // one workgroup per CU (the LDS of a tile allows no second one), a
    // multiple of the 8 XCDs
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      return hipErrorInvalidValue;
    const uint32_t g8 = (uint32_t(cus) + 7) / 8 * 8;
    grid = std::min<uint32_t>(grid, g8);
  }
  hipLaunchKernelGGL(kern, dim3(grid, 1, mask ? 2 : 1), dim3(kThreads), lds, s, d);
  return hipGetLastError();
}

hipError_t launch_rot_dot_groups(const DotGroup* groups, uint32_t ngroups, const int8_t* b, uint64_t first_entry,
                                 uint64_t n, uint64_t ld, bool persistent, hipStream_t s, bool galois) {
  if (ngroups > uint32_t(kMaxDotGroups)) return hipErrorInvalidValue;
  uint32_t rmin = 32;
  for (uint32_t gi = 0; gi < ngroups; ++gi) {
    if (groups[gi].q == 0) continue;
    if (groups[gi].r < 13) return hipErrorInvalidValue;
    rmin = std::min(rmin, groups[gi].r);
  }
  // the staging of the fewest rotations (the most query slots) sizes the launch
  if (galois)
    return rmin >= 22 ? launch_rot_groups_cfg<kKGalois, 3>(groups, ngroups, b, first_entry, n, ld, persistent, s)
                      : launch_rot_groups_cfg<kKGalois, 5>(groups, ngroups, b, first_entry, n, ld, persistent, s);
  return rmin >= 22 ? launch_rot_groups_cfg<kK, 3>(groups, ngroups, b, first_entry, n, ld, persistent, s)
                    : launch_rot_groups_cfg<kK, 5>(groups, ngroups, b, first_entry, n, ld, persistent, s);
}

hipError_t launch_rot_dot(const int8_t* qop, const uint32_t* qidx, uint32_t q, uint32_t r, const int8_t* rot,
                          const int8_t* b,
                          uint64_t first_entry, uint64_t n, uint16_t* code, uint16_t* mask, uint64_t ld,
                          hipStream_t s, int kind, bool galois) {
  // 0: 8 waves of 64 x 64, loads 6 steps ahead; 2: HBM -> LDS copies, 8
  // stages; 3: database fragments straight into registers
  if (galois) {
    switch (kind) {
      case 2: return launch_rot_dma<kKGalois>(qop, qidx, q, r, rot, b, first_entry, n, code, mask, ld, s);
      case 3: return launch_rot_gb<kKGalois, 2, 2, 4, 2, 4, 3>(qop, qidx, q, r, rot, b, first_entry, n, code, mask, ld, s);
      default:
        if (r >= 22) return launch_rot_cfg<kKGalois, 2, 2, 4, 2, 4, 3>(qop, qidx, q, r, rot, b, first_entry, n, code, mask, ld, s);
        return launch_rot_cfg<kKGalois, 2, 2, 4, 2, 4, 5>(qop, qidx, q, r, rot, b, first_entry, n, code, mask, ld, s);
    }
  }
  switch (kind) {
    case 2: return launch_rot_dma<kK>(qop, qidx, q, r, rot, b, first_entry, n, code, mask, ld, s);
    case 3: return launch_rot_gb<kK, 2, 2, 4, 2, 4, 3>(qop, qidx, q, r, rot, b, first_entry, n, code, mask, ld, s);
    default:
      if (r >= 22) return launch_rot_cfg<kK, 2, 2, 4, 2, 4, 3>(qop, qidx, q, r, rot, b, first_entry, n, code, mask, ld, s);
      return launch_rot_cfg<kK, 2, 2, 4, 2, 4, 5>(qop, qidx, q, r, rot, b, first_entry, n, code, mask, ld, s);
  }
}

}  // namespace imc
