// dot.hip -- party-local dot products of the shared protocol (Alg. 3, the
// code and mask inner products; App. C: two plain dot products per MPC dot
// product) as i8 MFMA with i32 accumulation over balanced byte limbs.
//
// v = lo + 256 hi (mod 2^16), lo, hi signed bytes.  For u, v in Z_2^16:
//   u v = lo_u lo_v + 256 (lo_u hi_v + hi_u lo_v)  (mod 2^16)
// (the hi*hi term carries 2^16 and vanishes), so each output needs
// acc0 = sum lo lo and acc1 = sum (lo hi + hi lo): three MFMA streams into two
// accumulators.  |acc0| <= 25600 * 2^14 < 2^31 and |acc1| <= 2 * 25600 * 2^14
// < 2^31, so no accumulator wraps.
#include "device.h"
#include "launch.h"

namespace imc {


// ---------------------------------------------------------------------------
// Rotation expand: query operand rows (row-major, unrotated) -> rotated rows
// in the MFMA-native tiled layout [row-block][plane 4][k-chunk 1600][32][16 B].
// ---------------------------------------------------------------------------
struct Rot {
  int8_t s[IMC_MAX_ROT_DEV];
};

template <int K>
__global__ void __launch_bounds__(256) expand_kernel(const int8_t* __restrict__ qop, const uint32_t* __restrict__ qidx,
                                                     uint32_t q, uint32_t r, Rot rot, uint32_t rows_pad,
                                                     int8_t* __restrict__ a) {
  using G = Geo<K>;
  uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint64_t total = uint64_t(rows_pad) * kPlanes * G::kChunks;
  if (t >= total) return;
  uint32_t slot = uint32_t(t % 32);
  uint64_t rest = t / 32;
  uint32_t kc = uint32_t(rest % G::kChunks);
  rest /= G::kChunks;
  uint32_t plane = uint32_t(rest % kPlanes);
  uint32_t rb = uint32_t(rest / kPlanes);
  uint32_t row = rb * 32 + slot;
  uint4 v = make_uint4(0, 0, 0, 0);
  if (row < q * r) {
    uint32_t qi = row / r, ri = row % r;
    if (qidx) qi = qidx[qi];
    int s = rot.s[ri];
    uint32_t k0 = kc * 16;
    uint32_t h = k0 / kCodeBits, i0 = k0 - h * kCodeBits;
    uint32_t rrow = i0 / kRowLen, w0 = i0 - rrow * kRowLen;
    const int8_t* src = qop + uint64_t(qi) * G::kQopRowBytes + uint64_t(plane) * G::kK + h * kCodeBits + rrow * kRowLen;
    uint32_t wv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int w = int(w0) + 4 * j - 4 * s;
      w = (w % kRowLen + kRowLen) % kRowLen;
      wv[j] = *reinterpret_cast<const uint32_t*>(src + w);
    }
    v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
  }
  *reinterpret_cast<uint4*>(a + uint64_t(rb) * G::kBlockBytes + uint64_t(plane) * G::kPlaneBlockBytes + uint64_t(kc) * 512 +
                            slot * 16) = v;
}

// Same, with an explicit row table (query index, rotation) per row: rows of
// many uneven batches expanded into one operand.  A row whose query index is
// out of range becomes a zero row.
template <int K>
__global__ void __launch_bounds__(256) expand_rows_kernel(const int8_t* __restrict__ qop, uint32_t q,
                                                          const imc_row* __restrict__ rows, uint32_t nrows,
                                                          uint32_t rows_pad, int8_t* __restrict__ a) {
  using G = Geo<K>;
  uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint64_t total = uint64_t(rows_pad) * kPlanes * G::kChunks;
  if (t >= total) return;
  uint32_t slot = uint32_t(t % 32);
  uint64_t rest = t / 32;
  uint32_t kc = uint32_t(rest % G::kChunks);
  rest /= G::kChunks;
  uint32_t plane = uint32_t(rest % kPlanes);
  uint32_t rb = uint32_t(rest / kPlanes);
  uint32_t row = rb * 32 + slot;
  uint4 v = make_uint4(0, 0, 0, 0);
  if (row < nrows && rows[row].query_index < q) {
    const uint32_t qi = rows[row].query_index;
    const int s = rows[row].rot % kRowLen;
    uint32_t k0 = kc * 16;
    uint32_t h = k0 / kCodeBits, i0 = k0 - h * kCodeBits;
    uint32_t rrow = i0 / kRowLen, w0 = i0 - rrow * kRowLen;
    const int8_t* src = qop + uint64_t(qi) * G::kQopRowBytes + uint64_t(plane) * G::kK + h * kCodeBits + rrow * kRowLen;
    uint32_t wv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int w = int(w0) + 4 * j - 4 * s;
      w = (w % kRowLen + kRowLen) % kRowLen;
      wv[j] = *reinterpret_cast<const uint32_t*>(src + w);
    }
    v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
  }
  *reinterpret_cast<uint4*>(a + uint64_t(rb) * G::kBlockBytes + uint64_t(plane) * G::kPlaneBlockBytes + uint64_t(kc) * 512 +
                            slot * 16) = v;
}

// ---------------------------------------------------------------------------
// dot kernel.  Workgroup tile BM rows x BN entries, WAVES_M x WAVES_N waves of
// (32 WM) x (32 WN) outputs (WM x WN MFMA 32x32x32 blocks, two accumulators
// each).  Per K-step (32 bytes of k per plane) the workgroup stages its
// operand slices in LDS once -- A: BM/32 row-blocks, B: BN/32 entry-blocks,
// each 2 planes x 2 k-chunks x 32 slots x 16 B, i.e. exactly the tiled HBM
// layout -- so fragment reads are 1 KB contiguous per wave.  Three LDS stages
// and NSETS register sets keep the global loads NSETS + 2 steps ahead and the
// fragment reads one step ahead of the MFMAs.  blockIdx.z = 0
// code, 1 mask.
// ---------------------------------------------------------------------------
struct DotArgs {
  const int8_t* a;       // rotated query operand, tiled, rows_pad rows
  const int8_t* b;       // party's database region
  uint16_t* out[2];      // code, mask: [rows][ld]
  uint64_t ld;
  uint32_t rows;         // q * r
  uint32_t a_blocks;     // row-blocks present in a
  uint64_t b_block0;     // first database block (first_entry_id / 32)
  uint64_t b_blocks;     // database blocks holding columns [0, n)
  uint64_t n;            // columns
  uint32_t mt, nt;       // tiles along rows / columns
  uint32_t persistent;   // grid smaller than the tile count: loop over tiles
};

template <int WM, int WN, int WAVES_M, int WAVES_N>
struct DotCfg {
  static constexpr int kBM = 32 * WM * WAVES_M, kBN = 32 * WN * WAVES_N;
  static constexpr int kThreads = 64 * WAVES_M * WAVES_N;
  static constexpr int kABlk = kBM / 32, kBBlk = kBN / 32;
  static constexpr int kChunksPerStep = (kABlk + kBBlk) * 2 * 2 * 32;   // 16-byte chunks
  static constexpr int kPerThread = kChunksPerStep / kThreads;
  static constexpr int kStageBytes = kChunksPerStep * 16;
  static_assert(kChunksPerStep % kThreads == 0, "chunks must divide evenly");
};

template <int K, int WM, int WN, int WAVES_M, int WAVES_N, int NSETS>
__global__ void __launch_bounds__(64 * WAVES_M * WAVES_N) dot_kernel(DotArgs args) {
  using C = DotCfg<WM, WN, WAVES_M, WAVES_N>;
  using G = Geo<K>;
  extern __shared__ __align__(16) int8_t lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  const int vec = blockIdx.z;
  // XCD-aware order: workgroup i runs on XCD i % 8; the workgroups one XCD
  // holds at a time are all row tiles of a few column tiles, so each database
  // slice is fetched from HBM once and served to them from that XCD's L2.
  // With a persistent grid (args.persistent) each workgroup walks its XCD's
  // tile sequence with stride gridDim.x / 8; otherwise one tile per workgroup.
  const uint32_t i = blockIdx.x;
  const uint32_t xcd = i & 7;
  const uint32_t s_end = ((args.nt + 7) / 8) * args.mt;
  const uint32_t s_step = args.persistent ? (gridDim.x >> 3) : s_end;
  for (uint32_t s = i >> 3; s < s_end; s += s_step) {
  const uint32_t u = s % args.mt, tg = s / args.mt;
  const uint32_t t = tg * 8 + xcd;
  if (t >= args.nt) continue;

  // Global source of each 16-byte chunk this thread stages per K-step.
  // Chunk c: block (A row-blocks first, then B entry-blocks), plane, k-chunk, slot.
  const int8_t* src[C::kPerThread];
#pragma unroll
  for (int j = 0; j < C::kPerThread; ++j) {
    const int c = tid + j * C::kThreads;
    const int blk = c >> 7, rem = c & 127;
    const int plane = rem >> 6, kcl = (rem >> 5) & 1, slot = rem & 31;
    const int8_t* base;
    if (blk < C::kABlk) {
      uint32_t rb = u * C::kABlk + blk;
      rb = rb < args.a_blocks ? rb : args.a_blocks - 1;
      base = args.a + size_t(rb) * G::kBlockBytes;
    } else {
      uint64_t cb = uint64_t(t) * C::kBBlk + (blk - C::kABlk);
      cb = cb < args.b_blocks ? cb : args.b_blocks - 1;
      base = args.b + size_t(args.b_block0 + cb) * G::kBlockBytes;
    }
    src[j] = base + size_t(2 * vec + plane) * G::kPlaneBlockBytes + size_t(kcl) * 512 + slot * 16;
  }

  v16i acc0[WM][WN], acc1[WM][WN];
#pragma unroll
  for (int x = 0; x < WM; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) { acc0[x][y][e] = 0; acc1[x][y][e] = 0; }

  constexpr int kSteps = G::kChunks / 2;   // steps of 32 bytes of k
  static_assert(kSteps % NSETS == 0, "the K loop is unrolled by NSETS");
  v4i rs[NSETS][C::kPerThread];
#define IMC_GLOAD(R, KS)                                                              \
  _Pragma("unroll") for (int c_ = 0; c_ < C::kPerThread; ++c_)                        \
      R[c_] = *reinterpret_cast<const v4i*>(src[c_] + size_t(2 * (KS)) * 512);
#define IMC_LSTORE(R, STAGE)                                                          \
  _Pragma("unroll") for (int c_ = 0; c_ < C::kPerThread; ++c_)                        \
      *reinterpret_cast<v4i*>(lds + (STAGE) * C::kStageBytes + (tid + c_ * C::kThreads) * 16) = R[c_];
#define IMC_FRAGS(ALO, AHI, BLO, BHI, STAGE)                                          \
  {                                                                                   \
    const int8_t* st_ = lds + (STAGE) * C::kStageBytes;                               \
    _Pragma("unroll") for (int x_ = 0; x_ < WM; ++x_) {                               \
      const int8_t* p_ = st_ + (wm * WM + x_) * 2048 + lane * 16;                     \
      ALO[x_] = *reinterpret_cast<const v4i*>(p_);                                    \
      AHI[x_] = *reinterpret_cast<const v4i*>(p_ + 1024);                             \
    }                                                                                 \
    _Pragma("unroll") for (int y_ = 0; y_ < WN; ++y_) {                               \
      const int8_t* p_ = st_ + (C::kABlk + wn * WN + y_) * 2048 + lane * 16;          \
      BLO[y_] = *reinterpret_cast<const v4i*>(p_);                                    \
      BHI[y_] = *reinterpret_cast<const v4i*>(p_ + 1024);                             \
    }                                                                                 \
  }

  // Pipeline over three LDS stages: step j is global-loaded NSETS iterations
  // ahead into register set (j - 2) % NSETS, written to stage j % 3 two
  // iterations ahead, and its fragments are read from LDS one iteration ahead,
  // while the MFMAs of the current step run.  Iteration k overwrites stage
  // (k + 2) % 3, last read at iteration k - 2.  Indices past the last step
  // are clamped (redundant reloads instead of branches keep the sets in VGPRs).
  v4i falo[WM], fahi[WM], fblo[WN], fbhi[WN];     // fragments of the current step
  v4i nalo[WM], nahi[WM], nblo[WN], nbhi[WN];     // fragments of the next step
  {
    v4i r0[C::kPerThread];
    IMC_GLOAD(r0, 0)
    IMC_LSTORE(r0, 0)
    IMC_GLOAD(r0, 1)
    IMC_LSTORE(r0, 1)
  }
#pragma unroll
  for (int set = 0; set < NSETS; ++set) { IMC_GLOAD(rs[set], set + 2) }
  __syncthreads();
  IMC_FRAGS(falo, fahi, fblo, fbhi, 0)
  for (int k0 = 0; k0 < kSteps; k0 += NSETS) {
#pragma unroll
    for (int uu = 0; uu < NSETS; ++uu) {
      const int k = k0 + uu;
      IMC_FRAGS(nalo, nahi, nblo, nbhi, (k + 1) % 3)
#pragma unroll
      for (int x = 0; x < WM; ++x)
#pragma unroll
        for (int y = 0; y < WN; ++y) {
          acc0[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(falo[x], fblo[y], acc0[x][y], 0, 0, 0);
          acc1[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(falo[x], fbhi[y], acc1[x][y], 0, 0, 0);
          acc1[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fahi[x], fblo[y], acc1[x][y], 0, 0, 0);
        }
      IMC_LSTORE(rs[uu], (k + 2) % 3)             // step k + 2
      __syncthreads();
      IMC_GLOAD(rs[uu], min(k + 2 + NSETS, kSteps - 1))
#pragma unroll
      for (int x = 0; x < WM; ++x) { falo[x] = nalo[x]; fahi[x] = nahi[x]; }
#pragma unroll
      for (int y = 0; y < WN; ++y) { fblo[y] = nblo[y]; fbhi[y] = nbhi[y]; }
    }
  }
#undef IMC_FRAGS
#undef IMC_GLOAD
#undef IMC_LSTORE
#undef IMC_COMPUTE

  // Epilogue: 32x32 block, lane l holds column l%32, register e holds row
  // 8*(e/4) + 4*(l/32) + e%4.
  uint16_t* out = args.out[vec];
#pragma unroll
  for (int x = 0; x < WM; ++x)
#pragma unroll
    for (int y = 0; y < WN; ++y) {
      const uint64_t col = uint64_t(t) * C::kBN + (wn * WN + y) * 32 + (lane & 31);
      if (col >= args.n) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const uint32_t row = u * C::kBM + (wm * WM + x) * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (row < args.rows) {
          const uint32_t z = uint32_t(acc0[x][y][e]) + (uint32_t(acc1[x][y][e]) << 8);
          out[uint64_t(row) * args.ld + col] = uint16_t(z);
        }
      }
    }
  __syncthreads();   // the next tile's prologue reuses the LDS stages
  }
}

hipError_t launch_expand(const int8_t* qop, const uint32_t* qidx, uint32_t q, uint32_t r, const int8_t* rot, int8_t* a,
                         uint32_t rows_pad, hipStream_t s, bool galois) {
  Rot rr;
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) rr.s[i] = i < int(r) ? rot[i] : 0;
  const uint64_t chunks = galois ? Geo<kKGalois>::kChunks : Geo<kK>::kChunks;
  const uint64_t total = uint64_t(rows_pad) * kPlanes * chunks;
  if (!fits_grid(total, 256)) return hipErrorInvalidValue;
  const dim3 grid(unsigned((total + 255) / 256));
  if (galois)
    hipLaunchKernelGGL(expand_kernel<kKGalois>, grid, dim3(256), 0, s, qop, qidx, q, r, rr, rows_pad, a);
  else
    hipLaunchKernelGGL(expand_kernel<kK>, grid, dim3(256), 0, s, qop, qidx, q, r, rr, rows_pad, a);
  return hipGetLastError();
}

template <int K, int WM, int WN, int WAVES_M, int WAVES_N, int NSETS>
static hipError_t launch_dot_cfg(DotArgs d, uint32_t rows, uint64_t n, hipStream_t s, bool persistent) {
  using C = DotCfg<WM, WN, WAVES_M, WAVES_N>;
  d.mt = (rows + C::kBM - 1) / C::kBM;
  d.nt = uint32_t((n + C::kBN - 1) / C::kBN);
  const uint32_t ntg = (d.nt + 7) / 8;
  if (uint64_t(ntg) * 8 * d.mt > 0x7FFFFFFFull) return hipErrorInvalidValue;
  uint32_t blocks = ntg * 8 * d.mt;
  d.persistent = 0;
  if (persistent) {
    // one resident workgroup per CU (two waves per SIMD)
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint32_t want = uint32_t(((cus + 7) / 8) * 8);
    if (want < blocks) {
      blocks = want;
      d.persistent = 1;
    }
  }
  const dim3 grid(blocks, 1, d.out[1] ? 2 : 1);   // z: code, mask (no mask dot when masks are public)
  const size_t lds = 3 * size_t(C::kStageBytes);
  auto kern = dot_kernel<K, WM, WN, WAVES_M, WAVES_N, NSETS>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, dim3(C::kThreads), lds, s, d);
  return hipGetLastError();
}

hipError_t launch_expand_rows(const int8_t* qop, uint32_t q, const imc_row* rows, uint32_t nrows, int8_t* a,
                              uint32_t rows_pad, hipStream_t s, bool galois) {
  const uint64_t chunks = galois ? Geo<kKGalois>::kChunks : Geo<kK>::kChunks;
  const uint64_t total = uint64_t(rows_pad) * kPlanes * chunks;
  if (!fits_grid(total, 256)) return hipErrorInvalidValue;
  const dim3 grid(unsigned((total + 255) / 256));
  if (galois)
    hipLaunchKernelGGL(expand_rows_kernel<kKGalois>, grid, dim3(256), 0, s, qop, q, rows, nrows, rows_pad, a);
  else
    hipLaunchKernelGGL(expand_rows_kernel<kK>, grid, dim3(256), 0, s, qop, q, rows, nrows, rows_pad, a);
  return hipGetLastError();
}

template <int K>
static hipError_t launch_dot_k(DotArgs d, uint32_t rows, uint64_t n, hipStream_t s, int variant) {
  const bool persistent = (variant & IMC_DOT_PERSISTENT) != 0;
  switch (variant & 0xF) {
    case 2: return launch_dot_cfg<K, 2, 2, 2, 2, 2>(d, rows, n, s, persistent);    // 128 x 128, 4 waves of 64 x 64
    case 3: return launch_dot_cfg<K, 2, 2, 4, 2, 1>(d, rows, n, s, persistent);    // 256 x 128, loads 3 steps ahead
    default: return launch_dot_cfg<K, 2, 2, 4, 2, 2>(d, rows, n, s, persistent);   // 256 x 128, loads 4 steps ahead
  }
}

hipError_t launch_dot(const int8_t* a, uint32_t rows, uint32_t a_blocks, const int8_t* b, uint64_t first_entry,
                      uint64_t n, uint16_t* code, uint16_t* mask, uint64_t ld, hipStream_t s, int variant,
                      bool galois) {
  if (rows == 0 || n == 0) return hipSuccess;
  DotArgs d;
  d.a = a;
  d.b = b;
  d.out[0] = code;
  d.out[1] = mask;
  d.ld = ld;
  d.rows = rows;
  d.a_blocks = a_blocks;
  d.b_block0 = first_entry / 32;
  d.b_blocks = (n + 31) / 32;
  d.n = n;
  return galois ? launch_dot_k<kKGalois>(d, rows, n, s, variant) : launch_dot_k<kK>(d, rows, n, s, variant);
}

}  // namespace imc
