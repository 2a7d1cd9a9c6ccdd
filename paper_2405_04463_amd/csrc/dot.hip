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

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// Rotation expand: query operand rows (row-major, unrotated) -> rotated rows
// in the MFMA-native tiled layout [row-block][plane 4][k-chunk 1600][32][16 B].
// ---------------------------------------------------------------------------
struct Rot {
  int8_t s[IMC_MAX_ROT_DEV];
};

__global__ void __launch_bounds__(256) expand_kernel(const int8_t* __restrict__ qop, uint32_t q, uint32_t r, Rot rot,
                                                     uint32_t rows_pad, int8_t* __restrict__ a) {
  uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint64_t total = uint64_t(rows_pad) * kPlanes * kChunks;
  if (t >= total) return;
  uint32_t slot = uint32_t(t % 32);
  uint64_t rest = t / 32;
  uint32_t kc = uint32_t(rest % kChunks);
  rest /= kChunks;
  uint32_t plane = uint32_t(rest % kPlanes);
  uint32_t rb = uint32_t(rest / kPlanes);
  uint32_t row = rb * 32 + slot;
  uint4 v = make_uint4(0, 0, 0, 0);
  if (row < q * r) {
    uint32_t qi = row / r, ri = row % r;
    int s = rot.s[ri];
    uint32_t k0 = kc * 16;
    uint32_t h = k0 / kCodeBits, i0 = k0 - h * kCodeBits;
    uint32_t rrow = i0 / kRowLen, w0 = i0 - rrow * kRowLen;
    const int8_t* src = qop + uint64_t(qi) * kQopRowBytes + uint64_t(plane) * kK + h * kCodeBits + rrow * kRowLen;
    uint32_t wv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int w = int(w0) + 4 * j - 4 * s;
      w = (w % kRowLen + kRowLen) % kRowLen;
      wv[j] = *reinterpret_cast<const uint32_t*>(src + w);
    }
    v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
  }
  *reinterpret_cast<uint4*>(a + uint64_t(rb) * kBlockBytes + uint64_t(plane) * kPlaneBlockBytes + uint64_t(kc) * 512 +
                            slot * 16) = v;
}

// ---------------------------------------------------------------------------
// dot kernel: workgroup tile 128 rows x 128 entries, 4 waves of 64 x 64 (2x2
// MFMA 32x32x32 blocks).  Operand fragments are 1 KB contiguous in the tiled
// layout (lanes 0..31: chunk 2ks, lanes 32..63: chunk 2ks+1), loaded straight
// into registers.  blockIdx.z = 0 code, 1 mask.
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
};

__device__ __forceinline__ v4i ldfrag(const int8_t* base, int ks, int lane) {
  return *reinterpret_cast<const v4i*>(base + size_t(2 * ks + (lane >> 5)) * 512 + (lane & 31) * 16);
}

__global__ void __launch_bounds__(256) dot_kernel(DotArgs args) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int vec = blockIdx.z;
  // XCD-aware order: workgroup i runs on XCD i % 8; the workgroups one XCD
  // holds at a time share database tiles (all row tiles of a column tile).
  const uint32_t i = blockIdx.x;
  const uint32_t xcd = i & 7, s = i >> 3;
  const uint32_t u = s % args.mt, tg = s / args.mt;
  const uint32_t t = tg * 8 + xcd;
  if (t >= args.nt) return;

  const int8_t* abase[2];
  const int8_t* bbase[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    uint32_t rb = u * 4 + wm * 2 + x;
    rb = rb < args.a_blocks ? rb : args.a_blocks - 1;
    abase[x] = args.a + size_t(rb) * kBlockBytes + size_t(2 * vec) * kPlaneBlockBytes;
    uint64_t cb = uint64_t(t) * 4 + wn * 2 + x;
    cb = cb < args.b_blocks ? cb : args.b_blocks - 1;
    bbase[x] = args.b + size_t(args.b_block0 + cb) * kBlockBytes + size_t(2 * vec) * kPlaneBlockBytes;
  }

  v16i acc0[2][2], acc1[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) { acc0[x][y][e] = 0; acc1[x][y][e] = 0; }

  v4i alo[2], ahi[2], blo[2], bhi[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    alo[x] = ldfrag(abase[x], 0, lane);
    ahi[x] = ldfrag(abase[x] + kPlaneBlockBytes, 0, lane);
    blo[x] = ldfrag(bbase[x], 0, lane);
    bhi[x] = ldfrag(bbase[x] + kPlaneBlockBytes, 0, lane);
  }
  constexpr int kSteps = kChunks / 2;   // 800 steps of 32 bytes of k
  for (int ks = 0; ks < kSteps; ++ks) {
    v4i nalo[2], nahi[2], nblo[2], nbhi[2];
    const int kn = ks + 1 < kSteps ? ks + 1 : ks;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      nalo[x] = ldfrag(abase[x], kn, lane);
      nahi[x] = ldfrag(abase[x] + kPlaneBlockBytes, kn, lane);
      nblo[x] = ldfrag(bbase[x], kn, lane);
      nbhi[x] = ldfrag(bbase[x] + kPlaneBlockBytes, kn, lane);
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        acc0[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(alo[x], blo[y], acc0[x][y], 0, 0, 0);
        acc1[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(alo[x], bhi[y], acc1[x][y], 0, 0, 0);
        acc1[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ahi[x], blo[y], acc1[x][y], 0, 0, 0);
      }
#pragma unroll
    for (int x = 0; x < 2; ++x) { alo[x] = nalo[x]; ahi[x] = nahi[x]; blo[x] = nblo[x]; bhi[x] = nbhi[x]; }
  }

  // Epilogue: 32x32 block, lane l holds column l%32, register e holds row
  // 8*(e/4) + 4*(l/32) + e%4.
  uint16_t* out = args.out[vec];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      uint64_t col = uint64_t(t) * 128 + wn * 64 + y * 32 + (lane & 31);
      if (col >= args.n) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        uint32_t row = u * 128 + wm * 64 + x * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (row < args.rows) {
          uint32_t z = uint32_t(acc0[x][y][e]) + (uint32_t(acc1[x][y][e]) << 8);
          out[uint64_t(row) * args.ld + col] = uint16_t(z);
        }
      }
    }
}

hipError_t launch_expand(const int8_t* qop, uint32_t q, uint32_t r, const int8_t* rot, int8_t* a, uint32_t rows_pad,
                         hipStream_t s) {
  Rot rr;
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) rr.s[i] = i < int(r) ? rot[i] : 0;
  uint64_t total = uint64_t(rows_pad) * kPlanes * kChunks;
  hipLaunchKernelGGL(expand_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, qop, q, r, rr, rows_pad, a);
  return hipGetLastError();
}

hipError_t launch_dot(const int8_t* a, uint32_t rows, uint32_t a_blocks, const int8_t* b, uint64_t first_entry,
                      uint64_t n, uint16_t* code, uint16_t* mask, uint64_t ld, hipStream_t s) {
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
  d.mt = (rows + 127) / 128;
  d.nt = uint32_t((n + 127) / 128);
  uint32_t ntg = (d.nt + 7) / 8;
  dim3 grid(ntg * 8 * d.mt, 1, 2);
  hipLaunchKernelGGL(dot_kernel, grid, dim3(256), 0, s, d);
  return hipGetLastError();
}

}  // namespace imc
