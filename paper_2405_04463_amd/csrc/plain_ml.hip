// plain_ml.hip -- the mask overlap for the setting with masks in plain
// (Sec. 4.3, Alg. 2): the parties know every mask, so ml = |m' AND M| with
// m' the rotated query mask (Sec. 3) is a public integer that each party
// computes for itself; only the code dot is secret-shared.
//
// ml is a popcount "GEMM" over packed bits (200 u64 words per mask): one
// AND and one popcount per word pair, bound by the vector ALUs.  Query
// rotations are applied once per row by rotate_masks_kernel, so the main
// kernel reads plain packed rows.
#include "device.h"
#include "launch.h"

namespace imc {

struct RotMaskArgs {
  const uint64_t* masks;   // [q][200]
  uint64_t* out;           // [q*r][200]
  uint64_t q;
  int32_t r;
  int8_t rot[IMC_MAX_ROT_DEV];
};

// Word w of row qi*r + ri = bits 64w .. 64w+63 of rot_s(m_qi), s = rot[ri]:
// bit i of the rotated mask is bit rot_src(i, s) of the mask.
__global__ void __launch_bounds__(256) rotate_masks_kernel(RotMaskArgs a) {
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint64_t rows = a.q * uint64_t(a.r);
  if (t >= rows * kWords) return;
  const uint64_t row = t / kWords;
  const int w = int(t % kWords);
  const uint64_t* m = a.masks + (row / uint64_t(a.r)) * kWords;
  const int s = a.rot[row % uint64_t(a.r)];
  uint64_t v = 0;
#pragma unroll 8
  for (int b = 0; b < 64; ++b) {
    const int src = rot_src(64 * w + b, s);
    v |= ((m[src >> 6] >> (src & 63)) & 1ull) << b;
  }
  a.out[row * kWords + w] = v;
}

constexpr int kMlTM = 64, kMlTN = 128, kMlKC = 8;   // rows, entries, words per LDS stage

struct MlArgs {
  const uint64_t* rm;      // [rows][200] rotated query masks
  const uint64_t* dm;      // [n][200] database masks
  uint16_t* ml;            // [rows][ld]
  uint64_t rows, n, ld;
  uint32_t mt, nt;         // row tiles, entry tiles
};

// Workgroup tile 64 rows x 128 entries; thread (tr, tc) owns rows 4tr..4tr+3
// and entries tc + 16j.  Consecutive workgroups of one XCD walk the row tiles
// of one entry tile, so the entry masks are read from HBM about once per XCD.
// Held to 128 registers (it needs 125 then, no spills): four waves per SIMD
// instead of the three that 129 allowed.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) plain_ml_kernel(MlArgs a) {
  __shared__ uint64_t sa[kMlKC][kMlTM + 1];
  __shared__ uint64_t sb[kMlKC][kMlTN + 1];
  const uint32_t i = blockIdx.x, xcd = i & 7, s8 = i >> 3;
  const uint32_t u = s8 % a.mt, tt = (s8 / a.mt) * 8 + xcd;
  if (tt >= a.nt) return;
  const uint64_t r0 = uint64_t(u) * kMlTM, e0 = uint64_t(tt) * kMlTN;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  uint32_t acc[4][8];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 8; ++y) acc[x][y] = 0;

  for (int k0 = 0; k0 < kWords; k0 += kMlKC) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = tid + 256 * j, rr = c >> 3, ww = c & 7;
      const uint64_t row = r0 + rr;
      sa[ww][rr] = row < a.rows ? a.rm[row * kWords + k0 + ww] : 0ull;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = tid + 256 * j, ee = c >> 3, ww = c & 7;
      const uint64_t e = e0 + ee;
      sb[ww][ee] = e < a.n ? a.dm[e * kWords + k0 + ww] : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int ww = 0; ww < kMlKC; ++ww) {
      uint64_t x[4], y[8];
#pragma unroll
      for (int p = 0; p < 4; ++p) x[p] = sa[ww][4 * tr + p];
#pragma unroll
      for (int q = 0; q < 8; ++q) y[q] = sb[ww][tc + 16 * q];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[p][q] += uint32_t(__popcll(x[p] & y[q]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const uint64_t row = r0 + 4 * tr + p;
    if (row >= a.rows) continue;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint64_t e = e0 + tc + 16 * q;
      if (e < a.n) a.ml[row * a.ld + e] = uint16_t(acc[p][q]);
    }
  }
}

hipError_t launch_rotate_masks(const uint64_t* masks, uint64_t q, const imc_ids_dev& ids, uint64_t* out,
                               hipStream_t s) {
  const uint64_t threads = q * uint64_t(ids.r) * kWords;
  if (threads == 0) return hipSuccess;
  RotMaskArgs a;
  a.masks = masks;
  a.out = out;
  a.q = q;
  a.r = ids.r;
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) a.rot[i] = i < ids.r ? ids.rot[i] : 0;
  if (!fits_grid(threads, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rotate_masks_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_plain_ml(const uint64_t* row_masks, uint64_t rows, const uint64_t* db_masks, uint64_t n,
                           uint16_t* ml, uint64_t ld, hipStream_t s) {
  if (rows == 0 || n == 0) return hipSuccess;
  MlArgs a;
  a.rm = row_masks;
  a.dm = db_masks;
  a.ml = ml;
  a.rows = rows;
  a.n = n;
  a.ld = ld;
  a.mt = uint32_t((rows + kMlTM - 1) / kMlTM);
  a.nt = uint32_t((n + kMlTN - 1) / kMlTN);
  const uint64_t groups = uint64_t((a.nt + 7) / 8) * 8 * a.mt;
  if (groups > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(plain_ml_kernel, dim3(unsigned(groups)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace imc
