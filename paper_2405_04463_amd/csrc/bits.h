// bits.h -- bit-sliced helpers shared by the comparison kernels: 64
// comparisons per lane, bit o of every u64 word belonging to column 64w + o.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imc {

// Ties `pos` to `dep` for the compiler only (no instruction): keeps a block's
// generation after the gates that precede it, so at most a few blocks are
// live at once instead of the whole tape.
__device__ __forceinline__ uint64_t after(uint64_t pos, uint64_t dep) {
  uint32_t lo = uint32_t(pos), d = uint32_t(dep);
  asm volatile("" : "+v"(lo) : "v"(d));
  return (pos & 0xFFFFFFFF00000000ull) | lo;
}

__device__ __forceinline__ uint64_t word64(const uint32_t* w, int u) {
  return uint64_t(w[2 * u]) | (uint64_t(w[2 * u + 1]) << 32);
}

// 64 u16 values (one per comparison) -> 16 bit planes: plane[b] bit o = bit b of v[o].
// R[j] = v[j] | v[j+32] << 16 for j < 32; a 32x32 bit transpose turns row j
// into column j; plane b = R[b] | R[b+16] << 32.
__device__ __forceinline__ void to_planes(const uint32_t W[32], uint64_t plane[16]) {
  uint32_t R[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const uint32_t lo = W[j >> 1], hi = W[16 + (j >> 1)];
    R[j] = (j & 1) ? ((lo >> 16) | (hi & 0xFFFF0000u)) : ((lo & 0xFFFFu) | (hi << 16));
  }
#pragma unroll
  for (int lv = 0; lv < 5; ++lv) {
    const int s = 16 >> lv;
    const uint32_t m = lv == 0 ? 0x0000FFFFu : lv == 1 ? 0x00FF00FFu : lv == 2 ? 0x0F0F0F0Fu
                     : lv == 3 ? 0x33333333u : 0x55555555u;   // bits b with (b & s) == 0
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      if (j & s) continue;
      const uint32_t t = ((R[j] >> s) ^ R[j + s]) & m;
      R[j + s] ^= t;
      R[j] ^= t << s;
    }
  }
#pragma unroll
  for (int b = 0; b < 16; ++b) plane[b] = uint64_t(R[b]) | (uint64_t(R[b + 16]) << 32);
}

// Load 64 u16 of one row starting at column col0 (valid columns < nval).
__device__ __forceinline__ void load64(const uint16_t* row, uint64_t col0, int nval, bool vec_ok, uint32_t W[32]) {
  if (vec_ok && nval == 64) {
    const uint4* p = reinterpret_cast<const uint4*>(row + col0);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint4 v = p[i];
      W[4 * i] = v.x; W[4 * i + 1] = v.y; W[4 * i + 2] = v.z; W[4 * i + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const uint32_t a = (2 * i < nval) ? row[col0 + 2 * i] : 0u;
      const uint32_t b = (2 * i + 1 < nval) ? row[col0 + 2 * i + 1] : 0u;
      W[i] = a | (b << 16);
    }
  }
}

// a -= b over NB bit planes (mod 2^NB).
template <int NB>
__device__ __forceinline__ void sub_planes(uint64_t (&a)[NB], const uint64_t (&b)[NB]) {
  uint64_t br = 0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const uint64_t x = a[j], y = b[j];
    a[j] = x ^ y ^ br;
    br = (~x & y) | (~(x ^ y) & br);
  }
}

}  // namespace imc
