// device.h -- device-side building blocks shared by the library's kernels:
// the ChaCha12 PRF (the protocol's RNG.Gen, App. D), its stream addressing,
// balanced byte limbs, and the layout constants of the HBM buffers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imc {

constexpr int kCodeBits = 12800;         // l (Sec. 3)
constexpr int kWords = 200;              // u64 words per packed code
constexpr int kRowLen = 800;             // elements per angular row (200 columns x 4 bits)
constexpr int kK = 2 * kCodeBits;        // K of one dot: [own | prev] halves, 25,600
constexpr int kChunks = kK / 16;         // 16-byte k-chunks per limb plane, 1600
constexpr int kPlanes = 4;               // code lo, code hi, mask lo, mask hi
constexpr size_t kPlaneBlockBytes = size_t(kChunks) * 32 * 16;          // 819,200
constexpr size_t kBlockBytes = kPlanes * kPlaneBlockBytes;              // 32 entries, 3,276,800
constexpr size_t kEntryBytes = kBlockBytes / 32;                       // 102,400
constexpr size_t kQopRowBytes = size_t(kPlanes) * kK;                  // 102,400

// Operand geometry of one dot product with K byte-limb elements per vector
// and plane: K = 25,600 for the replicated form ([own | previous] halves) and
// 12,800 for the Galois-ring Shamir form (one share).
template <int K>
struct Geo {
  static constexpr int kK = K;
  static constexpr int kChunks = K / 16;                                      // 16-byte k-chunks per plane
  static constexpr size_t kPlaneBlockBytes = size_t(kChunks) * 32 * 16;       // 32 entries
  static constexpr size_t kBlockBytes = kPlanes * kPlaneBlockBytes;
  static constexpr size_t kQopRowBytes = size_t(kPlanes) * K;
  static_assert(K % kRowLen == 0 && K % 32 == 0, "K spans whole angular rows");
};
constexpr int kKGalois = kCodeBits;                                           // 12,800

// One angular row of a query operand plane as the rotation-aware kernels keep
// it in LDS: 800 bytes with 64 bytes of circular padding on both sides, so
// that a row rotated by s (|s| <= 15, 4s bytes) is read in place.
constexpr int kSegPad = 64;                       // >= 4 * 15 and a multiple of 16
constexpr int kSegBytes = kRowLen + 2 * kSegPad;  // 928
constexpr int kSegChunks = kSegBytes / 16;        // 58

// PRF domains: high byte of the 64-bit stream id.
constexpr uint32_t kDomShareDb = 1, kDomShareQuery = 2, kDomReshare = 3, kDomCmp = 4, kDomOr = 5;
constexpr uint32_t kDomGaloisDb = 6, kDomGaloisQuery = 7, kDomOrPairs = 8;
constexpr uint32_t kDomCmpPlain = 9, kDomCmpLift18 = 10, kDomCmpConst32 = 11;
constexpr uint32_t kDomShare32Db = 12, kDomShare32Query = 13, kDomReshare32 = 14;

// Per 64-entry group, each key's tape holds u64 words (8 per ChaCha block),
// 32 blocks reserved per group.  The comparison kernels document which words
// each of their AND gates and BitInject values take.
constexpr int kTapeBlocksPerGroup = 32;

// MFMA operand and accumulator vectors.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

struct Key {
  uint32_t w[8];
};
struct Keys3 {
  Key k[3];
};

__device__ __forceinline__ uint32_t rotl32(uint32_t v, int c) { return __builtin_rotateleft32(v, c); }

#define IMC_QR(a, b, c, d)          \
  a += b; d ^= a; d = rotl32(d, 16); \
  c += d; b ^= c; b = rotl32(b, 12); \
  a += b; d ^= a; d = rotl32(d, 8);  \
  c += d; b ^= c; b = rotl32(b, 7);

// ChaCha block function with 12 rounds; words 12..15 = (pos lo, pos hi,
// stream lo, stream hi); out = working state + input state.
__device__ __forceinline__ void chacha12(const Key& key, uint64_t stream, uint64_t pos, uint32_t out[16]) {
  const uint32_t c0 = 0x61707865u, c1 = 0x3320646eu, c2 = 0x79622d32u, c3 = 0x6b206574u;
  uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
  uint32_t x4 = key.w[0], x5 = key.w[1], x6 = key.w[2], x7 = key.w[3];
  uint32_t x8 = key.w[4], x9 = key.w[5], x10 = key.w[6], x11 = key.w[7];
  uint32_t x12 = uint32_t(pos), x13 = uint32_t(pos >> 32), x14 = uint32_t(stream), x15 = uint32_t(stream >> 32);
  const uint32_t i12 = x12, i13 = x13, i14 = x14, i15 = x15;
#pragma unroll 1
  for (int r = 0; r < 6; ++r) {   // kept rolled: ~100 instructions of code per inlined block
    IMC_QR(x0, x4, x8, x12) IMC_QR(x1, x5, x9, x13) IMC_QR(x2, x6, x10, x14) IMC_QR(x3, x7, x11, x15)
    IMC_QR(x0, x5, x10, x15) IMC_QR(x1, x6, x11, x12) IMC_QR(x2, x7, x8, x13) IMC_QR(x3, x4, x9, x14)
  }
  out[0] = x0 + c0; out[1] = x1 + c1; out[2] = x2 + c2; out[3] = x3 + c3;
  out[4] = x4 + key.w[0]; out[5] = x5 + key.w[1]; out[6] = x6 + key.w[2]; out[7] = x7 + key.w[3];
  out[8] = x8 + key.w[4]; out[9] = x9 + key.w[5]; out[10] = x10 + key.w[6]; out[11] = x11 + key.w[7];
  out[12] = x12 + i12; out[13] = x13 + i13; out[14] = x14 + i14; out[15] = x15 + i15;
}
// N ChaCha12 blocks (keys, streams and positions may differ) in one round
// loop, so the N independent states interleave (4N quarter-rounds per step).
template <int N>
__device__ __forceinline__ void chacha12_n(const Key* const keys[N], const uint64_t stream[N], const uint64_t pos[N],
                                           uint32_t out[N][16]) {
  uint32_t x[N][16];
#pragma unroll
  for (int b = 0; b < N; ++b) {
    x[b][0] = 0x61707865u; x[b][1] = 0x3320646eu; x[b][2] = 0x79622d32u; x[b][3] = 0x6b206574u;
#pragma unroll
    for (int i = 0; i < 8; ++i) x[b][4 + i] = keys[b]->w[i];
    x[b][12] = uint32_t(pos[b]); x[b][13] = uint32_t(pos[b] >> 32);
    x[b][14] = uint32_t(stream[b]); x[b][15] = uint32_t(stream[b] >> 32);
  }
#pragma unroll 1
  for (int r = 0; r < 6; ++r) {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      IMC_QR(x[b][0], x[b][4], x[b][8], x[b][12]) IMC_QR(x[b][1], x[b][5], x[b][9], x[b][13])
      IMC_QR(x[b][2], x[b][6], x[b][10], x[b][14]) IMC_QR(x[b][3], x[b][7], x[b][11], x[b][15])
    }
#pragma unroll
    for (int b = 0; b < N; ++b) {
      IMC_QR(x[b][0], x[b][5], x[b][10], x[b][15]) IMC_QR(x[b][1], x[b][6], x[b][11], x[b][12])
      IMC_QR(x[b][2], x[b][7], x[b][8], x[b][13]) IMC_QR(x[b][3], x[b][4], x[b][9], x[b][14])
    }
  }
#pragma unroll
  for (int b = 0; b < N; ++b) {
    out[b][0] = x[b][0] + 0x61707865u; out[b][1] = x[b][1] + 0x3320646eu;
    out[b][2] = x[b][2] + 0x79622d32u; out[b][3] = x[b][3] + 0x6b206574u;
#pragma unroll
    for (int i = 0; i < 8; ++i) out[b][4 + i] = x[b][4 + i] + keys[b]->w[i];
    out[b][12] = x[b][12] + uint32_t(pos[b]); out[b][13] = x[b][13] + uint32_t(pos[b] >> 32);
    out[b][14] = x[b][14] + uint32_t(stream[b]); out[b][15] = x[b][15] + uint32_t(stream[b] >> 32);
  }
}
#undef IMC_QR

__device__ __forceinline__ uint64_t row_stream(uint32_t dom, uint64_t qid, int rot) {
  return (uint64_t(dom) << 56) | ((qid & 0xFFFFFFFFFFFFull) << 8) | uint64_t(uint8_t(rot + 16));
}

__device__ __forceinline__ uint64_t share_stream(uint32_t dom, int vec, int comp, uint64_t id) {
  return (uint64_t(dom) << 56) | (uint64_t(vec) << 52) | (uint64_t(comp) << 48) | (id & 0xFFFFFFFFFFFFull);
}

// Balanced byte limbs of a Z_2^16 value: v = lo + 256*hi (mod 2^16), lo, hi in [-128, 127].
__device__ __forceinline__ void limbs(uint16_t v, int8_t& lo, int8_t& hi) {
  int l = int(int8_t(v & 0xFF));
  lo = int8_t(l);
  hi = int8_t(uint8_t(((int(v) - l) >> 8) & 0xFF));
}

// Rotation by s of element i in [0, 12800): source element of rot_s(v)[i].
__device__ __forceinline__ int rot_src(int i, int s) {
  int row = i / kRowLen, w = i - row * kRowLen;
  int src = w - 4 * s;
  src += (src < 0) ? kRowLen : 0;
  src -= (src >= kRowLen) ? kRowLen : 0;
  return row * kRowLen + src;
}

}  // namespace imc
