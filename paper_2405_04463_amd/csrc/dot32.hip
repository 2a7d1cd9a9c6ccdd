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
// k-chunk g holds x_p[16g..], k-chunk 800 + g holds x_{p-1}[16g..].
__global__ void __launch_bounds__(256) share32_db_kernel(Key dk, int vec, const uint64_t* codes, const uint64_t* masks,
                                                         uint64_t n, uint64_t first, uint8_t* d0, uint8_t* d1,
                                                         uint8_t* d2) {
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * (kCodeBits / 16)) return;
  const uint64_t j = t / (kCodeBits / 16);
  const int g = int(t % (kCodeBits / 16));
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
  int8_t rot[IMC_MAX_ROT_DEV];
};

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
  uint32_t z[3][8], G[3][8];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      z[p][j] = j < nval ? a.add[p][off + j] : 0u;
      G[p][j] = a.vec ? F[p][2 * j + 1] : F[p][2 * j];
    }
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int pm = (p + 2) % 3;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j >= nval) continue;
      const uint32_t own = z[p][j] + G[p][j] - G[pm][j];
      const uint32_t prev = z[pm][j] + G[pm][j] - G[(pm + 2) % 3][j];
      a.msg[p][off + j] = own;                 // party p -> party p+1
      a.rep[p][off + j] = own;
      a.rep[p][a.plane + off + j] = prev;      // received from party p-1
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_share32_db(const Key& dk, int vec, const uint64_t* codes, const uint64_t* masks, uint64_t n,
                             uint64_t first, uint8_t* const db[3], hipStream_t s) {
  const uint64_t threads = n * (kCodeBits / 16);
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(share32_db_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, dk, vec, codes, masks,
                     n, first, db[0], db[1], db[2]);
  return hipGetLastError();
}

hipError_t launch_share32_query(const Key& dk, int vec, const uint64_t* codes, const uint64_t* masks, uint64_t q,
                                uint64_t qid_base, int8_t* const op[3], hipStream_t s) {
  const uint64_t threads = q * (kCodeBits / 16);
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(share32_query_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, dk, vec, codes,
                     masks, q, qid_base, op[0], op[1], op[2]);
  return hipGetLastError();
}

hipError_t launch_dot32(const int8_t* qop, uint32_t q, uint32_t r, const int8_t* rot, const int8_t* b,
                        uint64_t first_entry, uint64_t n, uint32_t* out, uint64_t ld, hipStream_t s) {
  const uint32_t rows = q * r;
  if (rows == 0 || n == 0) return hipSuccess;
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
  for (int i = 0; i < IMC_MAX_ROT_DEV; ++i) a.rot[i] = i < ids.r ? ids.rot[i] : 0;
  const uint64_t threads = rows * ((n + 7) / 8);
  hipLaunchKernelGGL(reshare32_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

size_t db32_bytes(uint64_t capacity) { return size_t((capacity + 31) / 32) * kBlock32Bytes; }
size_t query32_op_bytes(uint64_t q) { return size_t(q) * kQop32RowBytes; }

}  // namespace imc
