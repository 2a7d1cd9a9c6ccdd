// share.hip -- enrolment and query sharing (Sec. 4.1.1 masked bits; App. C
// replicated sharing by a dealer), and appends of query shares to a database.
#include "device.h"
#include "launch.h"

namespace imc {

// Masked bit (T,U,F) = (-1,0,1): c' = m - 2 (c AND m) in Z_2^16; mask bit m as 0/1.
__device__ __forceinline__ uint16_t secret_elem(int vec, uint32_t cbits, uint32_t mbits, int b) {
  uint32_t c = (cbits >> b) & 1u, m = (mbits >> b) & 1u;
  return vec == 0 ? uint16_t(m - 2u * (c & m)) : uint16_t(m);
}

// One thread: 32 consecutive elements [32a, 32a+32) of one vector of one item,
// i.e. one ChaCha block per dealer component.  comps[c][j] for j < 32.
__device__ __forceinline__ void share32(const Key& dk, uint32_t dom, int vec, uint64_t id, int a,
                                        const uint64_t* code, const uint64_t* mask, uint16_t comps[3][32]) {
  uint32_t b0[16], b1[16];
  chacha12(dk, share_stream(dom, vec, 0, id), uint64_t(a), b0);
  chacha12(dk, share_stream(dom, vec, 1, id), uint64_t(a), b1);
  uint64_t cw = code[a >> 1], mw = mask[a >> 1];
  uint32_t cb = uint32_t(cw >> ((a & 1) * 32)), mb = uint32_t(mw >> ((a & 1) * 32));
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    uint16_t x = secret_elem(vec, cb, mb, j);
    uint16_t s0 = uint16_t((j & 1) ? (b0[j >> 1] >> 16) : (b0[j >> 1] & 0xFFFF));
    uint16_t s1 = uint16_t((j & 1) ? (b1[j >> 1] >> 16) : (b1[j >> 1] & 0xFFFF));
    comps[0][j] = s0;
    comps[1][j] = s1;
    comps[2][j] = uint16_t(x - s0 - s1);
  }
}

// Write 16 consecutive elements (k-chunk kc) of one half into the tiled
// database layout of one party, as lo and hi limb planes.
__device__ __forceinline__ void store_chunk(uint8_t* region, uint64_t e, int vec, int kc, const uint16_t* v) {
  uint8_t* base = region + (e >> 5) * kBlockBytes + size_t(kc) * 512 + (e & 31) * 16;
  uint32_t lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    int8_t l, h;
    limbs(v[j], l, h);
    lo[j >> 2] |= uint32_t(uint8_t(l)) << (8 * (j & 3));
    hi[j >> 2] |= uint32_t(uint8_t(h)) << (8 * (j & 3));
  }
  *reinterpret_cast<uint4*>(base + size_t(2 * vec) * kPlaneBlockBytes) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
  *reinterpret_cast<uint4*>(base + size_t(2 * vec + 1) * kPlaneBlockBytes) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
}

struct DbOut {
  uint8_t* p[3];
};

// Thread layout: 32 consecutive entries per 32 lanes, then (a, vec) pairs.
__global__ void __launch_bounds__(256) share_db_kernel(Key dk, const uint64_t* __restrict__ codes,
                                                       const uint64_t* __restrict__ masks, uint64_t n,
                                                       uint64_t first, DbOut db) {
  uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint64_t chunk = t / (32 * 800);
  uint32_t within = uint32_t(t % (32 * 800));
  uint32_t combo = within / 32, sub = within % 32;
  uint64_t idx = chunk * 32 + sub;
  if (idx >= n) return;
  int a = int(combo % 400), vec = int(combo / 400);
  uint64_t e = first + idx;
  uint16_t comps[3][32];
  share32(dk, kDomShareDb, vec, e, a, codes + idx * kWords, masks + idx * kWords, comps);
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    int pm = (p + 2) % 3;
    if (!db.p[p]) continue;   // this party's region is not held here
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      store_chunk(db.p[p], e, vec, 2 * a + h, &comps[p][16 * h]);                 // x_p at k = i
      store_chunk(db.p[p], e, vec, 800 + 2 * a + h, &comps[pm][16 * h]);         // x_{p-1} at k = 12800 + i
    }
  }
}

struct QOut {
  int8_t* op[3];
  uint16_t* raw[3];  // may be null
};

// Query operand: [q][plane 4][25600] i8; k < 12800: x_p + x_{p-1}; k >= 12800: x_p.
__global__ void __launch_bounds__(256) share_query_kernel(Key dk, const uint64_t* __restrict__ codes,
                                                          const uint64_t* __restrict__ masks, uint64_t q,
                                                          uint64_t qid_base, QOut out) {
  uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint64_t qi = t / 800;
  if (qi >= q) return;
  int combo = int(t % 800);
  int a = combo % 400, vec = combo / 400;
  uint16_t comps[3][32];
  share32(dk, kDomShareQuery, vec, qid_base + qi, a, codes + qi * kWords, masks + qi * kWords, comps);
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    int pm = (p + 2) % 3;
    int8_t* row = out.op[p] + qi * kQopRowBytes;
    uint32_t lo_s[8], hi_s[8], lo_o[8], hi_o[8];
#pragma unroll
    for (int w = 0; w < 8; ++w) lo_s[w] = hi_s[w] = lo_o[w] = hi_o[w] = 0;
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      int8_t l, h;
      limbs(uint16_t(comps[p][j] + comps[pm][j]), l, h);
      lo_s[j >> 2] |= uint32_t(uint8_t(l)) << (8 * (j & 3));
      hi_s[j >> 2] |= uint32_t(uint8_t(h)) << (8 * (j & 3));
      limbs(comps[p][j], l, h);
      lo_o[j >> 2] |= uint32_t(uint8_t(l)) << (8 * (j & 3));
      hi_o[j >> 2] |= uint32_t(uint8_t(h)) << (8 * (j & 3));
    }
    uint4* d0 = reinterpret_cast<uint4*>(row + size_t(2 * vec) * kK + 32 * a);
    uint4* d1 = reinterpret_cast<uint4*>(row + size_t(2 * vec + 1) * kK + 32 * a);
    uint4* d2 = reinterpret_cast<uint4*>(row + size_t(2 * vec) * kK + kCodeBits + 32 * a);
    uint4* d3 = reinterpret_cast<uint4*>(row + size_t(2 * vec + 1) * kK + kCodeBits + 32 * a);
    d0[0] = make_uint4(lo_s[0], lo_s[1], lo_s[2], lo_s[3]); d0[1] = make_uint4(lo_s[4], lo_s[5], lo_s[6], lo_s[7]);
    d1[0] = make_uint4(hi_s[0], hi_s[1], hi_s[2], hi_s[3]); d1[1] = make_uint4(hi_s[4], hi_s[5], hi_s[6], hi_s[7]);
    d2[0] = make_uint4(lo_o[0], lo_o[1], lo_o[2], lo_o[3]); d2[1] = make_uint4(lo_o[4], lo_o[5], lo_o[6], lo_o[7]);
    d3[0] = make_uint4(hi_o[0], hi_o[1], hi_o[2], hi_o[3]); d3[1] = make_uint4(hi_o[4], hi_o[5], hi_o[6], hi_o[7]);
    if (out.raw[p]) {
      uint16_t* r = out.raw[p] + qi * (2 * 2 * kCodeBits) + size_t(vec) * 2 * kCodeBits;
#pragma unroll
      for (int j = 0; j < 32; j += 2) {
        *reinterpret_cast<uint32_t*>(r + 32 * a + j) = uint32_t(comps[p][j]) | (uint32_t(comps[p][j + 1]) << 16);
        *reinterpret_cast<uint32_t*>(r + kCodeBits + 32 * a + j) =
            uint32_t(comps[pm][j]) | (uint32_t(comps[pm][j + 1]) << 16);
      }
    }
  }
}

// Append: party p's raw query shares (comp 0 = x_p, comp 1 = x_{p-1}) into slot e.
struct RawIn {
  const uint16_t* p[3];
};

__global__ void __launch_bounds__(256) append_kernel(RawIn raw, uint64_t qi, DbOut db, uint64_t e) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;   // one 16-element chunk of one (party, vec, half)
  if (t >= 3 * 2 * 2 * 800) return;
  int c = t % 800, h = (t / 800) % 2, vec = (t / 1600) % 2, p = t / 3200;
  if (!db.p[p]) return;   // this party's region is not held here
  const uint16_t* src = raw.p[p] + qi * (2 * 2 * kCodeBits) + size_t(vec) * 2 * kCodeBits + size_t(h) * kCodeBits + 16 * c;
  uint16_t v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = src[j];
  store_chunk(db.p[p], e, vec, h * 800 + c, v);
}

// ---------------------------------------------------------------------------
// Shamir sharing over the Galois ring GR = Z_2^16[X]/(X^2 - X - 1) (Sec.
// 4.3.2).  Elements 2i, 2i+1 of a vector form g_i = x_2i + x_2i+1 X; the
// dealer draws r_i in GR and party p receives g_i + r_i alpha_p at the points
// alpha = (1, X, 1 + X).  With X^2 = X + 1:
//   r X       = r1 + (r0 + r1) X
//   r (1 + X) = (r0 + r1) + (r0 + 2 r1) X.
// On the query side party p stores lambda_p times its share, lambda_p being
// its Lagrange coefficient for interpolating a degree-2 polynomial at 0 from
// the three points: 1/(X - 1) = X (as X (X - 1) = X^2 - X = 1), so
//   lambda_0 = X (1 + X) / ((X - 1) X) = (1 + X) X = 1 + 2X,
//   lambda_1 = (1 + X) / (1 - X)        = -(1 + 2X),
//   lambda_2 = X / ((-X)(-1))           = 1,
// and (l0 + l1 X)(s0 + s1 X) = (l0 s0 + l1 s1) + (l0 s1 + l1 s0 + l1 s1) X.
// The dot product then only needs constant terms: sum_i (a0 b0 + a1 b1), a
// plain length-12,800 dot product of the coefficient vectors.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t galois_stream(uint32_t dom, int vec, uint64_t id) {
  return (uint64_t(dom) << 56) | (uint64_t(vec) << 52) | (id & 0xFFFFFFFFFFFFull);
}

// One thread: elements [32a, 32a + 32) (pairs 16a .. 16a + 15) of one vector
// of one item, one ChaCha block; sh[p][j] = party p's share coefficients.
__device__ __forceinline__ void galois_share32(const Key& dk, uint32_t dom, int vec, uint64_t id, int a,
                                               const uint64_t* code, const uint64_t* mask, uint16_t sh[3][32]) {
  uint32_t b[16];
  chacha12(dk, galois_stream(dom, vec, id), uint64_t(a), b);
  uint64_t cw = code[a >> 1], mw = mask[a >> 1];
  uint32_t cb = uint32_t(cw >> ((a & 1) * 32)), mb = uint32_t(mw >> ((a & 1) * 32));
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint16_t g0 = secret_elem(vec, cb, mb, 2 * i), g1 = secret_elem(vec, cb, mb, 2 * i + 1);
    const uint16_t r0 = uint16_t(b[i] & 0xFFFF), r1 = uint16_t(b[i] >> 16);
    sh[0][2 * i] = uint16_t(g0 + r0);
    sh[0][2 * i + 1] = uint16_t(g1 + r1);
    sh[1][2 * i] = uint16_t(g0 + r1);
    sh[1][2 * i + 1] = uint16_t(g1 + r0 + r1);
    sh[2][2 * i] = uint16_t(g0 + r0 + r1);
    sh[2][2 * i + 1] = uint16_t(g1 + r0 + 2 * r1);
  }
}

// 16 consecutive elements (k-chunk kc) of one vector into a Galois-form
// database region as lo and hi limb planes.
__device__ __forceinline__ void store_chunk_galois(uint8_t* region, uint64_t e, int vec, int kc, const uint16_t* v) {
  using G = Geo<kKGalois>;
  uint8_t* base = region + (e >> 5) * G::kBlockBytes + size_t(kc) * 512 + (e & 31) * 16;
  uint32_t lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    int8_t l, h;
    limbs(v[j], l, h);
    lo[j >> 2] |= uint32_t(uint8_t(l)) << (8 * (j & 3));
    hi[j >> 2] |= uint32_t(uint8_t(h)) << (8 * (j & 3));
  }
  *reinterpret_cast<uint4*>(base + size_t(2 * vec) * G::kPlaneBlockBytes) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
  *reinterpret_cast<uint4*>(base + size_t(2 * vec + 1) * G::kPlaneBlockBytes) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
}

__global__ void __launch_bounds__(256) galois_share_db_kernel(Key dk, const uint64_t* __restrict__ codes,
                                                              const uint64_t* __restrict__ masks, uint64_t n,
                                                              uint64_t first, DbOut db) {
  uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint64_t chunk = t / (32 * 800);
  uint32_t within = uint32_t(t % (32 * 800));
  uint32_t combo = within / 32, sub = within % 32;
  uint64_t idx = chunk * 32 + sub;
  if (idx >= n) return;
  int a = int(combo % 400), vec = int(combo / 400);
  uint64_t e = first + idx;
  uint16_t sh[3][32];
  galois_share32(dk, kDomGaloisDb, vec, e, a, codes + idx * kWords, masks + idx * kWords, sh);
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    if (!db.p[p]) continue;
    store_chunk_galois(db.p[p], e, vec, 2 * a, &sh[p][0]);
    store_chunk_galois(db.p[p], e, vec, 2 * a + 1, &sh[p][16]);
  }
}

// Query operand: [q][plane 4][12800] i8 limbs of lambda_p times party p's share.
// raw[p] (optional): the plain share, u16 [q][vec 2][12800], for appends.
__global__ void __launch_bounds__(256) galois_share_query_kernel(Key dk, const uint64_t* __restrict__ codes,
                                                                 const uint64_t* __restrict__ masks, uint64_t q,
                                                                 uint64_t qid_base, QOut out) {
  using G = Geo<kKGalois>;
  uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint64_t qi = t / 800;
  if (qi >= q) return;
  int combo = int(t % 800);
  int a = combo % 400, vec = combo / 400;
  uint16_t sh[3][32];
  galois_share32(dk, kDomGaloisQuery, vec, qid_base + qi, a, codes + qi * kWords, masks + qi * kWords, sh);
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    int8_t* row = out.op[p] + qi * G::kQopRowBytes;
    uint32_t lo[8], hi[8];
#pragma unroll
    for (int w = 0; w < 8; ++w) lo[w] = hi[w] = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint16_t s0 = sh[p][2 * i], s1 = sh[p][2 * i + 1];
      uint16_t c0 = s0, c1 = s1;                       // lambda_2 = 1
      if (p < 2) {                                     // (1 + 2X)(s0 + s1 X) = (s0 + 2 s1) + (2 s0 + 3 s1) X
        c0 = uint16_t(s0 + 2 * s1);
        c1 = uint16_t(2 * s0 + 3 * s1);
        if (p == 1) {                                  // lambda_1 = -lambda_0
          c0 = uint16_t(0 - c0);
          c1 = uint16_t(0 - c1);
        }
      }
      int8_t l, h;
      limbs(c0, l, h);
      lo[i >> 1] |= uint32_t(uint8_t(l)) << (16 * (i & 1));
      hi[i >> 1] |= uint32_t(uint8_t(h)) << (16 * (i & 1));
      limbs(c1, l, h);
      lo[i >> 1] |= uint32_t(uint8_t(l)) << (16 * (i & 1) + 8);
      hi[i >> 1] |= uint32_t(uint8_t(h)) << (16 * (i & 1) + 8);
    }
    uint4* d0 = reinterpret_cast<uint4*>(row + size_t(2 * vec) * G::kK + 32 * a);
    uint4* d1 = reinterpret_cast<uint4*>(row + size_t(2 * vec + 1) * G::kK + 32 * a);
    d0[0] = make_uint4(lo[0], lo[1], lo[2], lo[3]); d0[1] = make_uint4(lo[4], lo[5], lo[6], lo[7]);
    d1[0] = make_uint4(hi[0], hi[1], hi[2], hi[3]); d1[1] = make_uint4(hi[4], hi[5], hi[6], hi[7]);
    if (out.raw[p]) {
      uint16_t* r = out.raw[p] + qi * (2 * kCodeBits) + size_t(vec) * kCodeBits + 32 * a;
#pragma unroll
      for (int j = 0; j < 32; j += 2)
        *reinterpret_cast<uint32_t*>(r + j) = uint32_t(sh[p][j]) | (uint32_t(sh[p][j + 1]) << 16);
    }
  }
}

// Append: party p's plain Galois share of query qi into slot e of its region.
__global__ void __launch_bounds__(256) galois_append_kernel(RawIn raw, uint64_t qi, DbOut db, uint64_t e) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;   // one 16-element chunk of one (party, vec)
  if (t >= 3 * 2 * 800) return;
  int c = t % 800, vec = (t / 800) % 2, p = t / 1600;
  if (!db.p[p]) return;
  const uint16_t* src = raw.p[p] + qi * (2 * kCodeBits) + size_t(vec) * kCodeBits + 16 * c;
  uint16_t v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = src[j];
  store_chunk_galois(db.p[p], e, vec, c, v);
}

hipError_t launch_galois_share_db(const Key& dk, const uint64_t* codes, const uint64_t* masks, uint64_t n,
                                  uint64_t first, uint8_t* const db[3], hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t threads = ((n + 31) / 32) * 32 * 800;
  DbOut o{{db[0], db[1], db[2]}};
  if (!fits_grid(threads, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(galois_share_db_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, dk, codes, masks,
                     n, first, o);
  return hipGetLastError();
}

hipError_t launch_galois_share_query(const Key& dk, const uint64_t* codes, const uint64_t* masks, uint64_t q,
                                     uint64_t qid_base, int8_t* const op[3], uint16_t* const raw[3], hipStream_t s) {
  if (q == 0) return hipSuccess;
  uint64_t threads = q * 800;
  QOut o{{op[0], op[1], op[2]}, {raw ? raw[0] : nullptr, raw ? raw[1] : nullptr, raw ? raw[2] : nullptr}};
  if (!fits_grid(threads, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(galois_share_query_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, dk, codes,
                     masks, q, qid_base, o);
  return hipGetLastError();
}

hipError_t launch_galois_append(const uint16_t* const raw[3], uint64_t qi, uint8_t* const db[3], uint64_t e,
                                hipStream_t s) {
  RawIn r{{raw[0], raw[1], raw[2]}};
  DbOut o{{db[0], db[1], db[2]}};
  hipLaunchKernelGGL(galois_append_kernel, dim3((3 * 2 * 800 + 255) / 256), dim3(256), 0, s, r, qi, o, e);
  return hipGetLastError();
}

hipError_t launch_share_db(const Key& dk, const uint64_t* codes, const uint64_t* masks, uint64_t n, uint64_t first,
                           uint8_t* const db[3], hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t threads = ((n + 31) / 32) * 32 * 800;
  DbOut o{{db[0], db[1], db[2]}};
  if (!fits_grid(threads, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(share_db_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, dk, codes, masks, n,
                     first, o);
  return hipGetLastError();
}

hipError_t launch_share_query(const Key& dk, const uint64_t* codes, const uint64_t* masks, uint64_t q,
                              uint64_t qid_base, int8_t* const op[3], uint16_t* const raw[3], hipStream_t s) {
  if (q == 0) return hipSuccess;
  uint64_t threads = q * 800;
  QOut o{{op[0], op[1], op[2]}, {raw ? raw[0] : nullptr, raw ? raw[1] : nullptr, raw ? raw[2] : nullptr}};
  if (!fits_grid(threads, 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(share_query_kernel, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s, dk, codes, masks, q,
                     qid_base, o);
  return hipGetLastError();
}

hipError_t launch_append(const uint16_t* const raw[3], uint64_t qi, uint8_t* const db[3], uint64_t e, hipStream_t s) {
  RawIn r{{raw[0], raw[1], raw[2]}};
  DbOut o{{db[0], db[1], db[2]}};
  hipLaunchKernelGGL(append_kernel, dim3((3 * 2 * 2 * 800 + 255) / 256), dim3(256), 0, s, r, qi, o, e);
  return hipGetLastError();
}

}  // namespace imc
