// api.cpp -- the C ABI (include/irismpc.h): argument checks, the context and
// its scratch, and dispatch to the kernels.  Every argument error is found
// here, before anything is enqueued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/irismpc.h"
#include "device.h"
#include "launch.h"

struct imc_ctx {
  int device;
  imc::Key dealer;
  imc::Keys3 party;
  uint32_t max_rows;
  int dot_variant;                // dot kernel tile configuration (params->flags & 0xF)
  int8_t* rot_op;                 // rotated query operand, max_rows (rounded to 32) rows
  size_t rot_op_bytes;
  unsigned long long* bad;        // open-check counter
};

// Device array behind imc_dot_shares_rows_noalloc: the expanded rotated query
// rows of one call (IMC_NOALLOC_MAX_ROWS rows in blocks of 32).  Each GPU the
// library runs on holds its own copy until the process ends.  In host code
// the name is only a handle for hipGetSymbolAddress: kernels and copies take
// the per-device address resolved at context creation.
static __device__ __align__(256) int8_t scratch[(IMC_NOALLOC_MAX_ROWS / 32) * imc::kBlockBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
std::atomic<int8_t*> g_scratch[kMaxDevices];   // address of `scratch` on each device, null until resolved

// Resolve `scratch` on `device`, which must be the current device.  Once per device.
imc_status resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return IMC_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device].load(std::memory_order_acquire)) return IMC_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return IMC_EDEVICE;
  g_scratch[device].store(static_cast<int8_t*>(ptr), std::memory_order_release);
  return IMC_OK;
}

imc::Key load_key(const uint8_t* b) {
  imc::Key k;
  for (int i = 0; i < 8; ++i)
    k.w[i] = uint32_t(b[4 * i]) | (uint32_t(b[4 * i + 1]) << 8) | (uint32_t(b[4 * i + 2]) << 16) |
             (uint32_t(b[4 * i + 3]) << 24);
  return k;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

imc_status dev_status(hipError_t e) { return e == hipSuccess ? IMC_OK : IMC_EDEVICE; }

// Make the context's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) return;
    ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (ok && hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

imc_status check_ids(const imc_ids* ids) {
  if (!ids) return IMC_EINVAL;
  if (ids->r < 1 || ids->r > IMC_MAX_ROT) return IMC_EINVAL;
  for (int i = 0; i < ids->r; ++i)
    if (ids->rot[i] < -15 || ids->rot[i] > 15) return IMC_EINVAL;
  if (ids->first_entry_id % 64) return IMC_EINVAL;
  if (ids->query_id_base >= (1ull << 48)) return IMC_EINVAL;
  return IMC_OK;
}

size_t blocks_for(size_t capacity) { return (capacity + 31) / 32; }

bool tiles_ok(uint32_t flags) {
  const uint32_t t = flags & 0xFu;
  return (flags & ~0x1Fu) == 0 && t <= IMC_DOT_TILES_MAX && t != 5;
}

}  // namespace

extern "C" {

const char* imc_strerror(imc_status s) {
  switch (s) {
    case IMC_OK: return "ok";
    case IMC_EINVAL: return "invalid argument";
    case IMC_ESHAPE: return "inconsistent sizes";
    case IMC_ENOMEM: return "out of device memory";
    case IMC_EDEVICE: return "HIP error";
    case IMC_ECORRUPT: return "components of a sharing disagree";
    case IMC_EUNSUPPORTED: return "unsupported parameter";
    default: return "unknown status";
  }
}

size_t imc_db_bytes(size_t capacity) { return blocks_for(capacity) * imc::kBlockBytes; }
size_t imc_query_op_bytes(size_t q) { return q * imc::kQopRowBytes; }
size_t imc_query_raw_bytes(size_t q) { return q * 2 * 2 * imc::kCodeBits * sizeof(uint16_t); }
size_t imc_galois_db_bytes(size_t capacity) { return blocks_for(capacity) * imc::Geo<imc::kKGalois>::kBlockBytes; }
size_t imc_galois_query_op_bytes(size_t q) { return q * imc::Geo<imc::kKGalois>::kQopRowBytes; }
size_t imc_galois_query_raw_bytes(size_t q) { return q * 2 * imc::kCodeBits * sizeof(uint16_t); }
size_t imc_or_tree_ws_bytes(size_t q, size_t r, size_t nw) { return imc::or_tree_ws_bytes(q, r, nw); }
size_t imc_db32_bytes(size_t capacity) { return imc::db32_bytes(capacity); }
size_t imc_query32_op_bytes(size_t q) { return imc::query32_op_bytes(q); }

imc_status imc_create(const imc_params* p, int device, imc_ctx** out) {
  if (!p || !out) return IMC_EINVAL;
  *out = nullptr;
  if (p->code_bits != IMC_CODE_BITS || p->thr_a != 16384u) return IMC_EUNSUPPORTED;
  if (!tiles_ok(p->flags)) return IMC_EUNSUPPORTED;
  if (p->max_rows == 0) return IMC_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return IMC_EDEVICE;
  if (device < 0 || device >= ndev) return IMC_EINVAL;
  DeviceGuard g(device);
  if (!g.ok) return IMC_EDEVICE;
  imc_ctx* c = new (std::nothrow) imc_ctx();
  if (!c) return IMC_ENOMEM;
  c->device = device;
  c->dealer = load_key(p->dealer_key);
  for (int k = 0; k < 3; ++k) c->party.k[k] = load_key(p->party_key[k]);
  c->max_rows = p->max_rows;
  c->dot_variant = int(p->flags & 0x1Fu);
  c->rot_op_bytes = blocks_for(p->max_rows) * imc::kBlockBytes;
  if (hipMalloc(reinterpret_cast<void**>(&c->rot_op), c->rot_op_bytes) != hipSuccess) {
    delete c;
    return IMC_ENOMEM;
  }
  if (hipMalloc(reinterpret_cast<void**>(&c->bad), sizeof(unsigned long long)) != hipSuccess) {
    (void)hipFree(c->rot_op);
    delete c;
    return IMC_ENOMEM;
  }
  const imc_status rs = resolve_scratch(device);   // the device is current (guard above)
  if (rs != IMC_OK) {
    (void)hipFree(c->rot_op);
    (void)hipFree(c->bad);
    delete c;
    return rs;
  }
  *out = c;
  return IMC_OK;
}

void imc_destroy(imc_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(c->rot_op);
  (void)hipFree(c->bad);
  delete c;
}

namespace {

imc_status share_db_impl(imc_ctx* c, const uint64_t* codes, const uint64_t* masks, size_t n, uint64_t first,
                         void* const db[3], size_t capacity, imc_stream stream, bool galois) {
  if (!c || !db) return IMC_EINVAL;
  if (n && (!codes || !masks)) return IMC_EINVAL;
  int held = 0;
  for (int p = 0; p < 3; ++p) {
    if (db[p] && !aligned(db[p], 256)) return IMC_EINVAL;
    held += db[p] != nullptr;
  }
  if (!held) return IMC_EINVAL;
  if (!aligned(codes, 8) || !aligned(masks, 8)) return IMC_EINVAL;
  if (first > capacity || n > capacity - first) return IMC_ESHAPE;
  if (first + n > (1ull << 48)) return IMC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  uint8_t* d[3] = {static_cast<uint8_t*>(db[0]), static_cast<uint8_t*>(db[1]), static_cast<uint8_t*>(db[2])};
  if (galois) return dev_status(imc::launch_galois_share_db(c->dealer, codes, masks, n, first, d, hipStream_t(stream)));
  return dev_status(imc::launch_share_db(c->dealer, codes, masks, n, first, d, hipStream_t(stream)));
}

imc_status share_query_impl(imc_ctx* c, const uint64_t* codes, const uint64_t* masks, size_t q, uint64_t qid_base,
                            void* const qop[3], void* const qraw[3], imc_stream stream, bool galois) {
  if (!c || !qop) return IMC_EINVAL;
  if (q && (!codes || !masks)) return IMC_EINVAL;
  if (!aligned(codes, 8) || !aligned(masks, 8)) return IMC_EINVAL;
  for (int p = 0; p < 3; ++p) {
    if (!qop[p] || !aligned(qop[p], 16)) return IMC_EINVAL;
    if (qraw && (!qraw[p] || !aligned(qraw[p], 16))) return IMC_EINVAL;
  }
  if (qid_base + q > (1ull << 48)) return IMC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  int8_t* op[3] = {static_cast<int8_t*>(qop[0]), static_cast<int8_t*>(qop[1]), static_cast<int8_t*>(qop[2])};
  uint16_t* raw[3] = {nullptr, nullptr, nullptr};
  if (qraw)
    for (int p = 0; p < 3; ++p) raw[p] = static_cast<uint16_t*>(qraw[p]);
  if (galois)
    return dev_status(imc::launch_galois_share_query(c->dealer, codes, masks, q, qid_base, op, qraw ? raw : nullptr,
                                                     hipStream_t(stream)));
  return dev_status(imc::launch_share_query(c->dealer, codes, masks, q, qid_base, op, qraw ? raw : nullptr,
                                            hipStream_t(stream)));
}

imc_status dot_shares_impl(imc_ctx* c, int party, const void* qop, const uint32_t* qidx, size_t q, const imc_ids* ids,
                           const void* db, size_t capacity, size_t n, uint16_t* code_dot, uint16_t* mask_dot,
                           size_t ld, imc_stream stream, bool galois) {
  if (!c || party < 0 || party > 2) return IMC_EINVAL;
  if (qidx && !aligned(qidx, 4)) return IMC_EINVAL;
  imc_status st = check_ids(ids);
  if (st != IMC_OK) return st;
  const size_t rows = q * size_t(ids->r);
  if (rows == 0 || n == 0) return IMC_OK;
  if (!qop || !db || !code_dot) return IMC_EINVAL;   // mask_dot NULL: code dot only
  if (!aligned(qop, 16) || !aligned(db, 256) || !aligned(code_dot, 2) || !aligned(mask_dot, 2)) return IMC_EINVAL;
  if (rows > c->max_rows) return IMC_ESHAPE;
  if (ld < n) return IMC_ESHAPE;
  if (ids->first_entry_id > capacity || n > capacity - ids->first_entry_id) return IMC_ESHAPE;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  const int v = c->dot_variant;
  const int tiles = v & 0xF;
  const bool rot_tiles = tiles == IMC_DOT_TILES_AUTO || tiles == IMC_DOT_TILES_ROTATION ||
                         tiles == IMC_DOT_TILES_ROTATION_LDSCOPY || tiles == IMC_DOT_TILES_ROTATION_DIRECT;
  const int kind = tiles == IMC_DOT_TILES_ROTATION_LDSCOPY ? 2 : tiles == IMC_DOT_TILES_ROTATION_DIRECT ? 3 : 0;
  if (rot_tiles && imc::rot_dot_applies(uint32_t(ids->r), kind)) {
    // rotations read straight from the unrotated operand staged in LDS
    return dev_status(imc::launch_rot_dot(static_cast<const int8_t*>(qop), qidx, uint32_t(q), uint32_t(ids->r), ids->rot,
                                          static_cast<const int8_t*>(db), ids->first_entry_id, n, code_dot, mask_dot,
                                          ld, hipStream_t(stream), kind, galois));
  }
  const uint32_t rows_pad = uint32_t(blocks_for(rows) * 32);
  hipError_t e = imc::launch_expand(static_cast<const int8_t*>(qop), qidx, uint32_t(q), uint32_t(ids->r), ids->rot,
                                    c->rot_op, rows_pad, hipStream_t(stream), galois);
  if (e != hipSuccess) return IMC_EDEVICE;
  e = imc::launch_dot(c->rot_op, uint32_t(rows), rows_pad / 32, static_cast<const int8_t*>(db), ids->first_entry_id,
                      n, code_dot, mask_dot, ld, hipStream_t(stream), v, galois);
  return dev_status(e);
}

// `a` receives the expanded rows (room for max_rows rows); a null `a` means the
// static array of the current device (imc_dot_shares_rows_noalloc).
imc_status dot_shares_rows_impl(imc_ctx* c, int party, const void* qop, size_t q, const imc_row* rows, size_t nrows,
                                const void* db, size_t capacity, uint64_t first_entry_id, size_t n,
                                uint16_t* code_dot, uint16_t* mask_dot, size_t ld, imc_stream stream, bool galois,
                                int8_t* a, size_t max_rows) {
  if (!c || party < 0 || party > 2) return IMC_EINVAL;
  if (nrows == 0 || n == 0) return IMC_OK;
  if (!qop || !rows || !db || !code_dot || q == 0) return IMC_EINVAL;   // mask_dot NULL: code dot only
  if (!aligned(qop, 16) || !aligned(rows, 8) || !aligned(db, 256) || !aligned(code_dot, 2) || !aligned(mask_dot, 2))
    return IMC_EINVAL;
  if (first_entry_id % 64) return IMC_EINVAL;
  if (nrows > max_rows) return IMC_ESHAPE;
  if (ld < n) return IMC_ESHAPE;
  if (first_entry_id > capacity || n > capacity - first_entry_id) return IMC_ESHAPE;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  if (!a) {
    a = g_scratch[c->device].load(std::memory_order_acquire);   // resolved by imc_create
    if (!a) return IMC_EDEVICE;
  }
  // every row the dot kernel reads (padding rows as zeros) is written here first
  const uint32_t rows_pad = uint32_t(blocks_for(nrows) * 32);
  hipError_t e = imc::launch_expand_rows(static_cast<const int8_t*>(qop), uint32_t(q), rows, uint32_t(nrows), a,
                                         rows_pad, hipStream_t(stream), galois);
  if (e != hipSuccess) return IMC_EDEVICE;
  int v = c->dot_variant;
  if ((v & 0xF) == IMC_DOT_TILES_AUTO || (v & 0xF) >= IMC_DOT_TILES_ROTATION)
    v = (v & ~0xF) | IMC_DOT_TILES_EXPANDED_256x128;
  e = imc::launch_dot(a, uint32_t(nrows), rows_pad / 32, static_cast<const int8_t*>(db), first_entry_id, n,
                      code_dot, mask_dot, ld, hipStream_t(stream), v, galois);
  return dev_status(e);
}

imc_status append_impl(imc_ctx* c, const void* const qraw[3], size_t qi, void* const db[3], size_t capacity,
                       uint64_t entry_id, imc_stream stream, bool galois) {
  if (!c || !qraw || !db) return IMC_EINVAL;
  int held = 0;
  for (int p = 0; p < 3; ++p) {
    if (!db[p]) continue;   // region not held on this device
    if (!qraw[p] || !aligned(db[p], 256) || !aligned(qraw[p], 2)) return IMC_EINVAL;
    ++held;
  }
  if (!held) return IMC_EINVAL;
  if (entry_id >= capacity) return IMC_ESHAPE;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  const uint16_t* raw[3] = {static_cast<const uint16_t*>(qraw[0]), static_cast<const uint16_t*>(qraw[1]),
                            static_cast<const uint16_t*>(qraw[2])};
  uint8_t* d[3] = {static_cast<uint8_t*>(db[0]), static_cast<uint8_t*>(db[1]), static_cast<uint8_t*>(db[2])};
  if (galois) return dev_status(imc::launch_galois_append(raw, qi, d, entry_id, hipStream_t(stream)));
  return dev_status(imc::launch_append(raw, qi, d, entry_id, hipStream_t(stream)));
}

}  // namespace

imc_status imc_share_db(imc_ctx* c, const uint64_t* codes, const uint64_t* masks, size_t n, uint64_t first,
                        void* const db[3], size_t capacity, imc_stream stream) {
  return share_db_impl(c, codes, masks, n, first, db, capacity, stream, false);
}
imc_status imc_galois_share_db(imc_ctx* c, const uint64_t* codes, const uint64_t* masks, size_t n, uint64_t first,
                               void* const db[3], size_t capacity, imc_stream stream) {
  return share_db_impl(c, codes, masks, n, first, db, capacity, stream, true);
}
imc_status imc_share_query(imc_ctx* c, const uint64_t* codes, const uint64_t* masks, size_t q, uint64_t qid_base,
                           void* const qop[3], void* const qraw[3], imc_stream stream) {
  return share_query_impl(c, codes, masks, q, qid_base, qop, qraw, stream, false);
}
imc_status imc_galois_share_query(imc_ctx* c, const uint64_t* codes, const uint64_t* masks, size_t q,
                                  uint64_t qid_base, void* const qop[3], void* const qraw[3], imc_stream stream) {
  return share_query_impl(c, codes, masks, q, qid_base, qop, qraw, stream, true);
}
imc_status imc_dot_shares(imc_ctx* c, int party, const void* qop, size_t q, const imc_ids* ids, const void* db,
                          size_t capacity, size_t n, uint16_t* code_dot, uint16_t* mask_dot, size_t ld,
                          imc_stream stream) {
  return dot_shares_impl(c, party, qop, nullptr, q, ids, db, capacity, n, code_dot, mask_dot, ld, stream, false);
}
imc_status imc_galois_dot_shares(imc_ctx* c, int party, const void* qop, size_t q, const imc_ids* ids, const void* db,
                                 size_t capacity, size_t n, uint16_t* code_dot, uint16_t* mask_dot, size_t ld,
                                 imc_stream stream) {
  return dot_shares_impl(c, party, qop, nullptr, q, ids, db, capacity, n, code_dot, mask_dot, ld, stream, true);
}
namespace {
imc_status dot_groups_impl(imc_ctx* c, int party, const imc_dot_group* groups, size_t n_groups, const void* db,
                           size_t capacity, uint64_t first_entry_id, size_t n, size_t ld, imc_stream stream,
                           bool galois) {
  if (!c || party < 0 || party > 2) return IMC_EINVAL;
  if (n_groups > IMC_MAX_DOT_GROUPS || (n_groups && !groups)) return IMC_EINVAL;
  if (first_entry_id % 64) return IMC_EINVAL;
  imc::DotGroup g[IMC_MAX_DOT_GROUPS];
  uint32_t used = 0;
  int masks = -1;   // 0: no group has a mask output, 1: every group has one
  for (size_t i = 0; i < n_groups; ++i) {
    const imc_dot_group& x = groups[i];
    if (x.q == 0) continue;
    if (x.r < 13 || x.r > IMC_MAX_ROT) return IMC_EINVAL;
    for (int j = 0; j < x.r; ++j)
      if (x.rot[j] < -15 || x.rot[j] > 15) return IMC_EINVAL;
    if (!x.qop || !x.code_dot || !aligned(x.qop, 16) || !aligned(x.code_dot, 2) || !aligned(x.mask_dot, 2))
      return IMC_EINVAL;
    const int m = x.mask_dot ? 1 : 0;
    if (masks >= 0 && m != masks) return IMC_EINVAL;
    masks = m;
    if (x.q >= (1ull << 31) / uint64_t(x.r)) return IMC_ESHAPE;
    g[used++] = imc::DotGroup{static_cast<const int8_t*>(x.qop), uint32_t(x.q), uint32_t(x.r), x.rot, x.code_dot,
                              x.mask_dot};
  }
  if (used == 0 || n == 0) return IMC_OK;
  if (!db || !aligned(db, 256)) return IMC_EINVAL;
  if (ld < n) return IMC_ESHAPE;
  if (first_entry_id > capacity || n > capacity - first_entry_id) return IMC_ESHAPE;
  DeviceGuard dg(c->device);
  if (!dg.ok) return IMC_EDEVICE;
  const bool persistent = (c->dot_variant & IMC_DOT_PERSISTENT) != 0;
  return dev_status(imc::launch_rot_dot_groups(g, used, static_cast<const int8_t*>(db), first_entry_id, n, ld,
                                               persistent, hipStream_t(stream), galois));
}
}  // namespace

imc_status imc_dot_shares_groups(imc_ctx* c, int party, const imc_dot_group* groups, size_t n_groups, const void* db,
                                 size_t capacity, uint64_t first_entry_id, size_t n, size_t ld, imc_stream stream) {
  return dot_groups_impl(c, party, groups, n_groups, db, capacity, first_entry_id, n, ld, stream, false);
}
imc_status imc_galois_dot_shares_groups(imc_ctx* c, int party, const imc_dot_group* groups, size_t n_groups,
                                        const void* db, size_t capacity, uint64_t first_entry_id, size_t n, size_t ld,
                                        imc_stream stream) {
  return dot_groups_impl(c, party, groups, n_groups, db, capacity, first_entry_id, n, ld, stream, true);
}

imc_status imc_dot_shares_gather(imc_ctx* c, int party, const void* qop, const uint32_t* qidx, size_t q,
                                 const imc_ids* ids, const void* db, size_t capacity, size_t n, uint16_t* code_dot,
                                 uint16_t* mask_dot, size_t ld, imc_stream stream) {
  if (!qidx) return IMC_EINVAL;
  return dot_shares_impl(c, party, qop, qidx, q, ids, db, capacity, n, code_dot, mask_dot, ld, stream, false);
}
imc_status imc_galois_dot_shares_gather(imc_ctx* c, int party, const void* qop, const uint32_t* qidx, size_t q,
                                        const imc_ids* ids, const void* db, size_t capacity, size_t n,
                                        uint16_t* code_dot, uint16_t* mask_dot, size_t ld, imc_stream stream) {
  if (!qidx) return IMC_EINVAL;
  return dot_shares_impl(c, party, qop, qidx, q, ids, db, capacity, n, code_dot, mask_dot, ld, stream, true);
}
imc_status imc_dot_shares_rows(imc_ctx* c, int party, const void* qop, size_t q, const imc_row* rows, size_t nrows,
                               const void* db, size_t capacity, uint64_t first_entry_id, size_t n, uint16_t* code_dot,
                               uint16_t* mask_dot, size_t ld, imc_stream stream) {
  if (!c) return IMC_EINVAL;
  return dot_shares_rows_impl(c, party, qop, q, rows, nrows, db, capacity, first_entry_id, n, code_dot, mask_dot, ld,
                              stream, false, c->rot_op, c->max_rows);
}
imc_status imc_dot_shares_rows_noalloc(imc_ctx* c, int party, const void* qop, size_t q, const imc_row* rows,
                                       size_t nrows, const void* db, size_t capacity, uint64_t first_entry_id,
                                       size_t n, uint16_t* code_dot, uint16_t* mask_dot, size_t ld,
                                       imc_stream stream) {
  return dot_shares_rows_impl(c, party, qop, q, rows, nrows, db, capacity, first_entry_id, n, code_dot, mask_dot, ld,
                              stream, false, nullptr, IMC_NOALLOC_MAX_ROWS);
}
imc_status imc_galois_dot_shares_rows(imc_ctx* c, int party, const void* qop, size_t q, const imc_row* rows,
                                      size_t nrows, const void* db, size_t capacity, uint64_t first_entry_id,
                                      size_t n, uint16_t* code_dot, uint16_t* mask_dot, size_t ld,
                                      imc_stream stream) {
  if (!c) return IMC_EINVAL;
  return dot_shares_rows_impl(c, party, qop, q, rows, nrows, db, capacity, first_entry_id, n, code_dot, mask_dot, ld,
                              stream, true, c->rot_op, c->max_rows);
}
imc_status imc_append_db(imc_ctx* c, const void* const qraw[3], size_t qi, void* const db[3], size_t capacity,
                         uint64_t entry_id, imc_stream stream) {
  return append_impl(c, qraw, qi, db, capacity, entry_id, stream, false);
}
imc_status imc_galois_append_db(imc_ctx* c, const void* const qraw[3], size_t qi, void* const db[3], size_t capacity,
                                uint64_t entry_id, imc_stream stream) {
  return append_impl(c, qraw, qi, db, capacity, entry_id, stream, true);
}

imc_status imc_mask_in_batch(imc_ctx* c, uint64_t* const match[3], size_t q, size_t r, size_t mw_ld, size_t word,
                             size_t group, imc_stream stream) {
  if (!c || !match) return IMC_EINVAL;
  for (int p = 0; p < 3; ++p)
    if (!match[p] || !aligned(match[p], 8)) return IMC_EINVAL;
  if (q > 64 || r < 1 || r > IMC_MAX_ROT || group < 1) return IMC_EINVAL;
  if (word >= mw_ld) return IMC_ESHAPE;
  if (q == 0) return IMC_OK;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  return dev_status(imc::launch_mask_in_batch(match, q, uint32_t(r), mw_ld, word, group, hipStream_t(stream)));
}

imc_status imc_or_pairs(imc_ctx* c, const uint8_t* const in[3], size_t count, uint64_t id, uint8_t* const out[3],
                        imc_stream stream) {
  if (!c || !in || !out) return IMC_EINVAL;
  for (int p = 0; p < 3; ++p)
    if (!in[p] || !out[p]) return IMC_EINVAL;
  if (count == 0) return IMC_OK;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  return dev_status(imc::launch_or_pairs(c->party, in, count, id, out, hipStream_t(stream)));
}

imc_status imc_or_bits(imc_ctx* c, const uint8_t* const a[3], const uint8_t* const b[3], size_t count, uint64_t id,
                       uint8_t* const out[3], imc_stream stream) {
  if (!c || !a || !b || !out) return IMC_EINVAL;
  for (int p = 0; p < 3; ++p)
    if (!a[p] || !b[p] || !out[p]) return IMC_EINVAL;
  if (count == 0) return IMC_OK;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  return dev_status(imc::launch_or_bits(c->party, a, b, count, id, out, hipStream_t(stream)));
}

imc_status imc_set_dot_tiles(imc_ctx* c, uint32_t flags) {
  if (!c) return IMC_EINVAL;
  if (!tiles_ok(flags)) return IMC_EUNSUPPORTED;
  c->dot_variant = int(flags);
  return IMC_OK;
}

imc_status imc_reshare(imc_ctx* c, const uint16_t* const add_code[3], const uint16_t* const add_mask[3], size_t rows,
                       size_t n, size_t ld, const imc_ids* ids, uint16_t* const msg[3], uint16_t* const rep_code[3],
                       uint16_t* const rep_mask[3], imc_stream stream) {
  if (!c || !add_code || !msg) return IMC_EINVAL;
  if (add_mask && rep_code && !rep_mask) return IMC_EINVAL;   // add_mask NULL: code shares only
  imc_status st = check_ids(ids);
  if (st != IMC_OK) return st;
  if (rows % size_t(ids->r)) return IMC_ESHAPE;
  if (ld < n) return IMC_ESHAPE;
  if (rows == 0 || n == 0) return IMC_OK;
  // 16-byte vector accesses are taken when ld % 8 == 0: every plane must then be 16-byte aligned
  const size_t va = ld % 8 == 0 ? 16 : 2;
  for (int p = 0; p < 3; ++p) {
    if (!add_code[p] || !msg[p]) return IMC_EINVAL;
    if (add_mask && !add_mask[p]) return IMC_EINVAL;
    if (!aligned(add_code[p], va) || !aligned(msg[p], va)) return IMC_EINVAL;
    if (add_mask && !aligned(add_mask[p], va)) return IMC_EINVAL;
    if (!rep_code) continue;                      // the messages alone
    if (!rep_code[p] || !aligned(rep_code[p], va)) return IMC_EINVAL;
    if (add_mask && (!rep_mask[p] || !aligned(rep_mask[p], va))) return IMC_EINVAL;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  return dev_status(
      imc::launch_reshare(c->party, add_code, add_mask, rows, n, ld, *ids, msg, rep_code, rep_mask, hipStream_t(stream)));
}

size_t imc_compare_msg_bytes(int variant, size_t rows, size_t n) {
  const size_t groups = (rows * ((n + 63) / 64) + 63) / 64;   // workgroups of 64 match words
  return imc::compare_msg_planes(variant) * groups * 64 * sizeof(uint64_t);
}

imc_status imc_compare_threshold(imc_ctx* c, const uint16_t* const rep_code[3], const uint16_t* const rep_mask[3],
                                 size_t rows, size_t n, size_t ld, const imc_ids* ids, void* msg_ws,
                                 size_t msg_ws_bytes, uint64_t* const match[3], size_t mw_ld, imc_stream stream) {
  if (!c || !rep_code || !rep_mask || !match) return IMC_EINVAL;
  imc_status st = check_ids(ids);
  if (st != IMC_OK) return st;
  if (rows % size_t(ids->r)) return IMC_ESHAPE;
  if (ld < n || mw_ld < (n + 63) / 64) return IMC_ESHAPE;
  if (rows == 0 || n == 0) return IMC_OK;
  // 16-byte vector accesses are taken when ld % 8 == 0: every plane must then be 16-byte aligned
  const size_t va = ld % 8 == 0 ? 16 : 2;
  for (int p = 0; p < 3; ++p) {
    if (!rep_code[p] || !rep_mask[p] || !match[p]) return IMC_EINVAL;
    if (!aligned(rep_code[p], va) || !aligned(rep_mask[p], va) || !aligned(match[p], 8)) return IMC_EINVAL;
  }
  if (msg_ws) {
    if (!aligned(msg_ws, 8)) return IMC_EINVAL;
    if (msg_ws_bytes < imc_compare_msg_bytes(0, rows, n)) return IMC_ESHAPE;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  if (msg_ws) {
    const void* code[3] = {rep_code[0], rep_code[1], rep_code[2]};
    const void* mask[3] = {rep_mask[0], rep_mask[1], rep_mask[2]};
    return dev_status(imc::launch_compare_msg(0, c->party, code, false, mask, nullptr, rows, n, ld, *ids, match,
                                              mw_ld, static_cast<uint64_t*>(msg_ws), hipStream_t(stream)));
  }
  return dev_status(imc::launch_compare(c->party, rep_code, rep_mask, rows, n, ld, *ids, match, mw_ld,
                                        hipStream_t(stream)));
}

imc_status imc_compare_threshold_msgs(imc_ctx* c, const uint16_t* const msgs[3], size_t rows, size_t n, size_t ld,
                                      const imc_ids* ids, void* msg_ws, size_t msg_ws_bytes,
                                      uint64_t* const match[3], size_t mw_ld, imc_stream stream) {
  if (!c || !msgs || !match) return IMC_EINVAL;
  imc_status st = check_ids(ids);
  if (st != IMC_OK) return st;
  if (rows % size_t(ids->r)) return IMC_ESHAPE;
  if (ld < n || mw_ld < (n + 63) / 64) return IMC_ESHAPE;
  if (rows == 0 || n == 0) return IMC_OK;
  const size_t va = ld % 8 == 0 ? 16 : 2;
  for (int p = 0; p < 3; ++p) {
    if (!msgs[p] || !match[p]) return IMC_EINVAL;
    if (!aligned(msgs[p], va) || !aligned(match[p], 8)) return IMC_EINVAL;
  }
  if (msg_ws) {
    if (!aligned(msg_ws, 8)) return IMC_EINVAL;
    if (msg_ws_bytes < imc_compare_msg_bytes(0, rows, n)) return IMC_ESHAPE;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  if (msg_ws)
    return dev_status(imc::launch_compare_msgs(c->party, msgs, rows, n, ld, *ids, match, mw_ld,
                                               static_cast<uint64_t*>(msg_ws), hipStream_t(stream)));
  // the register simulation reads each party's own component only
  const uint16_t* mask[3] = {msgs[0] + rows * ld, msgs[1] + rows * ld, msgs[2] + rows * ld};
  return dev_status(imc::launch_compare(c->party, msgs, mask, rows, n, ld, *ids, match, mw_ld, hipStream_t(stream)));
}

static_assert(sizeof(imc_query_entry) == 48 && offsetof(imc_query_entry, match) == 16 &&
                  offsetof(imc_query_entry, match_plane) == 40,
              "query entry layout");

imc_status imc_reshare_queries(imc_ctx* c, const uint16_t* const add_code[3], const uint16_t* const add_mask[3],
                               size_t q, size_t n, size_t ld, const imc_ids* ids, const imc_query_entry* table,
                               uint16_t* const msg[3], uint16_t* const rep_code[3], uint16_t* const rep_mask[3],
                               imc_stream stream) {
  if (!c || !add_code || !msg || !rep_code) return IMC_EINVAL;
  if (add_mask && !rep_mask) return IMC_EINVAL;
  if (!table || !aligned(table, 8) || !ids) return IMC_EINVAL;
  imc_ids idt = *ids;
  idt.query_id_base = 0;   // ignored: every query's id comes from the table
  imc_status st = check_ids(&idt);
  if (st != IMC_OK) return st;
  if (ld < n || q >= (size_t(1) << 31)) return IMC_ESHAPE;
  const size_t rows = q * size_t(idt.r);
  if (rows == 0 || n == 0) return IMC_OK;
  const size_t va = ld % 8 == 0 ? 16 : 2;
  for (int p = 0; p < 3; ++p) {
    if (!add_code[p] || !msg[p] || !rep_code[p]) return IMC_EINVAL;
    if (add_mask && (!add_mask[p] || !rep_mask[p])) return IMC_EINVAL;
    if (!aligned(add_code[p], va) || !aligned(msg[p], va) || !aligned(rep_code[p], va)) return IMC_EINVAL;
    if (add_mask && (!aligned(add_mask[p], va) || !aligned(rep_mask[p], va))) return IMC_EINVAL;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  imc::QueryTab qt;
  qt.tab = table;
  return dev_status(imc::launch_reshare(c->party, add_code, add_mask, rows, n, ld, idt, msg, rep_code, rep_mask,
                                        hipStream_t(stream), qt));
}

imc_status imc_compare_threshold_queries(imc_ctx* c, const uint16_t* const rep_code[3],
                                         const uint16_t* const rep_mask[3], size_t q, size_t n, size_t ld,
                                         const imc_ids* ids, const imc_query_entry* table, void* msg_ws,
                                         size_t msg_ws_bytes, size_t mw_ld, imc_stream stream) {
  if (!c || !rep_code || !rep_mask) return IMC_EINVAL;
  if (!table || !aligned(table, 8) || !ids) return IMC_EINVAL;
  imc_ids idt = *ids;
  idt.query_id_base = 0;   // ignored: every query's id comes from the table
  imc_status st = check_ids(&idt);
  if (st != IMC_OK) return st;
  if (ld < n || mw_ld < (n + 63) / 64 || q >= (size_t(1) << 31)) return IMC_ESHAPE;
  const size_t r = size_t(idt.r), rows = q * r;
  if (rows == 0 || n == 0) return IMC_OK;
  const size_t va = ld % 8 == 0 ? 16 : 2;
  for (int p = 0; p < 3; ++p) {
    if (!rep_code[p] || !rep_mask[p]) return IMC_EINVAL;
    if (!aligned(rep_code[p], va) || !aligned(rep_mask[p], va)) return IMC_EINVAL;
  }
  if (msg_ws) {
    if (!aligned(msg_ws, 8)) return IMC_EINVAL;
    if (msg_ws_bytes < imc_compare_msg_bytes(0, r, n)) return IMC_ESHAPE;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  uint64_t* const no_match[3] = {nullptr, nullptr, nullptr};   // each query's come from the table
  imc::QueryTab qt;
  qt.tab = table;
  if (!msg_ws)
    return dev_status(imc::launch_compare(c->party, rep_code, rep_mask, rows, n, ld, idt, no_match, mw_ld,
                                          hipStream_t(stream), qt));
  // launches of as many whole queries as the buffer's workgroup blocks hold
  const size_t nw = (n + 63) / 64;
  const size_t blocks = msg_ws_bytes / (imc::compare_msg_planes(0) * 64 * sizeof(uint64_t));
  const size_t per = std::min(q, blocks * 64 / nw / r);   // >= 1: the buffer holds one query
  qt.plane_rows = rows;
  for (size_t q0 = 0; q0 < q; q0 += per) {
    const size_t k = std::min(per, q - q0);
    const void* code[3], *mask[3];
    for (int p = 0; p < 3; ++p) {
      code[p] = rep_code[p] + q0 * r * ld;
      mask[p] = rep_mask[p] + q0 * r * ld;
    }
    qt.tab = table + q0;
    const imc_status e = dev_status(imc::launch_compare_msg(0, c->party, code, false, mask, nullptr, k * r, n, ld,
                                                            idt, no_match, mw_ld, static_cast<uint64_t*>(msg_ws),
                                                            hipStream_t(stream), qt));
    if (e != IMC_OK) return e;
  }
  return IMC_OK;
}

imc_status imc_compare_variant(imc_ctx* c, int variant, const void* const rep_code[3], int code_bits,
                               const void* const rep_mask[3], const uint16_t* ml_pub, size_t rows, size_t n,
                               size_t ld, const imc_ids* ids, void* msg_ws, size_t msg_ws_bytes,
                               uint64_t* const match[3], size_t mw_ld, imc_stream stream) {
  if (!c || !rep_code || !match) return IMC_EINVAL;
  if (variant < IMC_CMP_PLAIN_MASK || variant > IMC_CMP_CONST32) return IMC_EINVAL;
  if (code_bits != 16 && !(code_bits == 32 && variant == IMC_CMP_CONST32)) return IMC_EINVAL;
  imc_status st = check_ids(ids);
  if (st != IMC_OK) return st;
  if (rows % size_t(ids->r)) return IMC_ESHAPE;
  if (ld < n || mw_ld < (n + 63) / 64) return IMC_ESHAPE;
  if (rows == 0 || n == 0) return IMC_OK;
  const size_t cw = code_bits / 8, mwid = variant == IMC_CMP_CONST32 ? 4 : 2;
  for (int p = 0; p < 3; ++p) {
    if (!rep_code[p] || !match[p]) return IMC_EINVAL;
    if (!aligned(rep_code[p], cw) || !aligned(match[p], 8)) return IMC_EINVAL;
    if (variant != IMC_CMP_PLAIN_MASK && (!rep_mask || !rep_mask[p] || !aligned(rep_mask[p], mwid)))
      return IMC_EINVAL;
  }
  if (variant == IMC_CMP_PLAIN_MASK && (!ml_pub || !aligned(ml_pub, 2))) return IMC_EINVAL;
  if (msg_ws) {
    if (!aligned(msg_ws, 8)) return IMC_EINVAL;
    if (msg_ws_bytes < imc_compare_msg_bytes(variant, rows, n)) return IMC_ESHAPE;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  if (msg_ws)
    return dev_status(imc::launch_compare_msg(variant, c->party, rep_code, code_bits == 32,
                                              variant == IMC_CMP_PLAIN_MASK ? nullptr : rep_mask, ml_pub, rows, n,
                                              ld, *ids, match, mw_ld, static_cast<uint64_t*>(msg_ws),
                                              hipStream_t(stream)));
  return dev_status(imc::launch_compare_variant(variant, c->party, rep_code, code_bits == 32,
                                                variant == IMC_CMP_PLAIN_MASK ? nullptr : rep_mask, ml_pub, rows, n,
                                                ld, *ids, match, mw_ld, hipStream_t(stream)));
}

imc_status imc_rotate_masks(imc_ctx* c, const uint64_t* masks, size_t q, const imc_ids* ids, uint64_t* out,
                            imc_stream stream) {
  if (!c) return IMC_EINVAL;
  imc_status st = check_ids(ids);
  if (st != IMC_OK) return st;
  if (q == 0) return IMC_OK;
  if (!masks || !out || !aligned(masks, 8) || !aligned(out, 8)) return IMC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  return dev_status(imc::launch_rotate_masks(masks, q, *ids, out, hipStream_t(stream)));
}

imc_status imc_plain_ml(imc_ctx* c, const uint64_t* row_masks, size_t rows, const uint64_t* db_masks, size_t n,
                        uint16_t* ml, size_t ld, imc_stream stream) {
  if (!c) return IMC_EINVAL;
  if (ld < n) return IMC_ESHAPE;
  if (rows == 0 || n == 0) return IMC_OK;
  if (!row_masks || !db_masks || !ml) return IMC_EINVAL;
  if (!aligned(row_masks, 8) || !aligned(db_masks, 8) || !aligned(ml, 2)) return IMC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  return dev_status(imc::launch_plain_ml(row_masks, rows, db_masks, n, ml, ld, hipStream_t(stream)));
}

imc_status imc_share32_db(imc_ctx* c, int vec, const uint64_t* codes, const uint64_t* masks, size_t n,
                          uint64_t first, void* const db[3], size_t capacity, imc_stream stream) {
  if (!c || !db || (vec != 0 && vec != 1)) return IMC_EINVAL;
  if (n && (!codes || !masks)) return IMC_EINVAL;
  int held = 0;
  for (int p = 0; p < 3; ++p) {
    if (db[p] && !aligned(db[p], 256)) return IMC_EINVAL;
    held += db[p] != nullptr;
  }
  if (!held) return IMC_EINVAL;
  if (!aligned(codes, 8) || !aligned(masks, 8)) return IMC_EINVAL;
  if (first > capacity || n > capacity - first) return IMC_ESHAPE;
  if (first + n > (1ull << 48)) return IMC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  uint8_t* d[3] = {static_cast<uint8_t*>(db[0]), static_cast<uint8_t*>(db[1]), static_cast<uint8_t*>(db[2])};
  return dev_status(imc::launch_share32_db(c->dealer, vec, codes, masks, n, first, d, hipStream_t(stream)));
}

imc_status imc_share32_query(imc_ctx* c, int vec, const uint64_t* codes, const uint64_t* masks, size_t q,
                             uint64_t qid_base, void* const qop[3], imc_stream stream) {
  if (!c || !qop || (vec != 0 && vec != 1)) return IMC_EINVAL;
  if (q && (!codes || !masks)) return IMC_EINVAL;
  if (!aligned(codes, 8) || !aligned(masks, 8)) return IMC_EINVAL;
  for (int p = 0; p < 3; ++p)
    if (!qop[p] || !aligned(qop[p], 16)) return IMC_EINVAL;
  if (qid_base + q > (1ull << 48)) return IMC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  int8_t* op[3] = {static_cast<int8_t*>(qop[0]), static_cast<int8_t*>(qop[1]), static_cast<int8_t*>(qop[2])};
  return dev_status(imc::launch_share32_query(c->dealer, vec, codes, masks, q, qid_base, op, hipStream_t(stream)));
}

imc_status imc_dot32_shares(imc_ctx* c, int party, const void* qop, size_t q, const imc_ids* ids, const void* db,
                            size_t capacity, size_t n, uint32_t* dot, size_t ld, imc_stream stream) {
  if (!c || party < 0 || party > 2) return IMC_EINVAL;
  imc_status st = check_ids(ids);
  if (st != IMC_OK) return st;
  const size_t rows = q * size_t(ids->r);
  if (rows == 0 || n == 0) return IMC_OK;
  if (!qop || !db || !dot) return IMC_EINVAL;
  if (!aligned(qop, 16) || !aligned(db, 256) || !aligned(dot, 4)) return IMC_EINVAL;
  if (rows > 0xFFFFFFFFull) return IMC_ESHAPE;
  if (ld < n) return IMC_ESHAPE;
  if (ids->first_entry_id > capacity || n > capacity - ids->first_entry_id) return IMC_ESHAPE;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  return dev_status(imc::launch_dot32(static_cast<const int8_t*>(qop), uint32_t(q), uint32_t(ids->r), ids->rot,
                                      static_cast<const int8_t*>(db), ids->first_entry_id, n, dot, ld,
                                      hipStream_t(stream)));
}

imc_status imc_reshare32(imc_ctx* c, int vec, const uint32_t* const add[3], size_t rows, size_t n, size_t ld,
                         const imc_ids* ids, uint32_t* const msg[3], uint32_t* const rep[3], imc_stream stream) {
  if (!c || !add || !msg || !rep || (vec != 0 && vec != 1)) return IMC_EINVAL;
  imc_status st = check_ids(ids);
  if (st != IMC_OK) return st;
  if (rows % size_t(ids->r)) return IMC_ESHAPE;
  if (ld < n) return IMC_ESHAPE;
  if (rows == 0 || n == 0) return IMC_OK;
  for (int p = 0; p < 3; ++p) {
    if (!add[p] || !msg[p] || !rep[p]) return IMC_EINVAL;
    if (!aligned(add[p], 4) || !aligned(msg[p], 4) || !aligned(rep[p], 4)) return IMC_EINVAL;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  return dev_status(imc::launch_reshare32(c->party, vec, add, rows, n, ld, *ids, msg, rep, hipStream_t(stream)));
}

imc_status imc_or_tree(imc_ctx* c, const uint64_t* const match[3], size_t q, size_t nw, size_t mw_ld,
                       const imc_ids* ids, void* ws, size_t ws_bytes, uint8_t* const dup[3], imc_stream stream) {
  if (!c || !match || !dup) return IMC_EINVAL;
  imc_status st = check_ids(ids);
  if (st != IMC_OK) return st;
  if (q == 0) return IMC_OK;
  if (nw == 0 || mw_ld < nw) return IMC_ESHAPE;
  if (ws_bytes < imc::or_tree_ws_bytes(q, size_t(ids->r), nw)) return IMC_ESHAPE;
  const size_t len0 = size_t(ids->r) * nw;
  if (len0 > 1 && (!ws || !aligned(ws, 8))) return IMC_EINVAL;
  for (int p = 0; p < 3; ++p)
    if (!match[p] || !dup[p] || !aligned(match[p], 8)) return IMC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  return dev_status(imc::launch_or_tree(c->party, match, q, nw, mw_ld, *ids, ws, dup, hipStream_t(stream)));
}

imc_status imc_open(imc_ctx* c, int kind, const void* const rep[3], size_t count, void* out, int check,
                    imc_stream stream) {
  if (!c || !rep || kind < IMC_OPEN_U8_XOR || kind > IMC_OPEN_U32_ADD) return IMC_EINVAL;
  if (count == 0) return IMC_OK;
  static const size_t width[4] = {1, 8, 2, 4};
  if (!out || !aligned(out, width[kind])) return IMC_EINVAL;
  for (int p = 0; p < 3; ++p)
    if (!rep[p] || !aligned(rep[p], width[kind])) return IMC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return IMC_EDEVICE;
  hipStream_t s = hipStream_t(stream);
  if (imc::launch_open(kind, rep, count, out, check, c->bad, s) != hipSuccess) return IMC_EDEVICE;
  if (!check) return IMC_OK;
  unsigned long long bad = 0;
  if (hipMemcpyAsync(&bad, c->bad, sizeof bad, hipMemcpyDeviceToHost, s) != hipSuccess) return IMC_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return IMC_EDEVICE;
  return bad ? IMC_ECORRUPT : IMC_OK;
}


}  // extern "C"
