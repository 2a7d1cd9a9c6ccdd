// launch.h -- host-side launchers of the library's kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/irismpc.h"

#define IMC_MAX_ROT_DEV IMC_MAX_ROT

namespace imc {

struct Key;
struct Keys3;
typedef imc_ids imc_ids_dev;

// True when `threads` threads in workgroups of `block` fit the grid's x limit.
inline bool fits_grid(uint64_t threads, uint64_t block) { return (threads + block - 1) / block <= 0x7FFFFFFFull; }

hipError_t launch_share_db(const Key& dk, const uint64_t* codes, const uint64_t* masks, uint64_t n, uint64_t first,
                           uint8_t* const db[3], hipStream_t s);
hipError_t launch_share_query(const Key& dk, const uint64_t* codes, const uint64_t* masks, uint64_t q,
                              uint64_t qid_base, int8_t* const op[3], uint16_t* const raw[3], hipStream_t s);
hipError_t launch_append(const uint16_t* const raw[3], uint64_t qi, uint8_t* const db[3], uint64_t e, hipStream_t s);
hipError_t launch_galois_share_db(const Key& dk, const uint64_t* codes, const uint64_t* masks, uint64_t n,
                                  uint64_t first, uint8_t* const db[3], hipStream_t s);
hipError_t launch_galois_share_query(const Key& dk, const uint64_t* codes, const uint64_t* masks, uint64_t q,
                                     uint64_t qid_base, int8_t* const op[3], uint16_t* const raw[3], hipStream_t s);
hipError_t launch_galois_append(const uint16_t* const raw[3], uint64_t qi, uint8_t* const db[3], uint64_t e,
                                hipStream_t s);

hipError_t launch_expand(const int8_t* qop, const uint32_t* qidx, uint32_t q, uint32_t r, const int8_t* rot, int8_t* a,
                         uint32_t rows_pad, hipStream_t s, bool galois);
bool rot_dot_applies(uint32_t r, int kind);
hipError_t launch_rot_dot(const int8_t* qop, const uint32_t* qidx, uint32_t q, uint32_t r, const int8_t* rot,
                          const int8_t* b,
                          uint64_t first_entry, uint64_t n, uint16_t* code, uint16_t* mask, uint64_t ld,
                          hipStream_t s, int kind, bool galois);
// One query group of a fused rotation-aware launch (imc_dot_shares_groups).
struct DotGroup {
  const int8_t* qop;
  uint32_t q, r;
  const int8_t* rot;
  uint16_t* code;
  uint16_t* mask;
};
hipError_t launch_rot_dot_groups(const DotGroup* groups, uint32_t ngroups, const int8_t* b, uint64_t first_entry,
                                 uint64_t n, uint64_t ld, bool persistent, hipStream_t s, bool galois);
hipError_t launch_expand_rows(const int8_t* qop, uint32_t q, const imc_row* rows, uint32_t nrows, int8_t* a,
                              uint32_t rows_pad, hipStream_t s, bool galois);
hipError_t launch_dot(const int8_t* a, uint32_t rows, uint32_t a_blocks, const int8_t* b, uint64_t first_entry,
                      uint64_t n, uint16_t* code, uint16_t* mask, uint64_t ld, hipStream_t s, int variant,
                      bool galois);

// A call's optional table of per-query ids, column counts and match buffers
// (imc_query_entry, one per query of the launch), and the row count of the
// planes' allocation when a launch covers only some of its rows (plane 1
// of an input at plane_rows * ld; 0: the launch's own rows).
struct QueryTab {
  const imc_query_entry* tab = nullptr;
  uint64_t plane_rows = 0;
};
hipError_t launch_reshare(const Keys3& keys, const uint16_t* const add_code[3], const uint16_t* const add_mask[3],
                          uint64_t rows, uint64_t n, uint64_t ld, const imc_ids_dev& ids, uint16_t* const msg[3],
                          uint16_t* const rep_code[3], uint16_t* const rep_mask[3], hipStream_t s,
                          const QueryTab& qt = QueryTab{});
hipError_t launch_compare(const Keys3& keys, const uint16_t* const rep_code[3], const uint16_t* const rep_mask[3],
                          uint64_t rows, uint64_t n, uint64_t ld, const imc_ids_dev& ids, uint64_t* const match[3],
                          uint64_t mw_ld, hipStream_t s, const QueryTab& qt = QueryTab{});
// MPCLift with the parties' replicated components read from the resharing's
// messages: party p's own = msgs[p], its second = msgs[p-1] ([code, mask][rows][ld]).
hipError_t launch_compare_msgs(const Keys3& keys, const uint16_t* const msgs[3], uint64_t rows, uint64_t n,
                               uint64_t ld, const imc_ids_dev& ids, uint64_t* const match[3], uint64_t mw_ld,
                               uint64_t* msg, hipStream_t s);
hipError_t launch_compare_variant(int variant, const Keys3& keys, const void* const rep_code[3], bool code32,
                                  const void* const rep_mask[3], const uint16_t* ml_pub, uint64_t rows, uint64_t n,
                                  uint64_t ld, const imc_ids_dev& ids, uint64_t* const match[3], uint64_t mw_ld,
                                  hipStream_t s);
size_t compare_msg_planes(int variant);
hipError_t launch_compare_msg(int variant, const Keys3& keys, const void* const rep_code[3], bool code32,
                              const void* const rep_mask[3], const uint16_t* ml_pub, uint64_t rows, uint64_t n,
                              uint64_t ld, const imc_ids_dev& ids, uint64_t* const match[3], uint64_t mw_ld,
                              uint64_t* msg, hipStream_t s, const QueryTab& qt = QueryTab{});
hipError_t launch_rotate_masks(const uint64_t* masks, uint64_t q, const imc_ids_dev& ids, uint64_t* out,
                               hipStream_t s);
hipError_t launch_plain_ml(const uint64_t* row_masks, uint64_t rows, const uint64_t* db_masks, uint64_t n,
                           uint16_t* ml, uint64_t ld, hipStream_t s);
hipError_t launch_share32_db(const Key& dk, int vec, const uint64_t* codes, const uint64_t* masks, uint64_t n,
                             uint64_t first, uint8_t* const db[3], hipStream_t s);
hipError_t launch_share32_query(const Key& dk, int vec, const uint64_t* codes, const uint64_t* masks, uint64_t q,
                                uint64_t qid_base, int8_t* const op[3], hipStream_t s);
hipError_t launch_dot32(const int8_t* qop, uint32_t q, uint32_t r, const int8_t* rot, const int8_t* b,
                        uint64_t first_entry, uint64_t n, uint32_t* out, uint64_t ld, hipStream_t s);
hipError_t launch_reshare32(const Keys3& keys, int vec, const uint32_t* const add[3], uint64_t rows, uint64_t n,
                            uint64_t ld, const imc_ids_dev& ids, uint32_t* const msg[3], uint32_t* const rep[3],
                            hipStream_t s);
size_t db32_bytes(uint64_t capacity);
size_t query32_op_bytes(uint64_t q);
size_t or_tree_ws_bytes(uint64_t q, uint64_t r, uint64_t nw);
hipError_t launch_or_tree(const Keys3& keys, const uint64_t* const match[3], uint64_t q, uint64_t nw, uint64_t mw_ld,
                          const imc_ids_dev& ids, void* ws, uint8_t* const dup[3], hipStream_t s);
hipError_t launch_mask_in_batch(uint64_t* const match[3], uint64_t q, uint32_t r, uint64_t mw_ld, uint64_t word,
                                uint64_t group, hipStream_t s);
hipError_t launch_or_pairs(const Keys3& keys, const uint8_t* const in[3], uint64_t count, uint64_t id,
                           uint8_t* const out[3], hipStream_t s);
hipError_t launch_or_bits(const Keys3& keys, const uint8_t* const x[3], const uint8_t* const y[3], uint64_t count,
                          uint64_t id, uint8_t* const out[3], hipStream_t s);
hipError_t launch_open(int kind, const void* const rep[3], uint64_t count, void* out, int check,
                       unsigned long long* bad, hipStream_t s);

}  // namespace imc
