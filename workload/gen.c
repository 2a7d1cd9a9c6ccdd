/*
 * gen.c -- seeded synthetic iris codes and masks.
 *
 * Input generation only: this file holds none of the protocol's arithmetic.
 * Every 64-bit word is SplitMix64 (Steele, Lea, Flood 2014) evaluated at a
 * counter, so any entry is regenerated from (seed, class, id) alone:
 *   word(seed, key) = mix(seed + (key + 1) * 0x9E3779B97F4A7C15)
 *   key = (class << 60) | (id << 13) | index          (index < 8192)
 * Code bits are the words themselves (Bernoulli 0.5).  Mask bit i is the
 * 16-bit lane (i & 3) of word (i >> 2) compared with 58982 (p = 0.89999).
 */
#include <stdint.h>
#include <string.h>

#define WL_L 12800
#define WL_W 200

static uint64_t wl_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t wl_word(uint64_t seed, uint64_t cls, uint64_t id, uint64_t index) {
  uint64_t key = (cls << 60) | ((id & 0x7FFFFFFFFFFull) << 13) | (index & 0x1FFFull);
  return wl_mix(seed + (key + 1) * 0x9E3779B97F4A7C15ull);
}

/* n entries with ids first..first+n-1: codes, masks [n][200] u64. */
void wl_codes(uint64_t seed, uint64_t cls_code, uint64_t cls_mask, uint64_t first, long n,
              uint64_t* codes, uint64_t* masks) {
#pragma omp parallel for schedule(static)
  for (long e = 0; e < n; ++e) {
    uint64_t id = first + (uint64_t)e;
    uint64_t* c = codes + (size_t)e * WL_W;
    uint64_t* m = masks + (size_t)e * WL_W;
    for (int w = 0; w < WL_W; ++w) c[w] = wl_word(seed, cls_code, id, (uint64_t)w);
    memset(m, 0, WL_W * sizeof(uint64_t));
    for (int q = 0; q < WL_L / 4; ++q) {
      uint64_t r = wl_word(seed, cls_mask, id, (uint64_t)q);
      for (int t = 0; t < 4; ++t) {
        int i = 4 * q + t;
        if (((r >> (16 * t)) & 0xFFFFu) < 58982u) m[i >> 6] |= 1ull << (i & 63);
      }
    }
  }
}
