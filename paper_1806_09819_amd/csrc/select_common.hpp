// Ranking keys and parent draws shared by the selection kernel and the
// surrogate's candidate plan (Algorithm 1: sort, truncation selection;
// tournament selection as the requested variant).
#pragma once

#include "internal.hpp"

namespace leea {

// Unique 64-bit key of a slot's fitness: the high word is an
// order-reversing map of the float (larger fitness -> smaller key, -0 ->
// +0, every NaN -> 0xFFFFFFFF), the low word the slot index.
__device__ __forceinline__ uint64_t rank_key(float f, uint32_t slot) {
  uint32_t hi;
  if (f != f) {
    hi = 0xFFFFFFFFu;
  } else {
    uint32_t b = __float_as_uint(f);
    if ((b << 1) == 0u) b = 0u;  // -0 -> +0
    hi = (b & 0x80000000u) ? b : (~b & 0x7FFFFFFFu);
  }
  return ((uint64_t)hi << 32) | slot;
}

// Rank of one parent: truncation = floor(w * n_trunc / 2^32) from word p;
// tournament = best of k ranks floor(w * pop / 2^32) from words p*k + c.
__device__ __forceinline__ uint32_t parent_rank(const Key& key, uint32_t gen, uint32_t slot,
                                                int p, int selection, int tk, uint32_t n_trunc,
                                                uint32_t pop) {
  if (selection == 0) {
    const uint4 w = draw(key, kSel, gen, slot, 0u);
    return (uint32_t)(((uint64_t)word_of(w, p) * n_trunc) >> 32);
  }
  uint32_t best = 0xFFFFFFFFu;
  int blk = -1;
  uint4 w = make_uint4(0u, 0u, 0u, 0u);
  for (int c = 0; c < tk; ++c) {
    const int idx = p * tk + c;
    if ((idx >> 2) != blk) {
      blk = idx >> 2;
      w = draw(key, kSel, gen, slot, (uint32_t)blk);
    }
    const uint32_t r = (uint32_t)(((uint64_t)word_of(w, idx & 3) * pop) >> 32);
    best = r < best ? r : best;
  }
  return best;
}

}  // namespace leea
