// pp_sort.h -- spatial sort of the near/far split (pp_sort.hip) with a chosen
// Morton resolution (not part of the C ABI).
#pragma once

#include "pp_internal.h"

namespace ppk {

// Morton bits per axis for a bunch of n particles: about 8 cells per particle,
// ceil(log2(n) / 3) + 1, at most 10.  Host and device use this one function.
__host__ __device__ inline int morton_bits_for(int64_t n) {
  int need = 0;
  while (need < 10 && (int64_t(1) << (3 * need)) < n) ++need;
  return need + 1 > 10 ? 10 : need + 1;
}

// As launch_sort, with sort keys (bunch << key_shift) | code, where each
// bunch's code has 3 morton_bits_for(n) bits and key_shift (3..30) is the
// widest of them; key_bits = key_shift plus the bits of the largest bunch
// index, sorted in ceil(key_bits / 8) radix passes.
// With resort false the permutation of the previous full sort (same key_bits)
// is reused: only the bound, the gather into the sorted mirror, the rank and
// the group boxes are recomputed from the current positions.
hipError_t launch_sort_bits(const SortArgs& a, int key_shift, int key_bits, int32_t n_groups_total, bool resort,
                            hipStream_t s);

}  // namespace ppk
