// pp_sym64.h -- the FP64 symmetric pair sum (pp_sym64.hip): arguments and
// launchers (not part of the C ABI).
#pragma once

#include "pp_internal.h"

namespace ppk {

// Same rounds, bands and slot indexing as the mixed symmetric schedule
// (SymArgs), with FP64 sources (unscaled SI positions, normalised charges)
// and FP64 partial slots.
struct SymArgs64 {
  const BunchDev* bunches;
  const SymItem* items;
  const double *x, *y, *z, *qt;
  double* slot;            // (((r - r0) * nbt + block) * 2 + side) * SLOT_PLANES + plane) * block_size + offset
  int32_t r0;              // first sub-round of the launch (SymItem::r)
  int32_t nbt;
  int32_t split;           // items per block pair (1, 2 or 4)
};

struct SymFoldArgs64 {
  const BunchDev* bunches;
  const int32_t* bid;
  int64_t n_total;
  const double* slot;
  double* acc;             // SYM_PLANES planes of length n_total
  int32_t r0, r1;          // sub-rounds
  int32_t nbt;
  int32_t block_size;
  int32_t split;
  int32_t rounds;          // the sym_rounds tuning value
};

// Wavefronts per item; a block is SYM64_WG * i_per_lane particles.  Four
// wavefronts, not the mixed kernel's eight: the 4-receiver FP64 sweep needs
// 164 VGPRs, so a CU holds 3 wavefronts per SIMD, which only 4-wavefront items
// can fill (8-wavefront items leave it at 2 and measured 5% slower at 1M).
constexpr int SYM64_WAVES = 4;
constexpr int SYM64_WG = SYM64_WAVES * 64;

// receivers per lane 1, 2 or 4
hipError_t launch_sym64(const SymArgs64& a, int32_t first, int32_t count, int i_per_lane, bool uniform_q,
                        bool with_phi, hipStream_t s);
hipError_t launch_sym64_fold(const SymFoldArgs64& a, bool with_phi, hipStream_t s);
int sym64_blocks_per_cu(int i_per_lane);

}  // namespace ppk
