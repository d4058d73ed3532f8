// pp_fold.h -- the sweep of the symmetric schedules' fold over one band of
// partial slots, shared by the mixed and the FP64 fold kernels.
#pragma once

#include "pp_device.h"
#include "pp_internal.h"

namespace ppk {

// Adds one particle's slots of one component for the sub-rounds [r0, r1) of
// a band to its receiver-side (rs, rc) and source-side (ss, sc) compensated
// sums: sub-round by sub-round, the receiver side before the source side,
// with two-sum (the order that makes the sum independent of the order the
// items ran in).  slot0: the particle's receiver-side slot of this component
// in sub-round r0; round_stride: elements between sub-rounds; sl: elements
// between the receiver and source sides.  The particle is at block X of a
// bunch of nbk blocks; block pairs are split in 2^s_log2 parts, the
// particle's source part is `part`, and an item spans 2^m_log2 rounds (both
// powers of two, so no division is needed per sub-round).
//
// The loads of FOLD_U consecutive sub-rounds are issued before any of their
// additions.  A thread's loads do not depend on its sums, so this changes no
// result, but at small particle counts (a wavefront or two per SIMD) it
// replaces one exposed memory round trip per sub-round with one per FOLD_U.
// A load past r1 is redirected to sub-round r0 (inside the band) and its
// value is never added.
template <typename T>
__device__ __forceinline__ void fold_sweep(const T* __restrict__ slot0, int64_t round_stride, int64_t sl, int r0,
                                           int r1, int s_log2, int part, int nbk, int m_log2, int X, T& rs, T& rc,
                                           T& ss, T& sc) {
  constexpr int FOLD_U = 8;
  const int half = nbk / 2;
  const int smask = (1 << s_log2) - 1, mmask = (1 << m_log2) - 1;
  for (int v0 = r0; v0 < r1; v0 += FOLD_U) {
    T xr[FOLD_U], xs[FOLD_U];
    bool hr[FOLD_U], hs[FOLD_U];
#pragma unroll
    for (int u = 0; u < FOLD_U; ++u) {
      const int v = v0 + u;
      const int r = v >> s_log2;
      hr[u] = hs[u] = false;
      if (v < r1) {
        if (r == 0) {
          hr[u] = true;  // the diagonal items: receiver side only
        } else if (r <= half) {
          // receiver side: the item of block X whose group of rounds starts
          // at round r (one slot for the group); source side: item (X - r, X)
          // of round r.  With an even block count the round r = nbk / 2 holds
          // only the items with I < nbk / 2.
          hr[u] = ((r - 1) & mmask) == 0 && sym_group_rounds(nbk, 1 << m_log2, r, X) > 0;
          const int js = X - r < 0 ? X - r + nbk : X - r;
          hs[u] = !(2 * r == nbk && js >= half) && (v & smask) == part;
        }
      }
      const T* base = slot0 + (int64_t)((v < r1 ? v : r0) - r0) * round_stride;
      xr[u] = hr[u] ? base[0] : T(0);
      xs[u] = hs[u] ? base[sl] : T(0);
    }
#pragma unroll
    for (int u = 0; u < FOLD_U; ++u) {
      if (hr[u]) {
        if (v0 + u == 0) {
          rs = xr[u];
          rc = T(0);
        } else {
          two_sum(rs, rc, xr[u]);
        }
      }
      if (hs[u]) two_sum(ss, sc, xs[u]);
    }
  }
}

// log2 of a power of two
__device__ __forceinline__ int ilog2_pow2(int v) { return __builtin_ctz((unsigned)v); }

}  // namespace ppk
