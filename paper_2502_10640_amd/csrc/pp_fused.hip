// pp_fused.hip -- fused small-bunch step for gfx950: the whole field sum of a
// few receivers and their update in one workgroup.
//
// Sec. 2.1's direct sum (Eq. (B)) for bunches of a few thousand particles
// (the paper's own 4^3 .. 32^3 cubes) is set by latency, not arithmetic: the
// two-kernel step (pair sum over source chunks into partial slots, then a
// combine-and-kick kernel) waits on serial memory round trips in each kernel
// and on the kernel boundary between them.  Here a workgroup owns R receivers
// outright: it streams every source of the bunch through LDS in tiles of
// 1024, 256 / R lanes share each receiver (each takes every (256 / R)-th
// source of a tile), their partial sums are added in FP64 in a fixed order
// (a butterfly inside each wavefront, then the wavefronts in order), and the
// same workgroup applies the update (the field, the
// acceleration of Eqs. (D)/(F), or the kick of Eq. (H) with the next step's
// drift of Eq. (G) and source pack).  A step is one kernel; nothing but the
// kernel boundary orders one step's updates before the next step's sums.
// The kick-and-drift writes the next positions' sources into the other of two
// source buffers, so that workgroups still summing this step read unchanged
// sources.
//
// Summation (as the ordered kernel): each lane sums 64 of its terms in plain
// arithmetic of the path's precision and adds that to a (sum, compensation)
// pair by two-sum; the butterfly adds the lanes' pairs in FP64.  The order of
// every addition depends only on the bunch's size and the tiling, so a bunch
// gives the same bits alone or in a batch, and run to run.
#include "pp_device.h"
#include "pp_device64.h"
#include "pp_internal.h"
#include "pp_update.h"

#include <type_traits>

namespace ppk {
namespace {

constexpr int TS = 1024;         // sources per LDS tile
constexpr int PLAIN_TERMS = 64;  // terms per lane in one plain partial sum

// Sums of one lane for its receiver over tile entries s, s + S, ... < jn.
template <int S, bool UQ, bool PHI, bool DIAG>
__device__ __forceinline__ void tile_mixed(const float4* __restrict__ th, const float4* __restrict__ tl, int s, int jn,
                                           int jbase, int li, float xh, float yh, float zh, float xl, float yl,
                                           float zl, float eps2, float& tx, float& ty, float& tz, float& tp) {
#pragma unroll 4
  for (int m = s; m < jn; m += S) {
    const float4 h = th[m];
    const float4 l = tl[m];
    const float dx = (xh - h.x) + (xl - l.x);
    const float dy = (yh - h.y) + (yl - l.y);
    const float dz = (zh - h.z) + (zl - l.z);
    float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
    // self term j == i: rsq(+inf) = 0 removes it from E and phi
    if (DIAG && jbase + m == li) r2 = __builtin_inff();
    const float inv = __builtin_amdgcn_rsqf(r2);
    const float inv2 = inv * inv;
    const float sc = UQ ? inv2 * inv : (h.w * inv) * inv2;
    tx = fmaf(dx, sc, tx);
    ty = fmaf(dy, sc, ty);
    tz = fmaf(dz, sc, tz);
    if (PHI) tp += UQ ? inv : h.w * inv;
  }
}

template <int S, bool UQ, bool PHI, bool DIAG>
__device__ __forceinline__ void tile_fp64(const double4* __restrict__ tj, int s, int jn, int jbase, int li, double xi,
                                          double yi, double zi, double eps2, const SeriesConst& sc, double& tx,
                                          double& ty, double& tz, double& tp) {
#pragma unroll 4
  for (int m = s; m < jn; m += S) {
    const double4 p = tj[m];
    const double dx = xi - p.x;
    const double dy = yi - p.y;
    const double dz = zi - p.z;
    double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
    bool self = false;
    if (DIAG) {
      self = (jbase + m == li);
      if (self) r2 = 1.0;
    }
    double inv = 0.0;
    const double s3 = inv_r3_64<PHI>(r2, sc, inv);
    double f = UQ ? s3 : p.w * s3;
    double ph = UQ ? inv : p.w * inv;
    if (DIAG && self) { f = 0.0; ph = 0.0; }
    tx = fma(dx, f, tx);
    ty = fma(dy, f, ty);
    tz = fma(dz, f, tz);
    if (PHI) tp += ph;
  }
}

// One workgroup of FT threads per item: receivers [i0, i0 + R) of bunch b.
// Inside a wavefront the receiver index runs fastest (lane l serves receiver
// l mod R), so the 64 / R lanes of one source step read only 64 / R distinct
// sources from LDS, each a broadcast to R lanes; the S = FT / R source
// subsets of a receiver are the lane groups of the FT / 64 wavefronts (subset
// s = 64 / R x w + l / R takes the tile's sources s, s + S, ...).  Larger
// workgroups split the sources further and keep more wavefronts per SIMD
// without more source traffic.  Each thread loads TS / FT sources of a tile
// with independent loads, and the next
// tile's loads are in flight while the current tile is summed: at small bunch
// sizes a lane's share of a tile is a few dozen pairs, too little to wait out
// one load round trip per tile.
template <bool MIXED, int R, int FT, bool UQ, bool PHI, int MODE>
__global__ __launch_bounds__(FT) void fused_kernel(FusedArgs a) {
  static_assert(R >= 1 && 64 % R == 0, "a wavefront holds whole groups of the R receivers");
  constexpr int LPT = TS / FT;            // sources each thread loads per tile
  constexpr int SW = 64 / R;              // source subsets per wavefront
  constexpr int S = (FT / 64) * SW;       // source subsets per receiver
  constexpr int TILES_PER_SUM = PLAIN_TERMS * S / TS > 0 ? PLAIN_TERMS * S / TS : 1;
  __shared__ float4 s_hi[MIXED ? TS : 1];
  __shared__ float4 s_lo[MIXED ? TS : 1];
  __shared__ double4 s_j[MIXED ? 1 : TS];
  __shared__ double s_red[FT / 64][R][4];

  const FusedItem it = a.items[blockIdx.x];
  const BunchDev& B = a.bunches[it.b];
  const int64_t off = B.off;
  const int n = (int)B.n;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int r = l % R, s = w * SW + l / R;
  const int li = it.i0 + r;

  // the receiver in registers (an out-of-range slot reads particle 0; never stored)
  const int64_t gi = off + (li < n ? li : 0);
  float xh = 0.f, yh = 0.f, zh = 0.f, xl = 0.f, yl = 0.f, zl = 0.f;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if constexpr (MIXED) {
    xh = a.xh[gi]; yh = a.yh[gi]; zh = a.zh[gi];
    xl = a.xl[gi]; yl = a.yl[gi]; zl = a.zl[gi];
  } else {
    xi = a.x[gi]; yi = a.y[gi]; zi = a.z[gi];
  }
  // (S, C) per component in the path's precision, and the plain tile sums
  using T = typename std::conditional<MIXED, float, double>::type;
  T Sx = 0, Sy = 0, Sz = 0, Cx = 0, Cy = 0, Cz = 0, Sp = 0, Cp = 0;
  T tx = 0, ty = 0, tz = 0, tp = 0;
  const float eps2s = B.eps2s;
  const double eps2 = B.eps2;
  const SeriesConst sc = series_const();
  const int ilo = it.i0, ihi = it.i0 + R;

  // the next tile's sources, LPT per thread (entries tid + u FT of the tile)
  float4 rh[LPT], rl[LPT];
  double4 rj[LPT];
#pragma unroll
  for (int u = 0; u < LPT; ++u) {
    rh[u] = rl[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    rj[u] = make_double4(0.0, 0.0, 0.0, 0.0);
  }
  auto load_tile = [&](int jt) {
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int j = jt + tid + u * FT;
      if (j < n) {
        const int64_t gj = off + j;
        if constexpr (MIXED) {
          rh[u] = make_float4(a.xh[gj], a.yh[gj], a.zh[gj], UQ ? 1.f : a.qt[gj]);
          rl[u] = make_float4(a.xl[gj], a.yl[gj], a.zl[gj], 0.f);
        } else {
          rj[u] = make_double4(a.x[gj], a.y[gj], a.z[gj], UQ ? 1.0 : a.qt64[gj]);
        }
      }
    }
  };
  load_tile(0);
  int tiles = 0;
  for (int jt = 0; jt < n; jt += TS) {
    const int jn = min(TS, n - jt);
    __syncthreads();  // the previous tile is no longer read
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      if constexpr (MIXED) {
        s_hi[tid + u * FT] = rh[u];
        s_lo[tid + u * FT] = rl[u];
      } else {
        s_j[tid + u * FT] = rj[u];
      }
    }
    __syncthreads();
    load_tile(jt + TS);  // the next tile, while this one is summed
    const bool diag = jt < ihi && jt + jn > ilo;
    if constexpr (MIXED) {
      if (diag)
        tile_mixed<S, UQ, PHI, true>(s_hi, s_lo, s, jn, jt, li, xh, yh, zh, xl, yl, zl, eps2s, tx, ty, tz, tp);
      else
        tile_mixed<S, UQ, PHI, false>(s_hi, s_lo, s, jn, jt, li, xh, yh, zh, xl, yl, zl, eps2s, tx, ty, tz, tp);
    } else {
      if (diag)
        tile_fp64<S, UQ, PHI, true>(s_j, s, jn, jt, li, xi, yi, zi, eps2, sc, tx, ty, tz, tp);
      else
        tile_fp64<S, UQ, PHI, false>(s_j, s, jn, jt, li, xi, yi, zi, eps2, sc, tx, ty, tz, tp);
    }
    if (++tiles == TILES_PER_SUM || jt + TS >= n) {
      tiles = 0;
      two_sum(Sx, Cx, tx);
      two_sum(Sy, Cy, ty);
      two_sum(Sz, Cz, tz);
      if (PHI) two_sum(Sp, Cp, tp);
      tx = ty = tz = tp = T(0);
    }
  }

  // a receiver's S lanes: FP64 xor butterfly over the SW lanes of each
  // wavefront (masks R .. 32; every lane ends with the same bits, a + b ==
  // b + a), then the four wavefronts' sums in wavefront order
  double ex = (double)Sx + (double)Cx, ey = (double)Sy + (double)Cy, ez = (double)Sz + (double)Cz;
  double ph = PHI ? (double)Sp + (double)Cp : 0.0;
#pragma unroll
  for (int m = R; m < 64; m <<= 1) {
    ex += __shfl_xor(ex, m, 64);
    ey += __shfl_xor(ey, m, 64);
    ez += __shfl_xor(ez, m, 64);
    if (PHI) ph += __shfl_xor(ph, m, 64);
  }
  if (l < R) {
    s_red[w][l][0] = ex;
    s_red[w][l][1] = ey;
    s_red[w][l][2] = ez;
    s_red[w][l][3] = ph;
  }
  __syncthreads();
  if (tid < R && li < n) {
    double e[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      e[q] = s_red[0][tid][q];
#pragma unroll
      for (int ww = 1; ww < FT / 64; ++ww) e[q] += s_red[ww][tid][q];
    }
    update_particle<MIXED, MODE>(a.upd, B, off + li, e[0], e[1], e[2], e[3], PHI);
  }
}

template <bool MIXED, int R, int FT, bool UQ, bool PHI>
hipError_t go_mode(const FusedArgs& a, FinalMode mode, int n_items, hipStream_t st) {
#define PP_FUSED(MD) \
  hipLaunchKernelGGL((fused_kernel<MIXED, R, FT, UQ, PHI, MD>), dim3(n_items), dim3(FT), 0, st, a)
  switch (mode) {
    case FIN_FIELD: PP_FUSED(FIN_FIELD); break;
    case FIN_ACCEL: PP_FUSED(FIN_ACCEL); break;
    case FIN_KICK: PP_FUSED(FIN_KICK); break;
    default: PP_FUSED(FIN_KICK_DRIFT); break;
  }
#undef PP_FUSED
  return hipGetLastError();
}

template <bool MIXED, int R, int FT>
hipError_t go_fused(const FusedArgs& a, FinalMode mode, bool uq, bool phi, int n_items, hipStream_t st) {
  // the potential is summed only for field evaluations that ask for it
  if (phi && mode == FIN_FIELD)
    return uq ? go_mode<MIXED, R, FT, true, true>(a, mode, n_items, st)
              : go_mode<MIXED, R, FT, false, true>(a, mode, n_items, st);
  return uq ? go_mode<MIXED, R, FT, true, false>(a, mode, n_items, st)
            : go_mode<MIXED, R, FT, false, false>(a, mode, n_items, st);
}

template <bool MIXED, int FT>
hipError_t go_fused_r(const FusedArgs& a, int receivers, FinalMode mode, bool uq, bool phi, int n_items,
                      hipStream_t st) {
  switch (receivers) {
    case 4: return go_fused<MIXED, 4, FT>(a, mode, uq, phi, n_items, st);
    case 8: return go_fused<MIXED, 8, FT>(a, mode, uq, phi, n_items, st);
    case 16: return go_fused<MIXED, 16, FT>(a, mode, uq, phi, n_items, st);
    case 32: return go_fused<MIXED, 32, FT>(a, mode, uq, phi, n_items, st);
    default: return hipErrorInvalidValue;
  }
}

template <bool MIXED>
hipError_t go_fused_w(const FusedArgs& a, int receivers, int threads, FinalMode mode, bool uq, bool phi,
                      int n_items, hipStream_t st) {
  switch (threads) {
    case 256: return go_fused_r<MIXED, 256>(a, receivers, mode, uq, phi, n_items, st);
    case 512: return go_fused_r<MIXED, 512>(a, receivers, mode, uq, phi, n_items, st);
    case 1024: return go_fused_r<MIXED, 1024>(a, receivers, mode, uq, phi, n_items, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_fused(const FusedArgs& a, bool mixed, int receivers, int threads, FinalMode mode, bool uniform_q,
                        bool with_phi, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  return mixed ? go_fused_w<true>(a, receivers, threads, mode, uniform_q, with_phi, n_items, s)
               : go_fused_w<false>(a, receivers, threads, mode, uniform_q, with_phi, n_items, s);
}

}  // namespace ppk
