// pp_sym64.hip -- symmetric FP64 pair sum for gfx950 (the FP64 path's
// schedule for large bunches).
//
// Same method as the mixed symmetric kernel (pp_sym.hip): the pair term of
// Eq. (A) is antisymmetric, so one reciprocal square root serves the two
// ordered interactions of an unordered pair.  Items pair a receiver block I (SYM64_WAVES wavefronts, i_per_lane receivers
// per lane in VGPRs) with a source block J swept in groups of 64 staged in
// LDS; in step s of a group lane l meets source (l + s) mod 64 and the
// source-side partial follows its source one lane down per step (two
// ds_bpermute per double), arriving at the source's home lane after the 64th
// step.  r^-3 comes from v_rsq_f64 and one third-order series correction
// (inv_r3_64).  Items write FP64 partial slots indexed (sub-round, block,
// side), one value per component rounded once from the item's compensated
// sum, a source-side slot per round and one receiver-side slot per item (an
// item covers sym_rounds consecutive rounds in large bunches); the fold adds
// them in sub-round order, so every addition has a fixed order.  A sub-round r S + h is part h of round r when block pairs are split
// in S parts of the source block's groups (S = 1: plain rounds).
//
// Positions are the unscaled FP64 state and separations are plain FP64
// differences (no hi/lo split and no spatial sort are needed at this
// precision).
#include "pp_device.h"
#include "pp_device64.h"
#include "pp_fold.h"
#include "pp_sym64.h"

#include <cmath>

namespace ppk {
namespace {

// Out-of-range receivers and sources of a ragged block sit at two distinct far
// points, +-1e149 on every axis, with charge weight 0.  Any separation they
// take part in has r2 ~ 1e299: finite and never zero (r2 = 0 would give
// y = inf and e = 1 - 0 * inf = NaN in inv_r3_64), with y ~ 1e-150 and
// y^3 ~ 1e-449, which underflows to exactly 0, so every field term of a padded
// particle is an exact zero without the weight.  Only its potential term
// (y ~ 1e-150) needs the weight: with uniform charges the items that contain
// padding and want the potential take the weighted sweep.
constexpr double FAR_RECV = 1e149;
constexpr double FAR_SRC = -1e149;

__device__ __forceinline__ double lane_read64(double v, int src_lane) {
  // value of v in lane src_lane (two ds_bpermute, LDS crossbar only)
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(bits & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(bits >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int K, bool UQ, bool PHI, bool DIAG>
__device__ __forceinline__ void sweep_group64(const double4* __restrict__ sj, int l, int gsel,
                                              const double (&xi)[K], const double (&yi)[K], const double (&zi)[K],
                                              const double (&qi)[K], double eps2, const SeriesConst& sc,
                                              double (&ti)[3][K], double (&tip)[K], double (&aj)[4]) {
  // aj: plain partial of the source met in step s, (l + s) mod 64, which moves
  // one lane down after every step; after the 64 steps lane l holds the whole
  // group's partial of its own source l (64 terms in a plain FP64 sum, as the
  // receiver side's tile sum).  The group is stored twice in LDS so step s
  // reads entry l + s with no wrap.
#pragma unroll 4
  for (int s = 0; s < 64; ++s) {
    const double4 h = sj[l + s];
    double dx[K], dy[K], dz[K], s3[K], inv[K];
    bool self[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      dx[k] = xi[k] - h.x;
      dy[k] = yi[k] - h.y;
      dz[k] = zi[k] - h.z;
      double r2 = fma(dz[k], dz[k], fma(dy[k], dy[k], fma(dx[k], dx[k], eps2)));
      // self term: receiver group gsel + k meets source lane l at step 0
      self[k] = DIAG && s == 0 && gsel == k;
      if (DIAG && self[k]) r2 = 1.0;
      s3[k] = inv_r3_64<PHI>(r2, sc, inv[k]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double f3 = s3[k];
      double ph = PHI ? inv[k] : 0.0;
      if (DIAG && self[k]) { f3 = 0.0; ph = 0.0; }
      const double fi = UQ ? f3 : h.w * f3;
      ti[0][k] = fma(dx[k], fi, ti[0][k]);
      ti[1][k] = fma(dy[k], fi, ti[1][k]);
      ti[2][k] = fma(dz[k], fi, ti[2][k]);
      if (PHI) tip[k] += UQ ? ph : h.w * ph;
      if (!DIAG) {
        const double fj = UQ ? f3 : qi[k] * f3;
        aj[0] = fma(-dx[k], fj, aj[0]);
        aj[1] = fma(-dy[k], fj, aj[1]);
        aj[2] = fma(-dz[k], fj, aj[2]);
        if (PHI) aj[3] += UQ ? ph : qi[k] * ph;
      }
    }
    if (!DIAG) {
      // lane l takes over the partial of source (l + s + 1) mod 64 from lane l + 1
#pragma unroll
      for (int q = 0; q < (PHI ? 4 : 3); ++q) aj[q] = lane_read64(aj[q], (l + 1) & 63);
    }
  }
}

struct SymShared64 {
  double4 sj[128];                 // source group twice: position, normalised charge
  double xw[SYM64_WAVES][4][64];   // per-wave source-side partials for the cross-wave combine
};

template <int K, bool UQ, bool PHI, bool DIAG>
__device__ void sym_item64(const SymArgs64& a, const SymItem& it, SymShared64& sh) {
  double4* sj = sh.sj;
  auto& xw = sh.xw;
  const BunchDev& B = a.bunches[it.b];
  const int n = (int)B.n;
  const int64_t off = B.off;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  constexpr int BS = SYM64_WAVES * 64 * K;
  const int ibase = it.I * BS;
  const int nbk = (n + BS - 1) / BS;
  const SeriesConst sc = series_const();  // series constants held in registers
  const double eps2 = B.eps2;
  const int64_t rho = it.r - a.r0;
  double* rslot = a.slot + ((rho * a.nbt + B.bbase + it.I) * 2) * (int64_t)(SLOT_PLANES * BS);

  double xi[K], yi[K], zi[K], qi[K];
  double Si[3][K], Ci[3][K], Sip[K], Cip[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int li = ibase + (w * K + k) * 64 + l;
    if (li < n) {
      const int64_t g = off + li;
      xi[k] = a.x[g]; yi[k] = a.y[g]; zi[k] = a.z[g];
      qi[k] = UQ ? 1.0 : a.qt[g];
    } else {
      xi[k] = yi[k] = zi[k] = FAR_RECV;
      qi[k] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) Si[c][k] = Ci[c][k] = 0.0;
    Sip[k] = Cip[k] = 0.0;
  }

  // this item's part of each of its source blocks J: groups [g0, g1) of
  // the block's BS / 64; rounds d0 .. d0 + nr - 1, the receiver side summed
  // over all of them
  const int gpart = BS / 64 / a.split;
  const int hpart = it.r % a.split, d0 = it.r / a.split;
  const int g0 = hpart * gpart, g1 = g0 + gpart;
  const int nr = DIAG ? 1 : it.nr;
  for (int kr = 0; kr < nr; ++kr) {
  const int jblk = DIAG ? it.I : (it.I + d0 + kr) % nbk;
  const int jbase0 = jblk * BS;
  const bool pad = (n - ibase < BS) || (n - jbase0 < BS);  // a ragged last block takes part
  const int64_t rho_s = (int64_t)(d0 + kr) * a.split + hpart - a.r0;
  double* sslot = a.slot + ((rho_s * a.nbt + B.bbase + jblk) * 2 + 1) * (int64_t)(SLOT_PLANES * BS);
  for (int g = g0; g < g1; ++g) {
    const int jg = jbase0 + g * 64;
    __syncthreads();  // LDS of the previous group is free
    if (w == 0) {
      const int lj = jg + l;
      double4 v;
      if (lj < n) {
        const int64_t gi = off + lj;
        v = make_double4(a.x[gi], a.y[gi], a.z[gi], UQ ? 1.0 : a.qt[gi]);
      } else {
        v = make_double4(FAR_SRC, FAR_SRC, FAR_SRC, 0.0);
      }
      sj[l] = v;
      sj[l + 64] = v;
    }
    __syncthreads();

    double ti[3][K], tip[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { ti[0][k] = ti[1][k] = ti[2][k] = tip[k] = 0.0; }
    double aj[4] = {0.0, 0.0, 0.0, 0.0};
    // in a diagonal item the receivers of wave w, slot k belong to group w*K + k
    if (UQ && PHI && pad)  // unit weights 1.0 for real particles give the same bits as the uniform path
      sweep_group64<K, false, PHI, DIAG>(sj, l, DIAG ? g - w * K : -1, xi, yi, zi, qi, eps2, sc, ti, tip, aj);
    else
      sweep_group64<K, UQ, PHI, DIAG>(sj, l, DIAG ? g - w * K : -1, xi, yi, zi, qi, eps2, sc, ti, tip, aj);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      two_sum(Si[0][k], Ci[0][k], ti[0][k]);
      two_sum(Si[1][k], Ci[1][k], ti[1][k]);
      two_sum(Si[2][k], Ci[2][k], ti[2][k]);
      if (PHI) two_sum(Sip[k], Cip[k], tip[k]);
    }
    if (!DIAG) {
#pragma unroll
      for (int q = 0; q < (PHI ? 4 : 3); ++q) xw[w][q][l] = aj[q];
      __syncthreads();
      // one thread per (source, component): waves 0-3 add the waves' partials
      // in wave order with two-sum and store the source-side partial, S + C
      const int q = tid >> 6;
      if (q < (PHI ? 4 : 3)) {
        double S = xw[0][q][l], C = 0.0;
        for (int ww = 1; ww < SYM64_WAVES; ++ww) two_sum(S, C, xw[ww][q][l]);
        if (jg + l < n) {
          const int o = g * 64 + l;
          sslot[q * BS + o] = S + C;
        }
      }
    }
  }
  }

  // receiver-side partial
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int o = (w * K + k) * 64 + l;
    if (ibase + o >= n) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) rslot[c * BS + o] = Si[c][k] + Ci[c][k];
    if (PHI) {
      rslot[3 * BS + o] = Sip[k] + Cip[k];
    }
  }
}

template <int K, bool UQ, bool PHI>
__global__ __launch_bounds__(SYM64_WG) void pair_sym64_kernel(SymArgs64 a, int32_t first) {
  __shared__ SymShared64 sh;
  const SymItem it = a.items[first + blockIdx.x];
  if (it.r < a.split)
    sym_item64<K, UQ, PHI, true>(a, it, sh);
  else
    sym_item64<K, UQ, PHI, false>(a, it, sh);
}

template <int K, bool UQ, bool PHI>
hipError_t go_sym64(const SymArgs64& a, int32_t first, int32_t count, hipStream_t s) {
  hipLaunchKernelGGL((pair_sym64_kernel<K, UQ, PHI>), dim3(count), dim3(SYM64_WG), 0, s, a, first);
  return hipGetLastError();
}

template <int K>
hipError_t go_sym64_k(const SymArgs64& a, int32_t first, int32_t count, bool uq, bool phi, hipStream_t s) {
  if (uq) return phi ? go_sym64<K, true, true>(a, first, count, s) : go_sym64<K, true, false>(a, first, count, s);
  return phi ? go_sym64<K, false, true>(a, first, count, s) : go_sym64<K, false, false>(a, first, count, s);
}

// One thread per position: adds the slots of sub-rounds [r0, r1) in order to
// the accumulators; sub-round 0 (the first part of the diagonal items) starts
// them.  Receiver side: every part of a block pair; source side: only the part
// that holds this position.
// One thread per (particle, component): grid y is the component (x, y, z,
// and the potential when asked for); each component's sums are independent.
__global__ __launch_bounds__(256) void sym64_fold_kernel(SymFoldArgs64 a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (p >= a.n_total) return;
  const int b = a.bid[p];
  if (b < 0) return;
  const BunchDev& B = a.bunches[b];
  const int BS = a.block_size;
  const int l = (int)(p - B.off);
  const int X = l / BS, o = l - X * BS;
  const int nbk = (int)((B.n + BS - 1) / BS);
  const int64_t P = a.n_total;
  // accumulator planes of component q: receiver S, C and source S, C
  const int pl = q < 3 ? q : 12;
  const int ps = q < 3 ? 3 : 1;
  double rs = 0, rc = 0, ss = 0, sc = 0;
  if (a.r0 != 0) {
    rs = a.acc[(pl + 0 * ps) * P + p];
    rc = a.acc[(pl + 1 * ps) * P + p];
    ss = a.acc[(pl + 2 * ps) * P + p];
    sc = a.acc[(pl + 3 * ps) * P + p];
  }
  const int64_t sl = (int64_t)SLOT_PLANES * BS;
  const int S = a.split, part = o / (BS / S);
  const int M = sym_rounds_for(nbk, a.rounds);
  fold_sweep<double>(a.slot + ((int64_t)B.bbase + X) * 2 * sl + (int64_t)q * BS + o, (int64_t)a.nbt * 2 * sl, sl, a.r0,
                  a.r1, ilog2_pow2(S), part, nbk, ilog2_pow2(M), X, rs, rc, ss, sc);
  a.acc[(pl + 0 * ps) * P + p] = rs;
  a.acc[(pl + 1 * ps) * P + p] = rc;
  a.acc[(pl + 2 * ps) * P + p] = ss;
  a.acc[(pl + 3 * ps) * P + p] = sc;
}

}  // namespace

int sym64_blocks_per_cu(int i_per_lane) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (i_per_lane) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_sym64_kernel<1, true, false>, SYM64_WG, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_sym64_kernel<2, true, false>, SYM64_WG, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_sym64_kernel<4, true, false>, SYM64_WG, 0); break;
    default: break;
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_sym64_fold(const SymFoldArgs64& a, bool with_phi, hipStream_t s) {
  const unsigned grid = (unsigned)((a.n_total + 255) / 256);
  if (with_phi)
    hipLaunchKernelGGL(sym64_fold_kernel, dim3(grid, 4), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(sym64_fold_kernel, dim3(grid, 3), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sym64(const SymArgs64& a, int32_t first, int32_t count, int i_per_lane, bool uniform_q,
                        bool with_phi, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  switch (i_per_lane) {
    case 1: return go_sym64_k<1>(a, first, count, uniform_q, with_phi, s);
    case 2: return go_sym64_k<2>(a, first, count, uniform_q, with_phi, s);
    case 4: return go_sym64_k<4>(a, first, count, uniform_q, with_phi, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ppk
