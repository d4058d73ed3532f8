// pp_sym.hip -- symmetric mixed-precision pair sum for gfx950.
//
// Coulomb's law Eq. (A) is antisymmetric in i and j (Sec. 2.1): the pair term
// q_j d / (|d|^2 + eps^2)^(3/2) added to E_i reappears, with q_i in place of
// q_j and the opposite sign, in E_j.  One v_rsq_f32 therefore serves two
// ordered interactions.  On gfx950 the reciprocal square root costs 10-12
// FP32 issue slots inside a pair evaluation, so this halves the dominant cost.
//
// An item pairs receiver block I (held in VGPRs, i_per_lane per lane, 4 waves)
// with source block J, swept in groups of 64 sources staged in LDS.  In step s
// of a group, lane l meets source (l + s) mod 64 (every lane reads a distinct
// LDS address; the group is stored twice so that the address needs no wrap).  The source-side partial of that source travels with it: after
// each step every lane takes over the partial of its upper neighbour
// (ds_bpermute, an explicit cross-lane move), so after the group's 64 steps
// each partial is back at its source's home lane (lane l owns source l): a
// plain FP32 sum of the wave's 64 K terms for that source.  The 4 waves'
// partials are then added in wave order with two-sum and stored, rounded
// once to fl(S + C), as the source-side partial of the item for that round.
// The receiver side is a plain FP32 sum over each group of 64 sources,
// two-summed into registers across the item's rounds (sym_rounds of them for
// large bunches: one receiver block in registers meets the source blocks of
// consecutive rounds), and stored, rounded once, as the receiver-side partial
// at the end of the item.  Worst-case bounds of the
// plain sums: 63 u of the terms' magnitudes on the receiver side (64 terms),
// (64 K - 1) u on the source side (64 K terms: 255 u at K = 4); errors of
// random sign grow as the square root of the count (measured at most 6e-7 of
// the terms' magnitude sum).
//
// Diagonal items (I == J, round 0) evaluate the ordered pairs inside one block
// with the self term masked and have a receiver-side partial only.  Every
// item writes slots of its own, so the items of many rounds run in one launch
// in any order; the fold kernel then adds the slots of each position in round
// order (receiver side and source side kept apart), which fixes the order of
// every addition.  With block pairs split in S parts (for bunches too small
// to fill the last wave of items), round r becomes sub-rounds r S + h and
// item h sweeps only part h of source block J's groups: a full receiver-side
// slot, the source-side slot at the offsets of its part only.
#include "pp_device.h"
#include "pp_fold.h"
#include "pp_internal.h"

#include <cmath>

namespace ppk {
namespace {

// Out-of-range particles of a ragged block sit here: any separation to a real
// particle squares to +inf in FP32, rsq(+inf) = 0, so their terms are exact
// zeros in both directions.
constexpr float SENTINEL = 1.5e19f;

// Steps of a source group unrolled per loop iteration (a divisor of 64).
// Measured on gfx950: 16 is fastest for 2 and 4 receivers per lane; with 1
// per lane a 16-step body needs 129 VGPRs and 4 steps (75 VGPRs) is 14-24%
// faster.
template <int K>
constexpr int sweep_unroll() { return K == 1 ? 4 : 16; }

__device__ __forceinline__ float lane_read(float v, int src_lane) {
  // value of v in lane src_lane of this wavefront (ds_bpermute: LDS crossbar, no LDS memory)
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

template <int K, bool UQ, bool PHI, bool DIAG, bool FAR>
__device__ __forceinline__ void sweep_group(const float4* __restrict__ sjh, const float4* __restrict__ sjl, int l,
                                            int gsel, const float (&xh)[K], const float (&yh)[K],
                                            const float (&zh)[K], const float (&xl)[K], const float (&yl)[K],
                                            const float (&zl)[K], const float (&qi)[K], float eps2,
                                            float (&ti)[3][K], float (&tip)[K], float (&aj)[4]) {
  // aj: plain partial of the source met in this step, (l + s) mod 64; it moves
  // one lane down every step so that it stays with its source.  The source
  // group is stored twice in LDS (entries 64..127 repeat 0..63), so step s
  // reads entry l + s with no wrap, at an immediate offset from the base of
  // its block of UNR steps.
  constexpr int UNR = sweep_unroll<K>();
  static_assert(64 % UNR == 0, "a group is a whole number of iterations");
  for (int s0 = 0; s0 < 64; s0 += UNR) {
    const float4* hb = sjh + (l + s0);
    const float4* lb = sjl + (l + s0);
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int s = s0 + u;
      const float4 h = hb[u];
      float dx[K], dy[K], dz[K], r2[K], inv[K];
      if (FAR) {
        // far group: plain FP32 separations of the high parts
#pragma unroll
        for (int k = 0; k < K; ++k) {
          dx[k] = xh[k] - h.x;
          dy[k] = yh[k] - h.y;
          dz[k] = zh[k] - h.z;
        }
      } else {
        const float4 lo = lb[u];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          dx[k] = (xh[k] - h.x) + (xl[k] - lo.x);
          dy[k] = (yh[k] - h.y) + (yl[k] - lo.y);
          dz[k] = (zh[k] - h.z) + (zl[k] - lo.z);
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        r2[k] = fmaf(dz[k], dz[k], fmaf(dy[k], dy[k], fmaf(dx[k], dx[k], eps2)));
        if (DIAG) {
          // self term: receiver group gsel + k, source lane l at step 0
          if (s == 0 && gsel == k) r2[k] = __builtin_inff();
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) inv[k] = __builtin_amdgcn_rsqf(r2[k]);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float s3 = (inv[k] * inv[k]) * inv[k];
        const float fi = UQ ? s3 : h.w * s3;
        ti[0][k] = fmaf(dx[k], fi, ti[0][k]);
        ti[1][k] = fmaf(dy[k], fi, ti[1][k]);
        ti[2][k] = fmaf(dz[k], fi, ti[2][k]);
        if (PHI) tip[k] += UQ ? inv[k] : h.w * inv[k];
        if (!DIAG) {
          const float fj = UQ ? s3 : qi[k] * s3;
          aj[0] = fmaf(-dx[k], fj, aj[0]);
          aj[1] = fmaf(-dy[k], fj, aj[1]);
          aj[2] = fmaf(-dz[k], fj, aj[2]);
          if (PHI) aj[3] += UQ ? inv[k] : qi[k] * inv[k];
        }
      }
      if (!DIAG) {
        // lane l takes over the partial of source (l + s + 1) mod 64 from lane l + 1
#pragma unroll
        for (int q = 0; q < (PHI ? 4 : 3); ++q) aj[q] = lane_read(aj[q], (l + 1) & 63);
      }
    }
  }
}

struct SymShared {
  float4 sjh[128];               // source group twice: hi position, normalised charge
  float4 sjl[128];               // source group twice: lo position
  float xw[SYM_WAVES][8][64];    // per-wave two-sum pairs for the cross-wave combine
};

template <int K, bool UQ, bool PHI, bool DIAG>
__device__ void sym_item(const SymArgs& a, const SymItem& it, SymShared& sh) {
  float4* sjh = sh.sjh;
  float4* sjl = sh.sjl;
  auto& xw = sh.xw;

  const BunchDev& B = a.bunches[it.b];
  const int n = (int)B.n;
  const int64_t off = B.off;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  constexpr int BS = SYM_WAVES * 64 * K;
  const int ibase = it.I * BS;
  const int nbk = (n + BS - 1) / BS;
  const float eps2 = B.eps2s;
  const int64_t rho = it.r - a.r0;
  float* rslot = a.slot + ((rho * a.nbt + B.bbase + it.I) * 2) * (int64_t)(SLOT_PLANES * BS);

  // near/far split: this wavefront's receiver box (the union of the boxes of
  // its K groups of 64 sorted receivers) and the threshold; the far/near
  // choice is uniform over the wavefront and may differ between wavefronts
  const bool split = !DIAG && a.near_frac > 0.f;
  float ib[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  float ubound = 0.f, anorm = 0.f;
  if (split) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int gl = ibase / 64 + w * K + k;  // group of the bunch
      if (gl * 64 < n) {
        const float* gx = a.gbox + (int64_t)(B.gbase + gl) * GBOX;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          ib[c] = fminf(ib[c], gx[c]);
          ib[3 + c] = fmaxf(ib[3 + c], gx[3 + c]);
        }
      }
    }
    // dropping lo moves separation component c by at most 2^-24 (|u_i,c| + |u_j,c|):
    // the threshold scales with the coordinate sizes of the two boxes, capped by
    // the bunch bound U
    ubound = __uint_as_float(a.ubits[it.b]);
    if (ib[0] <= ib[3]) {
      float s2 = 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float m = fmaxf(fabsf(ib[c]), fabsf(ib[3 + c]));
        s2 = fmaf(m, m, s2);
      }
      anorm = sqrtf(s2);
    }
  }

  float xh[K], yh[K], zh[K], xl[K], yl[K], zl[K], qi[K];
  float Si[3][K], Ci[3][K], Sip[K], Cip[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int li = ibase + (w * K + k) * 64 + l;
    if (li < n) {
      const int64_t g = off + li;
      xh[k] = a.xh[g]; yh[k] = a.yh[g]; zh[k] = a.zh[g];
      xl[k] = a.xl[g]; yl[k] = a.yl[g]; zl[k] = a.zl[g];
      qi[k] = UQ ? 1.f : a.qt[g];
    } else {
      xh[k] = yh[k] = zh[k] = SENTINEL;
      xl[k] = yl[k] = zl[k] = 0.f;
      qi[k] = 0.f;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) Si[c][k] = Ci[c][k] = 0.f;
    Sip[k] = Cip[k] = 0.f;
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
  const int64_t rho_s = (int64_t)(d0 + kr) * a.split + hpart - a.r0;
  float* sslot = a.slot + ((rho_s * a.nbt + B.bbase + jblk) * 2 + 1) * (int64_t)(SLOT_PLANES * BS);
  for (int g = g0; g < g1; ++g) {
    const int jg = jbase0 + g * 64;
    __syncthreads();  // LDS of the previous group is free
    if (w == 0) {
      const int lj = jg + l;
      float4 h, lo;
      if (lj < n) {
        const int64_t gi = off + lj;
        h = make_float4(a.xh[gi], a.yh[gi], a.zh[gi], UQ ? 1.f : a.qt[gi]);
        lo = make_float4(a.xl[gi], a.yl[gi], a.zl[gi], 0.f);
      } else {
        h = make_float4(SENTINEL, SENTINEL, SENTINEL, 0.f);
        lo = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      sjh[l] = h;
      sjh[l + 64] = h;
      sjl[l] = lo;
      sjl[l + 64] = lo;
    }
    __syncthreads();

    float ti[3][K], tip[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { ti[0][k] = ti[1][k] = ti[2][k] = tip[k] = 0.f; }
    float aj[4] = {0.f, 0.f, 0.f, 0.f};
    bool far = false;
    if (split) {
      if (jg >= n || ib[0] > ib[3]) {
        far = true;  // sentinel-only receivers or sources: every term is an exact zero on either path
      } else {
        const float* gb = a.gbox + (int64_t)(B.gbase + jg / 64) * GBOX;
        float gap2 = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float d = fmaxf(0.f, fmaxf(gb[c] - ib[3 + c], ib[c] - gb[3 + c]));
          gap2 = fmaf(d, d, gap2);
        }
        // D = near_frac * min(U, (|a| + |b|) / 2), |a|, |b| the norms of the boxes'
        // per-axis largest |coordinate| (|b| stored with the group box)
        const float dfar = a.near_frac * fminf(ubound, 0.5f * (anorm + gb[6]));
        far = gap2 > dfar * dfar;
      }
    }
    // in a diagonal item the receivers of wave w, slot k belong to group w*K + k
    if (far)
      sweep_group<K, UQ, PHI, DIAG, true>(sjh, sjl, l, -1, xh, yh, zh, xl, yl, zl, qi, eps2, ti, tip, aj);
    else
      sweep_group<K, UQ, PHI, DIAG, false>(sjh, sjl, l, DIAG ? g - w * K : -1, xh, yh, zh, xl, yl, zl, qi, eps2,
                                           ti, tip, aj);
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
      // one thread per (source, component): waves 0-3 combine the 4 waves'
      // pairs in wave order and store the source-side partial
      const int q = tid >> 6;  // 0..2 field components, 3 potential
      if (q < (PHI ? 4 : 3)) {
        float S = xw[0][q][l], C = 0.f;
        for (int ww = 1; ww < SYM_WAVES; ++ww) two_sum(S, C, xw[ww][q][l]);
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
__global__ __launch_bounds__(SYM_WG) void pair_sym_kernel(SymArgs a, int32_t first) {
  __shared__ SymShared sh;
  const SymItem it = a.items[first + blockIdx.x];
  if (it.r < a.split)
    sym_item<K, UQ, PHI, true>(a, it, sh);
  else
    sym_item<K, UQ, PHI, false>(a, it, sh);
}

template <int K, bool UQ, bool PHI>
hipError_t go_sym(const SymArgs& a, int32_t first, int32_t count, hipStream_t s) {
  hipLaunchKernelGGL((pair_sym_kernel<K, UQ, PHI>), dim3(count), dim3(SYM_WG), 0, s, a, first);
  return hipGetLastError();
}

template <int K>
hipError_t go_sym_k(const SymArgs& a, int32_t first, int32_t count, bool uq, bool phi, hipStream_t s) {
  if (uq) return phi ? go_sym<K, true, true>(a, first, count, s) : go_sym<K, true, false>(a, first, count, s);
  return phi ? go_sym<K, false, true>(a, first, count, s) : go_sym<K, false, false>(a, first, count, s);
}

// One thread per position: adds the slots of sub-rounds [r0, r1) in order to
// the accumulators; sub-round 0 (the first part of the diagonal items) starts
// them.  Receiver side: every part of a block pair; source side: only the part
// that holds this position.
// One thread per (particle, component): grid y is the component (x, y, z,
// and the potential when asked for); each component's sums are independent.
__global__ __launch_bounds__(256) void sym_fold_kernel(SymFoldArgs a) {
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
  float rs = 0, rc = 0, ss = 0, sc = 0;
  if (a.r0 != 0) {
    rs = a.acc[(pl + 0 * ps) * P + p];
    rc = a.acc[(pl + 1 * ps) * P + p];
    ss = a.acc[(pl + 2 * ps) * P + p];
    sc = a.acc[(pl + 3 * ps) * P + p];
  }
  const int64_t sl = (int64_t)SLOT_PLANES * BS;
  const int S = a.split, part = o / (BS / S);
  const int M = sym_rounds_for(nbk, a.rounds);
  fold_sweep<float>(a.slot + ((int64_t)B.bbase + X) * 2 * sl + (int64_t)q * BS + o, (int64_t)a.nbt * 2 * sl, sl, a.r0,
                  a.r1, ilog2_pow2(S), part, nbk, ilog2_pow2(M), X, rs, rc, ss, sc);
  a.acc[(pl + 0 * ps) * P + p] = rs;
  a.acc[(pl + 1 * ps) * P + p] = rc;
  a.acc[(pl + 2 * ps) * P + p] = ss;
  a.acc[(pl + 3 * ps) * P + p] = sc;
}

}  // namespace

hipError_t launch_sym_fold(const SymFoldArgs& a, bool with_phi, hipStream_t s) {
  const unsigned grid = (unsigned)((a.n_total + 255) / 256);
  if (with_phi)
    hipLaunchKernelGGL(sym_fold_kernel, dim3(grid, 4), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(sym_fold_kernel, dim3(grid, 3), dim3(256), 0, s, a);
  return hipGetLastError();
}

int sym_blocks_per_cu(int i_per_lane) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (i_per_lane) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_sym_kernel<1, true, false>, SYM_WG, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_sym_kernel<2, true, false>, SYM_WG, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pair_sym_kernel<4, true, false>, SYM_WG, 0); break;
    default: break;
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_sym(const SymArgs& a, int32_t first, int32_t count, int i_per_lane, bool uniform_q, bool with_phi,
                      hipStream_t s) {
  if (count <= 0) return hipSuccess;
  switch (i_per_lane) {
    case 1: return go_sym_k<1>(a, first, count, uniform_q, with_phi, s);
    case 2: return go_sym_k<2>(a, first, count, uniform_q, with_phi, s);
    case 4: return go_sym_k<4>(a, first, count, uniform_q, with_phi, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ppk
