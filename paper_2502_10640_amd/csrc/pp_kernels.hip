// pp_kernels.hip -- gfx950 kernels of the PP library.
//
// Hot path (arXiv 2502.10640 Sec. 2.1): the direct pair sum of Eq. (B) with
// Plummer softening over all ordered pairs, one kernel over a flattened work
// list that serves every bunch of the context (one workgroup per item for
// short lists, a persistent grid with a work counter for long ones; the
// symmetric schedules for large bunches are in pp_sym.hip and pp_sym64.hip).
// Receivers sit in registers (i_per_lane per lane), sources are staged through
// LDS in tiles of JT particles loaded with coalesced SoA reads and read back as
// same-address (broadcast) LDS loads.  The pairwise law is evaluated on the
// vector ALUs with v_rsq_f32 (mixed) or v_rsq_f64 and a series correction
// (FP64, inv_r3_64); no MFMA: an inverse-cube law is not a dense contraction.
//
// Per-receiver sums are exact-order deterministic: a plain sum over sum_tile
// sources, then a two-sum (Knuth) into a running (sum, compensation) pair.
// Each work item writes its own partial slot; the final kernel adds the
// chunk partials in a fixed order in FP64.  No floating-point atomics anywhere;
// the only atomic is the work counter, which decides who computes an item,
// never the order of an addition.
#include "pp_device.h"
#include "pp_device64.h"
#include "pp_internal.h"
#include "pp_update.h"

#include <cfloat>
#include <cmath>

#ifndef PP_MIXED_WAVES_PER_EU
#define PP_MIXED_WAVES_PER_EU 2
#endif

namespace ppk {
namespace {

// ---------------------------------------------------------------------------
// Mixed precision pair sum.  Separation d = (hi_i - hi_j) + (lo_i - lo_j):
// the high-part difference is a plain FP32 subtraction, the low parts carry
// the ~24 bits FP32 rounding of the positions dropped, so d keeps the
// accuracy of the FP64 positions even for close pairs far from the origin.
// ---------------------------------------------------------------------------
template <int K, bool UQ, bool PHI, bool DIAG>
__device__ __forceinline__ void acc_mixed(const float4* __restrict__ sh, const float4* __restrict__ sl,
                                          int jb, int je, int jbase, const int (&li)[K],
                                          const float (&xh)[K], const float (&yh)[K], const float (&zh)[K],
                                          const float (&xl)[K], const float (&yl)[K], const float (&zl)[K],
                                          float eps2, float (&tx)[K], float (&ty)[K], float (&tz)[K],
                                          float (&tp)[K]) {
  // Stages run across the K receivers so that K independent pairs are in
  // flight between a v_rsq_f32 and the first use of its result.
#pragma unroll 2
  for (int jj = jb; jj < je; ++jj) {
    const float4 h = sh[jj];
    const float4 l = sl[jj];
    float dx[K], dy[K], dz[K], r2[K], inv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      dx[k] = (xh[k] - h.x) + (xl[k] - l.x);
      dy[k] = (yh[k] - h.y) + (yl[k] - l.y);
      dz[k] = (zh[k] - h.z) + (zl[k] - l.z);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      r2[k] = fmaf(dz[k], dz[k], fmaf(dy[k], dy[k], fmaf(dx[k], dx[k], eps2)));
      if (DIAG) {
        // self term j == i: rsq(+inf) = 0 removes it from E and phi
        if (jbase + jj == li[k]) r2[k] = __builtin_inff();
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) inv[k] = __builtin_amdgcn_rsqf(r2[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float inv2 = inv[k] * inv[k];
      const float s = UQ ? inv2 * inv[k] : (h.w * inv[k]) * inv2;
      tx[k] = fmaf(dx[k], s, tx[k]);
      ty[k] = fmaf(dy[k], s, ty[k]);
      tz[k] = fmaf(dz[k], s, tz[k]);
      if (PHI) tp[k] += UQ ? inv[k] : h.w * inv[k];
    }
  }
}

template <int K, bool UQ, bool PHI>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(PP_MIXED_WAVES_PER_EU)))
void pair_mixed_kernel(PairArgs a, int32_t sum_tile) {
  __shared__ float4 s_hi[JT];
  __shared__ float4 s_lo[JT];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  for (int pass = 0;; ++pass) {
    int it;
    if (a.direct) {
      // one workgroup per item, in work-list order: no counter
      if (pass > 0) break;
      it = blockIdx.x;
    } else {
      __syncthreads();  // previous item done with s_item and the tile
      if (tid == 0) s_item = atomicAdd(a.counter, 1);
      __syncthreads();
      it = s_item;
    }
    if (it >= a.n_items) break;
    const WorkItem w = a.items[it];
    const BunchDev& B = a.bunches[w.b];
    const int64_t off = B.off;
    const int n = (int)B.n;
    const float eps2 = B.eps2s;

    int li[K];
    float xh[K], yh[K], zh[K], xl[K], yl[K], zl[K];
    float Sx[K], Sy[K], Sz[K], Cx[K], Cy[K], Cz[K], Sp[K], Cp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      li[k] = w.i0 + k * WG + tid;
      const int64_t g = off + (li[k] < n ? li[k] : 0);
      xh[k] = a.xh[g]; yh[k] = a.yh[g]; zh[k] = a.zh[g];
      xl[k] = a.xl[g]; yl[k] = a.yl[g]; zl[k] = a.zl[g];
      Sx[k] = Sy[k] = Sz[k] = Cx[k] = Cy[k] = Cz[k] = Sp[k] = Cp[k] = 0.f;
    }

    const int j0 = (int)((int64_t)w.chunk * B.chunk_len);
    const int j1 = (int)min((int64_t)n, (int64_t)j0 + B.chunk_len);
    const int ilo = w.i0, ihi = w.i0 + K * WG;

    float4 rh = make_float4(0.f, 0.f, 0.f, 0.f), rl = rh;
    if (j0 + tid < j1) {
      const int64_t g = off + j0 + tid;
      rh = make_float4(a.xh[g], a.yh[g], a.zh[g], a.qt[g]);
      rl = make_float4(a.xl[g], a.yl[g], a.zl[g], 0.f);
    }
    for (int jt = j0; jt < j1; jt += JT) {
      const int jn = min(JT, j1 - jt);
      __syncthreads();
      s_hi[tid] = rh;
      s_lo[tid] = rl;
      __syncthreads();
      if (jt + JT + tid < j1) {  // prefetch the next tile while this one is used
        const int64_t g = off + jt + JT + tid;
        rh = make_float4(a.xh[g], a.yh[g], a.zh[g], a.qt[g]);
        rl = make_float4(a.xl[g], a.yl[g], a.zl[g], 0.f);
      }
      const bool diag = (jt < ihi) && (jt + jn > ilo);
      for (int s0 = 0; s0 < jn; s0 += sum_tile) {
        const int se = min(jn, s0 + sum_tile);
        float tx[K], ty[K], tz[K], tp[K];
#pragma unroll
        for (int k = 0; k < K; ++k) tx[k] = ty[k] = tz[k] = tp[k] = 0.f;
        if (diag)
          acc_mixed<K, UQ, PHI, true>(s_hi, s_lo, s0, se, jt, li, xh, yh, zh, xl, yl, zl, eps2, tx, ty, tz, tp);
        else
          acc_mixed<K, UQ, PHI, false>(s_hi, s_lo, s0, se, jt, li, xh, yh, zh, xl, yl, zl, eps2, tx, ty, tz, tp);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          two_sum(Sx[k], Cx[k], tx[k]);
          two_sum(Sy[k], Cy[k], ty[k]);
          two_sum(Sz[k], Cz[k], tz[k]);
          if (PHI) two_sum(Sp[k], Cp[k], tp[k]);
        }
      }
    }
    const int64_t base = B.pbase + (int64_t)w.chunk * n;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (li[k] < n) {
        const int64_t s = base + li[k];
        a.pf[0 * a.P + s] = Sx[k]; a.pf[1 * a.P + s] = Sy[k]; a.pf[2 * a.P + s] = Sz[k];
        a.pf[3 * a.P + s] = Cx[k]; a.pf[4 * a.P + s] = Cy[k]; a.pf[5 * a.P + s] = Cz[k];
        if (PHI) { a.pf[6 * a.P + s] = Sp[k]; a.pf[7 * a.P + s] = Cp[k]; }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 pair sum (the plain reference path on the GPU).
// ---------------------------------------------------------------------------
template <int K, bool UQ, bool PHI, bool DIAG>
__device__ __forceinline__ void acc_fp64(const double4* __restrict__ sj, int jb, int je, int jbase,
                                         const int (&li)[K], const double (&xi)[K], const double (&yi)[K],
                                         const double (&zi)[K], double eps2, const SeriesConst& sc, double (&tx)[K],
                                         double (&ty)[K], double (&tz)[K], double (&tp)[K]) {
#pragma unroll 2
  for (int jj = jb; jj < je; ++jj) {
    const double4 p = sj[jj];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double dx = xi[k] - p.x;
      const double dy = yi[k] - p.y;
      const double dz = zi[k] - p.z;
      double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
      bool self = false;
      if (DIAG) {
        self = (jbase + jj == li[k]);
        if (self) r2 = 1.0;
      }
      double inv = 0.0;
      const double s3 = inv_r3_64<PHI>(r2, sc, inv);
      double s = UQ ? s3 : p.w * s3;
      double ph = UQ ? inv : p.w * inv;
      if (DIAG) {
        if (self) { s = 0.0; ph = 0.0; }
      }
      tx[k] = fma(dx, s, tx[k]);
      ty[k] = fma(dy, s, ty[k]);
      tz[k] = fma(dz, s, tz[k]);
      if (PHI) tp[k] += ph;
    }
  }
}

template <int K, bool UQ, bool PHI>
__global__ __launch_bounds__(WG) void pair_fp64_kernel(PairArgs a, int32_t sum_tile) {
  __shared__ double4 s_j[JT];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  for (int pass = 0;; ++pass) {
    int it;
    if (a.direct) {
      if (pass > 0) break;
      it = blockIdx.x;
    } else {
      __syncthreads();
      if (tid == 0) s_item = atomicAdd(a.counter, 1);
      __syncthreads();
      it = s_item;
    }
    if (it >= a.n_items) break;
    const WorkItem w = a.items[it];
    const BunchDev& B = a.bunches[w.b];
    const int64_t off = B.off;
    const int n = (int)B.n;
    const double eps2 = B.eps2;
    const SeriesConst sc = series_const();  // series constants held in registers

    int li[K];
    double xi[K], yi[K], zi[K];
    double Sx[K], Sy[K], Sz[K], Cx[K], Cy[K], Cz[K], Sp[K], Cp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      li[k] = w.i0 + k * WG + tid;
      const int64_t g = off + (li[k] < n ? li[k] : 0);
      xi[k] = a.x[g]; yi[k] = a.y[g]; zi[k] = a.z[g];
      Sx[k] = Sy[k] = Sz[k] = Cx[k] = Cy[k] = Cz[k] = Sp[k] = Cp[k] = 0.0;
    }
    const int j0 = (int)((int64_t)w.chunk * B.chunk_len);
    const int j1 = (int)min((int64_t)n, (int64_t)j0 + B.chunk_len);
    const int ilo = w.i0, ihi = w.i0 + K * WG;

    double4 r = make_double4(0.0, 0.0, 0.0, 0.0);
    if (j0 + tid < j1) {
      const int64_t g = off + j0 + tid;
      r = make_double4(a.x[g], a.y[g], a.z[g], a.qt64[g]);
    }
    for (int jt = j0; jt < j1; jt += JT) {
      const int jn = min(JT, j1 - jt);
      __syncthreads();
      s_j[tid] = r;
      __syncthreads();
      if (jt + JT + tid < j1) {
        const int64_t g = off + jt + JT + tid;
        r = make_double4(a.x[g], a.y[g], a.z[g], a.qt64[g]);
      }
      const bool diag = (jt < ihi) && (jt + jn > ilo);
      for (int s0 = 0; s0 < jn; s0 += sum_tile) {
        const int se = min(jn, s0 + sum_tile);
        double tx[K], ty[K], tz[K], tp[K];
#pragma unroll
        for (int k = 0; k < K; ++k) tx[k] = ty[k] = tz[k] = tp[k] = 0.0;
        if (diag)
          acc_fp64<K, UQ, PHI, true>(s_j, s0, se, jt, li, xi, yi, zi, eps2, sc, tx, ty, tz, tp);
        else
          acc_fp64<K, UQ, PHI, false>(s_j, s0, se, jt, li, xi, yi, zi, eps2, sc, tx, ty, tz, tp);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          two_sum(Sx[k], Cx[k], tx[k]);
          two_sum(Sy[k], Cy[k], ty[k]);
          two_sum(Sz[k], Cz[k], tz[k]);
          if (PHI) two_sum(Sp[k], Cp[k], tp[k]);
        }
      }
    }
    const int64_t base = B.pbase + (int64_t)w.chunk * n;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (li[k] < n) {
        const int64_t s = base + li[k];
        a.pd[0 * a.P + s] = Sx[k]; a.pd[1 * a.P + s] = Sy[k]; a.pd[2 * a.P + s] = Sz[k];
        a.pd[3 * a.P + s] = Cx[k]; a.pd[4 * a.P + s] = Cy[k]; a.pd[5 * a.P + s] = Cz[k];
        if (PHI) { a.pd[6 * a.P + s] = Sp[k]; a.pd[7 * a.P + s] = Cp[k]; }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Drift (Eq. (G)) fused with the mixed-path source pack; also resets the
// persistent work counter for the pair kernel that follows on the stream.
// ---------------------------------------------------------------------------
template <bool DRIFT, bool MIXED>
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *a.counter = 0;
  if (i >= a.n_total) return;
  const int b = a.bid[i];
  if (b < 0) return;
  const BunchDev& B = a.bunches[b];
  // bunch constants before the stores of x (which would otherwise order these loads after them)
  const double ox = B.origin[0], oy = B.origin[1], oz = B.origin[2], scale = B.scale;
  double x = a.x[i], y = a.y[i], z = a.z[i];
  if (DRIFT) {
    const double dt = B.dt;
    x = drift1(x, a.vx[i], a.ax[i], dt);
    y = drift1(y, a.vy[i], a.ay[i], dt);
    z = drift1(z, a.vz[i], a.az[i], dt);
    a.x[i] = x; a.y[i] = y; a.z[i] = z;
  }
  if (MIXED) mirror1(ox, oy, oz, scale, i, x, y, z, a.xh, a.yh, a.zh, a.xl, a.yl, a.zl);
  else if (a.sx) { a.sx[i] = x; a.sy[i] = y; a.sz[i] = z; }
}

// ---------------------------------------------------------------------------
// Chunk combine in FP64 + field output, acceleration (Eq. (D)/(F)) or kick
// (Eq. (H)).
// ---------------------------------------------------------------------------
// L lanes per particle.  The ordered-pair path uses L = FIN_LANES: lane t adds
// chunks t, t + L, ... in order, then an xor butterfly over the L lanes (every
// lane ends with the same bits, a + b == b + a); the rule depends only on the
// bunch's chunk count.  The symmetric path uses L = 1.
constexpr int FIN_LANES = 8;

template <bool MIXED, int MODE, int L>
__global__ __launch_bounds__(256) void final_kernel(FinalArgs a) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (MODE == FIN_KICK_DRIFT && gt == 0) *a.counter = 0;  // for the next pair kernel on the stream
  const int t = (int)(gt % L);
  const int64_t i = gt / L;
  // the L lanes of a particle take every branch below together
  if (i >= a.n_total) return;
  const int b = a.bid[i];
  if (b < 0) return;
  const BunchDev& B = a.bunches[b];
  // the bunch fields the chunk loop needs, read together
  const int64_t li = i - B.off, bn = B.n, pbase = B.pbase;
  const int n_chunks = a.sym ? 0 : B.n_chunks;
  const bool want_phi = (MODE == FIN_FIELD) && a.phi != nullptr;
  double ex = 0.0, ey = 0.0, ez = 0.0, ph = 0.0;
  if (!MIXED && a.sym) {
    // FP64 symmetric accumulators: receiver side (S, C) then source side (S, C)
    const double* f = a.pd;
    const int64_t P = a.P;
    ex = (f[0 * P + i] + f[3 * P + i]) + (f[6 * P + i] + f[9 * P + i]);
    ey = (f[1 * P + i] + f[4 * P + i]) + (f[7 * P + i] + f[10 * P + i]);
    ez = (f[2 * P + i] + f[5 * P + i]) + (f[8 * P + i] + f[11 * P + i]);
    if (want_phi) ph = (f[12 * P + i] + f[13 * P + i]) + (f[14 * P + i] + f[15 * P + i]);
  }
  if (MIXED && a.sym) {
    // receiver side (S, C) then source side (S, C), in that order
    const float* f = a.pf;
    const int64_t P = a.P;
    const int64_t r = a.rank ? (int64_t)a.rank[i] : i;  // accumulator slot (sorted order)
    ex = ((double)f[0 * P + r] + (double)f[3 * P + r]) + ((double)f[6 * P + r] + (double)f[9 * P + r]);
    ey = ((double)f[1 * P + r] + (double)f[4 * P + r]) + ((double)f[7 * P + r] + (double)f[10 * P + r]);
    ez = ((double)f[2 * P + r] + (double)f[5 * P + r]) + ((double)f[8 * P + r] + (double)f[11 * P + r]);
    if (want_phi) ph = ((double)f[12 * P + r] + (double)f[13 * P + r]) + ((double)f[14 * P + r] + (double)f[15 * P + r]);
  }
  // this lane's chunks in chunk order
#pragma unroll 4
  for (int c = t; c < n_chunks; c += L) {
    const int64_t s = pbase + (int64_t)c * bn + li;
    if (MIXED) {
      ex += (double)a.pf[0 * a.P + s] + (double)a.pf[3 * a.P + s];
      ey += (double)a.pf[1 * a.P + s] + (double)a.pf[4 * a.P + s];
      ez += (double)a.pf[2 * a.P + s] + (double)a.pf[5 * a.P + s];
      if (want_phi) ph += (double)a.pf[6 * a.P + s] + (double)a.pf[7 * a.P + s];
    } else {
      ex += a.pd[0 * a.P + s] + a.pd[3 * a.P + s];
      ey += a.pd[1 * a.P + s] + a.pd[4 * a.P + s];
      ez += a.pd[2 * a.P + s] + a.pd[5 * a.P + s];
      if (want_phi) ph += a.pd[6 * a.P + s] + a.pd[7 * a.P + s];
    }
  }
  if (L > 1) {
#pragma unroll
    for (int m = 1; m < L; m <<= 1) {
      ex += __shfl_xor(ex, m, L);
      ey += __shfl_xor(ey, m, L);
      ez += __shfl_xor(ez, m, L);
      if (want_phi) ph += __shfl_xor(ph, m, L);
    }
    if (t != 0) return;
  }
  update_particle<MIXED, MODE>(a, B, i, ex, ey, ez, ph, want_phi);
}

// ---------------------------------------------------------------------------
// Set-up kernels: bunch id per particle, per-bunch charge normalisation,
// per-bunch extents/validation.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fill_bid_kernel(int32_t* bid, int64_t n_total, const BunchDev* bunches,
                                                       int32_t n_bunches) {
  const int b = blockIdx.y;
  if (b >= n_bunches) return;  // the grid's y extent is the bunch count
  const BunchDev& B = bunches[b];
  for (int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; li < B.n;
       li += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = B.off + li;
    if (i < n_total) bid[i] = b;
  }
}

__global__ __launch_bounds__(256) void qprep_kernel(const BunchDev* bunches, const int32_t* bid, int64_t n_total,
                                                    const double* q, float* qt, double* qt64) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_total) return;
  const int b = bid[i];
  if (b < 0) return;
  const double v = q[i] / bunches[b].qref;
  if (qt) qt[i] = (float)v;
  if (qt64) qt64[i] = v;
}

// Extents for set-up: per bunch [min x, max x, min y, max y, min z, max z,
// min q, max q, min m, max m, non-finite count, 0].
constexpr int MM = MM_LEN;

__device__ __forceinline__ bool fin(double v) { return isfinite(v); }

__global__ __launch_bounds__(256) void minmax_part_kernel(const BunchDev* bunches, const double* x, const double* y,
                                                          const double* z, const double* q, const double* m,
                                                          double* part, int32_t G) {
  __shared__ double sh[256][MM];
  const int b = blockIdx.y, g = blockIdx.x, tid = threadIdx.x;
  const BunchDev& B = bunches[b];
  double r[MM];
  for (int k = 0; k < 10; k += 2) { r[k] = INFINITY; r[k + 1] = -INFINITY; }
  r[10] = 0.0; r[11] = 0.0;
  for (int64_t li = (int64_t)g * blockDim.x + tid; li < B.n; li += (int64_t)G * blockDim.x) {
    const int64_t i = B.off + li;
    const double v[5] = {x[i], y[i], z[i], q[i], m[i]};
    bool ok = true;
    for (int k = 0; k < 5; ++k) {
      ok = ok && fin(v[k]);
      r[2 * k] = fmin(r[2 * k], v[k]);
      r[2 * k + 1] = fmax(r[2 * k + 1], v[k]);
    }
    if (!ok) r[10] += 1.0;
  }
  for (int k = 0; k < MM; ++k) sh[tid][k] = r[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      for (int k = 0; k < 10; k += 2) {
        sh[tid][k] = fmin(sh[tid][k], sh[tid + s][k]);
        sh[tid][k + 1] = fmax(sh[tid][k + 1], sh[tid + s][k + 1]);
      }
      sh[tid][10] += sh[tid + s][10];
    }
    __syncthreads();
  }
  if (tid < MM) part[((int64_t)b * G + g) * MM + tid] = sh[0][tid];
}

__global__ void minmax_final_kernel(const double* part, double* out, int32_t G) {
  const int b = blockIdx.x, k = threadIdx.x;
  if (k >= MM) return;
  double r = (k < 10) ? ((k & 1) ? -INFINITY : INFINITY) : 0.0;
  for (int g = 0; g < G; ++g) {
    const double v = part[((int64_t)b * G + g) * MM + k];
    if (k < 10) r = (k & 1) ? fmax(r, v) : fmin(r, v);
    else r += v;
  }
  out[b * MM + k] = r;
}

__global__ __launch_bounds__(256) void check_finite_kernel(const int32_t* bid, int64_t n_total,
                                                           const double* const* arrays, int32_t n_arrays,
                                                           int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_total || bid[i] < 0) return;
  bool ok = true;
  for (int k = 0; k < n_arrays; ++k) ok = ok && isfinite(arrays[k][i]);
  if (!ok) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Diagnostics: two passes of per-block FP64 partial sums reduced in a fixed
// order (deterministic), then the derived quantities of the record.
// ---------------------------------------------------------------------------
template <int NQ>
__device__ void block_reduce_store(double (&v)[NQ], double* dst, int first_max, int n_max) {
  // wave-level tree, then across the 4 waves through LDS; fixed pattern.
  __shared__ double sh[WG / 64][D_N1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = 0; k < NQ; ++k) {
    double x = v[k];
    const bool is_max = (k >= first_max && k < first_max + n_max);
    for (int o = 32; o > 0; o >>= 1) {
      const double y = __shfl_down(x, o, 64);
      x = is_max ? fmax(x, y) : x + y;
    }
    if (lane == 0) sh[wv][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    const int k = threadIdx.x;
    const bool is_max = (k >= first_max && k < first_max + n_max);
    double x = sh[0][k];
    for (int w = 1; w < WG / 64; ++w) x = is_max ? fmax(x, sh[w][k]) : x + sh[w][k];
    dst[k] = x;
  }
}

__global__ __launch_bounds__(WG) void diag_pass1_kernel(DiagArgs a) {
  const int b = blockIdx.y, g = blockIdx.x;
  const BunchDev& B = a.bunches[b];
  const double w = a.weight[b];
  double v[D_N1];
  for (int k = 0; k < D_N1; ++k) v[k] = 0.0;
  for (int k = D_XMAX0; k < D_NONFIN; ++k) v[k] = -INFINITY;
  for (int64_t li = (int64_t)g * WG + threadIdx.x; li < B.n; li += (int64_t)a.G * WG) {
    const int64_t i = B.off + li;
    const double r[3] = {a.x[i], a.y[i], a.z[i]};
    const double u[3] = {a.vx[i], a.vy[i], a.vz[i]};
    const double m = a.m[i], q = a.q[i];
    v[D_KIN] += 0.5 * w * m * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    v[D_POT] += 0.5 * w * q * a.phi[i];
    v[D_MSUM] += m;
    bool ok = true;
    for (int c = 0; c < 3; ++c) {
      v[D_P0 + c] += w * m * u[c];
      v[D_MR0 + c] += m * r[c];
      v[D_MV0 + c] += m * u[c];
      v[D_X0 + c] += r[c];
      v[D_V0 + c] += u[c];
      v[D_XX0 + c] += r[c] * r[c];
      v[D_VV0 + c] += u[c] * u[c];
      v[D_XV0 + c] += r[c] * u[c];
      v[D_XMAX0 + c] = fmax(v[D_XMAX0 + c], r[c]);
      v[D_VMAX0 + c] = fmax(v[D_VMAX0 + c], u[c]);
      ok = ok && isfinite(r[c]) && isfinite(u[c]);
    }
    if (!ok) v[D_NONFIN] += 1.0;
  }
  block_reduce_store<D_N1>(v, a.part + ((int64_t)b * a.G + g) * D_N1, D_XMAX0, 6);
}

__global__ void diag_final1_kernel(DiagArgs a) {
  const int b = blockIdx.x, k = threadIdx.x;
  if (k >= D_N1) return;
  const bool is_max = (k >= D_XMAX0 && k < D_XMAX0 + 6);
  double x = is_max ? -INFINITY : 0.0;
  for (int g = 0; g < a.G; ++g) {
    const double y = a.part[((int64_t)b * a.G + g) * D_N1 + k];
    x = is_max ? fmax(x, y) : x + y;
  }
  a.rec[(int64_t)b * D_NREC + k] = x;
}

__global__ __launch_bounds__(WG) void diag_pass2_kernel(DiagArgs a) {
  const int b = blockIdx.y, g = blockIdx.x;
  const BunchDev& B = a.bunches[b];
  const double* rb = a.rec + (int64_t)b * D_NREC;
  const double nn = (double)B.n;
  double mr[3], mv[3];
  for (int c = 0; c < 3; ++c) { mr[c] = rb[D_X0 + c] / nn; mv[c] = rb[D_V0 + c] / nn; }
  double v[D_N2];
  for (int k = 0; k < D_N2; ++k) v[k] = 0.0;
  for (int64_t li = (int64_t)g * WG + threadIdx.x; li < B.n; li += (int64_t)a.G * WG) {
    const int64_t i = B.off + li;
    const double r[3] = {a.x[i] - mr[0], a.y[i] - mr[1], a.z[i] - mr[2]};
    const double u[3] = {a.vx[i] - mv[0], a.vy[i] - mv[1], a.vz[i] - mv[2]};
    for (int c = 0; c < 3; ++c) {
      v[c] += r[c] * r[c];
      v[3 + c] += u[c] * u[c];
      v[6 + c] += r[c] * u[c];
    }
  }
  block_reduce_store<D_N2>(v, a.part + ((int64_t)b * a.G + g) * D_N1, 0, 0);
}

// out layout per bunch (doubles, pp_diag order from `kinetic` on):
// kinetic potential total momentum[3] com[3] com_velocity[3] emittance[3]
// emittance_centered[3] x_rms[3] x_max[3] v_rms[3] v_max[3] nonfinite

__global__ void diag_final2_kernel(DiagArgs a, double* out) {
  const int b = blockIdx.x;
  if (threadIdx.x != 0) return;
  double* rb = a.rec + (int64_t)b * D_NREC;
  for (int k = 0; k < D_N2; ++k) {
    double x = 0.0;
    for (int g = 0; g < a.G; ++g) x += a.part[((int64_t)b * a.G + g) * D_N1 + k];
    rb[D_N1 + k] = x;
  }
  const double nn = (double)a.bunches[b].n;
  double* o = out + (int64_t)b * D_OUT;
  o[0] = rb[D_KIN];
  o[1] = rb[D_POT];
  o[2] = rb[D_KIN] + rb[D_POT];
  for (int c = 0; c < 3; ++c) {
    o[3 + c] = rb[D_P0 + c];
    o[6 + c] = rb[D_MR0 + c] / rb[D_MSUM];
    o[9 + c] = rb[D_MV0 + c] / rb[D_MSUM];
    const double xx = rb[D_XX0 + c] / nn, vv = rb[D_VV0 + c] / nn, xv = rb[D_XV0 + c] / nn;
    const double e2 = xx * vv - xv * xv;
    o[12 + c] = sqrt(e2 > 0.0 ? e2 : 0.0);
    const double cxx = rb[D_CXX0 + c] / nn, cvv = rb[D_CVV0 + c] / nn, cxv = rb[D_CXV0 + c] / nn;
    const double c2 = cxx * cvv - cxv * cxv;
    o[15 + c] = sqrt(c2 > 0.0 ? c2 : 0.0);
    o[18 + c] = sqrt(xx);
    o[21 + c] = rb[D_XMAX0 + c];
    o[24 + c] = sqrt(vv);
    o[27 + c] = rb[D_VMAX0 + c];
  }
  o[D_OUT_VALUES] = rb[D_NONFIN];
}

template <int K, bool UQ, bool PHI>
hipError_t go_pair(const PairArgs& a, bool mixed, int grid, int sum_tile, hipStream_t s) {
  if (mixed) {
    hipLaunchKernelGGL((pair_mixed_kernel<K, UQ, PHI>), dim3(grid), dim3(WG), 0, s, a, sum_tile);
  } else {
    if constexpr (K <= 4) {
      hipLaunchKernelGGL((pair_fp64_kernel<K, UQ, PHI>), dim3(grid), dim3(WG), 0, s, a, sum_tile);
    } else {
      return hipErrorInvalidValue;  // the FP64 path holds at most 4 receivers per lane
    }
  }
  return hipGetLastError();
}

template <int K>
hipError_t go_pair_k(const PairArgs& a, bool mixed, bool uq, bool phi, int grid, int sum_tile, hipStream_t s) {
  if (uq) return phi ? go_pair<K, true, true>(a, mixed, grid, sum_tile, s)
                     : go_pair<K, true, false>(a, mixed, grid, sum_tile, s);
  return phi ? go_pair<K, false, true>(a, mixed, grid, sum_tile, s)
             : go_pair<K, false, false>(a, mixed, grid, sum_tile, s);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int pair_regs_hint(bool mixed, int i_per_lane) { return (mixed ? 16 : 24) * i_per_lane; }

hipError_t launch_pair(const PairArgs& a, bool mixed, int i_per_lane, int sum_tile, bool uniform_q,
                       bool with_phi, int grid, hipStream_t s) {
  switch (i_per_lane) {
    case 1: return go_pair_k<1>(a, mixed, uniform_q, with_phi, grid, sum_tile, s);
    case 2: return go_pair_k<2>(a, mixed, uniform_q, with_phi, grid, sum_tile, s);
    case 4: return go_pair_k<4>(a, mixed, uniform_q, with_phi, grid, sum_tile, s);
    case 8: return go_pair_k<8>(a, mixed, uniform_q, with_phi, grid, sum_tile, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pack(const PackArgs& a, bool drift, bool mixed, hipStream_t s) {
  const unsigned nb = a.n_total > 0 ? blocks_for(a.n_total, 256) : 1;
  if (drift) {
    if (mixed) hipLaunchKernelGGL((pack_kernel<true, true>), dim3(nb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((pack_kernel<true, false>), dim3(nb), dim3(256), 0, s, a);
  } else {
    if (mixed) hipLaunchKernelGGL((pack_kernel<false, true>), dim3(nb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((pack_kernel<false, false>), dim3(nb), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <int L>
hipError_t go_final(const FinalArgs& a, bool mixed, FinalMode mode, hipStream_t s) {
  const unsigned nb = blocks_for(a.n_total * L, 256);
  if (nb == 0) return hipSuccess;
#define PP_FIN(M, MD) hipLaunchKernelGGL((final_kernel<M, MD, L>), dim3(nb), dim3(256), 0, s, a)
  if (mixed) {
    if (mode == FIN_FIELD) PP_FIN(true, FIN_FIELD);
    else if (mode == FIN_ACCEL) PP_FIN(true, FIN_ACCEL);
    else if (mode == FIN_KICK) PP_FIN(true, FIN_KICK);
    else PP_FIN(true, FIN_KICK_DRIFT);
  } else {
    if (mode == FIN_FIELD) PP_FIN(false, FIN_FIELD);
    else if (mode == FIN_ACCEL) PP_FIN(false, FIN_ACCEL);
    else if (mode == FIN_KICK) PP_FIN(false, FIN_KICK);
    else PP_FIN(false, FIN_KICK_DRIFT);
  }
#undef PP_FIN
  return hipGetLastError();
}

hipError_t launch_final(const FinalArgs& a, bool mixed, FinalMode mode, hipStream_t s) {
  if (a.sym) return go_final<1>(a, mixed, mode, s);
  return go_final<FIN_LANES>(a, mixed, mode, s);
}

hipError_t launch_qprep(const BunchDev* bunches, const int32_t* bid, int64_t n_total, const double* q, float* qt,
                        double* qt64, hipStream_t s) {
  const unsigned nb = blocks_for(n_total, 256);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(qprep_kernel, dim3(nb), dim3(256), 0, s, bunches, bid, n_total, q, qt, qt64);
  return hipGetLastError();
}

hipError_t launch_minmax(const BunchDev* bunches, int32_t n_bunches, const double* x, const double* y,
                         const double* z, const double* q, const double* m, double* out, int32_t G,
                         hipStream_t s) {
  // out must hold n_bunches * G * MM doubles of scratch followed by
  // n_bunches * MM results.
  double* part = out + (int64_t)n_bunches * MM;
  hipLaunchKernelGGL(minmax_part_kernel, dim3(G, n_bunches), dim3(256), 0, s, bunches, x, y, z, q, m, part, G);
  hipLaunchKernelGGL(minmax_final_kernel, dim3(n_bunches), dim3(64), 0, s, part, out, G);
  return hipGetLastError();
}

hipError_t launch_check_finite(const int32_t* bid, int64_t n_total, const double* const* arrays,
                               int32_t n_arrays, int32_t* flag, hipStream_t s) {
  const unsigned nb = blocks_for(n_total, 256);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(check_finite_kernel, dim3(nb), dim3(256), 0, s, bid, n_total, arrays, n_arrays, flag);
  return hipGetLastError();
}

hipError_t launch_fill_bid(int32_t* bid, int64_t n_total, const BunchDev* bunches, int32_t n_bunches,
                           hipStream_t s) {
  hipLaunchKernelGGL(fill_bid_kernel, dim3(256, n_bunches), dim3(256), 0, s, bid, n_total, bunches, n_bunches);
  return hipGetLastError();
}

hipError_t launch_diag(const DiagArgs& a, int32_t n_bunches, hipStream_t s) {
  // a.rec holds n_bunches * D_NREC doubles followed by n_bunches * D_OUT output doubles
  double* out = a.rec + (int64_t)n_bunches * D_NREC;
  hipLaunchKernelGGL(diag_pass1_kernel, dim3(a.G, n_bunches), dim3(WG), 0, s, a);
  hipLaunchKernelGGL(diag_final1_kernel, dim3(n_bunches), dim3(64), 0, s, a);
  hipLaunchKernelGGL(diag_pass2_kernel, dim3(a.G, n_bunches), dim3(WG), 0, s, a);
  hipLaunchKernelGGL(diag_final2_kernel, dim3(n_bunches), dim3(64), 0, s, a, out);
  return hipGetLastError();
}

}  // namespace ppk
