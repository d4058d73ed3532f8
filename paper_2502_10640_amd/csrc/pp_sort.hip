// pp_sort.hip -- spatial ordering for the near/far split of the symmetric
// pair sum.
//
// Every step the particles of each bunch are ordered along a Morton curve of
// their (scaled, FP32 high part) positions, so that a block of consecutive
// particles is compact in space.  Source groups of 64 whose bounding box lies
// farther than D from a receiver block's box can then use plain FP32
// separations (hi_i - hi_j): the rounding of the positions to FP32 changes a
// pair term by at most 2 sqrt(3) 2^-23 U / D relative (U bounds every scaled
// coordinate of the bunch), while closer groups keep the hi/lo separations.
//
// The sort is a stable least-significant-digit radix sort with 8-bit digits:
// tile histograms (order-free LDS counts), a digit-major exclusive scan, and a
// scatter that ranks equal digits with wavefront ballots, so the permutation
// is the same on every run.
#include "pp_device.h"
#include "pp_internal.h"

#include <cmath>

namespace ppk {
namespace {

// ---- per-bunch coordinate bound U (max |hi| over the bunch, any axis) -------
__global__ __launch_bounds__(256) void bound_zero_kernel(uint32_t* ubits, int32_t nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) ubits[b] = 0u;
}

__global__ __launch_bounds__(256) void bound_kernel(SortArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_total) return;
  const int b = a.bid[i];
  if (b < 0) return;
  const float m = fmaxf(fabsf(a.xh[i]), fmaxf(fabsf(a.yh[i]), fabsf(a.zh[i])));
  // non-negative floats order like their bit patterns
  atomicMax(&a.ubits[b], __float_as_uint(m));
}

// ---- keys --------------------------------------------------------------------
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  // 10 bits -> every third bit of 30
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t quant10(float u, float inv_u) {
  float t = (u * inv_u + 1.0f) * 512.0f;
  t = fminf(fmaxf(t, 0.0f), 1023.0f);
  return (uint32_t)t;
}

__global__ __launch_bounds__(256) void key_kernel(SortArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_total) return;
  const int b = a.bid[i];
  if (b < 0) return;
  const BunchDev& B = a.bunches[b];
  const float U = __uint_as_float(a.ubits[b]);
  const float inv_u = U > 0.f ? 1.0f / U : 0.f;
  const uint32_t m = spread3(quant10(a.xh[i], inv_u)) | (spread3(quant10(a.yh[i], inv_u)) << 1) |
                     (spread3(quant10(a.zh[i], inv_u)) << 2);
  const int64_t c = B.cstart + (i - B.off);
  a.keys[c] = ((uint64_t)(uint32_t)b << 30) | m;
  a.vals[c] = (int32_t)i;
}

// ---- radix sort pass ----------------------------------------------------------
constexpr int RT = 256;          // threads per sort workgroup
constexpr int TILE = SORT_TILE;  // elements per tile
static_assert(TILE % RT == 0, "a tile is whole rounds of the workgroup");

__global__ __launch_bounds__(RT) void hist_kernel(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                  uint32_t* __restrict__ hist, int32_t n_tiles) {
  __shared__ uint32_t h[256];
  const int t = blockIdx.x;
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)t * TILE;
  for (int k = 0; k < TILE / RT; ++k) {
    const int64_t e = base + k * RT + threadIdx.x;
    if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * n_tiles + t] = h[threadIdx.x];
}

// exclusive scan of hist (digit-major, length 256 * n_tiles), one workgroup
__global__ __launch_bounds__(1024) void scan_kernel(uint32_t* __restrict__ hist, int64_t len) {
  __shared__ uint32_t part[1024];
  const int tid = threadIdx.x;
  const int64_t per = (len + 1023) / 1024;
  const int64_t s0 = tid * per, s1 = min(len, s0 + per);
  uint32_t sum = 0u;
  for (int64_t e = s0; e < s1; ++e) sum += hist[e];
  part[tid] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 1024 segment sums
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint32_t run = tid > 0 ? part[tid - 1] : 0u;
  for (int64_t e = s0; e < s1; ++e) {
    const uint32_t v = hist[e];
    hist[e] = run;
    run += v;
  }
}

__global__ __launch_bounds__(RT) void scatter_kernel(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                                     uint64_t* __restrict__ kout, int32_t* __restrict__ vout,
                                                     int64_t n, int shift, const uint32_t* __restrict__ offs,
                                                     int32_t n_tiles) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wc[RT / 64][256];
  const int t = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  run[tid] = 0u;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)t * TILE;
  for (int k = 0; k < TILE / RT; ++k) {
    for (int q = tid; q < (RT / 64) * 256; q += RT) (&wc[0][0])[q] = 0u;
    __syncthreads();
    const int64_t e = base + k * RT + tid;
    const bool valid = e < n;
    uint64_t key = 0;
    int32_t val = 0;
    if (valid) { key = kin[e]; val = vin[e]; }
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    uint64_t match = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t bal = __ballot((d >> bit) & 1u);
      match &= ((d >> bit) & 1u) ? bal : ~bal;
    }
    const uint32_t rank_w = (uint32_t)__popcll(match & lt);
    if (valid && rank_w == 0) wc[w][d] = (uint32_t)__popcll(match);
    __syncthreads();
    if (valid) {
      uint32_t pre = run[d];
      for (int ww = 0; ww < w; ++ww) pre += wc[ww][d];
      const uint64_t dst = (uint64_t)offs[(int64_t)d * n_tiles + t] + pre + rank_w;
      kout[dst] = key;
      vout[dst] = val;
    }
    __syncthreads();
    {
      uint32_t add = 0u;
      for (int ww = 0; ww < RT / 64; ++ww) add += wc[ww][tid];
      run[tid] += add;
    }
    __syncthreads();
  }
}

// ---- sorted mirror, rank, boxes ---------------------------------------------
__global__ __launch_bounds__(256) void gather_kernel(SortArgs a) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_in) return;
  const int32_t i = a.vals[c];
  const int b = a.bid[i];
  const BunchDev& B = a.bunches[b];
  const int64_t p = B.off + (c - B.cstart);
  a.rank[i] = (int32_t)p;
  a.sxh[p] = a.xh[i]; a.syh[p] = a.yh[i]; a.szh[p] = a.zh[i];
  a.sxl[p] = a.xl[i]; a.syl[p] = a.yl[i]; a.szl[p] = a.zl[i];
  a.sqt[p] = a.qt[i];
}

// one thread per group of 64 sorted particles: box of the FP32 high parts
__global__ __launch_bounds__(256) void gbox_kernel(SortArgs a, int32_t n_groups_total) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups_total) return;
  // find the bunch: groups are numbered bunch by bunch
  int b = 0;
  while (b + 1 < a.nb && a.bunches[b + 1].gbase <= g) ++b;
  const BunchDev& B = a.bunches[b];
  const int64_t l0 = (int64_t)(g - B.gbase) * 64;
  const int64_t l1 = min(B.n, l0 + 64);
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t l = l0; l < l1; ++l) {
    const int64_t p = B.off + l;
    const float v[3] = {a.sxh[p], a.syh[p], a.szh[p]};
    for (int c = 0; c < 3; ++c) { lo[c] = fminf(lo[c], v[c]); hi[c] = fmaxf(hi[c], v[c]); }
  }
  for (int c = 0; c < 3; ++c) { a.gbox[(int64_t)g * 6 + c] = lo[c]; a.gbox[(int64_t)g * 6 + 3 + c] = hi[c]; }
}

// one thread per symmetric block: union of its groups' boxes
__global__ __launch_bounds__(256) void bbox_kernel(SortArgs a, int32_t n_blocks_total, int32_t groups_per_block) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_blocks_total) return;
  int b = 0;
  while (b + 1 < a.nb && a.bunches[b + 1].bbase <= q) ++b;
  const BunchDev& B = a.bunches[b];
  const int ng = (int)((B.n + 63) / 64);
  const int g0 = (q - B.bbase) * groups_per_block;
  const int g1 = min(ng, g0 + groups_per_block);
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int g = g0; g < g1; ++g) {
    const float* bx = a.gbox + (int64_t)(B.gbase + g) * 6;
    for (int c = 0; c < 3; ++c) { lo[c] = fminf(lo[c], bx[c]); hi[c] = fmaxf(hi[c], bx[3 + c]); }
  }
  for (int c = 0; c < 3; ++c) { a.bbox[(int64_t)q * 6 + c] = lo[c]; a.bbox[(int64_t)q * 6 + 3 + c] = hi[c]; }
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_sort(const SortArgs& a, int key_bits, int32_t n_groups_total, int32_t n_blocks_total,
                       int32_t groups_per_block, hipStream_t s) {
  hipLaunchKernelGGL(bound_zero_kernel, dim3(nblk(a.nb, 256)), dim3(256), 0, s, a.ubits, a.nb);
  hipLaunchKernelGGL(bound_kernel, dim3(nblk(a.n_total, 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(key_kernel, dim3(nblk(a.n_total, 256)), dim3(256), 0, s, a);
  const int32_t n_tiles = (int32_t)nblk(a.n_in, TILE);
  uint64_t* kin = a.keys;
  int32_t* vin = a.vals;
  uint64_t* kout = a.keys2;
  int32_t* vout = a.vals2;
  const int passes = (key_bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(hist_kernel, dim3(n_tiles), dim3(RT), 0, s, kin, a.n_in, shift, a.hist, n_tiles);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, a.hist, (int64_t)256 * n_tiles);
    hipLaunchKernelGGL(scatter_kernel, dim3(n_tiles), dim3(RT), 0, s, kin, vin, kout, vout, a.n_in, shift, a.hist,
                       n_tiles);
    uint64_t* tk = kin; kin = kout; kout = tk;
    int32_t* tv = vin; vin = vout; vout = tv;
  }
  SortArgs g = a;
  g.vals = vin;  // sorted order after an even or odd number of passes
  hipLaunchKernelGGL(gather_kernel, dim3(nblk(a.n_in, 256)), dim3(256), 0, s, g);
  hipLaunchKernelGGL(gbox_kernel, dim3(nblk(n_groups_total, 256)), dim3(256), 0, s, g, n_groups_total);
  hipLaunchKernelGGL(bbox_kernel, dim3(nblk(n_blocks_total, 256)), dim3(256), 0, s, g, n_blocks_total,
                     groups_per_block);
  return hipGetLastError();
}

}  // namespace ppk
