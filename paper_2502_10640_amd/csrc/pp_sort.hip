// pp_sort.hip -- spatial ordering for the near/far split of the symmetric
// pair sum.
//
// Every step the particles of each bunch are ordered along a Morton curve of
// their (scaled, FP32 high part) positions, so that a block of consecutive
// particles is compact in space.  Source groups of 64 whose bounding box lies
// farther than D from a wavefront's receiver box can then use plain FP32
// separations (hi_i - hi_j): the rounding of the positions to FP32 moves a
// separation by at most 2^-24 (|a| + |b|) (a, b: the two boxes' per-axis
// largest |coordinate|, both below U, the bunch's bound), so a pair term
// changes by at most 2^-23 (|a| + |b|) / D relative, while closer groups keep
// the hi/lo separations.  This file computes U, the order and the group boxes.
//
// A bunch's Morton code has as many bits per axis as gives it about 8 cells
// per particle (morton_bits_for: ceil(log2 n / 3) + 1, at most 10), and the
// bunch index sits just above the widest code of the context, so the sort
// takes as few 8-bit passes as that allows while a bunch's order depends on
// the bunch alone.
//
// The sort is a stable least-significant-digit radix sort with 8-bit digits:
// tile histograms (order-free LDS counts), a digit-major exclusive scan, and a
// scatter that ranks equal digits with wavefront ballots, so the permutation
// is the same on every run.
#include "pp_device.h"
#include "pp_internal.h"
#include "pp_sort.h"

#include <cmath>

namespace ppk {
namespace {

// ---- per-bunch coordinate bound U (max |hi| over the bunch, any axis) -------
__global__ __launch_bounds__(256) void bound_zero_kernel(uint32_t* ubits, int32_t nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) ubits[b] = 0u;
}

// each thread reduces 8 particles (stride 256 inside the workgroup's 2048),
// flushing when the bunch changes; a wavefront whose lanes end in one bunch
// reduces once more and makes a single atomic
constexpr int BOUND_PER = 8;

__global__ __launch_bounds__(256) void bound_kernel(SortArgs a) {
  const int64_t i0 = (int64_t)blockIdx.x * (256 * BOUND_PER) + threadIdx.x;
  int b = -1;
  float m = 0.f;
  for (int k = 0; k < BOUND_PER; ++k) {
    const int64_t i = i0 + (int64_t)k * 256;
    if (i >= a.n_total) break;
    const int bi = a.bid[i];
    if (bi < 0) continue;
    const float v = fmaxf(fabsf(a.xh[i]), fmaxf(fabsf(a.yh[i]), fabsf(a.zh[i])));
    if (bi != b) {
      // non-negative floats order like their bit patterns
      if (b >= 0) atomicMax(&a.ubits[b], __float_as_uint(m));
      b = bi;
      m = v;
    } else {
      m = fmaxf(m, v);
    }
  }
  const int b0 = __shfl(b, 0);
  if (__all(b == b0)) {
    if (b0 < 0) return;
    for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d));
    if ((threadIdx.x & 63) == 0) atomicMax(&a.ubits[b0], __float_as_uint(m));
  } else if (b >= 0) {
    atomicMax(&a.ubits[b], __float_as_uint(m));
  }
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

// u in [-U, U] to bpa bits (bpa <= 10)
__device__ __forceinline__ uint32_t quant(float u, float inv_u, int bpa) {
  float t = (u * inv_u + 1.0f) * (float)(1 << (bpa - 1));
  t = fminf(fmaxf(t, 0.0f), (float)((1 << bpa) - 1));
  return (uint32_t)t;
}

__global__ __launch_bounds__(256) void key_kernel(SortArgs a, int key_shift) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_total) return;
  const int b = a.bid[i];
  if (b < 0) return;
  const BunchDev& B = a.bunches[b];
  const float U = __uint_as_float(a.ubits[b]);
  const float inv_u = U > 0.f ? 1.0f / U : 0.f;
  const int bpa = morton_bits_for(B.n);  // the bunch's own resolution: same order alone or in a batch
  const uint32_t m = spread3(quant(a.xh[i], inv_u, bpa)) | (spread3(quant(a.yh[i], inv_u, bpa)) << 1) |
                     (spread3(quant(a.zh[i], inv_u, bpa)) << 2);
  const int64_t c = B.cstart + (i - B.off);
  a.keys[c] = ((uint64_t)(uint32_t)b << key_shift) | m;
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

// Exclusive scan of hist (digit-major: hist[d * n_tiles + t]) in two
// launches of one workgroup per digit: digit totals, then each digit's base
// (sum of the totals of smaller digits) plus the scan of its own row.
__global__ __launch_bounds__(256) void digit_total_kernel(const uint32_t* __restrict__ hist, int32_t n_tiles,
                                                          uint32_t* __restrict__ tot) {
  __shared__ uint32_t part[256];
  const int d = blockIdx.x, tid = threadIdx.x;
  uint32_t sum = 0u;
  for (int t = tid; t < n_tiles; t += 256) sum += hist[(int64_t)d * n_tiles + t];
  part[tid] = sum;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) tot[d] = part[0];
}

// inclusive Hillis-Steele scan of v over the 256 threads of the workgroup
__device__ uint32_t block_scan_incl(uint32_t v, uint32_t* buf) {
  const int tid = threadIdx.x;
  buf[tid] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t x = tid >= off ? buf[tid - off] : 0u;
    __syncthreads();
    buf[tid] += x;
    __syncthreads();
  }
  const uint32_t r = buf[tid];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void digit_scan_kernel(uint32_t* __restrict__ hist, int32_t n_tiles,
                                                         const uint32_t* __restrict__ tot) {
  __shared__ uint32_t buf[256];
  const int d = blockIdx.x, tid = threadIdx.x;
  // base of digit d: exclusive prefix of the digit totals
  const uint32_t incl = block_scan_incl(tot[tid], buf);
  __shared__ uint32_t base;
  if (tid == d) base = incl - tot[tid];
  __syncthreads();
  // this digit's row: thread tid scans a contiguous segment
  const int per = (n_tiles + 255) / 256;
  const int t0 = min(n_tiles, tid * per), t1 = min(n_tiles, t0 + per);
  uint32_t* row = hist + (int64_t)d * n_tiles;
  uint32_t seg = 0u;
  for (int t = t0; t < t1; ++t) seg += row[t];
  uint32_t run = base + block_scan_incl(seg, buf) - seg;
  for (int t = t0; t < t1; ++t) {
    const uint32_t v = row[t];
    row[t] = run;
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

// bunch of group g (groups are numbered bunch by bunch)
__device__ __forceinline__ int bunch_of_group(const BunchDev* bunches, int nb, int g) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bunches[mid].gbase <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// one wavefront per group of 64 sorted particles: box of the FP32 high parts
__global__ __launch_bounds__(256) void gbox_kernel(SortArgs a, int32_t n_groups_total) {
  const int g = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int l = threadIdx.x & 63;
  if (g >= n_groups_total) return;  // uniform over the wavefront
  const BunchDev& B = a.bunches[bunch_of_group(a.bunches, a.nb, g)];
  const int64_t li = (int64_t)(g - B.gbase) * 64 + l;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (li < B.n) {
    const int64_t p = B.off + li;
    lo[0] = hi[0] = a.sxh[p];
    lo[1] = hi[1] = a.syh[p];
    lo[2] = hi[2] = a.szh[p];
  }
  for (int d = 32; d >= 1; d >>= 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[c] = fminf(lo[c], __shfl_xor(lo[c], d));
      hi[c] = fmaxf(hi[c], __shfl_xor(hi[c], d));
    }
  }
  float s2 = 0.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float m = fmaxf(fabsf(lo[c]), fabsf(hi[c]));
    s2 = fmaf(m, m, s2);
  }
  const float v = l == 0 ? lo[0] : l == 1 ? lo[1] : l == 2 ? lo[2] : l == 3 ? hi[0] : l == 4 ? hi[1]
                : l == 5 ? hi[2] : l == 6 ? sqrtf(s2) : 0.f;
  if (l < GBOX) a.gbox[(int64_t)g * GBOX + l] = v;
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_sort(const SortArgs& a, int key_bits, int32_t n_groups_total, hipStream_t s) {
  return launch_sort_bits(a, 30, key_bits, n_groups_total, true, s);
}

hipError_t launch_sort_bits(const SortArgs& a, int key_shift, int key_bits, int32_t n_groups_total, bool resort,
                            hipStream_t s) {
  if (key_shift < 3 || key_shift > 30 || key_bits < key_shift || key_bits > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bound_zero_kernel, dim3(nblk(a.nb, 256)), dim3(256), 0, s, a.ubits, a.nb);
  hipLaunchKernelGGL(bound_kernel, dim3(nblk(a.n_total, 256 * BOUND_PER)), dim3(256), 0, s, a);
  const int32_t n_tiles = (int32_t)nblk(a.n_in, TILE);
  uint64_t* kin = a.keys;
  int32_t* vin = a.vals;
  uint64_t* kout = a.keys2;
  int32_t* vout = a.vals2;
  const int passes = (key_bits + 7) / 8;
  if (!resort) {
    // the previous sort left its permutation in the buffer of its last pass
    if (passes % 2 == 1) vin = a.vals2;
  } else {
    hipLaunchKernelGGL(key_kernel, dim3(nblk(a.n_total, 256)), dim3(256), 0, s, a, key_shift);
  }
  for (int p = 0; resort && p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(hist_kernel, dim3(n_tiles), dim3(RT), 0, s, kin, a.n_in, shift, a.hist, n_tiles);
    hipLaunchKernelGGL(digit_total_kernel, dim3(256), dim3(256), 0, s, a.hist, n_tiles, a.dtot);
    hipLaunchKernelGGL(digit_scan_kernel, dim3(256), dim3(256), 0, s, a.hist, n_tiles, a.dtot);
    hipLaunchKernelGGL(scatter_kernel, dim3(n_tiles), dim3(RT), 0, s, kin, vin, kout, vout, a.n_in, shift, a.hist,
                       n_tiles);
    uint64_t* tk = kin; kin = kout; kout = tk;
    int32_t* tv = vin; vin = vout; vout = tv;
  }
  SortArgs g = a;
  g.vals = vin;  // sorted order after an even or odd number of passes
  hipLaunchKernelGGL(gather_kernel, dim3(nblk(a.n_in, 256)), dim3(256), 0, s, g);
  hipLaunchKernelGGL(gbox_kernel, dim3(nblk((int64_t)n_groups_total * 64, 256)), dim3(256), 0, s, g,
                     n_groups_total);
  return hipGetLastError();
}

}  // namespace ppk
