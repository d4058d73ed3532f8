// pp_ubench.hip -- vector-ALU issue-rate micro-benchmarks for gfx950 (a
// separate library, libpp_ubench.so, used by `bench.py --mode ubench`; not
// part of the C ABI of include/pp.h).
//
// They measure what the pair kernels' issue model needs: how many FP32 lane
// operations a compute unit completes per shader clock for FMA, add, mul and
// v_rsq_f32 alone, for FMA and rsq streams interleaved (as in a pair
// evaluation), and the same for FP64 FMA, add, mul and v_rsq_f64.  Each thread runs 8 independent dependence
// chains so that issue, not latency, limits the rate; the grid is 8
// workgroups of 256 threads per CU.  Every chain's result is stored, so the
// compiler cannot drop the work.  The shader clock during the kernel is read
// from the kernel itself (the shader-clock counter against the fixed 100 MHz
// counter), so rates per clock do not depend on the clock the chip held.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;
constexpr int kThreads = 256;

enum Op : int32_t {
  OP_FMA = 0, OP_ADD = 1, OP_MUL = 2, OP_RSQ = 3, OP_FMA_RSQ = 4,
  OP_FMA64 = 5, OP_ADD64 = 6, OP_MUL64 = 7, OP_RSQ64 = 8
};

// ops[] holds per-thread inputs; out[] receives the chains' results; clk[2 *
// block] the block's shader-clock and real-time spans (thread 0).
template <int OP>
__global__ __launch_bounds__(kThreads) void valu_kernel(const float* in, float* out, int iters,
                                                        unsigned long long* clk) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  const unsigned long long c0 = clock64(), r0 = wall_clock64();
  if (OP >= OP_FMA64) {
    double a[kChains];
    const double m = 1.0 + 1e-9 * in[t & 1023], c = 1e-7;
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = 1.0 + (double)in[(t + k) & 1023];
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int k = 0; k < kChains; ++k) {
        if (OP == OP_FMA64) a[k] = fma(a[k], m, c);
        if (OP == OP_ADD64) a[k] = a[k] + c;
        if (OP == OP_MUL64) a[k] = a[k] * m;
        if (OP == OP_RSQ64) a[k] = __builtin_amdgcn_rsq(a[k]);
      }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    out[t] = (float)s;
  } else {
    float a[kChains];
    const float m = 1.0f + 1e-6f * in[t & 1023], c = 1e-7f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = 1.0f + in[(t + k) & 1023];
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int k = 0; k < kChains; ++k) {
        if (OP == OP_FMA) a[k] = fmaf(a[k], m, c);
        if (OP == OP_ADD) a[k] = a[k] + c;
        if (OP == OP_MUL) a[k] = a[k] * m;
        if (OP == OP_RSQ) a[k] = __builtin_amdgcn_rsqf(a[k]);
        if (OP == OP_FMA_RSQ) {
          // one rsq feeding and fed by FMAs, 8 FMA per rsq: a pair's mix
          const float r = __builtin_amdgcn_rsqf(fmaf(a[k], a[k], c));
          a[k] = fmaf(fmaf(fmaf(fmaf(fmaf(fmaf(fmaf(r, m, c), m, c), m, c), m, c), m, c), m, c), r, a[k]);
        }
      }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    out[t] = s;
  }
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = clock64() - c0;
    clk[2 * blockIdx.x + 1] = wall_clock64() - r0;
  }
}

}  // namespace

// Runs one micro-benchmark: `blocks` workgroups of 256 threads, `iters`
// iterations of 8 chains, on the legacy default stream; returns the elapsed
// milliseconds (HIP events), the mean per-block shader-clock cycles and
// real-time ticks (100 MHz).  Buffers are the caller's device memory: in (1024
// floats), out (blocks x 256 floats), clk (2 x blocks 64-bit words).
// Returns a hipError_t value (0 on success).
extern "C" int pp_ubench_valu(int op, int blocks, int iters, const float* in, float* out, unsigned long long* clk,
                              double* ms) {
  if (blocks < 1 || iters < 1 || !in || !out || !clk || !ms) return (int)hipErrorInvalidValue;
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return (int)e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return (int)e;
  }
  (void)hipEventRecord(e0, nullptr);
  switch (op) {
    case OP_FMA: hipLaunchKernelGGL(valu_kernel<OP_FMA>, dim3(blocks), dim3(kThreads), 0, nullptr, in, out, iters, clk); break;
    case OP_ADD: hipLaunchKernelGGL(valu_kernel<OP_ADD>, dim3(blocks), dim3(kThreads), 0, nullptr, in, out, iters, clk); break;
    case OP_MUL: hipLaunchKernelGGL(valu_kernel<OP_MUL>, dim3(blocks), dim3(kThreads), 0, nullptr, in, out, iters, clk); break;
    case OP_RSQ: hipLaunchKernelGGL(valu_kernel<OP_RSQ>, dim3(blocks), dim3(kThreads), 0, nullptr, in, out, iters, clk); break;
    case OP_FMA_RSQ:
      hipLaunchKernelGGL(valu_kernel<OP_FMA_RSQ>, dim3(blocks), dim3(kThreads), 0, nullptr, in, out, iters, clk);
      break;
    case OP_FMA64:
      hipLaunchKernelGGL(valu_kernel<OP_FMA64>, dim3(blocks), dim3(kThreads), 0, nullptr, in, out, iters, clk);
      break;
    case OP_ADD64:
      hipLaunchKernelGGL(valu_kernel<OP_ADD64>, dim3(blocks), dim3(kThreads), 0, nullptr, in, out, iters, clk);
      break;
    case OP_MUL64:
      hipLaunchKernelGGL(valu_kernel<OP_MUL64>, dim3(blocks), dim3(kThreads), 0, nullptr, in, out, iters, clk);
      break;
    case OP_RSQ64:
      hipLaunchKernelGGL(valu_kernel<OP_RSQ64>, dim3(blocks), dim3(kThreads), 0, nullptr, in, out, iters, clk);
      break;
    default:
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return (int)hipErrorInvalidValue;
  }
  e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float f = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
  *ms = f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (int)e;
}

// Frequency of the counter behind wall_clock64() [kHz] (device 0 attribute).
extern "C" int pp_ubench_wall_clock_khz(int* khz) {
  if (!khz) return (int)hipErrorInvalidValue;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, dev);
  return (int)e;
}
