// pp_noalloc.hip -- the field of one bunch without a context and without any
// device allocation (pp_field_noalloc in include/pp.h).
//
// The same kernels as a context's ordered-pair path (source mirror pack,
// charge normalisation, pair sum over a work list of receiver blocks and
// source chunks, FP64 combine of the chunk partials), with every buffer they
// need -- the bunch's constants, the work list, the source mirror and the
// partial sums -- carved out of one file-scope device array.  The set-up
// reduction (extents and charge range) and the bunch's constants are
// computed on the device by one small kernel with the arithmetic a context
// uses (ppk::frame_from_extents, ppk::ordered_chunking), so the result equals
// pp_field's for a context with the same ordered tiling, bit for bit.  No
// value travels through the host: the entry point only enqueues kernels and
// may be captured in a hipGraph.
#include "pp.h"
#include "pp_internal.h"

#include <mutex>
#include <string>

// Scratch of the allocation-free path: one copy per device, held until the
// process ends.  In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress (scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[(size_t)PP_NOALLOC_SCRATCH_MIB << 20];

namespace {

constexpr size_t kScratchBytes = (size_t)PP_NOALLOC_SCRATCH_MIB << 20;

// Tiling of the allocation-free path: the ordered-pair kernel, one receiver
// per lane, the default sum tile and chunking of a context.
constexpr int kK = 1;
constexpr int kSumTile = 64;
constexpr int kChunkPairsLog2 = 22;
constexpr int kGridPerCu = 4;
constexpr int kInitThreads = 1024;

// Errors of this path are reported through pp_last_error(NULL).
pp_status fail(pp_status s, const std::string& msg) {
  ppk::set_thread_error(msg);
  return s;
}

struct DeviceScratch {
  void* ptr = nullptr;
  int cus = 0;
  bool ready = false;
};
constexpr int kMaxDevices = 64;
DeviceScratch g_dev[kMaxDevices];
std::mutex g_mutex;

// Device address of this device's scratch and its CU count, looked up once
// per device with that device current.
pp_status scratch_ptr(int dev, void** out, int* cus) {
  std::lock_guard<std::mutex> lock(g_mutex);
  DeviceScratch& d = g_dev[dev];
  if (!d.ready) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PP_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    int n = 0;
    e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return fail(PP_ERR_DEVICE, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(e));
    d.ptr = p;
    d.cus = n > 0 ? n : 1;
    d.ready = true;
  }
  *out = d.ptr;
  *cus = d.cus;
  return PP_OK;
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

struct InitArgs {
  ppk::BunchDev* bunch;
  int32_t* counter;
  int32_t* bid;
  ppk::WorkItem* items;
  const double *x, *y, *z, *q;
  int64_t n;
  double weight, softening, kc;
  int32_t mixed;
  int32_t n_chunks;
  int64_t chunk_len;
  int32_t n_ib;             // receiver blocks of kK x WG
};

// One workgroup: the set-up reduction over the bunch (min and max of x, y, z
// and q; fmin/fmax, so the order does not matter), the bunch's constants, the
// bunch id of every particle and the work list.  Everything the later kernels
// read is rewritten here on every call.
__global__ __launch_bounds__(kInitThreads) void noalloc_init_kernel(InitArgs a) {
  __shared__ double sh[kInitThreads / 64][8];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double r[8];
  for (int k = 0; k < 8; k += 2) { r[k] = INFINITY; r[k + 1] = -INFINITY; }
  for (int64_t i = t; i < a.n; i += kInitThreads) {
    const double v[4] = {a.x[i], a.y[i], a.z[i], a.q[i]};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      r[2 * k] = fmin(r[2 * k], v[k]);
      r[2 * k + 1] = fmax(r[2 * k + 1], v[k]);
    }
    a.bid[i] = 0;
  }
  const int64_t n_items = (int64_t)a.n_ib * a.n_chunks;
  for (int64_t k = t; k < n_items; k += kInitThreads) {
    const int32_t ib = (int32_t)(k / a.n_chunks), ch = (int32_t)(k % a.n_chunks);
    a.items[k] = ppk::WorkItem{0, ch, ib * kK * ppk::WG, 0};
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    double v = r[k];
    for (int o = 32; o > 0; o >>= 1) {
      const double u = __shfl_down(v, o, 64);
      v = (k & 1) ? fmax(v, u) : fmin(v, u);
    }
    if (lane == 0) sh[w][k] = v;
  }
  __syncthreads();
  if (t != 0) return;
  double ext[ppk::MM_LEN] = {};
  for (int k = 0; k < 8; ++k) {
    double v = sh[0][k];
    for (int ww = 1; ww < kInitThreads / 64; ++ww) v = (k & 1) ? fmax(v, sh[ww][k]) : fmin(v, sh[ww][k]);
    ext[k] = v;  // x, y, z, then q at MM_Q
  }
  ppk::BunchDev B{};
  B.off = 0;
  B.n = a.n;
  B.dt = 1.0;
  ppk::frame_from_extents(ext, a.weight, a.softening, a.kc, a.mixed != 0, true, B);
  B.n_chunks = a.n_chunks;
  B.chunk_len = a.chunk_len;
  B.pbase = 0;
  *a.bunch = B;
  *a.counter = 0;
}

}  // namespace

extern "C" pp_status pp_field_noalloc(int64_t n, const double* x, const double* y, const double* z, const double* q,
                                      double weight, double softening, pp_precision prec, double* ex, double* ey,
                                      double* ez, double* phi, void* hip_stream) {
  ppk::set_thread_error("");
  if (!x || !y || !z || !q || !ex || !ey || !ez) return fail(PP_ERR_INVALID_ARG, "a required pointer is NULL");
  if (prec != PP_FP64 && prec != PP_MIXED) return fail(PP_ERR_INVALID_ARG, "unknown precision");
  if (n < 1 || n > PP_NOALLOC_MAX_N)
    return fail(PP_ERR_INVALID_ARG, "n must be in 1.." + std::to_string(PP_NOALLOC_MAX_N) +
                                        " for the allocation-free path (got " + std::to_string(n) + ")");
  if (!(weight > 0.0) || !std::isfinite(weight) || !(softening >= 0.0) || !std::isfinite(softening))
    return fail(PP_ERR_INVALID_ARG, "need weight > 0 and softening >= 0, both finite");
  const bool mixed = prec == PP_MIXED;
  hipStream_t s = (hipStream_t)hip_stream;

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(PP_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(PP_ERR_DEVICE, "device index beyond the supported 64");
  void* base = nullptr;
  int cus = 0;
  pp_status st = scratch_ptr(dev, &base, &cus);
  if (st != PP_OK) return st;

  // layout of the scratch for this call (every part 256-byte aligned)
  const ppk::Chunking ch = ppk::ordered_chunking(n, kK, kChunkPairsLog2, kGridPerCu, cus);
  const int64_t BI = (int64_t)kK * ppk::WG;
  const int64_t n_ib = (n + BI - 1) / BI;
  const int64_t n_items = n_ib * ch.n_chunks;
  const size_t esz = mixed ? sizeof(float) : sizeof(double);
  const int64_t P = ch.n_chunks * n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += up256(bytes);
    return (unsigned char*)base + at;
  };
  auto* bunch = (ppk::BunchDev*)take(sizeof(ppk::BunchDev));
  auto* counter = (int32_t*)take(4 * sizeof(int32_t));
  auto* bid = (int32_t*)take((size_t)n * sizeof(int32_t));
  auto* items = (ppk::WorkItem*)take((size_t)n_items * sizeof(ppk::WorkItem));
  float* mir = mixed ? (float*)take(7 * (size_t)n * sizeof(float)) : nullptr;
  double* qt64 = mixed ? nullptr : (double*)take((size_t)n * sizeof(double));
  void* part = take((size_t)ppk::N_PLANES * (size_t)P * esz);
  if (off > kScratchBytes)
    return fail(PP_ERR_INVALID_ARG, "the allocation-free path needs " + std::to_string(off) + " bytes of scratch for n = " +
                                        std::to_string(n) + " on this device; it has " + std::to_string(kScratchBytes));
  // host-side shape checks of what the kernels assume
  if (n_items > 65536 || ch.n_chunks < 1 || ch.chunk_len < 1)
    return fail(PP_ERR_INVALID_ARG, "work list outside the one-workgroup-per-item range");

  InitArgs ia{};
  ia.bunch = bunch;
  ia.counter = counter;
  ia.bid = bid;
  ia.items = items;
  ia.x = x; ia.y = y; ia.z = z; ia.q = q;
  ia.n = n;
  ia.weight = weight;
  ia.softening = softening;
  ia.kc = ppk::coulomb_k();
  ia.mixed = mixed ? 1 : 0;
  ia.n_chunks = (int32_t)ch.n_chunks;
  ia.chunk_len = ch.chunk_len;
  ia.n_ib = (int32_t)n_ib;
  hipLaunchKernelGGL(noalloc_init_kernel, dim3(1), dim3(kInitThreads), 0, s, ia);
  if ((e = hipGetLastError()) != hipSuccess)
    return fail(PP_ERR_DEVICE, std::string("set-up kernel: ") + hipGetErrorString(e));

  auto plane = [&](int k) { return mir + (size_t)k * (size_t)n; };
  ppk::PackArgs pa{};
  pa.bunches = bunch;
  pa.bid = bid;
  pa.n_total = n;
  // read only: the pack without drift does not write positions
  pa.x = const_cast<double*>(x); pa.y = const_cast<double*>(y); pa.z = const_cast<double*>(z);
  if (mixed) {
    pa.xh = plane(0); pa.yh = plane(1); pa.zh = plane(2);
    pa.xl = plane(3); pa.yl = plane(4); pa.zl = plane(5);
  }
  pa.counter = counter;
  if ((e = ppk::launch_pack(pa, false, mixed, s)) != hipSuccess)
    return fail(PP_ERR_DEVICE, std::string("pack: ") + hipGetErrorString(e));
  if ((e = ppk::launch_qprep(bunch, bid, n, q, mixed ? plane(6) : nullptr, qt64, s)) != hipSuccess)
    return fail(PP_ERR_DEVICE, std::string("charge normalisation: ") + hipGetErrorString(e));

  ppk::PairArgs pr{};
  pr.bunches = bunch;
  pr.items = items;
  pr.n_items = (int32_t)n_items;
  pr.counter = counter;
  pr.direct = 1;
  if (mixed) {
    pr.xh = plane(0); pr.yh = plane(1); pr.zh = plane(2);
    pr.xl = plane(3); pr.yl = plane(4); pr.zl = plane(5);
    pr.qt = plane(6);
    pr.pf = (float*)part;
  } else {
    pr.x = x; pr.y = y; pr.z = z;
    pr.qt64 = qt64;
    pr.pd = (double*)part;
  }
  pr.P = P;
  // the charges are not inspected on the host: the per-source charge path,
  // which gives the uniform path's bits when every charge is the same
  if ((e = ppk::launch_pair(pr, mixed, kK, kSumTile, false, phi != nullptr, (int)n_items, s)) != hipSuccess)
    return fail(PP_ERR_DEVICE, std::string("pair sum: ") + hipGetErrorString(e));

  ppk::FinalArgs fa{};
  fa.bunches = bunch;
  fa.bid = bid;
  fa.n_total = n;
  fa.pf = mixed ? (const float*)part : nullptr;
  fa.pd = mixed ? nullptr : (const double*)part;
  fa.P = P;
  fa.sym = 0;
  fa.ex = ex; fa.ey = ey; fa.ez = ez; fa.phi = phi;
  if ((e = ppk::launch_final(fa, mixed, ppk::FIN_FIELD, s)) != hipSuccess)
    return fail(PP_ERR_DEVICE, std::string("combine: ") + hipGetErrorString(e));
  return PP_OK;
}
