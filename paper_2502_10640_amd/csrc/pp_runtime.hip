// pp_runtime.hip -- host runtime behind the C ABI of include/pp.h.
//
// Owns the context: argument validation, device scratch, the per-bunch
// constants, the work list of the ordered-pair kernel and the round/band
// schedule of the symmetric one, the step sequence (drift+pack -> pair sum ->
// combine+kick, the kick fused with the next drift inside a run), hipGraph
// replay of the step loop, diagnostics, kernel timing, the default tiling and
// the autotuner.
#include "pp.h"
#include "pp_internal.h"
#include "pp_sym64.h"
#include "pp_sort.h"

#include <sys/stat.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <new>
#include <queue>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

using ppk::BunchDev;
using ppk::WorkItem;

namespace {

const double kCoulomb = ppk::coulomb_k();

thread_local std::string g_create_error;

// Device bytes held by every context of the process (pp_device_bytes).
std::atomic<int64_t> g_live_bytes{0};

// Test hook: PP_FAULT_INJECT = "alloc:N" or "launch:N" (N >= 1, default 1),
// read by pp_create, makes the N-th device allocation or kernel launch of that
// context fail without calling HIP, as an out-of-memory or a launch failure.
enum class Fault : int32_t { kNone = 0, kAlloc = 1, kLaunch = 2 };

struct Graph {
  hipGraphExec_t exec = nullptr;
  int64_t steps = 0;
  int64_t phase = 0;        // step index modulo kResortEvery at capture
  int64_t perm_offset = 0;  // step of the last sort inside the graph, relative to its first step - 1
};

// The far split's Morton order is recomputed at evaluations whose step index is
// a multiple of kResortEvery and reused in between (the bound, the sorted
// mirror, the rank and the group boxes are still computed every evaluation
// from the current positions, so the far test is always exact).
constexpr int64_t kResortEvery = 8;

}  // namespace

struct pp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // capture-only stream
  pp_precision prec = PP_MIXED;
  int32_t nb = 0;
  int64_t n_total = 0;
  int cus = 256;
  std::vector<pp_bunch> hb;
  std::vector<BunchDev> hbd;
  pp_state st{};
  bool uniform_q = true;
  double pairs = 0.0;  // ordered pairs per evaluation

  BunchDev* dbunch = nullptr;
  int32_t* bid = nullptr;
  double *ax = nullptr, *ay = nullptr, *az = nullptr;
  float* mir = nullptr;  // 7 planes: xh yh zh xl yl zl qt
  double* qt64 = nullptr;
  void* part = nullptr;
  size_t part_bytes = 0;
  int64_t P = 0;
  WorkItem* items = nullptr;
  size_t items_cap = 0;
  int32_t n_items = 0;
  int32_t* counter = nullptr;  // [0] work counter, [1] finite flag
  double* phi = nullptr;       // diagnostics potential
  double* dweight = nullptr;   // per-bunch weight
  double* diag_buf = nullptr;
  size_t diag_doubles = 0;
  double** arrptr = nullptr;   // device table of state pointers for the finite check
  double *cmp_buf = nullptr;   // autotune comparison buffers (lazy)
  ppk::SymItem* sitems = nullptr;  // symmetric schedule, round by round
  size_t sitems_cap = 0;
  struct Band { int32_t first, count, r0, r1; };
  std::vector<Band> bands;         // one item launch + one fold per band of rounds
  void* acc = nullptr;             // symmetric accumulators, SYM_PLANES x n_total (FP32 or FP64)
  void* slot = nullptr;            // per-item partial slots of one band (FP32 or FP64)
  size_t slot_bytes = 0;
  // spatial sort of the near/far split (allocated on first use)
  float* smir = nullptr;           // 7 planes in sorted order
  uint64_t* keys = nullptr;        // 2 x n_in (ping-pong)
  int32_t* vals = nullptr;         // 2 x n_in
  uint32_t* hist = nullptr;        // 256 x (sort tiles + 1): histograms, then digit totals
  int32_t* rank = nullptr;         // sorted slot of each particle
  uint32_t* ubits = nullptr;       // per-bunch coordinate bound
  float* gbox = nullptr;           // GBOX x 64-particle groups
  int64_t n_in = 0;                // particles inside bunches
  int32_t n_groups = 0, n_blocks = 0;
  // fused small-bunch schedule: work list, the second source buffer (mixed:
  // 6 mirror planes; FP64: 2 x 3 planes of positions) and which buffer holds
  // the positions the next evaluation reads
  ppk::FusedItem* fitems = nullptr;
  size_t fitems_cap = 0;
  int32_t n_fitems = 0;
  float* mir2 = nullptr;
  double* src64 = nullptr;
  int cur = 0;
  void* hpin = nullptr;        // pinned host staging for every host<->device copy
  size_t hpin_bytes = 0;

  pp_tuning tun{};
  bool tuned = false;
  bool a_valid = false;
  int64_t step = 0;
  Graph graph;

  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used;
  int64_t prof_evals = 0;

  std::string err;
  bool broken = false;

  std::unordered_map<void*, size_t> live;  // device allocations of this context and their sizes
  int64_t live_bytes = 0;
  Fault fault = Fault::kNone;              // injected fault (test hook) and the calls left before it
  int64_t fault_left = 0;
  double* mmbuf = nullptr;                 // set-up reductions (extents, charge range, mass check)

  float* xh() const { return mir; }
  float* plane(int k) const { return mir + (size_t)k * (size_t)n_total; }
  bool mixed() const { return prec == PP_MIXED; }
  bool sym() const { return tun.symmetric != 0; }
  bool far() const { return mixed() && sym() && tun.far_split > 0; }
  bool fused() const { return tun.fused != 0; }
  size_t acc_elem() const { return mixed() ? sizeof(float) : sizeof(double); }
  int key_shift = 30, key_bits = 30;  // sort key layout of the far split (set_sort_bits)
  int64_t perm_k = -1;  // step index of the evaluation whose positions the current order sorts (-1: none)
  int k_eff() const { return mixed() ? tun.i_per_lane : std::min(tun.i_per_lane, 4); }
  // particles per block of the symmetric schedule
  int64_t sym_block() const { return (int64_t)(mixed() ? ppk::SYM_WG : ppk::SYM64_WG) * tun.i_per_lane; }
};

namespace {

pp_status set_err(pp_ctx* c, pp_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return s;
}

pp_status dev_fail(pp_ctx* c, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  pp_status s = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? PP_ERR_OUT_OF_MEMORY : PP_ERR_DEVICE;
  if (c) c->broken = true;
  return set_err(c, s, msg);
}

#define PP_HIP(c, call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return dev_fail((c), e_, #call); \
  } while (0)

// True when the injected fault of kind k fires now (once).
bool fault_fires(pp_ctx* c, Fault k) {
  if (c->fault != k) return false;
  if (--c->fault_left > 0) return false;
  c->fault = Fault::kNone;
  return true;
}

void read_fault_hook(pp_ctx* c) {
  const char* e = std::getenv("PP_FAULT_INJECT");
  if (!e || !*e) return;
  const std::string v(e);
  const size_t colon = v.find(':');
  const std::string kind = v.substr(0, colon);
  long long n = 1;
  if (colon != std::string::npos) n = std::atoll(v.c_str() + colon + 1);
  if (n < 1) return;
  if (kind == "alloc") c->fault = Fault::kAlloc;
  else if (kind == "launch") c->fault = Fault::kLaunch;
  else return;
  c->fault_left = n;
}

// Every device allocation of a context: recorded (pp_device_bytes) and freed
// through dfree.
hipError_t dalloc_bytes(pp_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  if (fault_fires(c, Fault::kAlloc)) return hipErrorOutOfMemory;
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  c->live[*p] = bytes;
  c->live_bytes += (int64_t)bytes;
  g_live_bytes += (int64_t)bytes;
  return hipSuccess;
}

template <class T>
hipError_t dalloc(pp_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  const hipError_t e = dalloc_bytes(c, &q, std::max<size_t>(count, 1) * sizeof(T));
  *p = (T*)q;
  return e;
}

hipError_t dfree(pp_ctx* c, void* p) {
  if (!p) return hipSuccess;
  const auto it = c->live.find(p);
  if (it != c->live.end()) {
    c->live_bytes -= (int64_t)it->second;
    g_live_bytes -= (int64_t)it->second;
    c->live.erase(it);
  }
  return hipFree(p);
}

// Every kernel launch of a context passes this gate first.
hipError_t launch_gate(pp_ctx* c) { return fault_fires(c, Fault::kLaunch) ? hipErrorLaunchFailure : hipSuccess; }

#define PP_LAUNCH(c, call)          \
  do {                              \
    PP_HIP((c), launch_gate(c));    \
    PP_HIP((c), (call));            \
  } while (0)

// Frees a context-owned device buffer before it is reallocated (callers have
// synchronised the stream, so nothing of it is in flight); a failure is a
// device error of the context.
template <typename T>
pp_status release(pp_ctx* c, T*& p) {
  if (!p) return PP_OK;
  void* q = p;
  p = nullptr;
  PP_HIP(c, dfree(c, q));
  return PP_OK;
}

pp_status usable(pp_ctx* c) {
  if (!c) return set_err(nullptr, PP_ERR_INVALID_ARG, "null context");
  if (c->broken) return set_err(c, PP_ERR_STATE, "context is broken by an earlier device failure: " + c->err);
  return PP_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Host <-> device copies go through a pinned staging buffer owned by the
// context, enqueued on the context stream and waited for before returning:
// no asynchronous copy ever touches pageable memory.
pp_status ensure_pin(pp_ctx* c, size_t bytes) {
  if (bytes <= c->hpin_bytes) return PP_OK;
  if (c->hpin) {
    void* q = c->hpin;
    c->hpin = nullptr;
    c->hpin_bytes = 0;
    PP_HIP(c, hipHostFree(q));
  }
  c->hpin_bytes = 0;
  size_t want = std::max<size_t>(bytes, 1 << 16);
  PP_HIP(c, hipHostMalloc(&c->hpin, want, hipHostMallocDefault));
  c->hpin_bytes = want;
  return PP_OK;
}

pp_status h2d(pp_ctx* c, void* dst, const void* src, size_t bytes) {
  pp_status s;
  if (bytes == 0) return PP_OK;
  if ((s = ensure_pin(c, bytes)) != PP_OK) return s;
  std::memcpy(c->hpin, src, bytes);
  PP_HIP(c, hipMemcpyAsync(dst, c->hpin, bytes, hipMemcpyHostToDevice, c->stream));
  PP_HIP(c, hipStreamSynchronize(c->stream));
  return PP_OK;
}

pp_status d2h(pp_ctx* c, void* dst, const void* src, size_t bytes) {
  pp_status s;
  if (bytes == 0) return PP_OK;
  if ((s = ensure_pin(c, bytes)) != PP_OK) return s;
  PP_HIP(c, hipMemcpyAsync(c->hpin, src, bytes, hipMemcpyDeviceToHost, c->stream));
  PP_HIP(c, hipStreamSynchronize(c->stream));
  std::memcpy(dst, c->hpin, bytes);
  return PP_OK;
}

// ---------------------------------------------------------------------------
// Symmetric schedule.  Blocks of sym_block() particles per bunch; round
// 0 holds every diagonal item, round d >= 1 the block pairs (I, I + d mod nb)
// (for even nb and d = nb/2 only I < nb/2), so each unordered block pair occurs
// exactly once and a round gives every block at most one partial per side.
// Rounds are grouped into bands whose partial slots fit in kSlotBytes; a band
// is one launch of all its items followed by one fold.
// ---------------------------------------------------------------------------
constexpr size_t kSlotBytes = size_t(12) << 30;

// Sort key layout of the far split: each bunch's Morton code is as fine as its
// own size asks (morton_bits_for), the bunch index sits above the widest code.
void set_sort_bits(pp_ctx* c) {
  int bpa = 1;
  for (const auto& b : c->hb) bpa = std::max(bpa, ppk::morton_bits_for(b.n));
  int bunch_bits = 0;
  while ((int64_t(1) << bunch_bits) < c->nb) ++bunch_bits;
  c->key_shift = 3 * bpa;
  c->key_bits = c->key_shift + bunch_bits;
}

pp_status build_sym(pp_ctx* c) {
  pp_status st;
  set_sort_bits(c);
  const int64_t BS = c->sym_block();
  const int64_t S = c->tun.sym_split;
  const int M = c->tun.sym_rounds;
  // Sub-round d * S + h holds part h of every block pair of round d (round 0:
  // the diagonal blocks).  An item of a bunch with M_b = sym_rounds_for(...)
  // rounds per item sweeps rounds d .. d + nr - 1 (a group starting at round
  // 1, 1 + M_b, ...) and is listed at the sub-round of its first round;
  // round_first[v] is the first item listed at sub-round v.
  std::vector<ppk::SymItem> items;
  std::vector<int64_t> round_first;
  int64_t maxr = 0;
  int Mmax = 1;
  for (int b = 0; b < c->nb; ++b) {
    const int64_t nbk = (c->hb[b].n + BS - 1) / BS;
    if (nbk > INT32_MAX / 8) return set_err(c, PP_ERR_INVALID_ARG, "symmetric schedule: too many blocks");
    maxr = std::max(maxr, nbk / 2);
    Mmax = std::max(Mmax, ppk::sym_rounds_for(nbk, M));
  }
  for (int64_t d = 0; d <= maxr; ++d) {
    for (int64_t h = 0; h < S; ++h) {
      round_first.push_back((int64_t)items.size());
      const int32_t v = (int32_t)(d * S + h);
      for (int b = 0; b < c->nb; ++b) {
        const int64_t nbk = (c->hb[b].n + BS - 1) / BS;
        if (d > nbk / 2) continue;
        if (d == 0) {
          for (int64_t I = 0; I < nbk; ++I) items.push_back({b, (int32_t)I, (int32_t)I, v, 1});
          continue;
        }
        const int Mb = ppk::sym_rounds_for(nbk, M);
        if ((d - 1) % Mb != 0) continue;  // not the first round of a group
        for (int64_t I = 0; I < nbk; ++I) {
          const int nr = ppk::sym_group_rounds(nbk, Mb, d, I);
          if (nr > 0) items.push_back({b, (int32_t)I, (int32_t)((I + d) % nbk), v, nr});
        }
      }
    }
  }
  round_first.push_back((int64_t)items.size());
  if (items.size() > (size_t)INT32_MAX) return set_err(c, PP_ERR_INVALID_ARG, "symmetric schedule too long");
  const int64_t rounds = (maxr + 1) * S;
  const size_t per_round = (size_t)c->n_blocks * 2 * ppk::SLOT_PLANES * (size_t)BS * c->acc_elem();
  // Bands hold whole units of rounds (round 0, then groups of Mmax rounds, so
  // that no item's rounds fall in two bands): the fewest bands whose slots
  // fit, with the units shared out evenly (no short last band leaving the
  // GPU half idle).
  std::vector<int64_t> ub{0};
  for (int64_t d = 0; d <= maxr; d = (d == 0 ? 1 : d + Mmax)) ub.push_back(std::min(rounds, (d == 0 ? 1 : d + Mmax) * S));
  const int64_t n_units = (int64_t)ub.size() - 1;
  const int64_t cap = std::max<int64_t>(1, (int64_t)(kSlotBytes / per_round));
  int64_t per_band = n_units, band = 0;
  for (int64_t nbands = 1; nbands <= n_units; ++nbands) {
    per_band = (n_units + nbands - 1) / nbands;
    band = 0;
    for (int64_t u = 0; u < n_units; u += per_band) band = std::max(band, ub[std::min(n_units, u + per_band)] - ub[u]);
    if (band <= cap || per_band == 1) break;
  }
  c->bands.clear();
  for (int64_t u = 0; u < n_units; u += per_band) {
    const int64_t r0 = ub[u], r1 = ub[std::min(n_units, u + per_band)];
    c->bands.push_back({(int32_t)round_first[r0], (int32_t)(round_first[r1] - round_first[r0]), (int32_t)r0,
                        (int32_t)r1});
  }
  // Launch order inside the first band: the diagonal items (about 0.6 of an
  // off-diagonal item's time) go last, so the cheapest items fill the tail of
  // the launch (longest-first list scheduling).  Items are independent and the
  // fold adds slots in sub-round order, so the order changes no result.
  {
    const int64_t r1 = c->bands.front().r1;
    std::rotate(items.begin() + round_first[0], items.begin() + round_first[std::min(S, r1)],
                items.begin() + round_first[r1]);
  }
  const size_t slot_need = (size_t)band * per_round;
  if (slot_need > c->slot_bytes) {
    c->slot_bytes = 0;
    if ((st = release(c, c->slot)) != PP_OK) return st;
    PP_HIP(c, dalloc_bytes(c, &c->slot, slot_need));
    c->slot_bytes = slot_need;
  }
  if (items.size() > c->sitems_cap) {
    c->sitems_cap = 0;
    if ((st = release(c, c->sitems)) != PP_OK) return st;
    PP_HIP(c, dalloc(c, &c->sitems, items.size()));
    c->sitems_cap = items.size();
  }
  if (!c->acc) PP_HIP(c, dalloc_bytes(c, &c->acc, (size_t)ppk::SYM_PLANES * (size_t)c->n_total * c->acc_elem()));
  if (c->far() && !c->smir) {
    // host-side shape checks of what the sort kernels assume
    if (c->n_total > INT32_MAX) return set_err(c, PP_ERR_INVALID_ARG, "far split: more than 2^31 - 1 particles");
    const size_t n = (size_t)c->n_total, nin = (size_t)c->n_in;
    const size_t tiles = (nin + ppk::SORT_TILE - 1) / ppk::SORT_TILE;
    PP_HIP(c, dalloc(c, &c->smir, 7 * n));
    PP_HIP(c, dalloc(c, &c->keys, 2 * nin));
    PP_HIP(c, dalloc(c, &c->vals, 2 * nin));
    PP_HIP(c, dalloc(c, &c->hist, 256 * (tiles + 1)));  // + 256 digit totals
    PP_HIP(c, dalloc(c, &c->rank, n));
    PP_HIP(c, dalloc(c, &c->ubits, (size_t)c->nb));
    PP_HIP(c, dalloc(c, &c->gbox, (size_t)ppk::GBOX * (size_t)c->n_groups));
  }
  return h2d(c, c->sitems, items.data(), items.size() * sizeof(ppk::SymItem));
}

// ---------------------------------------------------------------------------
// Fused small-bunch schedule: one item per R receivers of a bunch, the
// items of the largest bunches first (their workgroups run longest); the
// second source buffer of the kick-and-drift.
// ---------------------------------------------------------------------------
pp_status build_fused(pp_ctx* c) {
  pp_status st;
  const int64_t R = c->tun.fused;
  std::vector<int> order(c->nb);
  for (int b = 0; b < c->nb; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return c->hb[x].n > c->hb[y].n; });
  std::vector<ppk::FusedItem> items;
  for (int b : order) {
    for (int64_t i0 = 0; i0 < c->hb[b].n; i0 += R) items.push_back({b, (int32_t)i0});
  }
  if (items.size() > (size_t)INT32_MAX) return set_err(c, PP_ERR_INVALID_ARG, "fused schedule too long");
  c->n_fitems = (int32_t)items.size();
  if (items.size() > c->fitems_cap) {
    c->fitems_cap = 0;
    if ((st = release(c, c->fitems)) != PP_OK) return st;
    PP_HIP(c, dalloc(c, &c->fitems, items.size()));
    c->fitems_cap = items.size();
  }
  const size_t n = (size_t)c->n_total;
  if (c->mixed() && !c->mir2) PP_HIP(c, dalloc(c, &c->mir2, 6 * n));
  if (!c->mixed() && !c->src64) PP_HIP(c, dalloc(c, &c->src64, 6 * n));
  return h2d(c, c->fitems, items.data(), items.size() * sizeof(ppk::FusedItem));
}

// ---------------------------------------------------------------------------
// Work list: items (bunch, j-chunk, first receiver), heaviest first.  The
// chunking rule is ppk::ordered_chunking.  Its fill cap (FILL_CHUNKS):
// measured at 4096 particles (16^3 cube, hipGraph replay), 32 chunks were
// 11-13% faster per step than 64 in both precisions.  Where rounding the chunk
// length up to 64 sources leaves fewer chunks the cap did not pay (3000
// particles: 24 chunks, one item per CU, 5% slower; 5000: 27 chunks, FP64 7%
// slower), so it applies only when exactly 32 chunks remain; at 2048, 8192 and
// 16384 particles the rule gives 32 or fewer anyway.
// ---------------------------------------------------------------------------
pp_status build_items(pp_ctx* c) {
  pp_status st;
  // kernels still in flight may read the old list and partial planes
  PP_HIP(c, hipStreamSynchronize(c->stream));
  const int K = c->k_eff();
  const int64_t BI = (int64_t)K * ppk::WG;

  struct Cand { WorkItem w; double cost; };
  std::vector<Cand> cand;
  int64_t pbase = 0;
  int64_t cbase = 0, gbase = 0, bbase = 0;
  for (int b = 0; b < c->nb; ++b) {
    const int64_t n = c->hb[b].n;
    const ppk::Chunking ch0 = ppk::ordered_chunking(n, K, c->tun.chunk_pairs_log2, c->tun.grid_per_cu, c->cus);
    const int64_t nch = ch0.n_chunks, chunk_len = ch0.chunk_len;
    BunchDev& B = c->hbd[b];
    B.n_chunks = (int32_t)nch;
    B.chunk_len = chunk_len;
    B.pbase = pbase;
    pbase += nch * n;
    // spatial-sort bases: compacted keys, 64-particle groups, symmetric blocks
    const int64_t bs = c->sym_block();
    if (cbase + n > INT32_MAX || gbase + (n + 63) / 64 > INT32_MAX)
      return set_err(c, PP_ERR_INVALID_ARG, "work list: more than 2^31 - 1 particles in bunches");
    B.cstart = cbase;
    B.gbase = (int32_t)gbase;
    B.bbase = (int32_t)bbase;
    cbase += n;
    gbase += (n + 63) / 64;
    bbase += (n + bs - 1) / bs;
    const int64_t nib = (n + BI - 1) / BI;
    for (int64_t ib = 0; ib < nib; ++ib) {
      for (int64_t ch = 0; ch < nch; ++ch) {
        const int64_t ni = std::min(BI, n - ib * BI);
        const int64_t nj = std::min(chunk_len, n - ch * chunk_len);
        // host-side shape checks of what the kernel assumes
        if (ni <= 0 || nj <= 0 || ib * BI > INT32_MAX || ch > INT32_MAX)
          return set_err(c, PP_ERR_INVALID_ARG, "work list: bunch too large for 32-bit local indices");
        cand.push_back({WorkItem{b, (int32_t)ch, (int32_t)(ib * BI), 0}, (double)ni * (double)nj});
      }
    }
  }
  c->n_in = cbase;
  c->n_groups = (int32_t)gbase;
  c->n_blocks = (int32_t)bbase;
  std::stable_sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) { return x.cost > y.cost; });
  if (cand.size() > (size_t)INT32_MAX) return set_err(c, PP_ERR_INVALID_ARG, "work list too long");
  std::vector<WorkItem> items(cand.size());
  for (size_t k = 0; k < cand.size(); ++k) items[k] = cand[k].w;
  c->n_items = (int32_t)items.size();

  // partial-sum planes
  const size_t esz = c->mixed() ? sizeof(float) : sizeof(double);
  const size_t need = (size_t)ppk::N_PLANES * (size_t)std::max<int64_t>(pbase, 1) * esz;
  if (need > c->part_bytes) {
    c->part_bytes = 0;
    if ((st = release(c, c->part)) != PP_OK) return st;
    PP_HIP(c, dalloc_bytes(c, &c->part, need));
    c->part_bytes = need;
  }
  c->P = pbase;
  if (items.size() > c->items_cap) {
    c->items_cap = 0;
    if ((st = release(c, c->items)) != PP_OK) return st;
    PP_HIP(c, dalloc(c, &c->items, items.size()));
    c->items_cap = items.size();
  }
  pp_status s;
  if ((s = h2d(c, c->items, items.data(), items.size() * sizeof(WorkItem))) != PP_OK) return s;
  if ((s = h2d(c, c->dbunch, c->hbd.data(), c->hbd.size() * sizeof(BunchDev))) != PP_OK) return s;
  if (c->fused()) return build_fused(c);
  return c->sym() ? build_sym(c) : PP_OK;
}

// ---------------------------------------------------------------------------
// Kernel argument blocks.
// ---------------------------------------------------------------------------
// Short work lists run one workgroup per item (the dispatcher hands them out
// in work-list order); long ones use the persistent grid and its counter, whose
// one atomic per item would serialise a list of many tiny items.
bool direct_items(const pp_ctx* c) { return c->n_items <= 65536; }

ppk::PairArgs pair_args(pp_ctx* c) {
  ppk::PairArgs a{};
  a.bunches = c->dbunch;
  a.items = c->items;
  a.n_items = c->n_items;
  a.counter = c->counter;
  a.direct = direct_items(c) ? 1 : 0;
  if (c->mixed()) {
    a.xh = c->plane(0); a.yh = c->plane(1); a.zh = c->plane(2);
    a.xl = c->plane(3); a.yl = c->plane(4); a.zl = c->plane(5);
    a.qt = c->plane(6);
    a.pf = (float*)c->part;
  } else {
    a.x = c->st.x; a.y = c->st.y; a.z = c->st.z;
    a.qt64 = c->qt64;
    a.pd = (double*)c->part;
  }
  a.P = c->P;
  return a;
}

ppk::PackArgs pack_args(pp_ctx* c) {
  ppk::PackArgs a{};
  a.bunches = c->dbunch;
  a.bid = c->bid;
  a.n_total = c->n_total;
  a.x = c->st.x; a.y = c->st.y; a.z = c->st.z;
  a.vx = c->st.vx; a.vy = c->st.vy; a.vz = c->st.vz;
  a.ax = c->ax; a.ay = c->ay; a.az = c->az;
  if (c->mixed()) {
    a.xh = c->plane(0); a.yh = c->plane(1); a.zh = c->plane(2);
    a.xl = c->plane(3); a.yl = c->plane(4); a.zl = c->plane(5);
  } else if (c->fused()) {
    a.sx = c->src64;
    a.sy = c->src64 + c->n_total;
    a.sz = c->src64 + 2 * c->n_total;
  }
  a.counter = c->counter;
  return a;
}

ppk::FinalArgs final_args(pp_ctx* c) {
  ppk::FinalArgs a{};
  a.bunches = c->dbunch;
  a.bid = c->bid;
  a.n_total = c->n_total;
  a.pf = (c->sym() && c->mixed()) ? (const float*)c->acc : (const float*)c->part;
  a.pd = (c->sym() && !c->mixed()) ? (const double*)c->acc : (const double*)c->part;
  a.P = c->sym() ? c->n_total : c->P;
  a.sym = c->sym() ? 1 : 0;
  a.rank = c->far() ? c->rank : nullptr;
  a.x = c->st.x; a.y = c->st.y; a.z = c->st.z;
  if (c->mixed()) {
    a.xh = c->plane(0); a.yh = c->plane(1); a.zh = c->plane(2);
    a.xl = c->plane(3); a.yl = c->plane(4); a.zl = c->plane(5);
  }
  a.counter = c->counter;
  a.q = c->st.q;
  a.m = c->st.m;
  a.vx = c->st.vx; a.vy = c->st.vy; a.vz = c->st.vz;
  a.ax = c->ax; a.ay = c->ay; a.az = c->az;
  return a;
}

int grid_size(pp_ctx* c) {
  if (direct_items(c)) return c->n_items;
  const int64_t g = (int64_t)c->cus * c->tun.grid_per_cu;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, c->n_items));
}

hipEvent_t take_event(pp_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// The three launches of one evaluation, on stream s.
pp_status enqueue_pack(pp_ctx* c, bool drift, hipStream_t s) {
  PP_LAUNCH(c, ppk::launch_pack(pack_args(c), drift, c->mixed(), s));
  c->cur = 0;  // the pack writes the first source buffer
  return PP_OK;
}

// Events around one pair-sum dispatch when profiling.
pp_status mark(pp_ctx* c, bool timed, bool begin, hipStream_t s) {
  if (!timed) return PP_OK;
  hipEvent_t e = take_event(c);
  if (!e) return dev_fail(c, hipErrorOutOfMemory, "hipEventCreate");
  PP_HIP(c, hipEventRecord(e, s));
  if (begin) c->ev_used.push_back({e, nullptr});
  else c->ev_used.back().second = e;
  return PP_OK;
}

// Reuse the current order at an evaluation of step k when it sorts the
// positions of the last multiple of kResortEvery up to k (or of k itself):
// a function of k and of the evaluations before it, so eager steps, graph
// replays, split runs and repeated evaluations of one step all agree.
bool perm_reusable(const pp_ctx* c, int64_t k) {
  return c->perm_k >= 0 && (c->perm_k == k || (k % kResortEvery != 0 && c->perm_k == k - k % kResortEvery));
}

// the order is aligned at the current step: the next evaluations follow the
// every-kResortEvery rule (what a captured graph assumes)
bool perm_aligned(const pp_ctx* c) {
  return !c->far() || c->perm_k == c->step - c->step % kResortEvery;
}

pp_status enqueue_pair(pp_ctx* c, bool phi, hipStream_t s, bool timed, int64_t k) {
  pp_status st;
  if (timed) ++c->prof_evals;
  if (c->sym() && !c->mixed()) {
    ppk::SymArgs64 sa{};
    sa.bunches = c->dbunch;
    sa.items = c->sitems;
    sa.x = c->st.x; sa.y = c->st.y; sa.z = c->st.z;
    sa.qt = c->qt64;
    sa.slot = (double*)c->slot;
    sa.nbt = c->n_blocks;
    sa.split = c->tun.sym_split;
    ppk::SymFoldArgs64 fa{};
    fa.bunches = c->dbunch;
    fa.bid = c->bid;
    fa.n_total = c->n_total;
    fa.slot = (const double*)c->slot;
    fa.acc = (double*)c->acc;
    fa.nbt = c->n_blocks;
    fa.block_size = (int32_t)c->sym_block();
    fa.split = c->tun.sym_split;
    fa.rounds = c->tun.sym_rounds;
    for (const auto& B : c->bands) {
      sa.r0 = B.r0;
      if ((st = mark(c, timed, true, s)) != PP_OK) return st;
      PP_LAUNCH(c, ppk::launch_sym64(sa, B.first, B.count, c->tun.i_per_lane, c->uniform_q, phi, s));
      if ((st = mark(c, timed, false, s)) != PP_OK) return st;
      fa.r0 = B.r0;
      fa.r1 = B.r1;
      PP_LAUNCH(c, ppk::launch_sym64_fold(fa, phi, s));
    }
  } else if (c->sym()) {
    ppk::SymArgs sa{};
    sa.bunches = c->dbunch;
    sa.items = c->sitems;
    sa.xh = c->plane(0); sa.yh = c->plane(1); sa.zh = c->plane(2);
    sa.xl = c->plane(3); sa.yl = c->plane(4); sa.zl = c->plane(5);
    sa.qt = c->plane(6);
    sa.slot = (float*)c->slot;
    sa.nbt = c->n_blocks;
    sa.split = c->tun.sym_split;
    if (c->far()) {
      ppk::SortArgs so{};
      so.bunches = c->dbunch;
      so.nb = c->nb;
      so.bid = c->bid;
      so.n_total = c->n_total;
      so.n_in = c->n_in;
      so.xh = c->plane(0); so.yh = c->plane(1); so.zh = c->plane(2);
      so.xl = c->plane(3); so.yl = c->plane(4); so.zl = c->plane(5);
      so.qt = c->plane(6);
      float* sp[7];
      for (int k = 0; k < 7; ++k) sp[k] = c->smir + (size_t)k * (size_t)c->n_total;
      so.sxh = sp[0]; so.syh = sp[1]; so.szh = sp[2];
      so.sxl = sp[3]; so.syl = sp[4]; so.szl = sp[5];
      so.sqt = sp[6];
      so.ubits = c->ubits;
      so.keys = c->keys; so.keys2 = c->keys + c->n_in;
      so.vals = c->vals; so.vals2 = c->vals + c->n_in;
      so.hist = c->hist;
      {
        const size_t tiles = ((size_t)c->n_in + ppk::SORT_TILE - 1) / ppk::SORT_TILE;
        so.dtot = c->hist + 256 * tiles;
      }
      so.rank = c->rank;
      so.gbox = c->gbox;
      const bool resort = !perm_reusable(c, k);
      if (resort) c->perm_k = k;
      PP_LAUNCH(c, ppk::launch_sort_bits(so, c->key_shift, c->key_bits, c->n_groups, resort, s));
      sa.xh = sp[0]; sa.yh = sp[1]; sa.zh = sp[2];
      sa.xl = sp[3]; sa.yl = sp[4]; sa.zl = sp[5];
      sa.qt = sp[6];
      sa.near_frac = std::ldexp(1.0f, -c->tun.far_split);
      sa.gbox = c->gbox;
      sa.ubits = c->ubits;
    }
    ppk::SymFoldArgs fa{};
    fa.bunches = c->dbunch;
    fa.bid = c->bid;
    fa.n_total = c->n_total;
    fa.slot = (const float*)c->slot;
    fa.acc = (float*)c->acc;
    fa.nbt = c->n_blocks;
    fa.block_size = (int32_t)c->sym_block();
    fa.split = c->tun.sym_split;
    fa.rounds = c->tun.sym_rounds;
    for (const auto& B : c->bands) {
      sa.r0 = B.r0;
      if ((st = mark(c, timed, true, s)) != PP_OK) return st;
      PP_LAUNCH(c, ppk::launch_sym(sa, B.first, B.count, c->tun.i_per_lane, c->uniform_q, phi, s));
      if ((st = mark(c, timed, false, s)) != PP_OK) return st;
      fa.r0 = B.r0;
      fa.r1 = B.r1;
      PP_LAUNCH(c, ppk::launch_sym_fold(fa, phi, s));
    }
  } else {
    if ((st = mark(c, timed, true, s)) != PP_OK) return st;
    PP_LAUNCH(c, ppk::launch_pair(pair_args(c), c->mixed(), c->k_eff(), c->tun.sum_tile, c->uniform_q, phi,
                                  grid_size(c), s));
    if ((st = mark(c, timed, false, s)) != PP_OK) return st;
  }
  return PP_OK;
}

pp_status enqueue_final(pp_ctx* c, ppk::FinalMode mode, double* ex, double* ey, double* ez, double* phi,
                        hipStream_t s) {
  ppk::FinalArgs a = final_args(c);
  a.ex = ex; a.ey = ey; a.ez = ez; a.phi = phi;
  PP_LAUNCH(c, ppk::launch_final(a, c->mixed(), mode, s));
  return PP_OK;
}

// One field evaluation and its update (mode): the pair stage then the
// combine kernel, or, on the fused schedule, one fused kernel reading the
// source buffer that holds the current positions (the kick-and-drift writes
// the other one).
pp_status enqueue_eval(pp_ctx* c, ppk::FinalMode mode, double* ex, double* ey, double* ez, double* phi,
                       hipStream_t s, bool timed, int64_t k) {
  pp_status st;
  if (!c->fused()) {
    if ((st = enqueue_pair(c, phi != nullptr, s, timed, k)) != PP_OK) return st;
    return enqueue_final(c, mode, ex, ey, ez, phi, s);
  }
  if (timed) ++c->prof_evals;
  const size_t n = (size_t)c->n_total;
  const int cur = c->cur, nxt = 1 - cur;
  ppk::FusedArgs fa{};
  fa.bunches = c->dbunch;
  fa.items = c->fitems;
  fa.upd = final_args(c);
  fa.upd.ex = ex; fa.upd.ey = ey; fa.upd.ez = ez; fa.upd.phi = phi;
  if (c->mixed()) {
    // buffer 0: the mirror's planes 0-5; buffer 1: mir2; the charge plane is shared
    auto buf = [&](int b, int p) { return b == 0 ? c->plane(p) : c->mir2 + (size_t)p * n; };
    fa.xh = buf(cur, 0); fa.yh = buf(cur, 1); fa.zh = buf(cur, 2);
    fa.xl = buf(cur, 3); fa.yl = buf(cur, 4); fa.zl = buf(cur, 5);
    fa.qt = c->plane(6);
    fa.upd.xh = buf(nxt, 0); fa.upd.yh = buf(nxt, 1); fa.upd.zh = buf(nxt, 2);
    fa.upd.xl = buf(nxt, 3); fa.upd.yl = buf(nxt, 4); fa.upd.zl = buf(nxt, 5);
  } else {
    const double* sb = c->src64 + (size_t)cur * 3 * n;
    fa.x = sb; fa.y = sb + n; fa.z = sb + 2 * n;
    fa.qt64 = c->qt64;
    double* nb = c->src64 + (size_t)nxt * 3 * n;
    fa.upd.sx = nb; fa.upd.sy = nb + n; fa.upd.sz = nb + 2 * n;
  }
  if ((st = mark(c, timed, true, s)) != PP_OK) return st;
  PP_LAUNCH(c, ppk::launch_fused(fa, c->mixed(), c->tun.fused, 256 * c->tun.i_per_lane, mode, c->uniform_q,
                                 phi != nullptr, c->n_fitems, s));
  if ((st = mark(c, timed, false, s)) != PP_OK) return st;
  if (mode == ppk::FIN_KICK_DRIFT) c->cur = nxt;
  return PP_OK;
}

pp_status ensure_accel(pp_ctx* c) {
  if (c->a_valid) return PP_OK;
  pp_status s;
  if ((s = enqueue_pack(c, false, c->stream)) != PP_OK) return s;
  if ((s = enqueue_eval(c, ppk::FIN_ACCEL, nullptr, nullptr, nullptr, nullptr, c->stream, c->prof, c->step)) !=
      PP_OK)
    return s;
  c->a_valid = true;
  return PP_OK;
}

// n >= 1 Velocity Verlet steps on stream s from step c->step: the first drift,
// then per step the pair stage and the kick; the kick of every step but the
// last also does the next step's drift and mirror pack (2n + 1 kernels of the
// ordered path instead of 3n, with the same arithmetic).
pp_status enqueue_steps(pp_ctx* c, int64_t n, hipStream_t s, bool timed) {
  pp_status r;
  if (n <= 0) return PP_OK;
  if ((r = enqueue_pack(c, true, s)) != PP_OK) return r;
  for (int64_t k = 0; k < n; ++k) {
    const ppk::FinalMode m = k + 1 < n ? ppk::FIN_KICK_DRIFT : ppk::FIN_KICK;
    if ((r = enqueue_eval(c, m, nullptr, nullptr, nullptr, nullptr, s, timed, c->step + k + 1)) != PP_OK) return r;
  }
  return PP_OK;
}

// Teardown of handles the context no longer uses: a failure here leaves
// nothing to recover, so the results of these destroy/free calls are dropped
// on purpose ((void) casts).
void drop_graph(pp_ctx* c) {
  if (c->graph.exec) (void)hipGraphExecDestroy(c->graph.exec);
  c->graph = Graph{};
}

pp_status capture_graph(pp_ctx* c, int64_t steps) {
  drop_graph(c);
  PP_HIP(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  pp_status st = PP_OK;
  // the captured steps' sort decisions update the host's record of the order
  // as if they had run; nothing has run yet, so it is restored afterwards and
  // advanced at each replay instead
  const int64_t perm_before = c->perm_k;
  st = enqueue_steps(c, steps, c->cap, false);
  const int64_t perm_after = c->perm_k;
  c->perm_k = perm_before;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (st != PP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return dev_fail(c, e, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return dev_fail(c, e, "hipGraphInstantiate");
  c->graph.exec = ex;
  c->graph.steps = steps;
  c->graph.phase = c->step % kResortEvery;
  c->graph.perm_offset = perm_after - c->step;
  return PP_OK;
}

pp_status check_finite(pp_ctx* c) {
  PP_HIP(c, hipMemsetAsync(c->counter + 1, 0, sizeof(int32_t), c->stream));
  PP_LAUNCH(c, ppk::launch_check_finite(c->bid, c->n_total, c->arrptr, 9, c->counter + 1, c->stream));
  int32_t flag = 0;
  pp_status s = d2h(c, &flag, c->counter + 1, sizeof(int32_t));
  if (s != PP_OK) return s;
  if (flag) return set_err(c, PP_ERR_NOT_FINITE, "non-finite position, velocity or acceleration");
  return PP_OK;
}

bool valid_tuning(const pp_tuning& t, bool mixed) {
  const int k = t.i_per_lane;
  if (!(k == 1 || k == 2 || k == 4 || k == 8)) return false;
  if (!mixed && k == 8) return false;
  if (t.sum_tile < 32 || t.sum_tile > 256 || (t.sum_tile & (t.sum_tile - 1))) return false;
  if (t.chunk_pairs_log2 < 16 || t.chunk_pairs_log2 > 30) return false;
  if (t.grid_per_cu < 1 || t.grid_per_cu > 16) return false;
  if (t.graph_steps < 1 || t.graph_steps > 1024) return false;
  if (t.symmetric != 0 && t.symmetric != 1) return false;
  // symmetric: 1, 2 or 4 receivers per lane; the near/far split is mixed only
  if (t.symmetric && k == 8) return false;
  // far_split <= 4 keeps the per-term bound 2 sqrt(3) 2^-23 2^f at 6.6e-6, inside the mixed tolerance
  if (t.far_split < 0 || t.far_split > 4 || (t.far_split > 0 && (!t.symmetric || !mixed))) return false;
  // parts per block pair: a divisor of the 8 (mixed) or 4 (FP64) groups of a
  // block at 1 receiver per lane
  if (!(t.sym_split == 1 || t.sym_split == 2 || t.sym_split == 4)) return false;
  // receiver-side rounds per symmetric item
  if (!(t.sym_rounds == 1 || t.sym_rounds == 2 || t.sym_rounds == 4 || t.sym_rounds == 8)) return false;
  // fused: 4, 8, 16 or 32 receivers per workgroup, on the ordered layout
  if (!(t.fused == 0 || t.fused == 4 || t.fused == 8 || t.fused == 16 || t.fused == 32)) return false;
  if (t.fused && (t.symmetric || t.far_split || k > 4)) return false;
  return true;
}

// Finish time of a greedy list schedule (each item to the earliest free slot,
// in launch order: n_off items of cost c_off, then n_diag of cost c_diag) on
// `slots` slots.  Beyond 64 items per slot the tail is bounded by one item.
double list_makespan(double n_off, double c_off, double n_diag, double c_diag, double slots) {
  const double total = n_off * c_off + n_diag * c_diag;
  if (n_off + n_diag > 64.0 * slots) return total / slots + std::max(c_off, c_diag);
  const int64_t P = (int64_t)slots;
  std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
  for (int64_t k = 0; k < P; ++k) free_at.push(0.0);
  double end = 0.0;
  auto place = [&](int64_t n, double cost) {
    for (int64_t k = 0; k < n; ++k) {
      const double t = free_at.top() + cost;
      free_at.pop();
      free_at.push(t);
      end = std::max(end, t);
    }
  };
  place((int64_t)n_off, c_off);
  place((int64_t)n_diag, c_diag);
  return end;
}

// Default tiling from the bunch sizes.  The symmetric schedule (mixed: with
// the near/far split at D = U / 8) is taken when a cost model says it is
// cheaper than the ordered-pair kernel.  Costs in units of one ordered pair in
// the ordered kernel of the same precision, from measurements on MI355X: an
// off-diagonal unordered pair 1.02, a diagonal-block pair 0.6, times a
// per-variant factor (mixed: 1.0 at 4 receivers per lane, 1.15 at 2; FP64:
// 1.28 at 4, 1.51 at 2, the FP64 sweep gaining less over its ordered kernel
// because its r^-3 costs more relative to the rest of a pair and the fold of
// FP64 slots costs 2-4%); 1 receiver per lane, ~1.4-2x slower in both
// precisions, is left to the autotuner.  The mixed sweep loses ground in
// small bunches (fewer wavefront boxes clear the far threshold, and the sort
// and the fold weigh more): charged as 1 + 1 / (bunch size / 1024).
// Splitting each block pair into S items adds a split overhead / BS of a
// block pair's cost per extra item (receiver loads, slot stores, the fold's
// extra reads; measured 1-4% per extra item): 32 on the mixed path, 24 on
// the FP64 path.  Padded blocks are paid in full, and the cost is the finish
// time of the launch's list schedule over the resident slots times the slot
// count (idle slots in the last wave included).  The mixed constants are
// fitted to the pair-stage times of every ordered and symmetric tiling
// (1, 2 or 4 per lane, split 1, 2 or 4) on uniform spheres of 12288-262144
// particles: the model's choice is within 4% of the fastest at every size.
constexpr double kSplitOverheadMixed = 32.0;
constexpr double kSplitOverheadFp64 = 24.0;

// Largest bunch the default tiling puts on the fused schedule.
constexpr int64_t kFusedDefaultMaxN = 8192;

pp_tuning default_tuning(bool mixed, const std::vector<pp_bunch>& hb, int cus) {
  int64_t min_n = INT64_MAX;
  double ordered = 0.0;
  for (const auto& b : hb) {
    min_n = std::min<int64_t>(min_n, b.n);
    ordered += (double)b.n * (double)b.n;
  }
  pp_tuning t{};
  t.i_per_lane = (mixed && min_n >= 16384) ? 2 : 1;
  t.sum_tile = 64;
  t.chunk_pairs_log2 = 22;
  t.grid_per_cu = 4;
  t.graph_steps = 16;
  t.symmetric = 0;
  t.sym_split = 1;
  // up to 8 rounds per symmetric item (sym_rounds_for: 2 from 256 blocks, 4
  // from 512, 8 from 1024): at 1M particles with 8-wavefront items the fold
  // and the rest of the step outside the pair kernel went 1.65 -> 1.19 ms
  // (mixed), 4.9 -> 3.0 ms (FP64); with 4-wavefront items 1M takes 1.2%
  // less per step at 8 than at 1 (`bench.py --tuning sym_rounds=1` against 8)
  t.sym_rounds = 8;
  struct Variant { int k; double bs, eff; int blocks_per_cu; };
  std::vector<Variant> vars;
  if (mixed) {
    vars.push_back({4, (double)ppk::SYM_WG * 4, 1.0, ppk::sym_blocks_per_cu(4)});
    vars.push_back({2, (double)ppk::SYM_WG * 2, 1.15, ppk::sym_blocks_per_cu(2)});
  } else {
    vars.push_back({4, (double)ppk::SYM64_WG * 4, 1.28, ppk::sym64_blocks_per_cu(4)});
    vars.push_back({2, (double)ppk::SYM64_WG * 2, 1.51, ppk::sym64_blocks_per_cu(2)});
  }
  double best = ordered;
  for (const Variant& v : vars) {
    // pair-weighted small-bunch factor of the mixed sweep
    double wsum = 0.0, psum = 0.0;
    for (const auto& b : hb) {
      const double nbk = std::ceil((double)b.n / v.bs);
      const double f = mixed ? 1.0 + 1.0 / std::ceil((double)b.n / 1024.0) : 1.0;
      wsum += nbk * nbk * f;
      psum += nbk * nbk;
    }
    const double eff = v.eff * wsum / psum;
    const double split_overhead = mixed ? kSplitOverheadMixed : kSplitOverheadFp64;
    for (int S : {1, 2, 4}) {
      double n_off = 0.0, n_diag = 0.0;
      for (const auto& b : hb) {
        const double nbk = std::ceil((double)b.n / v.bs);
        n_off += S * nbk * (nbk - 1.0) / 2.0;
        n_diag += S * nbk;
      }
      const double unit = v.bs * v.bs * eff, extra = (S - 1) * (split_overhead / v.bs) / S;
      const double slots = (double)cus * v.blocks_per_cu;
      const double cost =
          slots * list_makespan(n_off, unit * (1.02 / S + extra), n_diag, unit * (0.6 / S + extra), slots);
      if (cost < best) {
        best = cost;
        t.symmetric = 1;
        t.i_per_lane = v.k;
        t.sym_split = S;
        t.far_split = mixed ? 3 : 0;  // mixed: per-term change at most 3.3e-6 relative
      }
    }
  }
  // Small bunches: the fused schedule (one kernel per step).  Measured per
  // step on MI355X with hipGraph replay against the two-kernel ordered step,
  // at the fastest receivers per workgroup: 512 particles 9.8 -> 4.3 us,
  // 2048 11.5 -> 6.7, 4096 17.3 -> 13.5, 8192 42.9 -> 38.2 (mixed; FP64
  // 10.0 -> 4.2, 13.2 -> 7.5, 22.7 -> 16.4, 55.0 -> 49.0); at 16384 the
  // ordered and symmetric schedules are faster.  The fastest tiling gives
  // each CU about one workgroup of 512 threads: R = n / 256 receivers per
  // workgroup, a power of two in 4..32.
  int64_t max_n = 0;
  for (const auto& b : hb) max_n = std::max<int64_t>(max_n, b.n);
  if (max_n <= kFusedDefaultMaxN) {
    int64_t R = 4;
    while (R < 32 && 2 * R * 256 <= max_n) R *= 2;
    t.symmetric = 0;
    t.far_split = 0;
    t.sym_split = 1;
    t.fused = (int32_t)R;
    // workgroups of 512 threads; FP64 from 16 receivers per workgroup on
    // 1024 (`bench.py --mode steps`: 16.9 -> 16.3 us at 4096 particles,
    // 50.6 -> 48.5 us at 8192; at 2048 and in mixed precision 512 is faster)
    t.i_per_lane = (!mixed && R >= 16) ? 4 : 2;
  }
  return t;
}

pp_status apply_tuning(pp_ctx* c, const pp_tuning& t) {
  c->tun = t;
  c->perm_k = -1;
  drop_graph(c);
  return build_items(c);
}

// ---------------------------------------------------------------------------
// Autotuner: coordinate search over (i_per_lane, sum_tile, grid_per_cu,
// chunk size, schedule, far split, split of block pairs) by
// timed field evaluations on the context's own bunches; a candidate must
// reproduce the field of the starting tiling (relative L2 within the
// precision's tolerance) to be kept.  Choices are cached in a text file
// keyed by device, precision and problem size.
// ---------------------------------------------------------------------------
std::string tune_key(pp_ctx* c) {
  const int lp = (int)std::lround(std::log2(std::max(1.0, c->pairs)));
  const int lb = (int)std::lround(std::log2((double)c->nb));
  std::ostringstream o;
  o << "gfx950:" << c->cus << ":" << (c->mixed() ? "mixed" : "fp64") << ":p" << lp << ":b" << lb
    << ":q" << (c->uniform_q ? 1 : 0) << ":v7";
  std::string s = o.str();
  for (auto& ch : s)
    if (ch == ' ') ch = '_';
  return s;
}

std::string tune_path() {
  if (const char* e = std::getenv("PP_TUNE_CACHE")) return e;
  const char* h = std::getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/pp_mi355x_tune.txt";
}

bool tune_lookup(const std::string& key, pp_tuning* t) {
  // one record per line: key and the 8 tuning fields; other lines are skipped
  std::ifstream f(tune_path());
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream in(line);
    std::string k, extra;
    pp_tuning v{};
    if (!(in >> k >> v.i_per_lane >> v.sum_tile >> v.chunk_pairs_log2 >> v.grid_per_cu >> v.graph_steps >>
          v.symmetric >> v.far_split >> v.sym_split >> v.fused >> v.sym_rounds) || (in >> extra))
      continue;
    if (k == key) { *t = v; found = true; }
  }
  return found;
}

// mkdir -p without a shell: create each missing prefix of dir (0755)
bool make_dirs(const std::string& dir) {
  for (size_t pos = 1; pos <= dir.size(); ++pos) {
    if (pos == dir.size() || dir[pos] == '/') {
      const std::string prefix = dir.substr(0, pos);
      if (::mkdir(prefix.c_str(), 0755) != 0 && errno != EEXIST) return false;
    }
  }
  return true;
}

void tune_store(const std::string& key, const pp_tuning& t) {
  const std::string path = tune_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0 && !make_dirs(path.substr(0, slash))) return;
  std::ofstream f(path, std::ios::app);
  if (f)
    f << key << " " << t.i_per_lane << " " << t.sum_tile << " " << t.chunk_pairs_log2 << " " << t.grid_per_cu << " "
      << t.graph_steps << " " << t.symmetric << " " << t.far_split << " " << t.sym_split << " " << t.fused << " "
      << t.sym_rounds << "\n";
}

// Time of one field evaluation: the pair stage (the sort, the pair-sum
// dispatches, the folds; on the fused schedule the fused kernel, which also
// combines), and with `full` also the combine kernel.
pp_status time_eval(pp_ctx* c, int reps, double* ms, bool full = false) {
  hipEvent_t e0 = take_event(c), e1 = take_event(c);
  if (!e0 || !e1) return dev_fail(c, hipErrorOutOfMemory, "hipEventCreate");
  double tot = 0.0;
  pp_status st = PP_OK;
  for (int r = 0; r < reps && st == PP_OK; ++r) {
    if ((st = enqueue_pack(c, false, c->stream)) != PP_OK) break;
    PP_HIP(c, hipEventRecord(e0, c->stream));
    if (c->fused())
      st = enqueue_eval(c, ppk::FIN_FIELD, nullptr, nullptr, nullptr, nullptr, c->stream, false, c->step);
    else
      st = enqueue_pair(c, false, c->stream, false, c->step);
    if (st != PP_OK) break;
    if (full && !c->fused() &&
        (st = enqueue_final(c, ppk::FIN_FIELD, nullptr, nullptr, nullptr, nullptr, c->stream)) != PP_OK)
      break;
    PP_HIP(c, hipEventRecord(e1, c->stream));
    PP_HIP(c, hipEventSynchronize(e1));
    float f = 0.f;
    PP_HIP(c, hipEventElapsedTime(&f, e0, e1));
    tot += f;
  }
  c->ev_pool.push_back(e0);
  c->ev_pool.push_back(e1);
  *ms = tot / std::max(1, reps);
  return st;
}

pp_status field_into(pp_ctx* c, double* ex, double* ey, double* ez) {
  pp_status s;
  if ((s = enqueue_pack(c, false, c->stream)) != PP_OK) return s;
  return enqueue_eval(c, ppk::FIN_FIELD, ex, ey, ez, nullptr, c->stream, false, c->step);
}

pp_status l2_rel(pp_ctx* c, const double* ref, const double* got, double* rel) {
  // 3 * n_total doubles each; done on the host from a copy (set-up path only)
  const size_t n = (size_t)c->n_total * 3;
  std::vector<double> a(n), b(n);
  pp_status s;
  if ((s = d2h(c, a.data(), ref, n * sizeof(double))) != PP_OK) return s;
  if ((s = d2h(c, b.data(), got, n * sizeof(double))) != PP_OK) return s;
  double num = 0.0, den = 0.0;
  for (size_t k = 0; k < n; ++k) {
    const double d = b[k] - a[k];
    num += d * d;
    den += a[k] * a[k];
  }
  *rel = den > 0.0 ? std::sqrt(num / den) : std::sqrt(num);
  return PP_OK;
}

// Largest bunch the autotuner tries the fused schedule on: each of its
// workgroups streams the whole bunch, so its source traffic grows as n^2 / R.
constexpr int64_t kFusedMaxN = 65536;

pp_status autotune(pp_ctx* c) {
  const std::string key = tune_key(c);
  pp_tuning cached{};
  if (tune_lookup(key, &cached) && valid_tuning(cached, c->mixed())) {
    c->tuned = true;
    return apply_tuning(c, cached);
  }
  const size_t n3 = (size_t)c->n_total * 3;
  if (!c->cmp_buf) PP_HIP(c, dalloc(c, &c->cmp_buf, 2 * n3));
  double* ref = c->cmp_buf;
  double* got = c->cmp_buf + n3;
  pp_status s;
  pp_tuning best = c->tun;
  if ((s = apply_tuning(c, best)) != PP_OK) return s;
  if ((s = field_into(c, ref, ref + c->n_total, ref + 2 * c->n_total)) != PP_OK) return s;
  double best_ms = 0.0;
  // whole evaluations (the combine included), so that the fused schedule, which
  // combines inside its one kernel, is compared fairly
  if ((s = time_eval(c, 1, &best_ms, true)) != PP_OK) return s;   // warm-up
  if ((s = time_eval(c, 2, &best_ms, true)) != PP_OK) return s;
  const double tol = c->mixed() ? 1e-6 : 1e-13;
  auto trial = [&](pp_tuning t) -> pp_status {
    if (!valid_tuning(t, c->mixed())) return PP_OK;
    pp_status r;
    if ((r = apply_tuning(c, t)) != PP_OK) return r;
    double ms = 0.0;
    if ((r = time_eval(c, 2, &ms, true)) != PP_OK) return r;
    if (ms < best_ms * 0.98) {
      if ((r = field_into(c, got, got + c->n_total, got + 2 * c->n_total)) != PP_OK) return r;
      double rel = 0.0;
      if ((r = l2_rel(c, ref, got, &rel)) != PP_OK) return r;
      if (rel <= tol) { best = t; best_ms = ms; }
    }
    return PP_OK;
  };
  const int ks[] = {1, 2, 4, 8};
  for (int k : ks) { pp_tuning t = best; t.i_per_lane = k; if ((s = trial(t)) != PP_OK) return s; }
  const int tiles[] = {32, 64, 128, 256};
  for (int ts : tiles) { pp_tuning t = best; t.sum_tile = ts; if ((s = trial(t)) != PP_OK) return s; }
  const int gpc[] = {1, 2, 4, 8};
  for (int g : gpc) { pp_tuning t = best; t.grid_per_cu = g; if ((s = trial(t)) != PP_OK) return s; }
  for (int cp : {18, 20, 22, 24}) { pp_tuning t = best; t.chunk_pairs_log2 = cp; if ((s = trial(t)) != PP_OK) return s; }
  {
    for (int sym : {0, 1}) {
      for (int k : {1, 2, 4}) {
        pp_tuning t = best;
        t.symmetric = sym;
        t.i_per_lane = k;
        t.far_split = sym ? t.far_split : 0;
        t.fused = 0;
        if ((s = trial(t)) != PP_OK) return s;
      }
    }
    if (best.symmetric) {
      for (int f : {0, 2, 3, 4}) {
        pp_tuning t = best;
        t.far_split = f;
        if ((s = trial(t)) != PP_OK) return s;
      }
      for (int sp : {1, 2, 4}) {
        pp_tuning t = best;
        t.sym_split = sp;
        if ((s = trial(t)) != PP_OK) return s;
      }
      for (int sr : {1, 2, 4, 8}) {
        pp_tuning t = best;
        t.sym_rounds = sr;
        if ((s = trial(t)) != PP_OK) return s;
      }
    }
  }
  int64_t max_n = 0;
  for (const auto& b : c->hb) max_n = std::max(max_n, b.n);
  if (max_n <= kFusedMaxN) {
    for (int rec : {4, 8, 16, 32}) {
      for (int k : {1, 2, 4}) {
        pp_tuning t = best;
        t.symmetric = 0;
        t.far_split = 0;
        t.sym_split = 1;
        t.fused = rec;
        t.i_per_lane = k;
        if ((s = trial(t)) != PP_OK) return s;
      }
    }
  }
  if ((s = apply_tuning(c, best)) != PP_OK) return s;
  tune_store(key, best);
  c->tuned = true;
  return PP_OK;
}

// Set-up reductions over every bunch (per bunch: min and max of x, y, z, q
// and m, and the count of non-finite values), then the per-bunch constants.
constexpr int kMM = ppk::MM_LEN;
constexpr int kMMG = 64;

// Frame of the mixed path (origin at the midpoint of the bunch's extent, scale
// the power of two 2^-ceil(log2 half-extent), exact), the charge scaling and
// the field and potential factors.  At create it also validates q and m and
// picks the reference charge; later (pp_invalidate) it only re-centres the
// mixed path on the current positions, and a non-finite position leaves the
// frames unchanged (PP_ERR_NOT_FINITE).
pp_status setup_frames(pp_ctx* c, bool at_create) {
  PP_HIP(c, launch_gate(c));
  PP_HIP(c, ppk::launch_minmax(c->dbunch, c->nb, c->st.x, c->st.y, c->st.z, c->st.q, c->st.m, c->mmbuf, kMMG,
                               c->stream));
  std::vector<double> ext((size_t)c->nb * kMM);
  pp_status st = d2h(c, ext.data(), c->mmbuf, ext.size() * sizeof(double));  // waits for the reduction
  if (st != PP_OK) return st;
  std::vector<BunchDev> hbd = c->hbd;
  bool uniform = true;
  for (int b = 0; b < c->nb; ++b) {
    const double* r = &ext[(size_t)b * kMM];
    char buf[160];
    if (r[ppk::MM_NONFIN] != 0.0) {
      std::snprintf(buf, sizeof buf, "bunch %d: %.0f particles with non-finite r, q or m", b, r[ppk::MM_NONFIN]);
      return set_err(c, at_create ? PP_ERR_INVALID_ARG : PP_ERR_NOT_FINITE, buf);
    }
    if (at_create && !(r[ppk::MM_M] > 0.0)) {
      std::snprintf(buf, sizeof buf, "bunch %d: mass must be > 0", b);
      return set_err(c, PP_ERR_INVALID_ARG, buf);
    }
    const bool same_q =
        ppk::frame_from_extents(r, c->hb[b].weight, c->hb[b].softening, kCoulomb, c->mixed(), at_create, hbd[b]);
    if (!same_q) uniform = false;
  }
  if (at_create) c->uniform_q = uniform;
  c->hbd = hbd;
  return h2d(c, c->dbunch, c->hbd.data(), c->hbd.size() * sizeof(BunchDev));
}

void free_all(pp_ctx* c) {
  drop_graph(c);
  // every device allocation the context still holds (the buffers above and
  // any other), so that a context broken half-way through a call frees all
  while (!c->live.empty()) (void)dfree(c, c->live.begin()->first);
  if (c->hpin) (void)hipHostFree(c->hpin);
  for (auto& e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto& p : c->ev_used) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  if (c->cap) (void)hipStreamDestroy(c->cap);
}

}  // namespace

namespace ppk {
void set_thread_error(const std::string& msg) { g_create_error = msg; }
}  // namespace ppk

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int32_t pp_abi_version(void) { return PP_ABI_VERSION; }

const char* pp_last_error(const pp_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

pp_status pp_create(pp_ctx** out, const pp_bunch* bunches, int32_t n_bunches, int64_t n_total,
                    const pp_state* state, pp_precision prec, void* hip_stream) {
  g_create_error.clear();
  if (!out) return set_err(nullptr, PP_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!bunches || n_bunches < 1) return set_err(nullptr, PP_ERR_INVALID_ARG, "need at least one bunch");
  if (!state) return set_err(nullptr, PP_ERR_INVALID_ARG, "state is NULL");
  if (prec != PP_FP64 && prec != PP_MIXED) return set_err(nullptr, PP_ERR_INVALID_ARG, "unknown precision");
  if (n_total < 1) return set_err(nullptr, PP_ERR_INVALID_ARG, "n_total < 1");
  const pp_state& S = *state;
  if (!S.x || !S.y || !S.z || !S.vx || !S.vy || !S.vz || !S.q || !S.m)
    return set_err(nullptr, PP_ERR_INVALID_ARG, "state has a NULL array");
  int64_t prev_end = 0;
  for (int b = 0; b < n_bunches; ++b) {
    const pp_bunch& B = bunches[b];
    char buf[160];
    if (B.n < 1 || B.offset < prev_end || B.offset > n_total - B.n) {
      std::snprintf(buf, sizeof buf, "bunch %d: offset/n out of order, overlapping or outside n_total", b);
      return set_err(nullptr, PP_ERR_INVALID_ARG, buf);
    }
    if (B.n > (int64_t)INT32_MAX / 2) {
      std::snprintf(buf, sizeof buf, "bunch %d: 2^30 or more particles (local indices are 32-bit)", b);
      return set_err(nullptr, PP_ERR_INVALID_ARG, buf);
    }
    if (!finite_pos(B.weight) || !finite_pos(B.dt) || !std::isfinite(B.softening) || B.softening < 0.0) {
      std::snprintf(buf, sizeof buf, "bunch %d: need weight > 0, dt > 0, softening >= 0, all finite", b);
      return set_err(nullptr, PP_ERR_INVALID_ARG, buf);
    }
    prev_end = B.offset + B.n;
  }

  pp_ctx* c = new (std::nothrow) pp_ctx();
  if (!c) return set_err(nullptr, PP_ERR_OUT_OF_MEMORY, "host allocation failed");
  read_fault_hook(c);
  c->prec = prec;
  c->nb = n_bunches;
  c->n_total = n_total;
  c->st = S;
  c->hb.assign(bunches, bunches + n_bunches);
  c->hbd.resize(n_bunches);
  auto fail = [&](pp_status s) {
    g_create_error = c->err;
    free_all(c);
    delete c;
    return s;
  };
#define PP_CREATE_HIP(call)                                        \
  do {                                                             \
    hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return fail(dev_fail(c, e_, #call));     \
  } while (0)

  PP_CREATE_HIP(hipGetDevice(&c->device));
  int cus = 0;
  PP_CREATE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
  c->cus = std::max(1, cus);
  c->stream = (hipStream_t)hip_stream;  // NULL: the legacy default stream
  PP_CREATE_HIP(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));

  const size_t n = (size_t)n_total;
  PP_CREATE_HIP(dalloc(c, &c->dbunch, (size_t)n_bunches));
  PP_CREATE_HIP(dalloc(c, &c->dweight, (size_t)n_bunches));
  PP_CREATE_HIP(dalloc(c, &c->bid, n));
  PP_CREATE_HIP(dalloc(c, &c->ax, n));
  PP_CREATE_HIP(dalloc(c, &c->ay, n));
  PP_CREATE_HIP(dalloc(c, &c->az, n));
  PP_CREATE_HIP(dalloc(c, &c->counter, 4));
  PP_CREATE_HIP(dalloc(c, &c->arrptr, 9));
  if (prec == PP_MIXED) PP_CREATE_HIP(dalloc(c, &c->mir, 7 * n));
  else PP_CREATE_HIP(dalloc(c, &c->qt64, n));

  for (int b = 0; b < n_bunches; ++b) {
    BunchDev& B = c->hbd[b];
    std::memset(&B, 0, sizeof B);
    B.off = bunches[b].offset;
    B.n = bunches[b].n;
    B.dt = bunches[b].dt;
    B.n_chunks = 1;
    B.chunk_len = B.n;
  }
  std::vector<double> wts(n_bunches);
  for (int b = 0; b < n_bunches; ++b) wts[b] = bunches[b].weight;
  pp_status st0;
  if ((st0 = h2d(c, c->dweight, wts.data(), wts.size() * sizeof(double))) != PP_OK) return fail(st0);
  if ((st0 = h2d(c, c->dbunch, c->hbd.data(), c->hbd.size() * sizeof(BunchDev))) != PP_OK) return fail(st0);
  PP_CREATE_HIP(hipMemsetAsync(c->bid, 0xff, n * sizeof(int32_t), c->stream));  // -1: outside every bunch
  PP_CREATE_HIP(hipMemsetAsync(c->ax, 0, n * sizeof(double), c->stream));
  PP_CREATE_HIP(hipMemsetAsync(c->ay, 0, n * sizeof(double), c->stream));
  PP_CREATE_HIP(hipMemsetAsync(c->az, 0, n * sizeof(double), c->stream));
  PP_CREATE_HIP(hipMemsetAsync(c->counter, 0, 4 * sizeof(int32_t), c->stream));
  PP_CREATE_HIP(launch_gate(c));
  PP_CREATE_HIP(ppk::launch_fill_bid(c->bid, n_total, c->dbunch, n_bunches, c->stream));
  const double* tbl[9] = {S.x, S.y, S.z, S.vx, S.vy, S.vz, c->ax, c->ay, c->az};
  if ((st0 = h2d(c, c->arrptr, tbl, sizeof tbl)) != PP_OK) return fail(st0);

  // device reductions over the bunches: extents, charge range, mass check;
  // the per-bunch constants (frame of the mixed path, charge scaling)
  PP_CREATE_HIP(dalloc(c, &c->mmbuf, (size_t)n_bunches * kMM * (kMMG + 1)));
  if ((st0 = setup_frames(c, true)) != PP_OK) return fail(st0);
  for (int b = 0; b < n_bunches; ++b) c->pairs += (double)c->hbd[b].n * (double)(c->hbd[b].n - 1);
  PP_CREATE_HIP(launch_gate(c));
  PP_CREATE_HIP(ppk::launch_qprep(c->dbunch, c->bid, n_total, S.q, c->mixed() ? c->plane(6) : nullptr, c->qt64,
                                  c->stream));
  c->tun = default_tuning(c->mixed(), c->hb, c->cus);
  pp_status st = build_items(c);
  if (st != PP_OK) return fail(st);
#undef PP_CREATE_HIP
  *out = c;
  return PP_OK;
}

pp_status pp_field(pp_ctx* c, double* ex, double* ey, double* ez, double* phi) {
  pp_status s;
  if ((s = usable(c)) != PP_OK) return s;
  if (!ex || !ey || !ez) return set_err(c, PP_ERR_INVALID_ARG, "field outputs must not be NULL");
  if ((s = enqueue_pack(c, false, c->stream)) != PP_OK) return s;
  return enqueue_eval(c, ppk::FIN_FIELD, ex, ey, ez, phi, c->stream, false, c->step);
}

pp_status pp_push(pp_ctx* c, int64_t n_steps) {
  pp_status s;
  if ((s = usable(c)) != PP_OK) return s;
  if (n_steps < 0) return set_err(c, PP_ERR_INVALID_ARG, "n_steps < 0");
  if ((s = ensure_accel(c)) != PP_OK) return s;
  if ((s = enqueue_steps(c, n_steps, c->stream, c->prof)) != PP_OK) return s;
  c->step += n_steps;
  return PP_OK;
}

pp_status pp_step_batched(pp_ctx* c, int64_t n_steps, uint32_t flags) {
  pp_status s;
  if ((s = usable(c)) != PP_OK) return s;
  if (n_steps < 0) return set_err(c, PP_ERR_INVALID_ARG, "n_steps < 0");
  if (flags & ~(PP_GRAPH | PP_AUTOTUNE | PP_CHECK)) return set_err(c, PP_ERR_INVALID_ARG, "unknown flag");
  if ((flags & PP_AUTOTUNE) && !c->tuned) {
    if ((s = autotune(c)) != PP_OK) return s;
  }
  if ((s = ensure_accel(c)) != PP_OK) return s;
  int64_t left = n_steps;
  if ((flags & PP_GRAPH) && left >= c->tun.graph_steps) {
    // a graph's sort decisions assume the order aligned to the every-
    // kResortEvery rule: after an invalidation, step eagerly until it is
    while (left > 0 && !perm_aligned(c)) {
      if ((s = enqueue_steps(c, 1, c->stream, c->prof)) != PP_OK) return s;
      c->step += 1;
      --left;
    }
    while (left >= c->tun.graph_steps) {
      // one graph per step phase (its baked sort decisions depend on it)
      if (!c->graph.exec || c->graph.steps != c->tun.graph_steps ||
          (c->far() && c->graph.phase != c->step % kResortEvery)) {
        if ((s = capture_graph(c, c->tun.graph_steps)) != PP_OK) return s;
      }
      PP_LAUNCH(c, hipGraphLaunch(c->graph.exec, c->stream));
      if (c->far()) c->perm_k = c->step + c->graph.perm_offset;
      left -= c->graph.steps;
      c->step += c->graph.steps;
    }
  }
  if ((s = enqueue_steps(c, left, c->stream, c->prof)) != PP_OK) return s;
  c->step += left;
  if (flags & PP_CHECK) return check_finite(c);
  return PP_OK;
}

pp_status pp_diagnostics(pp_ctx* c, pp_diag* out) {
  pp_status s;
  if ((s = usable(c)) != PP_OK) return s;
  if (!out) return set_err(c, PP_ERR_INVALID_ARG, "out is NULL");
  const int G = (int)std::max<int64_t>(1, std::min<int64_t>(1024, 2048 / c->nb));
  if (!c->phi) PP_HIP(c, dalloc(c, &c->phi, (size_t)c->n_total));
  const size_t need = (size_t)c->nb * ((size_t)G * ppk::D_N1 + ppk::D_NREC + ppk::D_OUT);
  if (need > c->diag_doubles) {
    c->diag_doubles = 0;
    if ((s = release(c, c->diag_buf)) != PP_OK) return s;  // the last diagnostics call synchronised
    PP_HIP(c, dalloc(c, &c->diag_buf, need));
    c->diag_doubles = need;
  }
  if ((s = enqueue_pack(c, false, c->stream)) != PP_OK) return s;
  if ((s = enqueue_eval(c, ppk::FIN_FIELD, nullptr, nullptr, nullptr, c->phi, c->stream, false, c->step)) != PP_OK)
    return s;
  ppk::DiagArgs d{};
  d.bunches = c->dbunch;
  d.x = c->st.x; d.y = c->st.y; d.z = c->st.z;
  d.vx = c->st.vx; d.vy = c->st.vy; d.vz = c->st.vz;
  d.q = c->st.q; d.m = c->st.m; d.phi = c->phi;
  d.weight = c->dweight;
  d.part = c->diag_buf + (size_t)c->nb * (ppk::D_NREC + ppk::D_OUT);
  d.rec = c->diag_buf;
  d.G = G;
  PP_LAUNCH(c, ppk::launch_diag(d, c->nb, c->stream));
  std::vector<double> res((size_t)c->nb * ppk::D_OUT);
  if ((s = d2h(c, res.data(), c->diag_buf + (size_t)c->nb * ppk::D_NREC, res.size() * sizeof(double))) != PP_OK)
    return s;
  for (int b = 0; b < c->nb; ++b) {
    const double* r = &res[(size_t)b * ppk::D_OUT];
    pp_diag& o = out[b];
    o.step = c->step;
    o.n = c->hb[b].n;
    o.time = (double)c->step * c->hb[b].dt;
    static_assert(offsetof(pp_diag, nonfinite) - offsetof(pp_diag, kinetic) == ppk::D_OUT_VALUES * sizeof(double),
                  "the device record matches pp_diag from kinetic through v_max");
    std::memcpy(&o.kinetic, r, ppk::D_OUT_VALUES * sizeof(double));
    o.nonfinite = (int64_t)std::llround(r[ppk::D_OUT_VALUES]);
  }
  return PP_OK;
}

pp_status pp_invalidate(pp_ctx* c) {
  pp_status s;
  if ((s = usable(c)) != PP_OK) return s;
  c->a_valid = false;
  c->perm_k = -1;
  // re-centre the mixed path's frames on the current positions (the FP64 path
  // uses positions as they are)
  if (c->mixed()) return setup_frames(c, false);
  return PP_OK;
}

pp_status pp_get_tuning(const pp_ctx* c, pp_tuning* out) {
  if (!c || !out) return PP_ERR_INVALID_ARG;
  *out = c->tun;
  return PP_OK;
}

pp_status pp_set_tuning(pp_ctx* c, const pp_tuning* t) {
  pp_status s;
  if ((s = usable(c)) != PP_OK) return s;
  if (!t || !valid_tuning(*t, c->mixed())) return set_err(c, PP_ERR_INVALID_ARG, "tuning out of range");
  c->tuned = true;
  return apply_tuning(c, *t);
}

pp_status pp_time_field(pp_ctx* c, int32_t n_reps, double* ms, double* pairs) {
  pp_status s;
  if ((s = usable(c)) != PP_OK) return s;
  if (n_reps < 1 || !ms) return set_err(c, PP_ERR_INVALID_ARG, "n_reps < 1 or ms NULL");
  if ((s = time_eval(c, n_reps, ms)) != PP_OK) return s;
  if (pairs) *pairs = c->pairs;
  return PP_OK;
}

pp_status pp_set_profiling(pp_ctx* c, int32_t enable) {
  pp_status s;
  if ((s = usable(c)) != PP_OK) return s;
  c->prof = enable != 0;
  return PP_OK;
}

pp_status pp_get_profile(pp_ctx* c, pp_profile* out) {
  pp_status s;
  if ((s = usable(c)) != PP_OK) return s;
  if (!out) return set_err(c, PP_ERR_INVALID_ARG, "out is NULL");
  PP_HIP(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (auto& p : c->ev_used) {
    float f = 0.f;
    PP_HIP(c, hipEventElapsedTime(&f, p.first, p.second));
    tot += f;
    c->ev_pool.push_back(p.first);
    c->ev_pool.push_back(p.second);
  }
  out->evaluations = c->prof_evals;
  out->launches = (int64_t)c->ev_used.size();
  out->total_ms = tot;
  out->pairs = c->pairs;
  c->ev_used.clear();
  c->prof_evals = 0;
  return PP_OK;
}

int64_t pp_device_bytes(const pp_ctx* c) { return c ? c->live_bytes : g_live_bytes.load(); }

pp_status pp_sync(pp_ctx* c) {
  pp_status s;
  if ((s = usable(c)) != PP_OK) return s;
  PP_HIP(c, hipStreamSynchronize(c->stream));
  return PP_OK;
}

pp_status pp_destroy(pp_ctx* c) {
  if (!c) return PP_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);  // teardown: nothing to report to
  free_all(c);
  delete c;
  return PP_OK;
}

}  // extern "C"
