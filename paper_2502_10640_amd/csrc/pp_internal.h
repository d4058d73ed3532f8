// pp_internal.h -- device data layout shared by the gfx950 kernels and the
// host runtime of the PP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace ppk {

// Threads per workgroup of the pair-sum kernels; also the number of j
// particles staged in LDS per tile (one global load per thread per tile).
constexpr int WG = 256;
constexpr int JT = WG;
// Smallest j-chunk of the ordered-pair work list (a partly filled tile); used
// only where chunks of whole tiles would leave the GPU idle.
constexpr int CHUNK_MIN = 64;

// Per-bunch constants in device memory.
//   Mixed path: positions enter the pair sum as u = (r - origin) * scale with
//   scale a power of two (exact), split into FP32 hi + lo; the field is
//   E = kE * S with S = sum_j qt_j d_u / (|d_u|^2 + eps2s)^(3/2) and
//   kE = k w qref scale^2, the potential phi = kPhi * Psi with
//   kPhi = k w qref scale.
//   FP64 path: unscaled SI positions, S = sum_j qt_j d / (|d|^2 + eps2)^(3/2),
//   kE = k w qref, kPhi = k w qref.
//   qt_j = q_j / qref (exactly 1 for a bunch of identical charges).
struct BunchDev {
  int64_t off;        // first particle in the state arrays
  int64_t n;          // particles
  double dt;          // time step [s]
  double origin[3];   // mixed-path origin [m]
  double scale;       // mixed-path scale [1/m], power of two
  double qref;        // reference charge [C]
  double kE;          // field factor (see above)
  double kPhi;        // potential factor
  double eps2;        // FP64 path: eps^2 [m^2]
  float eps2s;        // mixed path: (eps * scale)^2
  int32_t n_chunks;   // j-chunks the bunch's sources are split into
  int64_t chunk_len;  // sources per chunk (multiple of JT, or of CHUNK_MIN for small bunches)
  int64_t pbase;      // first partial-sum slot of the bunch
  int64_t cstart;     // spatial sort: first position of the bunch in the compacted key array
  int32_t gbase;      // spatial sort: first 64-particle group box of the bunch
  int32_t bbase;      // symmetric schedule: first block of the bunch over all bunches
};

// Coulomb constant 1/(4 pi eps0) from the CODATA 2018 vacuum permittivity.
inline double coulomb_k() { return 1.0 / (4.0 * 3.14159265358979323846 * 8.8541878128e-12); }

// Set-up reductions over a bunch: min and max of x, y, z, q and m, the count
// of non-finite values, padding (MM_* slots of one record).
enum MinMaxSlot : int32_t { MM_X = 0, MM_Y = 2, MM_Z = 4, MM_Q = 6, MM_M = 8, MM_NONFIN = 10, MM_LEN = 12 };

// 2^-ceil(log2 h) for h > 0, exactly: frexp gives h = f 2^e with f in [0.5, 1),
// and ceil(log2 h) is e - 1 when f = 0.5 (h a power of two), else e.
__host__ __device__ inline double frame_scale(double h) {
  int e = 0;
  const double f = frexp(h, &e);
  return ldexp(1.0, f == 0.5 ? 1 - e : -e);
}

// Frame of the mixed path and the factors of the field and the potential of
// one bunch from its set-up extents r[MM_LEN] (the same arithmetic on the host
// and on the device): origin at the midpoint of the extent, scale
// 2^-ceil(log2 half-extent) (at least the softening; exact; 1 when both are
// zero, a bunch of one particle or of coincident ones, whose separations are
// all zero in any frame), and, with set_q, the reference charge (the charge
// of largest magnitude, 1 if all are zero).  Returns whether the charges are
// all equal and not zero: the uniform-charge kernels take every normalised
// charge q / qref as 1, which a bunch of neutral particles (q / qref = 0) is
// not.
__host__ __device__ inline bool frame_from_extents(const double* r, double weight, double softening, double kc,
                                                   bool mixed, bool set_q, BunchDev& B) {
#pragma clang fp contract(off)
  double half = 0.0;
  for (int a = 0; a < 3; ++a) {
    B.origin[a] = 0.5 * (r[2 * a] + r[2 * a + 1]);
    half = fmax(half, 0.5 * (r[2 * a + 1] - r[2 * a]));
  }
  half = fmax(half, softening);
  if (!(half > 0.0)) half = 1.0;
  B.scale = frame_scale(half);
  const double qlo = r[MM_Q], qhi = r[MM_Q + 1];
  if (set_q) {
    double qref = fabs(qhi) >= fabs(qlo) ? qhi : qlo;
    if (qref == 0.0) qref = 1.0;
    B.qref = qref;
  }
  const double qref = B.qref;
  if (mixed) {
    B.kE = kc * weight * qref * B.scale * B.scale;
    B.kPhi = kc * weight * qref * B.scale;
    const double es = softening * B.scale;
    B.eps2s = (float)(es * es);
  } else {
    B.kE = kc * weight * qref;
    B.kPhi = kc * weight * qref;
    B.eps2 = softening * softening;
  }
  return qlo == qhi && qlo != 0.0;
}

// Source chunks of one bunch of n particles in the ordered-pair work list
// (receiver blocks of i_per_lane x WG): a bunch's sources are split into
// chunks of about 2^chunk_pairs_log2 pair interactions, and into at least
// enough chunks for the bunch alone to give cus x grid_per_cu items (down to
// CHUNK_MIN-source chunks), with the fill alone capped at FILL_CHUNKS chunks
// while that still leaves two items per CU.  Depends only on the bunch's own
// size and the device, so a bunch gives the same bits alone or in a batch.
constexpr int64_t FILL_CHUNKS = 32;

struct Chunking {
  int64_t n_chunks;
  int64_t chunk_len;
};

inline Chunking ordered_chunking(int64_t n, int i_per_lane, int chunk_pairs_log2, int grid_per_cu, int cus) {
  const int64_t BI = (int64_t)i_per_lane * WG;
  const double full = (double)(n < BI ? n : BI) * (double)n;
  const int64_t max_ch = (n + CHUNK_MIN - 1) / CHUNK_MIN;
  const int64_t nib0 = (n + BI - 1) / BI;
  const int64_t fill = (int64_t)cus * grid_per_cu;
  // chunk length for a wanted chunk count, and the chunk count it gives;
  // chunks are whole LDS tiles (JT sources) where that still fills the GPU,
  // else multiples of CHUNK_MIN sources (a partly filled tile)
  auto chunking = [&](int64_t want, int64_t* len) {
    want = want < 1 ? 1 : (want > max_ch ? max_ch : want);
    const int64_t per = (n + want - 1) / want;
    const int64_t gran = per >= JT ? JT : CHUNK_MIN;
    *len = ((per + gran - 1) / gran) * gran;
    return (n + *len - 1) / *len;
  };
  const int64_t by_pairs = (int64_t)llround(full / ldexp(1.0, chunk_pairs_log2));
  const int64_t by_fill = (fill + nib0 - 1) / nib0;
  Chunking c{0, 0};
  c.n_chunks = chunking(by_pairs > by_fill ? by_pairs : by_fill, &c.chunk_len);
  if (by_fill > FILL_CHUNKS && by_pairs < FILL_CHUNKS) {
    int64_t len = 0;
    const int64_t capped = chunking(FILL_CHUNKS, &len);
    if (capped == FILL_CHUNKS && capped * nib0 >= 2 * (int64_t)cus) {
      c.n_chunks = capped;
      c.chunk_len = len;
    }
  }
  return c;
}

// One unit of pair work: receivers [i0, i0 + i_per_lane * WG) of bunch b
// against the sources of chunk `chunk` of the same bunch.
struct WorkItem {
  int32_t b;
  int32_t chunk;
  int32_t i0;
  int32_t pad;
};

struct PairArgs {
  const BunchDev* bunches;
  const WorkItem* items;
  int32_t n_items;
  int32_t* counter;        // persistent-kernel work counter (zeroed by the pack kernel)
  int32_t direct;          // 1: one workgroup per item (item = blockIdx.x), no counter
  // mixed-path source mirror, FP32 SoA over all particles
  const float* xh; const float* yh; const float* zh;
  const float* xl; const float* yl; const float* zl;
  const float* qt;
  // FP64-path sources
  const double* x; const double* y; const double* z;
  const double* qt64;
  // partial sums: planes of length P (mixed: float planes Sx Sy Sz Cx Cy Cz Sp Cp;
  // fp64: double planes Sx Sy Sz Cx Cy Cz Sp Cp)
  float* pf;
  double* pd;
  int64_t P;
};

// Number of partial-sum planes (field hi, field compensation, potential).
constexpr int N_PLANES = 8;

// Symmetric pair sum (Newton's third law): one rsq per unordered pair.  A bunch
// is cut into blocks of SYM_WAVES * 64 * i_per_lane particles.  An item is the
// receiver block I against the source block J != I (both sides evaluated),
// or a diagonal item I == J (ordered pairs inside the block, self excluded).
// Items are numbered by rounds: round 0 holds the diagonal items, round d >= 1
// the pairs (I, I + d mod n_blocks), so in one round every block has at most
// one receiver-side and one source-side partial.  Each item writes its two
// partials into slots of its own, indexed by (round, block, side); a fold
// kernel then adds the slots to the accumulators in round order.  Items of
// many rounds therefore run in one launch, in any order, and the order of
// every addition is still fixed.
constexpr int SYM_WAVES = 4;
constexpr int SYM_WG = SYM_WAVES * 64;
constexpr int SYM_PLANES = 16;  // Si(xyz) Ci(xyz) Sj(xyz) Cj(xyz) Sip Cip Sjp Cjp
// per slot: one value per component, the item's compensated partial (S, C)
// rounded to S + C (x, y, z, potential): one rounding of relative size u per
// item partial, below the bounds of the plain sums it comes from
constexpr int SLOT_PLANES = 4;

struct SymItem {
  int32_t b;
  int32_t I;
  int32_t J;
  // sub-round r * split + h: round r of block pairs (0 = diagonal) and the
  // part h < split of source block J's 64-source groups that the item sweeps
  int32_t r;
  // rounds the item sweeps, r, r + 1, ..., r + nr - 1 (source blocks
  // I + r .. I + r + nr - 1 mod the bunch's block count), all part h; its
  // receiver side is one partial over all of them (1 for diagonal items)
  int32_t nr;
};

// Receiver-side rounds per item of a bunch of nbk blocks for the tuning value
// sym_rounds (1, 2, 4 or 8): the largest power of two M <= sym_rounds with at
// least 128 M blocks (smaller bunches keep their items short, so that the
// last wave of items stays full; measured with 4-wavefront items at 8
// rounds allowed: 256 blocks best at 2, 512 at 4, 1024 at 8).  Groups of
// rounds start at rounds 1, 1 + M, 1 + 2 M, ...; a power of two, M divides
// every other bunch's M or is a multiple of it.  Depends only on the bunch's
// size and the tuning.
__host__ __device__ inline int sym_rounds_for(int64_t nbk, int sym_rounds) {
  int m = sym_rounds;
  while (m > 1 && nbk < 128 * (int64_t)m) m >>= 1;
  return m;
}

// Rounds of the group that starts at round r (r >= 1, (r - 1) % M == 0) for
// receiver block X of a bunch of nbk blocks: M rounds, fewer at the last
// group, and without the half round nbk / 2 of an even block count where
// X >= nbk / 2 (that round holds only I < nbk / 2).  0: no item.
__host__ __device__ inline int sym_group_rounds(int64_t nbk, int M, int64_t r, int64_t X) {
  const int64_t half = nbk / 2;
  int64_t nr = half - r + 1 < M ? half - r + 1 : M;
  if (nr <= 0) return 0;
  if (nbk % 2 == 0 && r + nr - 1 == half && X >= half) --nr;
  return (int)nr;
}

struct SymArgs {
  const BunchDev* bunches;
  const SymItem* items;
  const float *xh, *yh, *zh, *xl, *yl, *zl, *qt;
  // partial slots of the sub-rounds [r0, r0 + count): float index
  // (((r - r0) * nbt + block) * 2 + side) * SLOT_PLANES + plane) * block_size + offset,
  // block = bunch's first block + I (side 0, receiver) or + J (side 1, source);
  // an item writes the source side only at the offsets of its part of J
  float* slot;
  int32_t r0;
  int32_t nbt;             // blocks over all bunches
  int32_t split;           // items per block pair (1, 2 or 4)
  // near/far split (needs the spatial sort): a source group whose box is
  // farther than near_frac * min(U, (|a| + |b|) / 2) from a wavefront's receiver
  // box (a, b: the boxes' per-axis largest |coordinate|) uses plain FP32
  // separations; near_frac = 0 keeps hi/lo separations everywhere
  float near_frac;
  const float* gbox;       // [group][GBOX]: min xyz, max xyz of the FP32 high parts, |b|
  const uint32_t* ubits;   // per-bunch bound U on |scaled coordinate| (float bits)
};

// Fold of the slots of sub-rounds [r0, r1) into the accumulators (SYM_PLANES
// planes of length n_total, indexed by position), in sub-round order.
struct SymFoldArgs {
  const BunchDev* bunches;
  const int32_t* bid;
  int64_t n_total;
  const float* slot;
  float* acc;
  int32_t r0, r1;
  int32_t nbt;
  int32_t block_size;
  int32_t split;
  int32_t rounds;          // the sym_rounds tuning value
};

// Spatial sort (pp_sort.hip): keys per tile of the radix sort.
constexpr int SORT_TILE = 2048;
// Group box record: min xyz, max xyz, then |b| = the norm of the per-axis
// largest |coordinate| over the box, then padding.
constexpr int GBOX = 8;

struct SortArgs {
  const BunchDev* bunches;
  int32_t nb;
  const int32_t* bid;
  int64_t n_total;
  int64_t n_in;            // particles inside bunches
  const float *xh, *yh, *zh, *xl, *yl, *zl, *qt;    // mirror, particle order
  float *sxh, *syh, *szh, *sxl, *syl, *szl, *sqt;   // mirror, sorted order
  uint32_t* ubits;
  uint64_t *keys, *keys2;
  int32_t *vals, *vals2;
  uint32_t* hist;          // 256 x sort tiles, digit-major
  uint32_t* dtot;          // 256 digit totals
  int32_t* rank;           // sorted position of each particle
  float* gbox;
};

struct PackArgs {
  const BunchDev* bunches;
  const int32_t* bid;      // bunch of each particle, -1 outside every bunch
  int64_t n_total;
  double *x, *y, *z;
  const double *vx, *vy, *vz;
  const double *ax, *ay, *az;
  float *xh, *yh, *zh, *xl, *yl, *zl;
  double *sx, *sy, *sz;    // FP64 source copy of the positions (fused FP64 schedule), or null
  int32_t* counter;
};

enum FinalMode : int32_t {
  FIN_FIELD = 0,   // write E (and phi) to output arrays
  FIN_ACCEL = 1,   // a = (q/m) E
  FIN_KICK = 2,    // a' = (q/m) E; v += (a + a') dt / 2; a = a'
  FIN_KICK_DRIFT = 3  // FIN_KICK, then the next step's drift and mirror pack
                      // (the pack kernel's work, same arithmetic)
};

struct FinalArgs {
  const BunchDev* bunches;
  const int32_t* bid;
  int64_t n_total;
  const float* pf;
  const double* pd;
  int64_t P;
  const double* q;
  const double* m;
  double *vx, *vy, *vz;
  double *ax, *ay, *az;
  double *ex, *ey, *ez, *phi;   // FIN_FIELD outputs (phi may be null)
  int32_t sym;                  // partials are the symmetric accumulators
  const int32_t* rank;          // symmetric accumulators in sorted order: slot = rank[i]
  // FIN_KICK_DRIFT: positions, mixed mirror (or FP64 source copy, where
  // given) and the pair kernel's work counter
  double *x, *y, *z;
  float *xh, *yh, *zh, *xl, *yl, *zl;
  double *sx, *sy, *sz;
  int32_t* counter;
};

// Fused small-bunch schedule (pp_fused.hip): one workgroup per item computes
// the whole field of receivers [i0, i0 + R) of bunch b and applies the update.
struct FusedItem {
  int32_t b;
  int32_t i0;
};

struct FusedArgs {
  const BunchDev* bunches;
  const FusedItem* items;
  // this step's sources: mixed mirror planes (qt: normalised charge), or the
  // FP64 source copy and the FP64 normalised charge
  const float *xh, *yh, *zh, *xl, *yl, *zl, *qt;
  const double *x, *y, *z, *qt64;
  // the update (state, outputs; FIN_KICK_DRIFT: the next step's source
  // buffer in xh..zl or sx..sz)
  FinalArgs upd;
};

// Diagnostics: per-bunch reduction record in device memory (doubles).
enum DiagSlot : int32_t {
  D_KIN = 0, D_POT, D_MSUM, D_P0, D_P1, D_P2,
  D_MR0, D_MR1, D_MR2, D_MV0, D_MV1, D_MV2,
  D_X0, D_X1, D_X2, D_V0, D_V1, D_V2,
  D_XX0, D_XX1, D_XX2, D_VV0, D_VV1, D_VV2,
  D_XV0, D_XV1, D_XV2,
  D_NSUM,                       // number of sums of pass 1
  D_XMAX0 = D_NSUM, D_XMAX1, D_XMAX2, D_VMAX0, D_VMAX1, D_VMAX2,
  D_NONFIN,
  D_N1,                         // record length of pass 1
  // pass 2 (centred second moments)
  D_CXX0 = D_N1, D_CXX1, D_CXX2, D_CVV0, D_CVV1, D_CVV2, D_CXV0, D_CXV1, D_CXV2,
  D_NREC
};
constexpr int D_N2 = D_NREC - D_N1;

// Host record of one bunch written by the diagnostics kernels: the 30 values
// of pp_diag from `kinetic` through `v_max` in declaration order, then the
// non-finite count.
constexpr int D_OUT_VALUES = 30;
constexpr int D_OUT = D_OUT_VALUES + 1;

struct DiagArgs {
  const BunchDev* bunches;
  const double *x, *y, *z, *vx, *vy, *vz, *q, *m, *phi;
  const double* weight;   // per bunch
  double* part;           // [n_bunches][G][D_N1] block partials
  double* rec;            // [n_bunches][D_NREC] reduced record
  int32_t G;              // blocks per bunch
};

}  // namespace ppk

// Message returned by pp_last_error(NULL) on the calling thread (set by the
// calls that have no context).
#include <string>
namespace ppk {
void set_thread_error(const std::string& msg);
}  // namespace ppk

// Launchers (pp_kernels.hip).  Each returns the hipGetLastError() status.
namespace ppk {
hipError_t launch_pack(const PackArgs& a, bool drift, bool mixed, hipStream_t s);
hipError_t launch_pair(const PairArgs& a, bool mixed, int i_per_lane, int sum_tile, bool uniform_q,
                       bool with_phi, int grid, hipStream_t s);
hipError_t launch_final(const FinalArgs& a, bool mixed, FinalMode mode, hipStream_t s);
hipError_t launch_sym(const SymArgs& a, int32_t first, int32_t count, int i_per_lane, bool uniform_q, bool with_phi,
                      hipStream_t s);
hipError_t launch_sym_fold(const SymFoldArgs& a, bool with_phi, hipStream_t s);
int sym_blocks_per_cu(int i_per_lane);  // resident symmetric workgroups per CU (occupancy query)
hipError_t launch_sort(const SortArgs& a, int key_bits, int32_t n_groups_total, hipStream_t s);
hipError_t launch_qprep(const BunchDev* bunches, const int32_t* bid, int64_t n_total, const double* q,
                        float* qt, double* qt64, hipStream_t s);
hipError_t launch_minmax(const BunchDev* bunches, int32_t n_bunches, const double* x, const double* y,
                         const double* z, const double* q, const double* m, double* out, int32_t G,
                         hipStream_t s);
hipError_t launch_check_finite(const int32_t* bid, int64_t n_total, const double* const* arrays,
                               int32_t n_arrays, int32_t* flag, hipStream_t s);
hipError_t launch_diag(const DiagArgs& a, int32_t n_bunches, hipStream_t s);
hipError_t launch_fill_bid(int32_t* bid, int64_t n_total, const BunchDev* bunches, int32_t n_bunches,
                           hipStream_t s);
int pair_regs_hint(bool mixed, int i_per_lane);
// Fused small-bunch schedule: the launch of one evaluation, one workgroup of
// `threads` (256, 512 or 1024) per item of `receivers` (4, 8, 16 or 32).
hipError_t launch_fused(const FusedArgs& a, bool mixed, int receivers, int threads, FinalMode mode, bool uniform_q,
                        bool with_phi, int n_items, hipStream_t s);
}  // namespace ppk
