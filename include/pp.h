/*
 * pp.h -- C ABI of the MI355X (gfx950) particle-particle Coulomb library.
 *
 * The library implements the electrostatic particle-particle (PP) model of
 * arXiv 2502.10640 ("Comparison between electrostatic PP and PIC simulations
 * on electron bunch expansion"), Sec. 2.1:
 *   - the direct field sum over all macro-particle pairs, Eq. (B) built from
 *     Coulomb's law Eq. (A), here with optional Plummer softening eps
 *     (eps = 0 is Eq. (B) exactly):
 *       E_i = k sum_{j != i, same bunch} (w q_j) (r_i - r_j) / (|r_i - r_j|^2 + eps^2)^(3/2),
 *       k = 1 / (4 pi eps0);
 *   - the acceleration a_i = (q_i / m_i) E_i of Eqs. (D)/(F) (the macro
 *     weight w cancels);
 *   - the Velocity Verlet push of Eqs. (G)/(H):
 *       r(t+dt) = r + v dt + a dt^2 / 2,   v(t+dt) = v + [a(t) + a(t+dt)] dt / 2;
 *   - the beam diagnostics of Sec. 2.2 / 3.2 (emittance Eq. (I), rms and
 *     maximum of x and v_x) plus energy, momentum and centre of mass.
 * Several independent bunches ("batched" runs: one macro-weight / time-step
 * sweep of the paper per call) share one context; particles of different
 * bunches do not interact.
 *
 * Conventions for every call
 *   - Units are SI: m, m/s, C, kg, s, V/m, V, J.
 *   - Device pointers are HIP device addresses on the device that was current
 *     when pp_create ran; host pointers are ordinary process memory.
 *   - Every call returns a pp_status; no exception, abort or exit crosses the
 *     ABI.  On PP_ERR_INVALID_ARG nothing was enqueued and no state changed.
 *     After PP_ERR_DEVICE or PP_ERR_OUT_OF_MEMORY from a call other than
 *     pp_create the context is broken: later calls return PP_ERR_STATE and
 *     only pp_destroy is valid.  pp_last_error gives a message.
 *   - Work is enqueued on the context's stream and is asynchronous unless a
 *     call says otherwise.  One context must not be used from two host threads
 *     at once.  Different contexts are independent.
 *   - Failure testing: when the environment variable PP_FAULT_INJECT holds
 *     "alloc:N" or "launch:N" (N >= 1; "alloc" and "launch" mean N = 1) at
 *     pp_create, the N-th device allocation or kernel launch that context
 *     makes (counting from pp_create's first) fails without reaching the
 *     device, as an out-of-memory error or a launch failure.  The failing call
 *     returns PP_ERR_OUT_OF_MEMORY or PP_ERR_DEVICE and the context is broken
 *     as after a real failure.
 */
#ifndef PP_MI355X_PP_H
#define PP_MI355X_PP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PP_ABI_VERSION 4

typedef struct pp_ctx pp_ctx; /* opaque; owns its device scratch */

typedef enum {
  PP_OK = 0,
  PP_ERR_INVALID_ARG = 1,   /* bad argument; nothing happened            */
  PP_ERR_OUT_OF_MEMORY = 2, /* device allocation failed                  */
  PP_ERR_DEVICE = 3,        /* a HIP call failed                         */
  PP_ERR_NOT_FINITE = 4,    /* PP_CHECK found a non-finite r, v or a     */
  PP_ERR_STATE = 5          /* context unusable after an earlier failure */
} pp_status;

/* Arithmetic of the pair sum.
 *   PP_FP64  : every pair in FP64; per-particle field summed per j-tile and
 *              the tile sums combined with compensated (two-sum) addition.
 *   PP_MIXED : pair arithmetic in FP32 on positions split into FP32 high and
 *              low parts (so separations keep ~48 bits), tile sums in FP32
 *              combined across tiles by two-sum; the push, the accumulation
 *              of chunk partials and all reductions stay in FP64. */
typedef enum { PP_FP64 = 0, PP_MIXED = 1 } pp_precision;

/* One bunch: particles [offset, offset + n) of the state arrays.  Bunches
 * must be sorted by offset and must not overlap (gaps are allowed and are
 * left untouched).  Sec. 2.1: all macro-particles of a bunch share one
 * weight w (Q = q w, M = m w). */
typedef struct {
  int64_t offset;   /* >= 0; bunches in increasing, disjoint order */
  int64_t n;        /* 1 <= n < 2^30 particles                 */
  double weight;    /* w > 0, real particles per macro-particle */
  double softening; /* eps >= 0 [m]; 0 is the bare Eq. (B)     */
  double dt;        /* Velocity Verlet step > 0 [s]            */
} pp_bunch;

/* Particle state, device SoA of length n_total, FP64.  Borrowed: the caller
 * owns the memory, which must outlive the context.  r and v are read and
 * updated in place by pp_push / pp_step_batched; q and m are read only and
 * must not change while the context lives (they are inspected at create).
 * q is the real-particle charge, m the real-particle mass (> 0). */
typedef struct {
  double *x, *y, *z;
  double *vx, *vy, *vz;
  const double *q;
  const double *m;
} pp_state;

/* Diagnostics of one bunch (host record).  Averages <.> are plain means over
 * the bunch's particles (uniform weight).  Per-axis arrays are [x, y, z]. */
typedef struct {
  int64_t step;                  /* steps taken since create              */
  int64_t n;                     /* particles                             */
  double time;                   /* step * dt [s]                         */
  double kinetic;                /* sum (1/2) w m |v|^2 [J]               */
  double potential;              /* (1/2) sum w q phi [J], phi softened   */
  double total;                  /* kinetic + potential                   */
  double momentum[3];            /* sum w m v                             */
  double com[3];                 /* sum m r / sum m                       */
  double com_velocity[3];        /* sum m v / sum m                       */
  double emittance[3];           /* Eq. (I) on raw moments                */
  double emittance_centered[3];  /* Eq. (I) on moments about the means    */
  double x_rms[3];               /* <x^2>^(1/2) (raw)                     */
  double x_max[3];               /* max x                                 */
  double v_rms[3];               /* <v_x^2>^(1/2) (raw)                   */
  double v_max[3];               /* max v_x                               */
  int64_t nonfinite;             /* particles with non-finite r or v      */
} pp_diag;

/* Flags of pp_step_batched. */
#define PP_GRAPH 1u    /* replay the step loop from captured hipGraphs            */
#define PP_AUTOTUNE 2u /* time candidate tilings once and keep the fastest passing */
#define PP_CHECK 4u    /* synchronise after the steps; PP_ERR_NOT_FINITE if any r,
                          v or a is not finite                                  */

/* Kernel tiling of the pair sum.  Any valid tiling gives a correct result
 * (within the precision's tolerance); for one tiling results are bitwise
 * reproducible run to run. */
typedef struct {
  int32_t i_per_lane;    /* receivers held in registers per lane: 1, 2, 4 or 8  */
  int32_t sum_tile;      /* j per plain partial sum before the two-sum: 32..256,
                            power of two                                        */
  int32_t chunk_pairs_log2; /* j-chunk splitting: a receiver block's sources are
                            split into chunks of about 2^chunk_pairs_log2 pair
                            interactions (16..30).  The split depends only on
                            the bunch's own size, so a bunch gives the same
                            bits alone or in a batch.                           */
  int32_t grid_per_cu;   /* ordered kernel: workgroups per compute unit of its
                            persistent grid (work lists over 65536 items), and
                            the items per CU a bunch is split into, 1..16      */
  int32_t graph_steps;   /* steps captured per hipGraph with PP_GRAPH, 1..1024   */
  int32_t symmetric;     /* 1 evaluates each unordered pair once (Newton's
                            third law, Eq. (A) antisymmetry) in rounds of block
                            pairs, i_per_lane 1, 2 or 4 (blocks of 256
                            i_per_lane particles in either precision); 0
                            evaluates every ordered pair in the ordered-pair
                            kernel                                              */
  int32_t far_split;     /* PP_MIXED symmetric only: 0 keeps the hi/lo
                            separations (positions as FP32 high + low parts)
                            for every pair; f in 1..4 orders each bunch
                            along a Morton curve (recomputed at steps that are
                            multiples of 8, reused in between; the boxes below
                            always come from the current positions) and uses plain
                            FP32 separations for a 64-source group whose box is
                            farther than D = 2^-f min(U, (|a| + |b|)/2) from
                            the box of a wavefront's receivers (U: largest
                            scaled coordinate of the bunch; a, b: per-axis
                            largest |scaled coordinate| of the two boxes).
                            Each such term then differs from the hi/lo term by
                            at most 2 sqrt(3) 2^-23 2^f relative (6.6e-6 at
                            f = 4, inside the mixed tolerance).                 */
  int32_t sym_split;     /* symmetric only: 1, 2 or 4 items per block pair, each
                            sweeping that fraction of the source block's
                            64-source groups (diagonal blocks too), so that a
                            bunch of a few block pairs per compute unit still
                            fills the last wave of items.  Changes the order of
                            additions, hence the bits.  The ordered schedule
                            ignores it.                                         */
  int32_t fused;         /* 0, or the fused small-bunch schedule with that many
                            receivers per workgroup (4, 8, 16 or 32; needs
                            symmetric 0 and far_split 0; i_per_lane 1, 2 or 4
                            then gives workgroups of 256 x i_per_lane threads
                            that split each receiver's sources; sum_tile,
                            chunk_pairs_log2 and grid_per_cu do not apply):
                            one workgroup computes the whole field of its
                            receivers, every source of the bunch streamed
                            through LDS, and applies the update itself, so a
                            step is one kernel.  Changes the order of
                            additions, hence the bits.                          */
  int32_t sym_rounds;    /* symmetric only: up to 1, 2, 4 or 8 consecutive
                            rounds per item: a bunch takes the largest power
                            of two M <= sym_rounds with at least 128 M
                            blocks (else 1).  An item then keeps its
                            receiver block in registers across that many
                            source blocks: one receiver-side partial instead
                            of one per round, and the receiver block read once
                            (less slot and mirror traffic, longer items).
                            Changes the order of additions, hence the bits.    */
} pp_tuning;

/* Create a context over n_bunches bunches of a state of n_total particles:
 * the set-up of Sec. 2.1 (N_p macro-particles per bunch of one weight w, each
 * with the real-particle charge q and mass m of Eqs. (C)-(F)), ready for the
 * field sum of Eq. (B) and the Velocity Verlet steps of Eqs. (G)/(H).
 * Inspects q and m on the device (FP64 reductions) to validate them and to
 * pick per-bunch charge scaling; synchronises the stream once.
 * PP_MIXED: each bunch's positions enter the FP32 pair arithmetic relative to
 * a frame fixed here from the bunch's extent (origin at the midpoint, scale a
 * power of two near the half-extent R; exact in FP64).  The hi/lo split keeps
 * each coordinate to about 2^-48 of its size in that frame, so once a bunch's
 * centre has moved a distance D from the origin a separation d carries an
 * extra relative error of about 2^-48 (D + R) / |d|, beside the 2^-24 of the
 * FP32 pair arithmetic: negligible while D is well below 2^24 |d| (for the
 * closest pairs of a 10^6-particle sphere, about 10^3 - 10^4 R).  Before
 * that, the near/far split of the symmetric schedule, whose threshold grows
 * with the coordinates' size, finds fewer source groups far and the sum slows
 * down.  pp_invalidate re-centres the frames; call it once a bunch has moved
 * by more than a few R. 
 *   out         receives the context (host pointer, required)
 *   bunches     host array of n_bunches entries, read only during the call
 *   n_total     length of every state array; every bunch lies inside it
 *   state       host pointer to the device pointers of the state
 *   prec        PP_FP64 or PP_MIXED
 *   hip_stream  hipStream_t every call enqueues on; NULL is the device's
 *               legacy default stream (ordered with all blocking streams)
 * Errors: PP_ERR_INVALID_ARG (null pointers, n < 1 or n >= 2^30, bad offsets, w <= 0,
 * eps < 0, dt <= 0, non-finite parameters, m <= 0 or non-finite q/m on the
 * device), PP_ERR_OUT_OF_MEMORY, PP_ERR_DEVICE.  On error *out is NULL and
 * pp_last_error(NULL) holds the message. */
pp_status pp_create(pp_ctx **out, const pp_bunch *bunches, int32_t n_bunches, int64_t n_total,
                    const pp_state *state, pp_precision prec, void *hip_stream);

/* Field (and optionally potential) at the current positions, Eq. (B) with
 * softening, written to caller-owned device arrays of length n_total (entries
 * outside every bunch are not written).  phi = NULL skips the potential; with
 * phi the self term j = i is excluded as in E.  Two distinct particles at the
 * same position contribute a zero term to each other when eps > 0; with
 * eps = 0 their term is 0/0 as in Eq. (B) itself, so their field and
 * potential are not finite (every other particle's are unaffected; the
 * PP_CHECK flag of pp_step_batched reports such a state).  Asynchronous. */
pp_status pp_field(pp_ctx *ctx, double *ex, double *ey, double *ez, double *phi);

/* Allocation-free field of one bunch, without a context.  For callers that
 * cannot allocate device memory: code under hipGraph stream capture, tight
 * serving loops, harnesses that forbid hipMalloc.  It calls no hipMalloc,
 * hipFree or other allocating routine and reads nothing back to the host;
 * every buffer it needs (bunch constants, work list, source mirror, partial
 * sums) lies in one static device array of PP_NOALLOC_SCRATCH_MIB MiB per
 * device, held from the first call on a device until the process ends.
 *   n           particles, 1 <= n <= PP_NOALLOC_MAX_N (more: PP_ERR_INVALID_ARG)
 *   x, y, z, q  device arrays of length n, FP64: positions [m] and
 *               real-particle charges [C]; read only, not inspected on the host
 *               (a non-finite value gives non-finite results)
 *   weight, softening, prec   as for a pp_bunch / pp_create
 *   ex, ey, ez  device outputs of length n [V/m]; phi (nullable) [V]
 *   hip_stream  stream the kernels are enqueued on (NULL: the legacy default)
 * Writes E (and phi) of every particle exactly as pp_field does for a context
 * of this one bunch on the ordered-pair tiling (symmetric 0, fused 0,
 * i_per_lane 1, sum_tile 64, chunk_pairs_log2 22, grid_per_cu 4): the same
 * bits.
 * Asynchronous.  Calls on one device share its scratch, which keeps the last
 * call's contents (each call rewrites all it reads): calls that overlap in
 * time on one device (different streams, or different host threads) race and
 * must be ordered by the caller.  Errors: PP_ERR_INVALID_ARG (null pointer,
 * n out of range, weight <= 0, softening < 0, a layout beyond the scratch),
 * PP_ERR_DEVICE (a HIP call failed); pp_last_error(NULL) holds the message. */
#define PP_NOALLOC_MAX_N 65536
#define PP_NOALLOC_SCRATCH_MIB 24
pp_status pp_field_noalloc(int64_t n, const double *x, const double *y, const double *z, const double *q,
                           double weight, double softening, pp_precision prec, double *ex, double *ey,
                           double *ez, double *phi, void *hip_stream);

/* Advance every bunch by n_steps >= 0 Velocity Verlet steps (Sec. 2.1,
 * Eqs. (G)/(H), with a = (q/m) E of Eqs. (D)/(F)), each step a plain sequence
 * of kernel launches.  The acceleration at the
 * current positions is computed first if it is not known (first call, or after
 * pp_invalidate).  Asynchronous. */
pp_status pp_push(pp_ctx *ctx, int64_t n_steps);

/* Same trajectory as pp_push (bitwise, for the same tiling): Velocity Verlet
 * steps of Sec. 2.1, Eqs. (G)/(H), of every bunch (the paper's weight and
 * time-step sweeps of Sec. 2.2 as one batch), driven by the batched scheduler: one pair-sum stage per step serving every bunch from one
 * work list (or one round schedule); with PP_GRAPH the steps are replayed from hipGraphs
 * captured on first use; with PP_AUTOTUNE the tiling is chosen by timing
 * candidates once (the choice is kept in the context); PP_CHECK as above.
 * Asynchronous unless PP_AUTOTUNE runs a search or PP_CHECK is given. */
pp_status pp_step_batched(pp_ctx *ctx, int64_t n_steps, uint32_t flags);

/* Diagnostics of every bunch into out[0 .. n_bunches-1] (host memory): the
 * beam quantities the paper follows (Sec. 2.2: the emittance of Eq. (I);
 * Sec. 3.2: <x^2>^(1/2), x_max, <v_x^2>^(1/2), v_x,max), per axis, and the
 * conserved quantities (total energy with the potential of Eq. (B)'s pair
 * law, momentum, centre of mass).  Costs one potential evaluation (O(N^2) per
 * bunch) and FP64 reductions in a fixed order; synchronises the stream. */
pp_status pp_diagnostics(pp_ctx *ctx, pp_diag *out);

/* Declare that the caller changed r or v: a(t) is recomputed on the next
 * push and the far split's spatial order at the next evaluation.  PP_MIXED:
 * the frames of pp_create are re-centred on the current positions (a device
 * reduction; synchronises the stream).  A non-finite position gives
 * PP_ERR_NOT_FINITE and leaves the frames as they were (the context stays
 * usable). */
pp_status pp_invalidate(pp_ctx *ctx);

/* Read or replace the tiling.  Setting checks ranges (PP_ERR_INVALID_ARG) and
 * drops captured graphs and the far split's spatial order. */
pp_status pp_get_tuning(const pp_ctx *ctx, pp_tuning *out);
pp_status pp_set_tuning(pp_ctx *ctx, const pp_tuning *tuning);

/* Time one field evaluation of the current tiling with HIP events on the
 * context stream (synchronises): *ms receives the average over n_reps
 * evaluations of the pair-sum stage (spatial sort if any, pair-sum
 * dispatches, folds); *pairs the ordered pair interactions per evaluation
 * (sum over bunches of n (n - 1)). */
pp_status pp_time_field(pp_ctx *ctx, int32_t n_reps, double *ms, double *pairs);

/* Kernel timing of the pair sum inside pp_push / pp_step_batched.  With
 * profiling on, every pair-sum kernel dispatch made outside a hipGraph is
 * bracketed by HIP events on the context stream (the spatial sort and the
 * folds of the symmetric schedule are not). */
typedef struct {
  int64_t evaluations; /* field evaluations timed since the last read      */
  int64_t launches;    /* pair-sum kernel dispatches among them (the
                          symmetric schedule makes one per band of rounds) */
  double total_ms;     /* sum of the dispatches' durations [ms]            */
  double pairs;        /* ordered pair interactions per evaluation         */
} pp_profile;
pp_status pp_set_profiling(pp_ctx *ctx, int32_t enable);
/* Synchronises, returns and resets the counters. */
pp_status pp_get_profile(pp_ctx *ctx, pp_profile *out);

/* Synchronise the context stream. */
pp_status pp_sync(pp_ctx *ctx);

/* Device memory accounting: bytes of device memory ctx currently holds (its
 * scratch: acceleration, source mirror, partial sums, work lists, sort
 * buffers, diagnostics), or, for ctx = NULL, the total over every live context
 * of the process.  After pp_destroy of every context the total is 0, also for
 * contexts broken by a failure half-way through a call.  Host only; never
 * fails. */
int64_t pp_device_bytes(const pp_ctx *ctx);

/* Release every resource of the context (synchronises first).  NULL is a
 * no-op.  Valid in every state; the context must not be used afterwards. */
pp_status pp_destroy(pp_ctx *ctx);

/* Last error message of ctx, or of the calling thread's last failed
 * pp_create or pp_field_noalloc when ctx is NULL.  Never NULL; "" when there was none.  The
 * string lives until the next call on the same context (or thread). */
const char *pp_last_error(const pp_ctx *ctx);

/* PP_ABI_VERSION of the loaded library. */
int32_t pp_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PP_MI355X_PP_H */
