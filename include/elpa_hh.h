/*
 * elpa_hh.h -- C ABI of the MI355X (gfx950) back-transformation of
 * eigenvectors from tridiagonal to band form, the hot step of the two-stage
 * Hermitian eigensolver.
 *
 * Operation (Kus et al., "Optimizations of the Eigensolvers in the ELPA
 * Library", Sec. 2: the back-transformation V~ = Q^H V^ that follows the
 * tridiagonal solve of Eq. Esolv, applied in the two-stage method to the
 * band -> tridiagonal reflectors; Sec. 3.1 names this part of the
 * back-transformation as the compute-heavy kernel that BLAS cannot express):
 *
 *     Q <- H(0,0) H(0,1) ... H(n-2, J(n-2)-1) Q,     H(s,j) = I - tau v v^H
 *
 * for every reflector of the one-column-per-step bulge chase: sweep
 * s = 0..n-2, chase step j = 0..J(s)-1 with J(s) = ceil((n-1-s)/nbw), acting
 * on rows [r, r+L), r = s+1+j*nbw, L = min(nbw, n-r).  The last generated
 * reflector is applied first.  H (not H^H) is applied; the paper's Q_i is
 * our H^H, its beta_i our conj(tau).
 *
 * Layouts (all device memory unless stated otherwise):
 *   Q    n x nev, column major, element (i, c) at Q[i + c*ldq], ldq >= n,
 *        overwritten in place.  Complex values are interleaved (re, im).
 *   hh   reflector vectors, slot-major in generation order (s ascending,
 *        then j ascending): slot k occupies hh[k*nbw .. k*nbw+nbw-1] with
 *        hh[k*nbw] = 1, then v[1..L-1], then zeros up to nbw.
 *        Slot offsets follow from (n, nbw) alone (see
 *        elpa_hh_num_reflectors / elpa_hh_slot_offset).
 *   tau  one scalar per slot, same element type as Q; tau = 0 is identity.
 *
 * Element types: ELPA_R64 (double), ELPA_R32 (float), ELPA_C64 (complex
 * double, 16-byte elements).  hh, tau and Q share the element type.
 *
 * Ownership and asynchrony: the caller owns every buffer.  Calls are
 * asynchronous on `stream` (a hipStream_t; NULL = the null stream) and keep
 * no pointer after returning; buffers must stay valid until the stream has
 * executed the work.  Calls on different streams are independent and
 * thread-safe.
 *
 * Workspace: a call takes its device workspace from the library's workspace
 * cache (hipMalloc'd blocks kept per device after use; see
 * elpa_hh_workspace_cached / elpa_hh_workspace_release).  A block is reused by
 * a later call on the same stream at once and by a call on another stream
 * only once the work that last used it has completed, so calls on different
 * streams never wait for each other.  While a stream is being captured into a
 * graph, the call's workspace is a stream-ordered allocation owned by the
 * graph.
 *
 * Errors: every call returns a status code, the counterpart of the error
 * out-argument that every call of the paper's C interface takes (Sec. 4.1,
 * the example use of the C interface); ELPA_OK = 0 is success.  Every
 * argument is validated before anything is enqueued; on an error nothing is
 * enqueued and Q is untouched.  n <= 1 or nev == 0 is a valid no-op (returns
 * ELPA_OK without touching any pointer).  A workspace that cannot be
 * allocated (more than the device holds, or the allocator refuses) returns
 * ELPA_ERR_NOMEM with nothing enqueued.
 */
#ifndef ELPA_HH_H
#define ELPA_HH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* element types */
enum { ELPA_R64 = 0, ELPA_R32 = 1, ELPA_C64 = 2 };

/* return codes (the paper's C interface reports errors through an error
   argument of every call, Sec. 4.1; here the return value carries them) */
enum {
    ELPA_OK = 0,
    ELPA_ERR_ARG = -1,    /* bad size, ldq < n, nbw < 1, null pointer */
    ELPA_ERR_DTYPE = -2,  /* unknown element type */
    ELPA_ERR_ALIGN = -3,  /* pointer not aligned to the element size */
    ELPA_ERR_NOMEM = -4,  /* device workspace could not be allocated (nothing enqueued) */
    ELPA_ERR_DEVICE = -5, /* HIP launch or runtime failure */
    ELPA_ERR_PLAN = -6,   /* explicit plan not valid for this problem (or a field out of range) */
    ELPA_ERR_ADMIT = -7   /* the problem's workspace exceeds the memory the call may use
                             (the fixed scratch of elpa_hh_trafo_noalloc) */
};

/* kernel family selection */
enum {
    ELPA_PATH_AUTO = 0,   /* library choice */
    ELPA_PATH_REF = 1,    /* one reflector at a time, any nbw */
    ELPA_PATH_STRIPE = 2, /* register-window stripe kernel, k sweeps fused, one lane
                             per column (all element types) */
    ELPA_PATH_SPLIT = 3,  /* register-window stripe kernel, k sweeps fused, two lanes
                             per column and reflectors pre-packed in consumption order,
                             real ones applied in pairs (real fp64, fp32 and complex
                             fp64, nbw 32 or 64; the default) */
    ELPA_PATH_WY = 4      /* compact-WY aggregation of 16 reflectors at a time,
                             applied by MFMA tiles to an LDS-resident window (real fp64
                             and fp32, nbw 32 or 64) */
};

/* order of the tiles of one launch over the workgroup ids (elpa_hh_plan.order).
   The one-launch batched schedule deals each problem's stripes to one die
   (dies balanced by work, longest problems first) unless ELPA_ORDER_LINEAR,
   which numbers the stripes problem by problem in id order. */
enum {
    ELPA_ORDER_AUTO = 0,   /* library choice */
    ELPA_ORDER_LINEAR = 1, /* tile (block m, stripe c) at id (m - m0) * stripes + c */
    ELPA_ORDER_XCD = 2     /* ids dealt to the 8 accelerator dies (XCDs) round robin
                              each get a contiguous run of tiles, so the tiles that
                              share a sweep block's reflectors share one die's L2 */
};

/*
 * Explicit execution plan (tests, autotuning).  Zero fields mean "library
 * default".  path: ELPA_PATH_*; k: sweeps fused per pass (the stripe kernels
 * keep an (nbw + k - 1)-row window per column in registers; each row loaded
 * from memory meets k reflectors); steps: chase steps per tile of the stripe
 * kernels' launch schedule (fewer steps: more tiles per launch, more
 * launches); order: ELPA_ORDER_* ; streams: the stripes (independent
 * column groups) are split into this many groups whose launch sequences run
 * on concurrent library-owned streams, forked from and joined back into the
 * caller's stream (1 = everything on the caller's stream; at most 8;
 * 0 = library choice, 2); batch: schedule of the two-lane kernel in batched
 * calls, ELPA_BATCH_* (single-problem calls ignore it).
 * Results do not depend on order, streams or batch.
 * A plan that leaves the kernel open (path AUTO, k, steps and batch 0, or
 * NULL) runs the tuner's plan for the problem's size class when there is one
 * (elpa_hh_tune, elpa_hh_tuner_*), with the caller's order and streams where
 * those are set.
 */
typedef struct {
    int32_t path;
    int32_t k;
    int32_t steps;
    int32_t order;
    int32_t streams;
    int32_t batch;
} elpa_hh_plan;

/* schedule of a batched call's two-lane group (elpa_hh_plan.batch) */
enum {
    ELPA_BATCH_AUTO = 0,       /* the one with the smaller modelled time (see
                                  elpa_hh_trafo_batched) */
    ELPA_BATCH_ONE_LAUNCH = 1, /* every (problem, stripe) unit in one launch */
    ELPA_BATCH_DIAGONAL = 2    /* every problem's diagonal launch sequence side by side */
};

/*
 * Number of reflector slots N_refl = sum_s J(s) of an n x n band matrix of
 * semi-bandwidth nbw (the length of tau; hh holds N_refl*nbw elements).
 * Returns 0 for n <= 1 and -1 for nbw < 1 or n < 0.
 */
int64_t elpa_hh_num_reflectors(int64_t n, int64_t nbw);

/*
 * Slot index of the first reflector of sweep s (sum of J(s') for s' < s),
 * 0 <= s <= n-1 (s = n-1 gives N_refl).  Returns -1 on bad arguments.
 */
int64_t elpa_hh_slot_offset(int64_t n, int64_t nbw, int64_t s);

/*
 * Q <- H(0,0) ... H(n-2, J-1) Q as described above, with the library's plan.
 * hh, tau, Q: device pointers; stream: hipStream_t or NULL.
 */
int elpa_hh_trafo(int64_t n, int64_t nev, int64_t nbw, const void *hh,
                  const void *tau, void *Q, int64_t ldq, int32_t dtype,
                  void *stream);

/*
 * Same operation with an explicit plan (host pointer, may be NULL = auto).
 * ELPA_ERR_PLAN if the plan cannot run this problem (e.g. a stripe kernel
 * that is not built for this nbw / k / dtype).
 */
int elpa_hh_trafo_plan(int64_t n, int64_t nev, int64_t nbw, const void *hh,
                       const void *tau, void *Q, int64_t ldq, int32_t dtype,
                       void *stream, const elpa_hh_plan *plan);

/*
 * One problem of a batched call (host struct; the pointers are device
 * pointers with the same meaning, layout and alignment rules as the
 * arguments of elpa_hh_trafo).
 */
typedef struct {
    int64_t n, nev, nbw, ldq;
    const void *hh;
    const void *tau;
    void *Q;
    int32_t dtype;
    int32_t reserved;
} elpa_hh_problem;

/*
 * Batched back-transformation: the same operation for every problem in
 * probs[0..count) (host array, read before the call returns), asynchronous on
 * `stream`.  Problems may differ in n, nev and ldq.  Problems that share
 * (dtype, nbw) and run the two-lane stripe kernel (ELPA_PATH_SPLIT, the
 * default where one is compiled) run as one group, in one of two schedules:
 *   - ONE kernel launch: every workgroup carries one 32-column stripe of one
 *     problem through all of that problem's reflectors (sweep blocks
 *     descending, chase steps ascending), the problems ordered by decreasing
 *     work so that the longest stripes start first; no workgroup waits for
 *     another.  For batches of many problems, whose stripes fill the device.
 *   - the diagonal launch sequence of every problem side by side (launch t
 *     runs launch t's tiles of every problem): for a few large problems,
 *     whose stripes alone would leave the device idle.
 * plan->batch picks one (ELPA_BATCH_*); by default the library models both
 * (resident wave slots, per-unit and per-launch work) and runs the faster,
 * the single launch unless it is modelled more than 10 % slower; an explicit
 * plan->steps selects the diagonal sequence.  A reflector-packing launch and
 * a layout-conversion launch run before and one conversion launch after,
 * each over all problems of the group.  Problems whose plan picks the
 * one-lane or compact-WY family run as that family's diagonal launch
 * sequence (all problems of the group side by side, one launch per diagonal);
 * problems without a compiled stripe kernel run through the reference kernel
 * one by one.  Groups run in order on the stream.  Every problem is validated
 * first; if any is invalid nothing is enqueued and the code of the first
 * invalid problem is returned.  The Q buffers of different problems must not
 * overlap.  plan may be NULL (library choice) and applies to every group
 * (one launch needs one compiled kernel, so k is uniform within a group).
 */
int elpa_hh_trafo_batched(const elpa_hh_problem *probs, int64_t count, void *stream,
                          const elpa_hh_plan *plan);

/*
 * Allocation-free variant of elpa_hh_trafo, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same operation, arguments, layouts and validation
 * as elpa_hh_trafo.  The two-lane stripe kernel (the library default, nbw 32
 * or 64) runs entirely on the caller's stream with its workspace (the
 * stripe-major copy of Q and the packed reflectors) in a fixed device array of
 * ELPA_HH_NOALLOC_SCRATCH_BYTES per device, which the library holds from load
 * until the process ends; nbw without a two-lane kernel runs the reference
 * kernel, which needs no workspace.  No device memory is allocated or freed
 * and no tuned plan is consulted (the library's default k for (dtype, nbw);
 * 1 stripe group).
 * Limit: a problem whose workspace (elpa_hh_workspace_bytes with plan
 * {ELPA_PATH_SPLIT, 0, 0, 0, 1, 0}) exceeds ELPA_HH_NOALLOC_SCRATCH_BYTES is
 * refused with ELPA_ERR_ADMIT, nothing enqueued (fp64 up to about
 * n = nev = 4400).
 * Every call on a device shares that device's scratch, which keeps the last
 * call's contents (each call writes every scratch byte it reads first):
 * calls that overlap on one device, from different streams or threads, RACE
 * and give wrong results; serialise them (one stream, or events).
 */
#define ELPA_HH_NOALLOC_SCRATCH_BYTES (256u << 20)
int elpa_hh_trafo_noalloc(int64_t n, int64_t nev, int64_t nbw, const void *hh,
                          const void *tau, void *Q, int64_t ldq, int32_t dtype,
                          void *stream);

/*
 * Prepared batched call, so that a batched back-transformation can be
 * captured into a HIP graph and replayed (a served SCF sequence repeats the
 * same call on the same buffers at every step).  elpa_hh_trafo_batched
 * stages its descriptor tables through host memory and allocates its
 * workspace on every call; a prepared batch does both once:
 *
 * elpa_hh_batch_create: validates the problems and plan exactly as
 *   elpa_hh_trafo_batched (same codes; a group whose kernel family has no
 *   prepared form, i.e. other than the two-lane kernel, gives ELPA_ERR_PLAN),
 *   builds the same schedules, allocates the device workspace and tables on
 *   the current device (hipMalloc; ELPA_ERR_NOMEM if it cannot) and copies the
 *   tables there before returning (synchronous).  A batch in which exactly
 *   one problem has work (n > 1, nev > 0) is prepared as the single-problem
 *   call elpa_hh_trafo_plan(..., plan) makes: the same kernel choice (the
 *   compact-WY kernel where the library picks it for a single call), plan
 *   and stripe groups on library streams forked from the run's stream; a
 *   family without a caller-workspace form (the one-lane kernel) gives
 *   ELPA_ERR_PLAN.  probs is read during the call; the problems' device
 *   pointers are kept and must stay valid until destroy.
 * elpa_hh_batch_run: the back-transformation of every problem of the batch
 *   on `stream`, with the results of elpa_hh_trafo_batched, or for a batch of
 *   one problem with work those of elpa_hh_trafo_plan (bitwise, same kernels
 *   and schedule): kernel launches and event fork/join only, no
 *   allocation, no copy, no host synchronisation, so it may be captured into
 *   a graph.  Runs of one batch share its workspace: they must not overlap
 *   (one stream, or ordered by events).  ELPA_ERR_ARG on another device.
 * elpa_hh_batch_bytes: device bytes the batch holds.
 * elpa_hh_batch_destroy: frees it (the caller makes sure no run is pending).
 */
typedef struct elpa_hh_batch elpa_hh_batch;
int elpa_hh_batch_create(const elpa_hh_problem *probs, int64_t count, const elpa_hh_plan *plan,
                         elpa_hh_batch **out);
int elpa_hh_batch_run(elpa_hh_batch *batch, void *stream);
int64_t elpa_hh_batch_bytes(const elpa_hh_batch *batch);
int elpa_hh_batch_destroy(elpa_hh_batch *batch);

/*
 * Device workspace (bytes) that elpa_hh_trafo_plan takes from the workspace
 * cache for one problem under `plan` (NULL = library choice): the stripe-major copy
 * of Q and, for paths 3 and 4, the packed reflectors.  0 for no-ops and the
 * reference path, -1 for invalid arguments or a plan that cannot run.  A
 * batched call allocates the sum over its problems plus small descriptor
 * tables.  For admission control by memory footprint (serving loops).
 */
int64_t elpa_hh_workspace_bytes(int64_t n, int64_t nev, int64_t nbw, int32_t dtype,
                                const elpa_hh_plan *plan);

/*
 * Workspace cache of the current device (see Workspace above):
 * elpa_hh_workspace_cached returns the device bytes the cache holds (blocks in
 * use and idle); elpa_hh_workspace_release frees the idle blocks whose last
 * use has completed and returns the bytes freed (it may wait for the device,
 * as hipFree does).  The cache keeps at most 8 GiB of idle blocks per device
 * before it frees the least recently used ones, and frees all idle blocks
 * before an allocation is reported as failed.  ELPA_ERR_DEVICE if there is no
 * current device.
 */
int64_t elpa_hh_workspace_cached(void);
int64_t elpa_hh_workspace_release(void);

/*
 * Upper bound of the device workspace of elpa_hh_trafo_batched on the same
 * arguments (the kernels a batched call picks, plus its descriptor and
 * schedule tables); -1 for invalid arguments or a plan that cannot run.
 */
int64_t elpa_hh_workspace_bytes_batched(const elpa_hh_problem *probs, int64_t count,
                                        const elpa_hh_plan *plan);

/*
 * Whether an explicit plan can run (n, nbw, dtype): 1 yes, 0 no.
 */
int elpa_hh_plan_supported(int64_t nbw, int32_t dtype, const elpa_hh_plan *plan);

/*
 * The kernel a call would run for a problem of this size: *out = the plan
 * (`plan` as given, or the tuner's for the size class where `plan` leaves
 * the kernel open) with path and k filled in by the library's choice
 * (path ELPA_PATH_REF and k 0 for the reference kernel).  batched != 0: as a
 * problem of elpa_hh_trafo_batched (whose choice prefers the kernels with a
 * one-launch form, and k = 96 at nbw = 32), else as elpa_hh_trafo_plan.
 * steps, order, streams and batch stay 0 where the library picks them at
 * launch.  ELPA_ERR_PLAN if `plan` cannot run, ELPA_ERR_ARG / _DTYPE for bad
 * arguments.  Host only, nothing enqueued.
 */
int elpa_hh_chosen_plan(int64_t n, int64_t nev, int64_t nbw, int32_t dtype, int32_t batched,
                        const elpa_hh_plan *plan, elpa_hh_plan *out);

/*
 * Kernel timing (benchmarks, tests).  While enabled on a host thread, every
 * call made from that thread on the device that was current at enable time
 * records HIP events around its main kernel sequence (the tile launches of
 * the stripe paths, the launch of the reference path) on the caller's stream,
 * and around each of those launches on the stream it runs on.
 * elpa_hh_profile_last waits for the latest such call's events and reports;
 * ELPA_ERR_ARG if no call was recorded since enabling.
 * elpa_hh_profile_enable(0) disables and releases the events.
 * With several stripe-group streams, launches overlap: sum_launch_ms /
 * kernel_ms is the average number of launches in flight.
 */
typedef struct {
    double kernel_ms;     /* event time of the whole main kernel sequence */
    int64_t launches;     /* main-kernel launches in that time */
    int32_t path;         /* ELPA_PATH_* that ran */
    int32_t k;            /* sweeps fused per pass (0: reference path) */
    int64_t steps;        /* chase steps per tile (0: reference path) */
    double sum_launch_ms; /* sum over launches of each launch's event time */
    int32_t streams;      /* stripe-group streams used */
    int32_t reserved;
} elpa_hh_profile;

int elpa_hh_profile_enable(int on);
int elpa_hh_profile_last(elpa_hh_profile *out);

/*
 * Plan tuner.  The library keeps a per-process cache of plans keyed by
 * (dtype, nbw, size class of n, size class of nev); size classes are quarter
 * octaves (floor(4 log2 x)), so sizes within about 19 % share a plan.  Calls
 * without an explicit plan (NULL, or a plan whose fields are all 0) use the
 * cached plan of their class when there is one, and so do the workspace
 * queries; batched calls do so per problem (problems whose plans pick
 * different kernels run as separate launch sequences, in order, which can be
 * slower for a batch than one uniform plan: see elpa_hh_tune_batched).
 *
 * elpa_hh_tune times candidate plans on a scratch copy of Q (Q itself is not
 * modified; the call allocates ldq*nev elements and waits for `stream`) and
 * caches and returns the fastest.  level 0: each kernel family's default k;
 * 1: every compiled k; 2: also explicit chase steps per tile; every candidate
 * with 1 and 2 stripe-group streams.  Same arguments and errors as
 * elpa_hh_trafo (n <= 1 or nev == 0: ELPA_ERR_ARG, nothing to tune).
 *
 * elpa_hh_tuner_set stores an explicit plan for a class (ELPA_ERR_PLAN if it
 * cannot run), elpa_hh_tuner_get reads it (1 found, 0 not), _size counts the
 * entries, _clear empties the cache.  elpa_hh_tuner_save / _load write and
 * read a text file ("elpa_hh_tuner 1", then one line per entry: dtype nbw
 * n_class nev_class path k steps order streams); a file that does not parse
 * or names a plan that cannot run is refused as a whole (ELPA_ERR_ARG) and
 * the cache is left as it was; loaded entries replace entries of the same key.
 */
int elpa_hh_tune(int64_t n, int64_t nev, int64_t nbw, const void *hh, const void *tau,
                 const void *Q, int64_t ldq, int32_t dtype, void *stream, int32_t level,
                 elpa_hh_plan *best);

/*
 * Batch tuner: times uniform plans (one plan for every problem, among those
 * that every problem of the batch can run in a batched call; for the two-lane
 * family both batched schedules, ELPA_BATCH_ONE_LAUNCH and
 * ELPA_BATCH_DIAGONAL) on scratch
 * copies of the problems' Q (the Q buffers are not modified; the call
 * allocates the sum of the spans ldq*(nev-1)+n and waits for `stream`) and
 * returns the fastest in *best, to be passed to elpa_hh_trafo_batched.  The
 * result is not cached: a batch's best plan depends on the whole mix of sizes
 * sharing the device, not on one problem's size class.  level as for
 * elpa_hh_tune.  Errors: ELPA_ERR_ARG for count <= 0, a NULL probs or level
 * out of range, otherwise those of elpa_hh_trafo_batched.
 */
int elpa_hh_tune_batched(const elpa_hh_problem *probs, int64_t count, void *stream,
                         int32_t level, elpa_hh_plan *best);
int elpa_hh_tuner_set(int32_t dtype, int64_t nbw, int64_t n, int64_t nev,
                      const elpa_hh_plan *plan);
int elpa_hh_tuner_get(int32_t dtype, int64_t nbw, int64_t n, int64_t nev, elpa_hh_plan *out);
int64_t elpa_hh_tuner_size(void);
void elpa_hh_tuner_clear(void);
int elpa_hh_tuner_save(const char *path);
int elpa_hh_tuner_load(const char *path);

/*
 * On-the-fly autotuning over a sequence of similar solves (Kus et al.,
 * Sec. 4.3: an SCF cycle solves many similar problems, so every solve can try
 * one candidate setting and the best one is kept for the rest).
 *
 * elpa_hh_autotune_setup: candidates for problems of this (n, nev, nbw,
 *   dtype): ELPA_AUTOTUNE_FAST = the kernel family only (each family's
 *   default k); ELPA_AUTOTUNE_MEDIUM = also the blocking parameters of the
 *   back-transformation (every compiled k, chase steps per tile 0/2/4/8/16,
 *   1 or 2 stripe-group streams).  `fixed` (may be NULL): its nonzero path,
 *   k, steps and streams fields are kept at that value and excluded from the
 *   search.  Returns NULL for invalid arguments or if no candidate can run.
 *   The state's two HIP events are created on the device current at its
 *   first step.
 * elpa_hh_autotune_step: one solve of the sequence, i.e. elpa_hh_trafo_plan
 *   on these arguments with the next candidate (the first step of a fresh
 *   state runs the first candidate untimed, as a warm-up), timed with events
 *   on `stream`; *tuning = 1 while candidates remain, 0 once every candidate
 *   has been timed (the call then runs the fastest).  The result of every
 *   step is the back-transformation itself, whichever candidate ran.  The
 *   timing of a step is read at the next step (or by _best / _save), so a
 *   step does not wait for the GPU.  Errors as elpa_hh_trafo_plan.
 * elpa_hh_autotune_best: the fastest timed candidate so far (waits for a
 *   pending timing); ELPA_ERR_ARG if none is timed yet.
 * elpa_hh_autotune_set_best: stores it in the plan cache for this size
 *   class (elpa_hh_tuner_set), so calls without a plan use it.
 * elpa_hh_autotune_save / _load: the state as text ("elpa_hh_autotune 1",
 *   the problem, the next candidate, then one line per candidate with its
 *   time or -1), so tuning can stop and resume in a later run; _load returns
 *   NULL for a file that does not parse.
 * elpa_hh_autotune_free: releases the state and its events.
 */
enum { ELPA_AUTOTUNE_FAST = 0, ELPA_AUTOTUNE_MEDIUM = 1 };
typedef struct elpa_hh_autotune_state elpa_hh_autotune_state;
elpa_hh_autotune_state *elpa_hh_autotune_setup(int32_t level, int64_t n, int64_t nev,
                                               int64_t nbw, int32_t dtype,
                                               const elpa_hh_plan *fixed);
int elpa_hh_autotune_step(elpa_hh_autotune_state *st, const void *hh, const void *tau,
                          void *Q, int64_t ldq, void *stream, int32_t *tuning);
int elpa_hh_autotune_best(elpa_hh_autotune_state *st, elpa_hh_plan *best);
int elpa_hh_autotune_set_best(elpa_hh_autotune_state *st);
int elpa_hh_autotune_save(elpa_hh_autotune_state *st, const char *path);
elpa_hh_autotune_state *elpa_hh_autotune_load(const char *path);
int64_t elpa_hh_autotune_candidates(const elpa_hh_autotune_state *st);
void elpa_hh_autotune_free(elpa_hh_autotune_state *st);

/* Static message for a return code (never NULL). */
const char *elpa_strerror(int code);

/* Library version string (never NULL). */
const char *elpa_hh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ELPA_HH_H */
