/*
 * trig.h - C ABI of the MI355X trigger-station triplet selection library.
 *
 * Method (Singhal, Chattopadhyay, Friese, "Investigation of heterogeneous
 * computing platforms for real-time data analysis in the CBM experiment",
 * Sec. 3.2 "Algorithm"):
 *   1. form every triplet of hits with one hit from each of the three layers of
 *      the MUCH trigger station;
 *   2. fit each triplet together with the event vertex (0, 0) by a straight
 *      line through the vertex, separately in the x-z (bending) and y-z planes
 *      (x = m0 z, y = m1 z), and reject the triplet if the mean square
 *      deviation per degree of freedom exceeds the plane's threshold
 *      (0.03 for x-z, 0.025 for y-z);
 *   3. select the event if at least two triplets pass.
 * Input hits are grouped into events and carry coordinates (Sec. 3.2, last
 * paragraph; Sec. 5.3, trigger-station hits only and one coordinate array per
 * axis); the output is the per-event decision and the list of selected events
 * (Sec. 5.3, step 6).
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE memory unless a comment says "host".  The caller
 *     owns every buffer; the library never allocates, frees or synchronises
 *     inside trig_select.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *     is complete once that stream has been synchronised.
 *   - Return codes: TRIG_OK, or a negative TRIG_E* code; trig_strerror()
 *     describes a code, trig_last_error_detail() the last failure of the
 *     calling host thread.
 *
 * Floating point contract (the paper fixes none): decisions are taken in IEEE
 * binary32 with round-to-nearest-even, subnormals preserved and no fused
 * multiply-add, in the operation order below, so that an independent
 * implementation reproduces every count bit for bit.  Per plane c in {x, y},
 * for hits c_i, c_j, c_k of layers 0, 1, 2 (each line one binary32 rounding
 * per operation, left to right):
 *
 *   TRIG_TEST_MSD (default) - the fit of Sec. 3.2 step 2 written out: the
 *     least-squares slope of the line c = m z through the vertex, its
 *     residuals and their sum of squares Q:
 *         Szz = (z0*z0 + z1*z1) + z2*z2,   w = f32(1 / f64(Szz)),
 *         m = ((c_i*z0 + c_j*z1) + c_k*z2) * w,
 *         r_l = c_l - m*z_l,   Q = (r0*r0 + r1*r1) + r2*r2
 *   TRIG_TEST_MSD_BASIS - the same Q evaluated in an orthonormal basis of
 *     the plane orthogonal to z = (z0, z1, z2) (8 operations per triplet
 *     instead of 28; in exact arithmetic the same number, in binary32 a
 *     decision can differ from TRIG_TEST_MSD's within a few ulps of the cut):
 *       u = (z1, -z0, 0) / n01,   v = (z0 z2, z1 z2, -s01) / (n01 |z|),
 *       s01 = z0^2 + z1^2, n01 = sqrt(s01), |z| = sqrt(s01 + z2^2):
 *         a = U0*c_i + U1*c_j
 *         b = (V0*c_i + V1*c_j) + V2*c_k
 *         Q = a*a + b*b
 *     with U0 = f32(z1/n01), U1 = f32(-z0/n01), V0 = f32(z0 z2/d),
 *     V1 = f32(z1 z2/d), V2 = f32(-s01/d), d = n01 |z|, everything before the
 *     final rounding evaluated in binary64 in the order written.
 *   For both MSD tests the plane passes iff  f32(Q / ndf) <= msd_max[c]
 *   (a triplet is rejected only if its MSD is above the threshold).
 *   TRIG_TEST_SLOPE_WINDOW - s_l = c_l / z_l (binary32 division); the plane
 *     passes iff |s_j - s_i| < W_c and |s_k - s_i| < W_c.
 * A triplet passes iff both planes pass.  Every passing triplet is counted,
 * including triplets that share hits.
 */
#ifndef TRIG_H
#define TRIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRIG_ABI_VERSION 2u

/* Return codes. */
#define TRIG_OK 0
#define TRIG_EINVAL (-1)       /* bad argument (see trig_select) */
#define TRIG_EWORKSPACE (-2)   /* workspace missing or smaller than trig_workspace_bytes */
#define TRIG_EHIP (-3)         /* a HIP runtime call or kernel launch failed */
#define TRIG_EUNSUPPORTED (-4) /* flag/test combination not provided */

/* Per-event error values written to out_counts (accept is 0 for them). */
#define TRIG_COUNT_MALFORMED (-1) /* layer range reversed or outside [0, n_hits] */
#define TRIG_COUNT_OVERFLOW (-2)  /* n0*n1*n2 > INT32_MAX: count not representable */

/* Sticky bits OR-ed into *out_status (device) when such events occur. */
#define TRIG_STATUS_MALFORMED 1u
#define TRIG_STATUS_OVERFLOW 2u

/* Events in CSR form.  layer_offsets: device int32[3*n_events + 1]; the hits
 * of event e in layer l (l = 0, 1, 2 from the target outwards) are
 * [layer_offsets[3e+l], layer_offsets[3e+l+1]).  Offsets need not start at 0;
 * each event is checked on its own (0 <= o0 <= o1 <= o2 <= o3 <= n_hits). */
typedef struct {
    int32_t n_events;
    const int32_t *layer_offsets;
} trig_events_csr;

/* Hit coordinates, structure of arrays: device float32[n_hits] each, cm.
 * z is optional: NULL takes the layer positions of trig_params.z; otherwise
 * every hit carries its own z (staggered modules; the paper's hits carry a
 * position each, Sec. 3.2 last paragraph) and each triplet is fitted with
 * its hits' z:
 *   TRIG_TEST_MSD: Szz = (zi*zi + zj*zj) + zk*zk, w = 1 / Szz (binary32
 *     division), m = ((ci*zi + cj*zj) + ck*zk) * w, r_l = c_l - m*z_l,
 *     Q = (r0*r0 + r1*r1) + r2*r2;
 *   TRIG_TEST_SLOPE_WINDOW: s_l = c_l / z_l with each hit's z;
 *   TRIG_TEST_MSD_BASIS: not provided (TRIG_EUNSUPPORTED).
 * With per-hit z the batched, binned and autotuned forms run one wave per
 * event from HBM, pruning pairs on their slopes c / z (a bound that every
 * passing triplet meets, for events whose layer-0 and layer-1 z lie in
 * (0, inf)); the plain and persistent forms test every triplet. */
typedef struct {
    int32_t n_hits;
    const float *x;
    const float *y;
    const float *z;
} trig_hits;

/* Triplet test (see the floating point contract above). */
enum {
    TRIG_TEST_MSD = 0,
    TRIG_TEST_SLOPE_WINDOW = 1,
    TRIG_TEST_MSD_BASIS = 2
};

/* Execution form and output flags (bitwise OR).  Every form computes the same
 * counts and flags bit for bit, for every test. */
enum {
    TRIG_EXEC_PLAIN = 0u,       /* one wave per event, every triplet tested */
    TRIG_EXEC_PERSISTENT = 1u,  /* one persistent launch; alone: waves steal
                                   (event, pair-range) work units of the
                                   every-triplet loop from a global counter;
                                   with TRIG_EXEC_PRUNED: workgroups steal event
                                   blocks; with TRIG_EXEC_BINNED: workgroups
                                   steal event groups.  Needs workspace */
    TRIG_EXEC_BINNED = 2u,      /* binned form for high-multiplicity events:
                                   one wave per event sorts layers 1 and 2
                                   into cells of a slope-proportional key in
                                   LDS and tests only hits in the cells whose
                                   key interval can pass (MSD tests: bounds on
                                   the partial sums a and b that every passing
                                   triplet meets; window: the slope windows),
                                   with the interval ends rounded outwards;
                                   same counts.  Events with more than 256
                                   hits in layer 1 or 2 take the pruned path.
                                   Not with TRIG_EXEC_PRUNED or
                                   TRIG_EXEC_AUTOTUNE */
    TRIG_EXEC_AUTOTUNE = 4u,    /* run the form that trig_autotune recorded
                                   for this device, test and multiplicity
                                   class (floor(log2(mean hits per event))):
                                   the batched form with its launch shape
                                   (block_hits, block_waves, fill of
                                   block_events, block stealing on or off),
                                   or the binned form with or without
                                   stealing; without a record, the batched
                                   form with the built-in rule.  Non-zero
                                   block_* fields win over the record and
                                   select the batched form.  Needs the
                                   workspace of trig_workspace_bytes() for
                                   these flags */
    TRIG_OUT_COMPACT = 8u,      /* also write the ascending ids of accepted
                                   events; needs workspace */
    TRIG_EXEC_PRUNED = 16u,     /* batched form: workgroups stage blocks of
                                   consecutive events in LDS and complete only
                                   pairs that provably can pass (MSD tests: a
                                   bound on the pair's partial sum a that
                                   every passing triplet meets; window: the
                                   layer-1 window is part of the test); same
                                   counts */
    TRIG_ACCEPT_TWO_PARTICLES = 32u, /* acceptance by the trigger signature of
                                   Sec. 3.1, two particles pointing back to
                                   the target: accept iff two of the event's
                                   passing triplets have no hit in common
                                   (they differ in every layer's hit);
                                   min_triplets is not used.  out_counts keep
                                   the passing-triplet counts.  Any execution
                                   form; events with two or more passing
                                   triplets are then decided by one more
                                   kernel */
    TRIG_DECISION_ONLY = 64u    /* only the decision is wanted: out_counts[e]
                                   = min(count, K), K = min_triplets (2 with
                                   TRIG_ACCEPT_TWO_PARTICLES), errors
                                   unchanged, and an event's search may stop
                                   once its count reaches K; the accept flags
                                   are those of the full count */
};

typedef struct {
    uint32_t abi_version;     /* TRIG_ABI_VERSION */
    int32_t test;             /* TRIG_TEST_*; default TRIG_TEST_MSD */
    float z[3];               /* layer positions, cm, finite and > 0;
                                 default 400, 410, 420 */
    float msd_max[2];         /* MSD thresholds per degree of freedom, cm^2,
                                 x-z then y-z; >= 0, not NaN; default
                                 0.03f, 0.025f */
    int32_t ndf;              /* degrees of freedom of the fit, >= 1; default 2
                                 (three measurements, one slope) */
    float slope_window[2];    /* window test only: W_x, W_y >= 0; default
                                 0.005f, 0.005f */
    int32_t min_triplets;     /* accept iff count >= min_triplets (>= 0);
                                 default 2 */
    uint32_t flags;           /* TRIG_EXEC_* | TRIG_OUT_* */
    void *workspace;          /* device scratch owned by the caller, at least
                                 trig_workspace_bytes() bytes, 256-byte
                                 aligned; may be NULL when that is 0 */
    size_t workspace_bytes;
    int32_t *out_accepted_ids;  /* TRIG_OUT_COMPACT: device int32[n_events] */
    int32_t *out_n_accepted;    /* TRIG_OUT_COMPACT: device int32[1] */
    uint32_t *out_status;       /* optional device word; error bits are OR-ed
                                   in (never cleared by the library) */
    int32_t tile_pairs;         /* TRIG_EXEC_PERSISTENT without pruning: pairs
                                   per work unit (multiple of 64; 0 = library
                                   default) */
    int32_t block_events;       /* TRIG_EXEC_PRUNED: events per workgroup block
                                   (1..128; 0 = chosen from the mean number of
                                   hits per event) */
    int32_t block_hits;         /* TRIG_EXEC_PRUNED: LDS hit capacity of a
                                   workgroup: 1024, 2048 or 4096 (0 = chosen) */
    int32_t block_waves;        /* TRIG_EXEC_PRUNED: waves per workgroup: 1, 2
                                   or 4 (0 = chosen) */
    int32_t reserved[4];        /* must be zero */
} trig_params;

/* Fill *p (host) with the defaults above.  Returns TRIG_OK or TRIG_EINVAL for
 * a NULL pointer. */
int trig_params_init(trig_params *p);

/* Checks *p (host) the way trig_select does, ignoring the pointers that
 * TRIG_OUT_COMPACT needs; enqueues nothing.  Returns TRIG_OK, TRIG_EINVAL or
 * TRIG_EUNSUPPORTED. */
int trig_params_check(const trig_params *p);

/* Bytes of device workspace trig_select needs for this batch and these
 * parameters (0 for the plain form without compaction).  Host-only call: it
 * reads ev->n_events and p->flags, never device memory.  Returns 0 for invalid
 * arguments as well; trig_select then reports the error. */
size_t trig_workspace_bytes(const trig_events_csr *ev, const trig_params *p);

/* Count the passing triplets of every event and decide acceptance.
 *   ev, hits, p   host pointers to the descriptors above.
 *   out_counts    device int32[n_events]: passing triplets, or
 *                 TRIG_COUNT_MALFORMED / TRIG_COUNT_OVERFLOW.
 *   out_accept    device uint8[n_events]: 1 iff out_counts[e] >= min_triplets
 *                 (never for a negative count).
 *   stream        hipStream_t or NULL.
 * Errors (returned before anything is enqueued): TRIG_EINVAL for a NULL
 * required pointer, n_events < 0, n_hits < 0, an ABI mismatch, non-finite or
 * non-positive z, a negative or NaN threshold or window, ndf < 1,
 * min_triplets < 0, tile_pairs not a non-negative multiple of 64,
 * block_events outside 0..128, block_hits or block_waves not one of the listed
 * values, non-zero reserved fields; TRIG_EWORKSPACE; TRIG_EUNSUPPORTED.  TRIG_EHIP if a launch
 * fails.  n_events == 0 enqueues only the compaction count (0), if requested.
 * Data-dependent problems are reported per event (see TRIG_COUNT_*) without a
 * host synchronisation.  Concurrent calls on different streams need distinct
 * workspaces. */
int trig_select(const trig_events_csr *ev, const trig_hits *hits, const trig_params *p,
                int32_t *out_counts, uint8_t *out_accept, void *stream);

/* Bytes of the library's static device scratch used by trig_select_noalloc. */
#define TRIG_NOALLOC_SCRATCH_BYTES (4u << 20)

/* trig_select without a caller workspace and without any allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, outputs and errors
 * as trig_select, except that p->workspace must be NULL and
 * p->workspace_bytes 0 (else TRIG_EINVAL): the kernels use a static device
 * array of TRIG_NOALLOC_SCRATCH_BYTES that every GPU the library runs on
 * holds until the process ends (its address is looked up on the first call
 * on each device).  A batch whose trig_workspace_bytes() exceeds that size
 * gets TRIG_EWORKSPACE before anything is enqueued: with TRIG_EXEC_PERSISTENT
 * alone (8 bytes per event) about 520,000 events at most; every other form
 * up to n_events of 2^31 - 1.  The kernels reset what must start at zero;
 * the array keeps the last call's contents.  All calls on one GPU share the
 * array: calls that overlap in time on one GPU (other streams, other host
 * threads) race and must be serialised by the caller. */
int trig_select_noalloc(const trig_events_csr *ev, const trig_hits *hits, const trig_params *p,
                        int32_t *out_counts, uint8_t *out_accept, void *stream);

/* Result of trig_autotune (host). */
typedef struct {
    int32_t n_candidates;     /* launch shapes timed (0 for an empty batch) */
    int32_t mult_class;       /* multiplicity class of the batch */
    int32_t block_hits;       /* chosen batched-form shape (0 if binned) */
    int32_t block_waves;
    int32_t block_events;     /* events per block for this batch */
    int32_t persistent;       /* 1 if block stealing won */
    int32_t binned;           /* 1 if the binned form won */
    float ms_best;            /* mean kernel time of the chosen shape, ms */
    float ms_rule;            /* same for the built-in rule's shape */
} trig_autotune_result;

/* Times the batched form's launch shapes and the binned form on this batch
 * and records the fastest for the batch's multiplicity class (per device and
 * test), for later calls with TRIG_EXEC_AUTOTUNE.  Candidates: the built-in
 * rule's shape; block_hits 1024/2048/4096 x block_waves 2/4 x block fill
 * 0.5/0.7/0.85/1.0 of the LDS capacity (in mean event sizes) x block
 * stealing off/on; the binned form with and without stealing.  Each is timed `reps`
 * times (1..100) after one warm-up; every candidate computes the same
 * counts.  Arguments are those
 * of trig_select, with TRIG_EXEC_AUTOTUNE set in p->flags; block_* fields of
 * p are ignored while timing.  On return (the call synchronises `stream`)
 * out_counts, out_accept (and the compact outputs, if requested) hold the
 * result of an autotuned trig_select with the new record, and *out (may be
 * NULL) describes it.  Errors: those of trig_select; TRIG_EINVAL if
 * TRIG_EXEC_AUTOTUNE is not set or reps is out of range; TRIG_EHIP if an
 * event or synchronisation fails.  Not for concurrent use with other calls on
 * the same workspace. */
int trig_autotune(const trig_events_csr *ev, const trig_hits *hits, const trig_params *p,
                  int32_t *out_counts, uint8_t *out_accept, int32_t reps, trig_autotune_result *out,
                  void *stream);

/* Forgets every recorded launch shape (host); autotuned calls use the
 * built-in rule again. */
void trig_autotune_reset(void);

/* Autotune cache file (host).  trig_autotune_save writes every recorded
 * shape to the text file `path` (replacing it): a header line, then one line
 * per record with the device's architecture name and compute-unit count,
 * test, multiplicity class, form (batched or binned), block_hits,
 * block_waves, block fill and block stealing.  trig_autotune_load reads such
 * a file and records each line for every device of this process whose
 * architecture name and compute-unit count match (replacing the shape held
 * for that device, test and class); *n_recorded (may be NULL) receives the
 * number of (line, device) pairs recorded, 0 on a machine without a match.
 * The whole file is checked before anything is recorded.  Returns TRIG_OK,
 * or TRIG_EINVAL for a NULL path, a file that cannot be opened, read or
 * written, or a malformed line (detail in trig_last_error_detail). */
int trig_autotune_save(const char *path);
int trig_autotune_load(const char *path, int32_t *n_recorded);

/* The shape recorded for the current device, `test` and multiplicity class
 * (host).  *found = 1 and *out filled (block_events 0: it depends on the
 * batch; n_candidates, ms_best and ms_rule 0) if there is one, else
 * *found = 0.  Returns TRIG_OK, or TRIG_EINVAL for NULL pointers or a test
 * or class out of range. */
int trig_autotune_lookup(int32_t test, int32_t mult_class, int32_t *found, trig_autotune_result *out);

/* Profiling hook (host, per calling thread): the following trig_select calls
 * of this thread record `start` immediately before and `stop` immediately
 * after the launch of their dominant kernel (the triplet kernel of the chosen
 * form), on the call's stream, so that hipEventElapsedTime(start, stop) is
 * that kernel's duration.  Both are hipEvent_t handles created and owned by
 * the caller; NULL, NULL switches the hook off.  Returns TRIG_OK, or
 * TRIG_EINVAL if exactly one of them is NULL. */
int trig_set_kernel_events(void *start, void *stop);

/* Static description of a return code (host). */
const char *trig_strerror(int code);

/* Detail of the last failed call on this host thread (host), e.g. the HIP
 * error text; empty string if none. */
const char *trig_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* TRIG_H */
