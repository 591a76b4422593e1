/*
 * trig_serve.h - serving runtime of the trigger-station selection: timeslices
 * of different sizes arrive over time and are processed with continuous
 * batching on one GPU.
 *
 * The paper's deployment picture (Sec. 2 and Sec. 3.2): event data reach the
 * FLES compute nodes continuously, and on the GPU the transfer of one batch
 * can be hidden behind the computation of another (Sec. 5.3).  This runtime
 * does that for a stream of timeslices:
 *   - submit() copies a slice (host CSR offsets and x, y) into pinned staging
 *     owned by the server (large slices with a few host threads) and queues
 *     it;
 *   - a dispatcher thread admits queued slices first-come first-served as soon
 *     as a stream slot is free and the slice's device footprint (inputs,
 *     outputs, workspace) fits the server's HBM arena; each admitted slice is
 *     copied to the device, selected (trig_select on its own stream) and its
 *     results copied back, so the transfers and kernels of different slices
 *     overlap on the device;
 *   - poll() returns finished slices with their counts, flags, accepted ids
 *     and timestamps; release() returns their host memory.
 * A slice's results do not depend on what else is in flight.
 *
 * All pointers here are host pointers.  Return codes are those of trig.h plus
 * TRIG_EBUSY (staging memory or the pending queue is full: poll and retry)
 * and TRIG_ETIMEOUT (poll: nothing finished within the timeout).
 */
#ifndef TRIG_SERVE_H
#define TRIG_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "trig.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TRIG_EBUSY (-5)
#define TRIG_ETIMEOUT (-6)

typedef struct {
    size_t hbm_budget_bytes;     /* device arena for admitted slices (> 0) */
    size_t pinned_budget_bytes;  /* pinned host staging for queued and finished
                                    slices (> 0) */
    int32_t n_streams;           /* slices on the device at once, 1..64 */
    int32_t max_pending;         /* queued, not yet admitted slices (>= 1) */
    int32_t device;              /* HIP device ordinal */
    int32_t reserved;            /* must be zero */
    trig_params params;          /* selection parameters; the workspace and
                                    out_* fields are ignored (the server owns
                                    them) and TRIG_OUT_COMPACT is implied */
} trig_server_config;

typedef struct trig_server trig_server;

typedef struct {
    uint64_t ticket;
    int32_t status;              /* TRIG_OK or the trig_select error code */
    int32_t n_events;
    const int32_t *counts;       /* int32[n_events]; valid until release */
    const uint8_t *accept;       /* uint8[n_events] */
    const int32_t *accepted_ids; /* int32[n_accepted], ascending */
    int32_t n_accepted;
    uint32_t event_status;       /* OR of TRIG_STATUS_* bits of the slice */
    double t_submit;             /* seconds on the server's steady clock */
    double t_admit;
    double t_done;
} trig_slice_result;

typedef struct {
    uint64_t submitted, completed, rejected_busy;
    uint64_t events_completed;
    int32_t pending, in_flight, max_in_flight;
    size_t hbm_in_use, hbm_peak;
} trig_server_stats;

/* Creates a server (allocates the HBM arena and pinned staging, writes the
 * staging once so that its pages are in place, creates the streams and a
 * dispatcher thread).  Errors: TRIG_EINVAL for bad sizes or parameters
 * (trig_select's checks), TRIG_EHIP if an allocation fails. */
int trig_server_create(const trig_server_config *cfg, trig_server **out);

/* Queues one timeslice: offsets int32[3*n_events+1] and x, y float32[n_hits]
 * (host memory, read before the call returns).  *ticket identifies it.
 * TRIG_EBUSY: staging memory or the pending queue is full (nothing queued).
 * TRIG_EINVAL: bad arguments, or a footprint larger than the HBM arena. */
int trig_server_submit(trig_server *srv, const int32_t *offsets, const float *x, const float *y,
                       int32_t n_events, int32_t n_hits, uint64_t *ticket);

/* Returns one finished slice in *out (in completion order), waiting up to
 * timeout_ms (0 = do not wait, < 0 = wait without limit).  TRIG_ETIMEOUT if
 * none finished in time. */
int trig_server_poll(trig_server *srv, trig_slice_result *out, int32_t timeout_ms);

/* Frees the host buffers of a polled result.  TRIG_EINVAL for an unknown or
 * not yet polled ticket. */
int trig_server_release(trig_server *srv, uint64_t ticket);

/* Stops (paused != 0) or resumes admission of queued slices; slices already
 * on the device finish either way.  Lets a caller stage several slices and
 * release them together, or drain the device.  TRIG_EINVAL for NULL. */
int trig_server_pause(trig_server *srv, int32_t paused);

/* Current counters. */
int trig_server_stats_get(trig_server *srv, trig_server_stats *out);

/* Seconds on the server's steady clock (the clock of the result times). */
double trig_server_now(trig_server *srv);

/* Waits for every admitted slice, stops the dispatcher and frees everything.
 * Queued slices that were never admitted are dropped. */
int trig_server_destroy(trig_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* TRIG_SERVE_H */
