/*
 * trig_filter.h - trigger-station filtering on the device: the step before
 * the selection of trig.h.
 *
 * An event arrives with all of its hits, from every detector station, each
 * tagged with its station number.  Only the hits of the three trigger layers
 * (the last muon station) enter the triplet search, about 90 of some 5000 per
 * event.  The paper filters them out on the host before the transfer to the
 * GPU (Sec. 5.3, the i3 implementation, about two orders of magnitude less
 * time per event than with all hits); here the hits are already in device
 * memory and the filter produces the selection's input in place: per event
 * the hits of trigger layers 0, 1 and 2, each layer in the order of the
 * input, as the CSR offsets and fp32 x/y arrays that trig_events_csr and
 * trig_hits describe.
 *
 * Same conventions as trig.h: device pointers unless noted, a hipStream_t
 * `stream` (NULL = null stream), asynchronous, no allocation and no host
 * synchronisation inside the call, TRIG_OK (0) or a negative trig.h code.
 */
#ifndef TRIG_FILTER_H
#define TRIG_FILTER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* All hits of a batch of events (host struct, device arrays). */
typedef struct {
    int32_t n_events;
    const int64_t *offsets;  /* int64[n_events + 1]: hits of event e are [offsets[e], offsets[e+1]) */
    int64_t n_hits;          /* length of station, x, y */
    const uint8_t *station;  /* uint8[n_hits]: station number of each hit */
    const float *x;          /* fp32[n_hits], cm */
    const float *y;          /* fp32[n_hits], cm */
} trig_raw_events;

/* Filter parameters and outputs (host struct, device arrays). */
typedef struct {
    uint8_t layers[3];            /* station numbers of trigger layers 0, 1, 2; distinct */
    uint8_t reserved;             /* must be 0 */
    int32_t out_capacity;         /* length of out_x and out_y, in hits (>= 0) */
    int32_t *out_layer_offsets;   /* int32[3*n_events + 1]: the trig_events_csr offsets */
    float *out_x;                 /* fp32[out_capacity] */
    float *out_y;                 /* fp32[out_capacity] */
    uint32_t *out_status;         /* optional uint32: sticky bits, OR-ed in (see below) */
    void *workspace;              /* trig_filter_workspace_bytes(n_events) bytes, 256-byte aligned */
    size_t workspace_bytes;
} trig_filter_params;

/* Status bits the filter ORs into *out_status. */
#define TRIG_FILTER_MALFORMED 1u  /* an event range not within [0, n_hits], decreasing or longer than
                                     INT32_MAX hits: the event keeps no hit */
#define TRIG_FILTER_CAPACITY 4u   /* more trigger hits than out_capacity (or than INT32_MAX): hits past
                                     the capacity are not written, and the offsets past it are not valid */

/* Device workspace trig_filter_stations needs for n_events events (host-only
 * call; 0 for n_events < 0): per event 16 bytes of layer and record counts
 * and 512 bytes of window records (128 records of 16 bytes per 4 events),
 * plus 8 bytes per 16 events. */
size_t trig_filter_workspace_bytes(int32_t n_events);

/* Keep the hits of the trigger layers, event by event.
 *   ev  host pointer to the batch description above.
 *   p   host pointer to the parameters and output pointers above.
 * Afterwards (once the stream has reached it) out_layer_offsets[3e + l] is
 * the index in out_x/out_y of the first hit of event e in trigger layer l,
 * out_layer_offsets[3*n_events] the total, and the hits of each (event,
 * layer) keep their input order.  Kernels: per-event counts of the three
 * layers and records of the 32-hit windows that hold trigger hits (their
 * start and per-layer bit masks; one pass over the station numbers), an
 * exclusive scan of the workgroup totals, then a stable scatter of the
 * trigger hits through the records (x and y read for trigger hits only).
 * The events of a group of 4 (events w, w + 4, w + 8, w + 12 of each 16)
 * that need more than 128 records together are scattered from a second pass
 * over their station numbers instead.
 * Errors (returned before anything is enqueued): TRIG_EINVAL for a NULL
 * required pointer, n_events < 0, n_hits < 0, equal layer numbers, a non-zero
 * reserved field, out_capacity < 0, or a workspace that is too small or not
 * 256-byte aligned; TRIG_EHIP if a launch fails.  n_events == 0 writes
 * out_layer_offsets[0] = 0 only.  Concurrent calls need distinct workspaces. */
int trig_filter_stations(const trig_raw_events *ev, const trig_filter_params *p, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TRIG_FILTER_H */
