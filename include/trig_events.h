/*
 * trig_events.h - event building from a free-streaming hit stream: the step
 * before the station filter (trig_filter.h) and the selection (trig.h).
 *
 * The paper's selection runs on hits already grouped into events; its
 * outlook (Sec. 8) notes that the CBM data acquisition delivers
 * free-streaming data, hits with time stamps and no hardware trigger, so
 * that events have to be built from the hits' times first.  The paper gives
 * no algorithm.  This library builds events by time-gap clustering: in a
 * stream of hits ordered by time, an event is a maximal run of consecutive
 * hits in which no two neighbours are more than `gap` apart.  A new event
 * starts at the first hit and at every hit whose time exceeds the previous
 * hit's by more than `gap`.  Interactions closer in time than the gap (pile
 * up) form one event.  The output is the int64 event offsets over the
 * stream's order, which trig_raw_events (trig_filter.h) takes with the
 * stream's station numbers and x, y as they are.
 *
 * Same conventions as trig.h: device pointers unless noted, a hipStream_t
 * `stream` (NULL = null stream), asynchronous, no allocation and no host
 * synchronisation inside the call, TRIG_OK (0) or a negative trig.h code.
 */
#ifndef TRIG_EVENTS_H
#define TRIG_EVENTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status bits trig_build_events ORs into *out_status. */
#define TRIG_EVENTS_UNSORTED 1u  /* a hit's time is below the previous hit's: the stream is not in time
                                    order; such a hit never starts an event */
#define TRIG_EVENTS_CAPACITY 4u  /* more than out_capacity - 1 events: offsets past the capacity are not
                                    written (out_n_events still holds the number of events) */

/* Device workspace trig_build_events needs for n_hits hits (host-only call;
 * 0 for n_hits < 0): one bit per hit, 4 bytes per 4096 hits and 8 bytes per
 * 16384 hits, each part rounded up to 256 bytes. */
size_t trig_build_events_workspace_bytes(int64_t n_hits);

/* Build events from a time-ordered stream.
 *   t             int64[n_hits]: hit times, any integer unit (e.g. ns), non-decreasing.
 *   n_hits        number of hits, 0 <= n_hits <= 2^40.
 *   gap           largest time difference between neighbouring hits of one
 *                 event, >= 0 (same unit as t).  Hit h > 0 starts an event
 *                 iff t[h] > t[h-1] and t[h] - t[h-1] > gap, the difference
 *                 taken exactly (as unsigned 64-bit, which holds it whenever
 *                 t[h] > t[h-1]).
 *   out_offsets   int64[out_capacity]: out_offsets[e] = the first hit of
 *                 event e for e < E, out_offsets[E] = n_hits (E = number of
 *                 events: 0 for an empty stream, else at least 1).
 *   out_capacity  length of out_offsets, >= 1; E + 1 <= n_hits + 1 entries suffice.
 *   out_n_events  int64[1]: E (device; read it after the stream reaches the call).
 *   out_status    optional uint32: sticky bits, OR-ed in (above).
 *   workspace     trig_build_events_workspace_bytes(n_hits) bytes, 256-byte aligned.
 * Kernels: per 64 hits one ballot of the event starts (time differences of
 * neighbouring lanes) into a bit mask in the workspace and per-wave counts,
 * an exclusive scan of the workgroup counts, then each wave ranks its masks'
 * set bits and writes their hit indices.  The stream's times are read once.
 * Errors (returned before anything is enqueued): TRIG_EINVAL for a NULL
 * required pointer, n_hits outside [0, 2^40], gap < 0, out_capacity < 1, or a
 * workspace that is too small or not 256-byte aligned; TRIG_EHIP if a launch
 * fails.  Concurrent calls need distinct workspaces. */
int trig_build_events(const int64_t *t, int64_t n_hits, int64_t gap, int64_t *out_offsets, int64_t out_capacity,
                      int64_t *out_n_events, uint32_t *out_status, void *workspace, size_t workspace_bytes,
                      void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TRIG_EVENTS_H */
