/*
 * trig_probe.h - micro-benchmark kernels that measure the two ceilings the
 * selection kernels are compared against on the device they run on: the
 * fp32 vector-ALU instruction rate and the HBM copy bandwidth.  They also
 * calibrate hardware byte counters (a copy of known size).
 *
 * Same conventions as trig.h: device pointers, a hipStream_t `stream`
 * (NULL = null stream), asynchronous, TRIG_OK (0) or a negative code
 * (-1 invalid argument, -3 launch failure).
 */
#ifndef TRIG_PROBE_H
#define TRIG_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* fp32 VALU probe: n_blocks workgroups of 256 threads; each thread runs
 * `iters` iterations of 16 independent non-fused fp32 operations (8 v_mul_f32
 * + 8 v_add_f32, no FMA, no packed math) and writes one float to
 * out[global thread id] (device, n_blocks*256 floats) so that nothing is
 * optimised away.  fp32 ops per launch = n_blocks * 256 * iters * 16.
 * `seed` feeds the operands. */
int trig_probe_valu(int32_t n_blocks, int32_t iters, float seed, float *out, void *stream);

/* Copy probe: dst[i] = src[i] for i < n_vec4 (device float4 arrays, 16-byte
 * aligned), grid-stride loop over n_blocks workgroups of 256 threads.  Bytes
 * moved per launch = 32 * n_vec4. */
int trig_probe_copy(const void *src, void *dst, int64_t n_vec4, int32_t n_blocks, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TRIG_PROBE_H */
