/*
 * mcrt_probes.h -- probes of the gfx950 memory system that the roofline of
 * the photon-package life cycle is measured against (libmcrt_probes.so).
 *
 * The life cycle's walks gather one density value per cell crossing from
 * grids that live in L2, in the MALL or in HBM, and its tallies take FP64
 * atomic adds at scattered cells; these probes time the same access
 * patterns in isolation, with HIP events on the caller's stream:
 *   MCRT_PROBE_STREAM_READ       read buf once, 16-byte loads, in order
 *   MCRT_PROBE_GATHER            n_ops 4-byte loads at uniformly random
 *                                indices of buf (float elements), four in
 *                                flight per thread
 *   MCRT_PROBE_ATOMIC_SCATTERED  n_ops FP64 atomic adds (no return value) at
 *                                uniformly random indices of buf (double
 *                                elements)
 *   MCRT_PROBE_ATOMIC_COALESCED  n_ops FP64 atomic adds in which the 64
 *                                lanes of a wavefront add to 64 consecutive
 *                                doubles of a random 512-byte-aligned block
 * Indices come from a 64-bit mixing function of the op number and are
 * reduced modulo the element count, which must be a power of two for the
 * gather and the atomics (buf_bytes / 4 or / 8, at least 64 elements); the
 * streaming read takes any multiple of 16 bytes.  buf is the caller's device
 * memory; the atomics add 1.0 to its elements.  The probe runs once
 * untimed, then `reps` times; *ms_host receives the average milliseconds of
 * one run.  Returns 0, -1 for invalid arguments (nothing launched) or -3
 * for a HIP error.  Not part of the transport path.
 */
#ifndef MCRT_PROBES_H
#define MCRT_PROBES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCRT_PROBE_STREAM_READ 0
#define MCRT_PROBE_GATHER 1
#define MCRT_PROBE_ATOMIC_SCATTERED 2
#define MCRT_PROBE_ATOMIC_COALESCED 3

int mcrt_probe(int kind, void *buf_dev, uint64_t buf_bytes, uint64_t n_ops, int reps, double *ms_host,
               void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MCRT_PROBES_H */
