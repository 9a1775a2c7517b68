/*
 * navsim_probe: measurement helpers of libnavsim.so (not part of the step).
 *
 * The fused step's throughput is reported as a fraction of the LDS roofline
 * (the range scan of section 2.2.2 reads one bitmap word per grid cell it
 * visits, eq. 4-5).  The nominal LDS bandwidth is a datasheet figure; this
 * entry point measures what the chip actually delivers to a conflict-free
 * read pattern, so that the fraction can be quoted against both.
 *
 * Conventions are those of navsim.h (status codes, navsim_last_error()).
 */
#ifndef NAVSIM_PROBE_H
#define NAVSIM_PROBE_H

#include <stdint.h>

#include "navsim.h"

#ifdef __cplusplus
extern "C" {
#endif

/* LDS read bandwidth.  Launches `blocks` workgroups of `threads` threads (256,
 * 512 or 1024), each with a 64 KiB LDS buffer of 4096 16-byte words filled
 * with word i = (i * 2654435761, i ^ 0x9E3779B9, i + 7, ~i) (uint32, wrapping).
 * Thread t (t = threadIdx) runs `iters` iterations; iteration it reads the 16
 * words at index ((t + 64 it) mod 256) + 256 k, k = 0..15 (one 16-byte LDS
 * read each, the 64 lanes of a wavefront reading one aligned, contiguous
 * kilobyte per instruction), and xors them into a 4-word accumulator.  Thread
 * g = block * threads + t stores the xor of its accumulator's four words to
 * out[g].
 * One untimed launch, then `launches` launches timed with two HIP events on
 * the null stream of device `hip_device`.
 *   out_host           host [blocks * threads] or NULL: the stored words of the
 *                      last launch (for a check of what was read)
 *   ms_per_launch      host, receives the mean time per timed launch (ms)
 *   bytes_per_launch   host, receives blocks * threads * iters * 16 * 16
 * Errors: NAVSIM_E_INVALID_ARG (threads not 256/512/1024; blocks or iters
 * outside 1..2^20; launches outside 1..1000; NULL ms/bytes pointer),
 * NAVSIM_E_OOM, NAVSIM_E_HIP.  Allocates and frees its own device buffer;
 * synchronises the device. */
navsim_status navsim_probe_lds_read(int hip_device, int32_t threads, int32_t blocks,
                                    int32_t iters, int32_t launches, uint32_t *out_host,
                                    double *ms_per_launch, double *bytes_per_launch);

#ifdef __cplusplus
}
#endif

#endif /* NAVSIM_PROBE_H */
