/*
 * ecc_probe.h -- measurement probe shipped in libecc.so beside the engine
 * (include/ecc.h).  Not part of the consistency method: it measures the
 * bandwidth the memory hierarchy gives 16-byte gathers, the access the
 * forward kernel makes per view and plane, so that the kernel's gather rate
 * can be set against a measured peak of the level that serves it.
 */
#ifndef ECC_PROBE_H
#define ECC_PROBE_H

#include <stdint.h>

#include "ecc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Launches n_blocks workgroups of 256 threads on `stream` (asynchronous);
 * every thread issues `iters` 16-byte loads from buf_dev (device, `bytes`
 * bytes, a power of two from 1 KiB to 64 GiB, contents arbitrary, 16-byte
 * aligned) at offsets drawn from a
 * counter-based hash of (thread, iteration), and writes the sum of what it
 * read to out_dev[thread] (device, n_blocks * 256 floats, overwritten).
 *   pattern 0: each thread an independent random 16-byte element (a
 *              wavefront's 64 loads touch 64 cache lines);
 *   pattern 1: each wavefront one random 1 KiB block per iteration, thread i
 *              of the wavefront its i-th 16 bytes (contiguous).
 * Gathered bytes per launch = 16 * iters * 256 * n_blocks.  iters: a
 * multiple of 4 in [4, 4096]; n_blocks in [1, 2^20].
 * Errors: ECC_E_ARG (NULLs, sizes, pattern), ECC_E_HIP. */
ecc_status ecc_probe_gather(const void *buf_dev, uint64_t bytes, int32_t pattern, int32_t iters, int32_t n_blocks,
                            float *out_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ECC_PROBE_H */
