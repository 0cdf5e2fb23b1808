/* Measurement probe for the sampling kernels' memory roofline (libmoss_probe.so).
 *
 * Not part of the estimator.  The samplers spend their time on chains of dependent
 * loads at data-dependent places in the CSR and sampling tables (the neighbour picks
 * and the edge tests of Section 4.1.3 and Algorithms 1-4); what one GPU can sustain for
 * such loads over a buffer of the same size is the ceiling those kernels are held to.
 * This library measures it: every lane follows its own chain of loads, each load's
 * address a function of the value the previous one returned, uniformly spread over
 * the buffer.
 *
 * Every call is asynchronous on `stream` (a hipStream_t, NULL = the default stream),
 * takes device pointers, allocates nothing and returns 0 or a negative code:
 *   -1  bad argument (null pointer, zero size, grid or steps out of range)
 *   -2  the launch failed (hipGetLastError after it)
 */
#ifndef MOSS_PROBE_H
#define MOSS_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Fills buf[0..words) with 64-bit values that look uniformly random (the SplitMix64
 * output function of seed + i).  words >= 1. */
int moss_probe_fill(uint64_t* buf, uint64_t words, uint64_t seed, void* stream);

/* Dependent gathers: each lane t of the launch (blocks x 256 lanes) follows `chains`
 * chains side by side.  Chain c starts at a place given by (t, c) and then, `steps`
 * times, loads x = buf[j] and moves to j = floor((x ^ salt) * words / 2^64), where salt
 * is an odd constant of the chain (so that chains do not fall into one another).  A
 * chain's loads depend on one another, the chains of a lane do not, so a lane keeps
 * `chains` loads in flight: with one chain the probe measures the latency-bound rate,
 * with several the rate the memory system sustains for random lines.  Lane t writes
 * the sum of the values it loaded to out[t] (out holds blocks * 256 words), which
 * keeps the loads live.  blocks * 256 * chains * steps loads in all, each to a line
 * picked at random.  1 <= blocks <= 2^20, 1 <= steps <= 2^20, chains in {1, 2, 4, 8}. */
int moss_probe_gather(const uint64_t* buf, uint64_t words, uint32_t blocks, uint32_t steps, uint32_t chains,
                      uint64_t* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif
