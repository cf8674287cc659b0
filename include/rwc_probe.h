/*
 * rwc_probe.h -- measurement kernels that bound the FastWalk sampler from above.  They are
 * not part of the method; bench.py uses them to place the sampler against what the memory
 * system delivers for its access pattern.
 *
 * Same conventions as rwc.h: device pointers owned by the caller, `stream` is a hipStream_t,
 * return 0 or a negative rwc_status.  Both calls synchronise `stream` to time themselves.
 */
#ifndef RWC_PROBE_H
#define RWC_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Random-access gather roofline: `lanes` independent chains, each doing `chain_len`
 * dependent 8-byte loads at uniformly random word indices of table_dev[0, words); the next
 * index depends on the loaded value (as a walker's next state word depends on the current
 * one).  *ms_out receives the kernel time; accesses/s = lanes * chain_len / time.
 *   sink_dev  uint64 [lanes] scratch written only to keep the loads live. */
int rwc_probe_random_gather(const uint64_t* table_dev, uint64_t words, int64_t lanes, int32_t chain_len,
                            uint32_t seed, uint64_t* sink_dev, float* ms_out, void* stream);

/* Streaming copy of `words` 8-byte words (coalesced), the reference for HBM byte counters
 * and for the streaming bandwidth.  *ms_out receives the kernel time. */
int rwc_probe_copy(const uint64_t* src_dev, uint64_t* dst_dev, uint64_t words, float* ms_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RWC_PROBE_H */
