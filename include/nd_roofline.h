/*
 * nd_roofline.h -- measured memory ceilings of the device, for reporting the
 * hot path's kernels as a fraction of what the hardware can sustain.
 *
 * Not part of the decomposition: the peel and count kernels are bound by
 * random 16-byte table probes and random 32-bit atomic updates, so their
 * roofline is set by these rates rather than by streaming bandwidth.
 */
#ifndef ND_ROOFLINE_H
#define ND_ROOFLINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double copy_gbs;           /* coalesced device copy, read + write GB/s */
  double gather16_gops;      /* random 16-byte loads per ns (G/s) over table_bytes */
  double atomic_ret_gops;    /* random returning u32 atomic adds, G/s, over count_bytes */
  double atomic_noret_gops;  /* random non-returning u32 atomic adds, G/s */
} nd_roofline;

/* Runs the four probes on the current HIP device on `hip_stream`, with
 * buffers of table_bytes (gathers) and count_bytes (atomics), allocated and
 * freed inside the call.  Returns 0 on success, 5 if the buffers cannot be
 * allocated, 6 on a HIP error. */
int nd_roofline_measure(uint64_t table_bytes, uint64_t count_bytes, void *hip_stream,
                        nd_roofline *out);

#ifdef __cplusplus
}
#endif
#endif /* ND_ROOFLINE_H */
