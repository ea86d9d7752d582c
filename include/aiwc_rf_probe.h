/*
 * aiwc_rf_probe.h -- measurement probes of libaiwc_rf_probe.so (gfx950).
 *
 * Not part of the method: these calls measure hardware ceilings that the
 * tree-growing kernel is set against, and check one of its arithmetic shortcuts.  Its histogram build adds every in-bag row
 * of a searched node to one packed 64-bit LDS bin per candidate column (the
 * per-node (count, sum) histograms of the variance-reduction split search that
 * the model of Sec. III-B needs), so besides HBM bandwidth its second ceiling is
 * the rate at which the CUs retire LDS atomic adds.
 *
 * Same conventions as aiwc_rf.h: 0 or a negative AIWC_RF_E* code, host outputs
 * end in _host, `stream` is a hipStream_t passed as void* (NULL = default stream);
 * each call synchronizes the stream before it returns.
 */
#ifndef AIWC_RF_PROBE_H
#define AIWC_RF_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* LDS atomic add throughput of the whole device.
 *
 * `blocks` workgroups of 256 threads each give every wave a 256-bin histogram
 * in LDS and add 1 to it `iters` x 8 times per lane, with ds_add_u64 when
 * width_bits is 64 and ds_add_u32 when it is 32.  pattern 0: the 64 lanes of an
 * instruction hit 64 distinct consecutive bins (no bank conflicts); pattern 1:
 * every lane hits a pseudo-random bin (fixed per lane and unrolled position), the
 * histogram build's access pattern for uniformly spread codes.
 * adds_per_s_host: lane-adds per second over the timed launch (one warm-up launch
 * first); elapsed_ms_host: that launch's duration.  The sum of every histogram is
 * checked against blocks x 256 x iters x 8 (AIWC_RF_ERANGE if it differs).
 * EINVAL: blocks < 1, iters < 1, width_bits not 32 or 64, pattern not 0 or 1,
 * a null output pointer. */
int aiwc_rf_probe_lds_add(int32_t width_bits, int32_t pattern, int32_t blocks, int32_t iters,
                          double* adds_per_s_host, double* elapsed_ms_host, void* stream);

/* The tree-growing kernel's split-score division (a shortened IEEE divide
 * sequence, valid for numerators that are zero or in [1, 2^90] and denominators
 * in [1, 2^20]) against IEEE division, on `samples` quotients of the score's
 * domain: the square of an integer of a random bit length up to 41 over an
 * integer weight in [1, 2^18] or [1, 64], drawn from a counter hash of `seed`.
 * mismatches_host: the quotients whose bit patterns differ (0 expected).
 * EINVAL: samples outside [1, 2^40], a null output pointer. */
int aiwc_rf_probe_divide(int64_t samples, uint64_t seed, uint64_t* mismatches_host, void* stream);

/* Message of the calling thread's last failed probe call ("" after a success). */
const char* aiwc_rf_probe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AIWC_RF_PROBE_H */
