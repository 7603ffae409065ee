/*
 * rtmi_peaks.h -- microbenchmarks of the device rates the march's rooflines are quoted
 * against (librtmi_peaks.so, gfx950).
 *
 * The march has no dense contraction. Its bounds are memory-side: the record pass
 * gathers 36 bytes of j and kappa per ray-substep from L2 / the Infinity Cache (MALL) /
 * HBM, and the tile pass adds 8 deposits per ray-substep into a binary64 LDS tile. These
 * calls measure, on the current device, the peak of each such pattern with HIP events,
 * so that a benchmark can state an achieved fraction of a rate measured in the same run
 * rather than of a datasheet figure. They allocate and free their own buffers and
 * synchronise the device; they are measurement tools, not part of the march.
 *
 * Every call returns 0 or a negative code (-1 bad argument, -4 HIP failure) and writes
 * the best rate of `reps` timed launches to *rate. *bytes_or_ops (optional, may be NULL)
 * receives what one launch moved or performed, so that a counter run of the same call
 * can be checked against it.
 */
#ifndef RTMI_PEAKS_H
#define RTMI_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Device copy of `bytes` (16-byte loads and stores): bytes read + bytes written per
 * second. */
int32_t rtmi_peak_copy(int64_t bytes, int32_t reps, double* rate, double* bytes_or_ops);

/* Random whole-line gathers: every lane reads one 64-byte line (four 16-byte loads) at a
 * pseudo-random line of a `footprint`-byte table, `iters` times. Bytes gathered per
 * second. A footprint of a few MiB stays in each XCD's L2, ~128 MiB in the MALL, and
 * several GiB reach HBM. */
int32_t rtmi_peak_gather(int64_t footprint, int32_t iters, int32_t reps, double* rate,
                         double* bytes_or_ops);

/* LDS atomic adds (512-lane work-groups, three per compute unit as in the tile pass), the
 * lanes of an instruction on consecutive slots: kind 0 = binary64 (ds_add_f64), 1 = 64-bit
 * integer (ds_add_u64), 2 = binary32 (ds_add_f32); kind 3 = binary64 with every lane on a
 * pseudo-random slot of a 48 KB array (bank conflicts and occasional shared addresses, as
 * when lanes deposit along unrelated rays), 4 = the same in 64-bit integers, 5, 6, 7 =
 * kind 3 with only one lane in 2, 4 or 8 of each wavefront adding. Adds (of the lanes that
 * add) per second; -1 for another kind or an `iters` that is not a multiple of the slots
 * per lane. */
int32_t rtmi_peak_lds_atomic(int32_t kind, int32_t iters, int32_t reps, double* rate,
                             double* bytes_or_ops);

/* Global binary32 atomic adds without return: `scattered` = 0 gives consecutive lanes
 * consecutive addresses (16 lanes per 64-byte line), 1 puts every lane on its own
 * pseudo-random line of a `footprint`-byte buffer (at most 4 GiB). Adds per second. */
int32_t rtmi_peak_global_atomic(int64_t footprint, int32_t scattered, int32_t iters, int32_t reps,
                                double* rate, double* bytes_or_ops);

#ifdef __cplusplus
}
#endif

#endif /* RTMI_PEAKS_H */
