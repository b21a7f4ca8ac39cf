/* Machine-peak probes of libnsl (gfx950): the measured denominators of the
 * roofline fractions the benchmark reports next to the datasheet ones.  They
 * are not part of the mapping step; each is one kernel launch on the stream,
 * asynchronous, timed by the caller (HIP events), and returns NSL_OK or an
 * NSL_E_* status of nsl.h (invalid arguments are rejected before any launch).
 */
#ifndef NSL_PEAKS_H
#define NSL_PEAKS_H

#include <stddef.h>
#include <stdint.h>

#include "nsl.h"

#ifdef __cplusplus
extern "C" {
#endif

/* HBM bandwidth: dst = src over `bytes` bytes (device pointers, 16-byte
 * aligned, bytes a multiple of 16); moves 2 * bytes. */
int nsl_peak_copy(const void* src, void* dst, size_t bytes, hipStream_t stream);

/* Random-gather rate: n_threads threads (a multiple of 256) each read
 * `loads` (a multiple of 16) 4-byte entries of `table` (2^log2_entries
 * entries, device memory) at pseudo-random indices, and write one word each
 * to out [n_threads].  A table of a few MB stays in L2, one of tens of MB in
 * the Infinity Cache: the access pattern of the hash-grid gather. */
int nsl_peak_gather(const uint32_t* table, int log2_entries, uint32_t* out, int n_threads, int loads,
                    hipStream_t stream);

/* Matrix-core rate: n_workgroups workgroups of 256 threads, each wave
 * running 8 independent accumulation chains of `iters` MFMAs,
 * v_mfma_f32_16x16x4_f32 (bf16 = 0: 2048 FLOP each) or
 * v_mfma_f32_16x16x32_bf16 (bf16 = 1: 16384 FLOP each); out receives one
 * float per thread (n_workgroups * 256). */
int nsl_peak_mfma(int bf16, float* out, int n_workgroups, int iters, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* NSL_PEAKS_H */
