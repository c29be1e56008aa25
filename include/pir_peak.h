/*
 * pir_peak.h -- issue-rate microbenchmarks of the units RowSel runs on.
 *
 * Not part of RowSel.  The paper measures its GPU's attainable bandwidth
 * and integer throughput with micro-benchmarks before placing its kernels on
 * the roofline (sec. 4.3); these calls do the same for the MI355X, so the
 * benchmark can report each kernel against a measured ceiling beside the
 * datasheet one.  Each call launches one kernel over the whole GPU on
 * `hip_stream`, times it with HIP events, waits for it and returns the
 * rate.  Clocks come from the shader's own counters read inside the kernel
 * (s_memtime, which counts shader clock cycles, against s_memrealtime, a
 * 100 MHz constant clock), averaged over every wave.  Errors as in pir.h.
 */
#ifndef PIR_PEAK_H
#define PIR_PEAK_H

#include <stdint.h>
#include "pir.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Register-only loop of v_mfma_i32_32x32x32_i8 (the instruction of the
 * RowSel MFMA path): 8 independent accumulators per wave, `iters`
 * iterations of 16 MFMAs each, two waves per SIMD on every CU.
 * random_operands = 0: all operands zero, nothing else in the loop; 1: the
 * operands change every iteration (a 32-bit LCG step per word and lane
 * between the MFMAs), so the matrix cores switch as they do on real data.
 * Outputs: *tops = 2*32*32*32 int8 operations per MFMA over the kernel's
 * event time, in 10^12 per second; *mhz = the average shader clock during
 * the loop.  1 <= iters <= 2^24. */
pir_status pir_peak_mfma_i8(uint32_t iters, int random_operands, double *tops, double *mhz, void *hip_stream);

/* Loop of v_mad_u64_u32 (the 32x32+64-bit multiply-add of the VALU RowSel
 * kernels): 16 independent chains per lane, `iters` iterations.  Outputs: *gops = multiply-adds per second / 10^9 (one per
 * lane per instruction), *mhz as above.  16 waves per CU.  1 <= iters <= 2^24. */
pir_status pir_peak_valu_mad64(uint32_t iters, double *gops, double *mhz, void *hip_stream);

/* Streaming read of `bytes` (a multiple of 16) of device memory at src_dev,
 * 16-byte non-temporal loads, XOR-reduced into one word per block (written
 * to a word inside the call's own scratch).  *gbs = bytes / event time, in
 * 10^9 bytes per second. */
pir_status pir_peak_hbm_read(const void *src_dev, uint64_t bytes, double *gbs, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PIR_PEAK_H */
