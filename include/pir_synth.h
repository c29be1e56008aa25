/*
 * pir_synth.h -- seeded synthetic inputs generated on the device.
 *
 * Not part of RowSel.  These calls let benchmarks and tests build
 * multi-GiB inputs in HBM without a host round trip.  The generator is
 * SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) used as a counter-based
 * stream, implemented here from its published definition:
 *
 *   mix64(z)     = z ^= z>>30; z *= 0xBF58476D1CE4E5B9;
 *                  z ^= z>>27; z *= 0x94D049BB133111EB; z ^ (z>>31)
 *   draw(key, i) = mix64(key + (i+1) * 0x9E3779B97F4A7C15)   (mod 2^64)
 *
 * `key` is computed by the caller.  Element values:
 *   uniform_mod(key, i, q) = (draw(key, i) * q) >> 64
 *   bits16(key, i)         = draw(key, i) & 0xFFFF
 * All calls are asynchronous on `hip_stream`; errors as in pir.h.
 */
#ifndef PIR_SYNTH_H
#define PIR_SYNTH_H

#include <stdint.h>
#include "pir.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Queries of clients [b0, b0 + nb) of a [B][2][D0][L][N] tensor: out_dev
 * receives [nb][2][D0][L][N]; the element at flat index f of the FULL
 * tensor is uniform_mod(key, f, q[l]) with l = (f / N) % L.  q is a host
 * array of L primes. */
pir_status pir_synth_query(uint32_t *out_dev, uint64_t key, uint32_t b0, uint32_t nb,
                           uint32_t d0, uint32_t nprimes, uint32_t n, const uint32_t *q,
                           void *hip_stream);

/* DB coefficients of rows [row0, row0 + nrows): out_dev receives
 * [nrows][D1][L][N]; element (k, n, l, t) = bits16(key, (k*D1 + n)*N + t),
 * identical for every limb l (a coefficient < 2^16 is its own residue). */
pir_status pir_synth_db_coeffs(uint32_t *out_dev, uint64_t key, uint32_t row0,
                               uint32_t nrows, uint32_t d1, uint32_t nprimes, uint32_t n,
                               void *hip_stream);

/* Raw draws: out_dev[i] = draw(key, i0 + i) for i < count (uint64). */
pir_status pir_synth_draw(uint64_t *out_dev, uint64_t key, uint64_t i0, uint64_t count,
                          void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PIR_SYNTH_H */
