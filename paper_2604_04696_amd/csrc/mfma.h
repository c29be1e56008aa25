// MFMA RowSel jobs: shared by the single, grouped and serving entry points.
#pragma once

#include "common.h"

namespace pir {

// Per-prime constants of the epilogue.
struct EpiQ {
    double qd, qinv, c32, c47, c48;   // q, 1/q, 2^32, 2^47 and 2^48 mod q in binary64
    uint32_t q, pad;
};

// Recombination variants of combine_classes (modarith.h): direct, split at
// 2^15 (primes below 2^30 with a large 2^32 mod q), and wide (primes of
// 2^30 or more: split at 2^16, 64-bit final conversion).
enum : int { RECOMB_DIRECT = 0, RECOMB_SPLIT = 1, RECOMB_WIDE = 2 };

// One RowSel instance on the MFMA path.  Its output tiles are numbered
// [tile0, tile0 + tiles) in the launch's global tile order.
struct MfmaJob {
    const int8_t *qd;      // query digit planes [L*N][4][nkc][mstride][64]
    const int8_t *dbd;     // DB digit planes    [L*N][4][nkc][d1][64]
    uint32_t *out;         // staging [points][mp][sstride] (see out_transpose_kernel)
    uint32_t m_rows, mp, d1, nkc, L, N;
    uint32_t mstride;      // rows of a query plane (>= mp)
    uint32_t g_begin;      // first point group (groups of four points) of this job
    uint32_t wm;           // waves along m: 4 (128 x 64 tiles) or 2 (64 x 128 tiles); in
                           // grouped launches 1, 2, 4 or 8 (see pts)
    uint32_t pts;          // grouped launches: points a tile computes side by side (1 or 2);
                           // the tile is pts x 32wm x 32wn with pts * wm * wn = 8 waves
    uint32_t nblk_m, nblk_n, groups, tile0, tiles;
    uint32_t split;        // recombination variant of the job's primes (RECOMB_*)
    uint32_t sstride;      // staging row stride: d1 rounded up to a multiple of 4 (16-byte rows)
    EpiQ q[PIR_MAX_PRIMES];
};


MfmaJob make_mfma_job(const pir_db &db, const int8_t *qd, uint32_t *out, uint32_t B, uint32_t tile0,
                      uint32_t wm);
uint32_t pick_wm(uint32_t B);
void launch_mfma_jobs(const MfmaJob &one, const MfmaJob *jobs_dev, uint32_t njobs, uint32_t total_tiles,
                      hipStream_t st);
// The tile-shape-per-job kernel (grouped launches and serving steps): one
// job by value (jobs_dev == NULL) or a device table of njobs jobs sorted by
// tile0; `split` is the recombination variant every job of the launch takes.
// deep: the three-stage 192-row ring (only the 1 x 128x64 and 1 x 64x128
// shapes), else the two-stage 320-row ring (every shape).
void launch_mfma_grouped(const MfmaJob &one, const MfmaJob *jobs_dev, uint32_t njobs, uint32_t total_tiles,
                         uint32_t split, bool deep, hipStream_t st);
// Tile shape for one job of mp rows and d1 columns (serving steps); deep: run
// it through launch_mfma_grouped's fixed-shape kernel.
void pick_shape(uint32_t mp, uint32_t d1, uint32_t *pts, uint32_t *wm, bool *deep);
// A job for that kernel in tile shape pts x 32wm x 32wn (pts * wm * wn = 8).
MfmaJob make_shaped_job(const pir_db &db, const int8_t *qd, uint32_t *out, uint32_t B, uint32_t pts, uint32_t wm);
// The query-resident kernel (rowsel_mfma_qres.hip) for mp <= 128 rows
// (larger mp in row blocks of the unit's height): unit shape 0 is 32 rows x
// 128 columns, 1 is 64 x 128, 2 is 96 x 64, 3 is 128 x 64 (shapes
// [0, qres_shape_count())).  Its query planes have mstride rows, at least
// the job's row blocks times the shape's rows.
uint32_t qres_shape_count();
uint32_t qres_shape_for(uint32_t mp);
// whether a job of mp rows and nkc 64-row chunks of k runs in it
bool qres_preferred(uint32_t mp, uint32_t nkc);
uint32_t qres_rows(uint32_t shape);
uint32_t qres_cols(uint32_t shape);
uint32_t qres_min_chunks(uint32_t shape);   // 64-row chunks of k the kernel needs at least
MfmaJob make_qres_job(const pir_db &db, const int8_t *qd, uint32_t mstride, uint32_t *stage, uint32_t B,
                      uint32_t shape);
void launch_mfma_qres(const MfmaJob &job, hipStream_t st);
// Staging row stride of a DB with d1 columns (16-byte aligned rows).
inline uint32_t staging_stride(uint32_t d1) { return (d1 + 3) / 4 * 4; }

void launch_query_digits(const pir_db &db, const uint32_t *q, uint32_t B, int8_t *qd, hipStream_t st);
void launch_query_digits_rows(const pir_db &db, const uint32_t *q, uint32_t rows, int8_t *qd,
                              uint32_t mstride, uint32_t row0, hipStream_t st);

}  // namespace pir
