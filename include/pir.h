/*
 * pir.h -- C ABI of the MI355X RowSel library (libpir.so).
 *
 * RowSel is the database-scanning stage of OnionPIR-style lattice PIR
 * (GPIR, sec. 2.2 "RowSel"): of the D0 selector ciphertexts a client sends,
 * every one encrypts 0 except row i*'s, which encrypts 1; the server
 * multiplies them with the D0 x D1 plaintext database to obtain D1
 * ciphertexts that encrypt row i*.  In the NTT domain this is, for every
 * point p of the L*N RNS/NTT points (sec. 2.4.1) and every prime q_l,
 * an independent matrix product mod q_l (sec. 2.3):
 *
 *     M_out[p][m][n] = sum_{k < D0} M_in0[p][m][k] * M_in1[p][k][n]  mod q_l
 *
 * with m over the 2*B ciphertext polynomials of B clients (multi-client
 * batching, sec. 3.1), k over the DB rows and n over the DB columns.
 *
 * Index conventions used by every call below:
 *   p = l*N + j      (l: prime index, j: NTT point), a polynomial is [L][N]
 *   m = 2*b + c      (b: client, c: ciphertext component, 0 = first supplied)
 *   query  tensor  [B][2][D0][L][N]  uint32, residues in [0, q_l)
 *   DB     source  [D0][D1][L][N]    uint32 (coefficients or NTT values)
 *   output tensor  [B][2][D1][L][N]  uint32, canonical residues in [0, q_l)
 * All arrays are dense, row-major, and live in device memory unless stated.
 *
 * Results are exact: every output word equals the mathematical sum reduced
 * into [0, q_l), independent of the path, tile or batch composition.
 *
 * Threading and streams: calls take a hipStream_t (as void*, NULL = the
 * legacy default stream) and are asynchronous on it unless stated; the
 * caller keeps inputs and outputs alive until the stream passes the call.
 * A pir_db may be read by concurrent calls; loading into it must not overlap
 * a RowSel call that reads it.
 *
 * Errors: every call returns pir_status; no C++ exception crosses the ABI.
 * Argument and shape checks fail with PIR_EINVAL before anything is
 * enqueued; pir_last_error() returns a thread-local message describing the
 * most recent failure on the calling thread.
 */
#ifndef PIR_H
#define PIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PIR_OK = 0,
    PIR_EINVAL = -1,        /* bad argument, shape or parameter */
    PIR_ENOMEM = -2,        /* device allocation failed */
    PIR_EDEVICE = -3,       /* a HIP runtime call failed */
    PIR_EBUSY = -4,         /* serving: request not admitted now (capacity) */
    PIR_EUNSUPPORTED = -5   /* valid request this library does not implement */
} pir_status;

#define PIR_MAX_PRIMES 4

/* Ring and database parameters.
 *   n       ring degree N: a power of two, 8 <= N <= 16384
 *   nprimes L: number of RNS primes, 1..4 (the paper uses four, sec. 2.4.1)
 *   q[l]    primes with q = 1 (mod 2N) (needed for the negacyclic NTT), each
 *           a 32-bit word.  Below 2^30 the VALU kernels keep up to fifteen
 *           60-bit products in one 64-bit sum.  With any prime of 2^30 or
 *           more (products up to 2^64, the 32-bit primes of sec. 2.4.1) the
 *           VALU kernels keep 64-bit sums that count their wraps and the INT8
 *           MFMA path splits each residue r as r or r - q, whichever lies in
 *           [-2155905152, 2139062143], the reach of four signed 8-bit digits
 *           (2^32 - 1 consecutive integers, so every q < 2^32 is served)
 *   d0, d1  DB rows (selector count) and columns, each 1..65536 */
typedef struct {
    uint32_t n;
    uint32_t nprimes;
    uint32_t q[PIR_MAX_PRIMES];
    uint32_t d0;
    uint32_t d1;
} pir_params;

typedef enum {
    PIR_DOMAIN_COEFF = 0,   /* source holds coefficients; the library NTTs them */
    PIR_DOMAIN_NTT = 1      /* source already holds NTT values in natural order */
} pir_domain;

typedef enum {
    PIR_PATH_AUTO = 0,      /* pick by batch size from the layouts present */
    PIR_PATH_VALU = 1,      /* 32x32->64-bit integer multiply-add kernels */
    PIR_PATH_MFMA_I8 = 2    /* exact signed 8-bit digit split on INT8 MFMA */
} pir_path;

/* Device layouts a DB can hold (bit flags for pir_db_create). Each takes
 * L*N*D0*D1*4 bytes of HBM (the MFMA one pads D0 up to a multiple of 64). */
#define PIR_LAYOUT_VALU 1u
#define PIR_LAYOUT_MFMA 2u

typedef struct pir_db pir_db;   /* opaque, device resident, library owned */

/* Allocate an empty DB on the current HIP device.
 * Validates every parameter (PIR_EINVAL with a message otherwise); `layouts`
 * is a non-empty subset of PIR_LAYOUT_*.  On success *out owns the device
 * memory until pir_db_free.  Database organisation: D0 x D1 records, each a
 * plaintext polynomial kept in the NTT domain (sec. 2.2, sec. 6 on the
 * NTT-domain storage); the internal layouts are transposed slot-major so
 * RowSel reads them coalesced (sec. 5.2.1: the DB layout is free because it
 * is transposed before any query arrives). */
pir_status pir_db_create(const pir_params *params, uint32_t layouts, pir_db **out);

/* Load DB rows [row0, row0 + nrows) from a device buffer `src_dev` laid out
 * [nrows][D1][L][N] (uint32).  PIR_DOMAIN_COEFF: values are coefficients
 * (any uint32; reduced mod q_l), transformed by the negacyclic NTT with
 * natural point order ahat_i = a(psi_l^(2i+1)), psi_l = g^((q_l-1)/2N),
 * g the smallest generator mod q_l (sec. 2.4.1).  PIR_DOMAIN_NTT: values
 * must be residues < q_l and are taken as they are.  The source is only
 * read; it may be freed once the stream passes the call.  Temporary device
 * memory of nrows*D1*L*N*4 bytes is used for COEFF input. */
pir_status pir_db_load_ntt(pir_db *db, const uint32_t *src_dev, uint32_t row0,
                           uint32_t nrows, pir_domain domain, void *hip_stream);

/* Copy the DB parameters out. */
pir_status pir_db_params(const pir_db *db, pir_params *out);

/* Layout flags actually present. */
uint32_t pir_db_layouts(const pir_db *db);

/* Release a DB (NULL is a no-op).  Synchronises the device first and drops
 * the cached grouped-call plans whose item lists name this DB (a hipGraph
 * that captured such a call must not be replayed afterwards; plans of other
 * DBs, and graphs over them, are unaffected). */
void pir_db_free(pir_db *db);

/* RowSel for B clients against one DB (sec. 2.2, sec. 2.3, sec. 5.1.1):
 *   out[b][c][n][l][j] = sum_k q[b][c][k][l][j] * DB_ntt[k][n][l][j] mod q_l
 * q_dev:  [B][2][D0][L][N] residues < q_l (larger values give unspecified
 *         results; PIR_VALIDATE=1 in the environment checks them and fails
 *         with PIR_EINVAL instead)
 * out_dev: [B][2][D1][L][N]; must not overlap q_dev.
 * B = 0 is a no-op.  `path` must name a layout the DB holds (PIR_EINVAL
 * otherwise); PIR_PATH_AUTO picks, when both layouts exist, the streaming
 * VALU kernel for B <= 2 (B = 1 when a prime is 2^30 or more, where each
 * client is its own pass over the DB) and the INT8 MFMA kernels above.  On
 * the MFMA path 2B rounded up to 32 rows picks the kernel: from 64 rows up
 * (17 clients and more, with D0 above 64) the query-resident one (units of
 * 64, 96 or 128 rows), else the tiled one; PIR_MFMA_KERNEL=qres or =tile in
 * the environment forces one (tuning and tests; the results are the same
 * bit for bit). */
pir_status pir_rowsel(const pir_db *db, const uint32_t *q_dev, uint32_t B,
                      uint32_t *out_dev, pir_path path, void *hip_stream);

/* Allocation-free RowSel, for callers that cannot allocate device memory:
 * code under hipGraph stream capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Computes exactly what pir_rowsel computes on the VALU
 * path (the streaming kernel), bit for bit, for 1 <= B <= 4 clients against a
 * DB holding the VALU layout; B = 0 is a no-op.  Its staging (the output's
 * size: L*N*D1*2B*4 bytes, or L*N*D1*2*4 with a prime of 2^30 or more, where
 * clients run one pass each) lives in a library-owned device array of
 * PIR_NOALLOC_SCRATCH_BYTES per GPU, held from library load until the process
 * ends; larger calls fail with PIR_EINVAL before anything is enqueued (e.g.
 * N = 4096, L = 2, D1 = 512 allows B <= 2).  The call allocates nothing:
 * no hipMalloc, no stream-ordered scratch, no events (kernel timing is not
 * recorded, PIR_VALIDATE is not applied).  Every call on one GPU uses that
 * GPU's one array: calls that overlap on a GPU (two streams, or two threads)
 * race and give undefined output; calls ordered on one stream are safe.
 * Arguments, layouts and stream semantics as for pir_rowsel. */
#define PIR_NOALLOC_SCRATCH_BYTES (64u << 20)
pir_status pir_rowsel_noalloc(const pir_db *db, const uint32_t *q_dev, uint32_t B,
                              uint32_t *out_dev, void *hip_stream);

/* RowSel on selector ciphertexts given in the coefficient domain, the form
 * query expansion produces them in (sec. 2.2): every query polynomial is
 * first taken to the NTT domain with the convention of pir_db_load_ntt
 * (ahat_i = a(psi^(2i+1)), natural order; sec. 2.4.1), then multiplied as
 * in pir_rowsel, whose output it equals bit for bit on the transformed
 * query.
 * q_coeff_dev: [B][2][D0][L][N] coefficients; limb l is read mod q_l (any
 *         uint32 value is accepted).  out_dev as for pir_rowsel and must not
 *         overlap q_coeff_dev.
 * One launch transforms the query into an NTT-domain copy in stream-ordered
 * scratch (the query's size), which the chosen path then reads as
 * pir_rowsel would.  Same path choice, errors and stream semantics as
 * pir_rowsel. */
pir_status pir_rowsel_coeff(const pir_db *db, const uint32_t *q_coeff_dev, uint32_t B,
                            uint32_t *out_dev, pir_path path, void *hip_stream);

/* First ColTor stage (sec. 2.2, ColTor; the external product of sec. 2.4.2):
 * for each of B clients and each pair of ciphertexts (columns 2t, 2t+1)
 *   out[b][t] = ct[b][2t] + RGSW_b [x] (ct[b][2t+1] - ct[b][2t])
 * with [x] the external product: both polynomials of the difference are
 * taken to the coefficient domain, every coefficient is rebuilt mod
 * Q = prod q_l (RNS reconstruction), centred into (-Q/2, Q/2] and cut into
 * `ell` digits of base z = 2^log2z (digits 0..ell-2 in [-z/2, z/2), the
 * last one the rest: within [-z/2, z/2 + 1] since z^ell > Q), and the
 * 2*ell digit polynomials, back in the NTT domain, multiply-accumulate
 * against the RGSW rows.  A bit-b RGSW thus keeps column 2t (b = 0) or takes
 * column 2t+1 (b = 1).  An unpaired last column (odd ncols) passes through.
 * ring:    n and the primes (d0, d1 are ignored); the same rules as
 *          pir_db_create, and L*N <= 16384 (the paper's N = 4096 with four
 *          limbs is the largest), else PIR_EUNSUPPORTED
 * ct_dev:  [B][2][ncols][L][N] NTT-domain residues < q_l (the layout of
 *          pir_rowsel's output; larger values give unspecified results, and
 *          PIR_VALIDATE=1 checks ct_dev and rgsw_dev and fails with
 *          PIR_EINVAL instead)
 * rgsw_dev: [B][2][ell][2][L][N]: row (p, i) is the ciphertext pair that
 *          multiplies digit i of input polynomial p, NTT domain
 * out_dev: [B][2][(ncols+1)/2][L][N]; must overlap neither input.
 * 1 <= ell <= 8, 1 <= log2z <= 30, z^ell > Q and 2^(log2z-1) + 1 below every
 * prime, else PIR_EINVAL.  B = 0 is a no-op; ncols >= 1 otherwise.
 * Stream-ordered scratch holds the digits (B * ceil(ncols/2) * 2 * ell * N
 * int32) and, for N >= 256, the RGSW rows permuted to the transforms'
 * register order (the size of rgsw_dev).  Asynchronous on hip_stream like
 * pir_rowsel; a tournament is one call per stage on the previous output. */
pir_status pir_coltor_stage(const pir_params *ring, const uint32_t *ct_dev, uint32_t B, uint32_t ncols,
                            const uint32_t *rgsw_dev, uint32_t log2z, uint32_t ell, uint32_t *out_dev,
                            void *hip_stream);

/* One RowSel instance of a grouped call. */
typedef struct {
    const pir_db *db;
    const uint32_t *q_dev;   /* [B][2][D0][L][N] of this instance's DB */
    uint32_t B;
    uint32_t *out_dev;       /* [B][2][D1][L][N] */
} pir_rowsel_item;

/* Many RowSel instances of uneven shape (own DB, own batch) at once (the
 * counterpart of the paper's per-prime, N-chunked launches under CUDA
 * Graphs, sec. 5.2.2, with the tile parameters of sec. 5.1.1 chosen per
 * instance).  Every item must satisfy the pir_rowsel contract and live on
 * the current device; outputs of distinct items must not overlap one another
 * or any query.  Results equal `count` separate pir_rowsel calls bit for
 * bit.  MFMA path (PIR_PATH_MFMA_I8, or AUTO when every DB holds the MFMA
 * layout): one query-ingest launch per item, the GEMM launches of the
 * item list's plan (below), one output-transpose launch per item.  VALU
 * path: the items' RowSel launches back to back.
 * The first MFMA call for a given list of (db, B) allocates a plan (device
 * work table and scratch, kept for reuse) and must not be made while the
 * stream is being captured (PIR_EINVAL); later calls with the same list only
 * enqueue kernels and may be captured into a hipGraph, with any query/output
 * pointers.  Up to 8 plans that were never used under capture are cached
 * (least recently used ones are released beyond that); a plan used under
 * capture is kept until one of its DBs is freed, so a captured graph stays
 * valid until pir_db_free of one of its items' DBs.
 * Plan: each item gets its own kernel and tile shape.  Candidates: the
 * fixed-shape tiled kernel (1 x 128x64 and 1 x 64x128 tiles, three stages of
 * 192 operand rows), the shaped tiled kernel (`points` NTT points side by
 * side x `rows` GEMM rows x `columns` DB columns: 1 x 128x64, 1 x 64x128,
 * 1 x 32x256, 1 x 256x32, 2 x 64x64, 2 x 32x128, 2 x 128x32, two stages of
 * 320 rows; those within 25% of the fewest padded output words) and the
 * query-resident kernel (units of 1 x 32x128, 1 x 64x128, 1 x 96x64 and
 * 1 x 128x64; items whose D0 spans at least two or three 64-row chunks).
 * When the plan is built every candidate runs three times, alone, on the
 * call's own inputs, timed on its stream (the first call therefore
 * synchronizes the stream), and the
 * fastest is kept.  The tiled items then run either in one persistent launch
 * per tiled kernel and tile family (three at most) or in one launch each,
 * whichever of the two schedules ran faster at plan build; each
 * query-resident item has a launch of its own.  PIR_AUTOTUNE=0 in the
 * environment keeps the candidate with the fewest padded words and the
 * shared launches without timing; PIR_GROUPED_SHAPE="points,rows,columns"
 * forces one tiled shape on every item; PIR_GROUPED_RING=deep, wide or qres
 * restricts the candidates to the fixed-shape, the shaped or (where D0
 * allows) the query-resident kernel; PIR_GROUPED_SCHED=shared or split
 * forces a schedule.  The results are the same bit for bit in every case. */
pir_status pir_rowsel_grouped(const pir_rowsel_item *items, uint32_t count,
                              pir_path path, void *hip_stream);

/* The plan an item list's MFMA calls run, as built by a previous
 * pir_rowsel_grouped call with the same list of (db, B): for item i,
 * tiles[5i .. 5i+4] = points, rows, columns of its tile or work unit, its
 * kernel (0 fixed-shape tiled, 1 shaped tiled, 2 query-resident) and 1 if
 * its GEMM has a launch of its own, 0 if it shares one (zeros for an item
 * with B = 0).  Only the (db, B) pairs of `items` are read; `tiles` holds
 * PIR_GROUPED_TILE_WORDS * count words.  PIR_EINVAL if no plan exists for
 * the list or a pointer is NULL. */
#define PIR_GROUPED_TILE_WORDS 5
pir_status pir_rowsel_grouped_tiles(const pir_rowsel_item *items, uint32_t count, uint32_t *tiles);

/* ---------------------------------------------------------------- serving */
/* A RowSel server over one resident DB with continuous batching.  The DB's
 * L*N/4 point groups are swept in `chunks` steps; every step runs the INT8
 * MFMA RowSel of ALL admitted clients on one chunk of points.  A request is
 * admitted into a free client slot at any step boundary and completes after
 * one full sweep (`chunks` consecutive steps), so requests that arrive while
 * others are on the GPU join the running batch instead of waiting for it to
 * drain.  Every output word depends only on its own client's query and the
 * DB, so a request's result is bit-identical alone and in any mix.  Needs a
 * DB with the MFMA layout.  (The paper reports batched throughput only,
 * Tab. 1; this adds admission, latency and the sweep schedule.) */
typedef struct pir_server pir_server;

typedef struct {
    uint32_t max_clients;   /* admission cap (slots), 1..4096; 0 = 256 */
    uint32_t chunks;        /* sweep steps per pass over the DB, 1..L*N/4; 0 = 16 */
    uint32_t pipeline;      /* steps kept in flight on the device, 1..4; 0 = 1 (a request
                             * admitted at a step boundary joins the next step; with
                             * 2, one step later, for the same throughput on the
                             * 32 GiB benchmark DB) */
    uint32_t max_waiting;   /* requests that may wait for a slot; an arrival that
                               finds this many waiting completes at once with
                               PIR_EBUSY (others go on); 0 = no bound */
    uint64_t hbm_budget;    /* device bytes the server may allocate; 0 = 90% of the
                               free memory at creation.  Admission capacity is the
                               number of client slots (64 MiB per client at
                               N = 4096, L = 2, D0 = 1024) that fit beside the step
                               staging; creation fails with PIR_ENOMEM if not one fits */
} pir_server_opts;

typedef struct {
    uint64_t id;               /* caller's tag, echoed in the completion; unique among
                                  the live (submitted, not yet returned) requests */
    const uint32_t *q_dev;     /* [2][D0][L][N] one client's selectors (residues < q_l) */
    uint32_t *out_dev;         /* [2][D1][L][N]; must not overlap another live request's */
    void *ready_event;         /* hipEvent_t recorded after the work that writes q_dev,
                                  on the producer's stream; the server's reads of the
                                  query are ordered after it (hipStreamWaitEvent at
                                  submission, so the event may be reused once the call
                                  returns).  NULL: q_dev is already complete on the
                                  device when pir_serve_step is called */
} pir_request;

typedef struct {
    uint64_t id;
    int32_t status;            /* PIR_OK, or this request's own error (others go on) */
    uint32_t reserved;
    double t_submit, t_admit, t_done;   /* seconds on pir_clock() */
} pir_completion;

typedef struct {
    uint32_t capacity;         /* client slots that fit the budget (<= max_clients) */
    uint32_t active;           /* clients currently admitted */
    uint32_t waiting;          /* requests queued for admission */
    uint32_t inflight;         /* steps on the device */
    uint64_t steps;            /* steps launched so far */
    uint64_t admitted;         /* requests admitted so far */
    uint64_t completed;        /* requests completed so far */
    uint64_t device_bytes;     /* bytes the server allocated */
} pir_server_stats;

/* Monotonic clock (seconds) used for the completion time stamps. */
double pir_clock(void);

pir_status pir_server_create(const pir_db *db, const pir_server_opts *opts, pir_server **out);

/* One turn of the serving loop; never blocks on the device.  Queues the
 * `n_arrivals` requests (stamped t_submit = now; a malformed request completes
 * at once with PIR_EINVAL, one that finds `max_waiting` requests waiting with
 * PIR_EBUSY), retires finished steps, admits waiting requests into free slots
 * in arrival order, and launches steps until `pipeline` are in flight (none
 * while no client is admitted).  Copies up to `cap` finished requests, oldest
 * first, into `done` and sets *n_done; the rest are kept for the next call.
 * The caller keeps each request's buffers alive until its completion is
 * returned.  An arrival whose id equals that of a live request (or of another
 * arrival of the same call) fails the whole call with PIR_EINVAL before
 * anything is queued.  Admission capacity is fixed when the server is
 * created (hbm_budget); requests beyond it wait.  Not thread safe: one caller
 * per server. */
pir_status pir_serve_step(pir_server *srv, const pir_request *arrivals, uint32_t n_arrivals,
                          pir_completion *done, uint32_t cap, uint32_t *n_done);

pir_status pir_server_get_stats(const pir_server *srv, pir_server_stats *out);

/* Waits for the device, drops pending requests and frees the server. */
void pir_server_destroy(pir_server *srv);

/* ---------------------------------------------------------------- helpers */
/* Negacyclic NTT / inverse NTT of `count` contiguous length-n polynomials
 * mod prime q < 2^32, q = 1 (mod 2n) (same convention as pir_db_load_ntt).  Not part of RowSel's
 * hot path: used to build inputs and to check results (client-side
 * decryption).  in_dev may equal out_dev. */
pir_status pir_ntt_forward(const uint32_t *in_dev, uint32_t *out_dev, uint32_t count,
                           uint32_t n, uint32_t q, void *hip_stream);
pir_status pir_ntt_inverse(const uint32_t *in_dev, uint32_t *out_dev, uint32_t count,
                           uint32_t n, uint32_t q, void *hip_stream);

/* Kernel timing, for benchmarks and profiling.  After pir_kernel_timing(1),
 * every pir_rowsel and pir_rowsel_grouped call records two HIP events on
 * its stream around its main kernel: the streaming kernel (VALU path,
 * B <= 4), the tiled kernel (VALU path, B > 4) or the persistent INT8 GEMM
 * (MFMA path; the up to three GEMM launches of a grouped call count as one);
 * with 32-bit primes the streaming kernel runs once per client, each launch
 * timed.  Every serving step's GEMM is timed the same way.  Query ingest, output transposes and scratch allocation
 * fall outside the events.  pir_kernel_time_read waits for every recorded
 * event, stores how many launches were timed and their summed duration in
 * milliseconds, and forgets them (PIR_EINVAL if an out pointer is NULL).
 * pir_kernel_timing(0) stops recording and drops unread events.  Off by
 * default; recording is process-wide, costs two event records per call,
 * and must not be enabled while a stream is being captured into a graph. */
pir_status pir_kernel_timing(int enable);
pir_status pir_kernel_time_read(uint32_t *launches, double *total_ms);

/* Thread-local description of the last failure on this thread ("" if none). */
const char *pir_last_error(void);

/* Library version string. */
const char *pir_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PIR_H */
