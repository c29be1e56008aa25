/* Drives the host side of libpir.so's C ABI through its argument checks and
 * error paths (no device work: every call here fails validation, or finds no
 * device, before anything is enqueued), for a build whose host code carries
 * AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status 0 when every
 * call returns the documented status and leaves a message. */
#include <stdio.h>
#include <string.h>

#include "pir.h"
#include "pir_peak.h"
#include "pir_synth.h"

#define EXPECT(call, st) do { pir_status r_ = (call); \
    if (r_ != (st)) { fprintf(stderr, "FAIL: %s returned %d\n", #call, (int)r_); return 1; } \
    if (r_ != PIR_OK && strlen(pir_last_error()) == 0) { fprintf(stderr, "FAIL: %s left no message\n", #call); return 1; } \
} while (0)

int main(void)
{
    pir_params p;
    memset(&p, 0, sizeof p);
    p.n = 4096; p.nprimes = 2; p.q[0] = 1073692673u; p.q[1] = 1073668097u; p.d0 = 16; p.d1 = 16;
    pir_db *db = NULL;
    pir_params bad = p;
    bad.n = 3000;
    EXPECT(pir_db_create(&bad, PIR_LAYOUT_VALU, &db), PIR_EINVAL);
    bad = p; bad.q[1] = 1073668099u;
    EXPECT(pir_db_create(&bad, PIR_LAYOUT_VALU, &db), PIR_EINVAL);
    bad = p; bad.nprimes = 5;
    EXPECT(pir_db_create(&bad, PIR_LAYOUT_VALU, &db), PIR_EINVAL);
    bad = p; bad.d0 = 0;
    EXPECT(pir_db_create(&bad, PIR_LAYOUT_VALU, &db), PIR_EINVAL);
    EXPECT(pir_db_create(&p, 0, &db), PIR_EINVAL);
    EXPECT(pir_db_create(NULL, PIR_LAYOUT_VALU, &db), PIR_EINVAL);
    EXPECT(pir_db_load_ntt(NULL, NULL, 0, 1, PIR_DOMAIN_NTT, NULL), PIR_EINVAL);
    EXPECT(pir_rowsel(NULL, NULL, 1, NULL, PIR_PATH_AUTO, NULL), PIR_EINVAL);
    EXPECT(pir_rowsel_coeff(NULL, NULL, 1, NULL, PIR_PATH_AUTO, NULL), PIR_EINVAL);
    EXPECT(pir_rowsel_grouped(NULL, 3, PIR_PATH_AUTO, NULL), PIR_EINVAL);
    uint32_t tiles[3];
    EXPECT(pir_rowsel_grouped_tiles(NULL, 1, tiles), PIR_EINVAL);
    EXPECT(pir_rowsel_grouped_tiles(NULL, 0, NULL), PIR_EINVAL);
    EXPECT(pir_coltor_stage(NULL, NULL, 1, 2, NULL, 22, 5, NULL, NULL), PIR_EINVAL);
    EXPECT(pir_coltor_stage(&p, NULL, 1, 2, NULL, 40, 5, NULL, NULL), PIR_EINVAL);   /* log2z > 30 */
    EXPECT(pir_coltor_stage(&p, NULL, 1, 2, NULL, 22, 0, NULL, NULL), PIR_EINVAL);   /* ell = 0 */
    EXPECT(pir_server_create(NULL, NULL, NULL), PIR_EINVAL);
    EXPECT(pir_serve_step(NULL, NULL, 0, NULL, 0, NULL), PIR_EINVAL);
    EXPECT(pir_server_get_stats(NULL, NULL), PIR_EINVAL);
    EXPECT(pir_ntt_forward(NULL, NULL, 1, 3000, 12289, NULL), PIR_EINVAL);
    EXPECT(pir_ntt_inverse(NULL, NULL, 1, 1024, 12289 + 2, NULL), PIR_EINVAL);
    EXPECT(pir_kernel_time_read(NULL, NULL), PIR_EINVAL);
    double d = 0;
    EXPECT(pir_peak_mfma_i8(0, 0, &d, &d, NULL), PIR_EINVAL);
    EXPECT(pir_peak_valu_mad64(1u << 25, &d, &d, NULL), PIR_EINVAL);
    EXPECT(pir_peak_hbm_read(NULL, 16, &d, NULL), PIR_EINVAL);
    EXPECT(pir_rowsel_noalloc(NULL, NULL, 1, NULL, NULL), PIR_EINVAL);
    pir_db_free(NULL);
    pir_server_destroy(NULL);
    printf("abi driver ok: %s\n", pir_version());
    return 0;
}
