/*
 * Calls the host-side validation paths of the HIP library's C ABI
 * (include/oi.h): malformed graphs, null handles, out-of-range arguments.
 * Built with AddressSanitizer and UndefinedBehaviorSanitizer on the host
 * side (tests/test_sanitizers.py); needs no GPU.  Exits 0 when every call
 * returns the documented status.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "oi.h"

static int fails = 0;
#define EXPECT(call, want)                                                               \
    do {                                                                                 \
        oi_status got_ = (call);                                                         \
        if (got_ != (want)) {                                                            \
            fprintf(stderr, "line %d: %s gave %d, expected %d\n", __LINE__, #call, (int)got_, \
                    (int)(want));                                                        \
            ++fails;                                                                     \
        }                                                                                \
    } while (0)

int main(void)
{
    int64_t rp[4] = {0, 1, 2, 2}, rp_dec[4] = {0, 2, 1, 2}, rp_off[4] = {1, 1, 2, 2};
    int32_t col[2] = {1, 2}, col_bad[2] = {1, 3};
    float p[2] = {0.5f, 0.5f}, p_bad[2] = {0.5f, 1.5f};
    oi_graph* g = NULL;
    EXPECT(oi_graph_create(3, 2, rp, col_bad, p, 0, NULL, &g), OI_EINVAL);
    EXPECT(oi_graph_create(3, 2, rp, col, p_bad, 0, NULL, &g), OI_EINVAL);
    EXPECT(oi_graph_create(3, 2, rp_dec, col, p, 0, NULL, &g), OI_EINVAL);
    EXPECT(oi_graph_create(3, 2, rp_off, col, p, 0, NULL, &g), OI_EINVAL);
    EXPECT(oi_graph_create(0, 0, rp, col, p, 0, NULL, &g), OI_EINVAL);
    EXPECT(oi_graph_create(3, (int64_t)1 << 32, rp, col, p, 0, NULL, &g), OI_EINVAL);
    EXPECT(oi_graph_create(3, 2, NULL, col, p, 0, NULL, &g), OI_EINVAL);
    EXPECT(oi_graph_create(3, 2, rp, col, p, 0, NULL, NULL), OI_EINVAL);
    if (g != NULL) {
        fprintf(stderr, "a rejected graph was returned\n");
        ++fails;
    }
    if (oi_last_error() == NULL || strlen(oi_last_error()) == 0) {
        fprintf(stderr, "no error message\n");
        ++fails;
    }

    int32_t seeds[1] = {0};
    int64_t off[2] = {0, 1};
    uint32_t qids[1] = {0};
    uint64_t u64a, u64b;
    double d;
    float f;
    int64_t l;
    oi_result r;
    oi_timing t;
    EXPECT(oi_graph_set_probs(NULL, p, 0), OI_EINVAL);
    EXPECT(oi_graph_set_theta(NULL, p, 0), OI_EINVAL);
    EXPECT(oi_graph_get_probs(NULL, &f), OI_EINVAL);
    EXPECT(oi_set_stream(NULL, NULL), OI_EINVAL);
    EXPECT(oi_stage1_table(NULL, seeds, 1, 0, &l, &d, NULL, NULL, NULL, NULL), OI_EINVAL);
    EXPECT(oi_estimate(NULL, 0, seeds, 1, 0.1, 0.1, OI_MODE_SOIEA, 1, &r), OI_EINVAL);
    EXPECT(oi_estimate_batch(NULL, 1, off, seeds, qids, 0.1, 0.1, OI_MODE_SOIEA, 1, &r), OI_EINVAL);
    EXPECT(oi_timing_enable(NULL, 1), OI_EINVAL);
    EXPECT(oi_timing_get(NULL, &t), OI_EINVAL);
    EXPECT(oi_set_tuning(NULL, 0, 0, 0, 0, 0), OI_EINVAL);
    EXPECT(oi_set_routing(NULL, 0, 0), OI_EINVAL);
    EXPECT(oi_set_pipeline(NULL, 1), OI_EINVAL);
    EXPECT(oi_set_stage1_skip(NULL, 100), OI_EINVAL);
    EXPECT(oi_set_stage1_skip_cost(NULL, 8.0), OI_EINVAL);
    EXPECT(oi_set_first_level(NULL, 1), OI_EINVAL);
    EXPECT(oi_gather_probe(NULL, 1024, 0, &u64a, &u64b, &d), OI_EINVAL);
    EXPECT(oi_coin_probe(NULL, 1024, 4, 0, 0, &u64a, &d), OI_EINVAL);
    int a, b, c, e;
    int nv = oi_num_variants();
    if (nv < 1) {
        fprintf(stderr, "no sampler variants\n");
        ++fails;
    }
    for (int v = 0; v < nv; ++v) EXPECT(oi_variant_info(v, &a, &b, &c, &e), OI_OK);
    if (oi_variant_info(nv, &a, &b, &c, &e) == OI_OK || oi_variant_info(-1, &a, &b, &c, &e) == OI_OK) {
        fprintf(stderr, "out-of-range variant accepted\n");
        ++fails;
    }
    oi_graph_destroy(NULL);
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("host driver ok\n");
    return 0;
}
