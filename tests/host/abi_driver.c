/*
 * Host-side checks of the C ABI (include/peos.h) for the sanitizer build:
 * every entry point is called with arguments it must reject (null pointers,
 * out-of-range shapes and flags, extreme sizes) and the pure host functions
 * with valid ones.  No device work: it runs without a GPU.  Exit status 0
 * when every call returned what the header states.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/peos.h"

static int failures = 0;

#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

int main(void)
{
    size_t ib = 0, wb = 0;
    /* sizes */
    EXPECT(peos_index_bytes(1000, 128, 32, 8, 16, 0, &ib, &wb) == PEOS_OK && ib == 1000u * 896u);
    EXPECT(peos_index_bytes(10, 960, 32, 16, 16, PEOS_FLAG_BF16_BASE | PEOS_FLAG_FP16, &ib, &wb) == PEOS_OK);
    EXPECT(peos_index_bytes(10, 32, 32, 4, 16, PEOS_FLAG_COMPACT, &ib, &wb) == PEOS_OK && ib == 10u * 256u);
    EXPECT(peos_index_bytes(2147483647LL, 4096, 64, 32, 128, PEOS_FLAG_BF16_BASE, &ib, &wb) == PEOS_OK);
    EXPECT(peos_index_bytes(2147483648LL, 128, 32, 8, 16, 0, &ib, &wb) == PEOS_EINVAL);
    EXPECT(peos_index_bytes(0, 128, 32, 8, 16, 0, &ib, &wb) == PEOS_EINVAL);
    EXPECT(peos_index_bytes(10, 130, 32, 8, 16, 0, &ib, &wb) == PEOS_EINVAL);
    EXPECT(peos_index_bytes(10, 128, 65, 8, 16, 0, &ib, &wb) == PEOS_EINVAL);
    EXPECT(peos_index_bytes(10, 128, 32, 33, 16, 0, &ib, &wb) == PEOS_EINVAL);
    EXPECT(peos_index_bytes(10, 128, 32, 8, 144, 0, &ib, &wb) == PEOS_EINVAL);
    EXPECT(peos_index_bytes(10, 128, 32, 8, 16, 64, &ib, &wb) == PEOS_EINVAL);
    EXPECT(peos_index_bytes(10, 128, 32, 8, 16, PEOS_FLAG_COMPACT, &ib, &wb) == PEOS_EINVAL);
    EXPECT(peos_index_bytes(10, 32, 32, 4, 16, PEOS_FLAG_COMPACT | PEOS_FLAG_FP16, &ib, &wb) == PEOS_EINVAL);
    EXPECT(peos_index_bytes(10, 128, 32, 8, 16, 0, NULL, &wb) == PEOS_EINVAL);
    EXPECT(strstr(peos_last_error(), "null") != NULL);
    EXPECT(peos_dimension_permutation_ws_bytes(128, &wb) == PEOS_OK && wb > 0);
    EXPECT(peos_dimension_permutation_ws_bytes(0, &wb) == PEOS_EINVAL);
    /* messages */
    for (int c = -8; c <= 1; ++c) EXPECT(peos_strerror(c) != NULL && strlen(peos_strerror(c)) > 0);
    /* every entry point that needs an index, a server or a graph rejects null */
    peos_index* ix = NULL;
    EXPECT(peos_build_tables(NULL, 10, 32, NULL, 16, 0, 4, 16, NULL, NULL, 0, 0, NULL, 0, NULL, 0,
                             NULL, &ix) == PEOS_EINVAL && ix == NULL);
    EXPECT(peos_build_tables_ex(NULL, 10, 32, NULL, 16, 0, 4, 16, NULL, NULL, 0, 0, NULL, NULL, 0,
                                NULL, 0, NULL, NULL) == PEOS_EINVAL);
    EXPECT(peos_index_layout(NULL, NULL) == PEOS_EINVAL);
    EXPECT(peos_set_upper_layers(NULL, NULL) == PEOS_EINVAL);
    EXPECT(peos_query_tables(NULL, NULL, 1, NULL, NULL, NULL) == PEOS_EINVAL);
    EXPECT(peos_search_ws_bytes(NULL, 1, 10, 0, &wb) == PEOS_EINVAL);
    EXPECT(peos_search_tables(NULL, NULL, NULL, NULL, 1, NULL, NULL, 10, 10, 10, 0, 0.1f, 0, NULL,
                              NULL, NULL, NULL, 0, NULL) == PEOS_EINVAL);
    EXPECT(peos_search(NULL, NULL, 1, NULL, NULL, 10, 10, 10, 0, 0.1f, 0, NULL, NULL, NULL, NULL,
                       0, NULL) == PEOS_EINVAL);
    EXPECT(peos_search_static(NULL, NULL, 1, NULL, NULL, 10, 10, 10, 0, 0.1f, 0, NULL, NULL, NULL,
                              NULL) == PEOS_EINVAL);
    EXPECT(peos_set_search_tuning(NULL, 0, 0, 0, 0) == PEOS_EINVAL);
    EXPECT(peos_set_class_tuning(NULL, 0, 0, 0, 0) == PEOS_EINVAL);
    EXPECT(peos_set_long_rows(NULL, 1) == PEOS_EINVAL);
    peos_graph* g = NULL;
    EXPECT(peos_graph_create(NULL, NULL, 1, NULL, NULL, 10, 10, 10, 0, 0.1f, 0, NULL, NULL, NULL,
                             NULL, 0, &g) == PEOS_EINVAL && g == NULL);
    EXPECT(peos_graph_launch(NULL, NULL) == PEOS_EINVAL);
    peos_serve_config cfg;
    memset(&cfg, 0, sizeof cfg);
    peos_server* sv = NULL;
    EXPECT(peos_serve_open(NULL, &cfg, &sv) == PEOS_EINVAL && sv == NULL);
    uint64_t t = 0;
    EXPECT(peos_serve_submit(NULL, NULL, 1, 1, 1, NULL, NULL, &t) == PEOS_EINVAL);
    int32_t n_done = 0;
    EXPECT(peos_serve_poll(NULL, 0, NULL, 0, &n_done) == PEOS_EINVAL);
    int64_t counters[8];
    EXPECT(peos_serve_counters(NULL, counters) == PEOS_EINVAL);
    EXPECT(peos_probe_gather(NULL, 1, 1, 1, NULL, NULL) == PEOS_EINVAL);
    EXPECT(peos_dimension_permutation(NULL, 1, 4, NULL, 1, 1, NULL, NULL, 0, NULL) == PEOS_EINVAL);
    /* releasing nothing is a no-op */
    peos_free(NULL);
    peos_graph_destroy(NULL);
    peos_serve_close(NULL);
    if (failures) fprintf(stderr, "%d failures\n", failures);
    else printf("abi driver ok\n");
    return failures ? 1 : 0;
}
