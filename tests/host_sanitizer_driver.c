/* Drives the host runtime's argument checks, tail counts, footprints and
 * status strings; built with AddressSanitizer and UBSan by
 * test_host_sanitizers.py and run on the CPU (no device work is reached). */
#include <math.h>
#include <stdio.h>
#include <string.h>
#include "ara.h"
static int fails = 0;
#define CHECK(cond) do { if (!(cond)) { printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond); ++fails; } } while (0)
int main(void) {
    ara_tables* t = NULL;
    int64_t off[2] = {0, 2}, bad[2] = {1, 2};
    uint32_t ids[2] = {0, 1};
    CHECK(ara_create_tables(NULL, 0, NULL, 0, NULL, 0, 10, 0, NULL, NULL) == ARA_ERR_INVALID_ARG);
    CHECK(ara_create_tables(off, -1, NULL, 0, NULL, 0, 10, 0, NULL, &t) == ARA_ERR_INVALID_ARG);
    CHECK(ara_create_tables(off, 1, ids, 2, NULL, 0, 0, 0, NULL, &t) == ARA_ERR_INVALID_ARG);
    CHECK(ara_create_tables(bad, 1, ids, 2, NULL, 0, 4, 0, NULL, &t) == ARA_ERR_INVALID_ARG);
    CHECK(strstr(ara_last_error(), "offsets") != NULL);
    double y[4] = {0}, mean = 0, pml[1], tv[1];
    double ps[4] = {1.0, 0.0, NAN, 0.5};
    int64_t ns[4] = {4, 4, 4, 0};
    for (int i = 0; i < 4; ++i)
        CHECK(ara_risk_metrics(y, ns[i], &ps[i], 1, &mean, pml, tv, 0, NULL) == ARA_ERR_INVALID_ARG);
    CHECK(ara_run_layers(NULL, NULL, 1, NULL, 1, 0, NULL) == ARA_ERR_INVALID_ARG);
    CHECK(ara_backward(NULL, NULL, 0.99, NULL, NULL, 0, NULL) == ARA_ERR_INVALID_ARG);
    ara_destroy_tables(NULL);
    CHECK(strcmp(ara_status_string(ARA_OK), "ARA_OK") == 0);
    CHECK(strcmp(ara_status_string(99), "ARA_ERR_UNKNOWN") == 0);
    /* tail counts: exact integer arithmetic on the shortest decimal of p */
    int64_t m = 0;
    CHECK(ara_tail_count(1000000, 0.99, &m) == ARA_OK && m == 10000);
    CHECK(ara_tail_count(1000000, 0.989999999999, &m) == ARA_OK && m == 10001);
    CHECK(ara_tail_count(3, 1.0 / 3.0, &m) == ARA_OK && m == 3);
    CHECK(ara_tail_count(3, 2.0 / 3.0, &m) == ARA_OK && m == 2);
    CHECK(ara_tail_count(INT64_MAX, nextafter(1.0, 0.0), &m) == ARA_OK && m >= 1);
    CHECK(ara_tail_count(INT64_MAX, 5e-324, &m) == ARA_OK && m == INT64_MAX);
    CHECK(ara_tail_count(0, 0.5, &m) != ARA_OK);
    CHECK(ara_tail_count(10, 1.0, &m) != ARA_OK);
    double p = 1e-300;
    for (int i = 0; i < 2000; ++i, p = p * 1.41 + 1e-7) {
        if (p >= 1.0) p = 1e-12 * (i + 1);
        CHECK(ara_tail_count(1 + i * 7919LL, p, &m) == ARA_OK && m >= 1 && m <= 1 + i * 7919LL);
    }
    int64_t b = 0;
    CHECK(ara_yet_footprint(1000000, 1000000000, 2000000, 0, &b) == ARA_OK && b > 0);
    CHECK(ara_metrics_footprint(1000000, 2, 0, &b) == ARA_OK && b > 0);
    CHECK(ara_layout_info_get(NULL, NULL) == ARA_ERR_INVALID_ARG);
    printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails != 0;
}
