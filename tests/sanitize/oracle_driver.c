/* Drives every entry point of the oracle on small inputs, including its
 * argument errors, so that an AddressSanitizer / UndefinedBehaviorSanitizer
 * build can check the C code's memory accesses and arithmetic.  Exits 0 and
 * prints "ok" when every call returned what it should. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/mco.h"

#define CHECK(x)                                                              \
    do {                                                                      \
        if (!(x)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #x);  \
            return 1;                                                         \
        }                                                                     \
    } while (0)

static uint32_t lcg(uint32_t *s) { return *s = *s * 1664525u + 1013904223u; }

int main(void) {
    mco_ctx *c = NULL;
    CHECK(mco_create(&c) == MCO_OK);
    const int nx = 12, ny = 10, nz = 9;
    uint8_t ids[12 * 10 * 9];
    float rho[12 * 10 * 9];
    uint32_t s = 7;
    for (int i = 0; i < nx * ny * nz; ++i) {
        ids[i] = (uint8_t)(lcg(&s) % 5u);
        rho[i] = ids[i] ? 0.5f + (float)(lcg(&s) % 1000u) * 0.003f : 0.001205f;
    }
    CHECK(mco_load_phantom(c, ids, rho, nx, ny, nz, 1.5f) == MCO_OK);
    mco_geometry g = {300.0f, 600.0f, 16, 12, 3.0f, 3.0f, 8, 6, 0.7f, 0u};
    CHECK(mco_set_geometry(c, &g) == MCO_OK);
    const float e[3] = {40.5f, 60.5f, 80.5f}, w[3] = {1.0f, 2.0f, 0.5f};
    CHECK(mco_set_spectrum(c, e, w, 3) == MCO_OK);
    float eta[60];
    for (int i = 0; i < 60; ++i) eta[i] = (float)(i + 1) * 0.9f;
    CHECK(mco_set_detector_response(c, eta, 60) == MCO_OK);

    int64_t prim[16 * 12], scat[8 * 6], prim2[16 * 12], scat2[8 * 6];
    for (int reading = 0; reading < 2; ++reading) {
        CHECK(mco_set_reading(c, reading) == MCO_OK);
        for (int est = 0; est < 3; ++est) {
            CHECK(mco_set_estimator(c, est, est ? 3 : 1, est == 2 ? 0.05 : 0.0) == MCO_OK);
            for (uint32_t phys = 0; phys < 4; ++phys) {
                CHECK(mco_set_physics(c, phys) == MCO_OK);
                CHECK(mco_project(c, 0.3f, 1500, 11, prim, scat) == MCO_OK);
                CHECK(mco_project_mt(c, 0.3f, 1500, 11, prim2, scat2, 3) == MCO_OK);
                CHECK(memcmp(prim, prim2, sizeof prim) == 0);
                CHECK(memcmp(scat, scat2, sizeof scat) == 0);
                memset(prim2, 0, sizeof prim2);
                memset(scat2, 0, sizeof scat2);
                CHECK(mco_project_range(c, 0.3f, 0, 700, 11, prim2, scat2) == MCO_OK);
                CHECK(mco_project_range(c, 0.3f, 700, 800, 11, prim2, scat2) == MCO_OK);
                CHECK(memcmp(prim, prim2, sizeof prim) == 0);
            }
        }
    }
    CHECK(mco_set_estimator(c, 0, 1, 0.0) == MCO_OK);
    CHECK(mco_set_physics(c, 3u) == MCO_OK);
    uint16_t nint[100];
    uint32_t steps[100];
    uint8_t endc[100], first[100];
    CHECK(mco_debug_histories(c, 1.1f, 5, 100, 3, nint, steps, endc, first) == MCO_OK);
    float xf[300], eend[100];
    int32_t pix[100];
    CHECK(mco_debug_paths(c, 1.1f, 5, 100, 3, xf, pix, eend) == MCO_OK);
    double pe_img[16 * 12];
    CHECK(mco_primary_expected(c, 0.7f, 2, pe_img) == MCO_OK);
    float sim[3 * 10], full[6 * 10];
    for (int i = 0; i < 30; ++i) sim[i] = (float)i;
    CHECK(mco_interp_angles(sim, 3, 10, full) == MCO_OK);
    float cs[500], es[500];
    for (int proc = 0; proc < 4; ++proc)
        CHECK(mco_test_sample(c, proc, 4, 30.0f, 500, 9, cs, es) == MCO_OK);
    double pdf;
    float e2;
    CHECK(mco_pd_pdf(c, MCO_PROC_COMPTON, 1, 60.0f, 0.25, &pdf, &e2) == MCO_OK);
    CHECK(mco_pd_pdf(c, MCO_PROC_RAYLEIGH, 4, 60.0f, 1.0, &pdf, &e2) == MCO_OK);
    const float o[3] = {1.0f, 2.0f, -1.0f}, d[3] = {-1.0f, 0.0f, 0.0f};
    CHECK(mco_set_estimator(c, MCO_SCORE_POINT, 4, 0.0) == MCO_OK);
    memset(scat, 0, sizeof scat);
    CHECK(mco_pd_score_event(c, 0.0f, 1, 2, 0, o, d, 60.0f, 1, MCO_PROC_COMPTON, scat) ==
          MCO_OK);
    int iu, iv;
    CHECK(mco_detector_pixel(c, 0.0f, o, d, &iu, &iv) == MCO_OK);
    int J = 0;
    CHECK(mco_get_tables(c, &J, NULL, NULL, NULL, NULL) == MCO_OK && J > 2);
    float *t = (float *)malloc(sizeof(float) * (size_t)(3 * 5 + 1) * (size_t)J);
    CHECK(t != NULL);
    CHECK(mco_get_tables(c, &J, t, t + 5 * J, t + 10 * J, t + 15 * J) == MCO_OK);
    free(t);
    double xs[3];
    CHECK(mco_cross_sections(7.42, 0.555, 60.0, xs) == MCO_OK);
    CHECK(mco_sigma_kn(100.0) > 0.0);
    mco_stats st;
    CHECK(mco_get_stats(c, &st) == MCO_OK);
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    mco_philox4x32_10(ctr, key, out);
    float u[4];
    mco_uniform_batch(out, 4, u);
    float dr[3];
    const float din[3] = {0.0f, 0.0f, 1.0f};
    mco_test_rotate(din, 0.5f, 1.0, dr);

    /* argument errors */
    CHECK(mco_load_phantom(c, ids, rho, 0, ny, nz, 1.0f) != MCO_OK);
    CHECK(mco_set_geometry(c, NULL) != MCO_OK);
    mco_geometry bad = g;
    bad.snu = 5;
    CHECK(mco_set_geometry(c, &bad) != MCO_OK);
    CHECK(mco_set_spectrum(c, e, w, 0) != MCO_OK);
    CHECK(mco_set_physics(c, 8u) != MCO_OK);
    CHECK(mco_set_estimator(c, 7, 1, 0.0) != MCO_OK);
    CHECK(mco_test_sample(c, 9, 0, 30.0f, 1, 1, cs, es) != MCO_OK);
    CHECK(mco_primary_expected(c, 0.0f, 0, pe_img) != MCO_OK);
    CHECK(mco_interp_angles(sim, 0, 10, full) != MCO_OK);
    CHECK(mco_project(NULL, 0.0f, 1, 1, prim, scat) != MCO_OK);
    printf("%s\n", mco_last_error(c));
    mco_destroy(c);
    printf("ok\n");
    return 0;
}
