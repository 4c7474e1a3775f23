/* Runs every entry point of the FP64 oracle on small seeded inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer: out-of-bounds
 * accesses, use of freed memory, leaks, signed overflow and other undefined
 * behaviour abort the run with a report.  2D and 3D, fp labels with 2 and 4
 * regions, PC / PS / Poisson / deconvolving models, brute-force and cell-list
 * neighbours, plain and ranked acceptance, run in every gradient mode, with
 * one and two threads.  Exit status 0 when every call returned. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/sobrc_oracle.h"

static uint64_t rng_state = 88172645463325252ull;
static uint64_t rnd(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

static void blobs(const ora_params* P, int32_t* L, double* I)
{
    const int64_t n = (int64_t)P->nx * P->ny * P->nz;
    for (int64_t i = 0; i < n; ++i) {
        int x = (int)(i % P->nx), y = (int)((i / P->nx) % P->ny), z = (int)(i / ((int64_t)P->nx * P->ny));
        int l = 0;
        for (int k = 1; k < P->max_labels; ++k) {
            int cx = (int)(k * P->nx / (P->max_labels + 1)), cy = P->ny / 2, cz = P->nz / 2;
            int r = (P->nx < P->ny ? P->nx : P->ny) / 4 + 1;
            if ((x - cx) * (x - cx) + (y - cy) * (y - cy) + (z - cz) * (z - cz) <= r * r)
                l = k;
        }
        L[i] = l;
        I[i] = (double)l + ((double)(rnd() % 1000) / 1000.0 - 0.5) * 0.6 + 0.2;
    }
}

static void exercise(ora_params P)
{
    const int64_t n = (int64_t)P.nx * P.ny * P.nz;
    int32_t* L = malloc(sizeof(int32_t) * (size_t)n);
    double* I = malloc(sizeof(double) * (size_t)n);
    blobs(&P, L, I);
    int64_t np = ora_particles(&P, L, 0, NULL, NULL, NULL);
    int64_t* lin = malloc(sizeof(int64_t) * (size_t)(np + 1));
    int32_t* a = malloc(sizeof(int32_t) * (size_t)(np + 1));
    int32_t* b = malloc(sizeof(int32_t) * (size_t)(np + 1));
    double* g2 = malloc(sizeof(double) * (size_t)(np + 1));
    double* g1 = malloc(sizeof(double) * (size_t)(np + 1));
    double* g1b = malloc(sizeof(double) * (size_t)(np + 1));
    ora_particles(&P, L, np, lin, a, b);
    int64_t* cnt = calloc((size_t)P.max_labels, sizeof(int64_t));
    double* s1 = calloc((size_t)P.max_labels, sizeof(double));
    double* s2 = calloc((size_t)P.max_labels, sizeof(double));
    ora_region_stats(&P, I, L, cnt, s1, s2);
    ora_l2diff(&P, I, L, np, lin, a, b, g2);
    ora_sobolev(&P, np, lin, a, b, g2, g1, ORA_NEIGH_CELLS, 0, NULL);
    ora_sobolev(&P, np, lin, a, b, g2, g1b, ORA_NEIGH_BRUTE, 0, NULL);
    int64_t sel[3] = {0, np / 2, np > 0 ? np - 1 : 0};
    if (np > 0)
        ora_sobolev(&P, np, lin, a, b, g2, g1b, ORA_NEIGH_CELLS, 3, sel);
    for (int64_t i = 0; i < n; i += 7)
        (void)ora_simple(&P, L, i, L[i]);
    int32_t* L2 = malloc(sizeof(int32_t) * (size_t)n);
    memcpy(L2, L, sizeof(int32_t) * (size_t)n);
    uint8_t* done = malloc((size_t)(np + 1));
    (void)ora_accept_ranked(&P, L2, np, lin, a, b, g1, 1, done);
    (void)ora_energy_pc(&P, I, L);
    for (int mode = 0; mode < 3; ++mode) {
        memcpy(L2, L, sizeof(int32_t) * (size_t)n);
        int64_t nf = 0;
        (void)ora_step(&P, I, L2, mode == 2 ? 0 : mode, np, lin, a, b, g2, g1, &nf);
        int64_t hn[12], hf[12], hb[12];
        int32_t sw = -1;
        memcpy(L2, L, sizeof(int32_t) * (size_t)n);
        (void)ora_run(&P, I, L2, mode, 12, 1e-3, hn, hf, hb, &sw);
    }
    uint32_t* stamp = calloc((size_t)n, sizeof(uint32_t));
    (void)ora_reversals(n, L, L2, stamp, 0);
    free(stamp);
    free(done);
    free(L2);
    free(cnt);
    free(s1);
    free(s2);
    free(lin);
    free(a);
    free(b);
    free(g2);
    free(g1);
    free(g1b);
    free(L);
    free(I);
}

int main(void)
{
    ora_params P;
    memset(&P, 0, sizeof P);
    const int shapes[][4] = {{2, 23, 19, 1}, {3, 11, 9, 7}, {2, 1, 30, 1}, {3, 1, 12, 10}};
    for (int s = 0; s < 4; ++s)
        for (int variant = 0; variant < 5; ++variant) {
            P.ndim = shapes[s][0];
            P.nx = shapes[s][1];
            P.ny = shapes[s][2];
            P.nz = shapes[s][3];
            P.E = 6.0;
            P.eps = 1.0 / 24.0;
            P.lambda = 0.3;
            P.max_labels = variant == 1 ? 4 : 2;
            P.model = variant == 2 ? ORA_PS : ORA_PC;
            P.ps_radius = variant == 2 ? 3 : 0;
            P.noise = variant == 3 ? 1 : 0;
            P.psf_sigma = variant == 4 ? 1.5 : 0.0;
            P.topo = variant == 1 ? 1 : 0;
            P.threads = s == 1 ? 2 : 1;
            exercise(P);
        }
    double taps[64];
    (void)ora_psf_taps(2.0, taps);
    double th[4];
    P.ndim = 2; P.nx = 17; P.ny = 13; P.nz = 1; P.max_labels = 3; P.psf_sigma = 2.0; P.model = ORA_PC;
    P.noise = 0; P.threads = 1;
    int32_t L[17 * 13];
    double I[17 * 13], J[17 * 13];
    blobs(&P, L, I);
    ora_deconv_theta(&P, I, L, th);
    ora_deconv_model(&P, L, th, J);
    double g[50], out[50];
    for (int i = 0; i < 50; ++i)
        g[i] = (double)(rnd() % 100) / 100.0;
    ora_conv_closed_curve(50, 30.0, 6.0, 1.0 / 24.0, g, out);
    ora_auto ast;
    ora_auto_init(&ast, 2);
    (void)ora_auto_update(&ast, 2, 1e-3, 100, 4, 4);
    (void)ora_kernel(1.0, 6.0, 1.0 / 24.0);
    printf("oracle driver: all calls returned\n");
    return 0;
}
