/* Exercises every oracle entry point on small lattices; built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitize.py, so that an out-of-bounds access, a leak or
 * undefined behaviour in the oracle fails the test.  Deterministic inputs
 * from a small linear congruential generator (values only, no method
 * arithmetic). */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static unsigned long long lcg = 12345;
static double unif(void)
{
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) / 9007199254740992.0 - 0.5;
}

/* random SU(3) matrix near the identity: Gram-Schmidt of 1 + eps * noise */
static void su3(double complex *U)
{
    double complex a[9];
    for (int i = 0; i < 9; ++i) a[i] = (i % 4 == 0 ? 1.0 : 0.0) + 0.3 * (unif() + I * unif());
    for (int r = 0; r < 2; ++r) {
        for (int p = 0; p < r; ++p) {
            double complex d = 0;
            for (int c = 0; c < 3; ++c) d += conj(a[3 * p + c]) * a[3 * r + c];
            for (int c = 0; c < 3; ++c) a[3 * r + c] -= d * a[3 * p + c];
        }
        double n = 0;
        for (int c = 0; c < 3; ++c) n += creal(a[3 * r + c] * conj(a[3 * r + c]));
        for (int c = 0; c < 3; ++c) a[3 * r + c] /= sqrt(n);
    }
    a[6] = conj(a[1] * a[5] - a[2] * a[4]);
    a[7] = conj(a[2] * a[3] - a[0] * a[5]);
    a[8] = conj(a[0] * a[4] - a[1] * a[3]);
    memcpy(U, a, sizeof(a));
}

static int run(const int L[4], const int B[4])
{
    const int bcs[4] = {1, 1, 1, -1};
    long V = (long)L[0] * L[1] * L[2] * L[3];
    double complex *U = malloc(sizeof(double complex) * V * 36);
    double complex *C = malloc(sizeof(double complex) * V * 144);
    double complex *x = malloc(sizeof(double complex) * V * 12);
    double complex *y = malloc(sizeof(double complex) * V * 12);
    double complex *z = calloc((size_t)V * 12, sizeof(double complex));
    double complex *w = calloc((size_t)V * 12, sizeof(double complex));
    long sites[3] = {0, V / 2, V - 1};
    double complex ys[36];
    double complex cs[144];
    for (long l = 0; l < V * 4; ++l) su3(U + 9 * l);
    for (long i = 0; i < V * 12; ++i) x[i] = unif() + I * unif();
    or_clover_field(L, U, 1.0, C);
    or_clover_site(L, U, 1.0, V - 1, cs);
    or_apply_D(L, bcs, U, C, -0.2, x, y);
    or_apply_D_sites(L, bcs, U, 1.0, -0.2, x, sites, 3, ys);
    or_apply_D_sites_nv(L, bcs, U, 1.0, -0.2, x, 1, sites, 3, ys);
    int rc = 0;
    rc |= or_apply_DBB(L, B, bcs, U, C, -0.2, 0, x, z) != 0;
    rc |= or_mr_block(L, B, bcs, U, C, -0.2, 1, 3, x, z, w) < 0;
    rc |= or_mr_block_eo(L, B, bcs, U, C, -0.2, 1, 3, x, z, w) < 0;
    rc |= or_sap(L, B, bcs, U, C, -0.2, x, z, 2, 3) != 0;
    rc |= or_sap_eo(L, B, bcs, U, C, -0.2, x, z, 2, 3) != 0;
    or_info info;
    memset(z, 0, sizeof(double complex) * V * 12);
    or_fgmres(L, B, bcs, U, C, -0.2, x, z, 8, 1e-10, 20, 2, 3, NULL, NULL, &info);
    rc |= info.status != 0 || !(info.rel_residual <= 1e-10);
    /* invalid blockings are rejected, not read out of bounds */
    const int bad[4] = {3, 4, 4, 4};
    rc |= or_sap(L, bad, bcs, U, C, -0.2, x, z, 1, 1) != -1;
    rc |= or_apply_DBB(L, B, bcs, U, C, -0.2, V, x, z) != -1;
    free(U);
    free(C);
    free(x);
    free(y);
    free(z);
    free(w);
    return rc;
}

int main(void)
{
    const int L1[4] = {4, 4, 4, 4}, B1[4] = {2, 2, 2, 2};
    const int L2[4] = {4, 4, 8, 8}, B2[4] = {4, 4, 4, 4};
    int rc = run(L1, B1) | run(L2, B2);
    printf("oracle sanitizer driver: %s\n", rc ? "FAILED" : "ok");
    return rc;
}
