/*
 * Runs every entry point of the FP64 oracle (test infrastructure) on small
 * 2D and 3D grids at space orders 4 and 16, with sparse points on the last
 * cell of the computational grid and inside the damping layer, records of
 * 1, 2 and 9 samples, and checkpoint segments of 1, 3 and more than the
 * record. Built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitized.py: any out-of-range access, overflow or
 * leak ends the run with an error. Exit status 0 when every call returned 0
 * and every output is finite.
 */
#include <math.h>
#include <stdio.h>

#include "../../oracle/wave.c"

static double fact(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

/* centred second-difference weights of half-order M (closed form) */
static void weights(int M, double* a) {
    a[0] = 0.0;
    for (int j = 1; j <= M; ++j) {
        a[j] = 2.0 * ((j % 2) ? 1.0 : -1.0) * fact(M) * fact(M) / ((double)j * j * fact(M - j) * fact(M + j));
        a[0] -= 2.0 * a[j];
    }
}

/* the 2^D corners and weights of a point at fractional computational index s */
static void point(const grid_t* g, const double* s, long* node, double* w) {
    const int D = g->ndim;
    const long n[3] = {g->nx, g->ny, g->nz};
    const long stride[3] = {g->ny * g->nz, g->nz, 1};
    long base[3]; double f[3];
    for (int a = 0; a < D; ++a) {
        const int A = (D == 3) ? a : (a == 0 ? 0 : 2);
        base[a] = (long)floor(s[a]);
        f[a] = s[a] - (double)base[a];
        if (base[a] >= n[A] - 1) { base[a] = n[A] - 2; f[a] = 1.0; }
    }
    for (int k = 0; k < (1 << D); ++k) {
        long off = 0; double ww = 1.0;
        for (int a = 0; a < D; ++a) {
            const int A = (D == 3) ? a : (a == 0 ? 0 : 2);
            const int bit = (k >> (D - 1 - a)) & 1;
            off += (base[a] + bit) * stride[A];
            ww *= bit ? f[a] : 1.0 - f[a];
        }
        node[k] = off; w[k] = ww;
    }
}

static int finite_all(const double* x, long n) {
    for (long i = 0; i < n; ++i) if (!isfinite(x[i])) return 0;
    return 1;
}

static int run(int D, int M, long nt) {
    grid_t g;
    memset(&g, 0, sizeof g);
    g.ndim = D; g.M = M;
    g.nx = 14; g.ny = D == 3 ? 11 : 1; g.nz = 13;
    g.hx = g.hy = g.hz = 10.0;
    weights(M, g.alpha);
    const long N = g.nx * g.ny * g.nz;
    const int K = 1 << D;
    double* m = malloc(N * sizeof(double));
    double* eta = malloc(N * sizeof(double));
    for (long c = 0; c < N; ++c) { m[c] = 0.2 + 0.05 * sin(0.37 * c); eta[c] = (c % 7 == 0) ? 0.01 : 0.0; }
    double S = 0.0;
    for (int j = 0; j <= M; ++j) S += (j ? 2.0 : 1.0) * fabs(g.alpha[j]);
    const double dt = 0.5 * 2.0 / (sqrt(1.0 / 0.2) * sqrt(S * D / (g.hx * g.hx)));
    /* sources: last cell, inside the layer; receivers: first and last cells */
    const double sp[2][3] = {{g.nx - 1.0, g.ny - 1.0, g.nz - 1.0}, {0.4, 0.0, 2.7}};
    const double rp[3][3] = {{0.0, 0.0, 0.0}, {g.nx - 1.0, 0.5, g.nz - 1.5}, {6.3, 4.2, 6.6}};
    long sn[2 * 8], rn[3 * 8]; double sw[2 * 8], rw[3 * 8];
    for (int i = 0; i < 2; ++i) {
        double s[3] = {sp[i][0], D == 3 ? sp[i][1] : sp[i][2], sp[i][2]};
        point(&g, s, sn + i * K, sw + i * K);
    }
    for (int i = 0; i < 3; ++i) {
        double s[3] = {rp[i][0], D == 3 ? rp[i][1] : rp[i][2], rp[i][2]};
        point(&g, s, rn + i * K, rw + i * K);
    }
    double* q = malloc(nt * 2 * sizeof(double));
    double* y = malloc(nt * 3 * sizeof(double));
    for (long i = 0; i < nt * 2; ++i) q[i] = cos(0.3 * i);
    for (long i = 0; i < nt * 3; ++i) y[i] = sin(0.2 * i);
    double* d = malloc(nt * 3 * sizeof(double));
    double* us = malloc(nt * N * sizeof(double));
    double* x = malloc(nt * 2 * sizeof(double));
    double* vs = malloc(nt * N * sizeof(double));
    double* g1 = malloc(N * sizeof(double));
    double* g2 = malloc(N * sizeof(double));
    double* lap = malloc(N * sizeof(double));
    int ok = 1;
    ok &= oracle_forward_d(&g, m, eta, dt, nt, 2, K, sn, sw, q, 3, K, rn, rw, d, us, NULL, NULL) == 0;
    ok &= finite_all(d, nt * 3) && finite_all(us, nt * N);
    ok &= oracle_adjoint_d(&g, m, eta, dt, nt, 3, K, rn, rw, y, 2, K, sn, sw, x, vs) == 0;
    ok &= finite_all(x, nt * 2) && finite_all(vs, nt * N);
    const long segs[3] = {1, 3, nt + 2};
    for (int i = 0; i < 3; ++i) {
        ok &= oracle_gradient_d(&g, m, eta, dt, nt, 2, K, sn, sw, q, 3, K, rn, rw, y, segs[i], g1, g2) == 0;
        ok &= finite_all(g1, N) && finite_all(g2, N);
    }
    oracle_laplacian_d(&g, m, lap);
    ok &= finite_all(lap, N);
    /* the complex build (complex-step derivatives) on the same problem */
    double complex* mz = malloc(N * sizeof(double complex));
    double complex* qz = malloc(nt * 2 * sizeof(double complex));
    double complex* yz = malloc(nt * 3 * sizeof(double complex));
    double complex* dz = malloc(nt * 3 * sizeof(double complex));
    double complex* g1z = malloc(N * sizeof(double complex));
    double complex* g2z = malloc(N * sizeof(double complex));
    for (long c = 0; c < N; ++c) mz[c] = m[c] + I * 1e-30;
    for (long i = 0; i < nt * 2; ++i) qz[i] = q[i];
    for (long i = 0; i < nt * 3; ++i) yz[i] = y[i];
    ok &= oracle_forward_z(&g, mz, eta, dt, nt, 2, K, sn, sw, qz, 3, K, rn, rw, dz, NULL, NULL, NULL) == 0;
    ok &= oracle_gradient_z(&g, mz, eta, dt, nt, 2, K, sn, sw, qz, 3, K, rn, rw, yz, 2, g1z, g2z) == 0;
    free(mz); free(qz); free(yz); free(dz); free(g1z); free(g2z);
    free(m); free(eta); free(q); free(y); free(d); free(us); free(x); free(vs); free(g1); free(g2); free(lap);
    if (!ok) fprintf(stderr, "failed: D=%d M=%d nt=%ld\n", D, M, nt);
    return ok;
}

int main(void) {
    int ok = 1;
    const int Ms[2] = {2, 8};
    const long nts[3] = {1, 2, 9};
    for (int D = 2; D <= 3; ++D)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) ok &= run(D, Ms[i], nts[j]);
    printf(ok ? "oracle sanitized run ok\n" : "oracle sanitized run FAILED\n");
    return ok ? 0 : 1;
}
