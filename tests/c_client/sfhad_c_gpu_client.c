/* The C-ABI end to end from plain C99 on the GPU: device buffers and a
 * stream from the HIP runtime API, the 3D Euler volume term (FP64 and
 * FP32-split) through sfhad.h, checked against the oracle's dense definition
 * (the oracle's C library is linked by the test only).  Prints "ok". */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "sfhad.h"

/* the oracle's C entry points (test infrastructure) */
int oracle_operator(int n, int kind, double *x, double *w, double *D, double *Q);
int oracle_dense_volume(const double *u, long E, int n, int d, int flux, const double *Q, const double *w,
                        double gamma, double *out);

#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            return 1;                                                  \
        }                                                              \
    } while (0)

static double uniform(unsigned long long *s) {
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL; /* 64-bit LCG (Knuth's MMIX constants) */
    return (double)(*s >> 11) / 9007199254740992.0;
}

static double normwise(const double *y, const double *r, long count) {
    double worst = 0.0;
    for (int v = 0; v < 5; ++v) {
        double dmax = 0.0, rmax = 0.0;
        for (long i = 0; i < count; ++i) {
            const double d = fabs(y[v * count + i] - r[v * count + i]), a = fabs(r[v * count + i]);
            if (d > dmax) dmax = d;
            if (a > rmax) rmax = a;
        }
        if (dmax / rmax > worst) worst = dmax / rmax;
    }
    return worst;
}

int main(void) {
    const int n = 4, d = 3, N = 64;
    const long E = 37, cnt = E * N;
    const size_t bytes = sizeof(double) * 5 * (size_t)cnt;
    double *u = malloc(bytes), *y = malloc(bytes), *ref = malloc(bytes);
    CHECK(u && y && ref);
    unsigned long long s = 12345;
    for (long i = 0; i < cnt; ++i) {
        const double rho = 0.5 + uniform(&s), p = 0.5 + uniform(&s);
        double vel[3], q = 0.0;
        for (int k = 0; k < 3; ++k) {
            vel[k] = uniform(&s) - 0.5;
            q += vel[k] * vel[k];
        }
        u[i] = rho;
        for (int k = 0; k < 3; ++k) u[(1 + k) * cnt + i] = rho * vel[k];
        u[4 * cnt + i] = p / 0.4 + 0.5 * rho * q;
    }
    double x[4], w[4], D[16], Q[16];
    CHECK(oracle_operator(n, 0 /* Gauss-Legendre */, x, w, D, Q) == 0);
    CHECK(oracle_dense_volume(u, E, n, d, 1, Q, w, 1.4, ref) == 0);

    double *du = NULL, *dy = NULL;
    hipStream_t st;
    CHECK(hipMalloc((void **)&du, bytes) == hipSuccess);
    CHECK(hipMalloc((void **)&dy, bytes) == hipSuccess);
    CHECK(hipStreamCreate(&st) == hipSuccess);
    CHECK(hipMemcpy(du, u, bytes, hipMemcpyHostToDevice) == hipSuccess);

    /* the short entry point: GL nodes, gamma 1.4, FP64, null stream */
    CHECK(sf_hadamard_volume(du, E, n, d, SF_FLUX_EULER_CHANDRASHEKAR, dy) == SF_OK);
    CHECK(hipMemcpy(y, dy, bytes, hipMemcpyDeviceToHost) == hipSuccess);
    const double e64 = normwise(y, ref, cnt);

    /* the FP32-split form on a stream of our own */
    sf_opts o;
    CHECK(sf_opts_init(&o) == SF_OK);
    o.precision = SF_PREC_FP32_SPLIT;
    o.stream = (void *)st;
    CHECK(sf_hadamard_volume_ex(du, E, n, d, SF_FLUX_EULER_CHANDRASHEKAR, dy, &o) == SF_OK);
    CHECK(hipStreamSynchronize(st) == hipSuccess);
    CHECK(hipMemcpy(y, dy, bytes, hipMemcpyDeviceToHost) == hipSuccess);
    const double e32 = normwise(y, ref, cnt);

    /* an argument error leaves the device untouched and says why */
    CHECK(sf_hadamard_volume(du, E, n, d, SF_FLUX_EULER_CHANDRASHEKAR, du) == SF_ERR_ARG);

    CHECK(hipStreamDestroy(st) == hipSuccess);
    CHECK(hipFree(du) == hipSuccess);
    CHECK(hipFree(dy) == hipSuccess);
    free(u);
    free(y);
    free(ref);
    if (!(e64 <= 1e-12 && e32 <= 1e-5)) {
        fprintf(stderr, "errors: fp64 %.3e fp32-split %.3e\n", e64, e32);
        return 1;
    }
    printf("ok\n");
    return 0;
}
