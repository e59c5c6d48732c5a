/* A plain C99 client of the library's C-ABI: compiles against include/sfhad.h
 * alone and exercises the host-only entry points and the argument checks
 * (no device call).  Built and run by tests/test_c_client.py; prints "ok". */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "sfhad.h"

static int fails = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
            ++fails;                                                  \
        }                                                             \
    } while (0)

int main(void) {
    double x[8], w[8], Q[64], V[64], P[64], lm[8], lp[8];
    double s = 0.0, rowmax = 0.0, idmax = 0.0;
    int i, j, k;
    sf_opts o;
    const double M[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};

    CHECK(strncmp(sf_version(), "sfhad", 5) == 0);
    CHECK(strcmp(sf_status_string(SF_ERR_ARG), "SF_ERR_ARG") == 0);

    CHECK(sf_operator_1d(8, SF_NODES_GAUSS_LEGENDRE, x, w, Q) == SF_OK);
    for (i = 0; i < 8; ++i) s += w[i];
    CHECK(fabs(s - 2.0) < 1e-14);
    for (i = 0; i < 8; ++i) {
        double r = 0.0;
        for (j = 0; j < 8; ++j) r += Q[i * 8 + j];
        if (fabs(r) > rowmax) rowmax = fabs(r);
    }
    CHECK(rowmax < 1e-13);

    CHECK(sf_basis_1d(8, SF_NODES_GAUSS_LOBATTO, V, P) == SF_OK);
    for (i = 0; i < 8; ++i)
        for (j = 0; j < 8; ++j) {
            double a = 0.0;
            for (k = 0; k < 8; ++k) a += P[i * 8 + k] * V[k * 8 + j];
            a -= (i == j) ? 1.0 : 0.0;
            if (fabs(a) > idmax) idmax = fabs(a);
        }
    CHECK(idmax < 1e-12);

    CHECK(sf_surface_operator_1d(4, SF_NODES_GAUSS_LOBATTO, lm, lp) == SF_OK);
    CHECK(lm[0] == 1.0 && lp[3] == 1.0 && lm[3] == 0.0);

    CHECK(sf_hadamard_volume(NULL, 4, 4, 3, SF_FLUX_EULER_CHANDRASHEKAR, NULL) == SF_ERR_ARG);
    CHECK(strlen(sf_last_error()) > 0);
    CHECK(sf_hadamard_volume(NULL, 4, 17, 3, SF_FLUX_PRODUCT, NULL) == SF_ERR_UNSUPPORTED);
    CHECK(sf_opts_init(&o) == SF_OK);
    CHECK(o.gamma == 1.4 && o.stream == NULL);
    CHECK(sf_hadamard_volume_ex(NULL, 0, 8, 3, SF_FLUX_EULER_CHANDRASHEKAR, NULL, &o) == SF_OK);
    CHECK(sf_tensor_apply(NULL, 0, 4, 3, 5, M, NULL, NULL) == SF_OK);
    CHECK(sf_tensor_apply(NULL, 4, 4, 3, 5, NULL, NULL, NULL) == SF_ERR_ARG);
    CHECK(sf_hadamard_surface(NULL, NULL, 0, 4, 3, SF_FLUX_EULER_CHANDRASHEKAR, NULL, NULL, &o) == SF_OK);
    o.precision = SF_PREC_FP32_SPLIT;
    CHECK(sf_hadamard_volume_ex(NULL, 4, 8, 3, SF_FLUX_PRODUCT, NULL, &o) == SF_ERR_UNSUPPORTED);

    if (fails) return 1;
    printf("ok\n");
    return 0;
}
