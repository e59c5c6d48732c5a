/* Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
 * library's host sources (C-ABI validation, 1D operators and bases, the
 * serving scheduler) are compiled with the sanitizers and linked with the
 * unmodified device objects; this driver runs every host path that needs no
 * GPU -- operator and basis construction for every n and node set, the
 * argument checks of every compute entry point, and a simulated server fed
 * from two threads (admission, budget, batching, failed launches,
 * release and teardown).  Prints "ok". */
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sfhad.h"

#define CHECK(c)                                                                      \
    do {                                                                              \
        if (!(c)) {                                                                   \
            fprintf(stderr, "%s:%d: check failed: %s (%s)\n", __FILE__, __LINE__, #c, \
                    sf_last_error());                                                 \
            exit(1);                                                                  \
        }                                                                             \
    } while (0)

static double *tiny_state(long E, int n) {
    const long cnt = E * n * n * n;
    double *u = malloc(sizeof(double) * 5 * (size_t)cnt);
    for (long i = 0; i < cnt; ++i) {
        u[i] = 1.0;
        u[cnt + i] = 0.1;
        u[2 * cnt + i] = 0.0;
        u[3 * cnt + i] = -0.1;
        u[4 * cnt + i] = 2.5;
    }
    return u;
}

struct feeder {
    sf_server *srv;
    sf_mesh mesh[7];
    int rounds;
};

static void *feed(void *arg) {
    struct feeder *f = (struct feeder *)arg;
    for (int r = 0; r < f->rounds; ++r) {
        sf_ticket t[7];
        for (int k = 0; k < 7; ++k)
            CHECK(sf_submit(f->srv, f->mesh[k], (r + k) % 2 ? SF_PREC_FP32_SPLIT : SF_PREC_FP64, &t[k]) ==
                  SF_OK);
        for (int k = 0; k < 7; ++k) {
            const double *y = (const double *)1;
            double lat = -1.0;
            const int st = sf_wait(f->srv, t[k], &y, &lat);
            CHECK(st == SF_OK || st == SF_ERR_HIP);
            CHECK(y == NULL && lat >= 0.0);
            CHECK(sf_release(f->srv, t[k]) == SF_OK);
        }
    }
    return NULL;
}

int main(void) {
    /* operators and bases, every n and node set */
    double x[16], w[16], Q[256], V[256], P[256], lm[16], lp[16], Vr[16 * 16], Pr[16 * 16];
    for (int kind = 0; kind < 2; ++kind)
        for (int n = 2; n <= 16; ++n) {
            CHECK(sf_operator_1d(n, kind, x, w, Q) == SF_OK);
            CHECK(sf_basis_1d(n, kind, V, P) == SF_OK);
            CHECK(sf_surface_operator_1d(n, kind, lm, lp) == SF_OK);
            for (int m = n; m <= 16; ++m) CHECK(sf_basis_rect(n, m, kind, Vr, Pr) == SF_OK);
        }
    CHECK(sf_operator_1d(17, 0, x, w, Q) == SF_ERR_UNSUPPORTED);
    CHECK(sf_basis_rect(5, 4, 0, Vr, Pr) == SF_ERR_ARG);

    /* argument checks (no device call is reached) */
    char *bad = (char *)(uintptr_t)0x10000;
    double M[16];
    for (int i = 0; i < 16; ++i) M[i] = i == 0 || i == 5 || i == 10 || i == 15;
    sf_opts o;
    CHECK(sf_opts_init(&o) == SF_OK);
    CHECK(sf_hadamard_volume(NULL, 4, 4, 3, SF_FLUX_EULER_CHANDRASHEKAR, NULL) == SF_ERR_ARG);
    CHECK(sf_hadamard_volume((double *)bad, 4, 4, 3, SF_FLUX_EULER_CHANDRASHEKAR, (double *)bad) == SF_ERR_ARG);
    CHECK(sf_hadamard_volume_ex(NULL, 0, 8, 3, SF_FLUX_EULER_CHANDRASHEKAR, NULL, &o) == SF_OK);
    CHECK(dense_hadamard_volume(NULL, 4, 17, 3, SF_FLUX_PRODUCT, NULL) == SF_ERR_UNSUPPORTED);
    CHECK(sf_hadamard_surface(NULL, NULL, 0, 4, 3, SF_FLUX_EULER_CHANDRASHEKAR, NULL, NULL, &o) == SF_OK);
    CHECK(sf_hadamard_volume_surface((double *)bad, NULL, 4, 4, 3, 1, (double *)(bad + (1 << 20)), NULL, &o) ==
          SF_ERR_ARG);
    CHECK(sf_hadamard_volume_curvilinear((double *)bad, NULL, 4, 4, 1, (double *)(bad + (1 << 20)), NULL) ==
          SF_ERR_ARG);
    CHECK(sf_entropy_trace(NULL, 4, 4, NULL, NULL) == SF_ERR_ARG);
    CHECK(sf_entropy_variables(NULL, 0, NULL, 1.4, NULL) == SF_OK);
    CHECK(sf_conserved_variables((double *)bad, 4, (double *)(bad + 8), 1.4, NULL) == SF_ERR_ARG);
    CHECK(sf_tensor_apply(NULL, 0, 4, 3, 5, M, NULL, NULL) == SF_OK);
    CHECK(sf_tensor_apply_rect((double *)bad, 4, 4, 17, 3, 5, M, (double *)(bad + (1 << 20)), NULL) ==
          SF_ERR_UNSUPPORTED);
    CHECK(strlen(sf_status_string(SF_ERR_BUDGET)) > 0);

    /* the scheduler on a simulated device, fed from two threads */
    sf_server *srv = NULL;
    CHECK(sf_server_create_sim((size_t)64 << 20, 16, 0.5, &srv) == SF_OK);
    struct feeder f[2];
    for (int th = 0; th < 2; ++th) {
        f[th].srv = srv;
        f[th].rounds = 6;
        for (int k = 0; k < 7; ++k) {
            const int n = 2 + k;
            const long E = 17 + 13 * k + th;
            double *u = tiny_state(E, n);
            CHECK(sf_mesh_register(srv, u, E, n, SF_FLUX_EULER_CHANDRASHEKAR, k % 2, &f[th].mesh[k]) == SF_OK);
            free(u);
        }
    }
    CHECK(sf_server_sim_fail_launches(srv, 2) == SF_OK);
    pthread_t tid[2];
    for (int th = 0; th < 2; ++th) CHECK(pthread_create(&tid[th], NULL, feed, &f[th]) == 0);
    for (int th = 0; th < 2; ++th) CHECK(pthread_join(tid[th], NULL) == 0);
    int64_t queued = -1, inflight = -1, used = -1;
    CHECK(sf_server_stats(srv, &queued, &inflight, &used) == SF_OK);
    CHECK(queued == 0 && inflight == 0 && used == 0);
    /* a request larger than the whole budget, an unknown mesh, a double release */
    double *big = tiny_state(40000, 8);
    sf_mesh bm;
    CHECK(sf_mesh_register(srv, big, 40000, 8, SF_FLUX_EULER_CHANDRASHEKAR, 0, &bm) == SF_OK);
    free(big);
    sf_ticket t;
    CHECK(sf_submit(srv, bm, SF_PREC_FP64, &t) == SF_ERR_BUDGET);
    CHECK(sf_submit(srv, 987654, SF_PREC_FP64, &t) == SF_ERR_NOT_FOUND);
    CHECK(sf_submit(srv, f[0].mesh[0], SF_PREC_FP64, &t) == SF_OK);
    CHECK(sf_wait(srv, t, NULL, NULL) == SF_OK);
    CHECK(sf_release(srv, t) == SF_OK);
    CHECK(sf_release(srv, t) == SF_ERR_NOT_FOUND);
    CHECK(sf_mesh_unregister(srv, bm) == SF_OK);
    /* teardown with requests still queued */
    for (int k = 0; k < 5; ++k) CHECK(sf_submit(srv, f[1].mesh[k], SF_PREC_FP64, &t) == SF_OK);
    CHECK(sf_server_destroy(srv) == SF_OK);
    printf("ok\n");
    return 0;
}
