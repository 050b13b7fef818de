/*
 * A plain C caller of the ngfreg C ABI (include/ngfreg.h): the header is
 * compiled as C99 and the library linked without Python or torch.
 *
 *   ngf_c_check cpu   argument checks that need no device
 *   ngf_c_check gpu   a two-level registration (Sec. 2.1) of a synthetic
 *                     pair from host arrays: a smooth ball and the same
 *                     ball moved by one voxel along x; checks the report and
 *                     that the recovered displacement points along +x
 *
 * Exit status 0 on success; a failed check prints its reason.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ngfreg.h"

#define CHECK(cond, ...)                                                  \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);          \
            fprintf(stderr, __VA_ARGS__);                                 \
            fprintf(stderr, "\n");                                        \
            return 1;                                                     \
        }                                                                 \
    } while (0)

static ngf_params params(void) {
    ngf_params p;
    memset(&p, 0, sizeof p);
    p.alpha = 0.1;
    p.tau = 0.1;
    p.rho = 0.1;
    p.levels = 2;
    p.ratio = 2;
    p.max_iter = 30;
    p.lbfgs_mem = 5;
    p.tol_J = 1e-6;
    p.early_stop = 0;
    return p;
}

static int cpu_checks(void) {
    const char* v = ngf_version();
    ngf_ctx* c = NULL;
    ngf_params p;
    CHECK(v != NULL && strstr(v, "gfx950") != NULL, "version string %s", v ? v : "(null)");
    p = params();
    p.alpha = -1.0;
    CHECK(ngf_create(&p, NULL, &c) == NGF_E_ARG, "negative alpha accepted");
    p = params();
    p.ratio = 3;
    CHECK(ngf_create(&p, NULL, &c) == NGF_E_ARG, "ratio 3 accepted");
    p = params();
    p.lbfgs_mem = 0;
    CHECK(ngf_create(&p, NULL, &c) == NGF_E_ARG, "memory 0 accepted");
    CHECK(ngf_create(NULL, NULL, &c) == NGF_E_ARG, "null parameters accepted");
    CHECK(ngf_create(&p, NULL, NULL) == NGF_E_ARG, "null output accepted");
    CHECK(ngf_eval_J_grad(NULL, 0, NULL, NULL, NULL, NULL) == NGF_E_ARG, "null context");
    CHECK(ngf_register(NULL, NULL, NULL, NULL, NULL, 1, NULL) == NGF_E_ARG, "null context");
    printf("c abi cpu checks ok (%s)\n", v);
    return 0;
}

/* smooth ball of radius 8 voxels centred at (cx, 16, 16) */
static float ball(double x, double y, double z, double cx) {
    const double r = sqrt((x - cx) * (x - cx) + (y - 16.0) * (y - 16.0) + (z - 16.0) * (z - 16.0));
    return (float)(1.0 / (1.0 + exp(2.0 * (r - 8.0))));
}

static int gpu_registration(void) {
    enum { M = 32, MY = M / 2 + 1 };
    const size_t n = (size_t)M * M * M, ny = (size_t)3 * MY * MY * MY;
    float* R = malloc(n * sizeof(float));
    float* T = malloc(n * sizeof(float));
    float* y = malloc(ny * sizeof(float));
    ngf_params p = params();
    ngf_ctx* c = NULL;
    ngf_grid g;
    ngf_report rep;
    ngf_status st;
    double sx = 0.0, sy = 0.0, sz = 0.0, umax = 0.0;
    int cnt = 0, i, j, k, l;
    CHECK(R && T && y, "host allocation");
    for (i = 0; i < M; ++i)
        for (j = 0; j < M; ++j)
            for (k = 0; k < M; ++k) {
                const size_t q = ((size_t)i * M + j) * M + k;
                R[q] = ball(i + 0.5, j + 0.5, k + 0.5, 16.0);
                T[q] = ball(i + 0.5, j + 0.5, k + 0.5, 17.0);
            }
    CHECK(ngf_create(&p, NULL, &c) == NGF_OK, "ngf_create");
    g.m[0] = g.m[1] = g.m[2] = M;
    g.h[0] = g.h[1] = g.h[2] = 1.0;
    st = ngf_register(c, R, T, &g, y, 1, &rep);
    CHECK(st == NGF_OK, "ngf_register: %d (%s)", (int)st, ngf_last_error(c));
    CHECK(rep.levels == 2, "levels %d", rep.levels);
    for (l = 0; l < rep.levels; ++l) {
        printf("level %d: %d iterations, %d evaluations, J %.6f, info %d\n", l, rep.iters[l],
               rep.evals[l], rep.J[l], rep.info[l]);
        CHECK(rep.iters[l] >= 1 && rep.evals[l] > rep.iters[l] && isfinite(rep.J[l]),
              "level %d report", l);
        CHECK(rep.info[l] >= NGF_INFO_OK && rep.info[l] <= NGF_INFO_LINESEARCH_FAIL,
              "level %d info %d", l, rep.info[l]);
    }
    /* displacement u = y - X (node j at 2 j voxels) over the nodes near the ball */
    for (i = 0; i < MY; ++i)
        for (j = 0; j < MY; ++j)
            for (k = 0; k < MY; ++k) {
                const size_t q = ((size_t)i * MY + j) * MY + k;
                const double ux = y[q] - 2.0 * i, uy = y[ny / 3 + q] - 2.0 * j,
                             uz = y[2 * (ny / 3) + q] - 2.0 * k;
                const double d = sqrt((2.0 * i - 16.5) * (2.0 * i - 16.5) +
                                      (2.0 * j - 16.0) * (2.0 * j - 16.0) +
                                      (2.0 * k - 16.0) * (2.0 * k - 16.0));
                CHECK(isfinite(ux) && isfinite(uy) && isfinite(uz), "non-finite y");
                if (fabs(ux) > umax) umax = fabs(ux);
                if (d < 10.0) {
                    sx += ux;
                    sy += uy;
                    sz += uz;
                    ++cnt;
                }
            }
    sx /= cnt;
    sy /= cnt;
    sz /= cnt;
    printf("mean displacement near the ball: (%.3f, %.3f, %.3f) voxels, max |u_x| %.3f\n", sx, sy,
           sz, umax);
    CHECK(sx > 0.25 && sx > 4.0 * (fabs(sy) + fabs(sz)), "displacement not along +x");
    CHECK(umax < 4.0, "displacement too large");
    ngf_destroy(c);
    free(R);
    free(T);
    free(y);
    printf("c abi gpu registration ok\n");
    return 0;
}

int main(int argc, char** argv) {
    if (argc == 2 && strcmp(argv[1], "cpu") == 0) return cpu_checks();
    if (argc == 2 && strcmp(argv[1], "gpu") == 0) return gpu_registration();
    fprintf(stderr, "usage: %s cpu|gpu\n", argv[0]);
    return 2;
}
