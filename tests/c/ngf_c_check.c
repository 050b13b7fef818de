/*
 * A plain C caller of the ngfreg C ABI (include/ngfreg.h): the header is
 * compiled as C99 and the library linked without Python or torch.
 *
 *   ngf_c_check cpu   argument checks that need no device
 *   ngf_c_check gpu   a two-level registration (Sec. 2.1) of a synthetic
 *                     pair from host arrays: a smooth ball and the same
 *                     ball moved by one voxel along x; checks the report and
 *                     that the recovered displacement points along +x; then
 *                     at the result, with device buffers: the level form of
 *                     the differentiation (ngf_eval_J_grad_T) against
 *                     ngf_eval_J_grad, and the batched evaluation
 *                     (ngf_batch_build, ngf_batch_eval) of two pairs against
 *                     the single-pair one
 *
 * Device memory comes from the HIP runtime's C entry points, declared here
 * by hand (the caller includes no HIP header).
 * Exit status 0 on success; a failed check prints its reason.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ngfreg.h"

/* HIP runtime entry points used for device buffers (libamdhip64) */
int hipMalloc(void** ptr, size_t size);
int hipFree(void* ptr);
int hipMemcpy(void* dst, const void* src, size_t size, int kind);
enum { H2D = 1, D2H = 2 };

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
    {
        /* iteration log and L-BFGS checkpoint: record layout, argument checks */
        size_t bytes = 0;
        int32_t count = 0;
        char buf[8] = {0};
        CHECK(sizeof(ngf_iter_record) == 64, "iteration record of %u bytes",
              (unsigned)sizeof(ngf_iter_record));
        CHECK(ngf_set_iteration_log(NULL, 1) == NGF_E_ARG, "null context");
        CHECK(ngf_iteration_log(NULL, NULL, 0, &count) == NGF_E_ARG, "null context");
        CHECK(ngf_lbfgs_state_size(NULL, &bytes) == NGF_E_ARG, "null context");
        CHECK(ngf_lbfgs_save(NULL, buf, sizeof buf) == NGF_E_ARG, "null context");
        CHECK(ngf_lbfgs_load(NULL, buf, sizeof buf) == NGF_E_ARG, "null context");
    }
    printf("c abi cpu checks ok (%s)\n", v);
    return 0;
}

/* smooth ball of radius 8 voxels centred at (cx, 16, 16) */
static float ball(double x, double y, double z, double cx) {
    const double r = sqrt((x - cx) * (x - cx) + (y - 16.0) * (y - 16.0) + (z - 16.0) * (z - 16.0));
    return (float)(1.0 / (1.0 + exp(2.0 * (r - 8.0))));
}

/* relative L2 distance of two float vectors */
static double rel_l2(const float* a, const float* b, size_t n) {
    double num = 0.0, den = 0.0;
    size_t i;
    for (i = 0; i < n; ++i) {
        num += ((double)a[i] - b[i]) * ((double)a[i] - b[i]);
        den += (double)b[i] * b[i];
    }
    return sqrt(num / den);
}

/* At the registered y (host), with the pyramid the registration built. */
static int device_forms(ngf_ctx* c, const ngf_params* p, const float* R, const float* T,
                        const float* y) {
    enum { M = 32, MY = M / 2 + 1 };
    const size_t n = (size_t)M * M * M, ny = (size_t)3 * MY * MY * MY;
    float *dR = NULL, *dT = NULL, *dy = NULL, *dg = NULL, *dgy = NULL, *dgT = NULL, *dg2 = NULL;
    float* hg = malloc(ny * sizeof(float));
    float* hgy = malloc(ny * sizeof(float));
    float* hg2 = malloc(ny * sizeof(float));
    ngf_batch* b = NULL;
    ngf_grid g[2];
    double J = 0.0, JT = 0.0, Jb[2] = {0.0, 0.0};
    ngf_status st;
    CHECK(hg && hgy && hg2, "host allocation");
    CHECK(hipMalloc((void**)&dR, n * 4) == 0 && hipMalloc((void**)&dT, n * 4) == 0 &&
              hipMalloc((void**)&dy, ny * 4) == 0 && hipMalloc((void**)&dg, ny * 4) == 0 &&
              hipMalloc((void**)&dgy, ny * 4) == 0 && hipMalloc((void**)&dgT, n * 4) == 0 &&
              hipMalloc((void**)&dg2, ny * 4) == 0,
          "hipMalloc");
    CHECK(hipMemcpy(dR, R, n * 4, H2D) == 0 && hipMemcpy(dT, T, n * 4, H2D) == 0 &&
              hipMemcpy(dy, y, ny * 4, H2D) == 0,
          "hipMemcpy to the device");
    /* the plain form and the level form of the differentiation, same variants */
    CHECK(ngf_set_kernel(c, -2) == NGF_OK, "ngf_set_kernel");
    st = ngf_eval_J_grad(c, 0, dy, &J, dg, NULL);
    CHECK(st == NGF_OK, "ngf_eval_J_grad: %d (%s)", (int)st, ngf_last_error(c));
    st = ngf_eval_J_grad_T(c, 0, dy, NULL, &JT, NULL, dgy, dgT);
    CHECK(st == NGF_OK, "ngf_eval_J_grad_T: %d (%s)", (int)st, ngf_last_error(c));
    CHECK(hipMemcpy(hg, dg, ny * 4, D2H) == 0 && hipMemcpy(hgy, dgy, ny * 4, D2H) == 0,
          "hipMemcpy to the host");
    printf("level form: J %.9g (plain %.9g), grad y rel-L2 %.2e\n", JT, J, rel_l2(hgy, hg, ny));
    CHECK(fabs(JT - J) <= 1e-6 * fabs(J), "J of the level form");
    CHECK(rel_l2(hgy, hg, ny) <= 1e-5, "grad y of the level form");
    /* the batched evaluation: (R, T) and (T, R), compared with the single pair */
    {
        const float* Rs[2];
        const float* Ts[2];
        const float* ys[2];
        float* gs[2];
        Rs[0] = dR;
        Ts[0] = dT;
        Rs[1] = dT;
        Ts[1] = dR;
        ys[0] = dy;
        ys[1] = dy;
        gs[0] = dg2;
        gs[1] = dgy;
        g[0].m[0] = g[0].m[1] = g[0].m[2] = M;
        g[0].h[0] = g[0].h[1] = g[0].h[2] = 1.0;
        g[1] = g[0];
        CHECK(ngf_batch_create(p, 1, &b) == NGF_OK, "ngf_batch_create");
        CHECK(ngf_batch_set_kernel(b, -2) == NGF_OK, "ngf_batch_set_kernel");
        CHECK(ngf_batch_eval(b, 0, ys, Jb, gs, NULL) == NGF_E_STATE, "eval before build");
        st = ngf_batch_build(b, 2, Rs, Ts, g, NULL);
        CHECK(st == NGF_OK, "ngf_batch_build: %d (%s)", (int)st, ngf_batch_last_error(b));
        st = ngf_batch_eval(b, 0, ys, Jb, gs, NULL);
        CHECK(st == NGF_OK, "ngf_batch_eval: %d (%s)", (int)st, ngf_batch_last_error(b));
        CHECK(hipMemcpy(hg2, dg2, ny * 4, D2H) == 0, "hipMemcpy to the host");
        printf("batched: J %.9g and %.9g (single pair %.9g)\n", Jb[0], Jb[1], J);
        CHECK(Jb[0] == J && memcmp(hg2, hg, ny * 4) == 0, "batched pair 0 differs");
        CHECK(isfinite(Jb[1]) && Jb[1] > 0.0, "batched pair 1");
        ngf_batch_destroy(b);
    }
    hipFree(dR);
    hipFree(dT);
    hipFree(dy);
    hipFree(dg);
    hipFree(dgy);
    hipFree(dgT);
    hipFree(dg2);
    free(hg);
    free(hgy);
    free(hg2);
    printf("c abi gpu device forms ok\n");
    return 0;
}

/* The iteration log of a registration and an L-BFGS checkpoint, from C:
 * one record per accepted step plus one per level start, in level order; a
 * saved state replays the same steps after further ones. */
static int aux_forms(ngf_ctx* c, const float* R, const float* T, const ngf_grid* g) {
    enum { MY = 17 };
    const size_t ny = (size_t)3 * MY * MY * MY;
    ngf_report rep;
    ngf_iter_record* recs = NULL;
    int32_t count = 0, expect = 0, info = 0, l;
    size_t bytes = 0;
    void* state = NULL;
    float* dy = NULL;
    double Ja[3], Jb[3];
    int k;
    CHECK(ngf_set_iteration_log(c, 1) == NGF_OK, "iteration log on");
    CHECK(ngf_register(c, R, T, g, NULL, 1, &rep) == NGF_OK, "register: %s", ngf_last_error(c));
    CHECK(ngf_iteration_log(c, NULL, 0, &count) == NGF_OK, "log count");
    for (l = 0; l < rep.levels; ++l) expect += rep.iters[l] + 1;
    CHECK(count == expect, "%d records, expected %d", (int)count, (int)expect);
    recs = malloc((size_t)count * sizeof(ngf_iter_record));
    CHECK(recs != NULL, "host allocation");
    CHECK(ngf_iteration_log(c, recs, count, &count) == NGF_OK, "log copy");
    CHECK(recs[0].level == rep.levels - 1 && recs[0].iter == 0 && recs[0].evals == 1,
          "first record");
    CHECK(recs[count - 1].level == 0 && recs[count - 1].iter == rep.iters[0] &&
              recs[count - 1].J == rep.J[0],
          "last record");
    free(recs);
    CHECK(ngf_set_iteration_log(c, 0) == NGF_OK, "iteration log off");

    CHECK(hipMalloc((void**)&dy, ny * sizeof(float)) == 0, "hipMalloc");
    CHECK(ngf_identity(c, 0, dy) == NGF_OK, "identity");
    CHECK(ngf_lbfgs_reset(c, 0, dy) == NGF_OK, "reset: %s", ngf_last_error(c));
    for (k = 0; k < 2; ++k) CHECK(ngf_lbfgs_step(c, Ja, &info) == NGF_OK, "step");
    CHECK(ngf_lbfgs_state_size(c, &bytes) == NGF_OK && bytes > 2 * ny * sizeof(float),
          "state size %lu", (unsigned long)bytes);
    state = malloc(bytes);
    CHECK(state != NULL, "host allocation");
    CHECK(ngf_lbfgs_save(c, state, bytes) == NGF_OK, "save: %s", ngf_last_error(c));
    CHECK(ngf_lbfgs_save(c, state, bytes - 1) == NGF_E_ARG, "short buffer accepted");
    for (k = 0; k < 3; ++k) CHECK(ngf_lbfgs_step(c, &Ja[k], &info) == NGF_OK, "step");
    CHECK(ngf_lbfgs_load(c, state, bytes) == NGF_OK, "load: %s", ngf_last_error(c));
    for (k = 0; k < 3; ++k) CHECK(ngf_lbfgs_step(c, &Jb[k], &info) == NGF_OK, "step");
    for (k = 0; k < 3; ++k) CHECK(Ja[k] == Jb[k], "resumed step %d: %.17g vs %.17g", k, Jb[k], Ja[k]);
    free(state);
    hipFree(dy);
    printf("c abi gpu iteration log and checkpoint ok (%d records)\n", (int)count);
    return 0;
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
    printf("c abi gpu registration ok\n");
    if (device_forms(c, &p, R, T, y) != 0) return 1;
    if (aux_forms(c, R, T, &g) != 0) return 1;
    ngf_destroy(c);
    free(R);
    free(T);
    free(y);
    return 0;
}

int main(int argc, char** argv) {
    if (argc == 2 && strcmp(argv[1], "cpu") == 0) return cpu_checks();
    if (argc == 2 && strcmp(argv[1], "gpu") == 0) return gpu_registration();
    fprintf(stderr, "usage: %s cpu|gpu\n", argv[0]);
    return 2;
}
