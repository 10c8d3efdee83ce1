/* Host-only exercise of libfdlb under AddressSanitizer: quadrature of every order, problem
 * set-up of valid and invalid descriptions, batches, networks, tile descriptions, errors. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "fdlb.h"

static fdlb_problem_desc desc(int nx, int ny, int px, int py, int qxk, int qxn, int qyk, int qyn, double kn, int prec) {
    fdlb_problem_desc d;
    memset(&d, 0, sizeof d);
    d.nx = nx; d.ny = ny; d.lx = 1.0; d.ly = 1.0; d.periodic_x = px; d.periodic_y = py;
    d.wall_u[1] = 0.01; d.kn = kn; d.cfl = 0.9;
    d.qx_kind = qxk; d.qx_n = qxn; d.qy_kind = qyk; d.qy_n = qyn; d.precision = prec;
    return d;
}

int main(void) {
    int bad = 0;
    for (int n = 0; n <= 17; ++n) {
        double x[64], w[64];
        int r = fdlb_quad_half_range(n, x, w);
        if ((n >= 1 && n <= 16) != (r == FDLB_OK)) { printf("half %d -> %d\n", n, r); bad++; }
    }
    for (int n = 0; n <= 33; ++n) {
        double x[64], w[64];
        int r = fdlb_quad_full_range(n, x, w);
        if ((n >= 1 && n <= 32) != (r == FDLB_OK)) { printf("full %d -> %d\n", n, r); bad++; }
    }
    srand(1308);
    for (int i = 0; i < 400; ++i) {
        int px = rand() % 3 == 1, py = !px && rand() % 2;
        int nx = px ? 1 : 1 + rand() % 80, ny = py ? 1 : 1 + rand() % 80;
        int qxk = rand() % 2, qyk = rand() % 2, qxn = rand() % 9, qyn = rand() % 9;
        double kn = (rand() % 10 == 0) ? INFINITY : pow(10.0, -2.0 + 4.0 * rand() / (double)RAND_MAX);
        fdlb_problem_desc d = desc(nx, ny, px, py, qxk, qxn, qyk, qyn, kn, rand() % 4);
        fdlb_problem *p = NULL;
        int r = fdlb_problem_create(&d, &p);
        if (r == FDLB_OK) {
            int q = fdlb_problem_q(p);
            double *a = malloc(sizeof(double) * q * 3);
            fdlb_problem_velocities(p, a, a + q, a + 2 * q);
            (void)fdlb_problem_dt(p); (void)fdlb_state_bytes(p); (void)fdlb_workspace_bytes(p);
            (void)fdlb_checkpoint_bytes(p);
            for (int t = -2; t < 40; ++t) (void)fdlb_problem_set_tile(p, t);
            free(a);
            fdlb_problem_destroy(p);
        } else if (p != NULL || strlen(fdlb_last_error()) == 0) {
            printf("create %d: handle or message missing\n", r); bad++;
        }
    }
    fdlb_problem_desc ds[6];
    for (int i = 0; i < 6; ++i) ds[i] = desc(16 + 8 * i, 12 + 4 * i, 0, 0, FDLB_HALF, 2 + i % 3, FDLB_HALF, 2 + i % 2, 0.1 * (i + 1), FDLB_MIXED);
    fdlb_batch *b = NULL;
    if (fdlb_batch_create(ds, 6, &b) != FDLB_OK) { printf("batch: %s\n", fdlb_last_error()); bad++; }
    else {
        for (int i = -1; i <= 6; ++i) (void)fdlb_batch_problem_q(b, i);
        (void)fdlb_batch_state_bytes(b); (void)fdlb_batch_workspace_bytes(b);
        for (int t = -2; t < 40; ++t) (void)fdlb_batch_set_tile(b, t);
        fdlb_batch_destroy(b);
    }
    ds[3].nx = 0;
    if (fdlb_batch_create(ds, 6, &b) == FDLB_OK) { printf("batch with a bad member accepted\n"); bad++; }
    for (int h = 0; h <= 9; ++h) {
        fdlb_mlp *m = NULL;
        int r = fdlb_mlp_create(h, 1000, &m);
        if (r == FDLB_OK) {
            int64_t P = fdlb_mlp_param_count(m);
            float *th = malloc(sizeof(float) * P);
            fdlb_mlp_init_params(m, 7, th);
            (void)fdlb_mlp_workspace_bytes(m);
            free(th);
            fdlb_mlp_destroy(m);
        }
    }
    /* hybrid channels: valid and invalid descriptions, layouts (host only, never bound) */
    for (int k = 0; k < 200; ++k) {
        fdlb_hybrid_desc hd = {0};
        hd.ny = 2 + (k * 37) % 300;
        hd.layer = 1 + (k * 13) % (hd.ny / 2 + 2);   /* sometimes past ny / 2: invalid */
        hd.kn = (k % 11 == 0) ? INFINITY : 0.01 + 0.1 * (k % 7);
        hd.u_bottom = -0.01;
        hd.u_top = 0.01;
        hd.cfl = (k % 17 == 0) ? 1.5 : 0.9;
        hd.qx_kind = k % 2;
        hd.qx_n = (k % 2 == 0) ? 1 + k % 6 : 1 + k % 4;
        hd.n_half = 1 + k % 9;
        hd.n_full = 1 + k % 17;
        fdlb_hybrid *hy = NULL;
        int r = fdlb_hybrid_create(&hd, 1, &hy);
        if (r == FDLB_OK) {
            int32_t ql = 0, qb = 0;
            int64_t sd = 0;
            double dt = 0, om = 0;
            (void)fdlb_hybrid_info(hy, 0, &ql, &qb, &sd, &dt, &om);
            (void)fdlb_hybrid_info(hy, 1, NULL, NULL, NULL, NULL, NULL);
            (void)fdlb_hybrid_state_bytes(hy);
            (void)fdlb_hybrid_workspace_bytes(hy);
            if (fdlb_hybrid_step(hy, 1) != FDLB_ESTATE) { printf("unbound hybrid stepped\n"); bad++; }
            fdlb_hybrid_destroy(hy);
        } else if (hy != NULL) {
            printf("hybrid handle set on error\n");
            bad++;
        }
    }
    char buf[8];
    for (int prec = 0; prec < 3; ++prec)
        for (int t = -1; t < 40; ++t) (void)fdlb_tile_describe(prec, t, buf, sizeof buf);
    printf("host harness done, %d problems\n", bad);
    return bad != 0;
}
