/*
 * A C consumer of libfdlb with no Python: the lid-driven cavity (N x N cells, 4 half-range nodes
 * per half-line in each direction, Kn and precision from the command line) solved to a residual
 * tolerance, with device memory from hipMalloc and a stream of its own.
 *
 *   cavity_c N KN TOL PRECISION(0 fp64 | 1 fp32 | 2 mixed) [OUT_FILE]
 *
 * Prints one line: steps, float steps, final residual, status, centre-line maximum of u_x.
 * With OUT_FILE, writes the state's raw populations (Q N N doubles, [alpha][y][x]) there.
 */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "fdlb.h"

#define HIP_OK(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));                  \
            return 2;                                                                   \
        }                                                                               \
    } while (0)
#define FDLB_OK_(call)                                                                  \
    do {                                                                                \
        int c_ = (call);                                                                \
        if (c_ < 0) {                                                                   \
            fprintf(stderr, "%s: error %d: %s\n", #call, c_, fdlb_last_error());        \
            return 3;                                                                   \
        }                                                                               \
    } while (0)

int main(int argc, char **argv) {
    if (argc < 5) {
        fprintf(stderr, "usage: %s N KN TOL PRECISION [OUT_FILE]\n", argv[0]);
        return 1;
    }
    const int n = atoi(argv[1]);
    fdlb_problem_desc d = {0};
    d.nx = d.ny = n;
    d.wall_u[FDLB_WALL_TOP] = 0.01;
    d.kn = atof(argv[2]);
    d.cfl = 0.9;
    d.qx_kind = d.qy_kind = FDLB_HALF;
    d.qx_n = d.qy_n = 4;
    d.precision = atoi(argv[4]);
    const double tol = atof(argv[3]);

    fdlb_problem *p = NULL;
    FDLB_OK_(fdlb_problem_create(&d, &p));
    void *state = NULL, *work = NULL;
    hipStream_t stream;
    HIP_OK(hipStreamCreate(&stream));
    HIP_OK(hipMalloc(&state, fdlb_state_bytes(p)));
    HIP_OK(hipMalloc(&work, fdlb_workspace_bytes(p)));
    FDLB_OK_(fdlb_bind(p, state, work, stream));
    FDLB_OK_(fdlb_init_equilibrium(p, NULL, NULL, NULL, 0));

    fdlb_report rep = {0};
    const int status = fdlb_solve_steady(p, tol, 2000000, 200, 1, &rep);
    FDLB_OK_(status);

    const size_t cells = (size_t)n * n;
    double *ux = (double *)malloc(cells * sizeof(double));
    FDLB_OK_(fdlb_moments(p, NULL, ux, NULL, NULL));
    double umax = 0;
    for (int y = 0; y < n; ++y) {
        const double u = 0.5 * (ux[(size_t)y * n + n / 2 - 1] + ux[(size_t)y * n + n / 2]);
        if (u > umax) umax = u;
    }
    printf("steps %lld fp32_steps %lld residual %.17g status %d centre_umax %.17g\n", (long long)rep.steps,
           (long long)rep.steps_fp32, rep.residual, status, umax);
    if (argc > 5) {
        const size_t nf = (size_t)fdlb_problem_q(p) * cells;
        double *f = (double *)malloc(nf * sizeof(double));
        FDLB_OK_(fdlb_state_download(p, f));
        FILE *fp = fopen(argv[5], "wb");
        if (!fp || fwrite(f, sizeof(double), nf, fp) != nf) {
            fprintf(stderr, "cannot write %s\n", argv[5]);
            return 4;
        }
        fclose(fp);
        free(f);
    }
    free(ux);
    fdlb_problem_destroy(p);
    HIP_OK(hipFree(state));
    HIP_OK(hipFree(work));
    HIP_OK(hipStreamDestroy(stream));
    return 0;
}
