/* Drives every entry of the oracle once on small media, for a build with AddressSanitizer
   and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Exits 0 when every call
   returned what its contract says; the sanitizers abort on the first memory or undefined-
   behaviour error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "../../oracle/ali_oracle.h"

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)

static or_material ti(void) {
    or_material m = {241e9, 138e9, 216e9, 129e9, 129e9, 72e9, 8100.0, OR_WAVE_QP, 0, OR_GROUP_EXACT, 0};
    return m;
}

int main(void) {
    const int nx = 23, nz = 19, N = nx * nz;
    const double h = 2e-4;
    or_material mats[2] = {ti(), ti()};
    mats[1].c11 = 5900.0 * 5900.0 * 8100.0;
    mats[1].c33 = mats[1].c11;
    mats[1].c55 = 3200.0 * 3200.0 * 8100.0;
    mats[1].c13 = mats[1].c11 - 2.0 * mats[1].c55;
    uint8_t* id = malloc(N);
    double* th = malloc(sizeof(double) * N);
    for (int p = 0; p < N; ++p) {
        id[p] = (uint8_t)((p % nx) > nx / 2);
        th[p] = 0.3 + 0.01 * (p % 7);
    }
    double* T = malloc(sizeof(double) * N);
    double* T2 = malloc(sizeof(double) * N);
    int64_t* pop = malloc(sizeof(int64_t) * N);
    double* pv = malloc(sizeof(double) * N);

    /* velocities (every wave and speed rule) */
    for (int w = 0; w < 2; ++w)
        for (int tab = 0; tab < 2; ++tab)
            for (int g = 0; g < 2; ++g) {
                or_material m = ti();
                m.wave = w; m.vtab = tab; m.grule = g;
                for (int k = -7; k <= 7; ++k) {
                    const double a = 0.37 * k;
                    CHECK(or_phase_speed(&m, a) > 0.0 && or_group_speed(&m, a) > 0.0);
                    CHECK(isfinite(or_phase_speed_deriv(&m, a)) && isfinite(or_group_speed_deriv(&m, a)));
                }
            }
    or_material m = ti();
    double dv[4], dV[4];
    or_qp_phase_speed_dA(&m, 0.4, dv);
    or_qp_group_speed_dA(&m, 0.4, dV);
    CHECK(or_qp_group_speed_support(&m, 0.4) > 0.0 && or_qp_group_speed_paper(&m, 0.4) > 0.0);

    /* heap march, local operator, sweeper, seeded march */
    CHECK(or_solve_fmm(nx, nz, h, mats, 2, id, th, 5, 4, 2, T, pop, pv) == N);
    CHECK(or_sweep_solve(nx, nz, h, mats, 2, id, th, 5, 4, 2, 10000, T2) > 0);
    for (int p = 0; p < N; ++p) CHECK(T[p] == T2[p]);
    int ch = -1;
    CHECK(or_localfmm(nx, nz, h, mats, id, th, T, 10, 10, &ch) == T[10 * nx + 10]);
    uint8_t* fixed = calloc(N, 1);
    uint8_t* known = calloc(N, 1);
    fixed[4 * nx + 5] = 1;
    T2[4 * nx + 5] = 0.0;
    double t_stop = 0.0;
    CHECK(or_fmm_seeded(nx, nz, h, mats, 2, id, th, fixed, T2, 5, 4, 3, known, &t_stop) > 0);
    /* invalid input is refused */
    CHECK(or_solve_fmm(nx, nz, h, mats, 2, id, th, nx, 4, 2, T2, NULL, NULL) == -1);

    /* nested source grids */
    const int dens[2] = {9, 3}, rad[2] = {2, 5};
    CHECK(or_solve_refined(nx, nz, h, mats, 2, id, th, 5, 4, 2, dens, rad, 0.5, T2) == 0);

    /* dense Dijkstra, segment time, rays (changing and fixed families) */
    or_dijkstra_dense(nx, nz, h, mats, id, th, 5, 4, 3.0, T2);
    CHECK(or_segment_time(nx, nz, h, mats, id, th, 0.5, 0.5, 20.2, 17.9) > 0.0);
    double* pts = malloc(sizeof(double) * 2 * 512);
    for (int fam = -1; fam < 4; ++fam) {
        int np = 0;
        double tr = 0.0;
        const int st = or_trace_ray_family(nx, nz, h, mats, id, th, T, 5, 4, 20, 17, fam, 4, 8, 512, pts, &np, &tr);
        CHECK(st == 0 || st == -1);
        CHECK(np >= 0 && np <= 512);
    }
    int np = 0;
    double tr = 0.0;
    CHECK(or_trace_ray(nx, nz, h, mats, id, th, T, 5, 4, 20, 17, 4, 8, 512, pts, &np, &tr) == 0 && tr > 0.0);

    /* adjoint (orientation and stiffness), choices, frozen field, stencil partials */
    double* g = calloc(N, sizeof(double));
    g[17 * nx + 20] = 1.0;
    g[0] = -0.5;
    double* dth = malloc(sizeof(double) * N);
    double* dA = malloc(sizeof(double) * 4 * N);
    CHECK(or_adjoint(nx, nz, h, mats, 2, id, th, 5, 4, 2, g, T2, dth, dA) == 0);
    int* choice = malloc(sizeof(int) * N);
    memset(fixed, 0, N);
    for (int j = 2; j <= 6; ++j)
        for (int i = 3; i <= 7; ++i) fixed[j * nx + i] = 1;
    or_field_choices(nx, nz, h, mats, id, th, T, fixed, choice);
    or_frozen_field(nx, nz, h, mats, id, th, 5, 4, 2, choice, pop, N, T2);
    for (int p = 0; p < N; ++p) CHECK(T2[p] == T[p]);
    int off[6];
    or_stencil_offsets(3, off);
    double a, b, c, d, dA4[4];
    or_stencil_partials(&m, 0.4, h, off, 1e-6, 1.2e-6, 1.3e-6, &a, &b, &c, &d, dA4);
    for (int v = 1; v <= 8; v <<= 1) {
        or_set_reading_variant(v);
        CHECK(or_solve_fmm(nx, nz, h, mats, 2, id, th, 5, 4, 2, T2, NULL, NULL) == N);
    }
    or_set_reading_variant(0);
    free(id); free(th); free(T); free(T2); free(pop); free(pv); free(fixed); free(known); free(pts);
    free(g); free(dth); free(dA); free(choice);
    printf("oracle driver: every entry point ran clean\n");
    return 0;
}
