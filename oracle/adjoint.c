/*
 * adjoint.c -- oracle gradient of a receiver misfit with respect to the orientation at
 * every node, through the frozen choices of the fixed point.  TEST INFRASTRUCTURE ONLY.
 *
 * At the solution every non-fixed node D holds the value of one candidate of the
 * Section 4.3 choice: a stencil estimate U(tau_A, tau_B, tau_C, theta_D) (Section 4.2) or
 * a straight-ray update tau_N + L h / V(phi) from a known 8-neighbour; source-box nodes
 * hold straight-ray times from the source with the source node's orientation
 * (Section 4.4).  With the choices frozen, T is a composition of these maps in heap pop
 * order, so dL/dtheta follows by the chain rule taken in reverse pop order:
 *     lambda = dL/dT;  for D in reverse pop order: lambda(X) += lambda(D) dU_D/dtau_X,
 *     dL/dtheta_D += lambda(D) dU_D/dtheta_D.
 * The local partials differentiate the paper's geometric formulas (point E, foot point F,
 * |FD|, normal direction, phase speed at theta') by hand; the group-speed derivative used
 * by straight rays is a Richardson-extrapolated central difference.  With the velocity
 * table (Sections 3.2, 4.2) the speeds are the table's piecewise-linear interpolants, and
 * their derivatives the slopes of the whole-degree intervals (velocity.c: table_slope).
 *
 * The same reverse pass also gives dL/dA for the density-normalised stiffness A = C / rho
 * of every node (A11, A13, A33, A55): a stencil estimate depends on A_D through the phase
 * speed v(theta') only, a straight ray through the group speed of its node (for the source
 * box, the source node's), so dL/dA_D = lambda(D) dU_D/dA_D (+ box terms at the source).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "ali_oracle.h"

/* partial derivatives of one stencil estimate (same arguments as or_stencil_estimate) */
void or_stencil_partials(const or_material* m, double theta_ax, double h, const int off[6],
                         double ta, double tb, double tc, double* dta, double* dtb, double* dtc,
                         double* dth, double* dA) {
    double xA = off[0], yA = off[1], xB = off[2], yB = off[3], xC = off[4], yC = off[5];
    double Dl = tc - ta;
    double a = (tb - ta) / Dl;
    double da_ta = (a - 1.0) / Dl, da_tb = 1.0 / Dl, da_tc = -a / Dl;
    double xE = (1.0 - a) * xA + a * xC, yE = (1.0 - a) * yA + a * yC;
    double wx = xB - xE, wy = yB - yE;               /* E -> B */
    double dwx = -(xC - xA), dwy = -(yC - yA);        /* d/da */
    double ex = -xE, ey = -yE;                        /* E -> D */
    double dex = dwx, dey = dwy;
    double N = wx * ey - wy * ex;
    double dN = dwx * ey + wx * dey - dwy * ex - wy * dex;
    double wl = sqrt(wx * wx + wy * wy);
    double dwl = (wx * dwx + wy * dwy) / wl;
    double sg = N >= 0.0 ? 1.0 : -1.0;
    double fd = fabs(N) / wl * h;
    double dfd = h * (sg * dN * wl - fabs(N) * dwl) / (wl * wl);
    double theta_n = atan2(wy, wx);
    double dthn = (wx * dwy - wy * dwx) / (wl * wl);
    double theta_D = theta_ax + 0.5 * M_PI;
    double thp = fmod(theta_D - theta_n + 0.5 * M_PI, M_PI);
    double v = or_phase_speed(m, thp);
    double dv = or_phase_speed_deriv(m, thp);
    double dU_da = dfd / v - fd * dv / (v * v) * (-dthn);
    *dta = dU_da * da_ta;
    *dtb = 1.0 + dU_da * da_tb;
    *dtc = dU_da * da_tc;
    *dth = -fd * dv / (v * v);
    if (dA) {
        /* |FD| depends on the times only; the stiffness enters through v(theta') */
        double dvA[4];
        or_qp_phase_speed_dA(m, thp, dvA);
        for (int k = 0; k < 4; ++k) dA[k] = -fd * dvA[k] / (v * v);
    }
}

static const int NEIGH8[8][2] = {
    {-1, -1}, {0, -1}, {1, -1}, {-1, 0}, {1, 0}, {-1, 1}, {0, 1}, {1, 1},
};

/* choices at the fixed point: -2 fixed (source box), -1 unreached, 0..31 stencil,
   32 + k straight ray from the k-th 8-neighbour */
void or_field_choices(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                      const double* orient, const double* T, const uint8_t* fixed, int* choice) {
    for (int j = 0; j < nz; ++j)
        for (int i = 0; i < nx; ++i) {
            int64_t p = (int64_t)j * nx + i;
            if (fixed[p]) { choice[p] = -2; continue; }
            int ch = -1;
            or_localfmm(nx, nz, h, mats, mat_id, orient, T, i, j, &ch);
            choice[p] = isfinite(T[p]) ? ch : -1;
        }
}

/* value of node (i, j) under a frozen choice, from the current field */
static double frozen_value(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                           const double* orient, const double* T, int i, int j, int ch) {
    int64_t p = (int64_t)j * nx + i;
    const or_material* m = &mats[mat_id[p]];
    if (ch < 32) {
        int off[6];
        or_stencil_offsets(ch, off);
        double ta = T[(int64_t)(j + off[1]) * nx + i + off[0]];
        double tb = T[(int64_t)(j + off[3]) * nx + i + off[2]];
        double tc = T[(int64_t)(j + off[5]) * nx + i + off[4]];
        return or_stencil_estimate(m, orient[p], h, off, ta, tb, tc);
    }
    int di = NEIGH8[ch - 32][0], dj = NEIGH8[ch - 32][1];
    double tn = T[(int64_t)(j + dj) * nx + i + di];
    double phi = atan2((double)(-dj), (double)(-di)) - (orient[p] + 0.5 * M_PI);
    return tn + sqrt((double)(di * di + dj * dj)) * h / or_group_speed(m, phi);
}

void or_frozen_field(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                     const double* orient, int si, int sj, int R, const int* choice,
                     const int64_t* pop, int64_t npop, double* T) {
    int64_t N = (int64_t)nx * nz;
    uint8_t* fixed = calloc((size_t)N, 1);
    for (int64_t p = 0; p < N; ++p) T[p] = INFINITY;
    or_source_box(nx, nz, h, mats, mat_id, orient, si, sj, R, T, fixed);
    for (int64_t q = 0; q < npop; ++q) {
        int64_t p = pop[q];
        if (fixed[p] || choice[p] < 0) continue;
        T[p] = frozen_value(nx, nz, h, mats, mat_id, orient, T, (int)(p % nx), (int)(p / nx), choice[p]);
    }
    free(fixed);
}

/* lambda times the stiffness derivative of a straight-ray time L / V(phi) */
static void add_ray_dA(const or_material* m, double phi, double L, double l, double* out) {
    double V = or_qp_group_speed(m, phi);
    double dV[4];
    or_qp_group_speed_dA(m, phi, dV);
    for (int k = 0; k < 4; ++k) out[k] -= l * L * dV[k] / (V * V);
}

int or_adjoint(int nx, int nz, double h, const or_material* mats, int n_mats, const uint8_t* mat_id,
               const double* orient, int si, int sj, int R, const double* g, double* T_out,
               double* dtheta, double* dA) {
    int64_t N = (int64_t)nx * nz;
    if (dA)   /* the stiffness partials are written for the qP wave's run-time speeds */
        for (int k = 0; k < n_mats; ++k)
            if (mats[k].wave != OR_WAVE_QP || mats[k].vtab) return -1;
    double* T = T_out ? T_out : malloc(sizeof(double) * (size_t)N);
    int64_t* pop = malloc(sizeof(int64_t) * (size_t)N);
    int64_t npop = or_solve_fmm(nx, nz, h, mats, n_mats, mat_id, orient, si, sj, R, T, pop, NULL);
    if (npop < 0) { if (!T_out) free(T); free(pop); return -1; }
    double* Tbox = malloc(sizeof(double) * (size_t)N);
    uint8_t* fixed = calloc((size_t)N, 1);
    for (int64_t p = 0; p < N; ++p) Tbox[p] = INFINITY;
    or_source_box(nx, nz, h, mats, mat_id, orient, si, sj, R, Tbox, fixed);
    int* choice = malloc(sizeof(int) * (size_t)N);
    or_field_choices(nx, nz, h, mats, mat_id, orient, T, fixed, choice);
    double* lam = malloc(sizeof(double) * (size_t)N);
    memcpy(lam, g, sizeof(double) * (size_t)N);
    for (int64_t p = 0; p < N; ++p) dtheta[p] = 0.0;
    if (dA)
        for (int64_t p = 0; p < 4 * N; ++p) dA[p] = 0.0;
    int64_t ps = (int64_t)sj * nx + si;
    const or_material* msrc = &mats[mat_id[ps]];
    for (int64_t q = npop - 1; q >= 0; --q) {
        int64_t p = pop[q];
        int i = (int)(p % nx), j = (int)(p / nx);
        double l = lam[p];
        if (l == 0.0) continue;
        const or_material* m = &mats[mat_id[p]];
        if (fixed[p]) {
            /* straight ray from the source with the source node's orientation */
            int di = i - si, dj = j - sj;
            if (di == 0 && dj == 0) continue;
            double phi = atan2((double)dj, (double)di) - (orient[ps] + 0.5 * M_PI);
            double V = or_group_speed(msrc, phi);
            double r = sqrt((double)(di * di + dj * dj)) * h;
            dtheta[ps] += l * r * or_group_speed_deriv(msrc, phi) / (V * V);
            if (dA) add_ray_dA(msrc, phi, r, l, dA + 4 * ps);
            continue;
        }
        int ch = choice[p];
        if (ch < 0) continue;
        if (ch < 32) {
            int off[6];
            or_stencil_offsets(ch, off);
            int64_t pa = (int64_t)(j + off[1]) * nx + i + off[0];
            int64_t pb = (int64_t)(j + off[3]) * nx + i + off[2];
            int64_t pc = (int64_t)(j + off[5]) * nx + i + off[4];
            double da, db, dc, dth, dUA[4];
            or_stencil_partials(m, orient[p], h, off, T[pa], T[pb], T[pc], &da, &db, &dc, &dth, dUA);
            lam[pa] += l * da;
            lam[pb] += l * db;
            lam[pc] += l * dc;
            dtheta[p] += l * dth;
            if (dA)
                for (int k = 0; k < 4; ++k) dA[4 * p + k] += l * dUA[k];
        } else {
            int di = NEIGH8[ch - 32][0], dj = NEIGH8[ch - 32][1];
            int64_t pn = (int64_t)(j + dj) * nx + i + di;
            double phi = atan2((double)(-dj), (double)(-di)) - (orient[p] + 0.5 * M_PI);
            double V = or_group_speed(m, phi);
            double L = sqrt((double)(di * di + dj * dj)) * h;
            lam[pn] += l;
            dtheta[p] += l * L * or_group_speed_deriv(m, phi) / (V * V);
            if (dA) add_ray_dA(m, phi, L, l, dA + 4 * p);
        }
    }
    free(lam); free(choice); free(fixed); free(Tbox); free(pop);
    if (!T_out) free(T);
    return 0;
}
