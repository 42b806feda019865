/*
 * nested.c -- oracle nested fine grids around the source (paper Section 4.4, "propagation
 * around source").  TEST INFRASTRUCTURE ONLY.
 *
 * The march starts on the finest of a sequence of grids centred on the source node and
 * moves to the next coarser grid when the front leaves a square region; the last grid is
 * the working grid itself.  Level l has density d_l (nodes per working-grid spacing, odd,
 * each divisible by the next) and radius r_l (working-grid cells).  Following the paper:
 *   - a fine node takes the material and orientation of the nearest working-grid node (the
 *     odd density makes that node unique);
 *   - on the finest grid, the nodes whose nearest working-grid node is the source node
 *     (the region of constant material around it) get straight-ray times at the source
 *     material's group speed; they are the fixed start of the march;
 *   - the march on level l runs until it accepts a node farther than r_l (Chebyshev) from
 *     the source; the nodes accepted strictly earlier in time are known;
 *   - on the next grid the nodes that coincide with known nodes keep those times and are
 *     fixed (the integer density ratio makes them coincide); the march resumes from them,
 *     which is the paper's re-seeding of known nodes with unknown neighbours.
 * Readings (where the paper is silent): "known" at a switch is {tau < tau of the first node
 * beyond r_l}; the straight-ray region is a square of half-width vor_half working cells
 * (1/2 for the working grid's own cell).  Each fine grid spans r_l d_l + 2 of its own
 * cells around the source (clipped to the domain).  That is enough for an exact switch:
 * a node earlier than the first node beyond r_l has all its earlier neighbours inside the
 * radius, and that first node lies within 2 cells of the radius (its earlier neighbours
 * are inside the radius and the update reaches 2 cells); an update reads only earlier
 * neighbours, so cutting the grid there changes none of these values, and no node beyond
 * the radius can fall below the first one.
 */
#include <math.h>
#include <stdlib.h>
#include "ali_oracle.h"

/* nearest multiple index of a / d for odd d > 0 (round half never occurs) */
static int near_div(int a, int d) {
    int q = a + (d - 1) / 2;
    return q >= 0 ? q / d : -((-q + d - 1) / d);
}

typedef struct {
    int d, a_lo, a_hi, b_lo, b_hi, nx, nz;
    uint8_t* mat_id;
    double* orient;
    double* T;
    uint8_t* fixed;
    uint8_t* known;
    double t_stop;
} level_t;

static void level_alloc(level_t* L, int d, int W, int nx, int nz, int si, int sj,
                        const uint8_t* mat_id, const double* orient) {
    L->d = d;
    L->a_lo = -W < -si * d ? -si * d : -W;
    L->a_hi = W > (nx - 1 - si) * d ? (nx - 1 - si) * d : W;
    L->b_lo = -W < -sj * d ? -sj * d : -W;
    L->b_hi = W > (nz - 1 - sj) * d ? (nz - 1 - sj) * d : W;
    L->nx = L->a_hi - L->a_lo + 1;
    L->nz = L->b_hi - L->b_lo + 1;
    int64_t n = (int64_t)L->nx * L->nz;
    L->mat_id = malloc((size_t)n);
    L->orient = malloc(sizeof(double) * (size_t)n);
    L->T = malloc(sizeof(double) * (size_t)n);
    L->fixed = calloc((size_t)n, 1);
    L->known = calloc((size_t)n, 1);
    L->t_stop = INFINITY;
    for (int b = L->b_lo; b <= L->b_hi; ++b)
        for (int a = L->a_lo; a <= L->a_hi; ++a) {
            int64_t q = (int64_t)(b - L->b_lo) * L->nx + (a - L->a_lo);
            int64_t p = (int64_t)(sj + near_div(b, d)) * nx + (si + near_div(a, d));
            L->mat_id[q] = mat_id[p];
            L->orient[q] = orient[p];
            L->T[q] = INFINITY;
        }
}

static void level_free(level_t* L) {
    free(L->mat_id); free(L->orient); free(L->T); free(L->fixed); free(L->known);
}

int or_solve_refined(int nx, int nz, double h, const or_material* mats, int n_mats, const uint8_t* mat_id,
                     const double* orient, int si, int sj, int n_levels, const int* density,
                     const int* radius, double vor_half, double* T) {
    if (n_levels < 0 || n_levels > 8 || !(vor_half > 0.0)) return -1;
    if (si < 0 || sj < 0 || si >= nx || sj >= nz) return -1;
    for (int l = 0; l < n_levels; ++l) {
        int next = l + 1 < n_levels ? density[l + 1] : 1;
        if (density[l] < 3 || density[l] % 2 == 0 || density[l] % next != 0 || radius[l] < 0) return -1;
        if (l > 0 && radius[l] < radius[l - 1]) return -1;
    }
    level_t lv[9];
    const int64_t ps = (int64_t)sj * nx + si;
    const or_material* msrc = &mats[mat_id[ps]];
    for (int l = 0; l <= n_levels; ++l) {
        level_t* L = &lv[l];
        if (l < n_levels) level_alloc(L, density[l], radius[l] * density[l] + 2, nx, nz, si, sj, mat_id, orient);
        else level_alloc(L, 1, nx > nz ? nx : nz, nx, nz, si, sj, mat_id, orient);
        const double hl = h / L->d;
        if (l == 0) {
            /* straight rays inside the source node's own cell */
            for (int b = L->b_lo; b <= L->b_hi; ++b)
                for (int a = L->a_lo; a <= L->a_hi; ++a) {
                    if (!(fabs((double)a) < vor_half * L->d && fabs((double)b) < vor_half * L->d)) continue;
                    int64_t q = (int64_t)(b - L->b_lo) * L->nx + (a - L->a_lo);
                    double t = 0.0;
                    if (a != 0 || b != 0) {
                        double phi = atan2((double)b, (double)a) - (orient[ps] + 0.5 * M_PI);
                        t = sqrt((double)a * a + (double)b * b) * hl / or_group_speed(msrc, phi);
                    }
                    L->T[q] = t;
                    L->fixed[q] = 1;
                }
        } else {
            /* nodes that coincide with known nodes of the finer level keep their times */
            const level_t* F = &lv[l - 1];
            const int k = F->d / L->d;
            for (int b = L->b_lo; b <= L->b_hi; ++b)
                for (int a = L->a_lo; a <= L->a_hi; ++a) {
                    int fa = a * k, fb = b * k;
                    if (fa < F->a_lo || fa > F->a_hi || fb < F->b_lo || fb > F->b_hi) continue;
                    int64_t fq = (int64_t)(fb - F->b_lo) * F->nx + (fa - F->a_lo);
                    if (!F->known[fq] || !(F->T[fq] < F->t_stop)) continue;
                    int64_t q = (int64_t)(b - L->b_lo) * L->nx + (a - L->a_lo);
                    L->T[q] = F->T[fq];
                    L->fixed[q] = 1;
                }
        }
        const int stop = l < n_levels ? radius[l] * L->d : -1;
        int64_t r = or_fmm_seeded(L->nx, L->nz, hl, mats, n_mats, L->mat_id, L->orient, L->fixed, L->T,
                                  -L->a_lo, -L->b_lo, stop, L->known, &L->t_stop);
        if (r < 0) {
            for (int m = 0; m <= l; ++m) level_free(&lv[m]);
            return -1;
        }
    }
    const level_t* Lw = &lv[n_levels];
    for (int64_t p = 0; p < (int64_t)nx * nz; ++p) T[p] = Lw->T[p];
    for (int l = 0; l <= n_levels; ++l) level_free(&lv[l]);
    return 0;
}
