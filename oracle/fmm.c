/*
 * fmm.c -- oracle ALI-FMM (paper Sections 2 and 4).  TEST INFRASTRUCTURE ONLY.
 *
 * Plain FP64 code written for a reader holding the paper:
 *   - stencil table: Tables 1 and 2 (two printing errors corrected, see below);
 *   - one stencil's estimate: Section 4.1 (point E by linear interpolation) and 4.2
 *     (foot point F, distance |FD|, phase velocity along the normal at D's orientation);
 *   - stencil choice: Section 4.3;
 *   - drivers: heap Fast Marching (Section 2), straight-ray source box (Section 4.4).
 *
 * Readings taken where the paper is silent or ambiguous (parity unpinned except through
 * the invariants tested in the suite):
 *   R1 a stencil is usable only if all three support points are "known" (accepted by the
 *      heap), tau_A < tau_B <= tau_C (Section 4.1), and its estimate exceeds tau_C
 *      (a causality strengthening of "only used when tau_D > tau_A", Section 4.3);
 *   R2 square stencils (pairs 1-8) are preferred to triangles (9-16); inside a class the
 *      stencil with the smallest score wins (squares: tau_C - tau_B; triangles: distance
 *      of the diagonal point's time from the isosceles interpolant), ties by table order;
 *   R3 if no stencil is usable, a straight-ray update from each known 8-neighbour at the
 *      exact group speed of D's material stands in for the finite difference of the
 *      comparison method cited by the paper (not defined in this paper);
 *   R4 each time a diamond neighbour of D is accepted, D's estimate is recomputed from
 *      its current known set (not min(old, new)); heap keys are (tau, linear index).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "ali_oracle.h"

/* ---- Tables 1 and 2 ------------------------------------------------------------------
   Rows give (di, dj) of A, B, C relative to D = (i, j).  Corrections:
   - row 4-1 prints C = (i-1, j), which is not adjacent to A = (i+1, j-1); row 4-2
     prints the corrected 4-1.  Here 4-1 = {A(+1,-1), B(0,-1), C(+1,0)} and 4-2 swaps B, C.
   - row 8-2 prints B = (i-1, j-1); the pair member of 8-1 has B = (i+1, j-1). */
static const int STENCIL[32][6] = {
    /* 1-1 */ {-1, -1,  0, -1, -1,  0}, /* 1-2 */ {-1, -1, -1,  0,  0, -1},
    /* 2-1 */ {-1,  1,  0,  1, -1,  0}, /* 2-2 */ {-1,  1, -1,  0,  0,  1},
    /* 3-1 */ { 1,  1,  1,  0,  0,  1}, /* 3-2 */ { 1,  1,  0,  1,  1,  0},
    /* 4-1 */ { 1, -1,  0, -1,  1,  0}, /* 4-2 */ { 1, -1,  1,  0,  0, -1},
    /* 5-1 */ {-2,  0, -1, -1, -1,  1}, /* 5-2 */ {-2,  0, -1,  1, -1, -1},
    /* 6-1 */ { 0,  2,  1,  1, -1,  1}, /* 6-2 */ { 0,  2, -1,  1,  1,  1},
    /* 7-1 */ { 0, -2,  1, -1, -1, -1}, /* 7-2 */ { 0, -2, -1, -1,  1, -1},
    /* 8-1 */ { 2,  0,  1,  1,  1, -1}, /* 8-2 */ { 2,  0,  1, -1,  1,  1},
    /* 9-1 */ { 0,  2,  0,  1,  1,  1}, /* 9-2 */ { 0,  2,  1,  1,  0,  1},
    /*10-1 */ { 0, -2,  0, -1,  1, -1}, /*10-2 */ { 0, -2,  1, -1,  0, -1},
    /*11-1 */ { 0, -2,  0, -1, -1, -1}, /*11-2 */ { 0, -2, -1, -1,  0, -1},
    /*12-1 */ { 0,  2,  0,  1, -1,  1}, /*12-2 */ { 0,  2, -1,  1,  0,  1},
    /*13-1 */ {-2,  0, -1,  0, -1,  1}, /*13-2 */ {-2,  0, -1,  1, -1,  0},
    /*14-1 */ { 2,  0,  1,  0,  1,  1}, /*14-2 */ { 2,  0,  1,  1,  1,  0},
    /*15-1 */ { 2,  0,  1,  0,  1, -1}, /*15-2 */ { 2,  0,  1, -1,  1,  0},
    /*16-1 */ {-2,  0, -1,  0, -1, -1}, /*16-2 */ {-2,  0, -1, -1, -1,  0},
};

void or_stencil_offsets(int s, int out[6]) {
    for (int k = 0; k < 6; ++k) out[k] = STENCIL[s][k];
}

/* The 12-node diamond {|di| + |dj| <= 2} \ {0}, listed in increasing linear-index order
   (row-major: by dj, then di). */
static const int DIAMOND[12][2] = {
    {0, -2}, {-1, -1}, {0, -1}, {1, -1}, {-2, 0}, {-1, 0},
    {1, 0},  {2, 0},   {-1, 1}, {0, 1},  {1, 1},  {0, 2},
};
static int diamond_slot(int di, int dj) {
    for (int k = 0; k < 12; ++k)
        if (DIAMOND[k][0] == di && DIAMOND[k][1] == dj) return k;
    return -1;
}

/* The 8-neighbourhood used by the straight-ray fallback, row-major order. */
static const int NEIGH8[8][2] = {
    {-1, -1}, {0, -1}, {1, -1}, {-1, 0}, {1, 0}, {-1, 1}, {0, 1}, {1, 1},
};

/* ---- Section 4.1 / 4.2: one stencil ------------------------------------------------ */
double or_stencil_estimate(const or_material* m, double theta_ax, double h,
                           const int off[6], double ta, double tb, double tc) {
    double xA = off[0], yA = off[1], xB = off[2], yB = off[3], xC = off[4], yC = off[5];
    double xD = 0.0, yD = 0.0;
    /* E on AC with the travel time of B (linear interpolation of tau along AC) */
    double a = (tb - ta) / (tc - ta);
    double xE = (1.0 - a) * xA + a * xC;
    double yE = (1.0 - a) * yA + a * yC;
    /* distance from D to the wavefront estimate EB (foot point F) */
    double num = fabs((yE - yB) * (xD - xE) + (xB - xE) * (yD - yE));
    double den = sqrt((xB - xE) * (xB - xE) + (yB - yE) * (yB - yE));
    double fd = num / den * h;
    /* phase angle: normal to EB against the material frame at D.  The paper's
       orientation theta_D is the c22-axis direction = symmetry axis + 90 deg. */
    double theta_n = atan2(yB - yE, xB - xE);
    double theta_D = theta_ax + 0.5 * M_PI;
    double thp = fmod(theta_D - theta_n + 0.5 * M_PI, M_PI);
    double v = or_phase_speed(m, thp);
    return tb + fd / v;
}

/* ---- Section 4.3: choice among stencils (R1-R3) ------------------------------------ */
typedef struct {
    int nx, nz;
    double h;
    const or_material* mats;
    const uint8_t* mat_id;
    const double* orient;
    const double* T;
} ctx_t;

static int in_grid(const ctx_t* c, int i, int j) {
    return i >= 0 && j >= 0 && i < c->nx && j < c->nz;
}

/* Alternative readings of Sections 2 and 4.3, for the test that measures which readings
   reproduce the printed errors of Table 3 (never set otherwise; 0 = the readings the
   oracle stands for).  Per thread. */
static _Thread_local int g_variant = 0;
void or_set_reading_variant(int v) { g_variant = v; }

/* known12: bit k set <=> the k-th diamond neighbour is in the known set K. */
static double phi_core(const ctx_t* c, int i, int j, unsigned known12, int* choice) {
    const double r2m1 = sqrt(2.0) - 1.0, two_mr2 = 2.0 - sqrt(2.0);
    int idx = j * c->nx + i;
    const or_material* m = &c->mats[c->mat_id[idx]];
    double th = c->orient[idx];
    int best = -1, best_cls = 4;
    double best_score = 0.0, best_U = INFINITY;
    for (int s = 0; s < 32; ++s) {
        const int* o = STENCIL[s];
        int ia = i + o[0], ja = j + o[1], ib = i + o[2], jb = j + o[3], ic = i + o[4], jc = j + o[5];
        if (!in_grid(c, ia, ja) || !in_grid(c, ib, jb) || !in_grid(c, ic, jc)) continue;
        int ka = diamond_slot(o[0], o[1]), kb = diamond_slot(o[2], o[3]), kc = diamond_slot(o[4], o[5]);
        if (!((known12 >> ka) & 1u) || !((known12 >> kb) & 1u) || !((known12 >> kc) & 1u)) continue;
        double ta = c->T[ja * c->nx + ia], tb = c->T[jb * c->nx + ib], tc = c->T[jc * c->nx + ic];
        if (!(ta < tb && tb <= tc)) continue;                 /* ordering, Section 4.1 */
        double U = or_stencil_estimate(m, th, c->h, o, ta, tb, tc);
        if (!(g_variant & OR_VAR_NO_CAUSALITY) && !(U > tc)) continue;   /* causality (R1) */
        int cls = s < 16 ? 0 : 1;
        if ((g_variant & OR_VAR_UNIT_SQUARES_FIRST) && cls == 1) cls = 2;
        if ((g_variant & OR_VAR_UNIT_SQUARES_FIRST) && s >= 8 && s < 16) cls = 1;
        double score;
        if (s < 16) {
            score = tc - tb;                                  /* squares: tau_C - tau_B */
        } else if (s & 1) {
            /* second member of a triangular pair: tau_B closest to the isosceles value */
            score = fabs(tb - (r2m1 * ta + two_mr2 * tc));
        } else if (g_variant & OR_VAR_TRIANGLE_LITERAL) {
            score = fabs(tb - (r2m1 * ta + two_mr2 * tc));
        } else {
            /* first member: same calculation with B and C swapped */
            score = fabs(tc - (r2m1 * ta + two_mr2 * tb));
        }
        if (cls < best_cls || (cls == best_cls && score < best_score)) {
            best = s; best_cls = cls; best_score = score; best_U = U;
        }
    }
    if (best < 0) {
        /* R3: straight-ray update from a known 8-neighbour N, exact group speed of D */
        for (int k = 0; k < 8; ++k) {
            int di = NEIGH8[k][0], dj = NEIGH8[k][1];
            int ni = i + di, nj = j + dj;
            if (!in_grid(c, ni, nj)) continue;
            int slot = diamond_slot(di, dj);
            if (!((known12 >> slot) & 1u)) continue;
            double tn = c->T[nj * c->nx + ni];
            double phi = atan2((double)(-dj), (double)(-di)) - (th + 0.5 * M_PI);
            double dist = sqrt((double)(di * di + dj * dj)) * c->h;
            double U = tn + dist / or_group_speed(m, phi);
            if (!(U > tn)) continue;
            if (U < best_U) { best_U = U; best = 32 + k; }
        }
    }
    if (choice) *choice = best;
    return best_U;
}

static unsigned known12_from_grid(const ctx_t* c, const uint8_t* known, int i, int j) {
    unsigned msk = 0;
    for (int k = 0; k < 12; ++k) {
        int ni = i + DIAMOND[k][0], nj = j + DIAMOND[k][1];
        if (in_grid(c, ni, nj) && known[nj * c->nx + ni]) msk |= 1u << k;
    }
    return msk;
}

double or_phi_d(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                const double* orient, const double* T, const uint8_t* known,
                int i, int j, int* choice) {
    ctx_t c = {nx, nz, h, mats, mat_id, orient, T};
    return phi_core(&c, i, j, known12_from_grid(&c, known, i, j), choice);
}

/* ---- Section 4.4: straight rays around the source ----------------------------------- */
void or_source_box(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                   const double* orient, int si, int sj, int R, double* T, uint8_t* fixed) {
    int sidx = sj * nx + si;
    const or_material* m = &mats[mat_id[sidx]];
    double th = orient[sidx];
    for (int dj = -R; dj <= R; ++dj)
        for (int di = -R; di <= R; ++di) {
            int i = si + di, j = sj + dj;
            if (i < 0 || j < 0 || i >= nx || j >= nz) continue;
            double t = 0.0;
            if (di != 0 || dj != 0) {
                double phi = atan2((double)dj, (double)di) - (th + 0.5 * M_PI);
                t = sqrt((double)(di * di + dj * dj)) * h / or_group_speed(m, phi);
            }
            T[j * nx + i] = t;
            fixed[j * nx + i] = 1;
        }
}

/* ---- Section 2: heap Fast Marching -------------------------------------------------- */
static _Thread_local int64_t g_phi_evals = 0;   /* evaluations of Phi_D in this thread's last or_solve_fmm call */
int64_t or_last_phi_evals(void) { return g_phi_evals; }

typedef struct { double t; int64_t idx; int64_t ver; } hent;
typedef struct { hent* a; int64_t n, cap; } heap_t;

static int hless(const hent* x, const hent* y) {
    return x->t < y->t || (x->t == y->t && x->idx < y->idx);
}
static void hpush(heap_t* h, hent e) {
    if (h->n == h->cap) { h->cap = h->cap ? 2 * h->cap : 1024; h->a = realloc(h->a, h->cap * sizeof(hent)); }
    int64_t k = h->n++;
    h->a[k] = e;
    while (k > 0) {
        int64_t p = (k - 1) / 2;
        if (!hless(&h->a[k], &h->a[p])) break;
        hent t = h->a[k]; h->a[k] = h->a[p]; h->a[p] = t; k = p;
    }
}
static hent hpop(heap_t* h) {
    hent top = h->a[0];
    h->a[0] = h->a[--h->n];
    int64_t k = 0;
    for (;;) {
        int64_t l = 2 * k + 1, r = l + 1, s = k;
        if (l < h->n && hless(&h->a[l], &h->a[s])) s = l;
        if (r < h->n && hless(&h->a[r], &h->a[s])) s = r;
        if (s == k) break;
        hent t = h->a[k]; h->a[k] = h->a[s]; h->a[s] = t; k = s;
    }
    return top;
}

static int valid_inputs(int nx, int nz, double h, const or_material* mats, int n_mats,
                        const uint8_t* mat_id, const double* orient, int si, int sj) {
    if (nx < 3 || nz < 3 || !(h > 0.0)) return 0;
    if (si < 0 || sj < 0 || si >= nx || sj >= nz) return 0;
    for (int k = 0; k < n_mats; ++k) {
        const or_material* m = &mats[k];
        if (m->wave != mats[0].wave) return 0;
        if (m->wave == OR_WAVE_SH) {
            if (!(m->rho > 0.0 && m->c44 > 0.0 && m->c66 > 0.0)) return 0;
            continue;
        }
        if (m->wave != OR_WAVE_QP) return 0;
        if (!(m->rho > 0.0 && m->c11 > 0.0 && m->c33 > 0.0 && m->c55 > 0.0)) return 0;
        if (!(m->c11 * m->c33 > m->c13 * m->c13)) return 0;
    }
    for (int64_t p = 0; p < (int64_t)nx * nz; ++p) {
        if (mat_id[p] >= n_mats) return 0;
        if (!isfinite(orient[p])) return 0;
    }
    return 1;
}

/* The march from a set of fixed nodes (their T given).  Nodes are accepted in (tau, index)
   order; with stop_r >= 0 the march ends at the first accepted node farther than stop_r
   (Chebyshev) from (ci, cj), which is not marked known and whose time goes to *t_stop. */
static int64_t fmm_core(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                        const double* orient, const uint8_t* fixed, double* T, int ci, int cj, int stop_r,
                        uint8_t* known, int64_t* pop_order, double* pop_values, double* t_stop) {
    int64_t N = (int64_t)nx * nz;
    int64_t* ver = calloc(N, sizeof(int64_t));
    heap_t hp = {0, 0, 0};
    for (int64_t p = 0; p < N; ++p) {
        known[p] = 0;
        if (fixed[p]) hpush(&hp, (hent){T[p], p, 0});
        else T[p] = INFINITY;
    }
    ctx_t c = {nx, nz, h, mats, mat_id, orient, T};
    int64_t npop = 0;
    g_phi_evals = 0;
    if (t_stop) *t_stop = INFINITY;
    while (hp.n > 0) {
        hent e = hpop(&hp);
        if (known[e.idx] || e.ver != ver[e.idx]) continue;   /* stale entry */
        int pi = (int)(e.idx % nx), pj = (int)(e.idx / nx);
        if (stop_r >= 0 && (abs(pi - ci) > stop_r || abs(pj - cj) > stop_r)) {
            if (t_stop) *t_stop = e.t;
            break;
        }
        known[e.idx] = 1;
        if (pop_order) pop_order[npop] = e.idx;
        if (pop_values) pop_values[npop] = e.t;
        ++npop;
        for (int k = 0; k < 12; ++k) {
            int di = pi + DIAMOND[k][0], dj = pj + DIAMOND[k][1];
            if (!in_grid(&c, di, dj)) continue;
            int64_t d = (int64_t)dj * nx + di;
            if (known[d] || fixed[d]) continue;
            double u = phi_core(&c, di, dj, known12_from_grid(&c, known, di, dj), NULL);
            ++g_phi_evals;
            if ((g_variant & OR_VAR_MIN_UPDATE) && !(u < T[d])) continue;
            if (u != T[d]) {                                  /* R4: recompute */
                T[d] = u;
                ++ver[d];
                if (isfinite(u)) hpush(&hp, (hent){u, d, ver[d]});
            }
        }
    }
    free(hp.a); free(ver);
    return npop;
}

int64_t or_solve_fmm(int nx, int nz, double h, const or_material* mats, int n_mats,
                     const uint8_t* mat_id, const double* orient, int si, int sj, int R,
                     double* T, int64_t* pop_order, double* pop_values) {
    if (!valid_inputs(nx, nz, h, mats, n_mats, mat_id, orient, si, sj)) return -1;
    int64_t N = (int64_t)nx * nz;
    uint8_t* fixed = calloc(N, 1);
    uint8_t* known = calloc(N, 1);
    for (int64_t p = 0; p < N; ++p) T[p] = INFINITY;
    or_source_box(nx, nz, h, mats, mat_id, orient, si, sj, R, T, fixed);
    int64_t npop = fmm_core(nx, nz, h, mats, mat_id, orient, fixed, T, si, sj, -1, known, pop_order,
                            pop_values, NULL);
    free(fixed); free(known);
    return npop;
}

int64_t or_fmm_seeded(int nx, int nz, double h, const or_material* mats, int n_mats, const uint8_t* mat_id,
                      const double* orient, const uint8_t* fixed, double* T, int ci, int cj, int stop_r,
                      uint8_t* known, double* t_stop) {
    if (!valid_inputs(nx, nz, h, mats, n_mats, mat_id, orient, ci, cj)) return -1;
    return fmm_core(nx, nz, h, mats, mat_id, orient, fixed, T, ci, cj, stop_r, known, NULL, NULL, t_stop);
}

/* ---- The local operator and an independent sweeping driver -------------------------- */
double or_localfmm(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                   const double* orient, const double* T, int i, int j, int* choice) {
    ctx_t c = {nx, nz, h, mats, mat_id, orient, T};
    int64_t idx_d = (int64_t)j * nx + i;
    /* finite diamond neighbours sorted by key (tau, linear index) */
    int slot[12], m = 0;
    for (int k = 0; k < 12; ++k) {
        int ni = i + DIAMOND[k][0], nj = j + DIAMOND[k][1];
        if (in_grid(&c, ni, nj) && isfinite(T[nj * nx + ni])) slot[m++] = k;
    }
    for (int a = 1; a < m; ++a)                               /* insertion sort by key */
        for (int b = a; b > 0; --b) {
            int k1 = slot[b - 1], k2 = slot[b];
            int64_t i1 = (int64_t)(j + DIAMOND[k1][1]) * nx + (i + DIAMOND[k1][0]);
            int64_t i2 = (int64_t)(j + DIAMOND[k2][1]) * nx + (i + DIAMOND[k2][0]);
            double t1 = T[i1], t2 = T[i2];
            if (t2 < t1 || (t2 == t1 && i2 < i1)) { slot[b - 1] = k2; slot[b] = k1; }
            else break;
        }
    unsigned known12 = 0;
    for (int k = 0; k <= m; ++k) {
        int ch = -1;
        double u = k == 0 ? INFINITY : phi_core(&c, i, j, known12, &ch);
        if (k == m) { if (choice) *choice = ch; return u; }
        int kn = slot[k];
        int64_t in = (int64_t)(j + DIAMOND[kn][1]) * nx + (i + DIAMOND[kn][0]);
        double tn = T[in];
        if (u < tn || (u == tn && idx_d < in)) { if (choice) *choice = ch; return u; }
        known12 |= 1u << kn;
    }
    return INFINITY; /* not reached */
}

int or_sweep_solve(int nx, int nz, double h, const or_material* mats, int n_mats,
                   const uint8_t* mat_id, const double* orient, int si, int sj, int R,
                   int max_sweeps, double* T) {
    if (!valid_inputs(nx, nz, h, mats, n_mats, mat_id, orient, si, sj)) return -2;
    int64_t N = (int64_t)nx * nz;
    uint8_t* fixed = calloc(N, 1);
    for (int64_t p = 0; p < N; ++p) T[p] = INFINITY;
    or_source_box(nx, nz, h, mats, mat_id, orient, si, sj, R, T, fixed);
    int sweeps = 0, done = 0;
    while (!done && sweeps < max_sweeps) {
        int changed = 0;
        /* alternate the four raster directions */
        int dir = sweeps & 3;
        for (int jj = 0; jj < nz; ++jj)
            for (int ii = 0; ii < nx; ++ii) {
                int i = (dir & 1) ? nx - 1 - ii : ii;
                int j = (dir & 2) ? nz - 1 - jj : jj;
                int64_t p = (int64_t)j * nx + i;
                if (fixed[p]) continue;
                double u = or_localfmm(nx, nz, h, mats, mat_id, orient, T, i, j, NULL);
                if (!(u == T[p] || (isinf(u) && isinf(T[p])))) { T[p] = u; changed = 1; }
            }
        ++sweeps;
        done = !changed;
    }
    free(fixed);
    return done ? sweeps : -1;
}
