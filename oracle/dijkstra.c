/*
 * dijkstra.c -- dense-stencil Dijkstra reference and straight-segment times.
 * TEST INFRASTRUCTURE ONLY.
 *
 * The paper contrasts FMM with Dijkstra's algorithm on a graph whose edge weights are
 * single-segment travel times (Section 2).  With edges to every node within a radius and
 * exact segment times this is an independent discretisation of the same first-arrival
 * problem: it is exact for nodes a single straight segment reaches in a homogeneous
 * medium and an upper bound elsewhere.
 *
 * Segment time: the straight ray is cut where it crosses the boundaries of the
 * nearest-node cells; each piece travels at the group speed of its cell's material and
 * orientation along the segment direction (the time of a straight ray at group velocity,
 * Section 5.1).
 */
#include <math.h>
#include <stdlib.h>
#include "ali_oracle.h"

static int cmpd(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return x < y ? -1 : x > y;
}

double or_segment_time(int nx, int nz, double h, const or_material* mats,
                       const uint8_t* mat_id, const double* orient,
                       double x0, double z0, double x1, double z1) {
    double dx = x1 - x0, dz = z1 - z0;
    double len = sqrt(dx * dx + dz * dz);
    if (len == 0.0) return 0.0;
    double ang = atan2(dz, dx);
    /* parameters where the segment crosses the cell boundaries k + 1/2 */
    int cap = 2 * (int)(fabs(dx) + fabs(dz)) + 8, n = 0;
    double* ts = malloc(sizeof(double) * (size_t)cap);
    ts[n++] = 0.0;
    ts[n++] = 1.0;
    if (dx != 0.0) {
        double lo = fmin(x0, x1), hi = fmax(x0, x1);
        for (double b = floor(lo - 0.5) + 0.5; b <= hi; b += 1.0) {
            double t = (b - x0) / dx;
            if (t > 0.0 && t < 1.0 && n < cap) ts[n++] = t;
        }
    }
    if (dz != 0.0) {
        double lo = fmin(z0, z1), hi = fmax(z0, z1);
        for (double b = floor(lo - 0.5) + 0.5; b <= hi; b += 1.0) {
            double t = (b - z0) / dz;
            if (t > 0.0 && t < 1.0 && n < cap) ts[n++] = t;
        }
    }
    qsort(ts, (size_t)n, sizeof(double), cmpd);
    double total = 0.0;
    for (int k = 0; k + 1 < n; ++k) {
        double ta = ts[k], tb = ts[k + 1];
        if (tb <= ta) continue;
        double tm = 0.5 * (ta + tb);
        int ci = (int)floor(x0 + tm * dx + 0.5), cj = (int)floor(z0 + tm * dz + 0.5);
        if (ci < 0) ci = 0;
        if (cj < 0) cj = 0;
        if (ci >= nx) ci = nx - 1;
        if (cj >= nz) cj = nz - 1;
        int64_t p = (int64_t)cj * nx + ci;
        const or_material* m = &mats[mat_id[p]];
        double phi = ang - (orient[p] + 0.5 * M_PI);
        total += (tb - ta) * len * h / or_group_speed(m, phi);
    }
    free(ts);
    return total;
}

typedef struct { double t; int64_t idx; } dent;

static void dpush(dent** a, int64_t* n, int64_t* cap, dent e) {
    if (*n == *cap) { *cap = *cap ? 2 * *cap : 1024; *a = realloc(*a, (size_t)*cap * sizeof(dent)); }
    int64_t k = (*n)++;
    (*a)[k] = e;
    while (k > 0) {
        int64_t p = (k - 1) / 2;
        if ((*a)[p].t <= (*a)[k].t) break;
        dent t = (*a)[k]; (*a)[k] = (*a)[p]; (*a)[p] = t; k = p;
    }
}
static dent dpop(dent* a, int64_t* n) {
    dent top = a[0];
    a[0] = a[--(*n)];
    int64_t k = 0;
    for (;;) {
        int64_t l = 2 * k + 1, r = l + 1, s = k;
        if (l < *n && a[l].t < a[s].t) s = l;
        if (r < *n && a[r].t < a[s].t) s = r;
        if (s == k) break;
        dent t = a[k]; a[k] = a[s]; a[s] = t; k = s;
    }
    return top;
}

void or_dijkstra_dense(int nx, int nz, double h, const or_material* mats,
                       const uint8_t* mat_id, const double* orient, int si, int sj,
                       double rad, double* T) {
    int64_t N = (int64_t)nx * nz;
    int R = (int)floor(rad);
    uint8_t* done = calloc((size_t)N, 1);
    for (int64_t p = 0; p < N; ++p) T[p] = INFINITY;
    dent* hp = NULL;
    int64_t n = 0, cap = 0;
    T[(int64_t)sj * nx + si] = 0.0;
    dpush(&hp, &n, &cap, (dent){0.0, (int64_t)sj * nx + si});
    while (n > 0) {
        dent e = dpop(hp, &n);
        if (done[e.idx] || e.t > T[e.idx]) continue;
        done[e.idx] = 1;
        int pi = (int)(e.idx % nx), pj = (int)(e.idx / nx);
        for (int dj = -R; dj <= R; ++dj)
            for (int di = -R; di <= R; ++di) {
                if (di == 0 && dj == 0) continue;
                if ((double)(di * di + dj * dj) > rad * rad) continue;
                int qi = pi + di, qj = pj + dj;
                if (qi < 0 || qj < 0 || qi >= nx || qj >= nz) continue;
                int64_t q = (int64_t)qj * nx + qi;
                if (done[q]) continue;
                double t = e.t + or_segment_time(nx, nz, h, mats, mat_id, orient, pi, pj, qi, qj);
                if (t < T[q]) { T[q] = t; dpush(&hp, &n, &cap, (dent){t, q}); }
            }
    }
    free(hp);
    free(done);
}
