/*
 * rays.c -- oracle ray tracer through a finished travel-time field (paper Section 5.1).
 * TEST INFRASTRUCTURE ONLY.
 *
 * The field T has its source at S.  By reciprocity (Section 5.1) T(C) is also the time
 * from C to S, so a ray between a start point P0 and S is built from P0 one point at a
 * time: the next point lies on a plane (a grid line in 2-D) and minimises the straight
 * segment time from the last point plus T on the plane (Fermat).  Readings:
 *   - plane families: x = k, z = k, x + z = k, x - z = k, through grid nodes; the family
 *     is the one making the largest angle with the last segment (the first step uses the
 *     direction towards S);
 *   - the next plane is the family's plane at the rounded index of the last point plus
 *     one step towards the direction of travel;
 *   - candidates: points of that plane spaced 1/sub of the node spacing, at offsets
 *     q/sub, |q| <= window*sub - 1, from the grid node nearest to the straight-ahead
 *     intersection (the paper samples a finer subgrid and limits the candidates without
 *     giving a number); T at a candidate is linearly interpolated between the two grid
 *     nodes of the plane around it;
 *   - segment time: exact walk through the nearest-node cells at the group speed of each
 *     cell (equal to the paper's "orientation of the closest point" inside one cell);
 *   - a parabola through each local minimum of the candidate costs and its two
 *     neighbours; the next point is the vertex of the parabola with the smallest value
 *     (a minimum at the window edge is taken as is);
 *   - stop when the last point is closer than 1.6 node spacings to S, then append S;
 *   - fixed families (the paper's first variant: one family for the whole ray, each of the
 *     four tried and the fastest kept): the planes of that family strictly between the
 *     start and S, each crossed once in order.  The paper tests all points of the plane:
 *     every grid node of the plane is costed first, then the fine window above around the
 *     best node; the last point joins S directly, and a start on S's own plane gives the
 *     straight segment;
 *   - the ray's travel time is the sum of its segment times.
 */
#include <math.h>
#include <stdlib.h>
#include "ali_oracle.h"

/* plane families: normal N (the plane index of a point p is N.p) and the step E between
   consecutive grid nodes on one plane */
static const double FAM_N[4][2] = {{1, 0}, {0, 1}, {1, 1}, {1, -1}};
static const double FAM_E[4][2] = {{0, 1}, {1, 0}, {1, -1}, {1, 1}};

/* node of family f on plane index k with parameter m */
static void fam_node(int f, int k, int m, int* i, int* j) {
    switch (f) {
        case 0: *i = k; *j = m; break;          /* x = k, parameter z */
        case 1: *i = m; *j = k; break;          /* z = k, parameter x */
        case 2: *i = m; *j = k - m; break;      /* x + z = k, parameter x */
        default: *i = m; *j = m - k; break;     /* x - z = k, parameter x */
    }
}

/* parameters of the grid nodes on plane k of family f */
static void plane_range(int nx, int nz, int f, int k, int* lo, int* hi) {
    switch (f) {
        case 0: *lo = 0; *hi = nz - 1; break;
        case 1: *lo = 0; *hi = nx - 1; break;
        case 2: *lo = k - (nz - 1) > 0 ? k - (nz - 1) : 0; *hi = k < nx - 1 ? k : nx - 1; break;
        default: *lo = k > 0 ? k : 0; *hi = k + nz - 1 < nx - 1 ? k + nz - 1 : nx - 1; break;
    }
}

/* T at parameter u along plane k of family f: linear between the two grid nodes of the
   plane around u; +inf if either is outside the grid or unreached */
static double plane_T(int nx, int nz, const double* T, int f, int k, double u) {
    int m = (int)floor(u);
    double w = u - m;
    int i0, j0, i1, j1;
    fam_node(f, k, m, &i0, &j0);
    fam_node(f, k, m + 1, &i1, &j1);
    if (i0 < 0 || j0 < 0 || i0 >= nx || j0 >= nz) return INFINITY;
    double t0 = T[(int64_t)j0 * nx + i0];
    if (w == 0.0) return t0;
    if (i1 < 0 || j1 < 0 || i1 >= nx || j1 >= nz) return INFINITY;
    double t1 = T[(int64_t)j1 * nx + i1];
    return (1.0 - w) * t0 + w * t1;
}

int or_trace_ray(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                 const double* orient, const double* T, int si, int sj, int ri, int rj,
                 int window, int sub, int max_pts, double* pts, int* n_pts, double* t_ray) {
    return or_trace_ray_family(nx, nz, h, mats, mat_id, orient, T, si, sj, ri, rj, -1, window, sub, max_pts,
                               pts, n_pts, t_ray);
}

int or_trace_ray_family(int nx, int nz, double h, const or_material* mats, const uint8_t* mat_id,
                        const double* orient, const double* T, int si, int sj, int ri, int rj, int family,
                        int window, int sub, int max_pts, double* pts, int* n_pts, double* t_ray) {
    double px = ri, pz = rj;
    double dx = si - px, dz = sj - pz;
    int n = 0;
    double tt = 0.0;
    const int half = window * sub - 1;
    const int nc = 2 * half + 1;
    if (family < -1 || family > 3) return -1;
    double* cost = malloc(sizeof(double) * (size_t)nc);
    int* ok = malloc(sizeof(int) * (size_t)nc);
    pts[2 * n] = px; pts[2 * n + 1] = pz; ++n;
    int status = -1;
    /* a fixed family: the planes strictly between the start and S, in order; its plane
       index of S, and the side S lies on */
    const int kS = family >= 0 ? (int)(si * FAM_N[family][0] + sj * FAM_N[family][1]) : 0;
    const int k0 = family >= 0 ? (int)(ri * FAM_N[family][0] + rj * FAM_N[family][1]) : 0;
    const int fsgn = kS > k0 ? 1 : -1;
    while (n < max_pts) {
        int k, f, sgn;
        if (family < 0) {
            if (hypot(px - si, pz - sj) < 1.6) {
                if (px != si || pz != sj) {
                    tt += or_segment_time(nx, nz, h, mats, mat_id, orient, px, pz, si, sj);
                    pts[2 * n] = si; pts[2 * n + 1] = sj; ++n;
                }
                status = 0;
                break;
            }
            if (n + 1 >= max_pts) break;
            /* family whose planes make the largest angle with the direction of travel */
            f = 0;
            double best = 2.0, dl = hypot(dx, dz);
            for (int q = 0; q < 4; ++q) {
                double el = hypot(FAM_E[q][0], FAM_E[q][1]);
                double c = fabs(dx * FAM_E[q][0] + dz * FAM_E[q][1]) / (dl * el);   /* |cos| */
                if (c < best) { best = c; f = q; }
            }
            double dn0 = dx * FAM_N[f][0] + dz * FAM_N[f][1];
            sgn = dn0 > 0 ? 1 : -1;
            double ip0 = px * FAM_N[f][0] + pz * FAM_N[f][1];
            k = (int)floor(ip0 + 0.5) + sgn;
        } else {
            f = family;
            sgn = fsgn;
            double ip0 = px * FAM_N[f][0] + pz * FAM_N[f][1];
            k = (int)floor(ip0 + 0.5) + sgn;
            /* the next plane is S's (or the start already lies on it): close with S */
            if (kS == k0 || (k - kS) * sgn >= 0) {
                tt += or_segment_time(nx, nz, h, mats, mat_id, orient, px, pz, si, sj);
                pts[2 * n] = si; pts[2 * n + 1] = sj; ++n;
                status = 0;
                break;
            }
            if (n + 1 >= max_pts) break;
        }
        double dn = dx * FAM_N[f][0] + dz * FAM_N[f][1];
        double ip = px * FAM_N[f][0] + pz * FAM_N[f][1];
        /* point of parameter u on plane k: node(floor u) + frac(u) * E */
        int i00, j00;
        fam_node(f, k, 0, &i00, &j00);
        int m0;
        if (family < 0) {
            /* straight-ahead intersection and its parameter along the plane */
            double s = (k - ip) / dn;
            double xs = px + s * dx, zs = pz + s * dz;
            double ms = (f == 0) ? zs : xs;
            m0 = (int)floor(ms + 0.5);
        } else {
            /* a fixed family may meet the ray at any angle: every grid node of the plane
               is a candidate first, then the fine window around the best of them */
            int lo, hi;
            plane_range(nx, nz, f, k, &lo, &hi);
            double bc = INFINITY;
            m0 = lo;
            for (int mm = lo; mm <= hi; ++mm) {
                double tc = plane_T(nx, nz, T, f, k, (double)mm);
                if (!isfinite(tc)) continue;
                int ci, cj;
                fam_node(f, k, mm, &ci, &cj);
                double c = or_segment_time(nx, nz, h, mats, mat_id, orient, px, pz, ci, cj) + tc;
                if (c < bc) { bc = c; m0 = mm; }
            }
        }
        int any = 0;
        for (int q = 0; q < nc; ++q) {
            double u = m0 + (double)(q - half) / sub;
            ok[q] = 0;
            cost[q] = INFINITY;
            double tc = plane_T(nx, nz, T, f, k, u);
            if (!isfinite(tc)) continue;
            double cx = i00 + u * FAM_E[f][0], cz = j00 + u * FAM_E[f][1];
            cost[q] = or_segment_time(nx, nz, h, mats, mat_id, orient, px, pz, cx, cz) + tc;
            ok[q] = 1;
            any = 1;
        }
        if (!any) break;
        /* local minima, parabola refinement, smallest vertex */
        double bestv = INFINITY, bestpos = 0.0;
        int bestq = -1;
        for (int q = 0; q < nc; ++q) {
            if (!ok[q]) continue;
            int lok = q > 0 && ok[q - 1], rok = q < nc - 1 && ok[q + 1];
            if (lok && !(cost[q] < cost[q - 1])) continue;
            if (rok && !(cost[q] <= cost[q + 1])) continue;
            double v = cost[q], pos = 0.0;
            if (lok && rok) {
                double cm = cost[q - 1], c0 = cost[q], cp = cost[q + 1];
                double den = cm - 2.0 * c0 + cp;
                if (den > 0.0) {
                    pos = 0.5 * (cm - cp) / den;
                    v = c0 - 0.125 * (cp - cm) * (cp - cm) / den;
                }
            }
            if (v < bestv) { bestv = v; bestpos = pos; bestq = q; }
        }
        if (bestq < 0) break;
        double ub = m0 + ((double)(bestq - half) + bestpos) / sub;
        double qx = i00 + ub * FAM_E[f][0], qz = j00 + ub * FAM_E[f][1];
        tt += or_segment_time(nx, nz, h, mats, mat_id, orient, px, pz, qx, qz);
        dx = qx - px; dz = qz - pz;
        px = qx; pz = qz;
        pts[2 * n] = px; pts[2 * n + 1] = pz; ++n;
    }
    free(cost);
    free(ok);
    *n_pts = n;
    *t_ray = tt;
    return status;
}
