/*
 * velocity.c -- oracle velocities (paper Section 3).  TEST INFRASTRUCTURE ONLY.
 *
 * The medium is orthotropic/TI and waves stay in the plane that contains the symmetry
 * axis.  Following Section 3.2, the in-plane Christoffel matrix for phase direction
 * (cos th, sin th) (th from the c22 axis) is
 *     [ alpha beta ; beta gamma ],  alpha = cos^2 c22 + sin^2 c44,
 *                                   beta  = cos sin (c23 + c44),
 *                                   gamma = cos^2 c44 + sin^2 c33,
 * and the qP eigenvalue is the largest root ((alpha+gamma) + sqrt((alpha-gamma)^2+4beta^2))/2
 * (the eigenvalues of M divided by rho give v^2; Section 3.1).
 *
 * Group velocity (Section 3.1): differentiating rho w^2 = C_ijql k_j k_l p_q p_i (the
 * Christoffel equation as derived in the paper) with respect to k_m gives
 *     V_m = C_imql p_i p_q n_l / (rho v).
 * The printed final formula divides by rho*omega and places the polarisation on the first
 * two tensor indices; both are read as printing slips (omega -> v, and the index order
 * that the derivation itself produces).
 */
#include <math.h>
#include "ali_oracle.h"

/* In-plane stiffness tensor C_ijkl, i,j,k,l in {0 = y (c22 axis), 1 = z (symmetry
   axis)}, from the Voigt matrix with the paper's index map f(i,j) (Section 3.2):
   f(y,y) = 2, f(z,z) = 3, f(y,z) = 4. */
static double cvoigt(const or_material* m, int vi, int vj) {
    /* Voigt entries that matter in the plane: c22, c33, c23, c44 (paper notation). */
    if (vi > vj) { int t = vi; vi = vj; vj = t; }
    if (vi == 2 && vj == 2) return m->c11;   /* c22 */
    if (vi == 3 && vj == 3) return m->c33;   /* c33 */
    if (vi == 2 && vj == 3) return m->c13;   /* c23 */
    if (vi == 4 && vj == 4) return m->c55;   /* c44 (in-plane shear) */
    return 0.0;
}
static int fmap(int i, int j) { return i == j ? (i == 0 ? 2 : 3) : 4; }
static double cijkl(const or_material* m, int i, int j, int k, int l) {
    return cvoigt(m, fmap(i, j), fmap(k, l));
}

static void christoffel(const or_material* m, double th, double* al, double* be, double* ga) {
    double c = cos(th), s = sin(th);
    *al = c * c * m->c11 + s * s * m->c55;
    *be = c * s * (m->c13 + m->c55);
    *ga = c * c * m->c55 + s * s * m->c33;
}

static double qp_lambda(double al, double be, double ga) {
    return 0.5 * ((al + ga) + sqrt((al - ga) * (al - ga) + 4.0 * be * be));
}

double or_qp_phase_speed(const or_material* m, double th_p) {
    double al, be, ga;
    christoffel(m, th_p, &al, &be, &ga);
    return sqrt(qp_lambda(al, be, ga) / m->rho);
}

/* d v / d th_p of the qP phase speed, by differentiating the closed-form root:
   alpha' = 2 sin cos (c44 - c22), gamma' = 2 sin cos (c33 - c44),
   beta' = (cos^2 - sin^2)(c23 + c44), lambda' from the root, v' = lambda' / (2 rho v). */
double or_qp_phase_speed_deriv(const or_material* m, double th_p) {
    double al, be, ga;
    christoffel(m, th_p, &al, &be, &ga);
    double c = cos(th_p), s = sin(th_p);
    double dal = 2.0 * s * c * (m->c55 - m->c11);
    double dga = 2.0 * s * c * (m->c33 - m->c55);
    double dbe = (c * c - s * s) * (m->c13 + m->c55);
    double root = sqrt((al - ga) * (al - ga) + 4.0 * be * be);
    double dlam = 0.5 * ((dal + dga) + (root > 0.0 ? ((al - ga) * (dal - dga) + 4.0 * be * dbe) / root : 0.0));
    double v = sqrt(qp_lambda(al, be, ga) / m->rho);
    return dlam / (2.0 * m->rho * v);
}

/* qP eigenvalue (rho v^2) and unit polarisation p at phase angle th_p */
static double qp_polarisation(const or_material* m, double th_p, double p[2]) {
    double al, be, ga;
    christoffel(m, th_p, &al, &be, &ga);
    double lam = qp_lambda(al, be, ga);
    /* unit eigenvector of [al be; be ga] for lam: take the better conditioned of the two
       equivalent forms (be, lam-al) and (lam-ga, be). */
    double p0a = be, p1a = lam - al;
    double p0b = lam - ga, p1b = be;
    double na = p0a * p0a + p1a * p1a, nb = p0b * p0b + p1b * p1b;
    if (na >= nb) { double r = sqrt(na); p[0] = p0a / r; p[1] = p1a / r; }
    else          { double r = sqrt(nb); p[0] = p0b / r; p[1] = p1b / r; }
    if (na == 0.0 && nb == 0.0) {          /* degenerate (isotropic point): p = n */
        p[0] = cos(th_p); p[1] = sin(th_p);
    }
    return lam;
}

void or_qp_group_from_phase(const or_material* m, double th_p, double* g_angle, double* g_speed) {
    double p[2];
    double lam = qp_polarisation(m, th_p, p);
    double v = sqrt(lam / m->rho);
    double n[2] = {cos(th_p), sin(th_p)};
    double V[2] = {0.0, 0.0};
    for (int mm = 0; mm < 2; ++mm)
        for (int i = 0; i < 2; ++i)
            for (int q = 0; q < 2; ++q)
                for (int l = 0; l < 2; ++l)
                    V[mm] += cijkl(m, i, mm, q, l) * p[i] * p[q] * n[l];
    V[0] /= (m->rho * v);
    V[1] /= (m->rho * v);
    *g_angle = atan2(V[1], V[0]);
    *g_speed = sqrt(V[0] * V[0] + V[1] * V[1]);
}

/* Reduce an angle to [0, pi/2] using the two mirror symmetries of an orthotropic
   velocity curve (symmetric about the c22 axis and about the symmetry axis). */
static double reduce_quadrant(double a) {
    a = fmod(fabs(a), M_PI);
    if (a > 0.5 * M_PI) a = M_PI - a;
    return a;
}

double or_qp_group_speed(const or_material* m, double phi) {
    double target = reduce_quadrant(phi);
    double lo = 0.0, hi = 0.5 * M_PI, ga, gs;
    /* the qP group angle increases monotonically with the phase angle on [0, pi/2]
       (convex slowness curve; checked by the tests) -> plain bisection */
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        or_qp_group_from_phase(m, mid, &ga, &gs);
        if (ga < target) lo = mid; else hi = mid;
    }
    or_qp_group_from_phase(m, 0.5 * (lo + hi), &ga, &gs);
    return gs;
}

static double support_route(const or_material* m, double phi, double (*vphase)(const or_material*, double)) {
    /* maximise f(psi) = cos(phi - psi) / v(psi) over psi in (phi - pi/2, phi + pi/2):
       coarse scan, then golden-section refinement of the best bracket */
    const int N = 7200;
    double best = -1.0, bpsi = phi;
    for (int k = 1; k < N; ++k) {
        double psi = phi - 0.5 * M_PI + M_PI * (double)k / N;
        double f = cos(phi - psi) / vphase(m, psi);
        if (f > best) { best = f; bpsi = psi; }
    }
    double a = bpsi - M_PI / N, b = bpsi + M_PI / N;
    const double gr = 0.5 * (sqrt(5.0) - 1.0);
    double c = b - gr * (b - a), d = a + gr * (b - a);
    double fc = cos(phi - c) / vphase(m, c);
    double fd = cos(phi - d) / vphase(m, d);
    for (int it = 0; it < 200 && (b - a) > 1e-13; ++it) {
        if (fc > fd) { b = d; d = c; fd = fc; c = b - gr * (b - a); fc = cos(phi - c) / vphase(m, c); }
        else         { a = c; c = d; fc = fd; d = a + gr * (b - a); fd = cos(phi - d) / vphase(m, d); }
    }
    double f = fc > fd ? fc : fd;
    if (best > f) f = best;
    return 1.0 / f;
}

double or_qp_group_speed_support(const or_material* m, double phi) {
    return support_route(m, phi, or_qp_phase_speed);
}

/* d V_group / d phi by Richardson-extrapolated central differences of the exact group
   speed (step 1e-3 rad; truncation error far below the other tolerances). */
double or_qp_group_speed_deriv(const or_material* m, double phi) {
    const double h1 = 1e-3, h2 = 0.5e-3;
    double d1 = (or_qp_group_speed(m, phi + h1) - or_qp_group_speed(m, phi - h1)) / (2.0 * h1);
    double d2 = (or_qp_group_speed(m, phi + h2) - or_qp_group_speed(m, phi - h2)) / (2.0 * h2);
    return (4.0 * d2 - d1) / 3.0;
}

/* d v / d A of the qP phase speed at phase angle th_p, A = C / rho (order A11, A13, A33,
   A55).  First-order eigenvalue perturbation of the symmetric Christoffel matrix: the
   change of the qP eigenvalue is p^T dGamma p for the unit polarisation p, and
   v^2 = lambda / rho, so dv/dA_k = rho (p^T dGamma/dc_k p) / (2 rho v). */
void or_qp_phase_speed_dA(const or_material* m, double th_p, double dv[4]) {
    double p[2];
    double lam = qp_polarisation(m, th_p, p);
    double v = sqrt(lam / m->rho);
    double c = cos(th_p), s = sin(th_p);
    /* dGamma/dc11 = [c^2 0; 0 0], dGamma/dc13 = [0 cs; cs 0], dGamma/dc33 = [0 0; 0 s^2],
       dGamma/dc55 = [s^2 cs; cs c^2] */
    double g11 = p[0] * p[0] * c * c;
    double g13 = 2.0 * p[0] * p[1] * c * s;
    double g33 = p[1] * p[1] * s * s;
    double g55 = p[0] * p[0] * s * s + 2.0 * p[0] * p[1] * c * s + p[1] * p[1] * c * c;
    double k = 1.0 / (2.0 * v);
    dv[0] = g11 * k;
    dv[1] = g13 * k;
    dv[2] = g33 * k;
    dv[3] = g55 * k;
}

/* d V / d A of the exact qP group speed at fixed group angle phi (order A11, A13, A33, A55)
   by Richardson-extrapolated central differences of or_qp_group_speed, steps of 1e-3 and
   5e-4 times (A11 + A33) / 2. */
void or_qp_group_speed_dA(const or_material* m, double phi, double dV[4]) {
    const double scale = 0.5 * (m->c11 + m->c33) / m->rho;
    for (int k = 0; k < 4; ++k) {
        double d[2];
        for (int r = 0; r < 2; ++r) {
            const double st = (r == 0 ? 1e-3 : 0.5e-3) * scale;
            or_material mp = *m, mm = *m;
            double* cp = k == 0 ? &mp.c11 : k == 1 ? &mp.c13 : k == 2 ? &mp.c33 : &mp.c55;
            double* cm = k == 0 ? &mm.c11 : k == 1 ? &mm.c13 : k == 2 ? &mm.c33 : &mm.c55;
            *cp += st * m->rho;
            *cm -= st * m->rho;
            d[r] = (or_qp_group_speed(&mp, phi) - or_qp_group_speed(&mm, phi)) / (2.0 * st);
        }
        dV[k] = (4.0 * d[1] - d[0]) / 3.0;
    }
}

/* ---- SH: the wave polarised normal to the plane ----------------------------------------
   Its Christoffel entry is C_2j2l n_j n_l = c66 n1^2 + c44 n3^2 for the in-plane direction
   n = (n1 across the axis, n3 along it): an elliptical slowness curve, so the wave surface
   is an ellipse and the group speed has a closed form. */
double or_sh_phase_speed(const or_material* m, double th_p) {
    double c = cos(th_p), s = sin(th_p);
    return sqrt((m->c66 * c * c + m->c44 * s * s) / m->rho);
}

double or_sh_phase_speed_deriv(const or_material* m, double th_p) {
    double v = or_sh_phase_speed(m, th_p);
    return (m->c44 - m->c66) * sin(2.0 * th_p) / (2.0 * m->rho * v);
}

double or_sh_group_speed(const or_material* m, double phi) {
    double c = cos(phi), s = sin(phi);
    return 1.0 / sqrt(c * c * m->rho / m->c66 + s * s * m->rho / m->c44);
}

double or_sh_group_speed_deriv(const or_material* m, double phi) {
    double V = or_sh_group_speed(m, phi);
    /* V^-2 = cos^2 rho/c66 + sin^2 rho/c44 */
    double dinv2 = sin(2.0 * phi) * (m->rho / m->c44 - m->rho / m->c66);
    return -0.5 * V * V * V * dinv2;
}

double or_qp_group_speed_paper(const or_material* m, double phi) {
    /* c22, c33, c23, c44 of the paper's YZ plane are c11, c33, c13, c55 of the axis frame */
    const double c22 = m->c11, c33 = m->c33, c23 = m->c13, c44 = m->c55;
    const double a = reduce_quadrant(phi);
    if (a == 0.0) return sqrt(c22 / m->rho);              /* group = phase on the axes */
    if (a == 0.5 * M_PI) return sqrt(c33 / m->rho);
    /* delta cos 2th + eta sin 2th + kappa = 0 with y = tan th:
       y^2 (kappa - delta) + 2 eta y + (delta + kappa) = 0, the root of the qP mode for a
       group angle in (0, 90) degrees */
    const double delta = c22 + c33 - 2.0 * c44;
    const double eta = (c23 + c44) * (tan(a) - 1.0 / tan(a));
    const double kappa = c22 - c33;
    const double y = (-eta - sqrt(eta * eta + delta * delta - kappa * kappa)) / (kappa - delta);
    double th = fmod(atan(y), M_PI);
    if (th < 0.0) th += M_PI;
    const double lam = 0.5 * (cos(2.0 * th) * (c22 - c44) + sin(2.0 * th) * (c23 + c44) * tan(a) + (c22 + c44));
    return sqrt(lam / m->rho) / cos(th - a);
}

static double exact_phase_speed(const or_material* m, double th_p) {
    return m->wave == OR_WAVE_SH ? or_sh_phase_speed(m, th_p) : or_qp_phase_speed(m, th_p);
}
static double exact_group_speed(const or_material* m, double phi) {
    if (m->wave == OR_WAVE_SH) return or_sh_group_speed(m, phi);
    return m->grule == OR_GROUP_PAPER ? or_qp_group_speed_paper(m, phi) : or_qp_group_speed(m, phi);
}

/* the velocity table: f at whole degrees of the angle, linear in between (f is pi-periodic) */
static double table_lookup(const or_material* m, double ang, double (*f)(const or_material*, double)) {
    double d = fmod(ang * (180.0 / M_PI), 180.0);
    if (d < 0.0) d += 180.0;
    double i = floor(d);
    double w = d - i;
    double a = f(m, i * (M_PI / 180.0));
    if (w == 0.0) return a;
    double b = f(m, (i + 1.0) * (M_PI / 180.0));
    return (1.0 - w) * a + w * b;
}

/* derivative of the table's interpolant in the angle [per radian]: the slope of the
   whole-degree interval the angle lies in (at a whole degree, the interval above it, as
   table_lookup reads it) */
static double table_slope(const or_material* m, double ang, double (*f)(const or_material*, double)) {
    double d = fmod(ang * (180.0 / M_PI), 180.0);
    if (d < 0.0) d += 180.0;
    double i = floor(d);
    return (f(m, (i + 1.0) * (M_PI / 180.0)) - f(m, i * (M_PI / 180.0))) * (180.0 / M_PI);
}

double or_phase_speed(const or_material* m, double th_p) {
    return m->vtab ? table_lookup(m, th_p, exact_phase_speed) : exact_phase_speed(m, th_p);
}
double or_phase_speed_deriv(const or_material* m, double th_p) {
    if (m->vtab) return table_slope(m, th_p, exact_phase_speed);
    return m->wave == OR_WAVE_SH ? or_sh_phase_speed_deriv(m, th_p) : or_qp_phase_speed_deriv(m, th_p);
}
double or_group_speed(const or_material* m, double phi) {
    return m->vtab ? table_lookup(m, phi, exact_group_speed) : exact_group_speed(m, phi);
}
double or_group_speed_deriv(const or_material* m, double phi) {
    if (m->vtab) return table_slope(m, phi, exact_group_speed);
    return m->wave == OR_WAVE_SH ? or_sh_group_speed_deriv(m, phi) : or_qp_group_speed_deriv(m, phi);
}
double or_group_speed_support(const or_material* m, double phi) {
    return support_route(m, phi, or_phase_speed);
}
