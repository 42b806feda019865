// ali_velocity.hpp -- exact qP group speed on the device (float64), shared by the solver
// (straight-ray source box and fallback times) and the ray tracer (group-slowness tables).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace ali {

// ---------------------------------------------------------------------------------------
// Group speed along group angle phi measured from the symmetry axis (float64).
// Phase speed squared F(psi) = v^2 with psi the phase angle from the axis; the group
// direction is psi + atan(v'/v) and |V|^2 = v^2 + v'^2 (Section 3.1's |V| = |v|/cos).
// Inverted on [0, pi/2] (two mirror symmetries) by a bracketed Illinois iteration.
// ---------------------------------------------------------------------------------------
struct MatA { double a11, a13, a33, a55; };

__device__ inline void phase_F(const MatA& m, double psi, double& F, double& dF) {
    const double P = m.a11 + m.a33 + 2.0 * m.a55, Q = m.a33 - m.a11;
    const double R = m.a11 + m.a33 - 2.0 * m.a55, W = m.a13 + m.a55;
    double s, c;
    sincos(2.0 * psi, &s, &c);
    const double lin = Q + R * c;
    const double S = sqrt(lin * lin + 4.0 * W * W * s * s);
    F = 0.25 * (P + Q * c + S);
    const double dS = S > 0.0 ? (-2.0 * R * s * lin + 8.0 * W * W * s * c) / S : 0.0;
    dF = 0.25 * (-2.0 * Q * s + dS);
}

__device__ inline double group_angle_of(const MatA& m, double psi, double* speed) {
    double F, dF;
    phase_F(m, psi, F, dF);
    if (speed) *speed = sqrt(F + dF * dF / (4.0 * F));
    return psi + atan(dF / (2.0 * F));
}

// Phase angle x in [0, pi/2] whose group direction is phi folded onto [0, pi/2] (V is even
// and pi-periodic in phi); sgn is the sign that d/dphi takes through the fold.
__device__ inline double phase_of_group(const MatA& m, double phi, double& sgn_out) {
    const double half_pi = 1.57079632679489661923;
    // fold onto [0, pi/2]: V is even and pi-periodic in phi
    double a = fmod(fabs(phi), 2.0 * half_pi);
    double sgn = phi < 0.0 ? -1.0 : 1.0;
    if (a > half_pi) { a = 2.0 * half_pi - a; sgn = -sgn; }
    double lo = 0.0, hi = half_pi;
    double glo = -a, ghi = half_pi - a;
    double x = a;
    if (glo == 0.0) {
        x = 0.0;
    } else if (ghi == 0.0) {
        x = half_pi;
    } else {
        int side = 0;
        for (int it = 0; it < 100; ++it) {
            x = (lo * ghi - hi * glo) / (ghi - glo);
            if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
            const double g = group_angle_of(m, x, nullptr) - a;
            if (g == 0.0 || hi - lo < 1e-15) break;
            if (g < 0.0) {
                lo = x; glo = g;
                if (side == -1) ghi *= 0.5;
                side = -1;
            } else {
                hi = x; ghi = g;
                if (side == 1) glo *= 0.5;
                side = 1;
            }
        }
    }
    sgn_out = sgn;
    return x;
}

// Group speed V and, if dV != nullptr, dV/dphi.  With psi the phase angle whose group
// direction is phi, tan(phi - psi) = v'/v and dV/dphi = V v'/v (differentiate
// V^2 = v^2 + v'^2 and phi = psi + atan(v'/v) in psi and divide).
__device__ inline double group_speed(const MatA& m, double phi, double* dV = nullptr) {
    double sgn;
    const double x = phase_of_group(m, phi, sgn);
    double F, dF;
    phase_F(m, x, F, dF);
    const double spd = sqrt(F + dF * dF / (4.0 * F));
    if (dV) *dV = sgn * spd * dF / (2.0 * F);
    return spd;
}

// dF/dA of the phase speed squared at phase angle psi, A in the order a11, a13, a33, a55.
// F = (P + Q c + S) / 4 with S = sqrt((Q + R c)^2 + 4 W^2 s^2) (c, s of 2 psi) and P, Q, R,
// W linear in A.
__device__ inline void phase_F_dA(const MatA& m, double psi, double d[4]) {
    const double Q = m.a33 - m.a11, R = m.a11 + m.a33 - 2.0 * m.a55, W = m.a13 + m.a55;
    double s, c;
    sincos(2.0 * psi, &s, &c);
    const double lin = Q + R * c;
    const double S = sqrt(lin * lin + 4.0 * W * W * s * s);
    const double iS = S > 0.0 ? 1.0 / S : 0.0;
    const double fP = 0.25, fQ = 0.25 * (c + lin * iS), fR = 0.25 * lin * c * iS, fW = W * s * s * iS;
    d[0] = fP - fQ + fR;
    d[1] = fW;
    d[2] = fP + fQ + fR;
    d[3] = 2.0 * (fP - fR) + fW;
}

// Group speed V and dV/dA at a fixed group angle phi.  1/V(phi) is the largest value of
// cos(phi - psi) / v(psi) over phase angles psi, so by the envelope theorem only v moves:
// dV/dA = (V / v) dv/dA = V / (2 F) dF/dA at the phase angle that carries phi.
__device__ inline double group_speed_dA(const MatA& m, double phi, double d[4]) {
    double sgn;
    const double x = phase_of_group(m, phi, sgn);
    double F, dF;
    phase_F(m, x, F, dF);
    const double spd = sqrt(F + dF * dF / (4.0 * F));
    phase_F_dA(m, x, d);
    const double k = spd / (2.0 * F);
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] *= k;
    return spd;
}

// ---------------------------------------------------------------------------------------
// Velocity-table mode (the paper's cheaper variant): speeds at whole degrees of the angle
// from the symmetry axis, 0..90 (the curves are even and pi-periodic), linearly
// interpolated.  VT_N entries per material.
// ---------------------------------------------------------------------------------------
constexpr int VT_N = 91;

// group speed from the table gt[0..90] (group speed at whole degrees of the group angle)
__device__ inline double group_speed_tab(const double* __restrict__ gt, double phi) {
    const double pi = 3.14159265358979323846;
    double a = fmod(fabs(phi), pi);
    if (a > 0.5 * pi) a = pi - a;
    const double deg = a * (180.0 / pi);
    int i = (int)deg;
    i = i > 89 ? 89 : i;
    const double w = deg - i;
    return w == 0.0 ? gt[i] : (1.0 - w) * gt[i] + w * gt[i + 1];
}

// tables of one material: phase speed / h (vt) and group speed (gt) at whole degrees
template <typename mreal>
__global__ void k_vtables(const MatA* __restrict__ A, const double* __restrict__ ih, int n, mreal* __restrict__ vt,
                          double* __restrict__ gt) {
    const int m = blockIdx.x;
    const int k = threadIdx.x;
    if (m >= n || k >= VT_N) return;
    const double ang = k * (3.14159265358979323846 / 180.0);
    double F, dF;
    phase_F(A[m], ang, F, dF);
    if (vt) vt[m * VT_N + k] = (mreal)(sqrt(F) * ih[m]);
    if (gt) gt[m * VT_N + k] = group_speed(A[m], ang);
}

}  // namespace ali
