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

__device__ inline double group_speed(const MatA& m, double phi) {
    const double half_pi = 1.57079632679489661923;
    double a = fmod(fabs(phi), 2.0 * half_pi);
    if (a > half_pi) a = 2.0 * half_pi - a;
    double lo = 0.0, hi = half_pi;
    double glo = -a, ghi = half_pi - a;
    double spd;
    if (glo == 0.0) { group_angle_of(m, 0.0, &spd); return spd; }
    if (ghi == 0.0) { group_angle_of(m, half_pi, &spd); return spd; }
    int side = 0;
    double x = a;
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
    group_angle_of(m, x, &spd);
    return spd;
}


}  // namespace ali
