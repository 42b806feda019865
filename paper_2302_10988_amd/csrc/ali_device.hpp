// ali_device.hpp -- device-side arithmetic of the ALI update for gfx950.
//
// One node update (paper Sections 4.1-4.3): from the travel times of the 12-node diamond
// around D, evaluate every stencil of Tables 1-2 whose ordering tau_A < tau_B <= tau_C
// holds, keep the causal ones (estimate above tau_C), rank them (squares before
// triangles, then by score, then table order; straight-ray updates from 8-neighbours
// last) and return the value the heap-ordered Fast Marching method would assign.
//
// Estimate of one stencil, written for the GPU.  With a = (tau_B - tau_A)/(tau_C - tau_A),
// E = A + a (C - A), w = B - E and D at the origin, the paper's |FD| is
// |cross(w, D - E)| / |w| and cross(w, D - E) = k1 - a k2 with the integer stencil
// constants k1 = (B-A)x(D-A), k2 = (B-A)x(C-A) + (C-A)x(D-A).  The phase speed along the
// normal of EB needs only cos 2psi and sin 2psi of the normal against the symmetry axis,
// which are quadratic in w; so
//     |FD| / v = |k1 - a k2| / sqrt(G),   G = |w|^2 v^2
//     G = 1/4 ( P|w|^2 + Q c + sqrt((Q|w|^2 + R c)^2 + 4 W^2 s^2) )
// with c = |w|^2 cos 2psi, s = |w|^2 sin 2psi, P = A11+A33+2A55, Q = A33-A11,
// R = A11+A33-2A55, W = A13+A55 (A = stiffness / density), all divided by h^2 so that
// the result is in seconds.  No trigonometry and one sqrt + one rsqrt per stencil.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

namespace ali {

// ---------------------------------------------------------------------------------------
// math: raw hardware sqrt / rsqrt / rcp in float32 (<= 1 ulp), IEEE in float64
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ float dsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float drsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double drsqrt(double x) { return 1.0 / __builtin_sqrt(x); }
__device__ __forceinline__ float dratio(float num, float den) { return num * __builtin_amdgcn_rcpf(den); }
__device__ __forceinline__ double dratio(double num, double den) { return num / den; }
template <typename real> __device__ __forceinline__ real dinf();
template <> __device__ __forceinline__ float dinf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double dinf<double>() { return __builtin_huge_val(); }

// ---------------------------------------------------------------------------------------
// diamond slots, numbered in increasing linear-index order of the neighbour
//   0:(0,-2) 1:(-1,-1) 2:(0,-1) 3:(1,-1) 4:(-2,0) 5:(-1,0) 6:(1,0) 7:(2,0)
//   8:(-1,1) 9:(0,1) 10:(1,1) 11:(0,2)          offsets are (di, dj)
// slots 0..5 precede D in linear-index order, 6..11 follow it.
// ---------------------------------------------------------------------------------------
constexpr int SLOT_DI[12] = {0, -1, 0, 1, -2, -1, 1, 2, -1, 0, 1, 0};
constexpr int SLOT_DJ[12] = {-2, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 2};
// the same offsets for a slot number known only at run time
__host__ __device__ constexpr int SLOT_DI_RT(int k) {
    return (k == 1 || k == 5 || k == 8) ? -1 : (k == 3 || k == 6 || k == 10) ? 1 : k == 4 ? -2 : k == 7 ? 2 : 0;
}
__host__ __device__ constexpr int SLOT_DJ_RT(int k) { return k == 0 ? -2 : k <= 3 ? -1 : k <= 7 ? 0 : k <= 10 ? 1 : 2; }

// Tables 1-2 as 16 pairs (A, P, Q): member 1 has B = P, C = Q; member 2 swaps B and C.
// Pairs 1-4 are the unit squares, 5-8 the sqrt(2) squares, 9-16 the triangles (member 1:
// B axial, C diagonal).  Two printing errors are corrected: row 4-1's C and row 8-2's B.
constexpr int PAIR_A[16] = {1, 8, 10, 3, 4, 11, 0, 7, 11, 0, 0, 11, 4, 7, 7, 4};
constexpr int PAIR_P[16] = {2, 9, 6, 2, 1, 10, 3, 10, 9, 2, 2, 9, 5, 6, 6, 5};
constexpr int PAIR_Q[16] = {5, 5, 9, 6, 8, 8, 1, 3, 10, 3, 1, 8, 8, 10, 3, 1};

// the eight neighbours used by the straight-ray fallback, in linear-index order, and
// the grid direction of each (0: x axis, 1: (1,1) diagonal, 2: z axis, 3: (1,-1) diagonal)
constexpr int FB_SLOT[8] = {1, 2, 3, 5, 6, 8, 9, 10};
constexpr int FB_DIR[8] = {1, 2, 3, 0, 0, 3, 2, 1};

// stencil s = 2*pair + member (0-based member), table order 1-1, 1-2, 2-1, ..., 16-2
template <int S> struct Stencil {
    static constexpr int pair = S / 2;
    static constexpr bool second = (S & 1) != 0;
    static constexpr int sa = PAIR_A[pair];
    static constexpr int sb = second ? PAIR_Q[pair] : PAIR_P[pair];
    static constexpr int sc = second ? PAIR_P[pair] : PAIR_Q[pair];
    static constexpr int cls = pair < 8 ? 0 : 1;                 // 0 square, 1 triangle
    static constexpr int ax = SLOT_DI[sa], az = SLOT_DJ[sa];
    static constexpr int bx = SLOT_DI[sb] - ax, bz = SLOT_DJ[sb] - az;   // B - A
    static constexpr int cx = SLOT_DI[sc] - ax, cz = SLOT_DJ[sc] - az;   // C - A
    static constexpr int dx = -ax, dz = -az;                           // D - A
    static constexpr int k1 = bx * dz - bz * dx;
    static constexpr int k2 = (bx * cz - bz * cx) + (cx * dz - cz * dx);
    // kappa: the support point with the largest key; C unless tau_B == tau_C, then the
    // later of B and C in linear-index order
    static constexpr int tie_slot = sb > sc ? sb : sc;
};

// ---------------------------------------------------------------------------------------
// per-node constants
// ---------------------------------------------------------------------------------------
// mreal: type of the wavefront / phase-speed arithmetic; treal: type of travel times
// (stored values, scores, every comparison that makes a decision)
template <typename mreal, typename treal> struct NodeConst {
    static constexpr bool table = false;
    mreal c2t, s2t;         // cos 2theta, sin 2theta of the symmetry axis
    mreal P, Q, R, K4;      // phase-speed constants / h^2 (K4 = 4 W^2 / h^4)
    treal fb[4];            // straight-ray times to an 8-neighbour along the 4 grid directions
};

// The velocity-table variant: the phase speed comes from the node material's table of
// speeds / h at whole degrees (0..90) of the angle between the wavefront normal and the
// symmetry axis, linearly interpolated.
template <typename mreal, typename treal> struct NodeConstTab : NodeConst<mreal, treal> {
    static constexpr bool table = true;
    const mreal* vt;
};

// Running best candidate: rank = (class, score, table index), lexicographic.
template <typename real> struct Best {
    int cls;                // 0 square, 1 triangle, 2 straight ray, 3 none
    real score;
    real U;
    real kt;                // tau of the activation point (kappa)
    int ks;                 // diamond slot of the activation point
    int idx;                // table index 0..31, or 32 + neighbour order for a straight ray
    unsigned evals;         // single-stencil estimates computed (statistics only)
};

__device__ __forceinline__ float dfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double dfma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// travel time from the wavefront EB to D (|FD| / v) in the math type.  The multiply-adds
// are explicit fused operations and the build forbids implicit contraction, so every
// kernel that evaluates an estimate rounds it the same way.
template <typename real, typename treal, typename NC>
__device__ __forceinline__ real stencil_incr(const NC& n, real a, int bx, int bz,
                                             int cx, int cz, int k1, int k2) {
    // w = (B - A) - a (C - A)
    const real wx = dfma(-a, real(cx), real(bx));
    const real wz = dfma(-a, real(cz), real(bz));
    const real cr = dfma(-a, real(k2), real(k1));
    const real w2 = dfma(wx, wx, wz * wz);
    const real dd = dfma(wz, wz, -(wx * wx));        // |w|^2 cos 2phi_n
    const real xz = real(-2) * wx * wz;               // |w|^2 sin 2phi_n
    const real c = dfma(dd, n.c2t, xz * n.s2t);       // |w|^2 cos 2psi
    if constexpr (NC::table) {
        // psi in degrees from cos 2psi, then the table (v / h) between whole degrees
        real cc = c / w2;
        cc = cc > real(1) ? real(1) : (cc < real(-1) ? real(-1) : cc);
        const real deg = acos(cc) * real(28.647889756541160848);   // 90 / pi
        int i = (int)deg;
        i = i > 89 ? 89 : i;
        const real fr = deg - real(i);
        const real v = dfma(fr, n.vt[i + 1] - n.vt[i], n.vt[i]);
        return __builtin_fabs(cr) * drsqrt(w2 * v * v);
    }
    const real s2 = dfma(w2, w2, -(c * c));           // (|w|^2 sin 2psi)^2
    const real lin = dfma(n.Q, w2, n.R * c);
    const real G4 = dfma(n.P, w2, dfma(n.Q, c, dsqrt(dfma(lin, lin, n.K4 * s2))));   // 4 G
    // |FD|/v = |cr| / sqrt(G) = 2 |cr| / sqrt(4G)
    return real(2) * __builtin_fabs(cr) * drsqrt(G4);
}

// interpolation weight a = (tau_B - tau_A) / (tau_C - tau_A): differences in the time
// type, the ratio in the math type
template <typename mreal, typename treal>
__device__ __forceinline__ mreal interp_weight(treal ta, treal tb, treal tc) {
    return dratio((mreal)(tb - ta), (mreal)(tc - ta));
}

// Candidate of one member: estimate, causality, rank against the best so far.  Every lane
// runs the same instructions (selects, no branches).
template <typename mreal, typename real, typename NC>
__device__ __forceinline__ void member_candidate(const NC& n, const int8_t (&g)[6],
                                                 real tA, real tB, real tC, real score, bool ok, int cls,
                                                 int ks, int idx, Best<real>& best, real& minU) {
    best.evals += ok ? 1u : 0u;
    const mreal a = interp_weight<mreal, real>(tA, tB, tC);
    const real U = tB + (real)stencil_incr<mreal, real>(n, a, g[0], g[1], g[2], g[3], g[4], g[5]);
    const bool cand = ok && U > tC;                // causality
    minU = (cand && U < minU) ? U : minU;
    // table order is the evaluation order, so an equal score never displaces the best
    const bool better = cand && (cls < best.cls || (cls == best.cls && score < best.score));
    best.cls = better ? cls : best.cls;
    best.score = better ? score : best.score;
    best.U = better ? U : best.U;
    best.kt = better ? tC : best.kt;
    best.ks = better ? ks : best.ks;
    best.idx = better ? idx : best.idx;
}

// One stencil pair with compile-time geometry.  The two members order the same three
// points (member 1: B = P, C = Q; member 2: B = Q, C = P), so only one of them can satisfy
// tau_A < tau_B <= tau_C unless tau_P == tau_Q; the admissible member's geometry is picked
// by selects, so the lanes of a wave run the same instructions.  A tie evaluates member 2
// as well, after member 1 (table order).
template <typename mreal, typename real, int PAIR, typename NC>
__device__ __forceinline__ void eval_pair(const NC& n, const real (&t)[12],
                                          Best<real>& best, real& minU) {
    using S1 = Stencil<2 * PAIR>;
    using S2 = Stencil<2 * PAIR + 1>;
    const real inf = dinf<real>();
    const real tA = t[PAIR_A[PAIR]], tP = t[PAIR_P[PAIR]], tQ = t[PAIR_Q[PAIR]];
    const bool m1 = tP <= tQ;
    const real tB = m1 ? tP : tQ, tC = m1 ? tQ : tP;
    const bool ok = tA < tB && tC < inf;
    // score: squares by tau_C - tau_B; triangles (P axial, Q diagonal) by the distance of
    // the diagonal point's time from the isosceles interpolant (same for both members)
    const real r2m1 = real(0.41421356237309504880);   // sqrt(2) - 1
    const real tm = real(0.58578643762690495120);     // 2 - sqrt(2)
    const real score = S1::cls == 0 ? tC - tB : __builtin_fabs(tQ - (r2m1 * tA + tm * tP));
    const int ks = (tB == tC) ? S1::tie_slot : (m1 ? S1::sc : S2::sc);
    const int8_t g[6] = {(int8_t)(m1 ? S1::bx : S2::bx), (int8_t)(m1 ? S1::bz : S2::bz),
                         (int8_t)(m1 ? S1::cx : S2::cx), (int8_t)(m1 ? S1::cz : S2::cz),
                         (int8_t)(m1 ? S1::k1 : S2::k1), (int8_t)(m1 ? S1::k2 : S2::k2)};
    // a pair that no lane of the wave can use is skipped as a whole (wave-uniform branch;
    // lanes with ok == false contribute nothing through the selects either way)
    if (__ballot(ok) == 0ull) return;
    member_candidate<mreal, real>(n, g, tA, tB, tC, score, ok, S1::cls, ks, m1 ? 2 * PAIR : 2 * PAIR + 1, best, minU);
    if (tP == tQ && ok) {
        const int8_t g2[6] = {(int8_t)S2::bx, (int8_t)S2::bz, (int8_t)S2::cx, (int8_t)S2::cz, (int8_t)S2::k1, (int8_t)S2::k2};
        member_candidate<mreal, real>(n, g2, tA, tQ, tP, score, true, S1::cls, S1::tie_slot, 2 * PAIR + 1, best, minU);
    }
}

template <typename mreal, typename real, typename NC, int... P>
__device__ __forceinline__ void eval_pairs(const NC& n, const real (&t)[12],
                                           Best<real>& best, real& minU, std::integer_sequence<int, P...>) {
    (eval_pair<mreal, real, P>(n, t, best, minU), ...);
}

template <typename mreal, typename real, int K, typename NC>
__device__ __forceinline__ void eval_fallback(const NC& n, const real (&t)[12],
                                              Best<real>& best, real& minU) {
    const real tn = t[FB_SLOT[K]];
    const real U = tn + n.fb[FB_DIR[K]];
    const bool cand = tn < dinf<real>() && U > tn;
    minU = (cand && U < minU) ? U : minU;
    // class 2 ranks by value, then neighbour order (evaluated in that order)
    const bool better = cand && (best.cls > 2 || (best.cls == 2 && U < best.score));
    best.cls = better ? 2 : best.cls;
    best.score = better ? U : best.score;
    best.U = better ? U : best.U;
    best.kt = better ? tn : best.kt;
    best.ks = better ? FB_SLOT[K] : best.ks;
    best.idx = better ? 32 + K : best.idx;
}

template <typename mreal, typename real, typename NC, int... K>
__device__ __forceinline__ void eval_fallbacks(const NC& n, const real (&t)[12],
                                               Best<real>& best, real& minU,
                                               std::integer_sequence<int, K...>) {
    (eval_fallback<mreal, real, K>(n, t, best, minU), ...);
}

// key_D(u) > key(slot with time tk): D's linear index lies between slots 5 and 6
__device__ __forceinline__ bool key_after(float u, float tk, int ks) { return u > tk || (u == tk && ks <= 5); }
__device__ __forceinline__ bool key_after(double u, double tk, int ks) { return u > tk || (u == tk && ks <= 5); }

// ---------------------------------------------------------------------------------------
// Exact slow path: walk the activation points (8-neighbours with a finite time) in key
// order.  At each one, the candidate activated there is the best stencil (by class,
// score, table order) whose activation point it is, or else the straight ray from it.
// The answer is the first record (a candidate better than all activated before it) whose
// value lies below the key of the next record's activation point.  Used only when the
// fast test is inconclusive (rare).  First every pair is evaluated again with the fast
// path's arithmetic and wave-level skip, keeping per activation point the best member
// activated there; then the walk finds each next point by a scan over registers.  No
// table or memory access happens inside the walk.
// ---------------------------------------------------------------------------------------
__host__ __device__ constexpr int fb_slot_rt(int k) {
    return k == 0 ? 1 : k == 1 ? 2 : k == 2 ? 3 : k == 3 ? 5 : k == 4 ? 6 : k == 5 ? 8 : k == 6 ? 9 : 10;
}
__host__ __device__ constexpr int fb_dir_rt(int k) {
    return k == 0 ? 1 : k == 1 ? 2 : k == 2 ? 3 : k == 3 ? 0 : k == 4 ? 0 : k == 5 ? 3 : k == 6 ? 2 : 1;
}

// best stencil member activated at each 8-neighbour k (FB_SLOT[k])
template <typename real> struct ActBest {
    int ci[8];              // class * 64 + table index; 3 * 64: none
    real score[8];
    real U[8];
};

template <typename real>
__device__ __forceinline__ void act_member(int ks, int cls, int idx, real score, real U, bool cand,
                                           ActBest<real>& ab) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int c = ab.ci[k] >> 6;
        // members arrive in table order, so an equal score keeps the earlier one
        const bool upd = cand && ks == FB_SLOT[k] && (cls < c || (cls == c && score < ab.score[k]));
        ab.ci[k] = upd ? cls * 64 + idx : ab.ci[k];
        ab.score[k] = upd ? score : ab.score[k];
        ab.U[k] = upd ? U : ab.U[k];
    }
}

template <typename mreal, typename real, int PAIR, typename NC>
__device__ __forceinline__ void act_pair(const NC& n, const real (&t)[12], ActBest<real>& ab) {
    using S1 = Stencil<2 * PAIR>;
    using S2 = Stencil<2 * PAIR + 1>;
    const real inf = dinf<real>();
    const real tA = t[PAIR_A[PAIR]], tP = t[PAIR_P[PAIR]], tQ = t[PAIR_Q[PAIR]];
    const bool m1 = tP <= tQ;
    const real tB = m1 ? tP : tQ, tC = m1 ? tQ : tP;
    const bool ok = tA < tB && tC < inf;
    if (__ballot(ok) == 0ull) return;
    const real r2m1 = real(0.41421356237309504880);
    const real tm = real(0.58578643762690495120);
    const real score = S1::cls == 0 ? tC - tB : __builtin_fabs(tQ - (r2m1 * tA + tm * tP));
    const int ks = (tB == tC) ? S1::tie_slot : (m1 ? S1::sc : S2::sc);
    const mreal a = interp_weight<mreal, real>(tA, tB, tC);
    const real U = tB + (real)stencil_incr<mreal, real>(n, a, m1 ? S1::bx : S2::bx, m1 ? S1::bz : S2::bz,
                                                        m1 ? S1::cx : S2::cx, m1 ? S1::cz : S2::cz,
                                                        m1 ? S1::k1 : S2::k1, m1 ? S1::k2 : S2::k2);
    act_member<real>(ks, S1::cls, m1 ? 2 * PAIR : 2 * PAIR + 1, score, U, ok && U > tC, ab);
    if (tP == tQ && ok) {
        // tie: member 2 as well (B = Q, C = P), after member 1
        const mreal a2 = interp_weight<mreal, real>(tA, tQ, tP);
        const real U2 = tQ + (real)stencil_incr<mreal, real>(n, a2, S2::bx, S2::bz, S2::cx, S2::cz, S2::k1, S2::k2);
        act_member<real>(S1::tie_slot, S1::cls, 2 * PAIR + 1, score, U2, U2 > tP, ab);
    }
}

template <typename mreal, typename real, typename NC, int... P>
__device__ __forceinline__ void act_pairs(const NC& n, const real (&t)[12], ActBest<real>& ab,
                                          std::integer_sequence<int, P...>) {
    (act_pair<mreal, real, P>(n, t, ab), ...);
}

// v[q] for a run-time q: a switch (a chain of selects is folded back into an indexed
// load, which puts the array in scratch memory)
template <typename T> __device__ __forceinline__ T pick8(const T (&v)[8], int q) {
    switch (q) {
        case 1: return v[1]; case 2: return v[2]; case 3: return v[3]; case 4: return v[4];
        case 5: return v[5]; case 6: return v[6]; case 7: return v[7]; default: return v[0];
    }
}

template <typename mreal, typename real, typename NC>
__device__ __noinline__ real slow_update(const NC n, const real* __restrict__ lds,
                                         int me, int stride, int* choice) {
    const real inf = dinf<real>();
    real t[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = lds[me + SLOT_DJ[k] * stride + SLOT_DI[k]];
    ActBest<real> ab;
#pragma unroll
    for (int k = 0; k < 8; ++k) { ab.ci[k] = 3 * 64; ab.score[k] = inf; ab.U[k] = inf; }
    act_pairs<mreal, real>(n, t, ab, std::make_integer_sequence<int, 16>{});

    int rci = 3 * 64;                 // record: class * 64 + index
    real rscore = inf, rU = inf;
    real prev_t = -inf;
    int prev_k = -1;
#pragma unroll 1
    for (int step = 0; step < 8; ++step) {
        // next activation point in key order (time, then linear-index order = k order)
        int q = -1;
        real tq = inf;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const real tk = t[FB_SLOT[k]];
            const bool after = tk > prev_t || (tk == prev_t && k > prev_k);
            const bool take = tk < inf && after && (q < 0 || tk < tq);
            q = take ? k : q;
            tq = take ? tk : tq;
        }
        if (q < 0) break;
        int ci = pick8(ab.ci, q);
        real cs = pick8(ab.score, q), cu = pick8(ab.U, q);
        if ((ci >> 6) == 3) {
            // no stencil activated here: the straight ray from this neighbour
            const int d = fb_dir_rt(q);
            const real fbt = d == 0 ? n.fb[0] : d == 1 ? n.fb[1] : d == 2 ? n.fb[2] : n.fb[3];
            const real U = tq + fbt;
            if (U > tq) { ci = 2 * 64 + 32 + q; cs = U; cu = U; }
        }
        const int ccls = ci >> 6, cidx = ci & 63;
        if (ccls < 3) {
            const int rcls = rci >> 6, ridx = rci & 63;
            const bool better = ccls < rcls || (ccls == rcls && (cs < rscore || (cs == rscore && cidx < ridx)));
            if (better) {
                if (rcls < 3 && !key_after(rU, tq, fb_slot_rt(q))) { *choice = ridx; return rU; }   // record below next key
                rci = ci; rscore = cs; rU = cu;
            }
        }
        prev_t = tq;
        prev_k = q;
    }
    *choice = (rci >> 6) < 3 ? (rci & 63) : -1;
    return (rci >> 6) < 3 ? rU : inf;
}

// ---------------------------------------------------------------------------------------
// The local update.  Fast test: let B be the best candidate overall and kappa_B its
// activation key.  If every candidate's value lies above kappa_B, no record activated
// before B can satisfy the stopping rule, so the heap's answer is B's value.
// ---------------------------------------------------------------------------------------
// t: the 12 diamond values (copied from lds[me + dj*stride + di]); the slow path
// reads them again from lds.
// choice (nullable) receives the chosen candidate: table index 0..31, 32 + k for a
// straight ray from the k-th 8-neighbour, -1 for none.
template <typename mreal, typename real, typename NC>
__device__ __forceinline__ real local_update(const NC& n, const real (&t)[12],
                                             const real* __restrict__ lds, int me, int stride,
                                             unsigned& evals, int* choice = nullptr) {
    const real inf = dinf<real>();
    Best<real> best;
    best.cls = 3; best.score = inf; best.U = inf; best.kt = inf; best.ks = 0; best.idx = -1; best.evals = 0;
    real minU = inf;
    eval_pairs<mreal, real>(n, t, best, minU, std::make_integer_sequence<int, 16>{});
    eval_fallbacks<mreal, real>(n, t, best, minU, std::make_integer_sequence<int, 8>{});
    evals += best.evals;
    if (best.cls == 3) { if (choice) *choice = -1; return inf; }
    if (key_after(minU, best.kt, best.ks)) { if (choice) *choice = best.idx; return best.U; }
    int ch = -1;
    const real u = slow_update<mreal, real>(n, lds, me, stride, &ch);
    if (choice) *choice = ch;
    return u;
}

}  // namespace ali
