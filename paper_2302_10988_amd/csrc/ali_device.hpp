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
__host__ __device__ constexpr int fb_local(int slot) {
    return slot == 1 ? 0 : slot == 2 ? 1 : slot == 3 ? 2 : slot == 5 ? 3 : slot == 6 ? 4
         : slot == 8 ? 5 : slot == 9 ? 6 : slot == 10 ? 7 : -1;
}

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
    mreal c2t, s2t;         // cos 2theta, sin 2theta of the symmetry axis
    mreal P, Q, R, K4;      // phase-speed constants / h^2 (K4 = 4 W^2 / h^4)
    treal fb[4];            // straight-ray times to an 8-neighbour along the 4 grid directions
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

// travel time from the wavefront EB to D (|FD| / v) in the math type
template <typename real, typename treal>
__device__ __forceinline__ real stencil_incr(const NodeConst<real, treal>& n, real a, int bx, int bz,
                                             int cx, int cz, int k1, int k2) {
    // w = (B - A) - a (C - A)
    const real wx = real(bx) - a * real(cx);
    const real wz = real(bz) - a * real(cz);
    const real cr = real(k1) - a * real(k2);
    const real w2 = wx * wx + wz * wz;
    const real dd = wz * wz - wx * wx;            // |w|^2 cos 2phi_n
    const real xz = real(-2) * wx * wz;           // |w|^2 sin 2phi_n
    const real c = dd * n.c2t + xz * n.s2t;       // |w|^2 cos 2psi
    const real s2 = w2 * w2 - c * c;              // (|w|^2 sin 2psi)^2
    const real lin = n.Q * w2 + n.R * c;
    const real G4 = n.P * w2 + n.Q * c + dsqrt(lin * lin + n.K4 * s2);   // 4 G
    // |FD|/v = |cr| / sqrt(G) = 2 |cr| / sqrt(4G)
    return real(2) * __builtin_fabs(cr) * drsqrt(G4);
}

// interpolation weight a = (tau_B - tau_A) / (tau_C - tau_A): differences in the time
// type, the ratio in the math type
template <typename mreal, typename treal>
__device__ __forceinline__ mreal interp_weight(treal ta, treal tb, treal tc) {
    return dratio((mreal)(tb - ta), (mreal)(tc - ta));
}

template <typename mreal, typename real, int S>
__device__ __forceinline__ void eval_stencil(const NodeConst<mreal, real>& n, real ta, real tb, real tc,
                                             Best<real>& best, real& minU) {
    using St = Stencil<S>;
    ++best.evals;
    const mreal a = interp_weight<mreal, real>(ta, tb, tc);
    const real U = tb + (real)stencil_incr<mreal, real>(n, a, St::bx, St::bz, St::cx, St::cz, St::k1, St::k2);
    if (!(U > tc)) return;                        // causality
    real score;
    if (St::cls == 0) {
        score = tc - tb;
    } else {
        // triangles: distance of the diagonal point's time from the isosceles interpolant
        const real r2m1 = real(0.41421356237309504880);   // sqrt(2) - 1
        const real tm = real(0.58578643762690495120);     // 2 - sqrt(2)
        if (St::second) score = __builtin_fabs(tb - (r2m1 * ta + tm * tc));
        else            score = __builtin_fabs(tc - (r2m1 * ta + tm * tb));
    }
    minU = U < minU ? U : minU;
    // table order is the evaluation order, so an equal score never displaces the best
    const bool better = St::cls < best.cls || (St::cls == best.cls && score < best.score);
    if (better) {
        best.cls = St::cls;
        best.score = score;
        best.U = U;
        best.kt = tc;
        best.ks = (tb == tc) ? St::tie_slot : St::sc;
        best.idx = S;
    }
}

template <typename mreal, typename real, int PAIR>
__device__ __forceinline__ void eval_pair(const NodeConst<mreal, real>& n, const real (&t)[12],
                                          Best<real>& best, real& minU) {
    const real inf = dinf<real>();
    const real tA = t[PAIR_A[PAIR]], tP = t[PAIR_P[PAIR]], tQ = t[PAIR_Q[PAIR]];
    // ordering tau_A < tau_B <= tau_C with both B, C known (finite)
    if (tA < tP && tP <= tQ && tQ < inf) eval_stencil<mreal, real, 2 * PAIR>(n, tA, tP, tQ, best, minU);
    if (tA < tQ && tQ <= tP && tP < inf) eval_stencil<mreal, real, 2 * PAIR + 1>(n, tA, tQ, tP, best, minU);
}

template <typename mreal, typename real, int... P>
__device__ __forceinline__ void eval_all(const NodeConst<mreal, real>& n, const real (&t)[12],
                                         Best<real>& best, real& minU,
                                         std::integer_sequence<int, P...>) {
    (eval_pair<mreal, real, P>(n, t, best, minU), ...);
}

template <typename mreal, typename real, int K>
__device__ __forceinline__ void eval_fallback(const NodeConst<mreal, real>& n, const real (&t)[12],
                                              Best<real>& best, real& minU) {
    const real tn = t[FB_SLOT[K]];
    if (!(tn < dinf<real>())) return;
    const real U = tn + n.fb[FB_DIR[K]];
    if (!(U > tn)) return;
    minU = U < minU ? U : minU;
    // class 2 ranks by value, then neighbour order (evaluated in that order)
    if (best.cls > 2 || (best.cls == 2 && U < best.score)) {
        best.cls = 2;
        best.score = U;
        best.U = U;
        best.kt = tn;
        best.ks = FB_SLOT[K];
        best.idx = 32 + K;
    }
}

template <typename mreal, typename real, int... K>
__device__ __forceinline__ void eval_fallbacks(const NodeConst<mreal, real>& n, const real (&t)[12],
                                               Best<real>& best, real& minU,
                                               std::integer_sequence<int, K...>) {
    (eval_fallback<mreal, real, K>(n, t, best, minU), ...);
}

// key_D(u) > key(slot with time tk): D's linear index lies between slots 5 and 6
__device__ __forceinline__ bool key_after(float u, float tk, int ks) { return u > tk || (u == tk && ks <= 5); }
__device__ __forceinline__ bool key_after(double u, double tk, int ks) { return u > tk || (u == tk && ks <= 5); }

// ---------------------------------------------------------------------------------------
// Exact slow path: walk the activation points in key order.  For each of the eight
// possible activation points keep the best candidate activated there; the answer is the
// first record (a candidate better than all activated before it) whose value lies below
// the key of the next record.  Used only when the fast test below is inconclusive.
// ---------------------------------------------------------------------------------------
template <typename real> struct SlotBest {
    int cls[8];
    int idx[8];             // table index of a stencil, neighbour order of a straight ray
    real score[8];
    real U[8];
};

template <typename mreal, typename real, int S>
__device__ __forceinline__ void slow_stencil(const NodeConst<mreal, real>& n, real ta, real tb, real tc,
                                             SlotBest<real>& sb) {
    using St = Stencil<S>;
    const mreal a = interp_weight<mreal, real>(ta, tb, tc);
    const real U = tb + (real)stencil_incr<mreal, real>(n, a, St::bx, St::bz, St::cx, St::cz, St::k1, St::k2);
    if (!(U > tc)) return;
    real score;
    if (St::cls == 0) {
        score = tc - tb;
    } else {
        const real r2m1 = real(0.41421356237309504880);
        const real tm = real(0.58578643762690495120);
        if (St::second) score = __builtin_fabs(tb - (r2m1 * ta + tm * tc));
        else            score = __builtin_fabs(tc - (r2m1 * ta + tm * tb));
    }
    constexpr int kc = fb_local(St::sc);
    constexpr int kt = fb_local(St::tie_slot);
    static_assert(kc >= 0 && kt >= 0, "activation point outside the 8-neighbourhood");
    // two static slots; the tie case files the candidate under the later point
    if (tb == tc) {
        if (St::cls < sb.cls[kt] || (St::cls == sb.cls[kt] && score < sb.score[kt])) {
            sb.cls[kt] = St::cls; sb.idx[kt] = S; sb.score[kt] = score; sb.U[kt] = U;
        }
    } else {
        if (St::cls < sb.cls[kc] || (St::cls == sb.cls[kc] && score < sb.score[kc])) {
            sb.cls[kc] = St::cls; sb.idx[kc] = S; sb.score[kc] = score; sb.U[kc] = U;
        }
    }
}

template <typename mreal, typename real, int PAIR>
__device__ __forceinline__ void slow_pair(const NodeConst<mreal, real>& n, const real (&t)[12], SlotBest<real>& sb) {
    const real inf = dinf<real>();
    const real tA = t[PAIR_A[PAIR]], tP = t[PAIR_P[PAIR]], tQ = t[PAIR_Q[PAIR]];
    if (tA < tP && tP <= tQ && tQ < inf) slow_stencil<mreal, real, 2 * PAIR>(n, tA, tP, tQ, sb);
    if (tA < tQ && tQ <= tP && tP < inf) slow_stencil<mreal, real, 2 * PAIR + 1>(n, tA, tQ, tP, sb);
}

template <typename mreal, typename real, int... P>
__device__ __forceinline__ void slow_all(const NodeConst<mreal, real>& n, const real (&t)[12], SlotBest<real>& sb,
                                         std::integer_sequence<int, P...>) {
    (slow_pair<mreal, real, P>(n, t, sb), ...);
}

// The slow path re-reads the diamond from the caller's staging buffer (LDS) and takes
// the node constants by value, so the fast path never spills them to the stack.
template <typename mreal, typename real>
__device__ __noinline__ real slow_update(const NodeConst<mreal, real> n, const real* __restrict__ lds,
                                         int me, int stride, int* choice) {
    const real inf = dinf<real>();
    real t[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = lds[me + SLOT_DJ[k] * stride + SLOT_DI[k]];
    SlotBest<real> sb;
#pragma unroll
    for (int k = 0; k < 8; ++k) { sb.cls[k] = 3; sb.idx[k] = 99; sb.score[k] = inf; sb.U[k] = inf; }
    slow_all<mreal, real>(n, t, sb, std::make_integer_sequence<int, 16>{});
    // straight-ray candidates fill activation points without a stencil candidate
    unsigned rem = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const real tn = t[FB_SLOT[k]];
        if (sb.cls[k] == 3 && tn < inf) {
            const real U = tn + n.fb[FB_DIR[k]];
            if (U > tn) { sb.cls[k] = 2; sb.idx[k] = 32 + k; sb.score[k] = U; sb.U[k] = U; }
        }
        if (sb.cls[k] < 3) rem |= 1u << k;
    }
    // records in key order
    int rcls = 3, ridx = 99;
    real rscore = inf, rU = inf;
    for (int it = 0; it < 8 && rem; ++it) {
        int q = -1, ccls = 3, cidx = 99;
        real tq = inf, cscore = inf, cU = inf;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const real tk = t[FB_SLOT[k]];
            // strict < scanning in index order keeps the smaller index on equal times
            if (((rem >> k) & 1u) && (q < 0 || tk < tq)) {
                q = k; tq = tk; ccls = sb.cls[k]; cscore = sb.score[k]; cU = sb.U[k]; cidx = sb.idx[k];
            }
        }
        rem &= ~(1u << q);
        // rank = (class, score, table index / neighbour order)
        const bool better = ccls < rcls || (ccls == rcls && (cscore < rscore || (cscore == rscore && cidx < ridx)));
        if (better) {
            if (rcls < 3 && !key_after(rU, tq, FB_SLOT[q])) { *choice = ridx; return rU; }  // record below next key
            rcls = ccls; rscore = cscore; rU = cU; ridx = cidx;
        }
    }
    *choice = rcls < 3 ? ridx : -1;
    return rcls < 3 ? rU : inf;
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
template <typename mreal, typename real>
__device__ __forceinline__ real local_update(const NodeConst<mreal, real>& n, const real (&t)[12],
                                             const real* __restrict__ lds, int me, int stride,
                                             unsigned& evals, int* choice = nullptr) {
    const real inf = dinf<real>();
    Best<real> best;
    best.cls = 3; best.score = inf; best.U = inf; best.kt = inf; best.ks = 0; best.idx = -1; best.evals = 0;
    real minU = inf;
    eval_all<mreal, real>(n, t, best, minU, std::make_integer_sequence<int, 16>{});
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
