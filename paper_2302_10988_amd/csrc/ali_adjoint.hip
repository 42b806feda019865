// ali_adjoint.hip -- gradient of receiver travel times with respect to the orientation of
// the symmetry axis at every node and, on request, to its stiffness A = C / rho (gfx950).
//
// At the fixed point every non-fixed node D holds the value of one candidate of its
// local update (paper Sections 4.2-4.3): a stencil estimate U(tau_A, tau_B, tau_C,
// theta_D) or a straight-ray time from one 8-neighbour; source-box nodes hold straight-ray
// times that depend on the source node's orientation only (Section 4.4).  Holding those
// choices fixed, the field is a composition of smooth maps along a DAG (every candidate
// lies strictly above its support times), so for a loss L with g = dL/dT
//     lambda(X) = g(X) + sum over D whose candidate uses X of lambda(D) dU_D/dtau_X
//     dL/dtheta(D) = lambda(D) dU_D/dtheta_D   (+ source-box terms at the source node)
// Steps on the GPU:
//   1. forward solve (float64 travel times), kept on the device;
//   2. k_adj_prep: re-derive each node's choice with the forward's own local update on
//      the final field, and its partial derivatives in float64 (hand-differentiated
//      estimate formula); one record per node and field, and the node's band time (its
//      travel time rounded up to float32, the only form in which the relaxation reads it);
//   3. k_adj_relax: tiled relaxation of the lambda equation.  Each evaluation recomputes
//      lambda(X) from scratch as a sum in a fixed order, so the end state (no value
//      changes) is the exact solution and independent of the schedule; on a DAG the
//      relaxation ends after at most its depth in sweeps;
//   4. k_adj_grad / k_adj_box: per-node gradient summed over fields in field order
//      (deterministic), plus the source-box terms; k_adj_grad_a / k_adj_box_a do the same
//      for dL/dA = lambda(D) dU_D/dA_D, whose partials k_adj_prep writes when asked.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <math.h>
#include <stdint.h>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "ali_solve.hpp"

namespace ali {

// record of one node in one field: kind and up to three support slots (diamond slot
// numbers 0..11, 0xF = none) in a 16-bit code, plus the partial derivatives
enum : int { K_NONE = 0, K_STENCIL = 1, K_FALLBACK = 2, K_BOX = 3 };
constexpr unsigned NO_SLOT = 0xFu;
__host__ __device__ constexpr uint16_t make_code(int kind, unsigned a, unsigned b, unsigned c) {
    return (uint16_t)(((unsigned)kind << 12) | (c << 8) | (b << 4) | a);
}
constexpr uint16_t CODE_NONE = make_code(K_NONE, NO_SLOT, NO_SLOT, NO_SLOT);
// the kind takes bits 12..13; bit 14 marks a node whose right-hand side g may be nonzero
// (a receiver), so that the relaxation reads g only there
constexpr unsigned CODE_KIND_MASK = 0x3u;
constexpr unsigned CODE_RHS = 1u << 14;
__host__ __device__ constexpr int code_kind(unsigned code) { return (int)((code >> 12) & CODE_KIND_MASK); }

struct StGeo { int sa, sb, sc, bx, bz, cx, cz, k1, k2; };

// What the relaxation of lambda reads of a node D: dU_D/dtau at its A, B and C supports
// and its code, in one aligned record.  The weights are stored in the math type: float32
// under mixed arithmetic (whose travel times, and so the weights derived from them, carry
// float32-level error already), float64 otherwise.
template <typename wreal> struct alignas(4 * sizeof(wreal)) AdjW {
    wreal a, b, c;
    uint32_t code;
};
static_assert(sizeof(AdjW<float>) == 16 && sizeof(AdjW<double>) == 32, "pull records are whole vectors");

template <int S> __device__ __forceinline__ StGeo geo_of() {
    using St = Stencil<S>;
    return StGeo{St::sa, St::sb, St::sc, St::bx, St::bz, St::cx, St::cz, St::k1, St::k2};
}
template <int... S>
__device__ __forceinline__ StGeo stencil_geo(int s, std::integer_sequence<int, S...>) {
    StGeo g{0, 0, 0, 0, 0, 0, 0, 0, 0};
    ((s == S ? (void)(g = geo_of<S>()) : (void)0), ...);
    return g;
}

// Float64 node constants for the derivatives (the phase-speed constants / h^2, with
// K4 = 4 W^2, and the double angle of the axis).
struct NodeD { double c2t, s2t, P, Q, R, W, K4; };

// Partial derivatives of U = tau_B + 2|cr| / sqrt(G4) (the estimate of ali_device.hpp:
// a = (tau_B - tau_A) / (tau_C - tau_A), w = (B - A) - a (C - A), cr = k1 - a k2) with
// respect to tau_A, tau_B, tau_C and the axis angle theta (cos 2theta' = -2 sin 2theta,
// sin 2theta' = 2 cos 2theta).
__device__ void stencil_partials(const NodeD& n, const StGeo& g, double ta, double tb, double tc,
                                 double& dA, double& dB, double& dC, double& dT) {
    const double Dl = tc - ta;
    const double a = (tb - ta) / Dl;
    const double wx = g.bx - a * g.cx, wz = g.bz - a * g.cz;
    const double cr = g.k1 - a * g.k2;
    const double w2 = wx * wx + wz * wz;
    const double dd = wz * wz - wx * wx;
    const double xz = -2.0 * wx * wz;
    const double c = dd * n.c2t + xz * n.s2t;
    const double s2 = w2 * w2 - c * c;
    const double lin = n.Q * w2 + n.R * c;
    const double rt = sqrt(lin * lin + n.K4 * s2);
    const double G4 = n.P * w2 + n.Q * c + rt;
    const double inc = 2.0 * fabs(cr) / sqrt(G4);
    // d/da
    const double dwx = -(double)g.cx, dwz = -(double)g.cz, dcr = -(double)g.k2;
    const double dw2 = 2.0 * (wx * dwx + wz * dwz);
    const double ddd = 2.0 * (wz * dwz - wx * dwx);
    const double dxz = -2.0 * (dwx * wz + wx * dwz);
    const double dc = ddd * n.c2t + dxz * n.s2t;
    const double ds2 = 2.0 * w2 * dw2 - 2.0 * c * dc;
    const double dlin = n.Q * dw2 + n.R * dc;
    const double drt = rt > 0.0 ? (lin * dlin + 0.5 * n.K4 * ds2) / rt : 0.0;
    const double dG4 = n.P * dw2 + n.Q * dc + drt;
    const double dinc = inc * (dcr / cr - 0.5 * dG4 / G4);
    dA = dinc * (a - 1.0) / Dl;
    dB = 1.0 + dinc / Dl;
    dC = -dinc * a / Dl;
    // d/dtheta at fixed a
    const double dct = -2.0 * dd * n.s2t + 2.0 * xz * n.c2t;
    const double drt_t = rt > 0.0 ? (lin * n.R * dct - n.K4 * c * dct) / rt : 0.0;
    const double dG4_t = n.Q * dct + drt_t;
    dT = -0.5 * inc * dG4_t / G4;
}

// Partial derivatives of the same estimate with respect to the node's stiffness A = C / rho
// (a11, a13, a33, a55).  The increment 2|cr| / sqrt(G4) depends on A through G4 only, with
// G4 = P w2 + Q c + sqrt(lin^2 + K4 s2), lin = Q w2 + R c, and P = (a11 + a33 + 2 a55)/h^2,
// Q = (a33 - a11)/h^2, R = (a11 + a33 - 2 a55)/h^2, K4 = 4 W^2 with W = (a13 + a55)/h^2.
__device__ void stencil_partials_A(const NodeD& n, const StGeo& g, double ta, double tb, double tc, double ih2,
                                   double d[4]) {
    const double Dl = tc - ta;
    const double a = (tb - ta) / Dl;
    const double wx = g.bx - a * g.cx, wz = g.bz - a * g.cz;
    const double cr = g.k1 - a * g.k2;
    const double w2 = wx * wx + wz * wz;
    const double c = (wz * wz - wx * wx) * n.c2t + (-2.0 * wx * wz) * n.s2t;
    const double s2 = w2 * w2 - c * c;
    const double lin = n.Q * w2 + n.R * c;
    const double rt = sqrt(lin * lin + n.K4 * s2);
    const double G4 = n.P * w2 + n.Q * c + rt;
    const double inc = 2.0 * fabs(cr) / sqrt(G4);
    const double irt = rt > 0.0 ? 1.0 / rt : 0.0;
    // dG4 / d(P, Q, R, K4)
    const double gP = w2, gQ = c + lin * w2 * irt, gR = lin * c * irt, gK = 0.5 * s2 * irt;
    const double gW = 8.0 * n.W * gK;      // dG4/dK4 dK4/dW
    const double k = -0.5 * inc / G4 * ih2;
    d[0] = k * (gP - gQ + gR);
    d[1] = k * gW;
    d[2] = k * (gP + gQ + gR);
    d[3] = k * (2.0 * (gP - gR) + gW);
}

// The same partials with the velocity table (Sections 3.2 and 4.2): v is the node
// material's table of phase speed / h at whole degrees of psi, the angle between the
// wavefront normal and the symmetry axis folded into [0, 90] degrees, linear in between;
// its derivative is the slope of the interval psi lies in.  cos 2psi' = c / |w|^2 and
// sin 2psi' = s / |w|^2 for psi' = phi_n - theta (phi_n the normal's direction), and
// 2 psi = |2 psi'| folded, so d(2 psi) = sign(s) d(2 psi').
template <typename mreal>
__device__ void stencil_partials_tab(const NodeD& n, const StGeo& g, const mreal* __restrict__ vt, double ta,
                                     double tb, double tc, double& dA, double& dB, double& dC, double& dT) {
    constexpr double DEG = 57.295779513082320877;   // degrees per radian
    const double Dl = tc - ta;
    const double a = (tb - ta) / Dl;
    const double wx = g.bx - a * g.cx, wz = g.bz - a * g.cz;
    const double cr = g.k1 - a * g.k2;
    const double w2 = wx * wx + wz * wz;
    const double dd = wz * wz - wx * wx;
    const double xz = -2.0 * wx * wz;
    const double c = dd * n.c2t + xz * n.s2t;
    const double sn = xz * n.c2t - dd * n.s2t;
    double cc = c / w2;
    cc = cc > 1.0 ? 1.0 : (cc < -1.0 ? -1.0 : cc);
    const double deg = 0.5 * DEG * acos(cc);
    int i = (int)deg;
    i = i > 89 ? 89 : i;
    const double v0 = (double)vt[i], v1 = (double)vt[i + 1];
    const double v = v0 + (deg - i) * (v1 - v0);
    const double slope = v1 - v0;                        // dv / dpsi, per degree
    const double inc = fabs(cr) / (sqrt(w2) * v);
    const double sg = sn >= 0.0 ? 1.0 : -1.0;
    // d/da: the normal turns with a, d(2 phi_n) = (dd dxz - xz ddd) / |w|^4
    const double dwx = -(double)g.cx, dwz = -(double)g.cz, dcr = -(double)g.k2;
    const double dw2 = 2.0 * (wx * dwx + wz * dwz);
    const double ddd = 2.0 * (wz * dwz - wx * dwx);
    const double dxz = -2.0 * (dwx * wz + wx * dwz);
    const double dpsi_da = 0.5 * DEG * sg * (dd * dxz - xz * ddd) / (w2 * w2);
    const double dinc = inc * (dcr / cr - 0.5 * dw2 / w2 - slope * dpsi_da / v);
    dA = dinc * (a - 1.0) / Dl;
    dB = 1.0 + dinc / Dl;
    dC = -dinc * a / Dl;
    // d/dtheta at fixed a: d(2 psi') = -2 dtheta
    dT = inc * slope * sg * DEG / v;
}

// group speed from the table gt (whole degrees of the group angle folded into [0, 90],
// linear in between; as group_speed_tab) and its derivative in phi
__device__ inline double group_speed_tab_d(const double* __restrict__ gt, double phi, double* dV) {
    const double pi = 3.14159265358979323846;
    double a = fmod(fabs(phi), pi);
    double da = phi >= 0.0 ? 1.0 : -1.0;
    if (a > 0.5 * pi) { a = pi - a; da = -da; }
    const double deg = a * (180.0 / pi);
    int i = (int)deg;
    i = i > 89 ? 89 : i;
    const double w = deg - i;
    *dV = (gt[i + 1] - gt[i]) * (180.0 / pi) * da;
    return w == 0.0 ? gt[i] : (1.0 - w) * gt[i] + w * gt[i + 1];
}

// ---------------------------------------------------------------------------------------
// step 2: choices and partial derivatives, one work-group per (tile, field)
// ---------------------------------------------------------------------------------------
// WA: also write dU/dA of every node (4 float64 per node and field, wA[4 q + k]); for a
// source-box node that is the derivative with respect to the source node's stiffness.
// TAB: the velocity table (vtab: the forward's phase-speed tables, the node's offset in geo
// slot 6; gtab: the group-speed tables, VT_N per device material).
// Four waves per SIMD (128 registers): left to itself the compiler takes 149 and runs
// three, and the kernel waits on its dependent float64 chains, not on memory.
template <typename mreal, typename oreal, bool WA, bool TAB>
__global__ void __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(4)))
k_adj_prep(const FieldDev* __restrict__ fields, int n_fields, const MatDev<mreal>* __restrict__ mats_all,
           const uint8_t* __restrict__ mat_id_all, const oreal* __restrict__ orient_all,
           const float* __restrict__ nodeA_all,
           const mreal* __restrict__ geo_all, const double* __restrict__ fbt_all, int R,
           const double* __restrict__ T, AdjW<mreal>* __restrict__ W, double* __restrict__ wT,
           float* __restrict__ Tb, double* __restrict__ wA, const mreal* __restrict__ vtab,
           const double* __restrict__ gtab, unsigned long long* __restrict__ mismatches) {
    __shared__ double lt[LH * LSTRIDE];
    const uint32_t unit = blockIdx.x;
    const FieldDev fd = fields[field_of_unit(fields, n_fields, unit)];
    const int nx = fd.nx, nz = fd.nz;
    const double h = fd.h;
    const int tile = (int)(unit - fd.unit_off);
    const int i0 = (tile % fd.ntx) * TX, j0 = (tile / fd.ntx) * TZ;
    const double* __restrict__ Tf = T + fd.t_off;
    const MatDev<mreal>* __restrict__ mats = mats_all + fd.mat_off;
    const uint8_t* __restrict__ mat_id = mat_id_all + fd.node_off;
    const oreal* __restrict__ orient = orient_all + fd.node_off;
    const float* __restrict__ nodeA = nodeA_all ? nodeA_all + 4 * fd.node_off : nullptr;
    const mreal* __restrict__ geo = geo_all + GEO_N * fd.node_off;
    const double* __restrict__ fbt = fbt_all + 4 * fd.node_off;
    const double inf = dinf<double>();
    // stiffness / density of a node: its own (per-node mode) or its material's
    auto stiff = [&](int64_t n) -> MatA {
        if (nodeA) return MatA{(double)nodeA[4 * n], (double)nodeA[4 * n + 1], (double)nodeA[4 * n + 2],
                               (double)nodeA[4 * n + 3]};
        return mats[mat_id[n]].A;
    };
    const int tid = threadIdx.x;
    for (int q = tid; q < LW * LH; q += NTHREADS) {
        const int li = q % LW, lj = q / LW;
        const int gi = i0 - HALO + li, gj = j0 - HALO + lj;
        double v = inf;
        if (gi >= 0 && gj >= 0 && gi < nx && gj < nz) v = Tf[(int64_t)gj * nx + gi];
        lt[lj * LSTRIDE + li] = v;
    }
    __syncthreads();
    const int lx = tid % TX, lz = tid / TX;
    const int gi = i0 + lx, gj = j0 + lz;
    if (gi >= nx || gj >= nz) return;
    const int64_t p = (int64_t)gj * nx + gi;
    const int64_t q = fd.t_off + p;
    const int2 s = fd.src;
    const int me = (lz + HALO) * LSTRIDE + (lx + HALO);
    const double tD = lt[me];
    uint16_t cd = CODE_NONE;
    double a = 0.0, b = 0.0, c = 0.0, t = 0.0;
    double dA[4] = {0.0, 0.0, 0.0, 0.0};
    const int di = gi - s.x, dj = gj - s.y;
    if (abs(di) <= R && abs(dj) <= R) {
        // straight ray from the source at the source node's orientation and material
        cd = make_code(K_BOX, NO_SLOT, NO_SLOT, NO_SLOT);
        if (di != 0 || dj != 0) {
            const int64_t ps = (int64_t)s.y * nx + s.x;
            const double phi = atan2((double)dj, (double)di) - (double)orient[ps];
            const double L = sqrt((double)(di * di + dj * dj)) * h;
            double dV;
            const MatA As = stiff(ps);
            const double V = TAB ? group_speed_tab_d(gtab + (fd.mat_off + mat_id[ps]) * VT_N, phi, &dV)
                                 : group_speed(As, phi, &dV);
            t = L * dV / (V * V);
            if constexpr (WA) {
                group_speed_dA(As, phi, dA);
#pragma unroll
                for (int k = 0; k < 4; ++k) dA[k] *= -L / (V * V);
            }
        }
    } else if (tD < inf) {
        using NC = typename std::conditional<TAB, NodeConstTab<mreal, double>, NodeConst<mreal, double>>::type;
        NC nc;
        load_node_const<double, mreal>(nc, p, geo, fbt);
        if constexpr (TAB) nc.vt = vtab + (int)geo[GEO_N * p + 6];
        double tt[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) tt[k] = lt[me + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k]];
        unsigned ev = 0;
        int ch = -1;
        const double u = local_update<mreal, double>(nc, tt, lt, me, LSTRIDE, ev, &ch);
        if (!(u == tD)) atomicAdd(mismatches, 1ull);
        const MatA A = stiff(p);
        const double th = (double)orient[p];
        if (ch >= 0 && ch < 32) {
            const StGeo g = stencil_geo(ch, std::make_integer_sequence<int, 32>{});
            NodeD nd;
            sincos(2.0 * th, &nd.s2t, &nd.c2t);
            const double ih2 = 1.0 / (h * h);
            nd.P = (A.a11 + A.a33 + 2.0 * A.a55) * ih2;
            nd.Q = (A.a33 - A.a11) * ih2;
            nd.R = (A.a11 + A.a33 - 2.0 * A.a55) * ih2;
            nd.W = (A.a13 + A.a55) * ih2;
            nd.K4 = 4.0 * nd.W * nd.W;
            if constexpr (TAB) stencil_partials_tab(nd, g, nc.vt, tt[g.sa], tt[g.sb], tt[g.sc], a, b, c, t);
            else stencil_partials(nd, g, tt[g.sa], tt[g.sb], tt[g.sc], a, b, c, t);
            if constexpr (WA) stencil_partials_A(nd, g, tt[g.sa], tt[g.sb], tt[g.sc], ih2, dA);
            cd = make_code(K_STENCIL, (unsigned)g.sa, (unsigned)g.sb, (unsigned)g.sc);
        } else if (ch >= 32) {
            const int k = ch - 32;
            const int d = fb_dir_rt(k);
            const double quarter = 0.78539816339744830962;
            const double ang = d == 0 ? 0.0 : d == 1 ? quarter : d == 2 ? 2.0 * quarter : -quarter;
            const double len = (d & 1) ? 1.41421356237309504880 : 1.0;
            double dV;
            const double V = TAB ? group_speed_tab_d(gtab + (fd.mat_off + mat_id[p]) * VT_N, ang - th, &dV)
                                 : group_speed(A, ang - th, &dV);
            a = 1.0;
            t = len * h * dV / (V * V);
            if constexpr (WA) {
                group_speed_dA(A, ang - th, dA);
#pragma unroll
                for (int k = 0; k < 4; ++k) dA[k] *= -len * h / (V * V);
            }
            cd = make_code(K_FALLBACK, (unsigned)fb_slot_rt(k), NO_SLOT, NO_SLOT);
        }
    }
    AdjW<mreal> w;
    w.a = (mreal)a; w.b = (mreal)b; w.c = (mreal)c;
    w.code = cd;
    W[q] = w;
    wT[q] = t;
    Tb[q] = __double2float_ru(tD);
    if constexpr (WA) {
#pragma unroll
        for (int k = 0; k < 4; ++k) wA[4 * q + k] = dA[k];
    }
}

// ---------------------------------------------------------------------------------------
// step 3: relaxation of lambda, one work-group per active (tile, field)
// ---------------------------------------------------------------------------------------
// contribution to lambda at the node in LDS slot `me` from its 12 diamond neighbours
template <typename wreal>
__device__ __forceinline__ double pull_lambda(double gsum, int me, const double* __restrict__ ll,
                                              const uint16_t* __restrict__ lc, const wreal* __restrict__ la,
                                              const wreal* __restrict__ lb, const wreal* __restrict__ lcw) {
    double s = gsum;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const int o = me + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k];
        const unsigned cd = lc[o];
        const unsigned tgt = 11u - (unsigned)k;       // this node seen from the neighbour
        if ((cd & 0xFu) == tgt) s += ll[o] * (double)la[o];
        else if (((cd >> 4) & 0xFu) == tgt) s += ll[o] * (double)lb[o];
        else if (((cd >> 8) & 0xFu) == tgt) s += ll[o] * (double)lcw[o];
    }
    return s;
}

// Tile visit of the lambda relaxation, one wave per tile (NPL nodes per lane), laid out as
// the forward relaxation.  A node is evaluated only once the descending threshold has
// reached its travel time (ready); a marked node below the threshold is left pending and
// the tile remembers its largest pending time.  A changed lambda marks the node's
// supports: inside the tile for the next sweep, in a neighbouring tile through that
// tile's node mask for the next pass.
template <typename wreal>
__global__ void __launch_bounds__(RW) __attribute__((amdgpu_waves_per_eu(4)))
k_adj_relax(const PassItem* __restrict__ list, const AdjW<wreal>* __restrict__ W,
            const double* __restrict__ G, const float* __restrict__ Tb, const double* __restrict__ theta,
            double* __restrict__ lam, uint8_t* __restrict__ pend, double* __restrict__ maxdef,
            uint32_t* __restrict__ flags, uint32_t* __restrict__ gflag, double* __restrict__ gkey,
            uint32_t* __restrict__ marks_in, uint32_t* __restrict__ marks_out,
            const uint32_t* __restrict__ count, const uint32_t* __restrict__ part_base, uint32_t* __restrict__ idle,
            int inner, unsigned long long* __restrict__ counters) {
    __shared__ double ll[LH * LSTRIDE];
    __shared__ wreal la[LH * LSTRIDE], lb[LH * LSTRIDE], lcw[LH * LSTRIDE];
    __shared__ uint16_t lc[LH * LSTRIDE];
    __shared__ uint8_t dnext[NTHREADS];
    __shared__ uint8_t lpend[NTHREADS];
    // own nodes' travel times for the band test, rounded up to float32 (the band only
    // orders the evaluations; every use of the time in the schedule reads this value)
    __shared__ float ltn[NTHREADS];
    __shared__ uint16_t clist[NTHREADS];
    __shared__ uint32_t omask[9][NODE_WORDS];
    __shared__ uint32_t touched[NODE_WORDS];      // nodes whose lambda changed in this visit
    __shared__ ListMap s_map;                     // where the pass's list entries sit

    const ListMap map = read_list_map(count, part_base);
    const uint32_t n_units = map.pre[LIST_PARTS];
    if (n_units == 0u) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *idle = 1u;
        return;
    }
    put_list_map(s_map, map);
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        atomicAdd(&counters[2], 1ull);
        atomicAdd(&counters[3], (unsigned long long)n_units);
    }
    const XcdRange xr = xcd_range(n_units);
    // the slot of the first entry from the map in registers, each later one looked up in
    // the LDS copy while the entry before it is visited
    uint32_t slot = xr.begin < xr.end ? list_slot_reg(map, xr.begin) : 0u;
    for (uint32_t item = xr.begin; item < xr.end; item += xr.stride) {
    const PassItem pi = list[slot];
    if (item + xr.stride < xr.end) slot = __builtin_amdgcn_readfirstlane(list_slot(s_map, item + xr.stride));
    // opaque inside the item loop, so that per-lane staging offsets are not hoisted out of
    // it and held in registers through the sweeps
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    const uint32_t unit = pi.unit;
    const uint32_t bits = pi.bits;
    const int f = pi.f;
    const int nx = pi.nx, nz = pi.nz, tx = pi.tx, tz = pi.tz;
    const int ntx = (nx + TX - 1) / TX;
    const int i0 = tx * TX, j0 = tz * TZ;
    const int64_t fo = pi.t_off;

    // stage the tile and its halo: every load is issued before the first store to LDS
    constexpr int SQ = (LW * LH + RW - 1) / RW;
    double sl[SQ];
    AdjW<wreal> sw[SQ];
#pragma unroll
    for (int k = 0; k < SQ; ++k) {
        const int q = lane + RW * k;
        const int li = q % LW, lj = q / LW;
        const int gi = i0 - HALO + li, gj = j0 - HALO + lj;
        sl[k] = 0.0;
        sw[k].a = wreal(0); sw[k].b = wreal(0); sw[k].c = wreal(0);
        sw[k].code = CODE_NONE;
        if (q < LW * LH && gi >= 0 && gj >= 0 && gi < nx && gj < nz) {
            const int64_t p = fo + (int64_t)gj * nx + gi;
            sl[k] = lam[p];
            sw[k] = W[p];
        }
    }
    uint32_t mk = 0u;
    if (lane < NODE_WORDS) {
        mk = marks_in[(int64_t)unit * NODE_WORDS + lane];
        if (mk) marks_in[(int64_t)unit * NODE_WORDS + lane] = 0u;
    }
    const double th = theta[f];
    // the tile's own nodes: pending state and band time, read with the halo instead of at
    // every evaluation
    uint8_t pdv[NPL];
    float tv[NPL];
#pragma unroll
    for (int q = 0; q < NPL; ++q) {
        const int node = lane + RW * q;
        const int gi = i0 + node % TX, gj = j0 + node / TX;
        const bool in = gi < nx && gj < nz;
        const int64_t p = fo + (int64_t)gj * nx + gi;
        pdv[q] = in ? pend[p] : 0;
        tv[q] = in ? Tb[p] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < SQ; ++k) {
        const int q = lane + RW * k;
        if (q < LW * LH) {
            const int o = (q / LW) * LSTRIDE + q % LW;
            ll[o] = sl[k]; lc[o] = (uint16_t)sw[k].code; la[o] = sw[k].a; lb[o] = sw[k].b; lcw[o] = sw[k].c;
        }
    }
    for (int q = lane; q < 9 * NODE_WORDS; q += RW) omask[q / NODE_WORDS][q % NODE_WORDS] = 0u;
    for (int q = lane; q < NTHREADS; q += RW) dnext[q] = 0;
    if (lane < NODE_WORDS) touched[lane] = 0u;
    unsigned dmask = 0u, vmask = 0u, pmask = 0u;   // pmask: pending on entry
#pragma unroll
    for (int q = 0; q < NPL; ++q) {
        const int node = lane + RW * q;
        const int gi = i0 + node % TX, gj = j0 + node / TX;
        const bool valid = gi < nx && gj < nz;
        const uint8_t pd = pdv[q];
        lpend[node] = pd;
        ltn[node] = tv[q];
        pmask |= pd ? 1u << q : 0u;
        const bool marked = (__shfl(mk, (node >> 5)) >> (node & 31)) & 1u;
        vmask |= valid ? 1u << q : 0u;
        if (valid && ((bits & TF_SELF) || marked || pd)) dmask |= 1u << q;
    }
    __syncthreads();

    unsigned my_updates = 0;
    bool done = false;
    bool any_out = false;
    for (int it = 0;; ++it) {
        unsigned total = 0;
#pragma unroll
        for (int q = 0; q < NPL; ++q) {
            const unsigned long long m = __ballot((dmask >> q) & 1u);
            if ((dmask >> q) & 1u) clist[total + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)(lane + RW * q);
            total += (unsigned)__popcll(m);
        }
        __syncthreads();
        if (total == 0) { done = true; break; }
        if (it == inner) break;     // sweep cap: the marked nodes carry over to the next pass
        dmask = 0u;
        for (unsigned c = 0; c < total; c += RW) {
            if (c + lane < total) {
                const int node = clist[c + lane];
                const int nlx = node % TX, nlz = node / TX;
                const int nme = (nlz + HALO) * LSTRIDE + (nlx + HALO);
                // time band: a node below the threshold waits until the band reaches it,
                // by which time the nodes it pulls from are final or close to it
                const bool ready = ltn[node] >= th;
                lpend[node] = ready ? 0 : 1;
                if (ready) {
                    ++my_updates;
                    // the right-hand side: nonzero only at receivers, which the code flags
                    const double g0 = (lc[nme] & CODE_RHS) ? G[fo + (int64_t)(j0 + nlz) * nx + (i0 + nlx)] : 0.0;
                    const double v = pull_lambda(g0, nme, ll, lc, la, lb, lcw);
                    if (v != ll[nme]) {
                        ll[nme] = v;
                        atomicOr(&touched[node >> 5], 1u << (node & 31));
                        // lambda flows into this node's supports
                        const unsigned cd = lc[nme];
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
                            const unsigned sl = (cd >> (4 * r)) & 0xFu;
                            if (sl >= 12u) continue;
                            const int ax = nlx + SLOT_DI_RT((int)sl), az = nlz + SLOT_DJ_RT((int)sl);
                            if (ax >= 0 && az >= 0 && ax < TX && az < TZ) {
                                dnext[az * TX + ax] = 1;
                            } else {
                                const int ngi = i0 + ax, ngj = j0 + az;
                                if (ngi < 0 || ngj < 0 || ngi >= nx || ngj >= nz) continue;
                                const int ox = ax < 0 ? 0 : (ax < TX ? 1 : 2), oz = az < 0 ? 0 : (az < TZ ? 1 : 2);
                                const int nn = (az - (oz - 1) * TZ) * TX + (ax - (ox - 1) * TX);
                                atomicOr(&omask[oz * 3 + ox][nn >> 5], 1u << (nn & 31));
                                any_out = true;
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < NPL; ++q) {
            const int node = lane + RW * q;
            if (dnext[node]) {
                dnext[node] = 0;
                dmask |= vmask & (1u << q);
            }
        }
        __syncthreads();
    }

    // write back, carry unfinished nodes, record the largest pending time
    if (!done) {
#pragma unroll 1
        for (int q = 0; q < NPL; ++q)
            if ((dmask >> q) & 1u) {
                const int node = lane + RW * q;
                atomicOr(&omask[4][node >> 5], 1u << (node & 31));
                any_out = true;
            }
    }
    double dk = -dinf<double>();
#pragma unroll 1
    for (int q = 0; q < NPL; ++q) {
        const int node = lane + RW * q;
        const int lx = node % TX, lz = node / TX;
        const int gi = i0 + lx, gj = j0 + lz;
        if (gi >= nx || gj >= nz) continue;
        const int64_t p = fo + (int64_t)gj * nx + gi;
        // only this visit writes the tile's nodes: changed values and pending states
        if ((touched[node >> 5] >> (node & 31)) & 1u) lam[p] = ll[(lz + HALO) * LSTRIDE + (lx + HALO)];
        const uint8_t pd = lpend[node];
        if ((pd != 0) != (((pmask >> q) & 1u) != 0u)) pend[p] = pd;
        if (pd) { const double tp = ltn[node]; dk = tp > dk ? tp : dk; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double d2 = __shfl_xor(dk, o);
        dk = d2 > dk ? d2 : dk;
        my_updates += __shfl_xor(my_updates, o);
    }
    const bool out = __ballot(any_out) != 0ull;
    __syncthreads();
    if (out) {
        for (int q = lane; q < 9 * NODE_WORDS; q += RW) {
            const uint32_t w = omask[q / NODE_WORDS][q % NODE_WORDS];
            if (!w) continue;
            const int o = q / NODE_WORDS;
            const int64_t u2 = (int64_t)unit + (int64_t)(o / 3 - 1) * ntx + (o % 3 - 1);
            atomicOr(&marks_out[u2 * NODE_WORDS + q % NODE_WORDS], w);
            flag_tile(flags, gflag, unit - (uint32_t)(tz * ntx + tx), pi.group_off,
                      (tz + o / 3 - 1) * ntx + (tx + o % 3 - 1), TF_MARK);
        }
    }
    if (lane == 0) {
        if (my_updates) atomicAdd(&counters[4 + 2 * (blockIdx.x % STAT_SLOTS)], (unsigned long long)my_updates);
        maxdef[unit] = dk;
        if (gkey && dk > -dinf<double>()) key_max(&gkey[pi.group_off + (uint32_t)((tz * ntx + tx) / GROUP)], dk);
    }
    __syncthreads();
    }
}

// Scheduler of one adjoint pass (descending thresholds), one work-group per field; the
// tile keys are the largest pending times (the relaxation rewrites them).  K as in k_sched.
template <int K>
__global__ void __launch_bounds__(SCHED_T)
k_adj_sched(const FieldDev* __restrict__ fields, int advance, const double* __restrict__ step,
            uint32_t* __restrict__ flags, double* __restrict__ maxdef, uint32_t* __restrict__ gflag,
            double* __restrict__ gkey, double* __restrict__ theta, PassItem* __restrict__ list,
            uint32_t* __restrict__ cnt_cur, uint32_t* __restrict__ cnt_next, const uint32_t* __restrict__ part_base,
            uint32_t* __restrict__ done, int direct_tiles) {
    __shared__ uint32_t s_due[SCHED_T * K];
    schedule_field<true, double, SCHED_T, K>(blockIdx.x, fields, advance, step, flags, maxdef, gflag, gkey, theta, list,
                                          cnt_cur, cnt_next, part_base, done, s_due, direct_tiles);
}

// ---------------------------------------------------------------------------------------
// right-hand side: g = dL/dT at the receivers, one work-item per field (receivers in order)
// ---------------------------------------------------------------------------------------
// mode 0: g given per (field, receiver).  mode 1: misfit L = 1/2 sum (T - obs)^2, so
// g = T - obs; also writes T at the receivers and the per-field misfit.  The field's
// threshold starts at its latest receiver time (nodes later than every receiver carry no
// sensitivity), or -inf without a band.
template <typename greal, typename outreal>
__global__ void k_adj_rhs(int mode, int n_fields, const FieldDev* __restrict__ fields, const int2* __restrict__ rec,
                          const greal* __restrict__ in, const double* __restrict__ T, double* __restrict__ G,
                          outreal* __restrict__ trec, double* __restrict__ lossf, uint32_t* __restrict__ flags,
                          uint32_t* __restrict__ gflag, double* __restrict__ theta, int banded,
                          uint32_t* __restrict__ wcode, int wstride) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_fields) return;
    const FieldDev fd = fields[f];
    double L = 0.0;
    double tmax = -dinf<double>();
    // G is read only where the code carries CODE_RHS, so only the receiver nodes are
    // cleared (receivers on one node add up)
    for (int r = 0; r < fd.n_rec; ++r) {
        const int2 x = rec[fd.rec_off + r];
        G[fd.t_off + (int64_t)x.y * fd.nx + x.x] = 0.0;
    }
    for (int r = 0; r < fd.n_rec; ++r) {
        const int2 x = rec[fd.rec_off + r];
        const int64_t p = fd.t_off + (int64_t)x.y * fd.nx + x.x;
        double g = (double)in[fd.obs_off + r];
        if (mode == 1) {
            const double t = T[p];
            g = t - g;
            L += 0.5 * g * g;
            if (trec) trec[fd.obs_off + r] = (outreal)t;
        }
        G[p] += g;
        wcode[p * wstride] |= CODE_RHS;
        tmax = T[p] > tmax ? T[p] : tmax;
        const int t = (x.y / TZ) * fd.ntx + (x.x / TX);
        flags[fd.unit_off + t] |= TF_SELF;
        if (gflag) gflag[fd.group_off + t / GROUP] = 1u;
    }
    if (lossf) lossf[f] = L;
    theta[f] = banded ? tmax : -dinf<double>();
}

// misfit of each medium: its fields' misfits in field order
__global__ void k_adj_loss(const double* __restrict__ lossf, const int* __restrict__ first, int n_media,
                           double* __restrict__ out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_media) return;
    double s = 0.0;
    for (int f = first[m]; f < first[m + 1]; ++f) s += lossf[f];
    out[m] = s;
}

// ---------------------------------------------------------------------------------------
// step 4: gradient
// ---------------------------------------------------------------------------------------
// nodes of one medium, summed over its fields f0 .. f1 - 1 in field order
template <typename wreal>
__global__ void k_adj_grad(int64_t N, int f0, int f1, const FieldDev* __restrict__ fields,
                           const AdjW<wreal>* __restrict__ W, const double* __restrict__ wT,
                           const double* __restrict__ lam, double* __restrict__ dth) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    double s = 0.0;
    for (int f = f0; f < f1; ++f) {
        const int64_t q = fields[f].t_off + p;
        const int kind = code_kind(W[q].code);
        if (kind == K_STENCIL || kind == K_FALLBACK) s += lam[q] * wT[q];
    }
    dth[p] = s;
}

// dL/dA of the nodes of one medium (4 per node), summed over its fields in field order
template <typename wreal>
__global__ void k_adj_grad_a(int64_t N, int f0, int f1, const FieldDev* __restrict__ fields,
                             const AdjW<wreal>* __restrict__ W, const double* __restrict__ wA,
                             const double* __restrict__ lam, double* __restrict__ dA) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int f = f0; f < f1; ++f) {
        const int64_t q = fields[f].t_off + p;
        const int kind = code_kind(W[q].code);
        if (kind == K_STENCIL || kind == K_FALLBACK) {
            const double l = lam[q];
            s0 += l * wA[4 * q + 0];
            s1 += l * wA[4 * q + 1];
            s2 += l * wA[4 * q + 2];
            s3 += l * wA[4 * q + 3];
        }
    }
    dA[4 * p + 0] = s0;
    dA[4 * p + 1] = s1;
    dA[4 * p + 2] = s2;
    dA[4 * p + 3] = s3;
}

// source-box terms of field f, reduced in a fixed order
__global__ void k_adj_box(const FieldDev* __restrict__ fields, int R, const double* __restrict__ wT,
                          const double* __restrict__ lam, double* __restrict__ boxsum) {
    const int f = blockIdx.x;
    const FieldDev fd = fields[f];
    const int2 s = fd.src;
    const int w = 2 * R + 1;
    double acc = 0.0;
    for (int k = threadIdx.x; k < w * w; k += blockDim.x) {
        const int i = s.x - R + k % w, j = s.y - R + k / w;
        if (i < 0 || j < 0 || i >= fd.nx || j >= fd.nz) continue;
        const int64_t q = fd.t_off + (int64_t)j * fd.nx + i;
        acc += lam[q] * wT[q];
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int m = blockDim.x / 2; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) boxsum[f] = red[0];
}

// source-box terms of field f with respect to the source node's stiffness (4 values)
__global__ void k_adj_box_a(const FieldDev* __restrict__ fields, int R, const double* __restrict__ wA,
                            const double* __restrict__ lam, double* __restrict__ boxsum) {
    const int f = blockIdx.x;
    const FieldDev fd = fields[f];
    const int2 s = fd.src;
    const int w = 2 * R + 1;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < w * w; k += blockDim.x) {
        const int i = s.x - R + k % w, j = s.y - R + k / w;
        if (i < 0 || j < 0 || i >= fd.nx || j >= fd.nz) continue;
        const int64_t q = fd.t_off + (int64_t)j * fd.nx + i;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += lam[q] * wA[4 * q + c];
    }
    __shared__ double red[4][256];
#pragma unroll
    for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int m = blockDim.x / 2; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m)
#pragma unroll
            for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x < 4) boxsum[4 * f + threadIdx.x] = red[threadIdx.x][0];
}

// The box terms are added at the source nodes in field order: one work-item per medium
// when the media's node ranges are disjoint (each node then sees its terms in field order),
// else one work-item for all (media may share nodes).
__device__ __forceinline__ bool box_add_range(int n_media, const int* __restrict__ first, bool disjoint, int& f0,
                                              int& f1) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (disjoint) {
        if (m >= n_media) return false;
        f0 = first[m];
        f1 = first[m + 1];
        return true;
    }
    f0 = 0;
    f1 = first[n_media];
    return m == 0;
}

__global__ void k_adj_box_add_a(int n_media, const int* __restrict__ first, int disjoint,
                                const FieldDev* __restrict__ fields, const double* __restrict__ boxsum,
                                double* __restrict__ dA) {
    int f0, f1;
    if (!box_add_range(n_media, first, disjoint != 0, f0, f1)) return;
    for (int f = f0; f < f1; ++f) {
        const FieldDev& fd = fields[f];
        const int64_t p = fd.node_off + (int64_t)fd.src.y * fd.nx + fd.src.x;
        for (int c = 0; c < 4; ++c) dA[4 * p + c] += boxsum[4 * f + c];
    }
}

__global__ void k_adj_box_add(int n_media, const int* __restrict__ first, int disjoint,
                              const FieldDev* __restrict__ fields, const double* __restrict__ boxsum,
                              double* __restrict__ dth) {
    int f0, f1;
    if (!box_add_range(n_media, first, disjoint != 0, f0, f1)) return;
    for (int f = f0; f < f1; ++f) {
        const FieldDev& fd = fields[f];
        dth[fd.node_off + (int64_t)fd.src.y * fd.nx + fd.src.x] += boxsum[f];
    }
}

// ---------------------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------------------
template <typename mreal, typename oreal, typename greal, typename outreal>
static ali_status adjoint_impl(ali_handle* H, const ali_medium* media, int32_t n_media, const ali_material* mats,
                               int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient,
                               const ali_node* srcs, const ali_node* recv, int mode, const greal* d_in,
                               const ali_options* opt_in, outreal* d_T, outreal* d_trec, double* d_loss,
                               outreal* d_dth, outreal* d_dA, ali_adjoint_stats* stats) {
    ali_options opt;
    ali_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (!recv) return H->fail(ALI_EINVAL, "receivers are NULL");
    ali_status st = validate_batch(H, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, recv, opt.wave);
    if (st != ALI_OK) return st;
    if (d_dA && opt.wave != ALI_WAVE_QP)
        return H->fail(ALI_EUNSUPPORTED, "the stiffness gradient is available for the qP wave only");
    if (opt.velocity != ALI_VEL_CHRISTOFFEL && d_dA)
        return H->fail(ALI_EUNSUPPORTED, "the stiffness gradient differentiates the run-time speeds (velocity table given)");
    if (opt.adjoint_band_cells < 0 || opt.adjoint_inner_sweeps < 0 || opt.adjoint_inner_sweeps > 4096)
        return H->fail(ALI_EINVAL, "adjoint_band_cells must be >= 0 and adjoint_inner_sweeps in [0, 4096]");
    if (!d_in) return H->fail(ALI_EINVAL, mode == 1 ? "d_obs is NULL" : "d_dLdT is NULL");
    if (!d_dth) return H->fail(ALI_EINVAL, "d_dLdtheta is NULL");
    int64_t n_fields64 = 0, NF = 0;
    batch_sizes(media, n_media, &n_fields64, &NF);
    const int n_fields = (int)n_fields64;
    int64_t med_nodes = 0;
    int n_recv_total = 0;
    for (int m = 0; m < n_media; ++m) {
        med_nodes = std::max(med_nodes, media[m].node_offset + (int64_t)media[m].grid.nx * media[m].grid.nz);
        n_recv_total = std::max(n_recv_total, media[m].rec_offset + media[m].n_rec);
    }
    // do the media's node ranges overlap? (the box terms are then added by one work-item)
    bool disjoint = true;
    {
        std::vector<std::pair<int64_t, int64_t>> rng(n_media);
        for (int m = 0; m < n_media; ++m)
            rng[m] = std::make_pair(media[m].node_offset, media[m].node_offset + (int64_t)media[m].grid.nx * media[m].grid.nz);
        std::sort(rng.begin(), rng.end());
        for (int m = 1; m < n_media; ++m) disjoint &= rng[m].first >= rng[m - 1].second;
    }

    // forward fields in float64: the caller's buffer when it is float64, else scratch
    constexpr bool out64 = std::is_same<outreal, double>::value;
    void* d_work = nullptr;
    if (!(out64 && d_T) && !H->scratch("adjT", sizeof(double) * NF, &d_work))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    double* T = (out64 && d_T) ? (double*)d_T : (double*)d_work;

    ali_solve_stats fst{};
    ForwardState<double, mreal> fs;
    st = solve_fields<double, mreal, oreal>(H, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, recv, opt, T,
                                            &fst, &fs);
    if (st != ALI_OK) return st;
    hipStream_t S = H->stream;
    HIPCK(H, hipEventRecord(H->ev4, S));
    const int64_t nunits = fs.n_units;

    void *d_W, *d_wT, *d_Tb, *d_lam, *d_G, *d_dacc, *d_box, *d_lossf, *d_rec, *d_first;
    void *d_flags, *d_list, *d_count, *d_cnt, *d_pend, *d_maxdef, *d_theta, *d_step, *d_idle, *d_marks;
    void *d_gflag, *d_gkey;
    const int64_t ngroups = fs.n_groups;
    const int sched_k = sched_k_for(nunits);
    const int direct_tiles = direct_tiles_for(nunits, SCHED_T * sched_k);
    bool use_groups = false;
    for (const FieldDev& fd : fs.hfields) use_groups |= fd.ntx * fd.ntz > direct_tiles;
    if (!H->scratch("a_w", sizeof(AdjW<mreal>) * NF, &d_W) || !H->scratch("a_wT", sizeof(double) * NF, &d_wT) ||
        !H->scratch("a_tb", sizeof(float) * NF, &d_Tb) ||
        !H->scratch("a_lam", sizeof(double) * NF, &d_lam) || !H->scratch("a_G", sizeof(double) * NF, &d_G) ||
        !H->scratch("a_pend", sizeof(uint8_t) * NF, &d_pend) ||
        !H->scratch("a_dth", sizeof(double) * med_nodes, &d_dacc) ||
        !H->scratch("a_box", sizeof(double) * n_fields, &d_box) ||
        !H->scratch("a_lossf", sizeof(double) * n_fields, &d_lossf) ||
        !H->scratch("a_theta", sizeof(double) * n_fields, &d_theta) ||
        !H->scratch("a_step", sizeof(double) * n_fields, &d_step) ||
        !H->scratch("a_first", sizeof(int) * (n_media + 1), &d_first) ||
        !H->scratch("a_rec", sizeof(int2) * n_recv_total, &d_rec) ||
        !H->scratch("a_flags", sizeof(uint32_t) * nunits, &d_flags) ||
        !H->scratch("a_maxdef", sizeof(double) * nunits, &d_maxdef) ||
        !H->scratch("a_gflag", sizeof(uint32_t) * ngroups, &d_gflag) ||
        !H->scratch("a_gkey", sizeof(double) * ngroups, &d_gkey) ||
        !H->scratch("a_list", sizeof(PassItem) * nunits, &d_list) ||
        !H->scratch("a_count", sizeof(uint32_t) * (CNT_WORDS + n_fields), &d_count) ||
        !H->scratch("a_idle", sizeof(uint32_t), &d_idle) ||
        !H->scratch("a_marks", sizeof(uint32_t) * 2 * NODE_WORDS * nunits, &d_marks) ||
        !H->scratch("a_cnt", (4 + 2 * STAT_SLOTS) * sizeof(unsigned long long), &d_cnt))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    // stiffness gradient (on request): dU/dA per node and field, its sums, box terms
    void *d_wA = nullptr, *d_aacc = nullptr, *d_boxa = nullptr;
    if (d_dA && (!H->scratch("a_wA", 4 * sizeof(double) * NF, &d_wA) ||
                 !H->scratch("a_dA", 4 * sizeof(double) * med_nodes, &d_aacc) ||
                 !H->scratch("a_boxA", 4 * sizeof(double) * n_fields, &d_boxa)))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    // descending time band: band_cells node spacings at each medium's fastest phase speed
    // the adjoint's own band and sweep cap (0: those of the forward)
    const int abands = opt.adjoint_band_cells > 0 ? opt.adjoint_band_cells : opt.band_cells;
    const int ainner = opt.adjoint_inner_sweeps > 0 ? opt.adjoint_inner_sweeps : opt.inner_sweeps;
    const bool banded = abands > 0;
    std::vector<double> hstep(n_fields);
    for (int f = 0; f < n_fields; ++f) {
        const int m = fs.hfields[f].medium;
        hstep[f] = banded ? abands * media[m].grid.h / fs.vmax[m] : 0.0;
    }
    std::vector<int2> hr(n_recv_total);
    for (int r = 0; r < n_recv_total; ++r) hr[r] = make_int2(recv[r].i, recv[r].j);
    HIPCK(H, hipMemcpyAsync(d_rec, hr.data(), sizeof(int2) * n_recv_total, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemcpyAsync(d_step, hstep.data(), sizeof(double) * n_fields, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemcpyAsync(d_first, fs.medium_first_field.data(), sizeof(int) * (n_media + 1), hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemsetAsync(d_flags, 0, sizeof(uint32_t) * nunits, S));
    HIPCK(H, hipMemsetAsync(d_gflag, 0, sizeof(uint32_t) * ngroups, S));
    HIPCK(H, hipMemsetAsync(d_marks, 0, sizeof(uint32_t) * 2 * NODE_WORDS * nunits, S));
    HIPCK(H, hipMemsetAsync(d_count, 0, sizeof(uint32_t) * (CNT_WORDS + n_fields), S));
    const std::vector<uint32_t> part_base = list_part_base(fs.hfields);
    HIPCK(H, hipMemcpyAsync((uint32_t*)d_count + 2 * CNT_BLOCK, part_base.data(), sizeof(uint32_t) * LIST_PARTS,
                            hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemsetAsync(d_idle, 0, sizeof(uint32_t), S));
    HIPCK(H, hipMemsetAsync(d_cnt, 0, (4 + 2 * STAT_SLOTS) * sizeof(unsigned long long), S));

    const int B = 256;
    const unsigned gNF = (unsigned)((NF + B - 1) / B);
    if (d_dA)
        hipLaunchKernelGGL((k_adj_prep<mreal, oreal, true, false>), dim3((unsigned)nunits), dim3(NTHREADS), 0, S,
                           fs.fields, n_fields, fs.mats, d_mat_id, d_orient, opt.d_node_A, fs.geo, fs.fbt,
                           opt.src_box_radius, (const double*)T, (AdjW<mreal>*)d_W, (double*)d_wT, (float*)d_Tb,
                           (double*)d_wA, (const mreal*)nullptr, (const double*)nullptr,
                           (unsigned long long*)d_cnt + 1);
    else if (fs.vt)
        hipLaunchKernelGGL((k_adj_prep<mreal, oreal, false, true>), dim3((unsigned)nunits), dim3(NTHREADS), 0, S,
                           fs.fields, n_fields, fs.mats, d_mat_id, d_orient, opt.d_node_A, fs.geo, fs.fbt,
                           opt.src_box_radius, (const double*)T, (AdjW<mreal>*)d_W, (double*)d_wT, (float*)d_Tb,
                           (double*)nullptr, fs.vt, fs.gt, (unsigned long long*)d_cnt + 1);
    else
        hipLaunchKernelGGL((k_adj_prep<mreal, oreal, false, false>), dim3((unsigned)nunits), dim3(NTHREADS), 0, S,
                           fs.fields, n_fields, fs.mats, d_mat_id, d_orient, opt.d_node_A, fs.geo, fs.fbt,
                           opt.src_box_radius, (const double*)T, (AdjW<mreal>*)d_W, (double*)d_wT, (float*)d_Tb,
                           (double*)nullptr, (const mreal*)nullptr, (const double*)nullptr,
                           (unsigned long long*)d_cnt + 1);
    HIPCK(H, hipGetLastError());
    hipLaunchKernelGGL((k_fill<double>), dim3(gNF), dim3(B), 0, S, (double*)d_lam, NF, 0.0);
    hipLaunchKernelGGL((k_fill<uint8_t>), dim3(gNF), dim3(B), 0, S, (uint8_t*)d_pend, NF, (uint8_t)0);
    hipLaunchKernelGGL((k_fill<double>), dim3((unsigned)((nunits + B - 1) / B)), dim3(B), 0, S, (double*)d_maxdef,
                       nunits, -dinf_host<double>());
    hipLaunchKernelGGL((k_fill<double>), dim3((unsigned)((ngroups + B - 1) / B)), dim3(B), 0, S, (double*)d_gkey,
                       ngroups, -dinf_host<double>());
    hipLaunchKernelGGL((k_adj_rhs<greal, outreal>), dim3((unsigned)((n_fields + 63) / 64)), dim3(64), 0, S,
                       mode, n_fields, fs.fields, (const int2*)d_rec, d_in, (const double*)T, (double*)d_G, d_trec,
                       (double*)d_lossf, (uint32_t*)d_flags, use_groups ? (uint32_t*)d_gflag : nullptr, (double*)d_theta,
                       banded ? 1 : 0, &((AdjW<mreal>*)d_W)->code, (int)(sizeof(AdjW<mreal>) / sizeof(uint32_t)));
    HIPCK(H, hipGetLastError());
    if (mode == 1 && d_loss)
        hipLaunchKernelGGL(k_adj_loss, dim3((unsigned)((n_media + 63) / 64)), dim3(64), 0, S, (const double*)d_lossf,
                           (const int*)d_first, n_media, d_loss);

    // passes queued in batches; the idle flag ends the loop (see the forward driver)
    int iters = 0;
    bool converged = false;
    double relax_ms = 0.0;
    // far more work-groups than are resident (see the forward relaxation)
    const int grid_relax = (int)(nunits < (int64_t)128 * H->n_cu ? nunits : (int64_t)128 * H->n_cu);
    uint32_t* cnt = (uint32_t*)d_count;
    auto* const ksched = sched_k == SCHED_K ? &k_adj_sched<SCHED_K> : &k_adj_sched<SCHED_K_LARGE>;
    auto enqueue = [&](int p, bool timed, hipStream_t S) {
        hipLaunchKernelGGL(ksched, dim3((unsigned)n_fields), dim3(SCHED_T), 0, S, fs.fields, p > 0 ? 1 : 0,
                           (const double*)d_step, (uint32_t*)d_flags, (double*)d_maxdef, (uint32_t*)d_gflag,
                           (double*)d_gkey, (double*)d_theta,
                           (PassItem*)d_list, cnt + (p & 1) * CNT_BLOCK, cnt + ((p + 1) & 1) * CNT_BLOCK,
                           (const uint32_t*)(cnt + 2 * CNT_BLOCK), cnt + 2 * CNT_BLOCK + LIST_PARTS, direct_tiles);
        uint32_t* mk_in = (uint32_t*)d_marks + (size_t)(p & 1) * nunits * NODE_WORDS;
        uint32_t* mk_out = (uint32_t*)d_marks + (size_t)((p + 1) & 1) * nunits * NODE_WORDS;
        if (timed) (void)hipEventRecord(H->pev[2 * (p % PASS_BATCH)], S);
        hipLaunchKernelGGL(k_adj_relax<mreal>, dim3((unsigned)grid_relax), dim3(RW), 0, S,
                           (const PassItem*)d_list, (const AdjW<mreal>*)d_W,
                           (const double*)d_G, (const float*)d_Tb, (const double*)d_theta, (double*)d_lam,
                           (uint8_t*)d_pend, (double*)d_maxdef, (uint32_t*)d_flags,
                           use_groups ? (uint32_t*)d_gflag : nullptr, use_groups ? (double*)d_gkey : nullptr, mk_in,
                           mk_out,
                           (const uint32_t*)(cnt + (p & 1) * CNT_BLOCK), (const uint32_t*)(cnt + 2 * CNT_BLOCK),
                           (uint32_t*)d_idle, ainner,
                           (unsigned long long*)d_cnt);
        if (timed) (void)hipEventRecord(H->pev[2 * (p % PASS_BATCH) + 1], S);
    };
    while (iters < opt.max_sweeps) {
        const int batch = opt.max_sweeps - iters < PASS_BATCH ? opt.max_sweeps - iters : PASS_BATCH;
        const bool graph = opt.graph && batch == PASS_BATCH;
        if (graph) {
            const int first = iters == 0 ? 1 : 0;
            const std::string key = graph_key("adj", first, (const void*)&k_adj_relax<mreal>, fs.fields, n_fields, d_step, d_flags, d_maxdef, d_gflag, d_gkey, use_groups ? 1 : 0, direct_tiles, d_theta,
                                              d_list, d_count, d_marks, nunits, d_W, d_G, T, d_lam, d_pend, d_idle, ainner, d_cnt, grid_relax);
            HIPCK(H, hipEventRecord(H->ev2, S));
            st = launch_captured(H, key, [&](int b, hipStream_t cs) { enqueue(first ? b : PASS_BATCH + b, false, cs); });
            if (st != ALI_OK) return st;
            HIPCK(H, hipEventRecord(H->ev3, S));
        } else {
            for (int bb = 0; bb < batch; ++bb) enqueue(iters + bb, true, S);
        }
        HIPCK(H, hipGetLastError());
        HIPCK(H, hipMemcpyAsync(H->host_count, d_idle, sizeof(uint32_t), hipMemcpyDeviceToHost, S));
        HIPCK(H, hipStreamSynchronize(S));
        if (graph) {
            float kms = 0.f;
            HIPCK(H, hipEventElapsedTime(&kms, H->ev2, H->ev3));
            relax_ms += kms;
        } else {
            for (int bb = 0; bb < batch; ++bb) {
                float kms = 0.f;
                HIPCK(H, hipEventElapsedTime(&kms, H->pev[2 * ((iters + bb) % PASS_BATCH)],
                                             H->pev[2 * ((iters + bb) % PASS_BATCH) + 1]));
                relax_ms += kms;
            }
        }
        iters += batch;
        if (*H->host_count) { converged = true; break; }
    }

    for (int m = 0; m < n_media; ++m) {
        const int64_t N = (int64_t)media[m].grid.nx * media[m].grid.nz;
        hipLaunchKernelGGL(k_adj_grad<mreal>, dim3((unsigned)((N + B - 1) / B)), dim3(B), 0, S, N,
                           fs.medium_first_field[m], fs.medium_first_field[m + 1], fs.fields,
                           (const AdjW<mreal>*)d_W, (const double*)d_wT, (const double*)d_lam,
                           (double*)d_dacc + media[m].node_offset);
    }
    hipLaunchKernelGGL(k_adj_box, dim3((unsigned)n_fields), dim3(256), 0, S, fs.fields, opt.src_box_radius,
                       (const double*)d_wT, (const double*)d_lam, (double*)d_box);
    hipLaunchKernelGGL(k_adj_box_add, dim3((unsigned)((n_media + 63) / 64)), dim3(64), 0, S, n_media,
                       (const int*)d_first, disjoint ? 1 : 0, fs.fields, (const double*)d_box, (double*)d_dacc);
    for (int m = 0; m < n_media; ++m) {
        const int64_t N = (int64_t)media[m].grid.nx * media[m].grid.nz;
        hipLaunchKernelGGL((k_convert<outreal, double>), dim3((unsigned)((N + B - 1) / B)), dim3(B), 0, S,
                           d_dth + media[m].node_offset, (const double*)d_dacc + media[m].node_offset, N);
    }
    HIPCK(H, hipGetLastError());
    if (d_dA) {
        for (int m = 0; m < n_media; ++m) {
            const int64_t N = (int64_t)media[m].grid.nx * media[m].grid.nz;
            hipLaunchKernelGGL(k_adj_grad_a<mreal>, dim3((unsigned)((N + B - 1) / B)), dim3(B), 0, S, N,
                               fs.medium_first_field[m], fs.medium_first_field[m + 1], fs.fields,
                               (const AdjW<mreal>*)d_W, (const double*)d_wA, (const double*)d_lam,
                               (double*)d_aacc + 4 * media[m].node_offset);
        }
        hipLaunchKernelGGL(k_adj_box_a, dim3((unsigned)n_fields), dim3(256), 0, S, fs.fields, opt.src_box_radius,
                           (const double*)d_wA, (const double*)d_lam, (double*)d_boxa);
        hipLaunchKernelGGL(k_adj_box_add_a, dim3((unsigned)((n_media + 63) / 64)), dim3(64), 0, S, n_media,
                           (const int*)d_first, disjoint ? 1 : 0, fs.fields, (const double*)d_boxa,
                           (double*)d_aacc);
        for (int m = 0; m < n_media; ++m) {
            const int64_t N4 = 4 * (int64_t)media[m].grid.nx * media[m].grid.nz;
            hipLaunchKernelGGL((k_convert<outreal, double>), dim3((unsigned)((N4 + B - 1) / B)), dim3(B), 0, S,
                               d_dA + 4 * media[m].node_offset, (const double*)d_aacc + 4 * media[m].node_offset,
                               N4);
        }
        HIPCK(H, hipGetLastError());
    }
    if (d_T && !out64)
        hipLaunchKernelGGL((k_convert<outreal, double>), dim3(gNF), dim3(B), 0, S, d_T, (const double*)T, NF);
    HIPCK(H, hipGetLastError());
    HIPCK(H, hipEventRecord(H->ev1, S));
    std::vector<unsigned long long> cnt_h(4 + 2 * STAT_SLOTS);
    HIPCK(H, hipMemcpyAsync(cnt_h.data(), d_cnt, sizeof(unsigned long long) * cnt_h.size(), hipMemcpyDeviceToHost, S));
    HIPCK(H, hipStreamSynchronize(S));
    unsigned long long lam_updates = 0;
    for (int k = 0; k < STAT_SLOTS; ++k) lam_updates += cnt_h[4 + 2 * k];
    if (stats) {
        float ms = 0.f;
        HIPCK(H, hipEventElapsedTime(&ms, H->ev0, H->ev1));
        float fms = 0.f;
        HIPCK(H, hipEventElapsedTime(&fms, H->ev0, H->ev4));
        stats->forward = fst;
        stats->forward.ms = fms;
        stats->lambda_updates = (int64_t)lam_updates;
        stats->choice_mismatches = (int64_t)cnt_h[1];
        stats->tile_visits = (int64_t)cnt_h[3];
        stats->outer_iters = (int32_t)cnt_h[2];
        stats->converged = converged ? 1 : 0;
        stats->ms = ms;
        stats->relax_ms = relax_ms;
    }
    if (!converged) return H->fail(ALI_ENOCONV, "adjoint relaxation reached max_sweeps");
    return ALI_OK;
}

template <typename real>
__global__ void k_bilinear(int n_z, int n_x, int ncz, int ncx, const real* __restrict__ ctrl,
                           real* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)n_z * n_x) return;
    const int j = (int)(p / n_x), i = (int)(p % n_x);
    const double uz = (double)j * (ncz - 1) / (n_z - 1), ux = (double)i * (ncx - 1) / (n_x - 1);
    int cz = (int)floor(uz), cx = (int)floor(ux);
    cz = cz < ncz - 2 ? cz : ncz - 2;
    cx = cx < ncx - 2 ? cx : ncx - 2;
    const double fz = uz - cz, fx = ux - cx;
    const double c00 = (double)ctrl[(int64_t)cz * ncx + cx], c01 = (double)ctrl[(int64_t)cz * ncx + cx + 1];
    const double c10 = (double)ctrl[(int64_t)(cz + 1) * ncx + cx], c11 = (double)ctrl[(int64_t)(cz + 1) * ncx + cx + 1];
    out[p] = (real)((1.0 - fz) * ((1.0 - fx) * c00 + fx * c01) + fz * ((1.0 - fx) * c10 + fx * c11));
}

// weight of control c in the 1-D interpolant at node k (n nodes, nc controls)
__device__ __forceinline__ double lin_weight(int k, int n, int nc, int c) {
    const double u = (double)k * (nc - 1) / (n - 1);
    int c0 = (int)floor(u);
    c0 = c0 < nc - 2 ? c0 : nc - 2;
    const double f = u - c0;
    return c == c0 ? 1.0 - f : (c == c0 + 1 ? f : 0.0);
}

// transpose: one work-item per control value, summing its support rows and columns in order
template <typename real>
__global__ void k_bilinear_t(int n_z, int n_x, int ncz, int ncx, const real* __restrict__ g,
                             real* __restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ncz * ncx) return;
    const int a = q / ncx, b = q % ncx;
    // nodes whose interpolation cell touches control a: u in (a-1, a+1)
    const int jlo = a == 0 ? 0 : (int)floor((double)(a - 1) * (n_z - 1) / (ncz - 1));
    const int jhi = (int)ceil((double)(a + 1) * (n_z - 1) / (ncz - 1));
    const int ilo = b == 0 ? 0 : (int)floor((double)(b - 1) * (n_x - 1) / (ncx - 1));
    const int ihi = (int)ceil((double)(b + 1) * (n_x - 1) / (ncx - 1));
    double s = 0.0;
    for (int j = jlo; j <= jhi && j < n_z; ++j) {
        const double wz = lin_weight(j, n_z, ncz, a);
        if (wz == 0.0) continue;
        double r = 0.0;
        for (int i = ilo; i <= ihi && i < n_x; ++i) {
            const double wx = lin_weight(i, n_x, ncx, b);
            if (wx != 0.0) r += wx * (double)g[(int64_t)j * n_x + i];
        }
        s += wz * r;
    }
    out[q] = (real)s;
}

template <typename real>
static ali_status bilinear_impl(ali_handle* H, int32_t nz, int32_t nx, int32_t ncz, int32_t ncx,
                                const real* d_in, real* d_out, bool transpose) {
    if (nz < 2 || nx < 2 || ncz < 2 || ncx < 2) return H->fail(ALI_EINVAL, "need nz, nx, ncz, ncx >= 2");
    if ((int64_t)nz * nx > (int64_t)1 << 31) return H->fail(ALI_EINVAL, "grid too large");
    if (ncz > nz || ncx > nx) return H->fail(ALI_EINVAL, "more control points than nodes");
    if (!d_in || !d_out) return H->fail(ALI_EINVAL, "NULL array");
    if (set_device(H) != ALI_OK) return ALI_EDEVICE;
    const int B = 256;
    if (transpose) {
        const int nq = ncz * ncx;
        hipLaunchKernelGGL((k_bilinear_t<real>), dim3((unsigned)((nq + B - 1) / B)), dim3(B), 0, H->stream,
                           nz, nx, ncz, ncx, d_in, d_out);
    } else {
        const int64_t n = (int64_t)nz * nx;
        hipLaunchKernelGGL((k_bilinear<real>), dim3((unsigned)((n + B - 1) / B)), dim3(B), 0, H->stream,
                           nz, nx, ncz, ncx, d_in, d_out);
    }
    HIPCK(H, hipGetLastError());
    return ALI_OK;
}

}  // namespace ali

using namespace ali;

template <typename oreal, typename greal, typename outreal>
static ali_status adjoint_dispatch(ali_handle* h, const ali_medium* media, int32_t n_media, const ali_material* mats,
                                   int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient, const ali_node* srcs,
                                   const ali_node* recv, int mode, const greal* d_in, const ali_options* opt,
                                   outreal* d_T, outreal* d_trec, double* d_loss, outreal* d_dth,
                                   outreal* d_dA, ali_adjoint_stats* stats) {
    const int arith = opt ? opt->arith : ALI_ARITH_MIXED;
    if (arith == ALI_ARITH_MIXED)
        return adjoint_impl<float, oreal, greal, outreal>(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs,
                                                          recv, mode, d_in, opt, d_T, d_trec, d_loss, d_dth, d_dA,
                                                          stats);
    if (arith == ALI_ARITH_F64)
        return adjoint_impl<double, oreal, greal, outreal>(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs,
                                                           recv, mode, d_in, opt, d_T, d_trec, d_loss, d_dth, d_dA,
                                                           stats);
    return h->fail(ALI_EUNSUPPORTED, "the adjoint needs float64 travel times: use ALI_ARITH_MIXED or ALI_ARITH_F64");
}

extern "C" ali_status ali_adjoint(ali_handle* h, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                                  const uint8_t* d_mat_id, const float* d_orient, const ali_node* srcs,
                                  int32_t n_src, const ali_node* recv, int32_t n_recv, const float* d_dLdT,
                                  const ali_options* opt, float* d_T, float* d_dLdtheta,
                                  ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    const ali_medium md = single_medium(grid, n_mats, n_src, n_recv);
    return adjoint_dispatch<float, float, float>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, recv, 0, d_dLdT,
                                                 opt, d_T, (float*)nullptr, nullptr, d_dLdtheta,
                                                 (float*)nullptr, stats);
}

extern "C" ali_status ali_adjoint_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                                      const uint8_t* d_mat_id, const double* d_orient, const ali_node* srcs,
                                      int32_t n_src, const ali_node* recv, int32_t n_recv, const double* d_dLdT,
                                      const ali_options* opt, double* d_T, double* d_dLdtheta,
                                      ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    const ali_medium md = single_medium(grid, n_mats, n_src, n_recv);
    return adjoint_impl<double, double, double, double>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, recv, 0,
                                                        d_dLdT, opt, d_T, (double*)nullptr, nullptr, d_dLdtheta,
                                                        (double*)nullptr, stats);
}

extern "C" ali_status ali_adjoint_stiffness(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                            int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                            const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                            int32_t n_recv, const float* d_dLdT, const ali_options* opt,
                                            float* d_T, float* d_dLdtheta, float* d_dLdA,
                                            ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    if (!d_dLdA) return h->fail(ALI_EINVAL, "d_dLdA is NULL");
    const ali_medium md = single_medium(grid, n_mats, n_src, n_recv);
    return adjoint_dispatch<float, float, float>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, recv, 0, d_dLdT,
                                                 opt, d_T, (float*)nullptr, nullptr, d_dLdtheta, d_dLdA, stats);
}

extern "C" ali_status ali_adjoint_stiffness_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                                int32_t n_mats, const uint8_t* d_mat_id, const double* d_orient,
                                                const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                                int32_t n_recv, const double* d_dLdT, const ali_options* opt,
                                                double* d_T, double* d_dLdtheta, double* d_dLdA,
                                                ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    if (!d_dLdA) return h->fail(ALI_EINVAL, "d_dLdA is NULL");
    const ali_medium md = single_medium(grid, n_mats, n_src, n_recv);
    return adjoint_impl<double, double, double, double>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, recv, 0,
                                                        d_dLdT, opt, d_T, (double*)nullptr, nullptr, d_dLdtheta,
                                                        d_dLdA, stats);
}

extern "C" ali_status ali_misfit_gradient(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                          int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                          const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                          int32_t n_recv, const float* d_obs, const ali_options* opt,
                                          float* d_T, float* d_Trec, double* d_loss, float* d_dLdtheta,
                                          ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    const ali_medium md = single_medium(grid, n_mats, n_src, n_recv);
    return adjoint_dispatch<float, float, float>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, recv, 1, d_obs,
                                                 opt, d_T, d_Trec, d_loss, d_dLdtheta, (float*)nullptr, stats);
}

extern "C" ali_status ali_misfit_gradient_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                              int32_t n_mats, const uint8_t* d_mat_id, const double* d_orient,
                                              const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                              int32_t n_recv, const double* d_obs, const ali_options* opt,
                                              double* d_T, double* d_Trec, double* d_loss, double* d_dLdtheta,
                                              ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    const ali_medium md = single_medium(grid, n_mats, n_src, n_recv);
    return adjoint_impl<double, double, double, double>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, recv, 1,
                                                        d_obs, opt, d_T, d_Trec, d_loss, d_dLdtheta, (double*)nullptr,
                                                        stats);
}

extern "C" ali_status ali_misfit_gradient_stiffness(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                                    int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                                    const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                                    int32_t n_recv, const float* d_obs, const ali_options* opt,
                                                    float* d_T, float* d_Trec, double* d_loss, float* d_dLdtheta,
                                                    float* d_dLdA, ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    if (!d_dLdA) return h->fail(ALI_EINVAL, "d_dLdA is NULL");
    const ali_medium md = single_medium(grid, n_mats, n_src, n_recv);
    return adjoint_dispatch<float, float, float>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, recv, 1, d_obs,
                                                 opt, d_T, d_Trec, d_loss, d_dLdtheta, d_dLdA, stats);
}

extern "C" ali_status ali_misfit_gradient_stiffness_f64(ali_handle* h, const ali_grid* grid,
                                                        const ali_material* mats, int32_t n_mats,
                                                        const uint8_t* d_mat_id, const double* d_orient,
                                                        const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                                        int32_t n_recv, const double* d_obs, const ali_options* opt,
                                                        double* d_T, double* d_Trec, double* d_loss,
                                                        double* d_dLdtheta, double* d_dLdA,
                                                        ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    if (!d_dLdA) return h->fail(ALI_EINVAL, "d_dLdA is NULL");
    const ali_medium md = single_medium(grid, n_mats, n_src, n_recv);
    return adjoint_impl<double, double, double, double>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, recv, 1,
                                                        d_obs, opt, d_T, d_Trec, d_loss, d_dLdtheta, d_dLdA, stats);
}

extern "C" ali_status ali_misfit_gradient_batch_stiffness(ali_handle* h, const ali_medium* media, int32_t n_media,
                                                          const ali_material* mats, int32_t n_mats,
                                                          const uint8_t* d_mat_id, const float* d_orient,
                                                          const ali_node* srcs, const ali_node* recv,
                                                          const float* d_obs, const ali_options* opt, float* d_Trec,
                                                          double* d_loss, float* d_dLdtheta, float* d_dLdA,
                                                          ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!d_dLdA) return h->fail(ALI_EINVAL, "d_dLdA is NULL");
    return adjoint_dispatch<float, float, float>(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, recv, 1,
                                                 d_obs, opt, (float*)nullptr, d_Trec, d_loss, d_dLdtheta, d_dLdA,
                                                 stats);
}

extern "C" ali_status ali_misfit_gradient_batch(ali_handle* h, const ali_medium* media, int32_t n_media,
                                                const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                                const float* d_orient, const ali_node* srcs, const ali_node* recv,
                                                const float* d_obs, const ali_options* opt, float* d_Trec,
                                                double* d_loss, float* d_dLdtheta, ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    return adjoint_dispatch<float, float, float>(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, recv, 1,
                                                 d_obs, opt, (float*)nullptr, d_Trec, d_loss, d_dLdtheta,
                                                 (float*)nullptr, stats);
}

extern "C" ali_status ali_bilinear(ali_handle* h, int32_t nz, int32_t nx, int32_t ncz, int32_t ncx,
                                   const float* d_ctrl, float* d_orient) {
    if (!h) return ALI_EINVAL;
    return bilinear_impl<float>(h, nz, nx, ncz, ncx, d_ctrl, d_orient, false);
}

extern "C" ali_status ali_bilinear_transpose(ali_handle* h, int32_t nz, int32_t nx, int32_t ncz, int32_t ncx,
                                             const float* d_dLdtheta, float* d_dLdctrl) {
    if (!h) return ALI_EINVAL;
    return bilinear_impl<float>(h, nz, nx, ncz, ncx, d_dLdtheta, d_dLdctrl, true);
}

extern "C" ali_status ali_bilinear_f64(ali_handle* h, int32_t nz, int32_t nx, int32_t ncz, int32_t ncx,
                                       const double* d_ctrl, double* d_orient) {
    if (!h) return ALI_EINVAL;
    return bilinear_impl<double>(h, nz, nx, ncz, ncx, d_ctrl, d_orient, false);
}

extern "C" ali_status ali_bilinear_transpose_f64(ali_handle* h, int32_t nz, int32_t nx, int32_t ncz, int32_t ncx,
                                                 const double* d_dLdtheta, double* d_dLdctrl) {
    if (!h) return ALI_EINVAL;
    return bilinear_impl<double>(h, nz, nx, ncz, ncx, d_dLdtheta, d_dLdctrl, true);
}
