// ali_adjoint.hip -- gradient of receiver travel times with respect to the orientation of
// the symmetry axis at every node (gfx950).
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
//      estimate formula); one record per node and field;
//   3. k_adj_relax: tiled relaxation of the lambda equation.  Each evaluation recomputes
//      lambda(X) from scratch as a sum in a fixed order, so the end state (no value
//      changes) is the exact solution and independent of the schedule; on a DAG the
//      relaxation ends after at most its depth in sweeps;
//   4. k_adj_grad / k_adj_box: per-node gradient summed over fields in field order
//      (deterministic), plus the source-box terms.
#include <hip/hip_runtime.h>
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

struct StGeo { int sa, sb, sc, bx, bz, cx, cz, k1, k2; };

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

// Float64 node constants for the derivatives (the phase-speed constants / h^2 and the
// double angle of the axis).
struct NodeD { double c2t, s2t, P, Q, R, K4; };

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

// ---------------------------------------------------------------------------------------
// step 2: choices and partial derivatives, one work-group per (tile, field)
// ---------------------------------------------------------------------------------------
template <typename mreal, typename oreal>
__global__ void __launch_bounds__(NTHREADS)
k_adj_prep(int nx, int nz, int ntx, int ntz, double h, const MatDev<mreal>* __restrict__ mats,
           const uint8_t* __restrict__ mat_id, const oreal* __restrict__ orient,
           const mreal* __restrict__ geo, const double* __restrict__ fbt,
           const int2* __restrict__ src, int R, const double* __restrict__ T,
           uint16_t* __restrict__ code, double* __restrict__ wA, double* __restrict__ wB,
           double* __restrict__ wC, double* __restrict__ wT,
           unsigned long long* __restrict__ mismatches) {
    __shared__ double lt[LH * LSTRIDE];
    const int ntiles = ntx * ntz;
    const int f = blockIdx.x / ntiles;
    const int tile = blockIdx.x % ntiles;
    const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TZ;
    const int64_t N = (int64_t)nx * nz;
    const double* __restrict__ Tf = T + (int64_t)f * N;
    const double inf = dinf<double>();
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
    const int64_t q = (int64_t)f * N + p;
    const int2 s = src[f];
    const int me = (lz + HALO) * LSTRIDE + (lx + HALO);
    const double tD = lt[me];
    uint16_t cd = CODE_NONE;
    double a = 0.0, b = 0.0, c = 0.0, t = 0.0;
    const int di = gi - s.x, dj = gj - s.y;
    if (abs(di) <= R && abs(dj) <= R) {
        // straight ray from the source at the source node's orientation and material
        cd = make_code(K_BOX, NO_SLOT, NO_SLOT, NO_SLOT);
        if (di != 0 || dj != 0) {
            const int64_t ps = (int64_t)s.y * nx + s.x;
            const double phi = atan2((double)dj, (double)di) - (double)orient[ps];
            double dV;
            const double V = group_speed(mats[mat_id[ps]].A, phi, &dV);
            t = sqrt((double)(di * di + dj * dj)) * h * dV / (V * V);
        }
    } else if (tD < inf) {
        NodeConst<mreal, double> nc;
        load_node_const<double, mreal>(nc, p, mats, mat_id, geo, fbt);
        double tt[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) tt[k] = lt[me + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k]];
        unsigned ev = 0;
        int ch = -1;
        const double u = local_update<mreal, double>(nc, tt, lt, me, LSTRIDE, ev, &ch);
        if (!(u == tD)) atomicAdd(mismatches, 1ull);
        const MatA& A = mats[mat_id[p]].A;
        const double th = (double)orient[p];
        if (ch >= 0 && ch < 32) {
            const StGeo g = stencil_geo(ch, std::make_integer_sequence<int, 32>{});
            NodeD nd;
            sincos(2.0 * th, &nd.s2t, &nd.c2t);
            const double ih2 = 1.0 / (h * h);
            nd.P = (A.a11 + A.a33 + 2.0 * A.a55) * ih2;
            nd.Q = (A.a33 - A.a11) * ih2;
            nd.R = (A.a11 + A.a33 - 2.0 * A.a55) * ih2;
            const double W = (A.a13 + A.a55) * ih2;
            nd.K4 = 4.0 * W * W;
            stencil_partials(nd, g, tt[g.sa], tt[g.sb], tt[g.sc], a, b, c, t);
            cd = make_code(K_STENCIL, (unsigned)g.sa, (unsigned)g.sb, (unsigned)g.sc);
        } else if (ch >= 32) {
            const int k = ch - 32;
            const int d = fb_dir_rt(k);
            const double quarter = 0.78539816339744830962;
            const double ang = d == 0 ? 0.0 : d == 1 ? quarter : d == 2 ? 2.0 * quarter : -quarter;
            const double len = (d & 1) ? 1.41421356237309504880 : 1.0;
            double dV;
            const double V = group_speed(A, ang - th, &dV);
            a = 1.0;
            t = len * h * dV / (V * V);
            cd = make_code(K_FALLBACK, (unsigned)fb_slot_rt(k), NO_SLOT, NO_SLOT);
        }
    }
    code[q] = cd;
    wA[q] = a; wB[q] = b; wC[q] = c; wT[q] = t;
}

// ---------------------------------------------------------------------------------------
// step 3: relaxation of lambda, one work-group per active (tile, field)
// ---------------------------------------------------------------------------------------
// contribution to lambda at the node in LDS slot `me` from its 12 diamond neighbours
__device__ __forceinline__ double pull_lambda(double gsum, int me, const double* __restrict__ ll,
                                              const uint16_t* __restrict__ lc, const double* __restrict__ la,
                                              const double* __restrict__ lb, const double* __restrict__ lcw) {
    double s = gsum;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const int o = me + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k];
        const unsigned cd = lc[o];
        const unsigned tgt = 11u - (unsigned)k;       // this node seen from the neighbour
        if ((cd & 0xFu) == tgt) s += ll[o] * la[o];
        else if (((cd >> 4) & 0xFu) == tgt) s += ll[o] * lb[o];
        else if (((cd >> 8) & 0xFu) == tgt) s += ll[o] * lcw[o];
    }
    return s;
}

__global__ void __launch_bounds__(NTHREADS)
k_adj_relax(int nx, int nz, int ntx, int ntz, const uint32_t* __restrict__ list,
            const uint32_t* __restrict__ lbits, const uint16_t* __restrict__ code,
            const double* __restrict__ wA, const double* __restrict__ wB, const double* __restrict__ wC,
            const double* __restrict__ G, const double* __restrict__ T, const double* __restrict__ theta,
            double* __restrict__ lam, uint8_t* __restrict__ pend, double* __restrict__ maxdef,
            uint32_t* __restrict__ flags, int inner, unsigned long long* __restrict__ counters) {
    __shared__ double ll[LH * LSTRIDE];
    __shared__ double la[LH * LSTRIDE], lb[LH * LSTRIDE], lcw[LH * LSTRIDE];
    __shared__ uint16_t lc[LH * LSTRIDE];
    __shared__ double ltau[NTHREADS];
    __shared__ uint8_t lpend[NTHREADS];
    __shared__ uint8_t dirty[2][NTHREADS];
    __shared__ uint16_t clist[NTHREADS];
    __shared__ unsigned wcount[NTHREADS / 64];
    __shared__ unsigned edge_out, blk_updates;
    __shared__ unsigned long long def_key;

    const uint32_t unit = list[blockIdx.x];
    const uint32_t bits = lbits[blockIdx.x];
    const int ntiles = ntx * ntz;
    const int f = (int)(unit / (uint32_t)ntiles);
    const int tile = (int)(unit % (uint32_t)ntiles);
    const int tx = tile % ntx, tz = tile / ntx;
    const int i0 = tx * TX, j0 = tz * TZ;
    const int64_t N = (int64_t)nx * nz;
    const int64_t fo = (int64_t)f * N;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;

    for (int q = tid; q < LW * LH; q += NTHREADS) {
        const int li = q % LW, lj = q / LW;
        const int gi = i0 - HALO + li, gj = j0 - HALO + lj;
        const int o = lj * LSTRIDE + li;
        if (gi >= 0 && gj >= 0 && gi < nx && gj < nz) {
            const int64_t p = fo + (int64_t)gj * nx + gi;
            ll[o] = lam[p];
            lc[o] = code[p];
            la[o] = wA[p]; lb[o] = wB[p]; lcw[o] = wC[p];
        } else {
            ll[o] = 0.0;
            lc[o] = CODE_NONE;
            la[o] = 0.0; lb[o] = 0.0; lcw[o] = 0.0;
        }
    }
    const int lx = tid % TX, lz = tid / TX;
    const int gi = i0 + lx, gj = j0 + lz;
    const bool valid = gi < nx && gj < nz;
    const int64_t pme = fo + (int64_t)gj * nx + gi;
    const uint8_t pend0 = valid ? pend[pme] : 0;
    ltau[tid] = valid ? T[pme] : 0.0;
    lpend[tid] = pend0;
    const double th = theta[f];
    if (tid == 0) { edge_out = 0u; blk_updates = 0u; def_key = 0ull; }
    {
        const bool d = (bits & TF_SELF) ||
                       ((bits & TF_HALO_L) && lx < HALO) || ((bits & TF_HALO_R) && lx >= TX - HALO) ||
                       ((bits & TF_HALO_U) && lz < HALO) || ((bits & TF_HALO_D) && lz >= TZ - HALO) ||
                       ((bits & TF_HALO_UL) && lx == 0 && lz == 0) ||
                       ((bits & TF_HALO_UR) && lx == TX - 1 && lz == 0) ||
                       ((bits & TF_HALO_DL) && lx == 0 && lz == TZ - 1) ||
                       ((bits & TF_HALO_DR) && lx == TX - 1 && lz == TZ - 1);
        dirty[0][tid] = (valid && (d || pend0)) ? 1 : 0;
        dirty[1][tid] = 0;
    }
    __syncthreads();
    const int me = (lz + HALO) * LSTRIDE + (lx + HALO);
    const double orig = ll[me];
    unsigned my_updates = 0;
    bool done = false;
    for (int it = 0;; ++it) {
        const int cur = it & 1;
        const bool d = dirty[cur][tid] != 0;
        dirty[cur][tid] = 0;
        const unsigned long long m = __ballot(d);
        const unsigned below = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[wave] = (unsigned)__popcll(m);
        __syncthreads();
        unsigned base = 0, total = 0;
#pragma unroll
        for (int w = 0; w < NTHREADS / 64; ++w) {
            const unsigned c = wcount[w];
            base += w < wave ? c : 0u;
            total += c;
        }
        if (d) clist[base + below] = (uint16_t)tid;
        __syncthreads();
        if (total == 0) { done = true; break; }
        if (it == inner) break;
        if ((unsigned)tid < total) {
            const int node = clist[tid];
            const int nlx = node % TX, nlz = node / TX;
            const int nme = (nlz + HALO) * LSTRIDE + (nlx + HALO);
            // time band: a node below the threshold waits (pending) until the band
            // reaches it, by which time the nodes it pulls from are final or close to it
            const bool ready = ltau[node] >= th;
            lpend[node] = ready ? 0 : 1;
            double v = ll[nme];
            if (ready) {
                ++my_updates;
                v = pull_lambda(G[fo + (int64_t)(j0 + nlz) * nx + (i0 + nlx)], nme, ll, lc, la, lb, lcw);
            }
            if (v != ll[nme]) {
                ll[nme] = v;
                // lambda flows into this node's supports: mark those inside the tile
                const unsigned cd = lc[nme];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const unsigned sl = (cd >> (4 * r)) & 0xFu;
                    if (sl < 12u) {
                        int ax = nlx, az = nlz;
                        switch (sl) {
                            case 0: az -= 2; break;            case 1: ax -= 1; az -= 1; break;
                            case 2: az -= 1; break;            case 3: ax += 1; az -= 1; break;
                            case 4: ax -= 2; break;            case 5: ax -= 1; break;
                            case 6: ax += 1; break;            case 7: ax += 2; break;
                            case 8: ax -= 1; az += 1; break;   case 9: az += 1; break;
                            case 10: ax += 1; az += 1; break;  default: az += 2; break;
                        }
                        if (ax >= 0 && az >= 0 && ax < TX && az < TZ && i0 + ax < nx && j0 + az < nz)
                            dirty[cur ^ 1][az * TX + ax] = 1;
                    }
                }
            }
        }
        __syncthreads();
    }

    const double fin = ll[me];
    if (valid && fin != orig) {
        lam[fo + (int64_t)gj * nx + gi] = fin;
        unsigned e = 0;
        if (lx < HALO) e |= 1u;
        if (lx >= TX - HALO) e |= 2u;
        if (lz < HALO) e |= 4u;
        if (lz >= TZ - HALO) e |= 8u;
        if (lx == 0 && lz == 0) e |= 16u;
        if (lx == TX - 1 && lz == 0) e |= 32u;
        if (lx == 0 && lz == TZ - 1) e |= 64u;
        if (lx == TX - 1 && lz == TZ - 1) e |= 128u;
        if (e) atomicOr(&edge_out, e);
    }
    if (valid && lpend[tid] != pend0) pend[pme] = lpend[tid];
    // largest time of a pending node (non-negative doubles order as their bit patterns)
    if (valid && lpend[tid]) atomicMax(&def_key, (unsigned long long)__double_as_longlong(ltau[tid]) + 1ull);
    if (my_updates) atomicAdd(&blk_updates, my_updates);
    __syncthreads();
    if (tid == 0) {
        if (blk_updates) atomicAdd(&counters[0], (unsigned long long)blk_updates);
        const unsigned long long dk = def_key;
        maxdef[(int64_t)f * ntiles + tile] = dk ? __longlong_as_double((long long)(dk - 1ull)) : -dinf<double>();
        uint32_t* fl = flags + (int64_t)f * ntiles;
        const unsigned e = edge_out;
        const bool hasL = tx > 0, hasR = tx + 1 < ntx, hasU = tz > 0, hasD = tz + 1 < ntz;
        if (!done) atomicOr(&fl[tile], TF_SELF);
        if ((e & 1u) && hasL) atomicOr(&fl[tile - 1], TF_HALO_R);
        if ((e & 2u) && hasR) atomicOr(&fl[tile + 1], TF_HALO_L);
        if ((e & 4u) && hasU) atomicOr(&fl[tile - ntx], TF_HALO_D);
        if ((e & 8u) && hasD) atomicOr(&fl[tile + ntx], TF_HALO_U);
        if ((e & 16u) && hasL && hasU) atomicOr(&fl[tile - ntx - 1], TF_HALO_DR);
        if ((e & 32u) && hasR && hasU) atomicOr(&fl[tile - ntx + 1], TF_HALO_DL);
        if ((e & 64u) && hasL && hasD) atomicOr(&fl[tile + ntx - 1], TF_HALO_UR);
        if ((e & 128u) && hasR && hasD) atomicOr(&fl[tile + ntx + 1], TF_HALO_UL);
    }
}

__global__ void k_adj_compact(uint32_t* __restrict__ flags, const double* __restrict__ maxdef, int64_t n,
                              int ntiles, const double* __restrict__ theta, uint32_t* __restrict__ list,
                              uint32_t* __restrict__ lbits, uint32_t* __restrict__ count) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const uint32_t b = flags[u];
    const double md = maxdef[u];
    if (b || (md > -dinf<double>() && md >= theta[u / ntiles])) {
        flags[u] = 0;
        const uint32_t pos = atomicAdd(count, 1u);
        list[pos] = (uint32_t)u;
        lbits[pos] = b;
    }
}

__global__ void k_adj_zero(uint32_t* p) { *p = 0u; }

// nothing active: lower each field's threshold to its largest pending time, if any
__global__ void k_adj_jump(const double* __restrict__ maxdef, int ntiles, double* __restrict__ theta,
                           uint32_t* __restrict__ jumped) {
    const int f = blockIdx.x;
    double m = -dinf<double>();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
        const double v = maxdef[(int64_t)f * ntiles + t];
        m = v > m ? v : m;
    }
    __shared__ double red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x + w] > red[threadIdx.x] ? red[threadIdx.x + w] : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] > -dinf<double>()) {
        if (red[0] < theta[f]) theta[f] = red[0];
        atomicAdd(jumped, 1u);
    }
}

__global__ void k_adj_advance(double* __restrict__ theta, double step, int nf) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < nf) theta[f] -= step;
}

// ---------------------------------------------------------------------------------------
// right-hand side: g = dL/dT at the receivers, one thread per field (receivers in order)
// ---------------------------------------------------------------------------------------
// mode 0: g given per (field, receiver).  mode 1: misfit L = 1/2 sum (T - obs)^2, so
// g = T - obs; also writes T at the receivers and the per-field misfit.
template <typename greal, typename outreal>
__global__ void k_adj_rhs(int mode, int nf, int nrec, int nx, int64_t N, int ntx,
                          const int2* __restrict__ rec, const greal* __restrict__ in,
                          const double* __restrict__ T, double* __restrict__ G,
                          outreal* __restrict__ trec, double* __restrict__ lossf,
                          uint32_t* __restrict__ flags, int ntiles, double* __restrict__ theta,
                          int banded) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    double L = 0.0;
    double tmax = -dinf<double>();
    for (int r = 0; r < nrec; ++r) {
        const int2 x = rec[r];
        const int64_t p = (int64_t)f * N + (int64_t)x.y * nx + x.x;
        double g = (double)in[(int64_t)f * nrec + r];
        if (mode == 1) {
            const double t = T[p];
            g = t - g;
            L += 0.5 * g * g;
            if (trec) trec[(int64_t)f * nrec + r] = (outreal)t;
        }
        G[p] += g;
        tmax = T[p] > tmax ? T[p] : tmax;
        flags[(int64_t)f * ntiles + (x.y / TZ) * ntx + (x.x / TX)] |= TF_SELF;
    }
    if (lossf) lossf[f] = L;
    // nodes later than every receiver carry no sensitivity: the band starts there
    theta[f] = banded ? tmax : -dinf<double>();
}

__global__ void k_adj_loss(const double* __restrict__ lossf, int nf, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int f = 0; f < nf; ++f) s += lossf[f];
        *out = s;
    }
}

// ---------------------------------------------------------------------------------------
// step 4: gradient
// ---------------------------------------------------------------------------------------
__global__ void k_adj_grad(int64_t N, int nf, const uint16_t* __restrict__ code, const double* __restrict__ wT,
                           const double* __restrict__ lam, double* __restrict__ dth) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    double s = 0.0;
    for (int f = 0; f < nf; ++f) {
        const int64_t q = (int64_t)f * N + p;
        const int kind = code[q] >> 12;
        if (kind == K_STENCIL || kind == K_FALLBACK) s += lam[q] * wT[q];
    }
    dth[p] = s;
}

// source-box terms of field f, reduced in a fixed order
__global__ void k_adj_box(int nx, int nz, int64_t N, int R, const int2* __restrict__ src,
                          const double* __restrict__ wT, const double* __restrict__ lam,
                          double* __restrict__ boxsum) {
    const int f = blockIdx.x;
    const int2 s = src[f];
    const int w = 2 * R + 1;
    double acc = 0.0;
    for (int k = threadIdx.x; k < w * w; k += blockDim.x) {
        const int i = s.x - R + k % w, j = s.y - R + k / w;
        if (i < 0 || j < 0 || i >= nx || j >= nz) continue;
        const int64_t q = (int64_t)f * N + (int64_t)j * nx + i;
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

// one work-item adds the box terms at the source nodes in field order
__global__ void k_adj_box_add(int nf, int nx, const int2* __restrict__ src, const double* __restrict__ boxsum,
                              double* __restrict__ dth) {
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int f = 0; f < nf; ++f) dth[(int64_t)src[f].y * nx + src[f].x] += boxsum[f];
}

// ---------------------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------------------
template <typename mreal, typename oreal, typename greal, typename outreal>
static ali_status adjoint_impl(ali_handle* H, const ali_grid* grid, const ali_material* mats,
                               int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient,
                               const ali_node* srcs, int32_t n_src, const ali_node* recv, int32_t n_recv,
                               int mode, const greal* d_in, const ali_options* opt_in, outreal* d_T,
                               outreal* d_trec, double* d_loss, outreal* d_dth, ali_adjoint_stats* stats) {
    ali_options opt;
    ali_default_options(&opt);
    if (opt_in) opt = *opt_in;
    ali_status st = validate_medium(H, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src);
    if (st != ALI_OK) return st;
    if (!recv || n_recv < 1) return H->fail(ALI_EINVAL, "need at least one receiver");
    for (int r = 0; r < n_recv; ++r)
        if (recv[r].i < 0 || recv[r].j < 0 || recv[r].i >= grid->nx || recv[r].j >= grid->nz)
            return H->fail(ALI_EINVAL, "receiver " + std::to_string(r) + " outside the grid");
    if (!d_in) return H->fail(ALI_EINVAL, mode == 1 ? "d_obs is NULL" : "d_dLdT is NULL");
    if (!d_dth) return H->fail(ALI_EINVAL, "d_dLdtheta is NULL");
    const int nx = grid->nx, nz = grid->nz;
    const int64_t N = (int64_t)nx * nz;
    const int64_t NF = N * n_src;

    // forward field in float64: the caller's buffer when it is float64, else scratch
    constexpr bool out64 = std::is_same<outreal, double>::value;
    void* d_work = nullptr;
    if (!(out64 && d_T) && !H->scratch("adjT", sizeof(double) * NF, &d_work))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    double* T = (out64 && d_T) ? (double*)d_T : (double*)d_work;

    ali_solve_stats fst{};
    ForwardState<double, mreal> fs;
    st = solve_core<double, mreal, oreal>(H, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src,
                                                     opt, T, &fst, &fs);
    if (st != ALI_OK) return st;
    hipStream_t S = H->stream;
    HIPCK(H, hipEventRecord(H->ev4, S));
    const int ntx = fs.ntx, ntz = fs.ntz, ntiles = ntx * ntz;
    const int64_t nunits = (int64_t)ntiles * n_src;

    void *d_code, *d_wA, *d_wB, *d_wC, *d_wT, *d_lam, *d_G, *d_dacc, *d_box, *d_lossf, *d_rec;
    void *d_flags, *d_list, *d_lbits, *d_count, *d_cnt, *d_pend, *d_maxdef, *d_theta;
    if (!H->scratch("a_code", sizeof(uint16_t) * NF, &d_code) ||
        !H->scratch("a_wA", sizeof(double) * NF, &d_wA) || !H->scratch("a_wB", sizeof(double) * NF, &d_wB) ||
        !H->scratch("a_wC", sizeof(double) * NF, &d_wC) || !H->scratch("a_wT", sizeof(double) * NF, &d_wT) ||
        !H->scratch("a_lam", sizeof(double) * NF, &d_lam) || !H->scratch("a_G", sizeof(double) * NF, &d_G) ||
        !H->scratch("a_pend", sizeof(uint8_t) * NF, &d_pend) ||
        !H->scratch("a_dth", sizeof(double) * N, &d_dacc) || !H->scratch("a_box", sizeof(double) * n_src, &d_box) ||
        !H->scratch("a_lossf", sizeof(double) * n_src, &d_lossf) ||
        !H->scratch("a_theta", sizeof(double) * n_src, &d_theta) ||
        !H->scratch("a_rec", sizeof(int2) * n_recv, &d_rec) ||
        !H->scratch("a_flags", sizeof(uint32_t) * nunits, &d_flags) ||
        !H->scratch("a_maxdef", sizeof(double) * nunits, &d_maxdef) ||
        !H->scratch("a_list", sizeof(uint32_t) * nunits, &d_list) ||
        !H->scratch("a_lbits", sizeof(uint32_t) * nunits, &d_lbits) ||
        !H->scratch("a_count", sizeof(uint32_t), &d_count) ||
        !H->scratch("a_cnt", 2 * sizeof(unsigned long long), &d_cnt))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    std::vector<int2> hr(n_recv);
    for (int r = 0; r < n_recv; ++r) hr[r] = make_int2(recv[r].i, recv[r].j);
    HIPCK(H, hipMemcpyAsync(d_rec, hr.data(), sizeof(int2) * n_recv, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemsetAsync(d_flags, 0, sizeof(uint32_t) * nunits, S));
    HIPCK(H, hipMemsetAsync(d_cnt, 0, 2 * sizeof(unsigned long long), S));
    // descending time band: band_cells node spacings at the fastest phase speed
    const bool banded = opt.band_cells > 0;
    const double band = banded ? opt.band_cells * grid->h / max_phase_speed(mats, n_mats) : 0.0;

    const int B = 256;
    const unsigned gNF = (unsigned)((NF + B - 1) / B);
    hipLaunchKernelGGL((k_adj_prep<mreal, oreal>), dim3((unsigned)nunits), dim3(NTHREADS), 0, S,
                       nx, nz, ntx, ntz, grid->h, fs.mats, d_mat_id, d_orient, fs.geo, fs.fbt, fs.src,
                       opt.src_box_radius, (const double*)T, (uint16_t*)d_code, (double*)d_wA, (double*)d_wB,
                       (double*)d_wC, (double*)d_wT, (unsigned long long*)d_cnt + 1);
    HIPCK(H, hipGetLastError());
    hipLaunchKernelGGL((k_fill<double>), dim3(gNF), dim3(B), 0, S, (double*)d_G, NF, 0.0);
    hipLaunchKernelGGL((k_fill<double>), dim3(gNF), dim3(B), 0, S, (double*)d_lam, NF, 0.0);
    hipLaunchKernelGGL((k_fill<uint8_t>), dim3(gNF), dim3(B), 0, S, (uint8_t*)d_pend, NF, (uint8_t)0);
    hipLaunchKernelGGL((k_fill<double>), dim3((unsigned)((nunits + B - 1) / B)), dim3(B), 0, S, (double*)d_maxdef,
                       nunits, -dinf_host<double>());
    hipLaunchKernelGGL((k_adj_rhs<greal, outreal>), dim3((unsigned)((n_src + 63) / 64)), dim3(64), 0, S,
                       mode, n_src, n_recv, nx, N, ntx, (const int2*)d_rec, d_in, (const double*)T,
                       (double*)d_G, d_trec, (double*)d_lossf, (uint32_t*)d_flags, ntiles, (double*)d_theta,
                       banded ? 1 : 0);
    HIPCK(H, hipGetLastError());
    if (mode == 1 && d_loss)
        hipLaunchKernelGGL(k_adj_loss, dim3(1), dim3(64), 0, S, (const double*)d_lossf, n_src, d_loss);

    int iters = 0;
    int64_t visits = 0;
    bool converged = false;
    double relax_ms = 0.0;
    bool pending = false;
    uint32_t* h_count = H->host_count;
    for (;;) {
        hipLaunchKernelGGL(k_adj_zero, dim3(1), dim3(1), 0, S, (uint32_t*)d_count);
        hipLaunchKernelGGL(k_adj_compact, dim3((unsigned)((nunits + B - 1) / B)), dim3(B), 0, S,
                           (uint32_t*)d_flags, (const double*)d_maxdef, nunits, ntiles, (const double*)d_theta,
                           (uint32_t*)d_list, (uint32_t*)d_lbits, (uint32_t*)d_count);
        HIPCK(H, hipGetLastError());
        HIPCK(H, hipMemcpyAsync(h_count, d_count, sizeof(uint32_t), hipMemcpyDeviceToHost, S));
        HIPCK(H, hipStreamSynchronize(S));
        if (pending) {
            float kms = 0.f;
            HIPCK(H, hipEventElapsedTime(&kms, H->ev2, H->ev3));
            relax_ms += kms;
            pending = false;
        }
        const uint32_t n = *h_count;
        if (n == 0) {
            // nothing active: lower the thresholds to the largest pending times, if any
            hipLaunchKernelGGL(k_adj_zero, dim3(1), dim3(1), 0, S, (uint32_t*)d_count);
            hipLaunchKernelGGL(k_adj_jump, dim3((unsigned)n_src), dim3(256), 0, S, (const double*)d_maxdef,
                               ntiles, (double*)d_theta, (uint32_t*)d_count);
            HIPCK(H, hipGetLastError());
            HIPCK(H, hipMemcpyAsync(h_count, d_count, sizeof(uint32_t), hipMemcpyDeviceToHost, S));
            HIPCK(H, hipStreamSynchronize(S));
            if (*h_count == 0) { converged = true; break; }
            continue;
        }
        if (iters >= opt.max_sweeps) break;
        HIPCK(H, hipEventRecord(H->ev2, S));
        hipLaunchKernelGGL(k_adj_relax, dim3(n), dim3(NTHREADS), 0, S, nx, nz, ntx, ntz,
                           (const uint32_t*)d_list, (const uint32_t*)d_lbits, (const uint16_t*)d_code,
                           (const double*)d_wA, (const double*)d_wB, (const double*)d_wC,
                           (const double*)d_G, (const double*)T, (const double*)d_theta, (double*)d_lam,
                           (uint8_t*)d_pend, (double*)d_maxdef, (uint32_t*)d_flags, opt.inner_sweeps,
                           (unsigned long long*)d_cnt);
        HIPCK(H, hipGetLastError());
        HIPCK(H, hipEventRecord(H->ev3, S));
        if (banded)
            hipLaunchKernelGGL(k_adj_advance, dim3((unsigned)((n_src + 63) / 64)), dim3(64), 0, S,
                               (double*)d_theta, band, n_src);
        pending = true;
        ++iters;
        visits += n;
    }

    hipLaunchKernelGGL(k_adj_grad, dim3((unsigned)((N + B - 1) / B)), dim3(B), 0, S, N, n_src,
                       (const uint16_t*)d_code, (const double*)d_wT, (const double*)d_lam, (double*)d_dacc);
    hipLaunchKernelGGL(k_adj_box, dim3((unsigned)n_src), dim3(256), 0, S, nx, nz, N, opt.src_box_radius,
                       fs.src, (const double*)d_wT, (const double*)d_lam, (double*)d_box);
    hipLaunchKernelGGL(k_adj_box_add, dim3(1), dim3(64), 0, S, n_src, nx, fs.src, (const double*)d_box,
                       (double*)d_dacc);
    hipLaunchKernelGGL((k_convert<outreal, double>), dim3((unsigned)((N + B - 1) / B)), dim3(B), 0, S,
                       d_dth, (const double*)d_dacc, N);
    HIPCK(H, hipGetLastError());
    if (d_T && !out64)
        hipLaunchKernelGGL((k_convert<outreal, double>), dim3(gNF), dim3(B), 0, S, d_T, (const double*)T, NF);
    HIPCK(H, hipGetLastError());
    HIPCK(H, hipEventRecord(H->ev1, S));
    unsigned long long cnt[2] = {0, 0};
    HIPCK(H, hipMemcpyAsync(cnt, d_cnt, sizeof(cnt), hipMemcpyDeviceToHost, S));
    HIPCK(H, hipStreamSynchronize(S));
    if (stats) {
        float ms = 0.f;
        HIPCK(H, hipEventElapsedTime(&ms, H->ev0, H->ev1));
        float fms = 0.f;
        HIPCK(H, hipEventElapsedTime(&fms, H->ev0, H->ev4));
        stats->forward = fst;
        stats->forward.ms = fms;
        stats->lambda_updates = (int64_t)cnt[0];
        stats->choice_mismatches = (int64_t)cnt[1];
        stats->tile_visits = visits;
        stats->outer_iters = iters;
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

extern "C" ali_status ali_adjoint(ali_handle* h, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                                  const uint8_t* d_mat_id, const float* d_orient, const ali_node* srcs,
                                  int32_t n_src, const ali_node* recv, int32_t n_recv, const float* d_dLdT,
                                  const ali_options* opt, float* d_T, float* d_dLdtheta,
                                  ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    const int arith = opt ? opt->arith : ALI_ARITH_MIXED;
    if (arith == ALI_ARITH_MIXED)
        return adjoint_impl<float, float, float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, recv,
                                                        n_recv, 0, d_dLdT, opt, d_T, nullptr, nullptr, d_dLdtheta, stats);
    if (arith == ALI_ARITH_F64)
        return adjoint_impl<double, float, float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, recv,
                                                         n_recv, 0, d_dLdT, opt, d_T, nullptr, nullptr, d_dLdtheta, stats);
    return h->fail(ALI_EUNSUPPORTED, "the adjoint needs float64 travel times: use ALI_ARITH_MIXED or ALI_ARITH_F64");
}

extern "C" ali_status ali_adjoint_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                                      const uint8_t* d_mat_id, const double* d_orient, const ali_node* srcs,
                                      int32_t n_src, const ali_node* recv, int32_t n_recv, const double* d_dLdT,
                                      const ali_options* opt, double* d_T, double* d_dLdtheta,
                                      ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    return adjoint_impl<double, double, double, double>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, recv,
                                                        n_recv, 0, d_dLdT, opt, d_T, nullptr, nullptr, d_dLdtheta, stats);
}

extern "C" ali_status ali_misfit_gradient(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                          int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                          const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                          int32_t n_recv, const float* d_obs, const ali_options* opt,
                                          float* d_T, float* d_Trec, double* d_loss, float* d_dLdtheta,
                                          ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    const int arith = opt ? opt->arith : ALI_ARITH_MIXED;
    if (arith == ALI_ARITH_MIXED)
        return adjoint_impl<float, float, float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, recv,
                                                        n_recv, 1, d_obs, opt, d_T, d_Trec, d_loss, d_dLdtheta, stats);
    if (arith == ALI_ARITH_F64)
        return adjoint_impl<double, float, float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, recv,
                                                         n_recv, 1, d_obs, opt, d_T, d_Trec, d_loss, d_dLdtheta, stats);
    return h->fail(ALI_EUNSUPPORTED, "the adjoint needs float64 travel times: use ALI_ARITH_MIXED or ALI_ARITH_F64");
}

extern "C" ali_status ali_misfit_gradient_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                              int32_t n_mats, const uint8_t* d_mat_id, const double* d_orient,
                                              const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                              int32_t n_recv, const double* d_obs, const ali_options* opt,
                                              double* d_T, double* d_Trec, double* d_loss, double* d_dLdtheta,
                                              ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    return adjoint_impl<double, double, double, double>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, recv,
                                                        n_recv, 1, d_obs, opt, d_T, d_Trec, d_loss, d_dLdtheta, stats);
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
