// ali_solve.hip -- travel-time fields by tiled relaxation of the ALI update (gfx950).
//
// The paper orders node updates with a binary heap (Section 2).  Its result is the unique
// fixed point of a local operator: at node D, grow the known set in (tau, index) order
// over the diamond and stop once D's estimate precedes the next neighbour.  Any schedule
// that reaches a state where no node changes lands on that field, so the GPU relaxes
// tiles in parallel instead.  Each pass is two launches:
//   - k_sched (one work-group per field) advances the field's threshold and lists the
//     tiles that are due, each entry carrying what a visit needs to start staging;
//   - k_relax (one wave per tile visit) stages a 16 x 8 tile and its 2-node halo in LDS,
//     sweeps the marked nodes (packed into the lanes) until nothing changes or the inner
//     cap is reached, writes changed values back and marks the diamond neighbours of
//     changed nodes in the neighbouring tiles (unfinished nodes mark their own tile).
// Ordering: relaxing from +inf everywhere lets values computed from incomplete upstream
// information race through the whole grid and be corrected over and over.  A per-field
// time band limits that: an update whose value exceeds the field's threshold theta is
// stored as +inf and its value remembered per tile (min_rejected).  theta advances by a
// fixed step each pass (and jumps to the smallest rejected value when nothing is active);
// a tile wakes up when theta passes its min_rejected.  This restricted operator has the
// unrestricted field, cut at theta, as its unique fixed point, so the end state (nothing
// active, nothing rejected) is the same discrete fixed point, reached with far fewer
// corrections (a Dijkstra-like ordering at tile granularity).
// Fields of one call (one per source) share the medium and are relaxed in the same launch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "ali_solve.hpp"

namespace ali {

// ---------------------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------------------
// per-node constants of media m0 .. m0 + gridDim.y - 1 (one medium per grid row, so a batch
// of many small media takes one launch)
struct PrepDev {
    int64_t node_off;
    int nx, nz;
    double h;
    int n_mats, mat_off;
};

// largest qP phase speed of one stiffness over the same 181 directions as max_phase_speed
__device__ __forceinline__ double node_vmax(const MatA& A) {
    double v2max = 0.0;
    for (int q = 0; q <= 180; ++q) {
        const double psi = q * (3.14159265358979323846 / 360.0);
        const double c = cos(2.0 * psi), sn = sin(2.0 * psi);
        const double lin = (A.a33 - A.a11) + (A.a11 + A.a33 - 2.0 * A.a55) * c;
        const double v2 = 0.25 * ((A.a11 + A.a33 + 2.0 * A.a55) + (A.a33 - A.a11) * c +
                                  sqrt(lin * lin + 4.0 * (A.a13 + A.a55) * (A.a13 + A.a55) * sn * sn));
        v2max = v2 > v2max ? v2 : v2max;
    }
    return sqrt(v2max);
}

template <typename mreal, typename treal, typename oreal>
// gt_all (velocity-table mode, else NULL): group-speed tables of the device materials; the
// node's table offset goes to geo slot 6 and the straight-ray times come from the table.
// nodeA_all (else NULL): the per-node stiffness in place of the table (same node order as
// the ids); each medium's largest phase speed goes to vmax_bits[medium] (positive doubles
// order as their bit patterns, so an integer maximum finds it).
__global__ void k_prep(const PrepDev* __restrict__ media, int m0, const MatDev<mreal>* __restrict__ mats_all,
                       const uint8_t* __restrict__ mat_id_all, const oreal* __restrict__ orient_all,
                       mreal* __restrict__ geo_all, treal* __restrict__ fbt_all, const double* __restrict__ gt_all,
                       const float* __restrict__ nodeA_all, unsigned long long* __restrict__ vmax_bits,
                       int* __restrict__ err) {
    const PrepDev md = media[m0 + blockIdx.y];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)md.nx * md.nz) return;
    const MatDev<mreal>* __restrict__ mats = mats_all + md.mat_off;
    const uint8_t* __restrict__ mat_id = mat_id_all + md.node_off;
    const oreal* __restrict__ orient = orient_all + md.node_off;
    mreal* __restrict__ geo = geo_all + GEO_N * md.node_off;
    treal* __restrict__ fbt = fbt_all + 4 * md.node_off;
    const double h = md.h;
    const double th = (double)orient[p];
    const int mid = mat_id[p];
    if (!isfinite(th)) { atomicOr(err, 1); return; }
    if (mid >= md.n_mats) { atomicOr(err, 2); return; }
    MatA m = mats[mid].A;
    mreal P = mats[mid].P, Q = mats[mid].Q, R = mats[mid].R, K4 = mats[mid].K4;
    if (nodeA_all) {
        // the same constants as the host table, from this node's stiffness
        const float* a = nodeA_all + 4 * (md.node_off + p);
        m = MatA{(double)a[0], (double)a[1], (double)a[2], (double)a[3]};
        if (!(isfinite(m.a11) && isfinite(m.a13) && isfinite(m.a33) && isfinite(m.a55) && m.a11 > 0.0 &&
              m.a33 > 0.0 && m.a55 > 0.0 && m.a11 * m.a33 > m.a13 * m.a13)) {
            atomicOr(err, 4);
            return;
        }
        const double ih2 = 1.0 / (h * h);
        P = (mreal)((m.a11 + m.a33 + 2.0 * m.a55) * ih2);
        Q = (mreal)((m.a33 - m.a11) * ih2);
        R = (mreal)((m.a11 + m.a33 - 2.0 * m.a55) * ih2);
        const double W = (m.a13 + m.a55) * ih2;
        K4 = (mreal)(4.0 * W * W);
        atomicMax(&vmax_bits[m0 + blockIdx.y], (unsigned long long)__double_as_longlong(node_vmax(m)));
    }
    double s2, c2;
    sincos(2.0 * th, &s2, &c2);
    mreal* g = geo + GEO_N * p;
    g[0] = (mreal)c2;
    g[1] = (mreal)s2;
    g[2] = P;
    g[3] = Q;
    g[4] = R;
    g[5] = K4;
    g[6] = gt_all ? (mreal)((md.mat_off + mid) * VT_N) : mreal(0);
    g[7] = mreal(0);
    // straight-ray time to an 8-neighbour along x, (1,1), z, (1,-1)
    const double quarter = 0.78539816339744830962;
    const double len[4] = {1.0, 1.41421356237309504880, 1.0, 1.41421356237309504880};
    const double ang[4] = {0.0, quarter, 2.0 * quarter, -quarter};
#pragma unroll
    for (int d = 0; d < 4; ++d)
        fbt[4 * p + d] = (treal)(len[d] * h / (gt_all ? group_speed_tab(gt_all + (md.mat_off + mid) * VT_N, ang[d] - th)
                                                      : group_speed(m, ang[d] - th)));
}

// initial values of the fields f0 .. f0 + gridDim.y - 1 (all in one medium)
template <typename real, typename mreal, typename oreal>
__global__ void k_init(const FieldDev* __restrict__ fields, int f0, double h, const MatDev<mreal>* __restrict__ mats,
                       const double* __restrict__ gt, int n_mats, const uint8_t* __restrict__ mat_id,
                       const oreal* __restrict__ orient, const float* __restrict__ nodeA, int R,
                       real* __restrict__ T, uint32_t* __restrict__ flags) {
    const FieldDev fd = fields[f0 + blockIdx.y];
    const int nx = fd.nx;
    const int64_t N = (int64_t)nx * fd.nz;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int i = (int)(p % nx), j = (int)(p / nx);
    const int2 s = fd.src;
    const int di = i - s.x, dj = j - s.y;
    real v = dinf<real>();
    if (abs(di) <= R && abs(dj) <= R) {
        // straight ray at the group speed of the source node's material (Section 4.4)
        const int64_t ps = (int64_t)s.y * nx + s.x;
        if (di == 0 && dj == 0) {
            v = real(0);
        } else {
            const double phi = atan2((double)dj, (double)di) - (double)orient[ps];
            // an id outside the table is reported by k_prep; read a valid entry meanwhile
            const int mid = mat_id[ps] < n_mats ? mat_id[ps] : 0;
            const MatA A = nodeA ? MatA{(double)nodeA[4 * ps], (double)nodeA[4 * ps + 1], (double)nodeA[4 * ps + 2],
                                        (double)nodeA[4 * ps + 3]}
                                 : mats[mid].A;
            const double V = gt ? group_speed_tab(gt + mid * VT_N, phi) : group_speed(A, phi);
            v = (real)(sqrt((double)(di * di + dj * dj)) * h / V);
        }
    }
    T[fd.t_off + p] = v;
    // tiles that see the box (box radius + diamond radius) start active
    if (abs(di) <= R + HALO && abs(dj) <= R + HALO)
        flags[fd.unit_off + (j / TZ) * fd.ntx + (i / TX)] = TF_SELF;   // evaluate the whole tile
}

// Seeded fields: every tile holding a fixed node, and its 8 neighbours, starts with a
// visit of all its nodes (a fixed node reaches 2 nodes out, tiles are wider than that).
__global__ void k_seed_flags(const FieldDev* __restrict__ fields, int n_fields, int64_t n_units,
                             const uint32_t* __restrict__ fixmask, uint32_t* __restrict__ flags) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_units) return;
    uint32_t any = 0u;
#pragma unroll
    for (int w = 0; w < NODE_WORDS; ++w) any |= fixmask[u * NODE_WORDS + w];
    if (!any) return;
    const FieldDev fd = fields[field_of_unit(fields, n_fields, (uint32_t)u)];
    const int t = (int)(u - fd.unit_off);
    const int tx = t % fd.ntx, tz = t / fd.ntx;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dx = -1; dx <= 1; ++dx) {
            const int x = tx + dx, z = tz + dz;
            if (x < 0 || z < 0 || x >= fd.ntx || z >= fd.ntz) continue;
            atomicOr(&flags[fd.unit_off + (uint32_t)(z * fd.ntx + x)], (uint32_t)TF_SELF);
        }
}

// Scheduler of one relaxation pass (ascending thresholds), one work-group per field.
template <typename real>
__global__ void __launch_bounds__(SCHED_T)
k_sched(const FieldDev* __restrict__ fields, int advance, uint32_t* __restrict__ flags, real* __restrict__ minrej,
        real* __restrict__ theta, const real* __restrict__ step, PassItem* __restrict__ list,
        uint32_t* __restrict__ cnt_cur, uint32_t* __restrict__ cnt_next) {
    schedule_field<false, real>(fields, advance, step, flags, minrej, theta, list, cnt_cur, cnt_next);
}


// min of non-negative values in LDS through their integer bit patterns
__device__ __forceinline__ void lds_min(float* p, float v) {
    atomicMin(reinterpret_cast<unsigned*>(p), __float_as_uint(v));
}
__device__ __forceinline__ void lds_min(double* p, double v) {
    atomicMin(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}


// One tile visit by one wave (64 lanes, NPL nodes per lane; tile + halo staged in LDS).
// The nodes to evaluate are tracked per node.  The first sweep takes every node (TF_SELF),
// the band front (unreached nodes with a reached neighbour: new arrivals and values an
// earlier band rejected) and the nodes a neighbouring tile marked; each later sweep takes
// the nodes marked by changes inside the tile.  A change of node X marks a diamond
// neighbour D in the tile only if min(old, new) <= tau_D: the update at D reads only
// neighbours that precede D's own value in key order, so a neighbour that stays behind D
// cannot change it.  Across tiles the marks are unconditional (the other tile may be
// working on an older copy of X) and go to the neighbouring tile's node mask for the next
// pass.  Each sweep packs the marked nodes into the first lanes.
// SEEDED: the fixed nodes are the set bits of fixmask (one bit per node of each tile unit,
// NODE_WORDS words per unit) instead of the source box of radius R.
// TAB: phase speeds from the per-material tables vtab (offset in geo slot 6).
template <typename real, typename mreal, bool SEEDED, bool TAB>
__global__ void __launch_bounds__(RW) __attribute__((amdgpu_waves_per_eu(4)))
k_relax(const PassItem* __restrict__ list, const mreal* __restrict__ geo_all, const real* __restrict__ fbt_all,
        int R, int inner, const real* __restrict__ theta,
        real* __restrict__ T, uint32_t* __restrict__ flags, real* __restrict__ minrej,
        uint32_t* __restrict__ marks_in, uint32_t* __restrict__ marks_out,
        const uint32_t* __restrict__ count, uint32_t* __restrict__ idle,
        unsigned long long* __restrict__ counters, const uint32_t* __restrict__ fixmask,
        const mreal* __restrict__ vtab) {
    __shared__ real lt[LH * LSTRIDE];
    __shared__ uint8_t dnext[NTHREADS];
    __shared__ uint16_t clist[NTHREADS];
    __shared__ uint32_t omask[9][NODE_WORDS];     // marks for the 3x3 tile neighbourhood
    __shared__ uint32_t touched[NODE_WORDS];      // nodes whose value changed in this visit

    // the first entry is read together with the list length (the grid never exceeds the
    // list's capacity, so the read is in bounds; the entry is used only if it is live)
    PassItem pi = list[blockIdx.x];
    const uint32_t n_units = *count;
    if (n_units == 0u) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *idle = 1u;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        atomicAdd(&counters[2], 1ull);                  // passes with work
        atomicAdd(&counters[3], (unsigned long long)n_units);   // tile visits
    }
    // the work-groups walk the pass list with a grid stride
    for (uint32_t item = blockIdx.x; item < n_units; item += gridDim.x) {
    if (item != blockIdx.x) pi = list[item];
    const uint32_t unit = pi.unit;
    const uint32_t bits = pi.bits;
    const int f = pi.f;
    const int nx = pi.nx, nz = pi.nz, tx = pi.tx, tz = pi.tz;
    const int ntx = (nx + TX - 1) / TX;
    const int i0 = tx * TX, j0 = tz * TZ;
    real* __restrict__ Tf = T + pi.t_off;
    const mreal* __restrict__ geo = geo_all + GEO_N * pi.node_off;
    const real* __restrict__ fbt = fbt_all + 4 * pi.node_off;
    const real inf = dinf<real>();
    // the lane index is made opaque inside the item loop: otherwise the per-lane staging
    // offsets are hoisted out of the loop and held in registers through the sweeps
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));

    // stage the tile and its halo: every load is issued before the first store to LDS
    constexpr int SQ = (LW * LH + RW - 1) / RW;
    real sv[SQ];
#pragma unroll
    for (int k = 0; k < SQ; ++k) {
        const int q = lane + RW * k;
        const int li = q % LW, lj = q / LW;
        const int gi = i0 - HALO + li, gj = j0 - HALO + lj;
        sv[k] = (q < LW * LH && gi >= 0 && gj >= 0 && gi < nx && gj < nz) ? Tf[(int64_t)gj * nx + gi] : inf;
    }
    // incoming marks of this tile (read and cleared; this pass writes the other buffer)
    uint32_t mk = 0u, fm = 0u;
    if (lane < NODE_WORDS) {
        mk = marks_in[(int64_t)unit * NODE_WORDS + lane];
        if (mk) marks_in[(int64_t)unit * NODE_WORDS + lane] = 0u;
        if constexpr (SEEDED) fm = fixmask[(int64_t)unit * NODE_WORDS + lane];
    }
    const real th = theta[f];
#pragma unroll
    for (int k = 0; k < SQ; ++k) {
        const int q = lane + RW * k;
        if (q < LW * LH) lt[(q / LW) * LSTRIDE + q % LW] = sv[k];
    }
    for (int q = lane; q < 9 * NODE_WORDS; q += RW) omask[q / NODE_WORDS][q % NODE_WORDS] = 0u;
    for (int q = lane; q < NTHREADS; q += RW) dnext[q] = 0;
    if (lane < NODE_WORDS) touched[lane] = 0u;
    const int2 s = pi.src;
    __syncthreads();

    // the NPL nodes of this lane: node = lane + 64 q.
    // Loops over them stay rolled, and nothing per node is kept in registers across the
    // phases (the write-back finds changed nodes in the LDS change mask).
    unsigned dmask = 0u;              // bit q: node q of this lane is marked for this sweep
    unsigned amask = 0u;              // bit q: node q of this lane is evaluated at all
#pragma unroll 1
    for (int q = 0; q < NPL; ++q) {
        const int node = lane + RW * q;
        const int lx = node % TX, lz = node / TX;
        const int gi = i0 + lx, gj = j0 + lz;
        const int me = (lz + HALO) * LSTRIDE + (lx + HALO);
        bool fixed_node;
        if constexpr (SEEDED) fixed_node = (__shfl(fm, (node >> 5)) >> (node & 31)) & 1u;
        else fixed_node = abs(gi - s.x) <= R && abs(gj - s.y) <= R;
        const bool act = gi < nx && gj < nz && !fixed_node;
        amask |= act ? 1u << q : 0u;
        const real cur = lt[me];
        bool any = false;
#pragma unroll
        for (int k = 0; k < 12; ++k) any |= lt[me + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k]] < inf;
        const bool marked = (__shfl(mk, (node >> 5)) >> (node & 31)) & 1u;
        // a finite node with no finite neighbour left is evaluated too (it must turn +inf)
        if (act && (any || cur < inf) && ((bits & TF_SELF) || !(cur < inf) || marked)) dmask |= 1u << q;
    }

    real rej = inf;                   // smallest value this lane's updates rejected
    unsigned my_updates = 0, my_evals = 0;
    bool done = false;
    for (int it = 0;; ++it) {
        // pack the marked nodes
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
            bool chg = false;
            real lo = real(0);
            int node = 0;
            if (c + lane < total) {
                node = clist[c + lane];
                const int nlx = node % TX, nlz = node / TX;
                const int nme = (nlz + HALO) * LSTRIDE + (nlx + HALO);
                const int64_t p = (int64_t)(j0 + nlz) * nx + (i0 + nlx);
                using NC = typename std::conditional<TAB, NodeConstTab<mreal, real>, NodeConst<mreal, real>>::type;
                NC nc;
                load_node_const<real, mreal>(nc, p, geo, fbt);
                if constexpr (TAB) nc.vt = vtab + (int)geo[GEO_N * p + 6];
                real t[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) t[k] = lt[nme + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k]];
                ++my_updates;
                real u = local_update<mreal, real>(nc, t, lt, nme, LSTRIDE, my_evals);
                if (u > th && u < inf) { rej = u < rej ? u : rej; u = inf; }
                const real cv = lt[nme];
                if (!(u == cv || (u >= inf && cv >= inf))) {
                    lt[nme] = u;
                    chg = true;
                    lo = u < cv ? u : cv;
                    atomicOr(&touched[node >> 5], 1u << (node & 31));
                }
            }
            // every value of the chunk is stored before any neighbour is compared (the
            // comparisons must see the neighbours' new values)
            __syncthreads();
            if (chg) {
                const int nlx = node % TX, nlz = node / TX;
                const int nme = (nlz + HALO) * LSTRIDE + (nlx + HALO);
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    const int ax = nlx + SLOT_DI[k], az = nlz + SLOT_DJ[k];
                    if (ax >= 0 && az >= 0 && ax < TX && az < TZ &&
                        lo <= lt[nme + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k]])
                        dnext[az * TX + ax] = 1;
                }
            }
            __syncthreads();
        }
        // collect the marks for the next sweep
#pragma unroll
        for (int q = 0; q < NPL; ++q) {
            const int node = lane + RW * q;
            if (dnext[node]) {
                dnext[node] = 0;
                dmask |= amask & (1u << q);
            }
        }
        __syncthreads();
    }

    // write back; mark the diamond neighbours of changed nodes in the neighbouring tiles
    // (and, after the sweep cap, this tile's own unfinished nodes)
    bool any_out = false;
    if (!done) {
#pragma unroll 1
        for (int q = 0; q < NPL; ++q)
            if ((dmask >> q) & 1u) {
                const int node = lane + RW * q;
                atomicOr(&omask[4][node >> 5], 1u << (node & 31));
                any_out = true;
            }
    }
#pragma unroll 1
    for (int q = 0; q < NPL; ++q) {
        const int node = lane + RW * q;
        const int lx = node % TX, lz = node / TX;
        const int gi = i0 + lx, gj = j0 + lz;
        if (gi >= nx || gj >= nz) continue;
        // a node whose value changed (possibly back to where it started) is written back
        if (!((touched[node >> 5] >> (node & 31)) & 1u)) continue;
        Tf[(int64_t)gj * nx + gi] = lt[(lz + HALO) * LSTRIDE + (lx + HALO)];
        if (lx >= HALO && lx < TX - HALO && lz >= HALO && lz < TZ - HALO) continue;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const int ax = lx + SLOT_DI[k], az = lz + SLOT_DJ[k];
            if (ax >= 0 && az >= 0 && ax < TX && az < TZ) continue;
            const int ngi = gi + SLOT_DI[k], ngj = gj + SLOT_DJ[k];
            if (ngi < 0 || ngj < 0 || ngi >= nx || ngj >= nz) continue;
            const int ox = ax < 0 ? 0 : (ax < TX ? 1 : 2), oz = az < 0 ? 0 : (az < TZ ? 1 : 2);
            const int nn = (az - (oz - 1) * TZ) * TX + (ax - (ox - 1) * TX);
            atomicOr(&omask[oz * 3 + ox][nn >> 5], 1u << (nn & 31));
            any_out = true;
        }
    }
    // wave-wide reductions
    for (int o = 32; o > 0; o >>= 1) {
        const real r2 = __shfl_xor(rej, o);
        rej = r2 < rej ? r2 : rej;
        my_updates += __shfl_xor(my_updates, o);
        my_evals += __shfl_xor(my_evals, o);
    }
    const bool out = __ballot(any_out) != 0ull;
    __syncthreads();
    if (out) {
        // one lane per (neighbour tile, word): push the node marks and flag the tile
        for (int q = lane; q < 9 * NODE_WORDS; q += RW) {
            const uint32_t w = omask[q / NODE_WORDS][q % NODE_WORDS];
            if (!w) continue;
            const int o = q / NODE_WORDS;
            const int ntx2 = tx + o % 3 - 1, ntz2 = tz + o / 3 - 1;
            const int64_t u2 = (int64_t)unit + (int64_t)(ntz2 - tz) * ntx + (ntx2 - tx);
            atomicOr(&marks_out[u2 * NODE_WORDS + q % NODE_WORDS], w);
            atomicOr(&flags[u2], TF_MARK);
        }
    }
    if (lane == 0) {
        // statistics spread over STAT_SLOTS counter pairs (one address for all visits
        // would serialise every tile visit of a pass)
        if (my_updates) {
            unsigned long long* sc = counters + 4 + 2 * (blockIdx.x % STAT_SLOTS);
            atomicAdd(&sc[0], (unsigned long long)my_updates);
            atomicAdd(&sc[1], (unsigned long long)my_evals);
        }
        minrej[unit] = rej;
    }
    __syncthreads();     // LDS is reused by the next item
    }
}

// ---------------------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------------------
ali_status validate_batch(ali_handle* H, const ali_medium* media, int32_t n_media, const ali_material* mats,
                          int32_t n_mats, const void* d_mat_id, const void* d_orient, const ali_node* srcs,
                          const ali_node* recv, int wave) {
    if (!media || n_media < 1) return H->fail(ALI_EINVAL, "need at least one medium");
    if (!mats || n_mats < 1) return H->fail(ALI_EINVAL, "need at least one material");
    for (int k = 0; k < n_mats; ++k) {
        const ali_status st = check_material(H, mats[k], k, wave);
        if (st != ALI_OK) return st;
    }
    if (!d_mat_id || !d_orient) return H->fail(ALI_EINVAL, "medium arrays are NULL");
    if (!srcs) return H->fail(ALI_EINVAL, "sources are NULL");
    int64_t units = 0;
    for (int m = 0; m < n_media; ++m) {
        const ali_medium& md = media[m];
        const std::string tag = "medium " + std::to_string(m) + ": ";
        const ali_grid& g = md.grid;
        if (g.nx < 3 || g.nz < 3) return H->fail(ALI_EINVAL, tag + "grid needs nx, nz >= 3");
        if ((int64_t)g.nx * g.nz > (int64_t)1 << 31) return H->fail(ALI_EINVAL, tag + "grid too large");
        if (!(g.h > 0.0) || !isfinite(g.h)) return H->fail(ALI_EINVAL, tag + "grid spacing h must be finite and > 0");
        if (md.n_mats < 1 || md.n_mats > 256 || md.mat_offset < 0 || md.mat_offset + md.n_mats > n_mats)
            return H->fail(ALI_EINVAL, tag + "materials outside the table (1..256 per medium)");
        if (md.node_offset < 0) return H->fail(ALI_EINVAL, tag + "negative node offset");
        if (md.n_src < 1 || md.src_offset < 0) return H->fail(ALI_EINVAL, tag + "need at least one source");
        for (int k = 0; k < md.n_src; ++k) {
            const ali_node& sn = srcs[md.src_offset + k];
            if (sn.i < 0 || sn.j < 0 || sn.i >= g.nx || sn.j >= g.nz)
                return H->fail(ALI_EINVAL, tag + "source " + std::to_string(k) + " outside the grid");
        }
        if (recv) {
            if (md.n_rec < 1 || md.rec_offset < 0) return H->fail(ALI_EINVAL, tag + "need at least one receiver");
            for (int k = 0; k < md.n_rec; ++k) {
                const ali_node& r = recv[md.rec_offset + k];
                if (r.i < 0 || r.j < 0 || r.i >= g.nx || r.j >= g.nz)
                    return H->fail(ALI_EINVAL, tag + "receiver " + std::to_string(k) + " outside the grid");
            }
        }
        units += (int64_t)((g.nx + TX - 1) / TX) * ((g.nz + TZ - 1) / TZ) * md.n_src;
    }
    if (units >= (int64_t)INT32_MAX) return H->fail(ALI_EINVAL, "too many tiles in one call");
    return ALI_OK;
}

// real: travel-time type (storage, scores, decisions); mreal: wavefront / phase-speed
// math; oreal: orientation input.
template <typename real, typename mreal, typename oreal>
ali_status solve_fields(ali_handle* H, const ali_medium* media, int32_t n_media, const ali_material* mats,
                        int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient, const ali_node* srcs,
                        const ali_node* recv, const ali_options& opt, real* d_T, ali_solve_stats* stats,
                        ForwardState<real, mreal>* fs, const uint32_t* d_fixmask) {
    ali_status st = validate_batch(H, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, recv, opt.wave);
    if (st != ALI_OK) return st;
    // the records the kernels use (for SH, the in-plane record with the SH speeds)
    const std::vector<ali_material> wmats = wave_materials(mats, n_mats, opt.wave);
    mats = wmats.data();
    if (!d_T) return H->fail(ALI_EINVAL, "d_T is NULL");
    if (opt.src_box_radius < 0 || opt.src_box_radius > 64) return H->fail(ALI_EINVAL, "src_box_radius out of range [0, 64]");
    if (opt.max_sweeps < 1) return H->fail(ALI_EINVAL, "max_sweeps must be >= 1");
    if (opt.inner_sweeps < 1 || opt.inner_sweeps > 4096) return H->fail(ALI_EINVAL, "inner_sweeps out of range [1, 4096]");
    if (opt.band_cells < 0) return H->fail(ALI_EINVAL, "band_cells must be >= 0 (0 = no band)");
    if (opt.velocity != ALI_VEL_CHRISTOFFEL && opt.velocity != ALI_VEL_TABLE)
        return H->fail(ALI_EINVAL, "unknown velocity mode");
    if (opt.d_node_A && (opt.wave != ALI_WAVE_QP || opt.velocity != ALI_VEL_CHRISTOFFEL))
        return H->fail(ALI_EUNSUPPORTED, "per-node stiffness needs the qP wave and the run-time speeds");
    if (set_device(H) != ALI_OK) return ALI_EDEVICE;
    hipStream_t S = H->stream;

    // field table, per-medium material constants (they carry 1/h^2) and band steps
    ForwardState<real, mreal> local;
    ForwardState<real, mreal>& F = fs ? *fs : local;
    F.hfields.clear();
    F.medium_first_field.clear();
    F.vmax.clear();
    std::vector<MatDev<mreal>> hm;
    std::vector<int> dev_mat_off(n_media);
    std::vector<real> hstep, htheta;
    int64_t units = 0, fnodes = 0, med_nodes = 0;
    int obs = 0;
    for (int m = 0; m < n_media; ++m) {
        const ali_medium& md = media[m];
        dev_mat_off[m] = (int)hm.size();
        const std::vector<MatDev<mreal>> mm = make_matdev<mreal>(mats + md.mat_offset, md.n_mats, md.grid.h);
        hm.insert(hm.end(), mm.begin(), mm.end());
        const double vmax = max_phase_speed(mats + md.mat_offset, md.n_mats);
        F.vmax.push_back(vmax);
        const real band = opt.band_cells > 0 ? (real)(opt.band_cells * md.grid.h / vmax) : dinf_host<real>();
        F.medium_first_field.push_back((int)F.hfields.size());
        const int nx = md.grid.nx, nz = md.grid.nz;
        const int ntx = (nx + TX - 1) / TX, ntz = (nz + TZ - 1) / TZ;
        med_nodes = std::max(med_nodes, md.node_offset + (int64_t)nx * nz);
        for (int k = 0; k < md.n_src; ++k) {
            FieldDev fd;
            fd.nx = nx; fd.nz = nz; fd.ntx = ntx; fd.ntz = ntz;
            fd.h = md.grid.h;
            fd.node_off = md.node_offset;
            fd.t_off = fnodes;
            fd.unit_off = (uint32_t)units;
            fd.mat_off = dev_mat_off[m];
            fd.medium = m;
            fd.rec_off = md.rec_offset;
            fd.n_rec = recv ? md.n_rec : 0;
            fd.obs_off = obs;
            fd.src = make_int2(srcs[md.src_offset + k].i, srcs[md.src_offset + k].j);
            F.hfields.push_back(fd);
            units += (int64_t)ntx * ntz;
            fnodes += (int64_t)nx * nz;
            obs += fd.n_rec;
            hstep.push_back(band);
            htheta.push_back(band);
        }
    }
    F.medium_first_field.push_back((int)F.hfields.size());
    const int n_fields = (int)F.hfields.size();
    const int64_t nunits = units;
    F.n_units = nunits;
    F.field_nodes = fnodes;

    void *d_mats, *d_geo, *d_fbt, *d_fields, *d_flags, *d_list, *d_count, *d_upd, *d_err;
    void *d_theta, *d_step, *d_minrej, *d_marks, *d_idle;
    if (!H->scratch("mats", sizeof(MatDev<mreal>) * hm.size(), &d_mats) ||
        !H->scratch("fields", sizeof(FieldDev) * n_fields, &d_fields) ||
        !H->scratch("theta", sizeof(real) * n_fields, &d_theta) ||
        !H->scratch("step", sizeof(real) * n_fields, &d_step) ||
        !H->scratch("minrej", sizeof(real) * nunits, &d_minrej) ||
        !H->scratch("geo", sizeof(mreal) * GEO_N * med_nodes, &d_geo) ||
        !H->scratch("fbt", sizeof(real) * 4 * med_nodes, &d_fbt) ||
        !H->scratch("flags", sizeof(uint32_t) * nunits, &d_flags) ||
        !H->scratch("list", sizeof(PassItem) * nunits, &d_list) ||
        !H->scratch("marks", sizeof(uint32_t) * 2 * NODE_WORDS * nunits, &d_marks) ||
        !H->scratch("count", 2 * sizeof(uint32_t), &d_count) ||
        !H->scratch("idle", sizeof(uint32_t), &d_idle) ||
        !H->scratch("upd", (4 + 2 * STAT_SLOTS) * sizeof(unsigned long long), &d_upd) ||
        !H->scratch("err", sizeof(int), &d_err))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    F.mats = (const MatDev<mreal>*)d_mats;
    F.geo = (const mreal*)d_geo;
    F.fbt = (const real*)d_fbt;
    F.fields = (const FieldDev*)d_fields;

    HIPCK(H, hipEventRecord(H->ev0, S));
    HIPCK(H, hipMemcpyAsync(d_mats, hm.data(), sizeof(MatDev<mreal>) * hm.size(), hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemcpyAsync(d_fields, F.hfields.data(), sizeof(FieldDev) * n_fields, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemsetAsync(d_flags, 0, sizeof(uint32_t) * nunits, S));
    HIPCK(H, hipMemsetAsync(d_marks, 0, sizeof(uint32_t) * 2 * NODE_WORDS * nunits, S));
    HIPCK(H, hipMemsetAsync(d_upd, 0, (4 + 2 * STAT_SLOTS) * sizeof(unsigned long long), S));
    HIPCK(H, hipMemsetAsync(d_count, 0, 2 * sizeof(uint32_t), S));
    HIPCK(H, hipMemsetAsync(d_idle, 0, sizeof(uint32_t), S));
    HIPCK(H, hipMemsetAsync(d_err, 0, sizeof(int), S));

    const int B = 256;
    hipLaunchKernelGGL((k_fill<real>), dim3((unsigned)((nunits + B - 1) / B)), dim3(B), 0, S,
                       (real*)d_minrej, nunits, dinf_host<real>());
    // velocity-table mode: per device material, phase speed / h and group speed at whole
    // degrees (built on the device from the run-time speeds)
    const bool tab = opt.velocity == ALI_VEL_TABLE;
    void *d_vt = nullptr, *d_gt = nullptr;
    std::vector<MatA> hA;
    std::vector<double> hih;
    if (tab) {
        for (int m = 0; m < n_media; ++m)
            for (int k = 0; k < media[m].n_mats; ++k) {
                hA.push_back(hm[dev_mat_off[m] + k].A);
                hih.push_back(1.0 / media[m].grid.h);
            }
        void *d_A = nullptr, *d_ih = nullptr;
        const size_t nd = hA.size();
        if (!H->scratch("vt_A", sizeof(MatA) * nd, &d_A) || !H->scratch("vt_ih", sizeof(double) * nd, &d_ih) ||
            !H->scratch("vt", sizeof(mreal) * VT_N * nd, &d_vt) || !H->scratch("gt", sizeof(double) * VT_N * nd, &d_gt))
            return H->fail(ALI_ENOMEM, "device scratch allocation failed");
        HIPCK(H, hipMemcpyAsync(d_A, hA.data(), sizeof(MatA) * nd, hipMemcpyHostToDevice, S));
        HIPCK(H, hipMemcpyAsync(d_ih, hih.data(), sizeof(double) * nd, hipMemcpyHostToDevice, S));
        hipLaunchKernelGGL((k_vtables<mreal>), dim3((unsigned)nd), dim3(128), 0, S, (const MatA*)d_A,
                           (const double*)d_ih, (int)nd, (mreal*)d_vt, (double*)d_gt);
    }
    // per-node constants of every medium: one launch per 65535 media
    std::vector<PrepDev> hp(n_media);
    int64_t max_nodes = 0;
    for (int m = 0; m < n_media; ++m) {
        const ali_medium& md = media[m];
        hp[m] = PrepDev{md.node_offset, md.grid.nx, md.grid.nz, md.grid.h, md.n_mats, dev_mat_off[m]};
        max_nodes = std::max(max_nodes, (int64_t)md.grid.nx * md.grid.nz);
    }
    void *d_prep = nullptr, *d_vmaxb = nullptr;
    if (!H->scratch("prep", sizeof(PrepDev) * n_media, &d_prep) ||
        !H->scratch("vmaxb", sizeof(unsigned long long) * n_media, &d_vmaxb))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    HIPCK(H, hipMemcpyAsync(d_prep, hp.data(), sizeof(PrepDev) * n_media, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemsetAsync(d_vmaxb, 0, sizeof(unsigned long long) * n_media, S));
    for (int m0 = 0; m0 < n_media; m0 += 65535) {
        const int nm = std::min(n_media - m0, 65535);
        hipLaunchKernelGGL((k_prep<mreal, real, oreal>), dim3((unsigned)((max_nodes + B - 1) / B), (unsigned)nm),
                           dim3(B), 0, S, (const PrepDev*)d_prep, m0, (const MatDev<mreal>*)d_mats, d_mat_id,
                           d_orient, (mreal*)d_geo, (real*)d_fbt, (const double*)d_gt, opt.d_node_A,
                           (unsigned long long*)d_vmaxb, (int*)d_err);
    }
    for (int m = 0; m < n_media; ++m) {
        const ali_medium& md = media[m];
        const int64_t N = (int64_t)md.grid.nx * md.grid.nz;
        if (!d_fixmask)
            hipLaunchKernelGGL((k_init<real, mreal, oreal>), dim3((unsigned)((N + B - 1) / B), (unsigned)md.n_src),
                               dim3(B), 0, S, (const FieldDev*)d_fields, F.medium_first_field[m], md.grid.h,
                               (const MatDev<mreal>*)d_mats + dev_mat_off[m],
                               tab ? (const double*)d_gt + (size_t)VT_N * dev_mat_off[m] : (const double*)nullptr,
                               md.n_mats, d_mat_id + md.node_offset, d_orient + md.node_offset,
                               opt.d_node_A ? opt.d_node_A + 4 * md.node_offset : (const float*)nullptr,
                               opt.src_box_radius, d_T, (uint32_t*)d_flags);
    }
    if (d_fixmask)
        hipLaunchKernelGGL(k_seed_flags, dim3((unsigned)((nunits + B - 1) / B)), dim3(B), 0, S,
                           (const FieldDev*)d_fields, n_fields, nunits, d_fixmask, (uint32_t*)d_flags);
    HIPCK(H, hipGetLastError());

    int h_err = 0;
    std::vector<unsigned long long> hvb(opt.d_node_A ? n_media : 0);
    HIPCK(H, hipMemcpyAsync(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost, S));
    if (opt.d_node_A)
        HIPCK(H, hipMemcpyAsync(hvb.data(), d_vmaxb, sizeof(unsigned long long) * n_media, hipMemcpyDeviceToHost, S));
    HIPCK(H, hipStreamSynchronize(S));
    if (h_err & 1) return H->fail(ALI_EINVAL, "orientation contains NaN or Inf");
    if (h_err & 2) return H->fail(ALI_EINVAL, "material id out of range");
    if (h_err & 4) return H->fail(ALI_EINVAL, "per-node stiffness: a node is not finite and positive definite");
    if (opt.d_node_A) {
        // the band steps from the nodes' own largest phase speed
        for (int m = 0; m < n_media; ++m) {
            double v;
            memcpy(&v, &hvb[m], sizeof(double));
            F.vmax[m] = v;
            const real band = opt.band_cells > 0 ? (real)(opt.band_cells * media[m].grid.h / v) : dinf_host<real>();
            for (int f = F.medium_first_field[m]; f < F.medium_first_field[m + 1]; ++f) {
                hstep[f] = band;
                htheta[f] = band;
            }
        }
    }
    HIPCK(H, hipMemcpyAsync(d_theta, htheta.data(), sizeof(real) * n_fields, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemcpyAsync(d_step, hstep.data(), sizeof(real) * n_fields, hipMemcpyHostToDevice, S));

    // passes are queued in batches without host round trips; each batch ends with one
    // read of the idle flag (set by a relax launch that found an empty pass list: from
    // then on nothing changes)
    int iters = 0;
    bool converged = false;
    double relax_ms = 0.0;
    // a fixed grid (the pass size is known only on the device); work-groups beyond the
    // pass list exit at once
    const int grid_relax = (int)(nunits < (int64_t)32 * H->n_cu ? nunits : (int64_t)32 * H->n_cu);
    uint32_t* cnt = (uint32_t*)d_count;
    // one pass: schedule, then relax (events around the relax launch when timed)
    auto enqueue = [&](int p, bool timed, hipStream_t S) {
        hipLaunchKernelGGL((k_sched<real>), dim3((unsigned)n_fields), dim3(SCHED_T), 0, S,
                           (const FieldDev*)d_fields, p > 0 ? 1 : 0,
                           (uint32_t*)d_flags, (real*)d_minrej, (real*)d_theta, (const real*)d_step,
                           (PassItem*)d_list, cnt + (p & 1), cnt + ((p + 1) & 1));
        uint32_t* mk_in = (uint32_t*)d_marks + (size_t)(p & 1) * nunits * NODE_WORDS;
        uint32_t* mk_out = (uint32_t*)d_marks + (size_t)((p + 1) & 1) * nunits * NODE_WORDS;
        if (timed) (void)hipEventRecord(H->pev[2 * (p % PASS_BATCH)], S);
        const int R = d_fixmask ? -1 : opt.src_box_radius;
        const mreal* vt = (const mreal*)d_vt;
        if (d_fixmask && tab)
            hipLaunchKernelGGL((k_relax<real, mreal, true, true>), dim3((unsigned)grid_relax), dim3(RW), 0, S,
                               (const PassItem*)d_list, (const mreal*)d_geo, (const real*)d_fbt, R,
                               opt.inner_sweeps, (const real*)d_theta, d_T, (uint32_t*)d_flags, (real*)d_minrej,
                               mk_in, mk_out, (const uint32_t*)(cnt + (p & 1)), (uint32_t*)d_idle,
                               (unsigned long long*)d_upd, d_fixmask, vt);
        else if (d_fixmask)
            hipLaunchKernelGGL((k_relax<real, mreal, true, false>), dim3((unsigned)grid_relax), dim3(RW), 0, S,
                               (const PassItem*)d_list, (const mreal*)d_geo, (const real*)d_fbt, R,
                               opt.inner_sweeps, (const real*)d_theta, d_T, (uint32_t*)d_flags, (real*)d_minrej,
                               mk_in, mk_out, (const uint32_t*)(cnt + (p & 1)), (uint32_t*)d_idle,
                               (unsigned long long*)d_upd, d_fixmask, vt);
        else if (tab)
            hipLaunchKernelGGL((k_relax<real, mreal, false, true>), dim3((unsigned)grid_relax), dim3(RW), 0, S,
                               (const PassItem*)d_list, (const mreal*)d_geo, (const real*)d_fbt, R,
                               opt.inner_sweeps, (const real*)d_theta, d_T, (uint32_t*)d_flags, (real*)d_minrej,
                               mk_in, mk_out, (const uint32_t*)(cnt + (p & 1)), (uint32_t*)d_idle,
                               (unsigned long long*)d_upd, d_fixmask, vt);
        else
            hipLaunchKernelGGL((k_relax<real, mreal, false, false>), dim3((unsigned)grid_relax), dim3(RW), 0, S,
                               (const PassItem*)d_list, (const mreal*)d_geo, (const real*)d_fbt, R, opt.inner_sweeps, (const real*)d_theta, d_T,
                               (uint32_t*)d_flags, (real*)d_minrej, mk_in, mk_out, (const uint32_t*)(cnt + (p & 1)),
                               (uint32_t*)d_idle, (unsigned long long*)d_upd, d_fixmask, vt);
        if (timed) (void)hipEventRecord(H->pev[2 * (p % PASS_BATCH) + 1], S);
    };
    while (iters < opt.max_sweeps) {
        const int batch = opt.max_sweeps - iters < PASS_BATCH ? opt.max_sweeps - iters : PASS_BATCH;
        const bool graph = opt.graph && batch == PASS_BATCH;
        if (graph) {
            // the first batch differs from the others only in the first pass (no advance)
            const int first = iters == 0 ? 1 : 0;
            const void* kern = d_fixmask ? (tab ? (const void*)&k_relax<real, mreal, true, true>
                                                : (const void*)&k_relax<real, mreal, true, false>)
                                         : (tab ? (const void*)&k_relax<real, mreal, false, true>
                                                : (const void*)&k_relax<real, mreal, false, false>);
            const std::string key = graph_key("relax", first, kern, d_fields, n_fields,
                                              d_flags, d_minrej, d_theta, d_step, d_list, d_count,
                                              d_marks, nunits, d_geo, d_fbt, opt.src_box_radius,
                                              opt.inner_sweeps, d_T, d_idle, d_upd, grid_relax,
                                              (const void*)d_fixmask, d_vt);
            HIPCK(H, hipEventRecord(H->ev2, S));
            st = launch_captured(H, key, [&](int b, hipStream_t cs) { enqueue(first ? b : PASS_BATCH + b, false, cs); });
            if (st != ALI_OK) return st;
            HIPCK(H, hipEventRecord(H->ev3, S));
        } else {
            for (int b = 0; b < batch; ++b) enqueue(iters + b, true, S);
        }
        HIPCK(H, hipGetLastError());
        HIPCK(H, hipMemcpyAsync(H->host_count, d_idle, sizeof(uint32_t), hipMemcpyDeviceToHost, S));
        HIPCK(H, hipStreamSynchronize(S));
        if (graph) {
            float kms = 0.f;
            HIPCK(H, hipEventElapsedTime(&kms, H->ev2, H->ev3));
            relax_ms += kms;
        } else {
            for (int b = 0; b < batch; ++b) {
                float kms = 0.f;
                HIPCK(H, hipEventElapsedTime(&kms, H->pev[2 * ((iters + b) % PASS_BATCH)],
                                             H->pev[2 * ((iters + b) % PASS_BATCH) + 1]));
                relax_ms += kms;
            }
        }
        iters += batch;
        if (*H->host_count) { converged = true; break; }
    }
    std::vector<unsigned long long> cnt_h(4 + 2 * STAT_SLOTS);
    HIPCK(H, hipMemcpyAsync(cnt_h.data(), d_upd, sizeof(unsigned long long) * cnt_h.size(), hipMemcpyDeviceToHost, S));
    HIPCK(H, hipStreamSynchronize(S));
    unsigned long long upd[4] = {0, 0, cnt_h[2], cnt_h[3]};
    for (int k = 0; k < STAT_SLOTS; ++k) { upd[0] += cnt_h[4 + 2 * k]; upd[1] += cnt_h[5 + 2 * k]; }
    if (stats) {
        stats->node_updates = (int64_t)upd[0];
        stats->stencil_evals = (int64_t)upd[1];
        stats->relax_ms = relax_ms;
        stats->tile_visits = (int64_t)upd[3];
        stats->nodes = fnodes;
        stats->outer_iters = (int32_t)upd[2];
        stats->converged = converged ? 1 : 0;
        stats->ms = 0.0;
    }
    if (!converged) return H->fail(ALI_ENOCONV, "relaxation reached max_sweeps");
    return ALI_OK;
}

#define ALI_SOLVE_FIELDS(R, M, O)                                                                            \
    template ali_status solve_fields<R, M, O>(ali_handle*, const ali_medium*, int32_t, const ali_material*,  \
                                              int32_t, const uint8_t*, const O*, const ali_node*,            \
                                              const ali_node*, const ali_options&, R*, ali_solve_stats*,     \
                                              ForwardState<R, M>*, const uint32_t*);
ALI_SOLVE_FIELDS(double, float, float)
ALI_SOLVE_FIELDS(float, float, float)
ALI_SOLVE_FIELDS(double, double, float)
ALI_SOLVE_FIELDS(double, double, double)
#undef ALI_SOLVE_FIELDS

// Entry-point body: relax in `real` (on a scratch field when it differs from the output
// type), convert into d_out, time the whole call.
template <typename real, typename mreal, typename oreal, typename outreal>
static ali_status solve_impl(ali_handle* H, const ali_medium* media, int32_t n_media, const ali_material* mats,
                             int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient,
                             const ali_node* srcs, const ali_options* opt_in, outreal* d_out,
                             ali_solve_stats* stats) {
    ali_options opt;
    ali_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (!d_out) return H->fail(ALI_EINVAL, "d_T is NULL");
    ali_status st = validate_batch(H, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, nullptr, opt.wave);
    if (st != ALI_OK) return st;
    int64_t n_fields = 0, tot = 0;
    batch_sizes(media, n_media, &n_fields, &tot);
    constexpr bool same_out = std::is_same<real, outreal>::value;
    void* d_work = nullptr;
    if (!same_out && !H->scratch("Twork", sizeof(real) * tot, &d_work))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    real* d_T = same_out ? (real*)d_out : (real*)d_work;
    ali_solve_stats local{};
    st = solve_fields<real, mreal, oreal>(H, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, nullptr, opt,
                                          d_T, &local, nullptr);
    if (st != ALI_OK && st != ALI_ENOCONV) return st;
    hipStream_t S = H->stream;
    if (!same_out) {
        const int B = 256;
        hipLaunchKernelGGL((k_convert<outreal, real>), dim3((unsigned)((tot + B - 1) / B)), dim3(B), 0, S,
                           d_out, (const real*)d_T, tot);
        HIPCK(H, hipGetLastError());
    }
    HIPCK(H, hipEventRecord(H->ev1, S));
    HIPCK(H, hipStreamSynchronize(S));
    if (stats) {
        float ms = 0.f;
        HIPCK(H, hipEventElapsedTime(&ms, H->ev0, H->ev1));
        *stats = local;
        stats->ms = ms;
    }
    return st;
}

// ---------------------------------------------------------------------------------------
// allocation-free forward solve: every scratch buffer comes from one static device array
// ---------------------------------------------------------------------------------------
// Bytes the arena hands out for one single-medium forward solve: every scratch() request of
// solve_impl and solve_fields, in request order, each at a 256-byte aligned offset.
template <typename real, typename mreal>
static size_t forward_scratch_bytes(const ali_grid& g, int n_src, int n_mats, bool table) {
    const int64_t nodes = (int64_t)g.nx * g.nz;
    const int64_t units = (int64_t)((g.nx + TX - 1) / TX) * ((g.nz + TZ - 1) / TZ) * n_src;
    std::vector<size_t> req;
    if (!std::is_same<real, float>::value) req.push_back(sizeof(real) * nodes * n_src);   // Twork
    req.push_back(sizeof(MatDev<mreal>) * n_mats);                 // mats
    req.push_back(sizeof(FieldDev) * n_src);                       // fields
    req.push_back(sizeof(real) * n_src);                           // theta
    req.push_back(sizeof(real) * n_src);                           // step
    req.push_back(sizeof(real) * units);                           // minrej
    req.push_back(sizeof(mreal) * GEO_N * nodes);                  // geo
    req.push_back(sizeof(real) * 4 * nodes);                       // fbt
    req.push_back(sizeof(uint32_t) * units);                       // flags
    req.push_back(sizeof(PassItem) * units);                       // list
    req.push_back(sizeof(uint32_t) * 2 * NODE_WORDS * units);      // marks
    req.push_back(2 * sizeof(uint32_t));                           // count
    req.push_back(sizeof(uint32_t));                               // idle
    req.push_back((4 + 2 * STAT_SLOTS) * sizeof(unsigned long long));   // upd
    req.push_back(sizeof(int));                                    // err
    if (table) {
        req.push_back(sizeof(MatA) * n_mats);                      // vt_A
        req.push_back(sizeof(double) * n_mats);                    // vt_ih
        req.push_back(sizeof(mreal) * VT_N * n_mats);              // vt
        req.push_back(sizeof(double) * VT_N * n_mats);             // gt
    }
    req.push_back(sizeof(PrepDev));                                // prep
    req.push_back(sizeof(unsigned long long));                     // vmaxb
    size_t used = 0;
    for (size_t b : req) used = ((used + 255) & ~(size_t)255) + b;
    return used;
}

}  // namespace ali

// The static scratch array: file scope, one copy per device, held until the process ends.
// Host code never passes its name to a kernel or a copy (in host code the name stands for a
// host-side shadow, not a device address); it uses the address hipGetSymbolAddress returns
// on each device.
static __device__ __align__(256) unsigned char scratch[ALI_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_SCRATCH_DEVICES] = {};
}  // namespace

hipError_t ali::static_scratch_address(int device, void** ptr, size_t* bytes) {
    if (device < 0 || device >= MAX_SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    *bytes = ALI_NOALLOC_SCRATCH_BYTES;
    return hipSuccess;
}

using namespace ali;

template <typename oreal, typename outreal>
static ali_status solve_dispatch(ali_handle* h, const ali_medium* media, int32_t n_media, const ali_material* mats,
                                 int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient, const ali_node* srcs,
                                 const ali_options* opt, outreal* d_T, ali_solve_stats* stats) {
    const int arith = opt ? opt->arith : ALI_ARITH_MIXED;
    switch (arith) {
        case ALI_ARITH_MIXED:
            return solve_impl<double, float, oreal, outreal>(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, opt, d_T, stats);
        case ALI_ARITH_F32:
            return solve_impl<float, float, oreal, outreal>(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, opt, d_T, stats);
        case ALI_ARITH_F64:
            return solve_impl<double, double, oreal, outreal>(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, opt, d_T, stats);
    }
    return h->fail(ALI_EINVAL, "unknown arith mode");
}

extern "C" ali_status ali_solve_traveltime(ali_handle* h, const ali_grid* grid,
                                           const ali_material* mats, int32_t n_mats,
                                           const uint8_t* d_mat_id, const float* d_orient,
                                           const ali_node* srcs, int32_t n_src,
                                           const ali_options* opt, float* d_T,
                                           ali_solve_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    const ali_medium md = single_medium(grid, n_mats, n_src, 0);
    return solve_dispatch<float, float>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, opt, d_T, stats);
}

extern "C" ali_status ali_solve_traveltime_f64(ali_handle* h, const ali_grid* grid,
                                               const ali_material* mats, int32_t n_mats,
                                               const uint8_t* d_mat_id, const double* d_orient,
                                               const ali_node* srcs, int32_t n_src,
                                               const ali_options* opt, double* d_T,
                                               ali_solve_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    const ali_medium md = single_medium(grid, n_mats, n_src, 0);
    return solve_impl<double, double, double, double>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, opt, d_T, stats);
}

extern "C" ali_status ali_solve_batch(ali_handle* h, const ali_medium* media, int32_t n_media,
                                      const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                      const float* d_orient, const ali_node* srcs, const ali_options* opt,
                                      float* d_T, ali_solve_stats* stats) {
    if (!h) return ALI_EINVAL;
    return solve_dispatch<float, float>(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, opt, d_T, stats);
}

extern "C" ali_status ali_solve_traveltime_noalloc(ali_handle* h, const ali_grid* grid,
                                                   const ali_material* mats, int32_t n_mats,
                                                   const uint8_t* d_mat_id, const float* d_orient,
                                                   const ali_node* srcs, int32_t n_src,
                                                   const ali_options* opt, float* d_T,
                                                   ali_solve_stats* stats) {
    if (!h) return ALI_EINVAL;
    if (!grid) return h->fail(ALI_EINVAL, "grid is NULL");
    ali_options o;
    ali_default_options(&o);
    if (opt) o = *opt;
    o.graph = 0;          // instantiating a graph may allocate
    const ali_medium md = single_medium(grid, n_mats, n_src, 0);
    ali_status st = validate_batch(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, nullptr, o.wave);
    if (st != ALI_OK) return st;
    if (!h->static_base) return h->fail(ALI_EDEVICE, "the static scratch array is not available on this device");
    const bool table = o.velocity == ALI_VEL_TABLE;
    size_t need = 0;
    switch (o.arith) {
        case ALI_ARITH_MIXED: need = forward_scratch_bytes<double, float>(*grid, n_src, n_mats, table); break;
        case ALI_ARITH_F32: need = forward_scratch_bytes<float, float>(*grid, n_src, n_mats, table); break;
        case ALI_ARITH_F64: need = forward_scratch_bytes<double, double>(*grid, n_src, n_mats, table); break;
        default: return h->fail(ALI_EINVAL, "unknown arith mode");
    }
    if (need > h->static_bytes)
        return h->fail(ALI_EINVAL, "this solve needs " + std::to_string(need) + " bytes of device scratch; the "
                       "allocation-free entry point has " + std::to_string(h->static_bytes) +
                       " (ALI_NOALLOC_SCRATCH_BYTES): use ali_solve_traveltime");
    h->arena = true;
    h->arena_used = 0;
    h->arena_slots.clear();
    st = solve_dispatch<float, float>(h, &md, 1, mats, n_mats, d_mat_id, d_orient, srcs, &o, d_T, stats);
    h->arena = false;
    if (st == ALI_ENOMEM) h->err = "the static scratch array was too small for this solve: " + h->err;
    return st;
}

// candidate schedules of the autotuner: (band_cells, inner_sweeps)
static const int TUNE_BAND[ALI_TUNE_CANDIDATES] = {1, 1, 1, 2, 2, 3};
static const int TUNE_INNER[ALI_TUNE_CANDIDATES] = {1, 2, 4, 2, 4, 4};

extern "C" ali_status ali_autotune_batch(ali_handle* h, const ali_medium* media, int32_t n_media,
                                         const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                         const float* d_orient, const ali_node* srcs, ali_options* opt,
                                         float* d_T, double* ms_out) {
    if (!h) return ALI_EINVAL;
    if (!opt) return h->fail(ALI_EINVAL, "opt is NULL");
    ali_options best = *opt;
    double best_ms = INFINITY;
    for (int c = 0; c < ALI_TUNE_CANDIDATES; ++c) {
        ali_options o = *opt;
        o.band_cells = TUNE_BAND[c];
        o.inner_sweeps = TUNE_INNER[c];
        double ms = INFINITY;
        // two runs: the first may build the candidate's graphs
        for (int rep = 0; rep < 2; ++rep) {
            ali_solve_stats st{};
            const ali_status s = solve_dispatch<float, float>(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs,
                                                              &o, d_T, &st);
            if (s != ALI_OK) return s;
            ms = st.ms;
        }
        if (ms_out) ms_out[c] = ms;
        if (ms < best_ms) { best_ms = ms; best = o; }
    }
    *opt = best;
    return ALI_OK;
}
