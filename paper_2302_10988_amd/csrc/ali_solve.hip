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
#include "ali_marks.hpp"

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
                       real* __restrict__ T, uint32_t* __restrict__ flags, uint32_t* __restrict__ gflag) {
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
    if (abs(di) <= R + HALO && abs(dj) <= R + HALO) {
        const int t = (j / TZ) * fd.ntx + (i / TX);
        flags[fd.unit_off + t] = TF_SELF;   // evaluate the whole tile
        gflag[fd.group_off + t / GROUP] = 1u;
    }
}

// Seeded fields: every tile holding a fixed node, and its 8 neighbours, starts with a
// visit of all its nodes (a fixed node reaches 2 nodes out, tiles are wider than that).
__global__ void k_seed_flags(const FieldDev* __restrict__ fields, int n_fields, int64_t n_units,
                             const uint32_t* __restrict__ fixmask, uint32_t* __restrict__ flags,
                             uint32_t* __restrict__ gflag) {
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
            flag_tile(flags, gflag, fd.unit_off, fd.group_off, z * fd.ntx + x, (uint32_t)TF_SELF);
        }
}

// Scheduler of one relaxation pass (ascending thresholds), one work-group per field, each
// work-item holding K groups or tiles at a time.
template <typename real, int K>
__global__ void __launch_bounds__(SCHED_T)
k_sched(const FieldDev* __restrict__ fields, int advance, uint32_t* __restrict__ flags, real* __restrict__ minrej,
        uint32_t* __restrict__ gflag, real* __restrict__ gkey, real* __restrict__ theta, const real* __restrict__ step,
        PassItem* __restrict__ list, uint32_t* __restrict__ cnt_cur, uint32_t* __restrict__ cnt_next,
        const uint32_t* __restrict__ part_base, uint32_t* __restrict__ done, int direct_tiles) {
    __shared__ uint32_t s_due[SCHED_T * K];
    schedule_field<false, real, SCHED_T, K>(blockIdx.x, fields, advance, step, flags, minrej, gflag, gkey, theta, list,
                                         cnt_cur, cnt_next, part_base, done, s_due, direct_tiles);
}


// min of non-negative values in LDS through their integer bit patterns
__device__ __forceinline__ void lds_min(float* p, float v) {
    atomicMin(reinterpret_cast<unsigned*>(p), __float_as_uint(v));
}
__device__ __forceinline__ void lds_min(double* p, double v) {
    atomicMin(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}


// One visit by one wave of up to G_MAX tiles of the pass list at once (64 lanes, NPL
// nodes per lane and tile; every tile and its halo staged in LDS).  The marked nodes of
// all the visit's tiles are packed into the same 64-lane chunks, so a wave evaluates
// full chunks where one tile alone would fill a third of them; the tiles are otherwise
// independent, exactly as if separate waves visited them (each works on its own copy of
// its halo).  G, the tiles per visit, is the same for every wave of a pass: enough
// visits to occupy `slots` waves, at most G_MAX.
// The nodes to evaluate are tracked per node.  The first sweep takes every node (TF_SELF),
// the band front (unreached nodes with a reached neighbour: new arrivals and values an
// earlier band rejected) and the nodes a neighbouring tile marked; each later sweep takes
// the nodes marked by changes inside the tile.  A change of node X marks a diamond
// neighbour D in the tile only if min(old, new) <= tau_D: the update at D reads only
// neighbours that precede D's own value in key order, so a neighbour that stays behind D
// cannot change it.  Across tiles the marks are unconditional (the other tile may be
// working on an older copy of X) and go to the neighbouring tile's node mask for the next
// pass.
// SEEDED: the fixed nodes are the set bits of fixmask (one bit per node of each tile unit,
// NODE_WORDS words per unit) instead of the source box of radius R.
// TAB: phase speeds from the per-material tables vtab (offset in geo slot 6).
constexpr int G_MAX = 4;
constexpr int TILE_LDS = LH * LSTRIDE;

// LDS of one relaxation wave
template <typename real> struct RelaxLds {
    real lt[G_MAX * TILE_LDS];                // staged tiles and halos
    uint16_t clist[G_MAX * NTHREADS];         // packed nodes: tile * NTHREADS + node
    uint8_t dnext[G_MAX][NTHREADS];           // one byte per node: marked for the next sweep
    uint32_t own[G_MAX][NODE_WORDS];          // nodes left marked at the sweep cap
    uint32_t touched[G_MAX][NODE_WORDS];      // nodes whose value changed in this visit
    PassItem s_item[G_MAX];
    real s_th[G_MAX], s_rej[G_MAX];
    real s_lo[G_MAX];                         // smallest old or new value of a change in the tile
    uint32_t incm[G_MAX][NODE_WORDS];         // nodes whose value went up in this visit
    ListMap map;                              // where the pass's list entries sit
};

static_assert(TX == MARK_TX && TZ == MARK_TZ && NODE_WORDS == MARK_WORDS && HALO == 2,
              "the cross-tile marks are written for 16 x 8 tiles and the diamond of radius 2");

// The tiles of one pass of n_units (> 0) listed tiles visited one at a time by this wave
// (a grid stride over the list), for passes too small to give every wave several tiles:
// the list entry lives in scalar registers.  The wave's update and estimate counts are
// added to my_updates, my_evals.
template <typename real, typename mreal, bool SEEDED, bool TAB>
__device__ __forceinline__ void relax_single(RelaxLds<real>& L, uint32_t n_units, const ListMap& map,
                                             const PassItem* __restrict__ list, const mreal* __restrict__ geo_all,
                                             const real* __restrict__ fbt_all, int R, int inner,
                                             const real* __restrict__ theta, real* __restrict__ T,
                                             uint32_t* __restrict__ flags, real* __restrict__ minrej,
                                             uint32_t* __restrict__ gflag, real* __restrict__ gkey,
                                             uint32_t* __restrict__ marks_in, uint32_t* __restrict__ marks_out,
                                             const uint32_t* __restrict__ fixmask, const mreal* __restrict__ vtab,
                                             unsigned& my_updates, unsigned& my_evals) {
    real* lt = L.lt;
    uint8_t* dnext = L.dnext[0];
    uint16_t* clist = L.clist;
    uint32_t* touched = L.touched[0];
    const XcdRange xr = xcd_range(n_units);
    // the slot of the first entry from the map in registers, each later one looked up in
    // the LDS copy while the entry before it is visited
    uint32_t slot = xr.begin < xr.end ? list_slot_reg(map, xr.begin) : 0u;
    for (uint32_t item = xr.begin; item < xr.end; item += xr.stride) {
    const PassItem pi = list[slot];
    if (item + xr.stride < xr.end) slot = __builtin_amdgcn_readfirstlane(list_slot(L.map, item + xr.stride));
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
    for (int q = lane; q < NTHREADS; q += RW) dnext[q] = 0;
    if (lane < NODE_WORDS) touched[lane] = 0u;
    const int2 s = pi.src;
    __syncthreads();

    // the NPL nodes of this lane: node = lane + 64 q.
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

    // write back the changed nodes
#pragma unroll 1
    for (int q = 0; q < NPL; ++q) {
        const int node = lane + RW * q;
        // a node whose value changed (possibly back to where it started) is written back;
        // only nodes inside the grid are ever evaluated
        if (!((touched[node >> 5] >> (node & 31)) & 1u)) continue;
        const int lx = node % TX, lz = node / TX;
        Tf[(int64_t)(j0 + lz) * nx + (i0 + lx)] = lt[(lz + HALO) * LSTRIDE + (lx + HALO)];
    }
    // after the sweep cap, the tile's own unfinished nodes carry over to the next pass
#pragma unroll
    for (int q = 0; q < NPL; ++q) {
        const unsigned long long m = done ? 0ull : __ballot((dmask >> q) & 1u);
        if (lane == 0) {
            L.own[0][2 * q] = (uint32_t)m;
            L.own[0][2 * q + 1] = (uint32_t)(m >> 32);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const real r2 = __shfl_xor(rej, o);
        rej = r2 < rej ? r2 : rej;
    }
    __syncthreads();
    // lane o < 9: the marks for neighbourhood slot o (4: the tile itself); push the node
    // marks and flag the tile
    if (lane < 9) {
        const int ox = lane % 3 - 1, oz = lane / 3 - 1;
        uint32_t w[NODE_WORDS];
        if (lane == 4) {
#pragma unroll
            for (int k = 0; k < NODE_WORDS; ++k) w[k] = L.own[0][k];
        } else {
            uint32_t tw[NODE_WORDS];
#pragma unroll
            for (int k = 0; k < NODE_WORDS; ++k) tw[k] = touched[k];
            cross_marks(tw, tx, tz, nx, nz, ox, oz, w);
        }
        const int64_t u2 = (int64_t)unit + (int64_t)oz * ntx + ox;
        bool any = false;
#pragma unroll
        for (int k = 0; k < NODE_WORDS; ++k)
            if (w[k]) {
                atomicOr(&marks_out[u2 * NODE_WORDS + k], w[k]);
                any = true;
            }
        if (any) flag_tile(flags, gflag, unit - (uint32_t)(tz * ntx + tx), pi.group_off, (tz + oz) * ntx + tx + ox, TF_MARK);
    }
    if (lane == 0) {
        minrej[unit] = rej;
        if (gkey && rej < inf) key_min(&gkey[pi.group_off + (uint32_t)((tz * ntx + tx) / GROUP)], rej);
    }
    __syncthreads();     // LDS is reused by the next item
    }
}

// The visits of one pass of n_units (> 0) listed tiles, taken by this wave with a stride of
// the grid; the wave's update and estimate counts are added to *upd, *evals.
template <typename real, typename mreal, bool SEEDED, bool TAB>
__device__ __forceinline__ void relax_visits(RelaxLds<real>& L, uint32_t n_units, int slots, int gcap,
                                             const PassItem* __restrict__ list, const mreal* __restrict__ geo_all,
                                             const real* __restrict__ fbt_all, int R, int inner,
                                             const real* __restrict__ theta, real* __restrict__ T,
                                             uint32_t* __restrict__ flags, real* __restrict__ minrej,
                                             uint32_t* __restrict__ gflag, real* __restrict__ gkey,
                                             uint32_t* __restrict__ marks_in, uint32_t* __restrict__ marks_out,
                                             const uint32_t* __restrict__ fixmask, const mreal* __restrict__ vtab,
                                             unsigned& my_updates, unsigned& my_evals) {
    auto& lt = L.lt;
    auto& clist = L.clist;
    auto& dnext = L.dnext;
    auto& touched = L.touched;
    auto& s_item = L.s_item;
    auto& s_th = L.s_th;
    auto& s_rej = L.s_rej;
    // tiles per visit: spread the pass over `slots` waves, at most G_MAX tiles each
    const uint32_t per = n_units / (uint32_t)slots;
    const int G = per >= (uint32_t)gcap ? gcap : (per < 1u ? 1 : (int)per);
    const uint32_t n_visits = (n_units + (uint32_t)G - 1u) / (uint32_t)G;
    const real inf = dinf<real>();

    static_assert(sizeof(PassItem) == 4 * sizeof(uint4), "a pass-list entry is four 16-byte vectors");
    const XcdRange xr = xcd_range(n_visits);
    // the pass-list entries of a visit (lanes 0..4*ng-1, one 16-byte vector each): the
    // first visit's are read here, each later visit's while the one before it runs
    uint4 nitem = make_uint4(0u, 0u, 0u, 0u);
    auto fetch = [&](uint32_t v) {
        const uint32_t f0 = v * (uint32_t)G;
        const int n = n_units - f0 < (uint32_t)G ? (int)(n_units - f0) : G;
        if ((int)threadIdx.x < 4 * n)
            nitem = reinterpret_cast<const uint4*>(list + list_slot(L.map, f0 + threadIdx.x / 4u))[threadIdx.x % 4u];
    };
    if (xr.begin < xr.end) fetch(xr.begin);
    for (uint32_t visit = xr.begin; visit < xr.end; visit += xr.stride) {
    // the lane index is made opaque inside the visit loop: otherwise the per-lane staging
    // offsets are hoisted out of the loop and held in registers through the sweeps
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    const uint32_t first = visit * (uint32_t)G;
    const int ng = n_units - first < (uint32_t)G ? (int)(n_units - first) : G;   // tiles of this visit
    if (lane < 4 * ng) reinterpret_cast<uint4*>(s_item)[lane] = nitem;
    __syncthreads();
    if (visit + xr.stride < xr.end) fetch(visit + xr.stride);

    // stage every tile and its halo: all loads of a lane are issued before its first store
    constexpr int SQ = (LW * LH + RW - 1) / RW;
    real sv[G_MAX][SQ];
#pragma unroll
    for (int g = 0; g < G_MAX; ++g) {
        const PassItem& pi = s_item[g < ng ? g : 0];
        const int i0 = pi.tx * TX, j0 = pi.tz * TZ, nx = pi.nx, nz = pi.nz;
        const real* __restrict__ Tf = T + pi.t_off;
#pragma unroll
        for (int k = 0; k < SQ; ++k) {
            const int q = lane + RW * k;
            const int li = q % LW, lj = q / LW;
            const int gi = i0 - HALO + li, gj = j0 - HALO + lj;
            sv[g][k] = (g < ng && q < LW * LH && gi >= 0 && gj >= 0 && gi < nx && gj < nz)
                           ? Tf[(int64_t)gj * nx + gi] : inf;
        }
    }
    // incoming marks of each tile (read and cleared; this pass writes the other buffer):
    // lane 4 g + w holds word w of tile g
    uint32_t mk = 0u, fm = 0u;
    if (lane < NODE_WORDS * ng) {
        const uint32_t unit = s_item[lane / NODE_WORDS].unit;
        const int64_t a = (int64_t)unit * NODE_WORDS + lane % NODE_WORDS;
        mk = marks_in[a];
        if (mk) marks_in[a] = 0u;
        if constexpr (SEEDED) fm = fixmask[a];
    }
    if (lane < ng) {
        s_th[lane] = theta[s_item[lane].f];
        s_rej[lane] = inf;
        L.s_lo[lane] = inf;
    }
#pragma unroll
    for (int g = 0; g < G_MAX; ++g) {
#pragma unroll
        for (int k = 0; k < SQ; ++k) {
            const int q = lane + RW * k;
            if (g < ng && q < LW * LH) lt[g * TILE_LDS + (q / LW) * LSTRIDE + q % LW] = sv[g][k];
        }
    }
    static_assert(sizeof(L.dnext) % sizeof(uint64_t) == 0 && sizeof(L.dnext) <= RW * sizeof(uint64_t),
                  "at most one 8-byte word of sweep marks per lane");
    if (lane < (int)(sizeof(L.dnext) / sizeof(uint64_t))) reinterpret_cast<uint64_t*>(&dnext[0][0])[lane] = 0ull;
    if (lane < G_MAX * NODE_WORDS) {
        (&touched[0][0])[lane] = 0u;
        (&L.incm[0][0])[lane] = 0u;
    }
    __syncthreads();

    // the nodes of this lane: q = 0 .. NPL * G_MAX - 1, tile q / NPL, node lane + 64 (q % NPL).
    // Loops over them stay rolled, and nothing per node is kept in registers across the
    // phases (the write-back finds changed nodes in the LDS change mask).
    unsigned dmask = 0u;              // bit q: node q of this lane is marked for this sweep
    unsigned amask = 0u;              // bit q: node q of this lane is evaluated at all
#pragma unroll 1
    for (int q = 0; q < NPL * ng; ++q) {
        const int g = q / NPL;
        const int node = lane + RW * (q % NPL);
        const PassItem& pi = s_item[g];
        const int lx = node % TX, lz = node / TX;
        const int gi = pi.tx * TX + lx, gj = pi.tz * TZ + lz;
        const int me = g * TILE_LDS + (lz + HALO) * LSTRIDE + (lx + HALO);
        bool fixed_node;
        if constexpr (SEEDED) fixed_node = (__shfl(fm, g * NODE_WORDS + (node >> 5)) >> (node & 31)) & 1u;
        else fixed_node = abs(gi - pi.src.x) <= R && abs(gj - pi.src.y) <= R;
        const bool act = gi < pi.nx && gj < pi.nz && !fixed_node;
        amask |= act ? 1u << q : 0u;
        const real cur = lt[me];
        bool any = false;
#pragma unroll
        for (int k = 0; k < 12; ++k) any |= lt[me + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k]] < inf;
        const bool marked = (__shfl(mk, g * NODE_WORDS + (node >> 5)) >> (node & 31)) & 1u;
        // a finite node with no finite neighbour left is evaluated too (it must turn +inf)
        if (act && (any || cur < inf) && ((pi.bits & TF_SELF) || !(cur < inf) || marked)) dmask |= 1u << q;
    }

    bool done = false;
    for (int it = 0;; ++it) {
        // pack the marked nodes of all tiles
        unsigned total = 0;
#pragma unroll 1
        for (int q = 0; q < NPL * ng; ++q) {
            const unsigned long long m = __ballot((dmask >> q) & 1u);
            if ((dmask >> q) & 1u)
                clist[total + __popcll(m & ((1ull << lane) - 1ull))] =
                    (uint16_t)((q / NPL) * NTHREADS + lane + RW * (q % NPL));
            total += (unsigned)__popcll(m);
        }
        __syncthreads();
        if (total == 0) { done = true; break; }
        if (it == inner) break;     // sweep cap: the marked nodes carry over to the next pass
        dmask = 0u;
        for (unsigned c = 0; c < total; c += RW) {
            bool chg = false;
            real lo = real(0);
            int code = 0;
            if (c + lane < total) {
                code = clist[c + lane];
                const int g = code / NTHREADS, node = code % NTHREADS;
                const PassItem& pi = s_item[g];
                const int nlx = node % TX, nlz = node / TX;
                const int nme = g * TILE_LDS + (nlz + HALO) * LSTRIDE + (nlx + HALO);
                const int64_t p = (int64_t)(pi.tz * TZ + nlz) * pi.nx + (pi.tx * TX + nlx);
                const mreal* __restrict__ geo = geo_all + GEO_N * pi.node_off;
                const real* __restrict__ fbt = fbt_all + 4 * pi.node_off;
                using NC = typename std::conditional<TAB, NodeConstTab<mreal, real>, NodeConst<mreal, real>>::type;
                NC nc;
                load_node_const<real, mreal>(nc, p, geo, fbt);
                if constexpr (TAB) nc.vt = vtab + (int)geo[GEO_N * p + 6];
                real t[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) t[k] = lt[nme + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k]];
                ++my_updates;
                real u = local_update<mreal, real>(nc, t, lt, nme, LSTRIDE, my_evals);
                if (u > s_th[g] && u < inf) { lds_min(&s_rej[g], u); u = inf; }
                const real cv = lt[nme];
                if (!(u == cv || (u >= inf && cv >= inf))) {
                    lt[nme] = u;
                    chg = true;
                    lo = u < cv ? u : cv;
                    atomicOr(&touched[g][node >> 5], 1u << (node & 31));
                    lds_min(&L.s_lo[g], lo);
                    if (u > cv) atomicOr(&L.incm[g][node >> 5], 1u << (node & 31));
                }
            }
            // every value of the chunk is stored before any neighbour is compared (the
            // comparisons must see the neighbours' new values)
            __syncthreads();
            if (chg) {
                const int g = code / NTHREADS, node = code % NTHREADS;
                const int nlx = node % TX, nlz = node / TX;
                const int nme = g * TILE_LDS + (nlz + HALO) * LSTRIDE + (nlx + HALO);
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    const int ax = nlx + SLOT_DI[k], az = nlz + SLOT_DJ[k];
                    if (ax >= 0 && az >= 0 && ax < TX && az < TZ &&
                        lo <= lt[nme + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k]])
                        dnext[g][az * TX + ax] = 1;
                }
            }
            __syncthreads();
        }
        // collect (and clear) the marks for the next sweep: every node's byte is read by
        // the lane that owns the node
#pragma unroll 1
        for (int q = 0; q < NPL * ng; ++q) {
            const int g = q / NPL;
            const int node = lane + RW * (q % NPL);
            if (dnext[g][node]) {
                dnext[g][node] = 0;
                dmask |= amask & (1u << q);
            }
        }
        __syncthreads();
    }

    // write back the changed nodes (only nodes inside the grid are ever evaluated)
#pragma unroll 1
    for (int q = 0; q < NPL * ng; ++q) {
        const int g = q / NPL;
        const int node = lane + RW * (q % NPL);
        if (!((touched[g][node >> 5] >> (node & 31)) & 1u)) continue;
        const PassItem& pi = s_item[g];
        const int lx = node % TX, lz = node / TX;
        T[pi.t_off + (int64_t)(pi.tz * TZ + lz) * pi.nx + (pi.tx * TX + lx)] =
            lt[g * TILE_LDS + (lz + HALO) * LSTRIDE + (lx + HALO)];
    }
    // after the sweep cap, each tile's own unfinished nodes carry over to the next pass
#pragma unroll 1
    for (int q = 0; q < NPL * ng; ++q) {
        const unsigned long long m = done ? 0ull : __ballot((dmask >> q) & 1u);
        if (lane == 0) {
            L.own[q / NPL][2 * (q % NPL)] = (uint32_t)m;
            L.own[q / NPL][2 * (q % NPL) + 1] = (uint32_t)(m >> 32);
        }
    }
    __syncthreads();
    // lane 9 g + o: the marks of tile g for its neighbourhood slot o (4: the tile itself);
    // push the node marks and flag the tile
    if (lane < 9 * ng) {
        const int g = lane / 9, o = lane % 9;
        const int ox = o % 3 - 1, oz = o / 3 - 1;
        const PassItem& pi = s_item[g];
        const int ntx = (pi.nx + TX - 1) / TX;
        uint32_t w[NODE_WORDS];
        if (o == 4) {
            // unfinished nodes, and nodes whose value went up: a neighbouring tile may have
            // skipped marking them against their lower staged value (below)
#pragma unroll
            for (int k = 0; k < NODE_WORDS; ++k) w[k] = L.own[g][k] | L.incm[g][k];
        } else {
            uint32_t tw[NODE_WORDS];
#pragma unroll
            for (int k = 0; k < NODE_WORDS; ++k) tw[k] = touched[g][k];
            cross_marks(tw, pi.tx, pi.tz, pi.nx, pi.nz, ox, oz, w);
            // The causal filter across tiles, on this visit's staged copy of the neighbour:
            // a node D whose copy lies below every old and new value of the tile's changes
            // cannot depend on them.  If D's own tile raised D during this pass (the copy is
            // then out of date), that tile marks D itself for the next pass (above); a D that
            // went down or stayed keeps the argument.
            const real lo_t = L.s_lo[g];
#pragma unroll
            for (int k = 0; k < NODE_WORDS; ++k) {
                uint32_t m = w[k], keep = 0u;
                while (m) {
                    const int b = __builtin_ctz(m);
                    m &= m - 1u;
                    const int nn = 32 * k + b;   // node of the neighbouring tile
                    const int ax = nn % TX + TX * ox, az = nn / TX + TZ * oz;
                    const real td = lt[g * TILE_LDS + (az + HALO) * LSTRIDE + (ax + HALO)];
                    if (!(td < lo_t)) keep |= 1u << b;
                }
                w[k] = keep;
            }
        }
        const int64_t u2 = (int64_t)pi.unit + (int64_t)oz * ntx + ox;
        bool any = false;
#pragma unroll
        for (int k = 0; k < NODE_WORDS; ++k)
            if (w[k]) {
                atomicOr(&marks_out[u2 * NODE_WORDS + k], w[k]);
                any = true;
            }
        if (any)
            flag_tile(flags, gflag, pi.unit - (uint32_t)(pi.tz * ntx + pi.tx), pi.group_off,
                      (pi.tz + oz) * ntx + pi.tx + ox, TF_MARK);
    }
    if (lane < ng) {
        const PassItem& pi = s_item[lane];
        const real rej = s_rej[lane];
        minrej[pi.unit] = rej;
        const int ntx = (pi.nx + TX - 1) / TX;
        if (gkey && rej < inf) key_min(&gkey[pi.group_off + (uint32_t)((pi.tz * ntx + pi.tx) / GROUP)], rej);
    }
    __syncthreads();     // LDS is reused by the next visit
    }
}

// statistics of one wave, spread over STAT_SLOTS counter pairs (one address for all waves
// would serialise every visit of a pass)
__device__ __forceinline__ void relax_stats(unsigned long long* __restrict__ counters, unsigned my_updates,
                                            unsigned my_evals) {
    for (int o = 32; o > 0; o >>= 1) {
        my_updates += __shfl_xor(my_updates, o);
        my_evals += __shfl_xor(my_evals, o);
    }
    if (threadIdx.x == 0 && my_updates) {
        unsigned long long* sc = counters + 4 + 2 * (blockIdx.x % STAT_SLOTS);
        atomicAdd(&sc[0], (unsigned long long)my_updates);
        atomicAdd(&sc[1], (unsigned long long)my_evals);
    }
}

// One relaxation pass: the listed tiles of the pass (count), or, for an empty list, the
// idle flag that ends the solve.
template <typename real, typename mreal, bool SEEDED, bool TAB>
__global__ void __launch_bounds__(RW) __attribute__((amdgpu_waves_per_eu(4)))
k_relax(const PassItem* __restrict__ list, const mreal* __restrict__ geo_all, const real* __restrict__ fbt_all,
        int R, int inner, const real* __restrict__ theta,
        real* __restrict__ T, uint32_t* __restrict__ flags, real* __restrict__ minrej,
        uint32_t* __restrict__ gflag, real* __restrict__ gkey,
        uint32_t* __restrict__ marks_in, uint32_t* __restrict__ marks_out,
        const uint32_t* __restrict__ count, const uint32_t* __restrict__ part_base, uint32_t* __restrict__ idle,
        unsigned long long* __restrict__ counters, const uint32_t* __restrict__ fixmask,
        const mreal* __restrict__ vtab, int slots, int gcap) {
    __shared__ RelaxLds<real> L;
    const ListMap map = read_list_map(count, part_base);
    const uint32_t n_units = map.pre[LIST_PARTS];
    if (n_units == 0u) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *idle = 1u;
        return;
    }
    put_list_map(L.map, map);
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        atomicAdd(&counters[2], 1ull);                  // passes with work
        atomicAdd(&counters[3], (unsigned long long)n_units);   // tile visits
    }
    unsigned my_updates = 0, my_evals = 0;
    if (gcap <= 1 || n_units < 2u * (uint32_t)slots)
        relax_single<real, mreal, SEEDED, TAB>(L, n_units, map, list, geo_all, fbt_all, R, inner, theta, T, flags,
                                               minrej, gflag, gkey, marks_in, marks_out, fixmask, vtab, my_updates,
                                               my_evals);
    else
        relax_visits<real, mreal, SEEDED, TAB>(L, n_units, slots, gcap, list, geo_all, fbt_all, R, inner, theta, T, flags,
                                               minrej, gflag, gkey, marks_in, marks_out, fixmask, vtab, my_updates,
                                               my_evals);
    relax_stats(counters, my_updates, my_evals);
}

// ---------------------------------------------------------------------------------------
// persistent relaxation: every pass of a solve in one cooperative launch
// ---------------------------------------------------------------------------------------
// Grid barrier for a cooperative grid of one-wave work-groups: each group's arrival is
// counted on one of BAR_LEAVES leaf counters, the last arrival of a leaf counts on the top
// counter, and the last arrival there releases everyone by bumping the generation word.
// Each counter sits on its own 128-byte line.  The fences on both sides make every global
// write of the phase before visible to every work-group after it, across the dies.  Every
// wait is bounded: past `timeout` ticks of the constant-rate clock, or once another group
// has given up, the group sets *err and returns false (the host reports a device error).
constexpr int BAR_LEAVES = 64;
constexpr int BAR_WORDS = 64 + 32 * BAR_LEAVES;

__device__ __forceinline__ bool grid_sync(uint32_t* __restrict__ bar, uint32_t& gen, uint32_t* __restrict__ err,
                                          long long timeout) {
    __threadfence();
    int ok = 1;
    if (threadIdx.x == 0) {
        const uint32_t nb = gridDim.x;
        const uint32_t nleaf = nb < (uint32_t)BAR_LEAVES ? nb : (uint32_t)BAR_LEAVES;
        const uint32_t leaf = blockIdx.x % nleaf;
        const uint32_t leaf_n = nb / nleaf + (leaf < nb % nleaf ? 1u : 0u);
        const uint32_t want = gen + 1u;
        if (atomicAdd(&bar[64 + 32 * leaf], 1u) + 1u == leaf_n) {
            atomicExch(&bar[64 + 32 * leaf], 0u);
            __threadfence();
            if (atomicAdd(&bar[32], 1u) + 1u == nleaf) {
                atomicExch(&bar[32], 0u);
                __threadfence();
                __hip_atomic_store(&bar[0], want, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(&bar[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != want) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                wall_clock64() - t0 > timeout) {
                atomicOr(err, 1u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    ok = __shfl(ok, 0);
    __threadfence();
    gen += 1u;
    return ok != 0;
}

// All passes of a forward solve, from pass first_pass on, in one launch: the grid (every
// work-group resident, one wave each) schedules the fields (field f by group f mod grid),
// meets at a grid barrier, relaxes the listed tiles, meets again; an empty pass list ends
// the loop (*done = 1), as does max_passes.  The schedule and the visits are those of
// k_sched and k_relax, so the fields are bitwise those of the pass-by-pass launches.
template <typename real, typename mreal, bool SEEDED, bool TAB>
__global__ void __launch_bounds__(RW) __attribute__((amdgpu_waves_per_eu(4)))
k_relax_persist(const FieldDev* __restrict__ fields, int n_fields, const real* __restrict__ step,
                real* __restrict__ theta, PassItem* __restrict__ list, uint32_t* __restrict__ cnt,
                const mreal* __restrict__ geo_all, const real* __restrict__ fbt_all, int R, int inner,
                real* __restrict__ T, uint32_t* __restrict__ flags, real* __restrict__ minrej,
                uint32_t* __restrict__ gflag, real* __restrict__ gkey, uint32_t* __restrict__ marks, int64_t nunits,
                unsigned long long* __restrict__ counters, const uint32_t* __restrict__ fixmask,
                const mreal* __restrict__ vtab, int gcap, int direct_tiles, int first_pass, int max_passes,
                uint32_t* __restrict__ bar,
                uint32_t* __restrict__ err, uint32_t* __restrict__ done, long long timeout) {
    __shared__ RelaxLds<real> L;
    uint32_t gen = 0u;
    unsigned my_updates = 0, my_evals = 0;
    for (int p = 0; p < max_passes; ++p) {
        const int pp = first_pass + p;
        for (int f = blockIdx.x; f < n_fields; f += gridDim.x)
            schedule_field<false, real, RW, 2>(f, fields, pp > 0 ? 1 : 0, step, flags, minrej, gflag, gkey, theta, list,
                                            cnt + (pp & 1) * CNT_BLOCK, cnt + ((pp + 1) & 1) * CNT_BLOCK,
                                            cnt + 2 * CNT_BLOCK, cnt + 2 * CNT_BLOCK + LIST_PARTS,
                                            reinterpret_cast<uint32_t*>(L.lt), direct_tiles);
        if (!grid_sync(bar, gen, err, timeout)) break;
        const ListMap map = read_list_map<true>(cnt + (pp & 1) * CNT_BLOCK, cnt + 2 * CNT_BLOCK);
        const uint32_t n_units = map.pre[LIST_PARTS];
        if (n_units == 0u) {
            if (blockIdx.x == 0 && threadIdx.x == 0) *done = 1u;
            break;
        }
        put_list_map(L.map, map);
        __syncthreads();
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            atomicAdd(&counters[2], 1ull);
            atomicAdd(&counters[3], (unsigned long long)n_units);
        }
        uint32_t* mk_in = marks + (size_t)(pp & 1) * nunits * NODE_WORDS;
        uint32_t* mk_out = marks + (size_t)((pp + 1) & 1) * nunits * NODE_WORDS;
        if (gcap <= 1 || n_units < 2u * gridDim.x)
            relax_single<real, mreal, SEEDED, TAB>(L, n_units, map, list, geo_all, fbt_all, R, inner, theta, T,
                                                   flags, minrej, gflag, gkey, mk_in, mk_out, fixmask, vtab,
                                                   my_updates, my_evals);
        else
            relax_visits<real, mreal, SEEDED, TAB>(L, n_units, (int)gridDim.x, gcap, list, geo_all, fbt_all, R, inner,
                                                   theta, T, flags, minrej, gflag, gkey, mk_in, mk_out, fixmask, vtab,
                                                   my_updates, my_evals);
        if (!grid_sync(bar, gen, err, timeout)) break;
    }
    relax_stats(counters, my_updates, my_evals);
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
    if (opt.visit_tiles < 0 || opt.visit_tiles > G_MAX) return H->fail(ALI_EINVAL, "visit_tiles out of range [0, 4]");
    if (opt.persistent != 0 && opt.persistent != 1) return H->fail(ALI_EINVAL, "persistent must be 0 or 1");
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
    int64_t units = 0, fnodes = 0, med_nodes = 0, groups = 0;
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
            fd.group_off = (uint32_t)groups;
            fd.mat_off = dev_mat_off[m];
            fd.medium = m;
            fd.rec_off = md.rec_offset;
            fd.n_rec = recv ? md.n_rec : 0;
            fd.obs_off = obs;
            fd.src = make_int2(srcs[md.src_offset + k].i, srcs[md.src_offset + k].j);
            F.hfields.push_back(fd);
            units += (int64_t)ntx * ntz;
            groups += field_groups(ntx * ntz);
            fnodes += (int64_t)nx * nz;
            obs += fd.n_rec;
            hstep.push_back(band);
            htheta.push_back(band);
        }
    }
    F.medium_first_field.push_back((int)F.hfields.size());
    const int n_fields = (int)F.hfields.size();
    for (int f = 0; f < n_fields; ++f) F.hfields[f].part = list_part_of(f, n_fields);
    const int64_t nunits = units;
    F.n_units = nunits;
    F.n_groups = groups;
    // the scheduler reads small fields tile by tile; the group summaries are kept only if
    // some field of the call is scheduled by groups
    const int sched_k = sched_k_for(nunits);
    const int direct_tiles = direct_tiles_for(nunits, opt.persistent ? RW * 2 : SCHED_T * sched_k);
    bool use_groups = false;
    for (const FieldDev& fd : F.hfields) use_groups |= fd.ntx * fd.ntz > direct_tiles;
    F.field_nodes = fnodes;

    void *d_mats, *d_geo, *d_fbt, *d_fields, *d_flags, *d_list, *d_count, *d_upd, *d_err;
    void *d_theta, *d_step, *d_minrej, *d_marks, *d_idle, *d_gflag, *d_gkey;
    if (!H->scratch("mats", sizeof(MatDev<mreal>) * hm.size(), &d_mats) ||
        !H->scratch("fields", sizeof(FieldDev) * n_fields, &d_fields) ||
        !H->scratch("theta", sizeof(real) * n_fields, &d_theta) ||
        !H->scratch("step", sizeof(real) * n_fields, &d_step) ||
        !H->scratch("minrej", sizeof(real) * nunits, &d_minrej) ||
        !H->scratch("geo", sizeof(mreal) * GEO_N * med_nodes, &d_geo) ||
        !H->scratch("fbt", sizeof(real) * 4 * med_nodes, &d_fbt) ||
        !H->scratch("flags", sizeof(uint32_t) * nunits, &d_flags) ||
        !H->scratch("gflag", sizeof(uint32_t) * groups, &d_gflag) ||
        !H->scratch("gkey", sizeof(real) * groups, &d_gkey) ||
        !H->scratch("list", sizeof(PassItem) * nunits, &d_list) ||
        !H->scratch("marks", sizeof(uint32_t) * 2 * NODE_WORDS * nunits, &d_marks) ||
        !H->scratch("count", sizeof(uint32_t) * (CNT_WORDS + n_fields), &d_count) ||
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
    HIPCK(H, hipMemsetAsync(d_gflag, 0, sizeof(uint32_t) * groups, S));
    HIPCK(H, hipMemsetAsync(d_marks, 0, sizeof(uint32_t) * 2 * NODE_WORDS * nunits, S));
    HIPCK(H, hipMemsetAsync(d_upd, 0, (4 + 2 * STAT_SLOTS) * sizeof(unsigned long long), S));
    HIPCK(H, hipMemsetAsync(d_count, 0, sizeof(uint32_t) * (CNT_WORDS + n_fields), S));
    F.part_base = list_part_base(F.hfields);
    HIPCK(H, hipMemcpyAsync((uint32_t*)d_count + 2 * CNT_BLOCK, F.part_base.data(), sizeof(uint32_t) * LIST_PARTS,
                            hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemsetAsync(d_idle, 0, sizeof(uint32_t), S));
    HIPCK(H, hipMemsetAsync(d_err, 0, sizeof(int), S));

    const int B = 256;
    hipLaunchKernelGGL((k_fill<real>), dim3((unsigned)((nunits + B - 1) / B)), dim3(B), 0, S,
                       (real*)d_minrej, nunits, dinf_host<real>());
    hipLaunchKernelGGL((k_fill<real>), dim3((unsigned)((groups + B - 1) / B)), dim3(B), 0, S,
                       (real*)d_gkey, groups, dinf_host<real>());
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
    F.vt = (const mreal*)d_vt;
    F.gt = (const double*)d_gt;
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
                               opt.src_box_radius, d_T, (uint32_t*)d_flags, (uint32_t*)d_gflag);
    }
    if (d_fixmask)
        hipLaunchKernelGGL(k_seed_flags, dim3((unsigned)((nunits + B - 1) / B)), dim3(B), 0, S,
                           (const FieldDev*)d_fields, n_fields, nunits, d_fixmask, (uint32_t*)d_flags,
                           (uint32_t*)d_gflag);
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
    // pass list exit at once.  Far more work-groups than are resident at a time (128 per
    // compute unit against 16), each with few visits: a finished one is replaced by the
    // next in dispatch order, which balances visits of uneven cost (against 32 per compute
    // unit the 128-media batch forward takes 691 instead of 735 ms, its adjoint 671
    // instead of 756 ms)
    const int grid_relax = (int)(nunits < (int64_t)128 * H->n_cu ? nunits : (int64_t)128 * H->n_cu);
    // resident one-wave work-groups of the relaxation (4 per SIMD): a pass with more tiles
    // than this packs several tiles into each visit
    const int slots = 16 * H->n_cu;
    const int gcap = opt.visit_tiles > 0 ? opt.visit_tiles : G_MAX;
    uint32_t* cnt = (uint32_t*)d_count;
    // one pass: schedule, then relax (events around the relax launch when timed)
    auto* const ksched = sched_k == SCHED_K ? &k_sched<real, SCHED_K> : &k_sched<real, SCHED_K_LARGE>;
    auto enqueue = [&](int p, bool timed, hipStream_t S) {
        hipLaunchKernelGGL(ksched, dim3((unsigned)n_fields), dim3(SCHED_T), 0, S,
                           (const FieldDev*)d_fields, p > 0 ? 1 : 0,
                           (uint32_t*)d_flags, (real*)d_minrej, (uint32_t*)d_gflag, (real*)d_gkey,
                           (real*)d_theta, (const real*)d_step,
                           (PassItem*)d_list, cnt + (p & 1) * CNT_BLOCK, cnt + ((p + 1) & 1) * CNT_BLOCK,
                           (const uint32_t*)(cnt + 2 * CNT_BLOCK), cnt + 2 * CNT_BLOCK + LIST_PARTS, direct_tiles);
        uint32_t* mk_in = (uint32_t*)d_marks + (size_t)(p & 1) * nunits * NODE_WORDS;
        uint32_t* mk_out = (uint32_t*)d_marks + (size_t)((p + 1) & 1) * nunits * NODE_WORDS;
        if (timed) (void)hipEventRecord(H->pev[2 * (p % PASS_BATCH)], S);
        const int R = d_fixmask ? -1 : opt.src_box_radius;
        const mreal* vt = (const mreal*)d_vt;
        if (d_fixmask && tab)
            hipLaunchKernelGGL((k_relax<real, mreal, true, true>), dim3((unsigned)grid_relax), dim3(RW), 0, S,
                               (const PassItem*)d_list, (const mreal*)d_geo, (const real*)d_fbt, R,
                               opt.inner_sweeps, (const real*)d_theta, d_T, (uint32_t*)d_flags, (real*)d_minrej,
                               use_groups ? (uint32_t*)d_gflag : nullptr, use_groups ? (real*)d_gkey : nullptr, mk_in, mk_out, (const uint32_t*)(cnt + (p & 1) * CNT_BLOCK), (const uint32_t*)(cnt + 2 * CNT_BLOCK), (uint32_t*)d_idle,
                               (unsigned long long*)d_upd, d_fixmask, vt, slots, gcap);
        else if (d_fixmask)
            hipLaunchKernelGGL((k_relax<real, mreal, true, false>), dim3((unsigned)grid_relax), dim3(RW), 0, S,
                               (const PassItem*)d_list, (const mreal*)d_geo, (const real*)d_fbt, R,
                               opt.inner_sweeps, (const real*)d_theta, d_T, (uint32_t*)d_flags, (real*)d_minrej,
                               use_groups ? (uint32_t*)d_gflag : nullptr, use_groups ? (real*)d_gkey : nullptr, mk_in, mk_out, (const uint32_t*)(cnt + (p & 1) * CNT_BLOCK), (const uint32_t*)(cnt + 2 * CNT_BLOCK), (uint32_t*)d_idle,
                               (unsigned long long*)d_upd, d_fixmask, vt, slots, gcap);
        else if (tab)
            hipLaunchKernelGGL((k_relax<real, mreal, false, true>), dim3((unsigned)grid_relax), dim3(RW), 0, S,
                               (const PassItem*)d_list, (const mreal*)d_geo, (const real*)d_fbt, R,
                               opt.inner_sweeps, (const real*)d_theta, d_T, (uint32_t*)d_flags, (real*)d_minrej,
                               use_groups ? (uint32_t*)d_gflag : nullptr, use_groups ? (real*)d_gkey : nullptr, mk_in, mk_out, (const uint32_t*)(cnt + (p & 1) * CNT_BLOCK), (const uint32_t*)(cnt + 2 * CNT_BLOCK), (uint32_t*)d_idle,
                               (unsigned long long*)d_upd, d_fixmask, vt, slots, gcap);
        else
            hipLaunchKernelGGL((k_relax<real, mreal, false, false>), dim3((unsigned)grid_relax), dim3(RW), 0, S,
                               (const PassItem*)d_list, (const mreal*)d_geo, (const real*)d_fbt, R, opt.inner_sweeps, (const real*)d_theta, d_T,
                               (uint32_t*)d_flags, (real*)d_minrej, use_groups ? (uint32_t*)d_gflag : nullptr, use_groups ? (real*)d_gkey : nullptr, mk_in, mk_out,
                               (const uint32_t*)(cnt + (p & 1) * CNT_BLOCK), (const uint32_t*)(cnt + 2 * CNT_BLOCK),
                               (uint32_t*)d_idle, (unsigned long long*)d_upd, d_fixmask, vt, slots, gcap);
        if (timed) (void)hipEventRecord(H->pev[2 * (p % PASS_BATCH) + 1], S);
    };
    if (opt.persistent) {
        // every pass in one cooperative launch (all work-groups resident; the runtime
        // refuses a grid that does not fit instead of over-subscribing)
        void* kern = d_fixmask ? (tab ? (void*)&k_relax_persist<real, mreal, true, true>
                                      : (void*)&k_relax_persist<real, mreal, true, false>)
                               : (tab ? (void*)&k_relax_persist<real, mreal, false, true>
                                      : (void*)&k_relax_persist<real, mreal, false, false>);
        int per_cu = 0, lds_cu = 0;
        HIPCK(H, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, RW, 0));
        // and no more than the LDS of a compute unit holds, allocations rounded up to 512 B
        hipFuncAttributes fa;
        HIPCK(H, hipFuncGetAttributes(&fa, kern));
        HIPCK(H, hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, H->device));
        const size_t lds_wg = (fa.sharedSizeBytes + 511) & ~(size_t)511;
        if (lds_wg > 0 && (size_t)per_cu * lds_wg > (size_t)lds_cu) per_cu = (int)((size_t)lds_cu / lds_wg);
        if (per_cu < 1) return H->fail(ALI_EDEVICE, "persistent relaxation: no resident work-group fits a compute unit");
        const int grid_p = per_cu * H->n_cu;
        void *d_bar, *d_perr;
        if (!H->scratch("bar", sizeof(uint32_t) * BAR_WORDS, &d_bar) || !H->scratch("perr", 2 * sizeof(uint32_t), &d_perr))
            return H->fail(ALI_ENOMEM, "device scratch allocation failed");
        HIPCK(H, hipMemsetAsync(d_bar, 0, sizeof(uint32_t) * BAR_WORDS, S));
        HIPCK(H, hipMemsetAsync(d_perr, 0, 2 * sizeof(uint32_t), S));
        const FieldDev* a_fields = (const FieldDev*)d_fields;
        int a_nf = n_fields;
        const real* a_step = (const real*)d_step;
        real* a_theta = (real*)d_theta;
        PassItem* a_list = (PassItem*)d_list;
        uint32_t* a_cnt = cnt;
        const mreal* a_geo = (const mreal*)d_geo;
        const real* a_fbt = (const real*)d_fbt;
        int a_R = d_fixmask ? -1 : opt.src_box_radius;
        int a_inner = opt.inner_sweeps;
        real* a_T = d_T;
        uint32_t* a_flags = (uint32_t*)d_flags;
        real* a_minrej = (real*)d_minrej;
        uint32_t* a_gflag = use_groups ? (uint32_t*)d_gflag : nullptr;
        real* a_gkey = use_groups ? (real*)d_gkey : nullptr;
        uint32_t* a_marks = (uint32_t*)d_marks;
        int64_t a_nunits = nunits;
        unsigned long long* a_upd = (unsigned long long*)d_upd;
        const uint32_t* a_fix = d_fixmask;
        const mreal* a_vt = (const mreal*)d_vt;
        int a_gcap = gcap;
        int a_direct = direct_tiles;
        int a_first = 0, a_max = opt.max_sweeps;
        uint32_t* a_bar = (uint32_t*)d_bar;
        uint32_t* a_err = (uint32_t*)d_perr;
        uint32_t* a_done = (uint32_t*)d_perr + 1;
        long long a_timeout = H->barrier_timeout_ticks;
        void* args[] = {&a_fields, &a_nf, &a_step, &a_theta, &a_list, &a_cnt, &a_geo, &a_fbt, &a_R, &a_inner,
                        &a_T, &a_flags, &a_minrej, &a_gflag, &a_gkey, &a_marks, &a_nunits, &a_upd, &a_fix, &a_vt,
                        &a_gcap, &a_direct, &a_first, &a_max, &a_bar, &a_err, &a_done, &a_timeout};
        HIPCK(H, hipEventRecord(H->ev2, S));
        const hipError_t le = hipLaunchCooperativeKernel(kern, dim3((unsigned)grid_p), dim3(RW), args, 0, S);
        if (le != hipSuccess) {
            // e.g. while another process holds the device's cooperative-launch resources
            (void)hipGetLastError();
            H->coop_refused = true;
            return H->fail(ALI_EDEVICE, std::string("hipLaunchCooperativeKernel refused the persistent relaxation: ") +
                                            hipGetErrorString(le));
        }
        HIPCK(H, hipEventRecord(H->ev3, S));
        uint32_t pflags[2] = {0u, 0u};
        HIPCK(H, hipMemcpyAsync(pflags, d_perr, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, S));
        HIPCK(H, hipStreamSynchronize(S));
        float kms = 0.f;
        HIPCK(H, hipEventElapsedTime(&kms, H->ev2, H->ev3));
        relax_ms = kms;
        if (pflags[0]) return H->fail(ALI_EDEVICE, "persistent relaxation: a grid barrier timed out");
        converged = pflags[1] != 0u;
        iters = opt.max_sweeps;
    }
    while (!opt.persistent && iters < opt.max_sweeps) {
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
                                              d_flags, d_minrej, d_gflag, d_gkey, use_groups ? 1 : 0, direct_tiles,
                                              d_theta, d_step, d_list, d_count,
                                              d_marks, nunits, d_geo, d_fbt, opt.src_box_radius,
                                              opt.inner_sweeps, d_T, d_idle, d_upd, grid_relax, slots, gcap,
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
    const int64_t groups = (int64_t)field_groups(((g.nx + TX - 1) / TX) * ((g.nz + TZ - 1) / TZ)) * n_src;
    req.push_back(sizeof(uint32_t) * units);                       // flags
    req.push_back(sizeof(uint32_t) * groups);                      // gflag
    req.push_back(sizeof(real) * groups);                          // gkey
    req.push_back(sizeof(PassItem) * units);                       // list
    req.push_back(sizeof(uint32_t) * 2 * NODE_WORDS * units);      // marks
    req.push_back(sizeof(uint32_t) * (CNT_WORDS + n_src));         // count, finished fields
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

// candidate schedules of the autotuner: band_cells, inner_sweeps, visit_tiles, persistent
static const int TUNE[ALI_TUNE_CANDIDATES][4] = {
    {1, 2, 4, 0}, {1, 2, 2, 0}, {1, 2, 1, 0}, {1, 4, 4, 0}, {2, 2, 4, 0}, {2, 4, 4, 0}, {1, 2, 4, 1}};

// size bucket of a batch: powers of two of the field count, the largest side and the
// node-fields, with the options that change the work (arithmetic, wave, speeds, stiffness)
static std::string tune_bucket(const ali_medium* media, int32_t n_media, const ali_options& o) {
    int64_t nf = 0, nodes = 0;
    int side = 0;
    batch_sizes(media, n_media, &nf, &nodes);
    for (int m = 0; m < n_media; ++m) side = std::max(side, std::max(media[m].grid.nx, media[m].grid.nz));
    auto p2 = [](int64_t v) { int b = 0; while (((int64_t)1 << b) < v) ++b; return b; };
    return graph_key("tune", p2(nf), p2(side), p2(nodes), o.arith, o.wave, o.velocity, o.d_node_A ? 1 : 0);
}

extern "C" ali_status ali_autotune_batch(ali_handle* h, const ali_medium* media, int32_t n_media,
                                         const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                         const float* d_orient, const ali_node* srcs, ali_options* opt,
                                         float* d_T, double* ms_out) {
    if (!h) return ALI_EINVAL;
    if (!opt) return h->fail(ALI_EINVAL, "opt is NULL");
    ali_status st = validate_batch(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs, nullptr, opt->wave);
    if (st != ALI_OK) return st;
    const std::string key = tune_bucket(media, n_media, *opt);
    auto it = h->tuned.find(key);
    if (it != h->tuned.end()) {
        // tuned before on this handle for a batch of the same bucket
        const int c = it->second.first;
        opt->band_cells = TUNE[c][0];
        opt->inner_sweeps = TUNE[c][1];
        opt->visit_tiles = TUNE[c][2];
        opt->persistent = TUNE[c][3];
        if (ms_out)
            for (int k = 0; k < ALI_TUNE_CANDIDATES; ++k) ms_out[k] = it->second.second[k];
        return ALI_OK;
    }
    int best = -1;
    double best_ms = INFINITY;
    std::vector<double> times(ALI_TUNE_CANDIDATES, INFINITY);
    for (int c = 0; c < ALI_TUNE_CANDIDATES; ++c) {
        ali_options o = *opt;
        o.band_cells = TUNE[c][0];
        o.inner_sweeps = TUNE[c][1];
        o.visit_tiles = TUNE[c][2];
        o.persistent = TUNE[c][3];
        double ms = INFINITY;
        // two runs: the first may build the candidate's graphs.  A persistent candidate whose
        // cooperative launch the runtime refuses is left out (time +inf).
        h->coop_refused = false;
        for (int rep = 0; rep < 2; ++rep) {
            ali_solve_stats sst{};
            const ali_status s = solve_dispatch<float, float>(h, media, n_media, mats, n_mats, d_mat_id, d_orient, srcs,
                                                              &o, d_T, &sst);
            if (s != ALI_OK && o.persistent && h->coop_refused) { ms = INFINITY; break; }
            if (s != ALI_OK) return s;
            ms = sst.ms;
        }
        times[c] = ms;
        if (ms < best_ms) { best_ms = ms; best = c; }
    }
    h->tuned[key] = std::make_pair(best, times);
    opt->band_cells = TUNE[best][0];
    opt->inner_sweeps = TUNE[best][1];
    opt->visit_tiles = TUNE[best][2];
    opt->persistent = TUNE[best][3];
    if (ms_out)
        for (int k = 0; k < ALI_TUNE_CANDIDATES; ++k) ms_out[k] = times[k];
    return ALI_OK;
}
