// ali_solve.hpp -- pieces of the travel-time solver shared with the adjoint: tile
// geometry, per-material constants, small utility kernels, and the forward driver that
// leaves its working field and per-node constants on the device.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <vector>

#include "ali_device.hpp"
#include "ali_velocity.hpp"
#include "ali_handle.hpp"
#include "../../include/ali.h"

namespace ali {

// a work-group owns a TX x TZ tile plus a HALO-node ring (the diamond radius) in LDS.
// 16 x 8: a row of the tile is one 128-byte line of float64 times; against 16 x 16 the
// adjoint stages 40 % less per visit (64-field weld: forward + adjoint 53.6 -> 49.5 ms)
// for slightly more redundant forward updates (5.65 against 5.42 per node).
constexpr int TX = 16, TZ = 8, HALO = 2;
constexpr int LW = TX + 2 * HALO, LH = TZ + 2 * HALO;
constexpr int LSTRIDE = LW;                  // LDS row stride of a staged tile (rows contiguous)
constexpr int NTHREADS = TX * TZ;             // nodes of a tile
constexpr int RW = 64;                        // one wave per tile visit
constexpr int NPL = NTHREADS / RW;            // nodes per lane
constexpr int NODE_WORDS = NTHREADS / 32;     // 32-bit words of a per-tile node mask
constexpr int STAT_SLOTS = 256;               // spread of the statistics counters

// Work-group IDs go round-robin over the 8 dies (XCDs) of the chip, each with its own L2.
// A relaxation launch hands its n list entries (visits) out so that every die works
// through one contiguous eighth of the list: consecutive entries are neighbouring tiles
// of one field, whose halos overlap, so they meet in the same L2 instead of being
// fetched once per die.  Work-group b runs on die b % 8 and takes the entries
// begin, begin + stride, ... below end.  A grid that is not a multiple of 8 falls back to a
// plain grid stride.
constexpr uint32_t N_XCD = 8;
struct XcdRange { uint32_t begin, end, stride; };
__device__ __forceinline__ XcdRange xcd_range(uint32_t n) {
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    if (nb % N_XCD != 0u) return XcdRange{b, n, nb};
    const uint32_t x = b % N_XCD, per = (n + N_XCD - 1u) / N_XCD;
    const uint32_t lo = x * per, hi = lo + per < n ? lo + per : n;
    return XcdRange{lo + b / N_XCD, hi, nb / N_XCD};
}

// per-node constants of the relaxation: GEO_N values of the math type per node, namely
// cos 2theta, sin 2theta of the symmetry axis and P, Q, R, K4 of the node's material (two
// unused), so that a node's constants come in two aligned vector loads with no table
// lookup behind them
constexpr int GEO_N = 8;

template <typename real> inline real dinf_host() { return (real)INFINITY; }

// per-material constants on the device (phase-speed constants in the math type)
template <typename mreal> struct MatDev {
    mreal P, Q, R, K4;      // phase-speed constants / h^2
    MatA A;                 // stiffness / density, float64
};

template <typename mreal>
inline std::vector<MatDev<mreal>> make_matdev(const ali_material* mats, int n_mats, double h) {
    std::vector<MatDev<mreal>> hm(n_mats);
    for (int k = 0; k < n_mats; ++k) {
        const ali_material& m = mats[k];
        const double a11 = m.c11 / m.rho, a13 = m.c13 / m.rho, a33 = m.c33 / m.rho, a55 = m.c55 / m.rho;
        const double ih2 = 1.0 / (h * h);
        hm[k].P = (mreal)((a11 + a33 + 2.0 * a55) * ih2);
        hm[k].Q = (mreal)((a33 - a11) * ih2);
        hm[k].R = (mreal)((a11 + a33 - 2.0 * a55) * ih2);
        const double W = (a13 + a55) * ih2;
        hm[k].K4 = (mreal)(4.0 * W * W);
        hm[k].A = MatA{a11, a13, a33, a55};
    }
    return hm;
}

// fastest qP phase speed over the materials (sampled every half degree): the time band
// of the relaxations is a number of node spacings at this speed
inline double max_phase_speed(const ali_material* mats, int n_mats) {
    double vmax = 0.0;
    for (int k = 0; k < n_mats; ++k) {
        const ali_material& m = mats[k];
        const double a11 = m.c11 / m.rho, a13 = m.c13 / m.rho, a33 = m.c33 / m.rho, a55 = m.c55 / m.rho;
        for (int q = 0; q <= 180; ++q) {
            const double psi = q * (3.14159265358979323846 / 360.0);
            const double c = cos(2.0 * psi), sn = sin(2.0 * psi);
            const double lin = (a33 - a11) + (a11 + a33 - 2.0 * a55) * c;
            const double v2 = 0.25 * ((a11 + a33 + 2.0 * a55) + (a33 - a11) * c +
                                      sqrt(lin * lin + 4.0 * (a13 + a55) * (a13 + a55) * sn * sn));
            if (v2 > vmax * vmax) vmax = sqrt(v2);
        }
    }
    return vmax;
}

template <typename dst, typename srcT>
__global__ void k_convert(dst* __restrict__ out, const srcT* __restrict__ in, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (dst)in[i];
}

template <typename real>
__global__ void k_fill(real* __restrict__ p, int64_t n, real v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// flag bits of a tile: which parts of it need evaluation on its next visit
enum : uint32_t {
    TF_SELF = 1u,              // everything (first visit, or the previous visit hit the sweep cap)
    TF_HALO_L = 2u, TF_HALO_R = 4u, TF_HALO_U = 8u, TF_HALO_D = 16u,       // a halo side changed
    TF_HALO_UL = 32u, TF_HALO_UR = 64u, TF_HALO_DL = 128u, TF_HALO_DR = 256u, // a halo corner changed
    TF_MARK = 512u             // a neighbouring tile marked nodes of this tile (node mask)
};

template <typename real, typename mreal>
__device__ __forceinline__ void load_node_const(NodeConst<mreal, real>& nc, int64_t p,
                                                const mreal* __restrict__ geo,
                                                const real* __restrict__ fbt) {
    // both arrays come from the device allocator (256-byte aligned) and hold whole
    // per-node records of 8 and 4 values
    const mreal* g = static_cast<const mreal*>(__builtin_assume_aligned(geo, 32)) + GEO_N * p;
    const real* b = static_cast<const real*>(__builtin_assume_aligned(fbt, 32)) + 4 * p;
    mreal gv[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) gv[k] = g[k];
    nc.c2t = gv[0]; nc.s2t = gv[1];
    nc.P = gv[2]; nc.Q = gv[3]; nc.R = gv[4]; nc.K4 = gv[5];
#pragma unroll
    for (int d = 0; d < 4; ++d) nc.fb[d] = b[d];
}

// One field of a batch: a source in a medium.  Offsets count elements.
struct FieldDev {
    int nx, nz, ntx, ntz;
    double h;             // node spacing of the medium
    int64_t node_off;     // the medium's first node in the per-node arrays (materials, orientation)
    int64_t t_off;        // the field's first node in the per-field arrays (travel times)
    uint32_t unit_off;    // the field's first tile unit (flags, thresholds, node marks)
    uint32_t group_off;   // the field's first scheduler group (GROUP tiles each)
    int mat_off;          // the medium's first entry in the device material table
    int medium;
    int rec_off, n_rec;   // the medium's receivers (gradient calls)
    int obs_off;          // the field's first entry in per-receiver arrays
    int2 src;
    int part;             // the field's pass-list region
};

// One entry of a pass list: what a tile visit needs before its first load of field
// values, written by the scheduler so that the visit reads it in one round trip.
struct alignas(16) PassItem {
    uint32_t unit, bits;      // tile unit; the flag bits it was scheduled with
    int f, tx;                // field; tile column
    int tz, nx, nz;           // tile row; the field's grid
    uint32_t group_off;       // the field's first scheduler group
    int2 src;                 // the field's source node
    int64_t t_off;            // the field's first node in the per-field arrays
    int64_t node_off;         // the medium's first node in the per-node arrays
    int64_t pad1;
};
static_assert(sizeof(PassItem) == 64, "pass-list entries are four 16-byte vectors");

// The pass list is kept in LIST_PARTS regions: the fields are split into LIST_PARTS runs of
// consecutive fields (FieldDev::part), and each run appends its due tiles to its own
// region, reserving slots on the region's own counter.  A device-scope atomic on one
// address is served one at a time (~8 ns each): with one counter the reservations of a
// 4096-field batch queue behind each other, with 8 counters (each on its own 4 KiB page)
// only behind those of the same run.  Region r starts at slot part_base[r] of the list
// array (the tiles of the fields of the runs before it, so it can never overflow) and
// holds that pass's count of it.  The readers take the regions as one list, in region
// order (entry v of the pass is in region r when pre[r] <= v < pre[r + 1], pre being the
// running sum of the counts), so the list keeps its field order: the relaxation gives each
// die one contiguous eighth of it, and the fields of one medium, which share the per-node
// records, stay on one die's L2 (regions by field number mod 8 spread every medium over
// all dies and made the batch relaxation 1.6 % slower).
// The counter buffer of a solve holds CNT_WORDS words: the counters of even passes at
// word r * CNT_GAP, those of odd passes CNT_BLOCK words further, then the region offsets;
// one word per field follows them (the field has finished).
constexpr int LIST_PARTS = 8;
constexpr int CNT_GAP = 1024;
constexpr int CNT_BLOCK = LIST_PARTS * CNT_GAP;
constexpr int CNT_WORDS = 2 * CNT_BLOCK + LIST_PARTS;

// region of field f of n: LIST_PARTS runs of consecutive fields
inline int list_part_of(int64_t f, int64_t n) { return (int)(f * LIST_PARTS / n); }

// first slot of every list region for the fields of a call (FieldDev::part set)
inline std::vector<uint32_t> list_part_base(const std::vector<FieldDev>& fields) {
    std::vector<uint32_t> cap(LIST_PARTS, 0u), base(LIST_PARTS, 0u);
    for (size_t f = 0; f < fields.size(); ++f)
        cap[fields[f].part] += (uint32_t)(fields[f].ntx * fields[f].ntz);
    for (int r = 1; r < LIST_PARTS; ++r) base[r] = base[r - 1] + cap[r - 1];
    return base;
}

// Where one pass's entries sit: pre[r] entries precede region r (pre[LIST_PARTS]: all of
// them), base[r] is region r's first slot.  Read by each relaxation work-group at its start
// into scalar registers (uniform values), and copied to LDS for the lookups of later entries.
struct ListMap {
    uint32_t pre[LIST_PARTS + 1];
    uint32_t base[LIST_PARTS];
};

// The map of one pass from its counters (cnt: that pass's counter block) and the region
// offsets.  COHERENT: device-scope loads of the counters (a reader in the same launch as
// the schedulers).
template <bool COHERENT = false>
__device__ __forceinline__ ListMap read_list_map(const uint32_t* __restrict__ cnt,
                                                 const uint32_t* __restrict__ part_base) {
    ListMap m;
    m.pre[0] = 0u;
#pragma unroll
    for (int r = 0; r < LIST_PARTS; ++r) {
        uint32_t c;
        if constexpr (COHERENT)
            c = __builtin_amdgcn_readfirstlane(__hip_atomic_load(const_cast<uint32_t*>(cnt) + r * CNT_GAP,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        else
            c = cnt[r * CNT_GAP];
        m.base[r] = part_base[r];
        m.pre[r + 1] = m.pre[r] + c;
    }
    return m;
}

// copy of the map in LDS, written by one lane (the work-group synchronises before reading it)
__device__ __forceinline__ void put_list_map(ListMap& dst, const ListMap& m) {
    if ((threadIdx.x & 63u) == 0u) {
#pragma unroll
        for (int r = 0; r < LIST_PARTS; ++r) {
            dst.pre[r] = m.pre[r];
            dst.base[r] = m.base[r];
        }
        dst.pre[LIST_PARTS] = m.pre[LIST_PARTS];
    }
}

// slot in the list array of entry v (< pre[LIST_PARTS]) of the pass, from the LDS copy
__device__ __forceinline__ uint32_t list_slot(const ListMap& m, uint32_t v) {
    int r = 0;
#pragma unroll
    for (int q = 1; q < LIST_PARTS; ++q) r += v >= m.pre[q] ? 1 : 0;
    return m.base[r] + (v - m.pre[r]);
}

// the same from the map in registers: selects only (an indexed register array would be
// moved to scratch memory)
__device__ __forceinline__ uint32_t list_slot_reg(const ListMap& m, uint32_t v) {
    uint32_t s = m.base[0] + v;
#pragma unroll
    for (int q = 1; q < LIST_PARTS; ++q)
        if (v >= m.pre[q]) s = m.base[q] + (v - m.pre[q]);
    return s;
}

constexpr int SCHED_T = 256;  // work-items of a scheduler work-group (one group per field)
constexpr int SCHED_K = 8;    // scheduler groups per work-item held in registers
// the same in calls of more than DIRECT_ALL_UNITS tiles, where only fields of one span are
// read tile by tile: fewer registers (more resident scheduler work-groups) pay there
// (batch of 128 media: step 1.260 -> 1.249 s; 2 the same), while a smaller call, read tile
// by tile, would need two spans for fields of 1025-2048 tiles (64 fields of 512 x 512:
// forward +2.8 % with 4)
constexpr int SCHED_K_LARGE = 4;
// due groups a scheduler wave expands at once (batch step: 2 and 4 save 0.9 %, 8 nothing)
constexpr int SCHED_UNROLL = 2;
// Tiles of one scheduler group.  The scheduler reads a summary per group (the OR of its
// tiles' flags and the nearest of its tiles' keys) and only expands the groups that are
// due, one wave per group and one tile per lane, instead of reading every tile of every
// field on every pass.
constexpr int GROUP = 64;

__host__ __device__ inline uint32_t field_groups(int ntiles) { return (uint32_t)((ntiles + GROUP - 1) / GROUP); }

// Group summaries of the tile keys, kept exact with integer atomics on the key's bit
// pattern: keys are non-negative times, +inf (ascending: none) or -inf (descending: none),
// which order like their patterns read as signed integers.
__device__ __forceinline__ void key_min(double* p, double v) {
    atomicMin(reinterpret_cast<long long*>(p), (long long)__double_as_longlong(v));
}
__device__ __forceinline__ void key_min(float* p, float v) { atomicMin(reinterpret_cast<int*>(p), __float_as_int(v)); }
__device__ __forceinline__ void key_max(double* p, double v) {
    atomicMax(reinterpret_cast<long long*>(p), (long long)__double_as_longlong(v));
}
__device__ __forceinline__ void key_max(float* p, float v) { atomicMax(reinterpret_cast<int*>(p), __float_as_int(v)); }

// flag tile t (index within its field) and its scheduler group (gflag == NULL: no field
// of the call is scheduled by groups)
__device__ __forceinline__ void flag_tile(uint32_t* __restrict__ flags, uint32_t* __restrict__ gflag, uint32_t unit_off,
                                          uint32_t group_off, int t, uint32_t bits) {
    atomicOr(&flags[unit_off + (uint32_t)t], bits);
    if (gflag) atomicOr(&gflag[group_off + (uint32_t)(t / GROUP)], 1u);
}

// Fields of up to this many tiles have their tiles read directly by the scheduler, when
// the whole call has at most DIRECT_ALL_UNITS tiles; otherwise only fields of up to one
// scheduler span are (the group summaries spare the larger ones a full read per pass).
constexpr int64_t DIRECT_ALL_UNITS = (int64_t)1 << 18;
inline int direct_tiles_for(int64_t n_units, int span) { return n_units <= DIRECT_ALL_UNITS ? (1 << 30) : span; }
inline int sched_k_for(int64_t n_units) { return n_units <= DIRECT_ALL_UNITS ? SCHED_K : SCHED_K_LARGE; }

// Pass scheduler of field f, run by one work-group of NT work-items (a multiple of 64;
// every work-item of the group calls it), each holding K groups at a time.  s_due:
// NT * K words of LDS.
// Ascending (DESC = false, travel times): key[t] is the smallest value tile t rejected
// (+inf: none); the threshold rises by step each pass, and a tile is due when it is
// flagged or its key is at or below the threshold.  Descending (DESC = true, adjoint):
// key[t] is the largest key still pending in tile t (-inf: none); the threshold falls by
// step, and a tile is due when flagged or its key is at or above the threshold.  When no
// tile is due the threshold jumps to the nearest key.  Due tiles have their flags cleared
// and their keys reset (their visit in this pass writes them again) and are appended to
// the field's region of the pass list (part_base), counted by the region's counter in the
// block cnt_cur; the block cnt_next (the next pass's counters) is cleared here.  A field
// with nothing flagged and no pending key sets done[f] (cleared by the caller before the
// first pass) and is skipped from then on.
// Fields of at most direct_tiles tiles are read tile by tile (in spans of NT * K); larger
// ones through the group summaries gflag / gkey, which are exact: a group is due exactly
// when one of its tiles is; an expanded group's summary is rebuilt from its tiles that
// stay.
template <bool DESC, typename real, int NT, int K = SCHED_K>
__device__ __forceinline__ void schedule_field(int f, const FieldDev* __restrict__ fields, int advance,
                                               const real* __restrict__ step, uint32_t* __restrict__ flags,
                                               real* __restrict__ key, uint32_t* __restrict__ gflag,
                                               real* __restrict__ gkey, real* __restrict__ theta,
                                               PassItem* __restrict__ list, uint32_t* __restrict__ cnt_cur,
                                               uint32_t* __restrict__ cnt_next,
                                               const uint32_t* __restrict__ part_base, uint32_t* __restrict__ done,
                                               uint32_t* __restrict__ s_due, int direct_tiles) {
    constexpr int NW = NT / 64;
    constexpr int SPAN = NT * K;
    __shared__ real s_key[NW];
    __shared__ unsigned s_act[NW], s_cnt[NW], s_gcnt[NW];
    __shared__ uint32_t s_base;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (f == 0 && tid < LIST_PARTS) cnt_next[tid * CNT_GAP] = 0u;
    // a field that had nothing flagged and no pending key has finished: only its own tile
    // visits could bring new work, and it has none
    if (done[f]) return;
    const FieldDev fd = fields[f];
    const int ntiles = fd.ntx * fd.ntz;
    const int ngroups = (int)field_groups(ntiles);
    uint32_t* __restrict__ fl = flags + fd.unit_off;
    real* __restrict__ ky = key + fd.unit_off;
    uint32_t* __restrict__ gf = gflag + fd.group_off;
    real* __restrict__ gk = gkey + fd.group_off;
    const real inf = dinf<real>();
    const real none = DESC ? -inf : inf;
    uint32_t* __restrict__ rcnt = cnt_cur + fd.part * CNT_GAP;   // the field's region
    PassItem* __restrict__ rlist = list + part_base[fd.part];
    real th = theta[f];
    if (advance) th = DESC ? th - step[f] : th + step[f];
    auto due_key = [&](real k) { return k != none && (DESC ? k >= th : k <= th); };

    if (ntiles <= direct_tiles) {
        // read tile by tile, in spans of NT * K (a single span is read once)
        uint32_t fv[K];
        real kv[K];
        bool act = false;
        real near = none;
        for (int b0 = 0; b0 < ntiles; b0 += SPAN) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int t = b0 + tid + NT * k;
                fv[k] = t < ntiles ? fl[t] : 0u;
                kv[k] = t < ntiles ? ky[t] : none;
                act |= fv[k] != 0u || due_key(kv[k]);
                near = DESC ? (kv[k] > near ? kv[k] : near) : (kv[k] < near ? kv[k] : near);
            }
        }
        const bool wact = __ballot(act) != 0ull;
        for (int o = 32; o > 0; o >>= 1) {
            const real r = __shfl_xor(near, o);
            near = DESC ? (r > near ? r : near) : (r < near ? r : near);
        }
        if (lane == 0) { s_key[wv] = near; s_act[wv] = wact ? 1u : 0u; }
        __syncthreads();
        bool any = false;
        near = none;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            any |= s_act[w] != 0u;
            near = DESC ? (s_key[w] > near ? s_key[w] : near) : (s_key[w] < near ? s_key[w] : near);
        }
        if (!any && near != none && (DESC ? near < th : near > th)) th = near;   // idle: jump
        if (!any && near == none && tid == 0) done[f] = 1u;
        if (tid == 0) theta[f] = th;
        for (int b0 = 0; b0 < ntiles; b0 += SPAN) {
            if (ntiles > SPAN) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int t = b0 + tid + NT * k;
                    fv[k] = t < ntiles ? fl[t] : 0u;
                    kv[k] = t < ntiles ? ky[t] : none;
                }
            }
            unsigned dmask = 0u;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (fv[k] != 0u || due_key(kv[k])) dmask |= 1u << k;
            const unsigned mine = (unsigned)__popc(dmask);
            unsigned incl = mine;
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned v = __shfl_up(incl, o);
                if (lane >= o) incl += v;
            }
            if (lane == 63) s_cnt[wv] = incl;
            __syncthreads();
            unsigned wbase = 0u, total = 0u;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                wbase += w < wv ? s_cnt[w] : 0u;
                total += s_cnt[w];
            }
            if (tid == 0) s_base = total ? atomicAdd(rcnt, total) : 0u;
            __syncthreads();
            uint32_t pos = s_base + wbase + incl - mine;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!((dmask >> k) & 1u)) continue;
                const int t = b0 + tid + NT * k;
                fl[t] = 0u;
                ky[t] = none;
                PassItem it;
                it.unit = fd.unit_off + (uint32_t)t;
                it.bits = fv[k];
                it.f = f;
                it.tx = t % fd.ntx;
                it.tz = t / fd.ntx;
                it.nx = fd.nx;
                it.nz = fd.nz;
                it.group_off = fd.group_off;
                it.src = fd.src;
                it.t_off = fd.t_off;
                it.node_off = fd.node_off;
                it.pad1 = 0;
                rlist[pos++] = it;
            }
            __syncthreads();     // s_cnt and s_base are reused by the next span and field
        }
        return;
    }

    // is any group due at this threshold, and which key is nearest?
    uint32_t fv[K];
    real kv[K];
    bool act = false;
    real near = none;
    for (int b0 = 0; b0 < ngroups; b0 += SPAN) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int g = b0 + tid + NT * k;
            fv[k] = g < ngroups ? gf[g] : 0u;
            kv[k] = g < ngroups ? gk[g] : none;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            act |= fv[k] != 0u || due_key(kv[k]);
            near = DESC ? (kv[k] > near ? kv[k] : near) : (kv[k] < near ? kv[k] : near);
        }
    }
    const bool wact = __ballot(act) != 0ull;
    for (int o = 32; o > 0; o >>= 1) {
        const real r = __shfl_xor(near, o);
        near = DESC ? (r > near ? r : near) : (r < near ? r : near);
    }
    if (lane == 0) { s_key[wv] = near; s_act[wv] = wact ? 1u : 0u; }
    __syncthreads();
    bool any = false;
    near = none;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        any |= s_act[w] != 0u;
        near = DESC ? (s_key[w] > near ? s_key[w] : near) : (s_key[w] < near ? s_key[w] : near);
    }
    if (!any && near != none && (DESC ? near < th : near > th)) th = near;   // idle: jump
    if (!any && near == none && tid == 0) done[f] = 1u;
    if (tid == 0) theta[f] = th;

    for (int b0 = 0; b0 < ngroups; b0 += SPAN) {
        // the due groups of this span, compacted in LDS
        if (ngroups > SPAN) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int g = b0 + tid + NT * k;
                fv[k] = g < ngroups ? gf[g] : 0u;
                kv[k] = g < ngroups ? gk[g] : none;
            }
        }
        unsigned dmask = 0u;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (fv[k] != 0u || due_key(kv[k])) dmask |= 1u << k;
        const unsigned mine = (unsigned)__popc(dmask);
        unsigned incl = mine;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        if (lane == 63) s_gcnt[wv] = incl;
        __syncthreads();
        unsigned gbase = 0u, ndue = 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            gbase += w < wv ? s_gcnt[w] : 0u;
            ndue += s_gcnt[w];
        }
        uint32_t gpos = gbase + incl - mine;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if ((dmask >> k) & 1u) s_due[gpos++] = (uint32_t)(b0 + tid + NT * k);
        __syncthreads();
        // count the due tiles (one wave per due group, one tile per lane; each wave loads
        // the flags and keys of SCHED_UNROLL of its groups before it uses any of them)
        constexpr int U = SCHED_UNROLL;
        unsigned wcount = 0u;
        for (unsigned q = wv; q < ndue; q += U * NW) {
            uint32_t fu[U];
            real ku[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const unsigned qu = q + (unsigned)(u * NW);
                const int t = qu < ndue ? (int)s_due[qu] * GROUP + lane : ntiles;
                fu[u] = t < ntiles ? fl[t] : 0u;
                ku[u] = t < ntiles ? ky[t] : none;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) wcount += (unsigned)__popcll(__ballot(fu[u] != 0u || due_key(ku[u])));
        }
        if (lane == 0) s_cnt[wv] = wcount;
        __syncthreads();
        unsigned wbase = 0u, total = 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            wbase += w < wv ? s_cnt[w] : 0u;
            total += s_cnt[w];
        }
        if (tid == 0) s_base = total ? atomicAdd(rcnt, total) : 0u;
        __syncthreads();
        // append them in the same order, reset their flags and keys, rebuild the summaries
        uint32_t pos = s_base + wbase;
        for (unsigned q = wv; q < ndue; q += U * NW) {
            uint32_t fu[U];
            real ku[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const unsigned qu = q + (unsigned)(u * NW);
                const int t = qu < ndue ? (int)s_due[qu] * GROUP + lane : ntiles;
                fu[u] = t < ntiles ? fl[t] : 0u;
                ku[u] = t < ntiles ? ky[t] : none;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const unsigned qu = q + (unsigned)(u * NW);
                if (qu >= ndue) break;
                const int g = (int)s_due[qu];
                const int t = g * GROUP + lane;
                const uint32_t tf = fu[u];
                const real tk = ku[u];
                const bool d = t < ntiles && (tf != 0u || due_key(tk));
                const unsigned long long m = __ballot(d);
                if (d) {
                    fl[t] = 0u;
                    ky[t] = none;
                    PassItem it;
                    it.unit = fd.unit_off + (uint32_t)t;
                    it.bits = tf;
                    it.f = f;
                    it.tx = t % fd.ntx;
                    it.tz = t / fd.ntx;
                    it.nx = fd.nx;
                    it.nz = fd.nz;
                    it.group_off = fd.group_off;
                    it.src = fd.src;
                    it.t_off = fd.t_off;
                    it.node_off = fd.node_off;
                    it.pad1 = 0;
                    rlist[pos + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = it;
                }
                pos += (uint32_t)__popcll(m);
                real r = d ? none : tk;
                for (int o = 32; o > 0; o >>= 1) {
                    const real r2 = __shfl_xor(r, o);
                    r = DESC ? (r2 > r ? r2 : r) : (r2 < r ? r2 : r);
                }
                if (lane == 0) { gk[g] = r; gf[g] = 0u; }
            }
        }
        __syncthreads();     // s_cnt, s_gcnt, s_due and s_base are reused by the next span
    }
}

// field f owning tile unit u (fields are stored in unit order)
__device__ __forceinline__ int field_of_unit(const FieldDev* __restrict__ fields, int n_fields, uint32_t u) {
    int lo = 0, hi = n_fields - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fields[mid].unit_off <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// What the forward driver leaves on the device for a following adjoint on the same
// stream: the field table, per-material and per-node constants, and their host copies.
template <typename real, typename mreal> struct ForwardState {
    const MatDev<mreal>* mats = nullptr;
    const mreal* geo = nullptr;      // [medium nodes][2] cos 2theta, sin 2theta
    const real* fbt = nullptr;       // [medium nodes][4] straight-ray times to 8-neighbours
    const mreal* vt = nullptr;       // velocity-table mode: phase speed / h tables of the device materials
    const double* gt = nullptr;      // and their group-speed tables (VT_N entries each), else NULL
    const FieldDev* fields = nullptr;
    std::vector<FieldDev> hfields;
    std::vector<uint32_t> part_base;       // first slot of every pass-list region
    std::vector<int> medium_first_field;   // per medium, then the total
    std::vector<double> vmax;        // fastest phase speed per medium
    int64_t n_units = 0, n_groups = 0, field_nodes = 0;
};

// Validates a batch (media, materials for the wave, sources and, when recv != NULL,
// receivers).
ali_status validate_batch(ali_handle* H, const ali_medium* media, int32_t n_media, const ali_material* mats,
                          int32_t n_mats, const void* d_mat_id, const void* d_orient, const ali_node* srcs,
                          const ali_node* recv, int wave = ALI_WAVE_QP);

// Forward solve of every field of a batch into the working field d_T (fields in medium
// order, each [nz][nx]; type real).  Validates its arguments, records H->ev0 at its start,
// synchronises the stream before returning and fills every stats field except `ms`.
// Instantiated for <double, float, float>, <float, float, float>, <double, double, float>
// and <double, double, double>.
// Seeded mode (d_fixmask != NULL): the fields start from the values already in d_T, the
// nodes whose bit is set in d_fixmask keep their values and every other node must hold
// +inf; there is no source box.  d_fixmask has NODE_WORDS words per tile unit, units
// numbered as unit_offsets() does, bit (j % TZ) * TX + i % TX for node (i, j) of the tile.
template <typename real, typename mreal, typename oreal>
ali_status solve_fields(ali_handle* H, const ali_medium* media, int32_t n_media, const ali_material* mats,
                        int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient, const ali_node* srcs,
                        const ali_node* recv, const ali_options& opt, real* d_T, ali_solve_stats* stats,
                        ForwardState<real, mreal>* fs, const uint32_t* d_fixmask = nullptr);

// first tile unit of every field of a batch (fields in medium order, then source order)
inline std::vector<uint32_t> unit_offsets(const ali_medium* media, int32_t n_media) {
    std::vector<uint32_t> off;
    uint32_t u = 0;
    for (int m = 0; m < n_media; ++m) {
        const uint32_t per = (uint32_t)(((media[m].grid.nx + TX - 1) / TX) * ((media[m].grid.nz + TZ - 1) / TZ));
        for (int k = 0; k < media[m].n_src; ++k) {
            off.push_back(u);
            u += per;
        }
    }
    off.push_back(u);
    return off;
}

// number of fields and field nodes of a batch (after validation)
inline void batch_sizes(const ali_medium* media, int32_t n_media, int64_t* n_fields, int64_t* field_nodes) {
    int64_t f = 0, n = 0;
    for (int m = 0; m < n_media; ++m) {
        f += media[m].n_src;
        n += (int64_t)media[m].n_src * media[m].grid.nx * media[m].grid.nz;
    }
    *n_fields = f;
    *field_nodes = n;
}

// the single-medium entry points as a batch of one
inline ali_medium single_medium(const ali_grid* g, int32_t n_mats, int32_t n_src, int32_t n_rec) {
    ali_medium m;
    m.grid = *g;
    m.mat_offset = 0;
    m.n_mats = n_mats;
    m.node_offset = 0;
    m.src_offset = 0;
    m.n_src = n_src;
    m.rec_offset = 0;
    m.n_rec = n_rec;
    return m;
}

}  // namespace ali
