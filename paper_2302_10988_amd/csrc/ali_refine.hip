// ali_refine.hip -- nested fine grids around each source (paper Section 4.4, propagation
// around the source), gfx950.
//
// Every source gets a sequence of grids centred on its node, finest first; level l has
// density d_l (nodes per working-grid spacing, odd, each divisible by the next) and is
// used out to radius r_l working cells (Chebyshev).  Per level, for all sources at once:
//   1. k_level_medium: the level grid of each source takes the material and orientation
//      of the nearest working-grid node (odd densities make it unique);
//   2. seeds: on the finest level, straight rays at the source material's group speed in
//      the square of half-width `start_half_width` cells around the source (by default
//      the source node's own cell, where the material cannot change); on later levels the
//      nodes that coincide with known nodes of the previous level;
//   3. the relaxation of the level's fields (one medium per source, one field each) with
//      those seeds fixed: the same kernels as every forward solve;
//   4. k_level_stop: per source, the earliest time beyond r_l.  A heap march would switch
//      grids at that node, so the nodes known at the switch are those strictly earlier:
//      the fixed point of the level restricted to them equals the march (a node's value
//      depends only on earlier nodes).
// A level grid spans r_l d_l + 2 of its cells around the source: nodes earlier than the
// switch have all their earlier neighbours inside the radius, the switching node lies
// within 2 cells of it, and an update reads only earlier neighbours, so a larger grid
// would change none of the values that are handed on.
// The working grid itself is the last level: all sources' fields in one batch, seeded
// from the coarsest fine level.
//
// Section 4.5's subgrid size s (odd) refines the whole medium s-fold first (k_subgrid_medium,
// nearest node again); the levels above then run on that grid, and k_subgrid_pick returns
// every s-th node of its fields.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <chrono>
#include <string>
#include <type_traits>
#include <vector>

#include "ali_solve.hpp"

namespace ali {

// one source's grid at one level: node (a, b) of the level sits at working-grid position
// (si + a / d, sj + b / d); a in [a_lo, a_lo + nx), b in [b_lo, b_lo + nz)
struct LevelDev {
    int a_lo, b_lo, nx, nz;
    int si, sj;               // the source node on the working grid
    int d;                    // density relative to the working grid
    int stop;                 // level cells: the level is used out to this Chebyshev radius
    int64_t node_off;         // first node in the level's per-node arrays
    int64_t t_off;            // first node in the level's field array
    uint32_t unit_off;        // first tile unit
    int ntx;
    // the source's working medium: its first node, row length, spacing and materials
    int64_t w_node;
    int nx_w;
    int mat_off, n_mats;
    double h_w;
};

// nearest multiple index of a / d for odd d (a half never occurs)
__device__ __forceinline__ int near_div(int a, int d) {
    const int q = a + (d - 1) / 2;
    return q >= 0 ? q / d : -((-q + d - 1) / d);
}

template <typename oreal>
__global__ void k_level_medium(const LevelDev* __restrict__ lv, const uint8_t* __restrict__ mat_w,
                               const oreal* __restrict__ ori_w, const float* __restrict__ A_w,
                               uint8_t* __restrict__ mat_l, oreal* __restrict__ ori_l, float* __restrict__ A_l) {
    const LevelDev L = lv[blockIdx.y];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)L.nx * L.nz) return;
    const int a = L.a_lo + (int)(q % L.nx), b = L.b_lo + (int)(q / L.nx);
    const int64_t p = L.w_node + (int64_t)(L.sj + near_div(b, L.d)) * L.nx_w + (L.si + near_div(a, L.d));
    mat_l[L.node_off + q] = mat_w[p];
    ori_l[L.node_off + q] = ori_w[p];
    if (A_w)
        for (int k = 0; k < 4; ++k) A_l[4 * (L.node_off + q) + k] = A_w[4 * p + k];
}

__device__ __forceinline__ void set_fixed(uint32_t* __restrict__ fixmask, const LevelDev& L, int i, int j) {
    const uint32_t unit = L.unit_off + (uint32_t)((j / TZ) * L.ntx + i / TX);
    const int bit = (j % TZ) * TX + (i % TX);
    atomicOr(&fixmask[(int64_t)unit * NODE_WORDS + (bit >> 5)], 1u << (bit & 31));
}

// finest level: straight rays from the source inside |a|, |b| < half * d, +inf elsewhere
template <typename real, typename oreal>
__global__ void k_seed_start(const LevelDev* __restrict__ lv, double half, const MatA* __restrict__ A,
                             const double* __restrict__ gt, const uint8_t* __restrict__ mat_w, const oreal* __restrict__ ori_w,
                             const float* __restrict__ A_w, real* __restrict__ T, uint32_t* __restrict__ fixmask) {
    const LevelDev L = lv[blockIdx.y];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)L.nx * L.nz) return;
    const int i = (int)(q % L.nx), j = (int)(q / L.nx);
    const int a = L.a_lo + i, b = L.b_lo + j;
    real v = dinf<real>();
    const double lim = half * L.d;
    if (fabs((double)a) < lim && fabs((double)b) < lim) {
        double t = 0.0;
        if (a != 0 || b != 0) {
            const int64_t ps = L.w_node + (int64_t)L.sj * L.nx_w + L.si;
            const double phi = atan2((double)b, (double)a) - (double)ori_w[ps];
            // an id outside the table is reported by the solve's own check; read a valid entry
            const int mid = L.mat_off + (mat_w[ps] < L.n_mats ? mat_w[ps] : 0);
            const MatA As = A_w ? MatA{(double)A_w[4 * ps], (double)A_w[4 * ps + 1], (double)A_w[4 * ps + 2],
                                       (double)A_w[4 * ps + 3]}
                                : A[mid];
            const double V = gt ? group_speed_tab(gt + mid * VT_N, phi) : group_speed(As, phi);
            t = sqrt((double)a * a + (double)b * b) * (L.h_w / L.d) / V;
        }
        v = (real)t;
        set_fixed(fixmask, L, i, j);
    }
    T[L.t_off + q] = v;
}

// later levels: nodes that coincide with nodes of the finer level known before its stop
template <typename real>
__global__ void k_seed_transfer(const LevelDev* __restrict__ fine, const real* __restrict__ Tf,
                                const real* __restrict__ tstop, const LevelDev* __restrict__ lv,
                                real* __restrict__ T, uint32_t* __restrict__ fixmask) {
    const LevelDev L = lv[blockIdx.y];
    const LevelDev F = fine[blockIdx.y];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)L.nx * L.nz) return;
    const int i = (int)(q % L.nx), j = (int)(q / L.nx);
    const int k = F.d / L.d;
    const int fa = (L.a_lo + i) * k - F.a_lo, fb = (L.b_lo + j) * k - F.b_lo;
    real v = dinf<real>();
    if (fa >= 0 && fb >= 0 && fa < F.nx && fb < F.nz) {
        const real t = Tf[F.t_off + (int64_t)fb * F.nx + fa];
        if (t < tstop[blockIdx.y]) {
            v = t;
            set_fixed(fixmask, L, i, j);
        }
    }
    T[L.t_off + q] = v;
}

// per source: the smallest time farther than `stop` level cells from the source
template <typename real>
__global__ void k_level_stop(const LevelDev* __restrict__ lv, const real* __restrict__ T, real* __restrict__ tstop) {
    const LevelDev L = lv[blockIdx.x];
    real m = dinf<real>();
    for (int64_t q = threadIdx.x; q < (int64_t)L.nx * L.nz; q += blockDim.x) {
        const int a = L.a_lo + (int)(q % L.nx), b = L.b_lo + (int)(q / L.nx);
        if (abs(a) > L.stop || abs(b) > L.stop) {
            const real t = T[L.t_off + q];
            m = t < m ? t : m;
        }
    }
    __shared__ real red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x + s] < red[threadIdx.x] ? red[threadIdx.x + s]
                                                                                             : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) tstop[blockIdx.x] = red[0];
}

// the s-fold grid's medium: node (a, b) takes the material and orientation of working node
// (nearest a / s, nearest b / s)
template <typename oreal>
__global__ void k_subgrid_medium(int nx, int nx_s, int64_t n_s, int s, const uint8_t* __restrict__ mat,
                                 const oreal* __restrict__ ori, const float* __restrict__ A,
                                 uint8_t* __restrict__ mat_s, oreal* __restrict__ ori_s, float* __restrict__ A_s) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_s) return;
    const int a = (int)(q % nx_s), b = (int)(q / nx_s);
    const int64_t p = (int64_t)near_div(b, s) * nx + near_div(a, s);
    mat_s[q] = mat[p];
    ori_s[q] = ori[p];
    if (A)
        for (int k = 0; k < 4; ++k) A_s[4 * q + k] = A[4 * p + k];
}

// the fields at the working nodes: node (i, j) of field k is node (s i, s j) of the s-fold
// field k
template <typename outreal, typename real>
__global__ void k_subgrid_pick(int nx, int64_t nw, int64_t n_out, int nx_s, int64_t n_s, int s,
                               const real* __restrict__ Ts, outreal* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_out) return;
    const int64_t k = q / nw, r = q % nw;
    const int i = (int)(r % nx), j = (int)(r / nx);
    out[q] = (outreal)Ts[k * n_s + (int64_t)j * s * nx_s + (int64_t)i * s];
}

// the level record of a field of medium m with its source and its working medium filled in
// (the batch's fields come in medium order, then source order)
static LevelDev working_level(const ali_medium& m, const ali_node& src) {
    LevelDev L{};
    L.si = src.i; L.sj = src.j;
    L.w_node = m.node_offset;
    L.nx_w = m.grid.nx;
    L.mat_off = m.mat_offset;
    L.n_mats = m.n_mats;
    L.h_w = m.grid.h;
    return L;
}

// host: one level's grids (clipped to each field's working grid) and their offsets; one
// level medium per field
static std::vector<LevelDev> level_grids(const ali_medium* bm, int n_bm, const ali_node* srcs, int d, int W,
                                         int stop, std::vector<ali_medium>& media, std::vector<ali_node>& lsrc) {
    std::vector<LevelDev> lv;
    media.clear();
    lsrc.clear();
    int64_t node = 0;
    uint32_t unit = 0;
    for (int m = 0; m < n_bm; ++m) {
        const ali_grid& g = bm[m].grid;
        for (int k = 0; k < bm[m].n_src; ++k) {
            const ali_node& sn = srcs[bm[m].src_offset + k];
            LevelDev L = working_level(bm[m], sn);
            const int si = sn.i, sj = sn.j;
            L.d = d; L.stop = stop;
            L.a_lo = std::max(-W, -si * d);
            const int a_hi = std::min(W, (g.nx - 1 - si) * d);
            L.b_lo = std::max(-W, -sj * d);
            const int b_hi = std::min(W, (g.nz - 1 - sj) * d);
            L.nx = a_hi - L.a_lo + 1;
            L.nz = b_hi - L.b_lo + 1;
            L.node_off = node;
            L.t_off = node;              // one field per level medium
            L.unit_off = unit;
            L.ntx = (L.nx + TX - 1) / TX;
            ali_medium lm{};
            lm.grid.nx = L.nx; lm.grid.nz = L.nz; lm.grid.h = g.h / d;
            lm.mat_offset = bm[m].mat_offset; lm.n_mats = bm[m].n_mats;
            lm.node_offset = node;
            lm.src_offset = (int32_t)lv.size(); lm.n_src = 1;
            lm.rec_offset = 0; lm.n_rec = 0;
            media.push_back(lm);
            lsrc.push_back(ali_node{-L.a_lo, -L.b_lo});
            lv.push_back(L);
            node += (int64_t)L.nx * L.nz;
            unit += (uint32_t)(L.ntx * ((L.nz + TZ - 1) / TZ));
        }
    }
    return lv;
}

static void add_stats(ali_solve_stats& acc, const ali_solve_stats& s) {
    acc.node_updates += s.node_updates;
    acc.stencil_evals += s.stencil_evals;
    acc.tile_visits += s.tile_visits;
    acc.outer_iters += s.outer_iters;
    acc.relax_ms += s.relax_ms;
    acc.converged = acc.converged && s.converged;
}

// the nested grids of every source of a batch of working grids (a caller's medium or its
// s-fold refinement, or the media of a batch); one relaxation per level for all fields
// mreal: the wavefront math of the fine grids; wmreal: that of the working grid
template <typename real, typename mreal, typename wmreal, typename oreal, typename outreal>
static ali_status levels_impl(ali_handle* H, const ali_medium* bm, int32_t n_bm, const ali_material* mats,
                              int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient, const ali_node* srcs,
                              const ali_options& opt, const ali_refine& ref, outreal* d_out,
                              ali_solve_stats* stats, std::chrono::steady_clock::time_point t0) {
    if (!d_out) return H->fail(ALI_EINVAL, "d_T is NULL");
    ali_status st = validate_batch(H, bm, n_bm, mats, n_mats, d_mat_id, d_orient, srcs, nullptr, opt.wave);
    if (st != ALI_OK) return st;
    int64_t n_fields64 = 0, NF = 0;
    batch_sizes(bm, n_bm, &n_fields64, &NF);
    const int n_src = (int)n_fields64;      // one level grid per field
    const int nl = ref.n_levels;
    if (nl < 0 || nl > ALI_MAX_LEVELS) return H->fail(ALI_EINVAL, "n_levels out of range [0, ALI_MAX_LEVELS]");
    if (!(ref.start_half_width > 0.0) || !(ref.start_half_width <= 64.0))
        return H->fail(ALI_EINVAL, "start_half_width out of range (0, 64]");
    for (int l = 0; l < nl; ++l) {
        const int next = l + 1 < nl ? ref.density[l + 1] : 1;
        if (ref.density[l] < 3 || ref.density[l] % 2 == 0 || ref.density[l] > 255 || ref.density[l] % next != 0)
            return H->fail(ALI_EINVAL, "densities must be odd, in [3, 255], each divisible by the next");
        if (ref.radius[l] < 0 || (l > 0 && ref.radius[l] < ref.radius[l - 1]))
            return H->fail(ALI_EINVAL, "radii must be >= 0 and non-decreasing");
        if ((int64_t)ref.radius[l] * ref.density[l] + 2 > 4096)
            return H->fail(ALI_EINVAL, "a fine grid would exceed 8193 nodes per side");
    }
    if (nl > 0 && ref.start_half_width > ref.radius[0] + 1)
        return H->fail(ALI_EINVAL, "start_half_width exceeds the finest grid");
    if (set_device(H) != ALI_OK) return ALI_EDEVICE;
    hipStream_t S = H->stream;
    const int B = 256;

    // material table for the straight rays (A = C / rho)
    const std::vector<ali_material> wm = wave_materials(mats, n_mats, opt.wave);
    std::vector<MatA> hA(n_mats);
    for (int k = 0; k < n_mats; ++k)
        hA[k] = MatA{wm[k].c11 / wm[k].rho, wm[k].c13 / wm[k].rho, wm[k].c33 / wm[k].rho, wm[k].c55 / wm[k].rho};
    void *d_A = nullptr, *d_stop = nullptr, *d_fm = nullptr;
    if (!H->scratch("ref_A", sizeof(MatA) * n_mats, &d_A) || !H->scratch("ref_stop", sizeof(real) * n_src, &d_stop))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    HIPCK(H, hipMemcpyAsync(d_A, hA.data(), sizeof(MatA) * n_mats, hipMemcpyHostToDevice, S));
    // velocity-table mode: the straight rays take the group-speed table
    void* d_gt = nullptr;
    if (opt.velocity == ALI_VEL_TABLE) {
        if (!H->scratch("ref_gt", sizeof(double) * VT_N * n_mats, &d_gt))
            return H->fail(ALI_ENOMEM, "device scratch allocation failed");
        hipLaunchKernelGGL((k_vtables<double>), dim3((unsigned)n_mats), dim3(128), 0, S, (const MatA*)d_A,
                           (const double*)nullptr, n_mats, (double*)nullptr, (double*)d_gt);
    }

    ali_solve_stats acc{};
    acc.converged = 1;
    // the working level: the batch's own fields
    std::vector<LevelDev> wl;
    {
        const std::vector<uint32_t> uoff = unit_offsets(bm, n_bm);
        int64_t t = 0;
        for (int m = 0; m < n_bm; ++m)
            for (int k = 0; k < bm[m].n_src; ++k) {
                LevelDev L = working_level(bm[m], srcs[bm[m].src_offset + k]);
                L.d = 1; L.stop = -1;
                L.a_lo = -L.si; L.b_lo = -L.sj; L.nx = bm[m].grid.nx; L.nz = bm[m].grid.nz;
                L.node_off = bm[m].node_offset; L.t_off = t;
                L.unit_off = uoff[wl.size()];
                L.ntx = (L.nx + TX - 1) / TX;
                wl.push_back(L);
                t += (int64_t)L.nx * L.nz;
            }
    }
    constexpr bool same_out = std::is_same<real, outreal>::value;
    std::vector<LevelDev> prev;
    const real* Tprev = nullptr;
    const LevelDev* dprev = nullptr;
    for (int l = 0; l <= nl; ++l) {
        const bool last = l == nl;
        const int d = last ? 1 : ref.density[l];
        std::vector<ali_medium> media;
        std::vector<ali_node> lsrc;
        std::vector<LevelDev> lv;
        const uint8_t* mid = d_mat_id;
        const oreal* ori = d_orient;
        real* T = nullptr;
        int64_t nodes = 0, units = 0;
        if (!last) {
            lv = level_grids(bm, n_bm, srcs, d, ref.radius[l] * d + 2, ref.radius[l] * d, media, lsrc);
            nodes = lv.back().node_off + (int64_t)lv.back().nx * lv.back().nz;
            units = unit_offsets(media.data(), n_src).back();
        } else {
            // the working grids: the batch's media and sources as given
            media.assign(bm, bm + n_bm);
            lsrc.clear();
            lv = wl;
            nodes = NF;
            units = unit_offsets(bm, n_bm).back();
        }
        const std::string pp = std::to_string(l & 1);
        void *d_lv = nullptr, *d_T = nullptr, *d_mid = nullptr, *d_ori = nullptr, *d_nA = nullptr;
        // per-node stiffness: the level grids take the nearest node's, as the material
        ali_options lopt = opt;
        if (!H->scratch(("ref_lv" + pp).c_str(), sizeof(LevelDev) * n_src, &d_lv) ||
            !H->scratch("ref_fm", sizeof(uint32_t) * NODE_WORDS * units, &d_fm))
            return H->fail(ALI_ENOMEM, "device scratch allocation failed");
        if (last && same_out) {
            d_T = (void*)d_out;
        } else if (!H->scratch(("ref_T" + pp).c_str(), sizeof(real) * nodes, &d_T)) {
            return H->fail(ALI_ENOMEM, "device scratch allocation failed");
        }
        T = (real*)d_T;
        HIPCK(H, hipMemcpyAsync(d_lv, lv.data(), sizeof(LevelDev) * n_src, hipMemcpyHostToDevice, S));
        HIPCK(H, hipMemsetAsync(d_fm, 0, sizeof(uint32_t) * NODE_WORDS * units, S));
        int64_t maxn = 0;
        for (const LevelDev& L : lv) maxn = std::max(maxn, (int64_t)L.nx * L.nz);
        const dim3 g2((unsigned)((maxn + B - 1) / B), (unsigned)n_src);
        if (!last) {
            if (!H->scratch(("ref_mid" + pp).c_str(), nodes, &d_mid) ||
                !H->scratch(("ref_ori" + pp).c_str(), sizeof(oreal) * nodes, &d_ori) ||
                (opt.d_node_A && !H->scratch(("ref_nA" + pp).c_str(), sizeof(float) * 4 * nodes, &d_nA)))
                return H->fail(ALI_ENOMEM, "device scratch allocation failed");
            hipLaunchKernelGGL((k_level_medium<oreal>), g2, dim3(B), 0, S, (const LevelDev*)d_lv, d_mat_id,
                               d_orient, opt.d_node_A, (uint8_t*)d_mid, (oreal*)d_ori, (float*)d_nA);
            lopt.d_node_A = (const float*)d_nA;
            mid = (const uint8_t*)d_mid;
            ori = (const oreal*)d_ori;
        }
        if (l == 0)
            hipLaunchKernelGGL((k_seed_start<real, oreal>), g2, dim3(B), 0, S, (const LevelDev*)d_lv,
                               ref.start_half_width, (const MatA*)d_A, (const double*)d_gt, d_mat_id, d_orient,
                               opt.d_node_A, T, (uint32_t*)d_fm);
        else
            hipLaunchKernelGGL((k_seed_transfer<real>), g2, dim3(B), 0, S, dprev, Tprev, (const real*)d_stop,
                               (const LevelDev*)d_lv, T, (uint32_t*)d_fm);
        HIPCK(H, hipGetLastError());
        ali_solve_stats ls{};
        st = last ? solve_fields<real, wmreal, oreal>(H, media.data(), (int32_t)media.size(), mats, n_mats, mid, ori,
                                                      srcs, nullptr, lopt, T, &ls, nullptr, (const uint32_t*)d_fm)
                  : solve_fields<real, mreal, oreal>(H, media.data(), (int32_t)media.size(), mats, n_mats, mid, ori,
                                                     lsrc.data(), nullptr, lopt, T, &ls, nullptr,
                                                     (const uint32_t*)d_fm);
        if (st != ALI_OK && st != ALI_ENOCONV) return st;
        add_stats(acc, ls);
        if (!last) {
            hipLaunchKernelGGL((k_level_stop<real>), dim3((unsigned)n_src), dim3(B), 0, S, (const LevelDev*)d_lv,
                               (const real*)T, (real*)d_stop);
            HIPCK(H, hipGetLastError());
        } else if (!same_out) {
            hipLaunchKernelGGL((k_convert<outreal, real>), dim3((unsigned)((nodes + B - 1) / B)), dim3(B), 0, S,
                               d_out, (const real*)T, nodes);
            HIPCK(H, hipGetLastError());
        }
        Tprev = T;
        dprev = (const LevelDev*)d_lv;
        prev = lv;
    }
    HIPCK(H, hipStreamSynchronize(S));
    if (stats) {
        *stats = acc;
        stats->nodes = NF;
        stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!acc.converged) return H->fail(ALI_ENOCONV, "relaxation reached max_sweeps");
    return ALI_OK;
}

template <typename real, typename mreal, typename wmreal, typename oreal, typename outreal>
static ali_status refined_impl(ali_handle* H, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                               const uint8_t* d_mat_id, const oreal* d_orient, const ali_node* srcs, int32_t n_src,
                               const ali_options* opt_in, const ali_refine* ref_in, outreal* d_out,
                               ali_solve_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    ali_options opt;
    ali_default_options(&opt);
    if (opt_in) opt = *opt_in;
    ali_refine ref;
    ali_default_refine(&ref);
    if (ref_in) ref = *ref_in;
    const int s = ref.subgrid;
    if (!grid) return H->fail(ALI_EINVAL, "grid is NULL");
    if (s == 0 || s == 1) {
        const ali_medium mw = single_medium(grid, n_mats, n_src, 0);
        return levels_impl<real, mreal, wmreal, oreal, outreal>(H, &mw, 1, mats, n_mats, d_mat_id, d_orient, srcs,
                                                                opt, ref, d_out, stats, t0);
    }
    if (s < 0 || s % 2 == 0 || s > 15) return H->fail(ALI_EINVAL, "subgrid must be 0, 1 or odd in [3, 15]");
    if (!d_out) return H->fail(ALI_EINVAL, "d_T is NULL");
    // the caller's medium, sources included, is checked on its own grid first
    const ali_medium mw = single_medium(grid, n_mats, n_src, 0);
    ali_status st = validate_batch(H, &mw, 1, mats, n_mats, d_mat_id, d_orient, srcs, nullptr, opt.wave);
    if (st != ALI_OK) return st;
    ali_grid gs = *grid;
    const int64_t nxs = (int64_t)(grid->nx - 1) * s + 1, nzs = (int64_t)(grid->nz - 1) * s + 1;
    if (nxs * nzs > (int64_t)1 << 31) return H->fail(ALI_EINVAL, "the s-fold grid exceeds 2^31 nodes");
    gs.nx = (int32_t)nxs;
    gs.nz = (int32_t)nzs;
    gs.h = grid->h / s;
    std::vector<ali_node> ss(srcs, srcs + n_src);
    for (ali_node& q : ss) {
        q.i *= s;
        q.j *= s;
    }
    if (set_device(H) != ALI_OK) return ALI_EDEVICE;
    hipStream_t S = H->stream;
    const int B = 256;
    const int64_t NS = nxs * nzs, NW = (int64_t)grid->nx * grid->nz;
    void *d_mid = nullptr, *d_ori = nullptr, *d_Ts = nullptr, *d_nA = nullptr;
    if (!H->scratch("sub_mid", NS, &d_mid) || !H->scratch("sub_ori", sizeof(oreal) * NS, &d_ori) ||
        !H->scratch("sub_T", sizeof(real) * NS * n_src, &d_Ts) ||
        (opt.d_node_A && !H->scratch("sub_nA", sizeof(float) * 4 * NS, &d_nA)))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    hipLaunchKernelGGL((k_subgrid_medium<oreal>), dim3((unsigned)((NS + B - 1) / B)), dim3(B), 0, S, grid->nx,
                       gs.nx, NS, s, d_mat_id, d_orient, opt.d_node_A, (uint8_t*)d_mid, (oreal*)d_ori,
                       (float*)d_nA);
    HIPCK(H, hipGetLastError());
    ali_options sopt = opt;
    sopt.d_node_A = (const float*)d_nA;
    const ali_medium ms = single_medium(&gs, n_mats, n_src, 0);
    st = levels_impl<real, mreal, wmreal, oreal, real>(H, &ms, 1, mats, n_mats, (const uint8_t*)d_mid,
                                                       (const oreal*)d_ori, ss.data(), sopt, ref, (real*)d_Ts, stats,
                                                       t0);
    if (st != ALI_OK && st != ALI_ENOCONV) return st;
    const int64_t n_out = NW * n_src;
    hipLaunchKernelGGL((k_subgrid_pick<outreal, real>), dim3((unsigned)((n_out + B - 1) / B)), dim3(B), 0, S,
                       grid->nx, NW, n_out, gs.nx, NS, s, (const real*)d_Ts, d_out);
    HIPCK(H, hipGetLastError());
    HIPCK(H, hipStreamSynchronize(S));
    if (stats) stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

// dL/dtheta of the working grid from the s-fold grid's: every fine node takes the
// orientation of its nearest working node, so a working node's derivative is the sum over
// the fine nodes within (s - 1) / 2 of its position (s odd: the nearest node is unique),
// added row by row in a fixed order
template <typename outreal>
__global__ void k_subgrid_sum(int nx, int nz, int nx_s, int nz_s, int s, const outreal* __restrict__ g_s,
                              outreal* __restrict__ g) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)nx * nz) return;
    const int i = (int)(p % nx), j = (int)(p / nx), r = (s - 1) / 2;
    const int a0 = i * s - r < 0 ? 0 : i * s - r, a1 = i * s + r < nx_s - 1 ? i * s + r : nx_s - 1;
    const int b0 = j * s - r < 0 ? 0 : j * s - r, b1 = j * s + r < nz_s - 1 ? j * s + r : nz_s - 1;
    double acc = 0.0;
    for (int b = b0; b <= b1; ++b)
        for (int a = a0; a <= a1; ++a) acc += (double)g_s[(int64_t)b * nx_s + a];
    g[p] = (outreal)acc;
}

// The misfit gradient of the forward on the s-fold grid (Section 4.5's subgrid size with the
// straight-ray source box counted in fine nodes): the fine medium is built as for the
// refined forward, the single-medium misfit gradient `grad` runs on it with the sources and
// receivers on the nodes (s i, s j), and its dL/dtheta is summed back onto the working nodes.
template <typename oreal, typename outreal, typename F>
static ali_status subgrid_gradient_impl(ali_handle* H, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                                        const uint8_t* d_mat_id, const oreal* d_orient, const ali_node* srcs,
                                        int32_t n_src, const ali_node* recv, int32_t n_recv, const outreal* d_obs,
                                        const ali_options* opt_in, int32_t s, outreal* d_T, outreal* d_Trec,
                                        double* d_loss, outreal* d_dth, ali_adjoint_stats* stats, F grad) {
    if (!grid) return H->fail(ALI_EINVAL, "grid is NULL");
    if (s == 1)
        return grad(H, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, recv, n_recv, d_obs, opt_in, d_T, d_Trec,
                    d_loss, d_dth, stats);
    if (s < 3 || s % 2 == 0 || s > 15) return H->fail(ALI_EINVAL, "subgrid must be 1 or odd in [3, 15]");
    ali_options opt;
    ali_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.d_node_A) return H->fail(ALI_EUNSUPPORTED, "the subgrid misfit gradient takes per-material stiffness only");
    if (!d_dth) return H->fail(ALI_EINVAL, "d_dLdtheta is NULL");
    // the caller's medium, sources and receivers are checked on its own grid first
    const ali_medium mw = single_medium(grid, n_mats, n_src, n_recv);
    ali_status st = validate_batch(H, &mw, 1, mats, n_mats, d_mat_id, d_orient, srcs, recv, opt.wave);
    if (st != ALI_OK) return st;
    const int64_t nxs = (int64_t)(grid->nx - 1) * s + 1, nzs = (int64_t)(grid->nz - 1) * s + 1;
    if (nxs * nzs > (int64_t)1 << 31) return H->fail(ALI_EINVAL, "the s-fold grid exceeds 2^31 nodes");
    ali_grid gs = *grid;
    gs.nx = (int32_t)nxs;
    gs.nz = (int32_t)nzs;
    gs.h = grid->h / s;
    std::vector<ali_node> ss(srcs, srcs + n_src), rs(recv, recv + n_recv);
    for (ali_node& q : ss) { q.i *= s; q.j *= s; }
    for (ali_node& q : rs) { q.i *= s; q.j *= s; }
    if (set_device(H) != ALI_OK) return ALI_EDEVICE;
    hipStream_t S = H->stream;
    const int B = 256;
    const int64_t NS = nxs * nzs, NW = (int64_t)grid->nx * grid->nz;
    void *d_mid = nullptr, *d_ori = nullptr, *d_gs = nullptr, *d_Ts = nullptr;
    if (!H->scratch("sg_mid", NS, &d_mid) || !H->scratch("sg_ori", sizeof(oreal) * NS, &d_ori) ||
        !H->scratch("sg_dth", sizeof(outreal) * NS, &d_gs) ||
        (d_T && !H->scratch("sg_T", sizeof(outreal) * NS * n_src, &d_Ts)))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    hipLaunchKernelGGL((k_subgrid_medium<oreal>), dim3((unsigned)((NS + B - 1) / B)), dim3(B), 0, S, grid->nx,
                       gs.nx, NS, s, d_mat_id, d_orient, (const float*)nullptr, (uint8_t*)d_mid, (oreal*)d_ori,
                       (float*)nullptr);
    HIPCK(H, hipGetLastError());
    st = grad(H, &gs, mats, n_mats, (const uint8_t*)d_mid, (const oreal*)d_ori, ss.data(), n_src, rs.data(), n_recv,
              d_obs, &opt, (outreal*)d_Ts, d_Trec, d_loss, (outreal*)d_gs, stats);
    if (st != ALI_OK && st != ALI_ENOCONV) return st;
    hipLaunchKernelGGL((k_subgrid_sum<outreal>), dim3((unsigned)((NW + B - 1) / B)), dim3(B), 0, S, grid->nx,
                       grid->nz, gs.nx, gs.nz, s, (const outreal*)d_gs, d_dth);
    if (d_T)
        hipLaunchKernelGGL((k_subgrid_pick<outreal, outreal>), dim3((unsigned)((NW * n_src + B - 1) / B)), dim3(B), 0,
                           S, grid->nx, NW, NW * n_src, gs.nx, NS, s, (const outreal*)d_Ts, d_T);
    HIPCK(H, hipGetLastError());
    HIPCK(H, hipStreamSynchronize(S));
    return st;
}

// a batch of media: the nested grids of every field, one relaxation per level for all of them
template <typename real, typename mreal, typename wmreal, typename oreal, typename outreal>
static ali_status batch_refined_impl(ali_handle* H, const ali_medium* media, int32_t n_media,
                                     const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                     const oreal* d_orient, const ali_node* srcs, const ali_options* opt_in,
                                     const ali_refine* ref_in, outreal* d_out, ali_solve_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    ali_options opt;
    ali_default_options(&opt);
    if (opt_in) opt = *opt_in;
    ali_refine ref;
    ali_default_refine(&ref);
    if (ref_in) ref = *ref_in;
    if (ref.subgrid != 0 && ref.subgrid != 1)
        return H->fail(ALI_EUNSUPPORTED, "batch calls take subgrid 0 or 1 (the s-fold medium is a single-medium option)");
    return levels_impl<real, mreal, wmreal, oreal, outreal>(H, media, n_media, mats, n_mats, d_mat_id, d_orient,
                                                            srcs, opt, ref, d_out, stats, t0);
}

}  // namespace ali

using namespace ali;

extern "C" void ali_default_refine(ali_refine* r) {
    if (!r) return;
    *r = ali_refine{};
    r->n_levels = 3;
    r->density[0] = 27; r->density[1] = 9; r->density[2] = 3;
    r->radius[0] = 1; r->radius[1] = 6; r->radius[2] = 13;
    r->start_half_width = 0.5;
    r->subgrid = 1;
}

extern "C" ali_status ali_solve_traveltime_refined(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                                   int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                                   const ali_node* srcs, int32_t n_src, const ali_options* opt,
                                                   const ali_refine* ref, float* d_T, ali_solve_stats* stats) {
    if (!h) return ALI_EINVAL;
    const int arith = opt ? opt->arith : ALI_ARITH_MIXED;
    switch (arith) {
        // float32 wavefront math on the fine grids lets near score ties flip (beyond the
        // 1e-4 bar on the weld), so the default arithmetic computes them in float64; the
        // grid itself keeps the mixed arithmetic of ali_solve_traveltime
        case ALI_ARITH_MIXED:
            return refined_impl<double, double, float, float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs,
                                                                     n_src, opt, ref, d_T, stats);
        case ALI_ARITH_F64:
            return refined_impl<double, double, double, float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs,
                                                                      n_src, opt, ref, d_T, stats);
        case ALI_ARITH_F32:
            return refined_impl<float, float, float, float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs,
                                                                   n_src, opt, ref, d_T, stats);
    }
    return h->fail(ALI_EINVAL, "unknown arith mode");
}

extern "C" ali_status ali_solve_traveltime_refined_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                                       int32_t n_mats, const uint8_t* d_mat_id, const double* d_orient,
                                                       const ali_node* srcs, int32_t n_src, const ali_options* opt,
                                                       const ali_refine* ref, double* d_T, ali_solve_stats* stats) {
    if (!h) return ALI_EINVAL;
    return refined_impl<double, double, double, double, double>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs,
                                                                n_src, opt, ref, d_T, stats);
}

extern "C" ali_status ali_solve_batch_refined(ali_handle* h, const ali_medium* media, int32_t n_media,
                                              const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                              const float* d_orient, const ali_node* srcs, const ali_options* opt,
                                              const ali_refine* ref, float* d_T, ali_solve_stats* stats) {
    if (!h) return ALI_EINVAL;
    const int arith = opt ? opt->arith : ALI_ARITH_MIXED;
    switch (arith) {
        case ALI_ARITH_MIXED:   // the fine grids in float64 (see ali_solve_traveltime_refined)
            return batch_refined_impl<double, double, float, float, float>(h, media, n_media, mats, n_mats, d_mat_id,
                                                                           d_orient, srcs, opt, ref, d_T, stats);
        case ALI_ARITH_F64:
            return batch_refined_impl<double, double, double, float, float>(h, media, n_media, mats, n_mats, d_mat_id,
                                                                            d_orient, srcs, opt, ref, d_T, stats);
        case ALI_ARITH_F32:
            return batch_refined_impl<float, float, float, float, float>(h, media, n_media, mats, n_mats, d_mat_id,
                                                                         d_orient, srcs, opt, ref, d_T, stats);
    }
    return h->fail(ALI_EINVAL, "unknown arith mode");
}

extern "C" ali_status ali_solve_batch_refined_f64(ali_handle* h, const ali_medium* media, int32_t n_media,
                                                  const ali_material* mats, int32_t n_mats, const uint8_t* d_mat_id,
                                                  const double* d_orient, const ali_node* srcs,
                                                  const ali_options* opt, const ali_refine* ref, double* d_T,
                                                  ali_solve_stats* stats) {
    if (!h) return ALI_EINVAL;
    return batch_refined_impl<double, double, double, double, double>(h, media, n_media, mats, n_mats, d_mat_id, d_orient,
                                                              srcs, opt, ref, d_T, stats);
}

extern "C" ali_status ali_misfit_gradient_subgrid(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                                  int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                                  const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                                  int32_t n_recv, const float* d_obs, const ali_options* opt,
                                                  int32_t subgrid, float* d_T, float* d_Trec, double* d_loss,
                                                  float* d_dLdtheta, ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    return subgrid_gradient_impl<float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, recv, n_recv,
                                               d_obs, opt, subgrid, d_T, d_Trec, d_loss, d_dLdtheta, stats,
                                               ali_misfit_gradient);
}

extern "C" ali_status ali_misfit_gradient_subgrid_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                                      int32_t n_mats, const uint8_t* d_mat_id, const double* d_orient,
                                                      const ali_node* srcs, int32_t n_src, const ali_node* recv,
                                                      int32_t n_recv, const double* d_obs, const ali_options* opt,
                                                      int32_t subgrid, double* d_T, double* d_Trec, double* d_loss,
                                                      double* d_dLdtheta, ali_adjoint_stats* stats) {
    if (!h) return ALI_EINVAL;
    return subgrid_gradient_impl<double, double>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, recv,
                                                 n_recv, d_obs, opt, subgrid, d_T, d_Trec, d_loss, d_dLdtheta, stats,
                                                 ali_misfit_gradient_f64);
}
