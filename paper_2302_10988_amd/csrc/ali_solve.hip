// ali_solve.hip -- travel-time fields by tiled relaxation of the ALI update (gfx950).
//
// The paper orders node updates with a binary heap (Section 2).  Its result is the unique
// fixed point of a local operator: at node D, grow the known set in (tau, index) order
// over the diamond and stop once D's estimate precedes the next neighbour.  Any schedule
// that reaches a state where no node changes lands on that field, so the GPU relaxes
// tiles in parallel instead:
//   - each work-group owns a 16x16 tile plus a 2-node halo staged in LDS;
//   - it sweeps the update over the tile in place until a block-wide OR reports no
//     change (or the inner cap), skipping waves whose rows saw no change last sweep;
//   - changed values go back to HBM; a change within 2 nodes of an edge flags the
//     neighbouring tile(s), an unfinished tile flags itself;
//   - a compaction kernel turns the flags into the next pass's work list.
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
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "ali_solve.hpp"

namespace ali {

// ---------------------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------------------
template <typename mreal, typename treal, typename oreal>
__global__ void k_prep(int nx, int nz, double h, int n_mats, const MatDev<mreal>* __restrict__ mats,
                       const uint8_t* __restrict__ mat_id, const oreal* __restrict__ orient,
                       mreal* __restrict__ geo, treal* __restrict__ fbt, int* __restrict__ err) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)nx * nz) return;
    const double th = (double)orient[p];
    const int mid = mat_id[p];
    if (!isfinite(th)) { atomicOr(err, 1); return; }
    if (mid >= n_mats) { atomicOr(err, 2); return; }
    const MatA m = mats[mid].A;
    double s2, c2;
    sincos(2.0 * th, &s2, &c2);
    geo[2 * p + 0] = (mreal)c2;
    geo[2 * p + 1] = (mreal)s2;
    // straight-ray time to an 8-neighbour along x, (1,1), z, (1,-1)
    const double quarter = 0.78539816339744830962;
    const double len[4] = {1.0, 1.41421356237309504880, 1.0, 1.41421356237309504880};
    const double ang[4] = {0.0, quarter, 2.0 * quarter, -quarter};
#pragma unroll
    for (int d = 0; d < 4; ++d) fbt[4 * p + d] = (treal)(len[d] * h / group_speed(m, ang[d] - th));
}

template <typename real, typename mreal, typename oreal>
__global__ void k_init(int nx, int nz, int nf, double h, const MatDev<mreal>* __restrict__ mats,
                       const uint8_t* __restrict__ mat_id, const oreal* __restrict__ orient,
                       const int2* __restrict__ src, int R, real* __restrict__ T,
                       uint32_t* __restrict__ flags, int ntx, int ntz) {
    const int64_t N = (int64_t)nx * nz;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (p >= N) return;
    const int i = (int)(p % nx), j = (int)(p / nx);
    const int2 s = src[f];
    const int di = i - s.x, dj = j - s.y;
    real v = dinf<real>();
    if (abs(di) <= R && abs(dj) <= R) {
        // straight ray at the group speed of the source node's material (Section 4.4)
        const int64_t ps = (int64_t)s.y * nx + s.x;
        if (di == 0 && dj == 0) {
            v = real(0);
        } else {
            const double phi = atan2((double)dj, (double)di) - (double)orient[ps];
            v = (real)(sqrt((double)(di * di + dj * dj)) * h / group_speed(mats[mat_id[ps]].A, phi));
        }
    }
    T[(int64_t)f * N + p] = v;
    // tiles that see the box (box radius + diamond radius) start active
    if (abs(di) <= R + HALO && abs(dj) <= R + HALO) {
        flags[(int64_t)f * ntx * ntz + (j / TZ) * ntx + (i / TX)] = 1u;   // evaluate the whole tile
    }
}

template <typename real>
__global__ void k_compact(uint32_t* __restrict__ flags, real* __restrict__ minrej, int64_t n,
                          int ntiles, const real* __restrict__ theta, uint32_t* __restrict__ list,
                          uint32_t* __restrict__ lbits, uint32_t* __restrict__ count) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int f = (int)(u / ntiles);
    const uint32_t b = flags[u];
    if (b || minrej[u] <= theta[f]) {
        flags[u] = 0;
        minrej[u] = dinf<real>();     // recomputed by the visit
        const uint32_t pos = atomicAdd(count, 1u);
        list[pos] = (uint32_t)u;
        lbits[pos] = b;
    }
}

// nothing active: move each field's threshold up to its smallest rejected value
template <typename real>
__global__ void k_jump(const real* __restrict__ minrej, int ntiles, int nf, real* __restrict__ theta,
                       uint32_t* __restrict__ jumped) {
    const int f = blockIdx.x;
    real m = dinf<real>();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
        const real v = minrej[(int64_t)f * ntiles + t];
        m = v < m ? v : m;
    }
    __shared__ real red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x + w] < red[threadIdx.x] ? red[threadIdx.x + w] : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] < dinf<real>()) {
        if (red[0] > theta[f]) theta[f] = red[0];
        atomicAdd(jumped, 1u);
    }
}

template <typename real>
__global__ void k_advance(real* __restrict__ theta, const real* __restrict__ step, int nf) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < nf) theta[f] += step[f];
}

__global__ void k_zero_u32(uint32_t* p) { *p = 0u; }

// min of non-negative values in LDS through their integer bit patterns
__device__ __forceinline__ void lds_min(float* p, float v) {
    atomicMin(reinterpret_cast<unsigned*>(p), __float_as_uint(v));
}
__device__ __forceinline__ void lds_min(double* p, double v) {
    atomicMin(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}


// One tile visit.  The set of nodes to evaluate is tracked per node: a node whose value
// changes marks its diamond neighbours inside the tile for the next sweep, and each sweep
// packs the marked nodes into the first threads of the block so that idle waves skip the
// update altogether.  The first sweep evaluates the band front (unreached nodes with a
// reached neighbour: new arrivals and values rejected by an earlier band), nodes next to
// a halo side that a neighbouring tile changed, or every node (TF_SELF).
template <typename real, typename mreal>
__global__ void __launch_bounds__(NTHREADS)
k_relax(int nx, int nz, int ntx, int ntz, const uint32_t* __restrict__ list,
        const uint32_t* __restrict__ lbits,
        const MatDev<mreal>* __restrict__ mats, const uint8_t* __restrict__ mat_id,
        const mreal* __restrict__ geo, const real* __restrict__ fbt,
        const int2* __restrict__ src, int R, int inner, const real* __restrict__ theta,
        real* __restrict__ T, uint32_t* __restrict__ flags, real* __restrict__ minrej,
        unsigned long long* __restrict__ counters) {
    __shared__ real lt[LH * LSTRIDE];
    __shared__ real rej[NTHREADS];
    __shared__ uint8_t dirty[2][NTHREADS];
    __shared__ uint8_t act[NTHREADS];
    __shared__ uint16_t clist[NTHREADS];
    __shared__ unsigned wcount[NTHREADS / 64];
    __shared__ real blk_rej;
    __shared__ unsigned edge_out;
    __shared__ unsigned blk_updates, blk_evals;

    const uint32_t unit = list[blockIdx.x];
    const uint32_t bits = lbits[blockIdx.x];
    const int ntiles = ntx * ntz;
    const int f = (int)(unit / (uint32_t)ntiles);
    const int tile = (int)(unit % (uint32_t)ntiles);
    const int tx = tile % ntx, tz = tile / ntx;
    const int i0 = tx * TX, j0 = tz * TZ;
    const int64_t N = (int64_t)nx * nz;
    real* __restrict__ Tf = T + (int64_t)f * N;
    const real inf = dinf<real>();
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;

    // stage tile + halo
    for (int q = tid; q < LW * LH; q += NTHREADS) {
        const int li = q % LW, lj = q / LW;
        const int gi = i0 - HALO + li, gj = j0 - HALO + lj;
        real v = inf;
        if (gi >= 0 && gj >= 0 && gi < nx && gj < nz) v = Tf[(int64_t)gj * nx + gi];
        lt[lj * LSTRIDE + li] = v;
    }
    const int2 s = src[f];
    const real th = theta[f];
    // the node this thread owns for bookkeeping
    const int lx = tid % TX, lz = tid / TX;
    const int gi = i0 + lx, gj = j0 + lz;
    const bool valid = gi < nx && gj < nz;
    const bool active = valid && !(abs(gi - s.x) <= R && abs(gj - s.y) <= R);
    act[tid] = active ? 1 : 0;
    rej[tid] = inf;
    if (tid == 0) { edge_out = 0u; blk_updates = 0u; blk_evals = 0u; blk_rej = inf; }
    __syncthreads();

    const int me = (lz + HALO) * LSTRIDE + (lx + HALO);
    const real orig = lt[me];
    {
        bool any = false;
#pragma unroll
        for (int k = 0; k < 12; ++k) any |= lt[me + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k]] < inf;
        const bool d = (bits & TF_SELF) || !(orig < inf) ||
                       ((bits & TF_HALO_L) && lx < HALO) || ((bits & TF_HALO_R) && lx >= TX - HALO) ||
                       ((bits & TF_HALO_U) && lz < HALO) || ((bits & TF_HALO_D) && lz >= TZ - HALO) ||
                       ((bits & TF_HALO_UL) && lx == 0 && lz == 0) ||
                       ((bits & TF_HALO_UR) && lx == TX - 1 && lz == 0) ||
                       ((bits & TF_HALO_DL) && lx == 0 && lz == TZ - 1) ||
                       ((bits & TF_HALO_DR) && lx == TX - 1 && lz == TZ - 1);
        dirty[0][tid] = (active && any && d) ? 1 : 0;
        dirty[1][tid] = 0;
    }
    __syncthreads();

    unsigned my_updates = 0, my_evals = 0;
    bool done = false;
    for (int it = 0;; ++it) {
        const int cur = it & 1;
        // pack the marked nodes
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
            const int64_t p = (int64_t)(j0 + nlz) * nx + (i0 + nlx);
            NodeConst<mreal, real> nc;
            load_node_const<real, mreal>(nc, p, mats, mat_id, geo, fbt);
            real t[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) t[k] = lt[nme + SLOT_DJ[k] * LSTRIDE + SLOT_DI[k]];
            ++my_updates;
            real u = local_update<mreal, real>(nc, t, lt, nme, LSTRIDE, my_evals);
            real r = inf;
            if (u > th && u < inf) { r = u; u = inf; }
            rej[node] = r;
            const real cv = lt[nme];
            if (!(u == cv || (u >= inf && cv >= inf))) {
                lt[nme] = u;
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    const int ax = nlx + SLOT_DI[k], az = nlz + SLOT_DJ[k];
                    if (ax >= 0 && az >= 0 && ax < TX && az < TZ && act[az * TX + ax])
                        dirty[cur ^ 1][az * TX + ax] = 1;
                }
            }
        }
        __syncthreads();
    }

    // write back, tell neighbouring tiles which of their halo sides changed
    const real fin = lt[me];
    if (valid && !(fin == orig || (fin >= inf && orig >= inf))) {
        Tf[(int64_t)gj * nx + gi] = fin;
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
    if (rej[tid] < inf) lds_min(&blk_rej, rej[tid]);
    if (my_updates) { atomicAdd(&blk_updates, my_updates); atomicAdd(&blk_evals, my_evals); }
    __syncthreads();
    if (tid == 0) {
        if (blk_updates) {
            atomicAdd(&counters[0], (unsigned long long)blk_updates);
            atomicAdd(&counters[1], (unsigned long long)blk_evals);
        }
        uint32_t* fl = flags + (int64_t)f * ntiles;
        minrej[(int64_t)f * ntiles + tile] = blk_rej;
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

// ---------------------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------------------
// real: travel-time type (storage, scores, decisions); mreal: wavefront / phase-speed
// math; oreal: orientation input.
template <typename real, typename mreal, typename oreal>
ali_status solve_core(ali_handle* H, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                      const uint8_t* d_mat_id, const oreal* d_orient, const ali_node* srcs,
                      int32_t n_src, const ali_options& opt, real* d_T, ali_solve_stats* stats,
                      ForwardState<real, mreal>* fs) {
    ali_status st = validate_medium(H, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src);
    if (st != ALI_OK) return st;
    if (!d_T) return H->fail(ALI_EINVAL, "d_T is NULL");
    if (opt.src_box_radius < 0 || opt.src_box_radius > 64) return H->fail(ALI_EINVAL, "src_box_radius out of range [0, 64]");
    if (opt.max_sweeps < 1) return H->fail(ALI_EINVAL, "max_sweeps must be >= 1");
    if (opt.inner_sweeps < 1 || opt.inner_sweeps > 4096) return H->fail(ALI_EINVAL, "inner_sweeps out of range [1, 4096]");
    if (opt.band_cells < 0) return H->fail(ALI_EINVAL, "band_cells must be >= 0 (0 = no band)");

    const int nx = grid->nx, nz = grid->nz;
    const int64_t N = (int64_t)nx * nz;
    const int ntx = (nx + TX - 1) / TX, ntz = (nz + TZ - 1) / TZ;
    const int64_t nunits = (int64_t)ntx * ntz * n_src;
    if (nunits >= (int64_t)UINT32_MAX) return H->fail(ALI_EINVAL, "too many tiles in one call");
    if (set_device(H) != ALI_OK) return ALI_EDEVICE;
    hipStream_t S = H->stream;

    const std::vector<MatDev<mreal>> hm = make_matdev<mreal>(mats, n_mats, grid->h);
    // band step: band_cells node spacings at the fastest phase speed of the medium
    const double vmax = max_phase_speed(mats, n_mats);
    const real band = opt.band_cells > 0 ? (real)(opt.band_cells * grid->h / vmax) : dinf_host<real>();
    std::vector<real> hstep(n_src, band), htheta(n_src, band);

    void *d_mats, *d_geo, *d_fbt, *d_src, *d_flags, *d_list, *d_count, *d_upd, *d_err;
    void *d_theta, *d_step, *d_minrej, *d_lbits;
    if (!H->scratch("mats", sizeof(MatDev<mreal>) * n_mats, &d_mats) ||
        !H->scratch("theta", sizeof(real) * n_src, &d_theta) ||
        !H->scratch("step", sizeof(real) * n_src, &d_step) ||
        !H->scratch("minrej", sizeof(real) * nunits, &d_minrej) ||
        !H->scratch("geo", sizeof(mreal) * 2 * N, &d_geo) ||
        !H->scratch("fbt", sizeof(real) * 4 * N, &d_fbt) ||
        !H->scratch("src", sizeof(int2) * n_src, &d_src) ||
        !H->scratch("flags", sizeof(uint32_t) * nunits, &d_flags) ||
        !H->scratch("list", sizeof(uint32_t) * nunits, &d_list) ||
        !H->scratch("lbits", sizeof(uint32_t) * nunits, &d_lbits) ||
        !H->scratch("count", sizeof(uint32_t), &d_count) ||
        !H->scratch("upd", 2 * sizeof(unsigned long long), &d_upd) ||
        !H->scratch("err", sizeof(int), &d_err))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    std::vector<int2> hs(n_src);
    for (int k = 0; k < n_src; ++k) hs[k] = make_int2(srcs[k].i, srcs[k].j);

    HIPCK(H, hipEventRecord(H->ev0, S));
    HIPCK(H, hipMemcpyAsync(d_mats, hm.data(), sizeof(MatDev<mreal>) * n_mats, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemcpyAsync(d_src, hs.data(), sizeof(int2) * n_src, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemcpyAsync(d_theta, htheta.data(), sizeof(real) * n_src, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemcpyAsync(d_step, hstep.data(), sizeof(real) * n_src, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemsetAsync(d_flags, 0, sizeof(uint32_t) * nunits, S));
    HIPCK(H, hipMemsetAsync(d_upd, 0, 2 * sizeof(unsigned long long), S));
    HIPCK(H, hipMemsetAsync(d_err, 0, sizeof(int), S));

    const int B = 256;
    hipLaunchKernelGGL((k_fill<real>), dim3((unsigned)((nunits + B - 1) / B)), dim3(B), 0, S,
                       (real*)d_minrej, nunits, dinf_host<real>());
    hipLaunchKernelGGL((k_prep<mreal, real, oreal>), dim3((unsigned)((N + B - 1) / B)), dim3(B), 0, S,
                       nx, nz, grid->h, n_mats, (const MatDev<mreal>*)d_mats, d_mat_id, d_orient,
                       (mreal*)d_geo, (real*)d_fbt, (int*)d_err);
    HIPCK(H, hipGetLastError());
    hipLaunchKernelGGL((k_init<real, mreal, oreal>), dim3((unsigned)((N + B - 1) / B), (unsigned)n_src), dim3(B), 0, S,
                       nx, nz, n_src, grid->h, (const MatDev<mreal>*)d_mats, d_mat_id,
                       d_orient, (const int2*)d_src, opt.src_box_radius, d_T,
                       (uint32_t*)d_flags, ntx, ntz);
    HIPCK(H, hipGetLastError());

    int h_err = 0;
    HIPCK(H, hipMemcpyAsync(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost, S));
    HIPCK(H, hipStreamSynchronize(S));
    if (h_err & 1) return H->fail(ALI_EINVAL, "orientation contains NaN or Inf");
    if (h_err & 2) return H->fail(ALI_EINVAL, "material id out of range");

    int iters = 0;
    int64_t visits = 0;
    bool converged = false;
    double relax_ms = 0.0;
    bool pending_relax = false;
    uint32_t* h_count = H->host_count;
    const int ntiles = ntx * ntz;
    for (;;) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, S, (uint32_t*)d_count);
        hipLaunchKernelGGL((k_compact<real>), dim3((unsigned)((nunits + B - 1) / B)), dim3(B), 0, S,
                           (uint32_t*)d_flags, (real*)d_minrej, nunits, ntiles, (const real*)d_theta,
                           (uint32_t*)d_list, (uint32_t*)d_lbits, (uint32_t*)d_count);
        HIPCK(H, hipGetLastError());
        HIPCK(H, hipMemcpyAsync(h_count, d_count, sizeof(uint32_t), hipMemcpyDeviceToHost, S));
        HIPCK(H, hipStreamSynchronize(S));
        if (pending_relax) {
            float kms = 0.f;
            HIPCK(H, hipEventElapsedTime(&kms, H->ev2, H->ev3));
            relax_ms += kms;
            pending_relax = false;
        }
        const uint32_t n = *h_count;
        if (n == 0) {
            // nothing active: jump thresholds to the smallest rejected values, if any
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, S, (uint32_t*)d_count);
            hipLaunchKernelGGL((k_jump<real>), dim3((unsigned)n_src), dim3(256), 0, S,
                               (const real*)d_minrej, ntiles, n_src, (real*)d_theta, (uint32_t*)d_count);
            HIPCK(H, hipGetLastError());
            HIPCK(H, hipMemcpyAsync(h_count, d_count, sizeof(uint32_t), hipMemcpyDeviceToHost, S));
            HIPCK(H, hipStreamSynchronize(S));
            if (*h_count == 0) { converged = true; break; }
            continue;
        }
        if (iters >= opt.max_sweeps) break;
        HIPCK(H, hipEventRecord(H->ev2, S));
        hipLaunchKernelGGL((k_relax<real, mreal>), dim3(n), dim3(NTHREADS), 0, S,
                           nx, nz, ntx, ntz, (const uint32_t*)d_list, (const uint32_t*)d_lbits,
                           (const MatDev<mreal>*)d_mats,
                           d_mat_id, (const mreal*)d_geo, (const real*)d_fbt, (const int2*)d_src,
                           opt.src_box_radius, opt.inner_sweeps, (const real*)d_theta, d_T,
                           (uint32_t*)d_flags, (real*)d_minrej, (unsigned long long*)d_upd);
        HIPCK(H, hipGetLastError());
        HIPCK(H, hipEventRecord(H->ev3, S));
        if (opt.band_cells > 0)
            hipLaunchKernelGGL((k_advance<real>), dim3((unsigned)((n_src + 63) / 64)), dim3(64), 0, S,
                               (real*)d_theta, (const real*)d_step, n_src);
        pending_relax = true;
        ++iters;
        visits += n;
    }
    unsigned long long upd[2] = {0, 0};
    HIPCK(H, hipMemcpyAsync(upd, d_upd, sizeof(upd), hipMemcpyDeviceToHost, S));
    HIPCK(H, hipStreamSynchronize(S));
    if (stats) {
        stats->node_updates = (int64_t)upd[0];
        stats->stencil_evals = (int64_t)upd[1];
        stats->relax_ms = relax_ms;
        stats->tile_visits = visits;
        stats->nodes = N * n_src;
        stats->outer_iters = iters;
        stats->converged = converged ? 1 : 0;
        stats->ms = 0.0;
    }
    if (fs) {
        fs->mats = (const MatDev<mreal>*)d_mats;
        fs->geo = (const mreal*)d_geo;
        fs->fbt = (const real*)d_fbt;
        fs->src = (const int2*)d_src;
        fs->ntx = ntx;
        fs->ntz = ntz;
    }
    if (!converged) return H->fail(ALI_ENOCONV, "relaxation reached max_sweeps");
    return ALI_OK;
}

template ali_status solve_core<double, float, float>(ali_handle*, const ali_grid*, const ali_material*, int32_t,
    const uint8_t*, const float*, const ali_node*, int32_t, const ali_options&, double*, ali_solve_stats*,
    ForwardState<double, float>*);
template ali_status solve_core<float, float, float>(ali_handle*, const ali_grid*, const ali_material*, int32_t,
    const uint8_t*, const float*, const ali_node*, int32_t, const ali_options&, float*, ali_solve_stats*,
    ForwardState<float, float>*);
template ali_status solve_core<double, double, float>(ali_handle*, const ali_grid*, const ali_material*, int32_t,
    const uint8_t*, const float*, const ali_node*, int32_t, const ali_options&, double*, ali_solve_stats*,
    ForwardState<double, double>*);
template ali_status solve_core<double, double, double>(ali_handle*, const ali_grid*, const ali_material*, int32_t,
    const uint8_t*, const double*, const ali_node*, int32_t, const ali_options&, double*, ali_solve_stats*,
    ForwardState<double, double>*);

// Entry-point body: relax in `real` (on a scratch field when it differs from the output
// type), convert into d_out, time the whole call.
template <typename real, typename mreal, typename oreal, typename outreal>
static ali_status solve_impl(ali_handle* H, const ali_grid* grid, const ali_material* mats,
                             int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient,
                             const ali_node* srcs, int32_t n_src, const ali_options* opt_in,
                             outreal* d_out, ali_solve_stats* stats) {
    ali_options opt;
    ali_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (!d_out) return H->fail(ALI_EINVAL, "d_T is NULL");
    if (!grid) return H->fail(ALI_EINVAL, "grid is NULL");
    constexpr bool same_out = std::is_same<real, outreal>::value;
    const int64_t tot = (int64_t)grid->nx * grid->nz * (n_src > 0 ? n_src : 0);
    void* d_work = nullptr;
    if (!same_out && tot > 0 && !H->scratch("Twork", sizeof(real) * tot, &d_work))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    real* d_T = same_out ? (real*)d_out : (real*)d_work;
    ali_solve_stats local{};
    ali_status st = solve_core<real, mreal, oreal>(H, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src,
                                                   opt, d_T, &local, nullptr);
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

}  // namespace ali

using namespace ali;

extern "C" ali_status ali_solve_traveltime(ali_handle* h, const ali_grid* grid,
                                           const ali_material* mats, int32_t n_mats,
                                           const uint8_t* d_mat_id, const float* d_orient,
                                           const ali_node* srcs, int32_t n_src,
                                           const ali_options* opt, float* d_T,
                                           ali_solve_stats* stats) {
    if (!h) return ALI_EINVAL;
    const int arith = opt ? opt->arith : ALI_ARITH_MIXED;
    switch (arith) {
        case ALI_ARITH_MIXED:
            return solve_impl<double, float, float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, opt, d_T, stats);
        case ALI_ARITH_F32:
            return solve_impl<float, float, float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, opt, d_T, stats);
        case ALI_ARITH_F64:
            return solve_impl<double, double, float, float>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, opt, d_T, stats);
    }
    return h->fail(ALI_EINVAL, "unknown arith mode");
}

extern "C" ali_status ali_solve_traveltime_f64(ali_handle* h, const ali_grid* grid,
                                               const ali_material* mats, int32_t n_mats,
                                               const uint8_t* d_mat_id, const double* d_orient,
                                               const ali_node* srcs, int32_t n_src,
                                               const ali_options* opt, double* d_T,
                                               ali_solve_stats* stats) {
    if (!h) return ALI_EINVAL;
    return solve_impl<double, double, double, double>(h, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, opt, d_T, stats);
}
