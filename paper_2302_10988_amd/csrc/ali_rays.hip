// ali_rays.hip -- ray tracing through finished travel-time fields (paper Section 5.1).
//
// A ray runs from a receiver to the source of a field: by reciprocity the field value at
// a point is the time from that point to the source.  Each step chooses the plane family
// (x = k, z = k, x + z = k, x - z = k) that makes the largest angle with the last segment,
// moves to the family's next plane through grid nodes, and picks the point of that plane
// that minimises  straight-segment time + field time  (Fermat): a parabola through each
// local minimum of the sampled costs and its two neighbours, the smallest vertex wins.
// The ray stops within 1.6 node spacings of the source.
//
// GPU mapping: one wave per ray, one candidate per lane (2 * window * sub - 1 <= 63
// candidates spaced 1/sub of a node, field linearly interpolated along the plane);
// neighbours, local minima and the arg-min use wave shuffles, so a step costs one
// segment walk per lane plus a few cross-lane reductions.  The segment walk crosses the
// nearest-node cells and sums length / group speed; the group slowness comes from a
// per-material table over the group angle (2048 intervals on [0, pi/2], linear
// interpolation) built by exact inversion in float64.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <vector>

#include "ali_handle.hpp"
#include "ali_velocity.hpp"
#include "../../include/ali.h"

namespace ali {

constexpr int GT_N = 2048;                 // table intervals over [0, pi/2]
constexpr double HALF_PI = 1.57079632679489661923;

__global__ void k_gtable(const MatA* __restrict__ mats, const double* __restrict__ gt, int n_mats,
                         float* __restrict__ tab) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (q > GT_N || m >= n_mats) return;
    const double phi = HALF_PI * (double)q / GT_N;
    tab[(int64_t)m * (GT_N + 1) + q] = (float)(1.0 / (gt ? group_speed_tab(gt + m * VT_N, phi) : group_speed(mats[m], phi)));
}

struct RayMedium {
    int nx, nz;
    double h;
    const uint8_t* mat_id;
    const float* orient;
    const float* tab;                      // [n_mats][GT_N + 1] group slowness [s/m]
};

__device__ __forceinline__ float group_slowness(const RayMedium& M, const float* __restrict__ tab, int64_t p,
                                                float ang) {
    // reduce the angle against the cell's symmetry axis to [0, pi/2].  Below 3 pi (the
    // usual case) one or two exact subtractions give fmodf's exact remainder (Sterbenz:
    // a - k pi is exact for k pi <= a <= 2 k pi); beyond that, fmodf itself.
    constexpr float PI_F = 3.14159265358979f;
    float a = fabsf(ang - M.orient[p]);
    if (a >= 3.0f * PI_F) a = fmodf(a, PI_F);
    else if (a >= 2.0f * PI_F) a -= 2.0f * PI_F;
    else if (a >= PI_F) a -= PI_F;
    if (a > 1.57079632679490f) a = 3.14159265358979f - a;
    const float x = a * (float)(GT_N / HALF_PI);
    int i = (int)x;
    i = i < 0 ? 0 : (i >= GT_N ? GT_N - 1 : i);
    const float w = x - (float)i;
    const float* t = tab + (int64_t)M.mat_id[p] * (GT_N + 1);
    return t[i] + w * (t[i + 1] - t[i]);
}

// straight-segment time from (x0,z0) to (x1,z1) [grid units] through the nearest-node
// cells: cut at the cell boundaries k + 1/2, each piece at its midpoint cell's speed.
// The pieces are enumerated SEG_BATCH at a time with arithmetic only and their cells'
// data loaded together, so a walk costs two dependent memory round trips per batch
// rather than two per cell.  A step that crosses no boundary adds a zero-length piece
// (+0, which leaves the sum unchanged); the pieces are summed in walk order.
constexpr int SEG_BATCH = 4;
__device__ __forceinline__ double segment_time(const RayMedium& M, const float* __restrict__ tab, double x0,
                                               double z0, double x1, double z1) {
    const double dx = x1 - x0, dz = z1 - z0;
    const double len = sqrt(dx * dx + dz * dz);
    if (len == 0.0) return 0.0;
    const float ang = atan2f((float)dz, (float)dx);
    // next boundary crossings along x and z
    double tx = 2.0, tz = 2.0, sx = 0.0, sz = 0.0;
    if (dx != 0.0) {
        const double b = dx > 0.0 ? floor(x0 + 0.5) + 0.5 : floor(x0 + 0.5) - 0.5;
        tx = (b - x0) / dx;
        sx = 1.0 / fabs(dx);
    }
    if (dz != 0.0) {
        const double b = dz > 0.0 ? floor(z0 + 0.5) + 0.5 : floor(z0 + 0.5) - 0.5;
        tz = (b - z0) / dz;
        sz = 1.0 / fabs(dz);
    }
    double t = 0.0, total = 0.0;
    for (int guard = 0; guard < 4096 && t < 1.0; guard += SEG_BATCH) {
        double wgt[SEG_BATCH];
        uint32_t cell[SEG_BATCH];
#pragma unroll
        for (int k = 0; k < SEG_BATCH; ++k) {
            double tn = tx < tz ? tx : tz;
            if (tn > 1.0) tn = 1.0;
            const bool live = t < 1.0;
            const double tm = 0.5 * (t + tn);
            int ci = (int)floor(x0 + tm * dx + 0.5), cj = (int)floor(z0 + tm * dz + 0.5);
            ci = ci < 0 ? 0 : (ci >= M.nx ? M.nx - 1 : ci);
            cj = cj < 0 ? 0 : (cj >= M.nz ? M.nz - 1 : cj);
            wgt[k] = (live && tn > t) ? tn - t : 0.0;
            cell[k] = (uint32_t)cj * (uint32_t)M.nx + (uint32_t)ci;
            if (live) {
                t = tn;
                if (tx <= tn) tx += sx;
                if (tz <= tn) tz += sz;
            }
        }
        float sl[SEG_BATCH];
#pragma unroll
        for (int k = 0; k < SEG_BATCH; ++k) sl[k] = group_slowness(M, tab, (int64_t)cell[k], ang);
#pragma unroll
        for (int k = 0; k < SEG_BATCH; ++k) total += wgt[k] * len * M.h * (double)sl[k];
    }
    return total;
}

// plane families: normal N and step E between consecutive nodes of one plane
__device__ __forceinline__ void fam(int f, int& nxf, int& nzf, int& ex, int& ez) {
    switch (f) {
        case 0: nxf = 1; nzf = 0; ex = 0; ez = 1; break;     // x = k
        case 1: nxf = 0; nzf = 1; ex = 1; ez = 0; break;     // z = k
        case 2: nxf = 1; nzf = 1; ex = 1; ez = -1; break;    // x + z = k
        default: nxf = 1; nzf = -1; ex = 1; ez = 1; break;   // x - z = k
    }
}
// grid node of parameter m on plane k of family f
__device__ __forceinline__ void fam_node(int f, int k, int m, int& i, int& j) {
    switch (f) {
        case 0: i = k; j = m; break;
        case 1: i = m; j = k; break;
        case 2: i = m; j = k - m; break;
        default: i = m; j = m - k; break;
    }
}

// parameters of the grid nodes on plane k of family f
__device__ __forceinline__ void plane_range(int nx, int nz, int f, int k, int& lo, int& hi) {
    switch (f) {
        case 0: lo = 0; hi = nz - 1; break;
        case 1: lo = 0; hi = nx - 1; break;
        case 2: lo = k - (nz - 1) > 0 ? k - (nz - 1) : 0; hi = k < nx - 1 ? k : nx - 1; break;
        default: lo = k > 0 ? k : 0; hi = k + nz - 1 < nx - 1 ? k + nz - 1 : nx - 1; break;
    }
}

template <typename treal>
__device__ __forceinline__ double field_at(const treal* __restrict__ T, int nx, int nz, int i, int j) {
    if (i < 0 || j < 0 || i >= nx || j >= nz) return INFINITY;
    return (double)T[(int64_t)j * nx + i];
}

// rays per work-group (one wave each); media of up to RAY_LDS_MATS materials keep the
// slowness tables in LDS, shared by the work-group's rays
constexpr int RAYS_PER_GROUP = 4;
constexpr int RAY_LDS_MATS = 4;

// FIXED: one plane family (family 0..3) for the whole ray; otherwise the changing family.
template <typename treal, bool LDS_TAB, bool FIXED>
__global__ void __launch_bounds__(RAYS_PER_GROUP * 64)
k_trace(RayMedium M, int n_mats, int n_rays, const treal* __restrict__ Tall, const int2* __restrict__ srcs,
        const int2* __restrict__ recv, int n_recv, int window, int sub, int max_pts, int family,
        float2* __restrict__ paths, int32_t* __restrict__ npts, float* __restrict__ tray) {
    __shared__ float s_tab[LDS_TAB ? RAY_LDS_MATS * (GT_N + 1) : 1];
    if (LDS_TAB) {
        for (int i = threadIdx.x; i < n_mats * (GT_N + 1); i += RAYS_PER_GROUP * 64) s_tab[i] = M.tab[i];
        __syncthreads();
    }
    const float* __restrict__ tab = LDS_TAB ? s_tab : M.tab;
    const int r = blockIdx.x * RAYS_PER_GROUP + (int)(threadIdx.x >> 6);
    if (r >= n_rays) return;
    const int s = r / n_recv, k = r % n_recv;
    const int lane = threadIdx.x & 63;
    const int64_t N = (int64_t)M.nx * M.nz;
    const treal* __restrict__ T = Tall + (int64_t)s * N;
    float2* __restrict__ path = paths + (int64_t)r * max_pts;
    const int2 S = srcs[s], R0 = recv[k];
    const int half = window * sub - 1, nc = 2 * half + 1;
    double px = R0.x, pz = R0.y;
    double dx = S.x - px, dz = S.y - pz;
    // The path's time is off the step's critical path: segment number g is kept by lane
    // g mod 64, and every 64 segments the lanes walk their segments together.  Each lane
    // sums its segments in order; the lanes' sums are combined by a fixed butterfly.
    double part = 0.0;
    double hx0 = 0.0, hz0 = 0.0, hx1 = 0.0, hz1 = 0.0;
    bool held = false;
    int nseg = 0;
    auto keep = [&](double ax, double az, double bx, double bz) {
        if (lane == (nseg & 63)) { hx0 = ax; hz0 = az; hx1 = bx; hz1 = bz; held = true; }
        if ((nseg & 63) == 63) {
            if (held) part += segment_time(M, tab, hx0, hz0, hx1, hz1);
            held = false;
        }
        ++nseg;
    };
    int n = 0;
    if (lane == 0) path[0] = make_float2((float)px, (float)pz);
    ++n;
    bool reached = false;
    // a fixed family: plane indices of the start and of S, and a lower bound of every
    // table slowness (interpolation stays between two entries; the margin covers rounding)
    int kS = 0, k0 = 0, fsgn = 1;
    double minsl = 0.0;
    if constexpr (FIXED) {
        float ms = INFINITY;
        for (int i = lane; i < n_mats * (GT_N + 1); i += 64) ms = fminf(ms, tab[i]);
        for (int off = 32; off > 0; off >>= 1) ms = fminf(ms, __shfl_xor(ms, off));
        minsl = (double)ms * (1.0 - 1e-6);
        int a, b, ex, ez;
        fam(family, a, b, ex, ez);
        kS = a * S.x + b * S.y;
        k0 = a * R0.x + b * R0.y;
        fsgn = kS > k0 ? 1 : -1;
    }
    for (int guard = 0; guard < max_pts; ++guard) {
        int f, kk, m0;
        if constexpr (!FIXED) {
            if (hypot(px - S.x, pz - S.y) < 1.6) {
                if (px != S.x || pz != S.y) {
                    keep(px, pz, (double)S.x, (double)S.y);
                    if (lane == 0) path[n] = make_float2((float)S.x, (float)S.y);
                    ++n;
                }
                reached = true;
                break;
            }
            if (n + 1 >= max_pts) break;
            // family making the largest angle with the direction of travel (first wins ties)
            f = 0;
            double best = 2.0;
            const double dl = sqrt(dx * dx + dz * dz);
            for (int q = 0; q < 4; ++q) {
                int a, b, ex, ez;
                fam(q, a, b, ex, ez);
                const double c = fabs(dx * ex + dz * ez) / (dl * sqrt((double)(ex * ex + ez * ez)));
                if (c < best) { best = c; f = q; }
            }
            int fnx, fnz, ex, ez;
            fam(f, fnx, fnz, ex, ez);
            const double dn = dx * fnx + dz * fnz;
            const int sgn = dn > 0.0 ? 1 : -1;
            const double ip = px * fnx + pz * fnz;
            kk = (int)floor(ip + 0.5) + sgn;
            const double st = (kk - ip) / dn;
            const double xs = px + st * dx, zs = pz + st * dz;
            m0 = (int)floor((f == 0 ? zs : xs) + 0.5);
        } else {
            f = family;
            int fnx, fnz, ex, ez;
            fam(f, fnx, fnz, ex, ez);
            kk = (int)floor(px * fnx + pz * fnz + 0.5) + fsgn;
            // the next plane is S's (or the start lies on it): close with S
            if (kS == k0 || (kk - kS) * fsgn >= 0) {
                keep(px, pz, (double)S.x, (double)S.y);
                if (lane == 0) path[n] = make_float2((float)S.x, (float)S.y);
                ++n;
                reached = true;
                break;
            }
            if (n + 1 >= max_pts) break;
            // every grid node of the plane first (the lanes stride over them), then the
            // fine window around the best: smallest cost, then lowest parameter.  A node's
            // cost is at least lb = T + length at the smallest slowness of the tables, so
            // with c* the exact cost of the node of smallest lb, only nodes with lb <= c*
            // are walked; the others cost more than c* and cannot be the best.
            int lo, hi;
            plane_range(M.nx, M.nz, f, kk, lo, hi);
            double blb = INFINITY;
            int blm = lo;
            for (int mm = lo + lane; mm <= hi; mm += 64) {
                int ci, cj;
                fam_node(f, kk, mm, ci, cj);
                const double tc = field_at<treal>(T, M.nx, M.nz, ci, cj);
                const double lb = tc + sqrt((ci - px) * (ci - px) + (cj - pz) * (cj - pz)) * M.h * minsl;
                if (lb < blb) { blb = lb; blm = mm; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(blb, off);
                const int om = __shfl_xor(blm, off);
                if (ob < blb || (ob == blb && om < blm)) { blb = ob; blm = om; }
            }
            if (!(blb < INFINITY)) break;
            double cstar = 0.0;
            if (lane == 0) {
                int ci, cj;
                fam_node(f, kk, blm, ci, cj);
                cstar = segment_time(M, tab, px, pz, (double)ci, (double)cj) + field_at<treal>(T, M.nx, M.nz, ci, cj);
            }
            cstar = __shfl(cstar, 0);
            double bc = INFINITY;
            int bm = lo;
            for (int mm = lo + lane; mm <= hi; mm += 64) {
                int ci, cj;
                fam_node(f, kk, mm, ci, cj);
                const double tc = field_at<treal>(T, M.nx, M.nz, ci, cj);
                const double lb = tc + sqrt((ci - px) * (ci - px) + (cj - pz) * (cj - pz)) * M.h * minsl;
                if (tc < INFINITY && lb <= cstar) {
                    const double c = segment_time(M, tab, px, pz, (double)ci, (double)cj) + tc;
                    if (c < bc) { bc = c; bm = mm; }
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double oc = __shfl_xor(bc, off);
                const int om = __shfl_xor(bm, off);
                if (oc < bc || (oc == bc && om < bm)) { bc = oc; bm = om; }
            }
            m0 = bm;
        }
        int fnx, fnz, ex, ez;
        fam(f, fnx, fnz, ex, ez);
        int i00, j00;
        fam_node(f, kk, 0, i00, j00);
        // this lane's candidate (the segment walk does not wait for the field values)
        double cost = INFINITY;
        const bool mine = lane < nc;
        if (mine) {
            const double u = m0 + (double)(lane - half) / sub;
            const int mf = (int)floor(u);
            const double w = u - mf;
            int ia, ja, ib, jb;
            fam_node(f, kk, mf, ia, ja);
            fam_node(f, kk, mf + 1, ib, jb);
            double tc = field_at<treal>(T, M.nx, M.nz, ia, ja);
            const double t1 = w != 0.0 ? field_at<treal>(T, M.nx, M.nz, ib, jb) : 0.0;
            const double seg = segment_time(M, tab, px, pz, i00 + u * ex, j00 + u * ez);
            if (w != 0.0) tc = (1.0 - w) * tc + w * t1;
            if (tc < INFINITY) cost = seg + tc;
        }
        // neighbours' costs
        double cm = __shfl_up(cost, 1);
        double cp = __shfl_down(cost, 1);
        if (lane == 0) cm = INFINITY;
        if (lane >= nc - 1) cp = INFINITY;
        const bool ok = cost < INFINITY, lok = cm < INFINITY, rok = cp < INFINITY;
        double v = INFINITY, pos = 0.0;
        if (mine && ok && (!lok || cost < cm) && (!rok || cost <= cp)) {
            v = cost;
            if (lok && rok) {
                const double den = cm - 2.0 * cost + cp;
                if (den > 0.0) {
                    pos = 0.5 * (cm - cp) / den;
                    v = cost - 0.125 * (cp - cm) * (cp - cm) / den;
                }
            }
        }
        // arg-min over lanes: smallest value, then lowest lane
        double bv = v;
        int bl = lane;
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off);
            const int ol = __shfl_xor(bl, off);
            if (ov < bv || (ov == bv && ol < bl)) { bv = ov; bl = ol; }
        }
        if (!(bv < INFINITY)) break;
        const double bpos = __shfl(pos, bl);
        const double ub = m0 + ((double)(bl - half) + bpos) / sub;
        const double qx = i00 + ub * ex, qz = j00 + ub * ez;
        keep(px, pz, qx, qz);
        dx = qx - px; dz = qz - pz;
        px = qx; pz = qz;
        if (lane == 0) path[n] = make_float2((float)px, (float)pz);
        ++n;
    }
    if (held) part += segment_time(M, tab, hx0, hz0, hx1, hz1);
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if (lane == 0) {
        npts[r] = reached ? n : -n;
        tray[r] = (float)part;
    }
}

// fastest of the four fixed-family rays (reached rays only; the first family wins a tie)
__global__ void k_pick(int n_rays, int max_pts, const float2* __restrict__ paths4, const int32_t* __restrict__ npts4,
                       const float* __restrict__ tray4, float2* __restrict__ paths, int32_t* __restrict__ npts,
                       float* __restrict__ tray) {
    const int r = blockIdx.x;
    int best = 0;
    for (int f = 1; f < 4; ++f) {
        const int64_t a = (int64_t)f * n_rays + r, b = (int64_t)best * n_rays + r;
        const bool fa = npts4[a] > 0, fb = npts4[b] > 0;
        if ((fa && !fb) || (fa && fb && tray4[a] < tray4[b])) best = f;
    }
    const int64_t q = (int64_t)best * n_rays + r;
    const int32_t np = npts4[q];
    const int cnt = np > 0 ? np : -np;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x)
        paths[(int64_t)r * max_pts + i] = paths4[q * max_pts + i];
    if (threadIdx.x == 0) {
        npts[r] = np;
        tray[r] = tray4[q];
    }
}

template <typename treal>
static ali_status trace_impl(ali_handle* H, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                             const uint8_t* d_mat_id, const float* d_orient, const treal* d_T,
                             const ali_node* srcs, int32_t n_src, const ali_node* recv, int32_t n_recv,
                             const ali_options* opt_in, float* d_paths, int32_t* d_npts, float* d_tray) {
    ali_options opt;
    ali_default_options(&opt);
    if (opt_in) opt = *opt_in;
    ali_status st = validate_medium(H, grid, mats, n_mats, d_mat_id, d_orient, srcs, n_src, opt.wave);
    if (st != ALI_OK) return st;
    if (!d_T || !d_paths || !d_npts || !d_tray) return H->fail(ALI_EINVAL, "ray output or field pointer is NULL");
    if (!recv || n_recv < 1) return H->fail(ALI_EINVAL, "need at least one receiver");
    for (int k = 0; k < n_recv; ++k)
        if (recv[k].i < 0 || recv[k].j < 0 || recv[k].i >= grid->nx || recv[k].j >= grid->nz)
            return H->fail(ALI_EINVAL, "receiver " + std::to_string(k) + " outside the grid");
    if (opt.ray_window < 1 || opt.ray_sub < 1 || opt.ray_window * opt.ray_sub > 32)
        return H->fail(ALI_EINVAL, "ray_window * ray_sub must be in [1, 32]");
    if (opt.ray_max_pts < 2) return H->fail(ALI_EINVAL, "ray_max_pts must be >= 2");
    if (opt.ray_planes < ALI_RAY_CHANGING || opt.ray_planes > ALI_RAY_FASTEST_FIXED)
        return H->fail(ALI_EINVAL, "unknown ray_planes");
    if (opt.d_node_A) return H->fail(ALI_EUNSUPPORTED, "ray tracing takes the material table, not per-node stiffness");
    if (opt.velocity != ALI_VEL_CHRISTOFFEL && opt.velocity != ALI_VEL_TABLE)
        return H->fail(ALI_EINVAL, "unknown velocity mode");
    if ((int64_t)n_src * n_recv > (int64_t)1 << 30) return H->fail(ALI_EINVAL, "too many rays");
    if (set_device(H) != ALI_OK) return ALI_EDEVICE;
    hipStream_t S = H->stream;

    const std::vector<ali_material> wm = wave_materials(mats, n_mats, opt.wave);
    std::vector<MatA> hm(n_mats);
    for (int k = 0; k < n_mats; ++k)
        hm[k] = MatA{wm[k].c11 / wm[k].rho, wm[k].c13 / wm[k].rho, wm[k].c33 / wm[k].rho, wm[k].c55 / wm[k].rho};
    std::vector<int2> hs(n_src), hr(n_recv);
    for (int k = 0; k < n_src; ++k) hs[k] = make_int2(srcs[k].i, srcs[k].j);
    for (int k = 0; k < n_recv; ++k) hr[k] = make_int2(recv[k].i, recv[k].j);
    void *d_ma, *d_tab, *d_src, *d_rec;
    if (!H->scratch("ray_mats", sizeof(MatA) * n_mats, &d_ma) ||
        !H->scratch("ray_tab", sizeof(float) * (GT_N + 1) * n_mats, &d_tab) ||
        !H->scratch("ray_src", sizeof(int2) * n_src, &d_src) ||
        !H->scratch("ray_rec", sizeof(int2) * n_recv, &d_rec))
        return H->fail(ALI_ENOMEM, "device scratch allocation failed");
    HIPCK(H, hipMemcpyAsync(d_ma, hm.data(), sizeof(MatA) * n_mats, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemcpyAsync(d_src, hs.data(), sizeof(int2) * n_src, hipMemcpyHostToDevice, S));
    HIPCK(H, hipMemcpyAsync(d_rec, hr.data(), sizeof(int2) * n_recv, hipMemcpyHostToDevice, S));
    void* d_gt = nullptr;
    if (opt.velocity == ALI_VEL_TABLE) {
        if (!H->scratch("ray_gt", sizeof(double) * VT_N * n_mats, &d_gt))
            return H->fail(ALI_ENOMEM, "device scratch allocation failed");
        hipLaunchKernelGGL((k_vtables<double>), dim3((unsigned)n_mats), dim3(128), 0, S, (const MatA*)d_ma,
                           (const double*)nullptr, n_mats, (double*)nullptr, (double*)d_gt);
    }
    hipLaunchKernelGGL(k_gtable, dim3((GT_N + 1 + 255) / 256, (unsigned)n_mats), dim3(256), 0, S,
                       (const MatA*)d_ma, (const double*)d_gt, n_mats, (float*)d_tab);
    HIPCK(H, hipGetLastError());
    RayMedium M{grid->nx, grid->nz, grid->h, d_mat_id, d_orient, (const float*)d_tab};
    const int n_rays = n_src * n_recv;
    const unsigned groups = (unsigned)((n_rays + RAYS_PER_GROUP - 1) / RAYS_PER_GROUP);
    auto launch = [&](int family, float2* pth, int32_t* np, float* tr) {
        const bool lds = n_mats <= RAY_LDS_MATS;
        const dim3 g(groups), b(RAYS_PER_GROUP * 64);
#define ALI_TRACE_ARGS M, n_mats, n_rays, d_T, (const int2*)d_src, (const int2*)d_rec, n_recv, opt.ray_window, \
                       opt.ray_sub, opt.ray_max_pts, family, pth, np, tr
        if (family < 0 && lds) hipLaunchKernelGGL((k_trace<treal, true, false>), g, b, 0, S, ALI_TRACE_ARGS);
        else if (family < 0) hipLaunchKernelGGL((k_trace<treal, false, false>), g, b, 0, S, ALI_TRACE_ARGS);
        else if (lds) hipLaunchKernelGGL((k_trace<treal, true, true>), g, b, 0, S, ALI_TRACE_ARGS);
        else hipLaunchKernelGGL((k_trace<treal, false, true>), g, b, 0, S, ALI_TRACE_ARGS);
#undef ALI_TRACE_ARGS
    };
    if (opt.ray_planes == ALI_RAY_FASTEST_FIXED) {
        void *d_p4, *d_n4, *d_t4;
        const size_t npath = (size_t)n_rays * opt.ray_max_pts;
        if (!H->scratch("ray_p4", sizeof(float2) * 4 * npath, &d_p4) ||
            !H->scratch("ray_n4", sizeof(int32_t) * 4 * n_rays, &d_n4) ||
            !H->scratch("ray_t4", sizeof(float) * 4 * n_rays, &d_t4))
            return H->fail(ALI_ENOMEM, "device scratch allocation failed");
        for (int f = 0; f < 4; ++f)
            launch(f, (float2*)d_p4 + f * npath, (int32_t*)d_n4 + (size_t)f * n_rays, (float*)d_t4 + (size_t)f * n_rays);
        hipLaunchKernelGGL(k_pick, dim3((unsigned)n_rays), dim3(256), 0, S, n_rays, opt.ray_max_pts,
                           (const float2*)d_p4, (const int32_t*)d_n4, (const float*)d_t4, (float2*)d_paths, d_npts,
                           d_tray);
    } else {
        launch(opt.ray_planes == ALI_RAY_CHANGING ? -1 : opt.ray_planes - 1, (float2*)d_paths, d_npts, d_tray);
    }
    HIPCK(H, hipGetLastError());
    // the host arrays above must outlive the asynchronous copies
    HIPCK(H, hipStreamSynchronize(S));
    return ALI_OK;
}

}  // namespace ali

using namespace ali;

extern "C" ali_status ali_trace_rays(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                     int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                     const float* d_T, const ali_node* srcs, int32_t n_src,
                                     const ali_node* recv, int32_t n_recv, const ali_options* opt,
                                     float* d_paths, int32_t* d_npts, float* d_tray) {
    if (!h) return ALI_EINVAL;
    return trace_impl<float>(h, grid, mats, n_mats, d_mat_id, d_orient, d_T, srcs, n_src, recv, n_recv,
                             opt, d_paths, d_npts, d_tray);
}

extern "C" ali_status ali_trace_rays_f64(ali_handle* h, const ali_grid* grid, const ali_material* mats,
                                         int32_t n_mats, const uint8_t* d_mat_id, const float* d_orient,
                                         const double* d_T, const ali_node* srcs, int32_t n_src,
                                         const ali_node* recv, int32_t n_recv, const ali_options* opt,
                                         float* d_paths, int32_t* d_npts, float* d_tray) {
    if (!h) return ALI_EINVAL;
    return trace_impl<double>(h, grid, mats, n_mats, d_mat_id, d_orient, d_T, srcs, n_src, recv, n_recv,
                              opt, d_paths, d_npts, d_tray);
}
