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

// a work-group owns a TX x TZ tile plus a HALO-node ring (the diamond radius) in LDS
constexpr int TX = 16, TZ = 16, HALO = 2;
constexpr int LW = TX + 2 * HALO, LH = TZ + 2 * HALO;
constexpr int LSTRIDE = LW + 1;
constexpr int NTHREADS = TX * TZ;             // nodes of a tile
constexpr int RW = 64;                        // one wave per tile visit
constexpr int NPL = NTHREADS / RW;            // nodes per lane
constexpr int NODE_WORDS = NTHREADS / 32;     // 32-bit words of a per-tile node mask
constexpr int STAT_SLOTS = 256;               // spread of the statistics counters

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
                                                const MatDev<mreal>* __restrict__ mats,
                                                const uint8_t* __restrict__ mat_id,
                                                const mreal* __restrict__ geo,
                                                const real* __restrict__ fbt) {
    const MatDev<mreal>& m = mats[mat_id[p]];
    nc.P = m.P; nc.Q = m.Q; nc.R = m.R; nc.K4 = m.K4;
    nc.c2t = geo[2 * p + 0];
    nc.s2t = geo[2 * p + 1];
#pragma unroll
    for (int d = 0; d < 4; ++d) nc.fb[d] = fbt[4 * p + d];
}

// One field of a batch: a source in a medium.  Offsets count elements.
struct FieldDev {
    int nx, nz, ntx, ntz;
    double h;             // node spacing of the medium
    int64_t node_off;     // the medium's first node in the per-node arrays (materials, orientation)
    int64_t t_off;        // the field's first node in the per-field arrays (travel times)
    uint32_t unit_off;    // the field's first tile unit (flags, thresholds, node marks)
    int mat_off;          // the medium's first entry in the device material table
    int medium;
    int rec_off, n_rec;   // the medium's receivers (gradient calls)
    int obs_off;          // the field's first entry in per-receiver arrays
    int2 src;
};

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
    const FieldDev* fields = nullptr;
    std::vector<FieldDev> hfields;
    std::vector<int> medium_first_field;   // per medium, then the total
    std::vector<double> vmax;        // fastest phase speed per medium
    int64_t n_units = 0, field_nodes = 0;
};

// Validates a batch (media, materials, sources and, when recv != NULL, receivers).
ali_status validate_batch(ali_handle* H, const ali_medium* media, int32_t n_media, const ali_material* mats,
                          int32_t n_mats, const void* d_mat_id, const void* d_orient, const ali_node* srcs,
                          const ali_node* recv);

// Forward solve of every field of a batch into the working field d_T (fields in medium
// order, each [nz][nx]; type real).  Validates its arguments, records H->ev0 at its start,
// synchronises the stream before returning and fills every stats field except `ms`.
// Instantiated for <double, float, float>, <float, float, float>, <double, double, float>
// and <double, double, double>.
template <typename real, typename mreal, typename oreal>
ali_status solve_fields(ali_handle* H, const ali_medium* media, int32_t n_media, const ali_material* mats,
                        int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient, const ali_node* srcs,
                        const ali_node* recv, const ali_options& opt, real* d_T, ali_solve_stats* stats,
                        ForwardState<real, mreal>* fs);

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
