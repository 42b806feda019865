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

// What the forward driver leaves on the device for a following adjoint on the same
// stream: per-material and per-node constants of the medium and the source list.
template <typename real, typename mreal> struct ForwardState {
    const MatDev<mreal>* mats = nullptr;
    const mreal* geo = nullptr;      // [N][2] cos 2theta, sin 2theta
    const real* fbt = nullptr;       // [N][4] straight-ray times to 8-neighbours
    const int2* src = nullptr;       // [n_src]
    int ntx = 0, ntz = 0;
};

// Forward solve of n_src fields into the working field d_T ([n_src][nz][nx], type real).
// Validates its arguments, records H->ev0 at its start, synchronises the stream before
// returning and fills every stats field except `ms`.  Instantiated for
// <double, float, float>, <float, float, float>, <double, double, float> and
// <double, double, double>.
template <typename real, typename mreal, typename oreal>
ali_status solve_core(ali_handle* H, const ali_grid* grid, const ali_material* mats, int32_t n_mats,
                      const uint8_t* d_mat_id, const oreal* d_orient, const ali_node* srcs,
                      int32_t n_src, const ali_options& opt, real* d_T, ali_solve_stats* stats,
                      ForwardState<real, mreal>* fs);

}  // namespace ali
