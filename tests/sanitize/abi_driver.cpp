// Drives the C ABI through every kind of entry point on a small medium, for a build whose
// host code carries AddressSanitizer and UndefinedBehaviorSanitizer (device code is built
// as usual).  Without a GPU it checks the calls that need none and that ali_create fails
// cleanly; with one it runs forward solves (mixed, float64, allocation-free, persistent,
// nested source grids, batch, batch with nested grids), gradients (also on the refined medium and with the velocity
// table), rays, the autotuner and error paths, and checks each status.  Exits 0 when every
// status is the expected one; the sanitizers abort on the first host memory or
// undefined-behaviour error.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>
#include <vector>

#include "../../include/ali.h"

// the handle of the GPU part, for the library's message when a check fails
static ali_handle* g_handle = nullptr;

#define CHECK(c)                                                                      \
    do {                                                                              \
        if (!(c)) {                                                                   \
            fprintf(stderr, "check failed: %s (line %d); last error: %s\n", #c, __LINE__, \
                    ali_last_error(g_handle));                                        \
            return 1;                                                                 \
        }                                                                             \
    } while (0)
#define OK(call) CHECK((call) == ALI_OK)

template <typename T> static T* dev(const std::vector<T>& v) {
    T* p = nullptr;
    if (hipMalloc(&p, sizeof(T) * (v.empty() ? 1 : v.size())) != hipSuccess) return nullptr;
    if (!v.empty() && hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return p;
}

int main() {
    ali_options o;
    ali_default_options(&o);
    CHECK(o.band_cells == 1 && o.inner_sweeps == 2 && o.persistent == 0 && o.visit_tiles == 0);
    ali_refine r;
    ali_default_refine(&r);
    CHECK(r.n_levels == 3 && r.density[0] == 27);
    for (int s = 0; s >= -6; --s) CHECK(ali_status_string((ali_status)s) != nullptr);
    CHECK(strlen(ali_last_error(nullptr)) > 0);
    CHECK(ali_destroy(nullptr) == ALI_EINVAL && ali_set_stream(nullptr, nullptr) == ALI_EINVAL);
    CHECK(ali_set_barrier_timeout(nullptr, 1.0) == ALI_EINVAL);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        ali_handle* h = nullptr;
        CHECK(ali_create(&h, 0, nullptr) == ALI_EDEVICE && h == nullptr);
        printf("abi driver: no GPU; host-only entry points ran clean\n");
        return 0;
    }
    ali_handle* h = nullptr;
    OK(ali_create(&h, 0, nullptr));
    g_handle = h;
    CHECK(ali_set_barrier_timeout(h, -1.0) == ALI_EINVAL);

    const int nx = 40, nz = 33, N = nx * nz;
    const double hh = 2e-4;
    ali_grid g{nx, nz, hh};
    std::vector<ali_material> mats(2);
    mats[0] = ali_material{241e9, 138e9, 216e9, 129e9, 129e9, 72e9, 8100.0};
    const double c11 = 5900.0 * 5900.0 * 8100.0, c55 = 3200.0 * 3200.0 * 8100.0;
    mats[1] = ali_material{c11, c11 - 2 * c55, c11, c55, c55, c55, 8100.0};
    std::vector<uint8_t> id(N);
    std::vector<float> th(N);
    std::vector<double> th64(N);
    for (int p = 0; p < N; ++p) {
        id[p] = (uint8_t)((p % nx) > nx / 2);
        th[p] = (float)(0.3 + 0.01 * (p % 7));
        th64[p] = th[p];
    }
    std::vector<ali_node> src = {{5, 0}, {30, 0}}, rec = {{3, 32}, {20, 32}, {39, 32}};
    uint8_t* d_id = dev(id);
    float* d_th = dev(th);
    double* d_th64 = dev(th64);
    float* d_T = dev(std::vector<float>(2 * N));
    double* d_T64 = dev(std::vector<double>(2 * N));
    CHECK(d_id && d_th && d_th64 && d_T && d_T64);
    ali_solve_stats st{};
    OK(ali_solve_traveltime(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, nullptr, d_T, &st));
    CHECK(st.converged == 1 && st.node_updates > 0);
    OK(ali_solve_traveltime_f64(h, &g, mats.data(), 2, d_id, d_th64, src.data(), 2, nullptr, d_T64, &st));
    OK(ali_solve_traveltime_noalloc(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, nullptr, d_T, &st));
    ali_options op = o;
    op.persistent = 1;
    {
        // the runtime refuses a cooperative launch while another process (the test runner
        // that started this driver, say) holds the device's cooperative-launch resources:
        // then the call must fail cleanly and say so
        const ali_status ps = ali_solve_traveltime(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, &op, d_T, &st);
        CHECK(ps == ALI_OK || (ps == ALI_EDEVICE && strstr(ali_last_error(h), "hipLaunchCooperativeKernel")));
        if (ps != ALI_OK) printf("abi driver: persistent launch refused by the runtime (%s)\n", ali_last_error(h));
    }
    OK(ali_solve_traveltime_refined(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, nullptr, nullptr, d_T, &st));

    // rays through the fields
    const int maxp = 256;
    float* d_paths = dev(std::vector<float>(2 * 3 * maxp * 2));
    int32_t* d_np = dev(std::vector<int32_t>(6));
    float* d_tr = dev(std::vector<float>(6));
    ali_options orays = o;
    orays.ray_max_pts = maxp;
    OK(ali_solve_traveltime(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, nullptr, d_T, &st));
    OK(ali_trace_rays(h, &g, mats.data(), 2, d_id, d_th, d_T, src.data(), 2, rec.data(), 3, &orays, d_paths, d_np,
                      d_tr));

    // gradients
    std::vector<float> gr(6, 1.0f), obs(6, 2e-6f);
    float* d_g = dev(gr);
    float* d_obs = dev(obs);
    float* d_dth = dev(std::vector<float>(N));
    float* d_dA = dev(std::vector<float>(4 * N));
    float* d_trec = dev(std::vector<float>(6));
    double* d_loss = dev(std::vector<double>(2));
    ali_adjoint_stats ast{};
    OK(ali_adjoint(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, rec.data(), 3, d_g, nullptr, nullptr, d_dth, &ast));
    CHECK(ast.converged == 1 && ast.choice_mismatches == 0);
    OK(ali_adjoint_stiffness(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, rec.data(), 3, d_g, nullptr, nullptr,
                             d_dth, d_dA, &ast));
    OK(ali_misfit_gradient(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, rec.data(), 3, d_obs, nullptr, nullptr,
                           d_trec, d_loss, d_dth, &ast));
    // the same on the 3-fold refined medium, and the gradient with the velocity table
    float* d_Tsub = dev(std::vector<float>(2 * N));
    CHECK(d_Tsub);
    OK(ali_misfit_gradient_subgrid(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, rec.data(), 3, d_obs, nullptr, 3,
                                   d_Tsub, d_trec, d_loss, d_dth, &ast));
    CHECK(ali_misfit_gradient_subgrid(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, rec.data(), 3, d_obs, nullptr,
                                      4, nullptr, d_trec, d_loss, d_dth, &ast) == ALI_EINVAL);
    ali_options otab = o;
    otab.velocity = ALI_VEL_TABLE;
    OK(ali_adjoint(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, rec.data(), 3, d_g, &otab, nullptr, d_dth, &ast));
    CHECK(ali_adjoint_stiffness(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, rec.data(), 3, d_g, &otab, nullptr,
                                d_dth, d_dA, &ast) == ALI_EUNSUPPORTED);

    // a batch of two media (the second a copy of the first), its gradient and the autotuner
    std::vector<ali_medium> media(2);
    for (int m = 0; m < 2; ++m) {
        media[m].grid = g;
        media[m].mat_offset = 0;
        media[m].n_mats = 2;
        media[m].node_offset = 0;
        media[m].src_offset = m;
        media[m].n_src = 1;
        media[m].rec_offset = 0;
        media[m].n_rec = 3;
    }
    OK(ali_solve_batch(h, media.data(), 2, mats.data(), 2, d_id, d_th, src.data(), nullptr, d_T, &st));
    OK(ali_solve_batch_refined(h, media.data(), 2, mats.data(), 2, d_id, d_th, src.data(), nullptr, nullptr, d_T,
                               &st));
    ali_refine r3;
    ali_default_refine(&r3);
    r3.subgrid = 3;
    CHECK(ali_solve_batch_refined(h, media.data(), 2, mats.data(), 2, d_id, d_th, src.data(), nullptr, &r3, d_T,
                                  &st) == ALI_EUNSUPPORTED);
    OK(ali_misfit_gradient_batch(h, media.data(), 2, mats.data(), 2, d_id, d_th, src.data(), rec.data(), d_obs,
                                 nullptr, d_trec, d_loss, d_dth, &ast));
    ali_options tuned = o;
    double ms[ALI_TUNE_CANDIDATES];
    OK(ali_autotune_batch(h, media.data(), 2, mats.data(), 2, d_id, d_th, src.data(), &tuned, d_T, ms));
    OK(ali_autotune_batch(h, media.data(), 2, mats.data(), 2, d_id, d_th, src.data(), &tuned, d_T, ms));

    // error paths: a material that is not positive definite, a source outside, a huge
    // allocation-free solve, a bad option
    std::vector<ali_material> bad = mats;
    bad[0].c13 = 1e13;
    CHECK(ali_solve_traveltime(h, &g, bad.data(), 2, d_id, d_th, src.data(), 2, nullptr, d_T, &st) == ALI_EINVAL);
    std::vector<ali_node> out = {{nx, 0}};
    CHECK(ali_solve_traveltime(h, &g, mats.data(), 2, d_id, d_th, out.data(), 1, nullptr, d_T, &st) == ALI_EINVAL);
    ali_grid big{4096, 4096, hh};
    CHECK(ali_solve_traveltime_noalloc(h, &big, mats.data(), 2, d_id, d_th, src.data(), 1, nullptr, d_T, &st) ==
          ALI_EINVAL);
    CHECK(strlen(ali_last_error(h)) > 0);
    ali_options badopt = o;
    badopt.visit_tiles = 9;
    CHECK(ali_solve_traveltime(h, &g, mats.data(), 2, d_id, d_th, src.data(), 2, &badopt, d_T, &st) == ALI_EINVAL);

    for (void* p : {(void*)d_id, (void*)d_th, (void*)d_th64, (void*)d_T, (void*)d_T64, (void*)d_paths, (void*)d_np,
                    (void*)d_tr, (void*)d_g, (void*)d_obs, (void*)d_dth, (void*)d_dA, (void*)d_trec, (void*)d_loss,
                    (void*)d_Tsub})
        (void)hipFree(p);
    const ali_status ds = ali_destroy(h);
    g_handle = nullptr;
    CHECK(ds == ALI_OK);
    printf("abi driver: every entry point ran clean\n");
    return 0;
}
