// ali_capi.hip -- handle lifetime, options and status strings of the C ABI.
#include <hip/hip_runtime.h>
#include <new>

#include "ali_handle.hpp"

extern "C" void ali_default_options(ali_options* o) {
    if (!o) return;
    o->src_box_radius = 2;
    o->max_sweeps = 1000000;
    o->inner_sweeps = 2;
    o->band_cells = 1;
    o->ray_window = 4;
    o->ray_max_pts = 4096;
    o->arith = ALI_ARITH_MIXED;
    o->ray_sub = 8;
    o->graph = 1;
    o->wave = ALI_WAVE_QP;
    o->ray_planes = ALI_RAY_CHANGING;
    o->velocity = ALI_VEL_CHRISTOFFEL;
    o->d_node_A = nullptr;
    o->persistent = 0;
    o->visit_tiles = 0;
    o->adjoint_band_cells = 0;
    o->adjoint_inner_sweeps = 0;
}

extern "C" ali_status ali_create(ali_handle** out, int device, void* hip_stream) {
    if (!out) return ALI_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return ALI_EDEVICE;
    ali_handle* h = new (std::nothrow) ali_handle();
    if (!h) return ALI_ENOMEM;
    h->device = device;
    h->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess || hipEventCreate(&h->ev0) != hipSuccess ||
        hipEventCreate(&h->ev1) != hipSuccess || hipEventCreate(&h->ev2) != hipSuccess ||
        hipEventCreate(&h->ev3) != hipSuccess || hipEventCreate(&h->ev4) != hipSuccess ||
        hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void**)&h->host_count, sizeof(uint32_t) * 4, hipHostMallocDefault) != hipSuccess ||
        hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
        ali_destroy(h);
        return ALI_EDEVICE;
    }
    int wclk_khz = 0;
    if (hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || wclk_khz <= 0)
        wclk_khz = 100000;
    h->wall_clock_khz = wclk_khz;
    h->barrier_timeout_ticks = 5000LL * wclk_khz;
    for (int k = 0; k < 2 * ALI_PASS_BATCH; ++k)
        if (hipEventCreate(&h->pev[k]) != hipSuccess) {
            ali_destroy(h);
            return ALI_EDEVICE;
        }
    // the device's static scratch array (allocation-free entry point); a failed lookup
    // leaves it unset, and only that entry point then reports the error
    if (ali::static_scratch_address(device, &h->static_base, &h->static_bytes) != hipSuccess) {
        h->static_base = nullptr;
        h->static_bytes = 0;
    }
    *out = h;
    return ALI_OK;
}

extern "C" ali_status ali_destroy(ali_handle* h) {
    if (!h) return ALI_EINVAL;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : h->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->ev2) (void)hipEventDestroy(h->ev2);
    if (h->ev3) (void)hipEventDestroy(h->ev3);
    if (h->ev4) (void)hipEventDestroy(h->ev4);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (int k = 0; k < 2 * ALI_PASS_BATCH; ++k)
        if (h->pev[k]) (void)hipEventDestroy(h->pev[k]);
    if (h->host_count) (void)hipHostFree(h->host_count);
    delete h;
    return ALI_OK;
}

extern "C" ali_status ali_set_barrier_timeout(ali_handle* h, double seconds) {
    if (!h) return ALI_EINVAL;
    if (!(seconds >= 0.0) || seconds > 3600.0) return h->fail(ALI_EINVAL, "barrier timeout must be in [0, 3600] s");
    h->barrier_timeout_ticks = (long long)(seconds * 1000.0 * h->wall_clock_khz);
    return ALI_OK;
}

extern "C" ali_status ali_set_stream(ali_handle* h, void* hip_stream) {
    if (!h) return ALI_EINVAL;
    h->stream = (hipStream_t)hip_stream;
    return ALI_OK;
}

extern "C" const char* ali_status_string(ali_status s) {
    switch (s) {
        case ALI_OK: return "ok";
        case ALI_EINVAL: return "invalid argument";
        case ALI_ENOMEM: return "out of device memory";
        case ALI_EDEVICE: return "HIP device error";
        case ALI_ENOCONV: return "relaxation did not converge within max_sweeps";
        case ALI_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" const char* ali_last_error(const ali_handle* h) {
    return h ? h->err.c_str() : "null handle";
}
