// ali_handle.hpp -- handle state shared by the C-ABI entry points: device, stream,
// named scratch buffers grown on demand, timing events, last error message.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <map>
#include <string>
#include <vector>

#include "../../include/ali.h"

// relaxation passes queued between two host checks
constexpr int ALI_PASS_BATCH = 16;
// captured pass batches kept per handle (each signature includes the output pointer, so a
// caller that passes new buffers every call would otherwise grow the cache without bound).
// A call takes two per relaxation (first batch and the rest; a nested-grid solve two per
// level), so the bound leaves room for callers that alternate between several kinds of call.
constexpr size_t ALI_MAX_GRAPHS = 128;

struct ali_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;         // only records pass batches into graphs
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr, ev4 = nullptr;
    uint32_t* host_count = nullptr;           // pinned 4-byte readback slot
    hipEvent_t pev[2 * ALI_PASS_BATCH] = {};  // per-pass timing events of one batch
    int n_cu = 0;                             // compute units of the device
    long long barrier_timeout_ticks = 0;      // grid-barrier wait limit, ticks of the constant-rate clock
    int wall_clock_khz = 100000;              // rate of that clock
    bool coop_refused = false;                // the runtime refused the last cooperative launch
    std::map<std::string, hipGraphExec_t> graphs;   // captured pass batches by argument signature
    // autotuner choices by size bucket: candidate index and every candidate's time [ms]
    std::map<std::string, std::pair<int, std::vector<double>>> tuned;
    std::string err;
    struct Buf { void* p = nullptr; size_t bytes = 0; };
    std::map<std::string, Buf> bufs;
    // the device's static scratch array (address of the library's file-scope device array
    // on this handle's device, looked up once per device at create), and the carve-up of
    // it during an allocation-free call (arena != 0)
    void* static_base = nullptr;
    size_t static_bytes = 0;
    bool arena = false;
    size_t arena_used = 0;
    std::map<std::string, std::pair<size_t, size_t>> arena_slots;   // name -> (offset, bytes)

    ali_status fail(ali_status s, const std::string& msg) {
        err = msg;
        return s;
    }
    // device buffer `name` of at least `bytes`; contents are not preserved on growth.
    // During an allocation-free call the buffer is carved from the static array instead
    // (256-byte aligned, never hipMalloc); false if it does not fit.
    bool scratch(const char* name, size_t bytes, void** out) {
        if (arena) {
            auto it = arena_slots.find(name);
            if (it != arena_slots.end() && it->second.second >= bytes) {
                *out = (char*)static_base + it->second.first;
                return true;
            }
            const size_t off = (arena_used + 255) & ~(size_t)255;
            if (!static_base || off > static_bytes || bytes > static_bytes - off) return false;
            arena_slots[name] = std::make_pair(off, bytes);
            arena_used = off + bytes;
            *out = (char*)static_base + off;
            return true;
        }
        Buf& b = bufs[name];
        if (b.bytes < bytes) {
            if (b.p) (void)hipFree(b.p);
            b.p = nullptr;
            b.bytes = 0;
            size_t want = bytes < 256 ? 256 : bytes;
            if (hipMalloc(&b.p, want) != hipSuccess) { b.p = nullptr; return false; }
            b.bytes = want;
        }
        *out = b.p;
        return true;
    }
};

// A failed runtime call is reported through the handle; the runtime's last-error state is
// cleared, so that the failure (a refused cooperative launch, say) is not reported again by
// the error check of a later, unrelated call.
#define HIPCK(H, call)                                                                 \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (void)hipGetLastError();                                                   \
            return (H)->fail(ALI_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
        }                                                                              \
    } while (0)

namespace ali {

constexpr int PASS_BATCH = ALI_PASS_BATCH;

// Device address and size of the static scratch array of the allocation-free entry point
// on `device` (which must be current).  The address is looked up once per device and kept
// for the life of the process.
hipError_t static_scratch_address(int device, void** ptr, size_t* bytes);

// Enqueue `enqueue(b)` for b = 0 .. PASS_BATCH-1 on the handle's stream as one captured
// graph, instantiated once per signature `key` (every argument the kernels receive) and
// replayed afterwards.
// The batch is recorded on the handle's own capture stream (the caller's stream may be the
// legacy default stream, which cannot be captured) and replayed on the caller's stream.
// Callers synchronise the stream after every batch, so when the cache is full its graphs
// are idle and are all released before the next capture.
template <class F>
inline ali_status launch_captured(ali_handle* H, const std::string& key, F&& enqueue) {
    hipGraphExec_t exec = nullptr;
    auto it = H->graphs.find(key);
    if (it != H->graphs.end()) {
        exec = it->second;
    } else {
        if (H->graphs.size() >= ALI_MAX_GRAPHS) {
            for (auto& kv : H->graphs) (void)hipGraphExecDestroy(kv.second);
            H->graphs.clear();
        }
        hipGraph_t graph = nullptr;
        HIPCK(H, hipStreamBeginCapture(H->cap_stream, hipStreamCaptureModeThreadLocal));
        for (int b = 0; b < PASS_BATCH; ++b) enqueue(b, H->cap_stream);
        const hipError_t le = hipGetLastError();
        HIPCK(H, hipStreamEndCapture(H->cap_stream, &graph));
        if (le != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return H->fail(ALI_EDEVICE, std::string("launch during capture: ") + hipGetErrorString(le));
        }
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) return H->fail(ALI_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        H->graphs[key] = exec;
    }
    HIPCK(H, hipGraphLaunch(exec, H->stream));
    return ALI_OK;
}

// signature of a pass batch: the pointer and scalar arguments, printed
template <typename... A>
inline std::string graph_key(const char* tag, A... a) {
    std::string k(tag);
    const unsigned long long v[] = {(unsigned long long)a...};
    char buf[24];
    for (unsigned long long x : v) { snprintf(buf, sizeof(buf), ":%llx", x); k += buf; }
    return k;
}

inline ali_status set_device(ali_handle* H) {
    HIPCK(H, hipSetDevice(H->device));
    return ALI_OK;
}

// one material record, checked for the wave of the call
inline ali_status check_material(ali_handle* H, const ali_material& m, int k, int wave) {
    const double v[7] = {m.c11, m.c13, m.c33, m.c55, m.c44, m.c66, m.rho};
    for (double x : v)
        if (!isfinite(x)) return H->fail(ALI_EINVAL, "material " + std::to_string(k) + " has a non-finite entry");
    if (!(m.rho > 0.0)) return H->fail(ALI_EINVAL, "material " + std::to_string(k) + ": rho must be > 0");
    if (wave == ALI_WAVE_SH) {
        if (!(m.c44 > 0.0 && m.c66 > 0.0))
            return H->fail(ALI_EINVAL, "material " + std::to_string(k) + ": c44, c66 must be > 0 (SH)");
        return ALI_OK;
    }
    if (wave != ALI_WAVE_QP) return H->fail(ALI_EINVAL, "unknown wave");
    if (!(m.c11 > 0.0 && m.c33 > 0.0 && m.c55 > 0.0))
        return H->fail(ALI_EINVAL, "material " + std::to_string(k) + ": c11, c33, c55 must be > 0");
    if (!(m.c11 * m.c33 > m.c13 * m.c13))
        return H->fail(ALI_EINVAL, "material " + std::to_string(k) + ": c11*c33 must exceed c13^2");
    return ALI_OK;
}

// The record the kernels use.  For SH: c11 = c66, c33 = c44, c55 = min(c44, c66),
// c13 = -c55.  Its in-plane Christoffel matrix is diagonal, (c66 s^2 + c55 c^2,
// c55 s^2 + c44 c^2) / rho for s, c of the angle from the axis, and with c55 the smaller
// of c44, c66 the larger entry is (c66 s^2 + c44 c^2) / rho at every angle: the SH entry.
// The qP root, its group velocity and every derivative are then those of SH.
inline ali_material wave_record(const ali_material& m, int wave) {
    if (wave != ALI_WAVE_SH) return m;
    ali_material r = m;
    r.c11 = m.c66;
    r.c33 = m.c44;
    r.c55 = m.c44 < m.c66 ? m.c44 : m.c66;
    r.c13 = -r.c55;
    return r;
}

inline std::vector<ali_material> wave_materials(const ali_material* mats, int n_mats, int wave) {
    std::vector<ali_material> out(n_mats > 0 ? n_mats : 0);
    for (int k = 0; k < n_mats; ++k) out[k] = wave_record(mats[k], wave);
    return out;
}

// host-side validation shared by every entry point taking a medium
template <typename oreal>
inline ali_status validate_medium(ali_handle* H, const ali_grid* g, const ali_material* mats,
                                  int32_t n_mats, const uint8_t* d_mat_id, const oreal* d_orient,
                                  const ali_node* srcs, int32_t n_src, int wave = ALI_WAVE_QP) {
    if (!g) return H->fail(ALI_EINVAL, "grid is NULL");
    if (g->nx < 3 || g->nz < 3) return H->fail(ALI_EINVAL, "grid needs nx, nz >= 3");
    if ((int64_t)g->nx * g->nz > (int64_t)1 << 31) return H->fail(ALI_EINVAL, "grid too large");
    if (!(g->h > 0.0) || !isfinite(g->h)) return H->fail(ALI_EINVAL, "grid spacing h must be finite and > 0");
    if (!mats || n_mats < 1 || n_mats > 256) return H->fail(ALI_EINVAL, "need 1..256 materials");
    for (int k = 0; k < n_mats; ++k) {
        const ali_status st = check_material(H, mats[k], k, wave);
        if (st != ALI_OK) return st;
    }
    if (!d_mat_id || !d_orient) return H->fail(ALI_EINVAL, "medium arrays are NULL");
    if (!srcs || n_src < 1) return H->fail(ALI_EINVAL, "need at least one source");
    for (int k = 0; k < n_src; ++k)
        if (srcs[k].i < 0 || srcs[k].j < 0 || srcs[k].i >= g->nx || srcs[k].j >= g->nz)
            return H->fail(ALI_EINVAL, "source " + std::to_string(k) + " outside the grid");
    return ALI_OK;
}

}  // namespace ali
