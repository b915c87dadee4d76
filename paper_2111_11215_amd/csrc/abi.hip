// Status strings, last-error text and per-device properties of the library.
#include <cstdio>

#include "common.hpp"

namespace dvgo {

namespace {
thread_local char g_last_error[256] = {0};
constexpr int kMaxDevices = 64;
int g_cu_count[kMaxDevices] = {0};
}  // namespace

// ---- optional per-kernel timing: events around every launch of one kernel
namespace {
constexpr int kMaxPairs = 8192;
int g_prof_target = -1;
int g_prof_pairs = 0;
hipEvent_t g_ev[kMaxPairs][2];
bool g_ev_made = false;
double g_prof_ms = 0.0;
int64_t g_prof_launches = 0;

void prof_flush() {
    for (int i = 0; i < g_prof_pairs; ++i) {
        hipEventSynchronize(g_ev[i][1]);
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, g_ev[i][0], g_ev[i][1]) == hipSuccess) {
            g_prof_ms += ms;
            ++g_prof_launches;
        }
    }
    g_prof_pairs = 0;
}
}  // namespace

void prof_begin(int id, hipStream_t s) {
    if (id != g_prof_target) return;
    if (!g_ev_made) {
        for (int i = 0; i < kMaxPairs; ++i) {
            hipEventCreate(&g_ev[i][0]);
            hipEventCreate(&g_ev[i][1]);
        }
        g_ev_made = true;
    }
    if (g_prof_pairs == kMaxPairs) prof_flush();
    hipEventRecord(g_ev[g_prof_pairs][0], s);
}

void prof_end(int id, hipStream_t s) {
    if (id != g_prof_target) return;
    hipEventRecord(g_ev[g_prof_pairs][1], s);
    ++g_prof_pairs;
}

void record_hip_error(hipError_t e) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", hipGetErrorName(e), hipGetErrorString(e));
}

void record_text(const char* msg) { std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    if (g_cu_count[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        g_cu_count[dev] = n;
    }
    return g_cu_count[dev];
}

}  // namespace dvgo

extern "C" {

const char* dvgo_status_string(int32_t status) {
    switch (status) {
        case DVGO_OK: return "ok";
        case DVGO_E_ARG: return "invalid argument (null pointer, negative size or bad value)";
        case DVGO_E_SHAPE: return "inconsistent or unsupported sizes";
        case DVGO_E_DTYPE: return "unsupported element type or precision";
        case DVGO_E_CAPACITY: return "buffer or workspace too small";
        case DVGO_E_HIP: return "HIP launch failed (see dvgo_last_error)";
        case DVGO_E_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char* dvgo_last_error(void) { return dvgo::g_last_error; }

int32_t dvgo_version(void) { return 1; }

int32_t dvgo_profile_enable(int32_t kernel_id) {
    if (kernel_id < -1 || kernel_id >= dvgo::K_NUM_KERNELS) return DVGO_E_ARG;
    dvgo::prof_flush();
    dvgo::g_prof_target = kernel_id;
    dvgo::g_prof_ms = 0.0;
    dvgo::g_prof_launches = 0;
    return DVGO_OK;
}

int32_t dvgo_profile_read(double* total_ms, int64_t* launches) {
    if (!total_ms || !launches) return DVGO_E_ARG;
    dvgo::prof_flush();
    *total_ms = dvgo::g_prof_ms;
    *launches = dvgo::g_prof_launches;
    return DVGO_OK;
}

}  // extern "C"
