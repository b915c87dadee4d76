// Internal helpers shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "dvgo.h"

namespace dvgo {

// Records the last HIP error text for dvgo_last_error().
void record_hip_error(hipError_t e);
// Records a library message as the dvgo_last_error() text.
void record_text(const char* msg);

// Checks the launch just enqueued; returns DVGO_OK or DVGO_E_HIP.
inline int32_t launch_status() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        record_hip_error(e);
        return DVGO_E_HIP;
    }
    return DVGO_OK;
}

// Number of compute units of the current device (cached per device).
int device_cu_count();

// Kernel identifiers of the optional per-kernel event timing.
enum KernelId {
    K_RAY_SETUP = 0, K_MORTON_SORT, K_COUNT_KEPT, K_SCAN, K_FILL_KEPT, K_COARSE_MASK,
    K_PACK, K_RAY_BASE, K_GATHER, K_MLP_FWD, K_COMPOSE_FWD, K_COMPOSE_BWD, K_MLP_BWD, K_SCATTER,
    K_REDUCE, K_PHOTO_LOSS, K_ADAM, K_PROP_FWD, K_PROP_BWD, K_PROP_REDUCE, K_SCENE, K_BIN_COUNT,
    K_CELL_SCAN, K_BIN_PLACE, K_GRID_ADAM, K_GRID_ACTIVE, K_TOY_PIXEL, K_TOY_VERTEX, K_TOY_REDUCE, K_GRID_RESAMPLE, K_COARSE_STEP, K_VIEW_COUNT, K_NUM_KERNELS
};
// Bracket one launch with events when timing of `id` is enabled.
void prof_begin(int id, hipStream_t s);
void prof_end(int id, hipStream_t s);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// hipLaunchKernelGGL bracketed by the optional timing events of kernel `id`.
#define DVGO_LAUNCH(id, kernel, grid, block, shmem, stream, ...)                  \
    do {                                                                       \
        ::dvgo::prof_begin(::dvgo::id, (stream));                              \
        hipLaunchKernelGGL(kernel, grid, block, shmem, (stream), __VA_ARGS__); \
        ::dvgo::prof_end(::dvgo::id, (stream));                                \
    } while (0)

inline bool box_ok(const dvgo_box* b, int min_n) {
    if (!b) return false;
    for (int i = 0; i < 3; ++i) {
        if (!(b->xyz_max[i] > b->xyz_min[i])) return false;
        if (b->n[i] < min_n) return false;
    }
    return true;
}

// Grid description passed by value to kernels.  `scale` is (n-1)/(max-min)
// rounded once to float32 on the host.
struct GridArgs {
    float mn[3];
    float scale[3];
    int n[3];
};

inline GridArgs make_grid(const dvgo_box& b) {
    GridArgs g;
    for (int i = 0; i < 3; ++i) {
        g.mn[i] = b.xyz_min[i];
        volatile float span = b.xyz_max[i] - b.xyz_min[i];
        volatile float nm1 = static_cast<float>(b.n[i] - 1);
        g.scale[i] = nm1 / span;
        g.n[i] = b.n[i];
    }
    return g;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace dvgo

// ---------------------------------------------------------------------------
// Device-side float32 recipe of the discrete sampler (no contraction).
// ---------------------------------------------------------------------------
namespace dvgo_dev {

// t_k = t_near + ((float)k + p) * step, three roundings in this order.
__device__ __forceinline__ float recipe_tk(float tn, float p, int k, float step) {
#pragma clang fp contract(off)
    float kp = static_cast<float>(k) + p;
    float m = kp * step;
    return tn + m;
}

// x = o + t * d per component (multiply, then add).
__device__ __forceinline__ void recipe_x(const float o[3], const float d[3], float t, float x[3]) {
#pragma clang fp contract(off)
    for (int i = 0; i < 3; ++i) {
        float m = t * d[i];
        x[i] = o[i] + m;
    }
}

// Slab clip of the ray o + t d against the box [mn, mx] (float32 recipe, no
// contraction): per axis with d_i != 0, t0 = (mn_i - o_i) * (1/d_i) and
// t1 = (mx_i - o_i) * (1/d_i); a zero component misses unless o_i lies in
// the slab.  t_near = max(0, max_i min(t0, t1)), t_far = min_i max(t0, t1);
// the ray is valid iff it does not miss and t_near < t_far.
__device__ __forceinline__ bool recipe_slab(const float o[3], const float d[3], const float mn[3], const float mx[3],
                                            float* t_near, float* t_far) {
#pragma clang fp contract(off)
    float te = -INFINITY, tx = INFINITY;
    bool miss = false;
    for (int i = 0; i < 3; ++i) {
        if (d[i] == 0.0f) {
            if (o[i] < mn[i] || o[i] > mx[i]) miss = true;
        } else {
            const float inv = 1.0f / d[i];
            const float t0 = (mn[i] - o[i]) * inv;
            const float t1 = (mx[i] - o[i]) * inv;
            te = fmaxf(te, fminf(t0, t1));
            tx = fminf(tx, fmaxf(t0, t1));
        }
    }
    *t_near = fmaxf(te, 0.0f);
    *t_far = tx;
    return !miss && (*t_near < tx);
}

// Cell of the coarse grid holding x: clamp(floor((x-min)*scale), 0, n-2).
__device__ __forceinline__ int recipe_cell(const dvgo::GridArgs& g, const float x[3]) {
#pragma clang fp contract(off)
    int idx[3];
    for (int i = 0; i < 3; ++i) {
        float u = (x[i] - g.mn[i]) * g.scale[i];
        float fl = floorf(u);
        fl = fminf(fmaxf(fl, 0.0f), static_cast<float>(g.n[i] - 2));
        idx[i] = static_cast<int>(fl);
    }
    return (idx[0] * (g.n[1] - 1) + idx[1]) * (g.n[2] - 1) + idx[2];
}

// Trilinear interpolation of a float32 vertex grid for a discrete decision,
// in a fixed float32 recipe: per axis u = (x-min)*scale, fl = clamp(floor(u),
// 0, n-2), f = clamp(u-fl, 0, 1); corner c = (c>>2 &1, c>>1 &1, c &1) has
// weight (gx*gy)*gz; the value adds w_c*V_c one product at a time in corner
// order.
__device__ __forceinline__ float recipe_trilerp(const dvgo::GridArgs& g, const float* __restrict__ v,
                                                const float x[3]) {
#pragma clang fp contract(off)
    int i0[3];
    float gw[3][2];
    for (int i = 0; i < 3; ++i) {
        const float u = (x[i] - g.mn[i]) * g.scale[i];
        const float fl = fminf(fmaxf(floorf(u), 0.0f), static_cast<float>(g.n[i] - 2));
        const float f = fminf(fmaxf(u - fl, 0.0f), 1.0f);
        i0[i] = static_cast<int>(fl);
        gw[i][0] = 1.0f - f;
        gw[i][1] = f;
    }
    const int64_t sx = static_cast<int64_t>(g.n[1]) * g.n[2], sy = g.n[2];
    const int64_t base = i0[0] * sx + i0[1] * sy + i0[2];
    float c[8];
    for (int k = 0; k < 8; ++k) c[k] = v[base + ((k >> 2) & 1) * sx + ((k >> 1) & 1) * sy + (k & 1)];
    float val = 0.0f;
    for (int k = 0; k < 8; ++k) {
        const float w = (gw[0][(k >> 2) & 1] * gw[1][(k >> 1) & 1]) * gw[2][k & 1];
        const float term = w * c[k];
        val = k == 0 ? term : val + term;
    }
    return val;
}

// Sine and cosine of x for |x| <= 1024, for the encoded query position
// (whose arguments 2^j u stay within 16 in magnitude): Cody and Waite's
// reduction x = k pi/2 + r with pi/2 split into three parts (the first two
// with 12 significant bits, so that k times each is exact for |k| < 2^12),
// then the Taylor series of sin and cos on |r| <= pi/4 to the terms in r^11
// and r^12 (the first omitted terms are below 1e-11) in Horner form, and
// the quadrant k mod 4 picks and signs the pair.  About one unit in the last
// place, and free of the large-argument path that the library's sincosf
// carries in registers.
__device__ __forceinline__ void pe_sincos(float x, float* s, float* c) {
    constexpr float kTwoOverPi = 0x1.45f306p-1f;
    constexpr float kP1 = 0x1.922p+0f, kP2 = -0x1.2aep-18f, kP3 = -0x1.de974p-31f;
    const float k = rintf(x * kTwoOverPi);
    float r = fmaf(-k, kP1, x);
    r = fmaf(-k, kP2, r);
    r = fmaf(-k, kP3, r);
    const float r2 = r * r;
    float ps = -1.0f / 39916800.0f;
    ps = fmaf(ps, r2, 1.0f / 362880.0f);
    ps = fmaf(ps, r2, -1.0f / 5040.0f);
    ps = fmaf(ps, r2, 1.0f / 120.0f);
    ps = fmaf(ps, r2, -1.0f / 6.0f);
    const float sr = fmaf(ps * r2, r, r);
    float pc = 1.0f / 479001600.0f;
    pc = fmaf(pc, r2, -1.0f / 3628800.0f);
    pc = fmaf(pc, r2, 1.0f / 40320.0f);
    pc = fmaf(pc, r2, -1.0f / 720.0f);
    pc = fmaf(pc, r2, 1.0f / 24.0f);
    pc = fmaf(pc, r2, -0.5f);
    const float cr = fmaf(pc, r2, 1.0f);
    const int q = static_cast<int>(k) & 3;
    const float a = (q & 1) ? cr : sr, b = (q & 1) ? sr : cr;
    *s = (q & 2) ? -a : a;
    *c = ((q + 1) & 2) ? -b : b;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

}  // namespace dvgo_dev
