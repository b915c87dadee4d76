// Photometric loss (paper Eq. photo_loss) and the fused Adam step (the
// paper's optimiser, Sec. 5.2; update rule of Kingma and Ba with bias
// correction).  Both are streaming kernels bound by HBM bandwidth.
#include "adam.hpp"
#include "common.hpp"

namespace {

struct AdamArgs {
    float* p;
    float* g;
    float* m;
    float* v;
    uint16_t* shadow;
    int64_t n;
    dvgo::AdamCoef c;
};

// 16-byte vectors: every pointer 16-byte aligned, n4 = n/4 vectors; the
// last n % 4 values are taken by the first threads of the grid.
__global__ __launch_bounds__(256) void adam_vec_kernel(AdamArgs a) {
    const int64_t n4 = a.n >> 2;
    float4* P = reinterpret_cast<float4*>(a.p);
    float4* G = reinterpret_cast<float4*>(a.g);
    float4* M = reinterpret_cast<float4*>(a.m);
    float4* V = reinterpret_cast<float4*>(a.v);
    const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (int64_t i = tid; i < n4; i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        float4 p = P[i], g = G[i], m = M[i], v = V[i];
        dvgo::adam_update(a.c, p.x, g.x, m.x, v.x);
        dvgo::adam_update(a.c, p.y, g.y, m.y, v.y);
        dvgo::adam_update(a.c, p.z, g.z, m.z, v.z);
        dvgo::adam_update(a.c, p.w, g.w, m.w, v.w);
        P[i] = p;
        M[i] = m;
        V[i] = v;
        G[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (a.shadow) reinterpret_cast<uint2*>(a.shadow)[i] = dvgo::bf16x4_bits(p);
    }
    const int64_t t = 4 * n4 + tid;
    if (t < a.n) {
        float p = a.p[t], m = a.m[t], v = a.v[t];
        dvgo::adam_update(a.c, p, a.g[t], m, v);
        a.p[t] = p;
        a.m[t] = m;
        a.v[t] = v;
        a.g[t] = 0.0f;
        if (a.shadow) a.shadow[t] = dvgo::bf16_bits(p);
    }
}

__global__ __launch_bounds__(256) void adam_scalar_kernel(AdamArgs a, int64_t start) {
    for (int64_t i = start + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        float p = a.p[i], m = a.m[i], v = a.v[i];
        dvgo::adam_update(a.c, p, a.g[i], m, v);
        a.p[i] = p;
        a.m[i] = m;
        a.v[i] = v;
        a.g[i] = 0.0f;
        if (a.shadow) a.shadow[i] = dvgo::bf16_bits(p);
    }
}

// Single workgroup: grad = 2 (rgb - target)/B, loss = sum ||.||^2 / B.
__global__ __launch_bounds__(1024) void photo_loss_kernel(const float* __restrict__ rgb,
                                                         const float* __restrict__ target, int B,
                                                         float* __restrict__ grad, float* __restrict__ loss) {
    __shared__ float red[16];
    const float invB = 1.0f / static_cast<float>(B);
    float acc = 0.0f;
    for (int64_t i = threadIdx.x; i < 3LL * B; i += blockDim.x) {
        const float d = rgb[i] - target[i];
        acc += d * d;
        grad[i] = 2.0f * d * invB;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0 && loss) {
        float s = 0.0f;
        for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) s += red[w];
        *loss = s * invB;
    }
}

// Single workgroup: thread t adds the listed rays t, t + 256, ... in float64
// (each product of two float32 values is exact in float64; the three
// channels in order), then a fixed-shape tree sums the 256 partials, so the
// result does not depend on scheduling.  Ray indices outside [0, B) are
// skipped.
__global__ __launch_bounds__(256) void fd_reduce_kernel(const float* __restrict__ rgb,
                                                       const float* __restrict__ weight,
                                                       const int32_t* __restrict__ rays, int n, int B,
                                                       double* __restrict__ out) {
    __shared__ double part[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const int r = rays ? rays[i] : i;
        if (r < 0 || r >= B) continue;
        for (int c = 0; c < 3; ++c)
            acc += static_cast<double>(weight[3 * r + c]) * static_cast<double>(rgb[3 * r + c]);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0];
}

}  // namespace

extern "C" {

int32_t dvgo_fd_reduce_f64(const float* rgb, const float* weight, const int32_t* rays, int32_t n, int32_t B,
                           double* out, void* stream) {
    if (n < 0 || B < 0 || !out) return DVGO_E_ARG;
    if (!rays && n > B) return DVGO_E_SHAPE;
    if (n > 0 && (!rgb || !weight)) return DVGO_E_ARG;
    hipLaunchKernelGGL(fd_reduce_kernel, dim3(1), dim3(256), 0, dvgo::as_stream(stream), rgb, weight, rays, n, B,
                       out);
    return dvgo::launch_status();
}

int32_t dvgo_photo_loss(const float* rgb, const float* target, int32_t B, float* grad_rgb, float* loss,
                        void* stream) {
    if (B < 0) return DVGO_E_ARG;
    if (B > 0 && (!rgb || !target || !grad_rgb)) return DVGO_E_ARG;
    if (B == 0) return DVGO_OK;
    DVGO_LAUNCH(K_PHOTO_LOSS, photo_loss_kernel, dim3(1), dim3(1024), 0, dvgo::as_stream(stream), rgb, target, B,
                       grad_rgb, loss);
    return dvgo::launch_status();
}

int32_t dvgo_adam_step(float* p, float* g, float* m, float* v, uint16_t* shadow_bf16, int64_t n, float lr,
                       float beta1, float beta2, float eps, int32_t t, void* stream) {
    if (n < 0 || t < 1) return DVGO_E_ARG;
    if (n > 0 && (!p || !g || !m || !v)) return DVGO_E_ARG;
    if (!dvgo::adam_hyper_ok(beta1, beta2, eps, t)) return DVGO_E_ARG;
    if (n == 0) return DVGO_OK;
    AdamArgs a;
    a.p = p;
    a.g = g;
    a.m = m;
    a.v = v;
    a.shadow = shadow_bf16;
    a.n = n;
    a.c = dvgo::adam_coef(lr, beta1, beta2, eps, t);
    hipStream_t s = dvgo::as_stream(stream);
    auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    const bool vec = al16(p) && al16(g) && al16(m) && al16(v) &&
                     (!shadow_bf16 || (reinterpret_cast<uintptr_t>(shadow_bf16) & 7u) == 0);
    const int cus = dvgo::device_cu_count();
    int64_t done = 0;
    if (vec && n >= 4) {
        const int64_t n4 = n >> 2;
        int64_t blocks = (n4 + 255) / 256;
        if (blocks > static_cast<int64_t>(cus) * 8) blocks = static_cast<int64_t>(cus) * 8;
        DVGO_LAUNCH(K_ADAM, adam_vec_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a);
        if (int32_t st = dvgo::launch_status()) return st;
        done = n;   // the tail (n % 4 < 256 values) is handled in the same launch
    }
    if (done < n) {
        int64_t blocks = (n - done + 255) / 256;
        if (blocks > static_cast<int64_t>(cus) * 8) blocks = static_cast<int64_t>(cus) * 8;
        DVGO_LAUNCH(K_ADAM, adam_scalar_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a, done);
        if (int32_t st = dvgo::launch_status()) return st;
    }
    return DVGO_OK;
}

}  // extern "C"
