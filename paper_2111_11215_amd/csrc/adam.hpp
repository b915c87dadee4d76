// Adam update (the paper's optimiser, Sec. 5.2; rule of Kingma and Ba with
// bias correction) as one device function, shared by the streaming Adam
// kernel and the fused backward + grid update.
#pragma once
#include <cmath>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace dvgo {

struct AdamCoef {
    float lr, b1, b2, eps, inv_bc1, inv_bc2;
};

inline bool adam_hyper_ok(float beta1, float beta2, float eps, int32_t t) {
    return t >= 1 && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f;
}

// Bias corrections 1/(1 - beta^t) in double, then rounded once to float.
inline AdamCoef adam_coef(float lr, float beta1, float beta2, float eps, int32_t t) {
    AdamCoef c;
    c.lr = lr;
    c.b1 = beta1;
    c.b2 = beta2;
    c.eps = eps;
    c.inv_bc1 = static_cast<float>(1.0 / (1.0 - std::pow(static_cast<double>(beta1), t)));
    c.inv_bc2 = static_cast<float>(1.0 / (1.0 - std::pow(static_cast<double>(beta2), t)));
    return c;
}

// The moment updates are written as explicit fused multiply-adds (the new
// gradient's share rounded first), so that every kernel that inlines this
// function computes the same bits whatever the compiler would contract.
__device__ __forceinline__ void adam_update(const AdamCoef& c, float& p, float g, float& m, float& v) {
    m = __builtin_fmaf(c.b1, m, (1.0f - c.b1) * g);
    v = __builtin_fmaf(c.b2, v, ((1.0f - c.b2) * g) * g);
    const float mh = m * c.inv_bc1;
    const float vh = v * c.inv_bc2;
    p = p - (c.lr * mh) / (sqrtf(vh) + c.eps);
}

// float32 -> bfloat16 bits, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return static_cast<uint16_t>((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ uint2 bf16x4_bits(float4 p) {
    uint2 r;
    r.x = static_cast<uint32_t>(bf16_bits(p.x)) | (static_cast<uint32_t>(bf16_bits(p.y)) << 16);
    r.y = static_cast<uint32_t>(bf16_bits(p.z)) | (static_cast<uint32_t>(bf16_bits(p.w)) << 16);
    return r;
}

}  // namespace dvgo
