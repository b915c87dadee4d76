// Learned proposal (not in the paper): a small network that predicts, per
// ray, how the compositing weight is spread over 32 equal-count segments of
// its uniform samples, and the segment mask that keeps the segments holding
// most of it.  Inputs and weights are rounded to bfloat16, products are
// accumulated in float32; the selection runs in float64 so that it is
// reproducible from the float32 logits.
#include "common.hpp"

namespace {

constexpr int kIn = 54, kH = 64, kS = 32;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kS * kH, kParams = kOffB3 + kS;
constexpr int kPStride = (kParams + 63) / 64 * 64;
constexpr int kRaysPerBlock = 64;

__device__ __forceinline__ float bf16_round(float f) {   // round to nearest even, keep as float
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return f;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

struct PropArgs {
    const float* rays_o;
    const float* rays_d;
    const float* t_near;
    const uint8_t* valid;
    int B;
    float mn[3], mx[3];
    const float* w[3];
    const float* b[3];
};

// Load weights (bf16-rounded) and biases (float32) into LDS, flat layout.
__device__ void load_weights(const PropArgs& a, float* sw) {
    for (int i = threadIdx.x; i < kParams; i += blockDim.x) {
        float v;
        if (i < kOffB1) v = bf16_round(a.w[0][i - kOffW1]);
        else if (i < kOffW2) v = a.b[0][i - kOffB1];
        else if (i < kOffB2) v = bf16_round(a.w[1][i - kOffW2]);
        else if (i < kOffW3) v = a.b[1][i - kOffB2];
        else if (i < kOffB3) v = bf16_round(a.w[2][i - kOffW3]);
        else v = a.b[2][i - kOffB3];
        sw[i] = v;
    }
}

// Encoding: PE4 of the box-entry point in box coordinates, then PE4 of d.
__device__ void encode(const PropArgs& a, int r, float e[kIn]) {
    float d[3], u[3];
    const float tn = a.t_near[r];
    for (int i = 0; i < 3; ++i) {
        d[i] = a.rays_d[3 * r + i];
        const float x0 = a.rays_o[3 * r + i] + tn * d[i];
        u[i] = (x0 - 0.5f * (a.mn[i] + a.mx[i])) / (0.5f * (a.mx[i] - a.mn[i]));
    }
    const float* src[2] = {u, d};
    for (int part = 0; part < 2; ++part) {
        float* out = e + 27 * part;
        for (int c = 0; c < 3; ++c) out[c] = src[part][c];
        for (int fq = 0; fq < 4; ++fq)
            for (int c = 0; c < 3; ++c) {
                float sv, cv;
                sincosf(src[part][c] * static_cast<float>(1 << fq), &sv, &cv);
                out[3 + 6 * fq + c] = sv;
                out[6 + 6 * fq + c] = cv;
            }
    }
    for (int i = 0; i < kIn; ++i) e[i] = bf16_round(e[i]);
}

// Forward of one ray; h1, h2 are post-ReLU and rounded to bfloat16.
__device__ void forward(const float* sw, const float e[kIn], float h1[kH], float h2[kH], float z[kS]) {
    for (int o = 0; o < kH; ++o) {
        float acc = sw[kOffB1 + o];
        for (int k = 0; k < kIn; ++k) acc += sw[kOffW1 + o * kIn + k] * e[k];
        h1[o] = bf16_round(fmaxf(acc, 0.0f));
    }
    for (int o = 0; o < kH; ++o) {
        float acc = sw[kOffB2 + o];
        for (int k = 0; k < kH; ++k) acc += sw[kOffW2 + o * kH + k] * h1[k];
        h2[o] = bf16_round(fmaxf(acc, 0.0f));
    }
    for (int o = 0; o < kS; ++o) {
        float acc = sw[kOffB3 + o];
        for (int k = 0; k < kH; ++k) acc += sw[kOffW3 + o * kH + k] * h2[k];
        z[o] = acc;
    }
}

// Segment mask from float32 logits, float64 arithmetic, sequential sums.
__device__ uint32_t select_mask(const float z[kS], double cum_frac, double min_mass, float* pred_mass) {
    double m = 0.0;
    for (int s = 0; s < kS; ++s) m = fmax(m, static_cast<double>(z[s]));
    double e[kS + 1];
    double tot = 0.0;
    for (int s = 0; s < kS; ++s) {
        e[s] = exp(static_cast<double>(z[s]) - m);
        tot += e[s];
    }
    e[kS] = exp(0.0 - m);
    tot += e[kS];
    double q[kS];
    double mass = 0.0;
    for (int s = 0; s < kS; ++s) {
        q[s] = e[s] / tot;
        mass += q[s];
    }
    *pred_mass = static_cast<float>(mass);
    if (!(mass >= min_mass)) return 0xFFFFFFFFu;
    uint32_t chosen = 0;
    double acc = 0.0;
    const double target = cum_frac * mass;
    for (int it = 0; it < kS; ++it) {
        int best = -1;
        for (int s = 0; s < kS; ++s)
            if (!((chosen >> s) & 1u) && (best < 0 || q[s] > q[best])) best = s;
        chosen |= 1u << best;
        acc += q[best];
        if (acc >= target) break;
    }
    return chosen;
}

__global__ __launch_bounds__(kRaysPerBlock) void proposal_fwd_kernel(PropArgs a, int run_net, float cum_frac,
                                                                     float min_mass, float* __restrict__ logits,
                                                                     float* __restrict__ pred_mass,
                                                                     uint32_t* __restrict__ seg_mask) {
    __shared__ float sw[kParams];
    if (run_net) load_weights(a, sw);
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.B) return;
    float z[kS];
    if (run_net) {
        float e[kIn], h1[kH], h2[kH];
        encode(a, r, e);
        forward(sw, e, h1, h2, z);
        for (int s = 0; s < kS; ++s) logits[static_cast<int64_t>(r) * kS + s] = z[s];
    } else {
        for (int s = 0; s < kS; ++s) z[s] = logits[static_cast<int64_t>(r) * kS + s];
    }
    float pm;
    uint32_t mask = select_mask(z, cum_frac, min_mass, &pm);
    if (a.valid && !a.valid[r]) mask = 0xFFFFFFFFu;
    if (pred_mass) pred_mass[r] = pm;
    if (seg_mask) seg_mask[r] = mask;
}

// Backward over 64 rays per block: per-ray adjoint in registers, activations
// staged in LDS, each lane then accumulates whole weight rows over the rays.
__global__ __launch_bounds__(kRaysPerBlock) void proposal_bwd_kernel(PropArgs a, const float* __restrict__ seg_w,
                                                                     const float* __restrict__ log_t_end,
                                                                     float* __restrict__ partial,
                                                                     float* __restrict__ loss_part) {
    __shared__ float sw[kParams];
    __shared__ float sE[kRaysPerBlock * kIn];
    __shared__ float sH1[kRaysPerBlock * kH];
    __shared__ float sH2[kRaysPerBlock * kH];
    __shared__ float sD1[kRaysPerBlock * kH];
    __shared__ float sD2[kRaysPerBlock * kH];
    __shared__ float sDz[kRaysPerBlock * kS];
    load_weights(a, sw);
    __syncthreads();
    const int t = threadIdx.x;
    const int r = blockIdx.x * blockDim.x + t;
    const bool ok = r < a.B && (!a.valid || a.valid[r]);
    float e[kIn], h1[kH], h2[kH], z[kS];
    float kl = 0.0f;
    if (r < a.B) {
        encode(a, r, e);
        forward(sw, e, h1, h2, z);
    } else {
        for (int i = 0; i < kIn; ++i) e[i] = 0.0f;
        for (int i = 0; i < kH; ++i) h1[i] = h2[i] = 0.0f;
        for (int i = 0; i < kS; ++i) z[i] = 0.0f;
    }
    float dz[kS];
    {
        float m = 0.0f;
        for (int s = 0; s < kS; ++s) m = fmaxf(m, z[s]);
        float tot = expf(-m);
        for (int s = 0; s < kS; ++s) tot += expf(z[s] - m);
        const float invB = 1.0f / static_cast<float>(a.B);
        const float logtot = logf(tot) + m;   // log of the softmax denominator
        for (int s = 0; s < kS; ++s) {
            const float q = expf(z[s] - logtot);
            const float p = ok ? seg_w[static_cast<int64_t>(r) * kS + s] : 0.0f;
            dz[s] = ok ? (q - p) * invB : 0.0f;
            if (ok && p > 0.0f) kl += p * (logf(p) - (z[s] - logtot));
        }
        if (ok) {
            const float pt = expf(log_t_end[r]);
            if (pt > 0.0f) kl += pt * (log_t_end[r] + logtot);
        }
        kl *= invB;
    }
    float d2[kH], d1[kH];
    for (int k = 0; k < kH; ++k) {
        float acc = 0.0f;
        for (int o = 0; o < kS; ++o) acc += sw[kOffW3 + o * kH + k] * dz[o];
        d2[k] = h2[k] > 0.0f ? acc : 0.0f;
    }
    for (int k = 0; k < kH; ++k) {
        float acc = 0.0f;
        for (int o = 0; o < kH; ++o) acc += sw[kOffW2 + o * kH + k] * d2[o];
        d1[k] = h1[k] > 0.0f ? acc : 0.0f;
    }
    for (int i = 0; i < kIn; ++i) sE[t * kIn + i] = e[i];
    for (int i = 0; i < kH; ++i) {
        sH1[t * kH + i] = h1[i];
        sH2[t * kH + i] = h2[i];
        sD1[t * kH + i] = d1[i];
        sD2[t * kH + i] = d2[i];
    }
    for (int i = 0; i < kS; ++i) sDz[t * kS + i] = dz[i];
    for (int off = 32; off > 0; off >>= 1) kl += __shfl_xor(kl, off, 64);
    __syncthreads();
    float* out = partial + static_cast<int64_t>(blockIdx.x) * kPStride;
    // lane o owns row o of W1 and W2 (and of W3 for o < 32), plus the biases
    const int o = t;
    {
        float acc[kIn];
        for (int k = 0; k < kIn; ++k) acc[k] = 0.0f;
        float bacc = 0.0f;
        for (int rr = 0; rr < kRaysPerBlock; ++rr) {
            const float g = sD1[rr * kH + o];
            bacc += g;
            for (int k = 0; k < kIn; ++k) acc[k] += g * sE[rr * kIn + k];
        }
        for (int k = 0; k < kIn; ++k) out[kOffW1 + o * kIn + k] = acc[k];
        out[kOffB1 + o] = bacc;
    }
    {
        float acc[kH];
        for (int k = 0; k < kH; ++k) acc[k] = 0.0f;
        float bacc = 0.0f;
        for (int rr = 0; rr < kRaysPerBlock; ++rr) {
            const float g = sD2[rr * kH + o];
            bacc += g;
            for (int k = 0; k < kH; ++k) acc[k] += g * sH1[rr * kH + k];
        }
        for (int k = 0; k < kH; ++k) out[kOffW2 + o * kH + k] = acc[k];
        out[kOffB2 + o] = bacc;
    }
    if (o < kS) {
        float acc[kH];
        for (int k = 0; k < kH; ++k) acc[k] = 0.0f;
        float bacc = 0.0f;
        for (int rr = 0; rr < kRaysPerBlock; ++rr) {
            const float g = sDz[rr * kS + o];
            bacc += g;
            for (int k = 0; k < kH; ++k) acc[k] += g * sH2[rr * kH + k];
        }
        for (int k = 0; k < kH; ++k) out[kOffW3 + o * kH + k] = acc[k];
        out[kOffB3 + o] = bacc;
    }
    if (t == 0) loss_part[blockIdx.x] = kl;
}

__global__ void proposal_reduce_kernel(const float* __restrict__ partial, const float* __restrict__ loss_part,
                                       int nblk, float* __restrict__ grad, float* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kParams) {
        float s = 0.0f;
        for (int b = 0; b < nblk; ++b) s += partial[static_cast<int64_t>(b) * kPStride + p];
        grad[p] += s;
    }
    if (p == 0 && loss) {
        float s = 0.0f;
        for (int b = 0; b < nblk; ++b) s += loss_part[b];
        *loss = s;
    }
}

bool fill_args(PropArgs& a, const float* rays_o, const float* rays_d, const float* t_near, const uint8_t* valid,
               int32_t B, const dvgo_box* box, const dvgo_prop* prop) {
    if (B < 0 || !box) return false;
    for (int i = 0; i < 3; ++i)
        if (!(box->xyz_max[i] > box->xyz_min[i])) return false;
    if (B > 0 && (!rays_o || !rays_d || !t_near)) return false;
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.t_near = t_near;
    a.valid = valid;
    a.B = B;
    for (int i = 0; i < 3; ++i) {
        a.mn[i] = box->xyz_min[i];
        a.mx[i] = box->xyz_max[i];
    }
    if (prop) {
        if (!prop->w1 || !prop->b1 || !prop->w2 || !prop->b2 || !prop->w3 || !prop->b3) return false;
        a.w[0] = prop->w1; a.w[1] = prop->w2; a.w[2] = prop->w3;
        a.b[0] = prop->b1; a.b[1] = prop->b2; a.b[2] = prop->b3;
    } else {
        for (int i = 0; i < 3; ++i) a.w[i] = a.b[i] = nullptr;
    }
    return true;
}

}  // namespace

extern "C" {

int64_t dvgo_prop_param_count(void) { return kParams; }

size_t dvgo_proposal_workspace_bytes(int32_t B) {
    if (B < 0) return 0;
    const size_t nblk = (static_cast<size_t>(B) + kRaysPerBlock - 1) / kRaysPerBlock;
    return dvgo::align_up(nblk * kPStride * 4, 256) + dvgo::align_up(nblk * 4, 256);
}

// prop == NULL: `logits` is an input and only the selection runs.
int32_t dvgo_proposal_fwd(const float* rays_o, const float* rays_d, const float* t_near, const uint8_t* valid,
                          int32_t B, const dvgo_box* box, const dvgo_prop* prop, float cum_frac, float min_mass,
                          float* logits, float* pred_mass, uint32_t* seg_mask, void* stream) {
    PropArgs a;
    if (!fill_args(a, rays_o, rays_d, t_near, valid, B, box, prop)) return DVGO_E_ARG;
    if (B > 0 && !logits) return DVGO_E_ARG;
    if (!(cum_frac > 0.0f && cum_frac <= 1.0f) || !(min_mass >= 0.0f && min_mass <= 1.0f)) return DVGO_E_ARG;
    if (B == 0) return DVGO_OK;
    DVGO_LAUNCH(K_PROP_FWD, proposal_fwd_kernel, dim3((B + kRaysPerBlock - 1) / kRaysPerBlock), dim3(kRaysPerBlock), 0,
                       dvgo::as_stream(stream), a, prop != nullptr, cum_frac, min_mass, logits, pred_mass, seg_mask);
    return dvgo::launch_status();
}

int32_t dvgo_proposal_bwd(const float* rays_o, const float* rays_d, const float* t_near, const uint8_t* valid,
                          int32_t B, const dvgo_box* box, const dvgo_prop* prop, const float* seg_w,
                          const float* log_t_end, float* grad_prop, float* loss, void* workspace,
                          size_t workspace_bytes, void* stream) {
    PropArgs a;
    if (!prop || !fill_args(a, rays_o, rays_d, t_near, valid, B, box, prop)) return DVGO_E_ARG;
    if (B > 0 && (!seg_w || !log_t_end || !grad_prop)) return DVGO_E_ARG;
    if (workspace_bytes < dvgo_proposal_workspace_bytes(B) || (B > 0 && !workspace)) return DVGO_E_CAPACITY;
    if (B == 0) return DVGO_OK;
    const int nblk = (B + kRaysPerBlock - 1) / kRaysPerBlock;
    float* partial = static_cast<float*>(workspace);
    float* loss_part = reinterpret_cast<float*>(static_cast<char*>(workspace) +
                                                dvgo::align_up(static_cast<size_t>(nblk) * kPStride * 4, 256));
    hipStream_t s = dvgo::as_stream(stream);
    DVGO_LAUNCH(K_PROP_BWD, proposal_bwd_kernel, dim3(nblk), dim3(kRaysPerBlock), 0, s, a, seg_w, log_t_end, partial,
                       loss_part);
    if (int32_t st = dvgo::launch_status()) return st;
    DVGO_LAUNCH(K_PROP_REDUCE, proposal_reduce_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, partial, loss_part,
                       nblk, grad_prop, loss);
    return dvgo::launch_status();
}

}  // extern "C"
