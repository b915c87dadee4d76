// Learned proposal (not in the paper): a small network that predicts, per
// ray, how the compositing weight is spread over 32 equal-count segments of
// its uniform samples, and the segment mask that keeps the segments holding
// most of it.  The network runs on bfloat16 matrix cores (inputs, hidden
// activations and weights rounded to bfloat16, float32 accumulation), one
// wavefront per 32 rays; the selection follows an explicit float32 recipe so
// that it is reproducible bit for bit from the float32 logits.
#include "adam.hpp"
#include "common.hpp"

namespace {

constexpr int kIn = 54, kH = 64, kS = 32;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kS * kH, kParams = kOffB3 + kS;
constexpr int kPStride = (kParams + 63) / 64 * 64;

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

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x16 mma(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// Row within a 32-row accumulator tile of register r in lane half h.
__device__ __forceinline__ int acc_row(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }
// Feature consumed at chained step st, element i, by lane half h.
__device__ __forceinline__ int phi16(int st, int i, int h) { return 32 * (st >> 1) + acc_row(8 * (st & 1) + i, h); }

__device__ __forceinline__ f32x16 zero16() {
    f32x16 z;
    #pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = 0.0f;
    return z;
}

__device__ __forceinline__ bf16x8 pack8(const f32x16& v, int g) {
    bf16x8 r;
    #pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = static_cast<__bf16>(v[8 * g + e]);
    return r;
}

// Matrix-core operand fragments, built per lane straight from the float32
// weights (row-major [out][in]) with vector loads and rounded to bfloat16:
//   w1(mt, st):  W1[32mt+m][16st+8h+i]   (k >= 54 zero)
//   w2(mt, st):  W2[32mt+m][phi16(st,i,h)]
//   w3(st):      W3[m][phi16(st,i,h)]
//   w2t(mt, st): W2[phi16(st,i,h)][32mt+m]
//   w3t(mt, st): W3[phi16(st,i,h)][32mt+m]
// phi16(st, i, h) for i = 0..3 and 4..7 is two runs of 4 consecutive inputs.
__device__ __forceinline__ bf16x8 frag_w1(const float* w1, int mt, int st, int m, int h) {
    const float* row = w1 + (32 * mt + m) * kIn;
    const int k0 = 16 * st + 8 * h;
    bf16x8 r;
    #pragma unroll
    for (int j = 0; j < 4; ++j) {
        float2 v = make_float2(0.0f, 0.0f);
        if (k0 + 2 * j < kIn) v = *reinterpret_cast<const float2*>(row + k0 + 2 * j);   // kIn is even
        r[2 * j] = static_cast<__bf16>(v.x);
        r[2 * j + 1] = static_cast<__bf16>(v.y);
    }
    return r;
}

__device__ __forceinline__ bf16x8 frag_rows(const float* row0) {
    const float4 a = *reinterpret_cast<const float4*>(row0);
    const float4 b = *reinterpret_cast<const float4*>(row0 + 8);
    bf16x8 r;
    r[0] = static_cast<__bf16>(a.x); r[1] = static_cast<__bf16>(a.y);
    r[2] = static_cast<__bf16>(a.z); r[3] = static_cast<__bf16>(a.w);
    r[4] = static_cast<__bf16>(b.x); r[5] = static_cast<__bf16>(b.y);
    r[6] = static_cast<__bf16>(b.z); r[7] = static_cast<__bf16>(b.w);
    return r;
}

__device__ __forceinline__ int phi16_base(int st, int h) { return 32 * (st >> 1) + 16 * (st & 1) + 4 * h; }

__device__ __forceinline__ bf16x8 frag_w2(const float* w2, int mt, int st, int m, int h) {
    return frag_rows(w2 + (32 * mt + m) * kH + phi16_base(st, h));
}

__device__ __forceinline__ bf16x8 frag_w3(const float* w3, int st, int m, int h) {
    return frag_rows(w3 + m * kH + phi16_base(st, h));
}

__device__ __forceinline__ bf16x8 frag_cols(const float* w, int st, int col, int h) {
    bf16x8 r;
    #pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = static_cast<__bf16>(w[phi16(st, i, h) * kH + col]);
    return r;
}

// Encoding: PE4 of the box-entry point in box coordinates, then PE4 of d.
// The arguments are small (|x| <= 8 for in-box points and unit directions)
// and every value is rounded to bfloat16 before the first layer, so the
// hardware sine and cosine (absolute error below 1e-6 here) replace the
// full-range library sincos and its range reduction.
__device__ void encode(const PropArgs& a, int r, float tn, float e[kIn]) {
    float d[3], u[3];
    for (int i = 0; i < 3; ++i) {
        d[i] = a.rays_d[3 * r + i];
        const float x0 = a.rays_o[3 * r + i] + tn * d[i];
        u[i] = (x0 - 0.5f * (a.mn[i] + a.mx[i])) / (0.5f * (a.mx[i] - a.mn[i]));
    }
    #pragma unroll
    for (int part = 0; part < 2; ++part) {
        const float* src = part == 0 ? u : d;
        float* out = e + 27 * part;
        #pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = src[c];
        #pragma unroll
        for (int fq = 0; fq < 4; ++fq)
            #pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float x = src[c] * static_cast<float>(1 << fq);
                out[3 + 6 * fq + c] = __sinf(x);
                out[6 + 6 * fq + c] = __cosf(x);
            }
    }
}

struct PropFwd {
    bf16x8 enc[4];   // layer-1 B operand
    f32x16 h1[2], h2[2], z;
};

// Box entry t_near of ray r and whether the ray meets the box: the caller's
// clip, or (no t_near given) the sampler's slab clip of the same box, which
// gives the same bits (t_near 0 for a ray that misses, as the sampler
// stores it).
__device__ __forceinline__ bool ray_entry(const PropArgs& a, int r, float* tn) {
    if (a.t_near) {
        *tn = a.t_near[r];
        return !a.valid || a.valid[r];
    }
    float o[3], d[3], tx;
    for (int i = 0; i < 3; ++i) {
        o[i] = a.rays_o[3 * r + i];
        d[i] = a.rays_d[3 * r + i];
    }
    const bool v = dvgo_dev::recipe_slab(o, d, a.mn, a.mx, tn, &tx);
    if (!v) *tn = 0.0f;
    return v;
}

// Forward of the 32 rays of a wave (ray = lane % 32); tn: the ray's t_near.
__device__ void prop_forward(const PropArgs& a, int r, bool ray_ok, float tn, int lane, PropFwd& f) {
    const int h = lane >> 5, m = lane & 31;
    float e[kIn];
    if (ray_ok) encode(a, r, tn, e);
    #pragma unroll
    for (int st = 0; st < 4; ++st)
        #pragma unroll
        for (int i = 0; i < 8; ++i) {
            // both candidate indices are compile-time constants: no private-array indexing
            const int k0 = 16 * st + i, k1 = k0 + 8;
            const float v0 = k0 < kIn ? e[k0 < kIn ? k0 : 0] : 0.0f;
            const float v1 = k1 < kIn ? e[k1 < kIn ? k1 : 0] : 0.0f;
            f.enc[st][i] = static_cast<__bf16>(ray_ok ? (h ? v1 : v0) : 0.0f);
        }
    #pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc;
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) acc[rr] = a.b[0][32 * mt + acc_row(rr, h)];
        #pragma unroll
        for (int st = 0; st < 4; ++st) acc = mma(frag_w1(a.w[0], mt, st, m, h), f.enc[st], acc);
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) f.h1[mt][rr] = fmaxf(acc[rr], 0.0f);
    }
    bf16x8 hb[4];
    #pragma unroll
    for (int st = 0; st < 4; ++st) hb[st] = pack8(f.h1[st >> 1], st & 1);
    #pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc;
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) acc[rr] = a.b[1][32 * mt + acc_row(rr, h)];
        #pragma unroll
        for (int st = 0; st < 4; ++st) acc = mma(frag_w2(a.w[1], mt, st, m, h), hb[st], acc);
        f.h2[mt] = acc;   // pre-activation kept for the ReLU mask
    }
    #pragma unroll
    for (int st = 0; st < 4; ++st) {
        bf16x8 v;
        #pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = static_cast<__bf16>(fmaxf(f.h2[st >> 1][8 * (st & 1) + i], 0.0f));
        hb[st] = v;
    }
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) f.z[rr] = a.b[2][acc_row(rr, h)];
    #pragma unroll
    for (int st = 0; st < 4; ++st) f.z = mma(frag_w3(a.w[2], st, m, h), hb[st], f.z);
}

// exp(x) for x <= 0 in an explicit float32 recipe (every operation rounded,
// no contraction), so that the selection below is reproducible bit for bit:
// Cody-Waite reduction x = k ln2 + r with ln 2 in two parts (k * ln2_hi is
// exact for |k| < 2^9), the degree-7 Taylor polynomial of e^r by Horner's
// rule, then the scale 2^k.  x < -87 gives 0 (the result would leave the
// normal range).  At most 1.15 units in the last place from exp.
__device__ __forceinline__ float exp_recipe(float x) {
#pragma clang fp contract(off)
    const float kLog2e = 0x1.715476p+0f, kLn2Hi = 0x1.62e4p-1f, kLn2Lo = 0x1.7f7d1cp-20f;
    const float k = rintf(x * kLog2e);
    float r = x - k * kLn2Hi;
    r = r - k * kLn2Lo;
    float p = 0x1.a01a02p-13f;       // 1/7!
    p = p * r + 0x1.6c16c2p-10f;     // 1/6!
    p = p * r + 0x1.111112p-7f;      // 1/5!
    p = p * r + 0x1.555556p-5f;      // 1/4!
    p = p * r + 0x1.555556p-3f;      // 1/3!
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    return x < -87.0f ? 0.0f : ldexpf(p, static_cast<int>(k));
}

// Segment mask of one ray from its float32 logits, computed by the ray's two
// lanes (m, h = 0/1): each holds 16 logits, z[rr] of segment acc_row(rr, h).
// float32 recipe, no contraction: m = max(0, z), e = exp_recipe(z - m); the
// total (transmitted entry last), the probabilities e/tot and the mass are
// summed one term at a time in index order over both halves, so both lanes
// hold the identical sums; the selection takes the largest unchosen q each
// round (ties to the lower index), comparing the two halves' candidates, and
// adds it to the running sum until that reaches cum_frac * mass.
__device__ __forceinline__ int seg_rr(int s) { return 4 * (s >> 3) + (s & 3); }   // inverse of acc_row
__device__ __forceinline__ int seg_h(int s) { return (s >> 2) & 1; }

__device__ uint32_t select_mask_pair(const float z[16], int h, float cum_frac, float min_mass, float* pred_mass) {
#pragma clang fp contract(off)
    float mx = 0.0f;
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) mx = fmaxf(mx, z[rr]);
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    float e[16], pe[16];
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) e[rr] = exp_recipe(z[rr] - mx);
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) pe[rr] = __shfl_xor(e[rr], 32, 64);
    float tot = 0.0f;
    #pragma unroll
    for (int s = 0; s < kS; ++s) tot += seg_h(s) == h ? e[seg_rr(s)] : pe[seg_rr(s)];
    tot += exp_recipe(0.0f - mx);
    float q[16], pq[16];
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) q[rr] = e[rr] / tot;
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) pq[rr] = __shfl_xor(q[rr], 32, 64);
    float mass = 0.0f;
    #pragma unroll
    for (int s = 0; s < kS; ++s) mass += seg_h(s) == h ? q[seg_rr(s)] : pq[seg_rr(s)];
    *pred_mass = mass;
    if (!(mass >= min_mass)) return 0xFFFFFFFFu;
    const float target = cum_frac * mass;
    uint32_t own = 0, mask = 0;   // own: chosen bits over rr
    float acc = 0.0f;
    for (int it = 0; it < kS; ++it) {
        float bq = -1.0f;
        int bs = 64, brr = -1;
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr)
            if (!((own >> rr) & 1u) && q[rr] > bq) {
                bq = q[rr];
                bs = acc_row(rr, h);
                brr = rr;
            }
        const float oq = __shfl_xor(bq, 32, 64);
        const int os = __shfl_xor(bs, 32, 64);
        const bool theirs = oq > bq || (oq == bq && os < bs);
        const float wq = theirs ? oq : bq;
        const int ws = theirs ? os : bs;
        if (!theirs && brr >= 0) own |= 1u << brr;
        if (ws < kS) mask |= 1u << ws;
        acc += wq;
        if (acc >= target) break;
    }
    return mask;
}

constexpr int kRaysPerWave = 32;
constexpr int kWaves = 1;   // one wavefront (32 rays) per workgroup

__global__ __launch_bounds__(64) void proposal_fwd_kernel(PropArgs a, int run_net, float cum_frac, float min_mass,
                                                          float* __restrict__ logits, float* __restrict__ pred_mass,
                                                          uint32_t* __restrict__ seg_mask) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, h = lane >> 5;
    const int r = (blockIdx.x * kWaves + wave) * kRaysPerWave + m;
    const bool ray_ok = r < a.B;
    float tn = 0.0f;
    const bool meets = ray_ok && ray_entry(a, r, &tn);
    float z[16];
    if (run_net) {
        PropFwd f;
        prop_forward(a, r, ray_ok, tn, lane, f);
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            z[rr] = f.z[rr];
            if (ray_ok) logits[static_cast<int64_t>(r) * kS + acc_row(rr, h)] = f.z[rr];
        }
    } else {
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) z[rr] = ray_ok ? logits[static_cast<int64_t>(r) * kS + acc_row(rr, h)] : 0.0f;
    }
    float pm;
    uint32_t mask = select_mask_pair(z, h, cum_frac, min_mass, &pm);
    if (ray_ok && h == 0) {
        if (!meets) mask = 0xFFFFFFFFu;
        if (pred_mass) pred_mass[r] = pm;
        if (seg_mask) seg_mask[r] = mask;
    }
}

// Backward: per wave 32 rays; the KL gradient (q - p)/B, the adjoint chain
// on matrix cores, and the weight gradients with the ray index as the
// contraction dimension through [feature][ray] bfloat16 LDS staging.  Each
// wave writes its own partial of the flat gradient.
constexpr int kRP = 40;   // LDS pitch (bf16) of a staged feature row of 32 rays

__global__ __launch_bounds__(64) void proposal_bwd_kernel(PropArgs a, const float* __restrict__ seg_w,
                                                          const float* __restrict__ log_t_end,
                                                          float* __restrict__ partial,
                                                          float* __restrict__ loss_part) {
    __shared__ __attribute__((aligned(16))) __bf16 sT[kWaves][(64 * 5 + 32) * kRP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 31, h = lane >> 5;
    const int wglob = blockIdx.x * kWaves + wave;
    const int r = wglob * kRaysPerWave + m;
    const bool in_batch = r < a.B;
    float tn = 0.0f;
    const bool ok = in_batch && ray_entry(a, r, &tn);
    PropFwd f;
    prop_forward(a, r, in_batch, tn, lane, f);
    // softmax over the 32 logits and the implicit 0, split over the two halves
    float mx = 0.0f;
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) mx = fmaxf(mx, f.z[rr]);
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    float tot = 0.0f;
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) tot += expf(f.z[rr] - mx);
    tot += __shfl_xor(tot, 32, 64);
    tot += expf(-mx);
    const float logtot = logf(tot) + mx;
    const float invB = 1.0f / static_cast<float>(a.B);
    f32x16 dz;
    float kl = 0.0f;
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        const int sg = acc_row(rr, h);
        const float lq = f.z[rr] - logtot;
        const float p = ok ? seg_w[static_cast<int64_t>(r) * kS + sg] : 0.0f;
        dz[rr] = ok ? (expf(lq) - p) * invB : 0.0f;
        if (ok && p > 0.0f) kl += p * (logf(p) - lq);
    }
    if (ok && h == 0) {
        const float lt = log_t_end[r];
        const float pt = expf(lt);
        if (pt > 0.0f) kl += pt * (lt + logtot);
    }
    kl *= invB;
    // adjoint chain: d2 = (W3^T dz) * relu'(z2), d1 = (W2^T d2) * relu'(z1)
    bf16x8 zb[2] = {pack8(dz, 0), pack8(dz, 1)};
    f32x16 d2[2], d1[2];
    #pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = zero16();
        #pragma unroll
        for (int st = 0; st < 2; ++st) acc = mma(frag_cols(a.w[2], st, 32 * mt + m, h), zb[st], acc);
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) d2[mt][rr] = f.h2[mt][rr] > 0.0f ? acc[rr] : 0.0f;
    }
    bf16x8 db[4];
    #pragma unroll
    for (int st = 0; st < 4; ++st) db[st] = pack8(d2[st >> 1], st & 1);
    #pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = zero16();
        #pragma unroll
        for (int st = 0; st < 4; ++st) acc = mma(frag_cols(a.w[1], st, 32 * mt + m, h), db[st], acc);
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) d1[mt][rr] = f.h1[mt][rr] > 0.0f ? acc[rr] : 0.0f;
    }
    // stage [feature][ray] rows: enc 0..63, h1 64..127, h2 128..191, d1 192..255,
    // d2 256..319, dz 320..351 (bf16)
    __bf16* T = sT[wave];
    #pragma unroll
    for (int st = 0; st < 4; ++st)
        #pragma unroll
        for (int i = 0; i < 8; ++i) T[(16 * st + 8 * h + i) * kRP + m] = f.enc[st][i];
    #pragma unroll
    for (int mt = 0; mt < 2; ++mt)
        #pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int j = 32 * mt + acc_row(rr, h);
            T[(64 + j) * kRP + m] = static_cast<__bf16>(f.h1[mt][rr]);
            T[(128 + j) * kRP + m] = static_cast<__bf16>(fmaxf(f.h2[mt][rr], 0.0f));
            T[(192 + j) * kRP + m] = static_cast<__bf16>(d1[mt][rr]);
            T[(256 + j) * kRP + m] = static_cast<__bf16>(d2[mt][rr]);
        }
    #pragma unroll
    for (int rr = 0; rr < 16; ++rr) T[(320 + acc_row(rr, h)) * kRP + m] = static_cast<__bf16>(dz[rr]);
    for (int off = 32; off > 0; off >>= 1) kl += __shfl_xor(kl, off, 64);
    __syncthreads();
    float* out = partial + static_cast<int64_t>(wglob) * kPStride;
    bf16x8 ones;
    #pragma unroll
    for (int e = 0; e < 8; ++e) ones[e] = static_cast<__bf16>(m == 0 ? 1.0f : 0.0f);
    auto rowv = [&](int row, int st) { return *reinterpret_cast<const bf16x8*>(T + row * kRP + 16 * st + 8 * h); };
    // (gradient rows, activation rows, weight offset, bias offset, out rows, in cols)
    #pragma unroll
    for (int layer = 0; layer < 3; ++layer) {
        const int grow = layer == 0 ? 192 : (layer == 1 ? 256 : 320);
        const int arow = layer == 0 ? 0 : (layer == 1 ? 64 : 128);
        const int woff = layer == 0 ? kOffW1 : (layer == 1 ? kOffW2 : kOffW3);
        const int boff = layer == 0 ? kOffB1 : (layer == 1 ? kOffB2 : kOffB3);
        const int nout = layer == 2 ? kS : kH;
        const int nin = layer == 0 ? kIn : kH;
        for (int mt = 0; mt < nout / 32; ++mt) {
            f32x16 acc0 = zero16(), acc1 = zero16(), accb = zero16();
            #pragma unroll
            for (int st = 0; st < 2; ++st) {
                const bf16x8 av = rowv(grow + 32 * mt + m, st);
                acc0 = mma(av, rowv(arow + m, st), acc0);
                acc1 = mma(av, rowv(arow + 32 + m, st), acc1);
                accb = mma(av, ones, accb);
            }
            #pragma unroll
            for (int rr = 0; rr < 16; ++rr) {
                const int o = 32 * mt + acc_row(rr, h);
                if (m < nin) out[woff + o * nin + m] = acc0[rr];
                if (32 + m < nin) out[woff + o * nin + 32 + m] = acc1[rr];
                if (m == 0) out[boff + o] = accb[rr];
            }
        }
    }
    if (lane == 0) loss_part[wglob] = kl;
}

// Optional Adam step taken on each parameter right after its gradient is
// summed (param NULL: none).
struct PropAdam {
    float* param;
    float* m;
    float* v;
    dvgo::AdamCoef c;
};

// 64 parameters per workgroup, 16 wavefronts each summing every 16th
// partial row, then a fixed-order sum of the 16 (deterministic); the
// first workgroup also sums the loss partials.  With an Adam step the
// accumulated gradient is consumed at once: the parameter and its moments
// are updated and the gradient is cleared, the same bits as the streaming
// Adam kernel on the stored gradient.
__global__ __launch_bounds__(1024) void proposal_reduce_kernel(const float* __restrict__ partial,
                                                               const float* __restrict__ loss_part, int nwaves,
                                                               float* __restrict__ grad, float* __restrict__ loss,
                                                               PropAdam opt) {
    __shared__ float sh[16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    // (rows are summed in order, eight rows' loads in flight at a time; a
    // runtime-bounded one-row loop waits on each load)
    float s = 0.0f;
    if (p < kParams)
        for (int b0 = wave; b0 < nwaves; b0 += 16 * 8) {
            float v[8];
            #pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = b0 + 16 * u;
                v[u] = b < nwaves ? partial[static_cast<int64_t>(b) * kPStride + p] : 0.0f;
            }
            #pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
    sh[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && p < kParams) {
        float t = 0.0f;
        for (int w = 0; w < 16; ++w) t += sh[w][lane];
        const float g = grad[p] + t;
        if (opt.param) {
            float q = opt.param[p], m = opt.m[p], v = opt.v[p];
            dvgo::adam_update(opt.c, q, g, m, v);
            opt.param[p] = q;
            opt.m[p] = m;
            opt.v[p] = v;
            grad[p] = 0.0f;
        } else {
            grad[p] = g;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
        float l = 0.0f;
        for (int b0 = 0; b0 < nwaves; b0 += 8) {
            float v[8];
            #pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = b0 + u < nwaves ? loss_part[b0 + u] : 0.0f;
            #pragma unroll
            for (int u = 0; u < 8; ++u) l += v[u];
        }
        *loss = l;
    }
}

// t_near NULL (then valid NULL too): the kernels clip each ray themselves.
bool fill_args(PropArgs& a, const float* rays_o, const float* rays_d, const float* t_near, const uint8_t* valid,
               int32_t B, const dvgo_box* box, const dvgo_prop* prop) {
    if (B < 0 || !box) return false;
    for (int i = 0; i < 3; ++i)
        if (!(box->xyz_max[i] > box->xyz_min[i])) return false;
    if (B > 0 && (!rays_o || !rays_d)) return false;
    if (!t_near && valid) return false;
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
        // vector loads of the weight rows: W1 8-byte, W2 and W3 16-byte aligned
        if ((reinterpret_cast<uintptr_t>(prop->w1) & 7u) || (reinterpret_cast<uintptr_t>(prop->w2) & 15u) ||
            (reinterpret_cast<uintptr_t>(prop->w3) & 15u))
            return false;
        a.w[0] = prop->w1; a.w[1] = prop->w2; a.w[2] = prop->w3;
        a.b[0] = prop->b1; a.b[1] = prop->b2; a.b[2] = prop->b3;
    } else {
        for (int i = 0; i < 3; ++i) a.w[i] = a.b[i] = nullptr;
    }
    return true;
}

// The backward launch and the reduction; opt non-NULL adds the Adam step to
// the reduction.  B == 0 with an Adam step still takes the step (on the
// gradient as it stands), as the separate Adam call would.
int32_t proposal_bwd_impl(const float* rays_o, const float* rays_d, const float* t_near, const uint8_t* valid,
                          int32_t B, const dvgo_box* box, const dvgo_prop* prop, const float* seg_w,
                          const float* log_t_end, float* grad_prop, float* loss, const dvgo_adam_state* opt,
                          void* workspace, size_t workspace_bytes, void* stream) {
    PropArgs a;
    if (!prop || !fill_args(a, rays_o, rays_d, t_near, valid, B, box, prop)) return DVGO_E_ARG;
    if (B > 0 && (!seg_w || !log_t_end || !grad_prop)) return DVGO_E_ARG;
    if (opt && !grad_prop) return DVGO_E_ARG;
    PropAdam pa{};
    if (opt) {
        if (!opt->param || !opt->m || !opt->v) return DVGO_E_ARG;
        if (!dvgo::adam_hyper_ok(opt->beta1, opt->beta2, opt->eps, opt->t)) return DVGO_E_ARG;
        pa.param = opt->param;
        pa.m = opt->m;
        pa.v = opt->v;
        pa.c = dvgo::adam_coef(opt->lr, opt->beta1, opt->beta2, opt->eps, opt->t);
    }
    if (workspace_bytes < dvgo_proposal_workspace_bytes(B) || (B > 0 && !workspace)) return DVGO_E_CAPACITY;
    if (B == 0 && !opt) return DVGO_OK;
    const int nblk = (B + kRaysPerWave * kWaves - 1) / (kRaysPerWave * kWaves);
    const int nw = nblk * kWaves;
    float* partial = static_cast<float*>(workspace);
    float* loss_part = B > 0 ? reinterpret_cast<float*>(static_cast<char*>(workspace) +
                                                         dvgo::align_up(static_cast<size_t>(nw) * kPStride * 4, 256))
                             : nullptr;
    hipStream_t s = dvgo::as_stream(stream);
    if (B > 0) {
        DVGO_LAUNCH(K_PROP_BWD, proposal_bwd_kernel, dim3(nblk), dim3(64 * kWaves), 0, s, a, seg_w, log_t_end,
                    partial, loss_part);
        if (int32_t st = dvgo::launch_status()) return st;
    }
    DVGO_LAUNCH(K_PROP_REDUCE, proposal_reduce_kernel, dim3((kParams + 63) / 64), dim3(1024), 0, s, partial, loss_part,
                nw, grad_prop, B > 0 ? loss : nullptr, pa);
    return dvgo::launch_status();
}

}  // namespace

extern "C" {

int64_t dvgo_prop_param_count(void) { return kParams; }

size_t dvgo_proposal_workspace_bytes(int32_t B) {
    if (B < 0) return 0;
    const size_t nw = (static_cast<size_t>(B) + kRaysPerWave * kWaves - 1) / (kRaysPerWave * kWaves) * kWaves;
    return dvgo::align_up(nw * kPStride * 4, 256) + dvgo::align_up(nw * 4, 256);
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
    DVGO_LAUNCH(K_PROP_FWD, proposal_fwd_kernel, dim3((B + kRaysPerWave - 1) / kRaysPerWave), dim3(64 * kWaves), 0,
                       dvgo::as_stream(stream), a, prop != nullptr, cum_frac, min_mass, logits, pred_mass, seg_mask);
    return dvgo::launch_status();
}

int32_t dvgo_proposal_bwd(const float* rays_o, const float* rays_d, const float* t_near, const uint8_t* valid,
                          int32_t B, const dvgo_box* box, const dvgo_prop* prop, const float* seg_w,
                          const float* log_t_end, float* grad_prop, float* loss, void* workspace,
                          size_t workspace_bytes, void* stream) {
    return proposal_bwd_impl(rays_o, rays_d, t_near, valid, B, box, prop, seg_w, log_t_end, grad_prop, loss, nullptr,
                             workspace, workspace_bytes, stream);
}

int32_t dvgo_proposal_bwd_adam(const float* rays_o, const float* rays_d, const float* t_near, const uint8_t* valid,
                               int32_t B, const dvgo_box* box, const dvgo_prop* prop, const float* seg_w,
                               const float* log_t_end, float* grad_prop, const dvgo_adam_state* opt, float* loss,
                               void* workspace, size_t workspace_bytes, void* stream) {
    if (!opt) return DVGO_E_ARG;
    return proposal_bwd_impl(rays_o, rays_d, t_near, valid, B, box, prop, seg_w, log_t_end, grad_prop, loss, opt,
                             workspace, workspace_bytes, stream);
}

}  // extern "C"
