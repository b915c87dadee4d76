// Fine-stage ray sampler: ray-box clip, uniform sample counts, coarse
// alpha-mask skipping and the fine-density alpha skip, optional Morton ray
// order, compaction into a per-ray sample list (paper Sec. 4.2 "Fine-stage
// points sampling" and "Free space skipping", Eq. coarse_sample, training
// jitter of the supplementary implementation details).
#include <mutex>

#include "common.hpp"

using dvgo::GridArgs;
using namespace dvgo_dev;

namespace {

constexpr int kMortonBits = 5;
constexpr uint32_t kMortonInvalid = 1u << (3 * kMortonBits);
constexpr int kMaxMortonRays = 32768;     // 15-bit ray id packed beside the key
constexpr int kScanThreads = 1024;

struct BoxF {
    float mn[3];
    float mx[3];
    float mscale[3];   // 32/(max-min), float32
};

// One thread per ray: clip, uniform count, Morton key or identity order.
// Slab clip and uniform count of one ray (float32 recipe, no contraction).
struct Clip {
    float tn, tx;
    bool v;
    int n;
};

__device__ __forceinline__ Clip clip_ray(const float o[3], const float d[3], float p, const BoxF& box, float step,
                                         int max_samples) {
#pragma clang fp contract(off)
    Clip c;
    c.v = recipe_slab(o, d, box.mn, box.mx, &c.tn, &c.tx);
    const float tx = c.tx;
    c.n = 0;
    if (c.v) {
        // estimate, then settle on the exact prefix length (t_k is monotone in k)
        const float est = (tx - c.tn) / step - p;
        int k = static_cast<int>(fminf(fmaxf(floorf(est) - 2.0f, 0.0f), static_cast<float>(max_samples)));
        while (k > 0 && !(recipe_tk(c.tn, p, k - 1, step) < tx)) --k;
        while (k < max_samples && recipe_tk(c.tn, p, k, step) < tx) ++k;
        c.n = k;
    }
    return c;
}

__global__ void ray_setup_kernel(const float* __restrict__ rays_o, const float* __restrict__ rays_d,
                                 const float* __restrict__ jitter, int B, BoxF box, float step,
                                 int max_samples, int morton, float* __restrict__ t_near,
                                 float* __restrict__ t_far, uint8_t* __restrict__ valid,
                                 int* __restrict__ n_uniform, uint32_t* __restrict__ keys,
                                 int* __restrict__ perm) {
#pragma clang fp contract(off)
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B) return;
    float o[3], d[3];
    for (int i = 0; i < 3; ++i) {
        o[i] = rays_o[3 * r + i];
        d[i] = rays_d[3 * r + i];
    }
    const Clip c = clip_ray(o, d, jitter ? jitter[r] : 0.0f, box, step, max_samples);
    const float tn = c.tn, tx = c.tx;
    const bool v = c.v;
    t_near[r] = v ? tn : 0.0f;
    t_far[r] = v ? tx : 0.0f;
    valid[r] = v ? 1 : 0;
    n_uniform[r] = c.n;
    if (morton) {
        uint32_t key = kMortonInvalid;
        if (v) {
            const float tm = (tn + tx) * 0.5f;
            float m[3];
            recipe_x(o, d, tm, m);
            uint32_t q[3];
            for (int i = 0; i < 3; ++i) {
                float u = (m[i] - box.mn[i]) * box.mscale[i];
                float fl = fminf(fmaxf(floorf(u), 0.0f), static_cast<float>((1 << kMortonBits) - 1));
                q[i] = static_cast<uint32_t>(fl);
            }
            key = 0;
            for (int b = 0; b < kMortonBits; ++b) {
                key |= ((q[0] >> b) & 1u) << (3 * b + 2);
                key |= ((q[1] >> b) & 1u) << (3 * b + 1);
                key |= ((q[2] >> b) & 1u) << (3 * b);
            }
        }
        keys[r] = (key << 15) | static_cast<uint32_t>(r);
    } else {
        perm[r] = r;
    }
}

// Single-workgroup bitonic sort of the packed (key, ray) words in LDS.
__global__ __launch_bounds__(1024) void morton_sort_kernel(const uint32_t* __restrict__ keys, int B,
                                                           int npow2, int* __restrict__ perm) {
    __shared__ uint32_t s[kMaxMortonRays];
    const int tid = threadIdx.x;
    for (int i = tid; i < npow2; i += blockDim.x) s[i] = i < B ? keys[i] : 0xFFFFFFFFu;
    __syncthreads();
    for (int k = 2; k <= npow2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < npow2; i += blockDim.x) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint32_t a = s[i], b = s[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        s[i] = b;
                        s[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < B; i += blockDim.x) perm[i] = static_cast<int>(s[i] & 0x7FFFu);
}

struct KeepArgs {
    const float* rays_o;
    const float* rays_d;
    const float* jitter;
    const float* t_near;
    const int* n_uniform;
    const int* perm;
    const uint32_t* coarse_bits;
    const uint32_t* seg_mask;
    GridArgs cg;
    const float* fine_density;   // second free-space rule (nullptr: off)
    GridArgs fg;
    float fine_thr;
    float step;
    int B;
    // the counting pass's keep ballots, kKeepWords per ray slot, read back by
    // the fill (nullptr: the fill evaluates the keep rule again)
    uint64_t* words;
};

// Ballot words kept per ray slot: rays of up to 64 * kKeepWords uniform
// samples reuse the counting pass's keep decisions in the fill.
constexpr int kKeepWords = 16;

struct RayView {
    float o[3], d[3], tn, p;
    int r, n;
    uint32_t seg;
};

__device__ __forceinline__ RayView load_ray(const KeepArgs& a, int slot) {
    RayView v;
    v.r = a.perm[slot];
    v.n = a.n_uniform[v.r];
    for (int i = 0; i < 3; ++i) {
        v.o[i] = a.rays_o[3 * v.r + i];
        v.d[i] = a.rays_d[3 * v.r + i];
    }
    v.tn = a.t_near[v.r];
    v.p = a.jitter ? a.jitter[v.r] : 0.0f;
    v.seg = a.seg_mask ? a.seg_mask[v.r] : 0xFFFFFFFFu;
    return v;
}

__device__ __forceinline__ bool keep_sample(const KeepArgs& a, const RayView& v, int k) {
    if (k >= v.n) return false;
    if (a.seg_mask) {
        const int seg = static_cast<int>((32LL * k) / v.n);
        if (!((v.seg >> seg) & 1u)) return false;
    }
    if (a.coarse_bits || a.fine_density) {
        float x[3];
        recipe_x(v.o, v.d, recipe_tk(v.tn, v.p, k, a.step), x);
        if (a.coarse_bits) {
            const int c = recipe_cell(a.cg, x);
            if (!((a.coarse_bits[c >> 5] >> (c & 31)) & 1u)) return false;
        }
        // unknown space: skip a point whose fine post-activated alpha is
        // below tau^(f), i.e. whose interpolated raw density is below the
        // equivalent threshold
        if (a.fine_density && !(recipe_trilerp(a.fg, a.fine_density, x) >= a.fine_thr)) return false;
    }
    return true;
}

// Identity order: one wavefront per ray clips it (every lane the same
// float32 recipe; lane 0 writes) and counts its kept samples, in one pass.
// One ray per workgroup, so that a long ray holds only its own slot.
__global__ __launch_bounds__(64) void setup_count_kernel(KeepArgs a, BoxF box, int max_samples,
                                                          float* __restrict__ t_near, float* __restrict__ t_far,
                                                          uint8_t* __restrict__ valid, int* __restrict__ n_uniform,
                                                          int* __restrict__ perm, int* __restrict__ counts) {
    const int r = blockIdx.x;
    const int lane = threadIdx.x & 63;
    if (r >= a.B) return;
    RayView v;
    v.r = r;
    for (int i = 0; i < 3; ++i) {
        v.o[i] = a.rays_o[3 * r + i];
        v.d[i] = a.rays_d[3 * r + i];
    }
    v.p = a.jitter ? a.jitter[r] : 0.0f;
    v.seg = a.seg_mask ? a.seg_mask[r] : 0xFFFFFFFFu;
    const Clip c = clip_ray(v.o, v.d, v.p, box, a.step, max_samples);
    v.tn = c.v ? c.tn : 0.0f;
    v.n = c.n;
    if (lane == 0) {
        t_near[r] = v.tn;
        t_far[r] = c.v ? c.tx : 0.0f;
        valid[r] = c.v ? 1 : 0;
        n_uniform[r] = c.n;
        perm[r] = r;
    }
    int cnt = 0;
    for (int base = 0; base < v.n; base += 64) {
        const uint64_t m = __ballot(keep_sample(a, v, base + lane));
        cnt += __popcll(m);
        if (a.words && lane == 0) a.words[static_cast<int64_t>(r) * kKeepWords + (base >> 6)] = m;
    }
    if (lane == 0) counts[r] = cnt;
}

// One wavefront per ray slot: number of kept samples.
__global__ __launch_bounds__(256) void count_kept_kernel(KeepArgs a, int* __restrict__ counts) {
    const int slot = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (slot >= a.B) return;
    const RayView v = load_ray(a, slot);
    int cnt = 0;
    for (int base = 0; base < v.n; base += 64) {
        const uint64_t m = __ballot(keep_sample(a, v, base + lane));
        cnt += __popcll(m);
        if (a.words && lane == 0) a.words[static_cast<int64_t>(slot) * kKeepWords + (base >> 6)] = m;
    }
    if (lane == 0) counts[slot] = cnt;
}

// Inclusive prefix sum over a wavefront on DPP lane shifts: a Hillis-Steele
// scan inside each row of 16 lanes (row_shr by 1, 2, 4, 8; a lane whose
// source lies outside its row reads 0), then each row adds the totals of the
// rows before it, read from their last lanes.
template <int kCtrl>
__device__ __forceinline__ int dpp_row_shr(int v) {
    return __builtin_amdgcn_update_dpp(0, v, kCtrl, 0xf, 0xf, true);
}
__device__ __forceinline__ int wave_incl_scan_int(int v, int lane) {
    v += dpp_row_shr<0x111>(v);
    v += dpp_row_shr<0x112>(v);
    v += dpp_row_shr<0x114>(v);
    v += dpp_row_shr<0x118>(v);
    const int t0 = __builtin_amdgcn_readlane(v, 15), t1 = __builtin_amdgcn_readlane(v, 31),
              t2 = __builtin_amdgcn_readlane(v, 47);
    const int row = lane >> 4;
    return v + (row == 0 ? 0 : row == 1 ? t0 : row == 2 ? t0 + t1 : t0 + t1 + t2);
}

// Single-workgroup exclusive scan: ray_offset[i] = sum_{j<i} counts[j].  The
// total is below 2^31 (the host bounds B * max_samples), so the scan runs in
// 32-bit integers.  Each thread takes kPer consecutive counts, so one pass
// covers kScanThreads * kPer = 8192 rays.
__global__ __launch_bounds__(kScanThreads) void scan_offsets_kernel(const int* __restrict__ counts, int B,
                                                                   int* __restrict__ ray_offset,
                                                                   int64_t* __restrict__ n_kept) {
    constexpr int kPer = 8;
    __shared__ int wsum[kScanThreads / 64];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const bool vec = (reinterpret_cast<uintptr_t>(counts) & 15u) == 0;
    int carry = 0;   // same value in every thread
    for (int64_t base = 0; base < B; base += kScanThreads * kPer) {
        const int64_t i0 = base + tid * kPer;
        int v[kPer];
        if (vec && i0 + kPer <= B) {
            const int4 a = *reinterpret_cast<const int4*>(counts + i0);
            const int4 b = *reinterpret_cast<const int4*>(counts + i0 + 4);
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
            v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else {
            for (int u = 0; u < kPer; ++u) v[u] = i0 + u < B ? counts[i0 + u] : 0;
        }
        int local = 0;
        for (int u = 0; u < kPer; ++u) local += v[u];
        const int incl = wave_incl_scan_int(local, lane);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int wave_off = 0, total = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) {
            const int t = wsum[w];
            wave_off += w < wave ? t : 0;
            total += t;
        }
        int run = carry + wave_off + incl - local;
        for (int u = 0; u < kPer; ++u) {
            if (i0 + u < B) ray_offset[i0 + u] = run;
            run += v[u];
        }
        carry += total;
        __syncthreads();   // wsum is rewritten by the next pass
    }
    if (tid == 0) {
        ray_offset[B] = carry;
        *n_kept = carry;
    }
}

// Kept (ray, k) pairs of one ray in ascending k from list position pos0
// (one wavefront; pairs past the capacity are dropped).
__device__ __forceinline__ void fill_ray(const KeepArgs& a, const RayView& v, int64_t pos0, int64_t capacity,
                                         int* __restrict__ sample_ray, int* __restrict__ sample_k, int lane) {
    for (int base = 0; base < v.n; base += 64) {
        const int k = base + lane;
        const bool keep = keep_sample(a, v, k);
        const uint64_t mask = __ballot(keep);
        const int64_t pos = pos0 + lanes_below(mask);
        if (keep && pos < capacity) {
            sample_ray[pos] = v.r;
            sample_k[pos] = k;
        }
        pos0 += __popcll(mask);
    }
}

// The same from the counting pass's ballot words of ray slot `slot`: lane w
// loads word w, each 64-sample step takes its word from that lane.
__device__ __forceinline__ void fill_ray_words(const KeepArgs& a, int slot, int64_t pos0, int64_t capacity,
                                               int* __restrict__ sample_ray, int* __restrict__ sample_k,
                                               int lane) {
    const int r = a.perm[slot];
    const int n = a.n_uniform[r];
    const int nw = (n + 63) >> 6;
    const uint64_t own = lane < nw ? a.words[static_cast<int64_t>(slot) * kKeepWords + lane] : 0;
    const uint32_t lo = static_cast<uint32_t>(own), hi = static_cast<uint32_t>(own >> 32);
    for (int w = 0; w < nw; ++w) {
        // (readlane returns a signed int: the halves widen as unsigned)
        const uint32_t wl = __builtin_amdgcn_readlane(lo, w), wh = __builtin_amdgcn_readlane(hi, w);
        const uint64_t mask = (static_cast<uint64_t>(wh) << 32) | wl;
        const bool keep = (mask >> lane) & 1u;
        const int64_t pos = pos0 + lanes_below(mask);
        if (keep && pos < capacity) {
            sample_ray[pos] = r;
            sample_k[pos] = 64 * w + lane;
        }
        pos0 += __popcll(mask);
    }
}

// One wavefront per ray slot: write the kept (ray, k) pairs in ascending k.
__global__ __launch_bounds__(256) void fill_kept_kernel(KeepArgs a, const int* __restrict__ ray_offset,
                                                        int64_t capacity, int* __restrict__ sample_ray,
                                                        int* __restrict__ sample_k) {
    const int slot = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (slot >= a.B) return;
    if (a.words) {
        fill_ray_words(a, slot, ray_offset[slot], capacity, sample_ray, sample_k, lane);
        return;
    }
    const RayView v = load_ray(a, slot);
    fill_ray(a, v, ray_offset[slot], capacity, sample_ray, sample_k, lane);
}

// Ray offsets and the kept pairs in one launch, for batches of at most
// kFusedMaxRays rays.  A workgroup takes kFillRays consecutive ray slots, one
// per wavefront.  It sums the counts of every slot before its first (at most
// kFusedMaxRays / 1024 loads per thread, all issued before the sum), adds the
// counts of the slots before each wavefront's own, writes the slots' offsets
// (the workgroup holding the last slot also writes ray_offset[B] and n_kept)
// and fills.  Integer sums, so every offset equals the scan's.
constexpr int kFillRays = 16;
constexpr int kFusedMaxRays = 16384;

__global__ __launch_bounds__(1024) void offsets_fill_kernel(KeepArgs a, const int* __restrict__ counts,
                                                            int* __restrict__ ray_offset,
                                                            int64_t* __restrict__ n_kept, int64_t capacity,
                                                            int* __restrict__ sample_ray,
                                                            int* __restrict__ sample_k) {
    constexpr int kLoads = kFusedMaxRays / 1024;
    __shared__ int wpart[16];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int first = blockIdx.x * kFillRays;
    const int slot = first + wave;
    // counts of this workgroup's slots (lanes 0..15; clamped, masked below)
    const int own_i = first + (lane & (kFillRays - 1));
    const int own = counts[own_i < a.B ? own_i : a.B - 1];
    // counts of all slots before the workgroup's first
    int c[kLoads];
    #pragma unroll
    for (int u = 0; u < kLoads; ++u) {
        c[u] = 0;
        if (1024 * u < first) {   // workgroup-uniform
            const int i = tid + 1024 * u;
            c[u] = counts[i < first ? i : first - 1];
        }
    }
    int part = 0;
    #pragma unroll
    for (int u = 0; u < kLoads; ++u) part += tid + 1024 * u < first ? c[u] : 0;
    // workgroup sum: row scans, then the rows' totals, then the wavefronts'
    part += __builtin_amdgcn_update_dpp(0, part, 0x111, 0xf, 0xf, true);
    part += __builtin_amdgcn_update_dpp(0, part, 0x112, 0xf, 0xf, true);
    part += __builtin_amdgcn_update_dpp(0, part, 0x114, 0xf, 0xf, true);
    part += __builtin_amdgcn_update_dpp(0, part, 0x118, 0xf, 0xf, true);
    const int wsum = __builtin_amdgcn_readlane(part, 15) + __builtin_amdgcn_readlane(part, 31) +
                     __builtin_amdgcn_readlane(part, 47) + __builtin_amdgcn_readlane(part, 63);
    if (lane == 0) wpart[wave] = wsum;
    __syncthreads();
    int prefix = 0;
    for (int w = 0; w < 16; ++w) prefix += wpart[w];
    if (slot >= a.B) return;
    // slots of this workgroup before this wavefront's: inclusive row scan of
    // the own counts in lanes 0..15
    int oc = lane < kFillRays && first + lane < a.B ? own : 0;
    oc += __builtin_amdgcn_update_dpp(0, oc, 0x111, 0xf, 0xf, true);
    oc += __builtin_amdgcn_update_dpp(0, oc, 0x112, 0xf, 0xf, true);
    oc += __builtin_amdgcn_update_dpp(0, oc, 0x114, 0xf, 0xf, true);
    oc += __builtin_amdgcn_update_dpp(0, oc, 0x118, 0xf, 0xf, true);
    const int before = wave > 0 ? __builtin_amdgcn_readlane(oc, wave - 1) : 0;
    const int pos0 = prefix + before;
    if (lane == 0) {
        ray_offset[slot] = pos0;
        if (slot == a.B - 1) {
            const int total = prefix + __builtin_amdgcn_readlane(oc, wave);
            ray_offset[a.B] = total;
            *n_kept = total;
        }
    }
    if (a.words) {
        fill_ray_words(a, slot, pos0, capacity, sample_ray, sample_k, lane);
        return;
    }
    const RayView v = load_ray(a, slot);
    fill_ray(a, v, pos0, capacity, sample_ray, sample_k, lane);
}

// One thread per 32-cell word of the coarse keep mask.
__global__ void coarse_mask_kernel(const float* __restrict__ raw, int nx, int ny, int nz, float thr,
                                   uint32_t* __restrict__ bits, int64_t ncells) {
    const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nwords = (ncells + 31) / 32;
    if (w >= nwords) return;
    const int cy = ny - 1, cz = nz - 1;
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
        const int64_t c = w * 32 + b;
        if (c >= ncells) break;
        const int iz = static_cast<int>(c % cz);
        const int iy = static_cast<int>((c / cz) % cy);
        const int ix = static_cast<int>(c / (static_cast<int64_t>(cz) * cy));
        float m = -INFINITY;
        for (int dx = 0; dx < 2; ++dx)
            for (int dy = 0; dy < 2; ++dy)
                for (int dz = 0; dz < 2; ++dz)
                    m = fmaxf(m, raw[(static_cast<int64_t>(ix + dx) * ny + (iy + dy)) * nz + (iz + dz)]);
        if (m >= thr) word |= 1u << b;
    }
    bits[w] = word;
}

// Per-ray counts and Morton keys, each rounded up to 256 bytes, plus 256;
// the public workspace adds the keep ballot words.
constexpr size_t base_workspace_bytes(int32_t B) {
    return (static_cast<size_t>(B) * 4 + 255) / 256 * 256 * 2 + 256;
}

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of dvgo_sample_rays_noalloc: the workspace of up to
// kNoAllocMaxRays rays without the keep ballot words (per-ray counts and
// Morton keys; the fill evaluates the keep rule again), held by every GPU
// the library runs on until the
// process ends.  Host code never passes the array's name to a kernel: it is
// a host-side stand-in, not a device address.  Each device's own address of
// its copy comes from hipGetSymbolAddress, taken once per device with that
// device current, and is what the call hands its kernels.
// ---------------------------------------------------------------------------
constexpr int32_t kNoAllocMaxRays = 1 << 18;
constexpr size_t kNoAllocScratchBytes = base_workspace_bytes(kNoAllocMaxRays);

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
void* g_scratch_ptr[kMaxScratchDevices] = {nullptr};
std::mutex g_scratch_mutex;

// This device's address of `scratch` (looked up on its first use).
int32_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        dvgo::record_hip_error(e);
        return DVGO_E_HIP;
    }
    if (dev < 0 || dev >= kMaxScratchDevices) return DVGO_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            dvgo::record_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return DVGO_E_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DVGO_OK;
}
}  // namespace

extern "C" {

int32_t dvgo_coarse_mask_build(const float* raw, const dvgo_box* cbox, float raw_threshold, uint32_t* bits,
                               void* stream) {
    if (!raw || !bits || !dvgo::box_ok(cbox, 2)) return DVGO_E_ARG;
    const int64_t ncells = static_cast<int64_t>(cbox->n[0] - 1) * (cbox->n[1] - 1) * (cbox->n[2] - 1);
    const int64_t nwords = (ncells + 31) / 32;
    const int threads = 256;
    const unsigned blocks = static_cast<unsigned>((nwords + threads - 1) / threads);
    DVGO_LAUNCH(K_COARSE_MASK, coarse_mask_kernel, dim3(blocks), dim3(threads), 0, dvgo::as_stream(stream), raw,
                       cbox->n[0], cbox->n[1], cbox->n[2], raw_threshold, bits, ncells);
    return dvgo::launch_status();
}

size_t dvgo_sample_workspace_bytes(int32_t B) {
    if (B < 0) return 0;
    return base_workspace_bytes(B) + dvgo::align_up(static_cast<size_t>(B) * kKeepWords * 8, 256);
}

static int32_t sample_rays_impl(const float* rays_o, const float* rays_d, const float* jitter, int32_t B,
                         const dvgo_box* box, float step, int32_t max_samples, const uint32_t* coarse_bits,
                         const dvgo_box* coarse_box, const uint32_t* seg_mask, const dvgo_fine_filter* fine,
                         int32_t morton, float* t_near,
                         float* t_far, uint8_t* valid, int32_t* n_uniform, int32_t* perm, int32_t* ray_offset,
                         int32_t* sample_ray, int32_t* sample_k, int64_t capacity, int64_t* n_kept,
                         void* workspace, size_t workspace_bytes, bool keep_words, void* stream) {
    if (B < 0 || !box) return DVGO_E_ARG;
    if (!(step > 0.0f) || max_samples < 0 || capacity < 0) return DVGO_E_ARG;
    for (int i = 0; i < 3; ++i)
        if (!(box->xyz_max[i] > box->xyz_min[i])) return DVGO_E_ARG;
    if (coarse_bits && !dvgo::box_ok(coarse_box, 2)) return DVGO_E_ARG;
    if (fine && (!fine->density || !dvgo::box_ok(&fine->box, 2))) return DVGO_E_ARG;
    if (fine && static_cast<int64_t>(fine->box.n[0]) * fine->box.n[1] * fine->box.n[2] >= (1LL << 31))
        return DVGO_E_UNSUPPORTED;
    // clip only: no sample list asked for (capacity 0, ray_offset and n_kept NULL)
    const bool clip_only = capacity == 0 && !ray_offset && !n_kept;
    if (!clip_only && (!n_kept || !ray_offset)) return DVGO_E_ARG;
    if (B > 0 && (!rays_o || !rays_d || !t_near || !t_far || !valid || !n_uniform || !perm)) return DVGO_E_ARG;
    if (capacity > 0 && (!sample_ray || !sample_k)) return DVGO_E_ARG;
    if (morton && B > kMaxMortonRays) return DVGO_E_UNSUPPORTED;
    if (static_cast<int64_t>(B) * max_samples >= (1LL << 31)) return DVGO_E_UNSUPPORTED;
    if (workspace_bytes < (keep_words ? dvgo_sample_workspace_bytes(B) : base_workspace_bytes(B)) ||
        (B > 0 && !workspace))
        return DVGO_E_CAPACITY;

    hipStream_t s = dvgo::as_stream(stream);
    if (B == 0) {
        if (clip_only) return DVGO_OK;
        DVGO_LAUNCH(K_SCAN, scan_offsets_kernel, dim3(1), dim3(kScanThreads), 0, s,
                           static_cast<const int*>(nullptr), 0, ray_offset, n_kept);
        return dvgo::launch_status();
    }
    char* ws = static_cast<char*>(workspace);
    int* counts = reinterpret_cast<int*>(ws);
    uint32_t* keys = reinterpret_cast<uint32_t*>(ws + dvgo::align_up(static_cast<size_t>(B) * 4, 256));

    BoxF bf;
    for (int i = 0; i < 3; ++i) {
        bf.mn[i] = box->xyz_min[i];
        bf.mx[i] = box->xyz_max[i];
        volatile float span = box->xyz_max[i] - box->xyz_min[i];
        volatile float q = static_cast<float>(1 << kMortonBits);
        bf.mscale[i] = q / span;
    }
    KeepArgs ka;
    ka.rays_o = rays_o;
    ka.rays_d = rays_d;
    ka.jitter = jitter;
    ka.t_near = t_near;
    ka.n_uniform = n_uniform;
    ka.perm = perm;
    ka.coarse_bits = coarse_bits;
    ka.seg_mask = seg_mask;
    ka.cg = coarse_bits ? dvgo::make_grid(*coarse_box) : GridArgs{};
    ka.fine_density = fine ? fine->density : nullptr;
    ka.fg = fine ? dvgo::make_grid(fine->box) : GridArgs{};
    ka.fine_thr = fine ? fine->raw_threshold : 0.0f;
    ka.step = step;
    ka.B = B;
    ka.words = keep_words && max_samples <= 64 * kKeepWords
                   ? reinterpret_cast<uint64_t*>(ws + base_workspace_bytes(B))
                   : nullptr;
    const unsigned wblocks = static_cast<unsigned>((B + 3) / 4);
    if (!morton && !clip_only) {
        DVGO_LAUNCH(K_RAY_SETUP, setup_count_kernel, dim3(B), dim3(64), 0, s, ka, bf, max_samples, t_near,
                    t_far, valid, n_uniform, perm, counts);
        if (int32_t st = dvgo::launch_status()) return st;
    } else {
        const int t1 = 256;
        DVGO_LAUNCH(K_RAY_SETUP, ray_setup_kernel, dim3((B + t1 - 1) / t1), dim3(t1), 0, s, rays_o, rays_d, jitter, B,
                    bf, step, max_samples, morton, t_near, t_far, valid, n_uniform, keys, perm);
        if (int32_t st = dvgo::launch_status()) return st;
        if (morton) {
            int np2 = 2;
            while (np2 < B) np2 <<= 1;
            DVGO_LAUNCH(K_MORTON_SORT, morton_sort_kernel, dim3(1), dim3(1024), 0, s, keys, B, np2, perm);
            if (int32_t st = dvgo::launch_status()) return st;
        }
        if (clip_only) return DVGO_OK;
        DVGO_LAUNCH(K_COUNT_KEPT, count_kept_kernel, dim3(wblocks), dim3(256), 0, s, ka, counts);
        if (int32_t st = dvgo::launch_status()) return st;
    }
    if (B <= kFusedMaxRays) {
        DVGO_LAUNCH(K_FILL_KEPT, offsets_fill_kernel, dim3((B + kFillRays - 1) / kFillRays), dim3(1024), 0, s, ka,
                    counts, ray_offset, n_kept, capacity, sample_ray, sample_k);
        return dvgo::launch_status();
    }
    DVGO_LAUNCH(K_SCAN, scan_offsets_kernel, dim3(1), dim3(kScanThreads), 0, s, counts, B, ray_offset, n_kept);
    if (int32_t st = dvgo::launch_status()) return st;
    DVGO_LAUNCH(K_FILL_KEPT, fill_kept_kernel, dim3(wblocks), dim3(256), 0, s, ka, ray_offset, capacity, sample_ray,
                       sample_k);
    return dvgo::launch_status();
}

int32_t dvgo_sample_rays(const float* rays_o, const float* rays_d, const float* jitter, int32_t B,
                         const dvgo_box* box, float step, int32_t max_samples, const uint32_t* coarse_bits,
                         const dvgo_box* coarse_box, const uint32_t* seg_mask, const dvgo_fine_filter* fine,
                         int32_t morton, float* t_near,
                         float* t_far, uint8_t* valid, int32_t* n_uniform, int32_t* perm, int32_t* ray_offset,
                         int32_t* sample_ray, int32_t* sample_k, int64_t capacity, int64_t* n_kept,
                         void* workspace, size_t workspace_bytes, void* stream) {
    return sample_rays_impl(rays_o, rays_d, jitter, B, box, step, max_samples, coarse_bits, coarse_box, seg_mask,
                            fine, morton, t_near, t_far, valid, n_uniform, perm, ray_offset, sample_ray, sample_k, capacity,
                            n_kept, workspace, workspace_bytes, true, stream);
}

// The same call with its workspace in the library's static device array
// (see the declaration): the per-ray counts and Morton keys of up to
// kNoAllocMaxRays rays.  Every kernel of the call writes these before
// reading them, so nothing needs clearing between calls.
int32_t dvgo_sample_rays_noalloc(const float* rays_o, const float* rays_d, const float* jitter, int32_t B,
                                 const dvgo_box* box, float step, int32_t max_samples, const uint32_t* coarse_bits,
                                 const dvgo_box* coarse_box, const uint32_t* seg_mask,
                                 const dvgo_fine_filter* fine, int32_t morton,
                                 float* t_near, float* t_far, uint8_t* valid, int32_t* n_uniform, int32_t* perm,
                                 int32_t* ray_offset, int32_t* sample_ray, int32_t* sample_k, int64_t capacity,
                                 int64_t* n_kept, void* stream) {
    if (B > kNoAllocMaxRays) {
        dvgo::record_text("dvgo_sample_rays_noalloc: more rays than its static scratch holds (262144)");
        return DVGO_E_UNSUPPORTED;
    }
    void* ws = nullptr;
    if (int32_t st = scratch_address(&ws)) return st;
    return sample_rays_impl(rays_o, rays_d, jitter, B, box, step, max_samples, coarse_bits, coarse_box, seg_mask,
                            fine, morton, t_near, t_far, valid, n_uniform, perm, ray_offset, sample_ray, sample_k, capacity,
                            n_kept, ws, kNoAllocScratchBytes, false, stream);
}

}  // extern "C"
