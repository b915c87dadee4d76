/*
 * dvgo.h - C ABI of the MI355X (gfx950) library for the fine-stage per-ray
 * training step of direct voxel-grid radiance-field optimisation
 * (Sun, Sun and Chen, "Direct Voxel Grid Optimization", arXiv 2111.11215).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers: unless marked "host", every pointer is a device pointer to a
 *   caller-owned buffer (for example a torch tensor's data_ptr()).  The
 *   library allocates nothing: scratch memory is passed in as a workspace
 *   whose size the matching *_workspace_bytes query returns.
 * Streams: `stream` is a hipStream_t passed as void*; NULL is the default
 *   stream.  Every call is asynchronous with respect to the host and orders
 *   its kernels on that stream only.
 * Errors: every entry point returns a dvgo_status.  Arguments are validated
 *   on the host before anything is enqueued; on a non-zero status nothing has
 *   been enqueued.  DVGO_E_HIP means a launch failed; dvgo_last_error() then
 *   holds the HIP error text.  Conditions only the device can see (sample
 *   capacity overflow) are reported through device-side counters documented
 *   per call.
 * Layouts: rays [B][3] float32 with unit-norm directions; vertex grids
 *   spanning the box inclusively ("align-corners"), density [nx][ny][nz] and
 *   features channel-last [nx][ny][nz][C]; network weights row-major
 *   [out][in] float32.
 * Numerics: discrete decisions (ray validity, sample counts, kept samples,
 *   Morton order, proposal masks) follow an explicit float32 recipe with no
 *   contraction, documented per call, so they are reproducible bit for bit.
 */
#ifndef DVGO_H
#define DVGO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dvgo_status {
    DVGO_OK = 0,
    DVGO_E_ARG = -1,          /* null pointer, negative size, bad value      */
    DVGO_E_SHAPE = -2,        /* inconsistent sizes                          */
    DVGO_E_DTYPE = -3,        /* unsupported element type / precision code   */
    DVGO_E_CAPACITY = -4,     /* a caller buffer or workspace is too small   */
    DVGO_E_HIP = -5,          /* a HIP launch failed (see dvgo_last_error)   */
    DVGO_E_UNSUPPORTED = -6   /* valid but not implemented (e.g. size limit) */
} dvgo_status;

enum { DVGO_F32 = 0, DVGO_BF16 = 1 };
enum { DVGO_TOY_PRE = 0, DVGO_TOY_IN = 1, DVGO_TOY_POST = 2 };

/* Axis-aligned box with n[i] grid vertices per axis spanning it inclusively. */
typedef struct dvgo_box {
    float xyz_min[3];
    float xyz_max[3];
    int32_t n[3];
} dvgo_box;

/* Fine scene representation of the paper's Sec. 4.2 (Eq. fine_queries):
 * the density grid with post-activation (Eq. post_activation, shift b of
 * Eq. density_activation) and the feature grid.  `feat` is float32 or a
 * bfloat16 shadow (feat_dtype), channel-last; `channels` must be 12.  The
 * render calls index vertices and cells in 32 bits: a grid of 2^31 or more
 * vertices is DVGO_E_UNSUPPORTED. */
typedef struct dvgo_field {
    const float* density;
    const void* feat;
    int32_t feat_dtype;
    int32_t channels;
    dvgo_box box;
    float act_shift;
} dvgo_field;

/* The shallow colour network of Eq. fine_queries: input [feat(C), PE(d)(27)],
 * two ReLU layers of `hidden` (must be 128) and a sigmoid RGB output.
 * Weights are float32 masters [out][in]; `precision` selects the arithmetic
 * of its matrix products: DVGO_F32 (float32 matrix cores) or DVGO_BF16
 * (bfloat16 inputs, float32 accumulation).
 * pe_x = 5 selects the paper's network that also takes the encoded query
 * position (Eq. fine_queries with k_x = 5 frequencies, supplementary
 * implementation details): input [feat(C), PE_5(u)(33), PE(d)(27)] (72 for
 * C = 12), where u = (x - centre) / half-extent is the sample's position in
 * the field box's coordinates (centre and 2/(max - min) rounded once to
 * float32) and PE_5(u) = [u, sin(2^j u), cos(2^j u)], j = 0..4, three
 * components each.  In DVGO_BF16 the per-sample part [feat, PE_5(u)] is
 * rounded to bfloat16 as feat alone is otherwise.  pe_x = 0
 * (zero-initialised structs) is the 39-input network; other values are
 * DVGO_E_UNSUPPORTED. */
typedef struct dvgo_mlp {
    const float* w1; const float* b1;   /* [hidden][C+27] (pe_x 5: [hidden][C+60]), [hidden] */
    const float* w2; const float* b2;   /* [hidden][hidden], [hidden] */
    const float* w3; const float* b3;   /* [3][hidden], [3] */
    int32_t hidden;
    int32_t precision;
    int32_t pe_x;
} dvgo_mlp;

/* Flat gradient layout of dvgo_mlp: w1, b1, w2, b2, w3, b3 concatenated. */
int64_t dvgo_mlp_param_count(int32_t channels, int32_t hidden, int32_t pe_x);

/* Proposal network (not in the paper: a learned predictor of which of 32
 * equal-count ray segments carry the compositing weight): input 54 values
 * (positional encodings, 4 frequencies, of the box-entry point in box
 * coordinates and of the direction), two ReLU layers of 64, 32 logits.
 * float32 masters [out][in]; evaluated with bfloat16 matrix products. */
typedef struct dvgo_prop {
    const float* w1; const float* b1;   /* [64][54], [64] */
    const float* w2; const float* b2;   /* [64][64], [64] */
    const float* w3; const float* b3;   /* [32][64], [32] */
} dvgo_prop;
int64_t dvgo_prop_param_count(void);

/* ------------------------------------------------------------------------ */
/* The method's scalar hyperparameters (host functions, no device work).
 *
 * dvgo_low_density_bias: the softplus shift b of the low-density
 *   initialisation (paper Eq. low_density_init and its supplementary
 *   derivation): with a zero density grid every voxel of size `voxel` lets
 *   through 1 - alpha_init of the light, b = log((1 - alpha_init)^(-1/voxel)
 *   - 1), evaluated as log(expm1(-log1p(-alpha_init)/voxel)).
 *   alpha_init in (0, 1), voxel > 0, bias a host double; else DVGO_E_ARG.
 * dvgo_coarse_raw_threshold: the raw-density threshold of the free-space
 *   test (paper Sec. 4.2, "Known free space and unknown space"): a point is
 *   kept when alpha(softplus(raw + act_shift), step) >= tau; both activations
 *   increase with raw, so this is raw >= softplus^{-1}(-log(1-tau)/step) -
 *   act_shift, computed in float64 and rounded DOWN to float32 (a float32
 *   comparison against it never drops a point the exact test keeps).
 *   tau in (0, 1), step > 0, act_shift finite, threshold a host float; else
 *   DVGO_E_ARG.
 * dvgo_lr_at: the learning rate of the exponential schedule (paper Sec. 5.2
 *   and the supplementary implementation details: decayed to 0.1x at 20k
 *   iterations): lr = base_lr * decay^(it/decay_steps).  base_lr >= 0,
 *   it >= 0, decay_steps > 0, decay > 0, lr a host double; else DVGO_E_ARG. */
int32_t dvgo_low_density_bias(double alpha_init, double voxel, double* bias /*host*/);
int32_t dvgo_coarse_raw_threshold(double tau, double step, double act_shift, float* threshold /*host*/);
int32_t dvgo_lr_at(double base_lr, int64_t it, int64_t decay_steps, double decay, double* lr /*host*/);
/* dvgo_pg_resolution: vertices per axis of a progressively scaled grid
 *   (paper Sec. 4.2, "Progressive scaling": the voxel count starts at
 *   1/2^K of the final one for K checkpoints and doubles at each) before
 *   checkpoint k = 0..K: floor((n_final^3 / 2^(K-k))^(1/3)), at least 2.
 *   n_final >= 2, 0 <= k <= K, n a host int; else DVGO_E_ARG. */
int32_t dvgo_pg_resolution(int32_t n_final, int32_t n_checkpoints, int32_t k, int32_t* n /*host*/);

/* ------------------------------------------------------------------------ */
/* Coarse alpha mask (paper Sec. 4.2, "Known free space and unknown space"
 * and "Free space skipping", first rule).  One bit per cell of the frozen
 * coarse density grid raw [nx][ny][nz] (box cbox): bit c of word c>>5, with
 * c = (ix*(ny-1)+iy)*(nz-1)+iz, is set when the largest of the cell's 8
 * corner raw values is >= raw_threshold.  With raw_threshold =
 * softplus^{-1}(-log(1-tau)/delta) - b (rounded down to float32) every point
 * whose post-activated coarse alpha reaches tau lies in a kept cell.
 * bits: ceil((nx-1)(ny-1)(nz-1)/32) words, fully overwritten. */
int32_t dvgo_coarse_mask_build(const float* raw, const dvgo_box* cbox /*host*/,
                               float raw_threshold, uint32_t* bits, void* stream);

/* Second free-space rule of the paper's Sec. 4.2 ("Free space skipping"): a
 * sample in unknown space is skipped when the post-activated alpha of the
 * fine density grid at it is below tau^(f).  Both activations increase with
 * the raw value, so the sampler keeps a sample iff raw >= raw_threshold
 * (dvgo_coarse_raw_threshold(tau_f, step, b)), with raw interpolated from
 * `density` [n0][n1][n2] (box: its extent and vertex counts) in the float32
 * recipe: per axis u = (x-min)*((n-1)/(max-min)), fl = clamp(floor(u), 0,
 * n-2), f = clamp(u-fl, 0, 1); corner c = (c>>2 &1, c>>1 &1, c &1) has
 * weight ((gx*gy)*gz) with g = (1-f, f); raw = w_0 V_0 + ... + w_7 V_7
 * added one product at a time in corner order, no contraction. */
typedef struct dvgo_fine_filter {
    const float* density;
    dvgo_box box;
    float raw_threshold;
} dvgo_fine_filter;

/* ------------------------------------------------------------------------ */
/* Ray sampling of the fine stage (paper Eq. coarse_sample with the training
 * jitter of the supplementary details, Sec. 4.2 "Fine-stage points
 * sampling" and "Free space skipping" rule one).
 *
 * Per ray (float32 recipe, every operation rounded, no FMA):
 *   slab clip: per axis inv = 1/d, t0 = (min-o)*inv, t1 = (max-o)*inv
 *     (d = 0: unbounded if min <= o <= max, else a miss); t_enter = max fmin,
 *     t_exit = min fmax; t_near = max(t_enter, 0), t_far = t_exit;
 *     valid = t_near < t_far (invalid rays get t_near = t_far = 0);
 *   uniform samples t_k = t_near + ((float)k + p)*step, k >= 0, while
 *     t_k < t_far and k < max_samples: n_uniform = their count;
 *   kept samples: x_k = o + t_k*d; kept when the coarse bit of its cell
 *     (cell = clamp(floor((x-min)*((n-1)/(max-min))), 0, n-2)) is set
 *     (coarse_bits NULL: all kept) and, with seg_mask, when bit
 *     floor(32k/n_uniform) of seg_mask[r] is set, and, with `fine`, when
 *     the second free-space rule keeps it (see dvgo_fine_filter).
 * Ray order of the compact list: slot i holds ray perm[i]; perm is the
 *   identity, or with `morton` != 0 the rays sorted by (key, ray id) where key
 *   is the 15-bit Morton code (x most significant) of the segment midpoint
 *   o + ((t_near+t_far)*0.5)*d quantised to 32 cells per axis of `box`,
 *   invalid rays last (key 2^15).  morton requires B <= 32768.
 * Outputs: t_near, t_far [B]; valid [B] (0/1); n_uniform [B];
 *   perm [B]; ray_offset [B+1] (ray perm[i] owns samples ray_offset[i] ..
 *   ray_offset[i+1]-1, ascending k); sample_ray, sample_k [capacity];
 *   n_kept: device int64, the total kept.  When n_kept > capacity the list
 *   is truncated (samples at index >= capacity are not written) and the
 *   caller must retry with a larger capacity; capacity = B*max_samples never
 *   overflows.
 * Clip only: with capacity == 0 and ray_offset == n_kept == NULL, only
 *   t_near, t_far, valid, n_uniform and perm are produced (no counting of
 *   kept samples, no list).
 * jitter: [B] per-ray p in [0,1), or NULL for p = 0.
 * workspace: dvgo_sample_workspace_bytes(B) bytes. */
size_t dvgo_sample_workspace_bytes(int32_t B);
int32_t dvgo_sample_rays(const float* rays_o, const float* rays_d, const float* jitter,
                         int32_t B, const dvgo_box* box /*host*/, float step,
                         int32_t max_samples, const uint32_t* coarse_bits,
                         const dvgo_box* coarse_box /*host, or NULL*/,
                         const uint32_t* seg_mask, const dvgo_fine_filter* fine /*host, or NULL*/,
                         int32_t morton,
                         float* t_near, float* t_far, uint8_t* valid, int32_t* n_uniform,
                         int32_t* perm, int32_t* ray_offset, int32_t* sample_ray,
                         int32_t* sample_k, int64_t capacity, int64_t* n_kept,
                         void* workspace, size_t workspace_bytes, void* stream);

/* dvgo_sample_rays without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, outputs, recipe and
 * errors as dvgo_sample_rays; the call allocates nothing: its scratch (the
 * per-ray counts and Morton keys) lives in a static device array of the
 * library, 2 MiB + 256 bytes, which every GPU the library runs on holds
 * until the process ends.  Limit: B <= 262144 rays, else DVGO_E_UNSUPPORTED
 * with dvgo_last_error() saying so and nothing enqueued.  All calls on one
 * GPU share that array: calls that overlap on one GPU (concurrent streams,
 * or host threads with no ordering between their calls) race and must not
 * be issued; calls ordered on one stream are safe.  The array's device
 * address is looked up once per device, on the first call with that device
 * current. */
int32_t dvgo_sample_rays_noalloc(const float* rays_o, const float* rays_d, const float* jitter,
                                 int32_t B, const dvgo_box* box /*host*/, float step,
                                 int32_t max_samples, const uint32_t* coarse_bits,
                                 const dvgo_box* coarse_box /*host, or NULL*/,
                                 const uint32_t* seg_mask, const dvgo_fine_filter* fine /*host, or NULL*/,
                                 int32_t morton,
                                 float* t_near, float* t_far, uint8_t* valid, int32_t* n_uniform,
                                 int32_t* perm, int32_t* ray_offset, int32_t* sample_ray,
                                 int32_t* sample_k, int64_t capacity, int64_t* n_kept, void* stream);

/* ------------------------------------------------------------------------ */
/* Forward volume rendering (paper Eq. volume_rendering, Eq. fine_queries,
 * Eq. post_activation) of the samples listed by dvgo_sample_rays, per ray in
 * ascending k:
 *   raw_k = interp(x_k, density), sigma_k = softplus(raw_k + act_shift),
 *   alpha_k = 1 - exp(-sigma_k*step), T_k = exp(-step*sum_{j<k} sigma_j),
 *   w_k = T_k alpha_k, c_k = MLP([interp(x_k, feat), PE(d)]),
 *   rgb = sum w_k c_k + T_end*bg, depth = sum w_k t_k, acc = sum w_k,
 *   log_t_end = -step*sum sigma_k, seg_w[r][s] = sum of w_k over segment
 *   s = floor(32k/n_uniform).
 * Trilinear interpolation: u = (x-min)*((n-1)/(max-min)), i0 =
 *   clamp(floor(u), 0, n-2), f = clamp(u-i0, 0, 1).  PE(d) = [d, sin(2^j d),
 *   cos(2^j d)] for j = 0..3.
 * m == NULL renders density only (rgb must then be NULL; the other outputs
 *   are produced): the proposal's target pass.
 * Outputs indexed by ray id: rgb [B][3], depth, acc, log_t_end [B] (each
 *   NULL to skip except log_t_end, which the backward pass needs),
 *   seg_w [B][32] or NULL; sample_w [capacity] or NULL (w_k in compact-list
 *   order).  All are overwritten.
 * n_kept: the device count written by dvgo_sample_rays; samples beyond
 *   min(n_kept, capacity) are ignored.
 * bg: host float[3].
 * workspace: dvgo_render_workspace_bytes(B, capacity, channels, &field.box)
 *   bytes (0 for an unsupported channel count or an invalid box), which the
 *   backward needs; the forward alone needs only the smaller
 *   dvgo_render_fwd_workspace_bytes. */
size_t dvgo_render_workspace_bytes(int32_t B, int64_t capacity, int32_t channels,
                                   const dvgo_box* grid /*host*/);
size_t dvgo_render_fwd_workspace_bytes(int32_t B, int64_t capacity, int32_t channels,
                                       const dvgo_box* grid /*host*/);
int32_t dvgo_render_fwd(const dvgo_field* field /*host*/, const dvgo_mlp* mlp /*host or NULL*/,
                        const float* rays_o, const float* rays_d, const float* jitter,
                        const float* t_near, const int32_t* n_uniform, const int32_t* perm,
                        const int32_t* ray_offset, const int32_t* sample_ray,
                        const int32_t* sample_k, const int64_t* n_kept, int64_t capacity,
                        int32_t B, float step, const float* bg /*host[3]*/,
                        float* rgb, float* depth, float* acc, float* log_t_end, float* seg_w,
                        float* sample_w, void* workspace, size_t workspace_bytes, void* stream);

/* Backward pass of dvgo_render_fwd: the adjoint recomputes every per-sample
 * quantity and walks each ray from its end, starting from the forward's
 * log_t_end (no per-sample state is kept between the calls):
 *   S_{K+1} = T_end*(bg, 0, 0),  S_k = S_{k+1} + w_k*(c_k, t_k, 1),
 *   dL/dsigma_k = step * g.(T_{k+1}*(c_k, t_k, 1) - S_{k+1}),
 *   dL/draw_k = dL/dsigma_k * sigmoid(raw_k + act_shift),
 *   dL/dc_k = w_k * grad_rgb, then through the network to the features,
 * where g = (grad_rgb, grad_depth, grad_acc) (the latter two may be NULL).
 * Gradients are ACCUMULATED (+=) into grad_density [nx][ny][nz],
 * grad_feat [nx][ny][nz][C] (float32 whatever feat_dtype is) and grad_mlp
 * (flat, dvgo_mlp_param_count values; may be NULL with mlp == NULL).
 * Grid gradients: samples are binned by fine cell and each grid vertex sums
 * its neighbouring samples' contributions (no float atomics); the order of
 * samples within a cell, and so the last bits of a sum, may vary from run to
 * run.  Same workspace as dvgo_render_fwd. */
int32_t dvgo_render_bwd(const dvgo_field* field /*host*/, const dvgo_mlp* mlp /*host or NULL*/,
                        const float* rays_o, const float* rays_d, const float* jitter,
                        const float* t_near, const int32_t* n_uniform, const int32_t* perm,
                        const int32_t* ray_offset, const int32_t* sample_ray,
                        const int32_t* sample_k, const int64_t* n_kept, int64_t capacity,
                        int32_t B, float step, const float* bg /*host[3]*/,
                        const float* log_t_end, const float* grad_rgb, const float* grad_depth,
                        const float* grad_acc, float* grad_density, float* grad_feat,
                        float* grad_mlp, void* workspace, size_t workspace_bytes, void* stream);

/* Grid parameters and their Adam moments for dvgo_render_bwd_adam (all
 * device pointers, float32, updated in place):
 *   density, density_m, density_v  [nx][ny][nz];
 *   feat, feat_m, feat_v           [nx][ny][nz][C], 16-byte aligned;
 *   feat_shadow_bf16               [nx][ny][nz][C] bfloat16 bits, 8-byte
 *                                  aligned, or NULL (rewritten as bf16(feat)).
 *   active                         [ceil(nx*ny*nz/32)] uint32 words, or NULL:
 *                                  bit v (word v/32, bit v%32) must be set
 *                                  whenever any of vertex v's moments (its
 *                                  density's and its C features' m and v) is
 *                                  non-zero.  A vertex whose bit is clear and
 *                                  that no sample touches would take a step
 *                                  with m = v = 0 and a zero gradient, which
 *                                  leaves p, m and v unchanged bit for bit; it
 *                                  is skipped without reading them.  The call
 *                                  sets the bit of every vertex that steps with
 *                                  a non-zero gradient, so the mask stays valid
 *                                  across calls.  Zero-fill it together with
 *                                  zero moments, or derive it from given
 *                                  moments with dvgo_grid_active_init.  NULL:
 *                                  every vertex steps (dense Adam).
 * lr, beta1, beta2, eps and the step count t >= 1 as in dvgo_adam_step. */
typedef struct {
    float* density;
    float* density_m;
    float* density_v;
    float* feat;
    float* feat_m;
    float* feat_v;
    uint16_t* feat_shadow_bf16;
    float lr, beta1, beta2, eps;
    int32_t t;
    uint32_t* active;
} dvgo_grid_adam;

/* The activity mask of dvgo_grid_adam from given moments: active[v/32] bit
 * v%32 = 1 iff any of density_m[v], density_v[v], feat_m[v][0..C-1],
 * feat_v[v][0..C-1] is non-zero (C = 12).  Every word of active
 * [ceil(n_vertices/32)] is rewritten.  feat_m and feat_v 16-byte aligned,
 * active 4-byte aligned; n_vertices >= 0. */
int32_t dvgo_grid_active_init(const float* density_m, const float* density_v, const float* feat_m,
                              const float* feat_v, int64_t n_vertices, uint32_t* active, void* stream);

/* Backward pass and Adam step of both grids in one call: the result is that
 * of dvgo_render_bwd into zeroed grid gradients followed by dvgo_adam_step
 * on the density and the feature grid (the paper's optimiser, Sec. 5.2;
 * every vertex takes the step, with a zero gradient where no sample touches
 * it), but the grid gradients never reach memory: each vertex sums its
 * binned samples' contributions and updates its parameters and moments in
 * the same thread.  The network gradient is accumulated into grad_mlp as in
 * dvgo_render_bwd (its Adam step stays a separate dvgo_adam_step).  mlp must
 * not be NULL.  The field may read the same arrays opt updates (field->density
 * == opt->density, field->feat == opt->feat or its bfloat16 shadow): all
 * reads of the grids finish before the update within the call. */
int32_t dvgo_render_bwd_adam(const dvgo_field* field /*host*/, const dvgo_mlp* mlp /*host*/,
                             const float* rays_o, const float* rays_d, const float* jitter,
                             const float* t_near, const int32_t* n_uniform, const int32_t* perm,
                             const int32_t* ray_offset, const int32_t* sample_ray,
                             const int32_t* sample_k, const int64_t* n_kept, int64_t capacity,
                             int32_t B, float step, const float* bg /*host[3]*/,
                             const float* log_t_end, const float* grad_rgb,
                             const float* grad_depth, const float* grad_acc,
                             const dvgo_grid_adam* opt /*host*/, float* grad_mlp,
                             void* workspace, size_t workspace_bytes, void* stream);

/* Adam state of a flat float32 parameter array for a fused optimiser step:
 * param, m, v [n] device pointers, param in the flat layout of the gradient
 * it is stepped with (n = dvgo_mlp_param_count for dvgo_train_step's network
 * step, dvgo_prop_param_count for dvgo_proposal_bwd_adam); lr, beta1,
 * beta2, eps and t >= 1 as in dvgo_adam_step. */
typedef struct {
    float* param;
    float* m;
    float* v;
    float lr, beta1, beta2, eps;
    int32_t t;
} dvgo_adam_state;

/* Weights of the auxiliary losses of the fine stage's training objective
 * (paper Sec. 4.2 "Training objective for fine representation" and the
 * supplementary implementation details: 1e-2 and 1e-3), added to the
 * photometric loss by dvgo_train_step:
 *   w_pt_rgb * (1/B) sum_r sum_k w_k ||c_k - C*_r||^2 (per-point rgb; the
 *     weights w_k are held fixed: it supervises the colours only), and
 *   w_bg_entropy * (1/B) sum_r H(clamp(T_end, 1e-6, 1 - 1e-6)) with
 *     H(p) = -p log p - (1-p) log(1-p) (background entropy; its gradient is
 *     zero where the clamp is active). */
typedef struct dvgo_aux_loss {
    float w_pt_rgb;
    float w_bg_entropy;
} dvgo_aux_loss;

/* One whole training step of the fine stage in one call: dvgo_render_fwd
 * (colour and log T_end only), dvgo_photo_loss against target [B][3]
 * (Eq. photo_loss), and dvgo_render_bwd_adam, with the same result.  Inside
 * the call the adjoint reuses what the forward left in the workspace (the
 * packed network, the per-ray encodings, every sample's gathered density
 * and features and its colour) instead of evaluating them again; the
 * transmittance is still recomputed from each ray's end.  rgb [B][3] (or
 * NULL) receives the rendered colour, loss (device float or NULL) the loss
 * (its gradient is formed inside the compositing, bit-identical to
 * dvgo_photo_loss's; the loss sum itself runs in another fixed order);
 * the grids take their Adam step through opt and the network gradient is
 * accumulated into grad_mlp.  With mlp_opt NULL the network's Adam step is
 * the caller's dvgo_adam_step; otherwise the call also takes it, with the
 * same result bit for bit as dvgo_adam_step(mlp_opt->param, grad_mlp,
 * mlp_opt->m, mlp_opt->v, NULL, n, ...) after the accumulation (grad_mlp is
 * left zero).  The network weights that mlp points at must be
 * mlp_opt->param's (every read of them ends before the update within the
 * call).  With aux (host, or NULL for none) the loss and its gradient also
 * carry the auxiliary losses (dvgo_aux_loss); when the call has no samples
 * at all (capacity 0) they are left out.  Same arguments, workspace and
 * errors as the separate calls; negative aux weights are DVGO_E_ARG. */
int32_t dvgo_train_step(const dvgo_field* field /*host*/, const dvgo_mlp* mlp /*host*/,
                        const float* rays_o, const float* rays_d, const float* jitter,
                        const float* t_near, const int32_t* n_uniform, const int32_t* perm,
                        const int32_t* ray_offset, const int32_t* sample_ray,
                        const int32_t* sample_k, const int64_t* n_kept, int64_t capacity,
                        int32_t B, float step, const float* bg /*host[3]*/,
                        const float* target, float* rgb, float* loss,
                        const dvgo_grid_adam* opt /*host*/, float* grad_mlp,
                        const dvgo_adam_state* mlp_opt /*host or NULL*/,
                        const dvgo_aux_loss* aux /*host or NULL*/,
                        void* workspace, size_t workspace_bytes, void* stream);

/* Photometric loss of paper Eq. photo_loss: loss = (1/B) sum_r
 * ||rgb_r - target_r||^2 and grad_rgb = 2 (rgb - target)/B.  grad_rgb [B][3]
 * is overwritten; loss (device float, or NULL) is overwritten. */
int32_t dvgo_photo_loss(const float* rgb, const float* target, int32_t B, float* grad_rgb,
                        float* loss, void* stream);

/* Float64 reduction for central finite differences of the rendering
 * (checking the adjoint of Eq. volume_rendering against differences of
 * forward passes): *out = sum over i < n of sum_c weight[r][c] * rgb[r][c]
 * with r = rays[i] (rays [n] device int32), or r = i when rays is NULL
 * (then n <= B).  rgb and weight are [B][3] float32 on the device; out is
 * one device double, overwritten.  Every product is exact in float64 and
 * the sum runs in one fixed order, so equal inputs give equal bits.  Ray
 * indices outside [0, B) are skipped.  n = 0 writes 0. */
int32_t dvgo_fd_reduce_f64(const float* rgb, const float* weight, const int32_t* rays, int32_t n,
                           int32_t B, double* out, void* stream);

/* One Adam step (the paper's optimiser, Sec. 5.2) over n float32 values:
 *   m = beta1*m + (1-beta1)*g;  v = beta2*v + (1-beta2)*g^2;
 *   p -= lr * (m/(1-beta1^t)) / (sqrt(v/(1-beta2^t)) + eps);  g = 0;
 * and, when shadow_bf16 is not NULL, shadow = bf16(p) (round to nearest
 * even), the storage the bfloat16 feature gathers read.  t >= 1. */
int32_t dvgo_adam_step(float* p, float* g, float* m, float* v, uint16_t* shadow_bf16,
                       int64_t n, float lr, float beta1, float beta2, float eps, int32_t t,
                       void* stream);

/* ------------------------------------------------------------------------ */
/* Learned proposal (not in the paper).  Forward: logits z [B][32] of the
 * proposal network on each ray's encoding; q = softmax([z, 0]) over 33
 * entries (the last is the transmitted share), pred_mass = sum_{s<32} q_s;
 * seg_mask[r] = the smallest set of segments, by descending q (ties to the
 * lower index), whose q sum reaches cum_frac * pred_mass, or all ones when
 * pred_mass < min_mass or the ray is invalid.  The selection follows an
 * explicit float32 recipe from the float32 logits (no contraction), so the
 * mask is reproducible bit for bit: m = max(0, z_s); e_s = exp_f32(z_s - m),
 * e_T = exp_f32(-m), where exp_f32 is the Cody-Waite reduction
 * k = rint(x*log2e), r = (x - k*ln2_hi) - k*ln2_lo (ln2_hi = 0x1.62e4p-1,
 * ln2_lo = 0x1.7f7d1cp-20), the degree-7 Taylor polynomial of e^r by
 * Horner's rule and the scale 2^k (0 for x < -87); tot = e_0 + ... + e_31
 * + e_T, q_s = e_s/tot and pred_mass = q_0 + ... + q_31, each summed one
 * term at a time in that order; the chosen q are added in the order chosen
 * until the sum reaches cum_frac*pred_mass (float32 product).
 * cum_frac in (0, 1], min_mass in [0, 1], else DVGO_E_ARG.
 * valid/t_near come from dvgo_sample_rays; with t_near (and valid) NULL the
 * call clips each ray against box itself with the sampler's recipe, which
 * gives the same t_near and validity bit for bit (one launch instead of a
 * separate clip).  valid without t_near is DVGO_E_ARG. */
int32_t dvgo_proposal_fwd(const float* rays_o, const float* rays_d, const float* t_near,
                          const uint8_t* valid, int32_t B, const dvgo_box* box /*host*/,
                          const dvgo_prop* prop /*host*/, float cum_frac, float min_mass,
                          float* logits, float* pred_mass, uint32_t* seg_mask, void* stream);

/* Proposal backward: KL(p || q) summed over the valid rays and divided by
 * the batch size B (invalid rays contribute nothing), with target
 * p = (seg_w[r][0..31], exp(log_t_end[r])) from a density-only render;
 * dL/dz_s = (q_s - p_s)/B.  grad_prop (flat, dvgo_prop_param_count) is
 * ACCUMULATED; loss (device float or NULL) is overwritten.  t_near/valid
 * as in dvgo_proposal_fwd (NULL: clipped here). */
int32_t dvgo_proposal_bwd(const float* rays_o, const float* rays_d, const float* t_near,
                          const uint8_t* valid, int32_t B, const dvgo_box* box /*host*/,
                          const dvgo_prop* prop /*host*/, const float* seg_w,
                          const float* log_t_end, float* grad_prop, float* loss,
                          void* workspace, size_t workspace_bytes, void* stream);
size_t dvgo_proposal_workspace_bytes(int32_t B);

/* dvgo_proposal_bwd followed by the proposal's Adam step, the step taken in
 * the launch that sums the gradient (Adam with bias correction, the
 * optimiser of Sec. 5.2, on a network that is not in the paper): the same
 * result bit for bit as dvgo_proposal_bwd(..., grad_prop, loss, ...) then
 * dvgo_adam_step(opt->param, grad_prop, opt->m, opt->v, NULL,
 * dvgo_prop_param_count(), opt->lr, opt->beta1, opt->beta2, opt->eps,
 * opt->t).  grad_prop (device, may hold gradient from earlier calls) is
 * consumed and left zero; opt->param is normally the flat array that prop
 * points into (the weights are read before the step).  B == 0 still takes
 * the step.  opt NULL, a NULL pointer in it or bad hyper-parameters:
 * DVGO_E_ARG; workspace as for dvgo_proposal_bwd. */
int32_t dvgo_proposal_bwd_adam(const float* rays_o, const float* rays_d, const float* t_near,
                               const uint8_t* valid, int32_t B, const dvgo_box* box /*host*/,
                               const dvgo_prop* prop /*host*/, const float* seg_w,
                               const float* log_t_end, float* grad_prop,
                               const dvgo_adam_state* opt /*host*/, float* loss,
                               void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Coarse stage (paper Sec. 4.1, "Coarse geometry searching").
 *
 * dvgo_coarse_field: the coarse density grid (post-activated with shift
 * act_shift, Eq. density_activation) and the view-invariant colour grid
 * rgb [n0][n1][n2][3] (Eq. coarse_queries; the colour is the sigmoid of the
 * interpolated 3 channels, the output activation of the paper's Sec. 3).
 *
 * dvgo_coarse_step: one training step's forward and gradient over the
 * sample list of dvgo_sample_rays (the coarse stage samples every in-box
 * point: no coarse mask), per ray in ascending k, with the quadrature of
 * dvgo_render_fwd (bg host float[3]) and the loss
 *   L = (1/B) sum_r [ ||C_r - C*_r||^2 + w_pt sum_k w_k ||c_k - C*_r||^2
 *                     + w_bg H(clamp(T_end, 1e-6, 1 - 1e-6)) ],
 * H(p) = -p log p - (1-p) log(1-p); in the per-point term the weights w_k
 * are held fixed (it supervises the colours only); H's gradient is zero
 * where the clamp is active.  target [B][3]; rgb [B][3] (or NULL) receives
 * C_r; loss (device float) L; grad_density [n] and grad_rgb [n][3] are
 * ACCUMULATED (+=) with float atomics (the summation order varies between
 * runs).  The adjoint walks each ray from its end with the transmittance
 * recomputed by prefix sums.  max_samples (the sampler's) at most 4096, else
 * DVGO_E_UNSUPPORTED.  workspace: dvgo_coarse_workspace_bytes(B). */
typedef struct dvgo_coarse_field {
    const float* density;
    const float* rgb;
    dvgo_box box;
    float act_shift;
} dvgo_coarse_field;
size_t dvgo_coarse_workspace_bytes(int32_t B);
int32_t dvgo_coarse_step(const dvgo_coarse_field* field /*host*/, const float* rays_o, const float* rays_d,
                         const float* jitter, const float* t_near, const int32_t* perm, const int32_t* ray_offset,
                         const int32_t* sample_k, const int64_t* n_kept, int64_t capacity, int32_t B,
                         int32_t max_samples, float step, const float* bg /*host[3]*/, const float* target,
                         float w_pt, float w_bg, float* rgb, float* grad_density, float* grad_rgb, float* loss,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Prior 2 of Sec. 4.1 (view-count-based learning rate): counts [n] = the
 * number of the ncam training views each vertex of `box` (positions
 * min + j*((max-min)/(n-1)), float32) is visible to, and lr_scale [n] =
 * counts / max(counts).  Visible: inside the pinhole frustum, no occlusion
 * test: with p = R^T (x - centre), p_z < 0 and (focal p_x/(-p_z) + W/2,
 * -focal p_y/(-p_z) + H/2) in [0, W) x [0, H).  cams [ncam][12] device
 * float32: R row-major (camera-to-world, columns right, up, back) then the
 * centre.  workspace: dvgo_view_counts_workspace_bytes(). */
size_t dvgo_view_counts_workspace_bytes(void);
int32_t dvgo_view_counts(const dvgo_box* box /*host*/, const float* cams, int32_t ncam, int32_t H, int32_t W,
                         float focal, int32_t* counts, float* lr_scale, void* workspace, size_t workspace_bytes,
                         void* stream);

/* dvgo_adam_step with a per-element learning-rate factor: element i takes
 * the step with lr * lr_scale[i] (Prior 2's n_j / n_max on the coarse
 * density); g is zeroed.  No bfloat16 copy. */
int32_t dvgo_adam_step_scaled(float* p, float* g, float* m, float* v, const float* lr_scale, int64_t n,
                              float lr, float beta1, float beta2, float eps, int32_t t, void* stream);

/* ------------------------------------------------------------------------ */
/* Progressive scaling (paper Sec. 4.2, "Progressive scaling": at each
 * checkpoint the grids are resized by trilinear interpolation).  dst
 * [dst_box->n][channels] receives, at each of its vertices
 * x_j = min + j*((max-min)/(n-1)) (per axis, float32, on dst_box), the
 * trilinear interpolation of src [src_box->n][channels] (channel-last;
 * positions outside src_box clamp to its faces).  Every dst value is
 * written.  A bad box or channel count is DVGO_E_ARG. */
int32_t dvgo_grid_resample(const float* src, const dvgo_box* src_box /*host*/, int32_t channels, float* dst,
                           const dvgo_box* dst_box /*host*/, void* stream);

/* ------------------------------------------------------------------------ */
/* Test-time rendering of a whole image (paper Sec. 4.2 "Free space
 * skipping" in testing, and the test-time rendering of Sec. 5): the same
 * sampler and forward as training without jitter (p = 0) and without a
 * proposal.  Pinhole camera: pixel (i, j) of an H x W image casts the ray
 * from `origin` along normalize(c2w * ((j + 1/2 - W/2)/focal,
 * -(i + 1/2 - H/2)/focal, -1)), c2w row-major (columns: camera right, up
 * and back in world space), evaluated in float32.  Pixels are processed in
 * chunks of `chunk` rays: each chunk casts its rays, runs dvgo_sample_rays
 * (coarse_bits/coarse_box and the fine filter as there, or NULL) with capacity
 * chunk*max_samples (no overflow possible) and dvgo_render_fwd.
 * Outputs, row-major over pixels: rgb [H*W][3], depth and acc [H*W] (each
 * NULL to skip, rgb required); rays_o, rays_d [H*W][3] (NULL to skip)
 * receive the cast rays.  mlp required.  workspace:
 * dvgo_render_image_workspace_bytes(chunk, max_samples, &field.box)
 * (0 when chunk*max_samples reaches 2^31).  Errors as dvgo_render_fwd's. */
typedef struct dvgo_camera {
    float c2w[9];
    float origin[3];
    int32_t H, W;
    float focal;
} dvgo_camera;
size_t dvgo_render_image_workspace_bytes(int32_t chunk, int32_t max_samples, const dvgo_box* grid /*host*/);
int32_t dvgo_render_image(const dvgo_field* field /*host*/, const dvgo_mlp* mlp /*host*/,
                          const dvgo_camera* cam /*host*/, float step, int32_t max_samples,
                          const uint32_t* coarse_bits, const dvgo_box* coarse_box /*host, or NULL*/,
                          const dvgo_fine_filter* fine /*host, or NULL*/, const float* bg /*host[3]*/, int32_t chunk, float* rgb, float* depth, float* acc,
                          float* rays_o, float* rays_d, void* workspace, size_t workspace_bytes,
                          void* stream);

/* ------------------------------------------------------------------------ */
/* Image-fitting toy of the paper's Sec. 3 ("Sharp decision boundary via
 * post-activation"; Eq. pre_activation, in_activation, post_activation):
 * a grid V [gh][gw] (float32, gh, gw >= 2), its vertices spanning an H x W
 * image inclusively, is interpolated bilinearly at the pixel centres: pixel
 * (i, j) sits at u = (i + 1/2)*((gh-1)/H), v = (j + 1/2)*((gw-1)/W) (the
 * ratios rounded once to float32), cell i0 = clamp(floor(u), 0, gh-2) (and
 * j0), fractions clamped to [0, 1].  With softplus(x) = log(1 + e^x) (no
 * shift) and alpha(s) = 1 - exp(-s*delta), the predicted alpha is
 *   DVGO_TOY_PRE:  interp(alpha(softplus(V)));
 *   DVGO_TOY_IN:   alpha(interp(softplus(V)));
 *   DVGO_TOY_POST: alpha(softplus(interp(V))).
 * dvgo_toy2d_forward writes image [H][W].  dvgo_toy2d_loss_grad writes
 * loss (device float) = mean over pixels of (alpha - target)^2 and
 * grad [gh][gw] = dloss/dV (overwritten; each vertex sums its pixels'
 * contributions in row-major order, no atomics), with a workspace of
 * dvgo_toy2d_workspace_bytes(H, W) bytes.  delta > 0; a bad mode or size
 * is DVGO_E_ARG, H*W or gh*gw of 2^31 or more DVGO_E_UNSUPPORTED. */
size_t dvgo_toy2d_workspace_bytes(int32_t H, int32_t W);
int32_t dvgo_toy2d_forward(const float* V, int32_t gh, int32_t gw, int32_t H, int32_t W, int32_t mode,
                           float delta, float* image, void* stream);
int32_t dvgo_toy2d_loss_grad(const float* V, int32_t gh, int32_t gw, const float* target, int32_t H,
                             int32_t W, int32_t mode, float delta, float* grad, float* loss,
                             void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Data generation (not part of the training step): colour of each ray
 * through an analytic scene of soft spheres, rows (cx,cy,cz,r,rho,R,G,B):
 * density sum_i rho_i*sigmoid((r_i - |x-c_i|)/edge), colour the density-
 * weighted mean, composited by the same quadrature at midpoints
 * t_near + (k+1/2)*step inside the box, background bg (host float[3]). */
int32_t dvgo_scene_render(const float* rays_o, const float* rays_d, int32_t B,
                          const dvgo_box* box /*host*/, const float* spheres, int32_t n_spheres,
                          float edge, float step, const float* bg /*host[3]*/, float* rgb,
                          void* stream);

/* Human-readable text of a status; dvgo_last_error() is the last HIP error
 * text recorded by this thread (empty if none).  Static strings. */
const char* dvgo_status_string(int32_t status);
const char* dvgo_last_error(void);
int32_t dvgo_version(void);

/* Optional timing of one kernel (host-side, not thread-safe): with
 * kernel_id >= 0, every later launch of that kernel is bracketed by a pair of
 * HIP events recorded on the launch's own stream; dvgo_profile_read waits for
 * them and returns the summed elapsed milliseconds and the launch count since
 * the last dvgo_profile_enable.  kernel_id -1 turns timing off.  Ids:
 *   0 ray setup, 1 Morton sort, 2 count kept, 3 ray-offset scan (batches above 16384 rays), 4 fill kept (up
 *   to 16384 rays with the offsets in the same launch),
 *   5 coarse mask, 6 (unused), 7 weight pack + per-ray encoding, 8 gather, 9 MLP forward,
 *   10 compose forward, 11 compose backward, 12 MLP backward, 13 vertex
 *   gather (gradient scatter), 14 partial reduce, 15 photo loss, 16 Adam,
 *   17 proposal forward, 18 proposal backward, 19 proposal reduce, 20 scene
 *   render, 21 (unused: cell binning counts run inside 11), 22 cell scan,
 *   23 record placement when there is no network,
 *   24 vertex gather with the grids' Adam step (dvgo_render_bwd_adam),
 *   25 activity mask from moments (dvgo_grid_active_init), 26 toy pixels,
 *   27 toy vertex gradients, 28 toy loss reduction, 29 grid resample,
 *   30 coarse-stage step, 31 view counts. */
int32_t dvgo_profile_enable(int32_t kernel_id);
int32_t dvgo_profile_read(double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* DVGO_H */
