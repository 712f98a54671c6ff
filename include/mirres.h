/*
 * mirres.h — C ABI of the MI355X (gfx950) differentiable path tracer with
 * reservoir-resampled environment lighting: the rendering hot path of MIRReS
 * (arXiv 2406.16360).
 *
 * The problem statement (Sec. 3 "Method overview"): given a triangle mesh,
 * spatially-varying materials, an HDR environment map and calibrated
 * cameras, render images with physically based path tracing and
 * back-propagate image-space gradients to the materials and the environment
 * map.  Here:
 *   - rendering equation, Sec. 3 Eq. pbr_render, with the incident light
 *     split into visible environment light plus indirect light (Eq. incident);
 *   - direct light by resampled importance sampling with a streaming weighted
 *     reservoir (Sec. 4.1, Eq. restir; Appendix A "Spatial-temporal reuse"
 *     for the reservoir update), over environment-map and BRDF candidates;
 *   - indirect light by BRDF-sampled multi-bounce continuation truncated
 *     after `bounces` surface vertices (Sec. 4.2, Eqs. mc_indir, sec_bouce);
 *   - visibility by explicit ray-mesh intersection over a linear BVH
 *     (Appendix A "Visibility estimation");
 *   - gradients of the detached-sampling path functional (Sec. 4.2 detaches
 *     indirect rays; grad_mode selects that or the full path).
 *
 * Conventions shared by every entry point
 *   Memory     Arrays named d_* and every pointer inside mrs_scene / mrs_grads
 *              / mrs_options debug fields are DEVICE pointers, caller-owned,
 *              contiguous, float32 / int32 / uint32.  mrs_view arrays and the
 *              structs themselves are HOST memory, read during the call only.
 *              The library owns only mrs_bvh, mrs_tape and an internal
 *              workspace; release them with the *_destroy calls.
 *   Streams    `stream` is a hipStream_t (NULL = default stream).  All work
 *              is enqueued on it; calls return before the GPU finishes, except
 *              mrs_build_bvh, which waits for its own stream.
 *   Errors     Every call returns an mrs_status; nothing throws across the
 *              ABI.  mrs_last_error() gives a message for the last failing
 *              call on the calling thread (valid until the next call).
 *              Arguments are validated on the host before any GPU work.
 *   Layouts    mesh positions [nv][3], faces [nf][3] (int32 vertex indices),
 *              uv [nv][2]; per-vertex materials [nv][5] = (albedo r, g, b,
 *              roughness, metallic); textures albedo [th][tw][3],
 *              roughness [th][tw], metallic [th][tw] (row 0 at v = 0,
 *              bilinear, wrap); or the material field (mrs_field) at the
 *              hit point; env [eh][ew][3] linear HDR, equirectangular,
 *              +y up, row 0 at the +y pole.  Images are packed per view at
 *              pixel_offset: [sum_v W_v * H_v][3], row-major, row 0 on top.
 *   Random     Every uniform is Philox4x32-10 (Salmon et al., SC'11) with
 *              key = seed and counter = (pixel, sample_offset + sample, view,
 *              (vertex << 16) | block); the output is bit-deterministic for
 *              fixed inputs.
 */
#ifndef MIRRES_H
#define MIRRES_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MRS_OK = 0,
    MRS_EINVAL = -1,        /* invalid argument (message says which) */
    MRS_ENOMEM = -2,        /* device or pinned-host allocation failed */
    MRS_EHIP = -3,          /* a HIP runtime call failed */
    MRS_EOVERFLOW = -4,     /* a size exceeds a documented limit */
    MRS_EUNSUPPORTED = -5   /* option combination not implemented */
} mrs_status;

enum { MRS_MAT_VERTEX = 0, MRS_MAT_TEXTURE = 1, MRS_MAT_FIELD = 2 };
enum { MRS_BRDF_LAMBERT = 0, MRS_BRDF_LAMBERT_GGX = 1 };
enum { MRS_BG_ENV = 0, MRS_BG_BLACK = 1 };
enum { MRS_GRAD_FULL = 0, MRS_GRAD_PRIMARY = 1 };
enum { MRS_TAPE_AUTO = 0, MRS_TAPE_ON = 1, MRS_TAPE_OFF = 2 };

#define MRS_MAX_BOUNCES 8
#define MRS_MAX_VIEWS 65536

typedef struct mrs_bvh mrs_bvh;     /* opaque, library-owned */
typedef struct mrs_tape mrs_tape;   /* opaque, library-owned */

/* Material neural field F_m (Sec. 3 "Intrinsic decomposition": m = F_m(x),
 * a small MLP over a multi-resolution hash grid; Appendix A "Network
 * details": 16 levels, 2 features per entry, coarsest resolution 16, finest
 * 2048, 2-layer MLP with 32 hidden units).  The encoding follows Mueller et
 * al., "Instant Neural Graphics Primitives with a Multiresolution Hash
 * Encoding" (SIGGRAPH 2022), Sec. 3:
 *   level l in [0, L): resolution N_l = floor(N_min exp(l ln(N_max/N_min) /
 *     (L - 1)) + 1e-6), computed in double (N_0 = N_min when L = 1);
 *   u = clamp((x - lo) / (hi - lo), 0, 1) per axis, s = u N_l, cell
 *     c = min(floor(s), N_l - 1), fraction s - c;
 *   grid vertex v in [0, N_l]^3 -> slot v0 + (N_l + 1)(v1 + (N_l + 1) v2)
 *     while (N_l + 1)^3 <= T, else (v0 ^ 2654435761 v1 ^ 805459861 v2)
 *     mod 2^32 mod T;
 *   e[2l + j] = trilinear interpolation of table[l][slot][j] over the cell;
 *   z1 = W1 e + b1 (32), a = max(z1, 0), z2 = W2 a + b2 (4), m = sigmoid(z2)
 *     = (albedo r, g, b, roughness); the field's metallic is 0.
 * All arrays are device float32: table [L][T][2], w1 [32][2L] (row-major),
 * b1 [32], w2 [4][32], b2 [4]. */
#define MRS_FIELD_MAX_LEVELS 16
#define MRS_FIELD_MAX_LOG2_TABLE 24
#define MRS_FIELD_MAX_RES 1048576
typedef struct {
    int32_t levels;          /* L in [1, MRS_FIELD_MAX_LEVELS] */
    int32_t log2_table;      /* T = 2^log2_table slots per level, in [1, MRS_FIELD_MAX_LOG2_TABLE] */
    int32_t n_min, n_max;    /* 1 <= n_min <= n_max <= MRS_FIELD_MAX_RES */
    float   lo[3], hi[3];    /* box mapped onto the unit cube, hi > lo */
    const float *table, *w1, *b1, *w2, *b2;
} mrs_field;

/* Gradients of the field parameters (device, accumulated with +=, each
 * nullable; shapes as in mrs_field). */
typedef struct {
    float *table, *w1, *b1, *w2, *b2;
} mrs_field_grads;

/* Scene: mesh, materials, lighting (Sec. 3: mesh {V, F}, material m,
 * environment map L_env).  All pointers are device pointers. */
typedef struct {
    const float   *pos;   int32_t nv;     /* [nv][3] */
    const int32_t *faces; int32_t nf;     /* [nf][3] */
    const float   *uv;                    /* [nv][2]; required for MRS_MAT_TEXTURE */
    const mrs_bvh *bvh;                   /* from mrs_build_bvh over the same pos/faces */
    int32_t        mat_mode;              /* MRS_MAT_VERTEX, MRS_MAT_TEXTURE or MRS_MAT_FIELD */
    const float   *vmat;                  /* [nv][5] for MRS_MAT_VERTEX */
    const float   *albedo;                /* [th][tw][3] */
    const float   *rough;                 /* [th][tw] */
    const float   *metal;                 /* [th][tw] */
    int32_t        tw, th;
    const float   *env;                   /* [eh][ew][3], fewer than 2^27 texels, ew <= 65536 */
    int32_t        ew, eh;
    mrs_field      field;                 /* the material source for MRS_MAT_FIELD */
} mrs_scene;

/* Pinhole camera (Sec. 3 "Rendering": camera ray o + t d).  c2w is
 * row-major camera-to-world; the camera looks down -z with +y up.
 * pixel_offset places this view's pixels in the packed image. */
typedef struct {
    float    c2w[16];
    float    fov_y_deg;
    int32_t  w, h, spp;
    uint32_t sample_offset;
    int64_t  pixel_offset;
} mrs_view;

typedef struct {
    int32_t  bounces;        /* B in [1, MRS_MAX_BOUNCES]: surface vertices with NEE (Sec. 4.2: 3) */
    int32_t  ris_m;          /* M >= 1 RIS candidates per vertex (Eq. restir's m) */
    int32_t  ris_m_brdf;     /* M_b in [0, M]: BRDF candidates; the other M - M_b sample the env */
    int32_t  rr_start;       /* -1: no Russian roulette; else roulette after vertex k >= rr_start */
    uint64_t seed;           /* Philox key */
    int32_t  brdf;           /* MRS_BRDF_* */
    int32_t  background;     /* MRS_BG_*: radiance of camera rays that miss */
    int32_t  grad_mode;      /* MRS_GRAD_*: FULL (all vertices) or PRIMARY (Sec. 4.2 detach) */
    int32_t  tape_mode;      /* MRS_TAPE_*: keep per-vertex records for the adjoint or recompute */
    int64_t  tape_budget;    /* bytes the tape may use in AUTO mode; 0 = half of free device memory */
    int32_t  pool;           /* paths in flight; 0 = library default (2^27, a whole output chunk) */
    int32_t  block;          /* threads per block of the trace/shade kernels: 0 = default (64),
                                else a multiple of 64 in [64, 256] */
    float   *debug_sample_rgb;   /* nullable device [S][3]: per-sample radiance, S = sum W*H*spp */
    uint32_t*debug_hash;         /* nullable device [S]: per-sample decision hash */
    /* Reservoir reuse at primary vertices (Sec. 4.1 end; Appendix A
     * "Spatial-temporal reuse"), on when reuse_spatial > 0 or
     * reuse_temporal = 1.  Per call (one frame): each sample's initial RIS
     * reservoir at its primary vertex is merged with the previous frame's
     * final reservoir of the same sample (temporal; its confidence capped at
     * reuse_m_cap * ris_m), then with the temporally merged reservoirs of
     * reuse_spatial neighbours (same view and sample index, offsets uniform
     * in a (2 reuse_radius + 1)^2 pixel window without the centre).  Merging
     * weights input i at the merging vertex q by p_hat_q(y_i) W_i M_i and
     * gives W = sum w / (sum M p_hat_q(y)).  The primary vertex is shaded
     * with the merged sample; gradients hold it and its weight fixed.
     * Reservoir records are 8 floats per sample (y.x, y.y, y.z, W, M, 0, 0,
     * 0), indexed like debug_sample_rgb.  mrs_render_backward without a tape
     * recomputes the frame's reservoirs, so reservoir_prev must hold the same
     * records then; reservoir_out is written by mrs_render only. */
    int32_t  reuse_spatial;      /* neighbours merged, in [0, 16] */
    int32_t  reuse_radius;       /* window half-size in pixels, in [1, 64] */
    int32_t  reuse_temporal;     /* 1: merge reservoir_prev first */
    int32_t  reuse_m_cap;        /* temporal confidence cap in multiples of ris_m, >= 1 */
    const float *reservoir_prev; /* nullable device [S][8]: the previous frame's final reservoirs */
    float   *reservoir_out;      /* nullable device [S][8]: this frame's final reservoirs (must not alias prev) */
    /* 1: mrs_render_backward sums every gradient word in a fixed order, so
     * its output is bitwise reproducible for the same inputs, whatever the
     * order in which the device runs the work.  Each sample writes its
     * (word, value) pairs to slots of its own, a stable radix sort groups
     * them by word, and one thread adds each word's run in sample order
     * (library-owned: 368 B per bounce per sample of a 2^20-sample launch,
     * pairs and sorted copy, plus the sort's scratch).
     * For tests and debugging: several times slower than the default (0),
     * whose float atomics land in any order.  Texture and vertex materials
     * only: MRS_EINVAL with MRS_MAT_FIELD. */
    int32_t  deterministic;
} mrs_options;

/* Gradient outputs (device, ACCUMULATED with +=; the caller zeroes them).
 * Any pointer may be NULL to skip that group.  Shapes follow mrs_scene. */
typedef struct {
    float *vmat;     /* [nv][5] */
    float *albedo;   /* [th][tw][3] */
    float *rough;    /* [th][tw] */
    float *metal;    /* [th][tw] */
    float *env;      /* [eh][ew][3] */
    mrs_field_grads field;   /* MRS_MAT_FIELD: the field's parameters */
} mrs_grads;

/* Builds a linear BVH (Karras, HPG 2012; the paper's LBVH, Appendix A) over
 * the triangles.  d_pos [nv][3] and d_faces [nf][3] are device arrays; the
 * BVH keeps its own copy of the triangles in leaf order, so the inputs may be
 * freed afterwards.  Degenerate triangles are kept and never hit.  Rays
 * traverse a collapse of the binary tree into nodes of up to four children
 * chosen to minimise the summed surface area of the nodes.  Waits for
 * `stream` before returning.  Errors: MRS_EINVAL (null, nv/nf <= 0, a face
 * index outside [0, nv)), MRS_EOVERFLOW (nf > 2^27, or a tree so deep that a
 * traversal could overflow its stack of 160 entries), MRS_ENOMEM, MRS_EHIP. */
mrs_status mrs_build_bvh(const float *d_pos, int32_t nv, const int32_t *d_faces, int32_t nf,
                         void *stream, mrs_bvh **out);

/* Hierarchies mrs_build_bvh_with can build over the same Morton order. */
enum {
    MRS_BVH_LBVH = 0,   /* Karras radix tree: what mrs_build_bvh builds */
    MRS_BVH_PLOC = 1    /* Meister and Bittner, "Parallel Locally-Ordered Clustering for Bounding
                           Volume Hierarchy Construction" (TVCG 2018): rounds that merge mutual
                           nearest neighbours within 32 sorted positions by the surface area of
                           their union box, then one bottom-up sweep of treelet restructuring
                           (Karras and Aila, HPG 2013: the best binary topology over up to 7
                           subtrees by the surface area heuristic).  Fewer node visits per ray,
                           longer build. */
};

/* As mrs_build_bvh, with the hierarchy chosen by `builder` (an MRS_BVH_*
 * value).  Both give the same leaf size bound, node layout and hit results
 * (closest hit with ties to the lower face id); only the tree differs.
 * Errors: as mrs_build_bvh, plus MRS_EINVAL for an unknown builder. */
mrs_status mrs_build_bvh_with(const float *d_pos, int32_t nv, const int32_t *d_faces, int32_t nf,
                              int32_t builder, void *stream, mrs_bvh **out);
void       mrs_bvh_destroy(mrs_bvh *bvh);

/* Refits the BVH to new positions of the same vertices (faces unchanged):
 * the triangle records and every node box are recomputed bottom-up over the
 * unchanged tree, one launch per node height (the order is fixed at build).
 * This is the per-iteration update of the acceleration
 * structure while vertices move (the paper rebuilds its LBVH every
 * iteration, Appendix A "Visibility estimation").  Hit results stay exact for
 * any motion; only the tree quality degrades with large motion, when a
 * rebuild pays again.  d_pos [nv][3] is a device array.  Enqueued on `stream`
 * without waiting.  Errors: MRS_EINVAL (null, nv differs from the build). */
mrs_status mrs_bvh_refit(mrs_bvh *bvh, const float *d_pos, int32_t nv, void *stream);

/* BVH statistics (host): number of triangles, nodes, tree depth. */
mrs_status mrs_bvh_info(const mrs_bvh *bvh, int32_t *nf, int32_t *nodes, int32_t *depth);

/* Ray-mesh intersection for a batch of n rays (Eq. intersect; Appendix A
 * visibility test).  d_orig, d_dir: device float [n][3].  Closest hit
 * (any_hit = 0): d_hit [n][4] = (t, b1, b2, face id as int32 bits) with the
 * smallest t > 0, ties to the lower face id, face id -1 on a miss; b1, b2 are
 * the barycentric weights of the face's 2nd and 3rd vertex.  Any hit
 * (any_hit = 1): only the face id slot is meaningful (-1 none, >= 0 some
 * hit).  Errors: MRS_EINVAL (null pointers, n < 0), MRS_EHIP. */
mrs_status mrs_trace(const mrs_bvh *bvh, const float *d_orig, const float *d_dir, int64_t n, int32_t any_hit,
                     float *d_hit, void *stream);

/* Renders n_views views (Eq. pbr_render estimated per sample with RIS direct
 * light and BRDF-sampled indirect light) into d_image [sum W*H][3] (float32,
 * overwritten at each view's pixel_offset; other pixels untouched).  Each
 * pixel is the mean over its spp samples.  If tape_out is non-NULL and the
 * tape policy keeps a tape, *tape_out receives the per-vertex records for
 * mrs_render_backward (else *tape_out = NULL).  Errors: MRS_EINVAL (bad
 * sizes, options, or a BVH built for another triangle count), MRS_EOVERFLOW
 * (more than 2^32 - 1 samples, parameter arrays beyond their limits, an env
 * of 2^27 texels or more or wider than 65536 texels), MRS_ENOMEM, MRS_EHIP. */
mrs_status mrs_render(const mrs_scene *scene, const mrs_view *views, int32_t n_views,
                      const mrs_options *opt, float *d_image, mrs_tape **tape_out, void *stream);

/* Adjoint path replay: accumulates the gradient of sum_pixels
 * d_grad_image . image with respect to the materials and env texels into
 * `grads`.  Uses `tape` (from mrs_render with identical arguments) when
 * non-NULL, else re-renders chunk by chunk into a bounded tape
 * (recompute).  Errors: MRS_EINVAL (including a tape recorded for different
 * views, samples, bounces or seed), MRS_ENOMEM, MRS_EHIP. */
mrs_status mrs_render_backward(const mrs_scene *scene, const mrs_view *views, int32_t n_views,
                               const mrs_options *opt, const float *d_grad_image,
                               const mrs_grads *grads, const mrs_tape *tape, void *stream);

/* The material field alone at n points: d_x [n][3] positions, d_m [n][4]
 * outputs (albedo rgb, roughness), device float32.  Errors: MRS_EINVAL
 * (null, n < 0, field parameters out of range), MRS_EHIP. */
mrs_status mrs_field_eval(const mrs_field *field, const float *d_x, int64_t n, float *d_m, void *stream);

/* Pull-back of d_grad_m [n][4] = dL/dm at the points d_x [n][3] onto the
 * field's parameters, accumulated (+=) into `grads` (null members skipped).
 * Points whose four gradient values are all zero are skipped.  Errors: as
 * mrs_field_eval. */
mrs_status mrs_field_backward(const mrs_field *field, const float *d_x, const float *d_grad_m, int64_t n,
                              const mrs_field_grads *grads, void *stream);

/* Denoiser G-buffer (Appendix A "Denoiser": its normal and position
 * buffers): for the ray through every pixel centre, the closest hit's
 * position o + t d and unit geometric normal turned towards the camera;
 * zeros where the ray misses.  d_position, d_normal [sum W*H][3] device,
 * packed like the image.  Errors: as mrs_render. */
mrs_status mrs_gbuffer(const mrs_scene *scene, const mrs_view *views, int32_t n_views, float *d_position,
                       float *d_normal, void *stream);

#define MRS_DENOISE_MAX_LEVELS 3

/* Edge-avoiding a-trous wavelet transform (Appendix A "Denoiser", after
 * Dammertz et al., HPG 2010).  Level i (0-based) filters c_i into c_{i+1}
 * with 5 x 5 B3-spline taps h = (1, 4, 6, 4, 1)/16 spaced 2^i pixels apart,
 * weighted by w_rt w_n w_x = exp(-|dc_i|^2/sigma_rt^2 - |dn|^2/sigma_n^2 -
 * |dx|^2/sigma_x^2) and normalised by the weight sum; taps outside the view
 * are left out.  The paper runs three levels. */
typedef struct {
    int32_t levels;                      /* in [1, MRS_DENOISE_MAX_LEVELS] */
    float   sigma_rt, sigma_n, sigma_x;  /* > 0 */
} mrs_denoise_params;

/* Bytes of the caller-owned device workspace mrs_denoise needs (every
 * level's colour and weight sum, kept for the backward); -1 on bad input. */
int64_t mrs_denoise_work_bytes(const mrs_view *views, int32_t n_views, const mrs_denoise_params *p);

/* Denoises the packed colour image d_color_in [sum W*H][3] (views by their
 * w, h and pixel_offset; other mrs_view fields are ignored) with the
 * G-buffer into d_color_out, and keeps what the backward needs in d_work.
 * Errors: MRS_EINVAL (null, empty view, bad levels or sigmas), MRS_EHIP. */
mrs_status mrs_denoise(const mrs_view *views, int32_t n_views, const mrs_denoise_params *p,
                       const float *d_color_in, const float *d_normal, const float *d_position,
                       float *d_color_out, float *d_work, void *stream);

/* Adjoint of the last mrs_denoise with this d_work: writes (overwrites)
 * d_grad_in = dL/d color_in from d_grad_out = dL/d color_out, through the
 * filters and through the colour weights' dependence on the image.  The
 * G-buffer is not differentiated.  d_grad_in must not alias d_grad_out. */
mrs_status mrs_denoise_backward(const mrs_view *views, int32_t n_views, const mrs_denoise_params *p,
                                const float *d_normal, const float *d_position, const float *d_work,
                                const float *d_grad_out, float *d_grad_in, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * mrs_denoise forward without a caller workspace.  It computes the same
 * image as mrs_denoise with the same arguments, allocates nothing and keeps
 * no state for mrs_denoise_backward.
 *   Scratch   The intermediate levels of one view live in a static device
 *             array of MRS_DENOISE_SCRATCH_BYTES that each GPU the library
 *             runs on holds until the process ends.  Views are filtered one
 *             after another through it: a view needs 12 bytes per pixel for
 *             two levels and 24 for three (none for one level), so a view of
 *             up to 2,796,202 pixels fits at three levels.  Nothing in it needs
 *             to start at zero.  Every call on a GPU shares that GPU's array:
 *             calls that overlap on one GPU (other streams or threads) race and
 *             must be serialised by the caller.
 *   Buffers   As mrs_denoise; d_color_out must not overlap d_color_in.
 * Errors: as mrs_denoise, plus MRS_EOVERFLOW (a view beyond the scratch
 * limit, checked before any GPU work) and MRS_EHIP. */
#define MRS_DENOISE_SCRATCH_BYTES (64ll << 20)
mrs_status mrs_denoise_noalloc(const mrs_view *views, int32_t n_views, const mrs_denoise_params *p,
                               const float *d_color_in, const float *d_normal, const float *d_position,
                               float *d_color_out, void *stream);

/* Plans: a render (and optionally its adjoint) for fixed views, options and
 * bound device arrays, with every buffer the passes need allocated by the
 * plan at creation (pool, output, env tables, tape or recompute chunk tape).
 * Many views of uneven size and spp share one persistent wavefront pool that
 * is refilled from a global sample counter.  With use_graph the launch
 * sequence of each pass is captured once into a hipGraph (on a stream the
 * plan owns) and every later call replays it on `stream`.
 *   - The arrays bound at creation (scene arrays, d_image, d_grad_image,
 *     grads, debug outputs in opt) must stay allocated at the same addresses
 *     while the plan lives; their CONTENTS may change between calls (an
 *     optimiser updating textures and env in place is the intended use).
 *   - mrs_plan_backward accumulates into grads (the caller zeroes them) using
 *     the tape of the latest mrs_plan_forward when the plan keeps one
 *     (tape_mode / tape_budget as for mrs_render), else re-renders.
 *   - Calls on one plan must not overlap: issue them on one stream or
 *     synchronise in between.  Plans never share buffers with each other or
 *     with the eager calls.
 * Errors: MRS_EINVAL (as mrs_render; grads and d_grad_image must be both set
 * or both NULL; backward on a plan without grads), MRS_ENOMEM, MRS_EHIP. */
typedef struct mrs_plan mrs_plan;   /* opaque, library-owned */
mrs_status mrs_plan_create(const mrs_scene *scene, const mrs_view *views, int32_t n_views, const mrs_options *opt,
                           float *d_image, const float *d_grad_image, const mrs_grads *grads, int32_t use_graph,
                           mrs_plan **out);
mrs_status mrs_plan_forward(mrs_plan *plan, void *stream);
mrs_status mrs_plan_backward(mrs_plan *plan, void *stream);
/* samples per pass, whether the plan keeps a tape, whether it replays graphs */
mrs_status mrs_plan_info(const mrs_plan *plan, int64_t *samples, int32_t *keeps_tape, int32_t *graph);
/* waits for the device, then frees the plan and its buffers */
void       mrs_plan_destroy(mrs_plan *plan);

/* Bytes a tape for these views/options would take (host arithmetic): 36 per
 * path vertex; a tape recorded with field materials (MRS_MAT_FIELD) also keeps
 * the field's output at each vertex, 16 bytes more. */
int64_t    mrs_tape_bytes(const mrs_view *views, int32_t n_views, const mrs_options *opt);
/* Releases a tape.  Its device buffers are kept by the library as a spare for
 * the next tape on the same device (an optimisation loop renders with a tape
 * every step) until a larger tape replaces them or mrs_release_workspace
 * frees them.  NULL is ignored. */
void       mrs_tape_destroy(mrs_tape *tape);

/* Kernel timing for measurement: between mrs_profile_begin and
 * mrs_profile_end every kernel the library launches is bracketed by a pair
 * of HIP events on the launch's own stream.  mrs_profile_end waits for the
 * recorded events and writes up to `cap` entries (one per kernel class with
 * at least one launch: name, launches, summed device milliseconds) to `out`;
 * *n receives the number written.  Errors: MRS_EINVAL (null out/n),
 * MRS_EHIP. */
typedef struct {
    char    name[32];
    int64_t launches;
    double  ms;
} mrs_kernel_time;
mrs_status mrs_profile_begin(void);
mrs_status mrs_profile_end(mrs_kernel_time *out, int32_t cap, int32_t *n);

/* Stable radix sort of n (32-bit key, 32-bit value) pairs by key, ascending,
 * equal keys in their input order: the sort the library runs to put the
 * field pull-back's points in Morton order (App. A, material field) and to
 * group the deterministic adjoint's gradient pairs by record.  d_keys_in,
 * d_vals_in: device uint32 [n], read only; d_keys_out, d_vals_out: device
 * uint32 [n], written (they must not be the inputs); d_tmp: caller-owned
 * device scratch of at least mrs_sort_pairs_tmp_bytes(n) bytes (nothing is
 * allocated).  Enqueued on `stream` without waiting.  Errors: MRS_EINVAL
 * (n < 0, a null buffer, an output equal to its input, too little scratch),
 * MRS_EOVERFLOW (n > 2^31 - 1), MRS_EHIP. */
size_t     mrs_sort_pairs_tmp_bytes(int64_t n);
mrs_status mrs_sort_pairs_u32(const uint32_t *d_keys_in, uint32_t *d_keys_out, const uint32_t *d_vals_in,
                              uint32_t *d_vals_out, int64_t n, void *d_tmp, size_t tmp_bytes, void *stream);

/* Frees the library's internal device workspace and the spare tape buffers
 * (they regrow on demand). */
void        mrs_release_workspace(void);
const char *mrs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
