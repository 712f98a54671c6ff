/*
 * FP64 CPU oracle for the differentiable multi-bounce path tracer with
 * reservoir-resampled direct lighting (MIRReS, arXiv 2406.16360).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct reference the GPU path is judged against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU product path never links, calls or falls back to it.  It shares no
 * source with the HIP library.
 *
 * What it computes (paper references by section / equation):
 *   - the rendering equation (Sec. 3 "Stage 2", Eq. pbr_render) with the
 *     incident light split into visible environment light plus indirect
 *     light (Eq. incident), truncated after B surface vertices
 *     ("first three bounces", Sec. 4.2, Eq. sec_bouce);
 *   - direct light by resampled importance sampling with a streaming
 *     weighted reservoir (Sec. 4.1, Eq. restir; Appendix A "Spatial-temporal
 *     reuse" for the reservoir update rule), generalised to environment and
 *     BRDF candidates with balance-heuristic weights;
 *   - indirect light by BRDF-sampled continuation (Sec. 4.2, Eqs. pbr_indir
 *     and mc_indir);
 *   - visibility by an explicit ray-mesh intersection (Appendix A
 *     "Visibility estimation");
 *   - materials from per-vertex attributes, textures, or the material
 *     neural field F_m (Sec. 3 "Intrinsic decomposition");
 *   - gradients of the detached-sampling path functional with respect to
 *     material texels and environment texels, by forward-mode dual numbers,
 *     and with respect to the field parameters through the field's
 *     pull-back.
 *
 * Parity status per function is stated in the header comment of oracle.c.
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Material neural field F_m (Sec. 3 "Intrinsic decomposition": m = F_m(x),
 * an MLP over a multi-resolution hash grid; Appendix A "Network details":
 * 16 levels, 2 features per entry, resolutions 16 to 2048, 2-layer MLP with
 * 32 hidden units).  Encoding after Mueller et al., "Instant Neural Graphics
 * Primitives with a Multiresolution Hash Encoding" (SIGGRAPH 2022), Sec. 3:
 *   level l in [0, L): N_l = floor(N_min * exp(l * ln(N_max / N_min) / (L - 1))
 *                      + 1e-6)  (N_0 = N_min when L = 1);
 *   u = clamp((x - lo) / (hi - lo), 0, 1) per axis; s = u N_l;
 *   cell c = min(floor(s), N_l - 1), fraction t = s - c;
 *   grid vertex v in [0, N_l]^3 -> slot v0 + (N_l+1)(v1 + (N_l+1) v2) when
 *   (N_l + 1)^3 <= T, else (v0 * 1 ^ v1 * 2654435761 ^ v2 * 805459861)
 *   mod 2^32 mod T (T = 2^log2_table);
 *   features e[2l + j] = trilinear interpolation of table[l][slot][j];
 *   z1 = W1 e + b1 (32), a = max(z1, 0), z2 = W2 a + b2 (4),
 *   m = sigmoid(z2) = (albedo r, g, b, roughness); metallic is 0.
 * table [L][T][2], w1 [32][2L], b1 [32], w2 [4][32], b2 [4]. */
#define ORC_FIELD_MAXL 16
#define ORC_FIELD_HIDDEN 32
#define ORC_FIELD_OUT 4
typedef struct {
    int32_t levels, log2_table, n_min, n_max;
    float   lo[3], hi[3];
    const float *table, *w1, *b1, *w2, *b2;
} orc_field;

/* Scene.  All arrays are host memory owned by the caller and must outlive
 * the context built from them.  faces are int32 triples into pos.
 * mat_mode 0: vmat[nv][5] = (albedo rgb, roughness, metallic) per vertex.
 * mat_mode 1: uv[nv][2] plus textures albedo[th][tw][3], rough[th][tw],
 *             metal[th][tw].
 * mat_mode 2: the material field `field` evaluated at the hit point.
 * env[eh][ew][3] is linear HDR radiance, row 0 = +y pole. */
typedef struct {
    const float   *pos;   int32_t nv;
    const int32_t *faces; int32_t nf;
    const float   *uv;
    int32_t        mat_mode;
    const float   *vmat;
    const float   *albedo, *rough, *metal; int32_t tw, th;
    const float   *env;  int32_t ew, eh;
    const orc_field *field;
} orc_scene;

/* Pinhole view.  c2w is row-major 4x4 camera-to-world; the camera looks
 * down -z with +y up.  Sample s of pixel p uses Philox counter
 * word 1 = sample_offset + s. */
typedef struct {
    float    c2w[16];
    float    fov_y_deg;
    int32_t  w, h, spp;
    uint32_t sample_offset;
} orc_view;

/* Reservoir reuse at primary vertices (Sec. 4.1 end; App. A "Spatial-
 * temporal reuse"; the readings are listed in oracle.c).  prev / out hold
 * one 8-float record per sample, (y.x, y.y, y.z, W, M, 0, 0, 0): prev is
 * indexed by the global sample index (views in order, pixel-major, spp
 * minor), out by item. */
#define ORC_REUSE_MAXK 16
typedef struct {
    int32_t spatial;       /* neighbours merged, in [0, ORC_REUSE_MAXK] */
    int32_t radius;        /* window half-size R in pixels, in [1, 64] */
    int32_t temporal;      /* 1: merge prev of the same sample first */
    int32_t m_cap;         /* temporal confidence cap, in multiples of ris_m (>= 1) */
    const float *prev;     /* nullable [S][8] */
    double  *out;          /* nullable [n][8] */
} orc_reuse;

typedef struct {
    int32_t  bounces;      /* B >= 1 surface vertices with next-event estimation */
    int32_t  ris_m;        /* M >= 1 candidates per vertex */
    int32_t  ris_m_brdf;   /* M_b in [0, M]; the first M - M_b are env samples */
    int32_t  rr_start;     /* -1: no Russian roulette; else applied when k >= rr_start */
    uint64_t seed;
    int32_t  brdf;         /* 0: Lambert only, 1: Lambert + GGX */
    int32_t  background;   /* 0: env radiance on primary miss, 1: black */
    int32_t  grad_mode;    /* 0: full path, 1: primary vertex only */
    const orc_reuse *reuse; /* nullable: no reuse */
    /* Test hook for conditioning studies: every unit vector the path derives
     * (camera ray, geometric normal, candidate and continuation directions)
     * moves by up to `jitter` units of 2^-24 per component, from a Philox
     * stream keyed by jitter_seed, and is renormalised.  0: no change. */
    double   jitter;
    uint64_t jitter_seed;
} orc_options;

enum { ORC_C_CLOSEST_RAYS = 0, ORC_C_CLOSEST_NODES, ORC_C_CLOSEST_TRIS,
       ORC_C_SHADOW_RAYS, ORC_C_SHADOW_NODES, ORC_C_SHADOW_TRIS,
       ORC_C_HITS, ORC_C_NEE_VISIBLE, ORC_C_CANDIDATES, ORC_C_PRIMARY_MISS,
       ORC_NCOUNT };

typedef struct orc_ctx orc_ctx;

/* Builds the FP64 environment CDF and (if use_bvh) an FP64 SAH BVH.
 * Returns NULL on invalid input. */
orc_ctx *orc_create(const orc_scene *scene, int32_t use_bvh);
void     orc_destroy(orc_ctx *ctx);

/* Philox4x32-10 block (Salmon et al., SC'11). */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Per-sample radiance.  items[n][3] = (view, pixel y*W+x, sample index in
 * [0, spp)).  rgb[n][3] (required), hash[n] (nullable), counters[ORC_NCOUNT]
 * (nullable, accumulated).  Returns 0 or a negative error. */
int32_t orc_render(const orc_ctx *ctx, const orc_view *views, int32_t nviews,
                   const orc_options *opt, const int32_t *items, int64_t n,
                   double *rgb, uint32_t *hash, int64_t *counters, int32_t nthreads);

/* Gradient of sum_i dldc[i] . C_i with respect to the material and env
 * texels, accumulated (+=) into the given buffers (each nullable). */
int32_t orc_grad(const orc_ctx *ctx, const orc_view *views, int32_t nviews,
                 const orc_options *opt, const int32_t *items, int64_t n,
                 const double *dldc, double *g_vmat, double *g_albedo,
                 double *g_rough, double *g_metal, double *g_env, int32_t nthreads);

/* Gradient of sum_i dldc[i] . C_i for a field-material scene (mat_mode 2)
 * with respect to the field's table and MLP parameters (shapes as in
 * orc_field) and the env texels, accumulated (+=; each nullable).  Exact
 * chain rule: the derivative of the path functional with respect to the
 * field's output at each path vertex, pulled back through the field. */
int32_t orc_grad_field(const orc_ctx *ctx, const orc_view *views, int32_t nviews,
                       const orc_options *opt, const int32_t *items, int64_t n,
                       const double *dldc, double *g_table, double *g_w1, double *g_b1,
                       double *g_w2, double *g_b2, double *g_env, int32_t nthreads);

/* The field alone: m[n][4] at points x[n][3]; and the pull-back of
 * g[n][4] = dL/dm onto the parameters (accumulated, each nullable). */
int32_t orc_field_eval(const orc_field *f, const double *x, int64_t n, double *m);
int32_t orc_field_vjp(const orc_field *f, const double *x, const double *g, int64_t n,
                      double *g_table, double *g_w1, double *g_b1, double *g_w2, double *g_b2);
/* level resolutions N_l (test hook); returns L or a negative error */
int32_t orc_field_levels(const orc_field *f, int64_t *res);

/* Frozen-path evaluation: records the path of one item in rec_ctx's scene,
 * then evaluates the detached-sampling functional with the material and env
 * values of eval_ctx (same mesh).  Used for finite differences. */
int32_t orc_frozen(const orc_ctx *rec_ctx, const orc_ctx *eval_ctx,
                   const orc_view *views, int32_t nviews, const orc_options *opt,
                   const int32_t item[3], double rgb[3]);

/* Closest hit (any_hit = 0) or any hit (any_hit = 1) for n rays; brute = 1
 * tests every triangle.  prim = -1 on a miss. */
int32_t orc_trace(const orc_ctx *ctx, const double *o, const double *d, int64_t n,
                  int32_t any_hit, int32_t brute, int32_t *prim, double *t,
                  double *b1, double *b2);

/* Reuse neighbour offset j of a sample (test hook): the Philox block
 * (1, 0xFFE0 + j) mapped by integer arithmetic to [-R, R]^2. */
int32_t orc_reuse_offset(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t view, int32_t j,
                         int32_t radius, int32_t *dx, int32_t *dy);

/* Environment helpers (test hooks). */
int32_t orc_env_sample(const orc_ctx *ctx, double u0, double u1, double dir[3],
                       double *pdf, int32_t *texel);
double  orc_env_pdf(const orc_ctx *ctx, const double dir[3]);
int32_t orc_env_lookup(const orc_ctx *ctx, const double dir[3], double rgb[3]);

/* BRDF helpers (test hooks).  m = (albedo rgb, roughness, metallic), raw
 * (clamped inside).  brdf as in orc_options. */
void    orc_brdf_eval(const double n[3], const double wo[3], const double wi[3],
                      const double m[5], int32_t brdf, double f[3]);
double  orc_brdf_pdf(const double n[3], const double wo[3], const double wi[3],
                     const double m[5], int32_t brdf);
int32_t orc_brdf_sample(const double n[3], const double wo[3], const double m[5],
                        int32_t brdf, const double u[3], double wi[3]);
double  orc_ggx_d(double alpha, double cos_h);
double  orc_ggx_g1(double alpha, double cos_w);
void    orc_frame(const double n[3], double t[3], double b[3]);

#ifdef __cplusplus
}
#endif
#endif
