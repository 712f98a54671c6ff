/*
 * FP64 CPU oracle — TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written from the paper (MIRReS, arXiv 2406.16360) and the readings of its
 * silent or ambiguous points that the design document lists.  Each function
 * names the passage it follows.  Everything is double precision; inputs are
 * the float arrays the GPU path also reads, widened exactly.
 *
 * Pins (tests/test_oracle_*.py), so that no function here is trusted only
 * against itself:
 *   philox          - rocRAND's Philox4x32-10 engine (compiled from its public
 *                     header at test time) and the published known-answer
 *                     vectors of the Random123 distribution.
 *   env CDF/sampler - pdf integrates to 1 over the sphere; chi-square of the
 *                     sampler against the pdf; sampled texel equals the
 *                     texel looked up from the sampled direction.
 *   BRDF            - GGX normalisation of D(h)(n.h); Lambert albedo
 *                     integral; reciprocity; sampler chi-square against the
 *                     mixture pdf; f cos / pdf_vndf = F G1(wi) identity.
 *   intersection    - BVH closest/any hit equal brute force (plain
 *                     definition, unique with the lower-prim tie rule).
 *   estimator       - white furnace (exact per sample with BRDF-only
 *                     candidates), unoccluded plane (pixel = albedo * L),
 *                     unbiasedness against brute-force BRDF-sampled path
 *                     tracing on a tiny scene.
 *   gradient        - central finite differences of the frozen functional;
 *                     closed form dI/da = L on the plane.
 *   material field  - level resolutions of the paper's configuration (16 to
 *                     2048 in 16 geometric steps); dense levels reproduce
 *                     tables affine in the vertex coordinates; hashed levels
 *                     are a partition of unity, continuous across cell faces,
 *                     and read slot v0 mod T along the x axis; MLP closed
 *                     forms (W2 = 0, W1 = 0); pull-back against central
 *                     differences; a constant field renders like constant
 *                     per-vertex materials, with the output-bias gradient
 *                     equal to sigmoid' times the summed vertex gradient;
 *                     path gradients against differences of the frozen
 *                     functional.  The hash primes are the published ones
 *                     (Mueller et al. 2022) and are pinned only on the x axis.
 *   reservoir reuse - neighbour offsets uniform over the window (chi-square);
 *                     on an unoccluded Lambertian plane under a constant
 *                     environment with cosine-sampled candidates every merge
 *                     (spatial, temporal) still gives exactly albedo x L per
 *                     sample; with env candidates too the merged estimator's
 *                     mean over seeds is albedo x L; with no neighbour and no
 *                     history it reduces to plain RIS; texture and env
 *                     gradients with reuse against central differences of
 *                     the frozen functional.
 * Parity with numbers printed in the paper is unpinned: the paper prints no
 * per-pixel or per-gradient values for this path.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846
#define ORC_MAXB 16
#define R_MIN 0.05
#define F0_DIELECTRIC 0.04

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
static void cross3(const double a[3], const double b[3], double r[3]) {
    double x = a[1]*b[2] - a[2]*b[1], y = a[2]*b[0] - a[0]*b[2], z = a[0]*b[1] - a[1]*b[0];
    r[0] = x; r[1] = y; r[2] = z;
}
static void sub3(const double a[3], const double b[3], double r[3]) { r[0] = a[0]-b[0]; r[1] = a[1]-b[1]; r[2] = a[2]-b[2]; }
static void normalize3(double a[3]) { double l = sqrt(dot3(a, a)); a[0] /= l; a[1] /= l; a[2] /= l; }
/* clamp to [lo, hi]; NaN (no order) goes to lo: a material value that is
 * not a number takes the lower end of its range */
static double clampd(double x, double lo, double hi) { return !(x >= lo) ? lo : (x > hi ? hi : x); }

/* ------------------------------------------------------------------ */
/* dual numbers (value, derivative) for forward-mode differentiation   */
/* ------------------------------------------------------------------ */
typedef struct { double v, d; } dual;
static dual dc(double v) { dual r = { v, 0.0 }; return r; }
static dual dadd(dual a, dual b) { dual r = { a.v + b.v, a.d + b.d }; return r; }
static dual dsub(dual a, dual b) { dual r = { a.v - b.v, a.d - b.d }; return r; }
static dual dmul(dual a, dual b) { dual r = { a.v * b.v, a.d * b.v + a.v * b.d }; return r; }
static dual ddiv(dual a, dual b) { dual r = { a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v) }; return r; }
static dual dscale(dual a, double s) { dual r = { a.v * s, a.d * s }; return r; }
static dual dsqrt(dual a) { double s = sqrt(a.v); dual r = { s, s > 0 ? a.d / (2.0 * s) : 0.0 }; return r; }
/* clamp with the derivative passed on the closed interval (torch.clamp
 * rule); NaN goes to lo with no derivative, as in clampd */
static dual dclamp(dual a, double lo, double hi) {
    if (!(a.v >= lo)) return dc(lo);
    if (a.v > hi) return dc(hi);
    return a;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:  */
/* as easy as 1, 2, 3", SC'11): 10 rounds of two 32x32->64 multiplies,  */
/* with the key bumped by the Weyl constants between rounds.            */
/* ------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream layout: counter = (pixel, sample, view, (vertex << 16) | block),
 * key = seed.  Each 32-bit word becomes a uniform in [0, 1) from its top 24
 * bits, which is exact in both float and double. */
static void uniforms4(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t view,
                      uint32_t vertex, uint32_t block, double u[4]) {
    uint32_t ctr[4] = { pixel, sample, view, (vertex << 16) | (block & 0xFFFFu) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t r[4];
    orc_philox(ctr, key, r);
    for (int i = 0; i < 4; ++i) u[i] = (double)(r[i] >> 8) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------ */
/* FNV-1a (32-bit) over little-endian words: per-sample decision hash   */
/* ------------------------------------------------------------------ */
static uint32_t fnv_word(uint32_t h, uint32_t w) {
    for (int i = 0; i < 4; ++i) { h ^= (w >> (8 * i)) & 0xFFu; h *= 16777619u; }
    return h;
}
#define FNV_BASIS 2166136261u

/* The decision hash of a sample is the XOR of one hash per event, so the
 * events may be recorded in any order:
 *   miss at vertex k            fnv(k, 0xFFFFFFFF)
 *   surface vertex k            fnv(k, face id, selected candidate or ~0, continuation code)
 *                               code 0: last vertex, 1: continued, 2: no valid
 *                               continuation sample, 3: killed by roulette
 *   shadow ray of vertex k      fnv(k | 0x10000, 1 if unoccluded else 0) */
static uint32_t ev_miss(uint32_t k) { return fnv_word(fnv_word(FNV_BASIS, k), 0xFFFFFFFFu); }
static uint32_t ev_vertex(uint32_t k, uint32_t prim, uint32_t sel, uint32_t code) {
    return fnv_word(fnv_word(fnv_word(fnv_word(FNV_BASIS, k), prim), sel), code);
}
static uint32_t ev_nee(uint32_t k, uint32_t vis) { return fnv_word(fnv_word(FNV_BASIS, k | 0x10000u), vis); }
/*   BRDF candidate s of vertex k fnv(k | 0x20000, s, lobe, env texel of its direction)
 * (the continuation code distinguishes lobes: 1 diffuse, 4 specular) */
static uint32_t ev_cand(uint32_t k, uint32_t s, uint32_t lobe, uint32_t tex) {
    return fnv_word(fnv_word(fnv_word(fnv_word(FNV_BASIS, k | 0x20000u), s), lobe), tex);
}

/* ------------------------------------------------------------------ */
/* context                                                             */
/* ------------------------------------------------------------------ */
typedef struct { double lo[3], hi[3]; int32_t left, right, first, count; } bnode;

struct orc_ctx {
    orc_scene s;
    double *v;          /* [nf][9] triangle vertices in double */
    uint8_t *degenerate;
    /* environment sampling tables */
    double *ew;         /* [eh][ew] texel weights */
    double *marg;       /* [eh + 1] */
    double *cond;       /* [eh][ew + 1] */
    double total;
    /* BVH */
    bnode *nodes; int32_t nnodes;
    int32_t *order;     /* triangle ids in leaf order */
};

/* --- environment: sampling weights proportional to mean radiance times
 * the solid angle of the texel row (Sec. 4.1: the proposal follows L_env). */
static void env_build(orc_ctx *c) {
    int W = c->s.ew, H = c->s.eh;
    c->ew = (double *)calloc((size_t)W * H, sizeof(double));
    c->marg = (double *)calloc((size_t)H + 1, sizeof(double));
    c->cond = (double *)calloc((size_t)H * (W + 1), sizeof(double));
    double total = 0.0;
    for (int i = 0; i < H; ++i) {
        double st = sin(PI * (i + 0.5) / H);
        double row = 0.0;
        double *cr = c->cond + (size_t)i * (W + 1);
        cr[0] = 0.0;
        for (int j = 0; j < W; ++j) {
            const float *L = c->s.env + ((size_t)i * W + j) * 3;
            double m = 0.0;
            for (int ch = 0; ch < 3; ++ch) m += L[ch] > 0.0f ? (double)L[ch] : 0.0;
            double w = (m / 3.0) * st;
            c->ew[(size_t)i * W + j] = w;
            row += w;
            cr[j + 1] = row;
        }
        if (row > 0.0) for (int j = 1; j <= W; ++j) cr[j] /= row;
        cr[W] = 1.0;
        c->marg[i + 1] = c->marg[i] + row;
        total += row;
    }
    c->total = total;
    if (total > 0.0) for (int i = 1; i <= H; ++i) c->marg[i] /= total;
    c->marg[H] = 1.0;
}

/* smallest i in [0, n) with cdf[i + 1] > u  (cdf[n] == 1 > u) */
static int cdf_find(const double *cdf, int n, double u) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (cdf[mid + 1] > u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static double env_channel(const orc_ctx *c, int32_t texel, int ch) {
    double L = (double)c->s.env[(size_t)texel * 3 + ch];
    return L > 0.0 ? L : 0.0;
}

/* Equirectangular mapping, +y up: theta = acos(d_y), phi = atan2(d_x, -d_z),
 * u = phi / 2pi + 1/2, v = theta / pi; nearest texel. */
static int32_t env_texel_of(const orc_ctx *c, const double d[3]) {
    int W = c->s.ew, H = c->s.eh;
    double dy = clampd(d[1], -1.0, 1.0);
    double theta = acos(dy), phi = atan2(d[0], -d[2]);
    double u = phi / (2.0 * PI) + 0.5, v = theta / PI;
    int col = (int)floor(u * W), row = (int)floor(v * H);
    if (col < 0) col = 0; if (col > W - 1) col = W - 1;
    if (row < 0) row = 0; if (row > H - 1) row = H - 1;
    return row * W + col;
}

/* solid-angle density of the env sampler at direction d */
static double env_pdf_dir(const orc_ctx *c, const double d[3]) {
    if (c->total <= 0.0) return 0.0;
    double st = sqrt(fmax(0.0, 1.0 - d[1] * d[1]));
    if (st <= 0.0) return 0.0;
    int32_t t = env_texel_of(c, d);
    return c->ew[t] / c->total * (double)c->s.ew * (double)c->s.eh / (2.0 * PI * PI * st);
}

/* CDF inversion: row from the marginal, column from the row's conditional,
 * continuous offset inside the texel from the linear remainder.  Returns 0
 * when no valid sample exists. */
static int env_sample(const orc_ctx *c, double u0, double u1, double dir[3], double *pdf, int32_t *texel) {
    int W = c->s.ew, H = c->s.eh;
    if (c->total <= 0.0) return 0;
    int i = cdf_find(c->marg, H, u0);
    double fv = (u0 - c->marg[i]) / (c->marg[i + 1] - c->marg[i]);
    const double *cr = c->cond + (size_t)i * (W + 1);
    int j = cdf_find(cr, W, u1);
    double fu = (u1 - cr[j]) / (cr[j + 1] - cr[j]);
    double v = (i + fv) / H, u = (j + fu) / W;
    double theta = PI * v, phi = 2.0 * PI * (u - 0.5);
    double st = sin(theta);
    if (st <= 0.0) return 0;
    dir[0] = st * sin(phi); dir[1] = cos(theta); dir[2] = -st * cos(phi);
    *texel = i * W + j;
    *pdf = c->ew[(size_t)i * W + j] / c->total * (double)W * (double)H / (2.0 * PI * PI * st);
    return *pdf > 0.0;
}

/* ------------------------------------------------------------------ */
/* BVH (FP64, binned SAH, <= 4 triangles per leaf).  Only an accelerator: */
/* the closest hit it returns is the plain minimum over all triangles.    */
/* ------------------------------------------------------------------ */
typedef struct { double lo[3], hi[3]; } box3;
static void box_empty(box3 *b) { for (int a = 0; a < 3; ++a) { b->lo[a] = INFINITY; b->hi[a] = -INFINITY; } }
static void box_grow_pt(box3 *b, const double p[3]) { for (int a = 0; a < 3; ++a) { if (p[a] < b->lo[a]) b->lo[a] = p[a]; if (p[a] > b->hi[a]) b->hi[a] = p[a]; } }
static void box_grow(box3 *b, const box3 *o) { for (int a = 0; a < 3; ++a) { if (o->lo[a] < b->lo[a]) b->lo[a] = o->lo[a]; if (o->hi[a] > b->hi[a]) b->hi[a] = o->hi[a]; } }
static double box_area(const box3 *b) {
    double e0 = b->hi[0] - b->lo[0], e1 = b->hi[1] - b->lo[1], e2 = b->hi[2] - b->lo[2];
    if (e0 < 0 || e1 < 0 || e2 < 0) return 0.0;
    return 2.0 * (e0 * e1 + e1 * e2 + e2 * e0);
}

typedef struct { box3 *tb; double *cen; int32_t *ids; bnode *nodes; int32_t nn, cap; } bvh_build;

static int32_t bvh_rec(bvh_build *B, int32_t first, int32_t count) {
    if (B->nn == B->cap) { B->cap *= 2; B->nodes = (bnode *)realloc(B->nodes, sizeof(bnode) * B->cap); }
    int32_t me = B->nn++;
    box3 bb, cb; box_empty(&bb); box_empty(&cb);
    for (int32_t i = first; i < first + count; ++i) {
        box_grow(&bb, &B->tb[B->ids[i]]);
        box_grow_pt(&cb, &B->cen[3 * (size_t)B->ids[i]]);
    }
    /* pad so the FP64 slab test can never reject a triangle it contains */
    for (int a = 0; a < 3; ++a) {
        double pad = 1e-9 * (fabs(bb.lo[a]) + fabs(bb.hi[a]) + 1.0);
        B->nodes[me].lo[a] = bb.lo[a] - pad; B->nodes[me].hi[a] = bb.hi[a] + pad;
    }
    B->nodes[me].left = B->nodes[me].right = -1;
    B->nodes[me].first = first; B->nodes[me].count = count;
    if (count <= 4) return me;
    enum { NB = 16 };
    double best = INFINITY; int best_axis = -1, best_split = -1;
    for (int a = 0; a < 3; ++a) {
        double ext = cb.hi[a] - cb.lo[a];
        if (!(ext > 0.0)) continue;
        box3 bins[NB]; int cnt[NB];
        for (int k = 0; k < NB; ++k) { box_empty(&bins[k]); cnt[k] = 0; }
        for (int32_t i = first; i < first + count; ++i) {
            int k = (int)((B->cen[3 * (size_t)B->ids[i] + a] - cb.lo[a]) / ext * NB);
            if (k >= NB) k = NB - 1; if (k < 0) k = 0;
            cnt[k]++; box_grow(&bins[k], &B->tb[B->ids[i]]);
        }
        for (int s = 1; s < NB; ++s) {
            box3 l, r; box_empty(&l); box_empty(&r); int nl = 0, nr = 0;
            for (int k = 0; k < s; ++k) { box_grow(&l, &bins[k]); nl += cnt[k]; }
            for (int k = s; k < NB; ++k) { box_grow(&r, &bins[k]); nr += cnt[k]; }
            if (nl == 0 || nr == 0) continue;
            double cost = box_area(&l) * nl + box_area(&r) * nr;
            if (cost < best) { best = cost; best_axis = a; best_split = s; }
        }
    }
    int32_t mid;
    if (best_axis >= 0) {
        double ext = cb.hi[best_axis] - cb.lo[best_axis];
        int32_t i = first, j = first + count - 1;
        while (i <= j) {
            int k = (int)((B->cen[3 * (size_t)B->ids[i] + best_axis] - cb.lo[best_axis]) / ext * NB);
            if (k >= NB) k = NB - 1; if (k < 0) k = 0;
            if (k < best_split) ++i; else { int32_t t = B->ids[i]; B->ids[i] = B->ids[j]; B->ids[j] = t; --j; }
        }
        mid = i;
        if (mid == first || mid == first + count) mid = first + count / 2;
    } else {
        mid = first + count / 2;   /* coincident centroids: split the index range */
    }
    int32_t l = bvh_rec(B, first, mid - first);
    int32_t r = bvh_rec(B, mid, first + count - mid);
    B->nodes[me].left = l; B->nodes[me].right = r; B->nodes[me].count = 0;
    return me;
}

static void bvh_build_all(orc_ctx *c) {
    int32_t nf = c->s.nf;
    bvh_build B;
    B.tb = (box3 *)malloc(sizeof(box3) * (size_t)nf);
    B.cen = (double *)malloc(sizeof(double) * 3 * (size_t)nf);
    B.ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)nf);
    B.cap = 2 * nf + 1; B.nn = 0;
    B.nodes = (bnode *)malloc(sizeof(bnode) * B.cap);
    for (int32_t f = 0; f < nf; ++f) {
        box_empty(&B.tb[f]);
        for (int k = 0; k < 3; ++k) box_grow_pt(&B.tb[f], c->v + 9 * (size_t)f + 3 * k);
        for (int a = 0; a < 3; ++a) B.cen[3 * (size_t)f + a] = 0.5 * (B.tb[f].lo[a] + B.tb[f].hi[a]);
        B.ids[f] = f;
    }
    if (nf > 0) bvh_rec(&B, 0, nf);
    c->nodes = B.nodes; c->nnodes = B.nn; c->order = B.ids;
    free(B.tb); free(B.cen);
}

/* Moller-Trumbore in FP64; edges inclusive, strictly t > 0, degenerate
 * triangles never hit. */
static int tri_hit(const orc_ctx *c, int32_t f, const double o[3], const double d[3],
                   double *t, double *b1, double *b2) {
    if (c->degenerate[f]) return 0;
    const double *v0 = c->v + 9 * (size_t)f, *v1 = v0 + 3, *v2 = v0 + 6;
    double e1[3], e2[3], pv[3], s[3], qv[3];
    sub3(v1, v0, e1); sub3(v2, v0, e2);
    cross3(d, e2, pv);
    double det = dot3(e1, pv);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    sub3(o, v0, s);
    double u = dot3(s, pv) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    cross3(s, e1, qv);
    double v = dot3(d, qv) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    double tt = dot3(e2, qv) * inv;
    if (!(tt > 0.0)) return 0;
    *t = tt; *b1 = u; *b2 = v;
    return 1;
}

/* slab test of a node box against [0, tmax]; *tnear = entry distance */
static int box_hit(const bnode *nd, const double o[3], const double d[3], double tmax, double *tnear) {
    double t0 = 0.0, t1 = tmax;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            double inv = 1.0 / d[a];
            double ta = (nd->lo[a] - o[a]) * inv, tb = (nd->hi[a] - o[a]) * inv;
            if (ta > tb) { double x = ta; ta = tb; tb = x; }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
            if (t0 > t1) return 0;
        } else if (o[a] < nd->lo[a] || o[a] > nd->hi[a]) {
            return 0;
        }
    }
    *tnear = t0;
    return 1;
}

typedef struct { int32_t prim; double t, b1, b2; } hitrec;

static void leaf_closest(const orc_ctx *c, const bnode *nd, const double o[3], const double d[3], hitrec *h,
                         int64_t *tris) {
    double t, b1, b2;
    for (int32_t i = nd->first; i < nd->first + nd->count; ++i) {
        int32_t f = c->order[i];
        if (tris) (*tris)++;
        if (tri_hit(c, f, o, d, &t, &b1, &b2) && (t < h->t || (t == h->t && f < h->prim))) {
            h->prim = f; h->t = t; h->b1 = b1; h->b2 = b2;
        }
    }
}

/* Closest hit: smallest t > 0, ties to the lower primitive id (plain
 * definition of Eq. intersect for a triangle mesh).  The BVH only prunes:
 * visiting an internal node tests both child boxes (counted as two box
 * tests), hit leaves are tested at once, the nearer hit child is visited
 * next and the farther one is stacked with its entry distance and skipped
 * when popped if a closer hit was found meanwhile (boxes touching the current
 * closest distance are still visited, for the tie rule). */
static hitrec trace_closest(const orc_ctx *c, const double o[3], const double d[3], int brute,
                            int64_t *nodes, int64_t *tris) {
    hitrec h = { -1, INFINITY, 0.0, 0.0 };
    double t, b1, b2;
    if (brute || !c->nodes) {
        for (int32_t f = 0; f < c->s.nf; ++f) {
            if (tris) (*tris)++;
            if (tri_hit(c, f, o, d, &t, &b1, &b2) && (t < h.t || (t == h.t && f < h.prim))) {
                h.prim = f; h.t = t; h.b1 = b1; h.b2 = b2;
            }
        }
        return h;
    }
    double t0;
    if (nodes) (*nodes)++;
    if (!box_hit(&c->nodes[0], o, d, h.t, &t0)) return h;
    if (c->nodes[0].left < 0) { leaf_closest(c, &c->nodes[0], o, d, &h, tris); return h; }
    int32_t stack[512]; double stackt[512]; int sp = 0;
    int32_t cur = 0;
    for (;;) {
        const bnode *nd = &c->nodes[cur];
        int32_t ch[2] = { nd->left, nd->right };
        double tn[2] = { 0.0, 0.0 };
        int hit[2];
        for (int k = 0; k < 2; ++k) {
            if (nodes) (*nodes)++;
            hit[k] = box_hit(&c->nodes[ch[k]], o, d, h.t, &tn[k]);
            if (hit[k] && c->nodes[ch[k]].left < 0) { leaf_closest(c, &c->nodes[ch[k]], o, d, &h, tris); hit[k] = 0; }
        }
        if (hit[0] && hit[1]) {
            int nr = tn[0] <= tn[1] ? 0 : 1;
            stack[sp] = ch[1 - nr]; stackt[sp] = tn[1 - nr]; ++sp;
            cur = ch[nr];
            continue;
        }
        if (hit[0] || hit[1]) { cur = hit[0] ? ch[0] : ch[1]; continue; }
        int found = 0;
        while (sp) {
            --sp;
            if (stackt[sp] <= h.t) { cur = stack[sp]; found = 1; break; }
        }
        if (!found) break;
    }
    return h;
}

static int leaf_any(const orc_ctx *c, const bnode *nd, const double o[3], const double d[3], int64_t *tris) {
    double t, b1, b2;
    for (int32_t i = nd->first; i < nd->first + nd->count; ++i) {
        if (tris) (*tris)++;
        if (tri_hit(c, c->order[i], o, d, &t, &b1, &b2)) return 1;
    }
    return 0;
}

/* Visibility (Appendix A): 1 if any triangle is hit at t > 0; same visiting
 * order and counting as the closest-hit traversal, stopping at the first hit. */
static int trace_any(const orc_ctx *c, const double o[3], const double d[3], int brute,
                     int64_t *nodes, int64_t *tris) {
    double t, b1, b2;
    if (brute || !c->nodes) {
        for (int32_t f = 0; f < c->s.nf; ++f) {
            if (tris) (*tris)++;
            if (tri_hit(c, f, o, d, &t, &b1, &b2)) return 1;
        }
        return 0;
    }
    double t0;
    if (nodes) (*nodes)++;
    if (!box_hit(&c->nodes[0], o, d, INFINITY, &t0)) return 0;
    if (c->nodes[0].left < 0) return leaf_any(c, &c->nodes[0], o, d, tris);
    int32_t stack[512]; int sp = 0;
    int32_t cur = 0;
    for (;;) {
        const bnode *nd = &c->nodes[cur];
        int32_t ch[2] = { nd->left, nd->right };
        double tn[2] = { 0.0, 0.0 };
        int hit[2];
        for (int k = 0; k < 2; ++k) {
            if (nodes) (*nodes)++;
            hit[k] = box_hit(&c->nodes[ch[k]], o, d, INFINITY, &tn[k]);
            if (hit[k] && c->nodes[ch[k]].left < 0) {
                if (leaf_any(c, &c->nodes[ch[k]], o, d, tris)) return 1;
                hit[k] = 0;
            }
        }
        if (hit[0] && hit[1]) {
            int nr = tn[0] <= tn[1] ? 0 : 1;
            stack[sp++] = ch[1 - nr];
            cur = ch[nr];
            continue;
        }
        if (hit[0] || hit[1]) { cur = hit[0] ? ch[0] : ch[1]; continue; }
        if (!sp) break;
        cur = stack[--sp];
    }
    return 0;
}

static int field_valid(const orc_field *f);

orc_ctx *orc_create(const orc_scene *s, int32_t use_bvh) {
    if (!s || !s->pos || !s->faces || s->nv <= 0 || s->nf <= 0 || !s->env || s->ew <= 0 || s->eh <= 0) return NULL;
    if (s->mat_mode == 0 && !s->vmat) return NULL;
    if (s->mat_mode == 1 && (!s->uv || !s->albedo || !s->rough || !s->metal || s->tw <= 0 || s->th <= 0)) return NULL;
    if (s->mat_mode == 2 && !field_valid(s->field)) return NULL;
    if (s->mat_mode < 0 || s->mat_mode > 2) return NULL;
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    c->s = *s;
    c->v = (double *)malloc(sizeof(double) * 9 * (size_t)s->nf);
    c->degenerate = (uint8_t *)calloc((size_t)s->nf, 1);
    for (int32_t f = 0; f < s->nf; ++f) {
        for (int k = 0; k < 3; ++k) {
            int32_t vi = s->faces[3 * (size_t)f + k];
            if (vi < 0 || vi >= s->nv) { orc_destroy(c); return NULL; }
            for (int a = 0; a < 3; ++a) c->v[9 * (size_t)f + 3 * k + a] = (double)s->pos[3 * (size_t)vi + a];
        }
        double e1[3], e2[3], cr[3];
        sub3(c->v + 9 * (size_t)f + 3, c->v + 9 * (size_t)f, e1);
        sub3(c->v + 9 * (size_t)f + 6, c->v + 9 * (size_t)f, e2);
        cross3(e1, e2, cr);
        c->degenerate[f] = (cr[0] == 0.0 && cr[1] == 0.0 && cr[2] == 0.0);
    }
    env_build(c);
    if (use_bvh) bvh_build_all(c);
    return c;
}

void orc_destroy(orc_ctx *c) {
    if (!c) return;
    free(c->v); free(c->degenerate); free(c->ew); free(c->marg); free(c->cond);
    free(c->nodes); free(c->order); free(c);
}

/* ------------------------------------------------------------------ */
/* shading frame: the branchless orthonormal basis of Duff et al. (JCGT  */
/* 2017, sign +1 for z >= 0) built for m = R n and mapped back with R,   */
/* where R = (1/9)[[1,4,8],[4,7,-4],[8,-4,1]] is a fixed symmetric       */
/* orthogonal matrix.  Every such basis switches branch on some plane of */
/* normals; with R that plane (8x - 4y + z = 0) contains no axis-aligned  */
/* or symmetric face normal of the synthetic meshes, so float and double */
/* evaluations take the same branch except within rounding of it.       */
/* ------------------------------------------------------------------ */
static const double FRAME_R[3][3] = { { 1.0 / 9, 4.0 / 9, 8.0 / 9 },
                                      { 4.0 / 9, 7.0 / 9, -4.0 / 9 },
                                      { 8.0 / 9, -4.0 / 9, 1.0 / 9 } };
static void rmul(const double v[3], double r[3]) {
    for (int i = 0; i < 3; ++i) r[i] = FRAME_R[i][0] * v[0] + FRAME_R[i][1] * v[1] + FRAME_R[i][2] * v[2];
}
void orc_frame(const double n[3], double t[3], double b[3]) {
    double m[3], tl[3], bl[3];
    rmul(n, m);
    double sg = m[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sg + m[2]);
    double bb = m[0] * m[1] * a;
    tl[0] = 1.0 + sg * m[0] * m[0] * a; tl[1] = sg * bb; tl[2] = -sg * m[0];
    bl[0] = bb; bl[1] = sg + m[1] * m[1] * a; bl[2] = -m[1];
    rmul(tl, t);
    rmul(bl, b);
}

/* ------------------------------------------------------------------ */
/* BRDF: Lambert diffuse plus GGX microfacet specular (Disney-style      */
/* albedo + roughness (+ metallic), Sec. 3 "Intrinsic decomposition").   */
/* ------------------------------------------------------------------ */
double orc_ggx_d(double alpha, double ch) {
    double a2 = alpha * alpha;
    double den = ch * ch * (a2 - 1.0) + 1.0;
    return a2 / (PI * den * den);
}
double orc_ggx_g1(double alpha, double cw) {
    double c2 = cw * cw;
    double tan2 = (1.0 - c2) / c2;
    double lam = (-1.0 + sqrt(1.0 + alpha * alpha * tan2)) * 0.5;
    return 1.0 / (1.0 + lam);
}

static dual g1_d(dual a2, double cw) {
    double c2 = cw * cw;
    double tan2 = (1.0 - c2) / c2;
    dual root = dsqrt(dadd(dc(1.0), dscale(a2, tan2)));
    dual lam = dscale(dsub(root, dc(1.0)), 0.5);
    return ddiv(dc(1.0), dadd(dc(1.0), lam));
}

/* m: clamped material (albedo rgb, roughness, metallic) as duals */
static void brdf_eval_d(const double n[3], const double wo[3], const double wi[3], const dual m[5],
                        int spec, dual f[3]) {
    double ci = dot3(n, wi), co = dot3(n, wo);
    for (int c = 0; c < 3; ++c) f[c] = dc(0.0);
    if (!(ci > 0.0) || !(co > 0.0)) return;
    dual one_m_mu = dsub(dc(1.0), m[4]);
    for (int c = 0; c < 3; ++c) f[c] = dscale(dmul(one_m_mu, m[c]), 1.0 / PI);
    if (!spec) return;
    double h[3] = { wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2] };
    normalize3(h);
    double nh = dot3(n, h), oh = dot3(wo, h);
    dual alpha = dmul(m[3], m[3]);
    dual a2 = dmul(alpha, alpha);
    dual den = dadd(dscale(dsub(a2, dc(1.0)), nh * nh), dc(1.0));
    dual D = ddiv(a2, dscale(dmul(den, den), PI));
    dual G = dmul(g1_d(a2, co), g1_d(a2, ci));
    double fw = pow(1.0 - oh, 5.0);
    dual DG = dscale(dmul(D, G), 1.0 / (4.0 * ci * co));
    for (int c = 0; c < 3; ++c) {
        dual F0 = dadd(dscale(one_m_mu, F0_DIELECTRIC), dmul(m[4], m[c]));
        dual F = dadd(F0, dscale(dsub(dc(1.0), F0), fw));
        f[c] = dadd(f[c], dmul(DG, F));
    }
}

static void clamp_material(const double raw[5], double m[5]) {
    for (int c = 0; c < 3; ++c) m[c] = clampd(raw[c], 0.0, 1.0);
    m[3] = clampd(raw[3], R_MIN, 1.0);
    m[4] = clampd(raw[4], 0.0, 1.0);
}

static void brdf_eval_plain(const double n[3], const double wo[3], const double wi[3], const double m[5],
                            int spec, double f[3]) {
    dual md[5], fd[3];
    for (int i = 0; i < 5; ++i) md[i] = dc(m[i]);
    brdf_eval_d(n, wo, wi, md, spec, fd);
    for (int c = 0; c < 3; ++c) f[c] = fd[c].v;
}

/* probability of choosing the specular lobe in the BRDF mixture sampler */
static double spec_prob(const double m[5], int spec) {
    if (!spec) return 0.0;
    double mu = m[4], f0 = 0.0, dif = 0.0;
    for (int c = 0; c < 3; ++c) { f0 += F0_DIELECTRIC * (1.0 - mu) + mu * m[c]; dif += (1.0 - mu) * m[c]; }
    f0 /= 3.0; dif /= 3.0;
    double den = f0 + dif;
    if (!(den > 0.0)) return 0.5;
    return clampd(f0 / den, 0.1, 0.9);
}

/* mixture density: p_spec * VNDF-reflection pdf + (1 - p_spec) * cosine pdf */
static double mix_pdf(const double n[3], const double wo[3], const double wi[3], const double m[5], int spec) {
    double ci = dot3(n, wi), co = dot3(n, wo);
    if (!(ci > 0.0) || !(co > 0.0)) return 0.0;
    double ps = spec_prob(m, spec);
    double p = (1.0 - ps) * ci / PI;
    if (ps > 0.0) {
        double h[3] = { wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2] };
        normalize3(h);
        double alpha = m[3] * m[3];
        p += ps * orc_ggx_g1(alpha, co) * orc_ggx_d(alpha, dot3(n, h)) / (4.0 * co);
    }
    return p;
}

/* GGX visible-normal sampling (Heitz, JCGT 2018) in the local frame where
 * the normal is +z; returns the microfacet normal. */
static void vndf_local(const double wo[3], double alpha, double u1, double u2, double h[3]) {
    double vh[3] = { alpha * wo[0], alpha * wo[1], wo[2] };
    normalize3(vh);
    double lensq = vh[0] * vh[0] + vh[1] * vh[1];
    double T1[3], T2[3];
    if (lensq > 0.0) { double il = 1.0 / sqrt(lensq); T1[0] = -vh[1] * il; T1[1] = vh[0] * il; T1[2] = 0.0; }
    else { T1[0] = 1.0; T1[1] = 0.0; T1[2] = 0.0; }
    cross3(vh, T1, T2);
    double r = sqrt(u1), phi = 2.0 * PI * u2;
    double t1 = r * cos(phi), t2 = r * sin(phi);
    double s = 0.5 * (1.0 + vh[2]);
    t2 = (1.0 - s) * sqrt(1.0 - t1 * t1) + s * t2;
    double tz = sqrt(fmax(0.0, 1.0 - t1 * t1 - t2 * t2));
    double nh[3];
    for (int a = 0; a < 3; ++a) nh[a] = t1 * T1[a] + t2 * T2[a] + tz * vh[a];
    h[0] = alpha * nh[0]; h[1] = alpha * nh[1]; h[2] = fmax(0.0, nh[2]);
    normalize3(h);
}

/* BRDF mixture sampler: u0 selects the lobe, (u1, u2) the direction.
 * Returns 1 (diffuse) or 2 (specular) for a direction above the surface,
 * 0 otherwise. */
static int mix_sample(const double n[3], const double t[3], const double b[3], const double wo[3],
                      const double m[5], int spec, double u0, double u1, double u2, double wi[3]) {
    double ps = spec_prob(m, spec);
    double l[3];
    int lobe;
    if (u0 < ps) {
        double wl[3] = { dot3(wo, t), dot3(wo, b), dot3(wo, n) };
        double h[3];
        vndf_local(wl, m[3] * m[3], u1, u2, h);
        double oh = dot3(wl, h);
        for (int a = 0; a < 3; ++a) l[a] = 2.0 * oh * h[a] - wl[a];
        lobe = 2;
    } else {
        double r = sqrt(u1), phi = 2.0 * PI * u2;
        l[0] = r * cos(phi); l[1] = r * sin(phi); l[2] = sqrt(fmax(0.0, 1.0 - u1));
        lobe = 1;
    }
    for (int a = 0; a < 3; ++a) wi[a] = t[a] * l[0] + b[a] * l[1] + n[a] * l[2];
    return dot3(n, wi) > 0.0 ? lobe : 0;
}

/* ------------------------------------------------------------------ */
/* surface interaction and material fetch                              */
/* ------------------------------------------------------------------ */
/* Interpolation in affine form, so that equal inputs give that value
 * exactly (a material at a clamp boundary stays on it): per-vertex values
 * x0 + b1 (x1 - x0) + b2 (x2 - x0); textures bilinear as nested lerps
 * lerp(lerp(x00, x10, fx), lerp(x01, x11, fx), fy), lerp(a, b, f) = a + f (b - a). */
typedef struct {
    int32_t idx[4];   /* vertices v0, v1, v2 or texels (i0,j0), (i1,j0), (i0,j1), (i1,j1) */
    double f1, f2;    /* (b1, b2) or (fx, fy) */
    int nw;
} interp;

static long long wrapi(long long i, long long n) { long long r = i % n; return r < 0 ? r + n : r; }

static void material_interp(const orc_ctx *c, int32_t prim, double b1, double b2, interp *ip) {
    const int32_t *fv = c->s.faces + 3 * (size_t)prim;
    if (c->s.mat_mode == 0) {
        ip->nw = 3;
        ip->idx[0] = fv[0]; ip->idx[1] = fv[1]; ip->idx[2] = fv[2];
        ip->f1 = b1; ip->f2 = b2;
        return;
    }
    const float *uv = c->s.uv;
    double u0 = uv[2 * (size_t)fv[0]], u1 = uv[2 * (size_t)fv[1]], u2 = uv[2 * (size_t)fv[2]];
    double v0 = uv[2 * (size_t)fv[0] + 1], v1 = uv[2 * (size_t)fv[1] + 1], v2 = uv[2 * (size_t)fv[2] + 1];
    double u = u0 + b1 * (u1 - u0) + b2 * (u2 - u0);
    double v = v0 + b1 * (v1 - v0) + b2 * (v2 - v0);
    /* bilinear, texel centres at (i + 1/2) / W, wrap addressing */
    double x = u * c->s.tw - 0.5, y = v * c->s.th - 0.5;
    double x0 = floor(x), y0 = floor(y);
    long long i0 = wrapi((long long)x0, c->s.tw), i1 = wrapi((long long)x0 + 1, c->s.tw);
    long long j0 = wrapi((long long)y0, c->s.th), j1 = wrapi((long long)y0 + 1, c->s.th);
    ip->nw = 4;
    ip->idx[0] = (int32_t)(j0 * c->s.tw + i0);
    ip->idx[1] = (int32_t)(j0 * c->s.tw + i1);
    ip->idx[2] = (int32_t)(j1 * c->s.tw + i0);
    ip->idx[3] = (int32_t)(j1 * c->s.tw + i1);
    ip->f1 = x - x0; ip->f2 = y - y0;
}

/* ------------------------------------------------------------------ */
/* material neural field F_m (Sec. 3 "Intrinsic decomposition"; Appendix */
/* A "Network details"); hash encoding after Mueller et al. (SIGGRAPH    */
/* 2022), Sec. 3.  The definition it follows is spelled out in oracle.h. */
/* ------------------------------------------------------------------ */
static int field_valid(const orc_field *f) {
    if (!f || !f->table || !f->w1 || !f->b1 || !f->w2 || !f->b2) return 0;
    if (f->levels < 1 || f->levels > ORC_FIELD_MAXL || f->log2_table < 1 || f->log2_table > 26) return 0;
    if (f->n_min < 1 || f->n_max < f->n_min) return 0;
    for (int a = 0; a < 3; ++a) if (!(f->hi[a] > f->lo[a])) return 0;
    return 1;
}

/* N_l: geometric progression from N_min to N_max (Mueller et al., Eq. 2-3) */
static int64_t field_res(const orc_field *f, int l) {
    if (f->levels == 1) return f->n_min;
    double g = log((double)f->n_max / (double)f->n_min) / (double)(f->levels - 1);
    return (int64_t)floor((double)f->n_min * exp((double)l * g) + 1e-6);
}

/* slot of grid vertex v at a level of resolution N: one-to-one while the
 * level's (N+1)^3 vertices fit in the table, else the spatial hash */
static int64_t field_slot(int64_t N, int64_t T, const int64_t v[3]) {
    int64_t side = N + 1;
    if (side * side * side <= T) return v[0] + side * (v[1] + side * v[2]);
    uint32_t h = (uint32_t)v[0] * 1u ^ (uint32_t)v[1] * 2654435761u ^ (uint32_t)v[2] * 805459861u;
    return (int64_t)(h % (uint64_t)T);
}

/* the 8 cell corners of x at level l: slots and trilinear weights
 * (corner bit a set = upper vertex along axis a) */
static void field_corners(const orc_field *f, int l, const double x[3], int64_t slot[8], double w[8]) {
    int64_t N = field_res(f, l), T = (int64_t)1 << f->log2_table;
    int64_t c[3]; double t[3];
    for (int a = 0; a < 3; ++a) {
        double u = clampd((x[a] - (double)f->lo[a]) / ((double)f->hi[a] - (double)f->lo[a]), 0.0, 1.0);
        double sa = u * (double)N;
        int64_t ca = (int64_t)floor(sa);
        if (ca > N - 1) ca = N - 1;
        c[a] = ca; t[a] = sa - (double)ca;
    }
    for (int k = 0; k < 8; ++k) {
        int64_t v[3]; double wk = 1.0;
        for (int a = 0; a < 3; ++a) {
            int up = (k >> a) & 1;
            v[a] = c[a] + up;
            wk *= up ? t[a] : 1.0 - t[a];
        }
        slot[k] = field_slot(N, T, v);
        w[k] = wk;
    }
}

/* forward pass at one point: encoding e[2L], pre-activations z1[32], m[4] */
static void field_forward(const orc_field *f, const double x[3], double *e, double *z1, double m[4]) {
    const int L = f->levels, I = 2 * L;
    const int64_t T = (int64_t)1 << f->log2_table;
    for (int l = 0; l < L; ++l) {
        int64_t slot[8]; double w[8];
        field_corners(f, l, x, slot, w);
        for (int j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 8; ++k) acc += w[k] * (double)f->table[((size_t)l * T + slot[k]) * 2 + j];
            e[2 * l + j] = acc;
        }
    }
    double a[ORC_FIELD_HIDDEN];
    for (int h = 0; h < ORC_FIELD_HIDDEN; ++h) {
        double acc = (double)f->b1[h];
        for (int i = 0; i < I; ++i) acc += (double)f->w1[(size_t)h * I + i] * e[i];
        z1[h] = acc;
        a[h] = acc > 0.0 ? acc : 0.0;
    }
    for (int o = 0; o < ORC_FIELD_OUT; ++o) {
        double acc = (double)f->b2[o];
        for (int h = 0; h < ORC_FIELD_HIDDEN; ++h) acc += (double)f->w2[(size_t)o * ORC_FIELD_HIDDEN + h] * a[h];
        m[o] = 1.0 / (1.0 + exp(-acc));
    }
}

/* pull-back of g = dL/dm at one point onto the parameters (chain rule
 * through the sigmoid, the two layers, the ReLU and the interpolation) */
static void field_backward(const orc_field *f, const double x[3], const double g[4], double *g_table,
                           double *g_w1, double *g_b1, double *g_w2, double *g_b2) {
    const int L = f->levels, I = 2 * L, H = ORC_FIELD_HIDDEN;
    const int64_t T = (int64_t)1 << f->log2_table;
    double e[2 * ORC_FIELD_MAXL], z1[ORC_FIELD_HIDDEN], m[ORC_FIELD_OUT];
    field_forward(f, x, e, z1, m);
    double dz2[ORC_FIELD_OUT], dz1[ORC_FIELD_HIDDEN];
    for (int o = 0; o < ORC_FIELD_OUT; ++o) dz2[o] = g[o] * m[o] * (1.0 - m[o]);
    for (int h = 0; h < H; ++h) {
        double da = 0.0;
        for (int o = 0; o < ORC_FIELD_OUT; ++o) da += (double)f->w2[(size_t)o * H + h] * dz2[o];
        dz1[h] = z1[h] > 0.0 ? da : 0.0;
    }
    if (g_b2) for (int o = 0; o < ORC_FIELD_OUT; ++o) g_b2[o] += dz2[o];
    if (g_w2)
        for (int o = 0; o < ORC_FIELD_OUT; ++o)
            for (int h = 0; h < H; ++h) g_w2[(size_t)o * H + h] += dz2[o] * (z1[h] > 0.0 ? z1[h] : 0.0);
    if (g_b1) for (int h = 0; h < H; ++h) g_b1[h] += dz1[h];
    if (g_w1)
        for (int h = 0; h < H; ++h)
            for (int i = 0; i < I; ++i) g_w1[(size_t)h * I + i] += dz1[h] * e[i];
    if (g_table) {
        for (int l = 0; l < L; ++l) {
            int64_t slot[8]; double w[8];
            field_corners(f, l, x, slot, w);
            for (int j = 0; j < 2; ++j) {
                double de = 0.0;
                for (int h = 0; h < H; ++h) de += (double)f->w1[(size_t)h * I + 2 * l + j] * dz1[h];
                for (int k = 0; k < 8; ++k) g_table[((size_t)l * T + slot[k]) * 2 + j] += w[k] * de;
            }
        }
    }
}

int32_t orc_field_levels(const orc_field *f, int64_t *res) {
    if (!field_valid(f) || !res) return -1;
    for (int l = 0; l < f->levels; ++l) res[l] = field_res(f, l);
    return f->levels;
}

int32_t orc_field_eval(const orc_field *f, const double *x, int64_t n, double *m) {
    if (!field_valid(f) || n < 0 || (n > 0 && (!x || !m))) return -1;
    for (int64_t i = 0; i < n; ++i) {
        double e[2 * ORC_FIELD_MAXL], z1[ORC_FIELD_HIDDEN];
        field_forward(f, x + 3 * i, e, z1, m + 4 * i);
    }
    return 0;
}

int32_t orc_field_vjp(const orc_field *f, const double *x, const double *g, int64_t n,
                      double *g_table, double *g_w1, double *g_b1, double *g_w2, double *g_b2) {
    if (!field_valid(f) || n < 0 || (n > 0 && (!x || !g))) return -1;
    for (int64_t i = 0; i < n; ++i) field_backward(f, x + 3 * i, g + 4 * i, g_table, g_w1, g_b1, g_w2, g_b2);
    return 0;
}

static dual dlerp(dual a, dual b, double f) { return dadd(a, dscale(dsub(b, a), f)); }

/* parameter kinds for derivative seeds */
enum { PK_NONE = -1, PK_VMAT = 0, PK_ALBEDO, PK_ROUGH, PK_METAL, PK_ENV, PK_FIELD };
typedef struct { int kind; int64_t idx; } seed_t;

static dual param_value(const orc_ctx *c, int kind, int64_t idx, seed_t sd) {
    double v;
    switch (kind) {
        case PK_VMAT:   v = c->s.vmat[idx]; break;
        case PK_ALBEDO: v = c->s.albedo[idx]; break;
        case PK_ROUGH:  v = c->s.rough[idx]; break;
        case PK_METAL:  v = c->s.metal[idx]; break;
        default:        v = c->s.env[idx]; break;
    }
    dual r = { v, (sd.kind == kind && sd.idx == idx) ? 1.0 : 0.0 };
    return r;
}

/* material at a hit as duals, clamped: albedo, metallic in [0,1], roughness
 * in [R_MIN, 1] */
static void material_d(const orc_ctx *c, const interp *ip, seed_t sd, dual m[5]) {
    for (int ch = 0; ch < 5; ++ch) {
        dual x[4];
        for (int k = 0; k < ip->nw; ++k) {
            if (c->s.mat_mode == 0) x[k] = param_value(c, PK_VMAT, (int64_t)ip->idx[k] * 5 + ch, sd);
            else if (ch < 3) x[k] = param_value(c, PK_ALBEDO, (int64_t)ip->idx[k] * 3 + ch, sd);
            else if (ch == 3) x[k] = param_value(c, PK_ROUGH, ip->idx[k], sd);
            else x[k] = param_value(c, PK_METAL, ip->idx[k], sd);
        }
        if (ip->nw == 3)
            m[ch] = dadd(x[0], dadd(dscale(dsub(x[1], x[0]), ip->f1), dscale(dsub(x[2], x[0]), ip->f2)));
        else
            m[ch] = dlerp(dlerp(x[0], x[1], ip->f1), dlerp(x[2], x[3], ip->f1), ip->f2);
    }
    for (int ch = 0; ch < 3; ++ch) m[ch] = dclamp(m[ch], 0.0, 1.0);
    m[3] = dclamp(m[3], R_MIN, 1.0);
    m[4] = dclamp(m[4], 0.0, 1.0);
}

static void material_plain(const orc_ctx *c, const interp *ip, double m[5]) {
    dual md[5]; seed_t none = { PK_NONE, -1 };
    material_d(c, ip, none, md);
    for (int i = 0; i < 5; ++i) m[i] = md[i].v;
}

/* env radiance max(0, L) with its derivative on L >= 0; a NaN channel is
 * radiance 0 with no derivative, like a negative one */
static dual env_d(const orc_ctx *c, int32_t texel, int ch, seed_t sd) {
    dual x = param_value(c, PK_ENV, (int64_t)texel * 3 + ch, sd);
    if (!(x.v >= 0.0)) return dc(0.0);
    return x;
}

/* field material at point p (mat_mode 2) as duals, clamped like the other
 * sources; the derivative seed (PK_FIELD, 4 k + ch) marks output ch of the
 * field at path vertex k */
static void material_field_d(const orc_ctx *c, const double p[3], int k, seed_t sd, dual m[5]) {
    double e[2 * ORC_FIELD_MAXL], z1[ORC_FIELD_HIDDEN], fm[ORC_FIELD_OUT];
    field_forward(c->s.field, p, e, z1, fm);
    for (int ch = 0; ch < 4; ++ch) {
        dual x = { fm[ch], (sd.kind == PK_FIELD && sd.idx == 4 * (int64_t)k + ch) ? 1.0 : 0.0 };
        m[ch] = x;
    }
    m[4] = dc(0.0);
    for (int ch = 0; ch < 3; ++ch) m[ch] = dclamp(m[ch], 0.0, 1.0);
    m[3] = dclamp(m[3], R_MIN, 1.0);
}

/* ------------------------------------------------------------------ */
/* one path sample                                                      */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t prim; double b1, b2;
    double p[3], n[3], wo[3];
    int32_t nee;            /* 1: reservoir non-empty and shadow ray unoccluded */
    double y[3], W; int32_t ytex;
    double wi[3], q, rr;    /* continuation direction, mixture pdf, 1 / q_rr */
} vtx;

typedef struct {
    double d[3];
    int32_t nv, miss_tex;
    vtx v[ORC_MAXB];
} pathrec;

static void camera_ray(const orc_view *vw, int x, int y, double u0, double u1, double o[3], double d[3]) {
    double aspect = (double)vw->w / (double)vw->h;
    double th = tan(0.5 * (double)vw->fov_y_deg * PI / 180.0);
    double nx = 2.0 * (x + u0) / vw->w - 1.0;
    double ny = 1.0 - 2.0 * (y + u1) / vw->h;
    double dcam[3] = { nx * th * aspect, ny * th, -1.0 };
    for (int r = 0; r < 3; ++r) {
        d[r] = (double)vw->c2w[4 * r] * dcam[0] + (double)vw->c2w[4 * r + 1] * dcam[1] + (double)vw->c2w[4 * r + 2] * dcam[2];
        o[r] = (double)vw->c2w[4 * r + 3];
    }
    normalize3(d);
}

/* Conditioning hook (orc_options.jitter): unit vector d moved by up to
 * jitter x 2^-24 per component and renormalised, from the Philox stream of
 * (pixel, sample, view, vertex k, block 0xC000 + slot) under key jitter_seed:
 * slot 0 the camera ray, 1 the geometric normal, 2 the continuation
 * direction, 3 the field's input point, 16 + s candidate s.  It stands for
 * the rounding an FP32 evaluation of the same path commits. */
static void jitter_unit(const orc_options *opt, uint32_t pixel, uint32_t sc, uint32_t vi, int k, uint32_t slot,
                        double d[3]) {
    if (!(opt->jitter > 0.0)) return;
    double u[4];
    uniforms4(opt->jitter_seed, pixel, sc, vi, (uint32_t)k, 0xC000u + slot, u);
    const double eps = opt->jitter * (1.0 / 16777216.0);
    for (int a = 0; a < 3; ++a) d[a] += eps * (2.0 * u[a] - 1.0);
    normalize3(d);
}

/* Shading point of a surface hit (Sec. 3 "Rendering"): position from the
 * barycentrics, geometric normal turned towards the viewer, shading frame and
 * clamped material. */
typedef struct {
    int32_t prim; double b1, b2;
    double p[3], n[3], wo[3], t[3], b[3], m[5];
} shpt;

static void shading_point(const orc_ctx *c, const hitrec *hr, const double d[3], int k, shpt *S) {
    S->prim = hr->prim; S->b1 = hr->b1; S->b2 = hr->b2;
    const double *v0 = c->v + 9 * (size_t)hr->prim, *v1 = v0 + 3, *v2 = v0 + 6;
    double b0 = 1.0 - hr->b1 - hr->b2, e1[3], e2[3], ng[3];
    for (int a = 0; a < 3; ++a) S->p[a] = b0 * v0[a] + hr->b1 * v1[a] + hr->b2 * v2[a];
    sub3(v1, v0, e1); sub3(v2, v0, e2); cross3(e1, e2, ng); normalize3(ng);
    if (dot3(ng, d) > 0.0) { ng[0] = -ng[0]; ng[1] = -ng[1]; ng[2] = -ng[2]; }
    for (int a = 0; a < 3; ++a) { S->n[a] = ng[a]; S->wo[a] = -d[a]; }
    orc_frame(S->n, S->t, S->b);
    if (c->s.mat_mode == 2) {
        dual md[5]; seed_t none = { PK_NONE, -1 };
        material_field_d(c, S->p, k, none, md);
        for (int ch = 0; ch < 5; ++ch) S->m[ch] = md[ch].v;
    } else {
        interp ip; material_interp(c, hr->prim, hr->b1, hr->b2, &ip);
        material_plain(c, &ip, S->m);
    }
}

/* the normal of shading point S of vertex k after the conditioning hook,
 * and its frame; with the material field, also the point the field is
 * evaluated at (slot 3: each coordinate moved by up to jitter x 2^-24 of
 * max(1, |coordinate|), the rounding of an FP32 hit position) and the
 * material there */
static void jitter_normal(const orc_ctx *c, const orc_options *opt, uint32_t pixel, uint32_t sc, uint32_t vi, int k,
                          shpt *S) {
    if (!(opt->jitter > 0.0)) return;
    jitter_unit(opt, pixel, sc, vi, k, 1, S->n);
    orc_frame(S->n, S->t, S->b);
    if (c->s.mat_mode == 2) {
        double u[4];
        uniforms4(opt->jitter_seed, pixel, sc, vi, (uint32_t)k, 0xC000u + 3u, u);
        const double eps = opt->jitter * (1.0 / 16777216.0);
        for (int a = 0; a < 3; ++a) S->p[a] += eps * fmax(1.0, fabs(S->p[a])) * (2.0 * u[a] - 1.0);
        dual md[5]; seed_t none = { PK_NONE, -1 };
        material_field_d(c, S->p, k, none, md);
        for (int ch = 0; ch < 5; ++ch) S->m[ch] = md[ch].v;
    }
}

/* RIS over Me env + Mb BRDF candidates with a streaming weighted reservoir
 * (Sec. 4.1, Eq. restir; App. A "Spatial-temporal reuse"), candidate s drawn
 * from Philox block (k, s).  sel = selected candidate (-1 none); W = its
 * contribution weight w_sum / p_hat(y). */
typedef struct {
    int32_t sel, ytex;
    double y[3], fy[3], Ly[3], wsum, phat, W;
} risres;

static void ris_vertex(const orc_ctx *c, const shpt *S, const orc_options *opt, uint32_t pixel, uint32_t sc,
                       uint32_t vi, int k, risres *r, uint32_t *h, int64_t *cnt) {
    int spec = opt->brdf == 1;
    int Mb = opt->ris_m_brdf, Me = opt->ris_m - opt->ris_m_brdf;
    double u[4];
    r->sel = -1; r->ytex = -1; r->wsum = 0.0; r->phat = 0.0; r->W = 0.0;
    for (int a = 0; a < 3; ++a) { r->y[a] = 0.0; r->fy[a] = 0.0; r->Ly[a] = 0.0; }
    double co = dot3(S->n, S->wo);
    if (!(co > 0.0)) return;
    for (int s = 0; s < opt->ris_m; ++s) {
        cnt[ORC_C_CANDIDATES]++;
        uniforms4(opt->seed, pixel, sc, vi, (uint32_t)k, (uint32_t)s, u);
        double w[3], qe = 0.0, qb = 0.0;
        int32_t tex = -1;
        int ok;
        if (s < Me) {
            ok = env_sample(c, u[0], u[1], w, &qe, &tex);
            if (ok) {
                jitter_unit(opt, pixel, sc, vi, k, 16u + (uint32_t)s, w);
                qb = mix_pdf(S->n, S->wo, w, S->m, spec);
            }
        } else {
            int lb = mix_sample(S->n, S->t, S->b, S->wo, S->m, spec, u[0], u[1], u[2], w);
            ok = lb != 0;
            if (ok) {
                jitter_unit(opt, pixel, sc, vi, k, 16u + (uint32_t)s, w);
                qb = mix_pdf(S->n, S->wo, w, S->m, spec);
                qe = env_pdf_dir(c, w);
                tex = env_texel_of(c, w);
                *h ^= ev_cand((uint32_t)k, (uint32_t)s, (uint32_t)lb, (uint32_t)tex);
            }
        }
        if (!ok) continue;
        double ci = dot3(S->n, w);
        if (!(ci > 0.0)) continue;
        double f[3], L[3];
        brdf_eval_plain(S->n, S->wo, w, S->m, spec, f);
        for (int ch = 0; ch < 3; ++ch) L[ch] = env_channel(c, tex, ch);
        double phat = (L[0] * f[0] + L[1] * f[1] + L[2] * f[2]) / 3.0 * ci;
        double den = Me * qe + Mb * qb;
        if (!(phat > 0.0) || !(den > 0.0)) continue;
        double ws = phat / den;
        r->wsum += ws;
        if (u[3] < ws / r->wsum) {
            r->sel = s; r->phat = phat; r->ytex = tex;
            for (int a = 0; a < 3; ++a) { r->y[a] = w[a]; r->fy[a] = f[a]; r->Ly[a] = L[a]; }
        }
    }
    if (r->sel >= 0) r->W = r->wsum / r->phat;
}

/* ------------------------------------------------------------------ */
/* reservoir reuse at primary vertices (Sec. 4.1 end; App. A            */
/* "Spatial-temporal reuse"), in the readings the design document       */
/* lists: per frame, the initial RIS reservoir r0 of every sample is     */
/* merged with the previous frame's final reservoir of the same sample   */
/* (temporal, its confidence capped at m_cap * M), then with the        */
/* temporally merged reservoirs of `spatial` neighbours (same view and   */
/* sample index, offsets uniform in a (2R+1)^2 window without the       */
/* centre, from Philox block (1, 0xFFE0 + j) by integer arithmetic).     */
/* Merging is the confidence-weighted combine: input i with sample y_i,  */
/* contribution weight W_i and confidence M_i gets resampling weight     */
/* w_i = p_hat_q(y_i) W_i M_i at the merging vertex q; the pick follows  */
/* the streaming reservoir rule, and W = sum w / (sum M p_hat_q(y)).    */
/* ------------------------------------------------------------------ */
typedef struct { double y[3], W, M; } resv;

/* the RIS target at a shading point: mean over channels of L(y) f(y) cos */
static double phat_at(const orc_ctx *c, const shpt *S, int spec, const double y[3]) {
    double ci = dot3(S->n, y);
    if (!(ci > 0.0)) return 0.0;
    double f[3], L[3];
    brdf_eval_plain(S->n, S->wo, y, S->m, spec, f);
    int32_t tex = env_texel_of(c, y);
    for (int ch = 0; ch < 3; ++ch) L[ch] = env_channel(c, tex, ch);
    return (L[0] * f[0] + L[1] * f[1] + L[2] * f[2]) / 3.0 * ci;
}

static int merge_reservoirs(const orc_ctx *c, const shpt *S, int spec, const resv *in, const double *u, int n,
                            resv *out) {
    double wsum = 0.0, Msum = 0.0;
    int sel = -1;
    for (int i = 0; i < n; ++i) {
        if (!(in[i].M > 0.0)) continue;
        Msum += in[i].M;
        if (!(in[i].W > 0.0)) continue;
        double w = phat_at(c, S, spec, in[i].y) * in[i].W * in[i].M;
        if (!(w > 0.0)) continue;
        wsum += w;
        if (u[i] < w / wsum) sel = i;
    }
    out->M = Msum;
    out->W = 0.0;
    for (int a = 0; a < 3; ++a) out->y[a] = 0.0;
    if (sel >= 0) {
        for (int a = 0; a < 3; ++a) out->y[a] = in[sel].y[a];
        out->W = wsum / (Msum * phat_at(c, S, spec, out->y));
    }
    return sel;
}

static uint32_t ev_merge(uint32_t stage, uint32_t sel) { return fnv_word(fnv_word(FNV_BASIS, 0x40000u | stage), sel); }

static int64_t sample_index(const orc_view *views, int32_t vi, int32_t pixel, int32_t sidx) {
    int64_t base = 0;
    for (int v = 0; v < vi; ++v) base += (int64_t)views[v].w * views[v].h * views[v].spp;
    return base + (int64_t)pixel * views[vi].spp + sidx;
}

/* primary vertex of sample (vi, pixel, sidx) and its initial reservoir; 0
 * when the primary ray misses (no reservoir) */
static int primary_vertex(const orc_ctx *c, const orc_view *views, int32_t vi, int32_t pixel, int32_t sidx,
                          const orc_options *opt, shpt *S, resv *r0, uint32_t *h, int64_t *cnt) {
    const orc_view *vw = &views[vi];
    uint32_t sc = vw->sample_offset + (uint32_t)sidx;
    double u[4], o[3], d[3];
    uniforms4(opt->seed, (uint32_t)pixel, sc, (uint32_t)vi, 0, 0, u);
    camera_ray(vw, pixel % vw->w, pixel / vw->w, u[0], u[1], o, d);
    jitter_unit(opt, (uint32_t)pixel, sc, (uint32_t)vi, 0, 0, d);
    cnt[ORC_C_CLOSEST_RAYS]++;
    hitrec hr = trace_closest(c, o, d, 0, &cnt[ORC_C_CLOSEST_NODES], &cnt[ORC_C_CLOSEST_TRIS]);
    if (hr.prim < 0) return 0;
    shading_point(c, &hr, d, 0, S);
    jitter_normal(c, opt, (uint32_t)pixel, sc, (uint32_t)vi, 1, S);
    risres rr;
    ris_vertex(c, S, opt, (uint32_t)pixel, sc, (uint32_t)vi, 1, &rr, h, cnt);
    for (int a = 0; a < 3; ++a) r0->y[a] = rr.y[a];
    r0->W = rr.W;
    r0->M = dot3(S->n, S->wo) > 0.0 ? (double)opt->ris_m : 0.0;
    return 1;
}

/* temporal merge of a sample's initial reservoir with the previous frame's */
static void temporal_merge(const orc_ctx *c, const orc_view *views, int32_t vi, int32_t pixel, int32_t sidx,
                           const orc_options *opt, const shpt *S, const resv *r0, resv *r1, uint32_t *h) {
    const orc_reuse *ru = opt->reuse;
    *r1 = *r0;
    if (!ru->temporal || !ru->prev) return;
    const float *pr = ru->prev + 8 * sample_index(views, vi, pixel, sidx);
    resv in[2];
    in[0] = *r0;
    for (int a = 0; a < 3; ++a) in[1].y[a] = pr[a];
    in[1].W = pr[3];
    in[1].M = fmin((double)pr[4], (double)ru->m_cap * opt->ris_m);
    double u[4], uu[2];
    uniforms4(opt->seed, (uint32_t)pixel, views[vi].sample_offset + (uint32_t)sidx, (uint32_t)vi, 1, 0xFFD0u, u);
    uu[0] = 0.0; uu[1] = u[0];
    int sel = merge_reservoirs(c, S, opt->brdf == 1, in, uu, 2, r1);
    if (h) *h ^= ev_merge(1u, (uint32_t)sel);
}

/* final reservoir of sample (vi, pixel, sidx) at its primary vertex S,
 * given its initial reservoir r0 */
static void reuse_reservoir(const orc_ctx *c, const orc_view *views, int32_t vi, int32_t pixel, int32_t sidx,
                            const orc_options *opt, const shpt *S, const resv *r0, resv *r2, uint32_t *h,
                            int64_t *cnt) {
    const orc_reuse *ru = opt->reuse;
    const orc_view *vw = &views[vi];
    uint32_t sc = vw->sample_offset + (uint32_t)sidx;
    resv in[1 + ORC_REUSE_MAXK];
    double uu[1 + ORC_REUSE_MAXK];
    temporal_merge(c, views, vi, pixel, sidx, opt, S, r0, &in[0], h);
    uu[0] = 0.0;
    int n = 1;
    const int x = pixel % vw->w, y = pixel / vw->w, R = ru->radius, side = 2 * R + 1;
    for (int j = 0; j < ru->spatial; ++j) {
        uint32_t ctr[4] = { (uint32_t)pixel, sc, (uint32_t)vi, (1u << 16) | (0xFFE0u + (uint32_t)j) };
        uint32_t key[2] = { (uint32_t)opt->seed, (uint32_t)(opt->seed >> 32) };
        uint32_t r[4];
        orc_philox(ctr, key, r);
        int dx = (int)(((uint64_t)r[0] * (uint64_t)side) >> 32) - R;
        int dy = (int)(((uint64_t)r[1] * (uint64_t)side) >> 32) - R;
        int xn = x + dx, yn = y + dy;
        if ((dx == 0 && dy == 0) || xn < 0 || yn < 0 || xn >= vw->w || yn >= vw->h) continue;
        int32_t pn = yn * vw->w + xn;
        shpt Sn;
        resv r0n;
        uint32_t hn = 0;
        if (!primary_vertex(c, views, vi, pn, sidx, opt, &Sn, &r0n, &hn, cnt)) continue;
        temporal_merge(c, views, vi, pn, sidx, opt, &Sn, &r0n, &in[n], NULL);
        uu[n] = (double)(r[2] >> 8) * (1.0 / 16777216.0);
        ++n;
    }
    int sel = merge_reservoirs(c, S, opt->brdf == 1, in, uu, n, r2);
    *h ^= ev_merge(2u, (uint32_t)sel);
}

/* neighbour offset j of a sample (test hook): 1 if it lies in the window */
int32_t orc_reuse_offset(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t view, int32_t j, int32_t radius,
                         int32_t *dx, int32_t *dy) {
    if (radius < 1 || j < 0 || j >= ORC_REUSE_MAXK || !dx || !dy) return -1;
    uint32_t ctr[4] = { pixel, sample, view, (1u << 16) | (0xFFE0u + (uint32_t)j) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t r[4];
    orc_philox(ctr, key, r);
    const uint64_t side = 2 * (uint64_t)radius + 1;
    *dx = (int32_t)(((uint64_t)r[0] * side) >> 32) - radius;
    *dy = (int32_t)(((uint64_t)r[1] * side) >> 32) - radius;
    return 0;
}

static int reuse_on(const orc_options *opt) {
    return opt->reuse && (opt->reuse->spatial > 0 || opt->reuse->temporal);
}

/* Path tracing with RIS next-event estimation at every surface vertex
 * (Sec. 4.1, Eq. restir; Sec. 4.2, Eq. sec_bouce), and with reservoir reuse
 * at the primary vertex when enabled.  Fills rgb, hash and the path record
 * used for differentiation (the reused sample and its weight are held fixed
 * there like every other sampling decision).  res_out (nullable) receives the
 * primary vertex's final reservoir (y, W, M). */
static void trace_path(const orc_ctx *c, const orc_view *views, int32_t vi, int32_t pixel, int32_t sidx,
                       const orc_options *opt, double rgb[3], uint32_t *hash, pathrec *rec, int64_t *cnt,
                       double *res_out) {
    const orc_view *vw = &views[vi];
    uint32_t S = vw->sample_offset + (uint32_t)sidx;
    int spec = opt->brdf == 1;
    double u[4];
    uniforms4(opt->seed, (uint32_t)pixel, S, (uint32_t)vi, 0, 0, u);
    double o[3], d[3];
    camera_ray(vw, pixel % vw->w, pixel / vw->w, u[0], u[1], o, d);
    jitter_unit(opt, (uint32_t)pixel, S, (uint32_t)vi, 0, 0, d);
    double T[3] = { 1, 1, 1 };
    rgb[0] = rgb[1] = rgb[2] = 0.0;
    uint32_t h = 0;
    rec->nv = 0; rec->miss_tex = -1;
    if (res_out) for (int a = 0; a < 8; ++a) res_out[a] = 0.0;
    for (int a = 0; a < 3; ++a) rec->d[a] = d[a];
    for (int k = 1; k <= opt->bounces; ++k) {
        cnt[ORC_C_CLOSEST_RAYS]++;
        hitrec hr = trace_closest(c, o, d, 0, &cnt[ORC_C_CLOSEST_NODES], &cnt[ORC_C_CLOSEST_TRIS]);
        if (hr.prim < 0) {
            h ^= ev_miss((uint32_t)k);
            if (k == 1) {
                cnt[ORC_C_PRIMARY_MISS]++;
                if (opt->background == 0) {
                    int32_t t = env_texel_of(c, d);
                    rec->miss_tex = t;
                    for (int ch = 0; ch < 3; ++ch) rgb[ch] = env_channel(c, t, ch);
                }
            }
            break;
        }
        cnt[ORC_C_HITS]++;
        vtx *V = &rec->v[rec->nv++];
        V->prim = hr.prim; V->b1 = hr.b1; V->b2 = hr.b2;
        V->nee = 0; V->W = 0.0; V->ytex = -1; V->q = 0.0; V->rr = 1.0;
        shpt Sp;
        shading_point(c, &hr, d, rec->nv - 1, &Sp);
        jitter_normal(c, opt, (uint32_t)pixel, S, (uint32_t)vi, k, &Sp);
        for (int a = 0; a < 3; ++a) { V->p[a] = Sp.p[a]; V->n[a] = Sp.n[a]; V->wo[a] = Sp.wo[a]; }
        const double *m = Sp.m;
        double pn = fmax(fabs(V->p[0]), fmax(fabs(V->p[1]), fabs(V->p[2])));
        double eps = 1e-4 * fmax(1.0, pn);
        double org[3] = { V->p[0] + eps * V->n[0], V->p[1] + eps * V->n[1], V->p[2] + eps * V->n[2] };
        double co = dot3(V->n, V->wo);
        /* --- direct light: RIS (and reuse at the primary vertex) ---------- */
        risres R;
        ris_vertex(c, &Sp, opt, (uint32_t)pixel, S, (uint32_t)vi, k, &R, &h, cnt);
        int32_t sel = R.sel;
        double W = R.W;
        if (k == 1 && reuse_on(opt)) {
            resv r0, r2;
            for (int a = 0; a < 3; ++a) r0.y[a] = R.y[a];
            r0.W = R.W;
            r0.M = co > 0.0 ? (double)opt->ris_m : 0.0;
            reuse_reservoir(c, views, vi, pixel, sidx, opt, &Sp, &r0, &r2, &h, cnt);
            if (res_out) { for (int a = 0; a < 3; ++a) res_out[a] = r2.y[a]; res_out[3] = r2.W; res_out[4] = r2.M; }
            sel = r2.W > 0.0 ? 0 : -1;
            W = r2.W;
            if (sel >= 0) {
                for (int a = 0; a < 3; ++a) R.y[a] = r2.y[a];
                brdf_eval_plain(Sp.n, Sp.wo, R.y, Sp.m, spec, R.fy);
                R.ytex = env_texel_of(c, R.y);
                for (int ch = 0; ch < 3; ++ch) R.Ly[ch] = env_channel(c, R.ytex, ch);
            }
        }
        if (sel >= 0) {
            for (int a = 0; a < 3; ++a) V->y[a] = R.y[a];
            V->ytex = R.ytex;
            V->W = W;
            cnt[ORC_C_SHADOW_RAYS]++;
            int occl = trace_any(c, org, V->y, 0, &cnt[ORC_C_SHADOW_NODES], &cnt[ORC_C_SHADOW_TRIS]);
            h ^= ev_nee((uint32_t)k, occl ? 0u : 1u);
            if (!occl) {
                cnt[ORC_C_NEE_VISIBLE]++;
                V->nee = 1;
                double cy = dot3(V->n, V->y);
                for (int ch = 0; ch < 3; ++ch) rgb[ch] += T[ch] * R.Ly[ch] * R.fy[ch] * cy * V->W;
            }
        }
        if (k == opt->bounces) { h ^= ev_vertex((uint32_t)k, (uint32_t)hr.prim, (uint32_t)sel, 0u); break; }
        /* --- continuation (Eq. mc_indir): BRDF mixture sample ------------- */
        uniforms4(opt->seed, (uint32_t)pixel, S, (uint32_t)vi, (uint32_t)k, 0xFFFFu, u);
        double wi[3];
        int lobe = co > 0.0 ? mix_sample(V->n, Sp.t, Sp.b, V->wo, m, spec, u[0], u[1], u[2], wi) : 0;
        if (lobe) jitter_unit(opt, (uint32_t)pixel, S, (uint32_t)vi, k, 2, wi);
        double q = lobe ? mix_pdf(V->n, V->wo, wi, m, spec) : 0.0;
        if (!lobe || !(q > 0.0)) { h ^= ev_vertex((uint32_t)k, (uint32_t)hr.prim, (uint32_t)sel, 2u); break; }
        double f[3];
        brdf_eval_plain(V->n, V->wo, wi, m, spec, f);
        double ci = dot3(V->n, wi);
        for (int ch = 0; ch < 3; ++ch) T[ch] *= f[ch] * ci / q;
        V->q = q;
        for (int a = 0; a < 3; ++a) V->wi[a] = wi[a];
        if (opt->rr_start >= 0 && k >= opt->rr_start) {
            double qr = fmin(0.95, fmax(T[0], fmax(T[1], T[2])));
            if (!(qr > 0.0) || !(u[3] < qr)) { h ^= ev_vertex((uint32_t)k, (uint32_t)hr.prim, (uint32_t)sel, 3u); break; }
            for (int ch = 0; ch < 3; ++ch) T[ch] /= qr;
            V->rr = 1.0 / qr;
        }
        h ^= ev_vertex((uint32_t)k, (uint32_t)hr.prim, (uint32_t)sel, lobe == 2 ? 4u : 1u);
        for (int a = 0; a < 3; ++a) { o[a] = org[a]; d[a] = wi[a]; }
    }
    *hash = h;
}

/* Detached-sampling functional of a recorded path: directions, selections,
 * lobe and roulette decisions and every pdf / reservoir weight are
 * constants; materials (and env texels) are read from ctx, with a derivative
 * seed on one parameter.  C = sum_k T_k (.) D_k, T_{k+1} = T_k (.) beta_k. */
static void frozen_eval(const orc_ctx *c, const pathrec *rec, const orc_options *opt, seed_t sd, dual C[3]) {
    int spec = opt->brdf == 1;
    seed_t none = { PK_NONE, -1 };
    for (int ch = 0; ch < 3; ++ch) C[ch] = dc(0.0);
    if (rec->nv == 0) {
        if (rec->miss_tex >= 0) for (int ch = 0; ch < 3; ++ch) C[ch] = env_d(c, rec->miss_tex, ch, sd);
        return;
    }
    dual T[3] = { dc(1.0), dc(1.0), dc(1.0) };
    for (int k = 0; k < rec->nv; ++k) {
        const vtx *V = &rec->v[k];
        seed_t s_here = (opt->grad_mode == 1 && k > 0) ? none : sd;
        dual m[5];
        if (c->s.mat_mode == 2) {
            material_field_d(c, V->p, k, s_here, m);
        } else {
            interp ip; material_interp(c, V->prim, V->b1, V->b2, &ip);
            material_d(c, &ip, s_here, m);
        }
        if (V->nee) {
            dual f[3];
            brdf_eval_d(V->n, V->wo, V->y, m, spec, f);
            double cw = dot3(V->n, V->y) * V->W;
            for (int ch = 0; ch < 3; ++ch) {
                dual L = env_d(c, V->ytex, ch, s_here);
                C[ch] = dadd(C[ch], dmul(T[ch], dscale(dmul(L, f[ch]), cw)));
            }
        }
        if (k + 1 < rec->nv) {
            dual f[3];
            brdf_eval_d(V->n, V->wo, V->wi, m, spec, f);
            double s = dot3(V->n, V->wi) / V->q * V->rr;
            for (int ch = 0; ch < 3; ++ch) T[ch] = dmul(T[ch], dscale(f[ch], s));
        }
    }
}

/* ------------------------------------------------------------------ */
/* public entry points                                                  */
/* ------------------------------------------------------------------ */
static int check_args(const orc_ctx *c, const orc_view *views, int32_t nviews, const orc_options *opt,
                      const int32_t *items, int64_t n) {
    if (!c || !views || nviews <= 0 || !opt || (n > 0 && !items)) return -1;
    if (opt->bounces < 1 || opt->bounces > ORC_MAXB || opt->ris_m < 1 || opt->ris_m_brdf < 0 ||
        opt->ris_m_brdf > opt->ris_m) return -1;
    if (opt->reuse && (opt->reuse->spatial < 0 || opt->reuse->spatial > ORC_REUSE_MAXK || opt->reuse->radius < 1 ||
                       opt->reuse->radius > 64 || opt->reuse->m_cap < 1)) return -1;
    if (!(opt->jitter >= 0.0) || opt->jitter > 1e6) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int32_t v = items[3 * i], p = items[3 * i + 1], s = items[3 * i + 2];
        if (v < 0 || v >= nviews) return -1;
        if (p < 0 || (int64_t)p >= (int64_t)views[v].w * views[v].h || s < 0 || s >= views[v].spp) return -1;
    }
    return 0;
}

int32_t orc_render(const orc_ctx *c, const orc_view *views, int32_t nviews, const orc_options *opt,
                   const int32_t *items, int64_t n, double *rgb, uint32_t *hash, int64_t *counters,
                   int32_t nthreads) {
    if (check_args(c, views, nviews, opt, items, n) || !rgb) return -1;
    if (nthreads < 1) nthreads = 1;
    int64_t total[ORC_NCOUNT] = { 0 };
#pragma omp parallel num_threads(nthreads)
    {
        int64_t cnt[ORC_NCOUNT] = { 0 };
        pathrec *rec = (pathrec *)malloc(sizeof(pathrec));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            uint32_t hh;
            trace_path(c, views, items[3 * i], items[3 * i + 1], items[3 * i + 2], opt, rgb + 3 * i, &hh, rec, cnt,
                       (opt->reuse && opt->reuse->out) ? opt->reuse->out + 8 * i : NULL);
            if (hash) hash[i] = hh;
        }
        free(rec);
#pragma omp critical
        for (int k = 0; k < ORC_NCOUNT; ++k) total[k] += cnt[k];
    }
    if (counters) for (int k = 0; k < ORC_NCOUNT; ++k) counters[k] += total[k];
    return 0;
}

/* every parameter the frozen functional of this path reads */
static int path_params(const orc_ctx *c, const pathrec *rec, const orc_options *opt, seed_t *ps, int cap) {
    int np = 0;
#define ADDP(K, I) do { seed_t t_ = { (K), (I) }; int dup_ = 0; \
        for (int q_ = 0; q_ < np; ++q_) if (ps[q_].kind == t_.kind && ps[q_].idx == t_.idx) { dup_ = 1; break; } \
        if (!dup_ && np < cap) ps[np++] = t_; } while (0)
    if (rec->nv == 0 && rec->miss_tex >= 0)
        for (int ch = 0; ch < 3; ++ch) ADDP(PK_ENV, (int64_t)rec->miss_tex * 3 + ch);
    for (int k = 0; k < rec->nv; ++k) {
        if (opt->grad_mode == 1 && k > 0) break;
        const vtx *V = &rec->v[k];
        if (c->s.mat_mode == 2) {
            for (int ch = 0; ch < 4; ++ch) ADDP(PK_FIELD, 4 * (int64_t)k + ch);
            if (V->nee) for (int ch = 0; ch < 3; ++ch) ADDP(PK_ENV, (int64_t)V->ytex * 3 + ch);
            continue;
        }
        interp ip; material_interp(c, V->prim, V->b1, V->b2, &ip);
        for (int j = 0; j < ip.nw; ++j) {
            if (c->s.mat_mode == 0) {
                for (int ch = 0; ch < 5; ++ch) ADDP(PK_VMAT, (int64_t)ip.idx[j] * 5 + ch);
            } else {
                for (int ch = 0; ch < 3; ++ch) ADDP(PK_ALBEDO, (int64_t)ip.idx[j] * 3 + ch);
                ADDP(PK_ROUGH, ip.idx[j]);
                ADDP(PK_METAL, ip.idx[j]);
            }
        }
        if (V->nee) for (int ch = 0; ch < 3; ++ch) ADDP(PK_ENV, (int64_t)V->ytex * 3 + ch);
    }
#undef ADDP
    return np;
}

/* Shared gradient driver.  Per item: record the path, then one
 * forward-mode evaluation of the frozen functional per parameter it reads.
 * Texel and vertex parameters accumulate straight into dst[kind]; in field
 * mode the derivatives with respect to the field's outputs at each vertex are
 * collected and pulled back through the field (chain rule). */
typedef struct { double *table, *w1, *b1, *w2, *b2; } field_grads;

static int32_t grad_impl(const orc_ctx *c, const orc_view *views, int32_t nviews, const orc_options *opt,
                         const int32_t *items, int64_t n, const double *dldc, double *dst_of[6],
                         const field_grads *fg, int32_t nthreads) {
    if (check_args(c, views, nviews, opt, items, n) || !dldc) return -1;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        int64_t cnt[ORC_NCOUNT] = { 0 };
        pathrec *rec = (pathrec *)malloc(sizeof(pathrec));
        seed_t *ps = (seed_t *)malloc(sizeof(seed_t) * 64 * ORC_MAXB);
        double gfield[ORC_MAXB][4];
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            double rgb[3]; uint32_t hh;
            trace_path(c, views, items[3 * i], items[3 * i + 1], items[3 * i + 2], opt, rgb, &hh, rec, cnt, NULL);
            int np = path_params(c, rec, opt, ps, 64 * ORC_MAXB);
            memset(gfield, 0, sizeof(gfield));
            for (int j = 0; j < np; ++j) {
                dual C[3];
                frozen_eval(c, rec, opt, ps[j], C);
                double g = dldc[3 * i] * C[0].d + dldc[3 * i + 1] * C[1].d + dldc[3 * i + 2] * C[2].d;
                if (ps[j].kind == PK_FIELD) { gfield[ps[j].idx / 4][ps[j].idx % 4] = g; continue; }
                double *dst = dst_of[ps[j].kind];
                if (dst) {
#pragma omp atomic
                    dst[ps[j].idx] += g;
                }
            }
            if (c->s.mat_mode == 2 && fg) {
#pragma omp critical(field_pullback)
                for (int k = 0; k < rec->nv; ++k)
                    field_backward(c->s.field, rec->v[k].p, gfield[k], fg->table, fg->w1, fg->b1, fg->w2, fg->b2);
            }
        }
        free(ps); free(rec);
    }
    return 0;
}

int32_t orc_grad(const orc_ctx *c, const orc_view *views, int32_t nviews, const orc_options *opt,
                 const int32_t *items, int64_t n, const double *dldc, double *g_vmat, double *g_albedo,
                 double *g_rough, double *g_metal, double *g_env, int32_t nthreads) {
    if (c && c->s.mat_mode == 2) return -1;
    double *dst_of[6] = { g_vmat, g_albedo, g_rough, g_metal, g_env, NULL };
    return grad_impl(c, views, nviews, opt, items, n, dldc, dst_of, NULL, nthreads);
}

int32_t orc_grad_field(const orc_ctx *c, const orc_view *views, int32_t nviews, const orc_options *opt,
                       const int32_t *items, int64_t n, const double *dldc, double *g_table, double *g_w1,
                       double *g_b1, double *g_w2, double *g_b2, double *g_env, int32_t nthreads) {
    if (!c || c->s.mat_mode != 2) return -1;
    double *dst_of[6] = { NULL, NULL, NULL, NULL, g_env, NULL };
    field_grads fg = { g_table, g_w1, g_b1, g_w2, g_b2 };
    return grad_impl(c, views, nviews, opt, items, n, dldc, dst_of, &fg, nthreads);
}

int32_t orc_frozen(const orc_ctx *rc, const orc_ctx *ec, const orc_view *views, int32_t nviews,
                   const orc_options *opt, const int32_t item[3], double rgb[3]) {
    if (check_args(rc, views, nviews, opt, item, 1) || !ec || !rgb) return -1;
    if (ec->s.nf != rc->s.nf || ec->s.mat_mode != rc->s.mat_mode) return -1;
    int64_t cnt[ORC_NCOUNT] = { 0 };
    pathrec *rec = (pathrec *)malloc(sizeof(pathrec));
    double tmp[3]; uint32_t hh;
    trace_path(rc, views, item[0], item[1], item[2], opt, tmp, &hh, rec, cnt, NULL);
    seed_t none = { PK_NONE, -1 };
    dual C[3];
    frozen_eval(ec, rec, opt, none, C);
    for (int ch = 0; ch < 3; ++ch) rgb[ch] = C[ch].v;
    free(rec);
    return 0;
}

int32_t orc_trace(const orc_ctx *c, const double *o, const double *d, int64_t n, int32_t any_hit,
                  int32_t brute, int32_t *prim, double *t, double *b1, double *b2) {
    if (!c || !o || !d || !prim) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        if (any_hit) {
            prim[i] = trace_any(c, o + 3 * i, d + 3 * i, brute, NULL, NULL) ? 1 : -1;
        } else {
            hitrec h = trace_closest(c, o + 3 * i, d + 3 * i, brute, NULL, NULL);
            prim[i] = h.prim;
            if (t) t[i] = h.t;
            if (b1) b1[i] = h.b1;
            if (b2) b2[i] = h.b2;
        }
    }
    return 0;
}

int32_t orc_env_sample(const orc_ctx *c, double u0, double u1, double dir[3], double *pdf, int32_t *texel) {
    return env_sample(c, u0, u1, dir, pdf, texel);
}
double orc_env_pdf(const orc_ctx *c, const double dir[3]) { return env_pdf_dir(c, dir); }
int32_t orc_env_lookup(const orc_ctx *c, const double dir[3], double rgb[3]) {
    int32_t t = env_texel_of(c, dir);
    for (int ch = 0; ch < 3; ++ch) rgb[ch] = env_channel(c, t, ch);
    return t;
}

void orc_brdf_eval(const double n[3], const double wo[3], const double wi[3], const double raw[5],
                   int32_t brdf, double f[3]) {
    double m[5]; clamp_material(raw, m);
    brdf_eval_plain(n, wo, wi, m, brdf == 1, f);
}
double orc_brdf_pdf(const double n[3], const double wo[3], const double wi[3], const double raw[5], int32_t brdf) {
    double m[5]; clamp_material(raw, m);
    return mix_pdf(n, wo, wi, m, brdf == 1);
}
int32_t orc_brdf_sample(const double n[3], const double wo[3], const double raw[5], int32_t brdf,
                        const double u[3], double wi[3]) {
    double m[5]; clamp_material(raw, m);
    double t[3], b[3]; orc_frame(n, t, b);
    return mix_sample(n, t, b, wo, m, brdf == 1, u[0], u[1], u[2], wi);
}
