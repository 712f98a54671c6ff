// Kernels of the wavefront path tracer and of the adjoint path replay
// (device code plus the argument bundles the host fills).  Included by
// render.hip only.
//
// Forward (per super-chunk of samples, one persistent pool of P paths):
//   iterate: schedule (refill the pool from a global sample counter) ->
//            generate (camera rays for the new paths) ->
//            closest hit (SoA ray queue -> hit queue) ->
//            shade (surface interaction, material fetch, M-candidate RIS with a
//                   streaming weighted reservoir, shadow-ray emission,
//                   BRDF-mixture continuation, Russian roulette, wave-level
//                   ballot/prefix-sum compaction into the next queue) ->
//            shadow (any hit; unoccluded NEE added to the sample's radiance)
//   then resolve the per-sample radiance into per-pixel means.
// Backward: one thread per sample replays the path from the per-vertex tape
// (written by the forward pass, or regenerated chunk by chunk), sweeps the
// vertices in reverse and scatters material and env-texel gradients with
// global float atomics.
//
// Paper: Sec. 3 Eqs. pbr_render / incident, Sec. 4.1 Eq. restir with the
// reservoir rule of Appendix A, Sec. 4.2 Eqs. mc_indir / sec_bouce, and
// Appendix A "Visibility estimation".
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device.h"
#include "field.h"
#include "trace.h"

namespace mrs {
namespace {

// ============================================================================
// device-side argument bundles
// ============================================================================
struct IterCtr {
    uint32_t n_in;       // continuing paths entering the iteration
    uint32_t n_new;      // camera paths generated in the iteration
    uint32_t n_live;     // n_in + n_new
    uint32_t n_shadow;   // shadow rays emitted by the iteration's shade
    uint64_t gen_base;   // first sample index generated in the iteration
};
struct Sched { uint64_t next, end; };

struct SceneDev {
    const int32_t *faces;
    const float *uv, *vmat, *albedo, *rough, *metal;
    const float4 *fm;   // field mode: materials from the field pass (per pool entry in shade, per vertex in the adjoint)
    const float4 *tpack; // texture mode: per texel (albedo rgb, roughness), (metallic, -, -, -), packed per call
    int mat_mode, tw, th;
    const WideNode *nodes;   // traversal nodes
    const TriRec *tris;
    EnvTables env;
};

struct Opts {
    int B, M, Mb, rr_start, spec, background, grad_mode;
    uint32_t k0, k1;
};

struct Queue { float4 *o, *d, *t; };   // o.w = sample id, d.w = vertex k, t = throughput

struct Tape {
    float4 *hit;   // [B][S]: (b1, b2, leaf, env texel)
    float4 *y;     // [B][S]: (y, W when unoccluded else 0)
    float *rr;     // [B][S]: continuation factor, 0 = path ended
    uint64_t base; // sample index of entry 0
    uint64_t S;    // samples per vertex slice
    float4 *fm;    // field mode, when kept: [B][S] the field's output at the hit (else null)
};

struct ViewTable {
    const ViewDev *v;
    int n;
};

// ============================================================================
// small helpers
// ============================================================================
__device__ __forceinline__ int find_view(const ViewTable &vt, uint64_t g) {
    int lo = 0, hi = vt.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (vt.v[mid].sample_base <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

struct SampleId { int view; uint32_t pixel, sample; };
__device__ __forceinline__ SampleId decode(const ViewTable &vt, uint64_t g) {
    SampleId s;
    s.view = find_view(vt, g);
    const ViewDev &v = vt.v[s.view];
    uint64_t local = g - v.sample_base;
    s.pixel = (uint32_t)(local / (uint64_t)v.spp);
    s.sample = v.sample_offset + (uint32_t)(local % (uint64_t)v.spp);
    return s;
}

// pinhole camera ray in double, rounded once to float
__device__ __forceinline__ void camera_ray(const ViewDev &v, uint32_t pixel, float u0, float u1, V3 &o, V3 &d) {
    double x = (double)(pixel % (uint32_t)v.w), y = (double)(pixel / (uint32_t)v.w);
    double nx = 2.0 * (x + (double)u0) / v.w - 1.0;
    double ny = 1.0 - 2.0 * (y + (double)u1) / v.h;
    double dc[3] = {nx * v.tan_half * v.aspect, ny * v.tan_half, -1.0};
    double w[3];
    for (int r = 0; r < 3; ++r)
        w[r] = (double)v.rot[3 * r] * dc[0] + (double)v.rot[3 * r + 1] * dc[1] + (double)v.rot[3 * r + 2] * dc[2];
    double l = 1.0 / sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    d = V3{(float)(w[0] * l), (float)(w[1] * l), (float)(w[2] * l)};
    o = V3{v.org[0], v.org[1], v.org[2]};
}

struct Interp { int idx[4]; float w[4]; int n; };
struct MatRaw { V3 a; float r, mu; };

__device__ __forceinline__ int wrapi(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

// affine interpolation: equal inputs give that value exactly, so a material
// sitting on a clamp boundary stays on it (the clamp's derivative mask then
// agrees with any other evaluation order)
__device__ __forceinline__ float bary(float x0, float x1, float x2, float b1, float b2) {
    return x0 + b1 * (x1 - x0) + b2 * (x2 - x0);
}
__device__ __forceinline__ float lerpf(float a, float b, float f) { return a + f * (b - a); }
__device__ __forceinline__ float bilerp(float x00, float x10, float x01, float x11, float fx, float fy) {
    return lerpf(lerpf(x00, x10, fx), lerpf(x01, x11, fx), fy);
}

// material at a hit: per-vertex attributes by barycentrics, or bilinear
// textures (texel centres at (i + 1/2) / W, wrap) at the interpolated uv.
// ip receives the indices and the linear weights used by the adjoint.
__device__ __forceinline__ MatRaw fetch_material(const SceneDev &s, int prim, float b1, float b2, Interp &ip) {
    int v0 = s.faces[3 * prim], v1 = s.faces[3 * prim + 1], v2 = s.faces[3 * prim + 2];
    MatRaw m;
    if (s.mat_mode == MRS_MAT_VERTEX) {
        ip.n = 3;
        ip.idx[0] = v0; ip.idx[1] = v1; ip.idx[2] = v2; ip.idx[3] = v0;
        ip.w[0] = 1.0f - b1 - b2; ip.w[1] = b1; ip.w[2] = b2; ip.w[3] = 0.0f;
        const float *p0 = s.vmat + 5 * (size_t)v0, *p1 = s.vmat + 5 * (size_t)v1, *p2 = s.vmat + 5 * (size_t)v2;
        m.a = V3{bary(p0[0], p1[0], p2[0], b1, b2), bary(p0[1], p1[1], p2[1], b1, b2), bary(p0[2], p1[2], p2[2], b1, b2)};
        m.r = bary(p0[3], p1[3], p2[3], b1, b2);
        m.mu = bary(p0[4], p1[4], p2[4], b1, b2);
        return m;
    }
    // uv and the texel coordinates in double: in float, u itself is held to
    // 2^-24, which is 2.4e-4 of a texel of a 4096-wide texture, enough to move
    // a small bilinear weight by several percent of itself
    const double db1 = b1, db2 = b2;
    const double u0 = s.uv[2 * v0], u1 = s.uv[2 * v1], u2 = s.uv[2 * v2];
    const double w0 = s.uv[2 * v0 + 1], w1 = s.uv[2 * v1 + 1], w2 = s.uv[2 * v2 + 1];
    const double u = u0 + db1 * (u1 - u0) + db2 * (u2 - u0);
    const double v = w0 + db1 * (w1 - w0) + db2 * (w2 - w0);
    const double x = u * (double)s.tw - 0.5, y = v * (double)s.th - 0.5;
    const double x0 = floor(x), y0 = floor(y);
    const float fx = (float)(x - x0), fy = (float)(y - y0);
    int i0 = wrapi((int)x0, s.tw), i1 = wrapi((int)x0 + 1, s.tw);
    int j0 = wrapi((int)y0, s.th), j1 = wrapi((int)y0 + 1, s.th);
    ip.n = 4;
    ip.idx[0] = j0 * s.tw + i0; ip.w[0] = (1.0f - fx) * (1.0f - fy);
    ip.idx[1] = j0 * s.tw + i1; ip.w[1] = fx * (1.0f - fy);
    ip.idx[2] = j1 * s.tw + i0; ip.w[2] = (1.0f - fx) * fy;
    ip.idx[3] = j1 * s.tw + i1; ip.w[3] = fx * fy;
    if (s.tpack) {
        // two 16-byte loads per texel from its 32-byte record instead of five scattered ones
        const float4 t0 = s.tpack[2 * (size_t)ip.idx[0]], t1 = s.tpack[2 * (size_t)ip.idx[1]];
        const float4 t2 = s.tpack[2 * (size_t)ip.idx[2]], t3 = s.tpack[2 * (size_t)ip.idx[3]];
        const float m0 = s.tpack[2 * (size_t)ip.idx[0] + 1].x, m1 = s.tpack[2 * (size_t)ip.idx[1] + 1].x;
        const float m2 = s.tpack[2 * (size_t)ip.idx[2] + 1].x, m3 = s.tpack[2 * (size_t)ip.idx[3] + 1].x;
        m.a = V3{bilerp(t0.x, t1.x, t2.x, t3.x, fx, fy), bilerp(t0.y, t1.y, t2.y, t3.y, fx, fy),
                 bilerp(t0.z, t1.z, t2.z, t3.z, fx, fy)};
        m.r = bilerp(t0.w, t1.w, t2.w, t3.w, fx, fy);
        m.mu = bilerp(m0, m1, m2, m3, fx, fy);
        return m;
    }
    const float *a0 = s.albedo + 3 * (size_t)ip.idx[0], *a1 = s.albedo + 3 * (size_t)ip.idx[1];
    const float *a2 = s.albedo + 3 * (size_t)ip.idx[2], *a3 = s.albedo + 3 * (size_t)ip.idx[3];
    m.a = V3{bilerp(a0[0], a1[0], a2[0], a3[0], fx, fy), bilerp(a0[1], a1[1], a2[1], a3[1], fx, fy),
             bilerp(a0[2], a1[2], a2[2], a3[2], fx, fy)};
    m.r = bilerp(s.rough[ip.idx[0]], s.rough[ip.idx[1]], s.rough[ip.idx[2]], s.rough[ip.idx[3]], fx, fy);
    m.mu = bilerp(s.metal[ip.idx[0]], s.metal[ip.idx[1]], s.metal[ip.idx[2]], s.metal[ip.idx[3]], fx, fy);
    return m;
}

// field output (albedo rgb, roughness); the field's metallic is 0
__device__ __forceinline__ MatRaw field_material(float4 f) {
    MatRaw m;
    m.a = V3{f.x, f.y, f.z};
    m.r = f.w;
    m.mu = 0.0f;
    return m;
}

__device__ __forceinline__ Mat clamp_material(const MatRaw &r) {
    Mat m;
    m.a = V3{fminf(fmaxf(r.a.x, 0.0f), 1.0f), fminf(fmaxf(r.a.y, 0.0f), 1.0f), fminf(fmaxf(r.a.z, 0.0f), 1.0f)};
    m.r = fminf(fmaxf(r.r, kRoughMin), 1.0f);
    m.mu = fminf(fmaxf(r.mu, 0.0f), 1.0f);
    return m;
}

// Barycentrics (b1, b2) of the point where the ray o + t d meets the plane
// of triangle (a, b, c), in double (Moeller and Trumbore, JGT 1997).  The
// traversal's float test decides which triangle is hit; its float
// barycentrics carry a few ulps of the coordinates relative to the
// triangle's size (1e-4 for a 1e-3-wide triangle three units away), which a
// fine texture's bilinear weights then magnify.  Every consumer of a hit
// (shading, the field pass, the reuse pass) refines it the same way from the
// same ray, so they agree.  A ray parallel to the plane keeps the inputs.
__device__ __forceinline__ void refine_hit(const TriRec &tr, V3 o, V3 d, float &b1, float &b2) {
    const double ax = tr.a.x, ay = tr.a.y, az = tr.a.z;
    const double e1x = (double)tr.b.x - ax, e1y = (double)tr.b.y - ay, e1z = (double)tr.b.z - az;
    const double e2x = (double)tr.c.x - ax, e2y = (double)tr.c.y - ay, e2z = (double)tr.c.z - az;
    const double dx = d.x, dy = d.y, dz = d.z;
    const double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    const double det = e1x * px + e1y * py + e1z * pz;
    if (det == 0.0) return;
    const double inv = 1.0 / det;
    const double sx = (double)o.x - ax, sy = (double)o.y - ay, sz = (double)o.z - az;
    const double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    b1 = (float)((sx * px + sy * py + sz * pz) * inv);
    b2 = (float)((dx * qx + dy * qy + dz * qz) * inv);
}

// hit position from the leaf-order triangle and barycentrics (as surface())
__device__ __forceinline__ V3 hit_point(const TriRec *__restrict__ tris, int leaf, float b1, float b2) {
    TriRec tr = tris[leaf];
    return xyz(tr.a) * (1.0f - b1 - b2) + xyz(tr.b) * b1 + xyz(tr.c) * b2;
}

// Points of the field passes: the hits of an iteration's queue, and the
// vertices of the taped paths of an adjoint launch (slot (k - 1) n + j for
// vertex k of sample g0 + j; a vertex exists when every earlier vertex
// continued the path and its own entry is a hit).
struct PointsHits {
    const float4 *hits; const TriRec *tris; const IterCtr *ctr; int it;
    const float4 *qo, *qd;   // the iteration's rays (refined barycentrics, as in shading)
    __device__ __forceinline__ uint64_t count() const { return ctr[it].n_live; }
    __device__ __forceinline__ uint64_t gindex(uint64_t i) const { return i; }
    __device__ __forceinline__ bool get(uint64_t i, V3 &p) const {
        if (i >= count()) return false;
        const float4 h = hits[i];
        const int leaf = __float_as_int(h.w);
        if (leaf < 0) return false;
        float b1 = h.y, b2 = h.z;
        refine_hit(tris[leaf], xyz(qo[i]), xyz(qd[i]), b1, b2);
        p = hit_point(tris, leaf, b1, b2);
        return true;
    }
};

struct PointsTape {
    Tape tape; const TriRec *tris; uint64_t g0, n; int kmax;
    __host__ __device__ __forceinline__ uint64_t count() const { return (uint64_t)kmax * n; }
    __device__ __forceinline__ uint64_t gindex(uint64_t i) const { return i; }
    __device__ __forceinline__ bool get(uint64_t i, V3 &p) const {
        if (i >= count()) return false;
        const int k = (int)(i / n) + 1;
        const uint64_t col = g0 + (i - (uint64_t)(k - 1) * n) - tape.base;
        for (int kk = 1; kk < k; ++kk)
            if (!(tape.rr[(uint64_t)(kk - 1) * tape.S + col] > 0.0f)) return false;
        const float4 th = tape.hit[(uint64_t)(k - 1) * tape.S + col];
        const int leaf = __float_as_int(th.z);
        if (leaf < 0) return false;
        p = hit_point(tris, leaf, th.x, th.y);
        return true;
    }
};

struct Surf { V3 p, n; Frame F; int prim; };
__device__ __forceinline__ Surf surface(const SceneDev &s, int leaf, float b1, float b2, V3 d) {
    TriRec tr = s.tris[leaf];
    V3 a = xyz(tr.a), b = xyz(tr.b), c = xyz(tr.c);
    Surf S;
    S.prim = __float_as_int(tr.a.w);
    float b0 = 1.0f - b1 - b2;
    S.p = a * b0 + b * b1 + c * b2;
    V3 ng = normalize(cross(b - a, c - a));
    if (dot(ng, d) > 0.0f) ng = ng * -1.0f;
    S.n = ng;
    S.F = make_frame(ng);
    return S;
}

__device__ __forceinline__ V3 spawn(V3 p, V3 n) {
    float pn = fmaxf(fabsf(p.x), fmaxf(fabsf(p.y), fabsf(p.z)));
    return p + n * (1e-4f * fmaxf(1.0f, pn));
}

// ballot / prefix-sum append: one atomic per wave
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool pred) {
    uint64_t mask = __ballot(pred);
    if (mask == 0) return 0;
    int lane = __lane_id();
    int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    uint64_t below = lane == 0 ? 0ull : (mask & ((~0ull) >> (64 - lane)));
    return base + (uint32_t)__popcll(below);
}

// decision-hash events (XOR-combined per sample)
__device__ __forceinline__ uint32_t ev_vertex(uint32_t k, uint32_t prim, uint32_t sel, uint32_t cont) {
    return fnv_word(fnv_word(fnv_word(fnv_word(kFnvBasis, k), prim), sel), cont);
}
__device__ __forceinline__ uint32_t ev_miss(uint32_t k) { return fnv_word(fnv_word(kFnvBasis, k), 0xFFFFFFFFu); }
__device__ __forceinline__ uint32_t ev_nee(uint32_t k, uint32_t vis) { return fnv_word(fnv_word(kFnvBasis, k | 0x10000u), vis); }
__device__ __forceinline__ uint32_t ev_cand(uint32_t k, uint32_t s, uint32_t lobe, uint32_t tex) {
    return fnv_word(fnv_word(fnv_word(fnv_word(kFnvBasis, k | 0x20000u), s), lobe), tex);
}

// texture mode: the three texture arrays interleaved into 32-byte texel
// records, once per call (the textures are trainable inputs)
__global__ void k_pack_texels(const float *__restrict__ albedo, const float *__restrict__ rough,
                              const float *__restrict__ metal, uint64_t n, float4 *__restrict__ out) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[2 * i] = make_float4(albedo[3 * i], albedo[3 * i + 1], albedo[3 * i + 2], rough[i]);
    out[2 * i + 1] = make_float4(metal[i], 0.0f, 0.0f, 0.0f);
}

// ============================================================================
// environment tables (rebuilt every call: the env map is a trainable input)
// ============================================================================
// Row i: texel weights w_ij = mean_c max(0, L) * sin(pi (i + 1/2) / H), prefix
// sums in double, conditional CDF normalised by the row sum.
__global__ void k_env_rows(const float *__restrict__ env, int W, int H, double *__restrict__ wts,
                           double *__restrict__ cond, double *__restrict__ rowsum) {
    __shared__ double part[256];
    int i = blockIdx.x;
    double st = sin(3.14159265358979323846 * (i + 0.5) / H);
    double carry = 0.0;
    double *cr = cond + (size_t)i * (W + 1);
    if (threadIdx.x == 0) cr[0] = 0.0;
    for (int base = 0; base < W; base += 256) {
        int j = base + threadIdx.x;
        double w = 0.0;
        if (j < W) {
            const float *L = env + ((size_t)i * W + j) * 3;
            double m = (double)fmaxf(L[0], 0.0f) + (double)fmaxf(L[1], 0.0f) + (double)fmaxf(L[2], 0.0f);
            w = (m / 3.0) * st;
            wts[(size_t)i * W + j] = w;
        }
        part[threadIdx.x] = w;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {      // inclusive Hillis-Steele scan
            double v = threadIdx.x >= off ? part[threadIdx.x - off] : 0.0;
            __syncthreads();
            part[threadIdx.x] += v;
            __syncthreads();
        }
        if (j < W) cr[j + 1] = carry + part[threadIdx.x];
        double tot = part[255];
        __syncthreads();
        carry += tot;
    }
    __syncthreads();
    for (int j = threadIdx.x + 1; j <= W; j += 256) cr[j] = carry > 0.0 ? cr[j] / carry : cr[j];
    __syncthreads();
    if (threadIdx.x == 0) { cr[W] = 1.0; rowsum[i] = carry; }
}

// Marginal CDF over the rows, normalised, with marg[H] = 1 exactly, and the
// total weight in info[0].  One block of kMargThreads threads: each sums a
// contiguous run of rows, the run sums are scanned in LDS, and each thread
// then writes its rows' prefix sums (the serial loop it replaces waited on
// one load per row).
constexpr int kMargThreads = 256;
__global__ void __launch_bounds__(kMargThreads) k_env_marg(const double *__restrict__ rowsum, int H,
                                                            double *__restrict__ marg, double *__restrict__ info) {
    __shared__ double part[kMargThreads];
    const int t = threadIdx.x;
    const int chunk = (H + kMargThreads - 1) / kMargThreads;
    const int a = min(H, t * chunk), b = min(H, a + chunk);
    double s = 0.0;
    for (int i = a; i < b; ++i) s += rowsum[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kMargThreads; off <<= 1) {      // inclusive Hillis-Steele scan
        const double v = t >= off ? part[t - off] : 0.0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const double total = part[kMargThreads - 1];
    double acc = t > 0 ? part[t - 1] : 0.0;
    for (int i = a; i < b; ++i) {
        acc += rowsum[i];
        marg[i + 1] = i + 1 == H ? 1.0 : (total > 0.0 ? acc / total : acc);
    }
    if (t == 0) { marg[0] = 0.0; info[0] = total; }
}

// texel records (conditional CDF value, radiance, pdf_uv), the marginal
// intervals and the guide tables of both CDFs
__global__ void k_env_finish(const float *__restrict__ env, int W, int H, const double *__restrict__ wts,
                             const double *__restrict__ info, const double *__restrict__ marg,
                             const double *__restrict__ cond, char *__restrict__ rec, uint16_t *__restrict__ gcond,
                             int32_t *__restrict__ gmarg,
                             double2 *__restrict__ mpair, double *__restrict__ rcos, double2 *__restrict__ csphi) {
    int i = blockIdx.x;
    (void)info; (void)wts;
    if (i < H) {
        const double *cr = cond + (size_t)i * (W + 1);
        for (int j = threadIdx.x; j < W; j += blockDim.x) {
            const float *L = env + ((size_t)i * W + j) * 3;
            double t = (double)j / W;
            int lo = 0, hi = W - 1;   // smallest c with cr[c + 1] > t: the guide of cell j
            while (lo < hi) { int mid = (lo + hi) >> 1; if (cr[mid + 1] > t) hi = mid; else lo = mid + 1; }
            char *r = rec + (size_t)kEnvRecBytes * ((size_t)i * W + j);
            *(double *)r = cr[j];
            float *f = (float *)(r + 8);
            // max(0, L), a negative zero where L < 0 or NaN: the adjoint's gradient mask
            f[0] = env_store(L[0]); f[1] = env_store(L[1]); f[2] = env_store(L[2]);
            *(float *)(r + 20) = env_pdf_uv(make_double2(marg[i], marg[i + 1]), make_double2(cr[j], cr[j + 1]), W, H);
            gcond[(size_t)i * W + j] = (uint16_t)lo;
        }
        if (i == H - 1 && threadIdx.x < 4) ((int32_t *)(rec + (size_t)kEnvRecBytes * W * H))[threadIdx.x] = 0;
    } else {
        for (int t = threadIdx.x; t < H; t += blockDim.x) mpair[t] = make_double2(marg[t], marg[t + 1]);
        for (int t0 = threadIdx.x; t0 < H; t0 += blockDim.x) {
            double t = (double)t0 / H;
            int lo = 0, hi = H - 1;
            while (lo < hi) { int mid = (lo + hi) >> 1; if (marg[mid + 1] > t) hi = mid; else lo = mid + 1; }
            gmarg[t0] = lo;
        }
        // texel edges of the direction -> texel mapping
        for (int t0 = threadIdx.x; t0 <= H; t0 += blockDim.x) rcos[t0] = cospi((double)t0 / H);
        for (int t0 = threadIdx.x; t0 <= W; t0 += blockDim.x) {
            double sn, cs;
            sincospi(2.0 * (double)t0 / W - 1.0, &sn, &cs);
            csphi[t0] = make_double2(cs, sn);
        }
    }
}

// ============================================================================
// wavefront kernels
// ============================================================================
__global__ void k_fill_u32(uint32_t *__restrict__ p, size_t n, uint32_t v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_schedule(IterCtr *__restrict__ ctr, int it, Sched *__restrict__ sched, uint32_t P) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t n_in = ctr[it].n_in;
    uint64_t rem = sched->end - sched->next;
    uint32_t n_new = (uint32_t)std::min<uint64_t>(rem, (uint64_t)(P - n_in));
    ctr[it].n_new = n_new;
    ctr[it].n_live = n_in + n_new;
    ctr[it].gen_base = sched->next;
    sched->next += n_new;
}

struct GenArgs {
    ViewTable vt; Opts op; Queue q; IterCtr *ctr; int it;
    float4 *out; uint64_t out_base; uint32_t *hash;
    const float4 *prim;   // with reservoir reuse: the primary hits it traced, per sample (else null)
    float4 *hits;         // the iteration's hit records (written here for camera rays when prim is given)
};

__device__ __forceinline__ void generate_one(const GenArgs &a, const IterCtr &c, uint32_t i) {
    uint64_t g = c.gen_base + i;
    SampleId sid = decode(a.vt, g);
    Rng rng{a.op.k0, a.op.k1, sid.pixel, sid.sample, (uint32_t)sid.view};
    float4 u = rng.draw(0, 0);
    V3 o, d;
    camera_ray(a.vt.v[sid.view], sid.pixel, u.x, u.y, o, d);
    uint32_t slot = c.n_in + i;
    a.q.o[slot] = make_float4(o.x, o.y, o.z, __uint_as_float((uint32_t)g));
    a.q.d[slot] = make_float4(d.x, d.y, d.z, __int_as_float(1));
    a.q.t[slot] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
    if (a.prim) {   // the same ray's hit, already traced by the reuse pass
        const float4 p = a.prim[g];
        a.hits[slot] = make_float4(0.0f, p.x, p.y, p.z);
    }
    a.out[g - a.out_base] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (a.hash) a.hash[g - a.out_base] = 0u;
}

// Grid-stride over the iteration's new samples: the grid is sized for the
// device, not the pool, so an iteration that admits few or no samples costs a
// handful of blocks instead of pool / 256 of them.
__global__ void k_generate(GenArgs a) {
    const IterCtr c = a.ctr[a.it];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < c.n_new; i += gridDim.x * blockDim.x)
        generate_one(a, c, i);
}

struct TraceArgs {
    const WideNode *nodes; const TriRec *tris;
    Queue q; float4 *hits; IterCtr *ctr; int it;
    uint32_t *claim;      // kClaimWords zeroed claim counters
    int continuing_only;  // trace only the continuing rays (the camera rays' hits are given)
};

// persistent: launched with a fixed grid that fills the device once, held to
// 8 wavefronts per SIMD (64 VGPRs), the occupancy its grid is sized for
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_trace_closest(TraceArgs a) {
    extern __shared__ int lds_stack[];
    IterCtr &c = a.ctr[a.it];
    const uint32_t n = a.continuing_only ? c.n_in : c.n_live;
    if (blockIdx.x * blockDim.x >= n) return;
    persistent_trace<false>(
        a.nodes, a.tris, n, a.claim, lds_stack,
        [&](uint32_t i, V3 &o, V3 &d) { o = xyz(a.q.o[i]); d = xyz(a.q.d[i]); },
        [&](uint32_t i, const Hit &h, bool) {
            a.hits[i] = make_float4(h.t, h.b1, h.b2, __int_as_float(h.leaf));
        });
}

// ---------------------------------------------------------------------------
// RIS at a surface vertex (Sec. 4.1, Eq. restir): Me = M - Mb env candidates
// and Mb BRDF-mixture candidates, candidate s from Philox block (k, s),
// balance-heuristic weights p_hat / (Me q_env + Mb q_brdf), streaming
// weighted reservoir (App. A "Spatial-temporal reuse").
// ---------------------------------------------------------------------------
struct RisOut {
    float wsum, phat, cos_y, W;   // W < 0: take wsum / phat
    V3 y, fy, Ly;
    int sel, ytex;
    uint32_t hev;                 // decision-hash events of the BRDF candidates (or of the reuse)
};

// candidate s of the streaming reservoir (env candidate if kEnv)
template <bool kEnv, class MV>
__device__ __forceinline__ void ris_candidate(const EnvTables &env, const EnvBufs &eb, bool env_ok, const MV &marg,
                                              const Rng &rng, int k, int s, int Me, int Mb, const Lobe &L,
                                              const Frame &F, bool want_hash, RisOut &o) {
    float4 u = rng.draw((uint32_t)k, (uint32_t)s);
    V3 dir, wl;
    int tex;
    float4 lp;
    float qe, qb;
    if (kEnv) {
        if (!env_sample(env, eb, env_ok, marg, u.x, u.y, dir, tex, lp, qe)) return;
        wl = to_local(F, dir);
    } else {
        int lb = mix_sample(L, u.x, u.y, u.z, wl);
        if (!lb) return;
        dir = to_world(F, wl);
        tex = env_texel_of(env, dir);
        if (want_hash) o.hev ^= ev_cand((uint32_t)k, (uint32_t)s, (uint32_t)lb, (uint32_t)tex);
        lp = env_lp(eb, (uint32_t)tex);
        qe = env_pdf_dir(env_ok, dir, lp.w);
    }
    if (!(wl.z > 0.0f)) return;
    V3 f = brdf_eval_pdf(L, wl, qb);
    float phat = (lp.x * f.x + lp.y * f.y + lp.z * f.z) * (1.0f / 3.0f) * wl.z;
    float den = (float)Me * qe + (float)Mb * qb;
    if (!(phat > 0.0f) || !(den > 0.0f)) return;
    float w = phat / den;
    o.wsum += w;
    if (u.w < w / o.wsum) {
        o.sel = s; o.y = dir; o.fy = f; o.Ly = V3{lp.x, lp.y, lp.z}; o.phat = phat; o.ytex = tex; o.cos_y = wl.z;
    }
}

template <class MV>
__device__ __forceinline__ void ris_select(const EnvTables &env, const MV &marg, const Rng &rng, int k, int M, int Mb,
                                           const Lobe &L, const Frame &F, bool front, bool want_hash, RisOut &o) {
    const int Me = M - Mb;
    o.hev = 0;
    o.wsum = 0.0f; o.phat = 0.0f; o.cos_y = 0.0f; o.W = -1.0f;
    o.y = V3{0, 0, 0}; o.fy = V3{0, 0, 0}; o.Ly = V3{0, 0, 0};
    o.sel = -1; o.ytex = -1;
    if (!front) return;
    const bool env_ok = env_valid(env);
    const EnvBufs eb = env_bufs(env);
    // candidates in order s = 0 .. M - 1: the Me env candidates, then the Mb
    // BRDF ones, each kind in a loop of its own (no per-candidate branch)
    for (int s = 0; s < Me; ++s) ris_candidate<true>(env, eb, env_ok, marg, rng, k, s, Me, Mb, L, F, want_hash, o);
    for (int s = Me; s < M; ++s) ris_candidate<false>(env, eb, env_ok, marg, rng, k, s, Me, Mb, L, F, want_hash, o);
}

// A reservoir record: (y, W) and (M, decision-hash events of its own
// sample, -, -).  M = 0: no reservoir (primary miss or back-facing).
struct ResvRec { float4 yw; float4 mh; };

// the primary vertex's reused sample as an RIS result (sel 0, or -1 if empty)
__device__ __forceinline__ void reused_sample(const EnvTables &env, const Lobe &L, const Frame &F, const ResvRec &r,
                                              RisOut &o) {
    o.hev = __float_as_uint(r.mh.y);
    o.wsum = 0.0f; o.phat = 0.0f; o.cos_y = 0.0f; o.W = 0.0f;
    o.y = V3{0, 0, 0}; o.fy = V3{0, 0, 0}; o.Ly = V3{0, 0, 0};
    o.sel = -1; o.ytex = -1;
    if (!(r.yw.w > 0.0f)) return;
    const V3 y = xyz(r.yw);
    const V3 wl = to_local(F, y);
    if (!(wl.z > 0.0f)) return;
    const int tex = env_texel_of(env, y);
    const float4 lp = env_lp(env, tex);
    o.sel = 0; o.y = y; o.fy = brdf_eval(L, wl); o.Ly = V3{lp.x, lp.y, lp.z};
    o.ytex = tex; o.cos_y = wl.z; o.W = r.yw.w;
}

struct ShadeArgs {
    SceneDev s; ViewTable vt; Opts op;
    Queue q, qn; float4 *hits; IterCtr *ctr; int it;
    float4 *so, *sd, *sc;          // shadow queue: origin (w = sample), dir (w = k), contribution
    float4 *out; uint64_t out_base; uint32_t *hash;
    Tape tape; int use_tape;
    const ResvRec *resv; uint64_t resv_base;   // reuse: final reservoirs of the primary vertices (null: plain RIS)
};

constexpr int kShadeBlock = 256;

// One path vertex per thread.  A block first partitions its kShadeBlock queue
// entries so that the hits, which run the RIS loop, fill the leading
// wavefronts and the misses the trailing ones; results do not depend on
// which thread handles an entry.
// At least 4 wavefronts per SIMD (at most 128 VGPRs): the RIS loop waits on
// chains of dependent table loads, and occupancy is what hides them.
// kMargLds: the env's marginal intervals and guide (H <= kEnvLdsRows) are
// copied into LDS first, so the row search of an env candidate costs no
// vector-memory instructions.
#ifndef MRS_SHADE_WAVES
#define MRS_SHADE_WAVES 4
#endif
constexpr int kEnvLdsRows = 1024;
template <bool kMargLds>
__global__ __launch_bounds__(kShadeBlock) __attribute__((amdgpu_waves_per_eu(MRS_SHADE_WAVES))) void k_shade(ShadeArgs a) {
    __shared__ uint32_t s_idx[kShadeBlock];
    __shared__ uint32_t s_hit[kShadeBlock / 64], s_valid[kShadeBlock / 64];
    __shared__ double2 s_mpair[kMargLds ? kEnvLdsRows : 1];
    __shared__ int32_t s_gmarg[kMargLds ? kEnvLdsRows : 1];
    const uint32_t n = a.ctr[a.it].n_live;
    const uint32_t i0 = blockIdx.x * kShadeBlock;
    if (i0 >= n) return;
    if (kMargLds) {
        for (int t = threadIdx.x; t < a.s.env.H; t += kShadeBlock) {
            s_mpair[t] = a.s.env.mpair[t];
            s_gmarg[t] = a.s.env.gmarg[t];
        }
    }
    const MargView marg = kMargLds ? MargView{s_mpair, s_gmarg} : MargView{a.s.env.mpair, a.s.env.gmarg};
    {   // (the partition's barrier also publishes the LDS copy)
        const uint32_t e = i0 + threadIdx.x;
        const bool valid = e < n;
        const bool hit = valid && __float_as_int(a.hits[e].w) >= 0;
        const uint64_t mh = __ballot(hit), mv = __ballot(valid);
        const int w = threadIdx.x / 64, lane = __lane_id();
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        if (lane == 0) { s_hit[w] = (uint32_t)__popcll(mh); s_valid[w] = (uint32_t)__popcll(mv); }
        __syncthreads();
        uint32_t hits_before = 0, misses_before = 0, hits_total = 0;
        for (int q = 0; q < kShadeBlock / 64; ++q) {
            if (q < w) { hits_before += s_hit[q]; misses_before += s_valid[q] - s_hit[q]; }
            hits_total += s_hit[q];
        }
        if (hit) s_idx[hits_before + __popcll(mh & below)] = e;
        else if (valid) s_idx[hits_total + misses_before + __popcll(mv & ~mh & below)] = e;
        __syncthreads();
    }
    const bool active = threadIdx.x < n - i0;
    const uint32_t i = active ? s_idx[threadIdx.x] : 0u;
    bool emit = false, cont = false;
    float4 e_o, e_d, e_c, c_o, c_d, c_t;
    if (active) {
        float4 po = a.q.o[i], pd = a.q.d[i], pt = a.q.t[i], hr = a.hits[i];
        uint32_t g = __float_as_uint(po.w);
        int k = __float_as_int(pd.w);
        V3 d = xyz(pd), T = xyz(pt);
        int leaf = __float_as_int(hr.w);
        uint64_t ti = (uint64_t)(k - 1) * a.tape.S + (g - a.tape.base);
        uint32_t hev;
        if (leaf < 0) {
            int tex = -1;
            if (k == 1 && a.op.background == MRS_BG_ENV) {
                tex = env_texel_of(a.s.env, d);
                float4 L = env_lp(a.s.env, tex);
                a.out[g - a.out_base] = make_float4(L.x, L.y, L.z, 0.0f);
            }
            hev = ev_miss((uint32_t)k);
            if (a.use_tape) {
                a.tape.hit[ti] = make_float4(0.0f, 0.0f, __int_as_float(-1), __int_as_float(tex));
                a.tape.y[ti] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                a.tape.rr[ti] = 0.0f;
            }
        } else {
            SampleId sid = decode(a.vt, g);
            Rng rng{a.op.k0, a.op.k1, sid.pixel, sid.sample, (uint32_t)sid.view};
            float b1 = hr.y, b2 = hr.z;
            refine_hit(a.s.tris[leaf], xyz(po), d, b1, b2);
            Surf S = surface(a.s, leaf, b1, b2, d);
            Interp ip;
            Mat m = clamp_material(a.s.mat_mode == MRS_MAT_FIELD ? field_material(a.s.fm[i])
                                                                 : fetch_material(a.s, S.prim, b1, b2, ip));
            V3 wo = to_local(S.F, d * -1.0f);
            Lobe L = make_lobe(m, wo, a.op.spec);
            V3 org = spawn(S.p, S.n);
            // ---- RIS over Me env + Mb BRDF candidates, streaming WRS, or the
            // reused reservoir at the primary vertex ----
            RisOut ro;
            if (a.resv && k == 1) reused_sample(a.s.env, L, S.F, a.resv[g - a.resv_base], ro);
            else ris_select(a.s.env, marg, rng, k, a.op.M, a.op.Mb, L, S.F, wo.z > 0.0f, a.hash != nullptr, ro);
            const uint32_t hcand = ro.hev;
            const float wsum = ro.wsum, phat_y = ro.phat, cos_y = ro.cos_y;
            const V3 y = ro.y, fy = ro.fy, Ly = ro.Ly;
            const int sel = ro.sel, ytex = ro.ytex;
            float Wy = 0.0f;
            if (sel >= 0) {
                Wy = ro.W >= 0.0f ? ro.W : wsum / phat_y;
                emit = true;
                V3 cc = T * Ly * fy * (cos_y * Wy);
                e_o = make_float4(org.x, org.y, org.z, __uint_as_float(g));
                e_d = make_float4(y.x, y.y, y.z, __int_as_float(k));
                e_c = make_float4(cc.x, cc.y, cc.z, 0.0f);
            }
            // ---- continuation (BRDF mixture), Russian roulette ----
            uint32_t code = 0;
            float rrf = 0.0f;
            if (k < a.op.B) {
                code = 2;
                float4 u = rng.draw((uint32_t)k, kBlockCont);
                V3 wl;
                int lobe = wo.z > 0.0f ? mix_sample(L, u.x, u.y, u.z, wl) : 0;
                float q = 0.0f;
                V3 f = lobe ? brdf_eval_pdf(L, wl, q) : V3{0, 0, 0};
                if (lobe && q > 0.0f) {
                    V3 Tn = T * f * (wl.z / q);
                    bool alive = true;
                    rrf = 1.0f;
                    if (a.op.rr_start >= 0 && k >= a.op.rr_start) {
                        float qr = fminf(0.95f, maxc(Tn));
                        if (!(qr > 0.0f) || !(u.w < qr)) { alive = false; code = 3; rrf = 0.0f; }
                        else { Tn = Tn * (1.0f / qr); rrf = 1.0f / qr; }
                    }
                    if (alive) {
                        code = lobe == 2 ? 4 : 1;
                        cont = true;
                        V3 wn = to_world(S.F, wl);
                        c_o = make_float4(org.x, org.y, org.z, __uint_as_float(g));
                        c_d = make_float4(wn.x, wn.y, wn.z, __int_as_float(k + 1));
                        c_t = make_float4(Tn.x, Tn.y, Tn.z, 0.0f);
                    }
                }
            }
            hev = ev_vertex((uint32_t)k, (uint32_t)S.prim, (uint32_t)sel, code) ^ hcand;
            if (a.use_tape) {
                a.tape.hit[ti] = make_float4(b1, b2, __int_as_float(leaf), __int_as_float(ytex));
                a.tape.y[ti] = make_float4(y.x, y.y, y.z, Wy);
                a.tape.rr[ti] = cont ? rrf : 0.0f;
                if (a.tape.fm) a.tape.fm[ti] = a.s.fm[i];
            }
        }
        if (a.hash) a.hash[g - a.out_base] ^= hev;
    }
    // compaction: wave-aggregated appends (all lanes reach this point)
    uint32_t si = wave_append(&a.ctr[a.it].n_shadow, emit);
    if (emit) { a.so[si] = e_o; a.sd[si] = e_d; a.sc[si] = e_c; }
    uint32_t ci = wave_append(&a.ctr[a.it + 1].n_in, cont);
    if (cont) { a.qn.o[ci] = c_o; a.qn.d[ci] = c_d; a.qn.t[ci] = c_t; }
}

struct ShadowArgs {
    const WideNode *nodes; const TriRec *tris;
    float4 *so, *sd, *sc; IterCtr *ctr; int it;
    float4 *out; uint64_t out_base; uint32_t *hash;
    Tape tape; int use_tape;
};

// One shadow ray per thread.  (A persistent launch with ray replacement, as
// for closest hits, measured slower: any-hit rays are short, and each refill
// stalls the whole wavefront on the new rays' loads.)  A sample has at most
// one shadow ray per iteration, so the accumulation into its output slot
// needs no atomics.
__global__ __launch_bounds__(256) void k_trace_shadow(ShadowArgs a) {
    extern __shared__ int lds_stack[];
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.ctr[a.it].n_shadow) return;
    float4 o = a.so[i], d = a.sd[i];
    uint32_t g = __float_as_uint(o.w);
    int k = __float_as_int(d.w);
    bool occl = trace_any(a.nodes, a.tris, xyz(o), xyz(d), lds_stack);
    if (!occl) {
        float4 c = a.sc[i];
        float4 &acc = a.out[g - a.out_base];
        acc = make_float4(acc.x + c.x, acc.y + c.y, acc.z + c.z, 0.0f);
    } else if (a.use_tape) {
        a.tape.y[(uint64_t)(k - 1) * a.tape.S + (g - a.tape.base)].w = 0.0f;
    }
    if (a.hash) a.hash[g - a.out_base] ^= ev_nee((uint32_t)k, occl ? 0u : 1u);
}

struct ResolveArgs {
    ViewTable vt; const float4 *out; uint64_t out_base;
    uint64_t pix0, pix1;      // global (view-order) pixel range of the chunk
    float *image; float *dbg_rgb;
};

__device__ __forceinline__ int find_view_pix(const ViewTable &vt, uint64_t P) {
    int lo = 0, hi = vt.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (vt.v[mid].pix_base <= P) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// pixel = mean of its spp samples, summed in sample order (deterministic)
__global__ void k_resolve(ResolveArgs a) {
    uint64_t P = a.pix0 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (P >= a.pix1) return;
    const ViewDev &v = a.vt.v[find_view_pix(a.vt, P)];
    uint64_t p = P - v.pix_base;
    uint64_t g0 = v.sample_base + p * (uint64_t)v.spp - a.out_base;
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    for (int s = 0; s < v.spp; ++s) {
        float4 c = a.out[g0 + s];
        sx += c.x; sy += c.y; sz += c.z;
        if (a.dbg_rgb) {
            float *dst = a.dbg_rgb + 3 * (g0 + a.out_base + s);
            dst[0] = c.x; dst[1] = c.y; dst[2] = c.z;
        }
    }
    float inv = 1.0f / (float)v.spp;
    float *img = a.image + 3 * (uint64_t)(v.pixel_offset + (int64_t)p);
    img[0] = sx * inv; img[1] = sy * inv; img[2] = sz * inv;
}

// ============================================================================
// adjoint path replay
// ============================================================================
struct AdjArgs {
    SceneDev s; ViewTable vt; Opts op; Tape tape;
    uint64_t g0, n;
    const float *dimg;
    float *gvmat, *galb, *grough, *gmetal, *genv;   // the caller's arrays (null: not wanted)
    float *rec;            // gradient records (see below), zeroed before the first chunk
    uint32_t env_base;     // first word of the env records
    int mat_on;            // some material gradient array is wanted
    float4 *gvtx;          // field mode: dL/d(field output) per path vertex, slot (k - 1) n + j
    int field_on;          // field mode: some field gradient array is wanted
    uint64_t fm_stride;    // field mode: the field output of vertex (k, j) is s.fm[(k - 1) fm_stride + j]
};

// ---------------------------------------------------------------------------
// Gradient scatter.  The adjoint accumulates into an internal record buffer:
// one kMatRec-float record per material texel (texture mode: albedo rgb,
// roughness, metallic) or per mesh vertex (vertex mode: its five values), then
// one kEnvRec-float record per env texel (rgb).  The atomics are carried out
// past L2, one memory-side request per cache line an instruction touches, so
// a wavefront never issues its lanes' values as they come.  Per flush it
// takes one of two forms, the same for all its lanes:
//  - merged, when neighbouring lanes share records (the spp samples of a pixel
//    and the pixels of a row at the primary vertex of a fine texture): the
//    lanes sum their values per record in an LDS hash table (open addressing,
//    keyed by the record's first word), and the wavefront then issues one
//    atomic per distinct record word, a record's words from adjacent lanes;
//  - staged, otherwise (deeper vertices, textures coarser than the pixels):
//    the lanes write their (offset, value) pairs to LDS, lane after lane, and
//    the wavefront issues them transposed, a few lanes' consecutive record
//    words per instruction; merging would cost LDS round trips for nothing.
// k_grad_fold then adds the records into the caller's arrays.
// ---------------------------------------------------------------------------
constexpr int kMatRec = 8, kEnvRec = 4;
constexpr int kMatChannels = 5;      // albedo rgb, roughness, metallic per interpolation entry
constexpr int kEnvChannels = 3;      // rgb per env texel
constexpr int kEntriesPerFlush = 2;  // interpolation entries a lane adds per flush
constexpr int kScatSlots = 13;       // staged form: pairs a lane stages per flush
constexpr int kAggBits = 8;
constexpr int kAggSlots = 1 << kAggBits;   // merged form: hash slots per wavefront
constexpr uint32_t kAggEmpty = 0xFFFFFFFFu;
constexpr int kAdjBlock = 64;
// The largest flush of a lane: kEntriesPerFlush material records and one env
// record.  The staged form drops pairs past kScatSlots and the merged form
// needs free slots to end its probing, so these bounds keep the scatter lossless.
static_assert(kScatSlots >= kEntriesPerFlush * kMatChannels + kEnvChannels,
              "a flush stages more pairs than a lane has slots");
static_assert(64 * (kEntriesPerFlush + 1) <= kAggSlots * 3 / 4, "a flush can fill the hash table");
static_assert(kAggSlots % 64 == 0, "slots are cleared and compacted 64 at a time");
// LDS words per wavefront: the two forms share one region
constexpr int kStageWords = 64 * kScatSlots * 2 + 64;
constexpr int kAggWords = kAggSlots * (2 + kMatChannels);
constexpr int kScatWords = kStageWords > kAggWords ? kStageWords : kAggWords;

struct WaveScatter {
    uint32_t *lds;       // this wavefront's kScatWords words
    float *rec;
    uint32_t env_base;   // first word of the env records
    uint32_t lane;
    bool merge;          // form of the current flush (wavefront-uniform)
    bool clean;          // the hash table is empty (no staged flush since it was cleared)
    int n;               // staged form: pairs staged by this lane

    // staged form: [64][kScatSlots] offsets, values, [64] counts
    __device__ __forceinline__ uint32_t *s_off() { return lds; }
    __device__ __forceinline__ float *s_val() { return (float *)(lds + 64 * kScatSlots); }
    __device__ __forceinline__ int *s_cnt() { return (int *)(lds + 2 * 64 * kScatSlots); }
    // merged form: [kAggSlots] keys, [kAggSlots][kMatChannels] sums, [kAggSlots] compacted slots
    __device__ __forceinline__ uint32_t *h_key() { return lds; }
    __device__ __forceinline__ float *h_val() { return (float *)(lds + kAggSlots); }
    __device__ __forceinline__ uint32_t *h_list() { return lds + kAggSlots * (1 + kMatChannels); }

    __device__ __forceinline__ static void sync() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // Picks the form of the next flushes from each lane's first material
    // record and env record (kAggEmpty: none): merged when at least a quarter
    // of the lanes with a record share one with the lane before them.
    __device__ __forceinline__ void begin(uint32_t kmat, uint32_t kenv) {
        const uint32_t pm = __shfl_up(kmat, 1), pe = __shfl_up(kenv, 1);
        const bool same = lane > 0 && ((kmat != kAggEmpty && kmat == pm) || (kenv != kAggEmpty && kenv == pe));
        const int nsame = __popcll(__ballot(same));
        const int nact = __popcll(__ballot(kmat != kAggEmpty || kenv != kAggEmpty));
        merge = nact > 0 && 4 * nsame >= nact;
        if (merge && !clean) {
            for (uint32_t s = lane; s < (uint32_t)kAggSlots; s += 64) {
                h_key()[s] = kAggEmpty;
#pragma unroll
                for (int c = 0; c < kMatChannels; ++c) h_val()[s * kMatChannels + c] = 0.0f;
            }
            sync();
            clean = true;
        }
        if (!merge) clean = false;
    }
    // adds scale * g[c] to word c of the record at word offset `base` (zeros
    // are dropped; the products are formed where they are used, so that they
    // need no registers across the slot search)
    template <int NCH>
    __device__ __forceinline__ void add(uint32_t base, float scale, const float (&g)[NCH]) {
        if (!merge) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const float v = scale * g[c];
                if (v == 0.0f || n >= kScatSlots) continue;
                s_off()[lane * kScatSlots + n] = base + c;
                s_val()[lane * kScatSlots + n] = v;
                ++n;
            }
            return;
        }
        bool any = false;
#pragma unroll
        for (int c = 0; c < NCH; ++c) any |= scale * g[c] != 0.0f;
        if (!any) return;
        uint32_t h = (base * 2654435761u) >> (32 - kAggBits);   // multiplicative (Fibonacci) hashing
        int p = 0;
        for (; p < kAggSlots; ++p) {
            const uint32_t old = atomicCAS(h_key() + h, kAggEmpty, base);
            if (old == kAggEmpty || old == base) break;
            h = (h + 1) & (kAggSlots - 1);
        }
        if (p == kAggSlots) {                      // not reached (the table is never full)
#pragma unroll
            for (int c = 0; c < NCH; ++c)
                if (scale * g[c] != 0.0f) atomicAdd(rec + base + c, scale * g[c]);
            return;
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const float v = scale * g[c];
            if (v != 0.0f) atomicAdd(h_val() + h * kMatChannels + c, v);
        }
    }
    // issues what the flush holds; all lanes of the wavefront call it together
    __device__ __forceinline__ void flush() {
        if (!merge) {
            s_cnt()[lane] = n;
            sync();
#pragma unroll 1
            for (int j = 0; j < kScatSlots; ++j) {
                const uint32_t e = j * 64 + lane, src = e / kScatSlots, r = e - src * kScatSlots;
                if ((int)r < s_cnt()[src]) atomicAdd(rec + s_off()[e], s_val()[e]);
            }
            sync();
            n = 0;
            return;
        }
        sync();
        // compact the taken slots, material records first (kMatChannels words
        // each), then env records (kEnvChannels words each)
        uint32_t nm = 0, total = 0;
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
            for (int r = 0; r < kAggSlots / 64; ++r) {
                const uint32_t s = r * 64 + lane, k = h_key()[s];
                const bool take = k != kAggEmpty && ((k < env_base) == (pass == 0));
                const uint64_t m = __ballot(take);
                if (take) h_list()[total + __popcll(m & ((1ull << lane) - 1))] = s;
                total += (uint32_t)__popcll(m);
            }
            if (pass == 0) nm = total;
        }
        sync();
        const uint32_t wm = nm * kMatChannels, np = wm + (total - nm) * kEnvChannels;
        for (uint32_t e = lane; e < np; e += 64) {
            uint32_t i, c;
            if (e < wm) { i = e / kMatChannels; c = e - i * kMatChannels; }
            else { const uint32_t q = (e - wm) / kEnvChannels; c = e - wm - q * kEnvChannels; i = nm + q; }
            const uint32_t s = h_list()[i];
            const float v = h_val()[s * kMatChannels + c];
            if (v != 0.0f) atomicAdd(rec + h_key()[s] + c, v);
        }
        sync();
        for (uint32_t i = lane; i < total; i += 64) {
            const uint32_t s = h_list()[i];
            h_key()[s] = kAggEmpty;
#pragma unroll
            for (int c = 0; c < kMatChannels; ++c) h_val()[s * kMatChannels + c] = 0.0f;
        }
        sync();
    }
};

// Deterministic form of the scatter: each sample writes its (record word,
// value) pairs, in the order it produces them, to kPairsPerVertex * B slots
// of its own; a stable sort by word and ordered sums (k_det_sum) then add
// them up in sample order, so the gradients do not depend on the order in
// which atomics land.  Unused slots keep the key kAggEmpty.
constexpr int kPairsPerVertex = 2 * kEntriesPerFlush * kMatChannels + kEnvChannels;
struct PairSink {
    uint32_t *key;   // this sample's slots
    float *val;
    int cap, n;
    __device__ __forceinline__ void begin(uint32_t, uint32_t) {}
    template <int NCH>
    __device__ __forceinline__ void add(uint32_t base, float scale, const float (&g)[NCH]) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const float v = scale * g[c];
            if (v == 0.0f || n >= cap) continue;
            key[n] = base + c;
            val[n] = v;
            ++n;
        }
    }
    __device__ __forceinline__ void flush() {}
};

// material records of interpolation entries q0 and q1 (those that exist)
template <class Sink>
__device__ __forceinline__ void put_material(Sink &ws, const Interp &ip, int q0, const float (&gm)[kMatChannels]) {
#pragma unroll
    for (int q = q0; q < q0 + kEntriesPerFlush && q < ip.n; ++q) {   // unrolled: ip stays in registers
        const float w = ip.w[q];
        if (w == 0.0f) continue;
        ws.add(kMatRec * (uint32_t)ip.idx[q], w, gm);
    }
}

// Detached-sampling gradient of one sample: with directions, selections and
// all pdf / reservoir weights held fixed, C = sum_k T_k (.) D_k and
// T_{k+1} = T_k (.) beta_k, so dC/dm_k = T_k (.) (dD_k/dm_k + dbeta_k/dm_k (.) Li_{k+1})
// with Li_k = D_k + beta_k (.) Li_{k+1} accumulated from the last vertex back.
// The vertex loop of the scatter runs in step across the wavefront.
template <class Sink>
__device__ __forceinline__ void adjoint_sample(const AdjArgs &a, bool valid, uint64_t j, Sink &ws) {
    const int B = a.op.B;
    uint64_t g = a.g0 + j;
    V3 gp = V3{0, 0, 0};
    bool live = false;
    Rng rng{a.op.k0, a.op.k1, 0, 0, 0};
    V3 o, d;
    if (valid) {
        SampleId sid = decode(a.vt, g);
        const ViewDev &vw = a.vt.v[sid.view];
        rng = Rng{a.op.k0, a.op.k1, sid.pixel, sid.sample, (uint32_t)sid.view};
        const float *gi = a.dimg + 3 * (uint64_t)(vw.pixel_offset + (int64_t)sid.pixel);
        float inv_spp = 1.0f / (float)vw.spp;
        gp = V3{gi[0] * inv_spp, gi[1] * inv_spp, gi[2] * inv_spp};
        live = !(gp.x == 0.0f && gp.y == 0.0f && gp.z == 0.0f);
        if (live) {
            float4 u = rng.draw(0, 0);
            camera_ray(vw, sid.pixel, u.x, u.y, o, d);
        }
    }
    V3 Dk[MRS_MAX_BOUNCES], Bk[MRS_MAX_BOUNCES], Lk[MRS_MAX_BOUNCES], dk[MRS_MAX_BOUNCES];
    int nv = 0;
    int miss_tex = -1;    // env texel of a primary miss
    // pass 1: per-vertex direct term D_k and continuation weight beta_k
    for (int k = 1; live && k <= B; ++k) {
        uint64_t ti = (uint64_t)(k - 1) * a.tape.S + (g - a.tape.base);
        float4 th = a.tape.hit[ti];
        int leaf = __float_as_int(th.z);
        if (leaf < 0) {
            if (k == 1) miss_tex = __float_as_int(th.w);
            break;
        }
        dk[k - 1] = d;
        Surf S = surface(a.s, leaf, th.x, th.y, d);
        Interp ip;
        Mat m = clamp_material(a.s.mat_mode == MRS_MAT_FIELD ? field_material(a.s.fm[(uint64_t)(k - 1) * a.fm_stride + j])
                                                             : fetch_material(a.s, S.prim, th.x, th.y, ip));
        Lobe L = make_lobe(m, to_local(S.F, d * -1.0f), a.op.spec);
        float4 ty = a.tape.y[ti];
        V3 D = V3{0, 0, 0};
        if (ty.w > 0.0f) {
            V3 yl = to_local(S.F, xyz(ty));
            V3 f = brdf_eval(L, yl);
            float4 lp = env_lp(a.s.env, __float_as_int(th.w));
            D = V3{lp.x, lp.y, lp.z} * f * (yl.z * ty.w);
        }
        Dk[k - 1] = D;
        Bk[k - 1] = V3{0, 0, 0};
        nv = k;
        float rr = a.tape.rr[ti];
        if (!(rr > 0.0f) || k == B) break;
        float4 uc = rng.draw((uint32_t)k, kBlockCont);
        V3 wl;
        mix_sample(L, uc.x, uc.y, uc.z, wl);
        float q;
        V3 fc = brdf_eval_pdf(L, wl, q);
        if (!(q > 0.0f)) break;
        Bk[k - 1] = fc * (wl.z / q * rr);
        d = to_world(S.F, wl);
    }
    // suffix radiance Li_{k+1}
    V3 Li = V3{0, 0, 0};
    for (int k = nv; k >= 1; --k) {
        Lk[k - 1] = Li;
        Li = Dk[k - 1] + Bk[k - 1] * Li;
    }
    // pass 2: local derivatives, scattered through interpolation weights
    V3 T = V3{1, 1, 1};
    for (int k = 1; k <= B; ++k) {
        const bool has = live && k <= nv && !(a.op.grad_mode == MRS_GRAD_PRIMARY && k > 1);
        const bool miss = live && k == 1 && miss_tex >= 0;
        if (__ballot(has || miss) == 0) break;
        float gm[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        Interp ip;
        ip.n = 0;
        int etex = miss ? miss_tex : -1;
        V3 ge = gp;
        float4 elp = make_float4(0.0f, 0.0f, 0.0f, 0.0f);   // record of etex (its radiance signs mask the gradient)
        if (has) {
            uint64_t ti = (uint64_t)(k - 1) * a.tape.S + (g - a.tape.base);
            float4 th = a.tape.hit[ti];
            int leaf = __float_as_int(th.z);
            V3 dd = dk[k - 1];
            Surf S = surface(a.s, leaf, th.x, th.y, dd);
            const bool field = a.s.mat_mode == MRS_MAT_FIELD;
            MatRaw raw = field ? field_material(a.s.fm[(uint64_t)(k - 1) * a.fm_stride + j])
                               : fetch_material(a.s, S.prim, th.x, th.y, ip);
            Mat m = clamp_material(raw);
            Lobe L = make_lobe(m, to_local(S.F, dd * -1.0f), a.op.spec);
            V3 ga = V3{0, 0, 0};
            float gr = 0.0f, gmu = 0.0f;
            V3 w = gp * T;   // dL/dC weighted by throughput
            float4 ty = a.tape.y[ti];
            if (ty.w > 0.0f) {
                V3 yl = to_local(S.F, xyz(ty));
                int tex = __float_as_int(th.w);
                float4 lp = env_lp(a.s.env, tex);
                elp = lp;
                V3 Lv = V3{lp.x, lp.y, lp.z};
                float cw = yl.z * ty.w;
                BrdfGrad bg = brdf_grad(L, m, yl);
                V3 wl = w * Lv * cw;
                ga = ga + wl * bg.da;
                gr += dot(wl, bg.dr);
                gmu += dot(wl, bg.dmu);
                etex = tex;
                ge = w * brdf_eval(L, yl) * cw;
            }
            if (k < nv) {
                float rr = a.tape.rr[ti];
                float4 uc = rng.draw((uint32_t)k, kBlockCont);
                V3 wl;
                mix_sample(L, uc.x, uc.y, uc.z, wl);
                float q = mix_pdf(L, wl);
                if (q > 0.0f) {
                    BrdfGrad bg = brdf_grad(L, m, wl);
                    V3 wb = w * Lk[k - 1] * (wl.z / q * rr);
                    ga = ga + wb * bg.da;
                    gr += dot(wb, bg.dr);
                    gmu += dot(wb, bg.dmu);
                }
            }
            // clamp masks (the derivative passes on the closed interval) and
            // the arrays the caller wants
            const bool vertex = a.s.mat_mode == MRS_MAT_VERTEX;
            const bool alb = field ? a.field_on != 0 : vertex ? a.gvmat != nullptr : a.galb != nullptr;
            const bool rgh = field ? a.field_on != 0 : vertex ? a.gvmat != nullptr : a.grough != nullptr;
            const bool mtl = field ? false : vertex ? a.gvmat != nullptr : a.gmetal != nullptr;
            gm[0] = (alb && raw.a.x >= 0.0f && raw.a.x <= 1.0f) ? ga.x : 0.0f;
            gm[1] = (alb && raw.a.y >= 0.0f && raw.a.y <= 1.0f) ? ga.y : 0.0f;
            gm[2] = (alb && raw.a.z >= 0.0f && raw.a.z <= 1.0f) ? ga.z : 0.0f;
            gm[3] = (rgh && raw.r >= kRoughMin && raw.r <= 1.0f) ? gr : 0.0f;
            gm[4] = (mtl && raw.mu >= 0.0f && raw.mu <= 1.0f) ? gmu : 0.0f;
            if (field && a.field_on) a.gvtx[(uint64_t)(k - 1) * a.n + j] = make_float4(gm[0], gm[1], gm[2], gm[3]);
            T = T * Bk[k - 1];
        }
        // group 1: interpolation entries 0 and 1, and the env texel
        static_assert(kEntriesPerFlush == 2, "the two groups below cover the four bilinear entries");
        const bool env_rec = etex >= 0 && a.genv;
        ws.begin(has && a.mat_on && ip.n > 0 ? kMatRec * (uint32_t)ip.idx[0] : kAggEmpty,
                 env_rec ? a.env_base + kEnvRec * (uint32_t)etex : kAggEmpty);
        if (has && a.mat_on) put_material(ws, ip, 0, gm);
        if (env_rec) {
            if (!has) elp = env_lp(a.s.env, etex);   // a camera ray's miss
            const float v[kEnvChannels] = {signbit(elp.x) ? 0.0f : ge.x, signbit(elp.y) ? 0.0f : ge.y,
                                           signbit(elp.z) ? 0.0f : ge.z};
            ws.add(a.env_base + kEnvRec * (uint32_t)etex, 1.0f, v);
        }
        ws.flush();
        // group 2: interpolation entries 2 and 3
        if (has && a.mat_on) put_material(ws, ip, kEntriesPerFlush, gm);
        ws.flush();
    }
}

// one thread per sample, every lane in the vertex loop of the scatter
__global__ void __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(4))) k_adjoint(AdjArgs a) {
    __shared__ uint32_t s_scat[kAdjBlock / 64 * kScatWords];
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);   // wavefront-uniform
    WaveScatter ws{s_scat + w * kScatWords, a.rec, a.env_base, (uint32_t)__lane_id(), false, false, 0};
    uint64_t j = blockIdx.x * (uint64_t)kAdjBlock + threadIdx.x;
    adjoint_sample(a, j < a.n, j, ws);
}

// deterministic mode: one thread per sample, its pairs to keys / vals (see PairSink)
__global__ void __launch_bounds__(kAdjBlock) k_adjoint_det(AdjArgs a, uint32_t *keys, float *vals) {
    const uint64_t j = blockIdx.x * (uint64_t)kAdjBlock + threadIdx.x;
    const int cap = kPairsPerVertex * a.op.B;
    const uint64_t slot = j < a.n ? j : 0;   // lanes past the end add nothing
    PairSink ps{keys + slot * cap, vals + slot * cap, cap, 0};
    adjoint_sample(a, j < a.n, j, ps);
}

// Ordered sums over the pairs sorted (stably) by record word: the first pair
// of each run of equal words adds the run, in its sorted order, which is
// sample order, to the record.  Each word has one run, so no atomics.
__global__ void k_det_sum(const uint32_t *__restrict__ key, const float *__restrict__ val, uint64_t n,
                          float *__restrict__ rec) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = key[i];
    if (k == kAggEmpty || (i > 0 && key[i - 1] == k)) return;
    float sum = 0.0f;
    for (uint64_t q = i; q < n && key[q] == k; ++q) sum += val[q];
    rec[k] += sum;
}

// adds the gradient records into the caller's arrays, one record per thread
struct FoldArgs {
    const float *rec;
    uint32_t n_mat, n_env, env_base;
    int vertex_mode;
    float *gvmat, *galb, *grough, *gmetal, *genv;
};

__global__ void k_grad_fold(FoldArgs f) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i < f.n_mat) {
        const float4 r0 = *(const float4 *)(f.rec + kMatRec * i);
        const float r4 = f.rec[kMatRec * i + 4];
        if (f.vertex_mode) {
            if (f.gvmat) {
                float *p = f.gvmat + 5 * i;
                p[0] += r0.x; p[1] += r0.y; p[2] += r0.z; p[3] += r0.w; p[4] += r4;
            }
        } else {
            if (f.galb) { float *p = f.galb + 3 * i; p[0] += r0.x; p[1] += r0.y; p[2] += r0.z; }
            if (f.grough) f.grough[i] += r0.w;
            if (f.gmetal) f.gmetal[i] += r4;
        }
    }
    if (i < f.n_env && f.genv) {
        const float4 r = *(const float4 *)(f.rec + f.env_base + kEnvRec * i);
        float *p = f.genv + 3 * i;
        p[0] += r.x; p[1] += r.y; p[2] += r.z;
    }
}

__global__ void k_trace_batch(const WideNode *__restrict__ nodes, const TriRec *__restrict__ tris,
                              const float *__restrict__ orig, const float *__restrict__ dir, int64_t n, int any,
                              float4 *__restrict__ out) {
    extern __shared__ int lds_stack[];
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    V3 o = ld3(orig + 3 * i), d = ld3(dir + 3 * i);
    if (any) {
        bool h = trace_any(nodes, tris, o, d, lds_stack);
        out[i] = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(h ? 0 : -1));
    } else {
        Hit h = trace_closest(nodes, tris, o, d, lds_stack);
        out[i] = make_float4(h.t, h.b1, h.b2, __int_as_float(h.leaf >= 0 ? h.prim : -1));
    }
}

// denoiser G-buffer: closest hit of the ray through each pixel centre
struct GbufArgs {
    const WideNode *nodes; const TriRec *tris;
    ViewTable vt; uint64_t pixels;
    float *position, *normal;
};

__global__ void k_gbuffer(GbufArgs a) {
    extern __shared__ int lds_stack[];
    const uint64_t P = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (P >= a.pixels) return;
    const ViewDev &v = a.vt.v[find_view_pix(a.vt, P)];
    const uint32_t p = (uint32_t)(P - v.pix_base);
    V3 o, d;
    camera_ray(v, p, 0.5f, 0.5f, o, d);
    Hit h = trace_closest(a.nodes, a.tris, o, d, lds_stack);
    V3 x = V3{0, 0, 0}, n = V3{0, 0, 0};
    if (h.leaf >= 0) {
        const TriRec tr = a.tris[h.leaf];
        x = o + d * h.t;
        n = normalize(cross(xyz(tr.b) - xyz(tr.a), xyz(tr.c) - xyz(tr.a)));
        if (dot(n, d) > 0.0f) n = n * -1.0f;
    }
    float *px = a.position + 3 * (uint64_t)(v.pixel_offset + (int64_t)p);
    float *pn = a.normal + 3 * (uint64_t)(v.pixel_offset + (int64_t)p);
    px[0] = x.x; px[1] = x.y; px[2] = x.z;
    pn[0] = n.x; pn[1] = n.y; pn[2] = n.z;
}

__global__ void k_set_sched(Sched *s, uint64_t a, uint64_t b) {
    if (threadIdx.x == 0 && blockIdx.x == 0) { s->next = a; s->end = b; }
}

}  // namespace
}  // namespace mrs
