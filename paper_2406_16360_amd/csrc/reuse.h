// Reservoir reuse at the primary vertices (Sec. 4.1 end; App. A "Spatial-
// temporal reuse").  Per frame (one mrs_render call), before the path
// tracer runs:
//   1. k_reuse_primary  closest hit of every sample's camera ray;
//   2. k_reuse_init     the initial RIS reservoir r0 at each primary vertex
//                       (the same candidates the path tracer would draw);
//   3. k_reuse_temporal r1 = merge(r0, previous frame's reservoir of the same
//                       sample, its confidence capped at m_cap * M);
//   4. k_reuse_spatial  r2 = merge(r1, r1 of `spatial` neighbours: same view
//                       and sample index, offsets uniform in a (2R+1)^2
//                       window without the centre, from Philox block
//                       (1, 0xFFE0 + j) by integer arithmetic).
// The path tracer then shades each primary vertex with r2's sample and
// contribution weight instead of its own RIS result.  Merging is the
// confidence-weighted combine: input i (sample y_i, contribution weight W_i,
// confidence M_i) gets resampling weight w_i = p_hat_q(y_i) W_i M_i at the
// merging vertex q, the pick follows the streaming reservoir rule with the
// input's uniform, and W = sum w / (sum M p_hat_q(y)).  The reused sample and
// its weight are sampling decisions: the adjoint holds them fixed like every
// other one (the tape records them).
#pragma once
#include "wavefront.h"

namespace mrs {
namespace {

constexpr int kReuseMaxK = 16;

struct ReuseArgs {
    SceneDev s; ViewTable vt; Opts op;
    uint64_t S;                      // samples of the frame (every view)
    float4 *prim;                    // [S] primary hit: (b1, b2, leaf bits, -)
    const float4 *fmat;              // field mode: [S] field output at the primary hit
    ResvRec *r0, *r1;                // r0 also receives r2
    const float *prev;               // nullable [S][8] previous frame (y, W, M, ...)
    float *out;                      // nullable [S][8] this frame's final reservoirs
    int spatial, radius, temporal;
    float mcap;                      // temporal confidence cap (m_cap * M)
};

__device__ __forceinline__ uint32_t ev_merge(uint32_t stage, uint32_t sel) {
    return fnv_word(fnv_word(kFnvBasis, 0x40000u | stage), sel);
}

// the primary vertex of sample g rebuilt from its stored hit: frame, lobe
// (the material from the scene, or from the field pass in field mode)
struct PrimVtx { Surf S; Lobe L; V3 wo; Rng rng; SampleId sid; };

__device__ __forceinline__ bool prim_vertex(const ReuseArgs &a, uint64_t g, PrimVtx &v) {
    const float4 ph = a.prim[g];
    const int leaf = __float_as_int(ph.z);
    if (leaf < 0) return false;
    v.sid = decode(a.vt, g);
    const ViewDev &vw = a.vt.v[v.sid.view];
    v.rng = Rng{a.op.k0, a.op.k1, v.sid.pixel, v.sid.sample, (uint32_t)v.sid.view};
    const float4 u = v.rng.draw(0, 0);
    V3 o, d;
    camera_ray(vw, v.sid.pixel, u.x, u.y, o, d);
    v.S = surface(a.s, leaf, ph.x, ph.y, d);
    Interp ip;
    const Mat m = clamp_material(a.s.mat_mode == MRS_MAT_FIELD ? field_material(a.fmat[g])
                                                               : fetch_material(a.s, v.S.prim, ph.x, ph.y, ip));
    v.wo = to_local(v.S.F, d * -1.0f);
    v.L = make_lobe(m, v.wo, a.op.spec);
    return true;
}

// p_hat at the vertex: mean over channels of L(y) f(y), times the cosine
__device__ __forceinline__ float phat_at(const EnvTables &env, const PrimVtx &v, V3 y) {
    const V3 wl = to_local(v.S.F, y);
    if (!(wl.z > 0.0f)) return 0.0f;
    const V3 f = brdf_eval(v.L, wl);
    const float4 lp = env_lp(env, env_texel_of(env, y));
    return (lp.x * f.x + lp.y * f.y + lp.z * f.z) * (1.0f / 3.0f) * wl.z;
}

struct Merge {
    float wsum = 0.0f, Msum = 0.0f, phat = 0.0f;
    V3 y = V3{0, 0, 0};
    int sel = -1, n = 0;
    __device__ __forceinline__ void add(const EnvTables &env, const PrimVtx &v, V3 yi, float Wi, float Mi, float u) {
        const int i = n++;
        if (!(Mi > 0.0f)) return;
        Msum += Mi;
        if (!(Wi > 0.0f)) return;
        const float ph = phat_at(env, v, yi);
        const float w = ph * Wi * Mi;
        if (!(w > 0.0f)) return;
        wsum += w;
        if (u < w / wsum) { sel = i; y = yi; phat = ph; }
    }
    __device__ __forceinline__ ResvRec result(uint32_t hev) const {
        ResvRec r;
        const float W = sel >= 0 ? wsum / (Msum * phat) : 0.0f;
        r.yw = make_float4(y.x, y.y, y.z, W);
        r.mh = make_float4(Msum, __uint_as_float(hev), 0.0f, 0.0f);
        return r;
    }
};

__global__ void k_reuse_primary(ReuseArgs a) {
    extern __shared__ int lds_stack[];
    const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (g >= a.S) return;
    const SampleId sid = decode(a.vt, g);
    const ViewDev &vw = a.vt.v[sid.view];
    const Rng rng{a.op.k0, a.op.k1, sid.pixel, sid.sample, (uint32_t)sid.view};
    const float4 u = rng.draw(0, 0);
    V3 o, d;
    camera_ray(vw, sid.pixel, u.x, u.y, o, d);
    const Hit h = trace_closest(a.s.nodes, a.s.tris, o, d, lds_stack);
    float b1 = h.b1, b2 = h.b2;
    if (h.leaf >= 0) refine_hit(a.s.tris[h.leaf], o, d, b1, b2);
    a.prim[g] = make_float4(b1, b2, __int_as_float(h.leaf >= 0 ? h.leaf : -1), 0.0f);
}

// kMargLds: the env's marginal intervals and guide go to LDS first, as in
// shading (H <= kEnvLdsRows), so an env candidate's row search reads LDS
template <bool kMargLds>
__global__ __launch_bounds__(256) void k_reuse_init(ReuseArgs a) {
    __shared__ double2 s_mpair[kMargLds ? kEnvLdsRows : 1];
    __shared__ int32_t s_gmarg[kMargLds ? kEnvLdsRows : 1];
    if (kMargLds) {
        for (int t = threadIdx.x; t < a.s.env.H; t += blockDim.x) {
            s_mpair[t] = a.s.env.mpair[t];
            s_gmarg[t] = a.s.env.gmarg[t];
        }
        __syncthreads();
    }
    const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (g >= a.S) return;
    PrimVtx v;
    ResvRec r;
    r.yw = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    r.mh = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (prim_vertex(a, g, v)) {
        const MargView marg = kMargLds ? MargView{s_mpair, s_gmarg} : MargView{a.s.env.mpair, a.s.env.gmarg};
        const bool front = v.wo.z > 0.0f;
        RisOut ro;
        ris_select(a.s.env, marg, v.rng, 1, a.op.M, a.op.Mb, v.L, v.S.F, front, true, ro);
        const float W = ro.sel >= 0 ? ro.wsum / ro.phat : 0.0f;
        r.yw = make_float4(ro.y.x, ro.y.y, ro.y.z, W);
        r.mh = make_float4(front ? (float)a.op.M : 0.0f, __uint_as_float(ro.hev), 0.0f, 0.0f);
    }
    a.r0[g] = r;
}

__global__ __launch_bounds__(256) void k_reuse_temporal(ReuseArgs a) {
    const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (g >= a.S) return;
    const ResvRec r0 = a.r0[g];
    PrimVtx v;
    if (!a.temporal || !a.prev || !prim_vertex(a, g, v)) {
        a.r1[g] = r0;
        return;
    }
    const float *pr = a.prev + 8 * g;
    Merge mg;
    mg.add(a.s.env, v, xyz(r0.yw), r0.yw.w, r0.mh.x, 0.0f);
    const float u = v.rng.draw(1, 0xFFD0u).x;
    mg.add(a.s.env, v, V3{pr[0], pr[1], pr[2]}, pr[3], fminf(pr[4], a.mcap), u);
    a.r1[g] = mg.result(__float_as_uint(r0.mh.y) ^ ev_merge(1u, (uint32_t)mg.sel));
}

__global__ __launch_bounds__(256) void k_reuse_spatial(ReuseArgs a) {
    const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (g >= a.S) return;
    PrimVtx v;
    ResvRec r;
    r.yw = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    r.mh = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (prim_vertex(a, g, v)) {
        const ResvRec r1 = a.r1[g];
        Merge mg;
        mg.add(a.s.env, v, xyz(r1.yw), r1.yw.w, r1.mh.x, 0.0f);
        const ViewDev &vw = a.vt.v[v.sid.view];
        const int x = (int)(v.sid.pixel % (uint32_t)vw.w), y = (int)(v.sid.pixel / (uint32_t)vw.w);
        const uint64_t side = 2 * (uint64_t)a.radius + 1;
        const uint32_t s_local = (uint32_t)((g - vw.sample_base) % (uint64_t)vw.spp);
        for (int j = 0; j < a.spatial; ++j) {
            const uint4 q = philox(make_uint4(v.sid.pixel, v.sid.sample, (uint32_t)v.sid.view,
                                              (1u << 16) | (0xFFE0u + (uint32_t)j)), a.op.k0, a.op.k1);
            const int dx = (int)(((uint64_t)q.x * side) >> 32) - a.radius;
            const int dy = (int)(((uint64_t)q.y * side) >> 32) - a.radius;
            const int xn = x + dx, yn = y + dy;
            if ((dx == 0 && dy == 0) || xn < 0 || yn < 0 || xn >= vw.w || yn >= vw.h) continue;
            const uint64_t gn = vw.sample_base + (uint64_t)(yn * vw.w + xn) * (uint64_t)vw.spp + s_local;
            if (__float_as_int(a.prim[gn].z) < 0) continue;   // a neighbour without a primary vertex is no input
            const ResvRec rn = a.r1[gn];
            mg.add(a.s.env, v, xyz(rn.yw), rn.yw.w, rn.mh.x, u01(q.z));
        }
        r = mg.result(__float_as_uint(r1.mh.y) ^ ev_merge(2u, (uint32_t)mg.sel));
    }
    a.r0[g] = r;
    if (a.out) {
        float *o = a.out + 8 * g;
        o[0] = r.yw.x; o[1] = r.yw.y; o[2] = r.yw.z; o[3] = r.yw.w;
        o[4] = r.mh.x; o[5] = 0.0f; o[6] = 0.0f; o[7] = 0.0f;
    }
}

// points of the field pass over the primary hits
struct PointsPrimary {
    const float4 *prim; const TriRec *tris; uint64_t n;
    __host__ __device__ __forceinline__ uint64_t count() const { return n; }
    __device__ __forceinline__ uint64_t gindex(uint64_t i) const { return i; }
    __device__ __forceinline__ bool get(uint64_t i, V3 &p) const {
        if (i >= n) return false;
        const float4 h = prim[i];
        const int leaf = __float_as_int(h.z);
        if (leaf < 0) return false;
        p = hit_point(tris, leaf, h.x, h.y);
        return true;
    }
};

// host: the reuse passes of one frame on stream s (fmat: the field pass's
// output buffer in field mode)
inline void launch_reuse(const ReuseArgs &ra, const FieldDev &fd, float *fmat, hipStream_t s) {
    const unsigned nb = (unsigned)((ra.S + 255) / 256);
    k_reuse_primary<<<nb, 256, kLdsStackBytes * 256, s>>>(ra);
    if (ra.s.mat_mode == MRS_MAT_FIELD) {
        PointsPrimary src{ra.prim, ra.s.tris, ra.S};
        k_field_eval<PointsPrimary><<<(unsigned)((ra.S + kFieldTile - 1) / kFieldTile), 64, 0, s>>>(fd, src, fmat);
    }
    if (ra.s.env.H <= kEnvLdsRows) k_reuse_init<true><<<nb, 256, 0, s>>>(ra);
    else k_reuse_init<false><<<nb, 256, 0, s>>>(ra);
    k_reuse_temporal<<<nb, 256, 0, s>>>(ra);
    k_reuse_spatial<<<nb, 256, 0, s>>>(ra);
}

}  // namespace
}  // namespace mrs
