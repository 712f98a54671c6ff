// Device-side building blocks of the gfx950 path tracer: Philox4x32-10,
// small vector math, the shading frame, the Lambert + GGX BRDF with its
// mixture sampler and hand-written material derivatives, environment-map
// sampling, and the internal data layouts shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mirres.h"

namespace mrs {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;
constexpr float kRoughMin = 0.05f;
constexpr float kF0Dielectric = 0.04f;
constexpr uint32_t kBlockCont = 0xFFFFu;   // Philox block of the continuation sample
constexpr int kStackSize = 160;            // traversal stack (tree depth is checked at build)
constexpr int kLeafMax = 2;                // triangles per collapsed leaf

// ----------------------------------------------------------------------------
// vector helpers
// ----------------------------------------------------------------------------
struct V3 { float x, y, z; };
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return V3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ V3 operator*(V3 a, V3 b) { return V3{a.x * b.x, a.y * b.y, a.z * b.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 normalize(V3 a) { return a * (1.0f / sqrtf(dot(a, a))); }
__device__ __forceinline__ float maxc(V3 a) { return fmaxf(a.x, fmaxf(a.y, a.z)); }
__device__ __forceinline__ float meanc(V3 a) { return (a.x + a.y + a.z) * (1.0f / 3.0f); }
__device__ __forceinline__ V3 ld3(const float *p) { return V3{p[0], p[1], p[2]}; }
__device__ __forceinline__ V3 xyz(float4 a) { return V3{a.x, a.y, a.z}; }

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round's two
// 32 x 32 -> 64-bit products are written as 64-bit multiplies, which gfx950
// issues as one v_mad_u64_u32 each instead of a mul_hi / mul_lo pair.
// ----------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

struct Rng {
    uint32_t k0, k1, pixel, sample, view;
    __device__ __forceinline__ float4 draw(uint32_t vertex, uint32_t block) const {
        uint4 r = philox(make_uint4(pixel, sample, view, (vertex << 16) | (block & 0xFFFFu)), k0, k1);
        return make_float4(u01(r.x), u01(r.y), u01(r.z), u01(r.w));
    }
};

// FNV-1a (32-bit) over little-endian words, for the per-sample decision hash
__device__ __forceinline__ uint32_t fnv_word(uint32_t h, uint32_t w) {
#pragma unroll
    for (int i = 0; i < 4; ++i) { h ^= (w >> (8 * i)) & 0xFFu; h *= 16777619u; }
    return h;
}
constexpr uint32_t kFnvBasis = 2166136261u;

// ----------------------------------------------------------------------------
// shading frame: branchless orthonormal basis (Duff et al., JCGT 2017, sign
// +1 for z >= 0) built for m = R n and mapped back with R, where
// R = (1/9)[[1,4,8],[4,7,-4],[8,-4,1]] is symmetric and orthogonal.  The
// basis switches branch on the plane 8x - 4y + z = 0 of normals, which no
// axis-aligned or mirror-symmetric face normal lies on, so float rounding of
// a face normal cannot flip the whole frame except within rounding of it.
// ----------------------------------------------------------------------------
struct Frame { V3 t, b, n; };
__device__ __forceinline__ V3 frame_r(V3 v) {
    constexpr float k = 1.0f / 9.0f;
    return V3{k * (v.x + 4.0f * v.y + 8.0f * v.z), k * (4.0f * v.x + 7.0f * v.y - 4.0f * v.z),
              k * (8.0f * v.x - 4.0f * v.y + v.z)};
}
__device__ __forceinline__ Frame make_frame(V3 n) {
    V3 m = frame_r(n);
    float sg = m.z >= 0.0f ? 1.0f : -1.0f;
    float a = -1.0f / (sg + m.z);
    float bb = m.x * m.y * a;
    Frame f;
    f.t = frame_r(V3{1.0f + sg * m.x * m.x * a, sg * bb, -sg * m.x});
    f.b = frame_r(V3{bb, sg + m.y * m.y * a, -m.y});
    f.n = n;
    return f;
}
__device__ __forceinline__ V3 to_local(const Frame &f, V3 w) { return V3{dot(w, f.t), dot(w, f.b), dot(w, f.n)}; }
__device__ __forceinline__ V3 to_world(const Frame &f, V3 l) { return f.t * l.x + f.b * l.y + f.n * l.z; }

// ----------------------------------------------------------------------------
// material and BRDF: Lambert diffuse (1 - mu) a / pi plus GGX specular
// D G1(wo) G1(wi) F / (4 cos_i cos_o), F Schlick with F0 = 0.04 (1 - mu) + mu a
// ----------------------------------------------------------------------------
struct Mat {
    V3 a;           // clamped albedo
    float r, mu;    // clamped roughness, metallic
};

struct Lobe {       // per-vertex constants of the BRDF at a fixed wo (local frame)
    V3 wo;          // local outgoing direction, wo.z = cos_o
    V3 kd;          // (1 - mu) a / pi
    V3 f0;
    float a2;       // alpha^2, alpha = r^2
    float g1o;      // Smith G1(wo)
    float pspec;    // probability of the specular lobe in the mixture sampler
    int spec;       // GGX lobe enabled
};

__device__ __forceinline__ float ggx_g1(float a2, float c) {
    float c2 = c * c;
    float t2 = fmaxf(0.0f, 1.0f - c2) / c2;
    return 2.0f / (1.0f + sqrtf(1.0f + a2 * t2));
}

__device__ __forceinline__ Lobe make_lobe(const Mat &m, V3 wo, int spec) {
    Lobe L;
    L.wo = wo;
    L.spec = spec;
    float omm = 1.0f - m.mu;
    L.kd = m.a * (omm * kInvPi);
    L.f0 = V3{kF0Dielectric * omm + m.mu * m.a.x, kF0Dielectric * omm + m.mu * m.a.y,
              kF0Dielectric * omm + m.mu * m.a.z};
    float alpha = m.r * m.r;
    L.a2 = alpha * alpha;
    L.g1o = wo.z > 0.0f ? ggx_g1(L.a2, wo.z) : 0.0f;
    if (spec) {
        float f0m = meanc(L.f0);
        float dif = omm * meanc(m.a);
        float den = f0m + dif;
        L.pspec = den > 0.0f ? fminf(fmaxf(f0m / den, 0.1f), 0.9f) : 0.5f;
    } else {
        L.pspec = 0.0f;
    }
    return L;
}

// Microfacet terms for a local wi.  den is written in the cancellation-free
// form sin^2(theta_h) + alpha^2 cos^2(theta_h) (equal to the textbook
// (n.h)^2 (alpha^2 - 1) + 1 for a unit h).
struct Micro { float D, g1i, fw, nh2, den; };
__device__ __forceinline__ Micro micro(const Lobe &L, V3 wi) {
    V3 h = normalize(wi + L.wo);
    Micro m;
    m.nh2 = h.z * h.z;
    m.den = (h.x * h.x + h.y * h.y) + L.a2 * m.nh2;
    m.D = L.a2 / (kPi * m.den * m.den);
    m.g1i = ggx_g1(L.a2, wi.z);
    float oh = fmaxf(0.0f, dot(L.wo, h));
    float x = 1.0f - oh, x2 = x * x;
    m.fw = x2 * x2 * x;
    return m;
}

__device__ __forceinline__ V3 brdf_eval(const Lobe &L, V3 wi) {
    if (!(wi.z > 0.0f) || !(L.wo.z > 0.0f)) return V3{0, 0, 0};
    V3 f = L.kd;
    if (L.spec) {
        Micro m = micro(L, wi);
        float k = m.D * L.g1o * m.g1i / (4.0f * wi.z * L.wo.z);
        f = f + V3{(L.f0.x + (1.0f - L.f0.x) * m.fw) * k, (L.f0.y + (1.0f - L.f0.y) * m.fw) * k,
                   (L.f0.z + (1.0f - L.f0.z) * m.fw) * k};
    }
    return f;
}

// f and the mixture pdf of a local wi from one microfacet evaluation
__device__ __forceinline__ V3 brdf_eval_pdf(const Lobe &L, V3 wi, float &pdf) {
    pdf = 0.0f;
    if (!(wi.z > 0.0f) || !(L.wo.z > 0.0f)) return V3{0, 0, 0};
    V3 f = L.kd;
    pdf = (1.0f - L.pspec) * wi.z * kInvPi;
    if (L.spec) {
        Micro m = micro(L, wi);
        float k = m.D * L.g1o * m.g1i / (4.0f * wi.z * L.wo.z);
        f = f + V3{(L.f0.x + (1.0f - L.f0.x) * m.fw) * k, (L.f0.y + (1.0f - L.f0.y) * m.fw) * k,
                   (L.f0.z + (1.0f - L.f0.z) * m.fw) * k};
        pdf += L.pspec * L.g1o * m.D / (4.0f * L.wo.z);
    }
    return f;
}

__device__ __forceinline__ float mix_pdf(const Lobe &L, V3 wi) {
    if (!(wi.z > 0.0f) || !(L.wo.z > 0.0f)) return 0.0f;
    float p = (1.0f - L.pspec) * wi.z * kInvPi;
    if (L.pspec > 0.0f) {
        Micro m = micro(L, wi);
        p += L.pspec * L.g1o * m.D / (4.0f * L.wo.z);
    }
    return p;
}

// GGX visible-normal sample (Heitz, JCGT 2018) for isotropic alpha, local frame.
__device__ __forceinline__ V3 vndf(V3 wo, float alpha, float u1, float u2) {
    V3 vh = normalize(V3{alpha * wo.x, alpha * wo.y, wo.z});
    float lensq = vh.x * vh.x + vh.y * vh.y;
    V3 T1 = lensq > 0.0f ? V3{-vh.y, vh.x, 0.0f} * (1.0f / sqrtf(lensq)) : V3{1.0f, 0.0f, 0.0f};
    V3 T2 = cross(vh, T1);
    float r = sqrtf(u1);
    float sp, cp;
    sincospif(2.0f * u2, &sp, &cp);   // sin, cos of 2 pi u2 (exact argument)
    float t1 = r * cp, t2 = r * sp;
    float s = 0.5f * (1.0f + vh.z);
    t2 = (1.0f - s) * sqrtf(1.0f - t1 * t1) + s * t2;
    float tz = sqrtf(fmaxf(0.0f, 1.0f - t1 * t1 - t2 * t2));
    V3 nh = T1 * t1 + T2 * t2 + vh * tz;
    return normalize(V3{alpha * nh.x, alpha * nh.y, fmaxf(0.0f, nh.z)});
}

// Mixture sampler: u0 picks the lobe, (u1, u2) the direction.  Returns the
// lobe (1 diffuse, 2 specular) or 0 when the direction is below the surface.
__device__ __forceinline__ int mix_sample(const Lobe &L, float u0, float u1, float u2, V3 &wi) {
    int lobe;
    if (u0 < L.pspec) {
        V3 h = vndf(L.wo, sqrtf(L.a2), u1, u2);
        wi = h * (2.0f * dot(L.wo, h)) - L.wo;
        lobe = 2;
    } else {
        float r = sqrtf(u1), sp, cp;
        sincospif(2.0f * u2, &sp, &cp);
        wi = V3{r * cp, r * sp, sqrtf(fmaxf(0.0f, 1.0f - u1))};
        lobe = 1;
    }
    return wi.z > 0.0f ? lobe : 0;
}

// d f_c / d(albedo_c), d f / d(roughness), d f / d(metallic) at a local wi
// (hand-written from the closed forms of D, Smith G1 and Schlick F).
struct BrdfGrad { V3 da; V3 dr; V3 dmu; };
__device__ __forceinline__ BrdfGrad brdf_grad(const Lobe &L, const Mat &m, V3 wi) {
    BrdfGrad g;
    g.da = V3{0, 0, 0}; g.dr = V3{0, 0, 0}; g.dmu = V3{0, 0, 0};
    if (!(wi.z > 0.0f) || !(L.wo.z > 0.0f)) return g;
    float omm = 1.0f - m.mu;
    g.da = V3{omm * kInvPi, omm * kInvPi, omm * kInvPi};
    g.dmu = m.a * (-kInvPi);
    if (!L.spec) return g;
    Micro mi = micro(L, wi);
    float k = mi.D * L.g1o * mi.g1i / (4.0f * wi.z * L.wo.z);
    float ofw = 1.0f - mi.fw;
    // dF_c/da_c = mu (1 - fw); dF_c/dmu = (a_c - 0.04) (1 - fw)
    g.da = g.da + V3{k * m.mu * ofw, k * m.mu * ofw, k * m.mu * ofw};
    g.dmu = g.dmu + V3{k * (m.a.x - kF0Dielectric) * ofw, k * (m.a.y - kF0Dielectric) * ofw,
                       k * (m.a.z - kF0Dielectric) * ofw};
    // d ln D / d alpha = 2/alpha - 4 alpha cos^2(theta_h) / den
    float alpha = m.r * m.r;
    float dlnD = 2.0f / alpha - 4.0f * alpha * mi.nh2 / mi.den;
    // d ln G1 / d alpha = -alpha t2 / (R (1 + R)), R = sqrt(1 + alpha^2 t2)
    float co2 = L.wo.z * L.wo.z, ci2 = wi.z * wi.z;
    float to2 = fmaxf(0.0f, 1.0f - co2) / co2, ti2 = fmaxf(0.0f, 1.0f - ci2) / ci2;
    float Ro = sqrtf(1.0f + L.a2 * to2), Ri = sqrtf(1.0f + L.a2 * ti2);
    float dlnG = -alpha * to2 / (Ro * (1.0f + Ro)) - alpha * ti2 / (Ri * (1.0f + Ri));
    float dk = k * (dlnD + dlnG) * 2.0f * m.r;     // d alpha / d r = 2 r
    g.dr = V3{(L.f0.x + (1.0f - L.f0.x) * mi.fw) * dk, (L.f0.y + (1.0f - L.f0.y) * mi.fw) * dk,
              (L.f0.z + (1.0f - L.f0.z) * mi.fw) * dk};
    return g;
}

// ----------------------------------------------------------------------------
// environment map (equirectangular, +y up): theta = acos(d_y),
// phi = atan2(d_x, -d_z), u = phi / 2pi + 1/2, v = theta / pi; nearest texel
// ----------------------------------------------------------------------------
// The normalised marginal CDF is stored as intervals, entry i = (cdf[i],
// cdf[i + 1]), so one aligned 16-byte load gives both ends of a bin; the
// conditional CDFs sit in the texel records, one value per texel.
struct EnvTables {
    const double2 *mpair;   // [H] marginal CDF over rows, as intervals
    // [H][W] 24-byte texel records (layout at env_rec): the row's conditional
    // CDF at the texel's column, the radiance and the texel's sampling
    // density.  A BRDF candidate reads radiance and density with one 16-byte
    // load; an env candidate's walk reads interval, radiance and density
    // together.  The table is three quarters the size of one that stores both
    // interval ends.
    const char *rec;
    // [H][W] guides of the conditional CDFs: g[i][c] is the first column of
    // row i whose bin ends above c / W (16 bits: W <= 65536).  Env candidates
    // read them at uniformly spread cells, so their size counts.
    const uint16_t *gcond;
    const int32_t *gmarg;   // [H] guide: first candidate row for u0 in [t/H, (t+1)/H)
    int W, H;
    const double *total;    // device: total sampling weight (no valid sample when 0)
    const double *rcos;     // [H + 1] cos(i pi / H): the direction's y at the edge above row i
    const double2 *csphi;   // [W + 1] (cos, sin) of phi_j = pi (2 j / W - 1): the edge left of column j
};

// the marginal intervals and guide, from the tables or from a copy in LDS
struct MargView {
    const double2 *pair;
    const int32_t *guide;
};

// Nearest texel of direction d.  theta is atan2(sin theta, d_y) with
// sin theta = sqrt(d_x^2 + d_z^2): acos(d_y) (and 1 - d_y^2) lose most of
// their digits to cancellation near the poles.  The float mapping decides,
// except within kTexEdge of a texel width from a row or column edge: there
// the float value of u W or v H (atan2f and the scaling round it by up to
// ~1e-4 of a texel width) can land on the wrong side, so the side is settled
// in double against the edge itself.  theta >= i pi / H iff d_y <= cos(i pi / H), and
// phi >= phi_j iff d_x cos(phi_j) + d_z sin(phi_j) >= 0 (phi = atan2(d_x,
// -d_z) within pi of phi_j, which holds next to the float estimate).  The
// seam at phi = +-pi and the poles keep the clamped float estimate.
constexpr float kTexEdge = 2e-3f;
__device__ __forceinline__ int env_texel_of(const EnvTables &e, V3 d) {
    float dy = fminf(fmaxf(d.y, -1.0f), 1.0f);
    float theta = atan2f(sqrtf(d.x * d.x + d.z * d.z), d.y), phi = atan2f(d.x, -d.z);
    float x = (phi * (0.5f * kInvPi) + 0.5f) * (float)e.W, v = theta * kInvPi * (float)e.H;
    float fx = floorf(x), fv = floorf(v);
    float rx = x - fx, rv = v - fv;
    int col = min(max((int)fx, 0), e.W - 1), row = min(max((int)fv, 0), e.H - 1);
    if (rx < kTexEdge || rx > 1.0f - kTexEdge) {
        int j = (int)fx + (rx < 0.5f ? 0 : 1);    // the nearest column edge
        if (j > 0 && j < e.W) {
            const double2 cs = e.csphi[j];
            col = ((double)d.x * cs.x + (double)d.z * cs.y >= 0.0) ? j : j - 1;
        }
    }
    if (rv < kTexEdge || rv > 1.0f - kTexEdge) {
        int i = (int)fv + (rv < 0.5f ? 0 : 1);    // the nearest row edge
        if (i > 0 && i < e.H) row = ((double)dy <= e.rcos[i]) ? i : i - 1;
    }
    return row * e.W + col;
}

// whether the env sampler has any valid sample (read once per vertex by the
// callers, so that the loads inside a candidate loop are not split by it)
__device__ __forceinline__ bool env_valid(const EnvTables &e) { return *e.total > 0.0; }

// density of the env sampler over the unit square of texel coordinates,
// divided by 2 pi^2: row probability x column probability x W H / (2 pi^2),
// from the marginal interval pm of the row and the conditional interval pc
// of the texel
__device__ __forceinline__ float env_pdf_uv(double2 pm, double2 pc, int W, int H) {
    return (float)((pm.y - pm.x) * (pc.y - pc.x) * ((double)W * (double)H * 0.050660591821168885));
}

// solid-angle pdf of the env sampler at direction d, from the pdf_uv / (2 pi^2)
// of its texel; ok = env_valid(e)
__device__ __forceinline__ float env_pdf_dir(bool ok, V3 d, float puv) {
    if (!ok) return 0.0f;
    float st = sqrtf(d.x * d.x + d.z * d.z);   // sin theta without the cancellation of 1 - d_y^2 near the poles
    return st > 0.0f ? puv / st : 0.0f;
}

// 16-byte loads through a raw buffer resource over [base, base + bytes) (base
// and bytes uniform over the wavefront).  The compiler keeps each one a single
// buffer_load_dwordx4: from a plain pointer it splits a 16-byte record into
// narrower loads when its words are used on different paths, and every extra
// scattered load instruction costs the memory pipeline one more cycle per
// distinct cache line.  Offsets need only be 4-byte aligned.  An offset at or
// past the end reads zeros.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

// 24-byte texel records: texel t at byte 24 t holds cdf[j] (double, the
// row's conditional CDF at its column j), L_r, L_g, L_b (env_store) and
// env_pdf_uv of the texel (float, from its row's marginal interval and its
// conditional interval); the upper end cdf[j + 1] is the next record's first
// word, and 1 after a row's last texel (the build sets the row's last CDF
// value to exactly 1).  16 bytes of padding follow the last record, so that
// the second load of the last record stays in the buffer.  env_lp returns
// (L_r, L_g, L_b, pdf_uv).
constexpr uint32_t kEnvRecBytes = 24u;
// a radiance channel as the records hold it: max(0, L), where L < 0 or NaN
// gives a negative zero.  Its sign bit is then the adjoint's mask (the
// derivative of max(0, L) is taken as 1 for L >= 0), so the adjoint needs
// no read of the caller's env.
__device__ __forceinline__ float env_store(float L) { return L >= 0.0f ? L + 0.0f : -0.0f; }
__device__ __forceinline__ float4 env_lp(const EnvTables &e, int t) {
    return *(const float4 *)((const char *)e.rec + (size_t)kEnvRecBytes * t + 8);
}

// the env's texel records as a buffer resource (W H < 2^27 texels, so the
// byte offsets fit in 32 bits)
struct EnvBufs {
    __amdgpu_buffer_rsrc_t rec;
    int W;
};
__device__ __forceinline__ EnvBufs env_bufs(const EnvTables &e) {
    const uint32_t bytes = (uint32_t)e.W * (uint32_t)e.H * kEnvRecBytes + 16u;
    return EnvBufs{buffer_rsrc(e.rec, bytes), e.W};
}
__device__ __forceinline__ float4 env_lp(const EnvBufs &eb, uint32_t t) {
    const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(eb.rec, kEnvRecBytes * t + 8u, 0, 0);
    return make_float4(__uint_as_float(q.x), __uint_as_float(q.y), __uint_as_float(q.z), __uint_as_float(q.w));
}
// the whole record of texel t (column j of its row): its CDF interval, and
// its radiance and pdf_uv as env_lp returns them
__device__ __forceinline__ void env_rec(const EnvBufs &eb, uint32_t t, int j, double2 &iv, float4 &lp) {
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(eb.rec, kEnvRecBytes * t, 0, 0);
    const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(eb.rec, kEnvRecBytes * t + 16u, 0, 0);
    iv = make_double2(__hiloint2double((int)a.y, (int)a.x),
                      j == eb.W - 1 ? 1.0 : __hiloint2double((int)b.w, (int)b.z));
    lp = make_float4(__uint_as_float(a.z), __uint_as_float(a.w), __uint_as_float(b.x), __uint_as_float(b.y));
}

// smallest i with cdf[i + 1] > u (cdf[0] = 0 <= u < 1 = cdf[n]): the unique i
// with cdf[i] <= u < cdf[i + 1], over the intervals iv[i] = (cdf[i], cdf[i + 1]).
// The guide entry is only a starting point; walking back then forward makes
// the answer exact whatever the guide is.  p receives iv[i].
__device__ __forceinline__ int interval_walk(const double2 *iv, int start, int n, double u, double2 &p) {
    int i = min(max(start, 0), n - 1);
    p = iv[i];
    while (i > 0 && p.x > u) { --i; p = iv[i]; }
    while (i < n - 1 && !(p.y > u)) { ++i; p = iv[i]; }
    return i;
}
// the same walk over the texel records of a row (base = its first texel),
// which also gives the radiance of the texel found
__device__ __forceinline__ int interval_walk(const EnvBufs &eb, uint32_t base, int start, int n, double u,
                                             double2 &p, float4 &lp) {
    int i = min(max(start, 0), n - 1);
    env_rec(eb, base + i, i, p, lp);
    while (i > 0 && p.x > u) { --i; env_rec(eb, base + i, i, p, lp); }
    while (i < n - 1 && !(p.y > u)) { ++i; env_rec(eb, base + i, i, p, lp); }
    return i;
}

// CDF inversion (row from the marginal, column from the row's conditional,
// linear remainder inside the texel), in double like the tables.
__device__ __forceinline__ bool env_sample(const EnvTables &e, const EnvBufs &eb, bool ok, const MargView &mv,
                                           float u0f, float u1f, V3 &dir, int &texel, float4 &lp, float &pdf) {
    if (!ok) return false;
    double u0 = u0f, u1 = u1f;
    double2 pm, pc;
    int i = interval_walk(mv.pair, mv.guide[min((int)(u0 * e.H), e.H - 1)], e.H, u0, pm);
    // the CDF differences are formed in double, the in-texel fractions in float
    float fv = __fdividef((float)(u0 - pm.x), (float)(pm.y - pm.x));
    const uint32_t row = (uint32_t)i * (uint32_t)e.W;
    int j = interval_walk(eb, row, e.gcond[row + (uint32_t)min((int)(u1 * e.W), e.W - 1)], e.W, u1, pc, lp);
    float fu = __fdividef((float)(u1 - pc.x), (float)(pc.y - pc.x));
    float v = ((float)i + fv) / (float)e.H, u = ((float)j + fu) / (float)e.W;
    float st, ct, sp, cp;
    sincospif(v, &st, &ct);                   // theta = pi v
    sincospif(2.0f * u - 1.0f, &sp, &cp);     // phi = 2 pi (u - 1/2)
    if (!(st > 0.0f)) return false;
    dir = V3{st * sp, ct, -st * cp};
    texel = i * e.W + j;
    pdf = lp.w / st;
    return pdf > 0.0f;
}

// ----------------------------------------------------------------------------
// internal layouts
// ----------------------------------------------------------------------------
// BVH node: both children's boxes, so one 64-byte fetch tests two boxes.
//   n0 = (l.lo.x, l.hi.x, l.lo.y, l.hi.y), n1 = (r.lo.x, r.hi.x, r.lo.y, r.hi.y)
//   n2 = (l.lo.z, l.hi.z, r.lo.z, r.hi.z), n3 = (lref, rref, -, -)
// ref >= 0: internal node; ref < 0: leaf ~(first << 3 | (count - 1)) over the
// leaf-ordered triangle array.
struct BvhNode { float4 n0, n1, n2; int4 n3; };
// Traversal node: up to four descendants of a binary node that together
// cover its subtree (chosen by the build's surface-area collapse; a leaf
// stands for itself), their boxes quantised to 8 bits per bound against the
// union box, so one 64-byte fetch tests four boxes where a binary node tests
// two.  On axis a, child c spans
//   [o_a + qlo_a[c] 2^(e_a - 127), o_a + qhi_a[c] 2^(e_a - 127)],
// which holds the child's float box with a quantum to spare on both sides.
//   a = (o.x, o.y, o.z, bits e_x | e_y << 8 | e_z << 16 | count << 24)
//   q = (qlo_x, qhi_x, qlo_y, qhi_y), byte c of a word for child c
//   r = (qlo_z, qhi_z, ref_0, ref_1), s = (ref_2, ref_3, 0, 0)
// Child c < count has ref_c: >= 0 the binary index of a descendant node,
// whose traversal node is stored at that same index; < 0 a leaf, as in
// BvhNode.  Only the binary nodes that the collapse keeps have a traversal
// node.
struct WideNode { float4 a; uint4 q; uint4 r; uint4 s; };
// Triangle in leaf order: v0 (w = original face id), v1, v2.
struct TriRec { float4 a, b, c; };

struct ViewDev {
    float rot[9];
    float org[3];
    double tan_half, aspect;
    int32_t w, h, spp;
    uint32_t sample_offset;
    int64_t pixel_offset;
    uint64_t sample_base;   // first global sample index of the view
    uint64_t pix_base;      // first view-order pixel index of the view
};

}  // namespace mrs
