// Host side of libmirres: argument validation, buffer management, the
// launch sequence of the wavefront path tracer and of its adjoint, the
// eager C-ABI entry points and the plan API (buffers owned per plan, launch
// sequence captured once in a hipGraph and replayed).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device.h"
#include "reuse.h"
#include "runtime.h"
#include "wavefront.h"

// ============================================================================
// error state
// ============================================================================
namespace mrs {
static thread_local std::string g_err;
void clear_error() { g_err.clear(); }
mrs_status fail(mrs_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
mrs_status hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return MRS_OK;
    (void)hipGetLastError();
    return fail(MRS_EHIP, "%s: %s", what, hipGetErrorString(e));
}
}  // namespace mrs

extern "C" const char *mrs_last_error(void) { return mrs::g_err.c_str(); }

namespace mrs {
namespace {

#define TRY(x) do { mrs_status st_ = (x); if (st_ != MRS_OK) return st_; } while (0)
#define HIPTRY(x, what) TRY(hip_check((x), what))

// ============================================================================
// kernel timing: event pairs around every launch while profiling is on (not
// while a launch sequence is being captured into a graph)
// ============================================================================
enum KernelId { KID_ENV = 0, KID_SCHED, KID_GENERATE, KID_CLOSEST, KID_SHADE, KID_SHADOW, KID_RESOLVE, KID_ADJOINT,
                KID_TRACE, KID_FIELD, KID_FIELD_BWD, KID_REUSE, KID_PLAN_FWD, KID_PLAN_BWD, KID_COUNT };
const char *const kKernelNames[KID_COUNT] = {"env_tables", "schedule", "generate", "trace_closest", "shade",
                                             "trace_shadow", "resolve", "adjoint", "trace_batch", "field_eval",
                                             "field_backward", "reuse", "plan_forward_graph", "plan_backward_graph"};
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int kid; hipEvent_t a, b; };
    std::vector<Rec> recs;
    hipEvent_t next() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
};
Profiler g_prof;
thread_local bool t_capturing = false;

struct ProfScope {
    int kid; hipStream_t s; hipEvent_t a = nullptr;
    ProfScope(int k, hipStream_t st) : kid(k), s(st) {
        if (g_prof.on && !t_capturing && (a = g_prof.next())) (void)hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = g_prof.next();
        if (!b) return;
        (void)hipEventRecord(b, s);
        g_prof.recs.push_back({kid, a, b});
    }
};
#define PROF(kid, s) ProfScope prof_scope_((kid), (s))

// ============================================================================
// jobs and buffers
// ============================================================================
constexpr uint64_t kOutChunkMax = 1ull << 27;   // samples per super-chunk of the output buffer
constexpr uint32_t kPoolDefault = 1u << 27;      // paths in flight: a whole output chunk (160 B each: 21.5 GB)
constexpr int kBlockDefault = 64;                // threads per workgroup of the trace and shade kernels
constexpr uint64_t kTapeRecBytes = 36;           // tape bytes per path vertex
constexpr uint64_t kTapeFieldBytes = 16;         // and, in field mode, the field's output at the vertex
constexpr uint64_t kAdjChunk = 1ull << 24;        // samples per adjoint launch

struct Chunk { uint64_t c0, c1, pix0, pix1; };

// Device buffers one launch sequence works in: the library's shared
// workspace for eager calls, or a plan's own set.
struct Res {
    DevBuf wts, cond, marg, rowsum, info, erec, gcond, gmarg, mpair, rcos, csphi;   // environment tables
    DevBuf views;                                              // ViewDev table
    DevBuf qa_o, qa_d, qa_t, qb_o, qb_d, qb_t, hits, so, sd, sc; // path pool queues
    DevBuf ctr, sched, out;                                    // iteration counters, scheduler, sample radiance
    DevBuf ct_hit, ct_y, ct_rr, ct_fm;                         // chunk tape (recompute mode)
    DevBuf grec;                                               // adjoint gradient records
    DevBuf fm, fvtx, gvtx;                                     // field mode: pool materials, vertex materials and gradients
    DevBuf rprim, rfmat, rr0, rr1;                             // reuse: primary hits, their field output, reservoirs
    DevBuf fkey, fkey2, fval, fval2, fsort;                    // field mode: pull-back order (keys, values, sort scratch)
    DevBuf tpack;                                              // texture mode: interleaved texel records
    DevBuf dkey, dkey2, dval, dval2, dsort;                    // deterministic adjoint: pairs, sorted pairs, sort scratch
    void release_all() {
        for (DevBuf *b : {&wts, &cond, &marg, &rowsum, &info, &erec, &gcond, &gmarg, &mpair, &rcos, &csphi, &views, &qa_o, &qa_d, &qa_t, &qb_o,
                          &qb_d, &qb_t, &hits, &so, &sd, &sc, &ctr, &sched, &out, &ct_hit, &ct_y, &ct_rr, &ct_fm, &grec, &fm, &fvtx, &gvtx,
                          &rprim, &rfmat, &rr0, &rr1, &fkey, &fkey2, &fval, &fval2, &fsort, &tpack, &dkey, &dkey2, &dval, &dval2,
                          &dsort})
            b->release();
    }
};

// Layout of the adjoint's gradient records for a scene and the wanted arrays:
// kMatRec floats per material texel (or mesh vertex) when any material
// gradient is wanted, then kEnvRec floats per env texel when the env one is.
// Offsets fit in 32 bits: validate() bounds the parameter arrays.
struct GradRec {
    uint32_t n_mat = 0, n_env = 0, env_base = 0;
    size_t words = 0;
};
GradRec grad_rec(const mrs_scene *sc, const mrs_grads *gr) {
    GradRec g;
    const bool vertex = sc->mat_mode == MRS_MAT_VERTEX;
    if (sc->mat_mode != MRS_MAT_FIELD && (vertex ? gr->vmat != nullptr : (gr->albedo || gr->rough || gr->metal)))
        g.n_mat = vertex ? (uint32_t)sc->nv : (uint32_t)sc->tw * (uint32_t)sc->th;
    if (gr->env) g.n_env = (uint32_t)sc->ew * (uint32_t)sc->eh;
    g.env_base = kMatRec * g.n_mat;
    g.words = (size_t)kMatRec * g.n_mat + (size_t)kEnvRec * g.n_env;
    return g;
}

struct Workspace {
    std::mutex mu;
    Res res;
    ViewDev *staging = nullptr;   // pinned host copy of the view table
    size_t staging_n = 0;
    std::vector<ViewDev> uploaded;  // view table currently on the device
    hipEvent_t done = nullptr;    // end of the previous eager call
    hipStream_t last = nullptr;
    bool has_last = false;
};
Workspace g_ws;

bool field_wanted(const mrs_grads *gr) {
    return gr->field.table || gr->field.w1 || gr->field.b1 || gr->field.w2 || gr->field.b2;
}

// reservoir reuse settings of a job (all zero: no reuse)
struct Reuse {
    int on = 0, spatial = 0, radius = 1, temporal = 0;
    float mcap = 0.0f;            // temporal confidence cap, m_cap * M
    const float *prev = nullptr;  // [S][8]
    float *out = nullptr;         // [S][8]
};

struct Job {
    FieldDev fd{};                // field mode: the field's device view
    Reuse reuse;
    std::vector<ViewDev> vd;
    uint64_t S = 0, pixels = 0;
    SceneDev sd{};
    Opts op{};
    ViewTable vt{};
    uint32_t pool = kPoolDefault;
    int block = kBlockDefault;
    bool det = false;             // deterministic adjoint (ordered sums instead of atomics)
};

inline unsigned nblocks(uint64_t n, int b) { return (unsigned)std::max<uint64_t>(1, (n + b - 1) / b); }

// compute units of the current device (cached per device)
int device_cus() {
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    int c = cus[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cus[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

// Grid of a persistent traversal launch: enough blocks of b threads to hold
// every wavefront slot of the current device (32 wave64 per CU), capped by
// the blocks needed for n rays.  Extra blocks find the queue drained and exit.
unsigned persistent_blocks(uint64_t n, int b) {
    return std::min<unsigned>(nblocks(n, b), (unsigned)((uint64_t)device_cus() * 2048 / b));
}

// Grid of a grid-stride kernel over a queue whose length only the device
// knows: per_cu blocks per compute unit (several rounds of resident blocks,
// so the hardware still balances the tail), capped by the blocks needed for
// a full pool of n entries.
unsigned stride_blocks(uint64_t n, int b, int per_cu) {
    return std::min<unsigned>(nblocks(n, b), (unsigned)(device_cus() * per_cu));
}

mrs_status validate(const mrs_scene *sc, const mrs_view *views, int32_t n_views, const mrs_options *op, Job &job) {
    if (!sc) return fail(MRS_EINVAL, "scene is NULL");
    if (!views) return fail(MRS_EINVAL, "views is NULL");
    if (!op) return fail(MRS_EINVAL, "options is NULL");
    if (!sc->pos || !sc->faces || sc->nv <= 0 || sc->nf <= 0) return fail(MRS_EINVAL, "scene mesh is empty or NULL");
    if (!sc->bvh) return fail(MRS_EINVAL, "scene.bvh is NULL (build it with mrs_build_bvh)");
    if (sc->bvh->nf != sc->nf || sc->bvh->nv != sc->nv)
        return fail(MRS_EINVAL, "scene.bvh was built for %d vertices / %d triangles, scene has %d / %d", sc->bvh->nv,
                    sc->bvh->nf, sc->nv, sc->nf);
    if (sc->mat_mode == MRS_MAT_VERTEX) {
        if (!sc->vmat) return fail(MRS_EINVAL, "scene.vmat is NULL for per-vertex materials");
    } else if (sc->mat_mode == MRS_MAT_TEXTURE) {
        if (!sc->uv || !sc->albedo || !sc->rough || !sc->metal) return fail(MRS_EINVAL, "texture mode needs uv, albedo, rough, metal");
        if (sc->tw <= 0 || sc->th <= 0 || (int64_t)sc->tw * sc->th >= (1ll << 31)) return fail(MRS_EINVAL, "bad texture size %dx%d", sc->tw, sc->th);
    } else if (sc->mat_mode == MRS_MAT_FIELD) {
        const char *why = nullptr;
        if (!make_field_dev(&sc->field, job.fd, &why)) return fail(MRS_EINVAL, "scene.%s", why);
    } else {
        return fail(MRS_EINVAL, "unknown mat_mode %d", sc->mat_mode);
    }
    if (!sc->env || sc->ew <= 0 || sc->eh <= 0) return fail(MRS_EINVAL, "bad environment map %dx%d", sc->ew, sc->eh);
    // the env's 24-byte texel records are addressed with 32-bit byte offsets,
    // and its column guides are 16-bit
    if ((int64_t)sc->ew * sc->eh >= (1ll << 27))
        return fail(MRS_EOVERFLOW, "environment map %dx%d has 2^27 texels or more", sc->ew, sc->eh);
    if (sc->ew > 65536) return fail(MRS_EOVERFLOW, "environment map %dx%d is wider than 65536 texels", sc->ew, sc->eh);
    // gradient elements are addressed with 29-bit indices
    if (3ll * sc->ew * sc->eh >= (1ll << 29) || 5ll * sc->nv >= (1ll << 29) ||
        (sc->mat_mode == MRS_MAT_TEXTURE && 3ll * sc->tw * sc->th >= (1ll << 29)))
        return fail(MRS_EOVERFLOW, "parameter arrays too large (more than 2^29 gradient elements)");
    if (n_views < 1 || n_views > MRS_MAX_VIEWS) return fail(MRS_EINVAL, "n_views must be in [1, %d]", MRS_MAX_VIEWS);
    if (op->bounces < 1 || op->bounces > MRS_MAX_BOUNCES) return fail(MRS_EINVAL, "bounces must be in [1, %d]", MRS_MAX_BOUNCES);
    if (op->ris_m < 1 || op->ris_m > 0xFFFE) return fail(MRS_EINVAL, "ris_m must be in [1, 65534]");
    if (op->ris_m_brdf < 0 || op->ris_m_brdf > op->ris_m) return fail(MRS_EINVAL, "ris_m_brdf must be in [0, ris_m]");
    if (op->rr_start < -1) return fail(MRS_EINVAL, "rr_start must be -1 or >= 0");
    if (op->brdf != MRS_BRDF_LAMBERT && op->brdf != MRS_BRDF_LAMBERT_GGX) return fail(MRS_EINVAL, "unknown brdf %d", op->brdf);
    if (op->background != MRS_BG_ENV && op->background != MRS_BG_BLACK) return fail(MRS_EINVAL, "unknown background %d", op->background);
    if (op->grad_mode != MRS_GRAD_FULL && op->grad_mode != MRS_GRAD_PRIMARY) return fail(MRS_EINVAL, "unknown grad_mode %d", op->grad_mode);
    if (op->tape_mode < MRS_TAPE_AUTO || op->tape_mode > MRS_TAPE_OFF) return fail(MRS_EINVAL, "unknown tape_mode %d", op->tape_mode);
    if (op->pool < 0) return fail(MRS_EINVAL, "pool must be >= 0");
    if (op->block != 0 && (op->block < 64 || op->block > 256 || op->block % 64)) return fail(MRS_EINVAL, "block must be 0 or a multiple of 64 in [64, 256]");
    if (op->deterministic != 0 && op->deterministic != 1) return fail(MRS_EINVAL, "deterministic must be 0 or 1");
    if (op->deterministic && sc->mat_mode == MRS_MAT_FIELD)
        return fail(MRS_EINVAL, "deterministic mode covers texture and vertex materials, not the material field");
    if (op->reuse_spatial != 0 || op->reuse_temporal != 0) {
        if (op->reuse_spatial < 0 || op->reuse_spatial > kReuseMaxK) return fail(MRS_EINVAL, "reuse_spatial must be in [0, %d]", kReuseMaxK);
        if (op->reuse_radius < 1 || op->reuse_radius > 64) return fail(MRS_EINVAL, "reuse_radius must be in [1, 64]");
        if (op->reuse_temporal != 0 && op->reuse_temporal != 1) return fail(MRS_EINVAL, "reuse_temporal must be 0 or 1");
        if (op->reuse_m_cap < 1) return fail(MRS_EINVAL, "reuse_m_cap must be >= 1");
        job.reuse.on = 1;
        job.reuse.spatial = op->reuse_spatial;
        job.reuse.radius = op->reuse_radius;
        job.reuse.temporal = op->reuse_temporal;
        job.reuse.mcap = (float)op->reuse_m_cap * (float)op->ris_m;
        job.reuse.prev = op->reservoir_prev;
        job.reuse.out = op->reservoir_out;
    } else if (op->reservoir_out) {
        return fail(MRS_EINVAL, "reservoir_out needs reservoir reuse (reuse_spatial > 0 or reuse_temporal = 1)");
    }
    job.vd.resize(n_views);
    uint64_t S = 0, P = 0;
    for (int i = 0; i < n_views; ++i) {
        const mrs_view &v = views[i];
        if (v.w < 1 || v.h < 1 || v.spp < 1) return fail(MRS_EINVAL, "view %d: w, h, spp must be >= 1", i);
        if ((int64_t)v.w * v.h >= (1ll << 31)) return fail(MRS_EOVERFLOW, "view %d: more than 2^31 pixels", i);
        if (!(v.fov_y_deg > 0.0f && v.fov_y_deg < 180.0f)) return fail(MRS_EINVAL, "view %d: fov_y_deg must be in (0, 180)", i);
        if (v.pixel_offset < 0) return fail(MRS_EINVAL, "view %d: negative pixel_offset", i);
        ViewDev &d = job.vd[i];
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) d.rot[3 * r + c] = v.c2w[4 * r + c];
            d.org[r] = v.c2w[4 * r + 3];
        }
        d.tan_half = tan(0.5 * (double)v.fov_y_deg * 3.14159265358979323846 / 180.0);
        d.aspect = (double)v.w / (double)v.h;
        d.w = v.w; d.h = v.h; d.spp = v.spp;
        d.sample_offset = v.sample_offset;
        d.pixel_offset = v.pixel_offset;
        d.sample_base = S;
        d.pix_base = P;
        S += (uint64_t)v.w * v.h * v.spp;
        P += (uint64_t)v.w * v.h;
    }
    if (S >= (1ull << 32)) return fail(MRS_EOVERFLOW, "%llu samples exceed 2^32 - 1 per call", (unsigned long long)S);
    if (job.reuse.prev && job.reuse.out) {
        const uintptr_t a = (uintptr_t)job.reuse.prev, b = (uintptr_t)job.reuse.out, nb = sizeof(float) * 8 * S;
        if (a < b + nb && b < a + nb) return fail(MRS_EINVAL, "reservoir_out overlaps reservoir_prev");
    }
    job.S = S;
    job.pixels = P;
    job.op.B = op->bounces; job.op.M = op->ris_m; job.op.Mb = op->ris_m_brdf; job.op.rr_start = op->rr_start;
    job.op.spec = op->brdf == MRS_BRDF_LAMBERT_GGX; job.op.background = op->background; job.op.grad_mode = op->grad_mode;
    job.op.k0 = (uint32_t)op->seed; job.op.k1 = (uint32_t)(op->seed >> 32);
    job.pool = op->pool > 0 ? (uint32_t)op->pool : kPoolDefault;
    job.block = op->block > 0 ? op->block : kBlockDefault;
    job.det = op->deterministic != 0;
    return MRS_OK;
}

uint64_t signature(const Job &job) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    };
    for (const ViewDev &v : job.vd) mix(&v, sizeof(ViewDev));
    mix(&job.op, sizeof(Opts));
    const int ru[4] = {job.reuse.on, job.reuse.spatial, job.reuse.radius, job.reuse.temporal};
    mix(ru, sizeof(ru));
    mix(&job.reuse.mcap, sizeof(float));
    return h;
}

// pixel-aligned sample ranges of at most `cap` samples (a pixel is never split)
std::vector<Chunk> make_chunks(const Job &job, uint64_t cap) {
    std::vector<Chunk> out;
    Chunk cur{0, 0, 0, 0};
    for (const ViewDev &v : job.vd) {
        uint64_t npix = (uint64_t)v.w * v.h, done = 0;
        while (done < npix) {
            uint64_t room = cap > (cur.c1 - cur.c0) ? cap - (cur.c1 - cur.c0) : 0;
            uint64_t take = std::min<uint64_t>(npix - done, room / v.spp);
            if (take == 0) {
                if (cur.c1 > cur.c0) { out.push_back(cur); cur = Chunk{cur.c1, cur.c1, cur.pix1, cur.pix1}; continue; }
                take = 1;   // a single pixel larger than the cap
            }
            cur.c1 += take * v.spp;
            cur.pix1 += take;
            done += take;
        }
    }
    if (cur.c1 > cur.c0) out.push_back(cur);
    return out;
}

uint64_t max_chunk(const std::vector<Chunk> &cs) {
    uint64_t m = 0;
    for (const Chunk &c : cs) m = std::max(m, c.c1 - c.c0);
    return m;
}

// Wavefront iterations that cover a chunk of n samples through a pool of P
// paths (n <= P: every sample starts in the first iteration).  While samples
// wait, the pool is full and an iteration retires P path vertices, at most n B
// in all; the last sample admitted then needs at most B - 1 more.
int iterations(const Job &job, uint64_t n, uint32_t P) {
    const int B = job.op.B;
    return n <= P ? B : (int)((n * B + P - 1) / P) + B;
}

// scene pointers the kernels read (the BVH's validated face copy for shading)
void bind_scene(const mrs_scene *sc, Job &job) {
    job.sd.faces = sc->bvh->faces.as<int32_t>(); job.sd.uv = sc->uv; job.sd.vmat = sc->vmat;
    job.sd.albedo = sc->albedo; job.sd.rough = sc->rough; job.sd.metal = sc->metal;
    job.sd.mat_mode = sc->mat_mode; job.sd.tw = sc->tw; job.sd.th = sc->th;
    job.sd.nodes = sc->bvh->wnodes.as<WideNode>();
    job.sd.tris = sc->bvh->tris.as<TriRec>();
}

mrs_status reserve_env(const mrs_scene *sc, Res &r) {
    size_t W = sc->ew, H = sc->eh, nt = W * H;
    TRY(r.wts.reserve(sizeof(double) * nt));
    TRY(r.cond.reserve(sizeof(double) * H * (W + 1)));
    TRY(r.marg.reserve(sizeof(double) * (H + 1)));
    TRY(r.rowsum.reserve(sizeof(double) * H));
    TRY(r.info.reserve(sizeof(double) * 2));
    TRY(r.erec.reserve(24 * nt + 16));
    TRY(r.gmarg.reserve(sizeof(int32_t) * H));
    TRY(r.gcond.reserve(sizeof(uint16_t) * nt));
    TRY(r.mpair.reserve(sizeof(double2) * H));
    TRY(r.rcos.reserve(sizeof(double) * (H + 1)));
    TRY(r.csphi.reserve(sizeof(double2) * (W + 1)));
    return MRS_OK;
}

// Counter buffer of one super-chunk: IterCtr per iteration (+1), then, from
// the next 128-byte boundary, the claim counters of the persistent
// closest-hit launch of every iteration.  All of it is zeroed per chunk.
size_t claim_offset_words(int n_iter) { return ((sizeof(IterCtr) * (size_t)(n_iter + 1) + 127) / 128) * 32; }
size_t ctr_words(int n_iter) { return claim_offset_words(n_iter) + (size_t)n_iter * kClaimWords; }

mrs_status reserve_pool(Res &r, uint32_t P, uint64_t out_samples, int n_iter, bool field) {
    size_t q = sizeof(float4) * (size_t)P;
    for (DevBuf *b : {&r.qa_o, &r.qa_d, &r.qa_t, &r.qb_o, &r.qb_d, &r.qb_t, &r.hits, &r.so, &r.sd, &r.sc}) TRY(b->reserve(q));
    if (field) TRY(r.fm.reserve(q));
    TRY(r.ctr.reserve(4 * ctr_words(n_iter)));
    TRY(r.sched.reserve(sizeof(Sched)));
    TRY(r.out.reserve(sizeof(float4) * (size_t)out_samples));
    return MRS_OK;
}

// texture mode: the texel records the material fetch reads, packed per call
mrs_status reserve_tpack(const mrs_scene *sc, Res &r) {
    if (sc->mat_mode != MRS_MAT_TEXTURE) return MRS_OK;
    return r.tpack.reserve(2 * sizeof(float4) * (size_t)sc->tw * (size_t)sc->th);
}
mrs_status pack_texels(const mrs_scene *sc, Job &job, Res &r, hipStream_t s) {
    if (sc->mat_mode != MRS_MAT_TEXTURE) return MRS_OK;
    TRY(reserve_tpack(sc, r));
    const uint64_t n = (uint64_t)sc->tw * (uint64_t)sc->th;
    k_pack_texels<<<nblocks(n, 256), 256, 0, s>>>(sc->albedo, sc->rough, sc->metal, n, r.tpack.as<float4>());
    job.sd.tpack = r.tpack.as<float4>();
    return MRS_OK;
}

// env tables: kernels only (the validity flag stays on the device), so the
// sequence can be captured in a graph
mrs_status env_tables(const mrs_scene *sc, Job &job, Res &r, hipStream_t s) {
    TRY(reserve_env(sc, r));
    int W = sc->ew, H = sc->eh;
    {
        PROF(KID_ENV, s);
        k_env_rows<<<H, 256, 0, s>>>(sc->env, W, H, r.wts.as<double>(), r.cond.as<double>(), r.rowsum.as<double>());
        k_env_marg<<<1, kMargThreads, 0, s>>>(r.rowsum.as<double>(), H, r.marg.as<double>(), r.info.as<double>());
        k_env_finish<<<H + 1, 256, 0, s>>>(sc->env, W, H, r.wts.as<double>(), r.info.as<double>(), r.marg.as<double>(),
                                            r.cond.as<double>(), r.erec.as<char>(), r.gcond.as<uint16_t>(), r.gmarg.as<int32_t>(),
                                            r.mpair.as<double2>(), r.rcos.as<double>(), r.csphi.as<double2>());
    }
    EnvTables &e = job.sd.env;
    e.mpair = r.mpair.as<double2>(); e.rec = r.erec.as<char>();
    e.gmarg = r.gmarg.as<int32_t>();
    e.gcond = r.gcond.as<uint16_t>();
    e.total = r.info.as<double>();
    e.rcos = r.rcos.as<double>(); e.csphi = r.csphi.as<double2>();
    e.W = W; e.H = H;
    return MRS_OK;
}

// One super-chunk through the persistent pool.  The number of iterations is
// an upper bound (every full iteration retires P path vertices); iterations
// past the end find empty queues and exit at once.  No allocation happens
// when the buffers were reserved beforehand (graph capture relies on it).
mrs_status run_wavefront(const Job &job, const Chunk &ch, Tape tape, int use_tape, uint32_t *hash, Res &r,
                         hipStream_t s) {
    uint64_t n = ch.c1 - ch.c0;
    uint32_t P = (uint32_t)std::min<uint64_t>(job.pool, n);
    int n_iter = iterations(job, n, P);
    const bool field = job.sd.mat_mode == MRS_MAT_FIELD;
    TRY(reserve_pool(r, P, n, n_iter, field));
    size_t nctr = ctr_words(n_iter);
    k_fill_u32<<<nblocks(nctr, 256), 256, 0, s>>>(r.ctr.as<uint32_t>(), nctr, 0u);
    uint32_t *claim = r.ctr.as<uint32_t>() + claim_offset_words(n_iter);
    k_set_sched<<<1, 64, 0, s>>>(r.sched.as<Sched>(), ch.c0, ch.c1);
    Queue qa{r.qa_o.as<float4>(), r.qa_d.as<float4>(), r.qa_t.as<float4>()};
    Queue qb{r.qb_o.as<float4>(), r.qb_d.as<float4>(), r.qb_t.as<float4>()};
    IterCtr *ctr = r.ctr.as<IterCtr>();
    // with reservoir reuse the reuse pass has traced every camera ray of the
    // frame: the path tracer takes those hits instead of tracing again
    const float4 *prim = job.reuse.on ? r.rprim.as<float4>() : nullptr;
    int bs = job.block;
    for (int it = 0; it < n_iter; ++it) {
        {
            PROF(KID_SCHED, s);
            k_schedule<<<1, 64, 0, s>>>(ctr, it, r.sched.as<Sched>(), P);
        }
        {
            PROF(KID_GENERATE, s);
            GenArgs ga{job.vt, job.op, qa, ctr, it, r.out.as<float4>(), ch.c0, hash, prim, r.hits.as<float4>()};
            k_generate<<<stride_blocks(P, 256, 16), 256, 0, s>>>(ga);
        }
        {
            PROF(KID_CLOSEST, s);
            TraceArgs ta{job.sd.nodes, job.sd.tris, qa, r.hits.as<float4>(), ctr, it, claim + it * kClaimWords,
                         prim != nullptr};
            k_trace_closest<<<persistent_blocks(P, bs), bs, kLdsStackBytes * bs, s>>>(ta);
        }
        if (field) {
            PROF(KID_FIELD, s);
            PointsHits src{r.hits.as<float4>(), job.sd.tris, ctr, it, qa.o, qa.d};
            k_field_eval<PointsHits><<<nblocks(P, kFieldTile), 64, 0, s>>>(job.fd, src, r.fm.as<float>());
        }
        {
            PROF(KID_SHADE, s);
            ShadeArgs sa{job.sd, job.vt, job.op, qa, qb, r.hits.as<float4>(), ctr, it, r.so.as<float4>(),
                         r.sd.as<float4>(), r.sc.as<float4>(), r.out.as<float4>(), ch.c0, hash, tape, use_tape};
            sa.s.fm = r.fm.as<float4>();
            if (job.reuse.on) { sa.resv = r.rr0.as<ResvRec>(); sa.resv_base = 0; }
            if (job.sd.env.H <= kEnvLdsRows) k_shade<true><<<nblocks(P, kShadeBlock), kShadeBlock, 0, s>>>(sa);
            else k_shade<false><<<nblocks(P, kShadeBlock), kShadeBlock, 0, s>>>(sa);
        }
        {
            PROF(KID_SHADOW, s);
            ShadowArgs sh{job.sd.nodes, job.sd.tris, r.so.as<float4>(), r.sd.as<float4>(), r.sc.as<float4>(), ctr, it,
                          r.out.as<float4>(), ch.c0, hash, tape, use_tape};
            k_trace_shadow<<<nblocks(P, bs), bs, kLdsStackBytes * bs, s>>>(sh);
        }
        std::swap(qa, qb);
    }
    HIPTRY(hipGetLastError(), "wavefront launch");
    return MRS_OK;
}

// reservoir reuse buffers: primary hits, two record arrays (and the field's
// output at the primary hits in field mode), one entry per sample
mrs_status reserve_reuse(const Job &job, Res &r) {
    if (!job.reuse.on) return MRS_OK;
    TRY(r.rprim.reserve(sizeof(float4) * job.S));
    TRY(r.rr0.reserve(sizeof(ResvRec) * job.S));
    TRY(r.rr1.reserve(sizeof(ResvRec) * job.S));
    if (job.sd.mat_mode == MRS_MAT_FIELD) TRY(r.rfmat.reserve(sizeof(float4) * job.S));
    return MRS_OK;
}

// the final reservoirs of every primary vertex of the frame (into rr0);
// needs the env tables of the call
mrs_status run_reuse(const Job &job, Res &r, hipStream_t s) {
    TRY(reserve_reuse(job, r));
    PROF(KID_REUSE, s);
    ReuseArgs ra{job.sd, job.vt, job.op, job.S, r.rprim.as<float4>(), r.rfmat.as<float4>(), r.rr0.as<ResvRec>(),
                 r.rr1.as<ResvRec>(), job.reuse.prev, job.reuse.out, job.reuse.spatial, job.reuse.radius,
                 job.reuse.temporal, job.reuse.mcap};
    launch_reuse(ra, job.fd, r.rfmat.as<float>(), s);
    HIPTRY(hipGetLastError(), "reuse launch");
    return MRS_OK;
}

void resolve(const Job &job, const Chunk &ch, const Res &r, float *image, float *dbg_rgb, hipStream_t s) {
    PROF(KID_RESOLVE, s);
    ResolveArgs ra{job.vt, r.out.as<float4>(), ch.c0, ch.pix0, ch.pix1, image, dbg_rgb};
    k_resolve<<<nblocks(ch.pix1 - ch.pix0, 256), 256, 0, s>>>(ra);
}

// Field mode around each adjoint launch: the field at every taped vertex
// (the adjoint replays the materials), the adjoint writing dL/d(field
// output) per vertex, then the field's pull-back over the vertices that
// carry a gradient.  fvtx and gvtx hold B * min(kAdjChunk, samples) records.
mrs_status reserve_field_vertices(const Job &job, uint64_t samples, Res &r) {
    size_t n = (size_t)std::min<uint64_t>(kAdjChunk, samples) * job.op.B;
    TRY(r.fvtx.reserve(sizeof(float4) * n));
    TRY(r.gvtx.reserve(sizeof(float4) * n));
    for (DevBuf *b : {&r.fkey, &r.fkey2, &r.fval, &r.fval2}) TRY(b->reserve(sizeof(uint32_t) * n));
    TRY(r.fsort.reserve(std::max<size_t>(sort_pairs_tmp_bytes(n), 16)));
    return MRS_OK;
}

// Deterministic mode: kPairsPerVertex * B (record word, value) pairs per
// sample of a kDetChunk-sample adjoint launch, their sorted copies and the
// sort's scratch.
constexpr uint64_t kDetChunk = 1ull << 20;
mrs_status reserve_det_pairs(const Job &job, uint64_t samples, Res &r) {
    if (!job.det) return MRS_OK;
    const size_t n = (size_t)std::min<uint64_t>(kDetChunk, samples) * kPairsPerVertex * job.op.B;
    for (DevBuf *b : {&r.dkey, &r.dkey2, &r.dval, &r.dval2}) TRY(b->reserve(sizeof(uint32_t) * n));
    TRY(r.dsort.reserve(std::max<size_t>(sort_pairs_tmp_bytes(n), 16)));
    return MRS_OK;
}

mrs_status adjoint(const Job &job, const Tape &tp, uint64_t c0, uint64_t c1, const float *dimg, const mrs_grads *gr,
                   const GradRec &gl, float *rec, Res &r, hipStream_t s) {
    const bool field = job.sd.mat_mode == MRS_MAT_FIELD && field_wanted(gr);
    if (gl.words == 0 && !field) return MRS_OK;
    const FieldGrads fg{gr->field.table, gr->field.w1, gr->field.b1, gr->field.w2, gr->field.b2};
    const uint64_t step = job.det ? kDetChunk : kAdjChunk;
    for (uint64_t a0 = c0; a0 < c1; a0 += step) {
        uint64_t n = std::min<uint64_t>(step, c1 - a0);
        SceneDev sd = job.sd;
        uint64_t fm_stride = n;
        if (job.sd.mat_mode == MRS_MAT_FIELD) {
            if (tp.fm) {   // the forward kept the field's output at every vertex
                sd.fm = tp.fm + (a0 - tp.base);
                fm_stride = tp.S;
            } else {
                PROF(KID_FIELD, s);
                PointsTape src{tp, job.sd.tris, a0, n, job.op.B};
                k_field_eval<PointsTape><<<nblocks(src.count(), kFieldTile), 64, 0, s>>>(job.fd, src,
                                                                                          r.fvtx.as<float>());
                sd.fm = r.fvtx.as<float4>();
            }
        }
        const int kgrad = job.op.grad_mode == MRS_GRAD_PRIMARY ? 1 : job.op.B;
        if (field) {
            size_t words = 4 * (size_t)n * kgrad;
            k_fill_u32<<<nblocks(words, 256), 256, 0, s>>>(r.gvtx.as<uint32_t>(), words, 0u);
        }
        {
            PROF(KID_ADJOINT, s);
            AdjArgs aa{sd, job.vt, job.op, tp, a0, n, dimg, gr->vmat, gr->albedo, gr->rough, gr->metal, gr->env,
                       rec, gl.env_base, gl.n_mat > 0 ? 1 : 0, r.gvtx.as<float4>(), field ? 1 : 0, fm_stride};
            if (job.det) {
                const uint64_t np = n * kPairsPerVertex * (uint64_t)job.op.B;
                k_fill_u32<<<nblocks(np, 256), 256, 0, s>>>(r.dkey.as<uint32_t>(), np, kAggEmpty);
                k_adjoint_det<<<nblocks(n, kAdjBlock), kAdjBlock, 0, s>>>(aa, r.dkey.as<uint32_t>(), r.dval.as<float>());
                TRY(sort_pairs_u32(r.dkey.as<uint32_t>(), r.dkey2.as<uint32_t>(), r.dval.as<uint32_t>(),
                                   r.dval2.as<uint32_t>(), np, r.dsort, s));
                k_det_sum<<<nblocks(np, 256), 256, 0, s>>>(r.dkey2.as<uint32_t>(), r.dval2.as<float>(), np, rec);
            } else {
                k_adjoint<<<nblocks(n, kAdjBlock), kAdjBlock, 0, s>>>(aa);
            }
        }
        if (field) {
            PROF(KID_FIELD_BWD, s);
            // the vertices with a gradient in Morton order of their position, then the pull-back in that order
            PointsTape src{tp, job.sd.tris, a0, n, kgrad};
            const uint64_t cnt = src.count();
            k_field_keys<PointsTape><<<nblocks(cnt, 256), 256, 0, s>>>(job.fd, src, r.gvtx.as<float>(),
                                                                       r.fkey.as<uint32_t>(), r.fval.as<uint32_t>());
            TRY(sort_pairs_u32(r.fkey.as<uint32_t>(), r.fkey2.as<uint32_t>(), r.fval.as<uint32_t>(),
                               r.fval2.as<uint32_t>(), cnt, r.fsort, s));
            PointsPerm<PointsTape> ps{src, r.fval2.as<uint32_t>()};
            const uint64_t tiles = (cnt + kFieldTile - 1) / kFieldTile;
            k_field_backward<PointsPerm<PointsTape>><<<field_backward_blocks(tiles), 64, 0, s>>>(job.fd, ps,
                                                                                                 r.gvtx.as<float>(), fg);
        }
    }
    HIPTRY(hipGetLastError(), "adjoint launch");
    return MRS_OK;
}

// zero the gradient records before the first adjoint launch of a backward pass
void grad_rec_clear(const GradRec &gl, float *rec, hipStream_t s) {
    if (gl.words) k_fill_u32<<<nblocks(gl.words, 256), 256, 0, s>>>((uint32_t *)rec, gl.words, 0u);
}

// add the gradient records into the caller's arrays after the last one
void grad_rec_fold(const mrs_scene *sc, const GradRec &gl, const float *rec, const mrs_grads *gr, hipStream_t s) {
    uint32_t n = std::max(gl.n_mat, gl.n_env);
    if (n == 0) return;
    FoldArgs f{rec, gl.n_mat, gl.n_env, gl.env_base, sc->mat_mode == MRS_MAT_VERTEX ? 1 : 0,
               gr->vmat, gr->albedo, gr->rough, gr->metal, gr->env};
    k_grad_fold<<<nblocks(n, 256), 256, 0, s>>>(f);
}

// The last released tape's buffers, kept for the next tape on the same
// device: an optimisation loop renders with a tape every step, and a
// hipMalloc / hipFree pair of a few GB per step costs more than holding one
// tape.  mrs_release_workspace frees them.
struct SpareTape {
    std::mutex mu;
    int device = -1;
    DevBuf hit, y, rr, fm;
};
SpareTape g_spare;

void move_buf(DevBuf &dst, DevBuf &src) {
    dst.release();
    dst.p = src.p;
    dst.bytes = src.bytes;
    src.p = nullptr;
    src.bytes = 0;
}

mrs_status tape_alloc(mrs_tape *t, uint64_t S, int B, bool field) {
    size_t n = (size_t)S * B;
    int dev = -1;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lk(g_spare.mu);
        if (g_spare.device == dev) {
            if (g_spare.hit.bytes >= sizeof(float4) * n) move_buf(t->hit, g_spare.hit);
            if (g_spare.y.bytes >= sizeof(float4) * n) move_buf(t->y, g_spare.y);
            if (g_spare.rr.bytes >= sizeof(float) * n) move_buf(t->rr, g_spare.rr);
            if (field && g_spare.fm.bytes >= sizeof(float4) * n) move_buf(t->fm, g_spare.fm);
        }
    }
    TRY(t->hit.reserve(sizeof(float4) * n));
    TRY(t->y.reserve(sizeof(float4) * n));
    TRY(t->rr.reserve(sizeof(float) * n));
    if (field) TRY(t->fm.reserve(sizeof(float4) * n));
    t->device = dev;
    return MRS_OK;
}

// keeps a released tape's buffers as the spare (the larger of the two wins)
void tape_recycle(mrs_tape *t) {
    std::lock_guard<std::mutex> lk(g_spare.mu);
    if (g_spare.device != t->device) {
        g_spare.hit.release(); g_spare.y.release(); g_spare.rr.release(); g_spare.fm.release();
        g_spare.device = t->device;
    }
    if (t->hit.bytes > g_spare.hit.bytes) move_buf(g_spare.hit, t->hit);
    if (t->y.bytes > g_spare.y.bytes) move_buf(g_spare.y, t->y);
    if (t->rr.bytes > g_spare.rr.bytes) move_buf(g_spare.rr, t->rr);
    if (t->fm.bytes > g_spare.fm.bytes) move_buf(g_spare.fm, t->fm);
}

// tape policy: keep the per-vertex records when asked and affordable
mrs_status decide_tape(const Job &job, const mrs_options *opt, bool wanted, mrs_tape **out) {
    *out = nullptr;
    if (!wanted || opt->tape_mode == MRS_TAPE_OFF) return MRS_OK;
    const bool field = job.sd.mat_mode == MRS_MAT_FIELD;
    uint64_t bytes = job.S * job.op.B * (kTapeRecBytes + (field ? kTapeFieldBytes : 0));
    uint64_t budget = (uint64_t)opt->tape_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        HIPTRY(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
        budget = fr / 2;
    }
    if (opt->tape_mode != MRS_TAPE_ON && bytes > budget) return MRS_OK;
    mrs_tape *t = new mrs_tape();
    mrs_status st = tape_alloc(t, job.S, job.op.B, field);
    if (st != MRS_OK) {
        delete t;
        if (opt->tape_mode == MRS_TAPE_ON) return st;
        clear_error();   // AUTO falls back to recompute
        return MRS_OK;
    }
    t->samples = job.S; t->bounces = job.op.B; t->seed = opt->seed; t->signature = signature(job);
    *out = t;
    return MRS_OK;
}

Tape tape_view(const mrs_tape *t) {
    return Tape{t->hit.as<float4>(), t->y.as<float4>(), t->rr.as<float>(), 0, t->samples, t->fm.as<float4>()};
}

// forward launch sequence (eager or under capture)
mrs_status enqueue_forward(const Job &job, const std::vector<Chunk> &chunks, const mrs_scene *sc, Res &r,
                           const mrs_tape *tape, float *image, float *dbg_rgb, uint32_t *dbg_hash, hipStream_t s) {
    Job j = job;
    TRY(env_tables(sc, j, r, s));
    TRY(pack_texels(sc, j, r, s));
    if (j.reuse.on) TRY(run_reuse(j, r, s));
    Tape tp = tape ? tape_view(tape) : Tape{};
    for (const Chunk &ch : chunks) {
        // the hash buffer is indexed from the chunk start like the output
        TRY(run_wavefront(j, ch, tp, tape != nullptr, dbg_hash ? dbg_hash + ch.c0 : nullptr, r, s));
        resolve(j, ch, r, image, dbg_rgb, s);
    }
    return MRS_OK;
}

// backward launch sequence: replay the tape, or re-render chunk by chunk into
// a bounded tape and replay that
mrs_status enqueue_backward(const Job &job, const std::vector<Chunk> &chunks, const mrs_scene *sc, Res &r,
                            const mrs_tape *tape, const float *dimg, const mrs_grads *grads, hipStream_t s) {
    Job j = job;
    TRY(env_tables(sc, j, r, s));
    TRY(pack_texels(sc, j, r, s));
    const GradRec gl = grad_rec(sc, grads);
    if (gl.words) TRY(r.grec.reserve(4 * gl.words));
    if (sc->mat_mode == MRS_MAT_FIELD) TRY(reserve_field_vertices(j, j.S, r));
    TRY(reserve_det_pairs(j, j.S, r));
    float *rec = r.grec.as<float>();
    grad_rec_clear(gl, rec, s);
    if (tape) {
        TRY(adjoint(j, tape_view(tape), 0, j.S, dimg, grads, gl, rec, r, s));
    } else {
        // the re-render needs this frame's reservoirs: the same inputs give the same ones
        if (j.reuse.on) {
            Job jr = j;
            jr.reuse.out = nullptr;
            TRY(run_reuse(jr, r, s));
        }
        uint64_t cap = max_chunk(chunks);
        size_t n = (size_t)cap * j.op.B;
        TRY(r.ct_hit.reserve(sizeof(float4) * n));
        TRY(r.ct_y.reserve(sizeof(float4) * n));
        TRY(r.ct_rr.reserve(sizeof(float) * n));
        const bool field = sc->mat_mode == MRS_MAT_FIELD;
        if (field) TRY(r.ct_fm.reserve(sizeof(float4) * n));
        for (const Chunk &ch : chunks) {
            Tape tp{r.ct_hit.as<float4>(), r.ct_y.as<float4>(), r.ct_rr.as<float>(), ch.c0, cap,
                    field ? r.ct_fm.as<float4>() : nullptr};
            TRY(run_wavefront(j, ch, tp, 1, nullptr, r, s));
            TRY(adjoint(j, tp, ch.c0, ch.c1, dimg, grads, gl, rec, r, s));
        }
    }
    grad_rec_fold(sc, gl, rec, grads, s);
    return MRS_OK;
}

// eager calls share one workspace; a call on another stream first waits for
// the previous call to finish with it
mrs_status begin(hipStream_t s) {
    Workspace &w = g_ws;
    if (!w.done) HIPTRY(hipEventCreateWithFlags(&w.done, hipEventDisableTiming), "hipEventCreate");
    if (w.has_last && w.last != s) HIPTRY(hipStreamWaitEvent(s, w.done, 0), "hipStreamWaitEvent");
    return MRS_OK;
}
mrs_status finish(hipStream_t s) {
    Workspace &w = g_ws;
    HIPTRY(hipGetLastError(), "kernel launch");
    HIPTRY(hipEventRecord(w.done, s), "hipEventRecord");
    w.last = s;
    w.has_last = true;
    return MRS_OK;
}

// view table through pinned staging, reused once the previous call is done;
// skipped when the device already holds the same table (repeated calls over
// the same views, as in an optimisation loop)
mrs_status upload_views_eager(Job &job, hipStream_t s) {
    Workspace &w = g_ws;
    size_t nv = job.vd.size();
    job.vt.v = w.res.views.as<ViewDev>();
    job.vt.n = (int)nv;
    if (w.res.views.p && w.uploaded.size() == nv &&
        std::memcmp(w.uploaded.data(), job.vd.data(), sizeof(ViewDev) * nv) == 0)
        return MRS_OK;
    w.uploaded.clear();
    if (w.done) HIPTRY(hipEventSynchronize(w.done), "hipEventSynchronize");
    if (w.staging_n < nv) {
        if (w.staging) HIPTRY(hipHostFree(w.staging), "hipHostFree");
        w.staging = nullptr;
        w.staging_n = 0;
        HIPTRY(hipHostMalloc((void **)&w.staging, sizeof(ViewDev) * nv, hipHostMallocDefault), "hipHostMalloc");
        w.staging_n = nv;
    }
    std::memcpy(w.staging, job.vd.data(), sizeof(ViewDev) * nv);
    TRY(w.res.views.reserve(sizeof(ViewDev) * nv));
    HIPTRY(hipMemcpyAsync(w.res.views.p, w.staging, sizeof(ViewDev) * nv, hipMemcpyHostToDevice, s), "copy views");
    job.vt.v = w.res.views.as<ViewDev>();
    w.uploaded = job.vd;
    return MRS_OK;
}

}  // namespace
}  // namespace mrs

using namespace mrs;

// ============================================================================
// eager entry points
// ============================================================================
extern "C" mrs_status mrs_render(const mrs_scene *scene, const mrs_view *views, int32_t n_views,
                                 const mrs_options *opt, float *d_image, mrs_tape **tape_out, void *stream) {
    clear_error();
    if (tape_out) *tape_out = nullptr;
    if (!d_image) return fail(MRS_EINVAL, "mrs_render: image is NULL");
    Job job;
    TRY(validate(scene, views, n_views, opt, job));
    std::lock_guard<std::mutex> lk(g_ws.mu);
    hipStream_t s = (hipStream_t)stream;
    TRY(begin(s));
    TRY(upload_views_eager(job, s));
    bind_scene(scene, job);
    mrs_tape *tape = nullptr;
    TRY(decide_tape(job, opt, tape_out != nullptr, &tape));
    mrs_status st = enqueue_forward(job, make_chunks(job, kOutChunkMax), scene, g_ws.res, tape, d_image,
                                    opt->debug_sample_rgb, opt->debug_hash, s);
    if (st == MRS_OK) st = finish(s);
    if (st != MRS_OK) { delete tape; return st; }
    if (tape_out) *tape_out = tape;
    return MRS_OK;
}

extern "C" mrs_status mrs_gbuffer(const mrs_scene *scene, const mrs_view *views, int32_t n_views, float *d_position,
                                  float *d_normal, void *stream) {
    clear_error();
    if (!d_position || !d_normal) return fail(MRS_EINVAL, "mrs_gbuffer: output is NULL");
    // the G-buffer samples nothing: any valid option set passes validation
    mrs_options opt{};
    opt.bounces = 1;
    opt.ris_m = 1;
    opt.rr_start = -1;
    opt.brdf = MRS_BRDF_LAMBERT_GGX;
    opt.background = MRS_BG_ENV;
    Job job;
    TRY(validate(scene, views, n_views, &opt, job));
    std::lock_guard<std::mutex> lk(g_ws.mu);
    hipStream_t s = (hipStream_t)stream;
    TRY(begin(s));
    TRY(upload_views_eager(job, s));
    bind_scene(scene, job);
    GbufArgs ga{job.sd.nodes, job.sd.tris, job.vt, job.pixels, d_position, d_normal};
    k_gbuffer<<<nblocks(job.pixels, 256), 256, kLdsStackBytes * 256, s>>>(ga);
    return finish(s);
}

extern "C" mrs_status mrs_render_backward(const mrs_scene *scene, const mrs_view *views, int32_t n_views,
                                          const mrs_options *opt, const float *d_grad_image, const mrs_grads *grads,
                                          const mrs_tape *tape, void *stream) {
    clear_error();
    if (!d_grad_image) return fail(MRS_EINVAL, "mrs_render_backward: grad image is NULL");
    if (!grads) return fail(MRS_EINVAL, "mrs_render_backward: grads is NULL");
    Job job;
    TRY(validate(scene, views, n_views, opt, job));
    if (tape && (tape->samples != job.S || tape->bounces != job.op.B || tape->seed != opt->seed ||
                 tape->signature != signature(job)))
        return fail(MRS_EINVAL, "mrs_render_backward: tape was recorded for different views or options");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    hipStream_t s = (hipStream_t)stream;
    TRY(begin(s));
    TRY(upload_views_eager(job, s));
    bind_scene(scene, job);
    std::vector<Chunk> chunks = make_chunks(job, std::min<uint64_t>(kOutChunkMax, job.S));
    TRY(enqueue_backward(job, chunks, scene, g_ws.res, tape, d_grad_image, grads, s));
    return finish(s);
}

extern "C" int64_t mrs_tape_bytes(const mrs_view *views, int32_t n_views, const mrs_options *opt) {
    if (!views || !opt || n_views < 1) return -1;
    uint64_t S = 0;
    for (int i = 0; i < n_views; ++i)
        S += (uint64_t)std::max(0, views[i].w) * std::max(0, views[i].h) * std::max(0, views[i].spp);
    return (int64_t)(S * (uint64_t)std::max(0, opt->bounces) * kTapeRecBytes);
}

extern "C" void mrs_tape_destroy(mrs_tape *t) {
    if (!t) return;
    // No wait here: the only writers of a recycled buffer are a later eager
    // render, which is ordered after every earlier eager call (same stream, or
    // the workspace's completion event), and plan creation, which synchronises
    // the device first.
    tape_recycle(t);
    delete t;
}

extern "C" mrs_status mrs_trace(const mrs_bvh *bvh, const float *d_orig, const float *d_dir, int64_t n,
                                int32_t any_hit, float *d_hit, void *stream) {
    clear_error();
    if (!bvh || !d_orig || !d_dir || !d_hit) return fail(MRS_EINVAL, "mrs_trace: null argument");
    if (n < 0) return fail(MRS_EINVAL, "mrs_trace: n < 0");
    if (n == 0) return MRS_OK;
    hipStream_t s = (hipStream_t)stream;
    {
        PROF(KID_TRACE, s);
        k_trace_batch<<<nblocks((uint64_t)n, 256), 256, kLdsStackBytes * 256, s>>>(bvh->wnodes.as<WideNode>(), bvh->tris.as<TriRec>(),
                                                               d_orig, d_dir, n, any_hit ? 1 : 0, (float4 *)d_hit);
    }
    return hip_check(hipGetLastError(), "mrs_trace launch");
}

extern "C" mrs_status mrs_profile_begin(void) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.recs.clear();
    g_prof.used = 0;
    g_prof.on = true;
    return MRS_OK;
}

extern "C" mrs_status mrs_profile_end(mrs_kernel_time *out, int32_t cap, int32_t *n) {
    clear_error();
    if (!out || !n) return fail(MRS_EINVAL, "mrs_profile_end: null output");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = false;
    double ms[KID_COUNT] = {0};
    int64_t cnt[KID_COUNT] = {0};
    for (const Profiler::Rec &r : g_prof.recs) {
        HIPTRY(hipEventSynchronize(r.b), "hipEventSynchronize");
        float t = 0.0f;
        HIPTRY(hipEventElapsedTime(&t, r.a, r.b), "hipEventElapsedTime");
        ms[r.kid] += t;
        cnt[r.kid] += 1;
    }
    g_prof.recs.clear();
    g_prof.used = 0;
    int32_t k = 0;
    for (int i = 0; i < KID_COUNT && k < cap; ++i) {
        if (!cnt[i]) continue;
        std::memset(out[k].name, 0, sizeof(out[k].name));
        std::strncpy(out[k].name, kKernelNames[i], sizeof(out[k].name) - 1);
        out[k].launches = cnt[i];
        out[k].ms = ms[i];
        ++k;
    }
    *n = k;
    return MRS_OK;
}

#ifdef MRS_COUNT_VISITS
// measurement builds only: read and clear the traversal visit counters
extern "C" int mrs_debug_visits(unsigned long long out[4]) {
    if (hipDeviceSynchronize() != hipSuccess) return -1;
    if (hipMemcpyFromSymbol(out, HIP_SYMBOL(g_visit_counts), sizeof(unsigned long long) * 4) != hipSuccess) return -1;
    unsigned long long z[4] = {0, 0, 0, 0};
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_visit_counts), z, sizeof(z)) != hipSuccess) return -1;
    return 0;
}
#endif

extern "C" void mrs_release_workspace(void) {
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if (g_ws.done) (void)hipEventSynchronize(g_ws.done);
    g_ws.res.release_all();
    g_ws.uploaded.clear();
    std::lock_guard<std::mutex> lk2(g_spare.mu);
    g_spare.hit.release(); g_spare.y.release(); g_spare.rr.release(); g_spare.fm.release();
    g_spare.device = -1;
}

// ============================================================================
// plans: buffers owned per plan, launch sequences captured once and replayed
// ============================================================================
struct mrs_plan {
    Job job;
    Res res;
    mrs_scene scene{};
    std::vector<Chunk> fwd_chunks, bwd_chunks;
    float *image = nullptr, *dbg_rgb = nullptr;
    uint32_t *dbg_hash = nullptr;
    const float *dimg = nullptr;
    mrs_grads grads{};
    bool has_grads = false;
    mrs_tape *tape = nullptr;   // owned; kept when the budget allows
    bool use_graph = false;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    ~mrs_plan() {
        for (hipGraphExec_t &e : exec)
            if (e) (void)hipGraphExecDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
        delete tape;
    }
};

namespace {

mrs_status plan_enqueue(mrs_plan *p, int pass, hipStream_t s) {
    if (pass == 0)
        return enqueue_forward(p->job, p->fwd_chunks, &p->scene, p->res, p->tape, p->image, p->dbg_rgb, p->dbg_hash, s);
    return enqueue_backward(p->job, p->bwd_chunks, &p->scene, p->res, p->tape, p->dimg, &p->grads, s);
}

// capture the pass on the plan's own stream; all buffers exist already, so
// the sequence is kernel launches only
mrs_status plan_capture(mrs_plan *p, int pass) {
    if (!p->cap) HIPTRY(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking), "hipStreamCreate");
    HIPTRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    t_capturing = true;
    mrs_status st = plan_enqueue(p, pass, p->cap);
    t_capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (st != MRS_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    HIPTRY(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->exec[pass], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPTRY(e, "hipGraphInstantiate");
    return MRS_OK;
}

mrs_status plan_run(mrs_plan *p, int pass, hipStream_t s) {
    if (!p->use_graph) {
        TRY(plan_enqueue(p, pass, s));
        HIPTRY(hipGetLastError(), "plan launch");
        return MRS_OK;
    }
    if (!p->exec[pass]) TRY(plan_capture(p, pass));
    PROF(pass == 0 ? KID_PLAN_FWD : KID_PLAN_BWD, s);
    HIPTRY(hipGraphLaunch(p->exec[pass], s), "hipGraphLaunch");
    return MRS_OK;
}

}  // namespace

extern "C" mrs_status mrs_plan_create(const mrs_scene *scene, const mrs_view *views, int32_t n_views,
                                      const mrs_options *opt, float *d_image, const float *d_grad_image,
                                      const mrs_grads *grads, int32_t use_graph, mrs_plan **out) {
    clear_error();
    if (!out) return fail(MRS_EINVAL, "mrs_plan_create: out is NULL");
    *out = nullptr;
    if (!d_image) return fail(MRS_EINVAL, "mrs_plan_create: image is NULL");
    if ((grads == nullptr) != (d_grad_image == nullptr))
        return fail(MRS_EINVAL, "mrs_plan_create: grads and grad image must both be given or both be NULL");
    mrs_plan *p = new mrs_plan();
    mrs_status st = validate(scene, views, n_views, opt, p->job);
    if (st != MRS_OK) { delete p; return st; }
    p->scene = *scene;
    p->image = d_image;
    p->dbg_rgb = opt->debug_sample_rgb;
    p->dbg_hash = opt->debug_hash;
    p->dimg = d_grad_image;
    if (grads) { p->grads = *grads; p->has_grads = true; }
    p->use_graph = use_graph != 0;
    Job &job = p->job;
    bind_scene(scene, job);
    p->fwd_chunks = make_chunks(job, kOutChunkMax);
    p->bwd_chunks = make_chunks(job, std::min<uint64_t>(kOutChunkMax, job.S));
#define PTRY(x) do { st = (x); if (st != MRS_OK) { delete p; return st; } } while (0)
    // every buffer the passes use is allocated now (captures must not allocate)
    PTRY(hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize"));
    PTRY(p->res.views.alloc(sizeof(ViewDev) * job.vd.size()));
    PTRY(hip_check(hipMemcpy(p->res.views.p, job.vd.data(), sizeof(ViewDev) * job.vd.size(), hipMemcpyHostToDevice),
                   "copy views"));
    job.vt.v = p->res.views.as<ViewDev>();
    job.vt.n = (int)job.vd.size();
    PTRY(reserve_env(scene, p->res));
    uint64_t outmax = std::max(max_chunk(p->fwd_chunks), max_chunk(p->bwd_chunks));
    uint32_t P = (uint32_t)std::min<uint64_t>(job.pool, outmax);
    int n_iter = 0;
    for (const std::vector<Chunk> *cs : {&p->fwd_chunks, &p->bwd_chunks})
        for (const Chunk &c : *cs)
            n_iter = std::max(n_iter, iterations(job, c.c1 - c.c0, (uint32_t)std::min<uint64_t>(job.pool, c.c1 - c.c0)));
    PTRY(reserve_pool(p->res, P, outmax, n_iter, scene->mat_mode == MRS_MAT_FIELD));
    PTRY(reserve_reuse(job, p->res));
    PTRY(reserve_tpack(scene, p->res));
    if (p->has_grads) {
        if (size_t words = grad_rec(scene, grads).words) PTRY(p->res.grec.reserve(4 * words));
        if (scene->mat_mode == MRS_MAT_FIELD) PTRY(reserve_field_vertices(job, job.S, p->res));
        PTRY(reserve_det_pairs(job, job.S, p->res));
        PTRY(decide_tape(job, opt, true, &p->tape));
        if (!p->tape) {
            size_t n = (size_t)max_chunk(p->bwd_chunks) * job.op.B;
            PTRY(p->res.ct_hit.alloc(sizeof(float4) * n));
            PTRY(p->res.ct_y.alloc(sizeof(float4) * n));
            PTRY(p->res.ct_rr.alloc(sizeof(float) * n));
            if (scene->mat_mode == MRS_MAT_FIELD) PTRY(p->res.ct_fm.alloc(sizeof(float4) * n));
        }
    }
#undef PTRY
    *out = p;
    return MRS_OK;
}

extern "C" mrs_status mrs_plan_forward(mrs_plan *plan, void *stream) {
    clear_error();
    if (!plan) return fail(MRS_EINVAL, "mrs_plan_forward: plan is NULL");
    return plan_run(plan, 0, (hipStream_t)stream);
}

extern "C" mrs_status mrs_plan_backward(mrs_plan *plan, void *stream) {
    clear_error();
    if (!plan) return fail(MRS_EINVAL, "mrs_plan_backward: plan is NULL");
    if (!plan->has_grads) return fail(MRS_EINVAL, "mrs_plan_backward: plan was created without gradient buffers");
    return plan_run(plan, 1, (hipStream_t)stream);
}

extern "C" mrs_status mrs_plan_info(const mrs_plan *plan, int64_t *samples, int32_t *keeps_tape, int32_t *graph) {
    clear_error();
    if (!plan) return fail(MRS_EINVAL, "mrs_plan_info: plan is NULL");
    if (samples) *samples = (int64_t)plan->job.S;
    if (keeps_tape) *keeps_tape = plan->tape != nullptr;
    if (graph) *graph = plan->use_graph;
    return MRS_OK;
}

extern "C" void mrs_plan_destroy(mrs_plan *plan) {
    if (!plan) return;
    (void)hipDeviceSynchronize();
    delete plan;
}
