// Edge-avoiding a-trous wavelet denoiser for gfx950, forward and adjoint
// (the paper's "Denoiser" paragraph, Appendix A, after Dammertz et al., HPG
// 2010).  Level i filters c_i into c_{i+1} over 5 x 5 taps spaced 2^i pixels
// apart with the B3-spline weights h = (1, 4, 6, 4, 1) / 16 and the
// edge-stopping product w_rt w_n w_x, Gaussians of the colour (of c_i),
// normal and position differences; the result is normalised by the weight
// sum k.  Taps outside a view are left out.
//
// Each workgroup filters a 16 x 16 pixel tile and stages the tile plus its
// 2 * 2^i pixel apron in LDS, so the 25 taps of a pixel read LDS.  The
// adjoint is the exact derivative (the colour weight depends on c_i) in
// gather form, so no atomics are needed:
//   dL/dc_r = sum_q a_rq (g_q / k_q - 2 / s_rt^2 (c_r - c_q)(s_rq + s_qr)),
//   s_rq = g_r . (c_q - out_r) / k_r,
// where a is symmetric (a_rq = a_qr), g = dL/dc_{i+1}, out = c_{i+1}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "device.h"
#include "runtime.h"

namespace mrs {
namespace {

#define HIPTRY_ST(x, what) do { mrs_status st_ = hip_check((x), what); if (st_ != MRS_OK) return st_; } while (0)
#define TRY_ST(x) do { mrs_status st_ = (x); if (st_ != MRS_OK) return st_; } while (0)

constexpr int kTile = 16;
__constant__ float kB3[5] = {1.0f / 16, 4.0f / 16, 6.0f / 16, 4.0f / 16, 1.0f / 16};

struct LevelArgs {
    const float *c, *n, *x;        // this level's colour, the normal and position buffers
    const float *g, *out, *k;      // adjoint only: dL/d out, out = c_{i+1}, normalisation
    float *dst, *kdst;             // forward: c_{i+1} and k; adjoint: dL/dc_i
    int w, h, stride;
    int64_t off;                   // first pixel of the view in the G-buffer (and g, out, k)
    int64_t coff, doff;            // first pixel of the view in c and in dst (and kdst)
    float inv_rt2, inv_n2, inv_x2; // 1 / sigma^2
};

__device__ __forceinline__ float sq3(float ax, float ay, float az) { return ax * ax + ay * ay + az * az; }

// tile loader: `fields` float3 arrays (each with the view's first pixel at
// its own offset), pixel (ty, tx) of the apron-padded tile
template <int kFields>
__device__ __forceinline__ void stage(const float *const (&src)[kFields], const int64_t (&off)[kFields], float *lds,
                                      int span, int x0, int y0, int w, int h) {
    for (int t = threadIdx.y * kTile + threadIdx.x; t < span * span; t += kTile * kTile) {
        int ty = t / span, tx = t - ty * span;
        int gx = x0 + tx, gy = y0 + ty;
        if (gx < 0 || gx >= w || gy < 0 || gy >= h) continue;
        int64_t p = (int64_t)gy * w + gx;
#pragma unroll
        for (int f = 0; f < kFields; ++f) {
            const float *s = src[f] + 3 * (off[f] + p);
            float *d = lds + (size_t)(f * 3) * span * span + t;
            d[0] = s[0];
            d[span * span] = s[1];
            d[2 * span * span] = s[2];
        }
    }
}

__global__ __launch_bounds__(kTile *kTile) void k_eawt(LevelArgs a) {
    extern __shared__ float tile[];   // 9 planes of span^2: c, n, x
    const int s = a.stride, apron = 2 * s, span = kTile + 2 * apron, area = span * span;
    const int x0 = blockIdx.x * kTile - apron, y0 = blockIdx.y * kTile - apron;
    const float *src[3] = {a.c, a.n, a.x};
    const int64_t offs[3] = {a.coff, a.off, a.off};
    stage<3>(src, offs, tile, span, x0, y0, a.w, a.h);
    __syncthreads();
    const int gx = blockIdx.x * kTile + threadIdx.x, gy = blockIdx.y * kTile + threadIdx.y;
    if (gx >= a.w || gy >= a.h) return;
    const int me = (threadIdx.y + apron) * span + threadIdx.x + apron;
    const float *C = tile, *N = tile + 3 * area, *X = tile + 6 * area;
    const float cr = C[me], cg = C[area + me], cb = C[2 * area + me];
    const float nx = N[me], ny = N[area + me], nz = N[2 * area + me];
    const float px = X[me], py = X[area + me], pz = X[2 * area + me];
    float k = 0.0f, sr = 0.0f, sg = 0.0f, sb = 0.0f;
    for (int dy = -2; dy <= 2; ++dy) {
        const int qy = gy + dy * s;
        if (qy < 0 || qy >= a.h) continue;
        for (int dx = -2; dx <= 2; ++dx) {
            const int qx = gx + dx * s;
            if (qx < 0 || qx >= a.w) continue;
            const int q = me + dy * s * span + dx * s;
            const float qr = C[q], qg = C[area + q], qb = C[2 * area + q];
            const float e = sq3(cr - qr, cg - qg, cb - qb) * a.inv_rt2 +
                            sq3(nx - N[q], ny - N[area + q], nz - N[2 * area + q]) * a.inv_n2 +
                            sq3(px - X[q], py - X[area + q], pz - X[2 * area + q]) * a.inv_x2;
            const float wq = kB3[dy + 2] * kB3[dx + 2] * __expf(-e);
            k += wq;
            sr += wq * qr; sg += wq * qg; sb += wq * qb;
        }
    }
    const int64_t p = a.doff + (int64_t)gy * a.w + gx;
    const float ik = 1.0f / k;
    a.dst[3 * p] = sr * ik; a.dst[3 * p + 1] = sg * ik; a.dst[3 * p + 2] = sb * ik;
    if (a.kdst) a.kdst[p] = k;
}

__global__ __launch_bounds__(kTile *kTile) void k_eawt_adjoint(LevelArgs a) {
    // 16 planes of span^2: c, n, x, g, out (3 each) and k
    extern __shared__ float tile[];
    const int s = a.stride, apron = 2 * s, span = kTile + 2 * apron, area = span * span;
    const int x0 = blockIdx.x * kTile - apron, y0 = blockIdx.y * kTile - apron;
    const float *src[5] = {a.c, a.n, a.x, a.g, a.out};
    const int64_t offs[5] = {a.coff, a.off, a.off, a.off, a.off};
    stage<5>(src, offs, tile, span, x0, y0, a.w, a.h);
    float *K = tile + 15 * area;
    for (int t = threadIdx.y * kTile + threadIdx.x; t < area; t += kTile * kTile) {
        int ty = t / span, tx = t - ty * span;
        int gx = x0 + tx, gy = y0 + ty;
        if (gx >= 0 && gx < a.w && gy >= 0 && gy < a.h) K[t] = a.k[a.off + (int64_t)gy * a.w + gx];
    }
    __syncthreads();
    const int gx = blockIdx.x * kTile + threadIdx.x, gy = blockIdx.y * kTile + threadIdx.y;
    if (gx >= a.w || gy >= a.h) return;
    const int me = (threadIdx.y + apron) * span + threadIdx.x + apron;
    const float *C = tile, *N = tile + 3 * area, *X = tile + 6 * area, *G = tile + 9 * area, *O = tile + 12 * area;
    const float cr = C[me], cg = C[area + me], cb = C[2 * area + me];
    const float nx = N[me], ny = N[area + me], nz = N[2 * area + me];
    const float px = X[me], py = X[area + me], pz = X[2 * area + me];
    const float gr = G[me], gg = G[area + me], gb = G[2 * area + me];
    const float orr = O[me], og = O[area + me], ob = O[2 * area + me];
    const float ik = 1.0f / K[me];
    const float two = 2.0f * a.inv_rt2;
    float dr = 0.0f, dg = 0.0f, db = 0.0f;
    for (int dy = -2; dy <= 2; ++dy) {
        const int qy = gy + dy * s;
        if (qy < 0 || qy >= a.h) continue;
        for (int dx = -2; dx <= 2; ++dx) {
            const int qx = gx + dx * s;
            if (qx < 0 || qx >= a.w) continue;
            const int q = me + dy * s * span + dx * s;
            const float qr = C[q], qg = C[area + q], qb = C[2 * area + q];
            const float e = sq3(cr - qr, cg - qg, cb - qb) * a.inv_rt2 +
                            sq3(nx - N[q], ny - N[area + q], nz - N[2 * area + q]) * a.inv_n2 +
                            sq3(px - X[q], py - X[area + q], pz - X[2 * area + q]) * a.inv_x2;
            const float aq = kB3[dy + 2] * kB3[dx + 2] * __expf(-e);
            const float gqr = G[q], gqg = G[area + q], gqb = G[2 * area + q];
            const float ikq = 1.0f / K[q];
            const float s_rq = (gr * (qr - orr) + gg * (qg - og) + gb * (qb - ob)) * ik;
            const float s_qr = (gqr * (cr - O[q]) + gqg * (cg - O[area + q]) + gqb * (cb - O[2 * area + q])) * ikq;
            const float m = two * (s_rq + s_qr);
            dr += aq * (gqr * ikq - m * (cr - qr));
            dg += aq * (gqg * ikq - m * (cg - qg));
            db += aq * (gqb * ikq - m * (cb - qb));
        }
    }
    const int64_t p = a.doff + (int64_t)gy * a.w + gx;
    a.dst[3 * p] = dr; a.dst[3 * p + 1] = dg; a.dst[3 * p + 2] = db;
}

mrs_status check(const mrs_view *views, int32_t n_views, const mrs_denoise_params *dp, uint64_t &P) {
    if (!views || !dp || n_views < 1 || n_views > MRS_MAX_VIEWS) return fail(MRS_EINVAL, "denoise: bad views");
    if (dp->levels < 1 || dp->levels > MRS_DENOISE_MAX_LEVELS)
        return fail(MRS_EINVAL, "denoise: levels must be in [1, %d]", MRS_DENOISE_MAX_LEVELS);
    if (!(dp->sigma_rt > 0.0f) || !(dp->sigma_n > 0.0f) || !(dp->sigma_x > 0.0f))
        return fail(MRS_EINVAL, "denoise: sigmas must be positive");
    P = 0;
    for (int v = 0; v < n_views; ++v) {
        if (views[v].w < 1 || views[v].h < 1) return fail(MRS_EINVAL, "denoise: view %d is empty", v);
        if (views[v].pixel_offset < 0) return fail(MRS_EINVAL, "denoise: view %d has a negative pixel_offset", v);
        P = std::max<uint64_t>(P, (uint64_t)views[v].pixel_offset + (uint64_t)views[v].w * views[v].h);
    }
    return MRS_OK;
}

size_t lds_bytes(int planes, int stride) {
    size_t span = kTile + 4 * (size_t)stride;
    return (size_t)planes * span * span * sizeof(float);
}

LevelArgs level_args(const mrs_view &v, const mrs_denoise_params *dp, int stride) {
    LevelArgs a{};
    a.w = v.w; a.h = v.h; a.stride = stride; a.off = a.coff = a.doff = v.pixel_offset;
    a.inv_rt2 = 1.0f / (dp->sigma_rt * dp->sigma_rt);
    a.inv_n2 = 1.0f / (dp->sigma_n * dp->sigma_n);
    a.inv_x2 = 1.0f / (dp->sigma_x * dp->sigma_x);
    return a;
}

dim3 grid_of(const mrs_view &v) { return dim3((v.w + kTile - 1) / kTile, (v.h + kTile - 1) / kTile); }

}  // namespace
}  // namespace mrs

using namespace mrs;

// Work layout (floats): c_0 .. c_L (L + 1 colour images of P x 3), then
// k_0 .. k_{L-1} (L images of P), then one colour image of adjoint scratch.
extern "C" int64_t mrs_denoise_work_bytes(const mrs_view *views, int32_t n_views, const mrs_denoise_params *dp) {
    uint64_t P = 0;
    if (check(views, n_views, dp, P) != MRS_OK) return -1;
    const uint64_t L = (uint64_t)dp->levels;
    return (int64_t)(sizeof(float) * P * (3 * (L + 1) + L + 3));
}

extern "C" mrs_status mrs_denoise(const mrs_view *views, int32_t n_views, const mrs_denoise_params *dp,
                                  const float *d_color_in, const float *d_normal, const float *d_position,
                                  float *d_color_out, float *d_work, void *stream) {
    clear_error();
    uint64_t P = 0;
    mrs_status st = check(views, n_views, dp, P);
    if (st != MRS_OK) return st;
    if (!d_color_in || !d_normal || !d_position || !d_color_out || !d_work) return fail(MRS_EINVAL, "mrs_denoise: null buffer");
    hipStream_t s = (hipStream_t)stream;
    const int L = dp->levels;
    float *cimg = d_work, *kimg = d_work + 3 * P * (L + 1);
    HIPTRY_ST(hipMemcpyAsync(cimg, d_color_in, sizeof(float) * 3 * P, hipMemcpyDeviceToDevice, s), "copy colour");
    for (int i = 0; i < L; ++i) {
        const int stride = 1 << i;
        for (int v = 0; v < n_views; ++v) {
            LevelArgs a = level_args(views[v], dp, stride);
            a.c = cimg + 3 * P * i; a.n = d_normal; a.x = d_position;
            a.dst = cimg + 3 * P * (i + 1); a.kdst = kimg + P * i;
            k_eawt<<<grid_of(views[v]), dim3(kTile, kTile), lds_bytes(9, stride), s>>>(a);
        }
    }
    HIPTRY_ST(hipMemcpyAsync(d_color_out, cimg + 3 * P * L, sizeof(float) * 3 * P, hipMemcpyDeviceToDevice, s),
              "copy colour");
    return hip_check(hipGetLastError(), "mrs_denoise launch");
}

extern "C" mrs_status mrs_denoise_backward(const mrs_view *views, int32_t n_views, const mrs_denoise_params *dp,
                                           const float *d_normal, const float *d_position, const float *d_work,
                                           const float *d_grad_out, float *d_grad_in, void *stream) {
    clear_error();
    uint64_t P = 0;
    mrs_status st = check(views, n_views, dp, P);
    if (st != MRS_OK) return st;
    if (!d_normal || !d_position || !d_work || !d_grad_out || !d_grad_in)
        return fail(MRS_EINVAL, "mrs_denoise_backward: null buffer");
    hipStream_t s = (hipStream_t)stream;
    const int L = dp->levels;
    const float *cimg = d_work, *kimg = d_work + 3 * P * (L + 1);
    float *scratch = const_cast<float *>(d_work) + 3 * P * (L + 1) + P * L;
    // ping-pong so that the last level (i = 0) writes d_grad_in
    const float *g = d_grad_out;
    for (int i = L - 1; i >= 0; --i) {
        float *dst = ((i & 1) == 0) ? d_grad_in : scratch;
        const int stride = 1 << i;
        for (int v = 0; v < n_views; ++v) {
            LevelArgs a = level_args(views[v], dp, stride);
            a.c = cimg + 3 * P * i; a.n = d_normal; a.x = d_position;
            a.g = g; a.out = cimg + 3 * P * (i + 1); a.k = kimg + P * i;
            a.dst = dst;
            k_eawt_adjoint<<<grid_of(views[v]), dim3(kTile, kTile), lds_bytes(16, stride), s>>>(a);
        }
        g = dst;
    }
    return hip_check(hipGetLastError(), "mrs_denoise_backward launch");
}

// ============================================================================
// The forward without a caller workspace, for callers that cannot allocate
// device memory.  The intermediate levels of one view live in `scratch`, a
// static device array that each GPU holds from the library's first use on it
// until the process ends.  Views are filtered one after another through the
// same two images, so the limit is per view.
// ============================================================================
namespace mrs {
namespace {

constexpr size_t kScratchFloats = MRS_DENOISE_SCRATCH_BYTES / sizeof(float);
static __device__ __align__(256) float scratch[kScratchFloats];

// Device address of `scratch` on each device, looked up once per device with
// that device current.  The host-side symbol is not a device address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

mrs_status scratch_ptr(float **out) {
    int dev = -1;
    HIPTRY_ST(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MRS_EUNSUPPORTED, "mrs_denoise_noalloc: device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPTRY_ST(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(MRS_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = (float *)p;
    }
    *out = g_scratch_ptr[dev];
    return MRS_OK;
}

// colour images of one view the intermediate levels need: none for one
// level, one for two, two (ping-pong) for more
uint64_t noalloc_images(int levels) { return (uint64_t)std::min(levels - 1, 2); }

}  // namespace
}  // namespace mrs

extern "C" mrs_status mrs_denoise_noalloc(const mrs_view *views, int32_t n_views, const mrs_denoise_params *dp,
                                          const float *d_color_in, const float *d_normal, const float *d_position,
                                          float *d_color_out, void *stream) {
    clear_error();
    uint64_t P = 0;
    mrs_status st = check(views, n_views, dp, P);
    if (st != MRS_OK) return st;
    if (!d_color_in || !d_normal || !d_position || !d_color_out)
        return fail(MRS_EINVAL, "mrs_denoise_noalloc: null buffer");
    const uintptr_t in0 = (uintptr_t)d_color_in, out0 = (uintptr_t)d_color_out, nb = sizeof(float) * 3 * P;
    if (in0 < out0 + nb && out0 < in0 + nb) return fail(MRS_EINVAL, "mrs_denoise_noalloc: output overlaps the input");
    const int L = dp->levels;
    const uint64_t imgs = noalloc_images(L);
    for (int v = 0; v < n_views; ++v) {
        const uint64_t need = imgs * 3 * (uint64_t)views[v].w * (uint64_t)views[v].h;
        if (need > kScratchFloats)
            return fail(MRS_EOVERFLOW, "mrs_denoise_noalloc: view %d (%dx%d, %d levels) needs %llu scratch bytes, the limit is %llu",
                        v, views[v].w, views[v].h, L, (unsigned long long)(sizeof(float) * need),
                        (unsigned long long)MRS_DENOISE_SCRATCH_BYTES);
    }
    float *scr = nullptr;
    if (imgs) TRY_ST(scratch_ptr(&scr));
    hipStream_t s = (hipStream_t)stream;
    for (int v = 0; v < n_views; ++v) {
        const uint64_t img = 3 * (uint64_t)views[v].w * (uint64_t)views[v].h;
        for (int i = 0; i < L; ++i) {
            const int stride = 1 << i;
            LevelArgs a = level_args(views[v], dp, stride);
            a.n = d_normal; a.x = d_position; a.kdst = nullptr;
            if (i == 0) { a.c = d_color_in; } else { a.c = scr + img * ((i - 1) & 1); a.coff = 0; }
            if (i == L - 1) { a.dst = d_color_out; } else { a.dst = scr + img * (i & 1); a.doff = 0; }
            k_eawt<<<grid_of(views[v]), dim3(kTile, kTile), lds_bytes(9, stride), s>>>(a);
        }
    }
    return hip_check(hipGetLastError(), "mrs_denoise_noalloc launch");
}
