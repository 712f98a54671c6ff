// Material neural field F_m on gfx950: multi-resolution hash encoding and
// the 2-layer MLP (Sec. 3 "Intrinsic decomposition"; Appendix A "Network
// details"; encoding after Mueller et al., "Instant Neural Graphics
// Primitives with a Multiresolution Hash Encoding", SIGGRAPH 2022, Sec. 3),
// forward and pull-back.  The definition is spelled out at mrs_field in
// mirres.h.
//
// Work layout.  A wavefront takes a tile of 32 points.  Lanes l and l + 32
// encode the same point (l mod 32), each half-wave 8 of the 16 levels, so a
// lane issues 64 of the point's 128 corner gathers.  Half h holds levels
// 4(q >> 1) + 2h + (q & 1), q < 8, and its local feature s = 2q + j is the
// global feature drow(s, h) = 8(s >> 2) + 4h + (s & 3).
//
// v_mfma_f32_32x32x2f32 operand layout (lane l, half = l / 32):
//   A: lane l supplies A[l mod 32][half];  B: lane l supplies B[half][l mod 32];
//   D: register r of lane l holds D[drow(r, half)][l mod 32].
// First layer, Z1 = E W1^T: 16 steps, step s contracts features drow(s, 0)
// and drow(s, 1), A = the lane's encoding register s, B = W1[l mod 32][drow(s,
// half)]; lane l ends with hidden unit l mod 32 of points drow(r, half).
// Pull-back: dW1 = sum_p dz1_p e_p^T contracts over the points (A = dz1 in
// the layer's own output layout, B = e read back transposed from LDS), and
// dL/de = W1^T dz1 is a second chain whose output lands in the lanes that
// encoded each point (features drow(r, half) of point l mod 32), which then
// scatter it to the table with float atomics.  The second layer (32 -> 4) and
// the small transposes go through a per-wave LDS tile.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "device.h"

namespace mrs {
namespace {

constexpr int kFieldMaxL = MRS_FIELD_MAX_LEVELS;
constexpr int kFieldHidden = 32;
constexpr int kFieldOut = 4;
constexpr int kFieldTile = 32;       // points per wavefront
constexpr int kFieldStride = 33;     // LDS row stride (floats) of the transposes

typedef float f32x16 __attribute__((ext_vector_type(16)));

struct FieldDev {
    const float2 *table;             // [L][T]
    const float *w1, *b1, *w2, *b2;
    int L, I;                        // levels, features (2L)
    uint32_t tmask;                  // T - 1
    uint32_t log2T;
    double lo[3], inv[3];            // u = (x - lo) * inv, in double (see field_unit)
    int res[kFieldMaxL];             // N_l
    uint32_t dense;                  // bit l: level l indexed one-to-one
};

// host: validates the parameters and fills the device view
inline bool make_field_dev(const mrs_field *f, FieldDev &d, const char **why) {
    *why = nullptr;
    if (!f) { *why = "field is NULL"; return false; }
    if (!f->table || !f->w1 || !f->b1 || !f->w2 || !f->b2) { *why = "field array is NULL"; return false; }
    if (f->levels < 1 || f->levels > kFieldMaxL) { *why = "field levels out of [1, 16]"; return false; }
    if (f->log2_table < 1 || f->log2_table > MRS_FIELD_MAX_LOG2_TABLE) { *why = "field log2_table out of range"; return false; }
    if (f->n_min < 1 || f->n_max < f->n_min || f->n_max > MRS_FIELD_MAX_RES) { *why = "field resolutions out of range"; return false; }
    for (int a = 0; a < 3; ++a)
        if (!(f->hi[a] > f->lo[a]) || !std::isfinite(f->lo[a]) || !std::isfinite(f->hi[a])) {
            *why = "field box needs finite hi > lo";
            return false;
        }
    d.table = (const float2 *)f->table;
    d.w1 = f->w1; d.b1 = f->b1; d.w2 = f->w2; d.b2 = f->b2;
    d.L = f->levels;
    d.I = 2 * f->levels;
    d.log2T = (uint32_t)f->log2_table;
    d.tmask = (1u << f->log2_table) - 1u;
    for (int a = 0; a < 3; ++a) {
        d.lo[a] = (double)f->lo[a];
        d.inv[a] = 1.0 / ((double)f->hi[a] - (double)f->lo[a]);
    }
    d.dense = 0;
    const double g = f->levels > 1 ? std::log((double)f->n_max / (double)f->n_min) / (double)(f->levels - 1) : 0.0;
    for (int l = 0; l < kFieldMaxL; ++l) {
        int64_t N = l < f->levels ? (int64_t)std::floor((double)f->n_min * std::exp((double)l * g) + 1e-6) : 1;
        d.res[l] = (int)N;
        if (l < f->levels && (N + 1) * (N + 1) * (N + 1) <= ((int64_t)1 << f->log2_table)) d.dense |= 1u << l;
    }
    return true;
}

// blocks of a persistent pull-back: 16 single-wave blocks per CU, capped
// by the tiles
inline unsigned field_backward_blocks(uint64_t tiles) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    const uint64_t cap = (uint64_t)cus * 16;
    return (unsigned)(tiles < 1 ? 1 : (tiles < cap ? tiles : cap));
}

__device__ __forceinline__ int drow(int r, int half) { return 8 * (r >> 2) + 4 * half + (r & 3); }

// The 8 corners of the cell holding u at a level of resolution N: slots and
// trilinear weights (corner bit a set = upper vertex along axis a).  The
// cell and its fractions come from u N in double: at N = 2048 one float ulp
// of u moves the grid coordinate by about 1e-4 of a cell.
__device__ __forceinline__ void field_corners(const double (&u)[3], int N, bool dense, uint32_t tmask,
                                              uint32_t (&slot)[8], float (&w)[8], uint32_t (&c)[3]) {
    float t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double s = u[a] * (double)N;
        const int ci = min((int)floor(s), N - 1);
        c[a] = (uint32_t)ci;
        t[a] = (float)(s - (double)ci);
    }
    const uint32_t side = (uint32_t)N + 1u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t v0 = c[0] + (k & 1), v1 = c[1] + ((k >> 1) & 1), v2 = c[2] + ((k >> 2) & 1);
        w[k] = ((k & 1) ? t[0] : 1.0f - t[0]) * ((k & 2) ? t[1] : 1.0f - t[1]) * ((k & 4) ? t[2] : 1.0f - t[2]);
        slot[k] = dense ? v0 + side * (v1 + side * v2) : ((v0 ^ (v1 * 2654435761u) ^ (v2 * 805459861u)) & tmask);
    }
}

__device__ __forceinline__ void field_unit(const FieldDev &f, V3 x, double (&u)[3]) {
    u[0] = fmin(fmax(((double)x.x - f.lo[0]) * f.inv[0], 0.0), 1.0);
    u[1] = fmin(fmax(((double)x.y - f.lo[1]) * f.inv[1], 0.0), 1.0);
    u[2] = fmin(fmax(((double)x.z - f.lo[2]) * f.inv[2], 0.0), 1.0);
}

// level of this half-wave's step q (the two candidates are wave-uniform, so
// per-level constants stay in scalar registers)
__device__ __forceinline__ int half_level(int q, int half) { return 4 * (q >> 1) + 2 * half + (q & 1); }

// encoding of the lane's 8 levels: el[2q + j] = feature j of level half_level(q)
__device__ __forceinline__ void field_encode(const FieldDev &f, const double (&u)[3], bool valid, int half,
                                             float (&el)[16]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int la = 4 * (q >> 1) + (q & 1), lb = la + 2;
        const int l = half ? lb : la;
        el[2 * q] = 0.0f;
        el[2 * q + 1] = 0.0f;
        if (valid && l < f.L) {
            const int N = half ? f.res[lb] : f.res[la];
            const bool dense = (f.dense >> l) & 1u;
            uint32_t slot[8], cell[3];
            float w[8];
            field_corners(u, N, dense, f.tmask, slot, w, cell);
            const float2 *tab = f.table + ((size_t)l << f.log2T);
            float2 v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = tab[slot[k]];
            float e0 = 0.0f, e1 = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) { e0 += w[k] * v[k].x; e1 += w[k] * v[k].y; }
            el[2 * q] = e0;
            el[2 * q + 1] = e1;
        }
    }
}

// the B operands of the first layer for this lane: W1[l mod 32][drow(s, half)]
__device__ __forceinline__ void field_w1_cols(const FieldDev &f, int hid, int half, float (&w)[16]) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int feat = drow(s, half);
        w[s] = feat < f.I ? f.w1[hid * f.I + feat] : 0.0f;
    }
}

// the A operands of dL/de = W1^T dz1: W1[2s + half][l mod 32]
__device__ __forceinline__ void field_w1_rows(const FieldDev &f, int hid, int half, float (&w)[16]) {
#pragma unroll
    for (int s = 0; s < 16; ++s) w[s] = hid < f.I ? f.w1[(2 * s + half) * f.I + hid] : 0.0f;
}

__device__ __forceinline__ f32x16 field_layer1(const float (&el)[16], const float (&w1c)[16]) {
    f32x16 acc = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(el[s], w1c[s], acc, 0, 0, 0);
    return acc;
}

// second layer and sigmoid for point p = lane (lanes < 32), reading the
// hidden activations a[p][h] from the LDS tile
__device__ __forceinline__ void field_layer2(const FieldDev &f, const float *sT, int p, float (&m)[kFieldOut]) {
    float z[kFieldOut];
#pragma unroll
    for (int o = 0; o < kFieldOut; ++o) z[o] = f.b2[o];
#pragma unroll 8
    for (int h = 0; h < kFieldHidden; ++h) {
        const float a = sT[p * kFieldStride + h];
#pragma unroll
        for (int o = 0; o < kFieldOut; ++o) z[o] += f.w2[o * kFieldHidden + h] * a;
    }
#pragma unroll
    for (int o = 0; o < kFieldOut; ++o) m[o] = 1.0f / (1.0f + __expf(-z[o]));
}

// Points of a field launch.  get(i, x) gives the position of point i and
// whether it exists; count() bounds the point indices.
struct PointsArray {
    const float *x;
    uint64_t n;
    __device__ __forceinline__ uint64_t count() const { return n; }
    __device__ __forceinline__ uint64_t gindex(uint64_t i) const { return i; }
    __device__ __forceinline__ bool get(uint64_t i, V3 &p) const {
        if (i >= n) return false;
        p = V3{x[3 * i], x[3 * i + 1], x[3 * i + 2]};
        return true;
    }
};

// Forward: one tile of 32 points per 64-thread block.  m[i][4] = F(x_i).
template <class Src>
__global__ __launch_bounds__(64) void k_field_eval(FieldDev f, Src src, float *__restrict__ m) {
    __shared__ float sT[kFieldTile * kFieldStride];
    const int lane = threadIdx.x, half = lane >> 5, hid = lane & 31;
    const uint64_t i = (uint64_t)blockIdx.x * kFieldTile + hid;
    if ((uint64_t)blockIdx.x * kFieldTile >= src.count()) return;
    V3 x = V3{0, 0, 0};
    const bool valid = src.get(i, x);
    double u[3];
    field_unit(f, x, u);
    float el[16], w1c[16];
    field_encode(f, u, valid, half, el);
    field_w1_cols(f, hid, half, w1c);
    const f32x16 z = field_layer1(el, w1c);
    const float bh = f.b1[hid];
#pragma unroll
    for (int r = 0; r < 16; ++r) sT[drow(r, half) * kFieldStride + hid] = fmaxf(z[r] + bh, 0.0f);
    __syncthreads();
    if (half == 0 && valid) {
        float mo[kFieldOut];
        field_layer2(f, sT, hid, mo);
#pragma unroll
        for (int o = 0; o < kFieldOut; ++o) m[4 * i + o] = mo[o];
    }
}

struct FieldGrads { float *table, *w1, *b1, *w2, *b2; };

// 30-bit Morton code of u in [0, 1]^3 (10 bits per axis)
__device__ __forceinline__ uint32_t morton_spread10(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Sort keys of the pull-back's points: the Morton code of the point in the
// field's box for points that carry a gradient, all ones for the others
// (they sort last and are skipped).  Walking the points in this order makes
// a tile's 32 points a compact cluster, so its table atomics aggregate and
// share cache lines also for the spatially random bounce vertices.
template <class Src>
__global__ __launch_bounds__(256) void k_field_keys(FieldDev f, Src src, const float *__restrict__ g,
                                                    uint32_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= src.count()) return;
    uint32_t key = 0xFFFFFFFFu;
    V3 x;
    if ((g[4 * i] != 0.0f || g[4 * i + 1] != 0.0f || g[4 * i + 2] != 0.0f || g[4 * i + 3] != 0.0f) && src.get(i, x)) {
        double u[3];
        field_unit(f, x, u);
        const uint32_t q0 = (uint32_t)min(1023.0, u[0] * 1024.0), q1 = (uint32_t)min(1023.0, u[1] * 1024.0),
                       q2 = (uint32_t)min(1023.0, u[2] * 1024.0);
        key = morton_spread10(q0) | (morton_spread10(q1) << 1) | (morton_spread10(q2) << 2);
    }
    keys[i] = key;
    vals[i] = (uint32_t)i;
}

// the points of Src in the order of a permutation (from the key sort)
template <class Src>
struct PointsPerm {
    Src base; const uint32_t *perm;
    __host__ __device__ __forceinline__ uint64_t count() const { return base.count(); }
    __device__ __forceinline__ uint64_t gindex(uint64_t i) const { return perm[i]; }
    __device__ __forceinline__ bool get(uint64_t i, V3 &p) const { return i < count() && base.get(perm[i], p); }
};

// Table scatter of one level per half-wave: each pending lane adds w_k d_j
// into feature j of the slot of corner k (16 values).  Device-scope float
// atomics are carried out past L2, one memory-side request per cache line an
// instruction touches, so the values are not issued lane by lane:
//   - consecutive pending lanes of a half-wave whose points lie in the same
//     cell form a run (the points come in Morton order, so the points of a
//     cell are mostly adjacent); a segmented suffix sum over the half gives
//     each run's first lane the run's 16 totals;
//   - only those lanes issue: they stage their 16 (offset, value) pairs in
//     LDS, packed densely, corner pairs along x first (their slots are
//     adjacent on dense levels, and on hashed levels when the lower x is
//     even, since the x prime is 1), and the wavefront issues them
//     transposed: instruction j takes the pairs of runs 4j..4j+3, so it
//     touches a few cache lines instead of 64.
// Offsets count floats from the table gradient's base.  Every lane of the
// wavefront calls it.
constexpr int kScatterPairs = 16;
__device__ __forceinline__ void scatter_level(float *gtab, uint32_t base, const uint32_t (&slot)[8],
                                              const float (&w)[8], float d0, float d1, const uint32_t (&cell)[3],
                                              bool pending, uint32_t *s_off, float *s_val) {
    const int lane = __lane_id(), hl = lane & 31;
    const uint64_t pm = __ballot(pending);
    if (pm == 0) return;
    const uint32_t q0 = __shfl_up(cell[0], 1), q1 = __shfl_up(cell[1], 1), q2 = __shfl_up(cell[2], 1);
    const bool prev_pending = hl > 0 && ((pm >> (lane - 1)) & 1ull);
    const bool head = pending && (!prev_pending || q0 != cell[0] || q1 != cell[1] || q2 != cell[2]);
    const uint64_t hm = __ballot(head);
    float v[kScatterPairs];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[2 * k] = pending ? w[k] * d0 : 0.0f;
        v[2 * k + 1] = pending ? w[k] * d1 : 0.0f;
    }
    if (hm != pm) {   // some run has more than one lane
        // last lane of this lane's run: before the next head or non-pending
        // lane of the same half
        const uint64_t bnd = hm | ~pm;
        const uint64_t half_mask = lane < 32 ? 0x00000000FFFFFFFFull : 0xFFFFFFFF00000000ull;
        const uint64_t after = lane == 63 ? 0ull : (~0ull << (lane + 1));
        const uint64_t nb = bnd & half_mask & after;
        const int end = nb ? __ffsll((unsigned long long)nb) - 2 : (lane < 32 ? 31 : 63);
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
#pragma unroll
            for (int e = 0; e < kScatterPairs; ++e) {
                const float t = __shfl_down(v[e], o);
                if (lane + o <= end) v[e] += t;
            }
        }
    }
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int pos = kScatterPairs * __popcll(hm & below);
    if (head) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            s_off[pos + 2 * k] = base + 2 * slot[k];
            s_off[pos + 2 * k + 1] = base + 2 * slot[k] + 1;
            s_val[pos + 2 * k] = v[2 * k];
            s_val[pos + 2 * k + 1] = v[2 * k + 1];
        }
    }
    const int total = kScatterPairs * __popcll(hm);
    __syncthreads();
    for (int e = lane; e < total; e += 64) atomicAdd(gtab + s_off[e], s_val[e]);
    __syncthreads();
}

#ifndef MRS_FIELD_BWD_WAVES
#define MRS_FIELD_BWD_WAVES 2
#endif
template <class Src>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MRS_FIELD_BWD_WAVES)))
void k_field_backward(FieldDev f, Src src, const float *__restrict__ g, FieldGrads out) {
    __shared__ float sT[kFieldTile * kFieldStride];
    __shared__ float4 sG[kFieldTile];
    __shared__ uint32_t s_off[64 * kScatterPairs];
    __shared__ float s_val[64 * kScatterPairs];
    const int lane = threadIdx.x, half = lane >> 5, hid = lane & 31;
    const uint64_t ntiles = (src.count() + kFieldTile - 1) / kFieldTile;
    float w1c[16], w1r[16];
    field_w1_cols(f, hid, half, w1c);
    field_w1_rows(f, hid, half, w1r);
    const float bh = f.b1[hid];
    float w2h[kFieldOut];
#pragma unroll
    for (int o = 0; o < kFieldOut; ++o) w2h[o] = f.w2[o * kFieldHidden + hid];
    f32x16 gw1 = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    float gw2[kFieldOut] = {0.0f, 0.0f, 0.0f, 0.0f}, gb2[kFieldOut] = {0.0f, 0.0f, 0.0f, 0.0f}, gb1 = 0.0f;
    // each block walks a contiguous range of tiles: with the points in Morton
    // order its tiles are neighbours, so their table lines stay in cache
    const uint64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint64_t tb = blockIdx.x * per, te = tb + per < ntiles ? tb + per : ntiles;
    for (uint64_t t = tb; t < te; ++t) {
        const uint64_t i = t * kFieldTile + hid;
        V3 x = V3{0, 0, 0};
        bool valid = src.get(i, x);
        float gi[kFieldOut] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (valid) {
            const uint64_t ig = src.gindex(i);
#pragma unroll
            for (int o = 0; o < kFieldOut; ++o) gi[o] = g[4 * ig + o];
            valid = gi[0] != 0.0f || gi[1] != 0.0f || gi[2] != 0.0f || gi[3] != 0.0f;
        }
        double u[3];
        field_unit(f, x, u);
        float el[16];
        field_encode(f, u, valid, half, el);
        const f32x16 z = field_layer1(el, w1c);
        // second layer for point `hid` (lanes < 32), then dz2 to every lane
#pragma unroll
        for (int r = 0; r < 16; ++r) sT[drow(r, half) * kFieldStride + hid] = fmaxf(z[r] + bh, 0.0f);
        __syncthreads();
        if (half == 0) {
            float mo[kFieldOut];
            field_layer2(f, sT, hid, mo);
            float4 d;
            d.x = valid ? gi[0] * mo[0] * (1.0f - mo[0]) : 0.0f;
            d.y = valid ? gi[1] * mo[1] * (1.0f - mo[1]) : 0.0f;
            d.z = valid ? gi[2] * mo[2] * (1.0f - mo[2]) : 0.0f;
            d.w = valid ? gi[3] * mo[3] * (1.0f - mo[3]) : 0.0f;
            sG[hid] = d;
        }
        __syncthreads();
        // dz1 in the first layer's output layout; second-layer and bias sums
        float dz1[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float4 d = sG[drow(r, half)];
            const float z1 = z[r] + bh, a = fmaxf(z1, 0.0f);
            const float da = w2h[0] * d.x + w2h[1] * d.y + w2h[2] * d.z + w2h[3] * d.w;
            dz1[r] = z1 > 0.0f ? da : 0.0f;
            gw2[0] += d.x * a; gw2[1] += d.y * a; gw2[2] += d.z * a; gw2[3] += d.w * a;
            gb2[0] += d.x; gb2[1] += d.y; gb2[2] += d.z; gb2[3] += d.w;
            gb1 += dz1[r];
        }
        // dW1 += sum over the tile's points of dz1 e^T (e transposed via LDS)
#pragma unroll
        for (int s = 0; s < 16; ++s) sT[hid * kFieldStride + drow(s, half)] = el[s];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 16; ++s)
            gw1 = __builtin_amdgcn_mfma_f32_32x32x2f32(dz1[s], sT[drow(s, half) * kFieldStride + hid], gw1, 0, 0, 0);
        __syncthreads();
        // dL/de = W1^T dz1 (dz1 transposed via LDS)
#pragma unroll
        for (int r = 0; r < 16; ++r) sT[drow(r, half) * kFieldStride + hid] = dz1[r];
        __syncthreads();
        f32x16 de = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 16; ++s)
            de = __builtin_amdgcn_mfma_f32_32x32x2f32(w1r[s], sT[hid * kFieldStride + 2 * s + half], de, 0, 0, 0);
        __syncthreads();
        // scatter dL/de of the lane's levels through the corner weights
        if (out.table) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int la = 4 * (q >> 1) + (q & 1), lb = la + 2;
                const int l = half ? lb : la;
                if (__ballot(valid && l < f.L) == 0) continue;
                const int N = half ? f.res[lb] : f.res[la];
                uint32_t slot[8], cell[3];
                float w[8];
                field_corners(u, N, (f.dense >> (l & 31)) & 1u, f.tmask, slot, w, cell);
                const uint32_t base = (uint32_t)(l < f.L ? l : 0) << (f.log2T + 1);
                scatter_level(out.table, base, slot, w, de[2 * q], de[2 * q + 1], cell, valid && l < f.L, s_off,
                              s_val);
            }
        }
    }
    if (out.w1) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            if (hid < f.I) atomicAdd(out.w1 + drow(r, half) * f.I + hid, gw1[r]);
    }
    if (out.w2) {
#pragma unroll
        for (int o = 0; o < kFieldOut; ++o) atomicAdd(out.w2 + o * kFieldHidden + hid, gw2[o]);
    }
    if (out.b1) atomicAdd(out.b1 + hid, gb1);
    if (out.b2 && hid == 0) {
#pragma unroll
        for (int o = 0; o < kFieldOut; ++o) atomicAdd(out.b2 + o, gb2[o]);
    }
}

}  // namespace
}  // namespace mrs
