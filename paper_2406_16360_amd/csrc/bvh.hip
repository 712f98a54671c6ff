// BVH builders for gfx950 (the paper builds an LBVH with its own kernels,
// Appendix A "Visibility estimation"):
//   triangle boxes -> centroid bounds -> 63-bit Morton codes -> sort of
//   (code, index) pairs, then either
//   - LBVH (Karras, "Maximizing parallelism in the construction of BVHs,
//     octrees and k-d trees", HPG 2012): binary radix tree from longest
//     common prefixes, bottom-up boxes with per-node arrival counters; or
//   - PLOC (Meister and Bittner, TVCG 2018): rounds of nearest-neighbour
//     merging over the same order, then a bottom-up sweep of treelet
//     restructuring (Karras and Aila, HPG 2013; treelet.h);
//   -> node layout with both child boxes per node, small subtrees collapsed
//   into leaves of <= kLeafMax triangles, triangles copied in leaf order;
//   then the traversal nodes (four quantised child boxes) over that tree.
// Refit moves the triangles to new vertex positions and recomputes the boxes
// over the unchanged tree (the per-iteration update while vertices move).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "device.h"
#include "runtime.h"
#include "treelet.h"

namespace mrs {

namespace {

__global__ void k_tri_bounds(const float *__restrict__ pos, const int32_t *__restrict__ faces, int nf,
                             float4 *__restrict__ lo, float4 *__restrict__ hi) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    V3 a = ld3(pos + 3 * (size_t)faces[3 * (size_t)f]);
    V3 b = ld3(pos + 3 * (size_t)faces[3 * (size_t)f + 1]);
    V3 c = ld3(pos + 3 * (size_t)faces[3 * (size_t)f + 2]);
    lo[f] = make_float4(fminf(a.x, fminf(b.x, c.x)), fminf(a.y, fminf(b.y, c.y)), fminf(a.z, fminf(b.z, c.z)), 0.f);
    hi[f] = make_float4(fmaxf(a.x, fmaxf(b.x, c.x)), fmaxf(a.y, fmaxf(b.y, c.y)), fmaxf(a.z, fmaxf(b.z, c.z)), 0.f);
}

// centroid bounds: one block-level reduction per block, then one block
// reduces the partials.  out[2 * blk] = min, out[2 * blk + 1] = max.
__global__ void k_centroid_bounds(const float4 *__restrict__ lo, const float4 *__restrict__ hi, int n,
                                  float4 *__restrict__ out) {
    __shared__ float smin[3][256], smax[3][256];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float4 l = lo[i], h = hi[i];
        float c[3] = {0.5f * (l.x + h.x), 0.5f * (l.y + h.y), 0.5f * (l.z + h.z)};
        for (int a = 0; a < 3; ++a) { mn[a] = fminf(mn[a], c[a]); mx[a] = fmaxf(mx[a], c[a]); }
    }
    for (int a = 0; a < 3; ++a) { smin[a][threadIdx.x] = mn[a]; smax[a][threadIdx.x] = mx[a]; }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int a = 0; a < 3; ++a) {
                smin[a][threadIdx.x] = fminf(smin[a][threadIdx.x], smin[a][threadIdx.x + s]);
                smax[a][threadIdx.x] = fmaxf(smax[a][threadIdx.x], smax[a][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = make_float4(smin[0][0], smin[1][0], smin[2][0], 0.f);
        out[2 * blockIdx.x + 1] = make_float4(smax[0][0], smax[1][0], smax[2][0], 0.f);
    }
}

__device__ __forceinline__ uint64_t spread21(uint64_t x) {
    x &= 0x1FFFFFull;
    x = (x | x << 32) & 0x1F00000000FFFFull;
    x = (x | x << 16) & 0x1F0000FF0000FFull;
    x = (x | x << 8) & 0x100F00F00F00F00Full;
    x = (x | x << 4) & 0x10C30C30C30C30C3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

__global__ void k_morton(const float4 *__restrict__ lo, const float4 *__restrict__ hi, int n, int npow2,
                         const float4 *__restrict__ bounds, uint64_t *__restrict__ keys, uint32_t *__restrict__ ids) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npow2) return;
    if (i >= n) { keys[i] = ~0ull; ids[i] = 0xFFFFFFFFu; return; }
    float4 bl = bounds[0], bh = bounds[1];
    float4 l = lo[i], h = hi[i];
    float c[3] = {0.5f * (l.x + h.x), 0.5f * (l.y + h.y), 0.5f * (l.z + h.z)};
    float blo[3] = {bl.x, bl.y, bl.z}, bhi[3] = {bh.x, bh.y, bh.z};
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
        float ext = bhi[a] - blo[a];
        float t = ext > 0.f ? (c[a] - blo[a]) / ext : 0.5f;
        t = fminf(fmaxf(t, 0.f), 1.f);
        q[a] = (uint64_t)fminf(t * 2097152.0f, 2097151.0f);
    }
    keys[i] = (spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]);
    ids[i] = (uint32_t)i;
}

// one merge step of a bitonic sort over (key, id) pairs (ids break ties)
__global__ void k_bitonic(uint64_t *__restrict__ keys, uint32_t *__restrict__ ids, int npow2, int j, int k) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npow2) return;
    int p = i ^ j;
    if (p <= i) return;
    uint64_t ka = keys[i], kb = keys[p];
    uint32_t ia = ids[i], ib = ids[p];
    bool a_gt_b = ka > kb || (ka == kb && ia > ib);
    bool up = (i & k) == 0;
    if (a_gt_b == up) { keys[i] = kb; keys[p] = ka; ids[i] = ib; ids[p] = ia; }
}

// the same step for all j < 512 inside a block, in LDS
__global__ void k_bitonic_local(uint64_t *__restrict__ keys, uint32_t *__restrict__ ids, int npow2, int k, int jmax) {
    __shared__ uint64_t sk[1024];
    __shared__ uint32_t si[1024];
    int base = blockIdx.x * 1024;
    for (int t = threadIdx.x; t < 1024; t += blockDim.x) { sk[t] = keys[base + t]; si[t] = ids[base + t]; }
    __syncthreads();
    for (int j = jmax; j > 0; j >>= 1) {
        for (int t = threadIdx.x; t < 1024; t += blockDim.x) {
            int p = t ^ j;
            if (p > t) {
                uint64_t ka = sk[t], kb = sk[p];
                uint32_t ia = si[t], ib = si[p];
                bool a_gt_b = ka > kb || (ka == kb && ia > ib);
                bool up = ((base + t) & k) == 0;
                if (a_gt_b == up) { sk[t] = kb; sk[p] = ka; si[t] = ib; si[p] = ia; }
            }
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < 1024; t += blockDim.x) { keys[base + t] = sk[t]; ids[base + t] = si[t]; }
}

// longest common prefix of sorted keys i and j; -1 outside [0, n); equal keys
// fall back to the indices (Karras 2012, Sec. 4)
__device__ __forceinline__ int delta(const uint64_t *__restrict__ keys, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint64_t a = keys[i], b = keys[j];
    if (a == b) return 64 + __clz((uint32_t)(i ^ j));
    return __clzll(a ^ b);
}

// internal node i covers the sorted range [first, last]; children are
// internal nodes (id < n - 1) or leaves (id = n - 1 + leaf index)
__global__ void k_karras(const uint64_t *__restrict__ keys, int n, int32_t *__restrict__ child,
                         int32_t *__restrict__ parent, int2 *__restrict__ range) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(keys, n, i, i - d);
    int lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = delta(keys, n, i, j);
    int s = 0, t, div = 2;
    do {
        t = (l + div - 1) / div;
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
        div *= 2;
    } while (t > 1);
    int g = i + s * d + min(d, 0);
    int first = min(i, j), last = max(i, j);
    int lc = (first == g) ? (n - 1 + g) : g;
    int rc = (last == g + 1) ? (n - 1 + g + 1) : g + 1;
    child[2 * i] = lc;
    child[2 * i + 1] = rc;
    parent[lc] = i;
    parent[rc] = i;
    range[i] = make_int2(first, last);
}

// bottom-up boxes: the second thread to reach a node merges its children
__global__ void k_boxes(const float4 *__restrict__ tlo, const float4 *__restrict__ thi,
                        const uint32_t *__restrict__ ids, int n, const int32_t *__restrict__ child,
                        const int32_t *__restrict__ parent, int32_t *__restrict__ flags,
                        float4 *__restrict__ blo, float4 *__restrict__ bhi) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int leaf = n - 1 + k;
    uint32_t f = ids[k];
    blo[leaf] = tlo[f];
    bhi[leaf] = thi[f];
    __threadfence();
    int node = parent[leaf];
    while (node >= 0) {
        if (atomicAdd(&flags[node], 1) == 0) return;
        __threadfence();
        int a = child[2 * node], b = child[2 * node + 1];
        float4 la = blo[a], lb = blo[b], ha = bhi[a], hb = bhi[b];
        blo[node] = make_float4(fminf(la.x, lb.x), fminf(la.y, lb.y), fminf(la.z, lb.z), 0.f);
        bhi[node] = make_float4(fmaxf(ha.x, hb.x), fmaxf(ha.y, hb.y), fmaxf(ha.z, hb.z), 0.f);
        __threadfence();
        node = parent[node];
    }
}

// boxes are widened by a relative epsilon so the FP32 slab test stays
// conservative for every triangle inside
__device__ __forceinline__ float pad_lo(float x) { return x - (fabsf(x) * 4e-7f + 1e-30f); }
__device__ __forceinline__ float pad_hi(float x) { return x + (fabsf(x) * 4e-7f + 1e-30f); }

__device__ __forceinline__ int32_t child_ref(int c, int n, const int2 *__restrict__ range) {
    if (c >= n - 1) return ~(((c - (n - 1)) << 3) | 0);
    int2 r = range[c];
    int cnt = r.y - r.x + 1;
    if (cnt <= kLeafMax) return ~((r.x << 3) | (cnt - 1));
    return c;
}

__global__ void k_layout(int n, const int32_t *__restrict__ child, const int2 *__restrict__ range,
                         const float4 *__restrict__ blo, const float4 *__restrict__ bhi, BvhNode *__restrict__ nodes) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= max(n - 1, 1)) return;
    BvhNode nd;
    if (n == 1) {   // a single triangle: root with one leaf and an empty child
        float4 l = blo[0], h = bhi[0];
        nd.n0 = make_float4(pad_lo(l.x), pad_hi(h.x), pad_lo(l.y), pad_hi(h.y));
        nd.n1 = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
        nd.n2 = make_float4(pad_lo(l.z), pad_hi(h.z), INFINITY, -INFINITY);
        nd.n3 = make_int4(~0, ~0, 0, 0);
        nodes[0] = nd;
        return;
    }
    int a = child[2 * i], b = child[2 * i + 1];
    float4 la = blo[a], ha = bhi[a], lb = blo[b], hb = bhi[b];
    nd.n0 = make_float4(pad_lo(la.x), pad_hi(ha.x), pad_lo(la.y), pad_hi(ha.y));
    nd.n1 = make_float4(pad_lo(lb.x), pad_hi(hb.x), pad_lo(lb.y), pad_hi(hb.y));
    nd.n2 = make_float4(pad_lo(la.z), pad_hi(ha.z), pad_lo(lb.z), pad_hi(hb.z));
    nd.n3 = make_int4(child_ref(a, n, range), child_ref(b, n, range), 0, 0);
    nodes[i] = nd;
}

// triangle of sorted position k to leaf slot slot[k] (k itself when slot is null)
__global__ void k_tris(const float *__restrict__ pos, const int32_t *__restrict__ faces,
                       const uint32_t *__restrict__ ids, const int32_t *__restrict__ slot, int n,
                       TriRec *__restrict__ tris) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t f = ids[k];
    V3 a = ld3(pos + 3 * (size_t)faces[3 * (size_t)f]);
    V3 b = ld3(pos + 3 * (size_t)faces[3 * (size_t)f + 1]);
    V3 c = ld3(pos + 3 * (size_t)faces[3 * (size_t)f + 2]);
    TriRec t;
    t.a = make_float4(a.x, a.y, a.z, __int_as_float((int)f));
    t.b = make_float4(b.x, b.y, b.z, 0.f);
    t.c = make_float4(c.x, c.y, c.z, 0.f);
    tris[slot ? slot[k] : k] = t;
}

// depth of every leaf (walk to the root); the maximum bounds the stack.
// Leaf k is node leaf_base + k.
__global__ void k_depth(const int32_t *__restrict__ parent, int n, int leaf_base, int32_t *__restrict__ out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int d = 0, node = parent[leaf_base + k];
    while (node >= 0 && d < 1 << 20) { ++d; node = parent[node]; }
    atomicMax(out, d);
}

// ---------------------------------------------------------------------------
// PLOC: parallel locally-ordered clustering (Meister and Bittner, TVCG 2018)
// over the same Morton order.  Node ids: leaves 0..n-1 (sorted positions),
// merged nodes n.. in creation order.  Each round finds every cluster's
// nearest neighbour within kPlocRadius positions (smallest surface area of
// the union box, ties to the lower position), merges mutual pairs into new
// nodes placed where the left one was, and compacts.  Merge ids and the
// compaction come from prefix sums, so the tree is deterministic.
// ---------------------------------------------------------------------------
constexpr int kPlocRadius = 32;
constexpr int kPlocBlock = 256;

__global__ void k_ploc_init(const float4 *__restrict__ tlo, const float4 *__restrict__ thi,
                            const uint32_t *__restrict__ ids, int n, float4 *__restrict__ nlo,
                            float4 *__restrict__ nhi, int32_t *__restrict__ clus, int32_t *__restrict__ cnt) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    nlo[k] = tlo[ids[k]];
    nhi[k] = thi[ids[k]];
    clus[k] = k;
    cnt[k] = 1;
}

__global__ __launch_bounds__(kPlocBlock) void k_ploc_nn(const int32_t *__restrict__ clus, int count,
                                                        const float4 *__restrict__ nlo, const float4 *__restrict__ nhi,
                                                        int32_t *__restrict__ nn) {
    __shared__ float4 slo[kPlocBlock + 2 * kPlocRadius], shi[kPlocBlock + 2 * kPlocRadius];
    const int base = blockIdx.x * kPlocBlock - kPlocRadius;
    for (int t = threadIdx.x; t < kPlocBlock + 2 * kPlocRadius; t += kPlocBlock) {
        int p = base + t;
        if (p >= 0 && p < count) {
            int c = clus[p];
            slo[t] = nlo[c];
            shi[t] = nhi[c];
        }
    }
    __syncthreads();
    const int i = blockIdx.x * kPlocBlock + threadIdx.x;
    if (i >= count) return;
    const int s = threadIdx.x + kPlocRadius;
    const float4 l = slo[s], h = shi[s];
    float best = INFINITY;
    int bj = -1;
    for (int d = -kPlocRadius; d <= kPlocRadius; ++d) {
        int j = i + d;
        if (d == 0 || j < 0 || j >= count) continue;
        float4 l2 = slo[s + d], h2 = shi[s + d];
        float a = box_half_area(make_float4(fminf(l.x, l2.x), fminf(l.y, l2.y), fminf(l.z, l2.z), 0.f),
                            make_float4(fmaxf(h.x, h2.x), fmaxf(h.y, h2.y), fmaxf(h.z, h2.z), 0.f));
        if (a < best) { best = a; bj = j; }
    }
    nn[i] = bj;
}

// merge[i]: i starts a mutual pair (i < nn[i]); keep[i]: i survives the round
__global__ void k_ploc_flags(const int32_t *__restrict__ nn, int count, int32_t *__restrict__ merge,
                             int32_t *__restrict__ keep) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int j = nn[i];
    bool mutual = j >= 0 && nn[j] == i;
    merge[i] = mutual && i < j;
    keep[i] = !(mutual && i > j);
}

// totals of the two exclusive scans: out = (merges, survivors)
__global__ void k_ploc_totals(const int32_t *__restrict__ merge, const int32_t *__restrict__ mo,
                              const int32_t *__restrict__ keep, const int32_t *__restrict__ ko, int count,
                              int32_t *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = mo[count - 1] + merge[count - 1];
        out[1] = ko[count - 1] + keep[count - 1];
    }
}

__global__ void k_ploc_merge(const int32_t *__restrict__ clus, const int32_t *__restrict__ nn, int count,
                             const int32_t *__restrict__ merge, const int32_t *__restrict__ mo,
                             const int32_t *__restrict__ keep, const int32_t *__restrict__ ko, int next_id,
                             float4 *__restrict__ nlo, float4 *__restrict__ nhi, int2 *__restrict__ child,
                             int32_t *__restrict__ parent, int32_t *__restrict__ cnt, int32_t *__restrict__ clus_next) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    if (merge[i]) {
        int id = next_id + mo[i];
        int a = clus[i], b = clus[nn[i]];
        float4 la = nlo[a], lb = nlo[b], ha = nhi[a], hb = nhi[b];
        nlo[id] = make_float4(fminf(la.x, lb.x), fminf(la.y, lb.y), fminf(la.z, lb.z), 0.f);
        nhi[id] = make_float4(fmaxf(ha.x, hb.x), fmaxf(ha.y, hb.y), fmaxf(ha.z, hb.z), 0.f);
        child[id] = make_int2(a, b);
        parent[a] = id;
        parent[b] = id;
        cnt[id] = cnt[a] + cnt[b];
        clus_next[ko[i]] = id;
    } else if (keep[i]) {
        clus_next[ko[i]] = clus[i];
    }
}

// One bottom-up sweep of treelet restructuring over PLOC's merge tree: a
// thread starts at every triangle and climbs; the second child to arrive at
// a node finishes it, its whole subtree being final then (per-node arrival
// counters, as for the LBVH boxes).  Nodes of at least kTreeletLeaves triangles are treelet
// roots, the others only take their cost.  A block is one wavefront, and its
// lanes search the subsets of each treelet root together, one root after
// another: the subsets of one size at a time (each needs only smaller ones),
// about 120 dependent steps per treelet instead of about 1000 for one lane
// alone.  The split choices are those of the one-thread search.
// One sweep by default: a second and third lowered traversal time by no more
// than run-to-run noise.
constexpr int kTreeletBlock = 64;
#ifndef MRS_TREELET_PASSES
#define MRS_TREELET_PASSES 1
#endif
__global__ void __launch_bounds__(kTreeletBlock) k_treelet(MergeTree t, int32_t *__restrict__ arrive) {
    __shared__ float s_cost[kTreeletSets];
    __shared__ uint8_t s_split[kTreeletSets];
    __shared__ float4 s_llo[kTreeletLeaves], s_lhi[kTreeletLeaves];   // the current treelet's leaves
    __shared__ int s_lcnt[kTreeletLeaves];
    const TreeletScratch w{s_cost, s_split, 1};
    const int lane = threadIdx.x;
    const int k = blockIdx.x * kTreeletBlock + lane;
    int node = -1;
    if (k < t.n) {
        t.cost[k] = subtree_cost(box_half_area(t.lo[k], t.hi[k]), 1, 0.0f, 0.0f);
        node = t.parent[k];
    }
    // every lane stays in the loop until the wavefront is done: the subset
    // search needs all of them
    while (__ballot(node >= 0) != 0) {
        __threadfence();
        if (node >= 0 && atomicAdd(&arrive[node - t.n], 1) == 0) node = -1;   // the first arrival stops
        __threadfence();
        const bool root = node >= 0 && t.cnt[node] >= kTreeletLeaves;
        if (node >= 0 && !root) {
            const int2 c = t.child[node];
            t.cost[node] = subtree_cost(box_half_area(t.lo[node], t.hi[node]), t.cnt[node], t.cost[c.x], t.cost[c.y]);
        }
        // the roots of this step lie in disjoint subtrees
        for (uint64_t roots = __ballot(root); roots != 0; roots &= roots - 1) {
            const int r = __shfl(node, __ffsll((unsigned long long)roots) - 1);
            Treelet tl;
            treelet_form(t, r, tl);
            if (lane == 0) {   // the leaves' boxes from LDS, not from each lane's private copy
#pragma unroll
                for (int q = 0; q < kTreeletLeaves; ++q) {
                    s_llo[q] = tl.llo[q];
                    s_lhi[q] = tl.lhi[q];
                    s_lcnt[q] = tl.lcnt[q];
                }
            }
            __syncthreads();
            const uint32_t nsets = 1u << tl.nl;
            for (int size = 1; size <= tl.nl; ++size) {
                for (uint32_t s = (uint32_t)lane + 1; s < nsets; s += kTreeletBlock)
                    if (__popc(s) == size) treelet_subset(t, tl, s_llo, s_lhi, s_lcnt, s, w);
                __syncthreads();
            }
            if (lane == 0) treelet_finish(t, r, tl, treelet_keep_cost(t, r), w);
            __syncthreads();   // the tables serve the next root
        }
        if (node >= 0) node = t.parent[node];
    }
}

// slot of leaf k in depth-first order (left subtree first)
__global__ void k_ploc_slots(const int32_t *__restrict__ parent, const int2 *__restrict__ child,
                             const int32_t *__restrict__ cnt, int n, int32_t *__restrict__ slot) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int p = 0, node = k;
    for (int par = parent[node]; par >= 0; node = par, par = parent[node]) {
        int2 c = child[par];
        if (c.y == node) p += cnt[c.x];
    }
    slot[k] = p;
}

// Binary node layout for merged node id (slot (2n - 2) - id, the root first):
// a child with at most kLeafMax triangles becomes a leaf over its contiguous
// depth-first triangle range.
__global__ void k_ploc_layout(int n, const int2 *__restrict__ child, const int32_t *__restrict__ cnt,
                              const int32_t *__restrict__ slot, const float4 *__restrict__ nlo,
                              const float4 *__restrict__ nhi, BvhNode *__restrict__ nodes) {
    int id = n + blockIdx.x * blockDim.x + threadIdx.x;
    if (id > 2 * n - 2) return;
    int2 ch = child[id];
    int c2[2] = {ch.x, ch.y}, ref[2];
    for (int q = 0; q < 2; ++q) {
        int c = c2[q];
        if (cnt[c] <= kLeafMax) {
            int f = c;
            while (f >= n) f = child[f].x;   // leftmost leaf
            ref[q] = ~((slot[f] << 3) | (cnt[c] - 1));
        } else {
            ref[q] = (2 * n - 2) - c;
        }
    }
    float4 la = nlo[ch.x], ha = nhi[ch.x], lb = nlo[ch.y], hb = nhi[ch.y];
    BvhNode nd;
    nd.n0 = make_float4(pad_lo(la.x), pad_hi(ha.x), pad_lo(la.y), pad_hi(ha.y));
    nd.n1 = make_float4(pad_lo(lb.x), pad_hi(hb.x), pad_lo(lb.y), pad_hi(hb.y));
    nd.n2 = make_float4(pad_lo(la.z), pad_hi(ha.z), pad_lo(lb.z), pad_hi(hb.z));
    nd.n3 = make_int4(ref[0], ref[1], 0, 0);
    nodes[(2 * n - 2) - id] = nd;
}

// ---------------------------------------------------------------------------
// refit: new vertex positions over the unchanged tree
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *__restrict__ p, int n, int32_t v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// parent of every internal node slot, (slot << 1) | side; the root keeps -1
__global__ void k_node_parents(const BvhNode *__restrict__ nodes, int nnodes, int32_t *__restrict__ npar) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnodes) return;
    int4 r = nodes[i].n3;
    if (r.x >= 0) npar[r.x] = (i << 1) | 0;
    if (r.y >= 0) npar[r.y] = (i << 1) | 1;
}

// triangle records of the moved vertices (the face id travels in a.w)
__global__ void k_refit_tris(const float *__restrict__ pos, const int32_t *__restrict__ faces, int n,
                             TriRec *__restrict__ tris) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int f = __float_as_int(tris[q].a.w);
    V3 a = ld3(pos + 3 * (size_t)faces[3 * (size_t)f]);
    V3 b = ld3(pos + 3 * (size_t)faces[3 * (size_t)f + 1]);
    V3 c = ld3(pos + 3 * (size_t)faces[3 * (size_t)f + 2]);
    TriRec t;
    t.a = make_float4(a.x, a.y, a.z, __int_as_float(f));
    t.b = make_float4(b.x, b.y, b.z, 0.f);
    t.c = make_float4(c.x, c.y, c.z, 0.f);
    tris[q] = t;
}

__device__ __forceinline__ void leaf_box(const TriRec *__restrict__ tris, int ref, float4 &lo, float4 &hi) {
    const int code = ~ref, first = code >> 3, cnt = (code & 7) + 1;
    lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
    hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
    for (int q = first; q < first + cnt; ++q) {
        TriRec t = tris[q];
        lo.x = fminf(lo.x, fminf(t.a.x, fminf(t.b.x, t.c.x)));
        lo.y = fminf(lo.y, fminf(t.a.y, fminf(t.b.y, t.c.y)));
        lo.z = fminf(lo.z, fminf(t.a.z, fminf(t.b.z, t.c.z)));
        hi.x = fmaxf(hi.x, fmaxf(t.a.x, fmaxf(t.b.x, t.c.x)));
        hi.y = fmaxf(hi.y, fmaxf(t.a.y, fmaxf(t.b.y, t.c.y)));
        hi.z = fmaxf(hi.z, fmaxf(t.a.z, fmaxf(t.b.z, t.c.z)));
    }
}

// Bottom-up boxes over the node slots: a thread starts at every node whose
// children are both leaves and climbs; a node is finished by the thread that
// brings its last internal child (arrival counters, as in the build).  Child
// boxes are stored padded, as the build stores them; the unpadded node boxes
// feed the level above.
// One height of the refit: the nodes of height h (1 + the larger height of
// their inner children, leaves 0) take their boxes from their leaves'
// triangles and from their inner children, which earlier launches (smaller
// heights) have refitted; the launch boundary orders the levels, so no
// thread waits on another.  order[0, count) lists the level's node slots.
__global__ void k_refit_level(const int32_t *__restrict__ order, int count, BvhNode *__restrict__ nodes,
                              const TriRec *__restrict__ tris, float4 *__restrict__ nlo, float4 *__restrict__ nhi) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int node = order[t];
    const int4 r = nodes[node].n3;
    const int refs[2] = {r.x, r.y};
    float4 lo[2], hi[2];
    for (int q = 0; q < 2; ++q) {
        if (refs[q] < 0) leaf_box(tris, refs[q], lo[q], hi[q]);
        else { lo[q] = nlo[refs[q]]; hi[q] = nhi[refs[q]]; }
    }
    BvhNode &nd = nodes[node];
    nd.n0 = make_float4(pad_lo(lo[0].x), pad_hi(hi[0].x), pad_lo(lo[0].y), pad_hi(hi[0].y));
    nd.n1 = make_float4(pad_lo(lo[1].x), pad_hi(hi[1].x), pad_lo(lo[1].y), pad_hi(hi[1].y));
    nd.n2 = make_float4(pad_lo(lo[0].z), pad_hi(hi[0].z), pad_lo(lo[1].z), pad_hi(hi[1].z));
    nlo[node] = make_float4(fminf(lo[0].x, lo[1].x), fminf(lo[0].y, lo[1].y), fminf(lo[0].z, lo[1].z), 0.f);
    nhi[node] = make_float4(fmaxf(hi[0].x, hi[1].x), fmaxf(hi[0].y, hi[1].y), fmaxf(hi[0].z, hi[1].z), 0.f);
}

// first position of every height in the height-sorted node list (heights
// run without gaps from 1 to the root's)
__global__ void k_height_starts(const uint32_t *__restrict__ h, int n, int32_t *__restrict__ start) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (i == 0 || h[i] != h[i - 1])) start[h[i]] = i;
}

__global__ void k_iota(uint32_t *__restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

// Traversal nodes: a collapse of the binary tree into nodes of up to four
// children that minimises the summed surface area of the traversal nodes (the
// expected number of node fetches per ray under the surface-area model).  For
// a binary node n and j = 1..4 member slots of the traversal node above it,
//   S(n, 1) = A(n) + D(n, 4)        n heads a traversal node of its own,
//   S(n, j) = min(S(n, 1), D(n, j)) n may instead be opened, j >= 2,
//   D(n, k) = min over k1 of S(l, k1) + S(r, k - k1),
// with S = 0 for leaves and A(n) the surface area of n's box in its parent
// (the collapse of Ylitie, Karras and Laine, HPG 2017, for four children).
// The costs are computed bottom-up; the traversal nodes are then chosen from
// the root down, one level per launch.  A member of a traversal node is a
// binary node slot, (node << 1) | side, so that a refit takes its box and
// reference from the refitted slot and keeps the collapse.
__device__ __forceinline__ bool slot_of(const BvhNode &nd, int side, float &area, int &ref) {
    const float4 a = side ? nd.n1 : nd.n0;
    const float zl = side ? nd.n2.z : nd.n2.x, zh = side ? nd.n2.w : nd.n2.y;
    ref = side ? nd.n3.y : nd.n3.x;
    if (!(a.x <= a.y) || !(a.z <= a.w) || !(zl <= zh)) return false;   // empty slot
    const float dx = a.y - a.x, dy = a.w - a.z, dz = zh - zl;
    area = dx * dy + dy * dz + dz * dx;
    return true;
}
__device__ __forceinline__ float4 cost_of(const float4 *S, int ref) {
    return ref >= 0 ? S[ref] : make_float4(0.f, 0.f, 0.f, 0.f);
}
__device__ __forceinline__ float cost_j(float4 v, int j) { return j == 1 ? v.x : j == 2 ? v.y : j == 3 ? v.z : v.w; }
// D(n, k) from the children's costs a and b, with the best k1
__device__ __forceinline__ float split_cost(float4 a, float4 b, int k, int &k1) {
    float best = INFINITY;
    k1 = 1;
    for (int q = 1; q < k; ++q) {
        const float c = cost_j(a, q) + cost_j(b, k - q);
        if (c < best) { best = c; k1 = q; }
    }
    return best;
}

// S(n, 1..4) and the height of every binary node, bottom-up: a thread starts at every node
// whose children are both leaves and climbs; a node is finished by the thread
// that brings its last inner child (per-node arrival counters).
__global__ void k_wide_cost(int nnodes, const BvhNode *__restrict__ nodes, const int32_t *__restrict__ npar,
                            float4 *__restrict__ S, int32_t *__restrict__ arrive, uint32_t *__restrict__ height) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnodes) return;
    const int4 r0 = nodes[i].n3;
    if (r0.x >= 0 || r0.y >= 0) return;
    int node = i;
    while (true) {
        const BvhNode nd = nodes[node];
        const float4 a = cost_of(S, nd.n3.x), b = cost_of(S, nd.n3.y);
        float area = 0.0f;
        int ref, k1;
        const int p = npar[node];
        if (p >= 0) (void)slot_of(nodes[p >> 1], p & 1, area, ref);
        const float d2 = split_cost(a, b, 2, k1), d3 = split_cost(a, b, 3, k1), d4 = split_cost(a, b, 4, k1);
        const float s1 = area + d4;
        S[node] = make_float4(s1, fminf(s1, d2), fminf(s1, d3), fminf(s1, d4));
        height[node] = 1u + max(nd.n3.x >= 0 ? height[nd.n3.x] : 0u, nd.n3.y >= 0 ? height[nd.n3.y] : 0u);
        __threadfence();
        if (p < 0) break;
        const int parent = p >> 1;
        const int4 pr = nodes[parent].n3;
        const int need = (pr.x >= 0) + (pr.y >= 0);
        if (atomicAdd(&arrive[parent], 1) + 1 < need) break;
        __threadfence();
        node = parent;
    }
}

// level of the traversal node each binary node heads (-1: none); the root heads level 0
__global__ void k_wide_init(int32_t *__restrict__ level, int nnodes) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nnodes) level[i] = i == 0 ? 0 : -1;
}

// The members of every traversal node of level lv: the root's two slots share
// four members as D(n, 4) chose, and an inner slot with budget j >= 2 is
// opened when D(n, j) < S(n, 1) (depth first, left before right, so the
// members keep the tree's order).  Inner members head traversal nodes of the
// next level.  maxlv receives the deepest level.
__global__ void k_wide_level(const BvhNode *__restrict__ nodes, const float4 *__restrict__ S, int nnodes, int lv,
                             int32_t *__restrict__ level, int4 *__restrict__ cuts, int32_t *__restrict__ maxlv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnodes || level[i] != lv) return;
    // every stacked slot holds a budget >= 1 and the budgets sum to at most 4
    int st_slot[4], st_bud[4], sp = 0;
    int slot[4], ref[4];
    int n = 0;
    {
        const BvhNode nd = nodes[i];
        int k1, rf;
        float ar;
        (void)split_cost(cost_of(S, nd.n3.x), cost_of(S, nd.n3.y), 4, k1);
        const bool hl = slot_of(nd, 0, ar, rf), hr = slot_of(nd, 1, ar, rf);
        if (hl && hr) {
            st_slot[sp] = (i << 1) | 1; st_bud[sp++] = 4 - k1;
            st_slot[sp] = (i << 1) | 0; st_bud[sp++] = k1;
        } else if (hl || hr) {       // a one-triangle tree: the root has one slot
            st_slot[sp] = (i << 1) | (hl ? 0 : 1); st_bud[sp++] = 4;
        }
    }
    while (sp > 0) {
        --sp;
        const int sl = st_slot[sp], bud = st_bud[sp];
        float ar;
        int r;
        (void)slot_of(nodes[sl >> 1], sl & 1, ar, r);
        if (r < 0 || bud == 1 || cost_j(S[r], 1) <= cost_j(S[r], bud)) {
            slot[n] = sl; ref[n] = r; ++n;
            continue;
        }
        const BvhNode cn = nodes[r];
        int q1;
        (void)split_cost(cost_of(S, cn.n3.x), cost_of(S, cn.n3.y), bud, q1);
        st_slot[sp] = (r << 1) | 1; st_bud[sp++] = bud - q1;
        st_slot[sp] = (r << 1) | 0; st_bud[sp++] = q1;
    }
    int4 out = make_int4(-1, -1, -1, -1);
    int *o = &out.x;
    for (int c = 0; c < n; ++c) {
        o[c] = slot[c];
        if (ref[c] >= 0) level[ref[c]] = lv + 1;
    }
    cuts[i] = out;
    atomicMax(maxlv, lv);
}

// the smallest k with 253 * 2^k >= extent and 2^k >= one float ulp of
// magnitude m (decoded bounds then round by less than a quantum)
__device__ int wide_exponent(double extent, double m) {
    int k = -126;
    if (extent > 0.0) k = max(k, ilogb(extent / 253.0));
    while (ldexp(253.0, k) < extent) ++k;
    if (m > 0.0) k = max(k, ilogb(m) - 23);
    return min(k, 127);
}

// Traversal node of every binary node that heads one: the boxes of its
// members, quantised outwards against their union in double, one quantum of
// padding per side.
__global__ void k_wide_build(const BvhNode *__restrict__ nodes, int nnodes, const int32_t *__restrict__ level,
                             const int4 *__restrict__ cuts, WideNode *__restrict__ wn) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnodes || level[i] < 0) return;
    float lo[4][3], hi[4][3];
    int ref[4];
    int nc = 0;
    const int4 cut = cuts[i];
    const int cs[4] = {cut.x, cut.y, cut.z, cut.w};
    for (int c = 0; c < 4; ++c) {
        if (cs[c] < 0) continue;
        const BvhNode nd = nodes[cs[c] >> 1];
        const int side = cs[c] & 1;
        const float4 a = side ? nd.n1 : nd.n0;
        lo[nc][0] = a.x; hi[nc][0] = a.y; lo[nc][1] = a.z; hi[nc][1] = a.w;
        lo[nc][2] = side ? nd.n2.z : nd.n2.x; hi[nc][2] = side ? nd.n2.w : nd.n2.y;
        ref[nc] = side ? nd.n3.y : nd.n3.x;
        ++nc;
    }
    // members by surface area, largest first: any-hit traversal takes the
    // first hit member next, and a large one is the likelier to hold the
    // occluder (closest hit sorts the hit members by distance anyway)
    auto area = [&](int c) {
        const float dx = hi[c][0] - lo[c][0], dy = hi[c][1] - lo[c][1], dz = hi[c][2] - lo[c][2];
        return dx * dy + dy * dz + dz * dx;
    };
    for (int x = 1; x < nc; ++x)
        for (int y = x; y > 0 && area(y) > area(y - 1); --y) {
            for (int q = 0; q < 3; ++q) {
                float t = lo[y][q]; lo[y][q] = lo[y - 1][q]; lo[y - 1][q] = t;
                t = hi[y][q]; hi[y][q] = hi[y - 1][q]; hi[y - 1][q] = t;
            }
            const int r = ref[y]; ref[y] = ref[y - 1]; ref[y - 1] = r;
        }
    WideNode w;
    uint32_t meta = (uint32_t)nc << 24;
    uint32_t qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
    float org[3] = {0.0f, 0.0f, 0.0f};
    for (int ax = 0; ax < 3; ++ax) {
        double L = INFINITY, H = -INFINITY;
        for (int c = 0; c < nc; ++c) { L = fmin(L, (double)lo[c][ax]); H = fmax(H, (double)hi[c][ax]); }
        if (nc == 0) { L = 0.0; H = 0.0; }
        org[ax] = (float)L;                       // a float already: the smallest child bound
        const int k = wide_exponent(H - L, fmax(fabs(L), fabs(H)));
        meta |= (uint32_t)(k + 127) << (8 * ax);
        const double sc = ldexp(1.0, k);
        for (int c = 0; c < nc; ++c) {
            const double ql = floor(((double)lo[c][ax] - (double)org[ax]) / sc) - 1.0;
            const double qh = ceil(((double)hi[c][ax] - (double)org[ax]) / sc) + 1.0;
            qlo[ax] |= (uint32_t)fmin(fmax(ql, 0.0), 255.0) << (8 * c);
            qhi[ax] |= (uint32_t)fmin(fmax(qh, 0.0), 255.0) << (8 * c);
        }
    }
    for (int c = nc; c < 4; ++c) ref[c] = 0;
    w.a = make_float4(org[0], org[1], org[2], __uint_as_float(meta));
    w.q = make_uint4(qlo[0], qhi[0], qlo[1], qhi[1]);
    w.r = make_uint4(qlo[2], qhi[2], (uint32_t)ref[0], (uint32_t)ref[1]);
    w.s = make_uint4((uint32_t)ref[2], (uint32_t)ref[3], 0u, 0u);
    wn[i] = w;
}

__global__ void k_check_faces(const int32_t *__restrict__ faces, int nf, int nv, int32_t *__restrict__ bad) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    for (int k = 0; k < 3; ++k) {
        int v = faces[3 * (size_t)f + k];
        if (v < 0 || v >= nv) { atomicOr(bad, 1); return; }
    }
}

// Exclusive prefix sums of two int32 flag arrays at once (the merge and keep
// flags of a PLOC round): per-tile sums, one block scanning the tile sums,
// then each tile's outputs.  A thread owns kScanItems consecutive entries.
constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;
__device__ __forceinline__ int2 add2(int2 u, int2 v) { return make_int2(u.x + v.x, u.y + v.y); }

// in-place inclusive scan of sh[0 .. kScanThreads) (every thread of the block calls it)
__device__ __forceinline__ void block_scan2(int2 *sh) {
    const int t = threadIdx.x;
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int2 u = t >= off ? sh[t - off] : make_int2(0, 0);
        __syncthreads();
        sh[t] = add2(sh[t], u);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan2_tiles(const int32_t *__restrict__ a, const int32_t *__restrict__ b,
                                                              int n, int2 *__restrict__ part) {
    __shared__ int2 sh[kScanThreads];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int2 v = make_int2(0, 0);
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < n) { v.x += a[base + q]; v.y += b[base + q]; }
    sh[threadIdx.x] = v;
    __syncthreads();
    block_scan2(sh);
    if (threadIdx.x == kScanThreads - 1) part[blockIdx.x] = sh[kScanThreads - 1];
}

// exclusive scan of the nb tile sums in place, one block
__global__ void __launch_bounds__(kScanThreads) k_scan2_top(int2 *__restrict__ part, int nb) {
    __shared__ int2 sh[kScanThreads];
    int2 carry = make_int2(0, 0);
    for (int c = 0; c < nb; c += kScanThreads) {
        const int i = c + threadIdx.x;
        const int2 v = i < nb ? part[i] : make_int2(0, 0);
        sh[threadIdx.x] = v;
        __syncthreads();
        block_scan2(sh);
        const int2 incl = sh[threadIdx.x], total = sh[kScanThreads - 1];
        if (i < nb) part[i] = make_int2(carry.x + incl.x - v.x, carry.y + incl.y - v.y);
        carry = add2(carry, total);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan2_out(const int32_t *__restrict__ a, const int32_t *__restrict__ b,
                                                            int n, const int2 *__restrict__ part,
                                                            int32_t *__restrict__ oa, int32_t *__restrict__ ob) {
    __shared__ int2 sh[kScanThreads];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int2 v = make_int2(0, 0);
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < n) { v.x += a[base + q]; v.y += b[base + q]; }
    sh[threadIdx.x] = v;
    __syncthreads();
    block_scan2(sh);
    int2 run = add2(part[blockIdx.x], make_int2(sh[threadIdx.x].x - v.x, sh[threadIdx.x].y - v.y));
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < n) {
            oa[base + q] = run.x; ob[base + q] = run.y;
            run.x += a[base + q]; run.y += b[base + q];
        }
}

// the same exclusive sums for a short array, in one launch of one block
// that walks it tile by tile with a carry
constexpr int kScanOneMax = 1 << 16;
__global__ void __launch_bounds__(kScanThreads) k_scan2_one(const int32_t *__restrict__ a, const int32_t *__restrict__ b,
                                                            int n, int32_t *__restrict__ oa, int32_t *__restrict__ ob) {
    __shared__ int2 sh[kScanThreads];
    int2 carry = make_int2(0, 0);
    for (int c = 0; c < n; c += kScanTile) {
        const int base = c + threadIdx.x * kScanItems;
        int2 v = make_int2(0, 0);
        for (int q = 0; q < kScanItems; ++q)
            if (base + q < n) { v.x += a[base + q]; v.y += b[base + q]; }
        sh[threadIdx.x] = v;
        __syncthreads();
        block_scan2(sh);
        int2 run = add2(carry, make_int2(sh[threadIdx.x].x - v.x, sh[threadIdx.x].y - v.y));
        carry = add2(carry, sh[kScanThreads - 1]);
        __syncthreads();
        for (int q = 0; q < kScanItems; ++q)
            if (base + q < n) {
                oa[base + q] = run.x; ob[base + q] = run.y;
                run.x += a[base + q]; run.y += b[base + q];
            }
    }
}

inline int blocks(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }

}  // namespace

}  // namespace mrs

using namespace mrs;

namespace {

mrs_status build(const float *d_pos, int32_t nv, const int32_t *d_faces, int32_t nf, int32_t builder, void *stream,
                 mrs_bvh **out) {
    if (!out) return fail(MRS_EINVAL, "mrs_build_bvh: out is NULL");
    *out = nullptr;
    if (!d_pos || !d_faces) return fail(MRS_EINVAL, "mrs_build_bvh: null mesh pointer");
    if (nv <= 0 || nf <= 0) return fail(MRS_EINVAL, "mrs_build_bvh: nv and nf must be positive");
    if (nf > (1 << 27)) return fail(MRS_EOVERFLOW, "mrs_build_bvh: more than 2^27 triangles");
    hipStream_t s = (hipStream_t)stream;
    int n = nf;
    int npow2 = 1024;
    while (npow2 < n) npow2 *= 2;
    DevBuf tlo, thi, keys, ids, child, parent, range, flags, blo, bhi, part, depth, bad;
    DevBuf arrive, hgt, hsorted, hiota, hstart, sort_tmp;   // bottom-up passes, the refit's height order
    DevBuf pchild, cnt, clus, clus2, nn, mflag, kflag, mo, ko, tot, slot, scan_tmp, tcost, tarrive;   // PLOC
    const bool ploc = builder == MRS_BVH_PLOC && nf > 1;
    mrs_bvh *b = new mrs_bvh();
    b->nf = nf;
    b->nv = nv;
    b->nnodes = std::max(n - 1, 1);
    mrs_status st = MRS_OK;
#define TRY(x) do { st = (x); if (st != MRS_OK) goto done; } while (0)
    TRY(tlo.alloc(sizeof(float4) * n));
    TRY(thi.alloc(sizeof(float4) * n));
    TRY(keys.alloc(sizeof(uint64_t) * npow2));
    TRY(ids.alloc(sizeof(uint32_t) * npow2));
    TRY(child.alloc(sizeof(int32_t) * 2 * std::max(n - 1, 1)));
    TRY(parent.alloc(sizeof(int32_t) * (2 * n - 1)));
    TRY(range.alloc(sizeof(int2) * std::max(n - 1, 1)));
    TRY(flags.alloc(sizeof(int32_t) * std::max(n - 1, 1)));
    TRY(blo.alloc(sizeof(float4) * (2 * n - 1)));
    TRY(bhi.alloc(sizeof(float4) * (2 * n - 1)));
    TRY(part.alloc(sizeof(float4) * 2 * 257));
    TRY(depth.alloc(sizeof(int32_t)));
    TRY(bad.alloc(sizeof(int32_t)));
    TRY(b->nodes.alloc(sizeof(BvhNode) * b->nnodes));
    TRY(b->tris.alloc(sizeof(TriRec) * n));
    TRY(b->faces.alloc(sizeof(int32_t) * 3 * (size_t)n));
    TRY(hip_check(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s), "memset"));
    k_check_faces<<<blocks(n), 256, 0, s>>>(d_faces, nf, nv, (int32_t *)bad.p);
    {
        int32_t h_bad = 0;
        TRY(hip_check(hipMemcpyAsync(&h_bad, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy"));
        TRY(hip_check(hipStreamSynchronize(s), "sync"));
        if (h_bad) { st = fail(MRS_EINVAL, "mrs_build_bvh: face index out of [0, nv)"); goto done; }
    }
    TRY(hip_check(hipMemcpyAsync(b->faces.p, d_faces, sizeof(int32_t) * 3 * (size_t)n, hipMemcpyDeviceToDevice, s), "copy faces"));
    k_tri_bounds<<<blocks(n), 256, 0, s>>>(d_pos, d_faces, nf, (float4 *)tlo.p, (float4 *)thi.p);
    {
        // per-block partial (min, max) of the centroids, merged on the host
        int nb = std::min(256, blocks(n));
        k_centroid_bounds<<<nb, 256, 0, s>>>((float4 *)tlo.p, (float4 *)thi.p, n, (float4 *)part.p + 2);
        std::vector<float4> h(2 * nb);
        TRY(hip_check(hipMemcpyAsync(h.data(), (float4 *)part.p + 2, sizeof(float4) * 2 * nb, hipMemcpyDeviceToHost, s), "copy"));
        TRY(hip_check(hipStreamSynchronize(s), "sync"));
        float4 mn = h[0], mx = h[1];
        for (int i = 1; i < nb; ++i) {
            mn.x = std::min(mn.x, h[2 * i].x); mn.y = std::min(mn.y, h[2 * i].y); mn.z = std::min(mn.z, h[2 * i].z);
            mx.x = std::max(mx.x, h[2 * i + 1].x); mx.y = std::max(mx.y, h[2 * i + 1].y); mx.z = std::max(mx.z, h[2 * i + 1].z);
        }
        float4 hb[2] = {mn, mx};
        TRY(hip_check(hipMemcpyAsync(part.p, hb, sizeof(hb), hipMemcpyHostToDevice, s), "copy"));
        TRY(hip_check(hipStreamSynchronize(s), "sync"));
    }
    k_morton<<<blocks(npow2), 256, 0, s>>>((float4 *)tlo.p, (float4 *)thi.p, n, npow2, (float4 *)part.p,
                                         (uint64_t *)keys.p, (uint32_t *)ids.p);
    for (int k = 2; k <= npow2; k *= 2) {
        int j = k / 2;
        for (; j >= 512; j /= 2)
            k_bitonic<<<blocks(npow2), 256, 0, s>>>((uint64_t *)keys.p, (uint32_t *)ids.p, npow2, j, k);
        k_bitonic_local<<<npow2 / 1024, 256, 0, s>>>((uint64_t *)keys.p, (uint32_t *)ids.p, npow2, k, j);
    }
    TRY(hip_check(hipMemsetAsync(parent.p, 0xFF, sizeof(int32_t) * (2 * n - 1), s), "memset"));
    TRY(hip_check(hipMemsetAsync(depth.p, 0, sizeof(int32_t), s), "memset"));
    if (!ploc) {
        TRY(hip_check(hipMemsetAsync(flags.p, 0, sizeof(int32_t) * std::max(n - 1, 1), s), "memset"));
        if (n > 1)
            k_karras<<<blocks(n - 1), 256, 0, s>>>((uint64_t *)keys.p, n, (int32_t *)child.p, (int32_t *)parent.p,
                                                   (int2 *)range.p);
        k_boxes<<<blocks(n), 256, 0, s>>>((float4 *)tlo.p, (float4 *)thi.p, (uint32_t *)ids.p, n, (int32_t *)child.p,
                                          (int32_t *)parent.p, (int32_t *)flags.p, (float4 *)blo.p, (float4 *)bhi.p);
        k_layout<<<blocks(std::max(n - 1, 1)), 256, 0, s>>>(n, (int32_t *)child.p, (int2 *)range.p, (float4 *)blo.p,
                                                            (float4 *)bhi.p, (BvhNode *)b->nodes.p);
        k_tris<<<blocks(n), 256, 0, s>>>(d_pos, d_faces, (uint32_t *)ids.p, nullptr, n, (TriRec *)b->tris.p);
        k_depth<<<blocks(n), 256, 0, s>>>((int32_t *)parent.p, n, n - 1, (int32_t *)depth.p);
    } else {
        // rounds of nearest-neighbour merging until one cluster is left
        const size_t nn2 = 2 * (size_t)n - 1;
        TRY(pchild.alloc(sizeof(int2) * nn2));
        TRY(cnt.alloc(sizeof(int32_t) * nn2));
        for (DevBuf *d : {&clus, &clus2, &nn, &mflag, &kflag, &mo, &ko, &slot}) TRY(d->alloc(sizeof(int32_t) * n));
        TRY(tot.alloc(sizeof(int32_t) * 2));
        TRY(scan_tmp.alloc(sizeof(int2) * (size_t)blocks(n, kScanTile)));
        float4 *nlo = (float4 *)blo.p, *nhi = (float4 *)bhi.p;
        k_ploc_init<<<blocks(n), 256, 0, s>>>((float4 *)tlo.p, (float4 *)thi.p, (uint32_t *)ids.p, n, nlo, nhi,
                                              (int32_t *)clus.p, (int32_t *)cnt.p);
        int count = n, next_id = n, rounds = 0;
        while (count > 1) {
            k_ploc_nn<<<blocks(count, kPlocBlock), kPlocBlock, 0, s>>>((int32_t *)clus.p, count, nlo, nhi, (int32_t *)nn.p);
            k_ploc_flags<<<blocks(count), 256, 0, s>>>((int32_t *)nn.p, count, (int32_t *)mflag.p, (int32_t *)kflag.p);
            if (count <= kScanOneMax) {   // exclusive sums of the merge and keep flags
                k_scan2_one<<<1, kScanThreads, 0, s>>>((int32_t *)mflag.p, (int32_t *)kflag.p, count, (int32_t *)mo.p,
                                                       (int32_t *)ko.p);
            } else {
                const int nb = blocks(count, kScanTile);
                k_scan2_tiles<<<nb, kScanThreads, 0, s>>>((int32_t *)mflag.p, (int32_t *)kflag.p, count, (int2 *)scan_tmp.p);
                k_scan2_top<<<1, kScanThreads, 0, s>>>((int2 *)scan_tmp.p, nb);
                k_scan2_out<<<nb, kScanThreads, 0, s>>>((int32_t *)mflag.p, (int32_t *)kflag.p, count,
                                                        (const int2 *)scan_tmp.p, (int32_t *)mo.p, (int32_t *)ko.p);
            }
            k_ploc_totals<<<1, 64, 0, s>>>((int32_t *)mflag.p, (int32_t *)mo.p, (int32_t *)kflag.p, (int32_t *)ko.p,
                                           count, (int32_t *)tot.p);
            k_ploc_merge<<<blocks(count), 256, 0, s>>>((int32_t *)clus.p, (int32_t *)nn.p, count, (int32_t *)mflag.p,
                                                       (int32_t *)mo.p, (int32_t *)kflag.p, (int32_t *)ko.p, next_id,
                                                       nlo, nhi, (int2 *)pchild.p, (int32_t *)parent.p,
                                                       (int32_t *)cnt.p, (int32_t *)clus2.p);
            int32_t h_tot[2] = {0, 0};
            TRY(hip_check(hipGetLastError(), "ploc kernels"));
            TRY(hip_check(hipMemcpyAsync(h_tot, tot.p, sizeof(h_tot), hipMemcpyDeviceToHost, s), "copy"));
            TRY(hip_check(hipStreamSynchronize(s), "sync"));
            // the globally closest pair is always mutual, so every round merges
            if (h_tot[0] < 1 || h_tot[1] != count - h_tot[0] || ++rounds > n) {
                st = fail(MRS_EHIP, "mrs_build_bvh: clustering made no progress");
                goto done;
            }
            next_id += h_tot[0];
            count = h_tot[1];
            std::swap(clus.p, clus2.p);
        }
        // treelet restructuring of the merge tree: the clustering only pairs
        // nearby clusters, and a sweep rearranges small subtrees where that
        // left the surface-area cost high
        if (MRS_TREELET_PASSES > 0 && n >= kTreeletLeaves) {
            TRY(tcost.alloc(sizeof(float) * nn2));
            TRY(tarrive.alloc(sizeof(int32_t) * (n - 1)));
            const MergeTree mt{(int2 *)pchild.p, (int32_t *)parent.p, (int32_t *)cnt.p, nlo, nhi, (float *)tcost.p, n};
            for (int pass = 0; pass < MRS_TREELET_PASSES; ++pass) {
                k_fill_i32<<<blocks(n - 1), 256, 0, s>>>((int32_t *)tarrive.p, n - 1, 0);
                k_treelet<<<blocks(n, kTreeletBlock), kTreeletBlock, 0, s>>>(mt, (int32_t *)tarrive.p);
            }
        }
        k_ploc_slots<<<blocks(n), 256, 0, s>>>((int32_t *)parent.p, (int2 *)pchild.p, (int32_t *)cnt.p, n,
                                               (int32_t *)slot.p);
        k_ploc_layout<<<blocks(n - 1), 256, 0, s>>>(n, (int2 *)pchild.p, (int32_t *)cnt.p, (int32_t *)slot.p, nlo, nhi,
                                                    (BvhNode *)b->nodes.p);
        k_tris<<<blocks(n), 256, 0, s>>>(d_pos, d_faces, (uint32_t *)ids.p, (int32_t *)slot.p, n, (TriRec *)b->tris.p);
        k_depth<<<blocks(n), 256, 0, s>>>((int32_t *)parent.p, n, 0, (int32_t *)depth.p);
    }
    {
        int32_t h_depth = 0;
        TRY(hip_check(hipGetLastError(), "bvh kernels"));
        TRY(hip_check(hipMemcpyAsync(&h_depth, depth.p, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy"));
        TRY(hip_check(hipStreamSynchronize(s), "sync"));
        b->depth = h_depth;
        // a traversal node's members lie at most three binary levels below
        // it, and a triangle with d ancestors sits in a leaf at least d - 1
        // levels down, so its path meets at least ceil((d - 1) / 3) traversal
        // nodes; a tree that must overflow the stack is refused before the
        // collapse
        if (3 * ((h_depth + 1) / 3) + 2 > kStackSize) {
            st = fail(MRS_EOVERFLOW, "mrs_build_bvh: tree depth %d exceeds the traversal stack (%d entries)", h_depth,
                      kStackSize);
            goto done;
        }
    }
    // state for mrs_bvh_refit
    TRY(b->npar.alloc(sizeof(int32_t) * b->nnodes));
    TRY(b->nlo.alloc(sizeof(float4) * b->nnodes));
    TRY(b->nhi.alloc(sizeof(float4) * b->nnodes));
    TRY(arrive.alloc(sizeof(int32_t) * b->nnodes));
    TRY(hip_check(hipMemsetAsync(b->npar.p, 0xFF, sizeof(int32_t) * b->nnodes, s), "memset"));
    k_node_parents<<<blocks(b->nnodes), 256, 0, s>>>((BvhNode *)b->nodes.p, b->nnodes, (int32_t *)b->npar.p);
    // traversal nodes
    TRY(b->wnodes.alloc(sizeof(WideNode) * b->nnodes));
    TRY(b->wlevel.alloc(sizeof(int32_t) * b->nnodes));
    TRY(b->wcut.alloc(sizeof(int4) * b->nnodes));
    // the collapse costs live in nlo until the first refit needs it
    k_fill_i32<<<blocks(b->nnodes), 256, 0, s>>>((int32_t *)arrive.p, b->nnodes, 0);
    TRY(hgt.alloc(sizeof(uint32_t) * b->nnodes));
    k_wide_cost<<<blocks(b->nnodes), 256, 0, s>>>(b->nnodes, (const BvhNode *)b->nodes.p, (const int32_t *)b->npar.p,
                                                  (float4 *)b->nlo.p, (int32_t *)arrive.p, (uint32_t *)hgt.p);
    {   // the refit's order: node slots by height (stable, so slot order within a height)
        TRY(b->horder.alloc(sizeof(int32_t) * b->nnodes));
        TRY(hsorted.alloc(sizeof(uint32_t) * b->nnodes));
        TRY(hiota.alloc(sizeof(uint32_t) * b->nnodes));
        k_iota<<<blocks(b->nnodes), 256, 0, s>>>((uint32_t *)hiota.p, b->nnodes);
        TRY(sort_pairs_u32((const uint32_t *)hgt.p, (uint32_t *)hsorted.p, (const uint32_t *)hiota.p,
                           (uint32_t *)b->horder.p, (size_t)b->nnodes, sort_tmp, s));
        uint32_t h_top = 0;
        TRY(hip_check(hipMemcpyAsync(&h_top, (const uint32_t *)hsorted.p + (b->nnodes - 1), sizeof(uint32_t),
                                     hipMemcpyDeviceToHost, s), "copy"));
        TRY(hip_check(hipStreamSynchronize(s), "sync"));
        if (h_top < 1 || h_top > (uint32_t)b->nnodes) { st = fail(MRS_EHIP, "mrs_build_bvh: bad node heights"); goto done; }
        TRY(hstart.alloc(sizeof(int32_t) * (h_top + 2)));
        k_fill_i32<<<blocks(h_top + 2), 256, 0, s>>>((int32_t *)hstart.p, (int)h_top + 2, 0);
        k_height_starts<<<blocks(b->nnodes), 256, 0, s>>>((const uint32_t *)hsorted.p, b->nnodes, (int32_t *)hstart.p);
        b->hstart.assign(h_top + 2, 0);
        TRY(hip_check(hipMemcpyAsync(b->hstart.data(), hstart.p, sizeof(int32_t) * (h_top + 1), hipMemcpyDeviceToHost, s),
                      "copy"));
        TRY(hip_check(hipStreamSynchronize(s), "sync"));
        b->hstart[h_top + 1] = b->nnodes;
    }
    k_wide_init<<<blocks(b->nnodes), 256, 0, s>>>((int32_t *)b->wlevel.p, b->nnodes);
    k_fill_i32<<<1, 1, 0, s>>>((int32_t *)bad.p, 1, 0);      // receives the deepest traversal level
    for (int lv = 0; lv <= b->depth; ++lv)     // a level descends at least one binary level
        k_wide_level<<<blocks(b->nnodes), 256, 0, s>>>((const BvhNode *)b->nodes.p, (const float4 *)b->nlo.p,
                                                       b->nnodes, lv, (int32_t *)b->wlevel.p, (int4 *)b->wcut.p,
                                                       (int32_t *)bad.p);
    k_wide_build<<<blocks(b->nnodes), 256, 0, s>>>((const BvhNode *)b->nodes.p, b->nnodes, (const int32_t *)b->wlevel.p,
                                                   (const int4 *)b->wcut.p, (WideNode *)b->wnodes.p);
    TRY(hip_check(hipGetLastError(), "bvh parents and traversal nodes"));
    {
        int32_t h_lv = 0;
        TRY(hip_check(hipMemcpyAsync(&h_lv, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy"));
        TRY(hip_check(hipStreamSynchronize(s), "sync"));
        // a traversal node stacks at most 3 children, and a root-to-leaf path
        // meets at most h_lv + 1 traversal nodes
        if (3 * (h_lv + 1) + 2 > kStackSize) {
            st = fail(MRS_EOVERFLOW, "mrs_build_bvh: %d traversal levels exceed the traversal stack (%d entries)",
                      h_lv + 1, kStackSize);
            goto done;
        }
    }
#undef TRY
done:
    if (st != MRS_OK) { delete b; return st; }
    *out = b;
    return MRS_OK;
}

}  // namespace

extern "C" mrs_status mrs_build_bvh(const float *d_pos, int32_t nv, const int32_t *d_faces, int32_t nf,
                                    void *stream, mrs_bvh **out) {
    clear_error();
    return build(d_pos, nv, d_faces, nf, MRS_BVH_LBVH, stream, out);
}

extern "C" mrs_status mrs_build_bvh_with(const float *d_pos, int32_t nv, const int32_t *d_faces, int32_t nf,
                                         int32_t builder, void *stream, mrs_bvh **out) {
    clear_error();
    if (builder != MRS_BVH_LBVH && builder != MRS_BVH_PLOC) {
        if (out) *out = nullptr;
        return fail(MRS_EINVAL, "mrs_build_bvh_with: unknown builder %d", builder);
    }
    return build(d_pos, nv, d_faces, nf, builder, stream, out);
}

extern "C" void mrs_bvh_destroy(mrs_bvh *b) { delete b; }

extern "C" mrs_status mrs_bvh_refit(mrs_bvh *b, const float *d_pos, int32_t nv, void *stream) {
    clear_error();
    if (!b || !d_pos) return fail(MRS_EINVAL, "mrs_bvh_refit: null argument");
    if (nv != b->nv) return fail(MRS_EINVAL, "mrs_bvh_refit: %d vertices, the BVH was built for %d", nv, b->nv);
    hipStream_t s = (hipStream_t)stream;
    k_refit_tris<<<blocks(b->nf), 256, 0, s>>>(d_pos, (const int32_t *)b->faces.p, b->nf, (TriRec *)b->tris.p);
    for (size_t h = 1; h + 1 < b->hstart.size(); ++h) {   // one launch per height, leaves up
        const int first = b->hstart[h], count = b->hstart[h + 1] - first;
        k_refit_level<<<blocks(count), 256, 0, s>>>((const int32_t *)b->horder.p + first, count,
                                                    (BvhNode *)b->nodes.p, (const TriRec *)b->tris.p,
                                                    (float4 *)b->nlo.p, (float4 *)b->nhi.p);
    }
    k_wide_build<<<blocks(b->nnodes), 256, 0, s>>>((const BvhNode *)b->nodes.p, b->nnodes, (const int32_t *)b->wlevel.p,
                                                   (const int4 *)b->wcut.p, (WideNode *)b->wnodes.p);
    return hip_check(hipGetLastError(), "mrs_bvh_refit launch");
}

extern "C" mrs_status mrs_bvh_info(const mrs_bvh *b, int32_t *nf, int32_t *nodes, int32_t *depth) {
    clear_error();
    if (!b) return fail(MRS_EINVAL, "mrs_bvh_info: bvh is NULL");
    if (nf) *nf = b->nf;
    if (nodes) *nodes = b->nnodes;
    if (depth) *depth = b->depth;
    return MRS_OK;
}
