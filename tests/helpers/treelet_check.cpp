// Host-side checks of the BVH builder's treelet restructuring (the same
// __host__ __device__ routine the build kernel runs), printed as
// "name ok|FAIL detail" lines:
//  - optimum: on a tree of k <= 7 triangles the treelet spans the whole tree,
//    so the rebuilt cost must equal the minimum over every full binary tree on
//    those triangles, enumerated explicitly ((2k - 3)!! trees, each costed
//    from scratch);
//  - sweep: bottom-up sweeps over random trees of up to 3000 triangles keep
//    every triangle exactly once, consistent parents, counts and boxes, the
//    stored costs equal to a fresh evaluation, and never raise the cost.
#include <cmath>
#include <cstdio>
#include <functional>
#include <random>
#include <vector>

#include "../../paper_2406_16360_amd/csrc/treelet.h"

using namespace mrs;

namespace {

struct Tree {
    int n;
    std::vector<int2> child;
    std::vector<int32_t> parent, cnt;
    std::vector<float4> lo, hi;
    std::vector<float> cost;
    int root = 0;
    MergeTree view() { return MergeTree{child.data(), parent.data(), cnt.data(), lo.data(), hi.data(), cost.data(), n}; }
};

float4 fmin4(float4 a, float4 b) { return make_float4(fminf(a.x, b.x), fminf(a.y, b.y), fminf(a.z, b.z), 0.0f); }
float4 fmax4(float4 a, float4 b) { return make_float4(fmaxf(a.x, b.x), fmaxf(a.y, b.y), fmaxf(a.z, b.z), 0.0f); }

// n random triangle boxes, then random merges of neighbouring clusters
Tree random_tree(int n, std::mt19937 &rng, bool flat) {
    std::uniform_real_distribution<float> U(0.0f, 1.0f);
    Tree t;
    t.n = n;
    const int nn = 2 * n - 1;
    t.child.assign(nn, make_int2(-1, -1));
    t.parent.assign(nn, -1);
    t.cnt.assign(nn, 1);
    t.lo.resize(nn);
    t.hi.resize(nn);
    t.cost.assign(nn, 0.0f);
    std::vector<int> clus;
    for (int i = 0; i < n; ++i) {
        const float cx = U(rng), cy = U(rng), cz = flat ? 0.5f : U(rng), s = 0.02f * U(rng);
        t.lo[i] = make_float4(cx - s, cy - s, flat ? cz : cz - s, 0.0f);
        t.hi[i] = make_float4(cx + s, cy + s, cz + s, 0.0f);
        clus.push_back(i);
    }
    std::shuffle(clus.begin(), clus.end(), rng);
    int next = n;
    while (clus.size() > 1) {
        const size_t a = rng() % clus.size(), b = (a + 1) % clus.size();
        const int x = clus[a], y = clus[b], id = next++;
        t.child[id] = make_int2(x, y);
        t.parent[x] = t.parent[y] = id;
        t.cnt[id] = t.cnt[x] + t.cnt[y];
        t.lo[id] = fmin4(t.lo[x], t.lo[y]);
        t.hi[id] = fmax4(t.hi[x], t.hi[y]);
        clus[a] = id;
        clus.erase(clus.begin() + (long)b);
    }
    t.root = clus[0];
    return t;
}

float fresh_cost(const Tree &t, int x) {
    const float a = box_half_area(t.lo[x], t.hi[x]);
    if (x < t.n) return subtree_cost(a, 1, 0.0f, 0.0f);
    return subtree_cost(a, t.cnt[x], fresh_cost(t, t.child[x].x), fresh_cost(t, t.child[x].y));
}

// one bottom-up sweep in post order (children before parents, as the
// kernel's arrival counters guarantee)
void sweep(Tree &t, TreeletScratch w) {
    std::vector<int> post;
    std::function<void(int)> rec = [&](int x) {
        if (x >= t.n) { rec(t.child[x].x); rec(t.child[x].y); }
        post.push_back(x);
    };
    rec(t.root);
    MergeTree v = t.view();
    for (int x : post) {
        if (x < t.n) { t.cost[x] = subtree_cost(box_half_area(t.lo[x], t.hi[x]), 1, 0.0f, 0.0f); continue; }
        if (t.cnt[x] >= kTreeletLeaves) treelet_optimize(v, x, w);
        else t.cost[x] = subtree_cost(box_half_area(t.lo[x], t.hi[x]), t.cnt[x], t.cost[t.child[x].x], t.cost[t.child[x].y]);
    }
}

bool valid(const Tree &t, const char **why) {
    if (t.n == 1) return true;
    std::vector<int> seen(2 * t.n - 1, 0);
    bool ok = t.parent[t.root] == -1;
    if (!ok) *why = "root has a parent";
    std::function<void(int, int)> rec = [&](int x, int depth) {
        if (!ok) return;
        if (x < 0 || x >= 2 * t.n - 1 || depth > 2 * t.n) { ok = false; *why = "bad reference"; return; }
        if (++seen[x] > 1) { ok = false; *why = "node reached twice"; return; }
        if (x < t.n) return;
        const int2 c = t.child[x];
        rec(c.x, depth + 1);
        rec(c.y, depth + 1);
        if (!ok) return;
        if (t.parent[c.x] != x || t.parent[c.y] != x) { ok = false; *why = "parent mismatch"; }
        else if (t.cnt[x] != t.cnt[c.x] + t.cnt[c.y]) { ok = false; *why = "count mismatch"; }
        else {
            const float4 l = fmin4(t.lo[c.x], t.lo[c.y]), h = fmax4(t.hi[c.x], t.hi[c.y]);
            if (l.x != t.lo[x].x || l.y != t.lo[x].y || l.z != t.lo[x].z || h.x != t.hi[x].x || h.y != t.hi[x].y ||
                h.z != t.hi[x].z) { ok = false; *why = "box is not the union of the children"; }
        }
    };
    rec(t.root, 0);
    for (size_t i = 0; ok && i < seen.size(); ++i)
        if (seen[i] != 1) { ok = false; *why = "node unreached"; }
    return ok;
}

// explicit trees over leaves 0..k-1: node lists (left, right) with ids >= k;
// every tree on k leaves comes from one on k - 1 by hanging the new leaf
// above one of its nodes
struct Shape { std::vector<int2> inner; int root; };
void all_shapes(int k, std::vector<Shape> &out) {
    std::vector<Shape> cur{Shape{{}, 0}};
    for (int leaf = 1; leaf < k; ++leaf) {
        std::vector<Shape> nxt;
        for (const Shape &s : cur) {
            const int nodes = leaf + (int)s.inner.size();   // ids 0..leaf-1 leaves, then inner
            for (int at = 0; at < nodes; ++at) {
                // new numbering: leaves 0..leaf, inner nodes from leaf + 1
                Shape z;
                auto re = [&](int id) { return id < leaf ? id : id + 1; };
                for (const int2 &c : s.inner) z.inner.push_back(make_int2(re(c.x), re(c.y)));
                const int tgt = re(at);
                const int fresh = leaf + 1 + (int)z.inner.size();
                for (int2 &c : z.inner) {
                    if (c.x == tgt) c.x = fresh;
                    if (c.y == tgt) c.y = fresh;
                }
                z.inner.push_back(make_int2(tgt, leaf));
                z.root = re(s.root) == tgt ? fresh : re(s.root);
                nxt.push_back(z);
            }
        }
        cur.swap(nxt);
    }
    out = cur;
}

float shape_cost(const Shape &s, int k, const std::vector<float4> &lo, const std::vector<float4> &hi, int x,
                 float4 &bl, float4 &bh, int &cnt) {
    if (x < k) { bl = lo[x]; bh = hi[x]; cnt = 1; return subtree_cost(box_half_area(bl, bh), 1, 0.0f, 0.0f); }
    const int2 c = s.inner[x - k];
    float4 l1, h1, l2, h2;
    int c1, c2;
    const float a = shape_cost(s, k, lo, hi, c.x, l1, h1, c1), b = shape_cost(s, k, lo, hi, c.y, l2, h2, c2);
    bl = fmin4(l1, l2);
    bh = fmax4(h1, h2);
    cnt = c1 + c2;
    return subtree_cost(box_half_area(bl, bh), cnt, a, b);
}

}  // namespace

int main() {
    int fails = 0;
    std::vector<float> wc(kTreeletSets);
    std::vector<uint8_t> ws(kTreeletSets);
    const TreeletScratch w{wc.data(), ws.data(), 1};
    for (int k = 3; k <= kTreeletLeaves; ++k) {
        std::vector<Shape> shapes;
        all_shapes(k, shapes);
        long expect = 1;
        for (int f = 2 * k - 3; f > 1; f -= 2) expect *= f;
        for (int seed = 0; seed < 12; ++seed) {
            std::mt19937 rng(1000 * k + seed);
            Tree t = random_tree(k, rng, seed % 3 == 0);
            float best = INFINITY;
            for (const Shape &s : shapes) {
                float4 bl, bh;
                int c;
                best = fminf(best, shape_cost(s, k, t.lo, t.hi, s.root, bl, bh, c));
            }
            // force the root to be a treelet root whatever its size, as a
            // k-triangle root is below the kernel's threshold for k < 7
            sweep(t, w);
            treelet_optimize(t.view(), t.root, w);
            const char *why = "";
            bool ok = (long)shapes.size() == expect && valid(t, &why);
            const float got = fresh_cost(t, t.root);
            if (ok && !(std::fabs(got - best) <= 2e-5f * best)) { ok = false; why = "cost above the optimum"; }
            if (ok && !(std::fabs(t.cost[t.root] - got) <= 2e-5f * got)) { ok = false; why = "stored cost differs"; }
            printf("optimum k=%d seed=%d %s shapes=%zu best=%.6g got=%.6g %s\n", k, seed, ok ? "ok" : "FAIL",
                   shapes.size(), best, got, why);
            fails += !ok;
        }
    }
    const int small[4] = {1, 2, 7, 8};
    for (int seed = 0; seed < 16; ++seed) {
        std::mt19937 rng(seed);
        const int n = seed < 4 ? small[seed] : 1 + (int)(rng() % 3000);
        Tree t = random_tree(n, rng, seed % 2 == 1);
        const float before = fresh_cost(t, t.root);
        bool ok = true;
        const char *why = "";
        float prev = before;
        for (int pass = 0; pass < 3 && ok; ++pass) {
            sweep(t, w);
            ok = valid(t, &why);
            const float now = fresh_cost(t, t.root);
            if (ok && now > prev * 1.00001f) { ok = false; why = "cost went up"; }
            if (ok && !(std::fabs(t.cost[t.root] - now) <= 1e-4f * now)) { ok = false; why = "stored cost differs"; }
            prev = now;
        }
        printf("sweep n=%d seed=%d %s cost %.6g -> %.6g %s\n", n, seed, ok ? "ok" : "FAIL", before, prev, why);
        fails += !ok;
    }
    printf("failures %d\n", fails);
    return fails ? 1 : 0;
}
