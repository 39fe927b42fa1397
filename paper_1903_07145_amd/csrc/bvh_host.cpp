// Binned SAH BVH build on the host (Wald, "On fast construction of SAH-based
// bounding volume hierarchies", 2007): 64 bins per axis, C_trav = C_isect =
// 1, leaves of at most 2 triangles.  The result is written in the layout
// the traversal kernels read: depth-first "child pair" nodes (both child
// boxes and both child references in one 64-byte record) and leaf-ordered
// triangles.
#include "bvh_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace ipt {

namespace {

struct Box {
    float lo[3], hi[3];
    void reset() {
        for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    }
    void grow(const Box& b) {
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], b.lo[a]); hi[a] = std::max(hi[a], b.hi[a]); }
    }
    void grow(const float* p) {
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], p[a]); hi[a] = std::max(hi[a], p[a]); }
    }
    double area() const {
        if (!(hi[0] >= lo[0])) return 0.0;
        double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

struct BNode {
    Box box;
    int left, right;    // children (-1 for a leaf)
    int first, count;   // primitive range in `idx` for a leaf
};

constexpr int kBins = 64;   // the GPU builder's slab count
constexpr int kMaxLeaf = 2;   // the GPU builder's leaf size

// Slab of a centroid coordinate, clamped into [0, kBins - 1].
inline int slab(float c, float lo, float k) {
    float x = (c - lo) * k;
    return x >= (float)(kBins - 1) ? kBins - 1 : (x > 0.0f ? (int)x : 0);
}

}  // namespace

bool build_bvh_host(const float* verts, const int* tris, int64_t nt, BvhOut& out) {
    std::vector<Box> pb(nt);
    std::vector<float> cen(3 * nt);
    for (int64_t t = 0; t < nt; ++t) {
        pb[t].reset();
        for (int j = 0; j < 3; ++j) pb[t].grow(verts + 3 * (int64_t)tris[3 * t + j]);
        for (int a = 0; a < 3; ++a) cen[3 * t + a] = 0.5f * (pb[t].lo[a] + pb[t].hi[a]);
    }
    std::vector<int> idx(nt);
    for (int64_t t = 0; t < nt; ++t) idx[t] = (int)t;
    std::vector<BNode> nodes;
    nodes.reserve(2 * nt);
    struct Task { int node, first, count, depth; };
    std::vector<Task> stack;
    nodes.push_back(BNode{});
    stack.push_back({0, 0, (int)nt, 1});
    int max_depth = 0;
    while (!stack.empty()) {
        Task tk = stack.back();
        stack.pop_back();
        max_depth = std::max(max_depth, tk.depth);
        BNode nd;
        nd.box.reset();
        Box cb;
        cb.reset();
        for (int i = tk.first; i < tk.first + tk.count; ++i) {
            nd.box.grow(pb[idx[i]]);
            cb.grow(&cen[3 * (int64_t)idx[i]]);
        }
        nd.left = nd.right = -1;
        nd.first = tk.first;
        nd.count = tk.count;
        if (tk.count <= kMaxLeaf) {
            nodes[tk.node] = nd;
            continue;
        }
        // binned SAH over the three axes
        double best_cost = INFINITY;
        int best_axis = -1, best_split = -1;
        for (int a = 0; a < 3; ++a) {
            float ext = cb.hi[a] - cb.lo[a];
            if (!(ext > 0.0f)) continue;
            Box bb[kBins];
            int bc[kBins];
            for (int b = 0; b < kBins; ++b) { bb[b].reset(); bc[b] = 0; }
            float k = kBins / ext;
            for (int i = tk.first; i < tk.first + tk.count; ++i) {
                int p = idx[i];
                int b = slab(cen[3 * (int64_t)p + a], cb.lo[a], k);
                bb[b].grow(pb[p]);
                bc[b]++;
            }
            double rA[kBins];
            int rN[kBins];
            Box acc;
            acc.reset();
            int n = 0;
            for (int b = kBins - 1; b > 0; --b) {
                acc.grow(bb[b]);
                n += bc[b];
                rA[b] = acc.area();
                rN[b] = n;
            }
            acc.reset();
            n = 0;
            for (int b = 0; b < kBins - 1; ++b) {
                acc.grow(bb[b]);
                n += bc[b];
                if (n == 0 || rN[b + 1] == 0) continue;
                double c = acc.area() * n + rA[b + 1] * rN[b + 1];
                if (c < best_cost) { best_cost = c; best_axis = a; best_split = b; }
            }
        }
        int mid;
        if (best_axis >= 0) {
            float ext = cb.hi[best_axis] - cb.lo[best_axis];
            float k = kBins / ext;
            int a = best_axis;
            auto it = std::partition(idx.begin() + tk.first, idx.begin() + tk.first + tk.count, [&](int p) {
                int b = slab(cen[3 * (int64_t)p + a], cb.lo[a], k);
                return b <= best_split;
            });
            mid = (int)(it - idx.begin());
            if (mid == tk.first || mid == tk.first + tk.count) mid = tk.first + tk.count / 2;
        } else {
            mid = tk.first + tk.count / 2;   // all centroids coincide
        }
        nd.left = (int)nodes.size();
        nodes.push_back(BNode{});
        nd.right = (int)nodes.size();
        nodes.push_back(BNode{});
        nodes[tk.node] = nd;
        stack.push_back({nd.right, mid, tk.first + tk.count - mid, tk.depth + 1});
        stack.push_back({nd.left, tk.first, mid - tk.first, tk.depth + 1});
    }

    // SAH cost (relative to the root box area)
    double ar = nodes[0].box.area();
    double sah = 0.0;
    for (const BNode& n : nodes) {
        double r = ar > 0 ? n.box.area() / ar : 1.0;
        sah += n.left < 0 ? r * n.count : r;
    }

    // depth-first child-pair layout
    out.nodes.clear();
    out.leaf_order.clear();
    out.leaf_order.reserve(nt);
    auto pad_box = [](const Box& b, float* lo, float* hi) {
        for (int a = 0; a < 3; ++a) {
            float m = std::max(std::fabs(b.lo[a]), std::fabs(b.hi[a]));
            float pad = m * 9.5367431640625e-07f + 1e-30f;  // 2^-20 relative
            lo[a] = b.lo[a] - pad;
            hi[a] = b.hi[a] + pad;
        }
    };
    // each entry: the BNode to emit as a child-pair record at position pos
    struct Emit { int bnode, pos; };
    std::vector<Emit> es;
    auto child_ref = [&](int c, std::vector<Emit>& pending) -> int {
        const BNode& n = nodes[c];
        if (n.left < 0) {
            int first = (int)out.leaf_order.size();
            for (int i = n.first; i < n.first + n.count; ++i) out.leaf_order.push_back(idx[i]);
            return ~((first << 3) | (n.count - 1));
        }
        int pos = (int)(out.nodes.size() / 16);
        out.nodes.resize(out.nodes.size() + 16, 0.0f);
        pending.push_back({c, pos});
        return pos;
    };
    auto write = [&](int pos, const Box* b0, const Box* b1, int c0, int c1) {
        float* r = &out.nodes[16 * (size_t)pos];
        float lo0[3], hi0[3], lo1[3], hi1[3];
        pad_box(*b0, lo0, hi0);
        if (b1) pad_box(*b1, lo1, hi1);
        else for (int a = 0; a < 3; ++a) { lo1[a] = 0.0f; hi1[a] = 0.0f; }
        r[0] = lo0[0]; r[1] = lo0[1]; r[2] = lo0[2]; r[3] = hi0[0];
        r[4] = hi0[1]; r[5] = hi0[2]; r[6] = lo1[0]; r[7] = lo1[1];
        r[8] = lo1[2]; r[9] = hi1[0]; r[10] = hi1[1]; r[11] = hi1[2];
        std::memcpy(&r[12], &c0, 4);
        std::memcpy(&r[13], &c1, 4);
        r[14] = 0.0f;
        r[15] = 0.0f;
    };
    out.nodes.resize(16, 0.0f);
    if (nodes[0].left < 0) {
        std::vector<Emit> dummy;
        int c0 = child_ref(0, dummy);
        write(0, &nodes[0].box, nullptr, c0, 0x7FFFFFFF);
    } else {
        // iterative DFS: emit record for root at pos 0
        std::vector<Emit> todo;
        todo.push_back({0, 0});
        while (!todo.empty()) {
            Emit e = todo.back();
            todo.pop_back();
            const BNode& n = nodes[e.bnode];
            std::vector<Emit> pend;
            int c0 = child_ref(n.left, pend);
            int c1 = child_ref(n.right, pend);
            write(e.pos, &nodes[n.left].box, &nodes[n.right].box, c0, c1);
            // visit left subtree first (depth-first order of positions)
            for (int i = (int)pend.size() - 1; i >= 0; --i) todo.push_back(pend[i]);
        }
    }
    out.num_nodes = (int64_t)(out.nodes.size() / 16);
    out.depth = max_depth;
    out.sah_cost = sah;
    return (int64_t)out.leaf_order.size() == nt;
}

}  // namespace ipt
