// Four-child BVH nodes from the binary tree's child-pair records (host side).
//
// Greedy collapse: a node starts from a binary node's two children and, while
// it has fewer than four, replaces its inner child of largest surface area by
// that child's two children (the greedy collapse of wide BVHs); leaves stay
// leaves, and the boxes are the binary tree's (padded) child boxes.  Against
// folding exactly every other binary level, the apartment's rays visit 15.0
// instead of 16.2 nodes.
//
// Quantized nodes (after Ylitie, Karras and Laine 2017, "Efficient incoherent
// ray traversal on GPUs through compressed wide BVHs"): the four child boxes
// as 8-bit grid coordinates relative to a per-node origin, with a
// power-of-two cell size per axis.  Layout per node, 16 floats = 64 B:
//   row 0: origin x, y, z (float); biased exponents e_x, e_y, e_z (bytes 0-2)
//   row 1: x lo, x hi, y lo, y hi of the four children (one byte per child)
//   row 2: z lo, z hi, 0, 0
//   row 3: the four child references (as the float layout)
// A plane decodes to origin + q 2^e.  Every decoded box contains its child's
// float box widened by delta = 2^-20 of the node's largest extent on every
// side: that margin covers the rounding of the traversal's
// fma(q, 2^e / d, (origin - o) / d) for ray origins within or near the node,
// and the slab test's relative slack covers origins far from it.  An empty
// slot has q lo = 255, q hi = 0 (a box inside out, which the slab test
// rejects unless the ray starts some 10^6 node extents away) and, as its
// reference, the leaf code of the one-triangle leaf holding triangle 0
// (~0): should the slack ever admit the slot, the traversal tests a real
// triangle once more, which changes no hit, instead of following an
// invalid reference.  The traversal then needs no reference check.
#include "bvh_wide.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace ipt {

namespace {

int bits_i(float f) { int i; std::memcpy(&i, &f, sizeof i); return i; }
float bits_f(int i) { float f; std::memcpy(&f, &i, sizeof f); return f; }

struct Child {
    float lo[3], hi[3];
    int ref;
};

}  // namespace

int64_t collapse_wide(const std::vector<float>& pairs, std::vector<float>& wide, int* depth) {
    auto children = [&](int r, Child out[2]) {
        const float* n = &pairs[16 * (size_t)r];
        out[0] = Child{{n[0], n[1], n[2]}, {n[3], n[4], n[5]}, bits_i(n[12])};
        out[1] = Child{{n[6], n[7], n[8]}, {n[9], n[10], n[11]}, bits_i(n[13])};
    };
    std::vector<int> rec_of{0};        // four-child node id -> binary record
    std::vector<int> level{0};         // four-child node id -> its level
    wide.assign(32, 0.0f);
    wide.reserve(2 * pairs.size());
    std::vector<int> stack{0};         // four-child node ids to write
    int levels = 1;
    while (!stack.empty()) {
        const int id = stack.back();
        stack.pop_back();
        // the binary node's children, then, while a slot is free, the inner
        // child of largest surface area is replaced by its own children
        Child c2[2], g[4];
        children(rec_of[id], c2);
        int m = 0;
        for (int k = 0; k < 2; ++k)
            if (c2[k].ref != kWideNone) g[m++] = c2[k];
        while (m < 4) {
            int open = -1;
            double best_area = -1.0;
            for (int j = 0; j < m; ++j) {
                if (g[j].ref < 0) continue;
                const double dx = (double)g[j].hi[0] - g[j].lo[0], dy = (double)g[j].hi[1] - g[j].lo[1],
                             dz = (double)g[j].hi[2] - g[j].lo[2];
                const double area = dx * dy + dy * dz + dz * dx;
                if (area > best_area) { best_area = area; open = j; }
            }
            if (open < 0) break;
            Child gc[2];
            children(g[open].ref, gc);
            int k = 0;
            for (int j = 0; j < 2; ++j) {
                if (gc[j].ref == kWideNone) continue;
                if (k++ == 0) g[open] = gc[j];
                else g[m++] = gc[j];
            }
            if (k == 0) g[open] = g[--m];   // a record without children
        }
        int ref[4] = {kWideNone, kWideNone, kWideNone, kWideNone};
        std::vector<int> inner;
        for (int j = 0; j < m; ++j) {
            if (g[j].ref >= 0) {
                ref[j] = (int)rec_of.size();
                rec_of.push_back(g[j].ref);
                level.push_back(level[id] + 1);
                levels = std::max(levels, level[id] + 2);
                wide.resize(wide.size() + 32, 0.0f);
                inner.push_back(ref[j]);
            } else {
                ref[j] = g[j].ref;
            }
        }
        for (size_t k = inner.size(); k-- > 0;) stack.push_back(inner[k]);
        // an empty slot gets lo = hi = +inf on every axis: the slab test
        // gives it an entry distance of +inf (never entered)
        const float inf = std::numeric_limits<float>::infinity();
        float* o = &wide[32 * (size_t)id];
        for (int j = 0; j < 4; ++j)
            for (int a = 0; a < 3; ++a) {
                o[4 * (2 * a) + j] = j < m ? g[j].lo[a] : inf;
                o[4 * (2 * a + 1) + j] = j < m ? g[j].hi[a] : inf;
            }
        for (int j = 0; j < 4; ++j) {
            o[24 + j] = bits_f(ref[j]);
            o[28 + j] = 0.0f;
        }
    }
    if (depth) *depth = levels;
    return (int64_t)rec_of.size();
}

void quantize_wide(std::vector<float>& wide) {
    const size_t n = wide.size() / 32;
    std::vector<float> q(16 * n);
    for (size_t id = 0; id < n; ++id) {
        const float* o = &wide[32 * id];
        float lo[3][4], hi[3][4];
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 4; ++j) {
                lo[a][j] = o[4 * (2 * a) + j];
                hi[a][j] = o[4 * (2 * a + 1) + j];
            }
        const int ref[4] = {bits_i(o[24]), bits_i(o[25]), bits_i(o[26]), bits_i(o[27])};
        bool valid[4];
        double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int j = 0; j < 4; ++j) {
            valid[j] = ref[j] != kWideNone;
            if (!valid[j]) continue;
            for (int a = 0; a < 3; ++a) {
                mn[a] = std::min(mn[a], (double)lo[a][j]);
                mx[a] = std::max(mx[a], (double)hi[a][j]);
            }
        }
        float org[3] = {0, 0, 0};
        int ex[3] = {0, 0, 0};
        uint8_t ql[3][4], qh[3][4];
        double ext = 0.0;
        for (int a = 0; a < 3; ++a)
            if (mx[a] >= mn[a]) ext = std::max(ext, mx[a] - mn[a]);
        // a node of points (extent 0) still gets a positive margin
        const double delta = std::ldexp(std::max(ext, 1e-30), -20);
        for (int a = 0; a < 3; ++a) {
            for (int j = 0; j < 4; ++j) { ql[a][j] = 255; qh[a][j] = 0; }
            if (!(mx[a] >= mn[a])) continue;   // no valid child
            // origin: a float at or below the lowest plane minus the margin
            float og = (float)(mn[a] - delta);
            while ((double)og > mn[a] - delta) og = std::nextafter(og, -INFINITY);
            org[a] = og;
            const double span = mx[a] + delta - (double)og;
            int e = (int)std::ceil(std::log2(span / 255.0));
            e = std::max(e, -126);
            for (;; ++e) {
                const double cell = std::ldexp(1.0, e);
                bool ok = true;
                for (int j = 0; j < 4 && ok; ++j) {
                    if (!valid[j]) continue;
                    double l = std::floor((lo[a][j] - delta - (double)og) / cell);
                    double h = std::ceil((hi[a][j] + delta - (double)og) / cell);
                    // the decoded planes (exact: og + q 2^e in double) enclose the widened box
                    while (l > 0 && (double)og + l * cell > lo[a][j] - delta) l -= 1.0;
                    while ((double)og + h * cell < hi[a][j] + delta) h += 1.0;
                    if (l < 0 || h > 255) { ok = false; break; }
                    ql[a][j] = (uint8_t)l;
                    qh[a][j] = (uint8_t)h;
                }
                if (ok) break;
            }
            ex[a] = e;
        }
        auto pack = [](const uint8_t b[4]) {
            return bits_f((int)((uint32_t)b[0] | (uint32_t)b[1] << 8 | (uint32_t)b[2] << 16 | (uint32_t)b[3] << 24));
        };
        const uint32_t ew = (uint32_t)(ex[0] + 127) | (uint32_t)(ex[1] + 127) << 8 | (uint32_t)(ex[2] + 127) << 16;
        float* d = &q[16 * id];
        d[0] = org[0]; d[1] = org[1]; d[2] = org[2]; d[3] = bits_f((int)ew);
        d[4] = pack(ql[0]); d[5] = pack(qh[0]); d[6] = pack(ql[1]); d[7] = pack(qh[1]);
        d[8] = pack(ql[2]); d[9] = pack(qh[2]); d[10] = 0.0f; d[11] = 0.0f;
        for (int j = 0; j < 4; ++j) d[12 + j] = bits_f(valid[j] ? ref[j] : ~0);
    }
    wide.swap(q);
}

}  // namespace ipt
