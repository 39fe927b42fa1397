// Host-only harness for the tests: the host BVH builder followed by the
// four-child collapse (and, on request, the quantization), exposed through a
// plain C interface that ctypes can call without a GPU.
#include <cstring>
#include <vector>

#include "bvh_host.h"
#include "bvh_wide.h"

namespace {
std::vector<float> g_nodes;
std::vector<int> g_order;
}  // namespace

// Builds the tree of nt triangles; returns the number of four-child nodes
// (-1 if the host builder fails).  *levels: node levels of the four-child
// tree; *bin_depth: levels of the binary tree.
extern "C" long long harness_build(const float* verts, const int* tris, long long nt, int quantize, int* levels,
                                   int* bin_depth) {
    ipt::BvhOut b;
    if (!ipt::build_bvh_host(verts, tris, nt, b)) return -1;
    const long long n = ipt::collapse_wide(b.nodes, g_nodes, levels);
    if (quantize) ipt::quantize_wide(g_nodes);
    g_order = b.leaf_order;
    *bin_depth = b.depth;
    return n;
}

// Copies the last build: nodes (32 floats per node with float boxes, 16 when
// quantized) and the leaf order (leaf position -> input triangle id).
extern "C" void harness_copy(float* nodes, int* order) {
    std::memcpy(nodes, g_nodes.data(), sizeof(float) * g_nodes.size());
    std::memcpy(order, g_order.data(), sizeof(int) * g_order.size());
}
