// Four-child BVH nodes made on the host from the binary tree's child-pair
// records: the greedy collapse and the quantization of the child boxes.
// Plain C++ (no HIP types), so the host tests can build and check it.
#pragma once
#include <stdint.h>

#include <vector>

namespace ipt {

constexpr int kWideNone = 0x7FFFFFFF;   // empty child slot (the kernels' kNone)

// Child-pair records, 16 floats each (child 0 lo xyz, hi xyz; child 1 lo xyz,
// hi xyz; the two references as int bits: inner record index, leaf code
// ~(first << 3 | count - 1), or kWideNone; two padding floats), record 0 the
// root -> four-child nodes with float boxes, 32 floats each (rows lo.x, hi.x,
// lo.y, hi.y, lo.z, hi.z of the four children, one child per component, then
// the four references, then padding), node 0 the root, children of a node
// contiguous, depth first.  Returns the node count; *depth receives the
// number of node levels.
int64_t collapse_wide(const std::vector<float>& pairs, std::vector<float>& wide, int* depth);

// Four-child float-box nodes (32 floats each) -> quantized nodes (16 floats
// each, the layout the traversal reads), in place.
void quantize_wide(std::vector<float>& wide);

}  // namespace ipt
