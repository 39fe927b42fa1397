#pragma once
#include <stdint.h>

#include <vector>

namespace ipt {

struct BvhOut {
    std::vector<float> nodes;      // 16 floats (64 B) per child-pair node
    std::vector<int> leaf_order;   // leaf position -> input triangle id
    int64_t num_nodes = 0;
    int depth = 0;                 // levels of the binary tree
    double sah_cost = 0.0;
};

bool build_bvh_host(const float* verts, const int* tris, int64_t nt, BvhOut& out);

}  // namespace ipt
