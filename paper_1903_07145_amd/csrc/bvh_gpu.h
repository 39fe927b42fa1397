// GPU scene build: binned SAH BVH and the leaf-ordered triangle layout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace ipt {

struct GpuBvh {
    float4* nodes = nullptr;   // device, 4 x float4 per child-pair record (caller frees)
    int* leaf_order = nullptr; // device [nt]: leaf position -> input triangle id (caller frees)
    int64_t num_nodes = 0;     // child-pair records
    int depth = 0;             // levels of the binary tree (root = 1)
    double sah_cost = 0.0;     // sum over nodes of area/root area (x count at leaves)
};

// Build on `st` from device arrays verts [nv][3] and tris [nt][3].  Returns
// an empty string on success, else a message (nothing is left allocated).
std::string build_bvh_gpu(const float* d_verts, const int* d_tris, int64_t nt, hipStream_t st, GpuBvh& out);

// Leaf-ordered triangle records (v0, orig id) (v1, segment) (v2, light index),
// shading normals (when d_normals != NULL) and the inverse permutation
// pos_of [nt]; then lights[j].x = pos_of[lights[j].w].
hipError_t launch_scene_layout(const float* d_verts, const int* d_tris, const int* d_seg, const int* d_light_of_tri,
                               const float* d_normals, const int* d_leaf_order, int64_t nt, float4* trec,
                               float4* nrec, int* pos_of, int4* lights, int nlt, hipStream_t st);

}  // namespace ipt
