// Internal host/device interface between the C ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "guide_dev.h"
#include "ipt_math.h"

namespace ipt {

constexpr int kBlock = 256;       // threads per block of the path kernels
constexpr int kShortStack = 16;   // per-lane LDS stack entries (power of two)
constexpr int kOvfDepth = 48;     // per-lane global overflow entries
constexpr int kNone = 0x7FFFFFFF; // empty child slot
// BVH node width of the traversal: 4 (the binary tree collapsed into
// four-child nodes on the host, bvh_wide.cpp) or 2 (the binary tree's 64 B
// child-pair nodes)
#ifndef IPT_NODE_WIDTH
#define IPT_NODE_WIDTH 4
#endif
constexpr int kNodeWidth = IPT_NODE_WIDTH;
// 4-wide nodes with quantized child boxes (64 B, four float4 loads per
// visit) instead of float boxes (128 B, seven loads)
#ifndef IPT_NODE_QUANT
#define IPT_NODE_QUANT 1
#endif
constexpr int kNodeQuant = (IPT_NODE_WIDTH == 4) ? IPT_NODE_QUANT : 0;
// float4 rows per node in the node array
constexpr int kNodeRows = kNodeWidth == 4 ? (kNodeQuant ? 4 : 8) : 4;
constexpr int kMaxDepth = 16;     // max scattering vertices per path
constexpr int kMaxLdsLights = 1024;
constexpr int kMaxLdsParams = 4096;  // larger parameter vectors stay in global memory
constexpr int64_t kMaxParams = 1ll << 26;
// global parameter storage: the adjoint's float64 accumulator is replicated
// (block b adds into copy b mod R) within this many bytes, so paths that hit
// the same few parameters do not all contend for one address
constexpr size_t kGradCopyBytes = size_t(256) << 20;

// Checkpoint record flags (packed with tri+1 in the low 28 bits).
constexpr uint32_t kCkTriMask = 0x0FFFFFFFu;
constexpr uint32_t kCkVis = 1u << 28;    // next-event shadow ray unoccluded
constexpr uint32_t kCkCont = 1u << 29;   // path continued from this vertex
constexpr uint32_t kCkDrop = 1u << 30;   // (vertex 1) path dropped: non-finite

// Device view of a built scene.
struct SceneDev {
    const float4* nodes;   // kNodeRows float4 per node (layouts in api.hip)
    const float4* tris;    // 3 x float4 per leaf-ordered triangle:
                           //   (v0, orig id), (v1, segment), (v2, light index or -1)
    const float4* nrm;     // 3 x float4 per leaf-ordered triangle, or NULL
    const int4* lights;    // [nlt]: (leaf tri, emitter index, area bits, orig id)
    const int* seg_emitter;// [S]: emitter index or -1
    const int* pos_of;     // [nt]: input triangle id -> leaf position
    int S, E, nlt;
    int nm;                // material parameters per segment: 7 (Lambert + GGX) or 13 (Disney)
    float tmin;            // ray epsilon (1e-6 of the scene diagonal)
};

// Per-kernel work counters (kernel modes 0..2): rays cast, BVH nodes
// fetched, triangles tested, paths, path vertices, work units taken (a work
// unit is a pixel's whole sample range, or a chunk of it when a pixel's
// samples are split over lanes).
struct KStats {
    unsigned long long rays, nodes, tris, paths, vertices, units;
};

struct Counters {
    unsigned long long nonfinite;
    unsigned long long overflow;
    KStats k[3];
};

enum Mode { kColor = 0, kGradFwd = 1, kReplay = 2 };

struct PathArgs {
    SceneDev sc;
    const float* c2w;
    const float* fov;
    int V, W, H;
    const float* params;
    const float* sparams;
    int P;
    int frozen;              // sparams differs from params
    const float* cdf;        // [2 nlt]: inclusive prefix sums of light weights, then probabilities
    Rng rng;
    int spp, D, rr_depth, mis, profile, jitter;
    const int64_t* pixel_list;
    int64_t pix_begin, pix_count;  // work-pixel chunk
    // work unit = (sample chunk c, work pixel q): samples [c spc, min(spp, (c+1) spc))
    // of pixel q; unit index c * pix_count + q.  nchunk > 1 when the pixels are
    // too few to fill the grid one pixel per lane.
    int spc, nchunk;
    float* image;                  // colour: [pixels][3]
    float* part;                   // colour, nchunk > 1: per-unit sums [nchunk][pix_count][3]
    uint64_t* hash;                // [pixels*spp] or NULL
    float* path_L;                 // colour: [pixels*spp][3] per-path radiance or NULL
    float* dbg_vtx;                // colour: [pixels*spp][D+1][8] per-vertex record or NULL
    const uint8_t* mask;           // [pixels*spp] or NULL
    int4* ck_hit;                  // checkpoint planes, [(k-1)*spp + s][pix_count]
    float4* ck_a;
    float4* ck_c;
    const float* w;                // replay: adjoint image [pixels][3]
    double* grad_part;             // replay: [gridDim.x][P]
    unsigned* work;                // dynamic tile counter (zeroed before launch)
    Counters* err;
    int* ovf;                      // [kOvfDepth][grid threads]
    int replay_traverse;
    int params_global;             // parameters read from global memory; the adjoint adds float64
                                   // atomics into copy blockIdx.x mod grad_copies of
                                   // grad_part[grad_copies][P] (else per-block LDS copies and
                                   // partials grad_part[gridDim.x][P])
    int grad_copies;
    int count_stats;               // accumulate KStats into err->k[mode]
    int mat;                       // material model: 0 Lambert + GGX, 1 Disney (selects the kernels)
    // learned proposal (one-sample MIS with BRDF sampling)
    GuideDev gd;
    int guided;                    // a guide is attached (checkpoint plane ck_d is written)
    int guide_kind;                // proposal sampled: 0 none, 1 network (bfloat16 MFMA), 2 network
                                   // (float32 VALU), 3 cached rows
    float gmix;                    // probability of sampling the guide
    float4* ck_d;                  // guided: [(k-1)*spp + s][pix_count] (sampled direction, NEE density)
    float* grec;                   // training-record ring [cap][16] or NULL
    unsigned* grec_count;
    int grec_cap, grec_stride;
};

size_t path_lds_bytes(int mode, int P, int frozen, int S, int nlt, int guide_kind = 0, int params_global = 0);
int path_blocks_per_cu(int mode, size_t lds, int guide_kind = 0, int params_global = 0, int mat = 0);
hipError_t launch_guide_records(const PathArgs& a, hipStream_t st);
hipError_t launch_paths(int mode, const PathArgs& a, int grid, size_t lds, hipStream_t st);
// guide handle internals (guide.hip)
struct GuideHandle;
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st);
hipError_t launch_light_cdf(const SceneDev& sc, const float* sparams, float* cdf, hipStream_t st);
hipError_t launch_loss_adjoint(const float* img, const float* target, int64_t n3, int kind,
                               float* w, float* partials, int nparts, float* loss,
                               hipStream_t st);
hipError_t launch_colour_reduce(const float* part, int nchunk, int64_t pix_count, int spp, float* image,
                                hipStream_t st);
hipError_t launch_grad_reduce(const double* part, int nblocks, int P, float* grad, int accumulate,
                              hipStream_t st);
hipError_t launch_l1_reg(const float* p, float* g, const float* w, int P, float* loss, hipStream_t st);
hipError_t launch_adam(float* params, const float* grad, float* m, float* v, int P, int step,
                       float lr, float b1, float b2, float eps, const float* scale,
                       const float* lo, const float* hi, const uint8_t* trainable,
                       hipStream_t st);
hipError_t launch_trace_rays(const SceneDev& sc, const float* o, const float* d, const int* skip,
                             int64_t n, float tmin, int brute, int64_t nt, int* out_tri,
                             float* out_tuv, int* ovf, int grid, Counters* err, hipStream_t st);
int trace_rays_grid(int num_cu);

}  // namespace ipt
