// C ABI of the inverse path tracing library: validation, scene upload,
// workspace layout and launch sequencing on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ipt.h"
#include "bvh_gpu.h"
#include "bvh_host.h"
#include "bvh_wide.h"
#include "ipt_internal.h"

using namespace ipt;

static thread_local std::string g_err;

static ipt_status fail(ipt_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_OK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return fail(IPT_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_));          \
    } while (0)

extern "C" const char* ipt_last_error(void) { return g_err.c_str(); }

// guide internals (guide.hip)
GuideDev guide_dev(const ipt_guide_s* g);
float* guide_records(ipt_guide_s* g);
unsigned* guide_record_count(ipt_guide_s* g);
int guide_capacity(const ipt_guide_s* g);
int guide_record_stride(const ipt_guide_s* g);
int guide_cache_ready(const ipt_guide_s* g, const void* scene);
ipt_status guide_cache_build_impl(ipt_guide_s* g, const void* scene, const float4* tris, const float4* nrm,
                                  int64_t nt, float cell_area, int mode, hipStream_t st, int64_t* ncells);
ipt_status ipt_fail(ipt_status s, const char* msg) { return fail(s, "%s", msg); }

struct ipt_scene_s {
    int device = 0;
    int num_cu = 0;
    SceneDev dev{};
    float4* d_nodes = nullptr;
    float4* d_tris = nullptr;
    float4* d_nrm = nullptr;
    int4* d_lights = nullptr;
    int* d_segemit = nullptr;
    int* d_pos_of = nullptr;
    Counters* d_err = nullptr;
    int* d_ovf_rays = nullptr;   // overflow stacks of ipt_trace_rays
    int64_t nt = 0, nv = 0, nnodes = 0;
    int S = 0, E = 0, nlt = 0, depth = 0, has_normals = 0, bvh_builder = 0, params_global = 0;
    int mat = 0, nm = 7;   // material model and its parameters per segment
    double sah = 0.0, build_ms = 0.0;
    float diag = 0.0f;
    float bb_lo[3] = {0, 0, 0}, bb_hi[3] = {0, 0, 0};
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[3];
};

// Four-child nodes (default): the binary tree's child-pair records are
// collapsed and quantized on the host (bvh_wide.cpp) and uploaded in place of
// the binary ones; *levels receives the number of node levels.
static hipError_t collapse_bvh4(float4*& d_nodes, int64_t& nnodes, int* levels, hipStream_t st) {
    static_assert(kWideNone == kNone, "empty child slot marker");
    std::vector<float> pairs(16 * (size_t)nnodes);
    hipError_t e = hipMemcpyAsync(pairs.data(), d_nodes, sizeof(float) * pairs.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    std::vector<float> wide;
    const int64_t n4 = collapse_wide(pairs, wide, levels);
    if (kNodeQuant) quantize_wide(wide);
    float4* d4 = nullptr;
    e = hipMalloc((void**)&d4, sizeof(float) * wide.size());
    if (e == hipSuccess) e = hipMemcpyAsync(d4, wide.data(), sizeof(float) * wide.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        hipFree(d4);
        return e;
    }
    hipFree(d_nodes);
    d_nodes = d4;
    nnodes = n4;
    return hipSuccess;
}

static void prof_clear_events(ipt_scene_s* s) {
    for (auto& v : s->ev) {
        for (auto& p : v) {
            hipEventDestroy(p.first);
            hipEventDestroy(p.second);
        }
        v.clear();
    }
}

// Launch a path kernel, bracketed by events when profiling is on.
static hipError_t timed_launch(ipt_scene_s* s, int mode, PathArgs& a, int grid, size_t lds, hipStream_t st) {
    a.count_stats = s->prof ? 1 : 0;
    if (!s->prof) return launch_paths(mode, a, grid, lds, st);
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) return e;
    hipEventRecord(e0, st);
    e = launch_paths(mode, a, grid, lds, st);
    hipEventRecord(e1, st);
    s->ev[mode].push_back({e0, e1});
    return e;
}

// ---------------------------------------------------------------------------
// Scene build.
// ---------------------------------------------------------------------------
extern "C" ipt_status ipt_scene_free(ipt_scene_t s) {
    if (!s) return IPT_OK;
    prof_clear_events(s);
    hipFree(s->d_nodes);
    hipFree(s->d_tris);
    hipFree(s->d_nrm);
    hipFree(s->d_lights);
    hipFree(s->d_segemit);
    hipFree(s->d_pos_of);
    hipFree(s->d_err);
    hipFree(s->d_ovf_rays);
    delete s;
    return IPT_OK;
}

extern "C" ipt_status ipt_scene_build_ex(const float* verts, int64_t nv, const float* normals,
                                         const int32_t* tris, const int32_t* tri_seg, int64_t nt,
                                         int32_t num_segments, const int32_t* emitter_seg,
                                         int32_t num_emitters, const ipt_build_opts* bopts, void* hip_stream,
                                         ipt_scene_t* out) {
    const int builder = bopts ? bopts->bvh_builder : IPT_BVH_GPU;
    if (builder != IPT_BVH_GPU && builder != IPT_BVH_HOST) return fail(IPT_ERR_INVALID_ARG, "unknown bvh_builder %d", builder);
    const int storage = bopts ? bopts->param_storage : IPT_PARAMS_AUTO;
    if (storage != IPT_PARAMS_AUTO && storage != IPT_PARAMS_GLOBAL)
        return fail(IPT_ERR_INVALID_ARG, "unknown param_storage %d", storage);
    const int mat = bopts ? bopts->material_model : IPT_MATERIAL_GGX;
    if (mat != IPT_MATERIAL_GGX && mat != IPT_MATERIAL_DISNEY)
        return fail(IPT_ERR_INVALID_ARG, "unknown material_model %d", mat);
    const int nm = mat == IPT_MATERIAL_DISNEY ? 13 : 7;
    hipStream_t st = (hipStream_t)hip_stream;
    if (!out) return fail(IPT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!verts || !tris || !tri_seg) return fail(IPT_ERR_INVALID_ARG, "verts/tris/tri_seg is NULL");
    if (nv < 3 || nt < 1) return fail(IPT_ERR_INVALID_ARG, "need nv >= 3 and nt >= 1");
    if (nt >= (int64_t)kCkTriMask) return fail(IPT_ERR_NOT_SUPPORTED, "too many triangles (%lld)", (long long)nt);
    if (num_segments < 1) return fail(IPT_ERR_INVALID_ARG, "num_segments < 1");
    if (num_emitters < 0 || (num_emitters > 0 && !emitter_seg))
        return fail(IPT_ERR_INVALID_ARG, "bad emitter list");
    // coordinates up to 1e12 in magnitude: the quantized node planes scale
    // 1/d (at most 1e20) by 2^(e + 24) with cells 2^e of up to 2^33, which
    // then stays finite
    for (int64_t i = 0; i < 3 * nv; ++i) {
        if (!std::isfinite(verts[i])) return fail(IPT_ERR_BAD_SCENE, "vertex %lld is not finite", (long long)(i / 3));
        if (std::fabs(verts[i]) > 1e12f)
            return fail(IPT_ERR_BAD_SCENE, "vertex %lld has a coordinate beyond 1e12", (long long)(i / 3));
    }
    if (normals)
        for (int64_t i = 0; i < nv; ++i) {
            float x = normals[3 * i], y = normals[3 * i + 1], z = normals[3 * i + 2];
            if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z) || !(x * x + y * y + z * z > 0.0f))
                return fail(IPT_ERR_BAD_SCENE, "normal %lld is not a finite nonzero vector", (long long)i);
        }
    for (int64_t t = 0; t < nt; ++t) {
        for (int j = 0; j < 3; ++j)
            if (tris[3 * t + j] < 0 || tris[3 * t + j] >= nv)
                return fail(IPT_ERR_BAD_SCENE, "triangle %lld references vertex %d out of range", (long long)t,
                            tris[3 * t + j]);
        if (tri_seg[t] < 0 || tri_seg[t] >= num_segments)
            return fail(IPT_ERR_BAD_SCENE, "triangle %lld has segment %d out of range", (long long)t, tri_seg[t]);
    }
    std::vector<int> seg_emitter(num_segments, -1);
    for (int k = 0; k < num_emitters; ++k) {
        int s = emitter_seg[k];
        if (s < 0 || s >= num_segments) return fail(IPT_ERR_BAD_SCENE, "emitter %d segment %d out of range", k, s);
        if (seg_emitter[s] >= 0) return fail(IPT_ERR_BAD_SCENE, "segment %d listed twice as emitter", s);
        seg_emitter[s] = k;
    }
    int64_t P = nm * (int64_t)num_segments + 3 * (int64_t)num_emitters;
    if (P > kMaxParams)
        return fail(IPT_ERR_NOT_SUPPORTED, "parameter vector too long (%lld > %lld)", (long long)P, (long long)kMaxParams);


    // emitter table in ascending input-id order (leaf positions filled in on the device)
    std::vector<int4> lights;
    std::vector<int> light_of_tri(nt, -1);
    for (int64_t t = 0; t < nt; ++t) {
        int k = seg_emitter[tri_seg[t]];
        if (k < 0) continue;
        const float* a = verts + 3 * (int64_t)tris[3 * t];
        const float* b = verts + 3 * (int64_t)tris[3 * t + 1];
        const float* c = verts + 3 * (int64_t)tris[3 * t + 2];
        double e1[3], e2[3];
        for (int i = 0; i < 3; ++i) { e1[i] = (double)b[i] - a[i]; e2[i] = (double)c[i] - a[i]; }
        double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
               cz = e1[0] * e2[1] - e1[1] * e2[0];
        float area = (float)(0.5 * std::sqrt(cx * cx + cy * cy + cz * cz));
        if (!(area > 0.0f)) return fail(IPT_ERR_BAD_SCENE, "emitter triangle %lld has zero area", (long long)t);
        int4 L;
        L.x = -1;
        L.y = k;
        std::memcpy(&L.z, &area, 4);
        L.w = (int)t;
        light_of_tri[t] = (int)lights.size();
        lights.push_back(L);
    }
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < nv; ++i)
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], verts[3 * i + a]); hi[a] = std::max(hi[a], verts[3 * i + a]); }
    double diag = std::sqrt((double)(hi[0] - lo[0]) * (hi[0] - lo[0]) + (double)(hi[1] - lo[1]) * (hi[1] - lo[1]) +
                            (double)(hi[2] - lo[2]) * (hi[2] - lo[2]));

    ipt_scene_t s = new ipt_scene_s();
    HIP_OK(hipGetDevice(&s->device));
    HIP_OK(hipDeviceGetAttribute(&s->num_cu, hipDeviceAttributeMultiprocessorCount, s->device));
    // inputs on the device for the build (freed before returning)
    struct Tmp {
        std::vector<void*> p;
        ~Tmp() { for (void* q : p) (void)hipFree(q); }
    } tmp;
    auto up = [&](void** dst, const void* src, size_t bytes, bool temporary) -> hipError_t {
        hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 16));
        if (e != hipSuccess) return e;
        if (temporary) tmp.p.push_back(*dst);
        if (bytes) e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, st);
        return e;
    };
    float* d_verts = nullptr;
    float* d_vnrm = nullptr;
    int *d_tris = nullptr, *d_seg = nullptr, *d_lot = nullptr, *d_order = nullptr;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up((void**)&d_verts, verts, sizeof(float) * 3 * nv, true);
    if (e == hipSuccess) e = up((void**)&d_tris, tris, sizeof(int) * 3 * nt, true);
    if (e == hipSuccess) e = up((void**)&d_seg, tri_seg, sizeof(int) * nt, true);
    if (e == hipSuccess) e = up((void**)&d_lot, light_of_tri.data(), sizeof(int) * nt, true);
    if (e == hipSuccess && normals) e = up((void**)&d_vnrm, normals, sizeof(float) * 3 * nv, true);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        ipt_scene_free(s);
        return fail(e == hipErrorOutOfMemory ? IPT_ERR_OUT_OF_MEMORY : IPT_ERR_HIP, "scene upload: %s",
                    hipGetErrorString(e));
    }

    // BVH: on the device (default) or the host reference builder
    auto t0 = std::chrono::steady_clock::now();
    int depth = 0;
    double sah = 0.0;
    int64_t nnodes = 0;
    if (builder == IPT_BVH_GPU) {
        GpuBvh gb;
        std::string msg = build_bvh_gpu(d_verts, d_tris, nt, st, gb);
        if (!msg.empty()) {
            ipt_scene_free(s);
            return fail(IPT_ERR_HIP, "%s", msg.c_str());
        }
        s->d_nodes = gb.nodes;
        d_order = gb.leaf_order;
        tmp.p.push_back(d_order);
        depth = gb.depth;
        sah = gb.sah_cost;
        nnodes = gb.num_nodes;
    } else {
        BvhOut bvh;
        if (!build_bvh_host(verts, tris, nt, bvh)) {
            ipt_scene_free(s);
            return fail(IPT_ERR_BAD_SCENE, "BVH build failed");
        }
        e = up((void**)&s->d_nodes, bvh.nodes.data(), bvh.nodes.size() * sizeof(float), false);
        if (e == hipSuccess) e = up((void**)&d_order, bvh.leaf_order.data(), sizeof(int) * nt, true);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            ipt_scene_free(s);
            return fail(IPT_ERR_HIP, "BVH upload: %s", hipGetErrorString(e));
        }
        depth = bvh.depth;
        sah = bvh.sah_cost;
        nnodes = bvh.num_nodes;
    }
    int levels = depth;   // node levels of the traversal's tree
    if (kNodeWidth == 4) {
        e = collapse_bvh4(s->d_nodes, nnodes, &levels, st);
        if (e != hipSuccess) {
            ipt_scene_free(s);
            return fail(IPT_ERR_HIP, "BVH layout: %s", hipGetErrorString(e));
        }
    }
    auto t1 = std::chrono::steady_clock::now();
    // a node pushes at most width - 1 entries, so the stack holds at most
    // that many per level of the path to the current node
    if ((kNodeWidth - 1) * levels > kShortStack + kOvfDepth) {
        ipt_scene_free(s);
        return fail(IPT_ERR_NOT_SUPPORTED, "BVH of %d node levels exceeds the traversal stack", levels);
    }

    // leaf-ordered triangle records, shading normals, inverse permutation, light table
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_tris, sizeof(float4) * 3 * nt);
    if (e == hipSuccess && normals) e = hipMalloc((void**)&s->d_nrm, sizeof(float4) * 3 * nt);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_pos_of, sizeof(int) * std::max<int64_t>(nt, 4));
    if (e == hipSuccess) e = up((void**)&s->d_lights, lights.data(), lights.size() * sizeof(int4), false);
    if (e == hipSuccess) e = up((void**)&s->d_segemit, seg_emitter.data(), seg_emitter.size() * sizeof(int), false);
    if (e == hipSuccess)
        e = launch_scene_layout(d_verts, d_tris, d_seg, d_lot, d_vnrm, d_order, nt, s->d_tris, s->d_nrm, s->d_pos_of,
                                s->d_lights, (int)lights.size(), st);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_err, sizeof(Counters));
    if (e == hipSuccess) e = hipMemsetAsync(s->d_err, 0, sizeof(Counters), st);
    if (e == hipSuccess)
        e = hipMalloc((void**)&s->d_ovf_rays,
                      sizeof(int) * (size_t)kOvfDepth * trace_rays_grid(s->num_cu) * kBlock);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        ipt_scene_free(s);
        return fail(e == hipErrorOutOfMemory ? IPT_ERR_OUT_OF_MEMORY : IPT_ERR_HIP, "scene layout: %s",
                    hipGetErrorString(e));
    }
    s->nt = nt;
    s->nv = nv;
    s->nnodes = nnodes;
    s->S = num_segments;
    s->E = num_emitters;
    s->mat = mat;
    s->nm = nm;
    s->nlt = (int)lights.size();
    s->depth = depth;
    s->has_normals = normals != nullptr;
    s->sah = sah;
    s->bvh_builder = builder;
    s->params_global = (storage == IPT_PARAMS_GLOBAL || P > kMaxLdsParams) ? 1 : 0;
    s->build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    s->diag = (float)diag;
    for (int a = 0; a < 3; ++a) { s->bb_lo[a] = lo[a]; s->bb_hi[a] = hi[a]; }
    s->dev.nodes = s->d_nodes;
    s->dev.tris = s->d_tris;
    s->dev.nrm = s->d_nrm;
    s->dev.lights = s->d_lights;
    s->dev.seg_emitter = s->d_segemit;
    s->dev.pos_of = s->d_pos_of;
    s->dev.S = num_segments;
    s->dev.E = num_emitters;
    s->dev.nm = nm;
    s->dev.nlt = s->nlt;
    s->dev.tmin = (float)(1e-6 * diag);
    *out = s;
    return IPT_OK;
}

extern "C" ipt_status ipt_scene_build(const float* verts, int64_t nv, const float* normals,
                                      const int32_t* tris, const int32_t* tri_seg, int64_t nt,
                                      int32_t num_segments, const int32_t* emitter_seg,
                                      int32_t num_emitters, void* hip_stream, ipt_scene_t* out) {
    return ipt_scene_build_ex(verts, nv, normals, tris, tri_seg, nt, num_segments, emitter_seg, num_emitters, nullptr,
                              hip_stream, out);
}

extern "C" ipt_status ipt_scene_info(ipt_scene_t s, ipt_scene_info_t* out) {
    if (!s || !out) return fail(IPT_ERR_INVALID_ARG, "NULL scene or out");
    Counters c;
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(&c, s->d_err, sizeof(Counters), hipMemcpyDeviceToHost));
    out->num_triangles = s->nt;
    out->num_vertices = s->nv;
    out->num_nodes = s->nnodes;
    out->num_light_triangles = s->nlt;
    out->num_segments = s->S;
    out->num_emitters = s->E;
    out->bvh_depth = s->depth;
    out->has_normals = s->has_normals;
    out->sah_cost = s->sah;
    out->build_ms = s->build_ms;
    out->scene_diag = s->diag;
    out->nonfinite_paths = c.nonfinite;
    out->stack_overflows = c.overflow;
    out->bvh_builder = s->bvh_builder;
    out->params_global = s->params_global;
    out->node_bytes = 16 * kNodeRows;
    out->node_width = kNodeWidth;
    out->material_model = s->mat;
    out->params_per_segment = s->nm;
    return IPT_OK;
}

// ---------------------------------------------------------------------------
// Options and workspace.
// ---------------------------------------------------------------------------
static ipt_status check_opts(const ipt_scene_s* s, const ipt_cameras* cams, const ipt_render_opts* o,
                             int64_t* npix) {
    if (!cams || !o) return fail(IPT_ERR_INVALID_ARG, "NULL cameras or options");
    if (cams->num_views < 1 || cams->width < 1 || cams->height < 1 || !cams->cam_to_world || !cams->fov_y)
        return fail(IPT_ERR_INVALID_ARG, "bad cameras");
    if (o->spp < 1) return fail(IPT_ERR_INVALID_ARG, "spp must be >= 1");
    if (o->max_depth < 1 || o->max_depth > kMaxDepth) return fail(IPT_ERR_INVALID_ARG, "max_depth must be in [1, %d]", kMaxDepth);
    if (o->mis < 0 || o->mis > 3) return fail(IPT_ERR_INVALID_ARG, "mis must be 0..3");
    if (o->emission_profile < 0 || o->emission_profile > 1) return fail(IPT_ERR_INVALID_ARG, "emission_profile must be 0/1");
    if (o->guide && o->replay_traverse)
        return fail(IPT_ERR_NOT_SUPPORTED, "a guided gradient replays from vertex checkpoints only");
    if (!(o->guide_mix >= 0.0f && o->guide_mix < 1.0f)) return fail(IPT_ERR_INVALID_ARG, "guide_mix must be in [0, 1)");
    if (o->guide_mix > 0.0f && !o->guide) return fail(IPT_ERR_INVALID_ARG, "guide_mix > 0 needs a guide");
    if (o->guide_cached != 0 && o->guide_cached != 1) return fail(IPT_ERR_INVALID_ARG, "guide_cached must be 0 or 1");
    if (o->guide && o->guide_mix > 0.0f && o->guide_cached && !guide_cache_ready(o->guide, s))
        return fail(IPT_ERR_INVALID_ARG, "guide_cached: no cached proposal built for this scene (ipt_guide_cache_build)");
    int64_t all = (int64_t)cams->num_views * cams->width * cams->height;
    if (o->pixel_list) {
        if (o->num_pixels < 1) return fail(IPT_ERR_INVALID_ARG, "num_pixels must be >= 1 with a pixel list");
        *npix = o->num_pixels;
    } else {
        *npix = all;
    }
    return IPT_OK;
}

// Which proposal the path kernels evaluate: 0 none sampled, 1 network per
// vertex (bfloat16 MFMA), 2 network per vertex (float32 VALU), 3 cached rows.
static int guide_kind(const ipt_render_opts* o) {
    if (!o->guide || !(o->guide_mix > 0.0f)) return 0;
    return o->guide_cached ? 3 : (o->guide_fp32 ? 2 : 1);
}

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

struct Plan {
    int grid = 0;
    int grad_copies = 0;
    size_t off_counters = 0, off_cdf = 0, off_loss = 0, off_w = 0, off_img = 0, off_gpart = 0, off_ovf = 0,
           off_part = 0, off_ck = 0, end_fixed = 0;
    int64_t chunk = 0;         // work pixels per gradient chunk
    size_t ck_per_pixel = 0;   // checkpoint bytes per work pixel
};

// Persistent grid: blocks per CU from the occupancy calculator (at most 8),
// or IPT_BLOCKS_PER_CU when set (tuning).
static int path_grid(const ipt_scene_s* s, int P, int frozen, int gk) {
    const int pg = s->params_global;
    int occ = path_blocks_per_cu(kColor, path_lds_bytes(kColor, P, frozen, s->S, s->nlt, gk, pg), gk, pg, s->mat);
    occ = std::min(occ, path_blocks_per_cu(kGradFwd, path_lds_bytes(kGradFwd, P, frozen, s->S, s->nlt, gk, pg), gk, pg,
                                           s->mat));
    static const int forced = [] {
        const char* e = std::getenv("IPT_BLOCKS_PER_CU");
        return e ? std::atoi(e) : 0;
    }();
    if (forced > 0) occ = forced;
    occ = std::max(1, std::min(occ, 8));
    return s->num_cu * occ;
}

// Samples per work unit.  With fewer than two pixels per lane of the grid a
// pixel's samples are split over ceil(2 lanes / pixels) lanes (at most spp),
// so a small image with many samples per pixel still fills the GPU.
static void split_samples(int64_t npix, int spp, int grid, int& spc, int& nchunk) {
    const int64_t lanes = (int64_t)grid * kBlock;
    nchunk = 1;
    if (npix < 2 * lanes && spp > 1) nchunk = (int)std::min<int64_t>(spp, (2 * lanes + npix - 1) / npix);
    spc = (spp + nchunk - 1) / nchunk;
    nchunk = (spp + spc - 1) / spc;
}

static void make_plan(const ipt_scene_s* s, const ipt_render_opts* o, int64_t npix, bool with_loss, Plan& pl) {
    int P = s->nm * s->S + 3 * s->E;
    const int guided = o->guide != nullptr;
    pl.grid = path_grid(s, P, 1, guide_kind(o));
    size_t off = 0;
    pl.off_counters = off; off = al256(off + 64 * sizeof(unsigned));
    pl.off_cdf = off; off = al256(off + 2 * sizeof(float) * std::max(1, s->nlt));   // prefix sums, probabilities
    pl.off_loss = off; off = al256(off + sizeof(float) * 1024);
    pl.off_w = off; off = al256(off + (with_loss ? sizeof(float) * 3 * npix : 0));
    pl.off_img = off; off = al256(off + (with_loss ? sizeof(float) * 3 * npix : 0));
    // replay gradient: per-block partials, or with global parameters grad_copies
    // accumulators (as many as the grid has blocks, within kGradCopyBytes)
    pl.grad_copies = s->params_global ? (int)std::max<int64_t>(1, std::min<int64_t>(pl.grid,
                                            (int64_t)(kGradCopyBytes / (sizeof(double) * (size_t)P)))) : pl.grid;
    pl.off_gpart = off; off = al256(off + sizeof(double) * (size_t)pl.grad_copies * P);
    pl.off_ovf = off; off = al256(off + sizeof(int) * (size_t)kOvfDepth * pl.grid * kBlock);
    // colour sample sums when pixels are split over lanes: nchunk * npix <= 2 lanes + npix
    const int64_t lanes = (int64_t)pl.grid * kBlock;
    pl.off_part = off; off = al256(off + (npix < 2 * lanes ? sizeof(float) * 3 * (size_t)(2 * lanes + npix) : 0));
    pl.off_ck = off;
    pl.end_fixed = off;
    pl.ck_per_pixel = (size_t)(o->max_depth + 1) * o->spp * (sizeof(int4) + (guided ? 3 : 2) * sizeof(float4));
}

static size_t plan_min(const Plan& pl, int64_t npix) {
    int64_t c = std::min<int64_t>(npix, kBlock);
    return pl.end_fixed + 4 * 256 + (size_t)c * pl.ck_per_pixel;
}
static size_t plan_full(const Plan& pl, int64_t npix) { return pl.end_fixed + 4 * 256 + (size_t)npix * pl.ck_per_pixel; }

extern "C" ipt_status ipt_workspace_query(ipt_scene_t s, const ipt_cameras* cams, const ipt_render_opts* o,
                                          size_t* min_bytes, size_t* full_bytes) {
    if (!s || !min_bytes || !full_bytes) return fail(IPT_ERR_INVALID_ARG, "NULL argument");
    int64_t npix = 0;
    ipt_status st = check_opts(s, cams, o, &npix);
    if (st != IPT_OK) return st;
    Plan pl;
    make_plan(s, o, npix, true, pl);
    *min_bytes = plan_min(pl, npix);
    *full_bytes = plan_full(pl, npix);
    return IPT_OK;
}

static PathArgs base_args(const ipt_scene_s* s, const ipt_cameras* cams, const float* params, const float* sp,
                          const ipt_render_opts* o, unsigned char* ws, const Plan& pl) {
    PathArgs a{};
    a.sc = s->dev;
    a.c2w = cams->cam_to_world;
    a.fov = cams->fov_y;
    a.V = cams->num_views;
    a.W = cams->width;
    a.H = cams->height;
    a.params = params;
    a.sparams = sp ? sp : params;
    a.frozen = (sp && sp != params) ? 1 : 0;
    a.P = s->nm * s->S + 3 * s->E;
    a.mat = s->mat;
    a.cdf = (const float*)(ws + pl.off_cdf);
    a.rng.k0 = (uint32_t)o->seed ^ (o->stream_tag * 0x9E3779B9u);
    a.rng.k1 = (uint32_t)(o->seed >> 32);
    a.rng.iteration = o->iteration;
    a.spp = o->spp;
    a.D = o->max_depth;
    a.rr_depth = o->rr_depth;
    a.mis = o->mis;
    a.profile = o->emission_profile;
    a.jitter = o->jitter;
    a.pixel_list = o->pixel_list;
    a.hash = o->debug_path_hash;
    a.path_L = o->debug_path_radiance;
    a.dbg_vtx = o->debug_vertices;
    a.mask = o->path_mask;
    a.work = (unsigned*)(ws + pl.off_counters);
    a.err = s->d_err;
    a.ovf = (int*)(ws + pl.off_ovf);
    a.grad_part = (double*)(ws + pl.off_gpart);
    a.replay_traverse = o->replay_traverse;
    a.params_global = s->params_global;
    a.grad_copies = pl.grad_copies;
    a.guided = o->guide != nullptr;
    a.gmix = a.guided ? o->guide_mix : 0.0f;
    a.guide_kind = guide_kind(o);
    if (a.guided) a.gd = guide_dev(o->guide);
    return a;
}

static ipt_status do_render(ipt_scene_t s, const ipt_cameras* cams, const float* params, const float* sp,
                            const ipt_render_opts* o, int64_t npix, float* image, unsigned char* ws,
                            const Plan& pl, hipStream_t st, bool allow_profile = true) {
    PathArgs a = base_args(s, cams, params, sp, o, ws, pl);
    a.image = image;
    a.pix_begin = 0;
    a.pix_count = npix;
    split_samples(npix, o->spp, pl.grid, a.spc, a.nchunk);
    a.part = a.nchunk > 1 ? (float*)(ws + pl.off_part) : nullptr;
    HIP_OK(launch_light_cdf(s->dev, a.sparams, (float*)(ws + pl.off_cdf), st));
    HIP_OK(launch_zero_u32(a.work, 1, st));
    size_t lds = path_lds_bytes(kColor, a.P, a.frozen, s->S, s->nlt, a.guide_kind, a.params_global);
    int grid = (int)std::min<int64_t>(pl.grid, (npix * a.nchunk + kBlock - 1) / kBlock);
    if (allow_profile) {
        HIP_OK(timed_launch(s, kColor, a, std::max(1, grid), lds, st));
    } else {
        a.count_stats = 0;
        HIP_OK(launch_paths(kColor, a, std::max(1, grid), lds, st));
    }
    if (a.nchunk > 1) HIP_OK(launch_colour_reduce(a.part, a.nchunk, npix, o->spp, image, st));
    return IPT_OK;
}

static ipt_status do_grad(ipt_scene_t s, const ipt_cameras* cams, const float* params, const float* sp,
                          const ipt_render_opts* o, int64_t npix, const float* w, float* grad, unsigned char* ws,
                          size_t ws_bytes, const Plan& pl, hipStream_t st) {
    PathArgs a = base_args(s, cams, params, sp, o, ws, pl);
    a.w = w;
    split_samples(npix, o->spp, pl.grid, a.spc, a.nchunk);
    // chunk size from the space left for checkpoints
    size_t avail = ws_bytes > pl.end_fixed + 4 * 256 ? ws_bytes - pl.end_fixed - 4 * 256 : 0;
    int64_t chunk = (int64_t)(avail / pl.ck_per_pixel);
    if (chunk < npix) chunk = (chunk / kBlock) * kBlock;
    chunk = std::min<int64_t>(chunk, npix);
    if (chunk < 1) return fail(IPT_ERR_WORKSPACE_TOO_SMALL, "workspace too small for one gradient chunk");
    size_t rec = (size_t)(o->max_depth + 1) * o->spp * (size_t)chunk;
    unsigned char* ck = ws + pl.off_ck;
    a.ck_hit = (int4*)ck;
    a.ck_a = (float4*)(ck + al256(rec * sizeof(int4)));
    a.ck_c = (float4*)(ck + al256(rec * sizeof(int4)) + al256(rec * sizeof(float4)));
    a.ck_d = a.guided ? (float4*)(ck + al256(rec * sizeof(int4)) + 2 * al256(rec * sizeof(float4))) : nullptr;
    if (a.guided) {
        a.grec = guide_records(o->guide);
        a.grec_count = guide_record_count(o->guide);
        a.grec_cap = guide_capacity(o->guide);
        a.grec_stride = guide_record_stride(o->guide);
    }
    HIP_OK(launch_light_cdf(s->dev, a.sparams, (float*)(ws + pl.off_cdf), st));
    size_t lds_f = path_lds_bytes(kGradFwd, a.P, a.frozen, s->S, s->nlt, a.guide_kind, a.params_global);
    size_t lds_r = path_lds_bytes(kReplay, a.P, a.frozen, s->S, s->nlt, 0, a.params_global);
    if (a.params_global) HIP_OK(launch_zero_u32((unsigned*)a.grad_part, 2 * a.grad_copies * a.P, st));
    for (int64_t b = 0; b < npix; b += chunk) {
        a.pix_begin = b;
        a.pix_count = std::min<int64_t>(chunk, npix - b);
        int grid = (int)std::max<int64_t>(1, std::min<int64_t>(pl.grid, (a.pix_count * a.nchunk + kBlock - 1) / kBlock));
        HIP_OK(launch_zero_u32(a.work, 1, st));
        HIP_OK(timed_launch(s, kGradFwd, a, grid, lds_f, st));
        if (a.guided) HIP_OK(launch_guide_records(a, st));
        // the replay pulls tiles, so it runs on as many blocks as are resident
        int grid_r = std::min(grid, s->num_cu * std::max(1, path_blocks_per_cu(kReplay, lds_r, 0, a.params_global, a.mat)));
        HIP_OK(launch_zero_u32(a.work, 1, st));
        HIP_OK(timed_launch(s, kReplay, a, grid_r, lds_r, st));
        if (!a.params_global) HIP_OK(launch_grad_reduce(a.grad_part, grid_r, a.P, grad, b > 0 ? 1 : 0, st));
    }
    if (a.params_global) HIP_OK(launch_grad_reduce(a.grad_part, a.grad_copies, a.P, grad, 0, st));
    return IPT_OK;
}

extern "C" ipt_status ipt_render(ipt_scene_t s, const ipt_cameras* cams, const float* params,
                                 const float* sampling_params, const ipt_render_opts* o, float* image,
                                 void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (!s || !params || !image) return fail(IPT_ERR_INVALID_ARG, "NULL scene/params/image");
    int64_t npix = 0;
    ipt_status stt = check_opts(s, cams, o, &npix);
    if (stt != IPT_OK) return stt;
    Plan pl;
    make_plan(s, o, npix, false, pl);
    if (!workspace || workspace_bytes < pl.end_fixed)
        return fail(IPT_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", pl.end_fixed);
    return do_render(s, cams, params, sampling_params, o, npix, image, (unsigned char*)workspace, pl,
                     (hipStream_t)hip_stream);
}

// ---------------------------------------------------------------------------
// Allocation-free colour pass: the scratch that ipt_render takes from the
// caller's workspace (work counter, light table, traversal overflow stacks,
// per-chunk sample sums) lives in this file-scope device array instead.
// Host code must not use the name `scratch` as an address: it stands for
// the device symbol; the pointer comes from hipGetSymbolAddress, once per
// device, with that device current.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(40) << 20;
constexpr int kStaticBlocksPerCu = 2;     // bounds the overflow stacks to 48 x 512 x 256 ints
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_ptr[kMaxDevices];   // per device, set on its first call

static ipt_status scratch_for_device(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(IPT_ERR_NOT_SUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(IPT_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = (unsigned char*)p;
    }
    *out = g_scratch_ptr[dev];
    return IPT_OK;
}

// Layout of the colour pass's scratch for a grid of at most
// kStaticBlocksPerCu blocks per CU; returns the bytes it needs.
static size_t static_render_plan(const ipt_scene_s* s, const ipt_render_opts* o, int64_t npix, Plan& pl) {
    const int P = s->nm * s->S + 3 * s->E;
    pl.grid = std::min(path_grid(s, P, 1, guide_kind(o)), s->num_cu * kStaticBlocksPerCu);
    size_t off = 0;
    pl.off_counters = off; off = al256(off + 64 * sizeof(unsigned));
    pl.off_cdf = off; off = al256(off + 2 * sizeof(float) * std::max(1, s->nlt));
    pl.off_loss = pl.off_w = pl.off_img = pl.off_gpart = off;   // unused by the colour pass
    pl.grad_copies = 0;
    pl.off_ovf = off; off = al256(off + sizeof(int) * (size_t)kOvfDepth * pl.grid * kBlock);
    const int64_t lanes = (int64_t)pl.grid * kBlock;
    pl.off_part = off; off = al256(off + (npix < 2 * lanes ? sizeof(float) * 3 * (size_t)(2 * lanes + npix) : 0));
    pl.off_ck = off;
    pl.end_fixed = off;
    return off;
}

extern "C" ipt_status ipt_render_static(ipt_scene_t s, const ipt_cameras* cams, const float* params,
                                        const float* sampling_params, const ipt_render_opts* o, float* image,
                                        void* hip_stream) {
    if (!s || !params || !image) return fail(IPT_ERR_INVALID_ARG, "NULL scene/params/image");
    int64_t npix = 0;
    ipt_status stt = check_opts(s, cams, o, &npix);
    if (stt != IPT_OK) return stt;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev != s->device) return fail(IPT_ERR_INVALID_ARG, "scene built on device %d, current device %d", s->device, dev);
    Plan pl;
    const size_t need = static_render_plan(s, o, npix, pl);
    if (need > kStaticScratchBytes)
        return fail(IPT_ERR_NOT_SUPPORTED, "ipt_render_static needs %zu bytes of scratch (%d light triangles, "
                    "%lld pixels), more than its fixed %zu; use ipt_render with a workspace", need, s->nlt,
                    (long long)npix, kStaticScratchBytes);
    unsigned char* ws = nullptr;
    stt = scratch_for_device(dev, &ws);
    if (stt != IPT_OK) return stt;
    return do_render(s, cams, params, sampling_params, o, npix, image, ws, pl, (hipStream_t)hip_stream, false);
}

extern "C" ipt_status ipt_render_grad(ipt_scene_t s, const ipt_cameras* cams, const float* params,
                                      const float* sampling_params, const ipt_render_opts* o, const float* w,
                                      float* grad, void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (!s || !params || !w || !grad) return fail(IPT_ERR_INVALID_ARG, "NULL scene/params/w/grad");
    int64_t npix = 0;
    ipt_status stt = check_opts(s, cams, o, &npix);
    if (stt != IPT_OK) return stt;
    Plan pl;
    make_plan(s, o, npix, false, pl);
    if (!workspace || workspace_bytes < plan_min(pl, npix))
        return fail(IPT_ERR_WORKSPACE_TOO_SMALL, "workspace needs at least %zu bytes", plan_min(pl, npix));
    return do_grad(s, cams, params, sampling_params, o, npix, w, grad, (unsigned char*)workspace, workspace_bytes,
                   pl, (hipStream_t)hip_stream);
}

extern "C" ipt_status ipt_loss_grad(ipt_scene_t s, const ipt_cameras* cams, const float* params,
                                    const float* target, const ipt_render_opts* co, const ipt_render_opts* go,
                                    int32_t loss_kind, float* loss, float* grad, float* image_A, void* workspace,
                                    size_t workspace_bytes, void* hip_stream) {
    if (!s || !params || !target || !loss || !grad) return fail(IPT_ERR_INVALID_ARG, "NULL argument");
    if (loss_kind != 0 && loss_kind != 1) return fail(IPT_ERR_INVALID_ARG, "loss_kind must be 0 or 1");
    int64_t npa = 0, npb = 0;
    ipt_status stt = check_opts(s, cams, co, &npa);
    if (stt != IPT_OK) return stt;
    stt = check_opts(s, cams, go, &npb);
    if (stt != IPT_OK) return stt;
    if (npa != npb || (co->pixel_list == nullptr) != (go->pixel_list == nullptr))
        return fail(IPT_ERR_INVALID_ARG, "colour and gradient options must cover the same pixels");
    Plan pl;
    make_plan(s, go, npb, true, pl);
    if (!workspace || workspace_bytes < plan_min(pl, npb))
        return fail(IPT_ERR_WORKSPACE_TOO_SMALL, "workspace needs at least %zu bytes", plan_min(pl, npb));
    unsigned char* ws = (unsigned char*)workspace;
    hipStream_t st = (hipStream_t)hip_stream;
    float* img = image_A ? image_A : (float*)(ws + pl.off_img);
    float* w = (float*)(ws + pl.off_w);
    stt = do_render(s, cams, params, nullptr, co, npa, img, ws, pl, st);
    if (stt != IPT_OK) return stt;
    HIP_OK(launch_loss_adjoint(img, target, 3 * npa, loss_kind, w, (float*)(ws + pl.off_loss), 1024, loss, st));
    return do_grad(s, cams, params, nullptr, go, npb, w, grad, ws, workspace_bytes, pl, st);
}

extern "C" ipt_status ipt_sgd_step(float* params, const float* grad, float* m, float* v, int32_t P, int32_t step,
                                   const ipt_adam_opts* adam, const float* scale, const float* lo, const float* hi,
                                   const uint8_t* trainable, void* hip_stream) {
    if (!params || !grad || !m || !v || !adam) return fail(IPT_ERR_INVALID_ARG, "NULL argument");
    if (P < 1 || step < 1) return fail(IPT_ERR_INVALID_ARG, "need P >= 1 and step >= 1");
    if (!(adam->lr > 0.0f) || !(adam->beta1 >= 0.0f && adam->beta1 < 1.0f) ||
        !(adam->beta2 >= 0.0f && adam->beta2 < 1.0f) || !(adam->eps > 0.0f))
        return fail(IPT_ERR_INVALID_ARG, "bad Adam hyper-parameters");
    HIP_OK(launch_adam(params, grad, m, v, P, step, adam->lr, adam->beta1, adam->beta2, adam->eps, scale, lo, hi,
                       trainable, (hipStream_t)hip_stream));
    return IPT_OK;
}

extern "C" ipt_status ipt_l1_reg(const float* params, float* grad, const float* weight, int32_t P, float* loss,
                                 void* hip_stream) {
    if (!params || !grad || !weight || !loss) return fail(IPT_ERR_INVALID_ARG, "NULL argument");
    if (P < 1) return fail(IPT_ERR_INVALID_ARG, "P must be >= 1");
    HIP_OK(launch_l1_reg(params, grad, weight, P, loss, (hipStream_t)hip_stream));
    return IPT_OK;
}

extern "C" ipt_status ipt_trace_rays(ipt_scene_t s, const float* origins, const float* dirs, const int32_t* skip_tri,
                                     int64_t n, float tmin, int32_t brute_force, int32_t* out_tri, float* out_tuv,
                                     void* hip_stream) {
    if (!s || !origins || !dirs || !out_tri || !out_tuv) return fail(IPT_ERR_INVALID_ARG, "NULL argument");
    if (n < 0) return fail(IPT_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return IPT_OK;
    HIP_OK(launch_trace_rays(s->dev, origins, dirs, skip_tri, n, tmin, brute_force, s->nt, out_tri, out_tuv,
                             s->d_ovf_rays, trace_rays_grid(s->num_cu), s->d_err, (hipStream_t)hip_stream));
    return IPT_OK;
}

extern "C" ipt_status ipt_profile_enable(ipt_scene_t s, int32_t enable) {
    if (!s) return fail(IPT_ERR_INVALID_ARG, "NULL scene");
    s->prof = enable != 0;
    return IPT_OK;
}

extern "C" ipt_status ipt_profile_reset(ipt_scene_t s) {
    if (!s) return fail(IPT_ERR_INVALID_ARG, "NULL scene");
    HIP_OK(hipDeviceSynchronize());
    prof_clear_events(s);
    HIP_OK(hipMemset(&s->d_err->k[0], 0, sizeof(KStats) * 3));
    return IPT_OK;
}

extern "C" ipt_status ipt_profile_read(ipt_scene_t s, int32_t kernel, ipt_kernel_profile* out) {
    if (!s || !out || kernel < 0 || kernel > 2) return fail(IPT_ERR_INVALID_ARG, "bad argument");
    HIP_OK(hipDeviceSynchronize());
    double tot = 0.0;
    for (auto& p : s->ev[kernel]) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, p.first, p.second));
        tot += ms;
    }
    Counters c;
    HIP_OK(hipMemcpy(&c, s->d_err, sizeof(Counters), hipMemcpyDeviceToHost));
    out->launches = (int64_t)s->ev[kernel].size();
    out->total_ms = tot;
    out->rays = c.k[kernel].rays;
    out->nodes = c.k[kernel].nodes;
    out->tris = c.k[kernel].tris;
    out->paths = c.k[kernel].paths;
    out->vertices = c.k[kernel].vertices;
    out->units = c.k[kernel].units;
    return IPT_OK;
}

ipt_status guide_create_impl(int S, const float lo[3], const float hi[3], const ipt_guide_opts* o, void* stream,
                             ipt_guide_t* out);

extern "C" ipt_status ipt_guide_cache_build(ipt_guide_t g, ipt_scene_t s, float cell_area, int32_t mode,
                                            int64_t* num_cells, void* stream) {
    if (!g || !s) return fail(IPT_ERR_INVALID_ARG, "NULL guide or scene");
    return guide_cache_build_impl(g, s, s->d_tris, s->d_nrm, s->nt, cell_area, mode, (hipStream_t)stream, num_cells);
}

extern "C" ipt_status ipt_guide_create(ipt_scene_t s, const ipt_guide_opts* o, void* stream, ipt_guide_t* out) {
    if (!s || !o || !out) return fail(IPT_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (o->batch < 64 || o->batch % 64 || o->ring_capacity < 64 || !(o->lr > 0.0f) || o->record_stride < 1)
        return fail(IPT_ERR_INVALID_ARG, "guide options: batch multiple of 64, ring >= 64, lr > 0, stride >= 1");
    return guide_create_impl(s->S, s->bb_lo, s->bb_hi, o, stream, out);
}
