// Path kernels of the inverse path tracer (gfx950).
//
// Three passes share one set of shading functions, so they compute the same
// values:
//   kColor   - the Monte Carlo pixel estimate (Sec. 3.1, Eq. 1-2) with MIS of
//              BRDF sampling and light sampling (Appendix A.2, Appendix E);
//   kGradFwd - the gradient-stream forward pass: traces the independent
//              paths (Sec. 3.3: independent samples for the estimate and for
//              its gradient), stores per-vertex hit checkpoints, the local
//              contribution c_k and continuation weight a_k, then sweeps the
//              path backwards to turn them into the suffix radiance
//              R_{k+1} = c_{k+1} + a_{k+1} R_{k+2} (no division, so exact at
//              zero albedo or zero emission);
//   kReplay  - the adjoint: replays every path from its Philox counter (hits
//              from the checkpoints, or re-traced), carries the prefix
//              throughput T_{k-1} and adds, per vertex,
//              w . T_{k-1} (dc_k/dtheta + da_k/dtheta R_{k+1}) -- the product
//              rule of Eq. 5 (emission) and Eq. 6 (materials) -- into a block
//              private gradient in LDS.
//
// kColor and kGradFwd run as a per-lane state machine around ONE traversal
// call site that serves both closest-hit and shadow rays: every iteration
// each lane traces whatever ray it has pending, then advances its path.  A
// lane owns one pixel and walks its spp samples in order, so the pixel mean
// is formed in registers (deterministic, no atomics); a lane that finishes
// its pixel takes the next one at once (the wave takes as many pixels as it
// has idle lanes with one atomic).  The lanes of a wave thus stay in the same
// phase instead of serialising the divergent loops of a nested megakernel.
#include <hip/hip_runtime.h>

#include "ipt_internal.h"
#include "disney.h"

namespace ipt {

struct Lds {
    __bf16* gact;       // this wave's guide activation rows (guided kernels)
    float* params;
    float* sparams;
    int* seg_emitter;
    float* cdf;
    int4* lights;
    double* grad;       // replay: block gradient, float64 (the terms of some entries cancel)
    int* stack;
    bool lights_in_lds;
};

// per-wave guide activation rows (64 x kGRowStride bf16), 4 waves per block
constexpr size_t kGuideLds = 4 * 64 * kGRowStride * sizeof(__bf16);

size_t path_lds_bytes(int mode, int P, int frozen, int S, int nlt, int gk, int pglobal) {
    size_t b = 0;
    auto al = [](size_t x) { return (x + 15) & ~size_t(15); };
    if (pglobal) P = S = 0;                           // read from global memory
    b += al(sizeof(float) * P);                       // params
    if (frozen) b += al(sizeof(float) * P);           // sampling params
    b += al(sizeof(int) * S);                         // segment -> emitter
    if (nlt <= kMaxLdsLights) b += al(2 * sizeof(float) * nlt) + al(sizeof(int4) * nlt);
    if (mode == kReplay) b += al(sizeof(double) * P); // block gradient
    b += sizeof(int) * kShortStack * kBlock;          // short stacks
    if ((gk == 1 || gk == 2) && mode != kReplay) b += kGuideLds;   // network activations / outputs
    return b;
}

// PG (a compile-time copy of PathArgs::params_global) keeps each pointer's
// address space known, so LDS reads stay ds_read and the LDS gradient
// ds_add_f64 rather than flat accesses.
template <int PG>
__device__ void carve_lds(const PathArgs& a, int mode, unsigned char* smem, Lds& lds) {
    const int tid = threadIdx.x;
    unsigned char* p = smem;
    auto al = [](size_t x) { return (x + 15) & ~size_t(15); };
    constexpr int pg = PG;
    if constexpr (PG) {
        // parameters, segment table and the replay's gradient accumulator in global memory
        lds.params = (float*)a.params;
        lds.sparams = (float*)a.sparams;
        lds.seg_emitter = (int*)a.sc.seg_emitter;
    } else {
        lds.params = (float*)p; p += al(sizeof(float) * a.P);
        lds.sparams = lds.params;
        if (a.frozen) { lds.sparams = (float*)p; p += al(sizeof(float) * a.P); }
        lds.seg_emitter = (int*)p; p += al(sizeof(int) * a.sc.S);
    }
    lds.lights_in_lds = a.sc.nlt <= kMaxLdsLights;
    lds.cdf = nullptr;
    lds.lights = nullptr;
    if (lds.lights_in_lds) {
        lds.cdf = (float*)p; p += al(2 * sizeof(float) * a.sc.nlt);
        lds.lights = (int4*)p; p += al(sizeof(int4) * a.sc.nlt);
    }
    lds.grad = nullptr;
    if (mode == kReplay) {
        if constexpr (PG) lds.grad = a.grad_part + (size_t)(blockIdx.x % a.grad_copies) * a.P;
        else { lds.grad = (double*)p; p += al(sizeof(double) * a.P); }
    }
    lds.stack = (int*)p;
    p += sizeof(int) * kShortStack * kBlock;
    lds.gact = (__bf16*)p + (threadIdx.x >> 6) * 64 * kGRowStride;
    if constexpr (!pg) {
        for (int i = tid; i < a.P; i += kBlock) {
            lds.params[i] = a.params[i];
            if (a.frozen) lds.sparams[i] = a.sparams[i];
            if (mode == kReplay) lds.grad[i] = 0.0;
        }
        for (int i = tid; i < a.sc.S; i += kBlock) lds.seg_emitter[i] = a.sc.seg_emitter[i];
    }
    if (lds.lights_in_lds)
        for (int i = tid; i < a.sc.nlt; i += kBlock) {
            lds.cdf[i] = a.cdf[i];
            lds.cdf[a.sc.nlt + i] = a.cdf[a.sc.nlt + i];
            lds.lights[i] = a.sc.lights[i];
        }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Traversal with a per-lane short stack in LDS ([slot][lane] layout, so the
// 64 lanes of a wave hit 64 distinct banks) that spills its oldest entries to
// a per-lane global stack ([depth][thread], coalesced).
// ---------------------------------------------------------------------------
struct Stack {
    int* lds;     // kShortStack * kBlock
    int* ovf;
    int tid, gtid, gthreads;
    int sp;
    bool overflow;
    __device__ __forceinline__ void push(int x) {
        int slot = sp & (kShortStack - 1);
        if (sp >= kShortStack) {
            int d = sp - kShortStack;
            if (d >= kOvfDepth) { overflow = true; return; }
            ovf[(size_t)d * gthreads + gtid] = lds[slot * kBlock + tid];
        }
        lds[slot * kBlock + tid] = x;
        ++sp;
    }
    // Pushes the n (0..3) entries x0..x(n-1), x0 deepest.  With room for
    // three in the LDS window (and so no entry to move to the overflow
    // stack) all three slots are written, whatever n: the slots above the
    // new top hold no live entry.
    __device__ __forceinline__ void push_upto3(int n, int x0, int x1, int x2) {
        if (sp + 3 <= kShortStack) {
            int* s = lds + sp * kBlock + tid;
            s[0] = x0;
            s[kBlock] = x1;
            s[2 * kBlock] = x2;
            sp += n;
        } else {
            if (n > 0) push(x0);
            if (n > 1) push(x1);
            if (n > 2) push(x2);
        }
    }
    __device__ __forceinline__ int pop() {
        --sp;
        int slot = sp & (kShortStack - 1);
        int x = lds[slot * kBlock + tid];
        if (sp >= kShortStack) lds[slot * kBlock + tid] = ovf[(size_t)(sp - kShortStack) * gthreads + gtid];
        return x;
    }
};

__device__ __forceinline__ void init_stack(Stack& st, const PathArgs& a, int* lds_stack) {
    st.lds = lds_stack;
    st.ovf = a.ovf;
    st.tid = threadIdx.x;
    st.gtid = blockIdx.x * kBlock + threadIdx.x;
    st.gthreads = gridDim.x * kBlock;
    st.overflow = false;
    st.sp = 0;
}

struct Hit {
    int tri;     // leaf-ordered index, -1 on miss
    float t, u, v;
};

struct Work {
    uint32_t rays, nodes, tris, vertices, units;
};

__device__ __forceinline__ void load_tri(const SceneDev& sc, int i, V3& p0, V3& p1, V3& p2, int& orig,
                                         int& seg, int& light) {
    float4 a = sc.tris[3 * i], b = sc.tris[3 * i + 1], c = sc.tris[3 * i + 2];
    p0 = xyz(a); p1 = xyz(b); p2 = xyz(c);
    orig = __float_as_int(a.w);
    seg = __float_as_int(b.w);
    light = __float_as_int(c.w);
}

constexpr int kTravDone = (int)0x80000000;   // no node left (leaf codes are > INT_MIN)

// Bytes 0 and 2 (or 1 and 3) of a quantized plane row, zero-extended into the
// two 16-bit halves of a register: each half, read as fp16, is the subnormal
// q 2^-24 (kernels keep fp16 denormals, the default fp16/fp64 denormal mode;
// the BVH tests compare the hits with brute force bit for bit).
typedef _Float16 h2x __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2x bytes02(uint32_t w) { return __builtin_bit_cast(h2x, w & 0x00ff00ffu); }
__device__ __forceinline__ h2x bytes13(uint32_t w) {
    return __builtin_bit_cast(h2x, __builtin_amdgcn_perm(w, w, 0x0c030c01u));
}

// Traversal state of one lane, kept across calls when a call returns early.
struct Trav {
    int cur;        // next node: inner (>= 0), leaf code (< 0) or kTravDone
    int pend;       // leaf held for the leaf phase
    int best_orig;  // original id of the best hit (tie rule)
    Hit best;
};

__device__ __forceinline__ void trav_init(Trav& tv, float tmax, Stack& st, Work& wk) {
    tv.cur = 0;
    tv.pend = kTravDone;
    tv.best_orig = 0x7FFFFFFF;
    tv.best = Hit{-1, tmax, 0.0f, 0.0f};
    st.sp = 0;
    wk.rays++;
}

// The node phase ends early once no more than this many lanes of the wave
// are still looking for their first leaf (0: it runs until none is).
// Apartment step with binary nodes: 166.7 ms at 0; 159.0 / 157.8 / 157.3 /
// 157.1 / 158.0 / 169.9 / 204.3 ms at 2 / 3 / 4 / 6 / 8 / 16 / 32.  With
// quantized four-child nodes and two-triangle leaves, whose leaf phase is
// cheaper (testing the held leaves sooner also shortens the rays' best
// distance): 125.9 / 123.2 / 122.4 ms at 2 / 4 / 8 in one run, and
// 123.8 / 123.0 / 124.8 / 129.7 / 141.1 ms at 4 / 8 / 12 / 16 / 24 in another.
#ifndef IPT_NODE_BREAK
#define IPT_NODE_BREAK 8
#endif


// Advances the lanes' traversals; returns true for a lane whose traversal
// has finished (its hit is then in tv.best).  With exit_lanes > 0 the call
// also returns, after at least one node phase and one leaf phase (so every
// call advances every unfinished lane), as soon as no more than exit_lanes
// lanes of the wave are still traversing: those keep their state and resume
// on the next call, while the others shade and start new rays, instead of
// idling through the slowest rays' tail.
__device__ bool traverse_resume(const SceneDev& sc, const Ray& r, float tmin, float tmax, int skip0, int skip1,
                                bool any, Stack& st, Work& wk, Trav& tv, int exit_lanes) {
    int cur = tv.cur, pend = tv.pend, best_orig = tv.best_orig;
    Hit best = tv.best;
    // direction signs: which byte row of a quantized node is an axis's near plane
    const bool negx = r.inv.x < 0.0f, negy = r.inv.y < 0.0f, negz = r.inv.z < 0.0f;
    auto next_from_stack = [&]() -> int { return (st.sp > 0 && !st.overflow) ? st.pop() : kTravDone; };
    while (true) {
        // ---- node phase ----
        while (true) {
            if (cur < 0 && cur != kTravDone && pend == kTravDone) {
                pend = cur;
                cur = next_from_stack();
            }
            const bool inner = cur >= 0;
            const uint64_t searching = __ballot(inner && pend == kTravDone);
            if (!searching) break;
            // few lanes still looking for their first leaf: test the leaves
            // the others hold now, and let those lanes descend again with
            // the rest after the leaf phase (at least one leaf is pending,
            // so every pass of the outer loop makes progress)
            if (IPT_NODE_BREAK > 0 && __popcll(searching) <= IPT_NODE_BREAK && __any(pend != kTravDone)) break;
            if (inner && kNodeWidth == 4) {
                // four children: the nearest hit next, the others pushed far to near
                wk.nodes++;
                const float inf = __builtin_inff();
                float t[4];
                int c[4];
                if constexpr (kNodeQuant) {
                    // quantized child boxes: a plane is origin + q 2^e, so its
                    // slab distance is fma(q, 2^e / d, (origin - o) / d); the
                    // direction's sign picks each axis's near and far byte rows.
                    // The byte enters the fma as an fp16 operand of the
                    // mixed-precision fma (one instruction per plane instead of
                    // a conversion and an fma; the same value bit for bit)
                    const float4* n = sc.nodes + 4 * (size_t)cur;
                    const float4 h = n[0], qa = n[1], qb = n[2], cr = n[3];
                    c[0] = __float_as_int(cr.x); c[1] = __float_as_int(cr.y);
                    c[2] = __float_as_int(cr.z); c[3] = __float_as_int(cr.w);
                    // the references are needed only after the sort; tie them
                    // to this point so their load issues with the box rows
                    __asm__ volatile("" :: "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
                    const uint32_t ew = __float_as_uint(h.w);
                    // A carries an extra 2^24: a byte q, widened to 16 bits, is
                    // read as the fp16 subnormal q 2^-24, so the mixed-precision
                    // fma forms q 2^e / d + B exactly, with no conversion
                    const V3 A = v3(ldexpf(r.inv.x, (int)(ew & 0xffu) - 103),
                                    ldexpf(r.inv.y, (int)((ew >> 8) & 0xffu) - 103),
                                    ldexpf(r.inv.z, (int)((ew >> 16) & 0xffu) - 103));
                    const V3 B = v3((h.x - r.o.x) * r.inv.x, (h.y - r.o.y) * r.inv.y, (h.z - r.o.z) * r.inv.z);
                    const uint32_t xl = __float_as_uint(qa.x), xh = __float_as_uint(qa.y);
                    const uint32_t yl = __float_as_uint(qa.z), yh = __float_as_uint(qa.w);
                    const uint32_t zl = __float_as_uint(qb.x), zh = __float_as_uint(qb.y);
                    const uint32_t xn = negx ? xh : xl, xf = negx ? xl : xh;
                    const uint32_t yn = negy ? yh : yl, yf = negy ? yl : yh;
                    const uint32_t zn = negz ? zh : zl, zf = negz ? zl : zh;
                    const float tmx = best.t + sc.tmin;
                    // 16-bit lanes of children 0 and 2, and of children 1 and 3
                    const h2x e02[6] = {bytes02(xn), bytes02(xf), bytes02(yn), bytes02(yf), bytes02(zn), bytes02(zf)};
                    const h2x e13[6] = {bytes13(xn), bytes13(xf), bytes13(yn), bytes13(yf), bytes13(zn), bytes13(zf)};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const h2x* e = (i & 1) ? e13 : e02;
                        const int hi = i >> 1;
                        const float nx = fmaf((float)(hi ? e[0].y : e[0].x), A.x, B.x);
                        const float fx = fmaf((float)(hi ? e[1].y : e[1].x), A.x, B.x);
                        const float ny = fmaf((float)(hi ? e[2].y : e[2].x), A.y, B.y);
                        const float fy = fmaf((float)(hi ? e[3].y : e[3].x), A.y, B.y);
                        const float nz = fmaf((float)(hi ? e[4].y : e[4].x), A.z, B.z);
                        const float fz = fmaf((float)(hi ? e[5].y : e[5].x), A.z, B.z);
                        const float tn = fmaxf(fmaxf(nx, ny), fmaxf(nz, tmin));
                        const float tf = fminf(fminf(fx, fy), fminf(fz, tmx));
                        t[i] = tn <= tf * 1.0000005f ? tn : inf;
                    }
                } else {
                    // float child boxes; an empty slot's box is +inf on every
                    // axis, so its entry distance is +inf and it sorts last
                    const float4* n = sc.nodes + 8 * (size_t)cur;
                    const float4 lx = n[0], hx = n[1], ly = n[2], hy = n[3], lz = n[4], hz = n[5], cr = n[6];
                    c[0] = __float_as_int(cr.x); c[1] = __float_as_int(cr.y);
                    c[2] = __float_as_int(cr.z); c[3] = __float_as_int(cr.w);
                    t[0] = box_entry(r, v3(lx.x, ly.x, lz.x), v3(hx.x, hy.x, hz.x), tmin, best.t, sc.tmin);
                    t[1] = box_entry(r, v3(lx.y, ly.y, lz.y), v3(hx.y, hy.y, hz.y), tmin, best.t, sc.tmin);
                    t[2] = box_entry(r, v3(lx.z, ly.z, lz.z), v3(hx.z, hy.z, hz.z), tmin, best.t, sc.tmin);
                    t[3] = box_entry(r, v3(lx.w, ly.w, lz.w), v3(hx.w, hy.w, hz.w), tmin, best.t, sc.tmin);
                }
                // sorting network on (t, child) with selects, no branches;
                // equal distances keep their slot order
                auto cas = [&](int i, int j) {
                    const bool sw = t[j] < t[i];
                    const float ti = t[i], tj = t[j];
                    const int ci = c[i], cj = c[j];
                    t[i] = sw ? tj : ti;
                    t[j] = sw ? ti : tj;
                    c[i] = sw ? cj : ci;
                    c[j] = sw ? ci : cj;
                };
                cas(0, 1); cas(2, 3); cas(0, 2); cas(1, 3); cas(1, 2);
                if (t[0] < inf) {
                    // the entered children are a prefix of the sorted slots:
                    // push the nf after the nearest, farthest first
                    const int nf = (t[1] < inf ? 1 : 0) + (t[2] < inf ? 1 : 0) + (t[3] < inf ? 1 : 0);
                    st.push_upto3(nf, nf == 3 ? c[3] : (nf == 2 ? c[2] : c[1]), nf == 3 ? c[2] : c[1], c[1]);
                    cur = c[0];
                } else {
                    cur = next_from_stack();
                }
            } else if (inner) {
                wk.nodes++;
                const float4* n = sc.nodes + 4 * (size_t)cur;
                float4 n0 = n[0], n1 = n[1], n2 = n[2], n3 = n[3];
                int c0 = __float_as_int(n3.x), c1 = __float_as_int(n3.y);
                float t0 = box_entry(r, v3(n0.x, n0.y, n0.z), v3(n0.w, n1.x, n1.y), tmin, best.t, sc.tmin);
                float t1 = box_entry(r, v3(n1.z, n1.w, n2.x), v3(n2.y, n2.z, n2.w), tmin, best.t, sc.tmin);
                // box_entry returns +inf on a miss; best.t may itself be +inf
                bool h0 = t0 < __builtin_inff();
                bool h1 = (c1 != kNone) && t1 < __builtin_inff();
                if (h0 && h1) {
                    bool first0 = t0 <= t1;
                    st.push(first0 ? c1 : c0);
                    cur = first0 ? c0 : c1;
                } else if (h0) {
                    cur = c0;
                } else if (h1) {
                    cur = c1;
                } else {
                    cur = next_from_stack();
                }
            }
        }
        // ---- leaf phase ----
        if (pend != kTravDone) {
            int code = ~pend;
            int first = code >> 3, cnt = (code & 7) + 1;
            pend = kTravDone;
            wk.tris += cnt;
            for (int i = first; i < first + cnt; ++i) {
                if (i == skip0 || i == skip1) continue;
                V3 p0, p1, p2;
                int orig, seg, light;
                load_tri(sc, i, p0, p1, p2, orig, seg, light);
                float t, u, v;
                if (!tri_isect(r, p0, p1, p2, tmin, t, u, v)) continue;
                if (any) {
                    if (t < tmax) {
                        best.tri = i; best.t = t;
                        cur = kTravDone;
                        break;
                    }
                } else if (t < best.t || (t == best.t && orig < best_orig)) {
                    best.tri = i; best.t = t; best.u = u; best.v = v;
                    best_orig = orig;
                }
            }
        }
        const uint64_t live = __ballot(cur != kTravDone);
        if (!live) break;
        if (exit_lanes > 0 && __popcll(live) <= exit_lanes) break;
    }
    tv.cur = cur;
    tv.pend = pend;
    tv.best_orig = best_orig;
    const bool done = cur == kTravDone;
    if (done && !any && best.tri >= 0 && !(best.t < tmax)) best.tri = -1;
    tv.best = best;
    return done;
}

// Closest hit (any = false) or occlusion test (any = true: stops at the
// first hit in (tmin, tmax)), run to completion.  skip0/skip1 are leaf
// indices that are ignored.  Ties in t are resolved toward the smaller
// original id.
//
// Loop structure for 64-wide waves ("while-while" with speculative
// traversal, Aila and Laine 2009): the node phase visits inner nodes until
// every lane holds a leaf (a lane that already holds one keeps descending, and
// stops only at a second leaf), then the leaf phase tests the held leaves of
// all lanes together.  Node code and triangle code thus run with most lanes
// doing the same thing, instead of every iteration paying for both.
__device__ Hit traverse(const SceneDev& sc, const Ray& r, float tmin, float tmax, int skip0, int skip1, bool any,
                        Stack& st, Work& wk) {
    Trav tv;
    trav_init(tv, tmax, st, wk);
    traverse_resume(sc, r, tmin, tmax, skip0, skip1, any, st, wk, tv, 0);
    return tv.best;
}

// Brute-force closest hit (reference for the BVH).
__device__ Hit brute_closest(const SceneDev& sc, int64_t nt, const Ray& r, float tmin, int skip) {
    Hit best{-1, __builtin_inff(), 0.0f, 0.0f};
    int best_orig = 0x7FFFFFFF;
    for (int64_t i = 0; i < nt; ++i) {
        if ((int)i == skip) continue;
        V3 p0, p1, p2;
        int orig, seg, light;
        load_tri(sc, (int)i, p0, p1, p2, orig, seg, light);
        float t, u, v;
        if (!tri_isect(r, p0, p1, p2, tmin, t, u, v)) continue;
        if (t < best.t || (t == best.t && orig < best_orig)) {
            best.tri = (int)i; best.t = t; best.u = u; best.v = v;
            best_orig = orig;
        }
    }
    return best;
}

// ---------------------------------------------------------------------------
// Light selection from the cumulative table (first j with cdf[j] > u*total);
// cdf[n + j] holds light j's selection probability.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pick_light(const float* cdf, int n, float u) {
    float x = u * cdf[n - 1];
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cdf[mid] > x) hi = mid; else lo = mid + 1;
    }
    return lo;
}
__device__ __forceinline__ float light_prob(const float* cdf, int n, int j) {
    return cdf[n + j];
}

__device__ __forceinline__ void camera_ray(const PathArgs& a, int view, float px, float py, V3& o, V3& d) {
    const float* M = a.c2w + 16 * view;
    float th = tanf(0.5f * a.fov[view]);
    float asp = (float)a.W / (float)a.H;
    float cx = (2.0f * px / (float)a.W - 1.0f) * th * asp;
    float cy = (1.0f - 2.0f * py / (float)a.H) * th;
    V3 dw = v3(M[0] * cx + M[1] * cy - M[2], M[4] * cx + M[5] * cy - M[6], M[8] * cx + M[9] * cy - M[10]);
    o = v3(M[3], M[7], M[11]);
    d = normalize(dw);
}

__device__ __forceinline__ void lds_add(double* g, int i, float x) {
    if (x != 0.0f) atomicAdd(g + i, (double)x);
}

// ---------------------------------------------------------------------------
// Shading shared by all passes.
// ---------------------------------------------------------------------------
struct Shade {
    V3 p0, e1, e2, x, ng, ngf, ns, wo;
    V3 tx, ty;   // tangent frame of the Disney model (set by mat_frame)
    int tri, orig, seg, light, em;
    float u, v, t, cos_emit;
};

// Geometry of a hit: position from barycentrics, geometric and shading
// normals, both flipped toward the incoming ray (two-sided reflection).
__device__ __forceinline__ void make_shade(const SceneDev& sc, const Lds& lds, const Hit& hit, V3 d, Shade& g) {
    V3 p1, p2;
    load_tri(sc, hit.tri, g.p0, p1, p2, g.orig, g.seg, g.light);
    g.tri = hit.tri;
    g.u = hit.u;
    g.v = hit.v;
    g.t = hit.t;
    g.e1 = p1 - g.p0;
    g.e2 = p2 - g.p0;
    g.x = g.p0 + g.e1 * hit.u + g.e2 * hit.v;
    g.ng = normalize(cross(g.e1, g.e2));
    g.em = lds.seg_emitter[g.seg];
    g.cos_emit = -dot(d, g.ng);
    g.wo = v3(-d.x, -d.y, -d.z);
    g.ns = g.ng;
    if (sc.nrm) {
        float b0 = 1.0f - hit.u - hit.v;
        V3 n0 = xyz(sc.nrm[3 * hit.tri]), n1 = xyz(sc.nrm[3 * hit.tri + 1]), n2 = xyz(sc.nrm[3 * hit.tri + 2]);
        g.ns = normalize(n0 * b0 + n1 * hit.u + n2 * hit.v);
    }
    g.ngf = g.ng;
    if (dot(g.ng, g.wo) < 0.0f) { g.ngf = g.ng * -1.0f; g.ns = g.ns * -1.0f; }
}

// ---------------------------------------------------------------------------
// Material models (compile-time): 0 Lambert + GGX, 7 parameters per segment;
// 1 Disney (Sec. 4.1), 13.  The kernels see a material through these
// overloads only.
// ---------------------------------------------------------------------------
template <int MAT> struct MatSel { using M = Mat; static constexpr int NP = 7; };
template <> struct MatSel<1> { using M = DMat; static constexpr int NP = kDisneyParams; };

template <int MAT>
__device__ __forceinline__ typename MatSel<MAT>::M mat_load(const float* p, int seg) {
    if constexpr (MAT == 1) return load_dmat(p, seg);
    else return load_mat(p, seg);
}
// The Disney model's anisotropy needs a tangent frame at the vertex.
template <int MAT>
__device__ __forceinline__ void mat_frame(Shade& g) {
    if constexpr (MAT == 1) disney_frame(g.ns, g.e1, g.tx, g.ty);
}
// f(wo, wi); for Lambert + GGX also the GGX factor and its alpha derivative,
// which the adjoint uses directly (the Disney adjoint differentiates f).
__device__ __forceinline__ V3 mat_f(const Mat& m, const Shade& g, V3 wi, float& spec, float& dspec) {
    spec_term(g.ns, g.wo, wi, m.alpha, spec, dspec);
    return m.kd * kInvPi + m.ks * spec;
}
__device__ __forceinline__ V3 mat_f(const DMat& m, const Shade& g, V3 wi, float& spec, float& dspec) {
    spec = dspec = 0.0f;
    return disney_value(m, disney_geom(g.ns, g.tx, g.ty, g.wo, wi));
}
__device__ __forceinline__ V3 mat_f_only(const Mat& m, const Shade& g, V3 wi) {
    return m.kd * kInvPi + m.ks * spec_only(g.ns, g.wo, wi, m.alpha);
}
__device__ __forceinline__ V3 mat_f_only(const DMat& m, const Shade& g, V3 wi) {
    return disney_value(m, disney_geom(g.ns, g.tx, g.ty, g.wo, wi));
}
__device__ __forceinline__ float mat_pdf(const Mat& m, const Shade& g, V3 wi) { return brdf_pdf(m, g.ns, g.wo, wi); }
__device__ __forceinline__ float mat_pdf(const DMat& m, const Shade& g, V3 wi) {
    return disney_pdf(m, g.ns, g.tx, g.ty, g.wo, wi);
}
__device__ __forceinline__ bool mat_sample(const Mat& m, const Shade& g, float u3, float u4, float u5, V3& wi,
                                           int& lobe) {
    return brdf_sample(m, g.ns, g.wo, u3, u4, u5, wi, lobe);
}
__device__ __forceinline__ bool mat_sample(const DMat& m, const Shade& g, float u3, float u4, float u5, V3& wi,
                                           int& lobe) {
    return disney_sample(m, g.ns, g.tx, g.ty, g.wo, u3, u4, u5, wi, lobe);
}
template <class M> struct MatNP { static constexpr int value = 7; };
template <> struct MatNP<DMat> { static constexpr int value = kDisneyParams; };

// Adjoint of f at one vertex: w . d f / d theta_seg added to the block's
// gradient, for a channel weight w (the Lambert + GGX terms use the factors
// spec, dspec kept from the evaluation; the Disney model its hand-written
// reverse sweep).
__device__ __forceinline__ void mat_grad(double* grad, int mb, const Mat& m, const Shade&, V3, V3 w, float spec,
                                         float dspec) {
    lds_add(grad, mb + 0, w.x * kInvPi);
    lds_add(grad, mb + 1, w.y * kInvPi);
    lds_add(grad, mb + 2, w.z * kInvPi);
    lds_add(grad, mb + 3, w.x * spec);
    lds_add(grad, mb + 4, w.y * spec);
    lds_add(grad, mb + 5, w.z * spec);
    lds_add(grad, mb + 6, dot(w, m.ks) * dspec);
}
__device__ __forceinline__ void mat_grad(double* grad, int mb, const DMat& m, const Shade& g, V3 wi, V3 w, float,
                                         float) {
    float G[kDisneyParams];
    disney_grad(m, disney_geom(g.ns, g.tx, g.ty, g.wo, wi), w, G);
#pragma unroll
    for (int j = 0; j < kDisneyParams; ++j) lds_add(grad, mb + j, G[j]);
}

// MIS weight of an emitter hit at vertex k reached by a direction sampled
// with pdf prev_pdf (balance or power heuristic against light sampling).
__device__ __forceinline__ float emit_weight(const PathArgs& a, const float* cdf, const int4* lights, const Shade& g,
                                             int k, float prev_pdf) {
    if (k == 1) return 1.0f;
    if (a.mis == 1) return 0.0f;
    if (a.mis == 0) return 1.0f;
    float pa = light_prob(cdf, a.sc.nlt, g.light) / __int_as_float(lights[g.light].z);
    float pl = pa * g.t * g.t / g.cos_emit;
    return mis_weight(prev_pdf, pl, a.mis);
}

struct NeeS {
    V3 wl;
    float d2, dist, cy, larea;
    int lj, ltri, lk;
    bool shoot;   // geometric tests passed: a shadow ray is needed
};

// Pick an emitter triangle from the table and a uniform point on it.
__device__ __forceinline__ NeeS nee_setup(const SceneDev& sc, const float* cdf, const int4* lights, const Shade& g,
                                          const float u[8]) {
    NeeS n;
    n.lj = pick_light(cdf, sc.nlt, u[0]);
    int4 lrec = lights[n.lj];
    n.ltri = lrec.x;
    n.lk = lrec.y;
    n.larea = __int_as_float(lrec.z);
    V3 q0, q1, q2;
    int lorig, lseg, llight;
    load_tri(sc, lrec.x, q0, q1, q2, lorig, lseg, llight);
    float su = sqrtf(u[1]);
    float b1 = (1.0f - u[2]) * su, b2 = u[2] * su;
    // y - x from vertex differences and edge terms: the light point and the
    // shading point are never rounded to world coordinates first
    V3 dl = (q0 - g.p0) + ((q1 - q0) * b1 + (q2 - q0) * b2 - (g.e1 * g.u + g.e2 * g.v));
    V3 lng = normalize(cross(q1 - q0, q2 - q0));
    n.d2 = dot(dl, dl);
    n.dist = sqrtf(n.d2);
    n.wl = dl * (1.0f / n.dist);
    n.cy = -dot(n.wl, lng);
    float cxg = dot(n.wl, g.ngf);
    // grazing configurations (cosines below 1e-6: the light triangle itself,
    // a coplanar emitter) are skipped
    n.shoot = n.cy > 1e-6f && cxg > 1e-6f;
    return n;
}

struct NeeC {
    V3 c;            // local contribution (without the prefix throughput)
    V3 e, f;         // emission and BRDF value
    float g;         // cos_x cos_y / d^2 * MIS weight / p_area * profile
    float spec, dspec;
    bool valid;
};

// The light-sample contribution assuming the shadow ray is unoccluded.
// pb >= 0 overrides the BRDF-sampling density of the light direction (the
// combined density when a guide is used).
template <class M>
__device__ __forceinline__ NeeC nee_contrib(const PathArgs& a, const Lds& lds, const float* cdf, const Shade& g,
                                            const M& m, const M& ms, const NeeS& n, float pb_in = -1.0f) {
    NeeC r;
    r.spec = r.dspec = 0.0f;
    float cx = dot(g.ns, n.wl);
    r.valid = cx > 0.0f;
    r.c = v3(0.0f, 0.0f, 0.0f);
    r.e = r.c;
    r.f = r.c;
    r.g = 0.0f;
    if (!r.valid) return r;
    float parea = light_prob(cdf, a.sc.nlt, n.lj) / n.larea;
    float w = 1.0f;
    if (a.mis >= 2) {
        float pl = parea * n.d2 / n.cy;
        float pb = pb_in >= 0.0f ? pb_in : mat_pdf(ms, g, n.wl);
        w = mis_weight(pl, pb, a.mis);
    }
    float prof = a.profile ? n.cy : 1.0f;
    r.g = cx * n.cy / n.d2 * w / parea * prof;
    const float* ep = lds.params + MatNP<M>::value * a.sc.S + 3 * n.lk;
    r.e = v3(ep[0], ep[1], ep[2]);
    r.f = mat_f(m, g, n.wl, r.spec, r.dspec);
    r.c = r.f * r.e * r.g;
    return r;
}

struct ContS {
    V3 wi, av, ts;     // av, ts: continuation weight at params / sampling params (before RR)
    float pdf, g, spec, dspec, qrr;
    int lobe;
    bool ok;           // a direction above the surface with pdf > 0
    bool alive;        // survived Russian roulette
};

// Continuation weight of a sampled direction wi with sampling density pdf:
// validity (above both the geometric and the shading surface, pdf > 0),
// a = f cos / pdf at params, the same at sampling params (for Russian
// roulette), and the roulette decision.
template <class M>
__device__ __forceinline__ ContS cont_eval(const PathArgs& a, const Shade& g, const M& m, const M& ms, V3 wi,
                                           float pdf, int lobe, const float u[8], int k, V3 Ts) {
    ContS c;
    c.wi = wi;
    c.lobe = lobe;
    c.pdf = pdf;
    c.qrr = 1.0f;
    c.alive = false;
    c.av = v3(0.0f, 0.0f, 0.0f);
    c.ts = c.av;
    c.g = c.spec = c.dspec = 0.0f;
    c.ok = pdf > 0.0f && dot(wi, g.ngf) > 0.0f && dot(wi, g.ns) > 0.0f;
    if (!c.ok) return c;
    const V3 f = mat_f(m, g, wi, c.spec, c.dspec);
    float ci = dot(g.ns, wi);
    c.g = ci / pdf;
    c.av = f * c.g;
    c.ts = c.av;
    if (a.frozen) c.ts = mat_f_only(ms, g, wi) * c.g;
    c.alive = true;
    if (a.rr_depth >= 0 && k >= a.rr_depth) {
        c.qrr = fminf(fmaxf(maxc(Ts * c.ts), 0.1f), 0.95f);
        c.alive = u[6] < c.qrr;
    }
    return c;
}

// Sample the continuation direction.  Without a guide (mix == NULL): the
// lobe mixture at sampling parameters.  With a guide: the technique is the
// guide with probability gmix (u[7]), the BRDF otherwise, and the density is
// the combined gmix q + (1 - gmix) p_brdf (one-sample MIS).
// Density and sample of the proposal: the mixture of the network's outputs
// (per-vertex kinds) or a cached row (kind 3).
template <int GUIDE>
__device__ __forceinline__ float guide_pdf(const float* mix, V3 w) {
    if (GUIDE == 3) return cached_pdf(mix, w);
    return mixture_pdf(mix, w);
}
template <int GUIDE>
__device__ __forceinline__ V3 guide_sample(const float* mix, float u3, float u4, float u5) {
    if (GUIDE == 3) return cached_sample(mix, u3, u4, u5);
    return mixture_sample(mix, u3, u4, u5);
}

template <int GUIDE, class M>
__device__ __forceinline__ ContS cont_sample(const PathArgs& a, const Shade& g, const M& m, const M& ms,
                                             const float u[8], int k, V3 Ts, const float* mix, bool& used_guide) {
    V3 wi = v3(0.0f, 0.0f, 1.0f);
    int lobe = 0;
    used_guide = false;
    float pdf = 0.0f;
    if (GUIDE && mix && u[7] < a.gmix) {
        used_guide = true;
        wi = guide_sample<GUIDE>(mix, u[3], u[4], u[5]);
        pdf = a.gmix * guide_pdf<GUIDE>(mix, wi) + (1.0f - a.gmix) * mat_pdf(ms, g, wi);
    } else {
        bool okd = mat_sample(ms, g, u[3], u[4], u[5], wi, lobe);
        if (okd && dot(wi, g.ngf) > 0.0f && dot(wi, g.ns) > 0.0f) {
            pdf = mat_pdf(ms, g, wi);
            if (GUIDE && mix) pdf = a.gmix * guide_pdf<GUIDE>(mix, wi) + (1.0f - a.gmix) * pdf;
        }
    }
    return cont_eval(a, g, m, ms, wi, pdf, lobe, u, k, Ts);
}

// The cached proposal's one-sample MIS in two steps, so that both densities a
// vertex needs (continuation direction, light sample) come from one pass over
// its row: first the technique (u[7]) and the direction (u[3..5]) ...
struct ContDir {
    V3 wi;
    int lobe;
    bool ok;      // BRDF technique: a direction above the surface
    bool guide;   // the proposal's technique was chosen
};
template <class M>
__device__ __forceinline__ ContDir cont_direction_cached(const PathArgs& a, const Shade& g, const M& ms,
                                                         const float u[8], const float* row) {
    ContDir c;
    c.lobe = 0;
    c.guide = u[7] < a.gmix;
    if (c.guide) {
        c.wi = cached_sample(row, u[3], u[4], u[5]);
        c.ok = true;
    } else {
        c.wi = v3(0.0f, 0.0f, 1.0f);
        c.ok = mat_sample(ms, g, u[3], u[4], u[5], c.wi, c.lobe) && dot(c.wi, g.ngf) > 0.0f &&
               dot(c.wi, g.ns) > 0.0f;
    }
    return c;
}
// ... then, with the proposal's density q of that direction, the combined
// density and the continuation weight (as cont_sample).
template <class M>
__device__ __forceinline__ ContS cont_finish_cached(const PathArgs& a, const Shade& g, const M& m, const M& ms,
                                                    const float u[8], int k, V3 Ts, const ContDir& c, float q) {
    float pdf = 0.0f;
    if (c.guide || c.ok) pdf = a.gmix * q + (1.0f - a.gmix) * mat_pdf(ms, g, c.wi);
    return cont_eval(a, g, m, ms, c.wi, pdf, c.lobe, u, k, Ts);
}

// Streaming store of one 16 B checkpoint record: the records are read again
// only by a later kernel, so they should not displace the scene's nodes and
// triangles in the caches.
__device__ __forceinline__ void st_stream(float4* p, float4 v) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<f4*>(p));
}
__device__ __forceinline__ void st_stream(int4* p, int4 v) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    const i4 x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<i4*>(p));
}

// Backward sweep of the gradient forward pass: R_{k+1} into the c slot of
// vertex k; returns the path radiance.
__device__ __forceinline__ V3 suffix_sweep(const PathArgs& a, int klast, int s, int64_t q) {
    const size_t plane = (size_t)a.pix_count;
    V3 R = v3(0.0f, 0.0f, 0.0f);
    for (int k = klast; k >= 1; --k) {
        size_t ck = ((size_t)(k - 1) * a.spp + s) * plane + q;
        float4 c = a.ck_c[ck], av = a.ck_a[ck];
        a.ck_c[ck] = make_float4(R.x, R.y, R.z, 0.0f);
        R = v3(c.x, c.y, c.z) + v3(av.x, av.y, av.z) * R;
    }
    return R;
}

__device__ __forceinline__ void flush_stats(const PathArgs& a, int mode, const Work& wk, uint32_t npaths) {
    if (!a.count_stats) return;
    KStats* ks = &a.err->k[mode];
    atomicAdd(&ks->rays, (unsigned long long)wk.rays);
    atomicAdd(&ks->nodes, (unsigned long long)wk.nodes);
    atomicAdd(&ks->tris, (unsigned long long)wk.tris);
    atomicAdd(&ks->paths, (unsigned long long)npaths);
    atomicAdd(&ks->vertices, (unsigned long long)wk.vertices);
    atomicAdd(&ks->units, (unsigned long long)wk.units);
}

// ---------------------------------------------------------------------------
// Colour / gradient-forward kernel: per-lane state machine.
// ---------------------------------------------------------------------------
enum Phase { kNeedPixel = 0, kClosest = 1, kShadow = 2, kExit = 3 };

// At least 4 waves per SIMD: the path state needs ~158 VGPRs unconstrained
// (3 waves), and the fourth wave hides more node-fetch latency than the
// ~100 bytes of spilled state cost (apartment step 241 -> 214 ms).
#ifndef IPT_WAVES_PER_EU
#define IPT_WAVES_PER_EU 4
#endif
#define IPT_OCC __attribute__((amdgpu_waves_per_eu(IPT_WAVES_PER_EU, 8)))
// The guided kernels also hold the network's operands around the MLP call:
// at 2 waves per SIMD nothing spills (apartment guided step 537 ms at 4
// waves, 487 at 3, 449 at 2).
#ifndef IPT_WAVES_PER_EU_GUIDED
#define IPT_WAVES_PER_EU_GUIDED 2
#endif
// The Disney kernels hold two 13-float materials (rendering and sampling
// parameters) at each vertex: 3 waves per SIMD spill less (apartment with
// the Disney material: step 183.0 ms at 3 waves, 187.0 at 4, 215.2 at 2).
#ifndef IPT_WAVES_PER_EU_DISNEY
#define IPT_WAVES_PER_EU_DISNEY 3
#endif

// A traversal call returns once no more than this many lanes of the wave
// are still traversing (0: every traversal runs to completion in one call).
// Apartment step: 203 ms at 0, 188 / 187 / 190 / 195 ms at 8 / 16 / 24 / 32.
#ifndef IPT_TRAV_EXIT_LANES
#define IPT_TRAV_EXIT_LANES 16
#endif
// GUIDE: 0 none, 1 bfloat16 MFMA evaluation, 2 float32 VALU evaluation, 3 cached
// proposal; MAT: the material model (MatSel)
template <int MODE, int GUIDE, int PG, int MAT>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((GUIDE == 1 || GUIDE == 2) ? IPT_WAVES_PER_EU_GUIDED
                                   : (MAT == 1 ? IPT_WAVES_PER_EU_DISNEY : IPT_WAVES_PER_EU),
                                   8))) void path_sm_kernel(
    PathArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    Lds lds;
    carve_lds<PG>(a, MODE, smem, lds);
    Stack st;
    init_stack(st, a, lds.stack);
    const SceneDev& sc = a.sc;
    const float* cdf = lds.lights_in_lds ? lds.cdf : a.cdf;
    const int4* lights = lds.lights_in_lds ? lds.lights : sc.lights;
    const int lane = threadIdx.x & 63;
    const int64_t npix_img = (int64_t)a.V * a.W * a.H;
    const size_t plane = (size_t)a.pix_count;
    const int D = a.D;
    Work wk{0u, 0u, 0u, 0u, 0u};
    uint32_t npaths = 0;

    int ph = kNeedPixel;
    Trav tv;                 // traversal in progress (tracing) across iterations
    bool tracing = false;
    // work-unit state
    int64_t q = 0, wi = 0, pix = 0, unit = 0;
    int view = 0, px = 0, py = 0, s = 0, s_end = 0;
    const int64_t nunits = a.pix_count * a.nchunk;
    V3 acc = v3(0.0f, 0.0f, 0.0f);
    // path state: k = index of the vertex last processed
    uint64_t pid = 0, h = 0;
    int k = 0, klast = 0, prev_tri = -1;
    V3 T = acc, Ts = acc, L = acc, o = acc, d = acc;
    float prev_pdf = 0.0f;
    // vertex pending on a shadow ray
    V3 wl = acc, nee_LT = acc, nee_c = acc, cpart = acc;
    float sdist = 0.0f;
    int sltri = -1;
    uint32_t ev = 0, evtail = 0, ckx = 0;
    bool nee_valid = false;
    float* dvk = nullptr;

    auto start_path = [&]() {
        pid = (uint64_t)pix * (uint64_t)a.spp + (uint64_t)s;
        float j0 = 0.5f, j1 = 0.5f;
        if (a.jitter) jitter_uniforms(a.rng, pid, j0, j1);
        camera_ray(a, view, (float)px + j0, (float)py + j1, o, d);
        k = 0;
        klast = 0;
        prev_tri = -1;
        prev_pdf = 0.0f;
        T = v3(1.0f, 1.0f, 1.0f);
        Ts = T;
        L = v3(0.0f, 0.0f, 0.0f);
        h = 0xCBF29CE484222325ull;
        if (MODE == kColor && a.dbg_vtx) {
            float* dv = a.dbg_vtx + ((size_t)wi * a.spp + s) * 8 * (size_t)(D + 1);
            for (int i = 0; i < 8 * (D + 1); ++i) dv[i] = -1.0f;
        }
        ph = kClosest;
    };

    while (true) {
        // ---- lanes without a pixel take the next pixels (one atomic per wave) ----
        uint64_t need = __ballot(ph == kNeedPixel);
        if (need) {
            int first = __ffsll((unsigned long long)need) - 1;
            unsigned base = 0;
            if (lane == first) base = atomicAdd(a.work, (unsigned)__popcll(need));
            base = __shfl(base, first);
            if (ph == kNeedPixel) {
                unsigned rank = (unsigned)__popcll(need & ((1ull << lane) - 1ull));
                unit = (int64_t)base + rank;
                if (unit >= nunits) {
                    ph = kExit;
                } else {
                    wk.units++;
                    const int c = (int)(unit / a.pix_count);
                    q = unit - (int64_t)c * a.pix_count;
                    s = c * a.spc;
                    s_end = min(a.spp, s + a.spc);
                    wi = a.pix_begin + q;
                    pix = a.pixel_list ? a.pixel_list[wi] : wi;
                    if (pix < 0 || pix >= npix_img) {
                        if (MODE == kColor) {
                            float* out = a.nchunk > 1 ? a.part + 3 * (size_t)unit : a.image + 3 * wi;
                            out[0] = 0.0f;
                            out[1] = 0.0f;
                            out[2] = 0.0f;
                        }
                    } else {
                        view = (int)(pix / ((int64_t)a.W * a.H));
                        int64_t rem = pix - (int64_t)view * a.W * a.H;
                        py = (int)(rem / a.W);
                        px = (int)(rem - (int64_t)py * a.W);
                        acc = v3(0.0f, 0.0f, 0.0f);
                        start_path();
                    }
                }
            }
        }
        if (__ballot(ph != kExit) == 0) break;

        bool end_path = false;
        bool shade = false;      // vertex k still needs light sampling and a continuation
        Shade g;
        Hit hr;
        hr.tri = -1;
        hr.t = hr.u = hr.v = 0.0f;
        size_t ck = 0;
        if (ph == kClosest || ph == kShadow) {
            // ---- one traversal call site for closest-hit and shadow rays ----
            // a lane whose traversal returned unfinished resumes it here and
            // skips the rest of the iteration until it is done
            const bool any = ph == kShadow;
            const float tmax = any ? sdist * (1.0f - 1e-5f) : __builtin_inff();
            Ray ray = make_ray(o, any ? wl : d);
            if (!tracing) {
                trav_init(tv, tmax, st, wk);
                tracing = true;
            }
            const bool done = traverse_resume(sc, ray, sc.tmin, tmax, prev_tri, any ? sltri : -1, any, st, wk, tv,
                                              IPT_TRAV_EXIT_LANES);
            if (done) tracing = false;
            hr = tv.best;
            if (!done) {
                // still traversing
            } else if (any) {
                // ---- finish the vertex that waited for its shadow ray ----
                bool vis = hr.tri < 0;
                ev |= (uint32_t)vis << 2;
                if (vis && nee_valid) {
                    cpart = cpart + nee_c;
                    L = L + nee_LT;
                    if (dvk) { dvk[4] = L.x; dvk[5] = L.y; dvk[6] = L.z; dvk[7] = 1.0f; }
                }
                h = fnv1a(h, ev | evtail);
                if (MODE == kGradFwd) {
                    ck = ((size_t)(k - 1) * a.spp + s) * plane + q;
                    if (vis) a.ck_hit[ck].x = (int)(ckx | kCkVis);
                    st_stream(&a.ck_c[ck], make_float4(cpart.x, cpart.y, cpart.z, 0.0f));
                }
                end_path = evtail != 0;
                ph = kClosest;
            } else {
                // ---- closest hit: vertex k ----
                ++k;
                klast = k;
                wk.vertices++;
                ck = ((size_t)(k - 1) * a.spp + s) * plane + q;
                if (hr.tri < 0) {
                    h = fnv1a(h, 0xFFFFFFFFu);
                    if (MODE == kGradFwd) st_stream(&a.ck_hit[ck], make_int4(0, 0, 0, 0));
                    klast = k - 1;   // a miss contributes nothing: the sweep starts below it
                    end_path = true;
                } else {
                    make_shade(sc, lds, hr, d, g);
                    h = fnv1a(h, (uint32_t)g.orig);
                    dvk = nullptr;
                    if (MODE == kColor && a.dbg_vtx) {
                        dvk = a.dbg_vtx + (((size_t)wi * a.spp + s) * (size_t)(D + 1) + (k - 1)) * 8;
                        dvk[0] = (float)g.orig; dvk[1] = hr.u; dvk[2] = hr.v; dvk[3] = hr.t;
                        dvk[4] = L.x; dvk[5] = L.y; dvk[6] = L.z; dvk[7] = 0.0f;
                    }
                    ev = 0;
                    evtail = 0;
                    cpart = v3(0.0f, 0.0f, 0.0f);
                    if (g.em >= 0 && g.cos_emit > 0.0f) {
                        float w = emit_weight(a, cdf, lights, g, k, prev_pdf);
                        if (w > 0.0f) {
                            float prof = a.profile ? g.cos_emit : 1.0f;
                            const float* e = lds.params + MatSel<MAT>::NP * sc.S + 3 * g.em;
                            V3 c = v3(e[0], e[1], e[2]) * (prof * w);
                            cpart = c;
                            L = L + T * c;
                            if (dvk) { dvk[4] = L.x; dvk[5] = L.y; dvk[6] = L.z; }
                        }
                        ev |= 1u;
                    }
                    if (k == D + 1 || dot(g.ns, g.wo) <= 0.0f) {
                        // x_{D+1} only counts its emission; a shading normal facing
                        // away ends the path
                        if (k != D + 1) ev |= 2u;
                        end_path = true;
                        h = fnv1a(h, ev);
                        prev_tri = g.tri;
                        if (MODE == kGradFwd) {
                            st_stream(&a.ck_hit[ck], make_int4(g.tri + 1, __float_as_int(hr.u),
                                                               __float_as_int(hr.v), __float_as_int(hr.t)));
                            st_stream(&a.ck_a[ck], make_float4(0.0f, 0.0f, 0.0f, 0.0f));
                            st_stream(&a.ck_c[ck], make_float4(cpart.x, cpart.y, cpart.z, 0.0f));
                        }
                    } else {
                        shade = true;
                    }
                }
            }
        }

        // ---- guide evaluation for the lanes about to sample (all lanes active here) ----
        const float* mix = nullptr;
        if (GUIDE == 3) {
            // cached row of the hit's cell, on the side the path arrives from
            if (shade) mix = cache_row_at(a.gd, g.tri, g.u, g.v, dot(g.ng, g.wo) < 0.0f);
        } else if (GUIDE) {
            float* row = (float*)(lds.gact + lane * kGRowStride);
            if (GUIDE == 1) {
                if (shade) {
                    float f[9];
                    guide_features(a.gd, g.x, g.ns, g.wo, f);
                    guide_put_inputs(a.gd, lds.gact, f, g.seg);
                }
                if (__ballot(shade)) guide_mlp_wave(a.gd, lds.gact);
            } else if (shade) {
                float f[9];
                guide_features(a.gd, g.x, g.ns, g.wo, f);
                guide_mlp_fp32(a.gd, f, g.seg, row);
            }
            if (shade) {
                mixture_from_raw(row);
                mix = row;
            }
        }

        if (shade) {
            // ---- light sample and continuation of vertex k ----
            uint32_t flags = 0;
            bool shoot = false;
            V3 av = v3(0.0f, 0.0f, 0.0f);
            mat_frame<MAT>(g);
            const typename MatSel<MAT>::M m = mat_load<MAT>(lds.params, g.seg);
            const typename MatSel<MAT>::M ms = a.frozen ? mat_load<MAT>(lds.sparams, g.seg) : m;
            float u[8];
            vertex_uniforms(a.rng, pid, k, u);
            float pb_nee = -1.0f;
            // light sample accepted: its contribution waits for the shadow ray
            auto take_nee = [&](const NeeS& n) {
                NeeC nc = nee_contrib(a, lds, cdf, g, m, ms, n, pb_nee);
                shoot = true;
                nee_valid = nc.valid;
                nee_c = nc.c;
                nee_LT = T * nc.c;
                wl = n.wl;
                sdist = n.dist;
                sltri = n.ltri;
            };
            bool used_guide = false;
            ContS cs;
            if constexpr (GUIDE == 3) {
                // cached proposal: direction first, then both densities in one pass over the row
                NeeS n;
                n.shoot = false;
                n.lj = 0;
                const bool do_nee = a.mis != 0 && sc.nlt > 0;
                if (do_nee) {
                    n = nee_setup(sc, cdf, lights, g, u);
                    ev |= (uint32_t)n.lj << 8;
                }
                const ContDir cd = cont_direction_cached(a, g, ms, u, mix);
                float q_wi, q_wl;
                cached_pdf2(mix, cd.wi, n.shoot ? n.wl : cd.wi, q_wi, q_wl);
                if (n.shoot) {
                    pb_nee = a.gmix * q_wl + (1.0f - a.gmix) * mat_pdf(ms, g, n.wl);
                    take_nee(n);
                }
                cs = cont_finish_cached(a, g, m, ms, u, k, Ts, cd, q_wi);
                used_guide = cd.guide;
            } else {
                if (a.mis != 0 && sc.nlt > 0) {
                    NeeS n = nee_setup(sc, cdf, lights, g, u);
                    ev |= (uint32_t)n.lj << 8;
                    if (n.shoot) {
                        if (GUIDE && mix)
                            pb_nee = a.gmix * guide_pdf<GUIDE>(mix, n.wl) + (1.0f - a.gmix) * mat_pdf(ms, g, n.wl);
                        take_nee(n);
                    }
                }
                cs = cont_sample<GUIDE>(a, g, m, ms, u, k, Ts, mix, used_guide);
            }
            // lobe 1 at bit 3, lobe 2 (the Disney clearcoat) at bit 7
            ev |= (uint32_t)(cs.lobe & 1) << 3 | (uint32_t)(cs.lobe >> 1) << 7;
            if (used_guide) ev |= 64u;
            if (!cs.ok) {
                evtail = 16u;
            } else if (!cs.alive) {
                evtail = 32u;
            } else {
                float rq = 1.0f / cs.qrr;
                av = cs.av * rq;
                Ts = Ts * cs.ts * rq;
                flags |= kCkCont;
                prev_pdf = cs.pdf;
                T = T * av;
                d = cs.wi;
            }
            prev_tri = g.tri;
            o = g.x;
            if (MODE == kGradFwd) {
                ckx = (uint32_t)(g.tri + 1) | flags;
                st_stream(&a.ck_hit[ck], make_int4((int)ckx, __float_as_int(hr.u), __float_as_int(hr.v),
                                                   __float_as_int(hr.t)));
                st_stream(&a.ck_a[ck], make_float4(av.x, av.y, av.z, cs.pdf));
                if (a.guided) st_stream(&a.ck_d[ck], make_float4(cs.wi.x, cs.wi.y, cs.wi.z, pb_nee));
            }
            if (shoot) {
                ph = kShadow;   // the vertex finishes after its shadow ray
            } else {
                h = fnv1a(h, ev | evtail);
                if (MODE == kGradFwd) st_stream(&a.ck_c[ck], make_float4(cpart.x, cpart.y, cpart.z, 0.0f));
                end_path = evtail != 0;
            }
        }

        if (end_path) {
            ++npaths;
            size_t pidx = (size_t)wi * a.spp + s;
            bool use = a.mask ? a.mask[pidx] != 0 : true;
            if (MODE == kGradFwd) {
                const size_t c1 = (size_t)s * plane + q;
                if (a.guided) {
                    // the training records read R_{k+1} before the replay runs
                    V3 R = suffix_sweep(a, klast, s, q);
                    if (!finite3(R) || !finite3(L)) {
                        a.ck_hit[c1].x = (int)((uint32_t)a.ck_hit[c1].x | kCkDrop);
                        atomicAdd(&a.err->nonfinite, 1ull);
                    }
                } else if (!finite3(L)) {
                    a.ck_hit[c1].x = (int)((uint32_t)a.ck_hit[c1].x | kCkDrop);
                    atomicAdd(&a.err->nonfinite, 1ull);
                } else {
                    // the replay runs the sweep: the index of the path's last
                    // vertex goes into the unused fourth slot of vertex 1's c
                    a.ck_c[c1].w = __int_as_float(klast);
                }
            } else {
                if (!finite3(L)) atomicAdd(&a.err->nonfinite, 1ull);
                else if (use) acc = acc + L;
                if (a.path_L) {
                    a.path_L[3 * pidx] = L.x;
                    a.path_L[3 * pidx + 1] = L.y;
                    a.path_L[3 * pidx + 2] = L.z;
                }
            }
            if (a.hash) a.hash[pidx] = h;
            ++s;
            if (s < s_end) {
                start_path();
            } else {
                if (MODE == kColor) {
                    if (a.nchunk > 1) {   // sample sum of this unit; the reduce pass forms the mean
                        float* out = a.part + 3 * (size_t)unit;
                        out[0] = acc.x;
                        out[1] = acc.y;
                        out[2] = acc.z;
                    } else {
                        float inv = 1.0f / (float)a.spp;
                        a.image[3 * wi] = acc.x * inv;
                        a.image[3 * wi + 1] = acc.y * inv;
                        a.image[3 * wi + 2] = acc.z * inv;
                    }
                }
                ph = kNeedPixel;
            }
        }
    }
    if (st.overflow) atomicAdd(&a.err->overflow, 1ull);
    flush_stats(a, MODE, wk, npaths);
}

// ---------------------------------------------------------------------------
// Adjoint replay.  replay_kernel (one lane per pixel, tiles pulled by blocks)
// serves the check mode that re-traces paths; replay_sm_kernel below reads
// the vertex checkpoints.
// ---------------------------------------------------------------------------
template <int MAT>
__device__ void replay_path(const PathArgs& a, const Lds& lds, Stack& st, Work& wk, uint64_t pid, int64_t q, int s,
                            V3 org, V3 dir, V3 wpix) {
    const SceneDev& sc = a.sc;
    const float* cdf = lds.lights_in_lds ? lds.cdf : a.cdf;
    const int4* lights = lds.lights_in_lds ? lds.lights : sc.lights;
    const size_t plane = (size_t)a.pix_count;
    if ((uint32_t)a.ck_hit[(size_t)s * plane + q].x & kCkDrop) return;
    if (!a.guided) {
        // the backward sweep, here rather than at the end of each path in the
        // forward pass: every lane of the wave starts a path at once, so the
        // sweeps' round trips to memory overlap instead of holding up a wave
        // in which a few lanes end their paths
        const int klast = min(max(__float_as_int(a.ck_c[(size_t)s * plane + q].w), 0), a.D + 1);
        const V3 R = suffix_sweep(a, klast, s, q);
        if (!finite3(R)) {
            atomicAdd(&a.err->nonfinite, 1ull);
            return;
        }
    }
    V3 T = v3(1.0f, 1.0f, 1.0f), Ts = T;
    float prev_pdf = 0.0f;
    int prev_tri = -1;
    V3 o = org, d = dir;
    for (int k = 1; k <= a.D + 1; ++k) {
        size_t ck = ((size_t)(k - 1) * a.spp + s) * plane + q;
        int4 rec = a.ck_hit[ck];
        uint32_t flags = (uint32_t)rec.x;
        Hit hit;
        if (!a.replay_traverse) {
            hit.tri = (int)(flags & kCkTriMask) - 1;
            hit.u = __int_as_float(rec.y);
            hit.v = __int_as_float(rec.z);
            hit.t = __int_as_float(rec.w);
        } else {
            Ray ray = make_ray(o, d);
            hit = traverse(sc, ray, sc.tmin, __builtin_inff(), prev_tri, -1, false, st, wk);
        }
        if (hit.tri < 0) return;
        wk.vertices++;
        float4 rr = a.ck_c[ck];
        V3 Rn = v3(rr.x, rr.y, rr.z);   // R_{k+1}
        Shade g;
        make_shade(sc, lds, hit, d, g);
        V3 wT = wpix * T;
        // emission at this vertex: d/de = w_hit * profile
        if (g.em >= 0 && g.cos_emit > 0.0f) {
            float w = emit_weight(a, cdf, lights, g, k, prev_pdf);
            if (w > 0.0f) {
                float prof = a.profile ? g.cos_emit : 1.0f;
                int eb = MatSel<MAT>::NP * sc.S + 3 * g.em;
                lds_add(lds.grad, eb + 0, wT.x * prof * w);
                lds_add(lds.grad, eb + 1, wT.y * prof * w);
                lds_add(lds.grad, eb + 2, wT.z * prof * w);
            }
        }
        if (k == a.D + 1 || dot(g.ns, g.wo) <= 0.0f) return;
        mat_frame<MAT>(g);
        const typename MatSel<MAT>::M m = mat_load<MAT>(lds.params, g.seg);
        const typename MatSel<MAT>::M ms = a.frozen ? mat_load<MAT>(lds.sparams, g.seg) : m;
        float u[8];
        vertex_uniforms(a.rng, pid, k, u);
        float4 dk = a.guided ? a.ck_d[ck] : make_float4(0.0f, 0.0f, 0.0f, -1.0f);
        if (a.mis != 0 && sc.nlt > 0) {
            NeeS n = nee_setup(sc, cdf, lights, g, u);
            bool vis = false;
            if (n.shoot) {
                if (!a.replay_traverse) {
                    vis = (flags & kCkVis) != 0;
                } else {
                    Ray sr = make_ray(g.x, n.wl);
                    vis = traverse(sc, sr, sc.tmin, n.dist * (1.0f - 1e-5f), g.tri, n.ltri, true, st, wk).tri < 0;
                }
            }
            if (vis) {
                // with a guide the forward pass stored the combined density of wl
                NeeC nc = nee_contrib(a, lds, cdf, g, m, ms, n, dk.w);
                if (nc.valid) {
                    constexpr int NP = MatSel<MAT>::NP;
                    int mb = NP * g.seg, eb = NP * sc.S + 3 * n.lk;
                    V3 we = wT * nc.e * nc.g;
                    mat_grad(lds.grad, mb, m, g, n.wl, we, nc.spec, nc.dspec);
                    V3 wf = wT * nc.f * nc.g;
                    lds_add(lds.grad, eb + 0, wf.x);
                    lds_add(lds.grad, eb + 1, wf.y);
                    lds_add(lds.grad, eb + 2, wf.z);
                }
            }
        }
        if (!(flags & kCkCont)) return;
        ContS cs;
        if (a.guided) {
            // the sampled direction and its density come from the checkpoint
            cs = cont_eval(a, g, m, ms, v3(dk.x, dk.y, dk.z), a.ck_a[ck].w, 0, u, k, Ts);
        } else {
            bool ug;
            cs = cont_sample<0>(a, g, m, ms, u, k, Ts, nullptr, ug);
        }
        float rq = 1.0f / cs.qrr;
        V3 wr = wT * Rn * (cs.g * rq);
        mat_grad(lds.grad, MatSel<MAT>::NP * g.seg, m, g, cs.wi, wr, cs.spec, cs.dspec);
        T = T * (cs.av * rq);
        Ts = Ts * cs.ts * rq;
        prev_pdf = cs.pdf;
        prev_tri = g.tri;
        o = g.x;
        d = cs.wi;
    }
}

template <int PG, int MAT>
__global__ __launch_bounds__(kBlock) void replay_kernel(PathArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned tile_sh;
    const int tid = threadIdx.x;
    Lds lds;
    carve_lds<PG>(a, kReplay, smem, lds);
    Stack st;
    init_stack(st, a, lds.stack);
    const int64_t npix_img = (int64_t)a.V * a.W * a.H;
    Work wk{0u, 0u, 0u, 0u, 0u};
    uint32_t npaths = 0;
    const int64_t nunits = a.pix_count * a.nchunk;
    while (true) {
        if (tid == 0) tile_sh = atomicAdd(a.work, 1u);
        __syncthreads();
        // every thread reads the tile before the second barrier: after it,
        // thread 0 may already be writing the next tile into tile_sh
        const int64_t tile0 = (int64_t)tile_sh * kBlock;
        __syncthreads();
        if (tile0 >= nunits) break;
        const int64_t unit = tile0 + tid;
        if (unit >= nunits) continue;
        wk.units++;
        const int c = (int)(unit / a.pix_count);
        const int64_t q = unit - (int64_t)c * a.pix_count;
        const int s_begin = c * a.spc, s_end = min(a.spp, s_begin + a.spc);
        int64_t wi = a.pix_begin + q;
        int64_t pix = a.pixel_list ? a.pixel_list[wi] : wi;
        if (pix < 0 || pix >= npix_img) continue;
        int view = (int)(pix / ((int64_t)a.W * a.H));
        int64_t rem = pix - (int64_t)view * a.W * a.H;
        int py = (int)(rem / a.W), px = (int)(rem - (int64_t)py * a.W);
        float inv = 1.0f / (float)a.spp;
        V3 wpix = v3(a.w[3 * wi] * inv, a.w[3 * wi + 1] * inv, a.w[3 * wi + 2] * inv);
        for (int s = s_begin; s < s_end; ++s) {
            uint64_t pid = (uint64_t)pix * (uint64_t)a.spp + (uint64_t)s;
            size_t pidx = (size_t)wi * a.spp + s;
            if (a.mask && a.mask[pidx] == 0) continue;
            float j0 = 0.5f, j1 = 0.5f;
            if (a.jitter) jitter_uniforms(a.rng, pid, j0, j1);
            V3 o, d;
            camera_ray(a, view, (float)px + j0, (float)py + j1, o, d);
            replay_path<MAT>(a, lds, st, wk, pid, q, s, o, d, wpix);
            ++npaths;
        }
    }
    if (st.overflow) atomicAdd(&a.err->overflow, 1ull);
    flush_stats(a, kReplay, wk, npaths);
    if constexpr (PG) return;   // the atomics went straight to the accumulator copies
    __syncthreads();
    double* out = a.grad_part + (size_t)blockIdx.x * a.P;
    for (int i = tid; i < a.P; i += kBlock) out[i] = lds.grad[i];
}

// Adjoint replay from vertex checkpoints as a per-lane state machine (the
// Disney material's replay): each pass of the loop replays one vertex of
// every lane's current path, and a lane whose path has ended takes the next
// one (the next sample of its unit, else a new unit, one atomic per wave)
// instead of idling until the longest path of the wave is done.  Same
// arithmetic, in the same order per path, as replay_path.
template <int PG, int MAT>
__global__ __launch_bounds__(kBlock) void replay_sm_kernel(PathArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    Lds lds;
    carve_lds<PG>(a, kReplay, smem, lds);
    const SceneDev& sc = a.sc;
    const float* cdf = lds.lights_in_lds ? lds.cdf : a.cdf;
    const int4* lights = lds.lights_in_lds ? lds.lights : sc.lights;
    const int64_t npix_img = (int64_t)a.V * a.W * a.H;
    const int64_t nunits = a.pix_count * a.nchunk;
    const size_t plane = (size_t)a.pix_count;
    const float inv_spp = 1.0f / (float)a.spp;
    Work wk{0u, 0u, 0u, 0u, 0u};
    uint32_t npaths = 0;
    // unit of work: samples [s, s_end) of work pixel q
    bool have_unit = false, exhausted = false;
    int64_t q = 0, wi = 0, pix = 0;
    int view = 0, px = 0, py = 0, s = 0, s_end = 0;
    V3 wpix = v3(0.0f, 0.0f, 0.0f);
    // path being replayed
    bool in_path = false;
    uint64_t pid = 0;
    int k = 0;
    V3 T = wpix, Ts = wpix, d = wpix;
    float prev_pdf = 0.0f;

    while (true) {
        // ---- lanes without a path: next sample of the unit, else a new unit ----
        while (true) {
            if (!in_path && have_unit) {
                while (s < s_end && !in_path) {
                    pid = (uint64_t)pix * (uint64_t)a.spp + (uint64_t)s;
                    const size_t pidx = (size_t)wi * a.spp + s;
                    if (a.mask && a.mask[pidx] == 0) { ++s; continue; }
                    ++npaths;
                    if ((uint32_t)a.ck_hit[(size_t)s * plane + q].x & kCkDrop) { ++s; continue; }
                    if (!a.guided) {
                        const int klast = min(max(__float_as_int(a.ck_c[(size_t)s * plane + q].w), 0), a.D + 1);
                        const V3 R = suffix_sweep(a, klast, s, q);
                        if (!finite3(R)) {
                            atomicAdd(&a.err->nonfinite, 1ull);
                            ++s;
                            continue;
                        }
                    }
                    float j0 = 0.5f, j1 = 0.5f;
                    if (a.jitter) jitter_uniforms(a.rng, pid, j0, j1);
                    V3 o;
                    camera_ray(a, view, (float)px + j0, (float)py + j1, o, d);
                    T = v3(1.0f, 1.0f, 1.0f);
                    Ts = T;
                    prev_pdf = 0.0f;
                    k = 1;
                    in_path = true;
                }
                if (!in_path) have_unit = false;
            }
            const uint64_t need = __ballot(!in_path && !have_unit && !exhausted);
            if (!need) break;
            const int first = __ffsll((unsigned long long)need) - 1;
            unsigned base = 0;
            if (lane == first) base = atomicAdd(a.work, (unsigned)__popcll(need));
            base = __shfl(base, first);
            if (!in_path && !have_unit && !exhausted) {
                const int64_t unit = (int64_t)base + (int64_t)__popcll(need & ((1ull << lane) - 1ull));
                if (unit >= nunits) {
                    exhausted = true;
                } else {
                    wk.units++;
                    const int c = (int)(unit / a.pix_count);
                    q = unit - (int64_t)c * a.pix_count;
                    s = c * a.spc;
                    s_end = min(a.spp, s + a.spc);
                    wi = a.pix_begin + q;
                    pix = a.pixel_list ? a.pixel_list[wi] : wi;
                    if (pix >= 0 && pix < npix_img) {
                        view = (int)(pix / ((int64_t)a.W * a.H));
                        const int64_t rem = pix - (int64_t)view * a.W * a.H;
                        py = (int)(rem / a.W);
                        px = (int)(rem - (int64_t)py * a.W);
                        wpix = v3(a.w[3 * wi] * inv_spp, a.w[3 * wi + 1] * inv_spp, a.w[3 * wi + 2] * inv_spp);
                        have_unit = true;
                    }
                }
            }
        }
        if (__ballot(in_path) == 0) break;   // every lane is exhausted
        if (!in_path) continue;

        // ---- vertex k of the lane's path ----
        bool done = true;
        const size_t ck = ((size_t)(k - 1) * a.spp + s) * plane + q;
        const int4 rec = a.ck_hit[ck];
        const uint32_t flags = (uint32_t)rec.x;
        Hit hit;
        hit.tri = (int)(flags & kCkTriMask) - 1;
        hit.u = __int_as_float(rec.y);
        hit.v = __int_as_float(rec.z);
        hit.t = __int_as_float(rec.w);
        if (hit.tri >= 0) {
            wk.vertices++;
            const float4 rr = a.ck_c[ck];
            const V3 Rn = v3(rr.x, rr.y, rr.z);   // R_{k+1}
            Shade g;
            make_shade(sc, lds, hit, d, g);
            const V3 wT = wpix * T;
            // emission at this vertex: d/de = w_hit * profile
            if (g.em >= 0 && g.cos_emit > 0.0f) {
                const float w = emit_weight(a, cdf, lights, g, k, prev_pdf);
                if (w > 0.0f) {
                    const float prof = a.profile ? g.cos_emit : 1.0f;
                    const int eb = MatSel<MAT>::NP * sc.S + 3 * g.em;
                    lds_add(lds.grad, eb + 0, wT.x * prof * w);
                    lds_add(lds.grad, eb + 1, wT.y * prof * w);
                    lds_add(lds.grad, eb + 2, wT.z * prof * w);
                }
            }
            if (k != a.D + 1 && dot(g.ns, g.wo) > 0.0f) {
                mat_frame<MAT>(g);
                const typename MatSel<MAT>::M m = mat_load<MAT>(lds.params, g.seg);
                const typename MatSel<MAT>::M ms = a.frozen ? mat_load<MAT>(lds.sparams, g.seg) : m;
                float u[8];
                vertex_uniforms(a.rng, pid, k, u);
                const float4 dk = a.guided ? a.ck_d[ck] : make_float4(0.0f, 0.0f, 0.0f, -1.0f);
                if (a.mis != 0 && sc.nlt > 0) {
                    const NeeS n = nee_setup(sc, cdf, lights, g, u);
                    if (n.shoot && (flags & kCkVis) != 0) {
                        // with a guide the forward pass stored the combined density of wl
                        const NeeC nc = nee_contrib(a, lds, cdf, g, m, ms, n, dk.w);
                        if (nc.valid) {
                            constexpr int NP = MatSel<MAT>::NP;
                            const int mb = NP * g.seg, eb = NP * sc.S + 3 * n.lk;
                            mat_grad(lds.grad, mb, m, g, n.wl, wT * nc.e * nc.g, nc.spec, nc.dspec);
                            const V3 wf = wT * nc.f * nc.g;
                            lds_add(lds.grad, eb + 0, wf.x);
                            lds_add(lds.grad, eb + 1, wf.y);
                            lds_add(lds.grad, eb + 2, wf.z);
                        }
                    }
                }
                if (flags & kCkCont) {
                    ContS cs;
                    if (a.guided) {
                        // the sampled direction and its density come from the checkpoint
                        cs = cont_eval(a, g, m, ms, v3(dk.x, dk.y, dk.z), a.ck_a[ck].w, 0, u, k, Ts);
                    } else {
                        bool ug;
                        cs = cont_sample<0>(a, g, m, ms, u, k, Ts, nullptr, ug);
                    }
                    const float rq = 1.0f / cs.qrr;
                    mat_grad(lds.grad, MatSel<MAT>::NP * g.seg, m, g, cs.wi, wT * Rn * (cs.g * rq), cs.spec, cs.dspec);
                    T = T * (cs.av * rq);
                    Ts = Ts * cs.ts * rq;
                    prev_pdf = cs.pdf;
                    d = cs.wi;
                    ++k;
                    done = false;
                }
            }
        }
        if (done) {
            in_path = false;
            ++s;
        }
    }
    flush_stats(a, kReplay, wk, npaths);
    if constexpr (PG) return;   // the atomics went straight to the accumulator copies
    __syncthreads();
    double* out = a.grad_part + (size_t)blockIdx.x * a.P;
    for (int i = tid; i < a.P; i += kBlock) out[i] = lds.grad[i];
}

// ---------------------------------------------------------------------------
// Guide training records from the gradient pass: after the forward pass and
// its backward sweep, vertex k of a path holds its hit, the sampled
// continuation direction w_i and density p_i, and R_{k+1}, the radiance
// arriving along w_i.  Every record_stride-th path contributes one record per
// continued vertex: (normalised position, shading normal, outgoing
// direction, segment, w_i, weight = luminance(R_{k+1}) / p_i).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void guide_records_kernel(PathArgs a) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.pix_count * a.spp) return;
    int64_t q = p / a.spp;
    int s = (int)(p - q * a.spp);
    int64_t wi = a.pix_begin + q;
    int64_t gpath = wi * a.spp + s;
    if (gpath % a.grec_stride != 0) return;
    if (a.mask && a.mask[gpath] == 0) return;
    const size_t plane = (size_t)a.pix_count;
    if ((uint32_t)a.ck_hit[(size_t)s * plane + q].x & kCkDrop) return;
    int64_t pix = a.pixel_list ? a.pixel_list[wi] : wi;
    int64_t npix_img = (int64_t)a.V * a.W * a.H;
    if (pix < 0 || pix >= npix_img) return;
    int view = (int)(pix / ((int64_t)a.W * a.H));
    int64_t rem = pix - (int64_t)view * a.W * a.H;
    int py = (int)(rem / a.W), px = (int)(rem - (int64_t)py * a.W);
    uint64_t pid = (uint64_t)pix * (uint64_t)a.spp + (uint64_t)s;
    float j0 = 0.5f, j1 = 0.5f;
    if (a.jitter) jitter_uniforms(a.rng, pid, j0, j1);
    V3 o, d;
    camera_ray(a, view, (float)px + j0, (float)py + j1, o, d);
    for (int k = 1; k <= a.D; ++k) {
        size_t ck = ((size_t)(k - 1) * a.spp + s) * plane + q;
        int4 rec = a.ck_hit[ck];
        uint32_t fl = (uint32_t)rec.x;
        int tri = (int)(fl & kCkTriMask) - 1;
        if (tri < 0 || !(fl & kCkCont)) break;
        V3 p0, p1, p2;
        int orig, seg, light;
        load_tri(a.sc, tri, p0, p1, p2, orig, seg, light);
        float u = __int_as_float(rec.y), v = __int_as_float(rec.z);
        V3 e1 = p1 - p0, e2 = p2 - p0;
        V3 x = p0 + e1 * u + e2 * v;
        V3 ng = normalize(cross(e1, e2));
        V3 wo = v3(-d.x, -d.y, -d.z);
        V3 ns = ng;
        if (a.sc.nrm) {
            float b0 = 1.0f - u - v;
            ns = normalize(xyz(a.sc.nrm[3 * tri]) * b0 + xyz(a.sc.nrm[3 * tri + 1]) * u + xyz(a.sc.nrm[3 * tri + 2]) * v);
        }
        if (dot(ng, wo) < 0.0f) ns = ns * -1.0f;
        float4 dk = a.ck_d[ck];
        float4 av = a.ck_a[ck];  // continuation factor f cos / p (and 1 / q_rr)
        float4 R = a.ck_c[ck];   // R_{k+1} after the sweep
        // product target f cos L_i: its ratio to the sampling density is a_k R_{k+1}
        float w = lum(v3(av.x * R.x, av.y * R.y, av.z * R.z));
        if (w > 0.0f && isfinite(w)) {
            unsigned slot = atomicAdd(a.grec_count, 1u) % (unsigned)a.grec_cap;
            float f[9];
            guide_features(a.gd, x, ns, wo, f);
            float4* r = (float4*)(a.grec + 16 * (size_t)slot);
            r[0] = make_float4(f[0], f[1], f[2], __int_as_float(seg));
            r[1] = make_float4(f[3], f[4], f[5], w);
            r[2] = make_float4(f[6], f[7], f[8], __int_as_float((int)gpath));
            r[3] = make_float4(dk.x, dk.y, dk.z, __int_as_float(k));
        }
        d = v3(dk.x, dk.y, dk.z);
    }
}

hipError_t launch_guide_records(const PathArgs& a, hipStream_t st) {
    int64_t n = a.pix_count * a.spp;
    hipLaunchKernelGGL(guide_records_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename K>
static int occ(K kern, size_t lds) {
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kBlock, lds);
    return (e != hipSuccess || nb < 1) ? 1 : nb;
}

template <int MODE, int PG, int MAT>
static int path_occ(int gk, size_t lds) {
    switch (gk) {
        case 1: return occ(path_sm_kernel<MODE, 1, PG, MAT>, lds);
        case 2: return occ(path_sm_kernel<MODE, 2, PG, MAT>, lds);
        case 3: return occ(path_sm_kernel<MODE, 3, PG, MAT>, lds);
        default: return occ(path_sm_kernel<MODE, 0, PG, MAT>, lds);
    }
}

template <int MODE, int PG, int MAT>
static void launch_path_kind(int gk, const PathArgs& a, int grid, size_t lds, hipStream_t st) {
    switch (gk) {
        case 1: hipLaunchKernelGGL((path_sm_kernel<MODE, 1, PG, MAT>), dim3(grid), dim3(kBlock), lds, st, a); break;
        case 2: hipLaunchKernelGGL((path_sm_kernel<MODE, 2, PG, MAT>), dim3(grid), dim3(kBlock), lds, st, a); break;
        case 3: hipLaunchKernelGGL((path_sm_kernel<MODE, 3, PG, MAT>), dim3(grid), dim3(kBlock), lds, st, a); break;
        default: hipLaunchKernelGGL((path_sm_kernel<MODE, 0, PG, MAT>), dim3(grid), dim3(kBlock), lds, st, a); break;
    }
}

template <int MAT>
static int blocks_per_cu_mat(int mode, size_t lds, int gk, int pg) {
    if (mode == kColor) return pg ? path_occ<kColor, 1, MAT>(gk, lds) : path_occ<kColor, 0, MAT>(gk, lds);
    if (mode == kGradFwd) return pg ? path_occ<kGradFwd, 1, MAT>(gk, lds) : path_occ<kGradFwd, 0, MAT>(gk, lds);
    if constexpr (MAT == 1) return pg ? occ(replay_sm_kernel<1, MAT>, lds) : occ(replay_sm_kernel<0, MAT>, lds);
    return pg ? occ(replay_kernel<1, MAT>, lds) : occ(replay_kernel<0, MAT>, lds);
}

int path_blocks_per_cu(int mode, size_t lds, int gk, int pg, int mat) {
    return mat == 1 ? blocks_per_cu_mat<1>(mode, lds, gk, pg) : blocks_per_cu_mat<0>(mode, lds, gk, pg);
}

template <int MAT>
static void launch_paths_mat(int mode, const PathArgs& a, int grid, size_t lds, hipStream_t st) {
    const int pg = a.params_global;
    if (mode == kColor) {
        if (pg) launch_path_kind<kColor, 1, MAT>(a.guide_kind, a, grid, lds, st);
        else launch_path_kind<kColor, 0, MAT>(a.guide_kind, a, grid, lds, st);
    } else if (mode == kGradFwd) {
        if (pg) launch_path_kind<kGradFwd, 1, MAT>(a.guide_kind, a, grid, lds, st);
        else launch_path_kind<kGradFwd, 0, MAT>(a.guide_kind, a, grid, lds, st);
    } else if (a.replay_traverse || MAT == 0) {
        // the lanes of a wave replay the same sample and vertex index of
        // consecutive pixels, so their checkpoint reads coalesce: for the
        // Lambert + GGX adjoint, whose work per vertex is light, that beats
        // refilling idle lanes (apartment replay 12.9 ms here, 26.7 ms with
        // replay_sm_kernel); the Disney adjoint, ten times the arithmetic per
        // vertex, gains from the refill (27.1 -> 23.3 ms).  Also the check
        // mode that re-traces each path instead of reading its checkpoints.
        if (pg) hipLaunchKernelGGL((replay_kernel<1, MAT>), dim3(grid), dim3(kBlock), lds, st, a);
        else hipLaunchKernelGGL((replay_kernel<0, MAT>), dim3(grid), dim3(kBlock), lds, st, a);
    } else if constexpr (MAT == 1) {
        if (pg) hipLaunchKernelGGL((replay_sm_kernel<1, MAT>), dim3(grid), dim3(kBlock), lds, st, a);
        else hipLaunchKernelGGL((replay_sm_kernel<0, MAT>), dim3(grid), dim3(kBlock), lds, st, a);
    }
}

// The proposal is compiled in only when it is sampled (guide_mix > 0); kind
// as in PathArgs::guide_kind, material model as in PathArgs::mat.
hipError_t launch_paths(int mode, const PathArgs& a, int grid, size_t lds, hipStream_t st) {
    if (a.mat == 1) launch_paths_mat<1>(mode, a, grid, lds, st);
    else launch_paths_mat<0>(mode, a, grid, lds, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batch ray casting (hit parity and BVH checks).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void trace_rays_kernel(SceneDev sc, const float* o, const float* d,
                                                            const int* skip, int64_t n, float tmin, int brute,
                                                            int64_t nt, int* out_tri, float* out_tuv, int* ovf,
                                                            Counters* err) {
    __shared__ int stk[kShortStack * kBlock];
    Stack st;
    st.lds = stk;
    st.ovf = ovf;
    st.tid = threadIdx.x;
    st.gtid = blockIdx.x * kBlock + threadIdx.x;
    st.gthreads = gridDim.x * kBlock;
    st.overflow = false;
    st.sp = 0;
    Work wk{0u, 0u, 0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        Ray r = make_ray(v3(o[3 * i], o[3 * i + 1], o[3 * i + 2]), v3(d[3 * i], d[3 * i + 1], d[3 * i + 2]));
        int sk = (skip && skip[i] >= 0 && skip[i] < nt) ? sc.pos_of[skip[i]] : -1;
        Hit h = brute ? brute_closest(sc, nt, r, tmin, sk)
                      : traverse(sc, r, tmin, __builtin_inff(), sk, -1, false, st, wk);
        int orig = -1;
        if (h.tri >= 0) orig = __float_as_int(sc.tris[3 * h.tri].w);
        out_tri[i] = orig;
        out_tuv[3 * i] = h.tri >= 0 ? h.t : 0.0f;
        out_tuv[3 * i + 1] = h.u;
        out_tuv[3 * i + 2] = h.v;
    }
    if (st.overflow) atomicAdd(&err->overflow, 1ull);
}

int trace_rays_grid(int num_cu) { return num_cu * 4; }

hipError_t launch_trace_rays(const SceneDev& sc, const float* o, const float* d, const int* skip, int64_t n,
                             float tmin, int brute, int64_t nt, int* out_tri, float* out_tuv, int* ovf, int grid,
                             Counters* err, hipStream_t st) {
    hipLaunchKernelGGL(trace_rays_kernel, dim3(grid), dim3(kBlock), 0, st, sc, o, d, skip, n, tmin, brute, nt,
                       out_tri, out_tuv, ovf, err);
    return hipGetLastError();
}

}  // namespace ipt
