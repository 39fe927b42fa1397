// Path kernels of the inverse path tracer (gfx950).
//
// One lane owns one pixel and walks its spp paths one after another, so the
// pixel mean is formed in registers (no atomics, deterministic).  Blocks are
// persistent: they pull 256-pixel tiles from a counter until the chunk is
// done.  The same path loop runs in three modes:
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
#include <hip/hip_runtime.h>

#include "ipt_internal.h"

namespace ipt {

struct Lds {
    float* params;
    float* sparams;
    int* seg_emitter;
    float* cdf;
    int4* lights;
    float* grad;
    int* stack;
    bool lights_in_lds;
};

size_t path_lds_bytes(int mode, int P, int frozen, int S, int nlt) {
    size_t b = 0;
    auto al = [](size_t x) { return (x + 15) & ~size_t(15); };
    b += al(sizeof(float) * P);                       // params
    if (frozen) b += al(sizeof(float) * P);           // sampling params
    b += al(sizeof(int) * S);                         // segment -> emitter
    if (nlt <= kMaxLdsLights) b += al(sizeof(float) * nlt) + al(sizeof(int4) * nlt);
    if (mode == kReplay) b += al(sizeof(float) * P);  // block gradient
    b += sizeof(int) * kShortStack * kBlock;          // short stacks
    return b;
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
    __device__ __forceinline__ int pop() {
        --sp;
        int slot = sp & (kShortStack - 1);
        int x = lds[slot * kBlock + tid];
        if (sp >= kShortStack) lds[slot * kBlock + tid] = ovf[(size_t)(sp - kShortStack) * gthreads + gtid];
        return x;
    }
};

struct Hit {
    int tri;     // leaf-ordered index, -1 on miss
    float t, u, v;
};

__device__ __forceinline__ void load_tri(const SceneDev& sc, int i, V3& p0, V3& p1, V3& p2, int& orig,
                                         int& seg, int& light) {
    float4 a = sc.tris[3 * i], b = sc.tris[3 * i + 1], c = sc.tris[3 * i + 2];
    p0 = xyz(a); p1 = xyz(b); p2 = xyz(c);
    orig = __float_as_int(a.w);
    seg = __float_as_int(b.w);
    light = __float_as_int(c.w);
}

// Closest hit (ANY = false) or occlusion test (ANY = true: returns tri >= 0
// as soon as anything lies in (tmin, tmax)).  skip0/skip1 are leaf indices
// that are ignored.  Ties in t are resolved toward the smaller original id.
struct Work {
    uint32_t rays, nodes, tris, vertices;
};

template <bool ANY>
__device__ Hit traverse(const SceneDev& sc, const Ray& r, float tmin, float tmax, int skip0, int skip1,
                        Stack& st, Work& wk) {
    Hit best{-1, tmax, 0.0f, 0.0f};
    wk.rays++;
    int best_orig = 0x7FFFFFFF;
    st.sp = 0;
    int entry = 0;
    while (true) {
        if (entry >= 0) {
            wk.nodes++;
            const float4* n = sc.nodes + 4 * (size_t)entry;
            float4 n0 = n[0], n1 = n[1], n2 = n[2], n3 = n[3];
            int c0 = __float_as_int(n3.x), c1 = __float_as_int(n3.y);
            float t0 = box_entry(r, v3(n0.x, n0.y, n0.z), v3(n0.w, n1.x, n1.y), tmin, best.t);
            float t1 = box_entry(r, v3(n1.z, n1.w, n2.x), v3(n2.y, n2.z, n2.w), tmin, best.t);
            // box_entry returns +inf on a miss; best.t may itself be +inf
            bool h0 = t0 < __builtin_inff();
            bool h1 = (c1 != kNone) && t1 < __builtin_inff();
            if (h0 && h1) {
                bool first0 = t0 <= t1;
                st.push(first0 ? c1 : c0);
                entry = first0 ? c0 : c1;
                continue;
            }
            if (h0) { entry = c0; continue; }
            if (h1) { entry = c1; continue; }
        } else {
            int code = ~entry;
            int first = code >> 3, cnt = (code & 7) + 1;
            wk.tris += cnt;
            for (int i = first; i < first + cnt; ++i) {
                if (i == skip0 || i == skip1) continue;
                V3 p0, p1, p2;
                int orig, seg, light;
                load_tri(sc, i, p0, p1, p2, orig, seg, light);
                float t, u, v;
                if (!tri_isect(r, p0, p1, p2, tmin, t, u, v)) continue;
                if (ANY) {
                    if (t < tmax) { best.tri = i; best.t = t; return best; }
                } else if (t < best.t || (t == best.t && orig < best_orig)) {
                    best.tri = i; best.t = t; best.u = u; best.v = v;
                    best_orig = orig;
                }
            }
        }
        if (st.sp == 0 || st.overflow) break;
        entry = st.pop();
    }
    if (!ANY && best.tri >= 0 && !(best.t < tmax)) best.tri = -1;
    return best;
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
// Light selection from the cumulative table (first j with cdf[j] > u*total).
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
    float prev = j > 0 ? cdf[j - 1] : 0.0f;
    return (cdf[j] - prev) / cdf[n - 1];
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

__device__ __forceinline__ void lds_add(float* g, int i, float x) {
    if (x != 0.0f) atomicAdd(g + i, x);
}

// ---------------------------------------------------------------------------
// One path.  Returns the path radiance; in kGradFwd also writes checkpoints;
// in kReplay adds w-weighted derivatives into lds.grad.
// ---------------------------------------------------------------------------
template <int MODE>
__device__ V3 run_path(const PathArgs& a, const Lds& lds, Stack& st, Work& wk, uint64_t pid, int64_t q, int s,
                       V3 org, V3 dir, V3 wpix, uint64_t& hash, bool& drop_out, float* dv) {
    const SceneDev& sc = a.sc;
    const float* cdf = lds.lights_in_lds ? lds.cdf : a.cdf;
    const int4* lights = lds.lights_in_lds ? lds.lights : sc.lights;
    const int D = a.D;
    const size_t plane = (size_t)a.pix_count;
    V3 T = v3(1.0f, 1.0f, 1.0f), Ts = T, L = v3(0.0f, 0.0f, 0.0f);
    float prev_pdf = 0.0f;
    int prev_tri = -1;
    uint64_t h = 0xCBF29CE484222325ull;
    V3 o = org, d = dir;
    int klast = 0;
    drop_out = false;
    if (MODE == kReplay) {
        int4 r1 = a.ck_hit[(size_t)s * plane + q];
        if (r1.x & kCkDrop) { drop_out = true; return L; }
    }
    for (int k = 1; k <= D + 1; ++k) {
        Hit hit;
        uint32_t ckflags = 0;
        V3 Rn = v3(0.0f, 0.0f, 0.0f);   // replay: R_{k+1}
        size_t ck = ((size_t)(k - 1) * a.spp + s) * plane + q;
        if (MODE == kReplay && !a.replay_traverse) {
            int4 rec = a.ck_hit[ck];
            uint32_t x = (uint32_t)rec.x;
            hit.tri = (int)(x & kCkTriMask) - 1;
            hit.u = __int_as_float(rec.y);
            hit.v = __int_as_float(rec.z);
            hit.t = __int_as_float(rec.w);
            ckflags = x;
        } else {
            Ray ray = make_ray(o, d);
            hit = traverse<false>(sc, ray, sc.tmin, __builtin_inff(), prev_tri, -1, st, wk);
            if (MODE == kReplay) ckflags = (uint32_t)a.ck_hit[ck].x;
        }
        if (MODE == kReplay) {
            float4 rr = a.ck_c[ck];
            Rn = v3(rr.x, rr.y, rr.z);
        }
        klast = k;
        wk.vertices++;
        V3 ck_c = v3(0.0f, 0.0f, 0.0f), ck_a = v3(0.0f, 0.0f, 0.0f);
        uint32_t flags = 0;
        if (hit.tri < 0) {
            h = fnv1a(h, 0xFFFFFFFFu);
            if (MODE == kGradFwd) a.ck_hit[ck] = make_int4(0, 0, 0, 0);
            klast = k - 1;   // a miss contributes nothing: the sweep starts below it
            break;
        }
        V3 p0, p1, p2;
        int orig, seg, light;
        load_tri(sc, hit.tri, p0, p1, p2, orig, seg, light);
        h = fnv1a(h, (uint32_t)orig);
        float* dvk = dv ? dv + 8 * (k - 1) : nullptr;
        if (dvk) {
            dvk[0] = (float)orig; dvk[1] = hit.u; dvk[2] = hit.v; dvk[3] = hit.t;
            dvk[4] = L.x; dvk[5] = L.y; dvk[6] = L.z; dvk[7] = 0.0f;
        }
        V3 e1 = p1 - p0, e2 = p2 - p0;
        V3 x = p0 + e1 * hit.u + e2 * hit.v;
        V3 ng = normalize(cross(e1, e2));
        int em = lds.seg_emitter[seg];
        float cos_emit = -dot(d, ng);
        uint32_t ev = 0;
        V3 wT = wpix * T;
        // ---- emitter hit (MIS weight against light sampling) ----
        if (em >= 0 && cos_emit > 0.0f) {
            float w = 1.0f;
            if (k > 1) {
                if (a.mis == 1) w = 0.0f;
                else if (a.mis >= 2) {
                    float pa = light_prob(cdf, sc.nlt, light) / __int_as_float(lights[light].z);
                    float pl = pa * hit.t * hit.t / cos_emit;
                    w = mis_weight(prev_pdf, pl, a.mis);
                }
            }
            if (w > 0.0f) {
                float prof = a.profile ? cos_emit : 1.0f;
                const float* e = lds.params + 7 * sc.S + 3 * em;
                V3 c = v3(e[0], e[1], e[2]) * (prof * w);
                ck_c = ck_c + c;
                L = L + T * c;
                if (dvk) { dvk[4] = L.x; dvk[5] = L.y; dvk[6] = L.z; }
                if (MODE == kReplay) {
                    int eb = 7 * sc.S + 3 * em;
                    lds_add(lds.grad, eb + 0, wT.x * prof * w);
                    lds_add(lds.grad, eb + 1, wT.y * prof * w);
                    lds_add(lds.grad, eb + 2, wT.z * prof * w);
                }
            }
            ev |= 1u;
        }
        if (k == D + 1) {
            h = fnv1a(h, ev);
            if (MODE == kGradFwd) {
                a.ck_hit[ck] = make_int4((int)((uint32_t)(hit.tri + 1) | flags), __float_as_int(hit.u),
                                         __float_as_int(hit.v), __float_as_int(hit.t));
                a.ck_c[ck] = make_float4(ck_c.x, ck_c.y, ck_c.z, 0.0f);
                a.ck_a[ck] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
            break;
        }
        // ---- shading frame: two-sided, flipped toward the incoming ray ----
        V3 wo = v3(-d.x, -d.y, -d.z);
        V3 ns = ng;
        if (sc.nrm) {
            float b0 = 1.0f - hit.u - hit.v;
            V3 n0 = xyz(sc.nrm[3 * hit.tri]), n1 = xyz(sc.nrm[3 * hit.tri + 1]), n2 = xyz(sc.nrm[3 * hit.tri + 2]);
            ns = normalize(n0 * b0 + n1 * hit.u + n2 * hit.v);
        }
        V3 ngf = ng;
        if (dot(ng, wo) < 0.0f) { ngf = ng * -1.0f; ns = ns * -1.0f; }
        bool cont = false;
        if (dot(ns, wo) <= 0.0f) {
            h = fnv1a(h, ev | 2u);
        } else {
            Mat m = load_mat(lds.params, seg);
            Mat ms = a.frozen ? load_mat(lds.sparams, seg) : m;
            float u[8];
            vertex_uniforms(a.rng, pid, k, u);
            // ---- next-event estimation ----
            if (a.mis != 0 && sc.nlt > 0) {
                int lj = pick_light(cdf, sc.nlt, u[0]);
                int4 lrec = lights[lj];
                V3 q0, q1, q2;
                int lorig, lseg, llight;
                load_tri(sc, lrec.x, q0, q1, q2, lorig, lseg, llight);
                float su = sqrtf(u[1]);
                float b1 = (1.0f - u[2]) * su, b2 = u[2] * su;
                // y - x from vertex differences and edge terms: the light point and
                // the shading point are never rounded to world coordinates first
                V3 dl = (q0 - p0) + ((q1 - q0) * b1 + (q2 - q0) * b2 - (e1 * hit.u + e2 * hit.v));
                V3 lng = normalize(cross(q1 - q0, q2 - q0));
                float d2 = dot(dl, dl), dist = sqrtf(d2);
                V3 wl = dl * (1.0f / dist);
                float cy = -dot(wl, lng);
                float cxg = dot(wl, ngf);
                bool vis = false;
                // grazing configurations (cosines below 1e-6: the light
                // triangle itself, a coplanar emitter) are skipped
                if (cy > 1e-6f && cxg > 1e-6f) {
                    if (MODE == kReplay && !a.replay_traverse) {
                        vis = (ckflags & kCkVis) != 0;
                    } else {
                        Ray sr = make_ray(x, wl);
                        Hit sh = traverse<true>(sc, sr, sc.tmin, dist * (1.0f - 1e-5f), hit.tri, lrec.x, st, wk);
                        vis = sh.tri < 0;
                    }
                }
                ev |= ((uint32_t)lj << 8) | ((uint32_t)vis << 2);
                if (vis) {
                    flags |= kCkVis;
                    float spec, dspec;
                    spec_term(ns, wo, wl, m.alpha, spec, dspec);
                    float cx = dot(ns, wl);
                    if (cx > 0.0f) {
                        int lk = lrec.y;
                        float parea = light_prob(cdf, sc.nlt, lj) / __int_as_float(lrec.z);
                        float w = 1.0f;
                        if (a.mis >= 2) {
                            float pl = parea * d2 / cy;
                            float pb = brdf_pdf(ms, ns, wo, wl);
                            if (a.gmix > 0.0f) pb = (1.0f - a.gmix) * pb;  // guide pdf added by the guide path
                            w = mis_weight(pl, pb, a.mis);
                        }
                        float prof = a.profile ? cy : 1.0f;
                        float g = cx * cy / d2 * w / parea * prof;
                        const float* ep = lds.params + 7 * sc.S + 3 * lk;
                        V3 e = v3(ep[0], ep[1], ep[2]);
                        V3 f = m.kd * kInvPi + m.ks * spec;
                        V3 c = f * e * g;
                        ck_c = ck_c + c;
                        L = L + T * c;
                        if (dvk) { dvk[4] = L.x; dvk[5] = L.y; dvk[6] = L.z; dvk[7] = 1.0f; }
                        if (MODE == kReplay) {
                            int mb = 7 * seg, eb = 7 * sc.S + 3 * lk;
                            V3 we = wT * e * g;
                            lds_add(lds.grad, mb + 0, we.x * kInvPi);
                            lds_add(lds.grad, mb + 1, we.y * kInvPi);
                            lds_add(lds.grad, mb + 2, we.z * kInvPi);
                            lds_add(lds.grad, mb + 3, we.x * spec);
                            lds_add(lds.grad, mb + 4, we.y * spec);
                            lds_add(lds.grad, mb + 5, we.z * spec);
                            lds_add(lds.grad, mb + 6, dot(we, m.ks) * dspec);
                            V3 wf = wT * f * g;
                            lds_add(lds.grad, eb + 0, wf.x);
                            lds_add(lds.grad, eb + 1, wf.y);
                            lds_add(lds.grad, eb + 2, wf.z);
                        }
                    }
                }
            }
            // ---- continue by sampling the material ----
            V3 wi;
            int lobe = 0;
            bool ok = brdf_sample(ms, ns, wo, u[3], u[4], u[5], wi, lobe);
            ev |= (uint32_t)lobe << 3;
            float pdf = 0.0f;
            if (ok && dot(wi, ngf) > 0.0f && dot(wi, ns) > 0.0f) pdf = brdf_pdf(ms, ns, wo, wi);
            if (!(pdf > 0.0f)) {
                h = fnv1a(h, ev | 16u);
            } else {
                float spec, dspec;
                spec_term(ns, wo, wi, m.alpha, spec, dspec);
                float ci = dot(ns, wi);
                float g = ci / pdf;
                V3 av = (m.kd * kInvPi + m.ks * spec) * g;
                V3 ts = av;
                if (a.frozen) ts = (ms.kd * kInvPi + ms.ks * spec_only(ns, wo, wi, ms.alpha)) * g;
                float qrr = 1.0f;
                bool alive = true;
                if (a.rr_depth >= 0 && k >= a.rr_depth) {
                    qrr = fminf(fmaxf(maxc(Ts * ts), 0.1f), 0.95f);
                    alive = u[6] < qrr;
                }
                if (MODE == kReplay) alive = (ckflags & kCkCont) != 0;
                if (!alive) {
                    h = fnv1a(h, ev | 32u);
                } else {
                    float rq = 1.0f / qrr;
                    av = av * rq;
                    Ts = Ts * ts * rq;
                    if (MODE == kReplay) {
                        int mb = 7 * seg;
                        float gq = g * rq;
                        V3 wr = wT * Rn * gq;
                        lds_add(lds.grad, mb + 0, wr.x * kInvPi);
                        lds_add(lds.grad, mb + 1, wr.y * kInvPi);
                        lds_add(lds.grad, mb + 2, wr.z * kInvPi);
                        lds_add(lds.grad, mb + 3, wr.x * spec);
                        lds_add(lds.grad, mb + 4, wr.y * spec);
                        lds_add(lds.grad, mb + 5, wr.z * spec);
                        lds_add(lds.grad, mb + 6, dot(wr, m.ks) * dspec);
                    }
                    h = fnv1a(h, ev);
                    ck_a = av;
                    flags |= kCkCont;
                    cont = true;
                    prev_pdf = pdf;
                    prev_tri = hit.tri;
                    T = T * av;
                    o = x;
                    d = wi;
                }
            }
        }
        if (MODE == kGradFwd) {
            a.ck_hit[ck] = make_int4((int)((uint32_t)(hit.tri + 1) | flags), __float_as_int(hit.u),
                                     __float_as_int(hit.v), __float_as_int(hit.t));
            a.ck_c[ck] = make_float4(ck_c.x, ck_c.y, ck_c.z, 0.0f);
            a.ck_a[ck] = make_float4(ck_a.x, ck_a.y, ck_a.z, 0.0f);
        }
        if (!cont) break;
    }
    if (MODE == kGradFwd) {
        // backward sweep: R_{k+1} into the c slot of vertex k
        V3 R = v3(0.0f, 0.0f, 0.0f);
        for (int k = klast; k >= 1; --k) {
            size_t ck = ((size_t)(k - 1) * a.spp + s) * plane + q;
            float4 c = a.ck_c[ck], av = a.ck_a[ck];
            a.ck_c[ck] = make_float4(R.x, R.y, R.z, 0.0f);
            R = v3(c.x, c.y, c.z) + v3(av.x, av.y, av.z) * R;
        }
        if (!finite3(R) || !finite3(L)) {
            size_t c1 = (size_t)s * plane + q;
            int4 r1 = a.ck_hit[c1];
            r1.x = (int)((uint32_t)r1.x | kCkDrop);
            a.ck_hit[c1] = r1;
            drop_out = true;
        }
    }
    hash = h;
    return L;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void path_kernel(PathArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned tile_sh;
    const int tid = threadIdx.x;
    // ---- carve LDS ----
    Lds lds;
    unsigned char* p = smem;
    auto al = [](size_t x) { return (x + 15) & ~size_t(15); };
    lds.params = (float*)p; p += al(sizeof(float) * a.P);
    lds.sparams = lds.params;
    if (a.frozen) { lds.sparams = (float*)p; p += al(sizeof(float) * a.P); }
    lds.seg_emitter = (int*)p; p += al(sizeof(int) * a.sc.S);
    lds.lights_in_lds = a.sc.nlt <= kMaxLdsLights;
    lds.cdf = nullptr; lds.lights = nullptr;
    if (lds.lights_in_lds) {
        lds.cdf = (float*)p; p += al(sizeof(float) * a.sc.nlt);
        lds.lights = (int4*)p; p += al(sizeof(int4) * a.sc.nlt);
    }
    lds.grad = nullptr;
    if (MODE == kReplay) { lds.grad = (float*)p; p += al(sizeof(float) * a.P); }
    lds.stack = (int*)p;
    for (int i = tid; i < a.P; i += kBlock) {
        lds.params[i] = a.params[i];
        if (a.frozen) lds.sparams[i] = a.sparams[i];
        if (MODE == kReplay) lds.grad[i] = 0.0f;
    }
    for (int i = tid; i < a.sc.S; i += kBlock) lds.seg_emitter[i] = a.sc.seg_emitter[i];
    if (lds.lights_in_lds)
        for (int i = tid; i < a.sc.nlt; i += kBlock) {
            lds.cdf[i] = a.cdf[i];
            lds.lights[i] = a.sc.lights[i];
        }
    __syncthreads();

    Stack st;
    st.lds = lds.stack;
    st.ovf = a.ovf;
    st.tid = tid;
    st.gtid = blockIdx.x * kBlock + tid;
    st.gthreads = gridDim.x * kBlock;
    st.overflow = false;
    st.sp = 0;

    const int64_t npix_img = (int64_t)a.V * a.W * a.H;
    Work wk{0u, 0u, 0u, 0u};
    uint32_t npaths = 0;
    while (true) {
        if (tid == 0) tile_sh = atomicAdd(a.work, 1u);
        __syncthreads();
        int64_t q = (int64_t)tile_sh * kBlock + tid;
        __syncthreads();
        if ((int64_t)tile_sh * kBlock >= a.pix_count) break;
        if (q >= a.pix_count) continue;
        int64_t wi = a.pix_begin + q;                     // work-pixel index
        int64_t pix = a.pixel_list ? a.pixel_list[wi] : wi;
        if (pix < 0 || pix >= npix_img) continue;
        int view = (int)(pix / ((int64_t)a.W * a.H));
        int64_t rem = pix - (int64_t)view * a.W * a.H;
        int py = (int)(rem / a.W), px = (int)(rem - (int64_t)py * a.W);
        V3 wpix = v3(0.0f, 0.0f, 0.0f);
        if (MODE == kReplay) {
            float inv = 1.0f / (float)a.spp;
            wpix = v3(a.w[3 * wi] * inv, a.w[3 * wi + 1] * inv, a.w[3 * wi + 2] * inv);
        }
        V3 acc = v3(0.0f, 0.0f, 0.0f);
        for (int s = 0; s < a.spp; ++s) {
            uint64_t pid = (uint64_t)pix * (uint64_t)a.spp + (uint64_t)s;
            size_t pidx = (size_t)wi * a.spp + s;
            bool use = a.mask ? a.mask[pidx] != 0 : true;
            if (MODE == kReplay && !use) continue;
            float j0 = 0.5f, j1 = 0.5f;
            if (a.jitter) jitter_uniforms(a.rng, pid, j0, j1);
            V3 o, d;
            camera_ray(a, view, (float)px + j0, (float)py + j1, o, d);
            uint64_t hsh;
            bool drop;
            float* dv = nullptr;
            if (MODE == kColor && a.dbg_vtx) {
                dv = a.dbg_vtx + pidx * 8 * (size_t)(a.D + 1);
                for (int k = 0; k < 8 * (a.D + 1); ++k) dv[k] = -1.0f;
            }
            V3 Lp = run_path<MODE>(a, lds, st, wk, pid, q, s, o, d, wpix, hsh, drop, dv);
            ++npaths;
            if (MODE == kColor) {
                if (!finite3(Lp)) {
                    atomicAdd(&a.err->nonfinite, 1ull);
                } else if (use) {
                    acc = acc + Lp;
                }
            }
            if (MODE == kGradFwd && drop) atomicAdd(&a.err->nonfinite, 1ull);
            if (MODE != kReplay && a.hash) a.hash[pidx] = hsh;
            if (MODE == kColor && a.path_L) {
                a.path_L[3 * pidx] = Lp.x;
                a.path_L[3 * pidx + 1] = Lp.y;
                a.path_L[3 * pidx + 2] = Lp.z;
            }
        }
        if (MODE == kColor) {
            float inv = 1.0f / (float)a.spp;
            a.image[3 * wi] = acc.x * inv;
            a.image[3 * wi + 1] = acc.y * inv;
            a.image[3 * wi + 2] = acc.z * inv;
        }
    }
    if (st.overflow) atomicAdd(&a.err->overflow, 1ull);
    if (a.count_stats) {
        KStats* ks = &a.err->k[MODE];
        atomicAdd(&ks->rays, (unsigned long long)wk.rays);
        atomicAdd(&ks->nodes, (unsigned long long)wk.nodes);
        atomicAdd(&ks->tris, (unsigned long long)wk.tris);
        atomicAdd(&ks->paths, (unsigned long long)npaths);
        atomicAdd(&ks->vertices, (unsigned long long)wk.vertices);
    }
    if (MODE == kReplay) {
        __syncthreads();
        float* out = a.grad_part + (size_t)blockIdx.x * a.P;
        for (int i = tid; i < a.P; i += kBlock) out[i] = lds.grad[i];
    }
}

int path_blocks_per_cu(int mode, size_t lds) {
    int nb = 0;
    hipError_t e;
    if (mode == kColor)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, path_kernel<kColor>, kBlock, lds);
    else if (mode == kGradFwd)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, path_kernel<kGradFwd>, kBlock, lds);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, path_kernel<kReplay>, kBlock, lds);
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

hipError_t launch_paths(int mode, const PathArgs& a, int grid, size_t lds, hipStream_t st) {
    if (mode == kColor)
        hipLaunchKernelGGL(path_kernel<kColor>, dim3(grid), dim3(kBlock), lds, st, a);
    else if (mode == kGradFwd)
        hipLaunchKernelGGL(path_kernel<kGradFwd>, dim3(grid), dim3(kBlock), lds, st, a);
    else
        hipLaunchKernelGGL(path_kernel<kReplay>, dim3(grid), dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batch ray casting (hit parity and BVH checks).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void trace_rays_kernel(SceneDev sc, const float* o, const float* d,
                                                            const int* skip, int64_t n, float tmin,
                                                            int brute, int64_t nt, int* out_tri,
                                                            float* out_tuv, int* ovf, Counters* err) {
    __shared__ int stk[kShortStack * kBlock];
    Stack st;
    st.lds = stk;
    st.ovf = ovf;
    st.tid = threadIdx.x;
    st.gtid = blockIdx.x * kBlock + threadIdx.x;
    st.gthreads = gridDim.x * kBlock;
    st.overflow = false;
    st.sp = 0;
    Work wk{0u, 0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        Ray r = make_ray(v3(o[3 * i], o[3 * i + 1], o[3 * i + 2]), v3(d[3 * i], d[3 * i + 1], d[3 * i + 2]));
        int sk = (skip && skip[i] >= 0 && skip[i] < nt) ? sc.pos_of[skip[i]] : -1;
        Hit h = brute ? brute_closest(sc, nt, r, tmin, sk)
                      : traverse<false>(sc, r, tmin, __builtin_inff(), sk, -1, st, wk);
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

hipError_t launch_trace_rays(const SceneDev& sc, const float* o, const float* d, const int* skip,
                             int64_t n, float tmin, int brute, int64_t nt, int* out_tri,
                             float* out_tuv, int* ovf, int grid, Counters* err, hipStream_t st) {
    hipLaunchKernelGGL(trace_rays_kernel, dim3(grid), dim3(kBlock), 0, st, sc, o, d, skip, n, tmin,
                       brute, nt, out_tri, out_tuv, ovf, err);
    return hipGetLastError();
}

}  // namespace ipt
