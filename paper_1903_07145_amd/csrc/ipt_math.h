// Device-side math of the path tracer: vectors, Philox, ray/box and
// ray/triangle tests, the material model and its sampler, MIS weights.
// Everything here is float32 except the exact-zero fallback of the
// watertight triangle test.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipt {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return v3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ V3 operator*(V3 a, V3 b) { return v3(a.x * b.x, a.y * b.y, a.z * b.z); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 normalize(V3 a) { return a * (1.0f / sqrtf(dot(a, a))); }
__device__ __forceinline__ float comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
__device__ __forceinline__ V3 xyz(float4 a) { return v3(a.x, a.y, a.z); }
__device__ __forceinline__ float maxc(V3 a) { return fmaxf(a.x, fmaxf(a.y, a.z)); }
__device__ __forceinline__ bool finite3(V3 a) {
    return isfinite(a.x) && isfinite(a.y) && isfinite(a.z);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit multiply per word gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}
__device__ __forceinline__ float u24(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

struct Rng {
    uint32_t k0, k1, iteration;
};
// The eight uniforms of vertex k of path `pid` (slots as in the header).
__device__ __forceinline__ void vertex_uniforms(const Rng& r, uint64_t pid, int k, float u[8]) {
    uint4 a = philox(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), 2u * k, r.iteration), r.k0, r.k1);
    uint4 b = philox(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), 2u * k + 1u, r.iteration), r.k0, r.k1);
    u[0] = u24(a.x); u[1] = u24(a.y); u[2] = u24(a.z); u[3] = u24(a.w);
    u[4] = u24(b.x); u[5] = u24(b.y); u[6] = u24(b.z); u[7] = u24(b.w);
}
__device__ __forceinline__ void jitter_uniforms(const Rng& r, uint64_t pid, float& u0, float& u1) {
    uint4 a = philox(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), 0u, r.iteration), r.k0, r.k1);
    u0 = u24(a.x);
    u1 = u24(a.y);
}

__device__ __forceinline__ uint64_t fnv1a(uint64_t h, uint32_t x) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h ^= (x >> (8 * i)) & 0xFFu;
        h *= 0x100000001B3ull;
    }
    return h;
}

// ---------------------------------------------------------------------------
// Rays.  Watertight ray/triangle test: Woop, Benthin, Wald, "Watertight
// Ray/Triangle Intersection", JCGT 2013.  The edge functions are evaluated
// without contraction so a shared edge gives exactly opposite values in the
// two triangles; an exact zero is re-evaluated in double.
// ---------------------------------------------------------------------------
struct Ray {
    V3 o, d;
    V3 inv;          // 1/d with zero components replaced by +-1e-20
    int kx, ky, kz;
    float Sx, Sy, Sz;
};

__device__ __forceinline__ Ray make_ray(V3 o, V3 d) {
    Ray r;
    r.o = o;
    r.d = d;
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = 0;
    if (ay > ax) kz = 1;
    if (az > fmaxf(ax, ay)) kz = 2;
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    float dz = comp(d, kz);
    if (dz < 0.0f) { int t = kx; kx = ky; ky = t; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.Sx = __fdiv_rn(comp(d, kx), dz);
    r.Sy = __fdiv_rn(comp(d, ky), dz);
    r.Sz = __fdiv_rn(1.0f, dz);
    // the hardware reciprocal (1 ulp): the slab distances only cull boxes,
    // and their relative slack covers it
    r.inv = v3(__builtin_amdgcn_rcpf(fabsf(d.x) > 1e-20f ? d.x : copysignf(1e-20f, d.x)),
               __builtin_amdgcn_rcpf(fabsf(d.y) > 1e-20f ? d.y : copysignf(1e-20f, d.y)),
               __builtin_amdgcn_rcpf(fabsf(d.z) > 1e-20f ? d.z : copysignf(1e-20f, d.z)));
    return r;
}

// Returns true with (t, u, v) if the triangle is hit at tmin < t; the caller
// applies the upper bound and the tie rule.
__device__ __forceinline__ bool tri_isect(const Ray& r, V3 p0, V3 p1, V3 p2, float tmin, float& t,
                                          float& u, float& v) {
    V3 A = p0 - r.o, B = p1 - r.o, C = p2 - r.o;
    float Akz = comp(A, r.kz), Bkz = comp(B, r.kz), Ckz = comp(C, r.kz);
    float Ax = __fsub_rn(comp(A, r.kx), __fmul_rn(r.Sx, Akz));
    float Ay = __fsub_rn(comp(A, r.ky), __fmul_rn(r.Sy, Akz));
    float Bx = __fsub_rn(comp(B, r.kx), __fmul_rn(r.Sx, Bkz));
    float By = __fsub_rn(comp(B, r.ky), __fmul_rn(r.Sy, Bkz));
    float Cx = __fsub_rn(comp(C, r.kx), __fmul_rn(r.Sx, Ckz));
    float Cy = __fsub_rn(comp(C, r.ky), __fmul_rn(r.Sy, Ckz));
    float U = __fsub_rn(__fmul_rn(Cx, By), __fmul_rn(Cy, Bx));
    float V = __fsub_rn(__fmul_rn(Ax, Cy), __fmul_rn(Ay, Cx));
    float W = __fsub_rn(__fmul_rn(Bx, Ay), __fmul_rn(By, Ax));
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        double CxBy = (double)Cx * (double)By, CyBx = (double)Cy * (double)Bx;
        double AxCy = (double)Ax * (double)Cy, AyCx = (double)Ay * (double)Cx;
        double BxAy = (double)Bx * (double)Ay, ByAx = (double)By * (double)Ax;
        U = (float)(CxBy - CyBx);
        V = (float)(AxCy - AyCx);
        W = (float)(BxAy - ByAx);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = U + V + W;
    if (det == 0.0f) return false;
    float Az = r.Sz * Akz, Bz = r.Sz * Bkz, Cz = r.Sz * Ckz;
    float T = U * Az + V * Bz + W * Cz;
    float rdet = 1.0f / det;
    float tt = T * rdet;
    if (!(tt > tmin)) return false;
    t = tt;
    u = V * rdet;
    v = W * rdet;
    return true;
}

// Slab test of one box; returns the entry distance or +inf on a miss.
// The exit distance gets a relative slack, so a triangle lying on a box face
// is never culled.  The bound tmax (the best hit so far) gets an absolute
// one, slack_abs: the triangle test's t carries an error of the order of the
// rounding of the scene coordinates, not of t, so without it a flat box
// could be culled against a hit whose t came out a few ulps of the
// coordinates short, and a tie between coplanar triangles would be decided
// by the tree instead of by the tie rule.
__device__ __forceinline__ float box_entry(const Ray& r, V3 lo, V3 hi, float tmin, float tmax, float slack_abs) {
    float tx0 = (lo.x - r.o.x) * r.inv.x, tx1 = (hi.x - r.o.x) * r.inv.x;
    float ty0 = (lo.y - r.o.y) * r.inv.y, ty1 = (hi.y - r.o.y) * r.inv.y;
    float tz0 = (lo.z - r.o.z) * r.inv.z, tz1 = (hi.z - r.o.z) * r.inv.z;
    float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), tmin));
    float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax + slack_abs));
    return tn <= tf * 1.0000005f ? tn : __builtin_inff();
}

// ---------------------------------------------------------------------------
// Material model: Lambert + GGX (Walter et al. 2007), separable Smith G1,
// alpha = roughness clamped to [1e-3, 1], no Fresnel.
// ---------------------------------------------------------------------------
struct Mat {
    V3 kd, ks;
    float alpha;   // raw value
};
__device__ __forceinline__ Mat load_mat(const float* p, int seg) {
    const float* m = p + 7 * seg;
    return Mat{v3(m[0], m[1], m[2]), v3(m[3], m[4], m[5]), m[6]};
}
__device__ __forceinline__ float clamp_alpha(float a) { return fminf(fmaxf(a, 1e-3f), 1.0f); }
__device__ __forceinline__ float alpha_live(float a) { return (a > 1e-3f && a < 1.0f) ? 1.0f : 0.0f; }
__device__ __forceinline__ float lum(V3 c) { return (c.x + c.y + c.z) * (1.0f / 3.0f); }

// GGX in the cancellation-free form a^2 / (pi (a^2 c^2 + s^2)^2), c = n.h,
// s^2 = |n x h|^2: near the lobe peak 1 - c^2 would lose all float32 digits.
__device__ __forceinline__ float ggx_D(float ch, float sh2, float a) {
    if (ch <= 0.0f) return 0.0f;
    float a2 = a * a, d = a2 * ch * ch + sh2;
    return a2 / (kPi * d * d);
}
__device__ __forceinline__ float ggx_dD(float ch, float sh2, float a) {
    if (ch <= 0.0f) return 0.0f;
    float a2 = a * a, d = a2 * ch * ch + sh2;
    return 2.0f * a * (sh2 - a2 * ch * ch) / (kPi * d * d * d);
}
__device__ __forceinline__ float sin2(V3 n, V3 h) {
    V3 c = cross(n, h);
    return dot(c, c);
}
__device__ __forceinline__ float smith_G1(float c, float a) {
    float s = sqrtf(a * a + (1.0f - a * a) * c * c);
    return 2.0f * c / (c + s);
}
__device__ __forceinline__ float smith_dG1(float c, float a) {
    float s = sqrtf(a * a + (1.0f - a * a) * c * c);
    return -2.0f * c * a * (1.0f - c * c) / (s * (c + s) * (c + s));
}

// spec = D G1 G1 / (4 co ci) (without ks) and d spec / d alpha.
__device__ __forceinline__ void spec_term(V3 n, V3 wo, V3 wi, float alpha_raw, float& spec,
                                          float& dspec) {
    float co = dot(n, wo), ci = dot(n, wi);
    spec = 0.0f;
    dspec = 0.0f;
    if (co <= 0.0f || ci <= 0.0f) return;
    V3 h = normalize(wo + wi);
    float ch = dot(n, h), sh2 = sin2(n, h);
    float a = clamp_alpha(alpha_raw);
    float D = ggx_D(ch, sh2, a), dD = ggx_dD(ch, sh2, a);
    float Go = smith_G1(co, a), Gi = smith_G1(ci, a);
    float dGo = smith_dG1(co, a), dGi = smith_dG1(ci, a);
    float rden = 1.0f / (4.0f * co * ci);
    spec = D * Go * Gi * rden;
    dspec = alpha_live(alpha_raw) * (dD * Go * Gi + D * dGo * Gi + D * Go * dGi) * rden;
}
__device__ __forceinline__ float spec_only(V3 n, V3 wo, V3 wi, float alpha_raw) {
    float co = dot(n, wo), ci = dot(n, wi);
    if (co <= 0.0f || ci <= 0.0f) return 0.0f;
    V3 h = normalize(wo + wi);
    float a = clamp_alpha(alpha_raw);
    return ggx_D(dot(n, h), sin2(n, h), a) * smith_G1(co, a) * smith_G1(ci, a) / (4.0f * co * ci);
}

__device__ __forceinline__ float lobe_prob(const Mat& m) {
    float ld = lum(m.kd), ls = lum(m.ks);
    if (ld + ls <= 0.0f) return 0.5f;
    return ls / (ld + ls);
}

// Solid-angle pdf of the lobe-mixture sampler.
__device__ __forceinline__ float brdf_pdf(const Mat& m, V3 n, V3 wo, V3 wi) {
    float ci = dot(n, wi), co = dot(n, wo);
    if (ci <= 0.0f || co <= 0.0f) return 0.0f;
    float ps = lobe_prob(m);
    float pd = ci * kInvPi;
    float pspec = 0.0f;
    V3 h = normalize(wo + wi);
    float ch = dot(n, h), oh = dot(wo, h);
    if (ch > 0.0f && oh > 0.0f) pspec = ggx_D(ch, sin2(n, h), clamp_alpha(m.alpha)) * ch / (4.0f * oh);
    return (1.0f - ps) * pd + ps * pspec;
}

// Orthonormal basis (Duff, Burgess, Christensen, Hery, Kensler, Liani,
// Villemin, JCGT 2017).
__device__ __forceinline__ void onb(V3 n, V3& t, V3& b) {
    float sg = n.z >= 0.0f ? 1.0f : -1.0f;
    float a = -1.0f / (sg + n.z);
    float bb = n.x * n.y * a;
    t = v3(1.0f + sg * n.x * n.x * a, sg * bb, -sg * n.x);
    b = v3(bb, sg + n.y * n.y * a, -n.y);
}

// Lobe mixture sampling: u3 selects the lobe, (u4,u5) the direction.
__device__ __forceinline__ bool brdf_sample(const Mat& m, V3 n, V3 wo, float u3, float u4, float u5,
                                            V3& wi, int& lobe) {
    V3 t, b;
    onb(n, t, b);
    float ps = lobe_prob(m);
    // sin/cos of 2 pi u5 without rounding the angle: 2 u5 is exact
    float s, c;
    sincospif(2.0f * u5, &s, &c);
    if (u3 < ps) {
        lobe = 1;
        float a = clamp_alpha(m.alpha);
        // Walter et al. 2007: tan^2 = a^2 u / (1 - u), cos^2 and sin^2 without
        // cancellation.  Their denominator 1 + (a^2 - 1) u is formed as
        // (1 - u) + a^2 u: 1 - u is exact for these 24-bit uniforms, while
        // rounding a^2 - 1 to float32 costs up to 6e-8 / den relative, 1e-3
        // for a near-mirror lobe (a ~ 5e-3) and u near 1
        float den = (1.0f - u4) + a * a * u4;
        float ch = sqrtf((1.0f - u4) / den), sh = sqrtf(a * a * u4 / den);
        V3 h = t * (sh * c) + b * (sh * s) + n * ch;
        float oh = dot(wo, h);
        if (oh <= 0.0f) return false;
        wi = h * (2.0f * oh) - wo;
    } else {
        lobe = 0;
        float r = sqrtf(u4), z = sqrtf(fmaxf(0.0f, 1.0f - u4));
        wi = t * (r * c) + b * (r * s) + n * z;
    }
    return true;
}

__device__ __forceinline__ float mis_weight(float a, float b, int mode) {
    if (mode == 3) { a *= a; b *= b; }
    return a / (a + b);
}

}  // namespace ipt
