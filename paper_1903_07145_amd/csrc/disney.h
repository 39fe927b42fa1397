// Disney material model (Burley 2012, "Physically-Based Shading at Disney";
// the paper's material, Sec. 4.1): base colour plus ten parameters meant to
// lie in [0, 1], 13 floats per segment in this order:
//   base r g b, subsurface, metallic, specular, specular tint, roughness,
//   anisotropic, sheen, sheen tint, clearcoat, clearcoat gloss.
// f = (1 - metallic) (base/pi mix(F_d, F_ss, subsurface) + sheen F_W(h.l)
//     C_sheen) + D_s F_s G_s / (4 n.l n.v) + clearcoat/4 D_c F_c G_c / (4 n.l n.v)
// with F_W(x) = (1 - x)^5; tint = base / lum(base), lum = 0.3 r + 0.6 g +
// 0.1 b (tint 1 when lum = 0); Burley's diffuse F_d with F_D90 = 1/2 + 2 r
// (h.l)^2; the subsurface term F_ss = 1.25 (F_90 product (1/(n.l + n.v) -
// 1/2) + 1/2) with F_90 = r (h.l)^2; anisotropic GGX D_s with a_x =
// max(1e-3, r^2 / k), a_y = max(1e-3, r^2 k), k = sqrt(1 - 0.9 anisotropic)
// and the matching anisotropic Smith G_s; F_s = mix(C_s0, 1, F_W(h.l)) with
// C_s0 = mix(0.08 specular mix(1, tint, specular tint), base, metallic);
// C_sheen = mix(1, tint, sheen tint); GTR1 clearcoat D_c with a =
// mix(0.1, 0.001, gloss), F_c = mix(0.04, 1, F_W(h.l)), G_c Smith with a =
// 0.25.  The tangent x is the hit triangle's first edge projected onto the
// plane of the shading normal, y = n x x.
//
// The evaluator is written once as a template over the scalar type: float
// for values, Dual (a value and one directional derivative, forward-mode
// differentiation) for the derivative with respect to one parameter.
#pragma once
#include "ipt_math.h"

namespace ipt {

constexpr int kDisneyParams = 13;
enum DisneyParam {
    kDsSubsurface = 3, kDsMetallic, kDsSpecular, kDsSpecTint, kDsRoughness, kDsAniso, kDsSheen, kDsSheenTint,
    kDsClearcoat, kDsCcGloss
};

struct Dual {
    float v, d;
    Dual() = default;
    __device__ __forceinline__ Dual(float v_, float d_ = 0.0f) : v(v_), d(d_) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual{a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator+(Dual a, float b) { return Dual{a.v + b, a.d}; }
__device__ __forceinline__ Dual operator+(float a, Dual b) { return Dual{a + b.v, b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual{a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, float b) { return Dual{a.v - b, a.d}; }
__device__ __forceinline__ Dual operator-(float a, Dual b) { return Dual{a - b.v, -b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual{a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, float b) { return Dual{a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator*(float a, Dual b) { return Dual{a * b.v, a * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const float q = a.v / b.v;
    return Dual{q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual operator/(Dual a, float b) { return Dual{a.v / b, a.d / b}; }
__device__ __forceinline__ Dual operator/(float a, Dual b) {
    const float q = a / b.v;
    return Dual{q, -q * b.d / b.v};
}
__device__ __forceinline__ Dual dsqrt(Dual a) {
    const float s = sqrtf(a.v);
    return Dual{s, a.d * 0.5f / s};
}
__device__ __forceinline__ float dsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ Dual dlog(Dual a) { return Dual{logf(a.v), a.d / a.v}; }
__device__ __forceinline__ float dlog(float a) { return logf(a); }
__device__ __forceinline__ float val(float a) { return a; }
__device__ __forceinline__ float val(Dual a) { return a.v; }
template <class T>
__device__ __forceinline__ T max_lo(T a, float lo) {
    return val(a) < lo ? T(lo) : a;
}

struct DMat {
    float p[kDisneyParams];
};
__device__ __forceinline__ DMat load_dmat(const float* p, int seg) {
    DMat m;
    const float* q = p + kDisneyParams * seg;
#pragma unroll
    for (int i = 0; i < kDisneyParams; ++i) m.p[i] = q[i];
    return m;
}

// Cosines and frame components of a (wo, wi) pair, in float.
struct DGeom {
    float ci, co, ch, cd, ix, iy, ox, oy, hx, hy, sh2;
    bool ok;
};

// Tangent frame: the first triangle edge projected onto the shading plane,
// or the branch-free basis of ipt_math.h when the edge is (nearly) along n.
__device__ __forceinline__ void disney_frame(V3 n, V3 e1, V3& x, V3& y) {
    V3 t = e1 - n * dot(n, e1);
    float lt = sqrtf(dot(t, t)), le = sqrtf(dot(e1, e1));
    if (lt > 1e-6f * le) {
        x = t * (1.0f / lt);
        y = cross(n, x);
    } else {
        onb(n, x, y);
    }
}

__device__ __forceinline__ DGeom disney_geom(V3 n, V3 x, V3 y, V3 wo, V3 wi) {
    DGeom g;
    g.ci = dot(n, wi);
    g.co = dot(n, wo);
    g.ok = g.ci > 0.0f && g.co > 0.0f;
    g.ch = g.cd = g.ix = g.iy = g.ox = g.oy = g.hx = g.hy = g.sh2 = 0.0f;
    if (!g.ok) return g;
    V3 h = normalize(wo + wi);
    g.ch = dot(n, h);
    g.cd = dot(wi, h);
    g.ix = dot(wi, x);
    g.iy = dot(wi, y);
    g.ox = dot(wo, x);
    g.oy = dot(wo, y);
    g.hx = dot(h, x);
    g.hy = dot(h, y);
    g.sh2 = sin2(n, h);
    return g;
}

__device__ __forceinline__ float schlick_w(float c) {
    float m = 1.0f - c;
    float m2 = m * m;
    return m2 * m2 * m;
}
template <class T>
__device__ __forceinline__ T g1_aniso(float c, float wx, float wy, T ax, T ay) {
    T tx = wx * ax, ty = wy * ay;
    return 2.0f * c / (c + dsqrt(c * c + tx * tx + ty * ty));
}
__device__ __forceinline__ float g1_iso(float c, float a) { return 2.0f * c / (c + sqrtf(a * a + (1.0f - a * a) * c * c)); }

// f (3 channels) for parameters p of scalar type T.
template <class T>
__device__ __forceinline__ void disney_f(const T* p, const DGeom& g, T f[3]) {
    T lum = 0.3f * p[0] + 0.6f * p[1] + 0.1f * p[2];
    const bool haslum = val(lum) > 0.0f;
    const float FL = schlick_w(g.ci), FV = schlick_w(g.co), FH = schlick_w(g.cd);
    const float cd2 = g.cd * g.cd;
    T r = p[kDsRoughness];
    T fd90 = 0.5f + 2.0f * cd2 * r;
    T fd = (1.0f + (fd90 - 1.0f) * FL) * (1.0f + (fd90 - 1.0f) * FV);
    T f90 = cd2 * r;
    T fss = 1.25f * ((1.0f + (f90 - 1.0f) * FL) * (1.0f + (f90 - 1.0f) * FV) * (1.0f / (g.ci + g.co) - 0.5f) + 0.5f);
    T diff = (fd + (fss - fd) * p[kDsSubsurface]) * kInvPi;
    T k = dsqrt(1.0f - 0.9f * p[kDsAniso]);
    T r2 = r * r;
    T ax = max_lo(r2 / k, 1e-3f), ay = max_lo(r2 * k, 1e-3f);
    T tx = g.hx / ax, ty = g.hy / ay;
    T dd = tx * tx + ty * ty + g.ch * g.ch;
    T Ds = 1.0f / (kPi * ax * ay * dd * dd);
    T Gs = g1_aniso(g.ci, g.ix, g.iy, ax, ay) * g1_aniso(g.co, g.ox, g.oy, ax, ay);
    T ac = 0.1f + (0.001f - 0.1f) * p[kDsCcGloss];
    T a2 = ac * ac;
    T Dc = (a2 - 1.0f) / (kPi * dlog(a2) * (g.ch * g.ch * a2 + g.sh2));
    const float Fc = 0.04f + 0.96f * FH;
    const float Gc = g1_iso(g.ci, 0.25f) * g1_iso(g.co, 0.25f);
    const float rden = 1.0f / (4.0f * g.ci * g.co);
    T spec = Ds * Gs * rden;
    T coat = (0.25f * Fc * Gc * rden) * p[kDsClearcoat] * Dc;
    T om = 1.0f - p[kDsMetallic];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T tint = haslum ? p[c] / lum : T(1.0f);
        T ts = 1.0f + (tint - 1.0f) * p[kDsSpecTint];
        T s0 = 0.08f * p[kDsSpecular] * ts;
        T cs0 = s0 + (p[c] - s0) * p[kDsMetallic];
        T Fs = cs0 + (1.0f - cs0) * FH;
        T sheen = FH * p[kDsSheen] * (1.0f + (tint - 1.0f) * p[kDsSheenTint]);
        f[c] = (diff * p[c] + sheen) * om + Fs * spec + coat;
    }
}

__device__ __forceinline__ V3 disney_value(const DMat& m, const DGeom& g) {
    if (!g.ok) return v3(0.0f, 0.0f, 0.0f);
    float f[3];
    disney_f<float>(m.p, g, f);
    return v3(f[0], f[1], f[2]);
}

// d f / d p_j (3 channels) by forward-mode differentiation.
__device__ __forceinline__ V3 disney_dparam(const DMat& m, const DGeom& g, int j) {
    Dual p[kDisneyParams];
#pragma unroll
    for (int i = 0; i < kDisneyParams; ++i) p[i] = Dual{m.p[i], i == j ? 1.0f : 0.0f};
    Dual f[3];
    disney_f<Dual>(p, g, f);
    return v3(f[0].d, f[1].d, f[2].d);
}

// Lobe probabilities of the sampler: diffuse (1 - metallic) lum(base),
// specular max(0.08 specular + (lum - 0.08 specular) metallic, 0.02),
// clearcoat 0.1 clearcoat; normalised.
__device__ __forceinline__ void disney_lobes(const DMat& m, float& pd, float& ps) {
    const float lum = 0.3f * m.p[0] + 0.6f * m.p[1] + 0.1f * m.p[2];
    const float sp = 0.08f * m.p[kDsSpecular];
    const float s0 = sp + (lum - sp) * m.p[kDsMetallic];
    const float wd = fmaxf(1.0f - m.p[kDsMetallic], 0.0f) * fmaxf(lum, 0.0f);
    const float ws = fmaxf(s0, 0.02f);
    const float wc = 0.1f * fmaxf(m.p[kDsClearcoat], 0.0f);
    const float inv = 1.0f / (wd + ws + wc);
    pd = wd * inv;
    ps = ws * inv;
}
__device__ __forceinline__ void disney_alphas(const DMat& m, float& ax, float& ay, float& ac) {
    const float r = m.p[kDsRoughness], k = sqrtf(1.0f - 0.9f * m.p[kDsAniso]);
    ax = fmaxf(r * r / k, 1e-3f);
    ay = fmaxf(r * r * k, 1e-3f);
    ac = 0.1f + (0.001f - 0.1f) * m.p[kDsCcGloss];
}

// Solid-angle pdf of the sampler for wi.
__device__ __forceinline__ float disney_pdf(const DMat& m, V3 n, V3 x, V3 y, V3 wo, V3 wi) {
    const float ci = dot(n, wi), co = dot(n, wo);
    if (ci <= 0.0f || co <= 0.0f) return 0.0f;
    float pd, ps, ax, ay, ac;
    disney_lobes(m, pd, ps);
    disney_alphas(m, ax, ay, ac);
    const float pc = 1.0f - pd - ps;
    V3 h = normalize(wo + wi);
    const float ch = dot(n, h), oh = dot(wo, h);
    float p = pd * ci * kInvPi;
    if (ch > 0.0f && oh > 0.0f) {
        const float tx = dot(h, x) / ax, ty = dot(h, y) / ay, dd = tx * tx + ty * ty + ch * ch;
        const float Ds = 1.0f / (kPi * ax * ay * dd * dd);
        const float a2 = ac * ac;
        const float Dc = (a2 - 1.0f) / (kPi * logf(a2) * (ch * ch * a2 + sin2(n, h)));
        p += (ps * Ds + pc * Dc) * ch / (4.0f * oh);
    }
    return p;
}

// Sample wi: u3 picks the lobe (0 diffuse, 1 specular, 2 clearcoat); (u4, u5)
// the direction: cosine hemisphere; anisotropic GGX normals (azimuth of
// (a_x cos 2 pi u5, a_y sin 2 pi u5), tan^2 theta_h = u4 / ((1 - u4) A),
// A = cos^2 phi / a_x^2 + sin^2 phi / a_y^2); GTR1 normals (cos^2 theta_h =
// (1 - a^(2 (1 - u4))) / (1 - a^2), azimuth 2 pi u5), reflected about wo.
// The forms keep float32 free of cancellation: 1 - u4 is exact for 24-bit
// uniforms, and GTR1's two powers go through expm1.
__device__ __forceinline__ bool disney_sample(const DMat& m, V3 n, V3 x, V3 y, V3 wo, float u3, float u4, float u5,
                                              V3& wi, int& lobe) {
    float pd, ps, ax, ay, ac;
    disney_lobes(m, pd, ps);
    disney_alphas(m, ax, ay, ac);
    float s, c;
    sincospif(2.0f * u5, &s, &c);
    if (u3 < pd) {
        lobe = 0;
        const float r = sqrtf(u4), z = sqrtf(fmaxf(0.0f, 1.0f - u4));
        wi = x * (r * c) + y * (r * s) + n * z;
        return true;
    }
    float ch, sh, cp, sp;
    if (u3 < pd + ps) {
        lobe = 1;
        const float vx = ax * c, vy = ay * s, lv = sqrtf(vx * vx + vy * vy);
        cp = vx / lv;
        sp = vy / lv;
        const float A = cp * cp / (ax * ax) + sp * sp / (ay * ay);
        const float den = (1.0f - u4) * A + u4;
        ch = sqrtf((1.0f - u4) * A / den);
        sh = sqrtf(u4 / den);
    } else {
        lobe = 2;
        const float L = logf(ac * ac), inv = 1.0f / (1.0f - ac * ac);
        ch = sqrtf(-expm1f((1.0f - u4) * L) * inv);
        sh = sqrtf(ac * ac * expm1f(-u4 * L) * inv);
        cp = c;
        sp = s;
    }
    V3 h = x * (sh * cp) + y * (sh * sp) + n * ch;
    const float oh = dot(wo, h);
    if (oh <= 0.0f) return false;
    wi = h * (2.0f * oh) - wo;
    return true;
}

}  // namespace ipt
