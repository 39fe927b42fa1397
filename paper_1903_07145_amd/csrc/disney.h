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
// disney_value evaluates f; disney_grad is its adjoint, written out by hand
// (reverse mode): for a channel weight w it returns w . d f / d p_j for all
// 13 parameters in one pass that costs about two evaluations.
#pragma once
#include "ipt_math.h"

namespace ipt {

constexpr int kDisneyParams = 13;
enum DisneyParam {
    kDsSubsurface = 3, kDsMetallic, kDsSpecular, kDsSpecTint, kDsRoughness, kDsAniso, kDsSheen, kDsSheenTint,
    kDsClearcoat, kDsCcGloss
};

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
__device__ __forceinline__ float g1_aniso(float c, float wx, float wy, float ax, float ay) {
    const float tx = wx * ax, ty = wy * ay;
    return 2.0f * c / (c + sqrtf(c * c + tx * tx + ty * ty));
}
__device__ __forceinline__ float g1_iso(float c, float a) { return 2.0f * c / (c + sqrtf(a * a + (1.0f - a * a) * c * c)); }

// f (3 channels) for parameters p.
__device__ __forceinline__ void disney_f(const float* p, const DGeom& g, float f[3]) {
    const float lum = 0.3f * p[0] + 0.6f * p[1] + 0.1f * p[2];
    const bool haslum = lum > 0.0f;
    const float FL = schlick_w(g.ci), FV = schlick_w(g.co), FH = schlick_w(g.cd);
    const float cd2 = g.cd * g.cd;
    const float r = p[kDsRoughness];
    const float fd90 = 0.5f + 2.0f * cd2 * r;
    const float fd = (1.0f + (fd90 - 1.0f) * FL) * (1.0f + (fd90 - 1.0f) * FV);
    const float f90 = cd2 * r;
    const float fss = 1.25f * ((1.0f + (f90 - 1.0f) * FL) * (1.0f + (f90 - 1.0f) * FV) * (1.0f / (g.ci + g.co) - 0.5f) + 0.5f);
    const float diff = (fd + (fss - fd) * p[kDsSubsurface]) * kInvPi;
    const float k = sqrtf(1.0f - 0.9f * p[kDsAniso]);
    const float r2 = r * r;
    const float ax = fmaxf(r2 / k, 1e-3f), ay = fmaxf(r2 * k, 1e-3f);
    const float tx = g.hx / ax, ty = g.hy / ay;
    const float dd = tx * tx + ty * ty + g.ch * g.ch;
    const float Ds = 1.0f / (kPi * ax * ay * dd * dd);
    const float Gs = g1_aniso(g.ci, g.ix, g.iy, ax, ay) * g1_aniso(g.co, g.ox, g.oy, ax, ay);
    const float ac = 0.1f + (0.001f - 0.1f) * p[kDsCcGloss];
    const float a2 = ac * ac;
    const float Dc = (a2 - 1.0f) / (kPi * logf(a2) * (g.ch * g.ch * a2 + g.sh2));
    const float Fc = 0.04f + 0.96f * FH;
    const float Gc = g1_iso(g.ci, 0.25f) * g1_iso(g.co, 0.25f);
    const float rden = 1.0f / (4.0f * g.ci * g.co);
    const float spec = Ds * Gs * rden;
    const float coat = (0.25f * Fc * Gc * rden) * p[kDsClearcoat] * Dc;
    const float om = 1.0f - p[kDsMetallic];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float tint = haslum ? p[c] / lum : 1.0f;
        const float ts = 1.0f + (tint - 1.0f) * p[kDsSpecTint];
        const float s0 = 0.08f * p[kDsSpecular] * ts;
        const float cs0 = s0 + (p[c] - s0) * p[kDsMetallic];
        const float Fs = cs0 + (1.0f - cs0) * FH;
        const float sheen = FH * p[kDsSheen] * (1.0f + (tint - 1.0f) * p[kDsSheenTint]);
        f[c] = (diff * p[c] + sheen) * om + Fs * spec + coat;
    }
}

__device__ __forceinline__ V3 disney_value(const DMat& m, const DGeom& g) {
    if (!g.ok) return v3(0.0f, 0.0f, 0.0f);
    float f[3];
    disney_f(m.p, g, f);
    return v3(f[0], f[1], f[2]);
}

// Adjoint of f: G[j] = sum_c w_c d f_c / d p_j for all 13 parameters, the
// forward quantities of disney_f followed by one reverse sweep.  A clamped
// quantity (alpha at 1e-3, tint at lum = 0) passes no derivative.
__device__ __forceinline__ void disney_grad(const DMat& m, const DGeom& g, V3 wv, float G[kDisneyParams]) {
#pragma unroll
    for (int j = 0; j < kDisneyParams; ++j) G[j] = 0.0f;
    if (!g.ok) return;
    const float* p = m.p;
    const float w[3] = {wv.x, wv.y, wv.z};
    // ---- forward ----
    const float lum = 0.3f * p[0] + 0.6f * p[1] + 0.1f * p[2];
    const bool haslum = lum > 0.0f;
    const float FL = schlick_w(g.ci), FV = schlick_w(g.co), FH = schlick_w(g.cd);
    const float cd2 = g.cd * g.cd;
    const float r = p[kDsRoughness];
    const float fd90 = 0.5f + 2.0f * cd2 * r;
    const float AL = 1.0f + (fd90 - 1.0f) * FL, AV = 1.0f + (fd90 - 1.0f) * FV;
    const float fd = AL * AV;
    const float f90 = cd2 * r;
    const float BL = 1.0f + (f90 - 1.0f) * FL, BV = 1.0f + (f90 - 1.0f) * FV;
    const float Q = 1.0f / (g.ci + g.co) - 0.5f;
    const float fss = 1.25f * (BL * BV * Q + 0.5f);
    const float sub = p[kDsSubsurface];
    const float diff = (fd + (fss - fd) * sub) * kInvPi;
    const float k = sqrtf(1.0f - 0.9f * p[kDsAniso]);
    const float r2 = r * r;
    const float axr = r2 / k, ayr = r2 * k;
    const bool axl = axr >= 1e-3f, ayl = ayr >= 1e-3f;   // unclamped: derivatives pass
    const float ax = axl ? axr : 1e-3f, ay = ayl ? ayr : 1e-3f;
    const float tx = g.hx / ax, ty = g.hy / ay;
    const float dd = tx * tx + ty * ty + g.ch * g.ch;
    const float Ds = 1.0f / (kPi * ax * ay * dd * dd);
    const float qix = g.ix * ax, qiy = g.iy * ay, qox = g.ox * ax, qoy = g.oy * ay;
    const float si = sqrtf(g.ci * g.ci + qix * qix + qiy * qiy), so = sqrtf(g.co * g.co + qox * qox + qoy * qoy);
    const float G1i = 2.0f * g.ci / (g.ci + si), G1o = 2.0f * g.co / (g.co + so);
    const float Gs = G1i * G1o;
    const float ac = 0.1f + (0.001f - 0.1f) * p[kDsCcGloss];
    const float a2 = ac * ac;
    const float L = logf(a2);
    const float E = g.ch * g.ch * a2 + g.sh2;
    const float Dc = (a2 - 1.0f) / (kPi * L * E);
    const float Fc = 0.04f + 0.96f * FH;
    const float Gc = g1_iso(g.ci, 0.25f) * g1_iso(g.co, 0.25f);
    const float rden = 1.0f / (4.0f * g.ci * g.co);
    const float spec = Ds * Gs * rden;
    const float kc = 0.25f * Fc * Gc * rden;
    const float met = p[kDsMetallic], om = 1.0f - met;
    const float spc = p[kDsSpecular], stint = p[kDsSpecTint], sh = p[kDsSheen], shtint = p[kDsSheenTint];
    // ---- reverse ----
    float dp[3] = {0.0f, 0.0f, 0.0f};
    float dspec = 0.0f, ddiff = 0.0f, dlum = 0.0f;
    float gmet = 0.0f, gspc = 0.0f, gstint = 0.0f, gsh = 0.0f, gshtint = 0.0f;
    const float W = w[0] + w[1] + w[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float pc = p[c];
        const float tint = haslum ? pc / lum : 1.0f;
        const float ts = 1.0f + (tint - 1.0f) * stint;
        const float s0 = 0.08f * spc * ts;
        const float cs0 = s0 + (pc - s0) * met;
        const float Fs = cs0 + (1.0f - cs0) * FH;
        const float shf = 1.0f + (tint - 1.0f) * shtint;
        const float sheen = FH * sh * shf;
        // f_c = (diff p_c + sheen_c) om + Fs_c spec + coat
        const float X = w[c] * om;
        gmet -= w[c] * (diff * pc + sheen);
        ddiff += X * pc;
        dp[c] += X * diff;
        dspec += w[c] * Fs;
        const float dcs0 = w[c] * spec * (1.0f - FH);
        const float ds0 = dcs0 * om;
        dp[c] += dcs0 * met;
        gmet += dcs0 * (pc - s0);
        gspc += ds0 * 0.08f * ts;
        const float dts = ds0 * 0.08f * spc;
        gstint += dts * (tint - 1.0f);
        float dtint = dts * stint;
        gsh += X * FH * shf;
        gshtint += X * FH * sh * (tint - 1.0f);
        dtint += X * FH * sh * shtint;
        if (haslum) {
            dp[c] += dtint / lum;
            dlum -= dtint * tint / lum;
        }
    }
    dp[0] += 0.3f * dlum;
    dp[1] += 0.6f * dlum;
    dp[2] += 0.1f * dlum;
    // coat = kc p_cc Dc(ac), ac = 0.1 + (0.001 - 0.1) p_gloss
    const float gcc = W * kc * Dc;
    const float dDc = W * kc * p[kDsClearcoat];
    const float dDc_da2 = Dc * (1.0f / (a2 - 1.0f) - 1.0f / (a2 * L) - g.ch * g.ch / E);
    const float ggloss = dDc * dDc_da2 * 2.0f * ac * (0.001f - 0.1f);
    // spec = Ds Gs rden
    const float dDs = dspec * Gs * rden, dGs = dspec * Ds * rden;
    const float dax = dDs * Ds * (4.0f * tx * tx / dd - 1.0f) / ax
                    - dGs * (G1o * G1i * g.ix * g.ix * ax / (si * (g.ci + si)) + G1i * G1o * g.ox * g.ox * ax / (so * (g.co + so)));
    const float day = dDs * Ds * (4.0f * ty * ty / dd - 1.0f) / ay
                    - dGs * (G1o * G1i * g.iy * g.iy * ay / (si * (g.ci + si)) + G1i * G1o * g.oy * g.oy * ay / (so * (g.co + so)));
    float dr2 = 0.0f, dk = 0.0f;
    if (axl) { dr2 += dax / k; dk -= dax * axr / k; }
    if (ayl) { dr2 += day * k; dk += day * r2; }
    // diff = (fd (1 - sub) + fss sub) / pi
    const float gsub = ddiff * (fss - fd) * kInvPi;
    const float dfd = ddiff * (1.0f - sub) * kInvPi, dfss = ddiff * sub * kInvPi;
    const float dfd90 = dfd * (AV * FL + AL * FV);
    const float df90 = dfss * 1.25f * Q * (BV * FL + BL * FV);
    const float dr = dr2 * 2.0f * r + dfd90 * 2.0f * cd2 + df90 * cd2;
    G[0] = dp[0];
    G[1] = dp[1];
    G[2] = dp[2];
    G[kDsSubsurface] = gsub;
    G[kDsMetallic] = gmet;
    G[kDsSpecular] = gspc;
    G[kDsSpecTint] = gstint;
    G[kDsRoughness] = dr;
    G[kDsAniso] = dk * (-0.45f / k);
    G[kDsSheen] = gsh;
    G[kDsSheenTint] = gshtint;
    G[kDsClearcoat] = gcc;
    G[kDsCcGloss] = ggloss;
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
