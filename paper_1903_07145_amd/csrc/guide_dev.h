// Learned path-guiding proposal: device side.
//
// A small MLP maps the features of a path vertex -- position normalised to
// the scene box ([-1,1]^3), shading normal, outgoing direction -- and a
// learned 16-d embedding of the vertex's segment to an 8-lobe von
// Mises-Fisher mixture over incident directions.  It is combined with BRDF
// sampling by one-sample MIS (Veach 1997): a direction is drawn from the
// mixture with probability c, from the BRDF otherwise, and weighted by the
// combined density c q + (1 - c) p_brdf, which is positive wherever the
// integrand is, so the estimator stays unbiased whatever the network says.
//
// Network: 25 -> 64 -> 64 -> 64 -> 64 -> 40, ReLU; per lobe j the outputs
// y[5j..5j+4] give mu = normalise(y[0..2]), kappa = softplus(y[3]) + 0.01
// (at most 1e4) and the mixture weight softmax(y[4]).
// vMF density: kappa / (2 pi (1 - exp(-2 kappa))) exp(kappa (mu.w - 1));
// sampling: w = 1 + log(u + (1 - u) exp(-2 kappa)) / kappa (Wenzel Jakob,
// "Numerically stable sampling of the von Mises Fisher distribution on S2",
// 2012), azimuth uniform.
#pragma once
#include <hip/hip_runtime.h>

#include "ipt_math.h"

namespace ipt {

constexpr int kGIn = 25;       // 9 features + 16 embedding
constexpr int kGEmb = 16;
constexpr int kGHid = 64;
constexpr int kGOut = 40;      // 8 lobes x (mu 3, kappa 1, logit 1)
constexpr int kGLobes = 8;
// float32 master parameter block: W1 [25][64], b1, W2..W4 [64][64], b2..b4, W5 [64][40], b5
constexpr int kGW1 = 0;
constexpr int kGB1 = kGW1 + kGIn * kGHid;
constexpr int kGW2 = kGB1 + kGHid;
constexpr int kGB2 = kGW2 + kGHid * kGHid;
constexpr int kGW3 = kGB2 + kGHid;
constexpr int kGB3 = kGW3 + kGHid * kGHid;
constexpr int kGW4 = kGB3 + kGHid;
constexpr int kGB4 = kGW4 + kGHid * kGHid;
constexpr int kGW5 = kGB4 + kGHid;
constexpr int kGB5 = kGW5 + kGHid * kGOut;
constexpr int kGParams = kGB5 + kGOut;   // 16744
// bfloat16 operand copies for MFMA, per layer: "t" = [N_pad][K_pad] (row =
// output neuron), "r" = [K_pad][N_pad] (row = input unit, for backward).
constexpr int kGK1 = 32;                 // layer-1 input padded to one K step
constexpr int kGN5 = 48;                 // layer-5 outputs padded to 3 tiles of 16
constexpr int kGN5r = 64;                // ... and to 2 K steps for the backward
constexpr int kGT1 = 0;                               // t1: 64 x 32
constexpr int kGT2 = kGT1 + kGHid * kGK1;             // t2..t4: 64 x 64
constexpr int kGT3 = kGT2 + kGHid * kGHid;
constexpr int kGT4 = kGT3 + kGHid * kGHid;
constexpr int kGT5 = kGT4 + kGHid * kGHid;            // t5: 48 x 64
constexpr int kGTEnd = kGT5 + kGN5 * kGHid;
constexpr int kGR2 = kGTEnd;                          // r2..r4: 64 x 64
constexpr int kGR3 = kGR2 + kGHid * kGHid;
constexpr int kGR4 = kGR3 + kGHid * kGHid;
constexpr int kGR5 = kGR4 + kGHid * kGHid;            // r5: 64 x 64 (cols >= 40 zero)
constexpr int kGR1 = kGR5 + kGHid * kGN5r;            // r1: 32 x 64 (rows >= 25 zero)
constexpr int kGBf16 = kGR1 + kGK1 * kGHid;
constexpr int kGRowStride = 80;   // LDS activation row: 64 bf16 + pad (bank spread); 160 B holds 40 f32

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Cached proposal: the network evaluated once per surface cell and side.
// Cells cut a triangle's barycentric domain into n^2 sub-triangles, n the
// smallest integer in [1, kCellMaxN] with area / n^2 <= cell_area; a row
// per (cell, side) holds the cell's mixture ready for the path kernels.
// Row layout (48 float32, 192 B): per lobe j (mu xyz, kappa) at 4 j, then
// lw[8] = log(weight_j * kappa_j / (2 pi (1 - e^{-2 kappa_j}))) at 32, then
// the cumulative weights cw[8] at 40.  Density: sum_j exp(kappa_j (mu_j.w
// - 1) + lw_j), one exponential per lobe.
constexpr int kCacheRow = 48;
constexpr int kCellMaxN = 64;

struct GuideDev {
    const float* w;          // float32 master parameters [kGParams]
    const float* emb;        // [S][16]
    const __bf16* wb;        // bfloat16 copies [kGBf16]
    const __bf16* embb;      // [S][16] bfloat16
    float3 lo, inv;          // scene box: p_n = 2 (p - lo) * inv - 1
    const float* cache;      // cached proposal rows [2 cells][kCacheRow] or NULL
    const int2* cells;       // per leaf-ordered triangle: (first cell, n)
};

__device__ __forceinline__ float softplus(float x) { return x > 20.0f ? x : log1pf(expf(x)); }

// vMF density kappa / (2 pi (1 - e^{-2 kappa})) e^{kappa (c - 1)}, c = mu.w.
// Hardware exponentials (v_exp_f32, relative error ~1e-6 here) and a fast
// divide: the density is evaluated for 8 lobes twice per guided vertex, and
// the library expf / expm1f cost several times more.  kappa >= 0.01 keeps
// 1 - e^{-2 kappa} >= 0.0198, so the subtraction loses no more than ~3e-6.
__device__ __forceinline__ float vmf_pdf(float kappa, float c) {
    return __fdividef(kappa, 2.0f * kPi * (1.0f - __expf(-2.0f * kappa))) * __expf(kappa * (c - 1.0f));
}

// Mixture stored per lobe as (mu.xyz, kappa, weight).
__device__ __forceinline__ float mixture_pdf(const float* mix, V3 w) {
    float q = 0.0f;
#pragma unroll
    for (int j = 0; j < kGLobes; ++j) {
        const float* l = mix + 5 * j;
        q += l[4] * vmf_pdf(l[3], l[0] * w.x + l[1] * w.y + l[2] * w.z);
    }
    return q;
}

// Lobe by u3, then the vMF sample by (u4, u5).
__device__ __forceinline__ V3 mixture_sample(const float* mix, float u3, float u4, float u5) {
    int j = kGLobes - 1;
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < kGLobes; ++i) {
        acc += mix[5 * i + 4];
        if (u3 < acc) { j = i; break; }
    }
    const float* l = mix + 5 * j;
    V3 mu = v3(l[0], l[1], l[2]);
    float kappa = l[3];
    float w = 1.0f + log1pf(-(1.0f - u4) * -expm1f(-2.0f * kappa)) / kappa;
    w = fminf(fmaxf(w, -1.0f), 1.0f);
    float sw = sqrtf(fmaxf(0.0f, 1.0f - w * w));
    float s, c;
    sincospif(2.0f * u5, &s, &c);
    V3 t, b;
    onb(mu, t, b);
    return t * (sw * c) + b * (sw * s) + mu * w;
}

// Raw network outputs -> mixture parameters (in place, 40 floats).
__device__ __forceinline__ void mixture_from_raw(float* y) {
    float mx = -3.4e38f;
#pragma unroll
    for (int j = 0; j < kGLobes; ++j) mx = fmaxf(mx, y[5 * j + 4]);
    float z = 0.0f;
#pragma unroll
    for (int j = 0; j < kGLobes; ++j) {
        float* l = y + 5 * j;
        float n2 = l[0] * l[0] + l[1] * l[1] + l[2] * l[2];
        float rn = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
        if (n2 > 0.0f) { l[0] *= rn; l[1] *= rn; l[2] *= rn; } else { l[0] = 0.0f; l[1] = 0.0f; l[2] = 1.0f; }
        l[3] = fminf(softplus(l[3]) + 0.01f, 1e4f);
        l[4] = __expf(l[4] - mx);
        z += l[4];
    }
    float rz = 1.0f / z;
#pragma unroll
    for (int j = 0; j < kGLobes; ++j) y[5 * j + 4] *= rz;
}

// Input features of a vertex (the 9 geometric ones).
__device__ __forceinline__ void guide_features(const GuideDev& gd, V3 x, V3 n, V3 wo, float f[9]) {
    f[0] = 2.0f * (x.x - gd.lo.x) * gd.inv.x - 1.0f;
    f[1] = 2.0f * (x.y - gd.lo.y) * gd.inv.y - 1.0f;
    f[2] = 2.0f * (x.z - gd.lo.z) * gd.inv.z - 1.0f;
    f[3] = n.x; f[4] = n.y; f[5] = n.z;
    f[6] = wo.x; f[7] = wo.y; f[8] = wo.z;
}

// Float32 evaluation on VALU, one query per lane (the reference mode used
// for parity with the float64 oracle; not the fast path).  out: 40 raw
// outputs.  noinline keeps its activation arrays out of the callers'
// register allocation.
__device__ __noinline__ void guide_mlp_fp32(const GuideDev& gd, const float f[9], int seg, float* out) {
    float x[kGIn];
    for (int i = 0; i < 9; ++i) x[i] = f[i];
    for (int i = 0; i < kGEmb; ++i) x[9 + i] = gd.emb[kGEmb * seg + i];
    float h[kGHid], g[kGHid];
    for (int n = 0; n < kGHid; ++n) {
        float s = gd.w[kGB1 + n];
        for (int k = 0; k < kGIn; ++k) s += x[k] * gd.w[kGW1 + k * kGHid + n];
        h[n] = fmaxf(s, 0.0f);
    }
    const int W[3] = {kGW2, kGW3, kGW4}, B[3] = {kGB2, kGB3, kGB4};
    for (int l = 0; l < 3; ++l) {
        for (int n = 0; n < kGHid; ++n) {
            float s = gd.w[B[l] + n];
            for (int k = 0; k < kGHid; ++k) s += h[k] * gd.w[W[l] + k * kGHid + n];
            g[n] = fmaxf(s, 0.0f);
        }
        for (int n = 0; n < kGHid; ++n) h[n] = g[n];
    }
    for (int n = 0; n < kGOut; ++n) {
        float s = gd.w[kGB5 + n];
        for (int k = 0; k < kGHid; ++k) s += h[k] * gd.w[kGW5 + k * kGOut + n];
        out[n] = s;
    }
}

// ---------------------------------------------------------------------------
// Wave-cooperative bfloat16 MFMA evaluation (float32 accumulation) of the 64
// queries of one wave.  act: this wave's LDS rows [64][kGRowStride] bf16;
// row q holds lane q's 25 inputs (bf16, zero padded to 32) on entry and its
// 40 raw outputs (float32) on exit.  All 64 lanes must be active.
//
// v_mfma_f32_16x16x32_bf16 lane layout (gfx950): A[i][k] with i = lane%16,
// k = (lane/16)*8 + e for the 8 elements e a lane holds; B[k][n] with n =
// lane%16 and the same k; D[i][n] with n = lane%16, i = 4*(lane/16) + r.
// Rows are independent, so each 16-query block is written back in place.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bf16x8 lds_row8(const __bf16* act, int row, int col) {
    return *(const bf16x8*)(act + row * kGRowStride + col);
}

template <int KSTEPS, int NBLK>
__device__ __forceinline__ void mfma_layer(__bf16* act, const __bf16* wt, int kpad, const float* bias, bool relu,
                                           float* outf) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = (lane >> 4) * 8;
    for (int qb = 0; qb < 4; ++qb) {
        f32x4 acc[NBLK];
#pragma unroll
        for (int nb = 0; nb < NBLK; ++nb) acc[nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            bf16x8 a = lds_row8(act, qb * 16 + li, ks * 32 + lk);
#pragma unroll
            for (int nb = 0; nb < NBLK; ++nb) {
                bf16x8 b = *(const bf16x8*)(wt + (nb * 16 + li) * kpad + ks * 32 + lk);
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nb], 0, 0, 0);
            }
        }
        // results of this query block replace its rows
#pragma unroll
        for (int nb = 0; nb < NBLK; ++nb) {
            const int col = nb * 16 + li;
            const float bv = bias[col < (outf ? kGOut : kGHid) ? col : 0];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = qb * 16 + (lane >> 4) * 4 + r;
                float v = acc[nb][r] + bv;
                if (outf) {
                    if (col < kGOut) ((float*)(act + row * kGRowStride))[col] = v;
                } else {
                    act[row * kGRowStride + col] = (__bf16)(relu ? fmaxf(v, 0.0f) : v);
                }
            }
        }
    }
}

__device__ __noinline__ void guide_mlp_wave(const GuideDev& gd, __bf16* act) {
    mfma_layer<1, 4>(act, gd.wb + kGT1, kGK1, gd.w + kGB1, true, nullptr);
    mfma_layer<2, 4>(act, gd.wb + kGT2, kGHid, gd.w + kGB2, true, nullptr);
    mfma_layer<2, 4>(act, gd.wb + kGT3, kGHid, gd.w + kGB3, true, nullptr);
    mfma_layer<2, 4>(act, gd.wb + kGT4, kGHid, gd.w + kGB4, true, nullptr);
    // the output layer writes float32 rows of 40 (160 B fit a row)
    mfma_layer<2, 3>(act, gd.wb + kGT5, kGHid, gd.w + kGB5, false, (float*)act);
}

// Writes lane's bf16 input row (25 values, zero padded to 32).
__device__ __forceinline__ void guide_put_inputs(const GuideDev& gd, __bf16* act, const float f[9], int seg) {
    const int lane = threadIdx.x & 63;
    __bf16* row = act + lane * kGRowStride;
#pragma unroll
    for (int i = 0; i < 9; ++i) row[i] = (__bf16)f[i];
#pragma unroll
    for (int i = 0; i < kGEmb; ++i) row[9 + i] = gd.embb[kGEmb * seg + i];
#pragma unroll
    for (int i = kGIn; i < kGK1; ++i) row[i] = (__bf16)0.0f;
}

// ---------------------------------------------------------------------------
// Cached proposal.
// ---------------------------------------------------------------------------
// Subdivision of a triangle with edges e1, e2: the smallest n in [1,
// kCellMaxN] with |e1 x e2| <= 2 n^2 cell_area, decided in float32 with a
// fixed operation order and no contraction (squared, so no square root).
__device__ __forceinline__ int cell_subdiv(V3 e1, V3 e2, float cell_area) {
#pragma clang fp contract(off)
    const float cx = e1.y * e2.z - e1.z * e2.y;
    const float cy = e1.z * e2.x - e1.x * e2.z;
    const float cz = e1.x * e2.y - e1.y * e2.x;
    const float a2 = (cx * cx + cy * cy) + cz * cz;
    const float two = 2.0f * cell_area;
    int n = 1;
    for (; n < kCellMaxN; ++n) {
        const float q = (float)(n * n) * two;
        if (q * q >= a2) break;
    }
    return n;
}

// Cell of barycentrics (u, v) (x = p0 + u e1 + v e2) in a triangle cut into
// n^2 sub-triangles: grid square (i, j) = (floor(n u), floor(n v)), lower
// half (fractions summing to <= 1) or upper half; row i holds 2 (n - i) - 1
// cells starting at 2 n i - i^2, lower half j at 2 j, upper half at 2 j + 1.
__device__ __forceinline__ int cell_of(float u, float v, int n) {
    const float x = u * (float)n, y = v * (float)n;
    int i = min(max((int)x, 0), n - 1);
    int j = min(max((int)y, 0), n - 1 - i);
    const float fx = x - (float)i, fy = y - (float)j;
    const int up = (i + j < n - 1 && fx + fy > 1.0f) ? 1 : 0;
    return 2 * n * i - i * i + 2 * j + up;
}

// Barycentric centroid of cell c of an n^2 subdivision.
__device__ __forceinline__ void cell_centroid(int c, int n, float& u, float& v) {
    int i = 0;
    while (c >= 2 * (n - i) - 1) {
        c -= 2 * (n - i) - 1;
        ++i;
    }
    const int j = c >> 1;
    const float o = (c & 1) ? (2.0f / 3.0f) : (1.0f / 3.0f);
    u = ((float)i + o) / (float)n;
    v = ((float)j + o) / (float)n;
}

// Row of the cached proposal for a hit on leaf-ordered triangle tri at (u,
// v), seen from its back side (geometric normal facing away) when back.
__device__ __forceinline__ const float* cache_row_at(const GuideDev& gd, int tri, float u, float v, bool back) {
    const int2 cr = gd.cells[tri];
    const int64_t c = (int64_t)cr.x + cell_of(u, v, cr.y);
    return gd.cache + (size_t)(2 * c + (back ? 1 : 0)) * kCacheRow;
}

// The row is read lobe by lobe (not unrolled): the path kernels keep their
// state in registers, and holding all 48 values would spill it.
__device__ __forceinline__ float cached_pdf(const float* row, V3 w) {
    const float4* r = (const float4*)row;
    float q = 0.0f;
#pragma unroll 1
    for (int j = 0; j < kGLobes; ++j) {
        const float4 m = r[j];
        q += __expf(m.w * ((m.x * w.x + m.y * w.y + m.z * w.z) - 1.0f) + row[32 + j]);
    }
    return q;
}

// Densities of two directions in one pass over the row (each lobe read
// once): the continuation direction and the light sample of a vertex.
#ifndef IPT_CACHE_UNROLL
#define IPT_CACHE_UNROLL 2
#endif
__device__ __forceinline__ void cached_pdf2(const float* row, V3 w1, V3 w2, float& q1, float& q2) {
    const float4* r = (const float4*)row;
    float a = 0.0f, b = 0.0f;
#pragma unroll IPT_CACHE_UNROLL
    for (int j = 0; j < kGLobes; ++j) {
        const float4 m = r[j];
        const float lw = row[32 + j];
        a += __expf(m.w * ((m.x * w1.x + m.y * w1.y + m.z * w1.z) - 1.0f) + lw);
        b += __expf(m.w * ((m.x * w2.x + m.y * w2.y + m.z * w2.z) - 1.0f) + lw);
    }
    q1 = a;
    q2 = b;
}

// Lobe by u3 against the cumulative weights, then the vMF sample by (u4, u5)
// (the same steps as mixture_sample).
__device__ __forceinline__ V3 cached_sample(const float* row, float u3, float u4, float u5) {
    const float4* r = (const float4*)row;
    const float4 c0 = r[10], c1 = r[11];
    int j = kGLobes - 1;
    if (u3 < c1.z) j = 6;
    if (u3 < c1.y) j = 5;
    if (u3 < c1.x) j = 4;
    if (u3 < c0.w) j = 3;
    if (u3 < c0.z) j = 2;
    if (u3 < c0.y) j = 1;
    if (u3 < c0.x) j = 0;
    const float4 m = r[j];
    V3 mu = v3(m.x, m.y, m.z);
    const float kappa = m.w;
    float w = 1.0f + log1pf(-(1.0f - u4) * -expm1f(-2.0f * kappa)) / kappa;
    w = fminf(fmaxf(w, -1.0f), 1.0f);
    const float sw = sqrtf(fmaxf(0.0f, 1.0f - w * w));
    float s, c;
    sincospif(2.0f * u5, &s, &c);
    V3 t, b;
    onb(mu, t, b);
    return t * (sw * c) + b * (sw * s) + mu * w;
}

// Mixture (per lobe mu xyz, kappa, weight) -> cached row.
__device__ __forceinline__ void write_cache_row(const float* mix, float* out) {
    float4* o = (float4*)out;
    float lw[8], cw[8];
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < kGLobes; ++j) {
        const float* l = mix + 5 * j;
        const float kappa = l[3];
        o[j] = make_float4(l[0], l[1], l[2], kappa);
        lw[j] = logf(l[4]) + logf(kappa / (2.0f * kPi * (-expm1f(-2.0f * kappa))));
        acc += l[4];
        cw[j] = acc;
    }
    o[8] = make_float4(lw[0], lw[1], lw[2], lw[3]);
    o[9] = make_float4(lw[4], lw[5], lw[6], lw[7]);
    o[10] = make_float4(cw[0], cw[1], cw[2], cw[3]);
    o[11] = make_float4(cw[4], cw[5], cw[6], cw[7]);
}

}  // namespace ipt
