// Learned path-guiding proposal: batch evaluation, online training (bfloat16
// MFMA, float32 accumulation and float32 master weights) and the C ABI.
//
// Training follows the neural-importance-sampling objective (Mueller et al.,
// "Neural Importance Sampling", 2019): for records (vertex features, sampled
// direction w_i, weight r_i = target(w_i) / p_i with p_i the density it was
// sampled with) the loss  -sum_i r_i log q(w_i) / sum_i r_i  is a Monte Carlo
// estimate (up to a constant) of the KL divergence from the normalised target
// to the mixture q.  The target is the product BRDF x cosine x incident
// radiance; records come from the gradient pass of the tracer itself (see
// ipt_render_grad).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/ipt.h"
#include "guide_dev.h"
#include "ipt_internal.h"

namespace ipt {

constexpr int kRecF = 16;   // floats per training record
constexpr long long kMaxCacheCells = 1ll << 24;   // cached proposal: cells per side

// ---------------------------------------------------------------------------
// Requantisation: float32 master -> bfloat16 operand copies.
// ---------------------------------------------------------------------------
__global__ void guide_quantize_kernel(const float* w, const float* emb, int S, __bf16* wb, __bf16* embb) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    // t layouts: [N_pad][K_pad]
    if (i < kGHid * kGK1) {   // t1: 64 x 32
        int n = i / kGK1, k = i % kGK1;
        wb[kGT1 + i] = (__bf16)(k < kGIn ? w[kGW1 + k * kGHid + n] : 0.0f);
    }
    if (i < kGHid * kGHid) {
        int n = i / kGHid, k = i % kGHid;
        wb[kGT2 + i] = (__bf16)w[kGW2 + k * kGHid + n];
        wb[kGT3 + i] = (__bf16)w[kGW3 + k * kGHid + n];
        wb[kGT4 + i] = (__bf16)w[kGW4 + k * kGHid + n];
        // r layouts: [in][out]
        int in = i / kGHid, out = i % kGHid;
        wb[kGR2 + i] = (__bf16)w[kGW2 + in * kGHid + out];
        wb[kGR3 + i] = (__bf16)w[kGW3 + in * kGHid + out];
        wb[kGR4 + i] = (__bf16)w[kGW4 + in * kGHid + out];
        wb[kGR5 + i] = (__bf16)(out < kGOut ? w[kGW5 + in * kGOut + out] : 0.0f);
    }
    if (i < kGN5 * kGHid) {   // t5: 48 x 64
        int n = i / kGHid, k = i % kGHid;
        wb[kGT5 + i] = (__bf16)(n < kGOut ? w[kGW5 + k * kGOut + n] : 0.0f);
    }
    if (i < kGK1 * kGHid) {   // r1: 32 x 64
        int in = i / kGHid, out = i % kGHid;
        wb[kGR1 + i] = (__bf16)(in < kGIn ? w[kGW1 + in * kGHid + out] : 0.0f);
    }
    if (i < S * kGEmb) embb[i] = (__bf16)emb[i];
}

// ---------------------------------------------------------------------------
// Batch evaluation: feat [n][9], seg [n] -> mixture [n][40] (mu, kappa,
// weight per lobe).  mode 0: bfloat16 MFMA; 1: float32 VALU.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void guide_eval_kernel(GuideDev gd, const float* feat, const int* seg, int64_t n,
                                                          float* out) {
    __shared__ __align__(16) __bf16 act_all[4 * 64 * kGRowStride];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __bf16* act = act_all + wave * 64 * kGRowStride;
    for (int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64; base < n; base += (int64_t)gridDim.x * 256) {
        int64_t i = base + lane;
        bool ok = i < n;
        float f[9];
        int sg = 0;
        for (int j = 0; j < 9; ++j) f[j] = ok ? feat[9 * i + j] : 0.0f;
        if (ok) sg = seg[i];
        guide_put_inputs(gd, act, f, sg);
        guide_mlp_wave(gd, act);
        float* row = (float*)(act + lane * kGRowStride);
        mixture_from_raw(row);
        if (ok)
            for (int j = 0; j < kGOut; ++j) out[kGOut * i + j] = row[j];
    }
}

__global__ __launch_bounds__(256) void guide_eval_fp32_kernel(GuideDev gd, const float* feat, const int* seg,
                                                               int64_t n, float* out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float f[9];
        for (int j = 0; j < 9; ++j) f[j] = feat[9 * i + j];
        float* o = out + kGOut * i;
        guide_mlp_fp32(gd, f, seg[i], o);
        mixture_from_raw(o);
    }
}

// ---------------------------------------------------------------------------
// Cached proposal: cell table (count, scan) and rows (network per cell and
// side).  The query of a cell is its centroid, the shading normal there
// (geometric normal without vertex normals), both negated for the back side,
// and the outgoing direction taken along that normal.
// ---------------------------------------------------------------------------
__global__ void cell_count_kernel(const float4* tris, int64_t nt, float cell_area, int2* cells) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nt) return;
    const V3 p0 = xyz(tris[3 * t]), p1 = xyz(tris[3 * t + 1]), p2 = xyz(tris[3 * t + 2]);
    const int n = cell_subdiv(p1 - p0, p2 - p0, cell_area);
    cells[t] = make_int2(n * n, n);
}

// Exclusive scan of the cell counts (x) in place, in triangle order, by one
// block; *total = number of cells.
__global__ __launch_bounds__(1024) void cell_scan_kernel(int2* cells, int64_t nt, long long* total) {
    __shared__ long long part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (nt + 1023) / 1024;
    const int64_t b = min(nt, (int64_t)tid * per), e = min(nt, b + per);
    long long sum = 0;
    for (int64_t i = b; i < e; ++i) sum += cells[i].x;
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const long long v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    long long run = part[tid] - sum;
    for (int64_t i = b; i < e; ++i) {
        const int c = cells[i].x;
        cells[i].x = (int)run;
        run += c;
    }
    if (tid == 1023) *total = part[1023];
}

// Features and segment of cache row r (cell r / 2, side r % 2).
__device__ __forceinline__ void cell_query(const GuideDev& gd, const float4* tris, const float4* nrm, int64_t nt,
                                           int64_t r, float f[9], int& seg) {
    const int64_t c = r >> 1;
    int64_t lo = 0, hi = nt - 1;   // last triangle whose first cell is <= c
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)gd.cells[mid].x <= c) lo = mid;
        else hi = mid - 1;
    }
    const int64_t t = lo;
    const int2 cr = gd.cells[t];
    float u, v;
    cell_centroid((int)(c - cr.x), cr.y, u, v);
    const float4 a0 = tris[3 * t], a1 = tris[3 * t + 1], a2 = tris[3 * t + 2];
    const V3 p0 = xyz(a0), e1 = xyz(a1) - p0, e2 = xyz(a2) - p0;
    const V3 x = p0 + e1 * u + e2 * v;
    V3 ng = normalize(cross(e1, e2));
    V3 ns = ng;
    if (nrm) ns = normalize(xyz(nrm[3 * t]) * (1.0f - u - v) + xyz(nrm[3 * t + 1]) * u + xyz(nrm[3 * t + 2]) * v);
    if (r & 1) ns = ns * -1.0f;
    seg = __float_as_int(a1.w);
    guide_features(gd, x, ns, ns, f);
}

__global__ __launch_bounds__(256) void guide_cache_fill_kernel(GuideDev gd, const float4* tris, const float4* nrm,
                                                                int64_t nt, int64_t nrows, float* out) {
    __shared__ __align__(16) __bf16 act_all[4 * 64 * kGRowStride];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __bf16* act = act_all + wave * 64 * kGRowStride;
    for (int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64; base < nrows; base += (int64_t)gridDim.x * 256) {
        const int64_t r = base + lane;
        const bool ok = r < nrows;
        float f[9];
        int sg = 0;
        cell_query(gd, tris, nrm, nt, ok ? r : nrows - 1, f, sg);
        guide_put_inputs(gd, act, f, sg);
        guide_mlp_wave(gd, act);
        float* row = (float*)(act + lane * kGRowStride);
        mixture_from_raw(row);
        if (ok) write_cache_row(row, out + (size_t)r * kCacheRow);
    }
}

__global__ __launch_bounds__(256) void guide_cache_fill_fp32_kernel(GuideDev gd, const float4* tris,
                                                                     const float4* nrm, int64_t nt, int64_t nrows,
                                                                     float* out) {
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * 256) {
        float f[9], y[kGOut];
        int sg = 0;
        cell_query(gd, tris, nrm, nt, r, f, sg);
        guide_mlp_fp32(gd, f, sg, y);
        mixture_from_raw(y);
        write_cache_row(y, out + (size_t)r * kCacheRow);
    }
}

// ---------------------------------------------------------------------------
// Training.
// ---------------------------------------------------------------------------
struct TrainArgs {
    GuideDev gd;
    const float* rec;        // ring [cap][kRecF]
    int64_t nrec;            // valid records
    int batch;
    uint32_t key0, key1, step;
    int direct;              // 1: record b of the batch is record b (no sampling)
    float* wsum;             // [1] sum of record weights in the batch
    float* lsum;             // [1] sum of w log q
    float* gw;               // [kGParams] gradient
    float* gemb;             // [S][16] gradient
    float* part;             // [gridDim.x][kGParams] per-block weight and bias gradients
    int b0;                  // first batch position of this launch
};

// Records per training launch (one 64-record block each writes a partial
// gradient row; a fixed-order reduction sums them).
constexpr int kTrainChunkBlocks = 256;

__device__ __forceinline__ int64_t batch_index(const TrainArgs& t, int b) {
    if (t.direct) return b;
    uint4 r = philox(make_uint4((uint32_t)b, 0u, 7u, t.step), t.key0, t.key1);
    uint64_t x = ((uint64_t)r.x << 32) | r.y;
    return (int64_t)(x % (uint64_t)t.nrec);
}

__global__ void guide_wsum_kernel(TrainArgs t) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int b = blockIdx.x * 256 + threadIdx.x; b < t.batch; b += gridDim.x * 256)
        s += t.rec[kRecF * batch_index(t, b) + 7];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(t.wsum, red[0]);
}

// d(-log q)/dy for one record (40 raw outputs y, direction w), times scale.
__device__ void mixture_grad(const float* y, V3 w, float scale, float* dy, float* logq) {
    float mix[kGOut];
    for (int j = 0; j < kGOut; ++j) mix[j] = y[j];
    mixture_from_raw(mix);
    float pj[kGLobes], q = 0.0f;
    for (int j = 0; j < kGLobes; ++j) {
        const float* l = mix + 5 * j;
        pj[j] = vmf_pdf(l[3], l[0] * w.x + l[1] * w.y + l[2] * w.z);
        q += l[4] * pj[j];
    }
    q = fmaxf(q, 1e-30f);
    *logq = logf(q);
    for (int j = 0; j < kGLobes; ++j) {
        const float* l = mix + 5 * j;
        const float* r = y + 5 * j;
        float resp = l[4] * pj[j] / q;                     // responsibility
        float c = l[0] * w.x + l[1] * w.y + l[2] * w.z;
        float kap = l[3];
        // d log p / d kappa = mu.w - L(kappa), L = coth - 1/kappa (Langevin)
        float Lk = kap < 0.1f ? kap * (1.0f / 3.0f) - kap * kap * kap * (1.0f / 45.0f)
                              : 1.0f / tanhf(kap) - 1.0f / kap;
        float raw_k = softplus(r[3]) + 0.01f;
        float dk_dy = raw_k < 1e4f ? 1.0f / (1.0f + expf(-r[3])) : 0.0f;
        float dlogq_dy3 = resp * (c - Lk) * dk_dy;
        float dlogq_dy4 = resp - l[4];
        // d log q / d mu = resp kappa w; through mu = v / |v|
        float nv = sqrtf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
        if (nv > 0.0f) {
            float s = resp * kap / nv;
            g0 = s * (w.x - c * l[0]);
            g1 = s * (w.y - c * l[1]);
            g2 = s * (w.z - c * l[2]);
        }
        dy[5 * j + 0] = -scale * g0;
        dy[5 * j + 1] = -scale * g1;
        dy[5 * j + 2] = -scale * g2;
        dy[5 * j + 3] = -scale * dlogq_dy3;
        dy[5 * j + 4] = -scale * dlogq_dy4;
    }
}

// A operand from an LDS buffer read transposed: A[i][k] = buf[k][i].
__device__ __forceinline__ bf16x8 lds_col8(const __bf16* buf, int stride, int col, int row0) {
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = buf[(row0 + e) * stride + col];
    return v;
}

constexpr int kTS = 64;   // training LDS row stride (bf16)

// One wave (64 records) per block: forward, loss, backward.
__global__ __launch_bounds__(64) void guide_train_kernel(TrainArgs t) {
    // 56 KB: inputs, four hidden activations, and two gradient buffers that
    // also hold the float32 outputs during the forward pass
    __shared__ __align__(16) __bf16 X[64 * kTS];
    __shared__ __align__(16) __bf16 H[4][64 * kTS];
    __shared__ __align__(16) __bf16 D2[2 * 64 * kTS];
    __bf16* dA = D2;
    __bf16* dB = D2 + 64 * kTS;
    float* Y = (float*)D2;
    const int lane = threadIdx.x;
    const int li = lane & 15, lk = (lane >> 4) * 8;
    const GuideDev& gd = t.gd;
    const int b = t.b0 + blockIdx.x * 64 + lane;
    const bool ok = b < t.batch;
    float* part = t.part + (size_t)blockIdx.x * kGParams;
    const float* rc = t.rec + kRecF * (ok ? batch_index(t, b) : 0);
    int seg = ok ? __float_as_int(rc[3]) : 0;
    // inputs
    {
        float f[9] = {rc[0], rc[1], rc[2], rc[4], rc[5], rc[6], rc[8], rc[9], rc[10]};
        __bf16* row = X + lane * kTS;
        for (int i = 0; i < 9; ++i) row[i] = (__bf16)f[i];
        for (int i = 0; i < kGEmb; ++i) row[9 + i] = gd.embb[kGEmb * seg + i];
        for (int i = kGIn; i < kTS; ++i) row[i] = (__bf16)0.0f;
    }
    for (int i = lane; i < 2 * 64 * kTS; i += 64) D2[i] = (__bf16)0.0f;
    __syncthreads();
    // forward: H[l] = relu(in W + b)
    const __bf16* ins[5] = {X, H[0], H[1], H[2], H[3]};
    const int tw[5] = {kGT1, kGT2, kGT3, kGT4, kGT5};
    const int bs[5] = {kGB1, kGB2, kGB3, kGB4, kGB5};
    for (int l = 0; l < 5; ++l) {
        const int kpad = l == 0 ? kGK1 : kGHid, ksteps = l == 0 ? 1 : 2, nblk = l == 4 ? 3 : 4;
        const __bf16* in = ins[l];
        for (int qb = 0; qb < 4; ++qb) {
            f32x4 acc[4];
            for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            for (int ks = 0; ks < ksteps; ++ks) {
                bf16x8 a = *(const bf16x8*)(in + (qb * 16 + li) * kTS + ks * 32 + lk);
                for (int nb = 0; nb < nblk; ++nb) {
                    bf16x8 bb = *(const bf16x8*)(gd.wb + tw[l] + (nb * 16 + li) * kpad + ks * 32 + lk);
                    acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[nb], 0, 0, 0);
                }
            }
            for (int nb = 0; nb < nblk; ++nb) {
                int col = nb * 16 + li;
                for (int r = 0; r < 4; ++r) {
                    int row = qb * 16 + (lane >> 4) * 4 + r;
                    if (l < 4) {
                        float v = acc[nb][r] + gd.w[bs[l] + col];
                        H[l][row * kTS + col] = (__bf16)fmaxf(v, 0.0f);
                    } else if (col < kGOut) {
                        Y[row * kGOut + col] = acc[nb][r] + gd.w[bs[l] + col];
                    }
                }
            }
        }
        __syncthreads();
    }
    // loss and dY (bf16, padded to 64 columns) into dA
    {
        float yr[kGOut];
        for (int j = 0; j < kGOut; ++j) yr[j] = Y[lane * kGOut + j];
        __syncthreads();   // Y shares memory with dA
        float w = ok ? rc[7] / fmaxf(*t.wsum, 1e-30f) : 0.0f;
        float dy[kGOut], lq = 0.0f;
        mixture_grad(yr, v3(rc[12], rc[13], rc[14]), w, dy, &lq);
        float wl = (ok && w > 0.0f) ? w * lq : 0.0f;
        for (int o = 32; o >= 1; o >>= 1) wl += __shfl_xor(wl, o, 64);
        if (lane == 0 && wl != 0.0f) atomicAdd(t.lsum, wl);
        __bf16* row = dA + lane * kTS;
        for (int j = 0; j < 64; ++j) row[j] = (__bf16)((ok && j < kGOut) ? dy[j] : 0.0f);
    }
    __syncthreads();
    // backward, layer l = 4 .. 0; dA holds dZ_l (pre-activation gradient)
    const int rw[5] = {kGR1, kGR2, kGR3, kGR4, kGR5};
    const int gwo[5] = {kGW1, kGW2, kGW3, kGW4, kGW5};
    __bf16* dz = dA;
    __bf16* dn = dB;
    for (int l = 4; l >= 0; --l) {
        const int nout = l == 4 ? kGOut : kGHid;
        const int nin = l == 0 ? kGIn : kGHid;
        const __bf16* in = ins[l];
        // bias gradient: column sums of dz
        if (lane < nout) {
            float s = 0.0f;
            for (int q = 0; q < 64; ++q) s += (float)dz[q * kTS + lane];
            part[bs[l] + lane] = s;
        }
        // dW[in][out] = sum_q in[q][in] dz[q][out]: A = in^T (M = inputs), B = dz (K = queries)
        const int mblk = l == 0 ? 2 : 4, nblk = l == 4 ? 3 : 4;
        for (int ib = 0; ib < mblk; ++ib) {
            f32x4 acc[4];
            for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            for (int ks = 0; ks < 2; ++ks) {
                bf16x8 a = lds_col8(in, kTS, ib * 16 + li, ks * 32 + lk);
                for (int nb = 0; nb < nblk; ++nb) {
                    bf16x8 bb = lds_col8(dz, kTS, nb * 16 + li, ks * 32 + lk);
                    acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[nb], 0, 0, 0);
                }
            }
            for (int nb = 0; nb < nblk; ++nb) {
                int col = nb * 16 + li;
                for (int r = 0; r < 4; ++r) {
                    int row = ib * 16 + (lane >> 4) * 4 + r;
                    if (row < nin && col < nout) part[gwo[l] + row * nout + col] = acc[nb][r];
                }
            }
        }
        // d(in) = dz W^T: A = dz (K = outputs), B[k = out][n = in] = W[in][out] (r layout)
        const int kpad_out = l == 4 ? kGN5r : kGHid;
        const int nblk_in = l == 0 ? 2 : 4;
        for (int qb = 0; qb < 4; ++qb) {
            f32x4 acc[4];
            for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            for (int ks = 0; ks < 2; ++ks) {
                bf16x8 a = *(const bf16x8*)(dz + (qb * 16 + li) * kTS + ks * 32 + lk);
                for (int nb = 0; nb < nblk_in; ++nb) {
                    bf16x8 bb = *(const bf16x8*)(gd.wb + rw[l] + (nb * 16 + li) * kpad_out + ks * 32 + lk);
                    acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[nb], 0, 0, 0);
                }
            }
            for (int nb = 0; nb < nblk_in; ++nb) {
                int col = nb * 16 + li;
                for (int r = 0; r < 4; ++r) {
                    int row = qb * 16 + (lane >> 4) * 4 + r;
                    float v = acc[nb][r];
                    if (l > 0) {
                        // through the ReLU of the layer below
                        float hv = (float)ins[l][row * kTS + col];
                        dn[row * kTS + col] = (__bf16)(hv > 0.0f ? v : 0.0f);
                    } else if (col >= 9 && col < kGIn) {
                        int rb = blockIdx.x * 64 + row;
                        if (rb < t.batch) {
                            int sg = __float_as_int(t.rec[kRecF * batch_index(t, rb) + 3]);
                            atomicAdd(t.gemb + kGEmb * sg + (col - 9), v);
                        }
                    }
                }
            }
        }
        __syncthreads();
        __bf16* tmp = dz;
        dz = dn;
        dn = tmp;
        // pad columns beyond the layer width stay zero: clear dn for the next round
        for (int i = lane; i < 64 * kTS; i += 64) dn[i] = (__bf16)0.0f;
        __syncthreads();
    }
}

__global__ void guide_adam_kernel(float* p, const float* g, float* m, float* v, int n, float lr, float c1, float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = 0.9f * m[i] + 0.1f * gi;
    float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

__global__ void neg_copy_kernel(const float* src, float* dst) { dst[0] = -src[0]; }

// Appends n caller records at the ring position the counter holds (read
// only here; a second launch advances it).
__global__ void guide_append_kernel(const float* src, int64_t n, float* ring, const unsigned* count, int cap) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * kRecF) return;
    int64_t r = i / kRecF;
    uint64_t slot = ((uint64_t)*count + (uint64_t)r) % (uint64_t)cap;
    ring[slot * kRecF + (i - r * kRecF)] = src[i];
}

__global__ void guide_count_add_kernel(unsigned* count, unsigned n) { *count += n; }

__global__ void zero_f32_kernel(float* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

}  // namespace ipt

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------
using namespace ipt;

struct ipt_guide_s {
    int S = 0;
    float3 lo{0, 0, 0}, inv{1, 1, 1};
    float* w = nullptr;       // params [kGParams] then embedding [S*16] (contiguous)
    float* m = nullptr;
    float* v = nullptr;
    float* g = nullptr;       // gradient, same layout
    __bf16* wb = nullptr;     // [kGBf16]
    __bf16* embb = nullptr;   // [S*16]
    float* rec = nullptr;     // ring [cap][kRecF]
    unsigned* rec_count = nullptr;
    float* scal = nullptr;    // [0] wsum, [1] lsum
    float* gpart = nullptr;   // [kTrainChunkBlocks][kGParams] per-block training gradients
    int cap = 0, batch = 0, stride = 1;
    float lr = 1e-3f;
    uint64_t seed = 0;
    int step = 0;
    float last_loss = 0.0f;
    // cached proposal (ipt_guide_cache_build)
    const void* cache_scene = nullptr;
    int64_t cache_nt = 0;
    float cache_area = 0.0f;
    int2* cells = nullptr;            // per leaf-ordered triangle: (first cell, n)
    float* cache = nullptr;           // [2 cache_cells][kCacheRow]
    long long* cache_total = nullptr;
    int64_t cache_cells = 0;
};

extern "C" const char* ipt_last_error(void);
ipt_status ipt_fail(ipt_status s, const char* msg);

GuideDev guide_dev(const ipt_guide_s* g) {
    GuideDev d;
    d.w = g->w;
    d.emb = g->w + kGParams;
    d.wb = g->wb;
    d.embb = g->embb;
    d.lo = g->lo;
    d.inv = g->inv;
    d.cache = g->cache;
    d.cells = g->cells;
    return d;
}
int guide_cache_ready(const ipt_guide_s* g, const void* scene) { return g->cache && g->cache_scene == scene; }
float* guide_records(ipt_guide_s* g) { return g->rec; }
unsigned* guide_record_count(ipt_guide_s* g) { return g->rec_count; }
int guide_capacity(const ipt_guide_s* g) { return g->cap; }
int guide_record_stride(const ipt_guide_s* g) { return g->stride; }

static hipError_t requantize(ipt_guide_s* g, hipStream_t st) {
    int n = kGHid * kGHid;
    if (g->S * kGEmb > n) n = g->S * kGEmb;
    hipLaunchKernelGGL(guide_quantize_kernel, dim3((n + 255) / 256), dim3(256), 0, st, g->w, g->w + kGParams, g->S,
                       g->wb, g->embb);
    return hipGetLastError();
}

// Host-side initial weights: He-normal hidden layers from a Philox stream
// (Box-Muller), a small output layer so the initial mixture is broad.
static void init_weights(std::vector<float>& w, int S, uint64_t seed) {
    uint32_t k0 = (uint32_t)seed ^ 0x51ED270Bu, k1 = (uint32_t)(seed >> 32);
    uint32_t ctr = 0;
    auto philox_h = [&](uint32_t c) {
        uint32_t x0 = c, x1 = 0, x2 = 0x6A09E667u, x3 = 0, a0 = k0, a1 = k1;
        for (int r = 0; r < 10; ++r) {
            uint64_t p0 = (uint64_t)0xD2511F53u * x0, p1 = (uint64_t)0xCD9E8D57u * x2;
            uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ a0, n2 = (uint32_t)(p0 >> 32) ^ x3 ^ a1;
            x1 = (uint32_t)p1; x3 = (uint32_t)p0; x0 = n0; x2 = n2;
            a0 += 0x9E3779B9u; a1 += 0xBB67AE85u;
        }
        return std::make_pair(x0, x1);
    };
    auto gauss = [&]() {
        auto r = philox_h(ctr++);
        double u1 = ((r.first >> 8) + 0.5) / 16777216.0, u2 = (r.second >> 8) / 16777216.0;
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    w.assign(kGParams + (size_t)S * kGEmb, 0.0f);
    auto fill = [&](int off, int fan_in, int n, double gain) {
        double sd = gain * std::sqrt(2.0 / fan_in);
        for (int i = 0; i < n; ++i) w[off + i] = (float)(sd * gauss());
    };
    fill(kGW1, kGIn, kGIn * kGHid, 1.0);
    fill(kGW2, kGHid, kGHid * kGHid, 1.0);
    fill(kGW3, kGHid, kGHid * kGHid, 1.0);
    fill(kGW4, kGHid, kGHid * kGHid, 1.0);
    fill(kGW5, kGHid, kGHid * kGOut, 0.05);
    for (int j = 0; j < kGLobes; ++j) w[kGB5 + 5 * j + 3] = -1.0f;   // kappa starts near 0.3
    for (int i = 0; i < S * kGEmb; ++i) w[kGParams + i] = (float)(0.1 * gauss());
}

ipt_status guide_create_impl(int S, const float lo[3], const float hi[3], const ipt_guide_opts* o, void* stream,
                             ipt_guide_t* out) {
    ipt_guide_s* g = new ipt_guide_s();
    g->S = S;
    g->lo = make_float3(lo[0], lo[1], lo[2]);
    g->inv = make_float3(1.0f / std::max(hi[0] - lo[0], 1e-6f), 1.0f / std::max(hi[1] - lo[1], 1e-6f),
                         1.0f / std::max(hi[2] - lo[2], 1e-6f));
    g->cap = o->ring_capacity;
    g->batch = o->batch;
    g->stride = std::max(1, o->record_stride);
    g->lr = o->lr;
    g->seed = o->seed;
    size_t np = kGParams + (size_t)S * kGEmb;
    std::vector<float> w0;
    init_weights(w0, S, o->seed);
    hipError_t e = hipSuccess;
    auto al = [&](void** p, size_t b) { if (e == hipSuccess) e = hipMalloc(p, b); };
    al((void**)&g->w, np * 4);
    al((void**)&g->m, np * 4);
    al((void**)&g->v, np * 4);
    al((void**)&g->g, np * 4);
    al((void**)&g->wb, (size_t)kGBf16 * 2);
    al((void**)&g->embb, (size_t)S * kGEmb * 2 + 16);
    al((void**)&g->rec, (size_t)g->cap * kRecF * 4);
    al((void**)&g->rec_count, 64);
    al((void**)&g->scal, 64);
    al((void**)&g->gpart, (size_t)kTrainChunkBlocks * kGParams * 4);
    if (e == hipSuccess) e = hipMemcpy(g->w, w0.data(), np * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(g->m, 0, np * 4);
    if (e == hipSuccess) e = hipMemset(g->v, 0, np * 4);
    if (e == hipSuccess) e = hipMemset(g->wb, 0, (size_t)kGBf16 * 2);
    if (e == hipSuccess) e = hipMemset(g->rec_count, 0, 64);
    if (e == hipSuccess) e = requantize(g, (hipStream_t)stream);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        ipt_guide_free(g);
        return ipt_fail(e == hipErrorOutOfMemory ? IPT_ERR_OUT_OF_MEMORY : IPT_ERR_HIP, hipGetErrorString(e));
    }
    *out = g;
    return IPT_OK;
}

extern "C" ipt_status ipt_guide_free(ipt_guide_t g) {
    if (!g) return IPT_OK;
    hipFree(g->w); hipFree(g->m); hipFree(g->v); hipFree(g->g);
    hipFree(g->wb); hipFree(g->embb); hipFree(g->rec); hipFree(g->rec_count); hipFree(g->scal);
    hipFree(g->gpart);
    hipFree(g->cells); hipFree(g->cache); hipFree(g->cache_total);
    delete g;
    return IPT_OK;
}

// Cell table (when the scene or the cell area changed: allocates) and rows
// (every call: refilled from the current weights; allocates nothing).
ipt_status guide_cache_build_impl(ipt_guide_s* g, const void* scene, const float4* tris, const float4* nrm,
                                  int64_t nt, float cell_area, int mode, hipStream_t st, int64_t* ncells) {
    if (!(cell_area > 0.0f) || !std::isfinite(cell_area) || (mode != 0 && mode != 1) || nt < 1)
        return ipt_fail(IPT_ERR_INVALID_ARG, "guide cache: cell_area > 0, mode 0 or 1, non-empty scene");
    hipError_t e = hipSuccess;
    if (!g->cache || g->cache_scene != scene || g->cache_nt != nt || g->cache_area != cell_area) {
        hipFree(g->cells); hipFree(g->cache); hipFree(g->cache_total);
        g->cells = nullptr; g->cache = nullptr; g->cache_total = nullptr;
        g->cache_scene = nullptr; g->cache_cells = 0;
        e = hipMalloc((void**)&g->cells, sizeof(int2) * (size_t)nt);
        if (e == hipSuccess) e = hipMalloc((void**)&g->cache_total, 64);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(cell_count_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, tris, nt,
                               cell_area, g->cells);
            hipLaunchKernelGGL(cell_scan_kernel, dim3(1), dim3(1024), 0, st, g->cells, nt, g->cache_total);
            e = hipGetLastError();
        }
        long long total = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&total, g->cache_total, sizeof(total), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess && total > kMaxCacheCells) {
            hipFree(g->cells); hipFree(g->cache_total);
            g->cells = nullptr; g->cache_total = nullptr;
            return ipt_fail(IPT_ERR_INVALID_ARG, "guide cache: more than 2^24 cells; use a larger cell_area");
        }
        if (e == hipSuccess) e = hipMalloc((void**)&g->cache, sizeof(float) * kCacheRow * 2 * (size_t)total);
        if (e != hipSuccess)
            return ipt_fail(e == hipErrorOutOfMemory ? IPT_ERR_OUT_OF_MEMORY : IPT_ERR_HIP, hipGetErrorString(e));
        g->cache_scene = scene;
        g->cache_nt = nt;
        g->cache_area = cell_area;
        g->cache_cells = total;
    }
    const int64_t nrows = 2 * g->cache_cells;
    const int blocks = (int)std::min<int64_t>((nrows + 255) / 256, 8192);
    if (mode == 0)
        hipLaunchKernelGGL(guide_cache_fill_kernel, dim3(blocks), dim3(256), 0, st, guide_dev(g), tris, nrm, nt,
                           nrows, g->cache);
    else
        hipLaunchKernelGGL(guide_cache_fill_fp32_kernel, dim3(blocks), dim3(256), 0, st, guide_dev(g), tris, nrm,
                           nt, nrows, g->cache);
    e = hipGetLastError();
    if (e != hipSuccess) return ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
    if (ncells) *ncells = g->cache_cells;
    return IPT_OK;
}

extern "C" ipt_status ipt_guide_eval(ipt_guide_t g, const float* feat, const int32_t* seg, int64_t n, int32_t mode,
                                     float* out, void* stream) {
    if (!g || !feat || !seg || !out || n < 0 || (mode != 0 && mode != 1))
        return ipt_fail(IPT_ERR_INVALID_ARG, "bad guide eval arguments");
    if (n == 0) return IPT_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (mode == 0)
        hipLaunchKernelGGL(guide_eval_kernel, dim3((int)blocks), dim3(256), 0, (hipStream_t)stream, guide_dev(g), feat,
                           seg, n, out);
    else
        hipLaunchKernelGGL(guide_eval_fp32_kernel, dim3((int)blocks), dim3(256), 0, (hipStream_t)stream,
                           guide_dev(g), feat, seg, n, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? IPT_OK : ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
}

// grad[i] += sum over blocks of part[block][i], i < kGParams (fixed order).
__global__ void guide_part_reduce_kernel(const float* part, int nblocks, float* grad) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kGParams) return;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * kGParams + i];
    grad[i] += s;
}

// Loss and gradient of one batch into grad [np]; scal[0] = sum of weights,
// scal[1] = sum_b (w_b / sum w) log q_b.
static void launch_loss_grad(ipt_guide_s* g, const float* rec, int64_t nrec, int batch, int direct, float* grad,
                             hipStream_t st) {
    size_t np = kGParams + (size_t)g->S * kGEmb;
    TrainArgs t;
    t.gd = guide_dev(g);
    t.rec = rec;
    t.nrec = nrec;
    t.batch = batch;
    t.key0 = (uint32_t)g->seed ^ 0xA5A5A5A5u;
    t.key1 = (uint32_t)(g->seed >> 32);
    t.step = (uint32_t)g->step;
    t.direct = direct;
    t.wsum = g->scal;
    t.lsum = g->scal + 1;
    t.gw = grad;
    t.gemb = grad + kGParams;
    t.part = g->gpart;
    hipLaunchKernelGGL(zero_f32_kernel, dim3((int)((np + 255) / 256)), dim3(256), 0, st, grad, (int)np);
    hipLaunchKernelGGL(zero_f32_kernel, dim3(1), dim3(64), 0, st, g->scal, 2);
    hipLaunchKernelGGL(guide_wsum_kernel, dim3(64), dim3(256), 0, st, t);
    const int chunk = kTrainChunkBlocks * 64;
    for (int b0 = 0; b0 < t.batch; b0 += chunk) {
        t.b0 = b0;
        const int nb = (std::min(chunk, t.batch - b0) + 63) / 64;
        hipLaunchKernelGGL(guide_train_kernel, dim3(nb), dim3(64), 0, st, t);
        hipLaunchKernelGGL(guide_part_reduce_kernel, dim3((kGParams + 255) / 256), dim3(256), 0, st, g->gpart, nb,
                           grad);
    }
}

extern "C" ipt_status ipt_guide_loss_grad(ipt_guide_t g, const float* rec, int64_t n, float* loss, float* grad,
                                          void* stream) {
    if (!g || !rec || !loss || !grad || n < 1 || n > (1 << 24))
        return ipt_fail(IPT_ERR_INVALID_ARG, "bad guide loss_grad arguments (1 <= n <= 2^24)");
    hipStream_t st = (hipStream_t)stream;
    launch_loss_grad(g, rec, n, (int)n, 1, grad, st);
    hipLaunchKernelGGL(neg_copy_kernel, dim3(1), dim3(1), 0, st, g->scal + 1, loss);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? IPT_OK : ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
}

extern "C" ipt_status ipt_guide_add_records(ipt_guide_t g, const float* rec, int64_t n, void* stream) {
    if (!g || (!rec && n > 0) || n < 0 || n > g->cap)
        return ipt_fail(IPT_ERR_INVALID_ARG, "bad record count (0 <= n <= ring capacity)");
    if (n == 0) return IPT_OK;
    hipStream_t st = (hipStream_t)stream;
    int64_t tot = n * kRecF;
    hipLaunchKernelGGL(guide_append_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, rec, n, g->rec,
                       g->rec_count, g->cap);
    hipLaunchKernelGGL(guide_count_add_kernel, dim3(1), dim3(1), 0, st, g->rec_count, (unsigned)n);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? IPT_OK : ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
}

extern "C" ipt_status ipt_guide_read_records(ipt_guide_t g, float* out, int64_t n, void* stream) {
    if (!g || (!out && n > 0) || n < 0 || n > g->cap)
        return ipt_fail(IPT_ERR_INVALID_ARG, "bad record count (0 <= n <= ring capacity)");
    if (n == 0) return IPT_OK;
    hipError_t e = hipMemcpyAsync(out, g->rec, (size_t)n * kRecF * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? IPT_OK : ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
}

extern "C" ipt_status ipt_guide_train(ipt_guide_t g, int32_t steps, float* loss_out, void* stream) {
    if (!g || steps < 0) return ipt_fail(IPT_ERR_INVALID_ARG, "bad guide train arguments");
    hipStream_t st = (hipStream_t)stream;
    unsigned cnt = 0;
    hipError_t e = hipMemcpy(&cnt, g->rec_count, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
    int64_t nrec = std::min<int64_t>(cnt, g->cap);
    if (nrec < 64) return ipt_fail(IPT_ERR_INVALID_ARG, "too few training records in the ring");
    size_t np = kGParams + (size_t)g->S * kGEmb;
    float lsum_tot = 0.0f;
    for (int s = 0; s < steps; ++s) {
        launch_loss_grad(g, g->rec, nrec, g->batch, 0, g->g, st);
        g->step++;
        float c1 = (float)(1.0 - std::pow(0.9, g->step)), c2 = (float)(1.0 - std::pow(0.999, g->step));
        hipLaunchKernelGGL(guide_adam_kernel, dim3((int)((np + 255) / 256)), dim3(256), 0, st, g->w, g->g, g->m,
                           g->v, (int)np, g->lr, c1, c2);
        e = requantize(g, st);
        if (e != hipSuccess) return ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
        if (loss_out && s == steps - 1) {
            float sc[2];
            e = hipMemcpyAsync(sc, g->scal, 8, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
            lsum_tot = -sc[1];
        }
    }
    if (loss_out) *loss_out = lsum_tot;
    e = hipGetLastError();
    return e == hipSuccess ? IPT_OK : ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
}

extern "C" ipt_status ipt_guide_weights(ipt_guide_t g, float* host_out, int32_t get, int64_t count) {
    if (!g || !host_out) return ipt_fail(IPT_ERR_INVALID_ARG, "NULL argument");
    size_t np = kGParams + (size_t)g->S * kGEmb;
    if (count != (int64_t)np) return ipt_fail(IPT_ERR_INVALID_ARG, "count must equal 16744 + 16 S");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = get ? hipMemcpy(host_out, g->w, np * 4, hipMemcpyDeviceToHost)
                : hipMemcpy(g->w, host_out, np * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && !get) e = requantize(g, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e == hipSuccess ? IPT_OK : ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
}

extern "C" ipt_status ipt_guide_records(ipt_guide_t g, int64_t* count) {
    if (!g || !count) return ipt_fail(IPT_ERR_INVALID_ARG, "NULL argument");
    unsigned c = 0;
    hipError_t e = hipMemcpy(&c, g->rec_count, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ipt_fail(IPT_ERR_HIP, hipGetErrorString(e));
    *count = c;
    return IPT_OK;
}
