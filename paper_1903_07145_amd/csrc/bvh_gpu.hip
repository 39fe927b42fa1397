// Binned SAH BVH build and scene layout on the GPU (gfx950).
//
// Split rule: the binned surface-area heuristic of Wald (2007, "On fast
// construction of SAH-based bounding volume hierarchies").  The centroids of
// a node's triangles fall into 64 equal slabs per axis; each of the 3 x 63
// slab boundaries costs A_L N_L + A_R N_R (C_trav = C_isect = 1) and the
// cheapest one wins (first minimum in axis order, then slab order).  A node
// whose centroids coincide is cut at its median position, and nodes of at
// most two triangles are leaves.  This is the rule of the host builder, so
// both produce the same tree.
//
// Two regimes:
//  * a node of more than 1024 triangles ("large") is split one tree level at
//    a time by passes spread over blocks of 1024 triangles: bin counts and
//    bounds are formed in LDS and merged with global atomics, one wave costs
//    the 189 candidate planes (one lane per axis), the partition is stable
//    (per-chunk left counts, prefix-summed on the host) and the child bounds
//    are reduced from the partitioned triangles;
//  * a node of at most 1024 triangles is finished by one block: its triangle
//    ids stay in LDS while the block walks the subtree, continuing with the
//    smaller child and pushing the larger one; the node held at least
//    halves with every push and only nodes above the leaf size are pushed,
//    so the stack never holds more than log2(1024 / 3) + 1 < 11 entries.
// The depth-first child-pair layout is then found in parallel: every
// subtree's internal-node count bottom-up (the second child to finish
// completes its parent), then each internal node's preorder position by one
// walk to the root: one slot per ancestor, plus the internal nodes of the
// left subtree of every ancestor it lies to the right of.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "bvh_gpu.h"

namespace ipt {

namespace {

// 64 slabs per axis: against 32, the apartment's rays visit 14.5 instead of
// 15.0 nodes and a step takes 1.7% less time (256 slabs: 1.9%, at three
// times the build time)
constexpr int kBins = 64;
constexpr int kAxBins = 3 * kBins;          // slabs over the three axes
constexpr int kBinWords = kAxBins * 7;      // count, lo xyz, hi xyz per slab
constexpr int kLoOff = kAxBins;             // [kLoOff + 3 s + j]: slab s lower bound on axis j
constexpr int kHiOff = kAxBins * 4;         // [kHiOff + 3 s + j]: upper bound
// Leaves of at most two triangles: against four, the apartment's rays test
// 4.05 instead of 8.14 triangles for 16.2 instead of 14.8 node visits, and a
// step takes 7% less time (one-triangle leaves: 7% more).
constexpr int kMaxLeaf = 2;
constexpr int kTB = 256;                    // threads per build block
constexpr int kWaves = kTB / 64;
constexpr int kSmallMax = 1024;             // nodes finished by one block
constexpr int kChunk = 1024;                // triangles per block in the large passes
constexpr int kSmallStack = 32;
constexpr int kNoChild = 0x7FFFFFFF;
constexpr float kInf = __builtin_huge_valf();

struct alignas(16) GNode {   // binary node while building
    float lo[3];
    int left;                // child ids, -1 at a leaf
    float hi[3];
    int right;
    int first, count, parent, depth;
};

struct LTask {               // a large node split at the current level
    int node, first, count, depth;
    float cblo[3], cbhi[3];  // centroid bounds
};
struct Chunk {
    int task, start, end, left_before;   // left_before: left triangles of the task's earlier chunks
};
struct Decision {
    int axis, split, nleft, pad;         // axis < 0: median cut
};
struct STask {
    int node, first, count, depth;
};

// Order-preserving map of floats to unsigned ints (min/max by integer atomics).
__device__ __forceinline__ unsigned ordf(float f) {
    unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unordf(unsigned u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}
float unordf_host(unsigned u) {
    unsigned v = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    float f;
    std::memcpy(&f, &v, 4);
    return f;
}

__device__ __forceinline__ float comp(const float4& v, int a) { return a == 0 ? v.x : (a == 1 ? v.y : v.z); }

__device__ __forceinline__ float wave_min(float x) {
    for (int o = 32; o >= 1; o >>= 1) x = fminf(x, __shfl_xor(x, o, 64));
    return x;
}
__device__ __forceinline__ float wave_max(float x) {
    for (int o = 32; o >= 1; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
    return x;
}
__device__ __forceinline__ int wave_sum(int x) {
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ __forceinline__ double wave_sum(double x) {
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Slab of centroid coordinate c on an axis with lower bound lo and scale
// k = kBins / extent; clamped into [0, kBins - 1] (NaN from a degenerate extent -> 0).
__device__ __forceinline__ int slab(float c, float lo, float k) {
    float x = (c - lo) * k;
    return x >= (float)(kBins - 1) ? kBins - 1 : (x > 0.0f ? (int)x : 0);
}

// Surface area of a box (0 for an empty box), in double as the host does.
__device__ double box_area(const float* lo, const float* hi) {
#pragma clang fp contract(off)
    if (!(hi[0] >= lo[0])) return 0.0;
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return 2.0 * (dx * dy + dy * dz + dz * dx);
}

// SAH sweep over the kBins slabs of one axis: first minimum of
// A_L N_L + A_R N_R over the kBins - 1 boundaries with both sides non-empty.
__device__ void sah_sweep(const unsigned* bins, int a, double& best, int& split) {
#pragma clang fp contract(off)
    best = kInf;
    split = -1;
    double rA[kBins];
    int rN[kBins];
    float lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
    int n = 0;
#pragma unroll
    for (int b = kBins - 1; b > 0; --b) {
        int s = a * kBins + b;
        for (int j = 0; j < 3; ++j) {
            lo[j] = fminf(lo[j], unordf(bins[kLoOff + 3 * s + j]));
            hi[j] = fmaxf(hi[j], unordf(bins[kHiOff + 3 * s + j]));
        }
        n += (int)bins[s];
        rA[b] = box_area(lo, hi);
        rN[b] = n;
    }
    for (int j = 0; j < 3; ++j) { lo[j] = kInf; hi[j] = -kInf; }
    n = 0;
#pragma unroll
    for (int b = 0; b < kBins - 1; ++b) {
        int s = a * kBins + b;
        for (int j = 0; j < 3; ++j) {
            lo[j] = fminf(lo[j], unordf(bins[kLoOff + 3 * s + j]));
            hi[j] = fmaxf(hi[j], unordf(bins[kHiOff + 3 * s + j]));
        }
        n += (int)bins[s];
        if (n == 0 || rN[b + 1] == 0) continue;
        double c = box_area(lo, hi) * n + rA[b + 1] * rN[b + 1];
        if (c < best) { best = c; split = b; }
    }
}

__device__ __forceinline__ void bins_init(unsigned* b, int i) {
    b[i] = i < kLoOff ? 0u : (i < kHiOff ? ordf(kInf) : ordf(-kInf));
}

// Exclusive rank of this thread among the threads of the block with f set
// (thread order), and their total.  Every thread of the block must call it.
__device__ __forceinline__ int block_rank(bool f, int& total, int* swave) {
    unsigned long long m = __ballot(f);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int r = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) swave[w] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int j = 0; j < kWaves; ++j) {
        int x = swave[j];
        if (j < w) off += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return off + r;
}

// ---------------------------------------------------------------------------
// Triangle bounds and the root.
// ---------------------------------------------------------------------------
__global__ void k_prim_boxes(const float* __restrict__ v, const int* __restrict__ tri, int64_t nt, float4* pb,
                             int* idx) {
    int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (t >= nt) return;
    float lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
    for (int j = 0; j < 3; ++j) {
        const float* p = v + 3 * (int64_t)tri[3 * t + j];
        for (int a = 0; a < 3; ++a) { lo[a] = fminf(lo[a], p[a]); hi[a] = fmaxf(hi[a], p[a]); }
    }
    pb[2 * t] = make_float4(lo[0], lo[1], lo[2], 0.0f);
    pb[2 * t + 1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
    idx[t] = (int)t;
}

// acc slots of 12 words: box lo xyz, box hi xyz, centroid lo xyz, centroid hi xyz
__global__ void k_init_acc(unsigned* acc, int nslots) {
    int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= 12 * nslots) return;
    int j = i % 12;
    acc[i] = (j < 3 || (j >= 6 && j < 9)) ? ordf(kInf) : ordf(-kInf);
}

__device__ void acc_merge(unsigned* acc, const float* b12) {
    int lane = threadIdx.x & 63;
    float r[12];
    for (int j = 0; j < 12; ++j) {
        bool is_min = j < 3 || (j >= 6 && j < 9);
        r[j] = is_min ? wave_min(b12[j]) : wave_max(b12[j]);
    }
    if (lane == 0)
        for (int j = 0; j < 12; ++j) {
            bool is_min = j < 3 || (j >= 6 && j < 9);
            if (is_min) atomicMin(acc + j, ordf(r[j]));
            else atomicMax(acc + j, ordf(r[j]));
        }
}

__device__ __forceinline__ void grow12(float* b, const float4& lo, const float4& hi) {
    for (int a = 0; a < 3; ++a) {
        float l = comp(lo, a), h = comp(hi, a), c = 0.5f * (l + h);
        b[a] = fminf(b[a], l);
        b[3 + a] = fmaxf(b[3 + a], h);
        b[6 + a] = fminf(b[6 + a], c);
        b[9 + a] = fmaxf(b[9 + a], c);
    }
}
__device__ __forceinline__ void reset12(float* b) {
    for (int j = 0; j < 12; ++j) b[j] = (j < 3 || (j >= 6 && j < 9)) ? kInf : -kInf;
}

__global__ __launch_bounds__(kTB) void k_root_reduce(const float4* pb, int64_t nt, unsigned* acc) {
    float b[12];
    reset12(b);
    for (int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x; t < nt; t += (int64_t)gridDim.x * kTB)
        grow12(b, pb[2 * t], pb[2 * t + 1]);
    acc_merge(acc, b);
}

// ---------------------------------------------------------------------------
// Large nodes: one level per round of passes.
// ---------------------------------------------------------------------------
__global__ void k_init_bins(unsigned* bins, int ntasks) {
    int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (i >= (int64_t)ntasks * kBinWords) return;
    bins_init(bins + (i / kBinWords) * kBinWords, (int)(i % kBinWords));
}

struct AxisScale {
    float k[3];
    bool use[3];
};
__device__ __forceinline__ AxisScale axis_scale(const float* cblo, const float* cbhi) {
    AxisScale s;
    for (int a = 0; a < 3; ++a) {
        float ext = cbhi[a] - cblo[a];
        s.use[a] = ext > 0.0f;
        s.k[a] = s.use[a] ? (float)kBins / ext : 0.0f;
    }
    return s;
}

__device__ __forceinline__ void bin_tri(unsigned* sb, const AxisScale& sc, const float* cblo, const float4& lo,
                                        const float4& hi) {
    for (int a = 0; a < 3; ++a) {
        if (!sc.use[a]) continue;
        float c = 0.5f * (comp(lo, a) + comp(hi, a));
        int s = a * kBins + slab(c, cblo[a], sc.k[a]);
        atomicAdd(&sb[s], 1u);
        for (int j = 0; j < 3; ++j) {
            atomicMin(&sb[kLoOff + 3 * s + j], ordf(comp(lo, j)));
            atomicMax(&sb[kHiOff + 3 * s + j], ordf(comp(hi, j)));
        }
    }
}

__global__ __launch_bounds__(kTB) void k_bin_large(const LTask* tasks, const Chunk* chunks, const float4* pb,
                                                   const int* idx, unsigned* bins) {
    __shared__ unsigned sb[kBinWords];
    const Chunk c = chunks[blockIdx.x];
    const LTask t = tasks[c.task];
    for (int i = threadIdx.x; i < kBinWords; i += kTB) bins_init(sb, i);
    __syncthreads();
    AxisScale sc = axis_scale(t.cblo, t.cbhi);
    for (int i = c.start + threadIdx.x; i < c.end; i += kTB) {
        int p = idx[i];
        bin_tri(sb, sc, t.cblo, pb[2 * p], pb[2 * p + 1]);
    }
    __syncthreads();
    unsigned* g = bins + (size_t)c.task * kBinWords;
    for (int s = threadIdx.x; s < kAxBins; s += kTB) {
        if (sb[s] == 0) continue;
        atomicAdd(&g[s], sb[s]);
        for (int j = 0; j < 3; ++j) {
            atomicMin(&g[kLoOff + 3 * s + j], sb[kLoOff + 3 * s + j]);
            atomicMax(&g[kHiOff + 3 * s + j], sb[kHiOff + 3 * s + j]);
        }
    }
}

// Choose the split from complete bins (threads 0..2 sweep one axis each).
__device__ void choose_split(const unsigned* bins, int count, double* scost, int* ssplit, int* sdec) {
    if (threadIdx.x < 3) sah_sweep(bins, threadIdx.x, scost[threadIdx.x], ssplit[threadIdx.x]);
    __syncthreads();
    if (threadIdx.x == 0) {
        double best = kInf;
        int axis = -1, split = -1;
        for (int a = 0; a < 3; ++a)
            if (ssplit[a] >= 0 && scost[a] < best) { best = scost[a]; axis = a; split = ssplit[a]; }
        int nleft = count / 2;
        if (axis >= 0) {
            nleft = 0;
            for (int b = 0; b <= split; ++b) nleft += (int)bins[axis * kBins + b];
        }
        sdec[0] = axis;
        sdec[1] = split;
        sdec[2] = nleft;
    }
    __syncthreads();
}

__global__ __launch_bounds__(64) void k_split_large(const LTask* tasks, const unsigned* bins, Decision* dec) {
    __shared__ double scost[3];
    __shared__ int ssplit[3], sdec[3];
    const LTask t = tasks[blockIdx.x];
    choose_split(bins + (size_t)blockIdx.x * kBinWords, t.count, scost, ssplit, sdec);
    if (threadIdx.x == 0) dec[blockIdx.x] = Decision{sdec[0], sdec[1], sdec[2], 0};
}

__device__ __forceinline__ bool goes_left(const float4& lo, const float4& hi, int rel, int count, int axis, int split,
                                          const float* cblo, const AxisScale& sc) {
    if (axis < 0) return rel < count / 2;
    float c = 0.5f * (comp(lo, axis) + comp(hi, axis));
    return slab(c, cblo[axis], sc.k[axis]) <= split;
}

__global__ __launch_bounds__(kTB) void k_part_count(const LTask* tasks, const Chunk* chunks, const Decision* dec,
                                                    const float4* pb, const int* idx, int* chunk_left) {
    __shared__ int sw[kWaves];
    const Chunk c = chunks[blockIdx.x];
    const LTask t = tasks[c.task];
    const Decision d = dec[c.task];
    AxisScale sc = axis_scale(t.cblo, t.cbhi);
    int n = 0;
    for (int i = c.start + threadIdx.x; i < c.end; i += kTB) {
        int p = idx[i];
        n += goes_left(pb[2 * p], pb[2 * p + 1], i - t.first, t.count, d.axis, d.split, t.cblo, sc) ? 1 : 0;
    }
    n = wave_sum(n);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int j = 0; j < kWaves; ++j) s += sw[j];
        chunk_left[blockIdx.x] = s;
    }
}

// Stable partition of each chunk into idx_tmp, plus the bounds of both children
// (acc slot 2 task + side).  err[0] is set if a position falls outside the task.
__global__ __launch_bounds__(kTB) void k_scatter(const LTask* tasks, const Chunk* chunks, const Decision* dec,
                                                 const float4* pb, const int* idx, int* idx_tmp, unsigned* acc,
                                                 int* err) {
    __shared__ int swave[kWaves];
    const Chunk c = chunks[blockIdx.x];
    const LTask t = tasks[c.task];
    const Decision d = dec[c.task];
    AxisScale sc = axis_scale(t.cblo, t.cbhi);
    const int right_before = (c.start - t.first) - c.left_before;
    int run_l = 0, run_r = 0;
    float bl[12], br[12];
    reset12(bl);
    reset12(br);
    for (int base = c.start; base < c.end; base += kTB) {
        int i = base + threadIdx.x;
        bool valid = i < c.end;
        int p = 0;
        bool left = false;
        float4 lo = make_float4(0, 0, 0, 0), hi = lo;
        if (valid) {
            p = idx[i];
            lo = pb[2 * p];
            hi = pb[2 * p + 1];
            left = goes_left(lo, hi, i - t.first, t.count, d.axis, d.split, t.cblo, sc);
        }
        int tot_l, tot_r;
        int rl = block_rank(valid && left, tot_l, swave);
        int rr = block_rank(valid && !left, tot_r, swave);
        if (valid) {
            int pos = left ? t.first + c.left_before + run_l + rl : t.first + d.nleft + right_before + run_r + rr;
            bool in_side = left ? (pos < t.first + d.nleft) : (pos >= t.first + d.nleft);
            if (pos >= t.first && pos < t.first + t.count && in_side) idx_tmp[pos] = p;
            else atomicExch(err, 1);
            grow12(left ? bl : br, lo, hi);
        }
        run_l += tot_l;
        run_r += tot_r;
    }
    acc_merge(acc + 24 * (size_t)c.task, bl);
    acc_merge(acc + 24 * (size_t)c.task + 12, br);
}

__global__ void k_copy_back(const Chunk* chunks, const int* idx_tmp, int* idx) {
    const Chunk c = chunks[blockIdx.x];
    for (int i = c.start + threadIdx.x; i < c.end; i += kTB) idx[i] = idx_tmp[i];
}

// ---------------------------------------------------------------------------
// Small nodes: one block finishes a whole subtree.  flags[0]: error,
// flags[1]: deepest level reached.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTB) void k_small(const STask* tasks, const float4* pb, int* idx, GNode* nodes,
                                               int* counter, int max_nodes, int* flags) {
    __shared__ int sidx[kSmallMax], stmp[kSmallMax];
    __shared__ unsigned sb[kBinWords];
    __shared__ float sred[kWaves][12];
    __shared__ int swave[kWaves];
    __shared__ int4 sstack[kSmallStack];
    __shared__ double scost[3];
    __shared__ int ssplit[3], sdec[3];
    __shared__ int4 scur;
    __shared__ int sdone;
    const STask T = tasks[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (T.count > kSmallMax || T.count <= kMaxLeaf) {   // the host never sends these
        if (tid == 0) atomicExch(flags, 1);
        return;
    }
    for (int j = tid; j < T.count; j += kTB) sidx[j] = idx[T.first + j];
    int sp = 0;      // stack depth (thread 0's copy is authoritative)
    int maxd = T.depth;
    if (tid == 0) {
        scur = make_int4(0, T.count, T.node, T.depth);
        sdone = 0;
    }
    __syncthreads();
    while (true) {
        const int4 cur = scur;
        const int f = cur.x, n = cur.y;
        // centroid bounds
        float cb[6] = {kInf, kInf, kInf, -kInf, -kInf, -kInf};
        for (int j = f + tid; j < f + n; j += kTB) {
            int p = sidx[j];
            float4 lo = pb[2 * p], hi = pb[2 * p + 1];
            for (int a = 0; a < 3; ++a) {
                float c = 0.5f * (comp(lo, a) + comp(hi, a));
                cb[a] = fminf(cb[a], c);
                cb[3 + a] = fmaxf(cb[3 + a], c);
            }
        }
        for (int a = 0; a < 3; ++a) { cb[a] = wave_min(cb[a]); cb[3 + a] = wave_max(cb[3 + a]); }
        if (lane == 0)
            for (int j = 0; j < 6; ++j) sred[w][j] = cb[j];
        for (int i = tid; i < kBinWords; i += kTB) bins_init(sb, i);
        __syncthreads();
        for (int a = 0; a < 3; ++a) {
            cb[a] = sred[0][a];
            cb[3 + a] = sred[0][3 + a];
            for (int q = 1; q < kWaves; ++q) {
                cb[a] = fminf(cb[a], sred[q][a]);
                cb[3 + a] = fmaxf(cb[3 + a], sred[q][3 + a]);
            }
        }
        AxisScale sc = axis_scale(cb, cb + 3);
        for (int j = f + tid; j < f + n; j += kTB) {
            int p = sidx[j];
            bin_tri(sb, sc, cb, pb[2 * p], pb[2 * p + 1]);
        }
        __syncthreads();
        choose_split(sb, n, scost, ssplit, sdec);
        const int axis = sdec[0], split = sdec[1], nleft = sdec[2];
        if (axis >= 0) {   // stable partition through stmp
            int run_l = 0, run_r = 0;
            for (int base = f; base < f + n; base += kTB) {
                int j = base + tid;
                bool valid = j < f + n;
                int p = valid ? sidx[j] : 0;
                bool left = false;
                if (valid) left = goes_left(pb[2 * p], pb[2 * p + 1], j - f, n, axis, split, cb, sc);
                int tl, tr;
                int rl = block_rank(valid && left, tl, swave);
                int rr = block_rank(valid && !left, tr, swave);
                if (valid) {
                    int pos = left ? run_l + rl : nleft + run_r + rr;
                    if (pos >= 0 && pos < n) stmp[f + pos] = p;
                    else atomicExch(flags, 1);
                }
                run_l += tl;
                run_r += tr;
            }
            __syncthreads();
            for (int j = f + tid; j < f + n; j += kTB) sidx[j] = stmp[j];
            __syncthreads();
        }
        // child bounds: [0..5] left box, [6..11] right box
        float cbx[12] = {kInf, kInf, kInf, -kInf, -kInf, -kInf, kInf, kInf, kInf, -kInf, -kInf, -kInf};
        for (int j = f + tid; j < f + n; j += kTB) {
            int p = sidx[j];
            float4 lo = pb[2 * p], hi = pb[2 * p + 1];
            float* b = (j - f < nleft) ? cbx : cbx + 6;
            for (int a = 0; a < 3; ++a) { b[a] = fminf(b[a], comp(lo, a)); b[3 + a] = fmaxf(b[3 + a], comp(hi, a)); }
        }
        for (int j = 0; j < 12; ++j) cbx[j] = (j % 6) < 3 ? wave_min(cbx[j]) : wave_max(cbx[j]);
        if (lane == 0)
            for (int j = 0; j < 12; ++j) sred[w][j] = cbx[j];
        __syncthreads();
        if (tid == 0) {
            for (int j = 0; j < 12; ++j) {
                float x = sred[0][j];
                for (int q = 1; q < kWaves; ++q) x = (j % 6) < 3 ? fminf(x, sred[q][j]) : fmaxf(x, sred[q][j]);
                cbx[j] = x;
            }
            int id = atomicAdd(counter, 2);
            if (id < 0 || id + 2 > max_nodes) {
                atomicExch(flags, 1);
                sdone = 1;
            } else {
                const int d1 = cur.w + 1;
                maxd = max(maxd, d1);
                GNode L, R;
                for (int a = 0; a < 3; ++a) {
                    L.lo[a] = cbx[a]; L.hi[a] = cbx[3 + a];
                    R.lo[a] = cbx[6 + a]; R.hi[a] = cbx[9 + a];
                }
                L.left = L.right = R.left = R.right = -1;
                L.first = T.first + f; L.count = nleft;
                R.first = T.first + f + nleft; R.count = n - nleft;
                L.parent = R.parent = cur.z;
                L.depth = R.depth = d1;
                nodes[id] = L;
                nodes[id + 1] = R;
                nodes[cur.z].left = id;
                nodes[cur.z].right = id + 1;
                int4 lc = make_int4(f, nleft, id, d1), rc = make_int4(f + nleft, n - nleft, id + 1, d1);
                int4 big = lc.y >= rc.y ? lc : rc, sml = lc.y >= rc.y ? rc : lc;
                if (big.y > kMaxLeaf) {
                    if (sp < kSmallStack) sstack[sp++] = big;
                    else { atomicExch(flags, 1); sdone = 1; }
                }
                if (!sdone) {
                    if (sml.y > kMaxLeaf) scur = sml;
                    else if (sp > 0) scur = sstack[--sp];
                    else sdone = 1;
                }
            }
        }
        __syncthreads();
        if (sdone) break;
    }
    for (int j = tid; j < T.count; j += kTB) idx[T.first + j] = sidx[j];
    if (tid == 0) atomicMax(flags + 1, maxd);
}

// ---------------------------------------------------------------------------
// Depth-first child-pair layout.
// ---------------------------------------------------------------------------
__global__ void k_fill_int(int* a, int64_t n, int v) {
    int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_icount(const GNode* nodes, int N, int* icount, int* visits) {
    int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= N || nodes[i].left >= 0) return;
    int c = i;
    for (int guard = 0; guard < N; ++guard) {
        int p = nodes[c].parent;
        if (p < 0) break;
        __threadfence();
        if (atomicAdd(&visits[p], 1) == 0) break;   // the other subtree is still open
        __threadfence();
        int cl = atomicAdd(&icount[nodes[p].left], 0), cr = atomicAdd(&icount[nodes[p].right], 0);
        atomicExch(&icount[p], 1 + cl + cr);
        c = p;
    }
}

__global__ void k_pos(const GNode* nodes, int N, const int* icount, int* pos) {
    int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= N) return;
    if (nodes[i].left < 0) { pos[i] = -1; return; }
    int s = 0, c = i;
    for (int guard = 0; guard < N; ++guard) {
        int p = nodes[c].parent;
        if (p < 0) break;
        s += 1;
        if (nodes[p].right == c) s += icount[nodes[p].left];
        c = p;
    }
    pos[i] = s;
}

__device__ void pad_box(const float* lo, const float* hi, float* plo, float* phi) {
#pragma clang fp contract(off)
    for (int a = 0; a < 3; ++a) {
        float m = fmaxf(fabsf(lo[a]), fabsf(hi[a]));
        float pad = m * 9.5367431640625e-07f + 1e-30f;   // 2^-20 relative
        plo[a] = lo[a] - pad;
        phi[a] = hi[a] + pad;
    }
}

__device__ __forceinline__ int child_ref(const GNode& c, int cid, const int* pos) {
    return c.left < 0 ? ~((c.first << 3) | (c.count - 1)) : pos[cid];
}

__global__ void k_write(const GNode* nodes, int N, const int* pos, int nrec, float4* out) {
    int i = blockIdx.x * kTB + threadIdx.x;
    if (i >= N) return;
    const GNode n = nodes[i];
    if (n.left < 0) return;
    const int r = pos[i];
    if (r < 0 || r >= nrec) return;
    const GNode L = nodes[n.left], R = nodes[n.right];
    float l0[3], h0[3], l1[3], h1[3];
    pad_box(L.lo, L.hi, l0, h0);
    pad_box(R.lo, R.hi, l1, h1);
    float4* o = out + 4 * (size_t)r;
    o[0] = make_float4(l0[0], l0[1], l0[2], h0[0]);
    o[1] = make_float4(h0[1], h0[2], l1[0], l1[1]);
    o[2] = make_float4(l1[2], h1[0], h1[1], h1[2]);
    o[3] = make_float4(__int_as_float(child_ref(L, n.left, pos)), __int_as_float(child_ref(R, n.right, pos)), 0.0f,
                       0.0f);
}

// A tree that is a single leaf: one record with one child.
__global__ void k_write_leaf_root(const GNode* nodes, float4* out) {
    const GNode n = nodes[0];
    float l0[3], h0[3];
    pad_box(n.lo, n.hi, l0, h0);
    out[0] = make_float4(l0[0], l0[1], l0[2], h0[0]);
    out[1] = make_float4(h0[1], h0[2], 0.0f, 0.0f);
    out[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    out[3] = make_float4(__int_as_float(~((n.first << 3) | (n.count - 1))), __int_as_float(kNoChild), 0.0f, 0.0f);
}

// SAH cost relative to the root area, and the deepest level.
__global__ __launch_bounds__(kTB) void k_stats(const GNode* nodes, int N, double* sah, int* maxdepth) {
    int i = blockIdx.x * kTB + threadIdx.x;
    double s = 0.0;
    int d = 0;
    if (i < N) {
        const GNode n = nodes[i];
        const GNode r = nodes[0];
        double ar = box_area(r.lo, r.hi);
        double x = ar > 0 ? box_area(n.lo, n.hi) / ar : 1.0;
        s = n.left < 0 ? x * n.count : x;
        d = n.depth;
    }
    s = wave_sum(s);
    for (int o = 32; o >= 1; o >>= 1) d = max(d, __shfl_xor(d, o, 64));
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(sah, s);
        atomicMax(maxdepth, d);
    }
}

// ---------------------------------------------------------------------------
// Scene layout.
// ---------------------------------------------------------------------------
__global__ void k_tri_records(const float* __restrict__ v, const int* __restrict__ tri, const int* __restrict__ seg,
                              const int* __restrict__ light_of_tri, const float* __restrict__ nrm,
                              const int* __restrict__ order, int64_t nt, float4* trec, float4* nrec, int* pos_of) {
    int64_t p = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (p >= nt) return;
    int t = order[p];
    for (int j = 0; j < 3; ++j) {
        int vi = tri[3 * (int64_t)t + j];
        const float* x = v + 3 * (int64_t)vi;
        int tag = j == 0 ? t : (j == 1 ? seg[t] : light_of_tri[t]);
        trec[3 * p + j] = make_float4(x[0], x[1], x[2], __int_as_float(tag));
        if (nrm) {
            const float* q = nrm + 3 * (int64_t)vi;
            nrec[3 * p + j] = make_float4(q[0], q[1], q[2], 0.0f);
        }
    }
    pos_of[t] = (int)p;
}

__global__ void k_light_pos(int4* lights, int nlt, const int* pos_of) {
    int j = blockIdx.x * kTB + threadIdx.x;
    if (j < nlt) lights[j].x = pos_of[lights[j].w];
}

// Device allocations released at scope exit unless released to the caller.
struct Arena {
    std::vector<void*> ptrs;
    hipError_t err = hipSuccess;
    template <class T>
    T* get(size_t n) {
        void* p = nullptr;
        if (err != hipSuccess) return nullptr;
        err = hipMalloc(&p, std::max<size_t>(n * sizeof(T), 16));
        if (err != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return (T*)p;
    }
    void release(void* p) {
        for (auto& q : ptrs)
            if (q == p) q = nullptr;
    }
    ~Arena() {
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
    }
};

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kTB - 1) / kTB); }

}  // namespace

#define BVH_HIP(x)                                                                       \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) return std::string(#x ": ") + hipGetErrorString(e_);        \
    } while (0)

std::string build_bvh_gpu(const float* d_verts, const int* d_tris, int64_t nt, hipStream_t st, GpuBvh& out) {
    out = GpuBvh{};
    if (nt < 1 || nt > (int64_t(1) << 27)) return "the GPU BVH builder takes 1 .. 2^27 triangles";
    Arena ar;
    const int64_t max_nodes = 2 * nt - 1;
    float4* pb = ar.get<float4>(2 * nt);
    int* idx = ar.get<int>(nt);
    int* idx_tmp = ar.get<int>(nt);
    GNode* nodes = ar.get<GNode>(max_nodes);
    unsigned* acc_root = ar.get<unsigned>(12);
    int* flags = ar.get<int>(4);   // [0] error, [1] max depth, [2] node counter
    if (ar.err != hipSuccess) return std::string("BVH scratch: ") + hipGetErrorString(ar.err);

    hipLaunchKernelGGL(k_prim_boxes, dim3(blocks_for(nt)), dim3(kTB), 0, st, d_verts, d_tris, nt, pb, idx);
    hipLaunchKernelGGL(k_init_acc, dim3(1), dim3(kTB), 0, st, acc_root, 1);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(kTB), 0, st, flags, (int64_t)4, 0);
    hipLaunchKernelGGL(k_root_reduce, dim3(std::min<unsigned>(blocks_for(nt), 1024)), dim3(kTB), 0, st, pb, nt,
                       acc_root);
    BVH_HIP(hipGetLastError());
    unsigned racc[12];
    BVH_HIP(hipMemcpyAsync(racc, acc_root, sizeof(racc), hipMemcpyDeviceToHost, st));
    BVH_HIP(hipStreamSynchronize(st));

    std::vector<GNode> hn(1);
    for (int a = 0; a < 3; ++a) {
        hn[0].lo[a] = unordf_host(racc[a]);
        hn[0].hi[a] = unordf_host(racc[3 + a]);
    }
    hn[0].left = hn[0].right = -1;
    hn[0].first = 0;
    hn[0].count = (int)nt;
    hn[0].parent = -1;
    hn[0].depth = 1;
    int host_depth = 1;
    std::vector<STask> small;
    std::vector<LTask> large;
    if (nt > kSmallMax) {
        LTask t{0, 0, (int)nt, 1, {}, {}};
        for (int a = 0; a < 3; ++a) { t.cblo[a] = unordf_host(racc[6 + a]); t.cbhi[a] = unordf_host(racc[9 + a]); }
        large.push_back(t);
    } else if (nt > kMaxLeaf) {
        small.push_back(STask{0, 0, (int)nt, 1});
    }

    // ---- large nodes, level by level
    if (!large.empty()) {
        const int64_t max_large = nt / (kSmallMax + 1) + 1;
        const int64_t max_chunks = nt / kChunk + max_large + 1;
        LTask* d_tasks = ar.get<LTask>(max_large);
        Chunk* d_chunks = ar.get<Chunk>(max_chunks);
        unsigned* d_bins = ar.get<unsigned>(max_large * kBinWords);
        Decision* d_dec = ar.get<Decision>(max_large);
        int* d_cleft = ar.get<int>(max_chunks);
        unsigned* d_acc = ar.get<unsigned>(max_large * 24);
        if (ar.err != hipSuccess) return std::string("BVH scratch: ") + hipGetErrorString(ar.err);
        std::vector<Chunk> chunks;
        std::vector<Decision> dec;
        std::vector<int> cleft;
        std::vector<unsigned> acc;
        while (!large.empty()) {
            const int ntask = (int)large.size();
            if (ntask > max_large) return "BVH build: too many large nodes in one level";
            chunks.clear();
            std::vector<int> chunk0(ntask + 1);
            for (int i = 0; i < ntask; ++i) {
                chunk0[i] = (int)chunks.size();
                for (int s = large[i].first; s < large[i].first + large[i].count; s += kChunk)
                    chunks.push_back(Chunk{i, s, std::min(s + kChunk, large[i].first + large[i].count), 0});
            }
            chunk0[ntask] = (int)chunks.size();
            const int nch = (int)chunks.size();
            if (nch > max_chunks) return "BVH build: chunk list overflow";
            BVH_HIP(hipMemcpyAsync(d_tasks, large.data(), sizeof(LTask) * ntask, hipMemcpyHostToDevice, st));
            BVH_HIP(hipMemcpyAsync(d_chunks, chunks.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_init_bins, dim3(blocks_for((int64_t)ntask * kBinWords)), dim3(kTB), 0, st, d_bins,
                               ntask);
            hipLaunchKernelGGL(k_bin_large, dim3(nch), dim3(kTB), 0, st, d_tasks, d_chunks, pb, idx, d_bins);
            hipLaunchKernelGGL(k_split_large, dim3(ntask), dim3(64), 0, st, d_tasks, d_bins, d_dec);
            hipLaunchKernelGGL(k_part_count, dim3(nch), dim3(kTB), 0, st, d_tasks, d_chunks, d_dec, pb, idx, d_cleft);
            BVH_HIP(hipGetLastError());
            dec.resize(ntask);
            cleft.resize(nch);
            BVH_HIP(hipMemcpyAsync(dec.data(), d_dec, sizeof(Decision) * ntask, hipMemcpyDeviceToHost, st));
            BVH_HIP(hipMemcpyAsync(cleft.data(), d_cleft, sizeof(int) * nch, hipMemcpyDeviceToHost, st));
            BVH_HIP(hipStreamSynchronize(st));
            for (int i = 0; i < ntask; ++i) {
                int sum = 0;
                for (int c = chunk0[i]; c < chunk0[i + 1]; ++c) {
                    chunks[c].left_before = sum;
                    sum += cleft[c];
                }
                if (sum != dec[i].nleft || sum <= 0 || sum >= large[i].count)
                    return "BVH build: inconsistent partition of a large node";
            }
            BVH_HIP(hipMemcpyAsync(d_chunks, chunks.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_init_acc, dim3(blocks_for(24 * (int64_t)ntask)), dim3(kTB), 0, st, d_acc,
                               2 * ntask);
            hipLaunchKernelGGL(k_scatter, dim3(nch), dim3(kTB), 0, st, d_tasks, d_chunks, d_dec, pb, idx, idx_tmp,
                               d_acc, flags);
            hipLaunchKernelGGL(k_copy_back, dim3(nch), dim3(kTB), 0, st, d_chunks, idx_tmp, idx);
            BVH_HIP(hipGetLastError());
            acc.resize(24 * (size_t)ntask);
            int hflags[4];
            BVH_HIP(hipMemcpyAsync(acc.data(), d_acc, sizeof(unsigned) * acc.size(), hipMemcpyDeviceToHost, st));
            BVH_HIP(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
            BVH_HIP(hipStreamSynchronize(st));
            if (hflags[0]) return "BVH build: partition position out of range";
            std::vector<LTask> next;
            for (int i = 0; i < ntask; ++i) {
                const LTask& t = large[i];
                const int id = (int)hn.size();
                hn[t.node].left = id;
                hn[t.node].right = id + 1;
                for (int side = 0; side < 2; ++side) {
                    const unsigned* a = &acc[24 * (size_t)i + 12 * side];
                    GNode ch;
                    for (int k = 0; k < 3; ++k) { ch.lo[k] = unordf_host(a[k]); ch.hi[k] = unordf_host(a[3 + k]); }
                    ch.left = ch.right = -1;
                    ch.first = side == 0 ? t.first : t.first + dec[i].nleft;
                    ch.count = side == 0 ? dec[i].nleft : t.count - dec[i].nleft;
                    ch.parent = t.node;
                    ch.depth = t.depth + 1;
                    host_depth = std::max(host_depth, ch.depth);
                    hn.push_back(ch);
                    if (ch.count <= kMaxLeaf) continue;
                    if (ch.count <= kSmallMax) {
                        small.push_back(STask{id + side, ch.first, ch.count, ch.depth});
                    } else {
                        LTask nt2{id + side, ch.first, ch.count, ch.depth, {}, {}};
                        for (int k = 0; k < 3; ++k) { nt2.cblo[k] = unordf_host(a[6 + k]); nt2.cbhi[k] = unordf_host(a[9 + k]); }
                        next.push_back(nt2);
                    }
                }
            }
            large.swap(next);
        }
    }

    // ---- small nodes: one block per subtree
    const int m = (int)hn.size();
    BVH_HIP(hipMemcpyAsync(nodes, hn.data(), sizeof(GNode) * m, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(kTB), 0, st, flags + 2, (int64_t)1, m);
    if (!small.empty()) {
        STask* d_small = ar.get<STask>(small.size());
        if (ar.err != hipSuccess) return std::string("BVH scratch: ") + hipGetErrorString(ar.err);
        BVH_HIP(hipMemcpyAsync(d_small, small.data(), sizeof(STask) * small.size(), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_small, dim3((unsigned)small.size()), dim3(kTB), 0, st, d_small, pb, idx, nodes,
                           flags + 2, (int)max_nodes, flags);
        BVH_HIP(hipGetLastError());
    }
    int hflags[4];
    BVH_HIP(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
    BVH_HIP(hipStreamSynchronize(st));
    if (hflags[0]) return "BVH build: small-node pass failed";
    const int N = hflags[2];
    if (N < 1 || N > max_nodes || (N & 1) == 0) return "BVH build: bad node count " + std::to_string(N);

    // ---- layout
    const int nrec = N > 1 ? (N - 1) / 2 : 1;
    float4* recs = ar.get<float4>(4 * (size_t)nrec);
    int* icount = ar.get<int>(N);
    int* visits = ar.get<int>(N);
    int* pos = ar.get<int>(N);
    double* d_sah = ar.get<double>(1);
    if (ar.err != hipSuccess) return std::string("BVH layout: ") + hipGetErrorString(ar.err);
    hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(N)), dim3(kTB), 0, st, icount, (int64_t)N, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(N)), dim3(kTB), 0, st, visits, (int64_t)N, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(kTB), 0, st, flags + 1, (int64_t)1, 0);
    BVH_HIP(hipMemsetAsync(d_sah, 0, sizeof(double), st));
    if (N > 1) {
        hipLaunchKernelGGL(k_icount, dim3(blocks_for(N)), dim3(kTB), 0, st, nodes, N, icount, visits);
        hipLaunchKernelGGL(k_pos, dim3(blocks_for(N)), dim3(kTB), 0, st, nodes, N, icount, pos);
        hipLaunchKernelGGL(k_write, dim3(blocks_for(N)), dim3(kTB), 0, st, nodes, N, pos, nrec, recs);
    } else {
        hipLaunchKernelGGL(k_write_leaf_root, dim3(1), dim3(1), 0, st, nodes, recs);
    }
    hipLaunchKernelGGL(k_stats, dim3(blocks_for(N)), dim3(kTB), 0, st, nodes, N, d_sah, flags + 1);
    BVH_HIP(hipGetLastError());
    double sah = 0.0;
    int root_icount = 0;
    BVH_HIP(hipMemcpyAsync(&sah, d_sah, sizeof(double), hipMemcpyDeviceToHost, st));
    BVH_HIP(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
    BVH_HIP(hipMemcpyAsync(&root_icount, icount, sizeof(int), hipMemcpyDeviceToHost, st));
    BVH_HIP(hipStreamSynchronize(st));
    if (N > 1 && root_icount != nrec) return "BVH layout: internal node count mismatch";
    out.nodes = recs;
    out.leaf_order = idx;
    ar.release(recs);
    ar.release(idx);
    out.num_nodes = nrec;
    out.depth = hflags[1];
    out.sah_cost = sah;
    return std::string();
}

hipError_t launch_scene_layout(const float* d_verts, const int* d_tris, const int* d_seg, const int* d_light_of_tri,
                               const float* d_normals, const int* d_leaf_order, int64_t nt, float4* trec,
                               float4* nrec, int* pos_of, int4* lights, int nlt, hipStream_t st) {
    hipLaunchKernelGGL(k_tri_records, dim3(blocks_for(nt)), dim3(kTB), 0, st, d_verts, d_tris, d_seg, d_light_of_tri,
                       d_normals, d_leaf_order, nt, trec, nrec, pos_of);
    if (nlt > 0) hipLaunchKernelGGL(k_light_pos, dim3(blocks_for(nlt)), dim3(kTB), 0, st, lights, nlt, pos_of);
    return hipGetLastError();
}

}  // namespace ipt
