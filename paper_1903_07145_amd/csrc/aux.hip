// Small kernels around the path kernels: light-selection table, loss and
// adjoint image, block-partial gradient reduction, projected Adam.
#include <hip/hip_runtime.h>

#include "ipt_internal.h"

namespace ipt {

__global__ void zero_u32_kernel(unsigned* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Light-selection table.  The paper keeps light-sampling probabilities
// proportional to the current emission of each object in a Fenwick tree
// (Appendix E).  Here every call rebuilds the inclusive prefix sums of
// weight_j = area_j * max(lum(e_k), 1e-3 * max lum) over emitter triangles
// (area only if every emission is zero) with one block: each of the 1024
// threads scans a contiguous run, the run totals are scanned in LDS, and the
// runs are rescanned with their offsets.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void light_cdf_kernel(const int4* lights, int nlt, int S, int E, int nm,
                                                         const float* sp, float* cdf) {
    __shared__ float part[1024];
    __shared__ float maxl_sh;
    const int tid = threadIdx.x;
    if (tid == 0) {
        float m = 0.0f;
        for (int k = 0; k < E; ++k) {
            const float* e = sp + nm * S + 3 * k;
            m = fmaxf(m, (e[0] + e[1] + e[2]) * (1.0f / 3.0f));
        }
        maxl_sh = m;
    }
    __syncthreads();
    const float maxl = maxl_sh;
    const int per = (nlt + 1023) / 1024;
    const int b = tid * per, e_ = min(nlt, b + per);
    auto weight = [&](int j) {
        int4 L = lights[j];
        float area = __int_as_float(L.z);
        if (!(maxl > 0.0f)) return area;
        const float* e = sp + nm * S + 3 * L.y;
        float l = (e[0] + e[1] + e[2]) * (1.0f / 3.0f);
        return area * fmaxf(l, 1e-3f * maxl);
    };
    float s = 0.0f;
    for (int j = b; j < e_; ++j) s += weight(j);
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        float v = tid >= off ? part[tid - off] : 0.0f;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    float run = tid > 0 ? part[tid - 1] : 0.0f;
    for (int j = b; j < e_; ++j) {
        run += weight(j);
        cdf[j] = run;
    }
    // selection probabilities directly as w_j / total: a difference of two
    // prefix sums would lose digits when there are many lights
    const float rtot = 1.0f / part[1023];
    for (int j = b; j < e_; ++j) cdf[nlt + j] = weight(j) * rtot;
}

hipError_t launch_light_cdf(const SceneDev& sc, const float* sparams, float* cdf, hipStream_t st) {
    if (sc.nlt <= 0) return hipSuccess;
    hipLaunchKernelGGL(light_cdf_kernel, dim3(1), dim3(1024), 0, st, sc.lights, sc.nlt, sc.S, sc.E, sc.nm,
                       sparams, cdf);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Loss and adjoint (Sec. 3.2 Eq. 3, Sec. 3.3 Eq. 4).  kind 0: E = mean (I-T)^2,
// w = 2 (I - T) / n; kind 1: E = mean |I - T|, w = sgn(I - T) / n.  (Eq. 4 as
// printed carries sgn(T - I), the descent direction; w here is dE/dI.)
// Block partial sums, then a one-block final sum: deterministic.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void loss_kernel(const float* img, const float* tgt, int64_t n3, int kind,
                                                   float* w, float* partials) {
    __shared__ float red[256];
    float acc = 0.0f;
    const float inv = 1.0f / (float)n3;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n3; i += (int64_t)gridDim.x * 256) {
        float r = img[i] - tgt[i];
        if (kind == 0) {
            acc += r * r;
            w[i] = 2.0f * r * inv;
        } else {
            acc += fabsf(r);
            w[i] = (r > 0.0f ? 1.0f : (r < 0.0f ? -1.0f : 0.0f)) * inv;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void loss_final_kernel(const float* partials, int n, int64_t n3, float* loss) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += (double)partials[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(red[0] / (double)n3);
}

hipError_t launch_loss_adjoint(const float* img, const float* target, int64_t n3, int kind, float* w,
                               float* partials, int nparts, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(loss_kernel, dim3(nparts), dim3(256), 0, st, img, target, n3, kind, w, partials);
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, partials, nparts, n3, loss);
    return hipGetLastError();
}

// grad[i] (+)= sum_b part[b][i], in block order (deterministic).
// Pixel means from the per-unit sample sums of a colour pass whose pixels were
// split over several lanes (fixed summation order: deterministic).
__global__ __launch_bounds__(256) void colour_reduce_kernel(const float* part, int nchunk, int64_t pix_count,
                                                            float inv_spp, float* image) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= 3 * pix_count) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * 3 * pix_count + i];
    image[i] = s * inv_spp;
}

hipError_t launch_colour_reduce(const float* part, int nchunk, int64_t pix_count, int spp, float* image,
                                hipStream_t st) {
    int64_t n = 3 * pix_count;
    hipLaunchKernelGGL(colour_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, nchunk,
                       pix_count, 1.0f / (float)spp, image);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void grad_reduce_kernel(const double* part, int nblocks, int P, float* grad,
                                                          int accumulate) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * P + i];
    grad[i] = accumulate ? (float)((double)grad[i] + s) : (float)s;
}

hipError_t launch_grad_reduce(const double* part, int nblocks, int P, float* grad, int accumulate,
                              hipStream_t st) {
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((P + 255) / 256), dim3(256), 0, st, part, nblocks, P,
                       grad, accumulate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adam (Kingma & Ba; Sec. 4.5) on theta = p / scale, bias-corrected, then a
// clamp of theta to [lo, hi] (the material parameters live in [0, 1]).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void adam_kernel(float* params, const float* grad, float* m, float* v, int P,
                                                   float c1, float c2, float lr, float b1, float b2, float eps,
                                                   const float* scale, const float* lo, const float* hi,
                                                   const uint8_t* trainable) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    if (trainable && !trainable[i]) return;
    float sc = scale ? scale[i] : 1.0f;
    float g = grad[i] * sc;
    float mi = b1 * m[i] + (1.0f - b1) * g;
    float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    float mh = mi / c1, vh = vi / c2;
    float th = params[i] / sc - lr * mh / (sqrtf(vh) + eps);
    if (lo) th = fmaxf(th, lo[i]);
    if (hi) th = fminf(th, hi[i]);
    params[i] = th * sc;
}

// L1 term: grad += w sgn(p); loss += sum w |p| (one wave-reduced atomic per wave).
__global__ __launch_bounds__(256) void l1_reg_kernel(const float* p, float* g, const float* w, int P, float* loss) {
    int i = blockIdx.x * 256 + threadIdx.x;
    float l = 0.0f;
    if (i < P && w[i] != 0.0f) {
        float x = p[i];
        float sg = x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f);
        g[i] += w[i] * sg;
        l = w[i] * fabsf(x);
    }
    for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
    if ((threadIdx.x & 63) == 0 && l != 0.0f) atomicAdd(loss, l);
}

hipError_t launch_l1_reg(const float* p, float* g, const float* w, int P, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(l1_reg_kernel, dim3((P + 255) / 256), dim3(256), 0, st, p, g, w, P, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* params, const float* grad, float* m, float* v, int P, int step, float lr,
                       float b1, float b2, float eps, const float* scale, const float* lo, const float* hi,
                       const uint8_t* trainable, hipStream_t st) {
    float c1 = (float)(1.0 - pow((double)b1, (double)step));
    float c2 = (float)(1.0 - pow((double)b2, (double)step));
    hipLaunchKernelGGL(adam_kernel, dim3((P + 255) / 256), dim3(256), 0, st, params, grad, m, v, P, c1, c2, lr,
                       b1, b2, eps, scale, lo, hi, trainable);
    return hipGetLastError();
}

}  // namespace ipt
