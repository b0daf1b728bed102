// Optimisation-step kernels around the rasterizer: L2 reconstruction loss,
// fused Adam over several parameter groups, and device-side frame selection
// so that a captured step graph can be replayed without host involvement.
#include <cstdint>
#include "block_scan.h"
#include "common.h"

namespace gft {

namespace {

constexpr int kLossUnroll = 4;   // float4 loads in flight per thread and array

// L2 loss (paper Eq. 9, L2 part): grad = w * 2 (p - t) / count, loss += w * sum (p - t)^2 / count.
// Grid (chunks, frames): a workgroup takes a strided share of one frame's
// elements, so no element index is divided; VEC: 16-byte accesses (the
// per-frame element count is a multiple of 4 and the arrays are aligned).
template <bool VEC>
__global__ void __launch_bounds__(256) k_l2_loss(const float* __restrict__ pred,
                                                 const float* __restrict__ targets,
                                                 const int32_t* __restrict__ frame_index,
                                                 int32_t n_frames, long long elems, float weight,
                                                 float* __restrict__ grad, float* __restrict__ loss) {
    __shared__ float red[4];
    const long long f = blockIdx.y;
    const float inv = 1.0f / (float)((long long)n_frames * elems);
    const float gs = weight * 2.0f * inv;
    const long long sidx = frame_index ? (long long)frame_index[f] : f;
    const float* pf = pred + f * elems;
    const float* tf = targets + sidx * elems;
    float* gf = grad + f * elems;
    float acc = 0.f;
    const long long stride = (long long)gridDim.x * blockDim.x;
    if constexpr (VEC) {
        const long long n4 = elems >> 2;
        const float4* p4 = reinterpret_cast<const float4*>(pf);
        const float4* t4 = reinterpret_cast<const float4*>(tf);
        float4* g4 = reinterpret_cast<float4*>(gf);
        const auto step = [&](const float4 pv, const float4 tv, long long i) {
            const float4 r = make_float4(pv.x - tv.x, pv.y - tv.y, pv.z - tv.z, pv.w - tv.w);
            g4[i] = make_float4(gs * r.x, gs * r.y, gs * r.z, gs * r.w);
            acc += (r.x * r.x + r.y * r.y) + (r.z * r.z + r.w * r.w);
        };
        long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
        // kLossUnroll strided float4 pairs loaded before any is used.
        for (; i + (kLossUnroll - 1) * stride < n4; i += kLossUnroll * stride) {
            float4 pv[kLossUnroll], tv[kLossUnroll];
#pragma unroll
            for (int u = 0; u < kLossUnroll; ++u) {
                pv[u] = p4[i + u * stride];
                tv[u] = t4[i + u * stride];
            }
#pragma unroll
            for (int u = 0; u < kLossUnroll; ++u) step(pv[u], tv[u], i + u * stride);
        }
        for (; i < n4; i += stride) step(p4[i], t4[i], i);
    } else {
        for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < elems; i += stride) {
            const float r = pf[i] - tf[i];
            gf[i] = gs * r;
            acc += r * r;
        }
    }
    acc = wave_reduce_sum(acc);
    if (lane_id() == 0) red[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0 && loss) atomicAdd(loss, weight * ((red[0] + red[1]) + (red[2] + red[3])) * inv);
}

constexpr int kMaxGroups = 16;
constexpr int kAdamChunk = 256 * 16;   // elements per workgroup: 4 float4 per thread
struct AdamArgs {
    float* p[kMaxGroups];
    const float* g[kMaxGroups];
    float* m[kMaxGroups];
    float* v[kMaxGroups];
    long long n[kMaxGroups];
    int bstart[kMaxGroups + 1];   // first workgroup of each group
    int vec[kMaxGroups];          // 1: the four arrays are 16-byte aligned
    float lr[kMaxGroups];
    float lr_final[kMaxGroups];
    int decay[kMaxGroups];
    int n_groups;
    float b1, b2, eps;
};

__global__ void k_step_increment(int32_t* step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) step[0] += 1;
}

__device__ __forceinline__ float adam_one(float& p, float g, float& m, float& v, float b1, float b2, float ibc1,
                                          float ibc2, float lr, float eps) {
    m = b1 * m + (1.0f - b1) * g;
    v = b2 * v + (1.0f - b2) * g * g;
    p -= lr * (m * ibc1) * __builtin_amdgcn_rcpf(sqrtf(v * ibc2) + eps);
    return p;
}

// One workgroup per chunk of kAdamChunk consecutive elements of one group:
// the group and its (possibly decayed) rate are uniform per workgroup, and
// the bias corrections are multiplied in as reciprocals.
__global__ void __launch_bounds__(256) k_adam(AdamArgs A, const int32_t* __restrict__ step) {
    const int t = *step;
    const float ibc1 = 1.0f / (1.0f - powf(A.b1, (float)t));
    const float ibc2 = 1.0f / (1.0f - powf(A.b2, (float)t));
    int gi = 0;
    while ((int)blockIdx.x >= A.bstart[gi + 1]) ++gi;
    float lr = A.lr[gi];
    if (A.decay[gi] > 0) {
        const float s = (float)min(t - 1, A.decay[gi]) / (float)A.decay[gi];
        lr = A.lr[gi] * powf(A.lr_final[gi] / A.lr[gi], s);
    }
    const long long n = A.n[gi];
    const long long j0 = (long long)(blockIdx.x - A.bstart[gi]) * kAdamChunk;
    float* P = A.p[gi];
    const float* G = A.g[gi];
    float* M = A.m[gi];
    float* V = A.v[gi];
    if (A.vec[gi] && j0 + kAdamChunk <= n) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const long long j = j0 + 4 * ((long long)k * 256 + threadIdx.x);
            float4 p = *reinterpret_cast<float4*>(P + j);
            const float4 g = *reinterpret_cast<const float4*>(G + j);
            float4 m = *reinterpret_cast<float4*>(M + j);
            float4 v = *reinterpret_cast<float4*>(V + j);
            adam_one(p.x, g.x, m.x, v.x, A.b1, A.b2, ibc1, ibc2, lr, A.eps);
            adam_one(p.y, g.y, m.y, v.y, A.b1, A.b2, ibc1, ibc2, lr, A.eps);
            adam_one(p.z, g.z, m.z, v.z, A.b1, A.b2, ibc1, ibc2, lr, A.eps);
            adam_one(p.w, g.w, m.w, v.w, A.b1, A.b2, ibc1, ibc2, lr, A.eps);
            *reinterpret_cast<float4*>(P + j) = p;
            *reinterpret_cast<float4*>(M + j) = m;
            *reinterpret_cast<float4*>(V + j) = v;
        }
    } else {
        const long long j1 = min(j0 + (long long)kAdamChunk, n);
        for (long long j = j0 + threadIdx.x; j < j1; j += 256) {
            float p = P[j], m = M[j], v = V[j];
            adam_one(p, G[j], m, v, A.b1, A.b2, ibc1, ibc2, lr, A.eps);
            P[j] = p;
            M[j] = m;
            V[j] = v;
        }
    }
}

__global__ void k_select_frames(gftorf_frame* __restrict__ frames, int32_t n_batch,
                                const gftorf_frame* __restrict__ seq, int32_t n_seq,
                                const float* __restrict__ bg_table, int32_t n_bg, int32_t n_quad,
                                const int32_t* __restrict__ step, int32_t* __restrict__ frame_index) {
    const int b = blockIdx.x;
    if (b >= n_batch) return;
    const long long s = *step;
    const int src = (int)(((long long)n_batch * s + b) % n_seq);
    const float* in = reinterpret_cast<const float*>(seq + src);
    float* out = reinterpret_cast<float*>(frames + b);
    constexpr int NFL = sizeof(gftorf_frame) / sizeof(float);
    for (int i = threadIdx.x; i < NFL; i += blockDim.x) out[i] = in[i];
    __syncthreads();
    if (bg_table) {
        const float* bg = bg_table + ((long long)(s % n_bg) * n_batch + b) * (3 + n_quad);
        gftorf_frame* fr = frames + b;
        for (int i = threadIdx.x; i < 3 + n_quad; i += blockDim.x) {
            if (i < 3) fr->bg_rgb[i] = bg[i];
            else fr->bg_quad[i - 3] = bg[i];
        }
    }
    if (threadIdx.x == 0 && frame_index) frame_index[b] = src;
}

}  // namespace

void launch_l2_loss(const float* pred, const float* targets, const int32_t* frame_index,
                    int32_t n_frames, int64_t elems, float weight, float* grad, float* loss,
                    hipStream_t s) {
    if (n_frames <= 0 || elems <= 0) return;
    const auto aligned = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    const bool vec = (elems & 3) == 0 && aligned(pred) && aligned(targets) && aligned(grad);
    long long per = vec ? elems / 4 : elems;
    // Vector path: about 16 accesses per thread, kLossUnroll at a time (a
    // quarter of the workgroups, hence of the loss atomics on one word, of 4
    // per thread); scalar path: about 4 per thread.
    const long long per_thread = vec ? 4 * kLossUnroll : 4;
    long long bx = (per + 256 * per_thread - 1) / (256 * per_thread);
    if (bx > 4096) bx = 4096;
    const dim3 grid((unsigned)bx, (unsigned)n_frames);
    { ProfScope _p("k_l2_loss", s);
    if (vec)
        hipLaunchKernelGGL(k_l2_loss<true>, grid, dim3(256), 0, s, pred, targets, frame_index, n_frames,
                           (long long)elems, weight, grad, loss);
    else
        hipLaunchKernelGGL(k_l2_loss<false>, grid, dim3(256), 0, s, pred, targets, frame_index, n_frames,
                           (long long)elems, weight, grad, loss);
    }
}

void launch_adam(const gftorf_adam_group* groups, int32_t n_groups, int32_t* step, float b1,
                 float b2, float eps, hipStream_t s) {
    { ProfScope _p("k_step_increment", s);
    hipLaunchKernelGGL(k_step_increment, dim3(1), dim3(64), 0, s, step);
    }
    const auto aligned = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    for (int base = 0; base < n_groups; base += kMaxGroups) {
        AdamArgs A{};
        const int ng = (n_groups - base) < kMaxGroups ? (n_groups - base) : kMaxGroups;
        A.n_groups = ng;
        A.b1 = b1;
        A.b2 = b2;
        A.eps = eps;
        A.bstart[0] = 0;
        for (int i = 0; i < ng; ++i) {
            const gftorf_adam_group& g = groups[base + i];
            A.p[i] = g.param;
            A.g[i] = g.grad;
            A.m[i] = g.m;
            A.v[i] = g.v;
            A.n[i] = g.n;
            A.vec[i] = aligned(g.param) && aligned(g.grad) && aligned(g.m) && aligned(g.v);
            A.lr[i] = g.lr;
            A.lr_final[i] = g.lr_final;
            A.decay[i] = g.decay_steps;
            A.bstart[i + 1] = A.bstart[i] + (int)((g.n + kAdamChunk - 1) / kAdamChunk);
        }
        for (int i = ng; i < kMaxGroups; ++i) A.bstart[i + 1] = A.bstart[ng];
        if (A.bstart[ng] == 0) continue;
        { ProfScope _p("k_adam", s);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)A.bstart[ng]), dim3(256), 0, s, A, step);
        }
    }
}

void launch_select_frames(gftorf_frame* frames, int32_t n_batch, const gftorf_frame* seq,
                          int32_t n_seq, const float* bg_table, int32_t n_bg, int32_t n_quad,
                          const int32_t* step, int32_t* frame_index, hipStream_t s) {
    { ProfScope _p("k_select_frames", s);
    hipLaunchKernelGGL(k_select_frames, dim3(n_batch), dim3(64), 0, s, frames, n_batch, seq, n_seq,
                       bg_table, n_bg, n_quad, step, frame_index);
    }
}

}  // namespace gft
