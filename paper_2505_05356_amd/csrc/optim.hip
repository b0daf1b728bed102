// Optimisation-step kernels around the rasterizer: L2 reconstruction loss,
// fused Adam over several parameter groups, and device-side frame selection
// so that a captured step graph can be replayed without host involvement.
#include "block_scan.h"
#include "common.h"

namespace gft {

namespace {

// L2 loss (paper Eq. 9, L2 part): grad = w * 2 (p - t) / count, loss += w * sum (p - t)^2 / count.
__global__ void __launch_bounds__(256) k_l2_loss(const float* __restrict__ pred,
                                                 const float* __restrict__ targets,
                                                 const int32_t* __restrict__ frame_index,
                                                 int32_t n_frames, long long elems, float weight,
                                                 float* __restrict__ grad, float* __restrict__ loss) {
    __shared__ float red[4];
    const long long total = (long long)n_frames * elems;
    const float inv = 1.0f / (float)total;
    float acc = 0.f;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long f = i / elems;
        const long long e = i - f * elems;
        const long long sidx = frame_index ? (long long)frame_index[f] : f;
        const float r = pred[i] - targets[sidx * elems + e];
        grad[i] = weight * 2.0f * r * inv;
        acc += r * r;
    }
    acc = wave_reduce_sum(acc);
    if (lane_id() == 0) red[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0 && loss) atomicAdd(loss, weight * ((red[0] + red[1]) + (red[2] + red[3])) * inv);
}

constexpr int kMaxGroups = 16;
struct AdamArgs {
    float* p[kMaxGroups];
    const float* g[kMaxGroups];
    float* m[kMaxGroups];
    float* v[kMaxGroups];
    long long start[kMaxGroups + 1];
    float lr[kMaxGroups];
    float lr_final[kMaxGroups];
    int decay[kMaxGroups];
    int n_groups;
    float b1, b2, eps;
};

__global__ void k_step_increment(int32_t* step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) step[0] += 1;
}

__global__ void __launch_bounds__(256) k_adam(AdamArgs A, const int32_t* __restrict__ step) {
    const int t = *step;
    const float bc1 = 1.0f - powf(A.b1, (float)t);
    const float bc2 = 1.0f - powf(A.b2, (float)t);
    const long long total = A.start[A.n_groups];
    int lr_g = -1;   // group whose (possibly decayed) rate is in lr
    float lr = 0.0f;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        int gi = 0;
        while (i >= A.start[gi + 1]) ++gi;
        if (gi != lr_g) {
            lr_g = gi;
            lr = A.lr[gi];
            if (A.decay[gi] > 0) {
                const float s = (float)min(t - 1, A.decay[gi]) / (float)A.decay[gi];
                lr = A.lr[gi] * powf(A.lr_final[gi] / A.lr[gi], s);
            }
        }
        const long long j = i - A.start[gi];
        const float g = A.g[gi][j];
        const float m = A.b1 * A.m[gi][j] + (1.0f - A.b1) * g;
        const float v = A.b2 * A.v[gi][j] + (1.0f - A.b2) * g * g;
        A.m[gi][j] = m;
        A.v[gi][j] = v;
        const float mh = m / bc1;
        const float vh = v / bc2;
        A.p[gi][j] -= lr * mh / (sqrtf(vh) + A.eps);
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
    const long long total = (long long)n_frames * elems;
    long long blocks = (total + 256 * 8 - 1) / (256 * 8);
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    { ProfScope _p("k_l2_loss", s);
    hipLaunchKernelGGL(k_l2_loss, dim3((unsigned)blocks), dim3(256), 0, s, pred, targets, frame_index,
                       n_frames, (long long)elems, weight, grad, loss);
    }
}

void launch_adam(const gftorf_adam_group* groups, int32_t n_groups, int32_t* step, float b1,
                 float b2, float eps, hipStream_t s) {
    { ProfScope _p("k_step_increment", s);
    hipLaunchKernelGGL(k_step_increment, dim3(1), dim3(64), 0, s, step);
    }
    for (int base = 0; base < n_groups; base += kMaxGroups) {
        AdamArgs A{};
        const int ng = (n_groups - base) < kMaxGroups ? (n_groups - base) : kMaxGroups;
        A.n_groups = ng;
        A.b1 = b1;
        A.b2 = b2;
        A.eps = eps;
        A.start[0] = 0;
        for (int i = 0; i < ng; ++i) {
            const gftorf_adam_group& g = groups[base + i];
            A.p[i] = g.param;
            A.g[i] = g.grad;
            A.m[i] = g.m;
            A.v[i] = g.v;
            A.lr[i] = g.lr;
            A.lr_final[i] = g.lr_final;
            A.decay[i] = g.decay_steps;
            A.start[i + 1] = A.start[i] + g.n;
        }
        long long blocks = (A.start[ng] + 256 * 4 - 1) / (256 * 4);
        if (blocks > 8192) blocks = 8192;
        if (blocks < 1) blocks = 1;
        { ProfScope _p("k_adam", s);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, s, A, step);
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
