// Deformation network of paper §4 ("MLP") on the gfx950 matrix cores.
//
// delta x = W_8 h_8 + b_8,  h_{l+1} = relu(W_l h_l + b_l),  h_0 = the positional
// encoding of (s_x x0, s_t t), for every (time, Gaussian) row.
//
// Kernels
//   k_mlp_pack    float32 parameters -> bfloat16 weight copies: W_l as
//                 [out][in] (forward) and W_l^T as [in][out] (backward), both
//                 zero-padded so every product is whole 16 x 16 x 32 tiles.
//   k_mlp_fwd     one workgroup of 4 waves per 128 rows: the encoding and
//                 every layer's activations stay in LDS (128 x 256 bf16),
//                 weights stream from L2; wave w computes output columns
//                 64w .. 64w+63 of all 128 rows with v_mfma_f32_16x16x32_bf16.
//                 Two workgroups share a CU (two waves per SIMD), so one's
//                 epilogue overlaps the other's products.  Training mode also
//                 stores h_0 .. h_8 and the ReLU decisions as bits.
//   k_mlp_bwd     the same tiling backwards: gz_8 = dL/d delta, then per layer
//                 g_l = gz_l W_l, gz_{l-1} = g_l * [h_l > 0] (the forward's
//                 bits); stores every gz_l and, from g_0, the gradient of the
//                 scaled centre input.  Two workgroups per CU, as the forward.
//   k_mlp_dw      dW_l = sum_rows gz_l h_l^T, db_l = sum_rows gz_l: rows are the
//                 contraction, split into fixed chunks, one partial per chunk;
//                 each 64-row stage of gz_l and h_l passes once through LDS.
//   k_mlp_reduce  sums the chunk partials in chunk order into the parameter
//                 layout; k_mlp_dx0 sums the centre gradient over the times.
//   k_blend       Eq. 7 with the network: per-frame offsets from the offsets
//                 at two integer timesteps; k_blend_bwd is its transpose.
//
// Saved activations and gradients use a row-blocked layout [rows/8][feat][8]:
// the eight rows of one feature are one 16-byte fragment of the weight-gradient
// product, and the row-parallel kernels write four of them per lane.  The
// forward also keeps the ReLU decisions of h_1 .. h_8 as bits, 16 bytes per
// lane and layer in the lane's own accumulator order, so the backward gates
// its gradients from 4 registers instead of re-reading the activations.
#include <mutex>

#include "mlp.h"

namespace gft {
namespace mlp {
namespace {

// Scratch of gftorf_mlp_fwd_noalloc: the bfloat16 weight copies of one
// inference forward.  Every GPU the library runs on holds its own copy until
// the process ends.  In host code this name is only a stand-in for the
// symbol: kernels receive the device address that noalloc_scratch resolves.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

// LDS row stride in bf16: the 16-byte pad puts the 16 rows of one fragment
// read in 16 distinct 4-bank groups.
constexpr int kLDX = kWidth + 8;

struct Args {
    const float* x0;
    int64_t n, rows;
    int lx, lt;
    float sx, st;
    float times[kMaxTimes];
    const gftorf_frame* frames;   // if set, time t is frames[t].time (device)
    const bf16* wf[kLayers];
    const bf16* wt[kLayers];
    const float* bias[kLayers];
    bf16* H[kLayers];
    bf16* GZ[kLayers];
    uint4* mask;   // [blocks][kDepth][256 threads]: word c, bit mask_bit(r, j) = [h > 0] of acc[r][c][j]
};

// D += A B on one 16 x 16 tile, K = 32.  Lane l supplies A[l % 16][8 (l / 16) + e]
// and B[8 (l / 16) + e][l % 16], e = 0..7; it receives D[4 (l / 16) + j][l % 16].
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Positional encoding: feature f of the network input.  Returns the input
// coordinate it reads (0..2 = x, 3 = t, -1 = padding) and its block: 0 = the
// coordinate itself, 2k + 1 = sin(2^k pi p), 2k + 2 = cos(2^k pi p).
__device__ __forceinline__ int feat_src(int f, int lx, int lt, int& blk) {
    const int nx = 3 * (1 + 2 * lx);
    if (f < nx) {
        blk = f / 3;
        return f - 3 * blk;
    }
    f -= nx;
    blk = f;
    return f < 1 + 2 * lt ? 3 : -1;
}

__device__ __forceinline__ float enc(float p, int blk) {
    if (blk == 0) return p;
    const float a = ldexpf(p, (blk - 1) >> 1);   // 2^k p, exact
    return ((blk - 1) & 1) ? cospif(a) : sinpif(a);
}

__device__ __forceinline__ float enc_d(float p, int blk) {   // d enc / d p
    if (blk == 0) return 1.0f;
    const int k = (blk - 1) >> 1;
    const float a = ldexpf(p, k), w = ldexpf(3.14159265358979f, k);
    return ((blk - 1) & 1) ? -w * sinpif(a) : w * cospif(a);
}

__device__ __forceinline__ float pick4(const float (&v)[4], int c) {
    return c == 0 ? v[0] : c == 1 ? v[1] : c == 2 ? v[2] : v[3];
}

// scaled inputs of row r (zeros for padding rows)
__device__ __forceinline__ void row_inputs(const Args& a, int64_t r, float (&xin)[4]) {
    xin[0] = xin[1] = xin[2] = xin[3] = 0.f;
    if (r >= a.rows) return;
    const int t = (int)(r / a.n);
    const int64_t k = r - (int64_t)t * a.n;
    for (int c = 0; c < 3; ++c) xin[c] = a.sx * a.x0[c * a.n + k];
    xin[3] = a.st * (a.frames ? a.frames[t].time : a.times[t]);
}

// acc[r][c] += X[16 r + .][.] * B[col0 + 16 c + .][.] over K: X in LDS
// (row-major, stride kLDX), B in global memory as [cols][K].
// With PIPE the next k-step's weight fragments are in flight while this one
// multiplies (pinned by a scheduling barrier); without it the compiler
// schedules the loads, which suits the backward, whose mask loads are
// already queued ahead of the product.
template <int K, bool PIPE>
__device__ __forceinline__ void gemm_128x64(const bf16* X, const bf16* __restrict__ B, int col0,
                                            f32x4 (&acc)[8][4], int lane) {
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    const bf16* bp = B + (size_t)(col0 + lr) * K + lk;
    bf16x8 b[4], bn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) b[c] = *(const bf16x8*)(bp + (size_t)16 * c * K);
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 32) {
        if (k0 + 32 < K) {
#pragma unroll
            for (int c = 0; c < 4; ++c) bn[c] = *(const bf16x8*)(bp + (size_t)16 * c * K + k0 + 32);
        }
        if (PIPE) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const bf16x8 x = *(const bf16x8*)(X + (16 * r + lr) * kLDX + lk + k0);
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = mfma(x, b[c], acc[r][c]);
        }
        if (k0 + 32 < K) {
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = bn[c];
        }
    }
}

// Bit of element j of accumulator row tile r in its column tile's mask word.
// The forward derives the four bits of a tile from the two 32-bit words of its
// bfloat16 ReLU outputs (each half non-negative): adding 0x7fff to a half sets
// its bit 15 exactly when the half is non-zero, without carrying into the
// other half; bits 15 and 31 of the two sums then shift into place together.
__device__ __forceinline__ constexpr int mask_bit(int r, int j) {
    return r + (j == 0 ? 0 : j == 1 ? 16 : j == 2 ? 8 : 24);
}

__device__ __forceinline__ uint32_t relu_bits(bf16x4 v, int r) {
    const uint2 d = __builtin_bit_cast(uint2, v);
    const uint32_t s0 = (d.x + 0x7fff7fffu) & 0x80008000u;   // j = 0 at bit 15, j = 1 at bit 31
    const uint32_t s1 = (d.y + 0x7fff7fffu) & 0x80008000u;   // j = 2, j = 3
    return (s0 >> (15 - r)) | (s1 >> (7 - r));
}

__device__ __forceinline__ void zero(f32x4 (&acc)[8][4]) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// offset (in bf16) of rows row .. row+3 (row % 4 == 0) of feature col in a
// row-blocked [rows/8][F][8] array
template <int F>
__device__ __forceinline__ size_t blk_off(int64_t row, int col) {
    return ((size_t)(row >> 3) * F + col) * 8 + (size_t)(row & 7);
}

// copy the first F columns of the 128 LDS rows to a row-blocked array
template <int F>
__device__ __forceinline__ void save_block(const bf16* X, bf16* __restrict__ dst, int64_t r0,
                                           int tid) {
    for (int p = tid; p < 16 * F; p += 256) {
        const int rb = p / F, f = p - rb * F;
        bf16x8 v;
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = X[(8 * rb + m) * kLDX + f];
        *(bf16x8*)(dst + ((size_t)(r0 / 8 + rb) * F + f) * 8) = v;
    }
}

template <bool SAVE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_mlp_fwd(Args a, float* __restrict__ delta) {
    __shared__ __attribute__((aligned(16))) bf16 X[kRows * kLDX];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * kRows;
    {   // h_0: two threads per row, 48 features each
        const int rr = tid >> 1, half = tid & 1;
        float xin[4];
        row_inputs(a, r0 + rr, xin);
        for (int f = 48 * half; f < 48 * half + 48; ++f) {
            int blk;
            const int c = feat_src(f, a.lx, a.lt, blk);
            X[rr * kLDX + f] = (bf16)(c < 0 ? 0.f : enc(pick4(xin, c), blk));
        }
    }
    __syncthreads();
    if (SAVE) save_block<kK0>(X, a.H[0], r0, tid);

    f32x4 acc[8][4];
    const int col0 = 64 * wv;
    for (int l = 0; l < kDepth; ++l) {
        // the products accumulate onto the bias
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float bb = a.bias[l][col0 + 16 * c + lr];
#pragma unroll
            for (int r = 0; r < 8; ++r) acc[r][c] = f32x4{bb, bb, bb, bb};
        }
        if (l == 0)
            gemm_128x64<kK0, true>(X, a.wf[0], col0, acc, lane);
        else
            gemm_128x64<kWidth, true>(X, a.wf[l], col0, acc, lane);
        __syncthreads();   // every wave has read this layer's input
        // rows r0 + 16 r + 4 lg .. +3 of feature col0 + 16 c + lr sit at
        // hb + (16 r / 8) * kWidth * 8 + 16 c * 8 in the row-blocked layout
        bf16* hb = a.H[l + 1] + ((size_t)(r0 / 8 + (lg >> 1)) * kWidth + col0 + lr) * 8 + 4 * (lg & 1);
        uint32_t mw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = col0 + 16 * c + lr;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                // bfloat16 first, then ReLU as a packed 16-bit integer max with 0:
                // a negative bfloat16 is a negative int16
                const bf16x4 z = __builtin_convertvector(acc[r][c], bf16x4);
                const s16x4 zi = __builtin_bit_cast(s16x4, z);
                const bf16x4 v = __builtin_bit_cast(bf16x4, __builtin_elementwise_max(zi, s16x4{0, 0, 0, 0}));
#pragma unroll
                for (int j = 0; j < 4; ++j) X[(16 * r + 4 * lg + j) * kLDX + col] = v[j];
                if (SAVE) {
                    *(bf16x4*)(hb + (size_t)r * (2 * kWidth * 8) + c * 128) = v;
                    mw[c] |= relu_bits(v, r);
                }
            }
        }
        if (SAVE) a.mask[((size_t)blockIdx.x * kDepth + l) * 256 + tid] = make_uint4(mw[0], mw[1], mw[2], mw[3]);
        __syncthreads();
    }
    // head: 128 rows x 16 (3 real) outputs; wave w takes rows 32w .. 32w+31
    f32x4 o2[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
    const bf16* bp = a.wf[kDepth] + (size_t)lr * kWidth + 8 * lg;
#pragma unroll 4
    for (int k0 = 0; k0 < kWidth; k0 += 32) {
        const bf16x8 b = *(const bf16x8*)(bp + k0);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const bf16x8 x = *(const bf16x8*)(X + (32 * wv + 16 * r + lr) * kLDX + 8 * lg + k0);
            o2[r] = mfma(x, b, o2[r]);
        }
    }
    if (lr < 3) {
        const float bb = a.bias[kDepth][lr];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = r0 + 32 * wv + 16 * r + 4 * lg + j;
                if (row < a.rows) {
                    const int t = (int)(row / a.n);
                    const int64_t k = row - (int64_t)t * a.n;
                    delta[((int64_t)t * 3 + lr) * a.n + k] = o2[r][j] + bb;
                }
            }
    }
}

// The ReLU decisions of the training forward as plain bytes, dec[row][layer][unit]
// (1 = active), read from (WRITE = false) or written into (WRITE = true) the
// bit words: one thread per word, i.e. per (128-row block, layer, forward
// thread), which holds the thread's 4 column tiles x 8 row tiles x 4 rows.
// Padding rows read nothing and are written inactive.
template <bool WRITE>
__global__ void __launch_bounds__(256) k_mlp_decisions(uint4* __restrict__ mask, uint8_t* __restrict__ dec,
                                                       int64_t rows, int64_t words) {
    const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (w >= words) return;
    const int tid = (int)(w & 255);
    const int l = (int)((w >> 8) % kDepth);
    const int64_t blk = (w >> 8) / kDepth;
    const int lane = tid & 63, wv = tid >> 6, lr = lane & 15, lg = lane >> 4;
    uint32_t mw[4] = {0u, 0u, 0u, 0u};
    if (!WRITE) {
        const uint4 m = mask[w];
        mw[0] = m.x, mw[1] = m.y, mw[2] = m.z, mw[3] = m.w;
    }
    for (int c = 0; c < 4; ++c) {
        const int col = 64 * wv + 16 * c + lr;
        for (int r = 0; r < 8; ++r)
            for (int j = 0; j < 4; ++j) {
                const int64_t row = blk * kRows + 16 * r + 4 * lg + j;
                if (row >= rows) continue;
                uint8_t* d = dec + (row * kDepth + l) * kWidth + col;
                if (WRITE)
                    mw[c] |= (*d != 0 ? 1u : 0u) << mask_bit(r, j);
                else
                    *d = (uint8_t)((mw[c] >> mask_bit(r, j)) & 1u);
            }
    }
    if (WRITE) mask[w] = make_uint4(mw[0], mw[1], mw[2], mw[3]);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_mlp_bwd(Args a, const float* __restrict__ d_delta,
                                                 float* __restrict__ dxr) {
    __shared__ __attribute__((aligned(16))) bf16 X[kRows * kLDX];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * kRows;
    {   // gz_8 = dL/d delta of the block's rows, padded to kHeadK columns
        const int rr = tid >> 1, half = tid & 1;
        const int64_t r = r0 + rr;
        float g[4] = {0.f, 0.f, 0.f, 0.f};
        if (r < a.rows) {
            const int t = (int)(r / a.n);
            const int64_t k = r - (int64_t)t * a.n;
            for (int c = 0; c < 3; ++c) g[c] = d_delta[((int64_t)t * 3 + c) * a.n + k];
        }
        for (int c = 16 * half; c < 16 * half + 16; ++c)
            X[rr * kLDX + c] = (bf16)(c < 3 ? pick4(g, c) : 0.f);
    }
    __syncthreads();
    save_block<kOutPad>(X, a.GZ[kDepth], r0, tid);

    f32x4 acc[8][4];
    const int col0 = 64 * wv;
    // the forward's ReLU decisions for h_{l+1} (layer l's output), loaded
    // before the product so that their latency hides behind it
    uint4 hm;
    auto load_masks = [&](int l) { hm = a.mask[((size_t)blockIdx.x * kDepth + l) * 256 + tid]; };
    // rows r0 + 16 r + 4 lg .. +3 of feature col0 + 16 c + lr of a row-blocked
    // array sit at base + r * 2 kWidth 8 + c * 128
    const size_t base = ((size_t)(r0 / 8 + (lg >> 1)) * kWidth + col0 + lr) * 8 + 4 * (lg & 1);
    load_masks(kDepth - 1);
    zero(acc);
    gemm_128x64<kHeadK, false>(X, a.wt[kDepth], col0, acc, lane);   // g_8 = gz_8 W_8
    for (int l = kDepth - 1; l >= 0; --l) {
        __syncthreads();
        // gz_l = g_{l+1} * [h_{l+1} > 0]
        bf16* gzb = a.GZ[l] + base;
        const uint32_t mw[4] = {hm.x, hm.y, hm.z, hm.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = col0 + 16 * c + lr;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const size_t o = (size_t)r * (2 * kWidth * 8) + c * 128;
                // bfloat16 first, then the gates as 16-bit masks: shifting the
                // word puts the bits of elements (0, 1), then (2, 3), at bits 15
                // and 31, and an arithmetic shift of each half by 15 spreads them
                uint2 z = __builtin_bit_cast(uint2, __builtin_convertvector(acc[r][c], bf16x4));
                z.x &= __builtin_bit_cast(uint32_t, __builtin_bit_cast(s16x2, mw[c] << (15 - r)) >> (short)15);
                z.y &= __builtin_bit_cast(uint32_t, __builtin_bit_cast(s16x2, mw[c] << (7 - r)) >> (short)15);
                const bf16x4 v = __builtin_bit_cast(bf16x4, z);
#pragma unroll
                for (int j = 0; j < 4; ++j) X[(16 * r + 4 * lg + j) * kLDX + col] = v[j];
                *(bf16x4*)(gzb + o) = v;
            }
        }
        __syncthreads();
        if (l > 0) {
            load_masks(l - 1);
            zero(acc);
            gemm_128x64<kWidth, false>(X, a.wt[l], col0, acc, lane);   // g_l = gz_l W_l
        }
    }
    // g_0 = gz_0 W_0 -> [128][96]: wave w takes rows 32w .. 32w+31, all 6 column tiles
    f32x4 g0[2][6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) g0[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    {
        const bf16* bp = a.wt[0] + (size_t)lr * kWidth + 8 * lg;
#pragma unroll 2
        for (int k0 = 0; k0 < kWidth; k0 += 32) {
            bf16x8 b[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) b[c] = *(const bf16x8*)(bp + (size_t)16 * c * kWidth + k0);
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const bf16x8 x = *(const bf16x8*)(X + (32 * wv + 16 * r + lr) * kLDX + 8 * lg + k0);
#pragma unroll
                for (int c = 0; c < 6; ++c) g0[r][c] = mfma(x, b[c], g0[r][c]);
            }
        }
    }
    __syncthreads();
    constexpr int kLDF = kK0 + 4;   // float stride of g_0 in LDS
    float* XF = reinterpret_cast<float*>(X);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) XF[(32 * wv + 16 * r + 4 * lg + j) * kLDF + 16 * c + lr] = g0[r][c][j];
    __syncthreads();
    {   // d(scaled centre) = sum over the x features of g_0 * d enc / d p; two threads per row
        const int rr = tid >> 1, half = tid & 1;
        const int64_t r = r0 + rr;
        float xin[4];
        row_inputs(a, r, xin);
        float s0 = 0.f, s1 = 0.f, s2 = 0.f;
        for (int f = 48 * half; f < 48 * half + 48; ++f) {
            int blk;
            const int c = feat_src(f, a.lx, a.lt, blk);
            if (c < 0 || c > 2) continue;
            const float v = XF[rr * kLDF + f] * enc_d(pick4(xin, c), blk);
            s0 += c == 0 ? v : 0.f;
            s1 += c == 1 ? v : 0.f;
            s2 += c == 2 ? v : 0.f;
        }
        s0 += __shfl_xor(s0, 1, 64);
        s1 += __shfl_xor(s1, 1, 64);
        s2 += __shfl_xor(s2, 1, 64);
        if (half == 0 && r < a.rows) {
            dxr[r * 3 + 0] = a.sx * s0;
            dxr[r * 3 + 1] = a.sx * s1;
            dxr[r * 3 + 2] = a.sx * s2;
        }
    }
}

// dW_l [NO][NI] and db_l [NO] of one row chunk.  8 waves: OG groups of output
// rows times IG groups of input columns; each wave keeps MT x NT tiles.
struct DwArgs {
    const bf16* GZ[kLayers];
    const bf16* H[kLayers];
    int64_t part_off[kLayers];
    int64_t part_stride, rows_pad, rows_per_chunk;
    float* part;
};

template <int NO, int NI, int OG, int IG>
__global__ void __launch_bounds__(512) k_mlp_dw(DwArgs d, int l0) {
    constexpr int MT = NO / 16 / OG, NT = NI / 16 / IG;
    static_assert(OG * IG == 8 && MT * 16 * OG == NO && NT * 16 * IG == NI, "tiling");
    // One stage is two k-steps of 32 rows = 8 row blocks of gz (NO features)
    // and h (NI features), 16 bytes per (row block, feature): staged once per
    // workgroup in LDS, double-buffered, and read from there by the 8 waves
    // (each gradient tile is read by IG waves and each activation tile by OG).
    constexpr int NC = 8 * (NO + NI);
    constexpr int PER = (NC + 511) / 512;
    __shared__ bf16x8 sbuf[2][NC];
    const int l = l0 + blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int o0 = (wv / IG) * MT * 16, i0 = (wv % IG) * NT * 16;
    const bf16* __restrict__ GZ = d.GZ[l];
    const bf16* __restrict__ H = d.H[l];
    const int64_t rs = (int64_t)blockIdx.x * d.rows_per_chunk;
    const int64_t re = min(rs + d.rows_per_chunk, d.rows_pad);   // both multiples of 64
    const int nk = rs < re ? (int)((re - rs) / 64) : 0;          // stages; chunks hold multiples of 64 rows
    f32x4 acc[MT][NT];
    // db on the matrix cores: the product with a fragment of ones sums every
    // output row over the chunk's rows (the waves of the first input group)
    f32x4 ab[MT];
    bf16x8 ones;
#pragma unroll
    for (int e = 0; e < 8; ++e) ones[e] = (bf16)1.0f;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        ab[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    // chunk q < 8 NO: gz row block q / NO, feature q % NO; else h likewise
    bf16x8 stg[PER];
    auto fetch = [&](int64_t kb) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int q = tid + 512 * p;
            if (q < NC) {
                if (q < 8 * NO) {
                    const int rb = q / NO, f = q - rb * NO;
                    stg[p] = *(const bf16x8*)(GZ + ((size_t)(kb + rb) * NO + f) * 8);
                } else {
                    const int qh = q - 8 * NO, rb = qh / NI, f = qh - rb * NI;
                    stg[p] = *(const bf16x8*)(H + ((size_t)(kb + rb) * NI + f) * 8);
                }
            }
        }
    };
    auto stage = [&](int b) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int q = tid + 512 * p;
            if (q < NC) sbuf[b][q] = stg[p];
        }
    };
    const int64_t kb0 = rs / 8;
    if (nk > 0) {
        fetch(kb0);
        stage(0);
    }
    __syncthreads();
    for (int k = 0; k < nk; ++k) {
        const int cur = k & 1;
        const bool more = k + 1 < nk;
        if (more) fetch(kb0 + 8 * (k + 1));   // in flight during this stage's products
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf16x8 av[MT], bv[NT];
#pragma unroll
            for (int m = 0; m < MT; ++m) av[m] = sbuf[cur][(4 * h + lg) * NO + o0 + 16 * m + lr];
#pragma unroll
            for (int t = 0; t < NT; ++t) bv[t] = sbuf[cur][8 * NO + (4 * h + lg) * NI + i0 + 16 * t + lr];
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[m][t] = mfma(av[m], bv[t], acc[m][t]);
            if (i0 == 0)
#pragma unroll
                for (int m = 0; m < MT; ++m) ab[m] = mfma(av[m], ones, ab[m]);
        }
        if (more) stage(cur ^ 1);   // the other buffer was last read before the previous barrier
        __syncthreads();
    }
    float* P = d.part + (int64_t)blockIdx.x * d.part_stride + d.part_off[l];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                P[(size_t)(o0 + 16 * m + 4 * lg + j) * NI + i0 + 16 * t + lr] = acc[m][t][j];
    if (i0 == 0 && lr == 0) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int j = 0; j < 4; ++j) P[(size_t)NO * NI + o0 + 16 * m + 4 * lg + j] = ab[m][j];
    }
}

struct RedArgs {
    int64_t off_w[kLayers], off_b[kLayers], part_off[kLayers];
    int out[kLayers], in[kLayers];
    int64_t n_params, part_stride;
    int n_chunks;
};

// parameter gradient = sum of the chunk partials, chunk 0 first
__global__ void __launch_bounds__(256) k_mlp_reduce(RedArgs r, const float* __restrict__ part,
                                                    float* __restrict__ d_params) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= r.n_params) return;
    int l = 0;
    while (l + 1 < kLayers && p >= r.off_w[l + 1]) ++l;
    int64_t src;
    if (p < r.off_b[l]) {
        const int64_t e = p - r.off_w[l];
        const int o = (int)(e / r.in[l]), i = (int)(e - (int64_t)o * r.in[l]);
        src = r.part_off[l] + (int64_t)o * pad_in(l) + i;
    } else {
        src = r.part_off[l] + (int64_t)pad_out(l) * pad_in(l) + (p - r.off_b[l]);
    }
    // eight partials loaded at a time, added in chunk order
    float s = 0.f;
    int c = 0;
    for (; c + 8 <= r.n_chunks; c += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(c + j) * r.part_stride + src];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; c < r.n_chunks; ++c) s += part[(int64_t)c * r.part_stride + src];
    d_params[p] = s;
}

__global__ void __launch_bounds__(256) k_mlp_dx0(const float* __restrict__ dxr, int64_t n, int T,
                                                 int accumulate, float* __restrict__ d_x0) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    for (int t = 0; t < T; ++t) {
        const float* g = dxr + ((int64_t)t * n + k) * 3;
        s0 += g[0];
        s1 += g[1];
        s2 += g[2];
    }
    if (accumulate) {
        s0 += d_x0[k];
        s1 += d_x0[n + k];
        s2 += d_x0[2 * n + k];
    }
    d_x0[k] = s0;
    d_x0[n + k] = s1;
    d_x0[2 * n + k] = s2;
}

struct PackArgs {
    int64_t off_w[kLayers];
    int out[kLayers], in[kLayers];
    bf16* wf[kLayers];
    bf16* wt[kLayers];
};

__global__ void __launch_bounds__(256) k_mlp_pack(PackArgs p, const float* __restrict__ params) {
    const int l = blockIdx.y;
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int out = p.out[l], in = p.in[l];
    const float* W = params + p.off_w[l];
    const int NO = pad_out(l), NI = pad_in(l), KO = pad_k(l);
    if (e < NO * NI) {
        const int o = e / NI, i = e - o * NI;
        p.wf[l][e] = (bf16)((o < out && i < in) ? W[(int64_t)o * in + i] : 0.f);
    }
    if (e < NI * KO) {
        const int i = e / KO, o = e - i * KO;
        p.wt[l][e] = (bf16)((o < out && i < in) ? W[(int64_t)o * in + i] : 0.f);
    }
}

// Eq. 7 weights of a frame (1, 0 without anchors)
__device__ __forceinline__ void eq7_weights(const gftorf_frame& fr, float& w1, float& w2) {
    if (fr.t_hi > fr.t_lo) {
        const float span = fr.t_hi - fr.t_lo;
        w1 = (fr.t_hi - fr.time) / span;
        w2 = (fr.time - fr.t_lo) / span;
    } else {
        w1 = 1.0f;
        w2 = 0.0f;
    }
}

// out[f] = w1_f steps[lo_f] + w2_f steps[hi_f], one thread per (frame, element)
__global__ void __launch_bounds__(256) k_blend(Blend b, const float* __restrict__ steps,
                                               const gftorf_frame* __restrict__ frames,
                                               float* __restrict__ out) {
    const int64_t per = 3 * b.n;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)b.n_frames * per) return;
    const int f = (int)(i / per);
    const int64_t e = i - (int64_t)f * per;
    float w1, w2;
    eq7_weights(frames[f], w1, w2);
    float v = w1 * steps[(int64_t)b.anchors[2 * f] * per + e];
    if (w2 != 0.0f) v += w2 * steps[(int64_t)b.anchors[2 * f + 1] * per + e];
    out[i] = v;
}

// d_steps[s] = sum over frames (in frame order) of the weight of s times d_frames[f]
__global__ void __launch_bounds__(256) k_blend_bwd(Blend b, const float* __restrict__ d_frames,
                                                   const gftorf_frame* __restrict__ frames,
                                                   float* __restrict__ d_steps) {
    const int64_t per = 3 * b.n;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)b.n_steps * per) return;
    const int st = (int)(i / per);
    const int64_t e = i - (int64_t)st * per;
    float acc = 0.0f;
    for (int f = 0; f < b.n_frames; ++f) {
        const int lo = b.anchors[2 * f], hi = b.anchors[2 * f + 1];
        if (lo != st && hi != st) continue;
        float w1, w2;
        eq7_weights(frames[f], w1, w2);
        const float g = d_frames[(int64_t)f * per + e];
        if (lo == st) acc += w1 * g;
        if (hi == st && w2 != 0.0f) acc += w2 * g;
    }
    d_steps[i] = acc;
}

Args make_args(const Layout& L, const Call& c) {
    Args a;
    a.x0 = c.x0;
    a.n = L.n;
    a.rows = L.rows;
    a.lx = L.lx;
    a.lt = L.lt;
    a.sx = c.sx;
    a.st = c.st;
    for (int t = 0; t < kMaxTimes; ++t) a.times[t] = t < L.n_times ? c.times[t] : 0.f;
    a.frames = c.frames;
    for (int l = 0; l < kLayers; ++l) {
        a.wf[l] = reinterpret_cast<const bf16*>(c.ws + L.wf[l]);
        a.wt[l] = reinterpret_cast<const bf16*>(c.ws + L.wt[l]);
        a.bias[l] = c.params + L.off_b[l];
        a.H[l] = L.training ? reinterpret_cast<bf16*>(c.ws + L.H[l]) : nullptr;
        a.GZ[l] = L.training ? reinterpret_cast<bf16*>(c.ws + L.GZ[l]) : nullptr;
    }
    a.mask = L.training ? reinterpret_cast<uint4*>(c.ws + L.mask) : nullptr;
    return a;
}

}  // namespace

hipError_t noalloc_scratch(char** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static char* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || reinterpret_cast<uintptr_t>(p) % 256) return hipErrorInvalidValue;
        addr[dev] = static_cast<char*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

bool make_layout(int lx, int lt, int width, int depth, int64_t n, int n_times, bool training,
                 Layout* L) {
    if (width != kWidth || depth != kDepth || lx < 0 || lt < 0 || n < 1 || n_times < 1 ||
        n_times > kMaxTimes)
        return false;
    const int n_in = 3 * (1 + 2 * lx) + 1 + 2 * lt;
    if (n_in > kK0 || n > (int64_t(1) << 40) / n_times) return false;
    L->lx = lx;
    L->lt = lt;
    L->n_in = n_in;
    int64_t off = 0;
    for (int l = 0; l < kLayers; ++l) {
        L->out[l] = l == kDepth ? 3 : kWidth;
        L->in[l] = l == 0 ? n_in : kWidth;
        L->off_w[l] = off;
        off += (int64_t)L->out[l] * L->in[l];
        L->off_b[l] = off;
        off += L->out[l];
    }
    L->n_params = off;
    L->n = n;
    L->n_times = n_times;
    L->rows = n * n_times;
    L->rows_pad = (L->rows + kRows - 1) / kRows * kRows;
    int64_t rpc = (L->rows_pad + kMaxChunks - 1) / kMaxChunks;
    rpc = (rpc + 63) / 64 * 64;   // whole 64-row stages of the weight-gradient kernel
    L->rows_per_chunk = rpc;
    L->n_chunks = (int)((L->rows_pad + rpc - 1) / rpc);
    int64_t po = 0;
    for (int l = 0; l < kLayers; ++l) {
        L->part_off[l] = po;
        po += (int64_t)pad_out(l) * pad_in(l) + pad_out(l);
    }
    L->part_stride = po;
    size_t b = 0;
    auto take = [&](size_t bytes) {
        const size_t at = b;
        b += (bytes + 255) / 256 * 256;
        return at;
    };
    for (int l = 0; l < kLayers; ++l) {
        L->wf[l] = take((size_t)pad_out(l) * pad_in(l) * 2);
        L->wt[l] = take((size_t)pad_in(l) * pad_k(l) * 2);
    }
    for (int l = 0; l < kLayers; ++l) L->H[l] = L->GZ[l] = 0;
    L->mask = L->dxr = L->part = 0;
    if (training) {
        for (int l = 0; l < kLayers; ++l) L->H[l] = take((size_t)L->rows_pad * pad_in(l) * 2);
        for (int l = 0; l < kLayers; ++l) L->GZ[l] = take((size_t)L->rows_pad * pad_out(l) * 2);
        // ReLU bits: 16 bytes per thread, layer and 128-row block = 2 bytes per row and unit
        L->mask = take((size_t)(L->rows_pad / kRows) * kDepth * 256 * 16);
        L->dxr = take((size_t)L->rows_pad * 3 * 4);
        L->part = take((size_t)L->n_chunks * L->part_stride * 4);
    }
    L->bytes = b;
    L->training = training;
    return true;
}

hipError_t launch_fwd(const Layout& L, const Call& c, float* delta, bool save, hipStream_t s) {
    PackArgs p;
    for (int l = 0; l < kLayers; ++l) {
        p.off_w[l] = L.off_w[l];
        p.out[l] = L.out[l];
        p.in[l] = L.in[l];
        p.wf[l] = reinterpret_cast<bf16*>(c.ws + L.wf[l]);
        p.wt[l] = reinterpret_cast<bf16*>(c.ws + L.wt[l]);
    }
    {
        ProfScope _p("k_mlp_pack", s);
        hipLaunchKernelGGL(k_mlp_pack, dim3(kWidth * kWidth / 256, kLayers), dim3(256), 0, s, p, c.params);
    }
    const Args a = make_args(L, c);
    const unsigned blocks = (unsigned)(L.rows_pad / kRows);
    ProfScope _f("k_mlp_fwd", s);
    if (save)
        hipLaunchKernelGGL(k_mlp_fwd<true>, dim3(blocks), dim3(256), 0, s, a, delta);
    else
        hipLaunchKernelGGL(k_mlp_fwd<false>, dim3(blocks), dim3(256), 0, s, a, delta);
    return hipGetLastError();
}

hipError_t launch_blend(const Blend& b, const float* steps, const gftorf_frame* frames, float* out,
                        hipStream_t s) {
    const int64_t total = (int64_t)b.n_frames * 3 * b.n;
    if (total == 0) return hipSuccess;
    ProfScope _p("k_blend", s);
    hipLaunchKernelGGL(k_blend, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, b, steps, frames, out);
    return hipGetLastError();
}

hipError_t launch_blend_bwd(const Blend& b, const float* d_frames, const gftorf_frame* frames,
                            float* d_steps, hipStream_t s) {
    const int64_t total = (int64_t)b.n_steps * 3 * b.n;
    if (total == 0) return hipSuccess;
    ProfScope _p("k_blend_bwd", s);
    hipLaunchKernelGGL(k_blend_bwd, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, b, d_frames,
                       frames, d_steps);
    return hipGetLastError();
}

hipError_t launch_bwd(const Layout& L, const Call& c, const float* d_delta, float* d_params,
                      float* d_x0, bool accumulate_x0, hipStream_t s) {
    const Args a = make_args(L, c);
    float* dxr = reinterpret_cast<float*>(c.ws + L.dxr);
    {
        ProfScope _b("k_mlp_bwd", s);
        hipLaunchKernelGGL(k_mlp_bwd, dim3((unsigned)(L.rows_pad / kRows)), dim3(256), 0, s, a,
                           d_delta, dxr);
    }
    DwArgs d;
    for (int l = 0; l < kLayers; ++l) {
        d.GZ[l] = a.GZ[l];
        d.H[l] = a.H[l];
        d.part_off[l] = L.part_off[l];
    }
    d.part_stride = L.part_stride;
    d.rows_pad = L.rows_pad;
    d.rows_per_chunk = L.rows_per_chunk;
    d.part = reinterpret_cast<float*>(c.ws + L.part);
    {
        ProfScope _w("k_mlp_dw", s);
        const unsigned nc = (unsigned)L.n_chunks;
        hipLaunchKernelGGL((k_mlp_dw<kWidth, kWidth, 4, 2>), dim3(nc, kDepth - 1), dim3(512), 0, s, d, 1);
        hipLaunchKernelGGL((k_mlp_dw<kWidth, kK0, 4, 2>), dim3(nc, 1), dim3(512), 0, s, d, 0);
        hipLaunchKernelGGL((k_mlp_dw<kOutPad, kWidth, 1, 8>), dim3(nc, 1), dim3(512), 0, s, d, kDepth);
    }
    RedArgs r;
    for (int l = 0; l < kLayers; ++l) {
        r.off_w[l] = L.off_w[l];
        r.off_b[l] = L.off_b[l];
        r.part_off[l] = L.part_off[l];
        r.out[l] = L.out[l];
        r.in[l] = L.in[l];
    }
    r.n_params = L.n_params;
    r.part_stride = L.part_stride;
    r.n_chunks = L.n_chunks;
    {
        ProfScope _r("k_mlp_reduce", s);
        hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)((L.n_params + 255) / 256)), dim3(256), 0, s, r,
                           d.part, d_params);
        if (d_x0)
            hipLaunchKernelGGL(k_mlp_dx0, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, s, dxr, L.n,
                               L.n_times, accumulate_x0 ? 1 : 0, d_x0);
    }
    return hipGetLastError();
}

hipError_t launch_decisions(const Layout& L, char* ws, uint8_t* dec, bool write, hipStream_t s) {
    if (!L.training) return hipErrorInvalidValue;
    uint4* mask = reinterpret_cast<uint4*>(ws + L.mask);
    const int64_t words = L.rows_pad / kRows * kDepth * 256;
    const unsigned blocks = (unsigned)((words + 255) / 256);
    if (write)
        hipLaunchKernelGGL(k_mlp_decisions<true>, dim3(blocks), dim3(256), 0, s, mask, dec, L.rows, words);
    else
        hipLaunchKernelGGL(k_mlp_decisions<false>, dim3(blocks), dim3(256), 0, s, mask, dec, L.rows, words);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace gft
