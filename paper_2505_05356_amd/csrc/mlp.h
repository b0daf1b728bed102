// Deformation network (paper §4, "MLP"): workspace layout and launchers.
#pragma once

#include "common.h"

namespace gft {
namespace mlp {

constexpr int kWidth = 256;      // hidden units
constexpr int kDepth = 8;        // hidden layers; layer kDepth is the linear head
constexpr int kLayers = kDepth + 1;
constexpr int kK0 = 96;          // encoded input features, zero-padded
constexpr int kOutPad = 16;      // head outputs (3) padded to one matrix tile
constexpr int kHeadK = 32;       // head outputs padded to one k-step (backward)
constexpr int kRows = 128;       // rows per workgroup of the row-parallel kernels
constexpr int kMaxChunks = 144;  // row chunks of the weight-gradient reduction (~4 blocks per CU)
constexpr int kMaxTimes = GFTORF_MLP_MAX_TIMES;

// Padded matrix shapes of layer l: forward weights [NO][NI], transposed
// weights [NI][KO], activations h_l with NI features, gradients of the
// layer's pre-activations with NO features.
__host__ __device__ constexpr int pad_out(int l) { return l == kDepth ? kOutPad : kWidth; }
__host__ __device__ constexpr int pad_in(int l) { return l == 0 ? kK0 : kWidth; }
__host__ __device__ constexpr int pad_k(int l) { return l == kDepth ? kHeadK : kWidth; }

struct Layout {
    int lx, lt, n_in;                 // frequencies, real input features
    int out[kLayers], in[kLayers];    // real layer shapes
    int64_t off_w[kLayers], off_b[kLayers], n_params;
    int64_t n, rows, rows_pad;
    int n_times;
    int64_t rows_per_chunk;
    int n_chunks;
    int64_t part_off[kLayers], part_stride;   // floats
    // byte offsets into the workspace
    size_t wf[kLayers], wt[kLayers], H[kLayers], GZ[kLayers], mask, dxr, part, bytes;
    bool training;
};

// false if the configuration is unsupported
bool make_layout(int lx, int lt, int width, int depth, int64_t n, int n_times, bool training,
                 Layout* L);

struct Call {
    const float* params;
    const float* x0;
    float sx, st;
    float times[kMaxTimes];          // host times, or
    const gftorf_frame* frames;      // device frame descriptors whose .time is read
    char* ws;
};

hipError_t launch_fwd(const Layout& L, const Call& c, float* delta, bool save, hipStream_t s);

// Allocation-free inference forward: the packed weights go to a file-scope
// device array of kNoAllocScratchBytes instead of a caller workspace.
constexpr size_t kNoAllocScratchBytes = GFTORF_MLP_NOALLOC_SCRATCH_BYTES;
// Device address of the current GPU's copy of that array, resolved with
// hipGetSymbolAddress on the first call on each device and kept.
hipError_t noalloc_scratch(char** out);

constexpr int kMaxBlendFrames = GFTORF_MAX_BLEND_FRAMES;
struct Blend {
    int32_t anchors[2 * kMaxBlendFrames];   // (lo, hi) step of every frame
    int32_t n_frames, n_steps;
    int64_t n;
};
hipError_t launch_blend(const Blend& b, const float* steps, const gftorf_frame* frames, float* out,
                        hipStream_t s);
hipError_t launch_blend_bwd(const Blend& b, const float* d_frames, const gftorf_frame* frames,
                            float* d_steps, hipStream_t s);
// The training forward's ReLU decisions in ws as bytes dec[rows][kDepth][kWidth]:
// read them out (write = false) or replace them (write = true).
hipError_t launch_decisions(const Layout& L, char* ws, uint8_t* dec, bool write, hipStream_t s);
hipError_t launch_bwd(const Layout& L, const Call& c, const float* d_delta, float* d_params,
                      float* d_x0, bool accumulate_x0, hipStream_t s);

}  // namespace mlp
}  // namespace gft
