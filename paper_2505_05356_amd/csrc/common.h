// Internal definitions shared by the gfx950 kernels and the host ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gftorf.h"

namespace gft {

constexpr double kSpeedOfLight = 299792458.0;   // m/s
constexpr float kLog2e = 1.4426950408889634f;

// Radix sort geometry: 256 threads (4 wave64), 8 keys per thread.
constexpr uint32_t kCulledKey = 0xffffffffu;   // depth key of a culled item
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;   // 2048 keys per tile
constexpr int kSortBuckets = 256;                       // <= 8 digit bits per pass
constexpr int kSortPasses = 4;                          // 32-bit keys
// Batches of at most this many sort tiles (all frames) sort with one launch
// per pass (decoupled look-back over the frame's earlier tiles) after one
// histogram launch; larger batches use three launches per pass.
constexpr int64_t kOneSweepMaxTiles = 256;
// Words of the one-sweep control block: the next tile of each pass, then the
// flag set when a look-back wait gave up.
constexpr int kSortCtlWords = 8;
constexpr int kSortFault = kSortPasses;

// Tile binning works on chunks of depth-sorted items of one frame, first into
// groups of 8x8 tiles (one LDS counter per group of a frame), then into tiles.
constexpr int kMaxTilesPerFrame = 1 << 20;
constexpr int kMaxGroupsPerFrame = 1024;   // groups of 8x8 tiles (LDS counters)
struct BinGeom {
    int C;                 // items per level-A chunk
    int QC;                // chunks per frame
    int ng;                // groups of 8x8 tiles per frame
    int S;                 // group-list entries per level-B segment
    int R;                 // segments per placement chunk (R * S entries)
    int64_t max_segments;  // bound on the level-B segments
};
BinGeom bin_geometry(int64_t n, int32_t n_frames, int ntx, int nty, uint64_t cap);

// Per-(frame, Gaussian) record in float4 units.
//   r0 = {u_hi, v_hi, u_lo, v_lo}   pixel centre as an unevaluated float pair
//   r1 = {red, green, blue, d}     colour and range to the optical centre
//   r2.. = {a sin psi_f, a cos psi_f} for each frequency f (two per float4)
// and, in an array of its own (the preprocess backward reads only it),
//   conic = {cA, cB, cC, o}        conic pre-scaled by -log2(e) (x 1/2 on A, C)
__host__ __device__ constexpr int record_float4s(int nf) { return 2 + (nf + 1) / 2; }
// The composite kernels stage an entry as float4 slots: 0 the centre
// relative to the tile, 1 the conic, 2 colour and range, 3.. the phasors.
__host__ __device__ constexpr int staged_float4s(int nf) { return record_float4s(nf) + 1; }
// Gradient record per (frame, Gaussian), in floats:
//   du, dv, dcA, dcB, dcC, do, dred, dgreen, dblue, dd, {d(a sin), d(a cos)} x nf
__host__ __device__ constexpr int grad_floats(int nf) { return ((10 + 2 * nf) + 3) / 4 * 4; }

// Workspace header, at offset 0 of the workspace.
struct Status {
    unsigned long long n_pairs;   // total pairs of the last forward
    unsigned long long cap;       // capacity (max_pairs)
    unsigned int overflow;
    unsigned int nonfinite;
    unsigned long long wcount_off;   // byte offset of the forward's per-work-item counts
    unsigned long long n_items;      // work items (frames x tiles) of the last forward
    unsigned int magic;              // kStatusMagic once a forward has filled the fields
    // sticky over every forward since the header was last cleared: OR of the
    // overflow flags and the largest pair count
    unsigned int overflow_seen;
    unsigned long long n_pairs_seen;
    unsigned int sort_fault;         // the last forward's depth sort gave up a look-back wait
    unsigned int pad;
};
static_assert(sizeof(Status) == 64, "the status header is the workspace's first 64 bytes");
constexpr unsigned int kStatusMagic = 0x47465352u;
// The (evaluations, composited) counts of every work item are summed on the
// host by gftorf_read_status, which synchronises anyway, so no forward pays a
// reduction launch for them.

// Everything a kernel needs to know about a call, passed by value.
struct Params {
    int64_t n;              // Gaussians
    int32_t F;              // frames
    int32_t W, H;
    int32_t tw, th, ntx, nty, n_tiles;
    int32_t nf, nphi, nq;
    double freq[GFTORF_MAX_FREQ];
    float cphi[GFTORF_MAX_PHASE], sphi[GFTORF_MAX_PHASE];
    float alpha_min, alpha_max, T_min, extent, dilation, near_z, s_int;
    int32_t bg_pow;
    unsigned long long cap;  // pair capacity
};

// Device pointers carved out of the caller's workspace.
struct Workspace {
    Status* status;
    float4* rec;            // [M][record_float4s]
    float4* conic;          // [M]
    uint32_t* cnt;          // [M] tiles covered
    uint32_t* nf_block;     // [ceil(n / 256)] non-finite Gaussians per preprocess block
    uint32_t* dkey[2];      // [M] depth keys (double buffer)
    uint32_t* dval[2];      // [M] item ids
    uint2* drect[2];        // [M] tile rectangles (x_lo | x_hi << 16, y_lo | y_hi << 16), sort payload
    uint32_t* counts;       // [F][256][max_sort_tiles] per-tile digit counts of the depth sort
    uint32_t* totals;       // [F][256] digit totals per frame
    uint32_t* sctl;         // [kSortCtlWords + F * kSortPasses * 256] one-sweep control words,
                            // then the digit counts of every frame and pass (shist)
    uint32_t* shist;        // = sctl + kSortCtlWords
    uint32_t* slook[2];     // [F * max_sort_tiles][256] look-back words (one-sweep batches only)
    uint32_t* cntA;         // [F][QC][ng] per-chunk group counts, then column prefixes
    uint32_t* lenA;         // [F * ng] group-list lengths
    uint2* granges;         // [F * ng] group-list ranges in gval
    uint32_t* seg_start;    // [F * ng + 1] first level-B segment of each group
    uint32_t* chunk_start;  // [F * ng + 1] first placement chunk (R segments) of each group
    uint4* chunk_info;      // [max chunks] per placement chunk: group, first and end entry, first segment
    uint32_t* gval;         // [cap] item ids of the group lists
    uint16_t* gloc;         // [cap] their rectangles clipped to the group, 3 bits per bound
    uint32_t* cntB;         // [max_segments][64] per-segment tile counts, then prefixes
    uint32_t* tcount;       // [F * n_tiles] pairs per (frame, tile)
    uint2* ranges;          // [F * n_tiles] [start, end) of each tile list in tval
    uint32_t* tval;         // [cap] item ids of the tile lists
    uint2* wcount;          // [F * n_tiles] forward (evaluations, composited) per work item
    float* grec;            // [M][grad_floats]
    int64_t M;
    int64_t max_sort_tiles;
    size_t bytes;
};

// Carves `base` (may be NULL to only compute the size).
inline Workspace carve(void* base, int64_t n, int32_t F, int nf, int ntx, int nty, uint64_t cap) {
    const int n_tiles = ntx * nty;
    Workspace w{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) & ~size_t(255);
        char* p = base ? static_cast<char*>(base) + off : nullptr;
        off += bytes;
        return p;
    };
    const int64_t M = n * F;
    const BinGeom g = bin_geometry(n, F, ntx, nty, cap);
    w.M = M;
    w.max_sort_tiles = (n + kSortTile - 1) / kSortTile;   // sort tiles per frame
    if (w.max_sort_tiles < 1) w.max_sort_tiles = 1;
    const int64_t K = (int64_t)F * n_tiles;
    w.status = reinterpret_cast<Status*>(take(sizeof(Status)));
    w.rec = reinterpret_cast<float4*>(take(sizeof(float4) * record_float4s(nf) * M));
    w.conic = reinterpret_cast<float4*>(take(sizeof(float4) * M));
    w.cnt = reinterpret_cast<uint32_t*>(take(4 * M));
    w.nf_block = reinterpret_cast<uint32_t*>(take(4 * (size_t)((n + 255) / 256 + 1)));
    for (int i = 0; i < 2; ++i) w.dkey[i] = reinterpret_cast<uint32_t*>(take(4 * M));
    for (int i = 0; i < 2; ++i) w.dval[i] = reinterpret_cast<uint32_t*>(take(4 * M));
    for (int i = 0; i < 2; ++i) w.drect[i] = reinterpret_cast<uint2*>(take(sizeof(uint2) * M));
    w.counts = reinterpret_cast<uint32_t*>(take(4 * (size_t)F * kSortBuckets * w.max_sort_tiles));
    w.totals = reinterpret_cast<uint32_t*>(take(4 * (size_t)F * kSortBuckets));
    w.sctl = reinterpret_cast<uint32_t*>(take(4 * ((size_t)kSortCtlWords + (size_t)F * kSortPasses * kSortBuckets)));
    w.shist = w.sctl ? w.sctl + kSortCtlWords : nullptr;
    const int64_t sort_tiles = (int64_t)F * w.max_sort_tiles;
    const size_t look_words = sort_tiles <= kOneSweepMaxTiles ? (size_t)sort_tiles * kSortBuckets : 0;
    for (int i = 0; i < 2; ++i) w.slook[i] = reinterpret_cast<uint32_t*>(take(4 * look_words));
    const int64_t KG = (int64_t)F * g.ng;
    w.cntA = reinterpret_cast<uint32_t*>(take(4 * (size_t)F * g.QC * g.ng));
    w.lenA = reinterpret_cast<uint32_t*>(take(4 * KG));
    w.granges = reinterpret_cast<uint2*>(take(sizeof(uint2) * KG));
    w.seg_start = reinterpret_cast<uint32_t*>(take(4 * (KG + 1)));
    w.chunk_start = reinterpret_cast<uint32_t*>(take(4 * (KG + 1)));
    w.chunk_info = reinterpret_cast<uint4*>(take(sizeof(uint4) * (size_t)((g.max_segments + g.R - 1) / g.R + KG)));
    w.gval = reinterpret_cast<uint32_t*>(take(4 * cap));
    w.gloc = reinterpret_cast<uint16_t*>(take(2 * cap));
    w.cntB = reinterpret_cast<uint32_t*>(take(4 * 64 * (size_t)g.max_segments));
    w.tcount = reinterpret_cast<uint32_t*>(take(4 * K));
    w.ranges = reinterpret_cast<uint2*>(take(sizeof(uint2) * K));
    w.tval = reinterpret_cast<uint32_t*>(take(4 * cap));
    w.wcount = reinterpret_cast<uint2*>(take(sizeof(uint2) * K));
    w.grec = reinterpret_cast<float*>(take(4 * (size_t)grad_floats(nf) * M));
    w.bytes = off + 256;
    return w;
}

// Block -> work-item remap so that each of the 8 XCDs (which receive blocks
// round-robin) processes one contiguous range of work items, keeping the
// records of neighbouring tiles and of one frame in that XCD's L2.
constexpr int kXcds = 8;   // accelerator complex dies, each with its own L2
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    constexpr int kX = kXcds;
    const int q = nb / kX, r = nb % kX;
    const int x = b % kX, i = b / kX;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ---- optional per-kernel timing with HIP events (capi.cpp) -----------------
// When profiling is on (gftorf_profile_begin), every launch is bracketed by
// two events on its stream; otherwise prof_start returns -1 and costs a load.
int prof_start(const char* name, hipStream_t s);
void prof_stop(int slot, hipStream_t s);
struct ProfScope {
    int slot;
    hipStream_t s;
    ProfScope(const char* name, hipStream_t st) : slot(prof_start(name, st)), s(st) {}
    ~ProfScope() { prof_stop(slot, s); }
};

// ---- host-side launchers (defined in the .hip files) -----------------------
void launch_preprocess(const Params& P, const gftorf_gaussians& g, const gftorf_frame* frames,
                       const Workspace& w, hipStream_t s);
int depth_sort_passes(int n_frames);
int launch_depth_sort(const Params& P, const Workspace& w, hipStream_t s);
// True when this batch sorts with one launch per pass (its few sort tiles
// make the look-back chains short); the preprocess then clears the sort's
// control words and digit counts.
inline bool one_sweep_sort(const Params& P, const Workspace& w) {
    return w.M > 0 && (int64_t)P.F * w.max_sort_tiles <= kOneSweepMaxTiles;
}
hipError_t launch_binning(const Params& P, const Workspace& w, int dbuf, hipStream_t s);
void launch_item_rects(const Workspace& w, int dbuf, uint2* out, hipStream_t s);
void launch_keys_from_ranges(const Params& P, const Workspace& w, uint32_t* keys,
                             unsigned long long limit, hipStream_t s);
hipError_t launch_composite_fwd(const Params& P, const gftorf_frame* frames, const Workspace& w,
                                const gftorf_outputs& out, hipStream_t s);
hipError_t launch_composite_bwd(const Params& P, const gftorf_frame* frames, const Workspace& w,
                                const gftorf_outputs& saved, const float* d_rgb,
                                const float* d_quad, const float* d_depth, float* d_bg,
                                hipStream_t s);
void launch_preprocess_bwd(const Params& P, const gftorf_gaussians& g, const gftorf_frame* frames,
                           const Workspace& w, const gftorf_gaussians_grad& grad, hipStream_t s);
void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void launch_l2_loss(const float* pred, const float* targets, const int32_t* frame_index,
                    int32_t n_frames, int64_t elems, float weight, float* grad, float* loss,
                    hipStream_t s);
void launch_adam(const gftorf_adam_group* groups, int32_t n_groups, int32_t* step, float b1,
                 float b2, float eps, hipStream_t s);
void launch_select_frames(gftorf_frame* frames, int32_t n_batch, const gftorf_frame* seq,
                          int32_t n_seq, const float* bg_table, int32_t n_bg, int32_t n_quad,
                          const int32_t* step, int32_t* frame_index, hipStream_t s);

}  // namespace gft
