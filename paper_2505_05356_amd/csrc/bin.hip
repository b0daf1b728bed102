// Tile binning: per-(frame, tile) Gaussian lists in depth order, built from
// the frame-major depth-sorted items without sorting (tile, Gaussian) pairs.
//
// The compositing loop of paper §3 walks, for every pixel, the Gaussians of
// its tile front to back.  Each item (frame, Gaussian) covers a rectangle of
// tiles; its entry for tile t must sit at start[t] + (number of items before
// it in depth order that cover t).  The lists are built in two levels:
//
// Level A -- items into groups of 8x8 tiles.  The depth-ordered items of a
//   frame are cut into chunks: per-chunk group counts (LDS), a column scan
//   over the chunks, an exclusive scan over (frame, group), then one wave per
//   chunk places its items in depth order into the group lists.  An item
//   touches only a few groups, so these lists are short.
// Level B -- group lists into tile lists.  Each group list is cut into
//   segments of 512 entries; one wave per segment, lane l owning tile l of
//   the group.  A counting pass, a column scan over each group's segments and
//   an exclusive scan over (frame, tile) give every lane a cursor; the
//   placing pass then walks the segment in order and each lane appends the
//   items that cover its tile.  Every tile list is written by one lane at a
//   time in increasing addresses, so the writes coalesce, and the order is
//   the depth order by construction.
#include "block_scan.h"
#include "common.h"

namespace gft {

namespace {

constexpr int kGroupW = 8, kGroupH = 8;   // tiles per group (one per lane)
constexpr int kLine = 32;                 // u32 entries per 128-byte cache line

__device__ __forceinline__ void unpack_rect(uint2 rc, uint32_t& xlo, uint32_t& xhi, uint32_t& ylo,
                                            uint32_t& yhi) {
    xlo = rc.x & 0xffff;
    xhi = rc.x >> 16;
    ylo = rc.y & 0xffff;
    yhi = rc.y >> 16;
}

struct Groups {
    int ngx, ngy, ng;   // groups per row, per column, per frame
};

__device__ __forceinline__ Groups groups_of(const Params& P) {
    Groups g;
    g.ngx = (P.ntx + kGroupW - 1) / kGroupW;
    g.ngy = (P.nty + kGroupH - 1) / kGroupH;
    g.ng = g.ngx * g.ngy;
    return g;
}

// ---- level A: items -> groups ----------------------------------------------

__global__ void __launch_bounds__(256) k_group_count(Params P, int C, int QC,
                                                     const uint32_t* __restrict__ dval,
                                                     const uint32_t* __restrict__ cnt,
                                                     const uint2* __restrict__ rect,
                                                     uint32_t* __restrict__ cntA) {
    __shared__ uint32_t lcnt[kMaxGroupsPerFrame];
    const Groups G = groups_of(P);
    const int chunk = blockIdx.x;
    const int f = chunk / QC, q = chunk - f * QC;
    for (int t = threadIdx.x; t < G.ng; t += 256) lcnt[t] = 0;
    __syncthreads();
    const long long beg = (long long)f * P.n + (long long)q * C;
    const long long end = min(beg + C, (long long)(f + 1) * P.n);
    for (long long j = beg + threadIdx.x; j < end; j += 256) {
        const uint32_t item = dval[j];
        if (cnt[item] == 0) continue;
        uint32_t xlo, xhi, ylo, yhi;
        unpack_rect(rect[item], xlo, xhi, ylo, yhi);
        for (uint32_t gy = ylo / kGroupH; gy <= yhi / kGroupH; ++gy)
            for (uint32_t gx = xlo / kGroupW; gx <= xhi / kGroupW; ++gx)
                atomicAdd(&lcnt[gy * G.ngx + gx], 1u);
    }
    __syncthreads();
    uint32_t* out = cntA + (size_t)chunk * G.ng;
    for (int t = threadIdx.x; t < G.ng; t += 256) out[t] = lcnt[t];
}

// grid (ceil(ng / 64), F), 1024 threads: lane = group within a block of 64,
// wave = one sixteenth of the frame's chunk rows.  Exclusive scan of every
// group's column over the chunks of its frame; totals per (frame, group).
__global__ void __launch_bounds__(1024) k_group_colscan(Params P, int QC, uint32_t* __restrict__ cntA,
                                                        uint32_t* __restrict__ lenA) {
    __shared__ uint32_t part[16][64];
    const Groups G = groups_of(P);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gi = blockIdx.x * 64 + lane;
    const int f = blockIdx.y;
    const int rows = (QC + 15) / 16;
    const int q0 = wave * rows, q1 = min(q0 + rows, QC);
    uint32_t* col = cntA + (size_t)f * QC * G.ng + gi;
    uint32_t s = 0;
    if (gi < G.ng)
        for (int q = q0; q < q1; ++q) s += col[(size_t)q * G.ng];
    part[wave][lane] = s;
    __syncthreads();
    uint32_t run = 0, total = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) run += part[w][lane];
        total += part[w][lane];
    }
    if (gi < G.ng) {
        for (int q = q0; q < q1; ++q) {
            const uint32_t v = col[(size_t)q * G.ng];
            col[(size_t)q * G.ng] = run;
            run += v;
        }
        if (wave == 0) lenA[(size_t)f * G.ng + gi] = total;
    }
}

// Single workgroup: group-list ranges (exclusive scan of the lengths) and the
// first level-B segment of every group.  The level-A lists are bounded by the
// pair capacity (every group entry yields at least one pair).
__global__ void __launch_bounds__(1024) k_group_scan(const uint32_t* __restrict__ lenA, int K, int S,
                                                     unsigned long long cap, uint2* __restrict__ granges,
                                                     uint32_t* __restrict__ seg_start) {
    __shared__ unsigned long long scratch[17];
    __shared__ uint32_t scratch32[17];
    unsigned long long carry = 0;
    uint32_t scarry = 0;
    for (int base = 0; base < K; base += 1024) {
        const int i = base + threadIdx.x;
        const unsigned long long v = i < K ? lenA[i] : 0ull;
        const uint32_t nsg = (uint32_t)((v + S - 1) / S);
        unsigned long long tot;
        uint32_t stot;
        const unsigned long long ex = block_exclusive_scan<unsigned long long, 1024>(v, scratch, &tot);
        const uint32_t sex = block_exclusive_scan<uint32_t, 1024>(nsg, scratch32, &stot);
        if (i < K) {
            const unsigned long long a = carry + ex, b = a + v;
            granges[i] = make_uint2((uint32_t)(a < cap ? a : cap), (uint32_t)(b < cap ? b : cap));
            seg_start[i] = scarry + sex;
        }
        carry += tot;
        scarry += stot;
    }
    if (threadIdx.x == 0) seg_start[K] = scarry;
}

// One wave per chunk: the chunk's items in depth order append themselves to
// the lists of the groups they touch.  The cursors live in LDS and advance by
// LDS atomics (in issue order within the wave, so depth order is kept); the
// group rectangles of 64 items are prepared in parallel before the ordered
// walk.
__global__ void __launch_bounds__(64) k_group_place(Params P, int C, int QC,
                                                    const uint32_t* __restrict__ dval,
                                                    const uint32_t* __restrict__ cnt,
                                                    const uint2* __restrict__ rect,
                                                    const uint32_t* __restrict__ cntA,
                                                    const uint2* __restrict__ granges,
                                                    uint32_t* __restrict__ gval) {
    __shared__ uint32_t cursor[kMaxGroupsPerFrame];
    __shared__ uint32_t sitem[64];
    __shared__ uint4 sgrp[64];   // first group, groups per row, area, 1 / row as float bits
    const Groups G = groups_of(P);
    const int chunk = blockIdx.x;
    const int f = chunk / QC, q = chunk - f * QC;
    const int lane = threadIdx.x;
    const uint32_t cap = (uint32_t)(P.cap < 0xffffffffull ? P.cap : 0xffffffffull);
    const uint32_t* pre = cntA + (size_t)chunk * G.ng;
    for (int t = lane; t < G.ng; t += 64) cursor[t] = granges[(size_t)f * G.ng + t].x + pre[t];
    const long long beg = (long long)f * P.n + (long long)q * C;
    const long long end = min(beg + C, (long long)(f + 1) * P.n);
    for (long long j0 = beg; j0 < end; j0 += 64) {
        __syncthreads();
        const int m = (int)min(64ll, end - j0);
        if (lane < m) {
            const uint32_t item = dval[j0 + lane];
            uint4 gr = make_uint4(0, 1, 0, 0);
            if (cnt[item] != 0) {
                uint32_t xlo, xhi, ylo, yhi;
                unpack_rect(rect[item], xlo, xhi, ylo, yhi);
                const uint32_t gx0 = xlo / kGroupW, gy0 = ylo / kGroupH;
                const uint32_t gw = xhi / kGroupW - gx0 + 1;
                gr = make_uint4(gy0 * (uint32_t)G.ngx + gx0, gw, gw * (yhi / kGroupH - gy0 + 1),
                                __float_as_uint(1.0f / (float)gw));
            }
            sitem[lane] = item;
            sgrp[lane] = gr;
        }
        __syncthreads();
        for (int i = 0; i < m; ++i) {
            const uint4 gr = sgrp[i];
            for (uint32_t k = lane; k < gr.z; k += 64) {
                // k -> (row, column) of the item's group rectangle; the quotient
                // of these small integers is exact with the float reciprocal
                const uint32_t r = (uint32_t)(((float)k + 0.5f) * __uint_as_float(gr.w));
                const uint32_t t = gr.x + r * (uint32_t)G.ngx + (k - r * gr.y);
                const uint32_t pos = atomicAdd(&cursor[t], 1u);
                if (pos < cap) gval[pos] = sitem[i];
            }
        }
    }
}

// ---- level B: group lists -> tile lists ----------------------------------------

struct Segment {
    int fg;             // frame * ng + group
    uint32_t beg, end;  // entries of the group list
};

// Segment b -> (frame, group) and its entries; fg < 0 if b is past the last.
__device__ __forceinline__ Segment find_segment(int b, const uint32_t* __restrict__ seg_start, int K,
                                                int S, const uint2* __restrict__ granges) {
    Segment s;
    s.fg = -1;
    if ((uint32_t)b >= seg_start[K]) return s;
    int lo = 0, hi = K;   // seg_start[lo] <= b < seg_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg_start[mid] <= (uint32_t)b) lo = mid; else hi = mid;
    }
    const uint2 r = granges[lo];
    s.fg = lo;
    s.beg = r.x + (uint32_t)(b - (int)seg_start[lo]) * (uint32_t)S;
    s.end = min(s.beg + (uint32_t)S, r.y);
    return s;
}

// Lane l of the wave owns tile (gx * 8 + l % 8, gy * 8 + l / 8) of the group.
struct LaneTile {
    int f;
    uint32_t tx, ty, tile;
    bool mine;
};

__device__ __forceinline__ LaneTile lane_tile(const Params& P, const Groups& G, int fg, int lane) {
    LaneTile t;
    t.f = fg / G.ng;
    const int gi = fg - t.f * G.ng;
    const uint32_t gy = gi / G.ngx, gx = gi - gy * G.ngx;
    t.tx = gx * kGroupW + lane % kGroupW;
    t.ty = gy * kGroupH + lane / kGroupW;
    t.mine = t.tx < (uint32_t)P.ntx && t.ty < (uint32_t)P.nty;
    t.tile = t.ty * (uint32_t)P.ntx + t.tx;
    return t;
}

// Counting pass: entries of the segment that cover each lane's tile.
__global__ void __launch_bounds__(64) k_tile_count(Params P, int S, const uint32_t* __restrict__ seg_start,
                                                   const uint2* __restrict__ granges,
                                                   const uint32_t* __restrict__ gval,
                                                   const uint2* __restrict__ rect,
                                                   uint32_t* __restrict__ cntB) {
    __shared__ uint2 srect[64];
    const Groups G = groups_of(P);
    const int K = P.F * G.ng;
    const uint32_t nseg = seg_start[K];
    const int lane = threadIdx.x;
    for (uint32_t b = blockIdx.x; b < nseg; b += gridDim.x) {
        const Segment sg = find_segment((int)b, seg_start, K, S, granges);
        const LaneTile lt = lane_tile(P, G, sg.fg, lane);
        uint32_t c = 0;
        for (uint32_t j0 = sg.beg; j0 < sg.end; j0 += 64) {
            const int m = (int)min(64u, sg.end - j0);
            __syncthreads();
            if (lane < m) srect[lane] = rect[gval[j0 + lane]];
            __syncthreads();
            for (int i = 0; i < m; ++i) {
                uint32_t xlo, xhi, ylo, yhi;
                unpack_rect(srect[i], xlo, xhi, ylo, yhi);
                c += (lt.mine && lt.tx >= xlo && lt.tx <= xhi && lt.ty >= ylo && lt.ty <= yhi) ? 1u : 0u;
            }
        }
        cntB[(size_t)b * 64 + lane] = c;
    }
}

// Placing pass.  Each lane appends the covering entries of its tile to a
// 32-entry LDS line buffer that mirrors the 128-byte line of the tile list
// it is filling; a full line is written by 32 lanes at once, so global
// stores are whole lines except at the ends of each lane's run.
__global__ void __launch_bounds__(64) k_tile_place(Params P, int S, const uint32_t* __restrict__ seg_start,
                                                   const uint2* __restrict__ granges,
                                                   const uint32_t* __restrict__ gval,
                                                   const uint2* __restrict__ rect,
                                                   const uint32_t* __restrict__ cntB,
                                                   const uint2* __restrict__ ranges,
                                                   uint32_t* __restrict__ tval) {
    __shared__ uint32_t sitem[64];
    __shared__ uint2 srect[64];
    __shared__ uint32_t lbuf_[64][kLine + 1];  // +1: lanes of one slot hit different banks
    // Lanes read lines other lanes wrote: LDS operations of one wave complete
    // in issue order, and volatile keeps the compiler from reordering them.
    volatile uint32_t(*lbuf)[kLine + 1] = lbuf_;
    const Groups G = groups_of(P);
    const int K = P.F * G.ng;
    const uint32_t nseg = seg_start[K];
    const int lane = threadIdx.x;
    const uint32_t cap = (uint32_t)(P.cap < 0xffffffffull ? P.cap : 0xffffffffull);

    // writes slots [lo, hi) of lane L's buffer to tval[base + slot]
    auto flush = [&](uint32_t base, uint32_t lo, uint32_t hi, int L) {
        const uint32_t k = (uint32_t)lane;
        if (k >= lo && k < hi && base + k < cap) tval[base + k] = lbuf[L][k];
    };

    for (uint32_t b = blockIdx.x; b < nseg; b += gridDim.x) {
        const Segment sg = find_segment((int)b, seg_start, K, S, granges);
        const LaneTile lt = lane_tile(P, G, sg.fg, lane);
        uint32_t c = 0;   // next list position of this lane's tile
        if (lt.mine) c = ranges[(size_t)lt.f * P.n_tiles + lt.tile].x + cntB[(size_t)b * 64 + lane];
        uint32_t base = c & ~(uint32_t)(kLine - 1);   // list position of buffer slot 0
        uint32_t lo = c - base;                       // first slot this lane owns
        for (uint32_t j0 = sg.beg; j0 < sg.end; j0 += 64) {
            const int m = (int)min(64u, sg.end - j0);
            __syncthreads();
            if (lane < m) {
                const uint32_t item = gval[j0 + lane];
                sitem[lane] = item;
                srect[lane] = rect[item];
            }
            __syncthreads();
            for (int i = 0; i < m; ++i) {
                uint32_t xlo, xhi, ylo, yhi;
                unpack_rect(srect[i], xlo, xhi, ylo, yhi);
                const bool cov = lt.mine && lt.tx >= xlo && lt.tx <= xhi && lt.ty >= ylo && lt.ty <= yhi;
                if (cov) {
                    lbuf[lane][c - base] = sitem[i];
                    ++c;
                }
                unsigned long long full = __ballot(c - base == (uint32_t)kLine);
                while (full) {
                    const int L = __builtin_ctzll(full);
                    full &= full - 1;
                    const uint32_t bL = __builtin_amdgcn_readlane(base, L);
                    const uint32_t lL = __builtin_amdgcn_readlane(lo, L);
                    flush(bL, lL, kLine, L);
                }
                if (c - base == (uint32_t)kLine) {
                    base += kLine;
                    lo = 0;
                }
            }
        }
        // partial last lines
        unsigned long long rest = __ballot(c - base > lo);
        while (rest) {
            const int L = __builtin_ctzll(rest);
            rest &= rest - 1;
            flush(__builtin_amdgcn_readlane(base, L), __builtin_amdgcn_readlane(lo, L),
                  __builtin_amdgcn_readlane(c - base, L), L);
        }
        __syncthreads();
    }
}

// One wave per (frame, group): exclusive scan of each lane's tile column over
// the group's segments; per-tile totals.
__global__ void __launch_bounds__(64) k_tile_colscan(Params P, const uint32_t* __restrict__ seg_start,
                                                     uint32_t* __restrict__ cntB,
                                                     uint32_t* __restrict__ tcount) {
    const Groups G = groups_of(P);
    const int fg = blockIdx.x;
    const int lane = threadIdx.x;
    const int f = fg / G.ng, gi = fg - f * G.ng;
    const uint32_t gy = gi / G.ngx, gx = gi - gy * G.ngx;
    const uint32_t tx = gx * kGroupW + lane % kGroupW, ty = gy * kGroupH + lane / kGroupW;
    uint32_t run = 0;
    for (uint32_t b = seg_start[fg]; b < seg_start[fg + 1]; ++b) {
        const uint32_t v = cntB[(size_t)b * 64 + lane];
        cntB[(size_t)b * 64 + lane] = run;
        run += v;
    }
    if (tx < (uint32_t)P.ntx && ty < (uint32_t)P.nty)
        tcount[(size_t)f * P.n_tiles + ty * P.ntx + tx] = run;
}

// Single workgroup: tile-list ranges = exclusive scan of the per-(frame, tile)
// totals; pair count, capacity and overflow into the status block.  Ranges
// are clamped to the capacity so that an overflowed forward stays in bounds.
__global__ void __launch_bounds__(1024) k_tile_keyscan(const uint32_t* __restrict__ tcount, long long K,
                                                       unsigned long long cap, uint2* __restrict__ ranges,
                                                       Status* status) {
    __shared__ unsigned long long scratch[17];
    unsigned long long carry = 0;
    for (long long base = 0; base < K; base += 1024) {
        const long long i = base + threadIdx.x;
        const unsigned long long v = i < K ? tcount[i] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_exclusive_scan<unsigned long long, 1024>(v, scratch, &tot);
        if (i < K) {
            const unsigned long long a = carry + ex, b = a + v;
            ranges[i] = make_uint2((uint32_t)(a < cap ? a : cap), (uint32_t)(b < cap ? b : cap));
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        status->n_pairs = carry;
        status->cap = cap;
        status->overflow = carry > cap ? 1u : 0u;
    }
}

// Introspection: expands the ranges into per-pair (frame, tile) keys.
__global__ void k_keys_from_ranges(const uint2* __restrict__ ranges, long long K,
                                   unsigned long long limit, uint32_t* __restrict__ keys) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K;
         i += (long long)gridDim.x * blockDim.x) {
        const uint2 r = ranges[i];
        for (uint32_t p = r.x; p < r.y && p < limit; ++p) keys[p] = (uint32_t)i;
    }
}

}  // namespace

BinGeom bin_geometry(int64_t n, int32_t n_frames, int ntx, int nty, uint64_t cap) {
    BinGeom g;
    // level-A chunks: enough waves to fill the chip, at least 128 items each
    const int64_t M = n * (int64_t)n_frames;
    int C = 128;
    while (C < 2048 && M / C > 4096) C *= 2;
    g.C = C;
    g.QC = n > 0 ? (int)((n + C - 1) / C) : 0;
    g.ng = ((ntx + kGroupW - 1) / kGroupW) * ((nty + kGroupH - 1) / kGroupH);
    // level-B segment: long runs per lane for large batches, more waves for small ones
    g.S = M >= (1 << 20) ? 512 : 128;
    // every segment but the last of each group list holds S entries, and the
    // group lists hold at most min(cap, M * groups) entries
    uint64_t entries = cap;
    if ((uint64_t)M * g.ng < entries) entries = (uint64_t)M * g.ng;
    g.max_segments = (int64_t)((entries + g.S - 1) / g.S) + (int64_t)n_frames * g.ng;
    return g;
}

hipError_t launch_binning(const Params& P, const Workspace& w, int dbuf, hipStream_t s) {
    const BinGeom g = bin_geometry(P.n, P.F, P.ntx, P.nty, P.cap);
    const int K = P.F * g.ng;
    const unsigned chunks = (unsigned)(P.F * g.QC);
    if (chunks) {
        ProfScope _p("k_group_count", s);
        hipLaunchKernelGGL(k_group_count, dim3(chunks), dim3(256), 0, s, P, g.C, g.QC, w.dval[dbuf],
                           w.cnt, w.rect, w.cntA);
    }
    if (chunks) {
        ProfScope _p("k_group_colscan", s);
        hipLaunchKernelGGL(k_group_colscan, dim3((g.ng + 63) / 64, P.F), dim3(1024), 0, s, P, g.QC,
                           w.cntA, w.lenA);
    } else {
        launch_fill_u32(w.lenA, 0u, K, s);
    }
    {
        ProfScope _p("k_group_scan", s);
        hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(1024), 0, s, w.lenA, K, g.S,
                           (unsigned long long)P.cap, w.granges, w.seg_start);
    }
    if (chunks) {
        ProfScope _p("k_group_place", s);
        hipLaunchKernelGGL(k_group_place, dim3(chunks), dim3(64), 0, s, P, g.C, g.QC, w.dval[dbuf],
                           w.cnt, w.rect, w.cntA, w.granges, w.gval);
    }
    // persistent level-B grid: every wave loops over segments
    const unsigned segs = (unsigned)(g.max_segments < 16384 ? g.max_segments : 16384);
    {
        ProfScope _p("k_tile_count", s);
        hipLaunchKernelGGL(k_tile_count, dim3(segs), dim3(64), 0, s, P, g.S, w.seg_start, w.granges,
                           w.gval, w.rect, w.cntB);
    }
    {
        ProfScope _p("k_tile_colscan", s);
        hipLaunchKernelGGL(k_tile_colscan, dim3(K), dim3(64), 0, s, P, w.seg_start, w.cntB, w.tcount);
    }
    {
        ProfScope _p("k_tile_keyscan", s);
        hipLaunchKernelGGL(k_tile_keyscan, dim3(1), dim3(1024), 0, s, w.tcount,
                           (long long)P.F * P.n_tiles, (unsigned long long)P.cap, w.ranges, w.status);
    }
    {
        ProfScope _p("k_tile_place", s);
        hipLaunchKernelGGL(k_tile_place, dim3(segs), dim3(64), 0, s, P, g.S, w.seg_start, w.granges,
                           w.gval, w.rect, w.cntB, w.ranges, w.tval);
    }
    return hipGetLastError();
}

void launch_keys_from_ranges(const Params& P, const Workspace& w, uint32_t* keys,
                             unsigned long long limit, hipStream_t s) {
    const long long K = (long long)P.F * P.n_tiles;
    hipLaunchKernelGGL(k_keys_from_ranges, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s,
                       w.ranges, K, limit, keys);
}

}  // namespace gft
