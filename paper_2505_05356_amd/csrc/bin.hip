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
constexpr int kSegment = 512;             // group-list entries per level-B wave

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

// One thread per (frame, group): exclusive scan of the group's column over
// the chunks of its frame; totals per (frame, group).
__global__ void k_group_colscan(Params P, int QC, uint32_t* __restrict__ cntA,
                                uint32_t* __restrict__ lenA) {
    const Groups G = groups_of(P);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.F * G.ng) return;
    const int f = i / G.ng, gi = i - f * G.ng;
    uint32_t* col = cntA + (size_t)f * QC * G.ng + gi;
    uint32_t run = 0;
    for (int q = 0; q < QC; ++q) {
        const uint32_t v = col[(size_t)q * G.ng];
        col[(size_t)q * G.ng] = run;
        run += v;
    }
    lenA[i] = run;
}

// Single workgroup: group-list ranges (exclusive scan of the lengths) and the
// first level-B segment of every group.  The level-A lists are bounded by the
// pair capacity (every group entry yields at least one pair).
__global__ void __launch_bounds__(1024) k_group_scan(const uint32_t* __restrict__ lenA, int K,
                                                     unsigned long long cap, uint2* __restrict__ granges,
                                                     uint32_t* __restrict__ seg_start) {
    __shared__ unsigned long long scratch[17];
    __shared__ uint32_t scratch32[17];
    unsigned long long carry = 0;
    uint32_t scarry = 0;
    for (int base = 0; base < K; base += 1024) {
        const int i = base + threadIdx.x;
        const unsigned long long v = i < K ? lenA[i] : 0ull;
        const uint32_t nsg = (uint32_t)((v + kSegment - 1) / kSegment);
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
// the lists of the groups they touch (LDS cursors, lanes over the groups).
__global__ void __launch_bounds__(64) k_group_place(Params P, int C, int QC,
                                                    const uint32_t* __restrict__ dval,
                                                    const uint32_t* __restrict__ cnt,
                                                    const uint2* __restrict__ rect,
                                                    const uint32_t* __restrict__ cntA,
                                                    const uint2* __restrict__ granges,
                                                    uint32_t* __restrict__ gval) {
    __shared__ uint32_t cursor[kMaxGroupsPerFrame];
    __shared__ uint32_t sitem[64];
    __shared__ uint2 srect[64];
    const Groups G = groups_of(P);
    const int chunk = blockIdx.x;
    const int f = chunk / QC, q = chunk - f * QC;
    const int lane = threadIdx.x;
    const uint32_t cap = (uint32_t)(P.cap < 0xffffffffull ? P.cap : 0xffffffffull);
    const uint32_t* pre = cntA + (size_t)chunk * G.ng;
    for (int t = lane; t < G.ng; t += 64) cursor[t] = granges[(size_t)f * G.ng + t].x + pre[t];
    const long long beg = (long long)f * P.n + (long long)q * C;
    const long long end = min(beg + C, (long long)(f + 1) * P.n);
    volatile uint32_t* cur = cursor;
    for (long long j0 = beg; j0 < end; j0 += 64) {
        __syncthreads();
        const int m = (int)min(64ll, end - j0);
        if (lane < m) {
            const uint32_t item = dval[j0 + lane];
            const bool ok = cnt[item] != 0;
            sitem[lane] = ok ? item : 0xffffffffu;
            srect[lane] = ok ? rect[item] : make_uint2(0, 0);
        }
        __syncthreads();
        for (int i = 0; i < m; ++i) {
            const uint32_t item = sitem[i];
            if (item == 0xffffffffu) continue;
            uint32_t xlo, xhi, ylo, yhi;
            unpack_rect(srect[i], xlo, xhi, ylo, yhi);
            const uint32_t gx0 = xlo / kGroupW, gy0 = ylo / kGroupH;
            const uint32_t gw = xhi / kGroupW - gx0 + 1;
            const uint32_t area = gw * (yhi / kGroupH - gy0 + 1);
            for (uint32_t k = lane; k < area; k += 64) {
                const uint32_t gy = gy0 + k / gw, gx = gx0 + k % gw;
                const uint32_t t = gy * (uint32_t)G.ngx + gx;
                const uint32_t pos = cur[t];
                cur[t] = pos + 1;
                if (pos < cap) gval[pos] = item;
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
                                                const uint2* __restrict__ granges) {
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
    s.beg = r.x + (uint32_t)(b - (int)seg_start[lo]) * kSegment;
    s.end = min(s.beg + (uint32_t)kSegment, r.y);
    return s;
}

// Lane l of the wave owns tile (gx * 8 + l % 8, gy * 8 + l / 8) of the group.
template <bool PLACE>
__global__ void __launch_bounds__(64) k_tile_pass(Params P, const uint32_t* __restrict__ seg_start,
                                                  const uint2* __restrict__ granges,
                                                  const uint32_t* __restrict__ gval,
                                                  const uint2* __restrict__ rect,
                                                  uint32_t* __restrict__ cntB,
                                                  const uint2* __restrict__ ranges,
                                                  uint32_t* __restrict__ tval) {
    __shared__ uint32_t sitem[64];
    __shared__ uint2 srect[64];
    const Groups G = groups_of(P);
    const int K = P.F * G.ng;
    const uint32_t nseg = seg_start[K];
    for (uint32_t b = blockIdx.x; b < nseg; b += gridDim.x) {
    const Segment sg = find_segment((int)b, seg_start, K, granges);
    const int lane = threadIdx.x;
    const int f = sg.fg / G.ng, gi = sg.fg - f * G.ng;
    const uint32_t gy = gi / G.ngx, gx = gi - gy * G.ngx;
    const uint32_t tx = gx * kGroupW + lane % kGroupW, ty = gy * kGroupH + lane / kGroupW;
    const bool mine = tx < (uint32_t)P.ntx && ty < (uint32_t)P.nty;
    const uint32_t tile = ty * (uint32_t)P.ntx + tx;
    const uint32_t cap = (uint32_t)(P.cap < 0xffffffffull ? P.cap : 0xffffffffull);
    uint32_t c = 0;
    if (PLACE && mine) c = ranges[(size_t)f * P.n_tiles + tile].x + cntB[(size_t)b * 64 + lane];
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
            const bool cov = mine && tx >= xlo && tx <= xhi && ty >= ylo && ty <= yhi;
            if (PLACE) {
                if (cov) {
                    if (c < cap) tval[c] = sitem[i];
                    ++c;
                }
            } else {
                c += cov ? 1u : 0u;
            }
        }
    }
    if (!PLACE) cntB[(size_t)b * 64 + lane] = c;
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
    // every segment but the last of each group list holds kSegment entries,
    // and the group lists hold at most min(cap, M * groups) entries
    uint64_t entries = cap;
    if ((uint64_t)M * g.ng < entries) entries = (uint64_t)M * g.ng;
    g.max_segments = (int64_t)((entries + kSegment - 1) / kSegment) + (int64_t)n_frames * g.ng;
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
        hipLaunchKernelGGL(k_group_colscan, dim3((K + 255) / 256), dim3(256), 0, s, P, g.QC, w.cntA,
                           w.lenA);
    } else {
        launch_fill_u32(w.lenA, 0u, K, s);
    }
    {
        ProfScope _p("k_group_scan", s);
        hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(1024), 0, s, w.lenA, K, (unsigned long long)P.cap,
                           w.granges, w.seg_start);
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
        hipLaunchKernelGGL(k_tile_pass<false>, dim3(segs), dim3(64), 0, s, P, w.seg_start, w.granges,
                           w.gval, w.rect, w.cntB, w.ranges, w.tval);
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
        hipLaunchKernelGGL(k_tile_pass<true>, dim3(segs), dim3(64), 0, s, P, w.seg_start, w.granges,
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
