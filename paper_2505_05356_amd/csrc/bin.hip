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
//   chunk places 64 items at a time, every lane at once: the lanes that share
//   a group come from four ballot masks (by group column and row), and a
//   lane's rank among them is its offset in that group's list.
// Level B -- group lists into tile lists.  Each group list is cut into
//   segments; one wave per segment.  A counting pass (an 8x8 difference array
//   per segment), a column scan over each group's segments and an exclusive
//   scan over (frame, tile) give every tile a cursor; the placing pass takes
//   64 entries at a time and, tile by tile, ballots the covering lanes, which
//   write one contiguous run of the tile's list in depth order.
#include "block_scan.h"
#include "common.h"

namespace gft {

namespace {

constexpr int kGroupW = 8, kGroupH = 8;   // tiles per group (one per lane)

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

// Group counts of each chunk of C items: one workgroup of 256 threads per CPW
// chunks (CPW = 512 / C, between 1 and 4, so that every thread counts two or
// more items and short chunks do not each pay a workgroup launch).
constexpr int kMaxChunksPerBlock = 4;

__global__ void __launch_bounds__(256) k_group_count(Params P, int C, int QC, int CPW,
                                                     const uint32_t* __restrict__ dkey,
                                                     const uint2* __restrict__ drect,
                                                     uint32_t* __restrict__ cntA) {
    __shared__ uint32_t lcnt[kMaxChunksPerBlock][kMaxGroupsPerFrame];
    const Groups G = groups_of(P);
    const int TPC = 256 / CPW;   // threads per chunk
    const int sub = (int)threadIdx.x / TPC, lt = (int)threadIdx.x - sub * TPC;
    const int chunk = blockIdx.x * CPW + sub;
    const bool have = chunk < P.F * QC;
    uint32_t* cnt = lcnt[sub];
    for (int t = lt; t < G.ng; t += TPC) cnt[t] = 0;
    __syncthreads();
    if (have) {
        const int f = chunk / QC, q = chunk - f * QC;
        const long long beg = (long long)f * P.n + (long long)q * C;
        const long long end = min(beg + C, (long long)(f + 1) * P.n);
        for (long long j = beg + lt; j < end; j += TPC) {
            if (dkey[j] == kCulledKey) continue;
            uint32_t xlo, xhi, ylo, yhi;
            unpack_rect(drect[j], xlo, xhi, ylo, yhi);
            for (uint32_t gy = ylo / kGroupH; gy <= yhi / kGroupH; ++gy)
                for (uint32_t gx = xlo / kGroupW; gx <= xhi / kGroupW; ++gx)
                    atomicAdd(&cnt[gy * G.ngx + gx], 1u);
        }
    }
    __syncthreads();
    if (have) {
        uint32_t* out = cntA + (size_t)chunk * G.ng;
        for (int t = lt; t < G.ng; t += TPC) out[t] = cnt[t];
    }
}

// grid (ng, F), 256 threads: one workgroup per (frame, group) column.
// Exclusive scan of the column over the chunks of its frame (each thread a
// run of consecutive chunks), and the column total.
__global__ void __launch_bounds__(256) k_group_colscan(Params P, int QC, uint32_t* __restrict__ cntA,
                                                       uint32_t* __restrict__ lenA) {
    __shared__ uint32_t scratch[8];
    const Groups G = groups_of(P);
    const int gi = blockIdx.x, f = blockIdx.y;
    const int per = (QC + 255) / 256;
    const int q0 = min((int)threadIdx.x * per, QC), q1 = min(q0 + per, QC);
    uint32_t* col = cntA + (size_t)f * QC * G.ng + gi;
    // 8 loads in flight per round (a thread's run is 4-8 chunks at 1.6M-16M
    // items)
    uint32_t s = 0;
    for (int q = q0; q < q1; q += 8) {
        uint32_t v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = q + i < q1 ? col[(size_t)(q + i) * G.ng] : 0u;
#pragma unroll
        for (int i = 0; i < 8; ++i) s += v[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan<uint32_t, 256>(s, scratch, &total);
    for (int q = q0; q < q1; q += 8) {
        uint32_t v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = q + i < q1 ? col[(size_t)(q + i) * G.ng] : 0u;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (q + i < q1) col[(size_t)(q + i) * G.ng] = run;
            run += v[i];
        }
    }
    if (threadIdx.x == 0) lenA[(size_t)f * G.ng + gi] = total;
}

// Single workgroup: group-list ranges (exclusive scan of the lengths) and the
// first level-B segment of every group.  The level-A lists are bounded by the
// pair capacity (every group entry yields at least one pair).
__global__ void __launch_bounds__(1024) k_group_scan(const uint32_t* __restrict__ lenA, int K, int S, int R,
                                                     unsigned long long cap, uint2* __restrict__ granges,
                                                     uint32_t* __restrict__ seg_start,
                                                     uint32_t* __restrict__ chunk_start) {
    __shared__ unsigned long long scratch[17];
    __shared__ uint32_t scratch32[17];
    unsigned long long carry = 0;
    uint32_t scarry = 0, ccarry = 0;
    for (int base = 0; base < K; base += 1024) {
        const int i = base + threadIdx.x;
        const unsigned long long v = i < K ? lenA[i] : 0ull;
        unsigned long long tot;
        uint32_t stot, ctot;
        const unsigned long long ex = block_exclusive_scan<unsigned long long, 1024>(v, scratch, &tot);
        const unsigned long long a = carry + ex, b = a + v;
        const unsigned long long ac = a < cap ? a : cap, bc = b < cap ? b : cap;
        // segments and chunks of the stored part of the list only (the lists
        // are cut at the capacity), so their counts stay within the
        // workspace's bound even when an overflowed batch has more entries
        const uint32_t nsg = (uint32_t)((bc - ac + S - 1) / S);
        const uint32_t nch = (nsg + R - 1) / R;
        const uint32_t sex = block_exclusive_scan<uint32_t, 1024>(nsg, scratch32, &stot);
        const uint32_t cex = block_exclusive_scan<uint32_t, 1024>(nch, scratch32, &ctot);
        if (i < K) {
            granges[i] = make_uint2((uint32_t)ac, (uint32_t)bc);
            seg_start[i] = scarry + sex;
            chunk_start[i] = ccarry + cex;
        }
        carry += tot;
        scarry += stot;
        ccarry += ctot;
    }
    if (threadIdx.x == 0) {
        seg_start[K] = scarry;
        chunk_start[K] = ccarry;
    }
}

// Rank of this lane among the lanes of `peers` below it.
__device__ __forceinline__ uint32_t rank_below(uint64_t peers) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
}

// Placing pass of level A.  Work item = (run of RA consecutive chunks of one
// frame, group row gy); one wave walks the run's depth-ordered items 64 at a
// time (lane = item) and, for each group column, ballots the lanes whose
// rectangle covers that group: each writes at the group's cursor plus its
// rank among them, so one store appends a contiguous run to the group list
// and depth order holds inside every list.  A wave appends each group's run
// over the whole run of chunks, so its stores fill whole cache lines instead
// of scattering a few entries per group and batch.
// FAST: the row's group lists all end strictly below the capacity (their
// ranges are clamped to it), so the stores need no check.  REG: the row has
// at most kGroupW groups, whose cursors stay in scalar registers under an
// unrolled, branch-free column loop (an empty ballot stores nothing);
// otherwise they live in LDS.  NB: runs of at least 16 batches load 8
// batches at a time (fewer waits per run); shorter runs load each batch
// while the previous one is placed (measured faster there).
template <bool FAST, bool REG, int NB>
__device__ __forceinline__ void place_group_row(const Groups& G, long long beg, long long end, uint32_t gy, int lane,
                                                uint32_t* cursor, uint32_t (&cur)[kGroupW], uint32_t cap,
                                                const uint32_t* __restrict__ dval,
                                                const uint32_t* __restrict__ dkey,
                                                const uint2* __restrict__ drect,
                                                uint32_t* __restrict__ gval, uint16_t* __restrict__ gloc) {
    const uint32_t oy = gy * kGroupH;
    // one batch: lane = item, covering the groups gx0 .. gx1 of the row
    auto place_batch_a = [&](uint32_t key, uint32_t item, uint2 rect) {
        int gx0 = 1, gx1 = 0;   // empty: never in a ballot
        uint32_t xlo = 0, xhi = 0, ylo = 0, yhi = 0;
        if (key != kCulledKey) {
            unpack_rect(rect, xlo, xhi, ylo, yhi);
            if (ylo / kGroupH <= gy && gy <= yhi / kGroupH) {
                gx0 = (int)(xlo / kGroupW);
                gx1 = (int)(xhi / kGroupW);
            }
        }
        // the rows of the rectangle clipped to this group row
        const uint32_t y0 = max(ylo, oy) - oy, y1 = min(yhi, oy + kGroupH - 1) - oy;
        const uint32_t ybits = (y0 << 6) | (y1 << 9);
        auto place = [&](int c, uint32_t at, uint64_t peers, bool mine) {
            if (mine) {
                const uint32_t pos = at + rank_below(peers);
                const uint32_t ox = (uint32_t)c * kGroupW;
                const uint32_t x0 = max(xlo, ox) - ox, x1 = min(xhi, ox + kGroupW - 1) - ox;
                if (FAST || pos < cap) {
                    gval[pos] = item;
                    gloc[pos] = (uint16_t)(x0 | (x1 << 3) | ybits);
                }
            }
        };
        if constexpr (REG) {
#pragma unroll
            for (int c = 0; c < kGroupW; ++c) {   // columns past the frame never match
                const bool mine = gx0 <= c && c <= gx1;
                const uint64_t peers = __ballot(mine);
                place(c, cur[c], peers, mine);
                cur[c] = (uint32_t)__builtin_amdgcn_readfirstlane((int)(cur[c] + (uint32_t)__popcll(peers)));
            }
        } else {
            for (int c = 0; c < G.ngx; ++c) {
                const bool mine = gx0 <= c && c <= gx1;
                const uint64_t peers = __ballot(mine);
                if (peers == 0ull) continue;
                const uint32_t at = cursor[c];
                place(c, at, peers, mine);
                if (lane == 0) cursor[c] = at + (uint32_t)__popcll(peers);
            }
            // lane 0's cursor writes precede the next batch's reads by every lane
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    };
    if constexpr (NB == 1) {
        // the next batch's key, item and rectangle are loaded while this
        // batch is placed
        uint32_t nkey = kCulledKey, nitem = 0;
        uint2 nrect = make_uint2(0u, 0u);
        if (beg + lane < end) {
            nkey = dkey[beg + lane];
            nitem = dval[beg + lane];
            nrect = drect[beg + lane];
        }
        for (long long j0 = beg; j0 < end; j0 += 64) {
            const uint32_t key = nkey, item = nitem;
            const uint2 rect = nrect;
            const long long jn = j0 + 64 + lane;
            nkey = kCulledKey;
            if (jn < end) {
                nkey = dkey[jn];
                nitem = dval[jn];
                nrect = drect[jn];
            }
            place_batch_a(key, item, rect);
        }
    } else {
        // NB batches at a time, all their loads in flight before the first
        // of them is placed
        for (long long r0 = beg; r0 < end; r0 += 64 * NB) {
            uint32_t bkey[NB], bitem[NB];
            uint2 brect[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const long long j = r0 + 64 * b + lane;
                bkey[b] = kCulledKey;
                bitem[b] = 0;
                brect[b] = make_uint2(0u, 0u);
                if (j < end) {
                    bkey[b] = dkey[j];
                    bitem[b] = dval[j];
                    brect[b] = drect[j];
                }
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (r0 + 64 * b >= end) break;   // wave-uniform
                place_batch_a(bkey[b], bitem[b], brect[b]);
            }
        }
    }
}

template <int NB>
__global__ void __launch_bounds__(64) k_group_place(Params P, int C, int QC, int RA,
                                                         const uint32_t* __restrict__ dval,
                                                         const uint32_t* __restrict__ dkey,
                                                         const uint2* __restrict__ drect,
                                                         const uint32_t* __restrict__ cntA,
                                                         const uint2* __restrict__ granges,
                                                         uint32_t* __restrict__ gval,
                                                         uint16_t* __restrict__ gloc) {
    extern __shared__ uint32_t cursor[];   // [ngx] list cursors of the work item's group row
    const Groups G = groups_of(P);
    const int lane = threadIdx.x;
    const uint32_t cap = (uint32_t)(P.cap < 0xffffffffull ? P.cap : 0xffffffffull);
    const uint32_t nrun = ((uint32_t)QC + (uint32_t)RA - 1) / (uint32_t)RA;   // runs of RA chunks per frame
    const uint32_t nitems = (uint32_t)P.F * nrun * (uint32_t)G.ngy;
    // the rows of one run are consecutive work items, so they read the run's
    // items through one L2; each XCD takes one contiguous eighth of the work
    // items
    const uint32_t per_xcd = gridDim.x / kXcds, xcd = blockIdx.x % kXcds;
    const uint32_t hi = (uint32_t)((uint64_t)nitems * (xcd + 1) / kXcds);
    for (uint32_t wi = (uint32_t)((uint64_t)nitems * xcd / kXcds) + blockIdx.x / kXcds; wi < hi; wi += per_xcd) {
        const uint32_t fr = wi / (uint32_t)G.ngy;
        const uint32_t gy = wi - fr * (uint32_t)G.ngy;
        const uint32_t f = fr / nrun, q = (fr - f * nrun) * (uint32_t)RA;   // the run's first chunk
        const uint32_t chunk = f * (uint32_t)QC + q;
        const long long beg = (long long)f * P.n + (long long)q * C;
        const long long end = min(beg + (long long)RA * C, (long long)(f + 1) * P.n);
        // cursors: the group list start plus the items of earlier chunks
        const size_t g0 = (size_t)f * G.ng + (size_t)gy * G.ngx;
        const uint32_t* pre = cntA + (size_t)chunk * G.ng + (size_t)gy * G.ngx;
        uint32_t el = 0;
        uint32_t cur[kGroupW];
        // the ranges are clamped to the capacity, so only an end strictly
        // below it proves that the whole list fits
        if (G.ngx <= kGroupW) {   // cursors of lanes 0 .. ngx-1, then wave-uniform
            uint32_t cl = 0;
            if (lane < G.ngx) {
                const uint2 gr = granges[g0 + lane];
                cl = gr.x + pre[lane];
                el = gr.y;
            }
#pragma unroll
            for (int c = 0; c < kGroupW; ++c) cur[c] = (uint32_t)__builtin_amdgcn_readlane((int)cl, c);
            if (__ballot(el >= cap) == 0ull)
                place_group_row<true, true, NB>(G, beg, end, gy, lane, cursor, cur, cap, dval, dkey, drect, gval, gloc);
            else
                place_group_row<false, true, NB>(G, beg, end, gy, lane, cursor, cur, cap, dval, dkey, drect, gval, gloc);
            continue;
        }
        __syncthreads();   // the previous work item's cursor reads are done
        for (int c = lane; c < G.ngx; c += 64) {
            const uint2 gr = granges[g0 + c];
            cursor[c] = gr.x + pre[c];
            el = max(el, gr.y);
        }
        __syncthreads();
        if (__ballot(el >= cap) == 0ull)
            place_group_row<true, false, NB>(G, beg, end, gy, lane, cursor, cur, cap, dval, dkey, drect, gval, gloc);
        else
            place_group_row<false, false, NB>(G, beg, end, gy, lane, cursor, cur, cap, dval, dkey, drect, gval, gloc);
    }
}

// ---- level B: group lists -> tile lists ----------------------------------------

// Largest i in [0, K) with a[i] <= v, for a nondecreasing a with a[0] <= v.
__device__ __forceinline__ int last_le(const uint32_t* __restrict__ a, int K, uint32_t v) {
    int lo = 0, hi = K;   // a[lo] <= v < a[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
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

// An entry's tile rectangle clipped to the 8x8 tiles of its group, in group
// coordinates, as stored by the level-A placement (3 bits per bound).
struct LocalRect {
    uint32_t x0, x1, y0, y1;
};

__device__ __forceinline__ LocalRect local_rect(uint32_t packed) {
    LocalRect r;
    r.x0 = packed & 7u;
    r.x1 = (packed >> 3) & 7u;
    r.y0 = (packed >> 6) & 7u;
    r.y1 = (packed >> 9) & 7u;
    return r;
}

// Bit y * 8 + x set for every tile (x, y) of the rectangle.
__device__ __forceinline__ uint64_t cover_mask(const LocalRect& r) {
    const uint64_t row = (uint64_t)(((2u << r.x1) - (1u << r.x0)) & 0xffu) * 0x0101010101010101ull;
    const uint64_t upto = r.y1 >= 7 ? ~0ull : ((1ull << (8 * (r.y1 + 1))) - 1);
    const uint64_t below = (1ull << (8 * r.y0)) - 1;
    return row & upto & ~below;
}

// Counting pass: entries of the segment that cover each lane's tile.  Every
// entry adds the four corners of its rectangle to an 8x8 difference array
// in LDS; a 2-D prefix sum across the lanes turns it into per-tile counts.
__global__ void __launch_bounds__(64) k_tile_count(Params P, int S, const uint32_t* __restrict__ seg_start,
                                                   const uint2* __restrict__ granges,
                                                   const uint16_t* __restrict__ gloc,
                                                   uint32_t* __restrict__ cntB) {
    __shared__ int diff[64];
    const Groups G = groups_of(P);
    const int K = P.F * G.ng;
    const uint32_t nseg = seg_start[K];
    const int lane = threadIdx.x;
    // each wave counts a run of consecutive segments: one search for the
    // group of the first, then the group advances with the segments (groups
    // with empty lists have no segments and are stepped over)
    const uint32_t per = (nseg + gridDim.x - 1) / gridDim.x;
    const uint32_t b0 = blockIdx.x * per, b1 = min(b0 + per, nseg);
    int fg = b0 < b1 ? last_le(seg_start, K, b0) : 0;
    for (uint32_t b = b0; b < b1; ++b) {
        while (seg_start[fg + 1] <= b) ++fg;
        const uint2 gr = granges[fg];
        const uint32_t sbeg = gr.x + (b - seg_start[fg]) * (uint32_t)S;
        const uint32_t send = min(sbeg + (uint32_t)S, gr.y);
        diff[lane] = 0;
        __syncthreads();
        for (uint32_t j = sbeg + lane; j < send; j += 64) {
            const LocalRect r = local_rect(gloc[j]);
            const bool xin = r.x1 + 1 < (uint32_t)kGroupW, yin = r.y1 + 1 < (uint32_t)kGroupH;
            atomicAdd(&diff[r.y0 * kGroupW + r.x0], 1);
            if (xin) atomicAdd(&diff[r.y0 * kGroupW + r.x1 + 1], -1);
            if (yin) atomicAdd(&diff[(r.y1 + 1) * kGroupW + r.x0], -1);
            if (xin && yin) atomicAdd(&diff[(r.y1 + 1) * kGroupW + r.x1 + 1], 1);
        }
        __syncthreads();
        int v = diff[lane];
        for (int d = 1; d < kGroupW; d <<= 1) {
            const int u = __shfl_up(v, d, 64);
            if (lane % kGroupW >= d) v += u;
        }
        for (int d = kGroupW; d < 64; d <<= 1) {
            const int u = __shfl_up(v, d, 64);
            if (lane >= d) v += u;
        }
        cntB[(size_t)b * 64 + lane] = (uint32_t)v;
        __syncthreads();   // diff is cleared for the next segment
    }
}

// Appends one batch of 64 entries (lane = entry) to the 8 tile lists of a
// group row: per tile a ballot of the covering lanes, each writing at the
// tile's cursor plus its rank among them.  FAST: every position of the row's
// lists is known to lie below both the capacity and 2^30 (the tile ranges'
// ends, which are clamped to the capacity, lie strictly below both), so the
// stores need no capacity check and address tval with a 32-bit byte offset
// from its base.
template <bool FAST>
__device__ __forceinline__ void place_batch(uint32_t row, uint32_t item, uint32_t (&cur)[kGroupW], uint32_t ncol,
                                            uint32_t cap, uint32_t* __restrict__ tval) {
    // no branch per tile: an empty ballot stores nothing and leaves the
    // cursor, and the row bits of tiles beyond the frame's edge are cleared
    row &= (1u << ncol) - 1u;
#pragma unroll
    for (int c = 0; c < kGroupW; ++c) {
        const bool mine = (row >> c) & 1u;
        const uint64_t peers = __ballot(mine);
        const uint32_t cnt = (uint32_t)__popcll(peers);
        if (mine) {
            const uint32_t pos = cur[c] + rank_below(peers);
            if constexpr (FAST) {
                *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(tval) + (pos << 2)) = item;
            } else {
                if (cur[c] + cnt <= cap || pos < cap) tval[pos] = item;
            }
        }
        cur[c] = (uint32_t)__builtin_amdgcn_readfirstlane((int)(cur[c] + cnt));
    }
}

// The entries [beg, end) of a group list, 64 at a time, appended to the
// lists of the group's tile row r.  The entries are loaded kRowBatches
// batches at a time, all loads in flight before the first batch is placed
// (a work item is at most R * S = kRowBatches * 64 entries), so a wave waits
// for its loads once per work item rather than once per batch.
constexpr int kRowBatches = 16;

template <bool FAST>
__device__ __forceinline__ void place_row(uint32_t beg, uint32_t end, uint32_t r, int lane, uint32_t (&cur)[kGroupW],
                                          uint32_t ncol, uint32_t cap, const uint32_t* __restrict__ gval,
                                          const uint16_t* __restrict__ gloc, uint32_t* __restrict__ tval) {
    for (uint32_t j0 = beg; j0 < end; j0 += 64 * kRowBatches) {
        uint32_t item[kRowBatches], loc[kRowBatches];
#pragma unroll
        for (int b = 0; b < kRowBatches; ++b) {
            const uint32_t j = j0 + 64 * b + lane;
            item[b] = 0;
            loc[b] = 0;
            if (j < end) {
                item[b] = gval[j];
                loc[b] = gloc[j];
            }
        }
#pragma unroll
        for (int b = 0; b < kRowBatches; ++b) {
            if (j0 + 64 * b >= end) break;   // wave-uniform
            uint32_t row = 0;   // bit c: the entry covers tile (c, r) of the group
            if (j0 + 64 * b + lane < end) {
                const LocalRect lr = local_rect(loc[b]);
                if (lr.y0 <= r && r <= lr.y1) row = ((2u << lr.x1) - (1u << lr.x0)) & 0xffu;
            }
            place_batch<FAST>(row, item[b], cur, ncol, cap, tval);
        }
    }
}

// Placing pass.  Work item = (chunk of R segments of one group list, tile row
// r of the group); one wave walks the chunk's entries 64 at a time (lane =
// entry) and places the entries covering each of the row's 8 tiles: a ballot
// gives the covering lanes, and each writes at the tile's cursor plus its
// rank among them, so one store instruction appends a contiguous run to that
// tile's list.  The 8 cursors are wave-uniform (scalar registers, the tile
// loop unrolled), and one wave appends each tile's run over R * S entries, so
// the runs span whole cache lines except at their two ends.
__global__ void __launch_bounds__(64) k_tile_place(Params P,
                                                   const uint32_t* __restrict__ chunk_start,
                                                   const uint4* __restrict__ chunk_info,
                                                   const uint32_t* __restrict__ gval,
                                                   const uint16_t* __restrict__ gloc,
                                                   const uint32_t* __restrict__ cntB,
                                                   const uint2* __restrict__ ranges,
                                                   uint32_t* __restrict__ tval) {
    const Groups G = groups_of(P);
    const int K = P.F * G.ng;
    const uint32_t nitems = chunk_start[K] * (uint32_t)kGroupH;
    const int lane = threadIdx.x;
    const uint32_t cap = (uint32_t)(P.cap < 0xffffffffull ? P.cap : 0xffffffffull);
    const uint32_t fast_end = min(cap, 1u << 30);   // lists ending below this take the fast stores
    // consecutive chunks of a group end and start runs in the same cache
    // lines: each XCD takes one contiguous eighth of the work items, so those
    // partial lines meet in one L2 (the grid is a multiple of 8 workgroups).
    // Inside it the work items are dealt round robin: the 8 rows of a chunk
    // go to neighbouring waves at about the same time, which read the chunk's
    // entries through L2 once (runs of consecutive items per wave measured
    // slower at 1M x 16 frames)
    const uint32_t per_xcd = gridDim.x / kXcds, xcd = blockIdx.x % kXcds;
    const uint32_t hi = (uint32_t)((uint64_t)nitems * (xcd + 1) / kXcds);
    for (uint32_t wi = (uint32_t)((uint64_t)nitems * xcd / kXcds) + blockIdx.x / kXcds; wi < hi; wi += per_xcd) {
        const uint32_t ch = wi / kGroupH;
        const uint32_t r = wi - ch * kGroupH;   // tile row of the group
        const uint4 ci = chunk_info[ch];   // group, first and end entry, first segment
        const int fg = (int)ci.x;
        const int f = fg / G.ng, gi = fg - f * G.ng;
        const uint32_t gy = gi / G.ngx, gx = gi - gy * G.ngx;
        const uint32_t ty = gy * kGroupH + r;
        if (ty >= (uint32_t)P.nty) continue;   // the row lies below the frame
        const uint32_t beg = ci.y, end = ci.z, b0 = ci.w;
        // cursors of the row's tiles (lane c < 8 loads tile c's), then wave-uniform
        uint32_t cl = 0, el = 0;
        const uint32_t txl = gx * kGroupW + (uint32_t)lane;
        if (lane < kGroupW && txl < (uint32_t)P.ntx) {
            const uint2 rg = ranges[(size_t)f * P.n_tiles + ty * P.ntx + txl];
            cl = rg.x + cntB[(size_t)b0 * 64 + r * kGroupW + lane];
            el = rg.y;
        }
        uint32_t cur[kGroupW];
#pragma unroll
        for (int c = 0; c < kGroupW; ++c) cur[c] = (uint32_t)__builtin_amdgcn_readlane((int)cl, c);
        const uint32_t ncol = min((uint32_t)kGroupW, (uint32_t)P.ntx - gx * kGroupW);   // tiles inside the frame
        // the ranges are clamped to the capacity, so only an end strictly
        // below it proves that the whole list fits
        if (__ballot(el >= fast_end) == 0ull)
            place_row<true>(beg, end, r, lane, cur, ncol, cap, gval, gloc, tval);
        else
            place_row<false>(beg, end, r, lane, cur, ncol, cap, gval, gloc, tval);
    }
}

// One workgroup of kColWaves waves per (frame, group): exclusive scan of each
// lane's tile column over the group's segments (each wave a share of them,
// then a prefix over the waves); per-tile totals.
constexpr int kColWaves = 8;

__global__ void __launch_bounds__(64 * kColWaves) k_tile_colscan(Params P, int S, int R,
                                                      const uint32_t* __restrict__ seg_start,
                                                      const uint32_t* __restrict__ chunk_start,
                                                      const uint2* __restrict__ granges,
                                                      uint32_t* __restrict__ cntB,
                                                      uint32_t* __restrict__ tcount,
                                                      uint4* __restrict__ chunk_info) {
    __shared__ uint32_t part[kColWaves][64];
    const Groups G = groups_of(P);
    const int fg = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int f = fg / G.ng, gi = fg - f * G.ng;
    const uint32_t gy = gi / G.ngx, gx = gi - gy * G.ngx;
    const uint32_t tx = gx * kGroupW + lane % kGroupW, ty = gy * kGroupH + lane / kGroupW;
    const uint32_t s0 = seg_start[fg], s1 = seg_start[fg + 1];
    {   // the group's placement chunks, so that a placing wave finds its
        // chunk's group and entries with one load
        const uint32_t c0 = chunk_start[fg], c1 = chunk_start[fg + 1];
        const uint2 gr = granges[fg];
        for (uint32_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
            const uint32_t i = c - c0;
            const uint32_t beg = gr.x + i * (uint32_t)(R * S);
            chunk_info[c] = make_uint4((uint32_t)fg, beg, min(beg + (uint32_t)(R * S), gr.y), s0 + i * (uint32_t)R);
        }
    }
    const uint32_t per = (s1 - s0 + kColWaves - 1) / kColWaves;
    const uint32_t b0 = min(s0 + wave * per, s1), b1 = min(b0 + per, s1);
    uint32_t sum = 0;
    uint32_t b = b0;
    for (; b + 8 <= b1; b += 8) {   // 8 independent loads in flight
        uint32_t v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = cntB[(size_t)(b + i) * 64 + lane];
#pragma unroll
        for (int i = 0; i < 8; ++i) sum += v[i];
    }
    for (; b < b1; ++b) sum += cntB[(size_t)b * 64 + lane];
    part[wave][lane] = sum;
    __syncthreads();
    uint32_t run = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kColWaves; ++w) {
        run += w < wave ? part[w][lane] : 0u;
        total += part[w][lane];
    }
    for (b = b0; b + 8 <= b1; b += 8) {
        uint32_t v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = cntB[(size_t)(b + i) * 64 + lane];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            cntB[(size_t)(b + i) * 64 + lane] = run;
            run += v[i];
        }
    }
    for (; b < b1; ++b) {
        const uint32_t v = cntB[(size_t)b * 64 + lane];
        cntB[(size_t)b * 64 + lane] = run;
        run += v;
    }
    if (wave == 0 && tx < (uint32_t)P.ntx && ty < (uint32_t)P.nty)
        tcount[(size_t)f * P.n_tiles + ty * P.ntx + tx] = total;
}

// Single workgroup: tile-list ranges = exclusive scan of the per-(frame, tile)
// totals; pair count, capacity and overflow into the status block.  Ranges
// are clamped to the capacity so that an overflowed forward stays in bounds.
__global__ void __launch_bounds__(1024) k_tile_keyscan(const uint32_t* __restrict__ tcount, long long K,
                                                       unsigned long long cap, uint2* __restrict__ ranges,
                                                       const uint32_t* __restrict__ nf_block, int n_blocks,
                                                       unsigned long long wcount_off, const uint32_t* sort_fault,
                                                       Status* status) {
    __shared__ unsigned long long scratch[17];
    unsigned long long carry = 0;
    // 4 consecutive tiles per thread, 4096 per round; the next round's counts
    // are loaded while this round is scanned
    uint32_t nv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const long long i = 4 * (long long)threadIdx.x + j;
        nv[j] = i < K ? tcount[i] : 0u;
    }
    for (long long base = 0; base < K; base += 4096) {
        const long long i0 = base + 4 * (long long)threadIdx.x;
        uint32_t v[4];
        unsigned long long sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = nv[j];
            sum += v[j];
            nv[j] = i0 + 4096 + j < K ? tcount[i0 + 4096 + j] : 0u;
        }
        unsigned long long tot;
        unsigned long long a = carry + block_exclusive_scan<unsigned long long, 1024>(sum, scratch, &tot);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned long long b = a + v[j];
            if (i0 + j < K) ranges[i0 + j] = make_uint2((uint32_t)(a < cap ? a : cap), (uint32_t)(b < cap ? b : cap));
            a = b;
        }
        carry += tot;
    }
    uint32_t nf = 0;   // non-finite Gaussians counted by the preprocess blocks
    for (int i = threadIdx.x; i < n_blocks; i += 1024) nf += nf_block[i];
    nf = wave_reduce_sum(nf);
    __shared__ uint32_t nf_sum;
    if (threadIdx.x == 0) nf_sum = 0;
    __syncthreads();
    if (lane_id() == 0 && nf) atomicAdd(&nf_sum, nf);
    __syncthreads();
    if (threadIdx.x == 0) {
        status->n_pairs = carry;
        status->cap = cap;
        status->overflow = carry > cap ? 1u : 0u;
        status->overflow_seen |= carry > cap ? 1u : 0u;
        if (carry > status->n_pairs_seen) status->n_pairs_seen = carry;
        status->nonfinite = nf_sum;
        status->sort_fault = sort_fault ? *sort_fault : 0u;
        status->wcount_off = wcount_off;
        status->n_items = (unsigned long long)K;
        status->magic = kStatusMagic;
    }
}

// Introspection: the sorted rectangles back in item order.
__global__ void k_item_rects(const uint32_t* __restrict__ dval, const uint2* __restrict__ drect, long long M,
                             uint2* __restrict__ out) {
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < M;
         j += (long long)gridDim.x * blockDim.x)
        out[dval[j]] = drect[j];
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
    while (C < 2048 && M / C > 16384) C *= 2;
    g.C = C;
    g.QC = n > 0 ? (int)((n + C - 1) / C) : 0;
    g.ng = ((ntx + kGroupW - 1) / kGroupW) * ((nty + kGroupH - 1) / kGroupH);
    // level-B segment: 128 entries (two batches of 64) -- short segments give
    // enough waves to hide the load latency of the placing pass
    g.S = 128;
    // placement chunk: 8 segments, so a wave appends 1024 entries' worth of
    // each tile's run
    g.R = 8;
    // every segment but the last of each group list holds S entries, and the
    // group lists hold at most min(cap, M * groups) entries
    uint64_t entries = cap;
    if ((uint64_t)M * g.ng < entries) entries = (uint64_t)M * g.ng;
    g.max_segments = (int64_t)((entries + g.S - 1) / g.S) + (int64_t)n_frames * g.ng;
    return g;
}

// Grid caps of the one-wave placing and counting kernels.  Their waves wait
// on loads most of the time, so a grid of several times the 8192 resident
// waves (32 per CU) keeps the chip busier than a resident-sized one: level A
// gets one wave per work item up to 128K items (1M x 16 frames: 94K); the
// level-B grids are sized from an upper bound on the segments, so their cap
// also bounds the waves that find no work.
constexpr int64_t kPlaceGridA = 131072;
constexpr int64_t kLevelBGrid = 32768;

hipError_t launch_binning(const Params& P, const Workspace& w, int dbuf, hipStream_t s) {
    const BinGeom g = bin_geometry(P.n, P.F, P.ntx, P.nty, P.cap);
    const int K = P.F * g.ng;
    const unsigned chunks = (unsigned)(P.F * g.QC);
    if (chunks) {
        ProfScope _p("k_group_count", s);
        const int cpw = g.C >= 512 ? 1 : (g.C >= 256 ? 2 : 4);   // 512 / C in [1, 4]
        hipLaunchKernelGGL(k_group_count, dim3((chunks + cpw - 1) / cpw), dim3(256), 0, s, P, g.C, g.QC, cpw,
                           w.dkey[dbuf], w.drect[dbuf], w.cntA);
    }
    if (chunks) {
        ProfScope _p("k_group_colscan", s);
        hipLaunchKernelGGL(k_group_colscan, dim3(g.ng, P.F), dim3(256), 0, s, P, g.QC,
                           w.cntA, w.lenA);
    } else {
        launch_fill_u32(w.lenA, 0u, K, s);
    }
    {
        ProfScope _p("k_group_scan", s);
        hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(1024), 0, s, w.lenA, K, g.S, g.R,
                           (unsigned long long)P.cap, w.granges, w.seg_start, w.chunk_start);
    }
    if (chunks) {
        ProfScope _p("k_group_place", s);
        const int ngy = (P.nty + kGroupH - 1) / kGroupH, ngx = (P.ntx + kGroupW - 1) / kGroupW;
        // runs of up to 512 items per wave while at least 8192 work items
        // remain (200k x 8 frames: runs of 4 chunks of 128; one 640 x 480
        // frame of 100k: 1 chunk; 1M x 16 frames: 1 chunk of 1024)
        int RA = g.C >= 512 ? 1 : 512 / g.C;
        while (RA > 1 && (int64_t)P.F * ((g.QC + RA - 1) / RA) * ngy < 8192) RA /= 2;
        const int64_t items = (int64_t)P.F * ((g.QC + RA - 1) / RA) * ngy;
        const unsigned grid = (unsigned)((items < kPlaceGridA ? items : kPlaceGridA) + 7) / 8 * 8;
        if ((int64_t)RA * g.C >= 1024)
            hipLaunchKernelGGL(k_group_place<8>, dim3(grid), dim3(64), 4 * (size_t)ngx, s, P, g.C, g.QC, RA,
                               w.dval[dbuf], w.dkey[dbuf], w.drect[dbuf], w.cntA, w.granges, w.gval, w.gloc);
        else
            hipLaunchKernelGGL(k_group_place<1>, dim3(grid), dim3(64), 4 * (size_t)ngx, s, P, g.C, g.QC, RA,
                               w.dval[dbuf], w.dkey[dbuf], w.drect[dbuf], w.cntA, w.granges, w.gval, w.gloc);
    }
    // persistent level-B grids: every wave loops over segments (counting) or
    // over (chunk, tile row) work items (placing; a multiple of 8 workgroups,
    // as its split of the work items over the XCDs needs)
    const unsigned segs = (unsigned)(g.max_segments < kLevelBGrid ? g.max_segments : kLevelBGrid);
    const int64_t max_items = ((g.max_segments + g.R - 1) / g.R + K) * kGroupH;
    const unsigned place_grid = (unsigned)((max_items < kLevelBGrid ? max_items : kLevelBGrid) + 7) / 8 * 8;
    {
        ProfScope _p("k_tile_count", s);
        hipLaunchKernelGGL(k_tile_count, dim3(segs), dim3(64), 0, s, P, g.S, w.seg_start, w.granges,
                           w.gloc, w.cntB);
    }
    {
        ProfScope _p("k_tile_colscan", s);
        hipLaunchKernelGGL(k_tile_colscan, dim3(K), dim3(64 * kColWaves), 0, s, P, g.S, g.R, w.seg_start,
                           w.chunk_start, w.granges, w.cntB, w.tcount, w.chunk_info);
    }
    {
        ProfScope _p("k_tile_keyscan", s);
        hipLaunchKernelGGL(k_tile_keyscan, dim3(1), dim3(1024), 0, s, w.tcount,
                           (long long)P.F * P.n_tiles, (unsigned long long)P.cap, w.ranges, w.nf_block,
                           (int)((P.n + 255) / 256),
                           (unsigned long long)(reinterpret_cast<char*>(w.wcount) - reinterpret_cast<char*>(w.status)),
                           one_sweep_sort(P, w) ? w.sctl + kSortFault : nullptr, w.status);
    }
    {
        ProfScope _p("k_tile_place", s);
        hipLaunchKernelGGL(k_tile_place, dim3(place_grid), dim3(64), 0, s, P, w.chunk_start, w.chunk_info,
                           w.gval, w.gloc, w.cntB, w.ranges, w.tval);
    }
    return hipGetLastError();
}

void launch_item_rects(const Workspace& w, int dbuf, uint2* out, hipStream_t s) {
    if (w.M == 0) return;
    const long long blocks = (w.M + 255) / 256;
    hipLaunchKernelGGL(k_item_rects, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s,
                       w.dval[dbuf], w.drect[dbuf], (long long)w.M, out);
}

void launch_keys_from_ranges(const Params& P, const Workspace& w, uint32_t* keys,
                             unsigned long long limit, hipStream_t s) {
    const long long K = (long long)P.F * P.n_tiles;
    hipLaunchKernelGGL(k_keys_from_ranges, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s,
                       w.ranges, K, limit, keys);
}

}  // namespace gft
