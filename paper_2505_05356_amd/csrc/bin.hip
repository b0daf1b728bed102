// Tile binning: per-(frame, tile) Gaussian lists in depth order, built from
// the frame-major depth-sorted items without sorting (tile, Gaussian) pairs.
//
// Each item covers a rectangle of tiles.  The pair of (item j, tile t) must
// land at start[t] + #{items before j in depth order that cover t}, which is
// the order the compositing loop of paper §3 walks.  The depth-ordered items
// of each frame are cut into chunks of C items:
//   k_bin_count   one workgroup per chunk: per-tile counts of the chunk in
//                 LDS (rectangles expanded with LDS atomics), written as one
//                 row of the [chunk][tile] count matrix;
//   k_bin_colscan exclusive scan of every tile's column over the chunks of
//                 its frame (16 waves split the rows), and per-tile totals;
//   k_bin_keyscan exclusive scan of the totals over (frame, tile): the list
//                 ranges, the pair count and the capacity check;
//   k_bin_place   one wave per chunk: LDS cursors start[t] + column prefix,
//                 then the chunk's items in depth order, the lanes expanding
//                 one item's rectangle at a time; each lane writes the item id
//                 at its tile's cursor and advances it.
// HBM traffic is the pair list written once (4 B per pair) plus the count
// matrix (4 B per chunk and tile, read and written twice), instead of an
// emitted key/value pair list and two radix passes over it.
#include "block_scan.h"
#include "common.h"

namespace gft {

namespace {

__device__ __forceinline__ void unpack_rect(uint2 rc, uint32_t& xlo, uint32_t& xhi, uint32_t& ylo,
                                            uint32_t& yhi) {
    xlo = rc.x & 0xffff;
    xhi = rc.x >> 16;
    ylo = rc.y & 0xffff;
    yhi = rc.y >> 16;
}

__global__ void __launch_bounds__(256) k_bin_count(Params P, int C, int QC,
                                                   const uint32_t* __restrict__ dval,
                                                   const uint32_t* __restrict__ cnt,
                                                   const uint2* __restrict__ rect,
                                                   uint32_t* __restrict__ cntmat) {
    extern __shared__ uint32_t lcnt[];
    const int chunk = blockIdx.x;
    const int f = chunk / QC, q = chunk - f * QC;
    const int nt = P.n_tiles;
    const int ntx = P.ntx;
    for (int t = threadIdx.x; t < nt; t += 256) lcnt[t] = 0;
    __syncthreads();
    const long long beg = (long long)f * P.n + (long long)q * C;
    const long long end = min(beg + C, (long long)(f + 1) * P.n);
    for (long long j = beg + threadIdx.x; j < end; j += 256) {
        const uint32_t item = dval[j];
        if (cnt[item] == 0) continue;
        uint32_t xlo, xhi, ylo, yhi;
        unpack_rect(rect[item], xlo, xhi, ylo, yhi);
        for (uint32_t ty = ylo; ty <= yhi; ++ty)
            for (uint32_t tx = xlo; tx <= xhi; ++tx) atomicAdd(&lcnt[ty * ntx + tx], 1u);
    }
    __syncthreads();
    uint32_t* out = cntmat + (size_t)chunk * nt;
    for (int t = threadIdx.x; t < nt; t += 256) out[t] = lcnt[t];
}

// grid (ceil(nt / 64), F), 1024 threads: lane = tile within a group of 64,
// wave = one sixteenth of the frame's chunk rows.
__global__ void __launch_bounds__(1024) k_bin_colscan(Params P, int QC, uint32_t* __restrict__ cntmat,
                                                      uint32_t* __restrict__ tcount) {
    __shared__ uint32_t part[16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nt = P.n_tiles;
    const int t = blockIdx.x * 64 + lane;
    const int f = blockIdx.y;
    const int rows = (QC + 15) / 16;
    const int q0 = wave * rows, q1 = min(q0 + rows, QC);
    uint32_t* col = cntmat + (size_t)f * QC * nt + t;
    uint32_t s = 0;
    if (t < nt)
        for (int q = q0; q < q1; ++q) s += col[(size_t)q * nt];
    part[wave][lane] = s;
    __syncthreads();
    uint32_t run = 0, total = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) run += part[w][lane];
        total += part[w][lane];
    }
    if (t < nt) {
        for (int q = q0; q < q1; ++q) {
            const uint32_t v = col[(size_t)q * nt];
            col[(size_t)q * nt] = run;
            run += v;
        }
        if (wave == 0) tcount[(size_t)f * nt + t] = total;
    }
}

// Single workgroup: list ranges = exclusive scan of the per-(frame, tile)
// totals; pair count, capacity and overflow into the status block.  Ranges
// are clamped to the capacity so that an overflowed forward stays in bounds.
__global__ void __launch_bounds__(1024) k_bin_keyscan(const uint32_t* __restrict__ tcount, long long K,
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

// One wave per chunk (blockDim 64).  Dynamic LDS: nt cursors.
__global__ void __launch_bounds__(64) k_bin_place(Params P, int C, int QC,
                                                  const uint32_t* __restrict__ dval,
                                                  const uint32_t* __restrict__ cnt,
                                                  const uint2* __restrict__ rect,
                                                  const uint32_t* __restrict__ cntmat,
                                                  const uint2* __restrict__ ranges,
                                                  uint32_t* __restrict__ tval) {
    extern __shared__ uint32_t cursor[];
    __shared__ uint32_t sitem[64];
    __shared__ uint2 srect[64];
    const int chunk = blockIdx.x;
    const int f = chunk / QC, q = chunk - f * QC;
    const int nt = P.n_tiles;
    const uint32_t ntx = (uint32_t)P.ntx;
    const int lane = threadIdx.x;
    const uint32_t cap = (uint32_t)(P.cap < 0xffffffffull ? P.cap : 0xffffffffull);
    const uint32_t* pre = cntmat + (size_t)chunk * nt;
    for (int t = lane; t < nt; t += 64) cursor[t] = ranges[(size_t)f * nt + t].x + pre[t];
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
            const uint32_t w = xhi - xlo + 1;
            const uint32_t area = w * (yhi - ylo + 1);
            const float inv_w = 1.0f / (float)w;
            for (uint32_t k = lane; k < area; k += 64) {
                // k / w by a float reciprocal, corrected to the exact quotient
                uint32_t ty = (uint32_t)((float)k * inv_w);
                if (ty * w > k) --ty;
                if ((ty + 1) * w <= k) ++ty;
                const uint32_t tx = k - ty * w;
                const uint32_t t = (ylo + ty) * ntx + xlo + tx;
                const uint32_t pos = cur[t];
                cur[t] = pos + 1;
                if (pos < cap) tval[pos] = item;
            }
        }
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

BinGeom bin_geometry(int64_t n, int n_tiles) {
    BinGeom g;
    int C = 512;
    while (C < 8192 && C < n_tiles / 4) C *= 2;
    g.C = C;
    g.QC = n > 0 ? (int)((n + C - 1) / C) : 0;
    return g;
}

hipError_t launch_binning(const Params& P, const Workspace& w, int dbuf, hipStream_t s) {
    const BinGeom g = bin_geometry(P.n, P.n_tiles);
    const unsigned chunks = (unsigned)(P.F * g.QC);
    const size_t lds = sizeof(uint32_t) * (size_t)P.n_tiles;
    if (chunks) {
        ProfScope _p("k_bin_count", s);
        hipLaunchKernelGGL(k_bin_count, dim3(chunks), dim3(256), lds, s, P, g.C, g.QC, w.dval[dbuf],
                           w.cnt, w.rect, w.cntmat);
    }
    if (chunks) {
        ProfScope _p("k_bin_colscan", s);
        hipLaunchKernelGGL(k_bin_colscan, dim3((P.n_tiles + 63) / 64, P.F), dim3(1024), 0, s, P, g.QC,
                           w.cntmat, w.tcount);
    } else {
        launch_fill_u32(w.tcount, 0u, (int64_t)P.F * P.n_tiles, s);
    }
    {
        ProfScope _p("k_bin_keyscan", s);
        hipLaunchKernelGGL(k_bin_keyscan, dim3(1), dim3(1024), 0, s, w.tcount,
                           (long long)P.F * P.n_tiles, (unsigned long long)P.cap, w.ranges, w.status);
    }
    if (chunks) {
        ProfScope _p("k_bin_place", s);
        hipLaunchKernelGGL(k_bin_place, dim3(chunks), dim3(64), lds, s, P, g.C, g.QC, w.dval[dbuf],
                           w.cnt, w.rect, w.cntmat, w.ranges, w.tval);
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
