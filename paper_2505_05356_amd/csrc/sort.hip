// Depth ordering and tile binning of the (frame, Gaussian) items.
//
// The compositing order the image formation model needs (paper §3: each
// pixel composites the Gaussians of its tile front to back) is produced in
// two sorts instead of one wide (frame, tile, depth) sort:
//   1. a stable LSD radix sort of the M = F * N items by their 32-bit depth
//      key (items start in (frame, index) order, so ties keep index order);
//   2. pair emission in that depth order: every item writes one
//      ((frame, tile) key, item) pair per covered tile;
//   3. a stable LSD radix sort of the P pairs by the (frame, tile) key only,
//      ceil(log2(F * n_tiles)) bits, which keeps the depth order inside each
//      tile.
// The pair sort is the largest byte mover of the forward; cutting its key
// from 46+ bits to ~14 bits cuts its passes from 6 to 2.
//
// Radix passes are reduce-then-scan (upsweep tile histograms, per-digit
// column scan, downsweep rank-and-scatter), with no inter-workgroup waiting.
// Ranking inside a tile is stable: wave-level peer matching with ballots,
// wave-private digit counters in LDS, then an LDS reorder so each digit run is
// written to HBM contiguously.  Counts of data-dependent size (P) are read
// from device memory, so no host synchronisation is needed and the launch
// sequence can be graph-captured; grids are sized by capacity and loop.
#include "block_scan.h"
#include "common.h"

namespace gft {

namespace {

struct Count {
    const unsigned long long* dev;   // device count (clamped to cap) or NULL
    unsigned long long host;         // used when dev == NULL
    unsigned long long cap;
};

__device__ __forceinline__ unsigned long long get_n(const Count& c) {
    if (!c.dev) return c.host;
    unsigned long long v = *c.dev;
    return v < c.cap ? v : c.cap;
}

template <int TAG>  // 0: depth sort of items, 1: (frame, tile) sort of pairs
__global__ void __launch_bounds__(kSortThreads) k_sort_upsweep(const uint32_t* __restrict__ keys,
                                                               Count cn, int shift, int nbits,
                                                               uint32_t* __restrict__ counts,
                                                               long long stride) {
    __shared__ uint32_t hist[4][kSortBuckets];
    const unsigned long long n = get_n(cn);
    const long long ntiles = (long long)((n + kSortTile - 1) / kSortTile);
    const uint32_t mask = (1u << nbits) - 1u;
    const int wave = threadIdx.x / 64;
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        for (int i = threadIdx.x; i < 4 * kSortBuckets; i += kSortThreads) (&hist[0][0])[i] = 0;
        __syncthreads();
        const unsigned long long base = (unsigned long long)tile * kSortTile;
#pragma unroll 4
        for (int it = 0; it < kSortItems; ++it) {
            const unsigned long long idx = base + it * kSortThreads + threadIdx.x;
            if (idx < n) atomicAdd(&hist[wave][(keys[idx] >> shift) & mask], 1u);
        }
        __syncthreads();
        const int d = threadIdx.x;
        counts[(long long)d * stride + tile] = hist[0][d] + hist[1][d] + hist[2][d] + hist[3][d];
        __syncthreads();
    }
}

// One workgroup per digit: exclusive scan of that digit's per-tile counts.
template <int TAG>
__global__ void __launch_bounds__(256) k_sort_scan(uint32_t* __restrict__ counts, Count cn,
                                                   long long stride, uint32_t* __restrict__ totals) {
    __shared__ uint32_t scratch[8];
    const unsigned long long n = get_n(cn);
    const long long ntiles = (long long)((n + kSortTile - 1) / kSortTile);
    uint32_t* row = counts + (long long)blockIdx.x * stride;
    uint32_t carry = 0;
    for (long long base = 0; base < ntiles; base += 256 * 4) {
        uint32_t v[4];
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long i = base + threadIdx.x * 4 + j;
            v[j] = i < ntiles ? row[i] : 0u;
            s += v[j];
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_scan<uint32_t, 256>(s, scratch, &tot);
        uint32_t run = carry + ex;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long i = base + threadIdx.x * 4 + j;
            if (i < ntiles) row[i] = run;
            run += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

template <int TAG>  // 0: depth sort of items, 1: (frame, tile) sort of pairs
__global__ void __launch_bounds__(kSortThreads) k_sort_downsweep(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, Count cn, int shift, int nbits, const uint32_t* __restrict__ counts,
    const uint32_t* __restrict__ totals, long long stride) {
    __shared__ uint32_t digit_base[kSortBuckets];
    __shared__ uint32_t whist[4][kSortBuckets];
    __shared__ uint32_t tile_start[kSortBuckets];
    __shared__ uint32_t tile_cnt[kSortBuckets];
    __shared__ uint32_t skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    __shared__ uint32_t scratch[8];

    const unsigned long long n = get_n(cn);
    const long long ntiles = (long long)((n + kSortTile - 1) / kSortTile);
    const uint32_t mask = (1u << nbits) - 1u;
    const int nb = 1 << nbits;
    const int tid = threadIdx.x;
    const int wave = tid / 64;
    const int lane = tid % 64;

    {   // exclusive scan of the digit totals -> global base of each digit
        uint32_t tot;
        uint32_t v = tid < nb ? totals[tid] : 0u;
        uint32_t ex = block_exclusive_scan<uint32_t, kSortThreads>(v, scratch, &tot);
        digit_base[tid] = ex;
    }
    __syncthreads();

    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const unsigned long long base = (unsigned long long)tile * kSortTile;
        for (int i = lane; i < kSortBuckets; i += 64) whist[wave][i] = 0;
        uint32_t k[kSortItems], v[kSortItems], rank[kSortItems];
        const unsigned long long wbase = base + (unsigned long long)wave * (kSortItems * 64);
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const unsigned long long idx = wbase + it * 64 + lane;
            const bool ok = idx < n;
            k[it] = ok ? kin[idx] : 0u;
            v[it] = ok ? vin[idx] : 0u;
            // digit, with bit `nbits` flagging an out-of-range lane
            rank[it] = ok ? ((k[it] >> shift) & mask) : (1u << nbits);
        }
        __syncthreads();  // whist cleared
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const uint32_t d = rank[it];
            unsigned long long peers = ~0ull;
            for (int b = 0; b <= nbits; ++b) {
                const bool bit = (d >> b) & 1u;
                const unsigned long long bal = __ballot(bit);
                peers &= bit ? bal : ~bal;
            }
            const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
            const uint32_t cnt = (uint32_t)__popcll(peers);
            // Wave-synchronous LDS counter: every lane of the peer group reads
            // the counter, then its highest lane advances it.  LDS operations
            // of one wave complete in issue order and the volatile accesses
            // keep the compiler from reordering them across iterations.
            volatile uint32_t* wh = whist[wave];
            uint32_t prev = 0;
            const bool valid = d < (uint32_t)nb;
            if (valid) prev = wh[d];
            if (valid && below == cnt - 1) wh[d] = prev + cnt;
            rank[it] = valid ? prev + below : 0xffffffffu;
        }
        __syncthreads();
        {   // wave offsets per digit and tile-local digit starts
            const int d = tid;
            uint32_t s = 0;
            for (int w = 0; w < 4; ++w) {
                const uint32_t c = whist[w][d];
                whist[w][d] = s;
                s += c;
            }
            tile_cnt[d] = s;
            uint32_t tot;
            uint32_t ex = block_exclusive_scan<uint32_t, kSortThreads>(s, scratch, &tot);
            tile_start[d] = ex;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            if (rank[it] != 0xffffffffu) {
                const uint32_t d = (k[it] >> shift) & mask;
                const uint32_t pos = tile_start[d] + whist[wave][d] + rank[it];
                skey[pos] = k[it];
                sval[pos] = v[it];
            }
        }
        __syncthreads();
        const unsigned long long rem = n - base;
        const int valid_n = rem < (unsigned long long)kSortTile ? (int)rem : kSortTile;
        for (int j = tid; j < valid_n; j += kSortThreads) {
            const uint32_t key = skey[j];
            const uint32_t d = (key >> shift) & mask;
            const unsigned long long g = (unsigned long long)digit_base[d] +
                                         counts[(long long)d * stride + tile] + (j - tile_start[d]);
            kout[g] = key;
            vout[g] = sval[j];
        }
        __syncthreads();
    }
}

// ---- pair emission ----------------------------------------------------------

__global__ void __launch_bounds__(kEmitThreads) k_emit_count(const uint32_t* __restrict__ dval,
                                                             const uint32_t* __restrict__ cnt,
                                                             long long M,
                                                             unsigned long long* __restrict__ chunk_sum) {
    __shared__ unsigned long long red[kEmitThreads / 64];
    const long long j0 = (long long)blockIdx.x * kEmitChunk;
    unsigned long long s = 0;
#pragma unroll
    for (int r = 0; r < kEmitItems; ++r) {
        const long long j = j0 + r * kEmitThreads + threadIdx.x;
        if (j < M) s += cnt[dval[j]];
    }
    s = wave_reduce_sum(s);
    if (lane_id() == 0) red[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kEmitThreads / 64; ++w) t += red[w];
        chunk_sum[blockIdx.x] = t;
    }
}

// Single workgroup: chunk sums -> exclusive offsets; total pairs and overflow.
__global__ void __launch_bounds__(1024) k_emit_scan(unsigned long long* __restrict__ chunk_sum,
                                                    long long n_chunks, Status* status,
                                                    unsigned long long cap,
                                                    unsigned long long* __restrict__ off_end) {
    __shared__ unsigned long long scratch[17];
    unsigned long long carry = 0;
    for (long long base = 0; base < n_chunks; base += 1024) {
        const long long i = base + threadIdx.x;
        const unsigned long long v = i < n_chunks ? chunk_sum[i] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_exclusive_scan<unsigned long long, 1024>(v, scratch, &tot);
        if (i < n_chunks) chunk_sum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        chunk_sum[n_chunks] = carry;
        *off_end = carry;
        status->n_pairs = carry;
        status->cap = cap;
        status->overflow = carry > cap ? 1u : 0u;
    }
}

// Each workgroup takes 1024 consecutive depth-sorted items, scans their tile
// counts and writes every item's first pair position; every item also marks
// the pair blocks whose first pair it owns, so the pair-writing kernel needs
// no search over the items.
__global__ void __launch_bounds__(kEmitThreads) k_emit_offsets(Params P, const uint32_t* __restrict__ dval,
                                                               const uint32_t* __restrict__ cnt,
                                                               const unsigned long long* __restrict__ chunk_off,
                                                               long long M,
                                                               unsigned long long* __restrict__ off,
                                                               uint32_t* __restrict__ first) {
    __shared__ uint32_t scratch[kEmitThreads / 64 + 1];
    const long long j0 = (long long)blockIdx.x * kEmitChunk;
    const int t = threadIdx.x;
    uint32_t c[kEmitItems];
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kEmitItems; ++r) {
        const long long j = j0 + t * kEmitItems + r;
        c[r] = j < M ? cnt[dval[j]] : 0u;
        s += c[r];
    }
    uint32_t total;
    uint32_t ex = block_exclusive_scan<uint32_t, kEmitThreads>(s, scratch, &total);
    const unsigned long long base = chunk_off[blockIdx.x];
    const unsigned long long cap = P.cap;
#pragma unroll
    for (int r = 0; r < kEmitItems; ++r) {
        const long long j = j0 + t * kEmitItems + r;
        if (j < M) {
            const unsigned long long o = base + ex;
            off[j] = o;
            if (c[r]) {
                const unsigned long long e = o + c[r];
                for (unsigned long long b = (o + kPairsPerBlock - 1) / kPairsPerBlock;
                     b * kPairsPerBlock < e && b * kPairsPerBlock < cap; ++b)
                    first[b] = (uint32_t)j;
            }
        }
        ex += c[r];
    }
}

// Pair writing, balanced by pairs: workgroup b writes pairs
// [b * 2048, (b + 1) * 2048), each thread 8 consecutive pairs (two 16-byte
// stores per array).  The items overlapping the block are staged in LDS from
// first[b]; a thread finds its first item by binary search and then walks.
__global__ void __launch_bounds__(kEmitThreads) k_emit_pairs(Params P, const uint32_t* __restrict__ dval,
                                                             const uint2* __restrict__ rect,
                                                             const unsigned long long* __restrict__ off,
                                                             const uint32_t* __restrict__ first,
                                                             long long M, const Status* __restrict__ status,
                                                             uint32_t* __restrict__ tkey,
                                                             uint32_t* __restrict__ tval) {
    constexpr int PB = kPairsPerBlock;
    __shared__ int loff[PB + 2];
    __shared__ uint32_t litem[PB + 1];
    __shared__ uint32_t lbase[PB + 1];
    __shared__ uint16_t lw[PB + 1];
    const unsigned long long np_all = status->n_pairs < P.cap ? status->n_pairs : P.cap;
    const unsigned long long b0 = (unsigned long long)blockIdx.x * PB;
    if (b0 >= np_all) return;
    const int npairs = (int)((np_all - b0) < (unsigned long long)PB ? (np_all - b0) : PB);
    const uint32_t j0 = first[blockIdx.x];
    const int t = threadIdx.x;
    const uint32_t n = (uint32_t)P.n;
    for (int i = t; i < PB + 1; i += kEmitThreads) {
        const long long j = (long long)j0 + i;
        int lo = 0x7fffffff;
        uint32_t item = 0, kb = 0;
        uint16_t w = 1;
        if (j < M) {
            const unsigned long long o = off[j];
            if (o < b0 + (unsigned long long)npairs) {
                lo = (int)((long long)o - (long long)b0);
                item = dval[j];
                const uint2 rc = rect[item];
                const uint32_t xlo = rc.x & 0xffff, xhi = rc.x >> 16, ylo = rc.y & 0xffff;
                w = (uint16_t)(xhi - xlo + 1);
                kb = (item / n) * (uint32_t)P.n_tiles + ylo * (uint32_t)P.ntx + xlo;
            }
        }
        loff[i] = lo;
        litem[i] = item;
        lbase[i] = kb;
        lw[i] = w;
    }
    if (t == 0) loff[PB + 1] = 0x7fffffff;
    __syncthreads();
    const int p0 = t * kPairsPerThread;
    if (p0 >= npairs) return;
    int lo = 0, hi = PB + 1;   // loff[lo] <= p0 < loff[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (loff[mid] <= p0) lo = mid; else hi = mid;
    }
    int slot = lo;
    uint32_t item = litem[slot], kb = lbase[slot], w = lw[slot];
    const uint32_t ntx = (uint32_t)P.ntx;
    uint32_t local = (uint32_t)(p0 - loff[slot]);
    uint32_t ty = local / w, tx = local - ty * w;
    int next = loff[slot + 1];
    uint32_t k[kPairsPerThread], v[kPairsPerThread];
#pragma unroll
    for (int q = 0; q < kPairsPerThread; ++q) {
        const int p = p0 + q;
        if (p == next) {
            ++slot;
            item = litem[slot];
            kb = lbase[slot];
            w = lw[slot];
            tx = ty = 0;
            next = loff[slot + 1];
        }
        k[q] = kb + ty * ntx + tx;
        v[q] = item;
        if (++tx == w) {
            tx = 0;
            ++ty;
        }
    }
    const unsigned long long g = b0 + p0;
    if (p0 + kPairsPerThread <= npairs) {
        uint4* kd = reinterpret_cast<uint4*>(tkey + g);
        uint4* vd = reinterpret_cast<uint4*>(tval + g);
        kd[0] = make_uint4(k[0], k[1], k[2], k[3]);
        kd[1] = make_uint4(k[4], k[5], k[6], k[7]);
        vd[0] = make_uint4(v[0], v[1], v[2], v[3]);
        vd[1] = make_uint4(v[4], v[5], v[6], v[7]);
    } else {
        for (int q = 0; q < npairs - p0; ++q) {
            tkey[g + q] = k[q];
            tval[g + q] = v[q];
        }
    }
}

__global__ void k_ranges(const uint32_t* __restrict__ keys, Count cn, uint2* __restrict__ ranges) {
    const unsigned long long n = get_n(cn);
    for (unsigned long long p = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (unsigned long long)gridDim.x * blockDim.x) {
        const uint32_t k = keys[p];
        if (p == 0 || keys[p - 1] != k) ranges[k].x = (uint32_t)p;
        if (p == n - 1 || keys[p + 1] != k) ranges[k].y = (uint32_t)(p + 1);
    }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f32(float* p, float v, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

unsigned grid_for(long long items, long long per_block, unsigned cap_blocks) {
    long long b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap_blocks) b = cap_blocks;
    return (unsigned)b;
}

// One stable LSD pass; ping-pong is managed by the caller.  TAG only names
// the instantiation (depth or pair sort) for profiling.
template <int TAG>
void radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                const Count& cn, long long max_items, int shift, int nbits, const Workspace& w,
                hipStream_t s) {
    static const char* names[2][3] = {
        {"k_sort_upsweep<depth>", "k_sort_scan<depth>", "k_sort_downsweep<depth>"},
        {"k_sort_upsweep<pairs>", "k_sort_scan<pairs>", "k_sort_downsweep<pairs>"}};
    const long long stride = w.max_sort_tiles;
    const unsigned g = grid_for(max_items, kSortTile, 2048);
    {
        ProfScope _p(names[TAG][0], s);
        hipLaunchKernelGGL(k_sort_upsweep<TAG>, dim3(g), dim3(kSortThreads), 0, s, kin, cn, shift,
                           nbits, w.counts, stride);
    }
    {
        ProfScope _p(names[TAG][1], s);
        hipLaunchKernelGGL(k_sort_scan<TAG>, dim3(1u << nbits), dim3(256), 0, s, w.counts, cn, stride,
                           w.totals);
    }
    {
        ProfScope _p(names[TAG][2], s);
        hipLaunchKernelGGL(k_sort_downsweep<TAG>, dim3(g), dim3(kSortThreads), 0, s, kin, vin, kout,
                           vout, cn, shift, nbits, w.counts, w.totals, stride);
    }
}

}  // namespace

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    { ProfScope _p("k_fill_u32", s);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256 * 4, 4096)), dim3(256), 0, s, p, v,
                       (long long)n);
    }
}

void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    { ProfScope _p("k_fill_f32", s);
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256 * 4, 4096)), dim3(256), 0, s, p, v,
                       (long long)n);
    }
}

// Depth sort of the M items (32-bit keys, 4 passes of 8 bits); the sorted
// arrays end in buffer 0 (an even number of passes).
void launch_depth_sort(const Params& P, const Workspace& w, hipStream_t s, int* result_buf) {
    Count cn{nullptr, (unsigned long long)w.M, (unsigned long long)w.M};
    int cur = 0;
    for (int pass = 0; pass < 4; ++pass) {
        radix_pass<0>(w.dkey[cur], w.dval[cur], w.dkey[cur ^ 1], w.dval[cur ^ 1], cn, w.M, 8 * pass,
                      8, w, s);
        cur ^= 1;
    }
    *result_buf = cur;
}

void launch_emit(const Params& P, const Workspace& w, int dbuf, hipStream_t s) {
    const unsigned chunks = (unsigned)w.n_chunks;
    if (chunks) {
        ProfScope _p("k_emit_count", s);
        hipLaunchKernelGGL(k_emit_count, dim3(chunks), dim3(kEmitThreads), 0, s, w.dval[dbuf], w.cnt,
                           (long long)w.M, w.chunk_sum);
    }
    {
        ProfScope _p("k_emit_scan", s);
        hipLaunchKernelGGL(k_emit_scan, dim3(1), dim3(1024), 0, s, w.chunk_sum, (long long)w.n_chunks,
                           w.status, (unsigned long long)P.cap, w.off + w.M);
    }
    if (chunks) {
        ProfScope _p("k_emit_offsets", s);
        hipLaunchKernelGGL(k_emit_offsets, dim3(chunks), dim3(kEmitThreads), 0, s, P, w.dval[dbuf],
                           w.cnt, w.chunk_sum, (long long)w.M, w.off, w.first);
    }
    const unsigned long long blocks = (P.cap + kPairsPerBlock - 1) / kPairsPerBlock;
    if (blocks) {
        ProfScope _p("k_emit_pairs", s);
        hipLaunchKernelGGL(k_emit_pairs, dim3((unsigned)blocks), dim3(kEmitThreads), 0, s, P,
                           w.dval[dbuf], w.rect, w.off, w.first, (long long)w.M, w.status, w.tkey[0],
                           w.tval[0]);
    }
}

// Stable sort of the pairs by (frame, tile); returns the buffer holding the result.
int launch_tile_sort(const Params& P, const Workspace& w, hipStream_t s) {
    Count cn{&w.status->n_pairs, 0ull, (unsigned long long)P.cap};
    const int bits = P.key_bits < 1 ? 1 : P.key_bits;
    const int passes = (bits + 7) / 8;
    const int per = (bits + passes - 1) / passes;
    int cur = 0, shift = 0;
    for (int pass = 0; pass < passes; ++pass) {
        const int nb = (shift + per <= bits) ? per : bits - shift;
        radix_pass<1>(w.tkey[cur], w.tval[cur], w.tkey[cur ^ 1], w.tval[cur ^ 1], cn,
                      (long long)P.cap, shift, nb, w, s);
        cur ^= 1;
        shift += nb;
    }
    return cur;
}

void launch_ranges(const Params& P, const Workspace& w, int tbuf, hipStream_t s) {
    launch_fill_u32(reinterpret_cast<uint32_t*>(w.ranges), 0u, 2ll * P.F * P.n_tiles, s);
    Count cn{&w.status->n_pairs, 0ull, (unsigned long long)P.cap};
    { ProfScope _p("k_ranges", s);
    hipLaunchKernelGGL(k_ranges, dim3(grid_for((long long)P.cap, 256 * 8, 8192)), dim3(256), 0, s,
                       w.tkey[tbuf], cn, w.ranges);
    }
}

}  // namespace gft
