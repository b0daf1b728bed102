// Depth ordering of the (frame, Gaussian) items.
//
// Every pixel composites the Gaussians of its tile front to back (paper §3),
// in ascending (depth key, Gaussian index) order per frame.  The M = F * N
// items start in (frame, index) order; a stable LSD radix sort over their
// 32-bit depth keys (4 passes of 8 bits), run segment by segment (one segment
// per frame), leaves them frame-major and depth-ordered inside each frame,
// ties in index order.  The tile lists are then built from this order by the
// binning kernels (bin.hip) without sorting any (tile, Gaussian) pairs.
//
// Radix passes are reduce-then-scan (upsweep tile histograms, per-(frame,
// digit) column scan, downsweep rank-and-scatter) with no inter-workgroup
// waiting.  Batches of few sort tiles, where those three launches per pass
// cost more than the work, instead count the digits of all four passes in
// one launch and sort each pass in one launch: a workgroup takes the next
// sort tile from an atomic counter, ranks its keys, publishes its per-digit
// counts and adds those of the frame's earlier tiles by decoupled look-back
// (a bounded wait: those tiles were taken earlier, so their workgroups are
// running), then scatters.  Sort tiles never straddle a frame.  Each item's tile rectangle
// rides along as payload, so the binning kernels read it in depth order
// without gathering it by item id.  Ranking inside a tile is
// stable: wave-level peer matching with ballots, wave-private digit counters
// in LDS, then an LDS reorder so that each digit run is written contiguously.
#include "block_scan.h"
#include "common.h"

namespace gft {

namespace {

// Sort tile `g` of the segmented layout: frame and element range.
struct SortTile {
    long long f, t, beg, end;
};

__device__ __forceinline__ SortTile sort_tile(long long g, long long n, long long tpf) {
    SortTile r;
    r.f = g / tpf;
    r.t = g - r.f * tpf;
    r.beg = r.f * n + r.t * kSortTile;
    r.end = min(r.beg + kSortTile, (r.f + 1) * n);
    return r;
}

// counts[(f * 256 + d) * tpf + t] = keys of digit d in tile t of frame f.
// CP copies of each wave's histogram, lane l counting into copy l % CP: the
// top byte of positive float depths takes few values, so its counts would
// otherwise serialise on a few LDS addresses.
template <int CP>
__global__ void __launch_bounds__(kSortThreads) k_sort_upsweep(const uint32_t* __restrict__ keys, long long n,
                                                               int F, long long tpf, int shift,
                                                               uint32_t* __restrict__ counts) {
    __shared__ uint32_t hist[4 * CP][kSortBuckets];
    const int copy = (threadIdx.x / 64) * CP + (int)(threadIdx.x % CP);
    const long long ntiles = (long long)F * tpf;
    // consecutive tiles write neighbouring counts of every digit row: one XCD
    const long long g0 = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    for (long long g = g0; g < ntiles; g += gridDim.x) {
        const SortTile st = sort_tile(g, n, tpf);
        for (int i = threadIdx.x; i < 4 * CP * kSortBuckets; i += kSortThreads) (&hist[0][0])[i] = 0;
        // a histogram needs no element order: each thread loads its 8 keys
        // as two 16-byte vectors where the tile is whole and 16-byte aligned,
        // all loads in flight before the first count
        uint32_t kv[kSortItems];
        const long long i0 = st.beg + (long long)threadIdx.x * 4;
        const bool vec = st.end - st.beg == kSortTile && (st.beg & 3) == 0;
        if (vec) {
            const uint4 a = *reinterpret_cast<const uint4*>(keys + i0);
            const uint4 b = *reinterpret_cast<const uint4*>(keys + i0 + 4 * kSortThreads);
            kv[0] = a.x, kv[1] = a.y, kv[2] = a.z, kv[3] = a.w;
            kv[4] = b.x, kv[5] = b.y, kv[6] = b.z, kv[7] = b.w;
        } else {
#pragma unroll
            for (int it = 0; it < kSortItems; ++it) {
                const long long idx = st.beg + it * kSortThreads + threadIdx.x;
                kv[it] = idx < st.end ? keys[idx] : 0u;
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const bool ok = vec || st.beg + it * kSortThreads + threadIdx.x < st.end;
            if (ok) atomicAdd(&hist[copy][(kv[it] >> shift) & 0xffu], 1u);
        }
        __syncthreads();
        const int d = threadIdx.x;
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < 4 * CP; ++q) c += hist[q][d];
        counts[(st.f * kSortBuckets + d) * tpf + st.t] = c;
        __syncthreads();
    }
}

// One workgroup per (digit, frame): exclusive scan of that row of per-tile
// counts; the row total goes to totals[f * 256 + d].
__global__ void __launch_bounds__(256) k_sort_scan(uint32_t* __restrict__ counts, long long tpf,
                                                   uint32_t* __restrict__ totals) {
    __shared__ uint32_t scratch[8];
    const long long rowi = (long long)blockIdx.y * kSortBuckets + blockIdx.x;
    uint32_t* row = counts + rowi * tpf;
    uint32_t carry = 0;
    for (long long base = 0; base < tpf; base += 256 * 4) {
        uint32_t v[4];
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long i = base + threadIdx.x * 4 + j;
            v[j] = i < tpf ? row[i] : 0u;
            s += v[j];
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_scan<uint32_t, 256>(s, scratch, &tot);
        uint32_t run = carry + ex;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long i = base + threadIdx.x * 4 + j;
            if (i < tpf) row[i] = run;
            run += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) totals[rowi] = carry;
}

__global__ void __launch_bounds__(kSortThreads) k_sort_downsweep(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, const uint2* __restrict__ rin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, uint2* __restrict__ rout, long long n, int F,
    long long tpf, int shift,
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ totals) {
    __shared__ uint32_t digit_base[kSortBuckets];
    __shared__ uint32_t whist[4][kSortBuckets];
    __shared__ uint32_t tile_start[kSortBuckets];
    __shared__ uint32_t out_base[kSortBuckets];
    __shared__ uint32_t skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    __shared__ uint2 srect[kSortTile];
    __shared__ uint32_t scratch[8];

    const long long ntiles = (long long)F * tpf;
    const int tid = threadIdx.x;
    const int wave = tid / 64;
    const int lane = tid % 64;
    long long cur_f = -1;

    // consecutive tiles write adjacent runs of every digit: one XCD
    const long long g0 = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    for (long long g = g0; g < ntiles; g += gridDim.x) {
        const SortTile st = sort_tile(g, n, tpf);
        if (st.f != cur_f) {   // start of each digit inside this frame's segment
            __syncthreads();
            uint32_t tot;
            const uint32_t ex = block_exclusive_scan<uint32_t, kSortThreads>(
                totals[st.f * kSortBuckets + tid], scratch, &tot);
            digit_base[tid] = ex;
            cur_f = st.f;
        }
        for (int i = lane; i < kSortBuckets; i += 64) whist[wave][i] = 0;
        // this tile's offset of digit `tid` among the frame's keys of that
        // digit, loaded now so the load overlaps the ranking
        const uint32_t tile_off = counts[(st.f * kSortBuckets + tid) * tpf + st.t];
        uint32_t k[kSortItems], v[kSortItems], rank[kSortItems];
        uint2 rc[kSortItems];
        const long long wbase = st.beg + (long long)wave * (kSortItems * 64);
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const long long idx = wbase + it * 64 + lane;
            const bool ok = idx < st.end;
            k[it] = ok ? kin[idx] : 0u;
            v[it] = ok ? vin[idx] : 0u;
            rc[it] = ok ? rin[idx] : make_uint2(0u, 0u);
            // digit, with bit 8 flagging an out-of-range lane
            rank[it] = ok ? ((k[it] >> shift) & 0xffu) : 0x100u;
        }
        __syncthreads();  // whist cleared, digit_base written
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const uint32_t d = rank[it];
            unsigned long long peers = ~0ull;
            for (int b = 0; b <= 8; ++b) {
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
            // keep the compiler from reordering them across iterations; the
            // pointer keeps its LDS address space, so they stay LDS
            // instructions rather than generic (flat) ones.
            volatile __attribute__((address_space(3))) uint32_t* wh =
                (volatile __attribute__((address_space(3))) uint32_t*)whist[wave];
            uint32_t prev = 0;
            const bool valid = d < (uint32_t)kSortBuckets;
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
            uint32_t tot;
            uint32_t ex = block_exclusive_scan<uint32_t, kSortThreads>(s, scratch, &tot);
            tile_start[d] = ex;
            // output position of the tile's element j of digit d, minus j
            // (mod 2^32: the true position is below n)
            out_base[d] = digit_base[d] + tile_off - ex;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            if (rank[it] != 0xffffffffu) {
                const uint32_t d = (k[it] >> shift) & 0xffu;
                const uint32_t pos = tile_start[d] + whist[wave][d] + rank[it];
                skey[pos] = k[it];
                sval[pos] = v[it];
                srect[pos] = rc[it];
            }
        }
        __syncthreads();
        // scatter: no global loads here, so the stores of all kSortItems
        // rounds issue back to back
        const int valid_n = (int)(st.end - st.beg);
        const long long fbase = st.f * n;
#pragma unroll
        for (int it = 0; it < kSortItems; ++it) {
            const int j = tid + it * kSortThreads;
            if (j < valid_n) {
                const uint32_t key = skey[j];
                const uint32_t d = (key >> shift) & 0xffu;
                const long long gpos = fbase + (long long)(uint32_t)(out_base[d] + (uint32_t)j);
                kout[gpos] = key;
                vout[gpos] = sval[j];
                rout[gpos] = srect[j];
            }
        }
        __syncthreads();
    }
}

// Digit counts of every pass of the one-sweep sort: shist[(f * 4 + pass) *
// 256 + d] += keys of frame f whose digit `pass` is d (the key multiset is
// the same in every pass).  One workgroup per sort tile, which also clears
// the tile's look-back words of the first pass.
__global__ void __launch_bounds__(kSortThreads) k_sort_hist(const uint32_t* __restrict__ keys, long long n,
                                                            long long tpf, uint32_t* __restrict__ shist,
                                                            uint32_t* __restrict__ look0) {
    __shared__ uint32_t hist[kSortThreads / 64][kSortPasses][kSortBuckets];
    const long long g = blockIdx.x;
    const SortTile st = sort_tile(g, n, tpf);
    const int tid = threadIdx.x, wave = tid / 64;
    look0[g * kSortBuckets + tid] = 0u;
    for (int i = tid; i < (kSortThreads / 64) * kSortPasses * kSortBuckets; i += kSortThreads)
        (&hist[0][0][0])[i] = 0u;
    uint32_t kv[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const long long idx = st.beg + it * kSortThreads + tid;
        kv[it] = idx < st.end ? keys[idx] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        if (st.beg + it * kSortThreads + tid < st.end)
#pragma unroll
            for (int p = 0; p < kSortPasses; ++p) atomicAdd(&hist[wave][p][(kv[it] >> (8 * p)) & 0xffu], 1u);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kSortPasses; ++p) {
        uint32_t v = 0;
        for (int w = 0; w < kSortThreads / 64; ++w) v += hist[w][p][tid];
        if (v) atomicAdd(&shist[(st.f * kSortPasses + p) * kSortBuckets + tid], v);
    }
}

// Look-back word of (tile, digit): count << 2 | state, state 1 = the tile's
// own count, 2 = the inclusive count of the frame's tiles up to this one.
constexpr uint32_t kLookAggregate = 1u, kLookInclusive = 2u;
// A tile waits at most this many polls for an earlier tile to publish; past
// it the sort raises the fault flag (reported by gftorf_read_status) instead
// of waiting on.
constexpr int kLookSpinLimit = 1 << 22;

__device__ __forceinline__ uint32_t look_load(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void look_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One stable pass over digit `pass` of every frame's segment, one workgroup
// per sort tile.  look holds the pass's look-back words (cleared by the
// previous launch); look_next, if not NULL, is cleared here for the next pass.
__global__ void __launch_bounds__(kSortThreads) k_sort_onesweep(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, const uint2* __restrict__ rin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, uint2* __restrict__ rout, long long n,
    long long tpf, int pass, const uint32_t* __restrict__ shist, uint32_t* __restrict__ sctl,
    uint32_t* __restrict__ look, uint32_t* __restrict__ look_next) {
    __shared__ uint32_t whist[4][kSortBuckets];
    __shared__ uint32_t tile_start[kSortBuckets];
    __shared__ uint32_t out_base[kSortBuckets];
    __shared__ uint32_t skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    __shared__ uint2 srect[kSortTile];
    __shared__ uint32_t scratch[8];
    __shared__ uint32_t s_tile;

    const int tid = threadIdx.x;
    const int wave = tid / 64;
    const int lane = tid % 64;
    const int shift = 8 * pass;
    // tiles are numbered in the order their workgroups start, so every tile
    // a workgroup waits for belongs to a workgroup that is already running
    if (tid == 0) s_tile = atomicAdd(&sctl[pass], 1u);
    for (int i = lane; i < kSortBuckets; i += 64) whist[wave][i] = 0;
    __syncthreads();
    const long long g = s_tile;
    const SortTile st = sort_tile(g, n, tpf);
    if (look_next) look_next[g * kSortBuckets + tid] = 0u;
    const uint32_t fcount = shist[(st.f * kSortPasses + pass) * kSortBuckets + tid];

    uint32_t k[kSortItems], v[kSortItems], rank[kSortItems];
    uint2 rc[kSortItems];
    const long long wbase = st.beg + (long long)wave * (kSortItems * 64);
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const long long idx = wbase + it * 64 + lane;
        const bool ok = idx < st.end;
        k[it] = ok ? kin[idx] : 0u;
        v[it] = ok ? vin[idx] : 0u;
        rc[it] = ok ? rin[idx] : make_uint2(0u, 0u);
        rank[it] = ok ? ((k[it] >> shift) & 0xffu) : 0x100u;   // bit 8: out of range
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const uint32_t d = rank[it];
        unsigned long long peers = ~0ull;
        for (int b = 0; b <= 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
        const uint32_t cnt = (uint32_t)__popcll(peers);
        // the wave-synchronous LDS counter of the three-launch downsweep
        volatile __attribute__((address_space(3))) uint32_t* wh =
            (volatile __attribute__((address_space(3))) uint32_t*)whist[wave];
        uint32_t prev = 0;
        const bool valid = d < (uint32_t)kSortBuckets;
        if (valid) prev = wh[d];
        if (valid && below == cnt - 1) wh[d] = prev + cnt;
        rank[it] = valid ? prev + below : 0xffffffffu;
    }
    __syncthreads();
    {   // wave offsets per digit, tile-local digit starts, and the tile's
        // place among the frame's tiles by look-back (thread = digit)
        const int d = tid;
        uint32_t cnt = 0;
        for (int w = 0; w < 4; ++w) {
            const uint32_t c = whist[w][d];
            whist[w][d] = cnt;
            cnt += c;
        }
        uint32_t tot;
        const uint32_t ts = block_exclusive_scan<uint32_t, kSortThreads>(cnt, scratch, &tot);
        tile_start[d] = ts;
        const uint32_t base = block_exclusive_scan<uint32_t, kSortThreads>(fcount, scratch, &tot);
        uint32_t* mine = look + g * kSortBuckets + d;
        uint32_t excl = 0;
        if (st.t == 0) {
            look_store(mine, (cnt << 2) | kLookInclusive);
        } else {
            look_store(mine, (cnt << 2) | kLookAggregate);
            const long long first = st.f * tpf;
            int spins = 0;
            for (long long j = g - 1; j >= first;) {
                const uint32_t wv = look_load(look + j * kSortBuckets + d);
                const uint32_t state = wv & 3u;
                if (state == 0u) {
                    if (++spins > kLookSpinLimit) {
                        sctl[kSortFault] = 1u;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += wv >> 2;
                if (state == kLookInclusive) break;
                --j;
            }
            look_store(mine, ((excl + cnt) << 2) | kLookInclusive);
        }
        // output position of the tile's element j of digit d, minus j
        // (mod 2^32: the true position is below n)
        out_base[d] = base + excl - ts;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        if (rank[it] != 0xffffffffu) {
            const uint32_t d = (k[it] >> shift) & 0xffu;
            const uint32_t pos = tile_start[d] + whist[wave][d] + rank[it];
            skey[pos] = k[it];
            sval[pos] = v[it];
            srect[pos] = rc[it];
        }
    }
    __syncthreads();
    const int valid_n = (int)(st.end - st.beg);
    const long long fbase = st.f * n;
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        const int j = tid + it * kSortThreads;
        if (j < valid_n) {
            const uint32_t key = skey[j];
            const uint32_t d = (key >> shift) & 0xffu;
            const long long gpos = fbase + (long long)(uint32_t)(out_base[d] + (uint32_t)j);
            kout[gpos] = key;
            vout[gpos] = sval[j];
            rout[gpos] = srect[j];
        }
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

// One stable LSD pass over the F segments of n elements; ping-pong is
// managed by the caller.
void radix_pass(const uint32_t* kin, const uint32_t* vin, const uint2* rin, uint32_t* kout, uint32_t* vout,
                uint2* rout, long long n, int F, int shift, const Workspace& w, hipStream_t s) {
    const long long tpf = w.max_sort_tiles;
    // one workgroup per sort tile up to 16K tiles (33.5M keys): the
    // downsweep measured 5% faster than with half as many workgroups
    // looping over two tiles each (16M keys)
    const unsigned g = grid_for((long long)F * tpf, 1, 16384);
    {
        ProfScope _p("k_sort_upsweep", s);
        if (shift == 24)
            hipLaunchKernelGGL(k_sort_upsweep<4>, dim3(g), dim3(kSortThreads), 0, s, kin, n, F, tpf, shift,
                               w.counts);
        else
            hipLaunchKernelGGL(k_sort_upsweep<1>, dim3(g), dim3(kSortThreads), 0, s, kin, n, F, tpf, shift,
                           w.counts);
    }
    {
        ProfScope _p("k_sort_scan", s);
        hipLaunchKernelGGL(k_sort_scan, dim3(kSortBuckets, F), dim3(256), 0, s, w.counts, tpf, w.totals);
    }
    {
        ProfScope _p("k_sort_downsweep", s);
        hipLaunchKernelGGL(k_sort_downsweep, dim3(g), dim3(kSortThreads), 0, s, kin, vin, rin, kout, vout, rout,
                           n, F, tpf, shift, w.counts, w.totals);
    }
}

}  // namespace

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    ProfScope _p("k_fill_u32", s);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256 * 4, 4096)), dim3(256), 0, s, p, v,
                       (long long)n);
}

void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    ProfScope _p("k_fill_f32", s);
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256 * 4, 4096)), dim3(256), 0, s, p, v,
                       (long long)n);
}

int depth_sort_passes(int) { return kSortPasses; }

// Frame-major depth sort of the M items; returns the buffer holding the result.
int launch_depth_sort(const Params& P, const Workspace& w, hipStream_t s) {
    int cur = 0;
    if (w.M == 0) return 0;
    if (one_sweep_sort(P, w)) {   // the preprocess has cleared sctl and shist
        const long long tpf = w.max_sort_tiles;
        const unsigned tiles = (unsigned)(P.F * tpf);
        {
            ProfScope _p("k_sort_hist", s);
            hipLaunchKernelGGL(k_sort_hist, dim3(tiles), dim3(kSortThreads), 0, s, w.dkey[0], (long long)P.n,
                               tpf, w.shist, w.slook[0]);
        }
        for (int pass = 0; pass < kSortPasses; ++pass) {
            ProfScope _p("k_sort_onesweep", s);
            hipLaunchKernelGGL(k_sort_onesweep, dim3(tiles), dim3(kSortThreads), 0, s, w.dkey[cur], w.dval[cur],
                               w.drect[cur], w.dkey[cur ^ 1], w.dval[cur ^ 1], w.drect[cur ^ 1], (long long)P.n,
                               tpf, pass, w.shist, w.sctl, w.slook[pass & 1],
                               pass + 1 < kSortPasses ? w.slook[(pass + 1) & 1] : nullptr);
            cur ^= 1;
        }
        return cur;
    }
    for (int pass = 0; pass < kSortPasses; ++pass) {
        radix_pass(w.dkey[cur], w.dval[cur], w.drect[cur], w.dkey[cur ^ 1], w.dval[cur ^ 1], w.drect[cur ^ 1],
                   P.n, P.F, 8 * pass, w, s);
        cur ^= 1;
    }
    return cur;
}

}  // namespace gft
