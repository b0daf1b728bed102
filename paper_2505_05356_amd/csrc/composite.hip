// Front-to-back compositing (forward) and back-to-front gradient recursion
// (backward) of RGB, mean depth and raw C-ToF quads, one workgroup per
// (frame, tile) work item: one thread per pixel in the forward, 4 pixels per
// lane in the backward.
//
// Forward (paper §3): for each pixel walk the tile's depth-sorted list and
//   alpha = min(alpha_max, o G(x)),  skip if alpha < alpha_min,
//   stop before compositing if T (1 - alpha) < T_min,
//   RGB += c alpha T (Eq. 2), D += d alpha T (Eq. 5),
//   S_f += a sin(psi_f) alpha T^2, C_f += a cos(psi_f) alpha T^2 (Eq. 4),
// then Q_{f,j} = cos(phi_j) S_f + sin(phi_j) C_f + q_bg T^p, because
// sin(psi + phi) = sin(psi) cos(phi) + cos(psi) sin(phi): two accumulators
// per frequency serve every phase offset.
//
// Backward (supplement C): walk the same list back to front from the last
// composited entry, recover T_k = T_{k+1} / (1 - alpha_k) from the saved
// T_final, and accumulate dL/dalpha_k with Eq. S2 (RGB, depth) and Eq. S3
// (quads) plus the background terms; then chain to the per-entry screen-space
// quantities.  Per-entry gradients are summed over the wave with DPP and
// added to the per-(frame, Gaussian) gradient record with one atomic per wave.
//
// Records of 64 list entries at a time are staged in LDS by each wave, in
// its own slice (the forward's waves walk their tile's list independently;
// the backward has one wave per tile in large batches and 2 or 4 waves, each
// with its own pixels, in small ones): one coalesced gather per entry of its
// 48-byte record and 16-byte conic, then every lane of the wave reads them as
// LDS broadcasts.  No MFMA: per (pixel, entry) this is ~20 FP32 VALU
// operations and one v_exp_f32.
#include "block_scan.h"
#include "common.h"

namespace gft {

namespace {

// Base-2 exponent q of the 2-D Gaussian at (px, py): the conic is stored
// prescaled by -log2(e) / 2 (-log2(e) for the cross term), so o G = o 2^q.
// One definition shared by the forward and the backward kernels, with
// contraction pinned, so both take identical skip / stop / clamp decisions:
// q = dy (C dy + B dx) + A dx^2, where the column terms B dx and A dx^2 are
// formed once per pixel column (splat_col) and reused by every pixel of it.
struct SplatCol {
    float dx, bdx, adx2;
};

__device__ __forceinline__ SplatCol splat_col(const float4 c, const float4 r1, float px) {
#pragma clang fp contract(off)
    SplatCol k;
    k.dx = px - c.x;
    k.bdx = r1.y * k.dx;
    k.adx2 = (r1.x * k.dx) * k.dx;
    return k;
}

__device__ __forceinline__ float splat_row(const SplatCol& k, const float4 c, const float4 r1, float py,
                                           float& dy) {
#pragma clang fp contract(off)
    dy = py - c.y;
    return __builtin_fmaf(dy, __builtin_fmaf(r1.z, dy, k.bdx), k.adx2);
}

// Below this exponent (log2 units) alpha < alpha_min with room to spare for
// the rounding of exp2, the product and the threshold itself.
constexpr float kSkipMargin = 1.0f / 64.0f;

// The staged form of an entry's centre for one tile: the centre relative to
// the tile origin (the hi + lo pair folded once per entry), and the exponent
// threshold thr with q < thr  =>  min(o 2^q, alpha_max) < alpha_min, which
// lets the backward skip an entry that no pixel of the tile can take without
// changing any decision.
// lamin = log2(alpha_min), or -inf when alpha_min = 0 (nothing skipped).
__device__ __forceinline__ float4 stage_centre(const float4 r0, float o, float ox, float oy, float lamin) {
    const float cu = (r0.x - ox) + r0.z;
    const float cv = (r0.y - oy) + r0.w;
    return make_float4(cu, cv, (lamin - __log2f(o)) - kSkipMargin, 0.f);
}

// Sum over the 64 lanes of a wave: DPP within rows of 16, then 4 readlanes.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xf,
                                                              0xf, true));
}

__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f32<0xb1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f32<0x4e>(v);    // quad_perm [2,3,0,1]
    v += dpp_f32<0x114>(v);   // row_shr:4
    v += dpp_f32<0x118>(v);   // row_shr:8 -> lane 15 of each row holds the row sum
    const int b = __builtin_bit_cast(int, v);
    return (__builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 15)) +
            __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 31))) +
           (__builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 47)) +
            __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 63)));
}

// Value of the lane whose index differs from this lane's in bit log2(D) and
// agrees in all lower bits (rotations within a row of 16 satisfy this for
// D = 4 and D = 8; D >= 16 uses a full cross-lane permute).
template <int D>
__device__ __forceinline__ float xchg(float x) {
    if constexpr (D == 1) return dpp_f32<0xb1>(x);          // quad_perm [1,0,3,2]
    else if constexpr (D == 2) return dpp_f32<0x4e>(x);     // quad_perm [2,3,0,1]
    else if constexpr (D == 4) return dpp_f32<0x124>(x);    // row_ror:4
    else if constexpr (D == 8) return dpp_f32<0x128>(x);    // row_ror:8
    else return __shfl_xor(x, D, 64);
}

// Reduce-scatter of NP per-lane fields by butterfly: at distance D each lane
// keeps the half of its live fields selected by bit log2(D) of its lane index
// and adds the partner's copy of that half.  NP - 1 exchanges instead of
// NP * log2(64) for NP independent reductions.
template <int NP, int D = 1>
__device__ __forceinline__ void butterfly(float* v, int lane) {
    if constexpr (D < NP) {
        constexpr int H = NP / (2 * D);
        const bool hi = (lane & D) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const float send = hi ? v[i] : v[i + H];
            const float keep = hi ? v[i + H] : v[i];
            v[i] = keep + xchg<D>(send);
        }
        butterfly<NP, 2 * D>(v, lane);
    }
}

template <int D>
__device__ __forceinline__ float allreduce_from(float r) {
    if constexpr (D < 64) return allreduce_from<2 * D>(r + xchg<D>(r));
    else return r;
}

// Field whose wave total lane `lane` holds after wave_reduce_fields<NP>.
template <int NP>
__host__ __device__ constexpr int field_of_lane(int lane) {
    int f = 0;
#pragma unroll
    for (int D = 1; D < NP; D *= 2)
        if (lane & D) f += NP / (2 * D);
    return f;
}

// Sums v[0..NP) over the 64 lanes; returns, in every lane, the total of
// field field_of_lane<NP>(lane).
template <int NP>
__device__ __forceinline__ float wave_reduce_fields(float (&v)[NP], int lane) {
    butterfly<NP>(v, lane);
    return allreduce_from<NP>(v[0]);
}

template <int TW, int TH, int NF>
__global__ void __launch_bounds__(TW * TH) k_composite_fwd(Params P, const gftorf_frame* __restrict__ frames,
                                                           const uint2* __restrict__ ranges,
                                                           const uint32_t* __restrict__ tval,
                                                           const float4* __restrict__ rec,
                                                           const float4* __restrict__ conic,
                                                           gftorf_outputs out, uint2* __restrict__ wcount) {
    constexpr int BS = TW * TH;
    static_assert(BS % 64 == 0, "a tile is a whole number of waves");
    // Each wave stages 64 list entries at a time into its own LDS slice and
    // walks them without a workgroup barrier, so a wave whose pixels are all
    // done (T < T_min) stops while the others continue. Most pixels stop after
    // ~100-200 entries, so short batches also waste few record loads.
    constexpr int NWV = BS / 64;
    constexpr int RS4 = record_float4s(NF);
    constexpr int SS4 = staged_float4s(NF);
    __shared__ float4 srec_w[NWV][SS4][64];

    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const int f = w / P.n_tiles;
    const int tile = w - f * P.n_tiles;
    const int ty = tile / P.ntx, tx = tile - ty * P.ntx;
    const int tid = threadIdx.x;
    const int x = tx * TW + (tid % TW), y = ty * TH + (tid / TW);
    const bool inside = x < P.W && y < P.H;
    // pixel centre relative to the tile origin (exact small values)
    const float fpx = (float)(tid % TW) + 0.5f, fpy = (float)(tid / TW) + 0.5f;
    const float ox = (float)(tx * TW), oy = (float)(ty * TH);
    const uint2 rg = ranges[w];
    const float amin = P.alpha_min, amax = P.alpha_max, tmin = P.T_min;
    const float lamin = amin > 0.f ? __log2f(amin) : -INFINITY;

    float T = 1.0f;
    float cr = 0.f, cg = 0.f, cb = 0.f, dep = 0.f;
    float S[NF], C[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) S[i] = C[i] = 0.f;
    bool done = !inside;
    uint32_t last = 0;
    uint32_t n_eval = 0, n_comp = 0;   // evaluated / composited (pixel, entry) pairs

    float4 (*srec)[64] = srec_w[tid / 64];
    const int lane = tid & 63;
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += 64) {
        if (__ballot(!done) == 0ull) break;
        const uint32_t j = b0 + lane;
        // the previous batch's LDS reads of every lane precede these writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (j < rg.y) {
            const uint32_t item = tval[j];
            const float4* r = rec + (size_t)item * RS4;
            const float4 r1 = conic[item];
            srec[0][lane] = stage_centre(r[0], r1.w, ox, oy, lamin);
            srec[1][lane] = r1;
#pragma unroll
            for (int q = 1; q < RS4; ++q) srec[q + 1][lane] = r[q];
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int cnt = __builtin_amdgcn_readfirstlane((int)min(64u, rg.y - b0));
        // Divergent per pixel (a lane that is done or skips an entry simply
        // idles): measured faster here than branch-free selects with
        // wave-uniform ballot exits.
        for (int k = 0; k < cnt; ++k) {
            if (done) continue;
            ++n_eval;
            const float4 c = srec[0][k], r1 = srec[1][k];
            float dy;
            const float qe = splat_row(splat_col(c, r1, fpx), c, r1, fpy, dy);
            const float a = fminf(r1.w * __builtin_amdgcn_exp2f(qe), amax);
            if (a < amin) continue;
            const float nT = T * (1.0f - a);
            if (nT < tmin) {   // stop before compositing
                done = true;
                continue;
            }
            const float4 r2 = srec[2][k];
            const float w1 = a * T;
            const float w2 = w1 * T;
            cr += r2.x * w1;
            cg += r2.y * w1;
            cb += r2.z * w1;
            dep += r2.w * w1;
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                const float4 rp = srec[3 + i / 2][k];
                S[i] += ((i & 1) ? rp.z : rp.x) * w2;
                C[i] += ((i & 1) ? rp.w : rp.y) * w2;
            }
            T = nT;
            ++n_comp;
            last = b0 - rg.x + (uint32_t)k + 1u;
        }
    }
    {   // workload counters of this work item (algorithmic FLOP accounting);
        // summed over work items on the host by gftorf_read_status, not by
        // same-address atomics
        __shared__ uint2 wred[BS / 64];
        uint32_t e = n_eval, c = n_comp;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            e += (uint32_t)__shfl_xor((int)e, o, 64);
            c += (uint32_t)__shfl_xor((int)c, o, 64);
        }
        if ((tid & 63) == 0) wred[tid / 64] = make_uint2(e, c);
        __syncthreads();
        if (tid == 0) {
            uint2 t = wred[0];
            for (int q = 1; q < BS / 64; ++q) {
                t.x += wred[q].x;
                t.y += wred[q].y;
            }
            wcount[w] = t;
        }
    }
    if (!inside) return;
    const gftorf_frame& fr = frames[f];
    const size_t HW = (size_t)P.H * P.W;
    const size_t pix = (size_t)y * P.W + x;
    if (out.rgb) {
        float* o = out.rgb + (size_t)f * 3 * HW + pix;
        o[0] = cr + fr.bg_rgb[0] * T;
        o[HW] = cg + fr.bg_rgb[1] * T;
        o[2 * HW] = cb + fr.bg_rgb[2] * T;
    }
    if (out.quad) {
        const float Tp = P.bg_pow == 2 ? T * T : T;
        float* o = out.quad + (size_t)f * P.nq * HW + pix;
#pragma unroll
        for (int i = 0; i < NF; ++i)
            for (int jj = 0; jj < P.nphi; ++jj) {
                const int qc = i * P.nphi + jj;
                if (fr.quad_mask == 0u || ((fr.quad_mask >> qc) & 1u))
                    o[qc * HW] = P.cphi[jj] * S[i] + P.sphi[jj] * C[i] + fr.bg_quad[qc] * Tp;
            }
    }
    if (out.phasor || out.d_tof || out.amplitude) {
        const float Tp = P.bg_pow == 2 ? T * T : T;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            float sh = 0.f, ch = 0.f;   // projections of the rendered quads (Eq. 1)
            for (int jj = 0; jj < P.nphi; ++jj) {
                const int qc = i * P.nphi + jj;
                const float q = P.cphi[jj] * S[i] + P.sphi[jj] * C[i] + fr.bg_quad[qc] * Tp;
                sh += P.cphi[jj] * q;
                ch += P.sphi[jj] * q;
            }
            const size_t o = ((size_t)f * P.nf + i) * HW + pix;
            if (out.phasor) {
                out.phasor[(((size_t)f * P.nf + i) * 2) * HW + pix] = ch;
                out.phasor[(((size_t)f * P.nf + i) * 2 + 1) * HW + pix] = sh;
            }
            if (out.d_tof) {
                float ph = atan2f(sh, ch);
                if (ph < 0.f) ph += 6.283185307179586f;
                out.d_tof[o] = (float)(kSpeedOfLight / (4.0 * M_PI * P.freq[i])) * ph;
            }
            if (out.amplitude) out.amplitude[o] = 0.5f * sqrtf(sh * sh + ch * ch);
        }
    }
    if (out.depth) out.depth[(size_t)f * HW + pix] = dep;
    out.T_final[(size_t)f * HW + pix] = T;
    out.n_contrib[(size_t)f * HW + pix] = (int32_t)last;
}

// Backward: WPT waves per (frame, tile) (1 for large batches; 2 or 4 when
// the batch has too few tiles to fill the chip), each walking the tile's list
// for its own pixels; each lane owns PPT pixels of the tile
// (pixel p = lane + 64 i), so the per-entry cross-lane reduction of the
// gradient fields is paid once for PPT pixels.
//
// The upstream gradients are constant per pixel, so the recursions of Eq. S2
// (RGB and depth, factor 1 - alpha) and Eq. S3 (quads, factor (1 - alpha)^2)
// only enter dL/dalpha through the per-entry values
//   u_k = sum_c dL/dc_c c_k,c + dL/dd d_k,  v_k = sum_f dL/dS_f a sin psi + dL/dC_f a cos psi
// and their suffix sums behind entry k, kept un-normalised:
//   A1 = sum_{j>k} u_j alpha_j T_j,  A2 = sum_{j>k} v_j alpha_j T_j^2.
// (The normalised accumulators of S2 / S3 are A1 / T_{k+1} and
// A2 / T_{k+1}^2.)  With the background term bg = c_bg . dL/dc T_final +
// p q_bg . dL/dq T_final^p,
//   dL/dalpha_k = T_k u_k + T_k^2 v_k - (A1 + 2 A2 + bg) / (1 - alpha_k),
// so one running sum A = A1 + 2 A2 + bg per pixel suffices:
//   A <- A + u_k alpha_k T_k + 2 v_k alpha_k T_k^2.
template <int TW, int TH, int NF, int WPT>
__global__ void __launch_bounds__(64) k_composite_bwd(
    Params P, const gftorf_frame* __restrict__ frames, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ tval, const float4* __restrict__ rec, const float4* __restrict__ conic,
    const float* __restrict__ T_final, const int32_t* __restrict__ n_contrib,
    const float* __restrict__ d_rgb, const float* __restrict__ d_quad, const float* __restrict__ d_depth,
    float* __restrict__ grec, float* __restrict__ d_bg) {
    constexpr int PPT = TW * TH / (64 * WPT);   // pixels per lane
    constexpr int B = 64;                      // list entries staged per batch
    constexpr int RS4 = record_float4s(NF);
    constexpr int SS4 = staged_float4s(NF);
    constexpr int GS = grad_floats(NF);
    constexpr int NG = 10 + 2 * NF;            // gradient fields per entry
    constexpr int NGP = NG <= 16 ? 16 : 32;    // padded to a power of two
    static_assert(field_of_lane<NGP>(0) == 0 && field_of_lane<NGP>(NGP / 2) == 1,
                  "lanes 0 and NGP / 2 hold the totals of fields 0 and 1");
    __shared__ float4 srec[SS4][B];
    __shared__ uint32_t sitem[B];

    // the WPT waves of a work item are consecutive after the remap: one XCD
    const int wl = xcd_remap(blockIdx.x, gridDim.x);
    const int w = wl / WPT, sub = wl - w * WPT;
    const int f = w / P.n_tiles;
    const int tile = w - f * P.n_tiles;
    const int ty = tile / P.ntx, tx = tile - ty * P.ntx;
    const int lane = threadIdx.x;
    const uint2 rg = ranges[w];
    const float amin = P.alpha_min, amax = P.alpha_max;
    const float lamin = amin > 0.f ? __log2f(amin) : -INFINITY;
    const float ox = (float)(tx * TW), oy = (float)(ty * TH);
    const gftorf_frame& fr = frames[f];
    const size_t HW = (size_t)P.H * P.W;

    float fpx[PPT], fpy[PPT], T[PPT], A[PPT];
    uint32_t last[PPT];
    float gr[PPT][3], gd[PPT], gS[PPT][NF], gC[PPT][NF];
    float bg_acc[3 + GFTORF_MAX_QUAD];
    const int nbg = 3 + P.nq;
    for (int c = 0; c < 3 + GFTORF_MAX_QUAD; ++c) bg_acc[c] = 0.f;
    uint32_t maxl = 0;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int pidx = lane + 64 * (sub + WPT * i);   // same column for all i
        const int x = tx * TW + pidx % TW, y = ty * TH + pidx / TW;
        const bool inside = x < P.W && y < P.H;
        fpx[i] = (float)(pidx % TW) + 0.5f;   // relative to the tile origin
        fpy[i] = (float)(pidx / TW) + 0.5f;
        const size_t pix = (size_t)y * P.W + x;
        float Tf = 1.f, Tp = 1.f, brd = 0.f, bqd = 0.f;
        last[i] = 0;
        gr[i][0] = gr[i][1] = gr[i][2] = gd[i] = 0.f;
#pragma unroll
        for (int k = 0; k < NF; ++k) gS[i][k] = gC[i][k] = 0.f;
        if (inside) {
            Tf = T_final[(size_t)f * HW + pix];
            last[i] = (uint32_t)n_contrib[(size_t)f * HW + pix];
            Tp = P.bg_pow == 2 ? Tf * Tf : Tf;
            if (d_rgb)
                for (int c = 0; c < 3; ++c) gr[i][c] = d_rgb[((size_t)f * 3 + c) * HW + pix];
            if (d_depth) gd[i] = d_depth[(size_t)f * HW + pix];
            for (int c = 0; c < 3; ++c) {
                brd += fr.bg_rgb[c] * gr[i][c];
                bg_acc[c] += gr[i][c] * Tf;
            }
            if (d_quad) {
#pragma unroll
                for (int k = 0; k < NF; ++k)
                    for (int jj = 0; jj < P.nphi; ++jj) {
                        const int qc = k * P.nphi + jj;
                        if (fr.quad_mask != 0u && !((fr.quad_mask >> qc) & 1u)) continue;   // not rendered
                        const float g = d_quad[((size_t)f * P.nq + qc) * HW + pix];
                        gS[i][k] += P.cphi[jj] * g;
                        gC[i][k] += P.sphi[jj] * g;
                        bqd += fr.bg_quad[qc] * g;
                        bg_acc[3 + qc] += g * Tp;
                    }
            }
        }
        // the suffix sum starts with the background term
        A[i] = brd * Tf + (float)P.bg_pow * bqd * Tp;
        T[i] = Tf;
        maxl = max(maxl, last[i]);
    }
    // background gradients: dL/dc_bg = sum d_rgb T_final, dL/dq_bg = sum d_quad T_final^p
    if (d_bg) {
        for (int c = 0; c < nbg; ++c) {
            const float v = wave_sum(bg_acc[c]);
            if (lane == 0 && v != 0.f) atomicAdd(&d_bg[(size_t)f * nbg + c], v);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) maxl = max(maxl, (uint32_t)__shfl_xor((int)maxl, o, 64));
    const float LN2 = 0.6931471805599453f;

    for (uint32_t hi = min(rg.x + maxl, rg.y); hi > rg.x; ) {
        const uint32_t lo = (hi - rg.x > (uint32_t)B) ? hi - B : rg.x;
        const int cnt = (int)(hi - lo);
        __syncthreads();
        if (lane < cnt) {
            const uint32_t item = tval[hi - 1 - lane];
            sitem[lane] = item;
            const float4* r = rec + (size_t)item * RS4;
            const float4 r1 = conic[item];
            srec[0][lane] = stage_centre(r[0], r1.w, ox, oy, lamin);
            srec[1][lane] = r1;
#pragma unroll
            for (int q = 1; q < RS4; ++q) srec[q + 1][lane] = r[q];
        }
        __syncthreads();
        for (int s = 0; s < cnt; ++s) {
            const uint32_t kidx = hi - 1 - (uint32_t)s - rg.x;   // position in the tile list
            const float4 c = srec[0][s], r1 = srec[1][s];
            // phase 1: which pixels can composite this entry (the forward's
            // decisions: not past the pixel's last entry, exponent above the
            // certain-skip threshold); an entry no pixel takes costs no more
            float dx[PPT], dy[PPT], qe[PPT];
            bool pass[PPT];
            bool anyp = false;
            const SplatCol col = splat_col(c, r1, fpx[0]);   // the lane's pixels share a column
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                dx[i] = col.dx;
                qe[i] = splat_row(col, c, r1, fpy[i], dy[i]);
                pass[i] = kidx < last[i] && !(qe[i] < c.z);
                anyp |= pass[i];
            }
            if (__ballot(anyp) == 0ull) continue;
            const float4 r2 = srec[2][s];
            float as[NF], ac[NF];
#pragma unroll
            for (int k = 0; k < NF; ++k) {
                const float4 rp = srec[3 + k / 2][s];
                as[k] = (k & 1) ? rp.z : rp.x;
                ac[k] = (k & 1) ? rp.w : rp.y;
            }
            // Sums start from their first term (pixel 0), not from 0 + term:
            // the compiler must keep an addition of +0 (it turns -0 into +0)
            float g[NGP];
#pragma unroll
            for (int q = NG; q < NGP; ++q) g[q] = 0.f;
            auto put = [](float& acc, float term, int i) { acc = i == 0 ? term : acc + term; };
            bool any = false;
            // Branch-free per pixel: inactive pixels contribute zero and keep
            // their state (selects instead of divergent blocks, so the field
            // registers are never copied at control-flow joins).
            // The conic and centre gradients only need, per lane (one pixel
            // column, so one dx), sum gq, sum gq dy and sum gq dy^2
            float p0, p1, p2;
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const float G = __builtin_amdgcn_exp2f(qe[i]);
                const float oG = r1.w * G;
                const float a = fminf(oG, amax);
                const bool act = pass[i] && a >= amin;
                any |= act;
                // ae = alpha of a composited entry, 0 otherwise: with ae = 0
                // every state update below is the identity (rcp(1) = 1)
                const float ae = act ? a : 0.0f;
                const float rom = __builtin_amdgcn_rcpf(1.0f - ae);
                const float Ti = T[i] * rom;
                const float T2 = Ti * Ti;
                const float u = gr[i][0] * r2.x + gr[i][1] * r2.y + gr[i][2] * r2.z + gd[i] * r2.w;
                float v = gS[i][0] * as[0] + gC[i][0] * ac[0];
#pragma unroll
                for (int k = 1; k < NF; ++k) v += gS[i][k] * as[k] + gC[i][k] * ac[k];
                const float dA = Ti * u + T2 * v - rom * A[i];
                T[i] = Ti;
                const float w1 = ae * Ti;
                const float w2 = ae * T2;
                A[i] += w1 * u + w2 * (2.0f * v);
                put(g[6], w1 * gr[i][0], i);
                put(g[7], w1 * gr[i][1], i);
                put(g[8], w1 * gr[i][2], i);
                put(g[9], w1 * gd[i], i);
#pragma unroll
                for (int k = 0; k < NF; ++k) {
                    put(g[10 + 2 * k], w2 * gS[i][k], i);
                    put(g[11 + 2 * k], w2 * gC[i][k], i);
                }
                // alpha = o 2^q unless clamped (then alpha has no gradient);
                // gq = dL/dq / ln 2
                const float dAe = (act && oG <= amax) ? dA : 0.0f;
                const float gq = dAe * a;
                put(g[5], G * dAe, i);                           // d/do
                const float gy = gq * dy[i];
                put(p0, gq, i);
                put(p1, gy, i);
                put(p2, gy * dy[i], i);
            }
            {
                const float dxl = dx[0];                         // the lane's column
                g[0] = dxl * p0;                                 // sum gx
                g[1] = p1;                                       // sum gy
                g[2] = (dxl * dxl) * p0;                         // d/dcA
                g[3] = dxl * p1;                                 // d/dcB
                g[4] = p2;                                       // d/dcC
            }
            if (__ballot(any) == 0ull) continue;
            // one reduce-scatter over the wave, then one atomic instruction whose
            // lanes add consecutive fields of the entry's gradient record
            float tot = wave_reduce_fields<NGP>(g, lane);
            const int fld = field_of_lane<NGP>(lane);
            // fields 0 and 1 hold sum gx and sum gy (lanes 0 and NGP / 2):
            // d/du = -(2 cA sum gx + cB sum gy), d/dv = -(2 cC sum gy + cB sum gx)
            const float sgx = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, tot), 0));
            const float sgy =
                __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, tot), NGP / 2));
            if (fld == 0) tot = -(2.0f * r1.x * sgx + r1.y * sgy);
            if (fld == 1) tot = -(2.0f * r1.z * sgy + r1.y * sgx);
            if (fld < 5) tot *= LN2;
            if (lane < NGP && fld < NG && tot != 0.f)
                atomicAdd(grec + (size_t)sitem[s] * GS + fld, tot);
        }
        hi = lo;
    }
}


template <int TW, int TH>
hipError_t fwd_nf(const Params& P, const gftorf_frame* frames, const Workspace& w,
                  const gftorf_outputs& out, hipStream_t s) {
    const unsigned blocks = (unsigned)(P.F * P.n_tiles);
#define GFT_FWD(NF_)                                                                             \
    hipLaunchKernelGGL((k_composite_fwd<TW, TH, NF_>), dim3(blocks), dim3(TW * TH), 0, s, P, frames, \
                       w.ranges, w.tval, w.rec, w.conic, out, w.wcount)
    {
        ProfScope _p("k_composite_fwd", s);
        switch (P.nf) {
            case 1: GFT_FWD(1); break;
            case 2: GFT_FWD(2); break;
            case 3: GFT_FWD(3); break;
            default: GFT_FWD(4); break;
        }
    }
#undef GFT_FWD
    return hipGetLastError();
}

template <int TW, int TH, int WPT>
hipError_t bwd_wpt(const Params& P, const gftorf_frame* frames, const Workspace& w,
                   const gftorf_outputs& sv, const float* dr, const float* dq, const float* dd,
                   float* dbg, hipStream_t s) {
    const unsigned blocks = (unsigned)(P.F * P.n_tiles * WPT);
#define GFT_BWD(NF_)                                                                                  \
    hipLaunchKernelGGL((k_composite_bwd<TW, TH, NF_, WPT>), dim3(blocks), dim3(64), 0, s, P, frames,     \
                       w.ranges, w.tval, w.rec, w.conic, sv.T_final, sv.n_contrib, dr, dq, dd, w.grec, dbg)
    switch (P.nf) {
        case 1: GFT_BWD(1); break;
        case 2: GFT_BWD(2); break;
        case 3: GFT_BWD(3); break;
        default: GFT_BWD(4); break;
    }
#undef GFT_BWD
    return hipGetLastError();
}

// Waves per work item of the backward: one while the batch's tiles give at
// least kBwdWaves waves (several per SIMD, 1024 SIMDs), else 2 (4 below a
// quarter of that) sharing each tile's list, so a small batch still fills
// the chip.  Measured on one 640 x 480 frame (1200 tiles): 133 us with one
// wave per tile, 108 us with two, 107 us with four.
constexpr int64_t kBwdWaves = 4096;

template <int TW, int TH>
hipError_t bwd_nf(const Params& P, const gftorf_frame* frames, const Workspace& w,
                  const gftorf_outputs& sv, const float* dr, const float* dq, const float* dd,
                  float* dbg, hipStream_t s) {
    ProfScope _p("k_composite_bwd", s);
    const int64_t items = (int64_t)P.F * P.n_tiles;
    if constexpr (TW * TH >= 256) {
        if (items * 4 <= kBwdWaves) return bwd_wpt<TW, TH, 4>(P, frames, w, sv, dr, dq, dd, dbg, s);
        if (items < kBwdWaves) return bwd_wpt<TW, TH, 2>(P, frames, w, sv, dr, dq, dd, dbg, s);
    }
    return bwd_wpt<TW, TH, 1>(P, frames, w, sv, dr, dq, dd, dbg, s);
}

}  // namespace

hipError_t launch_composite_fwd(const Params& P, const gftorf_frame* frames, const Workspace& w,
                                const gftorf_outputs& out, hipStream_t s) {
    if (P.tw == 8 && P.th == 8) return fwd_nf<8, 8>(P, frames, w, out, s);
    if (P.tw == 32 && P.th == 8) return fwd_nf<32, 8>(P, frames, w, out, s);
    return fwd_nf<16, 16>(P, frames, w, out, s);
}

hipError_t launch_composite_bwd(const Params& P, const gftorf_frame* frames, const Workspace& w,
                                const gftorf_outputs& saved, const float* d_rgb,
                                const float* d_quad, const float* d_depth, float* d_bg,
                                hipStream_t s) {
    if (P.tw == 8 && P.th == 8) return bwd_nf<8, 8>(P, frames, w, saved, d_rgb, d_quad, d_depth, d_bg, s);
    if (P.tw == 32 && P.th == 8) return bwd_nf<32, 8>(P, frames, w, saved, d_rgb, d_quad, d_depth, d_bg, s);
    return bwd_nf<16, 16>(P, frames, w, saved, d_rgb, d_quad, d_depth, d_bg, s);
}

}  // namespace gft
