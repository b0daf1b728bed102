// Per-(frame, Gaussian) projection and binning (forward) and the chain rule
// from screen-space gradients back to the Gaussian parameters (backward).
//
// Forward (paper §3, "GS image formation model", applied per time frame):
// evaluate the trajectory at the frame time, transform to camera space, form
// the EWA 2D covariance, its conic, the pixel centre, the tile rectangle and
// the depth key; then the per-Gaussian C-ToF factors of Eq. 3/4: the range
// d_k to the optical centre, the falloff amplitude a_k = s r_k / d_k^2 and
// the phase psi_k = 4 pi f d_k / c.  Everything that decides the tile lists
// (rectangle, key) is evaluated in binary64 in one fixed operation order with
// FMA contraction off, so the lists are reproducible bit for bit.
//
// Layout: one thread per Gaussian; the thread loops over the frames so the
// 24 parameter floats of a Gaussian are read from HBM once per batch.
// Outputs are indexed by item i = frame * n + gaussian, so consecutive
// threads write consecutive records.
#include "common.h"
#include "sh.h"

namespace gft {

namespace {

struct Gauss {
    double x0[3], v[3], a[3], s[3], q0[4], om[3];
    double logit, rgb[3], albedo;
    bool finite;
};

__device__ __forceinline__ float ld(const float* p, int64_t i) { return p ? p[i] : 0.0f; }

__device__ Gauss load_gauss(const gftorf_gaussians& g, int64_t k) {
    Gauss r;
    const int64_t n = g.n;
    bool fin = true;
    auto rd = [&](const float* p, int64_t i) {
        float x = ld(p, i);
        fin = fin && isfinite(x);
        return (double)x;
    };
    for (int c = 0; c < 3; ++c) {
        r.x0[c] = rd(g.mean, c * n + k);
        r.v[c] = rd(g.vel, c * n + k);
        r.a[c] = rd(g.acc, c * n + k);
        r.s[c] = rd(g.scale, c * n + k);
        r.om[c] = rd(g.omega, c * n + k);
        r.rgb[c] = rd(g.rgb, c * n + k);
    }
    for (int c = 0; c < 4; ++c) r.q0[c] = rd(g.quat, c * n + k);
    r.logit = rd(g.opacity_logit, k);
    r.albedo = rd(g.albedo, k);
    r.finite = fin;
    return r;
}

struct Binned {
    double m[3];      // position at frame time
    double q[4];      // unnormalised quaternion at frame time
    double p[3];      // camera-space position
    double S00, S01, S11, det;
    double u, v;
    int xlo, xhi, ylo, yhi;
    bool valid;
};

// The pinned binary64 operation sequence.  Every statement is one IEEE
// operation evaluated left to right; contraction is off in this scope.
__device__ Binned bin(const Gauss& G, const gftorf_frame& fr, const Params& P,
                      const double* dl) {
#pragma clang fp contract(off)
    Binned b;
    const double t = (double)fr.time;
    const double tt = t * t;
    if (fr.t_hi > fr.t_lo) {
        // Eq. 7: the straight line between the positions at the two anchors
        const double tl = (double)fr.t_lo, th = (double)fr.t_hi;
        const double span = th - tl;
        const double w1 = (th - t) / span, w2 = (t - tl) / span;
        const double tl2 = tl * tl, th2 = th * th;
        for (int c = 0; c < 3; ++c) {
            const double ml = (G.x0[c] + G.v[c] * tl) + (0.5 * G.a[c]) * tl2;
            const double mh = (G.x0[c] + G.v[c] * th) + (0.5 * G.a[c]) * th2;
            b.m[c] = w1 * ml + w2 * mh;
        }
    } else {
        for (int c = 0; c < 3; ++c) b.m[c] = (G.x0[c] + G.v[c] * t) + (0.5 * G.a[c]) * tt;
    }
    if (dl)   // the deformation network's offset of this frame (§4), added last
        for (int c = 0; c < 3; ++c) b.m[c] = b.m[c] + dl[c];

    const double w0 = G.q0[0], qx0 = G.q0[1], qy0 = G.q0[2], qz0 = G.q0[3];
    const double ox = G.om[0], oy = G.om[1], oz = G.om[2];
    const double ht = 0.5 * t;
    const double dw = -((ox * qx0 + oy * qy0) + oz * qz0);
    const double dxq = w0 * ox + (oy * qz0 - oz * qy0);
    const double dyq = w0 * oy + (oz * qx0 - ox * qz0);
    const double dzq = w0 * oz + (ox * qy0 - oy * qx0);
    const double qw = w0 + ht * dw;
    const double qx = qx0 + ht * dxq;
    const double qy = qy0 + ht * dyq;
    const double qz = qz0 + ht * dzq;
    b.q[0] = qw; b.q[1] = qx; b.q[2] = qy; b.q[3] = qz;

    const double ww = qw * qw, xx = qx * qx, yy = qy * qy, zz = qz * qz;
    const double nq = ((ww + xx) + yy) + zz;
    double M[3][3];
    M[0][0] = ((ww + xx) - yy) - zz;
    M[0][1] = 2.0 * (qx * qy - qw * qz);
    M[0][2] = 2.0 * (qx * qz + qw * qy);
    M[1][0] = 2.0 * (qx * qy + qw * qz);
    M[1][1] = ((ww - xx) + yy) - zz;
    M[1][2] = 2.0 * (qy * qz - qw * qx);
    M[2][0] = 2.0 * (qx * qz - qw * qy);
    M[2][1] = 2.0 * (qy * qz + qw * qx);
    M[2][2] = ((ww - xx) - yy) + zz;

    double Wc[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Wc[i][j] = (double)fr.R[3 * i + j];
    for (int i = 0; i < 3; ++i)
        b.p[i] = ((Wc[i][0] * b.m[0] + Wc[i][1] * b.m[1]) + Wc[i][2] * b.m[2]) + (double)fr.t[i];
    const double px = b.p[0], py = b.p[1], pz = b.p[2];

    const double fx = (double)fr.fx, fy = (double)fr.fy;
    const double iz = 1.0 / pz;
    const double ja = fx * iz;
    const double jb = fy * iz;
    const double jc = -(((fx * px) * iz) * iz);
    const double jd = -(((fy * py) * iz) * iz);
    double L[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            L[i][j] = (Wc[i][0] * M[0][j] + Wc[i][1] * M[1][j]) + Wc[i][2] * M[2][j];
    double U0[3], U1[3];
    for (int j = 0; j < 3; ++j) {
        const double sc = G.s[j] / nq;
        U0[j] = (ja * L[0][j] + jc * L[2][j]) * sc;
        U1[j] = (jb * L[1][j] + jd * L[2][j]) * sc;
    }
    const double dil = (double)P.dilation;
    b.S00 = ((U0[0] * U0[0] + U0[1] * U0[1]) + U0[2] * U0[2]) + dil;
    b.S01 = (U0[0] * U1[0] + U0[1] * U1[1]) + U0[2] * U1[2];
    b.S11 = ((U1[0] * U1[0] + U1[1] * U1[1]) + U1[2] * U1[2]) + dil;
    b.det = b.S00 * b.S11 - b.S01 * b.S01;
    b.u = (fx * px) * iz + (double)fr.cx;
    b.v = (fy * py) * iz + (double)fr.cy;

    // tiles whose pixel-centre ranges [t T + 1/2, (t + 1) T - 1/2] meet the
    // axis-aligned box of the extent ellipse, half-widths k sqrt(S00), k sqrt(S11)
    double xlo, xhi, ylo, yhi;
    const double ext = (double)P.extent;
    if (ext > 0.0) {
        const double hx = ext * sqrt(b.S00);
        const double hy = ext * sqrt(b.S11);
        // the tile sides are powers of two (8, 16, 32), so multiplying by
        // their reciprocals is exact and equals the correctly rounded division
        const double itw = 1.0 / (double)P.tw, ith = 1.0 / (double)P.th;
        xlo = fmax(floor(((b.u - hx) + 0.5) * itw), 0.0);
        xhi = fmin(floor(((b.u + hx) - 0.5) * itw), (double)(P.ntx - 1));
        ylo = fmax(floor(((b.v - hy) + 0.5) * ith), 0.0);
        yhi = fmin(floor(((b.v + hy) - 0.5) * ith), (double)(P.nty - 1));
    } else {
        xlo = 0.0; xhi = (double)(P.ntx - 1);
        ylo = 0.0; yhi = (double)(P.nty - 1);
    }
    b.valid = G.finite && (pz > (double)P.near_z) && (b.det > 0.0) && (xlo <= xhi) && (ylo <= yhi);
    b.xlo = b.valid ? (int)xlo : 0;
    b.xhi = b.valid ? (int)xhi : -1;
    b.ylo = b.valid ? (int)ylo : 0;
    b.yhi = b.valid ? (int)yhi : -1;
    return b;
}

__device__ __forceinline__ void optical_centre(const gftorf_frame& fr, double c[3]) {
    for (int i = 0; i < 3; ++i)
        c[i] = -((double)fr.R[i] * fr.t[0] + (double)fr.R[3 + i] * fr.t[1] +
                 (double)fr.R[6 + i] * fr.t[2]);
}

template <bool SH>
__global__ void __launch_bounds__(256) k_preprocess(Params P, gftorf_gaussians g,
                                                    const gftorf_frame* __restrict__ frames,
                                                    float4* __restrict__ rec, float4* __restrict__ conic,
                                                    uint2* __restrict__ rect,
                                                    uint32_t* __restrict__ cnt, uint32_t* __restrict__ dkey,
                                                    uint32_t* __restrict__ dval, uint32_t* __restrict__ nf_block,
                                                    uint32_t* __restrict__ sclear, int64_t nclear) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Gauss G = load_gauss(g, k < P.n ? k : 0);
    // non-finite Gaussians per block (summed by the tile-range scan)
    const int bad = __syncthreads_count(k < P.n && !G.finite);
    if (threadIdx.x == 0) nf_block[blockIdx.x] = (uint32_t)bad;
    // the one-sweep depth sort's control words and digit counts start at 0
    if (sclear)
        for (int64_t i = k; i < nclear; i += (int64_t)gridDim.x * blockDim.x) sclear[i] = 0u;
    if (k >= P.n) return;
    const int RS4 = record_float4s(P.nf);
    const double o = 1.0 / (1.0 + exp(-G.logit));
    for (int f = 0; f < P.F; ++f) {
        const gftorf_frame& fr = frames[f];
        double dl[3];
        if (g.delta)
            for (int c = 0; c < 3; ++c) dl[c] = (double)g.delta[((int64_t)f * 3 + c) * P.n + k];
        const Binned b = bin(G, fr, P, g.delta ? dl : nullptr);
        const int64_t item = (int64_t)f * P.n + k;
        uint32_t c = 0;
        if (b.valid) c = (uint32_t)((b.xhi - b.xlo + 1) * (b.yhi - b.ylo + 1));
        cnt[item] = c;
        rect[item] = make_uint2((uint32_t)b.xlo | ((uint32_t)(b.xhi & 0xffff) << 16),
                                (uint32_t)b.ylo | ((uint32_t)(b.yhi & 0xffff) << 16));
        dkey[item] = b.valid ? __float_as_uint((float)b.p[2]) : kCulledKey;
        dval[item] = (uint32_t)item;
        if (!b.valid) continue;

        const double idet = 1.0 / b.det;
        const double A = b.S11 * idet, B = -b.S01 * idet, C = b.S00 * idet;
        const double L2E = 1.4426950408889634;
        const float u_hi = (float)b.u, v_hi = (float)b.v;
        float4* r = rec + item * RS4;
        r[0] = make_float4(u_hi, v_hi, (float)(b.u - (double)u_hi), (float)(b.v - (double)v_hi));
        conic[item] = make_float4((float)(-0.5 * L2E * A), (float)(-L2E * B), (float)(-0.5 * L2E * C),
                                  (float)o);
        double cc[3];
        optical_centre(fr, cc);
        const double e0 = b.m[0] - cc[0], e1 = b.m[1] - cc[1], e2 = b.m[2] - cc[2];
        const double d = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        float rgb[3] = {(float)G.rgb[0], (float)G.rgb[1], (float)G.rgb[2]};
        double albedo = G.albedo;
        if (SH) {
            // view-dependent colour / reflectivity at the viewing direction
            const float id = (float)(1.0 / d);
            float Y[kMaxSH];
            sh_basis((float)e0 * id, (float)e1 * id, (float)e2 * id, g.sh_degree, Y);
            const int K = sh_count(g.sh_degree);
            const int64_t n = P.n;
            // degree 3 (all kMaxSH coefficients present): unguarded loads, so
            // they issue together instead of one guarded load at a time
            const bool full = K == kMaxSH;
            if (g.sh_rgb)
                for (int c = 0; c < 3; ++c) {
                    float acc = 0.5f;
                    if (full) {
#pragma unroll
                        for (int l = 0; l < kMaxSH; ++l) acc += Y[l] * g.sh_rgb[((int64_t)l * 3 + c) * n + k];
                    } else {
#pragma unroll
                        for (int l = 0; l < kMaxSH; ++l)
                            if (l < K) acc += Y[l] * g.sh_rgb[((int64_t)l * 3 + c) * n + k];
                    }
                    rgb[c] = fmaxf(acc, 0.0f);
                }
            if (g.sh_albedo) {
                float acc = 0.5f;
                if (full) {
#pragma unroll
                    for (int l = 0; l < kMaxSH; ++l) acc += Y[l] * g.sh_albedo[(int64_t)l * n + k];
                } else {
#pragma unroll
                    for (int l = 0; l < kMaxSH; ++l)
                        if (l < K) acc += Y[l] * g.sh_albedo[(int64_t)l * n + k];
                }
                albedo = (double)fmaxf(acc, 0.0f);
            }
        }
        r[1] = make_float4(rgb[0], rgb[1], rgb[2], (float)d);
        const double amp = (double)P.s_int * albedo / (d * d);
        float ph[2 * GFTORF_MAX_FREQ];
        for (int fi = 0; fi < P.nf; ++fi) {
            // psi = 4 pi f d / c = 2 pi * cycles; the fractional cycle is taken in
            // binary64 (psi reaches tens of radians), then one float32 sine and
            // cosine of 2 pi * frac (the hardware instructions take revolutions)
            double cyc = 2.0 * P.freq[fi] * d / kSpeedOfLight;
            cyc -= floor(cyc);
            const float cf = (float)cyc;
            const float sn = __builtin_amdgcn_sinf(cf), cs = __builtin_amdgcn_cosf(cf);
            ph[2 * fi] = (float)amp * sn;
            ph[2 * fi + 1] = (float)amp * cs;
        }
        for (int fi = P.nf; fi < 2 * ((P.nf + 1) / 2); ++fi) {
            ph[2 * fi] = 0.f;
            ph[2 * fi + 1] = 0.f;
        }
        for (int j = 0; j < (P.nf + 1) / 2; ++j)
            r[2 + j] = make_float4(ph[4 * j], ph[4 * j + 1], ph[4 * j + 2], ph[4 * j + 3]);
    }
}

// ---------------------------------------------------------------------------
// Backward: screen-space gradient records -> parameter gradients.
//
// FP32 throughout (the gradients carry no binning decision).  One thread per
// (Gaussian, frame) item: the GS lanes of a group are the frames of one
// Gaussian (frames f0, f0 + GS, ... when there are more than GS), and the
// per-frame contributions are summed inside the group with DPP in a fixed
// order, so the result is deterministic and needs no atomics.  The 2-D
// covariance gradient comes from the stored conic Q (computed in binary64):
// dL/dSigma' = -Q (dL/dQ) Q, with no determinant to lose precision in.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true));
}

// Sum over the GS consecutive lanes of a group (GS a power of two <= 64).
template <int GS>
__device__ __forceinline__ float group_sum(float v) {
    if constexpr (GS >= 2) v += dpp_f<0xb1>(v);    // quad_perm [1,0,3,2]
    if constexpr (GS >= 4) v += dpp_f<0x4e>(v);    // quad_perm [2,3,0,1]
    if constexpr (GS >= 8) v += dpp_f<0x141>(v);   // row_half_mirror: the other quad of the 8
    if constexpr (GS >= 16) v += dpp_f<0x140>(v);  // row_mirror: the other 8 of the row
    if constexpr (GS >= 32) v += __shfl_xor(v, 16, 64);
    if constexpr (GS >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

constexpr int kNG = 25;   // gradient values per Gaussian

template <int GS, bool SH>
__global__ void __launch_bounds__(256) k_preprocess_bwd(Params P, gftorf_gaussians g,
                                                        const gftorf_frame* __restrict__ frames,
                                                        const uint32_t* __restrict__ cnt,
                                                        const float4* __restrict__ conic,
                                                        const float* __restrict__ grec,
                                                        gftorf_gaussians_grad out) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = tid / GS;
    const int f0 = (int)(tid - k * GS);
    const int64_t n = P.n;
    const bool have = k < n;
    // acc: mean 0-2, vel 3-5, acc 6-8, scale 9-11, quat 12-15, omega 16-18,
    //      rgb 19-21, opacity logit 22, albedo 23 (24 unused)
    float acc[kNG];
#pragma unroll
    for (int i = 0; i < kNG; ++i) acc[i] = 0.f;
    // spherical-harmonic coefficient gradients: colour [l][c] at 3 l + c,
    // reflectivity [l] at 3 kMaxSH + l.  With fewer than 64 lanes per
    // Gaussian every lane has at most one frame (GS is the smallest power of
    // two >= F), so a lane keeps only that frame's basis values and upstream
    // factors, and the products are formed and summed over the group one at
    // a time after the frame loop; otherwise each lane accumulates them over
    // its frames.
    constexpr bool kOneFrame = GS < 64;
    constexpr int NSH = SH && !kOneFrame ? 4 * kMaxSH : 1;
    float ash[NSH];
#pragma unroll
    for (int i = 0; i < NSH; ++i) ash[i] = 0.f;
    constexpr int NY = SH && kOneFrame ? kMaxSH : 1;
    float ysv[NY], tcv[3] = {0.f, 0.f, 0.f}, trv = 0.f;
#pragma unroll
    for (int l = 0; l < NY; ++l) ysv[l] = 0.f;
    const int K = sh_count(g.sh_degree);
    if (have) {
        auto ld = [&](const float* p, int64_t i) { return p ? p[i] : 0.0f; };
        float x0[3], vv[3], aa[3], sc[3], q0[4], om[3];
        for (int c = 0; c < 3; ++c) {
            x0[c] = ld(g.mean, c * n + k);
            vv[c] = ld(g.vel, c * n + k);
            aa[c] = ld(g.acc, c * n + k);
            sc[c] = ld(g.scale, c * n + k);
            om[c] = ld(g.omega, c * n + k);
        }
        for (int c = 0; c < 4; ++c) q0[c] = ld(g.quat, c * n + k);
        const float albedo = ld(g.albedo, k);
        // SH coefficients of this Gaussian, loaded once; at degree 3 (all
        // kMaxSH present) unguarded, so the loads issue together
        float shr[SH ? 3 * kMaxSH : 1], sha[SH ? kMaxSH : 1];
        if constexpr (SH) {
            const bool full = K == kMaxSH;
#pragma unroll
            for (int i = 0; i < 3 * kMaxSH; ++i) shr[i] = 0.f;
#pragma unroll
            for (int l = 0; l < kMaxSH; ++l) sha[l] = 0.f;
            if (g.sh_rgb) {
                if (full) {
#pragma unroll
                    for (int i = 0; i < 3 * kMaxSH; ++i) shr[i] = g.sh_rgb[(int64_t)i * n + k];
                } else {
#pragma unroll
                    for (int i = 0; i < 3 * kMaxSH; ++i)
                        if (i < 3 * K) shr[i] = g.sh_rgb[(int64_t)i * n + k];
                }
            }
            if (g.sh_albedo) {
                if (full) {
#pragma unroll
                    for (int l = 0; l < kMaxSH; ++l) sha[l] = g.sh_albedo[(int64_t)l * n + k];
                } else {
#pragma unroll
                    for (int l = 0; l < kMaxSH; ++l)
                        if (l < K) sha[l] = g.sh_albedo[(int64_t)l * n + k];
                }
            }
        }
        auto kr = [&](int l, int c) {
            if constexpr (SH) return shr[3 * l + c];
            else return 0.f;
        };
        auto ka = [&](int l) {
            if constexpr (SH) return sha[l];
            else return 0.f;
        };
        const int GF = grad_floats(P.nf);
        const float L2E = 1.4426950408889634f;
        for (int f = f0; f < P.F; f += GS) {
            const int64_t item = (int64_t)f * n + k;
            if (cnt[item] == 0) {
                if (out.delta)
                    for (int c = 0; c < 3; ++c) out.delta[((int64_t)f * 3 + c) * n + k] = 0.f;
                continue;
            }
            const gftorf_frame& fr = frames[f];
            const float* gr = grec + item * GF;
            const float4 r1 = conic[item];
            const float t = fr.time;

            // trajectory and rotation at the frame time (as in the forward): the
            // centre is cx0 x0 + cv v + ca a, with Eq. 7's weights when the
            // frame interpolates between two anchors
            float cx0 = 1.0f, cv = t, ca = 0.5f * t * t;
            if (fr.t_hi > fr.t_lo) {
                const float span = fr.t_hi - fr.t_lo;
                const float w1 = (fr.t_hi - t) / span, w2 = (t - fr.t_lo) / span;
                cx0 = w1 + w2;
                cv = w1 * fr.t_lo + w2 * fr.t_hi;
                ca = 0.5f * (w1 * fr.t_lo * fr.t_lo + w2 * fr.t_hi * fr.t_hi);
            }
            float m[3];
            for (int c = 0; c < 3; ++c) m[c] = cx0 * x0[c] + cv * vv[c] + ca * aa[c];
            if (g.delta)
                for (int c = 0; c < 3; ++c) m[c] += g.delta[((int64_t)f * 3 + c) * n + k];
            const float ht = 0.5f * t;
            const float qw = q0[0] - ht * (om[0] * q0[1] + om[1] * q0[2] + om[2] * q0[3]);
            const float qx = q0[1] + ht * (q0[0] * om[0] + om[1] * q0[3] - om[2] * q0[2]);
            const float qy = q0[2] + ht * (q0[0] * om[1] + om[2] * q0[1] - om[0] * q0[3]);
            const float qz = q0[3] + ht * (q0[0] * om[2] + om[0] * q0[2] - om[1] * q0[1]);
            float Wc[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Wc[i][j] = fr.R[3 * i + j];
            float p[3];
            for (int i = 0; i < 3; ++i) p[i] = Wc[i][0] * m[0] + Wc[i][1] * m[1] + Wc[i][2] * m[2] + fr.t[i];

            // colour (flat), opacity (o from the record)
            if (!SH || !g.sh_rgb)
                for (int c = 0; c < 3; ++c) acc[19 + c] += gr[6 + c];
            acc[22] += gr[5] * r1.w * (1.0f - r1.w);

            // range d: depth channel + C-ToF amplitude and phase
            float e[3];
            for (int i = 0; i < 3; ++i)
                e[i] = m[i] + (Wc[0][i] * fr.t[0] + Wc[1][i] * fr.t[1] + Wc[2][i] * fr.t[2]);
            const float d2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
            const float d = sqrtf(d2);
            const float id = 1.0f / d;
            // view-dependent colour / reflectivity: basis at the viewing direction
            float Y[SH ? kMaxSH : 1], act_c[3] = {1.f, 1.f, 1.f}, r_item = albedo, act_r = 1.f;
            if constexpr (SH) {
                sh_basis(e[0] * id, e[1] * id, e[2] * id, g.sh_degree, Y);
                float cs3[3] = {0.5f, 0.5f, 0.5f}, rs = 0.5f;
#pragma unroll
                for (int l = 0; l < kMaxSH; ++l) {
                    for (int c = 0; c < 3; ++c) cs3[c] += Y[l] * kr(l, c);
                    rs += Y[l] * ka(l);
                }
                for (int c = 0; c < 3; ++c) act_c[c] = cs3[c] > 0.f ? 1.f : 0.f;   // clamp at 0
                if (g.sh_albedo) {
                    r_item = fmaxf(rs, 0.f);
                    act_r = rs > 0.f ? 1.f : 0.f;
                }
            }
            const float amp = P.s_int * r_item / d2;
            float gd = gr[9];
            float galb = 0.f;   // dL/dr of this item
            for (int fi = 0; fi < P.nf; ++fi) {
                float cyc = (float)(2.0 * P.freq[fi] / kSpeedOfLight) * d;
                cyc -= floorf(cyc);
                const float sn = __builtin_amdgcn_sinf(cyc), cs = __builtin_amdgcn_cosf(cyc);   // of 2 pi cyc
                const float gas = gr[10 + 2 * fi], gac = gr[11 + 2 * fi];
                const float dpsi = (float)(4.0 * M_PI * P.freq[fi] / kSpeedOfLight);
                // a sin psi, a cos psi with a = s r / d^2, psi = 4 pi f d / c
                gd += gas * (-2.0f * amp * id * sn + amp * cs * dpsi) +
                      gac * (-2.0f * amp * id * cs - amp * sn * dpsi);
                galb += (gas * sn + gac * cs) * P.s_int / d2;
            }
            float gm[3];
            for (int c = 0; c < 3; ++c) gm[c] = gd * e[c] * id;
            if (SH && g.sh_albedo) {
                // through r = max(0, 1/2 + sum Y k) and the viewing direction
            } else {
                acc[23] += galb;
            }
            if constexpr (SH) {
                float w[kMaxSH];   // dL/dY_l
#pragma unroll
                for (int l = 0; l < kMaxSH; ++l) {
                    w[l] = 0.f;
                    if (g.sh_rgb)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const float tc = gr[6 + c] * act_c[c];
                            if constexpr (!kOneFrame) ash[3 * l + c] += Y[l] * tc;
                            w[l] += kr(l, c) * tc;
                        }
                    if (g.sh_albedo) {
                        const float tr = galb * act_r;
                        if constexpr (!kOneFrame) ash[3 * kMaxSH + l] += Y[l] * tr;
                        w[l] += ka(l) * tr;
                    }
                }
                if constexpr (kOneFrame) {
#pragma unroll
                    for (int l = 0; l < kMaxSH; ++l) ysv[l] = Y[l];
                    if (g.sh_rgb)
                        for (int c = 0; c < 3; ++c) tcv[c] = gr[6 + c] * act_c[c];
                    if (g.sh_albedo) trv = galb * act_r;
                }
                // direction = e / d: dL/de = (I - dir dir^T) dL/ddir / d
                float gdir[3];
                sh_basis_grad(e[0] * id, e[1] * id, e[2] * id, g.sh_degree, w, gdir[0], gdir[1], gdir[2]);
                const float dot = (gdir[0] * e[0] + gdir[1] * e[1] + gdir[2] * e[2]) * id;
                for (int c = 0; c < 3; ++c) gm[c] += (gdir[c] - dot * e[c] * id) * id;
            }

            // conic gradient -> 2-D covariance gradient: -Q (dL/dQ) Q
            const float A = r1.x * (-2.0f / L2E), B = r1.y * (-1.0f / L2E), C = r1.z * (-2.0f / L2E);
            const float gA = -0.5f * L2E * gr[2], gB = -L2E * gr[3], gC = -0.5f * L2E * gr[4];
            const float h00 = A * gA + B * (0.5f * gB), h01 = A * (0.5f * gB) + B * gC;
            const float h10 = B * gA + C * (0.5f * gB), h11 = B * (0.5f * gB) + C * gC;
            const float Gp[2][2] = {{-(h00 * A + h01 * B), -(h00 * B + h01 * C)},
                                    {-(h00 * B + h01 * C), -(h10 * B + h11 * C)}};

            // T = J W and Sigma3 = R S^2 R^T
            const float px = p[0], py = p[1], pz = p[2];
            const float fx = fr.fx, fy = fr.fy;
            const float iz = 1.0f / pz, iz2 = iz * iz;
            const float J[2][3] = {{fx * iz, 0.0f, -fx * px * iz2}, {0.0f, fy * iz, -fy * py * iz2}};
            float T[2][3];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j) T[i][j] = J[i][0] * Wc[0][j] + J[i][1] * Wc[1][j] + J[i][2] * Wc[2][j];
            const float nq = qw * qw + qx * qx + qy * qy + qz * qz;
            const float M[3][3] = {{qw * qw + qx * qx - qy * qy - qz * qz, 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
                                   {2 * (qx * qy + qw * qz), qw * qw - qx * qx + qy * qy - qz * qz, 2 * (qy * qz - qw * qx)},
                                   {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), qw * qw - qx * qx - qy * qy + qz * qz}};
            const float inq = 1.0f / nq;
            float R[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) R[i][j] = M[i][j] * inq;
            const float s2[3] = {sc[0] * sc[0], sc[1] * sc[1], sc[2] * sc[2]};
            float Sig[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    Sig[i][j] = R[i][0] * s2[0] * R[j][0] + R[i][1] * s2[1] * R[j][1] + R[i][2] * s2[2] * R[j][2];

            // dL/dSigma3 = T^T G' T ; dL/dT = 2 G' T Sigma3 ; dL/dJ = dL/dT W^T
            float GT[2][3];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j) GT[i][j] = Gp[i][0] * T[0][j] + Gp[i][1] * T[1][j];
            float G3[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) G3[i][j] = T[0][i] * GT[0][j] + T[1][i] * GT[1][j];
            float gT[2][3];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j)
                    gT[i][j] = 2.0f * (GT[i][0] * Sig[0][j] + GT[i][1] * Sig[1][j] + GT[i][2] * Sig[2][j]);
            float gJ[2][3];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j)
                    gJ[i][j] = gT[i][0] * Wc[j][0] + gT[i][1] * Wc[j][1] + gT[i][2] * Wc[j][2];
            // camera-space position: J and the pixel centre u = fx px / pz + cx
            const float gu = gr[0], gv = gr[1];
            float gp[3];
            gp[0] = gJ[0][2] * (-fx * iz2) + gu * fx * iz;
            gp[1] = gJ[1][2] * (-fy * iz2) + gv * fy * iz;
            gp[2] = gJ[0][0] * (-fx * iz2) + gJ[0][2] * (2.0f * fx * px * iz2 * iz) + gJ[1][1] * (-fy * iz2) +
                    gJ[1][2] * (2.0f * fy * py * iz2 * iz) - gu * fx * px * iz2 - gv * fy * py * iz2;
            for (int c = 0; c < 3; ++c) gm[c] += Wc[0][c] * gp[0] + Wc[1][c] * gp[1] + Wc[2][c] * gp[2];

            // Sigma3 -> scale: dL/ds_k = 2 s_k (R^T G3 R)_kk ; rotation: dL/dR = 2 G3 R S^2
            for (int kk = 0; kk < 3; ++kk) {
                float a3 = 0.f;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) a3 += R[i][kk] * G3[i][j] * R[j][kk];
                acc[9 + kk] += 2.0f * sc[kk] * a3;
            }
            float gn = 0.f, gM[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    const float gR = 2.0f * (G3[i][0] * R[0][j] + G3[i][1] * R[1][j] + G3[i][2] * R[2][j]) * s2[j];
                    gn -= gR * M[i][j];
                    gM[i][j] = gR * inq;
                }
            gn *= inq * inq;   // R = M / n
            float gq[4];
            gq[0] = 2 * (qw * gM[0][0] - qz * gM[0][1] + qy * gM[0][2] + qz * gM[1][0] + qw * gM[1][1] -
                         qx * gM[1][2] - qy * gM[2][0] + qx * gM[2][1] + qw * gM[2][2]) + 2 * qw * gn;
            gq[1] = 2 * (qx * gM[0][0] + qy * gM[0][1] + qz * gM[0][2] + qy * gM[1][0] - qx * gM[1][1] -
                         qw * gM[1][2] + qz * gM[2][0] + qw * gM[2][1] - qx * gM[2][2]) + 2 * qx * gn;
            gq[2] = 2 * (-qy * gM[0][0] + qx * gM[0][1] + qw * gM[0][2] + qx * gM[1][0] + qy * gM[1][1] +
                         qz * gM[1][2] - qw * gM[2][0] + qz * gM[2][1] - qy * gM[2][2]) + 2 * qy * gn;
            gq[3] = 2 * (-qz * gM[0][0] - qw * gM[0][1] + qx * gM[0][2] + qw * gM[1][0] - qz * gM[1][1] +
                         qy * gM[1][2] + qx * gM[2][0] + qy * gM[2][1] + qz * gM[2][2]) + 2 * qz * gn;
            // q = q0 + (t/2) D(omega) q0 with D the left product by (0, omega)
            acc[12] += gq[0] + ht * (gq[1] * om[0] + gq[2] * om[1] + gq[3] * om[2]);
            acc[13] += gq[1] + ht * (-gq[0] * om[0] + gq[2] * om[2] - gq[3] * om[1]);
            acc[14] += gq[2] + ht * (-gq[0] * om[1] - gq[1] * om[2] + gq[3] * om[0]);
            acc[15] += gq[3] + ht * (-gq[0] * om[2] + gq[1] * om[1] - gq[2] * om[0]);
            acc[16] += ht * (-gq[0] * q0[1] + gq[1] * q0[0] - gq[2] * q0[3] + gq[3] * q0[2]);
            acc[17] += ht * (-gq[0] * q0[2] + gq[1] * q0[3] + gq[2] * q0[0] - gq[3] * q0[1]);
            acc[18] += ht * (-gq[0] * q0[3] - gq[1] * q0[2] + gq[2] * q0[1] + gq[3] * q0[0]);

            // per-frame centre (the deformation offset's gradient) and trajectory
            if (out.delta)
                for (int c = 0; c < 3; ++c) out.delta[((int64_t)f * 3 + c) * n + k] = gm[c];
            for (int c = 0; c < 3; ++c) {
                acc[c] += gm[c] * cx0;
                acc[3 + c] += gm[c] * cv;
                acc[6 + c] += gm[c] * ca;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kNG - 1; ++i) acc[i] = group_sum<GS>(acc[i]);
    if constexpr (SH && kOneFrame) {
        // the group's sum of each product, stored by the group's first lane
        const bool store = have && f0 == 0;
#pragma unroll
        for (int l = 0; l < kMaxSH; ++l) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float v = group_sum<GS>(ysv[l] * tcv[c]);
                if (store && l < K && out.sh_rgb) out.sh_rgb[((int64_t)l * 3 + c) * n + k] = v;
            }
            const float v = group_sum<GS>(ysv[l] * trv);
            if (store && l < K && out.sh_albedo) out.sh_albedo[(int64_t)l * n + k] = v;
        }
    }
    if constexpr (SH && !kOneFrame) {
#pragma unroll
        for (int i = 0; i < NSH; ++i) ash[i] = group_sum<GS>(ash[i]);
    }
    if (!have || f0 != 0) return;
    if constexpr (SH && !kOneFrame) {
#pragma unroll
        for (int l = 0; l < kMaxSH; ++l) {
            if (l >= K) continue;
            if (out.sh_rgb)
                for (int c = 0; c < 3; ++c) out.sh_rgb[((int64_t)l * 3 + c) * n + k] = ash[3 * l + c];
            if (out.sh_albedo) out.sh_albedo[(int64_t)l * n + k] = ash[3 * kMaxSH + l];
        }
    }
    for (int c = 0; c < 3; ++c) {
        if (out.mean) out.mean[c * n + k] = acc[c];
        if (out.vel) out.vel[c * n + k] = acc[3 + c];
        if (out.acc) out.acc[c * n + k] = acc[6 + c];
        if (out.scale) out.scale[c * n + k] = acc[9 + c];
        if (out.omega) out.omega[c * n + k] = acc[16 + c];
        if (out.rgb) out.rgb[c * n + k] = acc[19 + c];
    }
    for (int c = 0; c < 4; ++c)
        if (out.quat) out.quat[c * n + k] = acc[12 + c];
    if (out.opacity_logit) out.opacity_logit[k] = acc[22];
    if (out.albedo) out.albedo[k] = acc[23];
}

}  // namespace

void launch_preprocess(const Params& P, const gftorf_gaussians& g, const gftorf_frame* frames,
                       const Workspace& w, hipStream_t s) {
    const int threads = 256;
    const unsigned blocks = (unsigned)((P.n + threads - 1) / threads);
    if (blocks == 0) return;
    uint32_t* sclear = one_sweep_sort(P, w) ? w.sctl : nullptr;
    const int64_t nclear = kSortCtlWords + (int64_t)P.F * kSortPasses * kSortBuckets;
    { ProfScope _p("k_preprocess", s);
    if (g.sh_rgb || g.sh_albedo)
        hipLaunchKernelGGL(k_preprocess<true>, dim3(blocks), dim3(threads), 0, s, P, g, frames, w.rec,
                           w.conic, w.drect[0], w.cnt, w.dkey[0], w.dval[0], w.nf_block, sclear, nclear);
    else
        hipLaunchKernelGGL(k_preprocess<false>, dim3(blocks), dim3(threads), 0, s, P, g, frames, w.rec,
                           w.conic, w.drect[0], w.cnt, w.dkey[0], w.dval[0], w.nf_block, sclear, nclear);
    }
}

void launch_preprocess_bwd(const Params& P, const gftorf_gaussians& g, const gftorf_frame* frames,
                           const Workspace& w, const gftorf_gaussians_grad& grad, hipStream_t s) {
    // GS lanes per Gaussian: the smallest power of two >= frames, at most 64
    int gs = 1;
    while (gs < P.F && gs < 64) gs *= 2;
    const int threads = 256;
    const unsigned blocks = (unsigned)((P.n * gs + threads - 1) / threads);
    if (blocks == 0) return;
    ProfScope _p("k_preprocess_bwd", s);
    const bool sh = g.sh_rgb || g.sh_albedo;
#define GFT_PRE_BWD(G)                                                                                      \
    if (sh)                                                                                                  \
        hipLaunchKernelGGL((k_preprocess_bwd<G, true>), dim3(blocks), dim3(threads), 0, s, P, g, frames,      \
                           w.cnt, w.conic, w.grec, grad);                                            \
    else                                                                                                     \
        hipLaunchKernelGGL((k_preprocess_bwd<G, false>), dim3(blocks), dim3(threads), 0, s, P, g, frames,     \
                           w.cnt, w.conic, w.grec, grad)
    switch (gs) {
        case 1: GFT_PRE_BWD(1); break;
        case 2: GFT_PRE_BWD(2); break;
        case 4: GFT_PRE_BWD(4); break;
        case 8: GFT_PRE_BWD(8); break;
        case 16: GFT_PRE_BWD(16); break;
        case 32: GFT_PRE_BWD(32); break;
        default: GFT_PRE_BWD(64); break;
    }
#undef GFT_PRE_BWD
}

}  // namespace gft
