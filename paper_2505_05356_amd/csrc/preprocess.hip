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
// 24 parameter floats of a Gaussian are read from HBM once per batch; frame
// descriptors are wave-uniform (scalar loads).  Outputs are indexed by item
// i = frame * n + gaussian, so consecutive threads write consecutive records.
#include "common.h"

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
__device__ Binned bin(const Gauss& G, const gftorf_frame& fr, const Params& P) {
#pragma clang fp contract(off)
    Binned b;
    const double t = (double)fr.time;
    const double tt = t * t;
    for (int c = 0; c < 3; ++c) b.m[c] = (G.x0[c] + G.v[c] * t) + (0.5 * G.a[c]) * tt;

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
    const double mid = 0.5 * (b.S00 + b.S11);
    double disc = mid * mid - b.det;
    disc = disc > 0.0 ? disc : 0.0;
    const double lam = mid + sqrt(disc);
    b.u = (fx * px) * iz + (double)fr.cx;
    b.v = (fy * py) * iz + (double)fr.cy;

    double xlo, xhi, ylo, yhi;
    const double ext = (double)P.extent;
    if (ext > 0.0) {
        const double r = ceil(ext * sqrt(lam));
        const double tw = (double)P.tw, th = (double)P.th;
        xlo = fmax(floor((b.u - r) / tw), 0.0);
        xhi = fmin(floor((b.u + r) / tw), (double)(P.ntx - 1));
        ylo = fmax(floor((b.v - r) / th), 0.0);
        yhi = fmin(floor((b.v + r) / th), (double)(P.nty - 1));
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

__global__ void __launch_bounds__(256) k_preprocess(Params P, gftorf_gaussians g,
                                                    const gftorf_frame* __restrict__ frames,
                                                    float4* __restrict__ rec, uint2* __restrict__ rect,
                                                    uint32_t* __restrict__ cnt, uint32_t* __restrict__ dkey,
                                                    uint32_t* __restrict__ dval, Status* status) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    const Gauss G = load_gauss(g, k);
    if (!G.finite) atomicAdd(&status->nonfinite, 1u);
    const int RS4 = record_float4s(P.nf);
    const double o = 1.0 / (1.0 + exp(-G.logit));
    for (int f = 0; f < P.F; ++f) {
        const gftorf_frame& fr = frames[f];
        const Binned b = bin(G, fr, P);
        const int64_t item = (int64_t)f * P.n + k;
        uint32_t c = 0;
        if (b.valid) c = (uint32_t)((b.xhi - b.xlo + 1) * (b.yhi - b.ylo + 1));
        cnt[item] = c;
        rect[item] = make_uint2((uint32_t)b.xlo | ((uint32_t)(b.xhi & 0xffff) << 16),
                                (uint32_t)b.ylo | ((uint32_t)(b.yhi & 0xffff) << 16));
        dkey[item] = b.valid ? __float_as_uint((float)b.p[2]) : 0xffffffffu;
        dval[item] = (uint32_t)item;
        if (!b.valid) continue;

        const double idet = 1.0 / b.det;
        const double A = b.S11 * idet, B = -b.S01 * idet, C = b.S00 * idet;
        const double L2E = 1.4426950408889634;
        const float u_hi = (float)b.u, v_hi = (float)b.v;
        float4* r = rec + item * RS4;
        r[0] = make_float4(u_hi, v_hi, (float)(b.u - (double)u_hi), (float)(b.v - (double)v_hi));
        r[1] = make_float4((float)(-0.5 * L2E * A), (float)(-L2E * B), (float)(-0.5 * L2E * C),
                           (float)o);
        double cc[3];
        optical_centre(fr, cc);
        const double e0 = b.m[0] - cc[0], e1 = b.m[1] - cc[1], e2 = b.m[2] - cc[2];
        const double d = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        r[2] = make_float4((float)G.rgb[0], (float)G.rgb[1], (float)G.rgb[2], (float)d);
        const double amp = (double)P.s_int * G.albedo / (d * d);
        float ph[2 * GFTORF_MAX_FREQ];
        for (int fi = 0; fi < P.nf; ++fi) {
            // psi = 4 pi f d / c = 2 pi * cycles; reduce to the fractional cycle first
            double cyc = 2.0 * P.freq[fi] * d / kSpeedOfLight;
            cyc -= floor(cyc);
            double sn, cs;
            sincos(2.0 * M_PI * cyc, &sn, &cs);
            ph[2 * fi] = (float)(amp * sn);
            ph[2 * fi + 1] = (float)(amp * cs);
        }
        for (int fi = P.nf; fi < 2 * ((P.nf + 1) / 2); ++fi) {
            ph[2 * fi] = 0.f;
            ph[2 * fi + 1] = 0.f;
        }
        for (int j = 0; j < (P.nf + 1) / 2; ++j)
            r[3 + j] = make_float4(ph[4 * j], ph[4 * j + 1], ph[4 * j + 2], ph[4 * j + 3]);
    }
}

// ---------------------------------------------------------------------------
// Backward: screen-space gradient records -> parameter gradients.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_preprocess_bwd(Params P, gftorf_gaussians g,
                                                        const gftorf_frame* __restrict__ frames,
                                                        const uint32_t* __restrict__ cnt,
                                                        const float* __restrict__ grec,
                                                        gftorf_gaussians_grad out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    const Gauss G = load_gauss(g, k);
    const int GS = grad_floats(P.nf);
    double gx0[3] = {0, 0, 0}, gv[3] = {0, 0, 0}, ga[3] = {0, 0, 0}, gs[3] = {0, 0, 0};
    double gq0[4] = {0, 0, 0, 0}, gom[3] = {0, 0, 0}, grgb[3] = {0, 0, 0};
    double glogit = 0, galb = 0;
    const double o = 1.0 / (1.0 + exp(-G.logit));
    const double L2E = 1.4426950408889634;

    for (int f = 0; f < P.F; ++f) {
        const int64_t item = (int64_t)f * P.n + k;
        if (cnt[item] == 0) continue;
        const gftorf_frame& fr = frames[f];
        const float* gr = grec + item * GS;
        const double gu = gr[0], gvv = gr[1];
        const double gA = -0.5 * L2E * gr[2], gB = -L2E * gr[3], gC = -0.5 * L2E * gr[4];
        const double go = gr[5];
        const double gd_direct = gr[9];
        const Binned b = bin(G, fr, P);
        const double t = (double)fr.time;

        // colour, opacity
        for (int c = 0; c < 3; ++c) grgb[c] += gr[6 + c];
        glogit += go * o * (1.0 - o);

        // ---- range d: depth channel + C-ToF amplitude and phase -----------
        double cc[3];
        optical_centre(fr, cc);
        const double e[3] = {b.m[0] - cc[0], b.m[1] - cc[1], b.m[2] - cc[2]};
        const double d = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        const double amp = (double)P.s_int * G.albedo / (d * d);
        double gd = gd_direct;
        for (int fi = 0; fi < P.nf; ++fi) {
            double cyc = 2.0 * P.freq[fi] * d / kSpeedOfLight;
            cyc -= floor(cyc);
            double sn, cs;
            sincos(2.0 * M_PI * cyc, &sn, &cs);
            const double gas = gr[10 + 2 * fi], gac = gr[11 + 2 * fi];
            const double dpsi = 4.0 * M_PI * P.freq[fi] / kSpeedOfLight;
            // a sin psi, a cos psi with a = s r / d^2, psi = 4 pi f d / c
            gd += gas * (-2.0 * amp / d * sn + amp * cs * dpsi) +
                  gac * (-2.0 * amp / d * cs - amp * sn * dpsi);
            galb += (gas * sn + gac * cs) * (double)P.s_int / (d * d);
        }
        double gm[3];
        for (int c = 0; c < 3; ++c) gm[c] = gd * e[c] / d;

        // ---- conic -> 2D covariance ---------------------------------------
        const double a = b.S00, bb = b.S01, c2 = b.S11;
        const double id2 = 1.0 / (b.det * b.det);
        const double g_a = (gA * (-c2 * c2) + gB * (bb * c2) + gC * (-bb * bb)) * id2;
        const double g_b = (gA * (2.0 * bb * c2) + gB * (-(a * c2 + bb * bb)) + gC * (2.0 * a * bb)) * id2;
        const double g_c = (gA * (-bb * bb) + gB * (a * bb) + gC * (-a * a)) * id2;
        const double Gp[2][2] = {{g_a, 0.5 * g_b}, {0.5 * g_b, g_c}};

        // ---- rebuild T = J W and Sigma3 = Rq S^2 Rq^T ----------------------
        const double px = b.p[0], py = b.p[1], pz = b.p[2];
        const double fx = fr.fx, fy = fr.fy;
        const double iz = 1.0 / pz, iz2 = iz * iz;
        double Wc[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Wc[i][j] = fr.R[3 * i + j];
        const double J[2][3] = {{fx * iz, 0.0, -fx * px * iz2}, {0.0, fy * iz, -fy * py * iz2}};
        double T[2][3];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j)
                T[i][j] = J[i][0] * Wc[0][j] + J[i][1] * Wc[1][j] + J[i][2] * Wc[2][j];
        const double qw = b.q[0], qx = b.q[1], qy = b.q[2], qz = b.q[3];
        const double nq = qw * qw + qx * qx + qy * qy + qz * qz;
        double M[3][3] = {{qw * qw + qx * qx - qy * qy - qz * qz, 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
                          {2 * (qx * qy + qw * qz), qw * qw - qx * qx + qy * qy - qz * qz, 2 * (qy * qz - qw * qx)},
                          {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), qw * qw - qx * qx - qy * qy + qz * qz}};
        double R[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) R[i][j] = M[i][j] / nq;
        const double s2[3] = {G.s[0] * G.s[0], G.s[1] * G.s[1], G.s[2] * G.s[2]};
        double Sig[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                Sig[i][j] = R[i][0] * s2[0] * R[j][0] + R[i][1] * s2[1] * R[j][1] + R[i][2] * s2[2] * R[j][2];

        // dL/dSigma3 = T^T G' T ; dL/dT = 2 G' T Sigma3
        double GT[2][3];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j) GT[i][j] = Gp[i][0] * T[0][j] + Gp[i][1] * T[1][j];
        double G3[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) G3[i][j] = T[0][i] * GT[0][j] + T[1][i] * GT[1][j];
        double gT[2][3];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j)
                gT[i][j] = 2.0 * (GT[i][0] * Sig[0][j] + GT[i][1] * Sig[1][j] + GT[i][2] * Sig[2][j]);
        // dL/dJ = dL/dT W^T
        double gJ[2][3];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 3; ++j)
                gJ[i][j] = gT[i][0] * Wc[j][0] + gT[i][1] * Wc[j][1] + gT[i][2] * Wc[j][2];
        // camera-space position gradient: J and the pixel centre
        double gp[3];
        gp[0] = gJ[0][2] * (-fx * iz2) + gu * fx * iz;
        gp[1] = gJ[1][2] * (-fy * iz2) + gvv * fy * iz;
        gp[2] = gJ[0][0] * (-fx * iz2) + gJ[0][2] * (2.0 * fx * px * iz2 * iz) +
                gJ[1][1] * (-fy * iz2) + gJ[1][2] * (2.0 * fy * py * iz2 * iz) -
                gu * fx * px * iz2 - gvv * fy * py * iz2;
        for (int c = 0; c < 3; ++c) gm[c] += Wc[0][c] * gp[0] + Wc[1][c] * gp[1] + Wc[2][c] * gp[2];

        // ---- Sigma3 -> scale, rotation -------------------------------------
        // dL/ds_k = 2 s_k (R^T G3 R)_kk ; dL/dR = 2 G3 R S^2
        for (int kk = 0; kk < 3; ++kk) {
            double acc = 0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) acc += R[i][kk] * G3[i][j] * R[j][kk];
            gs[kk] += 2.0 * G.s[kk] * acc;
        }
        double gR[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                gR[i][j] = 2.0 * (G3[i][0] * R[0][j] + G3[i][1] * R[1][j] + G3[i][2] * R[2][j]) * s2[j];
        // R = M / n
        double gn = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) gn -= gR[i][j] * M[i][j];
        gn /= nq * nq;
        double gM[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) gM[i][j] = gR[i][j] / nq;
        double gq[4];
        gq[0] = 2 * (qw * gM[0][0] - qz * gM[0][1] + qy * gM[0][2] + qz * gM[1][0] + qw * gM[1][1] -
                     qx * gM[1][2] - qy * gM[2][0] + qx * gM[2][1] + qw * gM[2][2]) + 2 * qw * gn;
        gq[1] = 2 * (qx * gM[0][0] + qy * gM[0][1] + qz * gM[0][2] + qy * gM[1][0] - qx * gM[1][1] -
                     qw * gM[1][2] + qz * gM[2][0] + qw * gM[2][1] - qx * gM[2][2]) + 2 * qx * gn;
        gq[2] = 2 * (-qy * gM[0][0] + qx * gM[0][1] + qw * gM[0][2] + qx * gM[1][0] + qy * gM[1][1] +
                     qz * gM[1][2] - qw * gM[2][0] + qz * gM[2][1] - qy * gM[2][2]) + 2 * qy * gn;
        gq[3] = 2 * (-qz * gM[0][0] - qw * gM[0][1] + qx * gM[0][2] + qw * gM[1][0] - qz * gM[1][1] +
                     qy * gM[1][2] + qx * gM[2][0] + qy * gM[2][1] + qz * gM[2][2]) + 2 * qz * gn;

        // q = q0 + (t/2) D(omega) q0 with D the left product by (0, omega)
        const double ht = 0.5 * t;
        const double ox = G.om[0], oy = G.om[1], oz = G.om[2];
        const double w0 = G.q0[0], x0 = G.q0[1], y0 = G.q0[2], z0 = G.q0[3];
        gq0[0] += gq[0] + ht * (gq[1] * ox + gq[2] * oy + gq[3] * oz);
        gq0[1] += gq[1] + ht * (-gq[0] * ox + gq[2] * oz - gq[3] * oy);
        gq0[2] += gq[2] + ht * (-gq[0] * oy - gq[1] * oz + gq[3] * ox);
        gq0[3] += gq[3] + ht * (-gq[0] * oz + gq[1] * oy - gq[2] * ox);
        gom[0] += ht * (-gq[0] * x0 + gq[1] * w0 - gq[2] * z0 + gq[3] * y0);
        gom[1] += ht * (-gq[0] * y0 + gq[1] * z0 + gq[2] * w0 - gq[3] * x0);
        gom[2] += ht * (-gq[0] * z0 - gq[1] * y0 + gq[2] * x0 + gq[3] * w0);

        // ---- trajectory ----------------------------------------------------
        for (int c = 0; c < 3; ++c) {
            gx0[c] += gm[c];
            gv[c] += gm[c] * t;
            ga[c] += gm[c] * 0.5 * t * t;
        }
    }
    const int64_t n = P.n;
    for (int c = 0; c < 3; ++c) {
        if (out.mean) out.mean[c * n + k] = (float)gx0[c];
        if (out.vel) out.vel[c * n + k] = (float)gv[c];
        if (out.acc) out.acc[c * n + k] = (float)ga[c];
        if (out.scale) out.scale[c * n + k] = (float)gs[c];
        if (out.omega) out.omega[c * n + k] = (float)gom[c];
        if (out.rgb) out.rgb[c * n + k] = (float)grgb[c];
    }
    for (int c = 0; c < 4; ++c)
        if (out.quat) out.quat[c * n + k] = (float)gq0[c];
    if (out.opacity_logit) out.opacity_logit[k] = (float)glogit;
    if (out.albedo) out.albedo[k] = (float)galb;
}

}  // namespace

void launch_preprocess(const Params& P, const gftorf_gaussians& g, const gftorf_frame* frames,
                       const Workspace& w, hipStream_t s) {
    const int threads = 256;
    const unsigned blocks = (unsigned)((P.n + threads - 1) / threads);
    if (blocks == 0) return;
    { ProfScope _p("k_preprocess", s);
    hipLaunchKernelGGL(k_preprocess, dim3(blocks), dim3(threads), 0, s, P, g, frames, w.rec, w.rect,
                       w.cnt, w.dkey[0], w.dval[0], w.status);
    }
}

void launch_preprocess_bwd(const Params& P, const gftorf_gaussians& g, const gftorf_frame* frames,
                           const Workspace& w, const gftorf_gaussians_grad& grad, hipStream_t s) {
    const int threads = 256;
    const unsigned blocks = (unsigned)((P.n + threads - 1) / threads);
    if (blocks == 0) return;
    { ProfScope _p("k_preprocess_bwd", s);
    hipLaunchKernelGGL(k_preprocess_bwd, dim3(blocks), dim3(threads), 0, s, P, g, frames, w.cnt,
                       w.grec, grad);
    }
}

}  // namespace gft
