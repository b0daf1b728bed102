// Real spherical harmonics of degree <= 3 for the view-dependent colour and
// reflectivity of paper §3 (16 x 3 and 16 coefficients per Gaussian).
//
// Basis order (l, m) = (0,0), (1,-1), (1,0), (1,1), (2,-2) ... (3,3); the real
// harmonics are sqrt(2) Re Y_l^m (m > 0), sqrt(2) Im Y_l^|m| (m < 0) and
// Y_l^0 of the complex harmonics with the Condon-Shortley phase, written as
// polynomials in the unit direction (x, y, z).  The constants are the
// normalisations 1/(2 sqrt(pi)), sqrt(3/(4 pi)), sqrt(15/pi)/2,
// sqrt(5/pi)/4, sqrt(15/pi)/4, sqrt(35/(2 pi))/4, sqrt(105/pi)/2,
// sqrt(21/(2 pi))/4, sqrt(7/pi)/4 and sqrt(105/pi)/4.
#pragma once

namespace gft {

constexpr int kMaxSH = 16;

__host__ __device__ constexpr int sh_count(int degree) { return (degree + 1) * (degree + 1); }

namespace shc {
constexpr float K0 = 0.28209479177387814f;
constexpr float K1 = 0.4886025119029199f;
constexpr float K2a = 1.0925484305920792f;
constexpr float K2b = 0.31539156525252005f;
constexpr float K2c = 0.5462742152960396f;
constexpr float K3a = 0.5900435899266435f;
constexpr float K3b = 2.890611442640554f;
constexpr float K3c = 0.4570457994644658f;
constexpr float K3d = 0.3731763325901154f;
constexpr float K3e = 1.445305721320277f;
}  // namespace shc

// Y[0 .. kMaxSH): basis values at the unit direction; entries past the
// degree are zero.
__device__ __forceinline__ void sh_basis(float x, float y, float z, int degree, float (&Y)[kMaxSH]) {
    using namespace shc;
#pragma unroll
    for (int i = 0; i < kMaxSH; ++i) Y[i] = 0.f;
    Y[0] = K0;
    if (degree < 1) return;
    Y[1] = -K1 * y;
    Y[2] = K1 * z;
    Y[3] = -K1 * x;
    if (degree < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = K2a * x * y;
    Y[5] = -K2a * y * z;
    Y[6] = K2b * (2.f * zz - xx - yy);
    Y[7] = -K2a * x * z;
    Y[8] = K2c * (xx - yy);
    if (degree < 3) return;
    Y[9] = -K3a * y * (3.f * xx - yy);
    Y[10] = K3b * x * y * z;
    Y[11] = -K3c * y * (4.f * zz - xx - yy);
    Y[12] = K3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -K3c * x * (4.f * zz - xx - yy);
    Y[14] = K3e * z * (xx - yy);
    Y[15] = -K3a * x * (xx - 3.f * yy);
}

// Gradient of sum_i w_i Y_i(x, y, z) with respect to (x, y, z), the
// polynomials above differentiated term by term (the unit-length constraint
// is applied by the caller).
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, int degree, const float (&w)[kMaxSH],
                                              float& gx, float& gy, float& gz) {
    using namespace shc;
    gx = gy = gz = 0.f;
    if (degree < 1) return;
    gx += -K1 * w[3];
    gy += -K1 * w[1];
    gz += K1 * w[2];
    if (degree < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    gx += K2a * y * w[4] - 2.f * K2b * x * w[6] - K2a * z * w[7] + 2.f * K2c * x * w[8];
    gy += K2a * x * w[4] - K2a * z * w[5] - 2.f * K2b * y * w[6] - 2.f * K2c * y * w[8];
    gz += -K2a * y * w[5] + 4.f * K2b * z * w[6] - K2a * x * w[7];
    if (degree < 3) return;
    gx += -6.f * K3a * x * y * w[9] + K3b * y * z * w[10] + 2.f * K3c * x * y * w[11] -
          6.f * K3d * x * z * w[12] - K3c * (4.f * zz - 3.f * xx - yy) * w[13] + 2.f * K3e * x * z * w[14] -
          3.f * K3a * (xx - yy) * w[15];
    gy += -3.f * K3a * (xx - yy) * w[9] + K3b * x * z * w[10] - K3c * (4.f * zz - xx - 3.f * yy) * w[11] -
          6.f * K3d * y * z * w[12] + 2.f * K3c * x * y * w[13] - 2.f * K3e * y * z * w[14] +
          6.f * K3a * x * y * w[15];
    gz += K3b * x * y * w[10] - 8.f * K3c * y * z * w[11] + K3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12] -
          8.f * K3c * x * z * w[13] + K3e * (xx - yy) * w[14];
}

}  // namespace gft
