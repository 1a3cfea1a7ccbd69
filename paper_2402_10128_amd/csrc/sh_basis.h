// sh_basis.h -- real spherical harmonics of degree <= 3 (colour model of GES Sec. 4.1, as in Gaussian
// splatting), evaluated in a fixed binary32 operation order.
#pragma once
#include <hip/hip_runtime.h>

namespace ges {

// Real SH basis with the Condon-Shortley phase, degree <= 3, m-ordered.  Constants are the binary32
// values nearest to the normalisations sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (x sqrt 2 for m != 0).
constexpr float kC0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kC1 = 0.4886025119029199f;    // sqrt(3/pi)/2
constexpr float kC2a = 1.0925484305920792f;   // sqrt(15/pi)/2
constexpr float kC2b = 0.31539156525252005f;  // sqrt(5/pi)/4
constexpr float kC2c = 0.5462742152960396f;   // sqrt(15/pi)/4
constexpr float kC3a = 0.5900435899266435f;   // sqrt(35/(2 pi))/4
constexpr float kC3b = 2.890611442640554f;    // sqrt(105/pi)/2
constexpr float kC3c = 0.4570457994644658f;   // sqrt(21/(2 pi))/4
constexpr float kC3d = 0.3731763325901154f;   // sqrt(7/pi)/4
constexpr float kC3e = 1.445305721320277f;    // sqrt(105/pi)/4

__device__ __forceinline__ void sh_basis(float x, float y, float z, int degree, float* Y) {
  Y[0] = kC0;
  if (degree < 1) return;
  Y[1] = -kC1 * y;
  Y[2] = kC1 * z;
  Y[3] = -kC1 * x;
  if (degree < 2) return;
  float xx = x * x, yy = y * y, zz = z * z;
  float xy = x * y, yz = y * z, xz = x * z;
  Y[4] = kC2a * xy;
  Y[5] = -kC2a * yz;
  float t = 2.0f * zz; t = t - xx; t = t - yy;
  Y[6] = kC2b * t;
  Y[7] = -kC2a * xz;
  t = xx - yy;
  Y[8] = kC2c * t;
  if (degree < 3) return;
  float u;
  t = 3.0f * xx; t = t - yy; u = -kC3a * y; Y[9] = u * t;
  u = kC3b * xy; Y[10] = u * z;
  t = 4.0f * zz; t = t - xx; t = t - yy;
  u = -kC3c * y; Y[11] = u * t;
  float t2 = 2.0f * zz; float t3 = 3.0f * xx; t2 = t2 - t3; t3 = 3.0f * yy; t2 = t2 - t3;
  u = kC3d * z; Y[12] = u * t2;
  u = -kC3c * x; Y[13] = u * t;
  t = xx - yy;
  u = kC3e * z; Y[14] = u * t;
  t = 3.0f * yy; t = xx - t;
  u = -kC3a * x; Y[15] = u * t;
}

}  // namespace ges
