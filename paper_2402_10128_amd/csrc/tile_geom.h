// tile_geom.h -- exact tile membership test of a splat's alpha-floor ellipse (ELLIPSE tile rule).
//
// A tile is listed when the minimum of q(dx,dy) = a dx^2 + 2 b dx dy + c dy^2 over the box of the
// tile's pixel centres, less a rounding allowance of 1e-3 times the magnitude of its terms, does not
// exceed q_max.  Off-centre, the minimum over a box lies on an edge, where q is a 1-D quadratic
// minimised at the clamped stationary point -b e / c (resp. -b e / a), formed with the reciprocals
// 1/c and 1/a computed once per splat (correctly rounded).  Binary32, fixed operation order (files including this
// are compiled with -ffp-contract=off), so the preprocess, the histogram and the scatter kernels take
// identical decisions.
#pragma once
#include <hip/hip_runtime.h>

namespace ges {

__device__ __forceinline__ float geom_max(float a, float b) { return (a < b) ? b : a; }
__device__ __forceinline__ float geom_min(float a, float b) { return (b < a) ? b : a; }

__device__ __forceinline__ float edge_min(float a, float b, float c, float inv_c, float e, float lo, float hi) {
  float y = b * e;
  y = y * inv_c;
  y = -y;
  y = geom_max(y, lo);
  y = geom_min(y, hi);
  float A = a * e; A = A * e;
  float C = c * y; C = C * y;
  float B = b * e; B = B * y; B = B + B;
  float q = A + C;
  float mag = q + __builtin_fabsf(B);
  q = q + B;
  float slack = 1e-3f * mag;
  return q - slack;
}

__device__ __forceinline__ bool ellipse_hits_tile(float u, float v, float a, float b, float c, float inv_a,
                                                  float inv_c, float qm, int tx, int ty, int W, int H) {
  const float x0 = (float)(tx * 16), x1 = (float)min(tx * 16 + 15, W - 1);
  const float y0 = (float)(ty * 16), y1 = (float)min(ty * 16 + 15, H - 1);
  const float dxlo = u - x1, dxhi = u - x0, dylo = v - y1, dyhi = v - y0;
  if (dxlo <= 0.0f && dxhi >= 0.0f && dylo <= 0.0f && dyhi >= 0.0f) return true;
  const float m1 = edge_min(a, b, c, inv_c, dxlo, dylo, dyhi);
  const float m2 = edge_min(a, b, c, inv_c, dxhi, dylo, dyhi);
  const float m3 = edge_min(c, b, a, inv_a, dylo, dxlo, dxhi);
  const float m4 = edge_min(c, b, a, inv_a, dyhi, dxlo, dxhi);
  const float m = geom_min(geom_min(m1, m2), geom_min(m3, m4));
  return m <= qm;
}

}  // namespace ges
