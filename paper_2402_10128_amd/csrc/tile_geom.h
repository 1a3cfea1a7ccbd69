// tile_geom.h -- exact tile membership test of a splat's alpha-floor ellipse (ELLIPSE tile rule).
//
// A tile is listed when the minimum of q(dx,dy) = a dx^2 + 2 b dx dy + c dy^2 over the box of the
// tile's pixel centres, less a rounding allowance of 1e-5 times the magnitude of its terms, does not
// exceed q_max (the binary32 rounding of this minimum and of a pixel's q stays below 1e-6 of it).  Off-centre, the minimum over a box lies on an edge, where q is a 1-D quadratic
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
  float slack = 1e-5f * mag;
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

// Candidate tiles of a splat: the tiles of its rectangle that can meet the region the exact test above
// accepts.  That test accepts a point when q - 1e-5 m <= q_max, with m = a dx^2 + c dy^2 + |2 b dx dy|
// <= 2 q / (1 - rho), rho = |b| / sqrt(a c) < 1; so accepted points satisfy q <= q' = q_max / (1 - 2e-5 / (1 - rho)),
// an ellipse with half-extents X = sqrt(q' c / det), Y = sqrt(q' a / det) (q' enlarged by 2.5e-5 instead of
// 2e-5, extents by 1% and half a pixel, covering binary32 rounding here and in the test).  Candidates are
// enumerated row by row of tiles: in each row the tiles meeting the ellipse's extent over the row's band of
// pixel centres (its chord extremes, again enlarged by 1% of their offsets and half a pixel).  Near-degenerate conics
// (rho within 1e-4 of 1) keep the whole rectangle.  A superset only: the exact test decides.  The
// preprocess counts a splat's candidates with this code and the duplication enumerates them with it, from
// the same binary32 values, so both see the same tiles in the same order.  Being a superset with margins of
// 1e-3 and more, it uses the hardware's approximate square root and reciprocal (relative errors near 1e-7,
// the same instructions on both sides) rather than the correctly rounded sequences of the exact path.
struct SplatTiles {
  int tx0, ty0, tx1, ty1;        // box of rows and columns to enumerate
  uint32_t rows;                 // ty1 - ty0 + 1, or 0: no candidate
  bool spans;                    // per-row spans of the ellipse (else whole rows of the box)
  float u, v, a, b, c, qm, inv_a, inv_c;
  float q2, det, Xe, Y, ra;      // the enlarged ellipse: q', det, its half-width sqrt(q' c / det), the
                                 // band half-height Y (1% and half a pixel added) and 1/a (approximate)
};

__device__ __forceinline__ float geom_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float geom_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ void candidate_tiles(float u, float v, float a, float b, float c, float qm, int tx0, int ty0,
                                                int tx1, int ty1, bool ellipse, SplatTiles& s) {
  s.tx0 = tx0; s.ty0 = ty0; s.tx1 = tx1; s.ty1 = ty1;
  s.rows = (uint32_t)(ty1 - ty0 + 1);
  s.spans = false;
  s.u = u; s.v = v; s.a = a; s.b = b; s.c = c; s.qm = qm;
  s.inv_a = 1.0f / a;
  s.inv_c = 1.0f / c;
  s.q2 = 0.f; s.det = 0.f; s.Xe = 0.f; s.Y = 0.f; s.ra = 0.f;
  if (!ellipse) return;
  const float ac = a * c;
  const float det = ac - b * b;
  const float gap = 1.f - __builtin_fabsf(b) * geom_rcp(geom_sqrt(ac));
  if (!(det > 0.f) || !(gap > 1e-4f)) return;
  const float grow = 2.5e-5f * geom_rcp(gap);
  const float q2 = qm * geom_rcp(1.f - grow);
  const float rdet = geom_rcp(det);
  const float Xe = geom_sqrt(q2 * c * rdet);
  const float X = Xe * 1.01f + 0.5f;
  const float Y = geom_sqrt(q2 * a * rdet) * 1.01f + 0.5f;
  if (!(X < 1e7f) || !(Y < 1e7f)) return;
  // tile tx can meet [u - X, u + X] when 16 tx + 15 >= u - X and 16 tx <= u + X
  s.tx0 = max(s.tx0, (int)__builtin_ceilf((u - X - 15.f) * 0.0625f));
  s.tx1 = min(s.tx1, (int)__builtin_floorf((u + X) * 0.0625f));
  s.ty0 = max(s.ty0, (int)__builtin_ceilf((v - Y - 15.f) * 0.0625f));
  s.ty1 = min(s.ty1, (int)__builtin_floorf((v + Y) * 0.0625f));
  if (s.tx0 > s.tx1 || s.ty0 > s.ty1) { s.rows = 0u; return; }
  s.rows = (uint32_t)(s.ty1 - s.ty0 + 1);
  s.spans = true;
  s.q2 = q2; s.det = det; s.Xe = Xe; s.Y = Y; s.ra = geom_rcp(a);
}

// Chord of the enlarged ellipse at height f (relative to v): x offsets e with a e^2 + 2 b e f + c f^2 = q'.
__device__ __forceinline__ float chord_lo(const SplatTiles& s, float f) {
  float r = s.a * s.q2;
  float t = s.det * f; t = t * f;
  r = r - t;
  r = geom_max(r, 0.f);
  float e = s.b * f; e = -e;
  e = e - geom_sqrt(r);
  return e * s.ra;
}
__device__ __forceinline__ float chord_hi(const SplatTiles& s, float f) {
  float r = s.a * s.q2;
  float t = s.det * f; t = t * f;
  r = r - t;
  r = geom_max(r, 0.f);
  float e = s.b * f; e = -e;
  e = e + geom_sqrt(r);
  return e * s.ra;
}

// Candidate columns [lo, hi] of tile row ty (ty0 <= ty <= ty1); lo > hi: none.
__device__ __forceinline__ void row_span(const SplatTiles& s, int ty, int H, int& lo, int& hi) {
  lo = s.tx0;
  hi = s.tx1;
  if (!s.spans) return;
  const float y0 = (float)(ty * 16), y1 = (float)min(ty * 16 + 15, H - 1);
  const float Yh = s.Y;
  float f0 = y0 - s.v, f1 = y1 - s.v;
  f0 = geom_max(f0, -Yh);
  f1 = geom_min(f1, Yh);
  if (!(f0 <= f1)) { lo = 1; hi = 0; return; }
  // the extremes over the band: at its ends, or at the ellipse's leftmost / rightmost points
  // f = +- b X' / c (X' = sqrt(q' c / det)) when those lie inside the band
  const float Xe = s.Xe;
  float fl = s.b * Xe; fl = fl * s.inv_c;   // leftmost point at f = b X' / c
  const float fr = -fl;                     // rightmost point at f = -b X' / c
  float emin = geom_min(chord_lo(s, f0), chord_lo(s, f1));
  float emax = geom_max(chord_hi(s, f0), chord_hi(s, f1));
  if (f0 <= fl && fl <= f1) emin = -Xe;
  if (f0 <= fr && fr <= f1) emax = Xe;
  float m = __builtin_fabsf(emin) + __builtin_fabsf(emax);
  m = 0.005f * m;
  m = m + 0.5f;
  const float xl = (s.u + emin) - m, xr = (s.u + emax) + m;
  lo = max(s.tx0, (int)__builtin_ceilf((xl - 15.f) * 0.0625f));
  hi = min(s.tx1, (int)__builtin_floorf(xr * 0.0625f));
}

// Number of candidate tiles of a splat (the sum of its rows' spans).
__device__ __forceinline__ uint32_t candidate_count(const SplatTiles& s, int H) {
  uint32_t n = 0;
  for (uint32_t r = 0; r < s.rows; ++r) {
    int lo, hi;
    row_span(s, s.ty0 + (int)r, H, lo, hi);
    if (hi >= lo) n += (uint32_t)(hi - lo + 1);
  }
  return n;
}

}  // namespace ges
