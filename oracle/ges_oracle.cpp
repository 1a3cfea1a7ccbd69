// ges_oracle.cpp -- plain CPU oracle for the GES tile rasterizer.
//
// TEST INFRASTRUCTURE ONLY (see ges_oracle.h).  Built with g++ -O2 -ffp-contract=off, no fast-math,
// so every binary32 expression below is evaluated exactly as written: one rounding per operation,
// no fused multiply-add unless std::fma is spelled out.
//
// Paper: GES, arXiv 2402.10128.  Sections cited inline.
#include "ges_oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ------------------------------------------------------------------------------------------------
// Canonical binary32 exp and log.
//
// exp: Cody-Waite argument reduction x = k*ln2 + r with k = rint(x*log2(e)) and ln2 split into a
// 15-significant-bit head (so k*head is exact for |k| <= 2^9) and a binary32 tail; exp(r) by the
// degree-7 Taylor polynomial in Horner form; the result is scaled by 2^k through the exponent field.
// log: x = m * 2^e with m in [sqrt(1/2), sqrt(2)); log(m) = 2*atanh(s), s = (m-1)/(m+1), by the odd
// series up to s^9; log(x) = e*ln2_head + (e*ln2_tail + log(m)).
// Range edges: exp(x) = +inf for x > 88.72283935546875, 0 for x < -87.33654022216797 (the binary32
// min-normal boundary; the canonical function flushes below it); log(0) = -inf, log(x<0) = NaN.
// Constants are derived here from their definitions (the binary32 value nearest to each).
// ------------------------------------------------------------------------------------------------
struct CanonConsts {
  float log2e, ln2_hi, ln2_lo, sqrt2;
  float e2, e3, e4, e5, e6, e7;   // 1/k! for k = 2..7
  float l3, l5, l7, l9;           // 1/k
  CanonConsts() {
    const double ln2 = std::log(2.0);
    log2e = (float)(1.0 / ln2);
    ln2_hi = (float)(std::floor(ln2 * 32768.0) / 32768.0);
    ln2_lo = (float)(ln2 - (double)ln2_hi);
    sqrt2 = (float)std::sqrt(2.0);
    e2 = (float)(1.0 / 2.0);
    e3 = (float)(1.0 / 6.0);
    e4 = (float)(1.0 / 24.0);
    e5 = (float)(1.0 / 120.0);
    e6 = (float)(1.0 / 720.0);
    e7 = (float)(1.0 / 5040.0);
    l3 = (float)(1.0 / 3.0);
    l5 = (float)(1.0 / 5.0);
    l7 = (float)(1.0 / 7.0);
    l9 = (float)(1.0 / 9.0);
  }
};
const CanonConsts CC;

inline float bits_to_float(uint32_t b) { float f; std::memcpy(&f, &b, 4); return f; }
inline uint32_t float_to_bits(float f) { uint32_t b; std::memcpy(&b, &f, 4); return b; }

float exp_c(float x) {
  if (x != x) return x;
  if (x > 88.72283935546875f) return std::numeric_limits<float>::infinity();
  if (x < -87.33654022216797f) return 0.0f;
  float k = std::rint(x * CC.log2e);
  float r = x - k * CC.ln2_hi;
  r = r - k * CC.ln2_lo;
  float p = CC.e7;
  p = p * r; p = p + CC.e6;
  p = p * r; p = p + CC.e5;
  p = p * r; p = p + CC.e4;
  p = p * r; p = p + CC.e3;
  p = p * r; p = p + CC.e2;
  p = p * r; p = p + 1.0f;
  p = p * r; p = p + 1.0f;
  int ki = (int)k;
  if (ki > 127) {
    p = p * bits_to_float((uint32_t)(127 + 127) << 23);
    return p * 2.0f;
  }
  return p * bits_to_float((uint32_t)(ki + 127) << 23);
}

float log_c(float x) {
  if (x != x) return x;
  if (x < 0.0f) return std::numeric_limits<float>::quiet_NaN();
  if (x == 0.0f) return -std::numeric_limits<float>::infinity();
  if (x == std::numeric_limits<float>::infinity()) return x;
  int e = 0;
  uint32_t b = float_to_bits(x);
  if (b < 0x00800000u) {            // subnormal: scale by 2^23 (exact)
    x = x * 8388608.0f;
    b = float_to_bits(x);
    e = -23;
  }
  e += (int)((b >> 23) & 0xffu) - 127;
  float m = bits_to_float((b & 0x007fffffu) | 0x3f800000u);   // [1,2)
  if (m > CC.sqrt2) { m = m * 0.5f; e += 1; }
  float f = m - 1.0f;
  float den = m + 1.0f;
  float s = f / den;
  float s2 = s * s;
  float poly = CC.l9;
  poly = poly * s2; poly = poly + CC.l7;
  poly = poly * s2; poly = poly + CC.l5;
  poly = poly * s2; poly = poly + CC.l3;
  poly = poly * s2;
  float lm = s * poly;
  lm = s + lm;
  lm = lm + lm;
  float ef = (float)e;
  float lo = ef * CC.ln2_lo;
  lo = lo + lm;
  float hi = ef * CC.ln2_hi;
  return hi + lo;
}

// ln Gamma(x), x > 0, in binary32 for the exact shape modification (Sec. 4.2, Eq. probablity): the
// recurrence Gamma(x) = Gamma(x + 1) / x lifts x to at least 8 (the factors multiplied into one product),
// then Stirling's series with the terms 1/(12x), -1/(360x^3), 1/(1260x^5); finally minus ln of the product.
float lgamma_c(float x) {
  float prod = 1.0f;
  while (x < 8.0f) {
    prod = prod * x;
    x = x + 1.0f;
  }
  const float lz = log_c(x);
  float t = x - 0.5f;
  t = t * lz;
  t = t - x;
  t = t + 0.918938533204672742f;                // ln(2 pi) / 2
  const float iz = 1.0f / x;
  const float iz2 = iz * iz;
  float c = iz2 * (float)(1.0 / 1260.0);
  c = (float)(1.0 / 360.0) - c;
  c = c * iz2;
  c = (float)(1.0 / 12.0) - c;
  c = c * iz;
  t = t + c;
  return t - log_c(prod);
}

// Scalar policy: F32 mode uses the canonical functions, F64 mode libm.
template <class S> struct M;
template <> struct M<float> {
  static float ex(float x) { return exp_c(x); }
  static float lg(float x) { return log_c(x); }
  static float lgam(float x) { return lgamma_c(x); }
};
template <> struct M<double> {
  static double ex(double x) { return std::exp(x); }
  static double lg(double x) { return std::log(x); }
  static double lgam(double x) { return std::lgamma(x); }
};

// ------------------------------------------------------------------------------------------------
// Real spherical harmonics, degree <= 3, with the Condon-Shortley phase, m-ordered (m = -l..l),
// evaluated at a unit direction (x,y,z).  Normalisation constants from
// N_lm = sqrt((2l+1)/(4 pi) * (l-|m|)!/(l+|m|)!) (times sqrt(2) for m != 0), written out per (l,m)
// as closed forms.
// ------------------------------------------------------------------------------------------------
struct ShConsts {
  double c0, c1, c2a, c2b, c2c, c3a, c3b, c3c, c3d, c3e;
  ShConsts() {
    const double pi = std::acos(-1.0);
    c0 = (0.5 * std::sqrt(1.0 / pi));
    c1 = (0.5 * std::sqrt(3.0 / pi));
    c2a = (0.5 * std::sqrt(15.0 / pi));    // xy, yz, xz
    c2b = (0.25 * std::sqrt(5.0 / pi));    // 2z^2 - x^2 - y^2
    c2c = (0.25 * std::sqrt(15.0 / pi));   // x^2 - y^2
    c3a = (0.25 * std::sqrt(35.0 / (2.0 * pi)));   // y(3x^2-y^2), x(x^2-3y^2)
    c3b = (0.5 * std::sqrt(105.0 / pi));           // xyz
    c3c = (0.25 * std::sqrt(21.0 / (2.0 * pi)));   // y(4z^2-x^2-y^2), x(...)
    c3d = (0.25 * std::sqrt(7.0 / pi));            // z(2z^2-3x^2-3y^2)
    c3e = (0.25 * std::sqrt(105.0 / pi));          // z(x^2-y^2)
  }
};
const ShConsts SC;

// Basis values Y_k, k = l^2 + l + m, in the canonical operation order.
template <class S>
void sh_basis(S x, S y, S z, int degree, S* Y) {
  Y[0] = (S)SC.c0;
  if (degree < 1) return;
  Y[1] = (S)(-SC.c1) * y;
  Y[2] = (S)SC.c1 * z;
  Y[3] = (S)(-SC.c1) * x;
  if (degree < 2) return;
  S xx = x * x, yy = y * y, zz = z * z;
  S xy = x * y, yz = y * z, xz = x * z;
  Y[4] = (S)SC.c2a * xy;
  Y[5] = (S)(-SC.c2a) * yz;
  S t = (S)2 * zz; t = t - xx; t = t - yy;
  Y[6] = (S)SC.c2b * t;
  Y[7] = (S)(-SC.c2a) * xz;
  t = xx - yy;
  Y[8] = (S)SC.c2c * t;
  if (degree < 3) return;
  S u;
  t = (S)3 * xx; t = t - yy;  u = (S)(-SC.c3a) * y;  Y[9] = u * t;
  u = (S)SC.c3b * xy;         Y[10] = u * z;
  t = (S)4 * zz; t = t - xx; t = t - yy;
  u = (S)(-SC.c3c) * y;       Y[11] = u * t;
  S t2 = (S)2 * zz; S t3 = (S)3 * xx; t2 = t2 - t3; t3 = (S)3 * yy; t2 = t2 - t3;
  u = (S)SC.c3d * z;          Y[12] = u * t2;
  u = (S)(-SC.c3c) * x;       Y[13] = u * t;
  t = xx - yy;
  u = (S)SC.c3e * z;          Y[14] = u * t;
  t = (S)3 * yy; t = xx - t;
  u = (S)(-SC.c3a) * x;       Y[15] = u * t;
}

// ------------------------------------------------------------------------------------------------
// Ellipse-tile test (ELLIPSE tile culling).  A tile is kept when the minimum of the splat's quadratic
// form over the tile's box of pixel centres, less a rounding allowance of 1e-5 times the magnitude of
// its terms, does not exceed q_max.  The allowance covers the binary32 rounding of this minimum and of a
// pixel's own q (a few units in the last place of the terms, below 1e-6 of their magnitude), so every
// pixel that passes the alpha floor lies in a kept tile.  The minimum over a box lies at an interior point only if the
// centre is inside; otherwise on one of the four edges, where it is a 1-D quadratic minimised at the
// clamped stationary point -b e / c (resp. -b e / a), evaluated with the reciprocals 1/c and 1/a
// formed once per splat.
// ------------------------------------------------------------------------------------------------
template <class S>
S edge_min(S a, S b, S c, S inv_c, S e, S lo, S hi) {
  S y = b * e;
  y = y * inv_c;
  y = -y;
  y = std::max(y, lo);
  y = std::min(y, hi);
  S A = a * e; A = A * e;
  S C = c * y; C = C * y;
  S B = b * e; B = B * y; B = B + B;
  S q = A + C;
  S mag = q + std::fabs(B);
  q = q + B;
  S slack = (S)1e-5 * mag;
  return q - slack;
}

template <class S>
bool ellipse_hits_tile(S u, S v, S a, S b, S c, S qm, int tx, int ty, int W, int H) {
  S x0 = (S)(tx * OC_TILE), x1 = (S)std::min(tx * OC_TILE + OC_TILE - 1, W - 1);
  S y0 = (S)(ty * OC_TILE), y1 = (S)std::min(ty * OC_TILE + OC_TILE - 1, H - 1);
  S dxlo = u - x1, dxhi = u - x0, dylo = v - y1, dyhi = v - y0;
  if (dxlo <= (S)0 && dxhi >= (S)0 && dylo <= (S)0 && dyhi >= (S)0) return true;
  const S inv_a = (S)1 / a, inv_c = (S)1 / c;
  S m1 = edge_min(a, b, c, inv_c, dxlo, dylo, dyhi);
  S m2 = edge_min(a, b, c, inv_c, dxhi, dylo, dyhi);
  S m3 = edge_min(c, b, a, inv_a, dylo, dxlo, dxhi);
  S m4 = edge_min(c, b, a, inv_a, dyhi, dxlo, dxhi);
  S m = std::min(std::min(m1, m2), std::min(m3, m4));
  return m <= qm;
}

inline bool all_finite(const float* p, int k) {
  for (int i = 0; i < k; ++i) if (!std::isfinite(p[i])) return false;
  return true;
}

void cull(oc_record* o, int64_t i) {
  o->u[i] = o->v[i] = o->depth[i] = 0.0;
  o->conic[3 * i] = o->conic[3 * i + 1] = o->conic[3 * i + 2] = 0.0;
  o->qmax[i] = o->opacity[i] = 0.0;
  o->rgb[3 * i] = o->rgb[3 * i + 1] = o->rgb[3 * i + 2] = 0.0;
  o->radius[i] = 0;
  for (int k = 0; k < 4; ++k) o->rect[4 * i + k] = 0;
  o->tiles_touched[i] = 0;
  o->clamp_bits[i] = 0;
}

// ------------------------------------------------------------------------------------------------
// Preprocess of one splat (Sec. 4.1 and 4.2).  Every step is one binary32 (or binary64) operation in
// the order written.
// ------------------------------------------------------------------------------------------------
template <class S>
void preprocess_one(int64_t i, const oc_splats* sp, const oc_camera* cam, const oc_params* prm,
                    const S campos[3], oc_record* o) {
  const int K = (sp->sh_degree + 1) * (sp->sh_degree + 1);
  const float* mu = sp->means + 3 * i;
  const float* ls = sp->log_scales + 3 * i;
  const float* qq = sp->quats + 4 * i;
  const float* shc = sp->sh + (int64_t)3 * K * i;
  o->beta[i] = (double)sp->beta[i];
  if (!all_finite(mu, 3) || !all_finite(ls, 3) || !all_finite(qq, 4) || !std::isfinite(sp->opacity_logits[i]) ||
      !std::isfinite(sp->beta[i]) || !all_finite(shc, 3 * K)) {
    cull(o, i);
    return;
  }
  const S* R = nullptr;
  S Rc[9], tc[3];
  for (int k = 0; k < 9; ++k) Rc[k] = (S)cam->R[k];
  for (int k = 0; k < 3; ++k) tc[k] = (S)cam->t[k];
  R = Rc;
  const S mx = (S)mu[0], my = (S)mu[1], mz = (S)mu[2];

  // 1. camera-space position p = R mu + t; near-plane cull on z
  S p[3];
  for (int r = 0; r < 3; ++r) {
    S acc = R[3 * r] * mx;
    acc = acc + R[3 * r + 1] * my;
    acc = acc + R[3 * r + 2] * mz;
    p[r] = acc + tc[r];
  }
  const S z = p[2];
  if (!(z > (S)cam->near_z)) { cull(o, i); return; }

  // 2. activations: scale = exp(log-scale), opacity = sigmoid(logit)
  S s[3];
  for (int k = 0; k < 3; ++k) s[k] = M<S>::ex((S)ls[k]);
  S en = M<S>::ex(-(S)sp->opacity_logits[i]);
  S den = (S)1 + en;
  const S op = (S)1 / den;
  const S o255 = (S)255 * op;                     // alpha floor 1/255: need 255*o > 1
  if (!(o255 > (S)1)) { cull(o, i); return; }

  // 3. unit quaternion (w,x,y,z) and its rotation matrix
  S qw = (S)qq[0], qx = (S)qq[1], qy = (S)qq[2], qz = (S)qq[3];
  S nn = qw * qw; nn = nn + qx * qx; nn = nn + qy * qy; nn = nn + qz * qz;
  if (!(nn > (S)0)) { cull(o, i); return; }
  S nr = std::sqrt(nn);
  qw = qw / nr; qx = qx / nr; qy = qy / nr; qz = qz / nr;
  S Q[9];
  {
    S t;
    t = qy * qy; t = t + qz * qz; t = (S)2 * t; Q[0] = (S)1 - t;
    t = qx * qy; t = t - qw * qz; Q[1] = (S)2 * t;
    t = qx * qz; t = t + qw * qy; Q[2] = (S)2 * t;
    t = qx * qy; t = t + qw * qz; Q[3] = (S)2 * t;
    t = qx * qx; t = t + qz * qz; t = (S)2 * t; Q[4] = (S)1 - t;
    t = qy * qz; t = t - qw * qx; Q[5] = (S)2 * t;
    t = qx * qz; t = t - qw * qy; Q[6] = (S)2 * t;
    t = qy * qz; t = t + qw * qx; Q[7] = (S)2 * t;
    t = qx * qx; t = t + qy * qy; t = (S)2 * t; Q[8] = (S)1 - t;
  }

  // 4. shape modification (Eq. approx): scales multiplied by phi_rho(beta) = 2/(1+exp(-(rho*beta-2*rho)))
  //    in PHI mode; the GEF mode keeps the scales and uses beta in the falloff (Eq. ges).
  const S beta = (S)sp->beta[i];
  S phi;
  if (prm->falloff == OC_FALLOFF_PHI) {
    const S rho = (S)prm->rho;
    S t = rho * beta;
    S r2 = (S)2 * rho;
    t = t - r2;
    S e = M<S>::ex(-t);
    S d = (S)1 + e;
    phi = (S)2 / d;
  } else if (prm->falloff == OC_FALLOFF_PHI_EXACT) {
    // exact modification 2 Gamma(3/beta) / Gamma(1/beta), normalised to 1 at beta = 2 (Eq. probablity)
    if (!(beta > (S)0)) { cull(o, i); return; }
    const S a3 = (S)3 / beta, a1 = (S)1 / beta;
    S dl = M<S>::lgam(a3);
    dl = dl - M<S>::lgam(a1);
    phi = (S)2 * M<S>::ex(dl);
    if (!std::isfinite(phi) || !(phi > (S)0)) { cull(o, i); return; }
  } else {
    if (!(beta > (S)0)) { cull(o, i); return; }
    phi = (S)1;
  }
  S sc[3];
  for (int k = 0; k < 3; ++k) sc[k] = phi * s[k];

  // 5. Sigma = (R S)(R S)^T (Sec. 4.1)
  S Mm[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Mm[3 * r + c] = Q[3 * r + c] * sc[c];
  S Sig[9];
  for (int r = 0; r < 3; ++r)
    for (int c = r; c < 3; ++c) {
      S acc = Mm[3 * r] * Mm[3 * c];
      acc = acc + Mm[3 * r + 1] * Mm[3 * c + 1];
      acc = acc + Mm[3 * r + 2] * Mm[3 * c + 2];
      Sig[3 * r + c] = acc;
      Sig[3 * c + r] = acc;
    }

  // 6. EWA (Sec. 4.1): Sigma' = J W Sigma W^T J^T, W = camera rotation, J = perspective Jacobian at p
  //    with the view-frustum guard: x/z, y/z clamped to +-1.3 * half-FoV tangent.
  const S fx = (S)cam->fx, fy = (S)cam->fy;
  S limx = (S)0.5 * (S)cam->width;  limx = limx / fx;  limx = (S)1.3 * limx;
  S limy = (S)0.5 * (S)cam->height; limy = limy / fy;  limy = (S)1.3 * limy;
  S txz = p[0] / z, tyz = p[1] / z;
  uint8_t bits = 0;
  if (txz < -limx) { txz = -limx; bits |= 8; } else if (txz > limx) { txz = limx; bits |= 8; }
  if (tyz < -limy) { tyz = -limy; bits |= 16; } else if (tyz > limy) { tyz = limy; bits |= 16; }
  const S xc = txz * z, yc = tyz * z;
  const S z2 = z * z;
  const S J00 = fx / z, J11 = fy / z;
  S J02 = fx * xc; J02 = J02 / z2; J02 = -J02;
  S J12 = fy * yc; J12 = J12 / z2; J12 = -J12;
  S T[6];
  for (int c = 0; c < 3; ++c) {
    S a0 = J00 * R[c];
    T[c] = a0 + J02 * R[6 + c];
    S a1 = J11 * R[3 + c];
    T[3 + c] = a1 + J12 * R[6 + c];
  }
  S U[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) {
      S acc = T[3 * r] * Sig[c];
      acc = acc + T[3 * r + 1] * Sig[3 + c];
      acc = acc + T[3 * r + 2] * Sig[6 + c];
      U[3 * r + c] = acc;
    }
  S cv[3];  // cov00, cov01, cov11
  {
    S acc = U[0] * T[0]; acc = acc + U[1] * T[1]; acc = acc + U[2] * T[2]; cv[0] = acc;
    acc = U[0] * T[3]; acc = acc + U[1] * T[4]; acc = acc + U[2] * T[5]; cv[1] = acc;
    acc = U[3] * T[3]; acc = acc + U[4] * T[4]; acc = acc + U[5] * T[5]; cv[2] = acc;
  }
  cv[0] = cv[0] + (S)0.3;
  cv[2] = cv[2] + (S)0.3;
  S det = cv[0] * cv[2];
  det = det - cv[1] * cv[1];
  if (!(det > (S)0)) { cull(o, i); return; }
  const S ca = cv[2] / det;
  S cb = cv[1] / det; cb = -cb;
  const S ccc = cv[0] / det;

  // 7. mean2D (pixel centres at integer coordinates)
  S u = fx * p[0]; u = u / z; u = u + (S)cam->cx;
  S v = fy * p[1]; v = v / z; v = v + (S)cam->cy;

  // 8. alpha-floor threshold: alpha >= 1/255  <=>  q <= qmax
  //    PHI: exp(-q/2) o >= 1/255  <=>  q <= 2 ln(255 o)
  //    GEF: exp(-q^(beta/2)/2) o >= 1/255  <=>  q <= (2 ln(255 o))^(2/beta)
  S L2 = M<S>::lg(o255);
  L2 = (S)2 * L2;
  S qm;
  if (prm->falloff != OC_FALLOFF_GEF) {   // Gaussian falloff (PHI and PHI_EXACT)
    qm = L2;
  } else {
    S e = (S)2 / beta;
    S lgl = M<S>::lg(L2);
    e = e * lgl;
    qm = M<S>::ex(e);
  }
  if (!std::isfinite(qm)) { cull(o, i); return; }

  // 9. screen radius: largest eigenvalue of Sigma' and r = 1 + ceil(sqrt(qmax * lambda_max))
  S mid = cv[0] + cv[2]; mid = (S)0.5 * mid;
  S disc = mid * mid; disc = disc - det;
  disc = std::max((S)0, disc);
  S lam = mid + std::sqrt(disc);
  S rr = qm * lam;
  rr = std::sqrt(rr);
  rr = std::ceil(rr);
  if (!(rr <= (S)1048576)) rr = (S)1048576;
  const int radius = 1 + (int)rr;
  const S fr = (S)radius;

  // 10. tile rectangle: tiles holding a pixel centre inside [u-r,u+r] x [v-r,v+r]
  S xl = u - fr; xl = std::ceil(xl);
  S xh = u + fr; xh = std::floor(xh);
  S yl = v - fr; yl = std::ceil(yl);
  S yh = v + fr; yh = std::floor(yh);
  xl = std::max(xl, (S)0); xh = std::min(xh, (S)(cam->width - 1));
  yl = std::max(yl, (S)0); yh = std::min(yh, (S)(cam->height - 1));
  if (!(xl <= xh) || !(yl <= yh)) { cull(o, i); return; }
  const int tx0 = (int)xl / OC_TILE, tx1 = (int)xh / OC_TILE;
  const int ty0 = (int)yl / OC_TILE, ty1 = (int)yh / OC_TILE;
  int64_t touched = 0;
  if (prm->tile_cull == OC_TILES_SQUARE) {
    touched = (int64_t)(tx1 - tx0 + 1) * (ty1 - ty0 + 1);
  } else {
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx)
        if (ellipse_hits_tile<S>(u, v, ca, cb, ccc, qm, tx, ty, cam->width, cam->height)) ++touched;
  }
  if (touched == 0) { cull(o, i); return; }

  // 11. colour from SH (Sec. 4.1): direction from the camera centre to the mean, basis values,
  //     rgb = sum_k Y_k c_k + 0.5, clamped at 0.
  S d0 = mx - campos[0], d1 = my - campos[1], d2 = mz - campos[2];
  S len = d0 * d0; len = len + d1 * d1; len = len + d2 * d2;
  len = std::sqrt(len);
  S dx = d0 / len, dy = d1 / len, dz = d2 / len;
  S Y[16];
  sh_basis<S>(dx, dy, dz, sp->sh_degree, Y);
  S rgb[3];
  for (int ch = 0; ch < 3; ++ch) {
    S acc = Y[0] * (S)shc[ch];
    for (int k = 1; k < K; ++k) acc = acc + Y[k] * (S)shc[3 * k + ch];
    acc = acc + (S)0.5;
    if (acc < (S)0) { acc = (S)0; bits |= (uint8_t)(1u << ch); }
    rgb[ch] = acc;
  }

  o->u[i] = u; o->v[i] = v; o->depth[i] = z;
  o->conic[3 * i] = ca; o->conic[3 * i + 1] = cb; o->conic[3 * i + 2] = ccc;
  o->qmax[i] = qm; o->opacity[i] = op;
  o->rgb[3 * i] = rgb[0]; o->rgb[3 * i + 1] = rgb[1]; o->rgb[3 * i + 2] = rgb[2];
  o->radius[i] = radius;
  o->rect[4 * i] = tx0; o->rect[4 * i + 1] = ty0; o->rect[4 * i + 2] = tx1; o->rect[4 * i + 3] = ty1;
  o->tiles_touched[i] = touched;
  o->clamp_bits[i] = bits;
}

template <class S>
void camera_centre(const oc_camera* cam, S c[3]) {
  // c = -R^T t
  for (int j = 0; j < 3; ++j) {
    S acc = (S)cam->R[j] * (S)cam->t[0];
    acc = acc + (S)cam->R[3 + j] * (S)cam->t[1];
    acc = acc + (S)cam->R[6 + j] * (S)cam->t[2];
    c[j] = -acc;
  }
}

template <class S>
void preprocess_all(const oc_splats* sp, const oc_camera* cam, const oc_params* prm, oc_record* o) {
  S cp[3];
  camera_centre<S>(cam, cp);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < sp->n; ++i) preprocess_one<S>(i, sp, cam, prm, cp, o);
}

int tiles_x(const oc_camera* c) { return (c->width + OC_TILE - 1) / OC_TILE; }
int tiles_y(const oc_camera* c) { return (c->height + OC_TILE - 1) / OC_TILE; }

bool in_tile(int mode, const oc_record* r, int64_t i, const oc_camera* cam, const oc_params* p, int tx, int ty) {
  if (r->tiles_touched[i] == 0) return false;
  const int32_t* rc = r->rect + 4 * i;
  if (tx < rc[0] || tx > rc[2] || ty < rc[1] || ty > rc[3]) return false;
  if (p->tile_cull == OC_TILES_SQUARE) return true;
  if (mode == OC_MODE_F32)
    return ellipse_hits_tile<float>((float)r->u[i], (float)r->v[i], (float)r->conic[3 * i], (float)r->conic[3 * i + 1],
                                    (float)r->conic[3 * i + 2], (float)r->qmax[i], tx, ty, cam->width, cam->height);
  return ellipse_hits_tile<double>(r->u[i], r->v[i], r->conic[3 * i], r->conic[3 * i + 1], r->conic[3 * i + 2],
                                   r->qmax[i], tx, ty, cam->width, cam->height);
}

// ------------------------------------------------------------------------------------------------
// Per-pixel compositing (Sec. 4.2, Eq. transimttance, discretised front to back).
// For each splat j of the pixel's depth-sorted list:
//   q = a dx^2 + 2 b dx dy + c dy^2 with (dx,dy) = mean2D - pixel centre;
//   skip unless q <= qmax (the alpha floor alpha >= 1/255, decided exactly on q);
//   G = exp(-q/2) (PHI) or exp(-q^(beta/2)/2) (GEF); alpha = min(0.99, o G);
//   t = T (1 - alpha); stop before compositing when t < 1e-4;
//   C += alpha T rgb; T = t.
// Final colour C + T bg.
// In F32 mode q is the canonical binary32 expression
//   t1 = fma(a, dx, (2b) dy);  q = fma(t1, dx, (c dy) dy)
// and everything after it is binary64.
// ------------------------------------------------------------------------------------------------
constexpr double kAlphaMax = 0.99;
constexpr double kTMin = 1e-4;
constexpr double kFlagRel = 1e-3;   // termination decisions this close (relative) to 1e-4 are flagged

struct Splat2D {
  double u, v, a, b, c, qmax, o, r, g, bl, beta;
  float uf, vf, af, bbf, cf, qmf;
};

inline void load_splat(const oc_record* r, uint32_t i, Splat2D& s) {
  s.u = r->u[i]; s.v = r->v[i];
  s.a = r->conic[3 * i]; s.b = r->conic[3 * i + 1]; s.c = r->conic[3 * i + 2];
  s.qmax = r->qmax[i]; s.o = r->opacity[i];
  s.r = r->rgb[3 * i]; s.g = r->rgb[3 * i + 1]; s.bl = r->rgb[3 * i + 2];
  s.beta = r->beta[i];
  s.uf = (float)s.u; s.vf = (float)s.v; s.af = (float)s.a;
  float bf = (float)s.b;
  s.bbf = bf + bf;
  s.cf = (float)s.c; s.qmf = (float)s.qmax;
}

// Returns q (as double) and whether the splat passes the alpha-floor test.
inline bool pair_q(int mode, const Splat2D& s, int px, int py, double& q, double& dx, double& dy) {
  if (mode == OC_MODE_F32) {
    float fdx = s.uf - (float)px;
    float fdy = s.vf - (float)py;
    float t = s.bbf * fdy;
    t = std::fma(s.af, fdx, t);
    float w = s.cf * fdy;
    w = w * fdy;
    float qf = std::fma(t, fdx, w);
    dx = fdx; dy = fdy; q = qf;
    return qf <= s.qmf;
  }
  dx = s.u - (double)px;
  dy = s.v - (double)py;
  q = s.a * dx * dx + 2.0 * s.b * dx * dy + s.c * dy * dy;
  return q <= s.qmax;
}

inline double falloff(int falloff_mode, double q, double beta) {
  if (q < 0.0) q = 0.0;
  if (falloff_mode != OC_FALLOFF_GEF) return std::exp(-0.5 * q);
  return std::exp(-0.5 * std::pow(q, 0.5 * beta));
}

inline uint64_t mix64(uint64_t h, uint64_t x) {
  h ^= x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h;
}

struct PixelOut {
  double C[3], T;
  int32_t nc;
  bool flagged;
  double alt[3];
  int64_t examined, skipped, blended;
  uint64_t hash;
};

// Forward over one pixel's list.  force_flip_at: list position whose termination decision is inverted
// (-1 = none), used to produce the alternative branch of a flagged pixel.
void pixel_forward(int mode, const oc_params* p, const Splat2D* L, int64_t len, int px, int py,
                   int64_t force_flip_at, PixelOut& out, int64_t* near_pos) {
  double T = 1.0, C[3] = {0.0, 0.0, 0.0};
  int32_t nc = 0;
  int64_t ex = 0, sk = 0, bl = 0;
  uint64_t h = 0;
  double best_margin = 1e300;
  int64_t best_pos = -1;
  for (int64_t j = 0; j < len; ++j) {
    const Splat2D& s = L[j];
    double q, dx, dy;
    ++ex;
    if (!pair_q(mode, s, px, py, q, dx, dy)) { ++sk; continue; }
    double G = falloff(p->falloff, q, s.beta);
    double oG = s.o * G;
    bool clamped = oG > kAlphaMax;
    double alpha = clamped ? kAlphaMax : oG;
    double t = T * (1.0 - alpha);
    double margin = std::fabs(t - kTMin) / kTMin;
    bool stop = t < kTMin;
    if (j == force_flip_at) stop = !stop;
    if (margin < best_margin) { best_margin = margin; best_pos = j; }
    if (stop) { h = mix64(h, 0xdead0000ull + (uint64_t)j); break; }
    C[0] += s.r * alpha * T;
    C[1] += s.g * alpha * T;
    C[2] += s.bl * alpha * T;
    T = t;
    nc = (int32_t)(j + 1);
    ++bl;
    h = mix64(h, ((uint64_t)j << 1) | (clamped ? 1u : 0u));
  }
  out.C[0] = C[0] + T * p->bg[0];
  out.C[1] = C[1] + T * p->bg[1];
  out.C[2] = C[2] + T * p->bg[2];
  out.T = T;
  out.nc = nc;
  out.examined = ex; out.skipped = sk; out.blended = bl;
  out.hash = mix64(h, (uint64_t)nc);
  out.flagged = best_margin < kFlagRel;
  if (near_pos) *near_pos = out.flagged ? best_pos : -1;
}

void render_list(int mode, const oc_camera* cam, const oc_params* p, const Splat2D* L, int64_t len,
                 int x0, int y0, int x1, int y1, double* img, double* final_T, int32_t* n_contrib,
                 uint8_t* flags, double* alt, int64_t* acc /*[5]*/, uint64_t* hash) {
  for (int py = y0; py <= y1; ++py)
    for (int px = x0; px <= x1; ++px) {
      PixelOut o;
      int64_t np = -1;
      pixel_forward(mode, p, L, len, px, py, -1, o, &np);
      const int64_t pix = (int64_t)py * cam->width + px;
      for (int ch = 0; ch < 3; ++ch) img[3 * pix + ch] = o.C[ch];
      if (final_T) final_T[pix] = o.T;
      if (n_contrib) n_contrib[pix] = o.nc;
      if (flags) flags[pix] = o.flagged ? 1 : 0;
      if (alt) {
        if (o.flagged) {
          PixelOut a;
          pixel_forward(mode, p, L, len, px, py, np, a, nullptr);
          for (int ch = 0; ch < 3; ++ch) alt[3 * pix + ch] = a.C[ch];
        } else {
          for (int ch = 0; ch < 3; ++ch) alt[3 * pix + ch] = o.C[ch];
        }
      }
      acc[0] += o.examined; acc[1] += o.skipped; acc[2] += o.blended; acc[3] += o.flagged ? 1 : 0;
      *hash = mix64(*hash, mix64((uint64_t)pix, o.hash));
    }
}

// Reverse-mode pass over one pixel: recompute the forward contributions, then walk them back to front.
//   dC/dalpha_j = T_j (c_j - S_j) - T_final bg / (1 - alpha_j),  S_j = colour composited behind j
//   (S_{j-1} = alpha_j c_j + (1 - alpha_j) S_j);  dC/dc_j = alpha_j T_j.
//   alpha = o G if o G <= 0.99 (else the constant 0.99: zero derivative).
//   PHI: dG/dq = -G/2.  GEF: dG/dq = -(beta/4) q^(beta/2-1) G (q floored at 1e-12),
//        dG/dbeta = -(1/4) q^(beta/2) ln(q) G (0 at q = 0).
//   q = a dx^2 + 2 b dx dy + c dy^2, dx = u - px:  dq/du = 2(a dx + b dy), dq/dv = 2(b dx + c dy),
//   dq/da = dx^2, dq/db = 2 dx dy, dq/dc = dy^2.
// Two decisions of a pixel are taken on floating-point values that a binary32 implementation can
// legitimately take the other way: the termination test t < 1e-4 and the clamp o G > 0.99.  The
// pixel is ambiguous when either lies within kFlagRel (termination, relative) or kClampAbs (clamp)
// of its threshold; for such a pixel the contributions of the other branch of the nearest decision
// are also computed and |other - primary| is accumulated per splat into `delta` (the amount by which
// a correct implementation may differ from the primary result).
struct Contrib { int64_t j; double alpha, T, G, q, dx, dy; bool clamped; };
constexpr double kClampAbs = 1e-5;

struct PixelGrad { int64_t j; double v[10]; };

// Forward walk with optional forced flips; returns the composited pairs and the final transmittance.
double pixel_contribs(int mode, const oc_params* p, const Splat2D* L, int64_t len, int px, int py,
                      int64_t flip_term_at, int64_t flip_clamp_at, std::vector<Contrib>& cs, int64_t* ex_out,
                      double* term_margin, int64_t* term_pos, double* clamp_margin, int64_t* clamp_pos) {
  cs.clear();
  double T = 1.0;
  int64_t ex = 0;
  double tm = 1e300, cm = 1e300;
  int64_t tp = -1, cp = -1;
  for (int64_t j = 0; j < len; ++j) {
    const Splat2D& s = L[j];
    double q, dx, dy;
    ++ex;
    if (!pair_q(mode, s, px, py, q, dx, dy)) continue;
    double G = falloff(p->falloff, q, s.beta);
    double oG = s.o * G;
    bool clamped = oG > kAlphaMax;
    const double cmar = std::fabs(oG - kAlphaMax);
    if (cmar < cm) { cm = cmar; cp = j; }
    if (j == flip_clamp_at) clamped = !clamped;
    double alpha = clamped ? kAlphaMax : oG;
    double t = T * (1.0 - alpha);
    const double tmar = std::fabs(t - kTMin) / kTMin;
    if (tmar < tm) { tm = tmar; tp = j; }
    bool stop = t < kTMin;
    if (j == flip_term_at) stop = !stop;
    if (stop) break;
    cs.push_back(Contrib{j, alpha, T, G, q, dx, dy, clamped});
    T = t;
  }
  if (ex_out) *ex_out += ex;
  if (term_margin) { *term_margin = tm; *term_pos = tp; *clamp_margin = cm; *clamp_pos = cp; }
  return T;
}

void pixel_grads(const oc_params* p, const Splat2D* L, const std::vector<Contrib>& cs, double Tfin, const double g[3],
                 std::vector<PixelGrad>& out) {
  out.clear();
  const double bgg = p->bg[0] * g[0] + p->bg[1] * g[1] + p->bg[2] * g[2];
  double Sb[3] = {0.0, 0.0, 0.0};
  for (int64_t k = (int64_t)cs.size() - 1; k >= 0; --k) {
    const Contrib& c = cs[(size_t)k];
    const Splat2D& s = L[c.j];
    const double col[3] = {s.r, s.g, s.bl};
    double dalpha = 0.0;
    for (int ch = 0; ch < 3; ++ch) dalpha += g[ch] * c.T * (col[ch] - Sb[ch]);
    dalpha -= Tfin * bgg / (1.0 - c.alpha);
    for (int ch = 0; ch < 3; ++ch) Sb[ch] = c.alpha * col[ch] + (1.0 - c.alpha) * Sb[ch];
    double dG = 0.0, dop = 0.0;
    if (!c.clamped) { dG = s.o * dalpha; dop = c.G * dalpha; }
    double q = c.q < 0.0 ? 0.0 : c.q;
    double dq = 0.0, dbeta = 0.0;
    if (p->falloff != OC_FALLOFF_GEF) {
      dq = c.q < 0.0 ? 0.0 : -0.5 * c.G * dG;
    } else {
      double qf = std::max(q, 1e-12);
      dq = c.q < 0.0 ? 0.0 : -0.25 * s.beta * std::pow(qf, 0.5 * s.beta - 1.0) * c.G * dG;
      dbeta = q > 0.0 ? -0.25 * std::pow(q, 0.5 * s.beta) * std::log(q) * c.G * dG : 0.0;
    }
    const double dx = c.dx, dy = c.dy;
    PixelGrad pg;
    pg.j = c.j;
    pg.v[0] = dq * 2.0 * (s.a * dx + s.b * dy);
    pg.v[1] = dq * 2.0 * (s.b * dx + s.c * dy);
    pg.v[2] = dq * dx * dx;
    pg.v[3] = dq * 2.0 * dx * dy;
    pg.v[4] = dq * dy * dy;
    pg.v[5] = dop;
    pg.v[6] = c.alpha * c.T * g[0];
    pg.v[7] = c.alpha * c.T * g[1];
    pg.v[8] = c.alpha * c.T * g[2];
    pg.v[9] = dbeta;
    out.push_back(pg);
  }
}

// ------------------------------------------------------------------------------------------------
// Rounding-error bound of one pixel's terms in a binary32 implementation.
//
// The GPU evaluates each composited pair's contributions (the ten terms of pixel_grads) in binary32,
// with hardware exp2/log2/reciprocal, and recovers the transmittance back to front by division from
// the stored binary32 final transmittance.  The amount by which such an evaluation may differ from the
// binary64 terms above is bounded here by first-order running error analysis (Wilkinson; Higham,
// "Accuracy and Stability of Numerical Algorithms", 2nd ed., Sec. 3.3): every computed quantity x
// carries an absolute bound E(x), propagated by
//     E(a +- b) = E(a) + E(b) + u|a +- b|,   E(a b) = |a| E(b) + |b| E(a) + u|a b|,
//     E(f(x))   = |f'(x)| E(x) + e_f |f(x)|  for f in {exp2, log2, 1/x},
// with u = 2^-24 (binary32 round to nearest) and e_f = 2u (one ulp).  The model of the implementation:
//   * the record fields, dx, dy and q are binary32 values shared bit for bit with the oracle (exact);
//   * G = exp2(x) with x a rounded product of q (PHI) or of q^(beta/2) = exp2((beta/2) log2 q) (GEF)
//     by -log2(e)/2; log2 within one ulp of its result or 2u absolute where the result is below 1;
//   * alpha = o G rounded, or the binary32 constant 0.99 when clamped (|0.99f - 0.99| absolute);
//   * T: forward product T (1 - alpha) rounded per step, stored in binary32, then recovered back to
//     front by T / (1 - alpha) through a reciprocal and a product (covers any forward recomputation too);
//   * S (colour behind): S + alpha (c - S) or alpha c + (1 - alpha) S per step, each rounding at most
//     4u (|c| + |S|);
//   * each term is a product of those quantities with a few rounded operations, counted per term.
// Decisions (alpha floor, clamp, termination) are the oracle's; their ambiguity is `delta`'s business.
// The summation over a tile's pixels is not included: its bound depends on the summation order and is
// gamma * sum |terms| (`mass`).
// ------------------------------------------------------------------------------------------------
constexpr double kU = 0x1p-24;
constexpr double kUlp = 2.0 * kU;
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLog2e = 1.44269504088896340736;

inline double log2_abs_err(double l) { return kUlp * std::max(std::fabs(l), 1.0); }

struct TermBound { int64_t j; double e[10]; };

void pixel_error_bounds(const oc_params* p, const Splat2D* L, const std::vector<Contrib>& cs, double Tfin,
                        const double g[3], std::vector<TermBound>& out) {
  out.clear();
  const size_t m = cs.size();
  if (m == 0) return;
  const bool gef = p->falloff == OC_FALLOFF_GEF;
  const double clampErr = std::fabs(0.99 - (double)0.99f);
  // per contribution: relative error of G, absolute error of alpha and of (1 - alpha)
  std::vector<double> eG(m), Ea(m), Eom(m), Ef(m + 1), Eb(m + 1);
  std::vector<double> eqb(m, 0.0), El(m, 0.0);
  for (size_t k = 0; k < m; ++k) {
    const Contrib& c = cs[k];
    const Splat2D& s = L[c.j];
    const double q = c.q < 0.0 ? 0.0 : c.q;
    if (!gef) {
      // x = (-log2e/2) q: the constant and the product round (2u |x|), exp2 adds one ulp
      const double x = 0.5 * kLog2e * q;
      eG[k] = kLn2 * 2.0 * kU * x + kUlp;
    } else if (q > 0.0) {
      const double l = std::log2(q);
      El[k] = log2_abs_err(l);
      const double arg = 0.5 * s.beta * l;
      const double Earg = 0.5 * s.beta * El[k] + 2.0 * kU * std::fabs(arg);
      eqb[k] = kLn2 * Earg + kUlp;
      const double qb = std::exp2(arg);
      const double x = 0.5 * kLog2e * qb;
      eG[k] = kLn2 * x * (eqb[k] + 2.0 * kU) + kUlp;
    } else {
      eG[k] = 0.0;   // q = 0: G = exp2(0) = 1 exactly
    }
    Ea[k] = c.clamped ? clampErr : c.alpha * (eG[k] + kU);
    Eom[k] = Ea[k] + kU * (1.0 - c.alpha);
  }
  // forward transmittance, then the stored value and its recovery back to front
  Ef[0] = 0.0;
  for (size_t k = 0; k < m; ++k) {
    const double Tn = cs[k].T * (1.0 - cs[k].alpha);
    Ef[k + 1] = Ef[k] * (1.0 - cs[k].alpha) + cs[k].T * Eom[k] + kU * Tn;
  }
  Eb[m] = Ef[m] + kU * Tfin;
  for (size_t kk = m; kk-- > 0;) {
    const double om = 1.0 - cs[kk].alpha;
    const double Tn = cs[kk].T * om;
    Eb[kk] = Eb[kk + 1] / om + Tn * Eom[kk] / (om * om) + 3.0 * kU * cs[kk].T;
  }
  const double bgg = p->bg[0] * g[0] + p->bg[1] * g[1] + p->bg[2] * g[2];
  const double bgabs = std::fabs(p->bg[0] * g[0]) + std::fabs(p->bg[1] * g[1]) + std::fabs(p->bg[2] * g[2]);
  double S[3] = {0.0, 0.0, 0.0}, ES[3] = {0.0, 0.0, 0.0};
  for (size_t kk = m; kk-- > 0;) {
    const Contrib& c = cs[kk];
    const Splat2D& s = L[c.j];
    const double col[3] = {s.r, s.g, s.bl};
    const double om = 1.0 - c.alpha;
    const double T = c.T, ET = Eb[kk];
    TermBound tb;
    tb.j = c.j;
    for (int i = 0; i < 10; ++i) tb.e[i] = 0.0;
    // dL/dalpha = sum_ch g T (c - S) - Tfin bgg / (1 - alpha)
    double D = 0.0, ED = 0.0, absSum = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
      D += g[ch] * T * (col[ch] - S[ch]);
      ED += std::fabs(g[ch]) * (T * ES[ch] + std::fabs(col[ch] - S[ch]) * ET);
      absSum += std::fabs(g[ch]) * (std::fabs(col[ch]) + std::fabs(S[ch]));
    }
    ED += 5.0 * kU * T * absSum;
    const double bp = Tfin * bgg / om;
    ED += bgabs * (Eb[m] / om + Tfin * Eom[kk] / (om * om) + 6.0 * kU * Tfin / om);
    D -= bp;
    ED += kU * std::fabs(D);
    // colour: alpha T g
    for (int ch = 0; ch < 3; ++ch) {
      const double v = c.alpha * T * g[ch];
      tb.e[6 + ch] = std::fabs(g[ch]) * (c.alpha * ET + T * Ea[kk]) + 2.0 * kU * std::fabs(v);
    }
    if (!c.clamped) {
      const double G = c.G;
      const double gd = G * D;
      const double Egd = G * ED + std::fabs(D) * G * eG[kk] + kU * std::fabs(gd);
      tb.e[5] = Egd;
      const double q = c.q < 0.0 ? 0.0 : c.q;
      double dq = 0.0, Edq = 0.0;
      if (c.q < 0.0) {
        // q rounded below 0 at the centre: no dL/dq term on either side
      } else if (!gef) {
        dq = -0.5 * s.o * gd;
        Edq = 0.5 * s.o * Egd + 2.0 * kU * std::fabs(dq);
      } else {
        const double qf = std::max(q, 1e-12);
        const double lf = std::log2(qf);
        const double arg2 = (0.5 * s.beta - 1.0) * lf;
        const double Earg2 = std::fabs(0.5 * s.beta - 1.0) * log2_abs_err(lf) + 2.0 * kU * std::fabs(arg2);
        const double qpow = std::exp2(arg2);
        const double eqpow = kLn2 * Earg2 + kUlp;
        dq = -0.25 * s.beta * qpow * s.o * gd;
        Edq = 0.25 * s.beta * s.o * (qpow * Egd + std::fabs(gd) * qpow * eqpow) + 3.0 * kU * std::fabs(dq);
        if (q > 0.0) {
          const double l = std::log2(q);
          const double qb = std::exp2(0.5 * s.beta * l);
          const double w = qb * l;
          const double Ew = std::fabs(l) * qb * eqb[kk] + qb * El[kk] + kU * std::fabs(w);
          const double v9 = 0.25 * kLn2 * s.o * w * gd;
          tb.e[9] = 0.25 * kLn2 * s.o * (std::fabs(w) * Egd + std::fabs(gd) * Ew) + 3.0 * kU * std::fabs(v9);
        }
      }
      (void)dq;
      const double dx = c.dx, dy = c.dy;
      const double hu = s.a * dx + s.b * dy, hv = s.b * dx + s.c * dy;
      const double Ehu = 2.0 * kU * (std::fabs(s.a * dx) + std::fabs(s.b * dy));
      const double Ehv = 2.0 * kU * (std::fabs(s.b * dx) + std::fabs(s.c * dy));
      const double adq = std::fabs(dq);
      tb.e[0] = 2.0 * (std::fabs(hu) * Edq + adq * Ehu) + kU * 2.0 * adq * std::fabs(hu);
      tb.e[1] = 2.0 * (std::fabs(hv) * Edq + adq * Ehv) + kU * 2.0 * adq * std::fabs(hv);
      tb.e[2] = dx * dx * Edq + 2.0 * kU * adq * dx * dx;
      tb.e[3] = 2.0 * std::fabs(dx * dy) * Edq + 2.0 * kU * 2.0 * adq * std::fabs(dx * dy);
      tb.e[4] = dy * dy * Edq + 2.0 * kU * adq * dy * dy;
    }
    out.push_back(tb);
    // S <- alpha c + (1 - alpha) S
    for (int ch = 0; ch < 3; ++ch) {
      const double Sn = c.alpha * col[ch] + om * S[ch];
      ES[ch] = om * ES[ch] + std::fabs(col[ch] - S[ch]) * Ea[kk] + 4.0 * kU * (std::fabs(col[ch]) + std::fabs(S[ch]));
      S[ch] = Sn;
    }
  }
}

void pixel_backward(int mode, const oc_params* p, const Splat2D* L, const uint32_t* ids, int64_t len, int px,
                    int py, const double g[3], double* g2d, double* delta, double* mass, double* ebound,
                    int64_t* examined) {
  std::vector<Contrib> cs;
  std::vector<PixelGrad> prim, alt;
  double tm, cm;
  int64_t tp, cp;
  const double Tfin = pixel_contribs(mode, p, L, len, px, py, -1, -1, cs, examined, &tm, &tp, &cm, &cp);
  pixel_grads(p, L, cs, Tfin, g, prim);
  for (const PixelGrad& pg : prim) {
    double* gs = g2d + 10 * (int64_t)ids[pg.j];
    for (int k = 0; k < 10; ++k) {
#pragma omp atomic
      gs[k] += pg.v[k];
    }
    if (mass) {
      double* ms = mass + 10 * (int64_t)ids[pg.j];
      for (int k = 0; k < 10; ++k) {
        const double a = std::fabs(pg.v[k]);
#pragma omp atomic
        ms[k] += a;
      }
    }
  }
  if (ebound) {
    std::vector<TermBound> eb;
    pixel_error_bounds(p, L, cs, Tfin, g, eb);
    for (const TermBound& tb : eb) {
      double* es = ebound + 10 * (int64_t)ids[tb.j];
      for (int k = 0; k < 10; ++k) {
#pragma omp atomic
        es[k] += tb.e[k];
      }
    }
  }
  if (!delta) return;
  const bool term_amb = tm < kFlagRel, clamp_amb = cm < kClampAbs;
  if (!term_amb && !clamp_amb) return;
  // the other branch of the nearer decision
  const bool use_term = term_amb && (!clamp_amb || tm * kTMin <= cm);
  const double Tf2 = pixel_contribs(mode, p, L, len, px, py, use_term ? tp : -1, use_term ? -1 : cp, cs, nullptr,
                                    nullptr, nullptr, nullptr, nullptr);
  pixel_grads(p, L, cs, Tf2, g, alt);
  // |alt - prim| per splat: accumulate both lists keyed by list position
  std::vector<std::pair<int64_t, std::array<double, 10>>> acc;
  auto add = [&](const std::vector<PixelGrad>& v, double sgn) {
    for (const PixelGrad& pg : v) {
      size_t k = 0;
      while (k < acc.size() && acc[k].first != pg.j) ++k;
      if (k == acc.size()) { acc.push_back({pg.j, {}}); acc.back().second.fill(0.0); }
      for (int c = 0; c < 10; ++c) acc[k].second[(size_t)c] += sgn * pg.v[c];
    }
  };
  add(alt, 1.0);
  add(prim, -1.0);
  for (const auto& e : acc) {
    double* ds = delta + 10 * (int64_t)ids[e.first];
    for (int c = 0; c < 10; ++c) {
      const double d = std::fabs(e.second[(size_t)c]);
#pragma omp atomic
      ds[c] += d;
    }
  }
}

void gather_list(const oc_record* r, const uint32_t* ids, int64_t len, std::vector<Splat2D>& L) {
  L.resize((size_t)len);
  for (int64_t j = 0; j < len; ++j) load_splat(r, ids[j], L[(size_t)j]);
}

}  // namespace

// ================================================================================================
extern "C" {

void oc_exp_c(const float* x, float* y, int64_t n) {
  for (int64_t i = 0; i < n; ++i) y[i] = exp_c(x[i]);
}
void oc_lgamma_c(const float* x, float* y, int64_t n) {
  for (int64_t i = 0; i < n; ++i) y[i] = lgamma_c(x[i]);
}
void oc_log_c(const float* x, float* y, int64_t n) {
  for (int64_t i = 0; i < n; ++i) y[i] = log_c(x[i]);
}

int oc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oc_preprocess(int mode, const oc_splats* s, const oc_camera* cam, const oc_params* p, oc_record* out) {
  if (!s || !cam || !p || !out || s->n < 0 || s->sh_degree < 0 || s->sh_degree > 3) return -1;
  if (mode == OC_MODE_F32) preprocess_all<float>(s, cam, p, out);
  else if (mode == OC_MODE_F64) preprocess_all<double>(s, cam, p, out);
  else return -1;
  return 0;
}

int oc_splat_in_tile(int mode, const oc_record* r, int64_t i, const oc_camera* cam, const oc_params* p,
                     int32_t tx, int32_t ty) {
  return in_tile(mode, r, i, cam, p, tx, ty) ? 1 : 0;
}

int oc_tile_counts(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                   int64_t* counts) {
  const int TX = tiles_x(cam), TY = tiles_y(cam);
  std::memset(counts, 0, sizeof(int64_t) * (size_t)TX * TY);
  for (int64_t i = 0; i < n; ++i) {
    if (r->tiles_touched[i] == 0) continue;
    const int32_t* rc = r->rect + 4 * i;
    for (int ty = rc[1]; ty <= rc[3]; ++ty)
      for (int tx = rc[0]; tx <= rc[2]; ++tx)
        if (in_tile(mode, r, i, cam, p, tx, ty)) counts[(int64_t)ty * TX + tx] += 1;
  }
  return 0;
}

int oc_build_keys(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                  uint64_t* keys, uint32_t* values, int64_t num_keys, int64_t* ranges) {
  const int TX = tiles_x(cam), TY = tiles_y(cam);
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (r->tiles_touched[i] == 0) continue;
    const int32_t* rc = r->rect + 4 * i;
    const uint32_t dbits = [&] { float f = (float)r->depth[i]; uint32_t b; std::memcpy(&b, &f, 4); return b; }();
    for (int ty = rc[1]; ty <= rc[3]; ++ty)
      for (int tx = rc[0]; tx <= rc[2]; ++tx) {
        if (!in_tile(mode, r, i, cam, p, tx, ty)) continue;
        if (k >= num_keys) return -2;
        keys[k] = ((uint64_t)((int64_t)ty * TX + tx) << 32) | dbits;
        values[k] = (uint32_t)i;
        ++k;
      }
  }
  if (k != num_keys) return -3;
  // stable sort by key: ties (equal tile and depth bits) keep splat-index order
  std::vector<int64_t> perm((size_t)num_keys);
  for (int64_t j = 0; j < num_keys; ++j) perm[(size_t)j] = j;
  std::stable_sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) { return keys[x] < keys[y]; });
  std::vector<uint64_t> k2((size_t)num_keys);
  std::vector<uint32_t> v2((size_t)num_keys);
  for (int64_t j = 0; j < num_keys; ++j) { k2[(size_t)j] = keys[perm[(size_t)j]]; v2[(size_t)j] = values[perm[(size_t)j]]; }
  std::memcpy(keys, k2.data(), sizeof(uint64_t) * (size_t)num_keys);
  std::memcpy(values, v2.data(), sizeof(uint32_t) * (size_t)num_keys);
  const int64_t T = (int64_t)TX * TY;
  for (int64_t t = 0; t < 2 * T; ++t) ranges[t] = 0;
  for (int64_t j = 0; j < num_keys; ++j) {
    int64_t t = (int64_t)(keys[j] >> 32);
    if (j == 0 || (int64_t)(keys[j - 1] >> 32) != t) ranges[2 * t] = j;
    if (j == num_keys - 1 || (int64_t)(keys[j + 1] >> 32) != t) ranges[2 * t + 1] = j + 1;
  }
  return 0;
}

int oc_tile_list(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                 int32_t tile, uint32_t* out, int64_t cap, int64_t* len) {
  const int TX = tiles_x(cam);
  const int tx = tile % TX, ty = tile / TX;
  std::vector<uint32_t> ids;
  for (int64_t i = 0; i < n; ++i)
    if (in_tile(mode, r, i, cam, p, tx, ty)) ids.push_back((uint32_t)i);
  std::stable_sort(ids.begin(), ids.end(), [&](uint32_t x, uint32_t y) {
    float a = (float)r->depth[x], b = (float)r->depth[y];
    if (mode == OC_MODE_F64) return r->depth[x] < r->depth[y];
    return a < b;
  });
  *len = (int64_t)ids.size();
  for (int64_t j = 0; j < (int64_t)ids.size() && j < cap; ++j) out[j] = ids[(size_t)j];
  return 0;
}

int oc_render(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
              const uint32_t* values, const int64_t* ranges, const int32_t* tiles, int64_t n_tiles,
              double* img, double* final_T, int32_t* n_contrib, uint8_t* flags, double* alt, oc_stats* stats) {
  (void)n;
  const int TX = tiles_x(cam), TY = tiles_y(cam);
  const int64_t nt = tiles ? n_tiles : (int64_t)TX * TY;
  int64_t tot[5] = {0, 0, 0, 0, 0};
  uint64_t hash = 0;
#pragma omp parallel
  {
    int64_t acc[5] = {0, 0, 0, 0, 0};
    uint64_t h = 0;
    std::vector<Splat2D> L;
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < nt; ++k) {
      const int64_t t = tiles ? tiles[k] : k;
      const int tx = (int)(t % TX), ty = (int)(t / TX);
      const int64_t s0 = ranges[2 * t], s1 = ranges[2 * t + 1];
      gather_list(r, values + s0, s1 - s0, L);
      const int x0 = tx * OC_TILE, y0 = ty * OC_TILE;
      const int x1 = std::min(x0 + OC_TILE, cam->width) - 1, y1 = std::min(y0 + OC_TILE, cam->height) - 1;
      uint64_t ht = 0;
      render_list(mode, cam, p, L.data(), s1 - s0, x0, y0, x1, y1, img, final_T, n_contrib, flags, alt, acc, &ht);
      h += mix64((uint64_t)t, ht);   // order-independent combination across tiles
    }
#pragma omp critical
    {
      for (int i = 0; i < 5; ++i) tot[i] += acc[i];
      hash += h;
    }
  }
  (void)TY;
  if (stats) {
    stats->pairs_examined = tot[0]; stats->pairs_skipped = tot[1]; stats->pairs_blended = tot[2];
    stats->pixels_flagged = tot[3]; stats->decision_hash = hash;
  }
  return 0;
}

int oc_render_untiled(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                      double* img, double* final_T, int32_t* n_contrib, uint8_t* flags, double* alt,
                      oc_stats* stats) {
  std::vector<uint32_t> ids;
  for (int64_t i = 0; i < n; ++i)
    if (r->tiles_touched[i] > 0) ids.push_back((uint32_t)i);
  std::stable_sort(ids.begin(), ids.end(), [&](uint32_t x, uint32_t y) {
    if (mode == OC_MODE_F64) return r->depth[x] < r->depth[y];
    return (float)r->depth[x] < (float)r->depth[y];
  });
  std::vector<Splat2D> L;
  gather_list(r, ids.data(), (int64_t)ids.size(), L);
  int64_t tot[5] = {0, 0, 0, 0, 0};
  uint64_t hash = 0;
#pragma omp parallel
  {
    int64_t acc[5] = {0, 0, 0, 0, 0};
    uint64_t h = 0;
#pragma omp for schedule(dynamic, 1)
    for (int py = 0; py < cam->height; ++py) {
      uint64_t hr = 0;
      render_list(mode, cam, p, L.data(), (int64_t)L.size(), 0, py, cam->width - 1, py, img, final_T, n_contrib,
                  flags, alt, acc, &hr);
      h += mix64((uint64_t)py, hr);
    }
#pragma omp critical
    {
      for (int i = 0; i < 5; ++i) tot[i] += acc[i];
      hash += h;
    }
  }
  if (stats) {
    stats->pairs_examined = tot[0]; stats->pairs_skipped = tot[1]; stats->pairs_blended = tot[2];
    stats->pixels_flagged = tot[3]; stats->decision_hash = hash;
  }
  return 0;
}

int oc_backward_untiled(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                        const double* dL_dimg, double* g2d, double* delta, double* mass, double* ebound,
                        oc_stats* stats) {
  std::vector<uint32_t> ids;
  for (int64_t i = 0; i < n; ++i)
    if (r->tiles_touched[i] > 0) ids.push_back((uint32_t)i);
  std::stable_sort(ids.begin(), ids.end(), [&](uint32_t x, uint32_t y) {
    if (mode == OC_MODE_F64) return r->depth[x] < r->depth[y];
    return (float)r->depth[x] < (float)r->depth[y];
  });
  std::vector<Splat2D> L;
  gather_list(r, ids.data(), (int64_t)ids.size(), L);
  int64_t tot = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tot)
  for (int py = 0; py < cam->height; ++py)
    for (int px = 0; px < cam->width; ++px) {
      const int64_t pix = (int64_t)py * cam->width + px;
      pixel_backward(mode, p, L.data(), ids.data(), (int64_t)L.size(), px, py, dL_dimg + 3 * pix, g2d, delta, mass,
                     ebound, &tot);
    }
  if (stats) { std::memset(stats, 0, sizeof(*stats)); stats->pairs_examined = tot; }
  return 0;
}

int oc_backward(int mode, const oc_record* r, int64_t n, const oc_camera* cam, const oc_params* p,
                const uint32_t* values, const int64_t* ranges, const int32_t* tiles, int64_t n_tiles,
                const double* dL_dimg, double* g2d, double* delta, double* mass, double* ebound, oc_stats* stats) {
  (void)n;
  const int TX = tiles_x(cam), TY = tiles_y(cam);
  const int64_t nt = tiles ? n_tiles : (int64_t)TX * TY;
  int64_t tot = 0;
#pragma omp parallel
  {
    int64_t ex = 0;
    std::vector<Splat2D> L;
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < nt; ++k) {
      const int64_t t = tiles ? tiles[k] : k;
      const int tx = (int)(t % TX), ty = (int)(t / TX);
      const int64_t s0 = ranges[2 * t], s1 = ranges[2 * t + 1];
      gather_list(r, values + s0, s1 - s0, L);
      const int x0 = tx * OC_TILE, y0 = ty * OC_TILE;
      const int x1 = std::min(x0 + OC_TILE, cam->width) - 1, y1 = std::min(y0 + OC_TILE, cam->height) - 1;
      for (int py = y0; py <= y1; ++py)
        for (int px = x0; px <= x1; ++px) {
          const int64_t pix = (int64_t)py * cam->width + px;
          pixel_backward(mode, p, L.data(), values + s0, s1 - s0, px, py, dL_dimg + 3 * pix, g2d, delta, mass,
                         ebound, &ex);
        }
    }
#pragma omp critical
    tot += ex;
  }
  (void)TY;
  if (stats) { std::memset(stats, 0, sizeof(*stats)); stats->pairs_examined = tot; }
  return 0;
}

}  // extern "C"
