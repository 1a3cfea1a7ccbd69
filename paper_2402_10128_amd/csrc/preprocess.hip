// preprocess.hip -- per-splat projection of GES splats (forward) and its chain rule (backward).
//
// Forward (GES Sec. 4.1-4.2), one thread per splat, binary32 with a fixed operation order (this file
// is compiled with -ffp-contract=off; correctly rounded division and square root):
//   p = W mu + t;  s = exp(log s);  o = sigmoid(logit);  R = R(q/|q|)
//   PHI: S = phi_rho(beta) s with phi_rho(beta) = 2 / (1 + exp(-(rho beta - 2 rho)))   (Eq. approx)
//   Sigma = (R S)(R S)^T;  Sigma' = J W Sigma W^T J^T + 0.3 I  (EWA, J guard-clamped)
//   conic = Sigma'^-1;  mean2D = (fx x/z + cx, fy y/z + cy)
//   q_max: alpha >= 1/255 <=> q <= q_max; PHI q_max = 2 ln(255 o), GEF q_max = (2 ln(255 o))^(2/beta)
//   radius = 1 + ceil(sqrt(q_max lambda_max(Sigma'))); tile rectangle of the pixel centres within
//   the radius square; tiles_touched (SQUARE: the rectangle, ELLIPSE: tiles meeting the ellipse)
//   colour = sum_k Y_k(dir) c_k + 0.5 clamped at 0 (real SH, degree <= 3).
// Memory: coalesced per-wave reads of the 64 splats' parameters; one 64-byte record per splat.
#include "canon_math.h"
#include "ges_internal.h"
#include "tile_geom.h"

namespace ges {

__device__ __forceinline__ float max_c(float a, float b) { return geom_max(a, b); }
__device__ __forceinline__ float min_c(float a, float b) { return geom_min(a, b); }

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

__device__ __forceinline__ void write_culled(float4* rec, int64_t i) {
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  rec[4 * i + 0] = z;
  rec[4 * i + 1] = z;
  rec[4 * i + 2] = z;
  rec[4 * i + 3] = z;
}

__device__ __forceinline__ bool finite3(const float* p) {
  return __builtin_isfinite(p[0]) && __builtin_isfinite(p[1]) && __builtin_isfinite(p[2]);
}

__global__ void __launch_bounds__(256) preprocess_kernel(const DeviceBatch* __restrict__ db) {
  const int64_t blk = blockIdx.x;
  const int v = view_of_block(db->pre_prefix, db->nviews, blk);
  const ViewDesc& V = db->views[v];
  const int64_t i = (blk - db->pre_prefix[v]) * 256 + threadIdx.x;
  if (i >= V.n) return;
  float4* rec = V.rec;
  const int K = V.sh_coeffs;
  const float* mu = V.means + 3 * i;
  const float* ls = V.log_scales + 3 * i;
  const float4 qv = reinterpret_cast<const float4*>(V.quats)[i];
  const float logit = V.logits[i];
  const float beta = V.beta[i];
  const float* shc = V.sh + (int64_t)3 * K * i;
  const float mx = mu[0], my = mu[1], mz = mu[2];
  const float l0 = ls[0], l1 = ls[1], l2 = ls[2];

  bool ok = finite3(mu) && finite3(ls) && __builtin_isfinite(qv.x) && __builtin_isfinite(qv.y) &&
            __builtin_isfinite(qv.z) && __builtin_isfinite(qv.w) && __builtin_isfinite(logit) &&
            __builtin_isfinite(beta);
  float shv[48];
  for (int k = 0; k < 3 * K; ++k) {
    shv[k] = shc[k];
    ok = ok && __builtin_isfinite(shv[k]);
  }
  if (!ok) { write_culled(rec, i); return; }

  // 1. camera-space position
  float p[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    float acc = V.R[3 * r] * mx;
    acc = acc + V.R[3 * r + 1] * my;
    acc = acc + V.R[3 * r + 2] * mz;
    p[r] = acc + V.t[r];
  }
  const float z = p[2];
  if (!(z > V.near_z)) { write_culled(rec, i); return; }

  // 2. activations
  const float s0 = canon_exp(l0), s1 = canon_exp(l1), s2 = canon_exp(l2);
  const float en = canon_exp(-logit);
  const float den = 1.0f + en;
  const float op = 1.0f / den;
  const float o255 = 255.0f * op;
  if (!(o255 > 1.0f)) { write_culled(rec, i); return; }

  // 3. quaternion -> rotation
  float qw = qv.x, qx = qv.y, qy = qv.z, qz = qv.w;
  float nn = qw * qw; nn = nn + qx * qx; nn = nn + qy * qy; nn = nn + qz * qz;
  if (!(nn > 0.0f)) { write_culled(rec, i); return; }
  const float nr = __builtin_sqrtf(nn);
  qw = qw / nr; qx = qx / nr; qy = qy / nr; qz = qz / nr;
  float Q[9];
  {
    float t;
    t = qy * qy; t = t + qz * qz; t = 2.0f * t; Q[0] = 1.0f - t;
    t = qx * qy; t = t - qw * qz; Q[1] = 2.0f * t;
    t = qx * qz; t = t + qw * qy; Q[2] = 2.0f * t;
    t = qx * qy; t = t + qw * qz; Q[3] = 2.0f * t;
    t = qx * qx; t = t + qz * qz; t = 2.0f * t; Q[4] = 1.0f - t;
    t = qy * qz; t = t - qw * qx; Q[5] = 2.0f * t;
    t = qx * qz; t = t - qw * qy; Q[6] = 2.0f * t;
    t = qy * qz; t = t + qw * qx; Q[7] = 2.0f * t;
    t = qx * qx; t = t + qy * qy; t = 2.0f * t; Q[8] = 1.0f - t;
  }

  // 4. shape modification
  float phi;
  if (V.falloff == GES_FALLOFF_PHI) {
    float t = V.rho * beta;
    float r2 = 2.0f * V.rho;
    t = t - r2;
    float e = canon_exp(-t);
    float d = 1.0f + e;
    phi = 2.0f / d;
  } else {
    if (!(beta > 0.0f)) { write_culled(rec, i); return; }
    phi = 1.0f;
  }
  const float sc[3] = {phi * s0, phi * s1, phi * s2};

  // 5. Sigma = (R S)(R S)^T
  float Mm[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Mm[3 * r + c] = Q[3 * r + c] * sc[c];
  float Sig[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = r; c < 3; ++c) {
      float acc = Mm[3 * r] * Mm[3 * c];
      acc = acc + Mm[3 * r + 1] * Mm[3 * c + 1];
      acc = acc + Mm[3 * r + 2] * Mm[3 * c + 2];
      Sig[3 * r + c] = acc;
      Sig[3 * c + r] = acc;
    }

  // 6. EWA projection
  const float fx = V.fx, fy = V.fy;
  float txz = p[0] / z, tyz = p[1] / z;
  uint32_t bits = 0;
  if (txz < -V.limx) { txz = -V.limx; bits |= 8; } else if (txz > V.limx) { txz = V.limx; bits |= 8; }
  if (tyz < -V.limy) { tyz = -V.limy; bits |= 16; } else if (tyz > V.limy) { tyz = V.limy; bits |= 16; }
  const float xc = txz * z, yc = tyz * z;
  const float z2 = z * z;
  const float J00 = fx / z, J11 = fy / z;
  float J02 = fx * xc; J02 = J02 / z2; J02 = -J02;
  float J12 = fy * yc; J12 = J12 / z2; J12 = -J12;
  float T[6];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float a0 = J00 * V.R[c];
    T[c] = a0 + J02 * V.R[6 + c];
    float a1 = J11 * V.R[3 + c];
    T[3 + c] = a1 + J12 * V.R[6 + c];
  }
  float U[6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float acc = T[3 * r] * Sig[c];
      acc = acc + T[3 * r + 1] * Sig[3 + c];
      acc = acc + T[3 * r + 2] * Sig[6 + c];
      U[3 * r + c] = acc;
    }
  float cv0, cv1, cv2;
  {
    float acc = U[0] * T[0]; acc = acc + U[1] * T[1]; acc = acc + U[2] * T[2]; cv0 = acc;
    acc = U[0] * T[3]; acc = acc + U[1] * T[4]; acc = acc + U[2] * T[5]; cv1 = acc;
    acc = U[3] * T[3]; acc = acc + U[4] * T[4]; acc = acc + U[5] * T[5]; cv2 = acc;
  }
  cv0 = cv0 + 0.3f;
  cv2 = cv2 + 0.3f;
  float det = cv0 * cv2;
  det = det - cv1 * cv1;
  if (!(det > 0.0f)) { write_culled(rec, i); return; }
  const float ca = cv2 / det;
  float cb = cv1 / det; cb = -cb;
  const float cc = cv0 / det;

  // 7. mean2D
  float u = fx * p[0]; u = u / z; u = u + V.cx;
  float vv = fy * p[1]; vv = vv / z; vv = vv + V.cy;

  // 8. alpha-floor threshold
  float L2 = canon_log(o255);
  L2 = 2.0f * L2;
  float qm;
  if (V.falloff == GES_FALLOFF_PHI) {
    qm = L2;
  } else {
    float e = 2.0f / beta;
    float lgl = canon_log(L2);
    e = e * lgl;
    qm = canon_exp(e);
  }
  if (!__builtin_isfinite(qm)) { write_culled(rec, i); return; }

  // 9. radius
  float mid = cv0 + cv2; mid = 0.5f * mid;
  float disc = mid * mid; disc = disc - det;
  disc = max_c(0.0f, disc);
  const float lam = mid + __builtin_sqrtf(disc);
  float rr = qm * lam;
  rr = __builtin_sqrtf(rr);
  rr = __builtin_ceilf(rr);
  if (!(rr <= 1048576.0f)) rr = 1048576.0f;
  const int radius = 1 + (int)rr;
  const float fr = (float)radius;

  // 10. tile rectangle over pixel centres
  float xl = u - fr; xl = __builtin_ceilf(xl);
  float xh = u + fr; xh = __builtin_floorf(xh);
  float yl = vv - fr; yl = __builtin_ceilf(yl);
  float yh = vv + fr; yh = __builtin_floorf(yh);
  xl = max_c(xl, 0.0f); xh = min_c(xh, (float)(V.width - 1));
  yl = max_c(yl, 0.0f); yh = min_c(yh, (float)(V.height - 1));
  if (!(xl <= xh) || !(yl <= yh)) { write_culled(rec, i); return; }
  const int tx0 = (int)xl / kTile, tx1 = (int)xh / kTile;
  const int ty0 = (int)yl / kTile, ty1 = (int)yh / kTile;
  uint32_t touched = 0;
  if (V.tile_cull == GES_TILES_SQUARE) {
    touched = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
  } else {
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx)
        touched += ellipse_hits_tile(u, vv, ca, cb, cc, qm, tx, ty, V.width, V.height) ? 1u : 0u;
  }
  if (touched == 0) { write_culled(rec, i); return; }

  // 11. colour
  float d0 = mx - V.campos[0], d1 = my - V.campos[1], d2 = mz - V.campos[2];
  float len = d0 * d0; len = len + d1 * d1; len = len + d2 * d2;
  len = __builtin_sqrtf(len);
  const float dx = d0 / len, dy = d1 / len, dz = d2 / len;
  float Y[16];
  sh_basis(dx, dy, dz, V.sh_degree, Y);
  float rgb[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = Y[0] * shv[ch];
    for (int k = 1; k < K; ++k) acc = acc + Y[k] * shv[3 * k + ch];
    acc = acc + 0.5f;
    if (acc < 0.0f) { acc = 0.0f; bits |= (1u << ch); }
    rgb[ch] = acc;
  }

  rec[4 * i + 0] = make_float4(u, vv, ca, cb);
  rec[4 * i + 1] = make_float4(cc, qm, op, beta);
  rec[4 * i + 2] = make_float4(rgb[0], rgb[1], rgb[2], z);
  rec[4 * i + 3] = make_float4(__int_as_float((int)((uint32_t)radius | (bits << 24))),
                               __uint_as_float((uint32_t)tx0 | ((uint32_t)ty0 << 16)),
                               __uint_as_float((uint32_t)tx1 | ((uint32_t)ty1 << 16)), __uint_as_float(touched));
}

// ------------------------------------------------------------------------------------------------
// Backward: per splat, the chain rule from the accumulated 2-D gradients (u, v, conic a/b/c, opacity,
// colour, beta) to mean, log-scale, quaternion, opacity logit, SH coefficients and beta.
// Forward quantities are recomputed in binary32 (decisions -- culling, guard clamp, colour clamp --
// come from the record).  Culled splats get zero gradients.
// ------------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) preprocess_backward_kernel(const DeviceBatch* __restrict__ db,
                                                                   ges_splat_grads G) {
  const int64_t blk = blockIdx.x;
  const int v = view_of_block(db->pre_prefix, db->nviews, blk);
  const ViewDesc& V = db->views[v];
  const int64_t i = (blk - db->pre_prefix[v]) * 256 + threadIdx.x;
  if (i >= V.n) return;
  const int K = V.sh_coeffs;
  const float4 r3 = V.rec[4 * i + 3];
  const uint32_t touched = __float_as_uint(r3.w);
  if (touched == 0) {
    if (G.means) { G.means[3 * i] = 0.f; G.means[3 * i + 1] = 0.f; G.means[3 * i + 2] = 0.f; }
    if (G.log_scales) { G.log_scales[3 * i] = 0.f; G.log_scales[3 * i + 1] = 0.f; G.log_scales[3 * i + 2] = 0.f; }
    if (G.quats) reinterpret_cast<float4*>(G.quats)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (G.opacity_logits) G.opacity_logits[i] = 0.f;
    if (G.sh) for (int k = 0; k < 3 * K; ++k) G.sh[(int64_t)3 * K * i + k] = 0.f;
    if (G.beta) G.beta[i] = 0.f;
    return;
  }
  const uint32_t flags = (uint32_t)__float_as_int(r3.x) >> 24;
  const float4 r0 = V.rec[4 * i + 0];
  const float4 r1 = V.rec[4 * i + 1];
  const float* gp = V.grad2d + (int64_t)kGradStride * i;
  const float4 g0 = reinterpret_cast<const float4*>(gp)[0];
  const float4 g1 = reinterpret_cast<const float4*>(gp)[1];
  const float4 g2 = reinterpret_cast<const float4*>(gp)[2];
  const float gu = g0.x, gv = g0.y, ga = g0.z, gb = g0.w;
  const float gc = g1.x, gop = g1.y;
  const float grgb[3] = {g1.z, g1.w, g2.x};
  const float gbeta2 = g2.y;

  const float* mu = V.means + 3 * i;
  const float mx = mu[0], my = mu[1], mz = mu[2];
  const float4 qv = reinterpret_cast<const float4*>(V.quats)[i];
  const float beta = V.beta[i];
  const float* R = V.R;
  float p[3];
  for (int r = 0; r < 3; ++r) p[r] = R[3 * r] * mx + R[3 * r + 1] * my + R[3 * r + 2] * mz + V.t[r];
  const float z = p[2];
  const float s[3] = {__expf(V.log_scales[3 * i]), __expf(V.log_scales[3 * i + 1]), __expf(V.log_scales[3 * i + 2])};
  const float op = r1.z;

  // quaternion
  const float nn = qv.x * qv.x + qv.y * qv.y + qv.z * qv.z + qv.w * qv.w;
  const float nr = sqrtf(nn);
  const float qw = qv.x / nr, qx = qv.y / nr, qy = qv.z / nr, qz = qv.w / nr;
  float Q[9];
  Q[0] = 1.f - 2.f * (qy * qy + qz * qz); Q[1] = 2.f * (qx * qy - qw * qz); Q[2] = 2.f * (qx * qz + qw * qy);
  Q[3] = 2.f * (qx * qy + qw * qz); Q[4] = 1.f - 2.f * (qx * qx + qz * qz); Q[5] = 2.f * (qy * qz - qw * qx);
  Q[6] = 2.f * (qx * qz - qw * qy); Q[7] = 2.f * (qy * qz + qw * qx); Q[8] = 1.f - 2.f * (qx * qx + qy * qy);
  float phi = 1.f;
  if (V.falloff == GES_FALLOFF_PHI) phi = 2.f / (1.f + __expf(-(V.rho * beta - 2.f * V.rho)));
  const float S[3] = {phi * s[0], phi * s[1], phi * s[2]};
  float Mm[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Mm[3 * r + c] = Q[3 * r + c] * S[c];
  float Sig[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Sig[3 * r + c] = Mm[3 * r] * Mm[3 * c] + Mm[3 * r + 1] * Mm[3 * c + 1] + Mm[3 * r + 2] * Mm[3 * c + 2];

  const float fx = V.fx, fy = V.fy;
  const bool clx = (flags & 8u) != 0, cly = (flags & 16u) != 0;
  float txz = p[0] / z, tyz = p[1] / z;
  txz = fminf(V.limx, fmaxf(-V.limx, txz));
  tyz = fminf(V.limy, fmaxf(-V.limy, tyz));
  const float xc = clx ? txz * z : p[0];
  const float yc = cly ? tyz * z : p[1];
  const float iz = 1.f / z, iz2 = iz * iz, iz3 = iz2 * iz;
  const float J00 = fx * iz, J11 = fy * iz, J02 = -fx * xc * iz2, J12 = -fy * yc * iz2;
  float T[6];
  for (int c = 0; c < 3; ++c) {
    T[c] = J00 * R[c] + J02 * R[6 + c];
    T[3 + c] = J11 * R[3 + c] + J12 * R[6 + c];
  }

  // conic -> covariance: dL/dcov = -C G_C C with C = conic, G_C the symmetric gradient
  const float ca = r0.z, cb = r0.w, cc = r1.x;
  const float gx = -(ca * ca * ga + ca * cb * gb + cb * cb * gc);
  const float gy = -(2.f * ca * cb * ga + (ca * cc + cb * cb) * gb + 2.f * cb * cc * gc);
  const float gz = -(cb * cb * ga + cb * cc * gb + cc * cc * gc);
  // G2: gradient w.r.t. the full symmetric 2x2 covariance (off-diagonal split in half)
  const float G2[4] = {gx, 0.5f * gy, 0.5f * gy, gz};

  // cov = T Sigma T^T: dL/dSigma = T^T G2 T (symmetric), dL/dT = 2 G2 T Sigma
  float GT[6];   // G2 T (2x3)
  for (int c = 0; c < 3; ++c) {
    GT[c] = G2[0] * T[c] + G2[1] * T[3 + c];
    GT[3 + c] = G2[2] * T[c] + G2[3] * T[3 + c];
  }
  float GS[9];   // T^T (G2 T)
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) GS[3 * r + c] = T[r] * GT[c] + T[3 + r] * GT[3 + c];
  float gT[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      gT[3 * r + c] = 2.f * (GT[3 * r] * Sig[c] + GT[3 * r + 1] * Sig[3 + c] + GT[3 * r + 2] * Sig[6 + c]);
  // T = J W: dL/dJ = dL/dT W^T
  const float gJ00 = gT[0] * R[0] + gT[1] * R[1] + gT[2] * R[2];
  const float gJ02 = gT[0] * R[6] + gT[1] * R[7] + gT[2] * R[8];
  const float gJ11 = gT[3] * R[3] + gT[4] * R[4] + gT[5] * R[5];
  const float gJ12 = gT[3] * R[6] + gT[4] * R[7] + gT[5] * R[8];
  float gp0 = 0.f, gp1 = 0.f, gz_ = 0.f;
  gz_ += -fx * iz2 * gJ00 + 2.f * fx * xc * iz3 * gJ02 - fy * iz2 * gJ11 + 2.f * fy * yc * iz3 * gJ12;
  const float gxc = -fx * iz2 * gJ02, gyc = -fy * iz2 * gJ12;
  if (clx) gz_ += gxc * txz; else gp0 += gxc;
  if (cly) gz_ += gyc * tyz; else gp1 += gyc;
  // mean2D
  gp0 += gu * fx * iz;
  gp1 += gv * fy * iz;
  gz_ += -(gu * fx * p[0] + gv * fy * p[1]) * iz2;

  // Sigma = M M^T: dL/dM = 2 GS M
  float gM[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) gM[3 * r + c] = 2.f * (GS[3 * r] * Mm[c] + GS[3 * r + 1] * Mm[3 + c] + GS[3 * r + 2] * Mm[6 + c]);
  float gS[3] = {0.f, 0.f, 0.f};
  float gQ[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      gS[c] += gM[3 * r + c] * Q[3 * r + c];
      gQ[3 * r + c] = gM[3 * r + c] * S[c];
    }
  float gphi = gS[0] * s[0] + gS[1] * s[1] + gS[2] * s[2];
  if (G.log_scales)
    for (int c = 0; c < 3; ++c) G.log_scales[3 * i + c] = gS[c] * phi * s[c];
  if (G.beta) {
    float gb_ = 0.f;
    if (V.falloff == GES_FALLOFF_PHI) gb_ = gphi * V.rho * phi * (1.f - 0.5f * phi);
    else gb_ = gbeta2;
    G.beta[i] = gb_;
  }
  // rotation -> unit quaternion -> quaternion
  {
    const float w = qw, x = qx, y = qy, zq = qz;
    float gw = 2.f * (-zq * gQ[1] + y * gQ[2] + zq * gQ[3] - x * gQ[5] - y * gQ[6] + x * gQ[7]);
    float gxq = 2.f * (y * gQ[1] + zq * gQ[2] + y * gQ[3] - 2.f * x * gQ[4] - w * gQ[5] + zq * gQ[6] + w * gQ[7] - 2.f * x * gQ[8]);
    float gyq = 2.f * (-2.f * y * gQ[0] + x * gQ[1] + w * gQ[2] + x * gQ[3] + zq * gQ[5] - w * gQ[6] + zq * gQ[7] - 2.f * y * gQ[8]);
    float gzq = 2.f * (-2.f * zq * gQ[0] - w * gQ[1] + x * gQ[2] + w * gQ[3] - 2.f * zq * gQ[4] + y * gQ[5] + x * gQ[6] + y * gQ[7]);
    const float dot = gw * w + gxq * x + gyq * y + gzq * zq;
    if (G.quats)
      reinterpret_cast<float4*>(G.quats)[i] =
          make_float4((gw - w * dot) / nr, (gxq - x * dot) / nr, (gyq - y * dot) / nr, (gzq - zq * dot) / nr);
  }
  if (G.opacity_logits) G.opacity_logits[i] = gop * op * (1.f - op);

  // colour: SH coefficients and the view direction
  float gmu[3] = {0.f, 0.f, 0.f};
  {
    const float e0 = mx - V.campos[0], e1 = my - V.campos[1], e2 = mz - V.campos[2];
    const float len = sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
    const float x = e0 / len, y = e1 / len, zz_ = e2 / len;
    float Y[16];
    sh_basis(x, y, zz_, V.sh_degree, Y);
    float gc3[3];
    for (int ch = 0; ch < 3; ++ch) gc3[ch] = (flags & (1u << ch)) ? 0.f : grgb[ch];
    const float* shc = V.sh + (int64_t)3 * K * i;
    if (G.sh)
      for (int k = 0; k < K; ++k)
        for (int ch = 0; ch < 3; ++ch) G.sh[(int64_t)3 * K * i + 3 * k + ch] = Y[k] * gc3[ch];
    if (V.sh_degree > 0) {
      // dL/dY_k = sum_ch gc3[ch] sh[k][ch]
      float gY[16];
      for (int k = 0; k < K; ++k) gY[k] = gc3[0] * shc[3 * k] + gc3[1] * shc[3 * k + 1] + gc3[2] * shc[3 * k + 2];
      float gdx = 0.f, gdy = 0.f, gdz = 0.f;
      gdy += -kC1 * gY[1]; gdz += kC1 * gY[2]; gdx += -kC1 * gY[3];
      if (V.sh_degree > 1) {
        const float xx = x * x, yy = y * y, z2v = zz_ * zz_;
        gdx += kC2a * y * gY[4]; gdy += kC2a * x * gY[4];
        gdy += -kC2a * zz_ * gY[5]; gdz += -kC2a * y * gY[5];
        gdx += -2.f * kC2b * x * gY[6]; gdy += -2.f * kC2b * y * gY[6]; gdz += 4.f * kC2b * zz_ * gY[6];
        gdx += -kC2a * zz_ * gY[7]; gdz += -kC2a * x * gY[7];
        gdx += 2.f * kC2c * x * gY[8]; gdy += -2.f * kC2c * y * gY[8];
        if (V.sh_degree > 2) {
          gdx += -kC3a * 6.f * x * y * gY[9]; gdy += -kC3a * (3.f * xx - 3.f * yy) * gY[9];
          gdx += kC3b * y * zz_ * gY[10]; gdy += kC3b * x * zz_ * gY[10]; gdz += kC3b * x * y * gY[10];
          gdx += 2.f * kC3c * x * y * gY[11]; gdy += -kC3c * (4.f * z2v - xx - 3.f * yy) * gY[11];
          gdz += -8.f * kC3c * y * zz_ * gY[11];
          gdx += -6.f * kC3d * x * zz_ * gY[12]; gdy += -6.f * kC3d * y * zz_ * gY[12];
          gdz += kC3d * (6.f * z2v - 3.f * xx - 3.f * yy) * gY[12];
          gdx += -kC3c * (4.f * z2v - 3.f * xx - yy) * gY[13]; gdy += 2.f * kC3c * x * y * gY[13];
          gdz += -8.f * kC3c * x * zz_ * gY[13];
          gdx += 2.f * kC3e * x * zz_ * gY[14]; gdy += -2.f * kC3e * y * zz_ * gY[14]; gdz += kC3e * (xx - yy) * gY[14];
          gdx += -kC3a * (3.f * xx - 3.f * yy) * gY[15]; gdy += 6.f * kC3a * x * y * gY[15];
        }
      }
      // d = e/|e|: dL/de = (dL/dd - d (d . dL/dd)) / |e|
      const float dd = gdx * x + gdy * y + gdz * zz_;
      gmu[0] += (gdx - x * dd) / len;
      gmu[1] += (gdy - y * dd) / len;
      gmu[2] += (gdz - zz_ * dd) / len;
    }
  }
  // p = W mu + t
  if (G.means) {
    for (int c = 0; c < 3; ++c) G.means[3 * i + c] = gmu[c] + R[c] * gp0 + R[3 + c] * gp1 + R[6 + c] * gz_;
  }
}

hipError_t launch_preprocess(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  if (b.pre_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(preprocess_kernel, dim3((unsigned)b.pre_blocks), dim3(256), 0, stream, dbatch);
  return hipGetLastError();
}

hipError_t launch_preprocess_backward(const DeviceBatch* dbatch, const Batch& b, const ges_splat_grads* grads,
                                      hipStream_t stream) {
  if (b.pre_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(preprocess_backward_kernel, dim3((unsigned)b.pre_blocks), dim3(256), 0, stream, dbatch, *grads);
  return hipGetLastError();
}

}  // namespace ges
