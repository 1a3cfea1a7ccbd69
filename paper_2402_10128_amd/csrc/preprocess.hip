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
#include "sh_basis.h"

namespace ges {

__device__ __forceinline__ float max_c(float a, float b) { return geom_max(a, b); }
__device__ __forceinline__ float min_c(float a, float b) { return geom_min(a, b); }

__device__ __forceinline__ void write_culled(const ViewDesc& V, int64_t i) {
  float4* rec = V.rec;
  V.vis[i] = 0u;
  V.item_key[i] = kNoKey;
  V.item_cand[i] = 0u;
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  rec[4 * i + 0] = z;
  rec[4 * i + 1] = z;
  rec[4 * i + 2] = z;
  rec[4 * i + 3] = z;
}

__device__ __forceinline__ bool finite3(const float* p) {
  return __builtin_isfinite(p[0]) && __builtin_isfinite(p[1]) && __builtin_isfinite(p[2]);
}

template <int D>
__device__ __forceinline__ void preprocess_splat(const ViewDesc& V, int64_t i) {
  constexpr int K = (D + 1) * (D + 1);
  float4* rec = V.rec;
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
  if (!ok) { write_culled(V, i); return; }

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
  if (!(z > V.near_z)) { write_culled(V, i); return; }

  // 2. activations
  const float s0 = canon_exp(l0), s1 = canon_exp(l1), s2 = canon_exp(l2);
  const float en = canon_exp(-logit);
  const float den = 1.0f + en;
  const float op = 1.0f / den;
  const float o255 = 255.0f * op;
  if (!(o255 > 1.0f)) { write_culled(V, i); return; }

  // 3. quaternion -> rotation
  float qw = qv.x, qx = qv.y, qy = qv.z, qz = qv.w;
  float nn = qw * qw; nn = nn + qx * qx; nn = nn + qy * qy; nn = nn + qz * qz;
  if (!(nn > 0.0f)) { write_culled(V, i); return; }
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
  } else if (V.falloff == GES_FALLOFF_PHI_EXACT) {
    if (!(beta > 0.0f)) { write_culled(V, i); return; }
    const float a3 = 3.0f / beta, a1 = 1.0f / beta;
    float dl = canon_lgamma(a3);
    dl = dl - canon_lgamma(a1);
    phi = 2.0f * canon_exp(dl);
    if (!__builtin_isfinite(phi) || !(phi > 0.0f)) { write_culled(V, i); return; }
  } else {
    if (!(beta > 0.0f)) { write_culled(V, i); return; }
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
  if (!(det > 0.0f)) { write_culled(V, i); return; }
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
  if (V.falloff != GES_FALLOFF_GEF) {   // Gaussian falloff (PHI, PHI_EXACT)
    qm = L2;
  } else {
    float e = 2.0f / beta;
    float lgl = canon_log(L2);
    e = e * lgl;
    qm = canon_exp(e);
  }
  if (!__builtin_isfinite(qm)) { write_culled(V, i); return; }

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
  if (!(xl <= xh) || !(yl <= yh)) { write_culled(V, i); return; }
  const int tx0 = (int)xl / kTile, tx1 = (int)xh / kTile;
  const int ty0 = (int)yl / kTile, ty1 = (int)yh / kTile;

  float shv[3 * K];
  if constexpr ((3 * K) % 4 == 0) {
    // rows of 12 K bytes are 16-byte aligned (the base pointer is checked on the host); read only
    // for splats that survived culling
#pragma unroll
    for (int k = 0; k < 3 * K / 4; ++k) {
      const float4 x = reinterpret_cast<const float4*>(shc)[k];
      shv[4 * k] = x.x; shv[4 * k + 1] = x.y; shv[4 * k + 2] = x.z; shv[4 * k + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) shv[k] = shc[k];
  }
  // a non-finite SH coefficient culls the splat like any other non-finite parameter
  bool sh_ok = true;
#pragma unroll
  for (int k = 0; k < 3 * K; ++k) sh_ok = sh_ok && __builtin_isfinite(shv[k]);
  if (!sh_ok) { write_culled(V, i); return; }
  // 11. colour
  float d0 = mx - V.campos[0], d1 = my - V.campos[1], d2 = mz - V.campos[2];
  float len = d0 * d0; len = len + d1 * d1; len = len + d2 * d2;
  len = __builtin_sqrtf(len);
  const float dx = d0 / len, dy = d1 / len, dz = d2 / len;
  float Y[16];
  sh_basis(dx, dy, dz, D, Y);
  float rgb[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = Y[0] * shv[ch];
#pragma unroll
    for (int k = 1; k < K; ++k) acc = acc + Y[k] * shv[3 * k + ch];
    acc = acc + 0.5f;
    if (acc < 0.0f) { acc = 0.0f; bits |= (1u << ch); }
    rgb[ch] = acc;
  }

  // the splat's depth-sort key and its number of candidate tiles (SQUARE: the rectangle); the candidate
  // count stands in for tiles_touched and the visibility bit until the duplication has counted the tiles
  // the exact test accepts (it rewrites the two words only where that count differs), with the clamp flags
  // for the backward pass
  uint32_t cand;
  {
    SplatTiles st;
    candidate_tiles(u, vv, ca, cb, cc, qm, tx0, ty0, tx1, ty1, V.tile_cull == GES_TILES_ELLIPSE, st);
    cand = candidate_count(st, V.height);
  }
  V.item_key[i] = __float_as_uint(z);
  V.item_cand[i] = cand;
  V.vis[i] = (cand ? kVisBit : 0u) | bits;
  rec[4 * i + 0] = make_float4(u, vv, ca, cb);
  rec[4 * i + 1] = make_float4(cc, qm, op, beta);
  rec[4 * i + 2] = make_float4(rgb[0], rgb[1], rgb[2], z);
  rec[4 * i + 3] = make_float4(__int_as_float((int)((uint32_t)radius | (bits << 24))),
                               __uint_as_float((uint32_t)tx0 | ((uint32_t)ty0 << 16)),
                               __uint_as_float((uint32_t)tx1 | ((uint32_t)ty1 << 16)), __uint_as_float(cand));
}

__global__ void __launch_bounds__(256) preprocess_kernel(const DeviceBatch* __restrict__ db) {
  const int64_t blk = blockIdx.x;
  const int v = view_of_block(db->pre_prefix, db->nviews, blk);
  const ViewDesc& V = db->views[v];
  const int64_t i = (blk - db->pre_prefix[v]) * 256 + threadIdx.x;
  if (i >= V.n) return;
  switch (V.sh_degree) {   // uniform per block: one view per block
    case 0: preprocess_splat<0>(V, i); break;
    case 1: preprocess_splat<1>(V, i); break;
    case 2: preprocess_splat<2>(V, i); break;
    default: preprocess_splat<3>(V, i); break;
  }
}

hipError_t launch_preprocess(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  if (b.pre_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(preprocess_kernel, dim3((unsigned)b.pre_blocks), dim3(256), 0, stream, dbatch);
  return hipGetLastError();
}

}  // namespace ges
