// preprocess_bwd.hip -- chain rule of the per-splat preprocess (GES Sec. 4.1-4.2), one thread per splat.
//
// From the accumulated gradients of a splat's 2-D quantities (mean2D, conic a/b/c, opacity, colour and,
// with the GEF falloff, beta) to its mean, log-scale, quaternion, opacity logit, SH coefficients and
// beta.  Forward quantities are recomputed in binary32; the decisions (culling, guard clamp of the
// Jacobian, colour clamp) come from the record.  Nothing here feeds a decision, so this file is built
// with contraction and fast division allowed.
// Memory: ~600 B per splat at SH degree 3 (parameters, record, 2-D gradients in; parameter gradients
// out): HBM-bound.
#include "ges_internal.h"
#include "sh_basis.h"

namespace ges {

template <int D>
__device__ __forceinline__ void backward_splat(const ViewDesc& V, const ges_splat_grads& G, int64_t i) {
  constexpr int K = (D + 1) * (D + 1);
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
  const double2* gp = reinterpret_cast<const double2*>(V.grad2d + (int64_t)kGradStride * i);
  const double2 g01 = gp[0], g23 = gp[1], g45 = gp[2], g67 = gp[3], g89 = gp[4];
  const float gu = (float)g01.x, gv = (float)g01.y, ga = (float)g23.x, gb = (float)g23.y;
  const float gc = (float)g45.x, gop = (float)g45.y;
  const float grgb[3] = {(float)g67.x, (float)g67.y, (float)g89.x};
  const float gbeta2 = (float)g89.y;

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
    sh_basis(x, y, zz_, D, Y);
    float gc3[3];
    for (int ch = 0; ch < 3; ++ch) gc3[ch] = (flags & (1u << ch)) ? 0.f : grgb[ch];
    const float* shc = V.sh + (int64_t)3 * K * i;
    if (G.sh)
      for (int k = 0; k < K; ++k)
        for (int ch = 0; ch < 3; ++ch) G.sh[(int64_t)3 * K * i + 3 * k + ch] = Y[k] * gc3[ch];
    if (D > 0) {
      // dL/dY_k = sum_ch gc3[ch] sh[k][ch]
      float gY[16];
      for (int k = 0; k < K; ++k) gY[k] = gc3[0] * shc[3 * k] + gc3[1] * shc[3 * k + 1] + gc3[2] * shc[3 * k + 2];
      float gdx = 0.f, gdy = 0.f, gdz = 0.f;
      gdy += -kC1 * gY[1]; gdz += kC1 * gY[2]; gdx += -kC1 * gY[3];
      if (D > 1) {
        const float xx = x * x, yy = y * y, z2v = zz_ * zz_;
        gdx += kC2a * y * gY[4]; gdy += kC2a * x * gY[4];
        gdy += -kC2a * zz_ * gY[5]; gdz += -kC2a * y * gY[5];
        gdx += -2.f * kC2b * x * gY[6]; gdy += -2.f * kC2b * y * gY[6]; gdz += 4.f * kC2b * zz_ * gY[6];
        gdx += -kC2a * zz_ * gY[7]; gdz += -kC2a * x * gY[7];
        gdx += 2.f * kC2c * x * gY[8]; gdy += -2.f * kC2c * y * gY[8];
        if (D > 2) {
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

__global__ void __launch_bounds__(256) preprocess_backward_kernel(const DeviceBatch* __restrict__ db,
                                                                   ges_splat_grads G) {
  const int64_t blk = blockIdx.x;
  const int v = view_of_block(db->pre_prefix, db->nviews, blk);
  const ViewDesc& V = db->views[v];
  const int64_t i = (blk - db->pre_prefix[v]) * 256 + threadIdx.x;
  if (i >= V.n) return;
  switch (V.sh_degree) {
    case 0: backward_splat<0>(V, G, i); break;
    case 1: backward_splat<1>(V, G, i); break;
    case 2: backward_splat<2>(V, G, i); break;
    default: backward_splat<3>(V, G, i); break;
  }
}

hipError_t launch_preprocess_backward(const DeviceBatch* dbatch, const Batch& b, const ges_splat_grads* grads,
                                      hipStream_t stream) {
  if (b.pre_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(preprocess_backward_kernel, dim3((unsigned)b.pre_blocks), dim3(256), 0, stream, dbatch, *grads);
  return hipGetLastError();
}

}  // namespace ges
