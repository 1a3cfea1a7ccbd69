// preprocess_bwd.hip -- chain rule of the per-splat preprocess (GES Sec. 4.1-4.2), one thread per splat.
//
// From the accumulated gradients of a splat's 2-D quantities (mean2D, conic a/b/c, opacity, colour and,
// with the GEF falloff, beta) to its mean, log-scale, quaternion, opacity logit, SH coefficients and
// beta.  The chain runs in binary64: forward quantities (scales, opacity, rotation, covariance, the
// conic, the view direction) are recomputed in binary64 from the binary32 inputs, and only the decisions
// (visibility, guard clamp of the Jacobian, colour clamp) come from the forward pass, through a 4-byte
// visibility word per splat.  Several of the sums cancel (e.g. the scale gradient of an axis along the
// view ray), and binary32 there leaves an error proportional to the splat's whole gradient; the FP64
// vector rate of gfx950 equals its non-packed FP32 rate and the kernel is memory-bound, so binary64
// costs little.  Nothing here feeds a decision, so this file is built with contraction allowed.
// Memory: per visible splat the 2-D gradient row, the parameters (240 B at SH degree 3) and the
// parameter gradients (240 B); per culled splat the visibility word and zero gradients.  The SH rows
// (192 B at degree 3) of a wave's 64 splats are staged in LDS and written as one contiguous block.
#include "ges_internal.h"

namespace ges {

// Real SH normalisations in binary64 (same values as the forward's binary32 constants, unrounded).
constexpr double kD0 = 0.28209479177387814;   // 1/(2 sqrt(pi))
constexpr double kD1 = 0.4886025119029199;    // sqrt(3/pi)/2
constexpr double kD2a = 1.0925484305920792;   // sqrt(15/pi)/2
constexpr double kD2b = 0.31539156525252005;  // sqrt(5/pi)/4
constexpr double kD2c = 0.5462742152960396;   // sqrt(15/pi)/4
constexpr double kD3a = 0.5900435899266435;   // sqrt(35/(2 pi))/4
constexpr double kD3b = 2.890611442640554;    // sqrt(105/pi)/2
constexpr double kD3c = 0.4570457994644658;   // sqrt(21/(2 pi))/4
constexpr double kD3d = 0.3731763325901154;   // sqrt(7/pi)/4
constexpr double kD3e = 1.445305721320277;    // sqrt(105/pi)/4

__device__ __forceinline__ void sh_basis_f64(double x, double y, double z, int degree, double* Y) {
  Y[0] = kD0;
  if (degree < 1) return;
  Y[1] = -kD1 * y; Y[2] = kD1 * z; Y[3] = -kD1 * x;
  if (degree < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kD2a * x * y; Y[5] = -kD2a * y * z; Y[6] = kD2b * (2.0 * zz - xx - yy); Y[7] = -kD2a * x * z;
  Y[8] = kD2c * (xx - yy);
  if (degree < 3) return;
  Y[9] = -kD3a * y * (3.0 * xx - yy);
  Y[10] = kD3b * x * y * z;
  Y[11] = -kD3c * y * (4.0 * zz - xx - yy);
  Y[12] = kD3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
  Y[13] = -kD3c * x * (4.0 * zz - xx - yy);
  Y[14] = kD3e * z * (xx - yy);
  Y[15] = -kD3a * x * (xx - 3.0 * yy);
}

// Gradient, parameter and moment stores are non-temporal: 720 MB of gradients per 3M-splat frame stream past
// the caches (measured on that frame: 0.29 -> 0.27 ms for the backward, and the parameters the next frame's
// preprocess reads stay in the last-level cache).
typedef float NtF4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void nt_store4(float4* d, float4 v) {
  NtF4 x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, reinterpret_cast<NtF4*>(d));
}

// Output of one parameter gradient: stored when the caller asked for gradients, and with kAdam also
// applied at once as an Adam update of the parameter (the gradient never goes through memory).
template <bool kAdam, int P>
__device__ __forceinline__ void emit(float* g, const AdamSplats& A, int64_t idx, float val) {
  if constexpr (kAdam) {
    if (A.gin[P]) val = A.gin[P][idx] + val;      // the other views' gradients, then this view's
  }
  if (g) {
    if (A.accumulate) g[idx] = g[idx] + val;
    else __builtin_nontemporal_store(val, g + idx);
  }
  if constexpr (kAdam) {
    float p = A.p[P][idx], m = A.m[P][idx], v = A.v[P][idx];
    adam_update(p, val, m, v, A.b1, A.b2, A.eps, A.step_size[P], A.inv_sqrt_bc2);
    __builtin_nontemporal_store(p, A.p[P] + idx);
    __builtin_nontemporal_store(m, A.m[P] + idx);
    __builtin_nontemporal_store(v, A.v[P] + idx);
  }
}

template <bool kAdam, int P>
__device__ __forceinline__ void emit4(float* g, const AdamSplats& A, int64_t idx4, float4 val) {
  if constexpr (kAdam) {
    if (A.gin[P]) {
      const float4 o = reinterpret_cast<const float4*>(A.gin[P])[idx4];
      val = make_float4(o.x + val.x, o.y + val.y, o.z + val.z, o.w + val.w);
    }
  }
  if (g) {
    float4* d = reinterpret_cast<float4*>(g) + idx4;
    if (A.accumulate) {
      const float4 o = *d;
      *d = make_float4(o.x + val.x, o.y + val.y, o.z + val.z, o.w + val.w);
    } else {
      nt_store4(d, val);
    }
  }
  if constexpr (kAdam) {
    float4 p = reinterpret_cast<const float4*>(A.p[P])[idx4];
    float4 m = reinterpret_cast<const float4*>(A.m[P])[idx4];
    float4 v = reinterpret_cast<const float4*>(A.v[P])[idx4];
    adam_update(p.x, val.x, m.x, v.x, A.b1, A.b2, A.eps, A.step_size[P], A.inv_sqrt_bc2);
    adam_update(p.y, val.y, m.y, v.y, A.b1, A.b2, A.eps, A.step_size[P], A.inv_sqrt_bc2);
    adam_update(p.z, val.z, m.z, v.z, A.b1, A.b2, A.eps, A.step_size[P], A.inv_sqrt_bc2);
    adam_update(p.w, val.w, m.w, v.w, A.b1, A.b2, A.eps, A.step_size[P], A.inv_sqrt_bc2);
    nt_store4(reinterpret_cast<float4*>(A.p[P]) + idx4, p);
    nt_store4(reinterpret_cast<float4*>(A.m[P]) + idx4, m);
    nt_store4(reinterpret_cast<float4*>(A.v[P]) + idx4, v);
  }
}

// Digamma psi(x) for x > 0 in binary64: psi(x) = psi(x + k) - sum 1/(x + j) up to x + k >= 6, then the
// asymptotic series ln x - 1/(2x) - 1/(12x^2) + 1/(120x^4) - 1/(252x^6) + 1/(240x^8) - 1/(132x^10).
__device__ __forceinline__ double digamma(double x) {
  double acc = 0.0;
  while (x < 6.0) {
    acc -= 1.0 / x;
    x += 1.0;
  }
  const double i = 1.0 / x, i2 = i * i;
  const double series = i2 * (1.0 / 12 - i2 * (1.0 / 120 - i2 * (1.0 / 252 - i2 * (1.0 / 240 - i2 / 132))));
  return acc + log(x) - 0.5 * i - series;
}

constexpr int kRowPad = 13;   // float4 slots per staged SH-gradient row (12 used at degree 3; 13 spreads LDS banks)



// Chain rule of splat i.  SH-gradient rows of degrees 1 and 3 (whole float4s) go to `row` in LDS; other
// degrees are written straight to memory.
template <int D, bool kAdam>
__device__ __forceinline__ void backward_splat(const ViewDesc& V, const ges_splat_grads& G, const AdamSplats& A,
                                               int64_t i, float4* row) {
  constexpr int K = (D + 1) * (D + 1);
  const uint32_t vis = V.vis[i];
  const int64_t sh0 = (int64_t)3 * K * i;
  if (!(vis & kVisBit)) {
    if (V.keep_grad2d) {   // inspection: the rows of unlisted splats read as zero
      double2* gz = reinterpret_cast<double2*>(V.grad2d + (int64_t)kGradStride * i);
#pragma unroll
      for (int k = 0; k < kGradStride / 2; ++k) gz[k] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      emit<kAdam, kParMeans>(G.means, A, 3 * i + c, 0.f);
      emit<kAdam, kParScales>(G.log_scales, A, 3 * i + c, 0.f);
    }
    emit4<kAdam, kParQuats>(G.quats, A, i, make_float4(0.f, 0.f, 0.f, 0.f));
    emit<kAdam, kParOpacity>(G.opacity_logits, A, i, 0.f);
    emit<kAdam, kParBeta>(G.beta, A, i, 0.f);
    if constexpr ((3 * K) % 4 == 0) {
#pragma unroll
      for (int m = 0; m < 3 * K / 4; ++m) row[m] = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      for (int k = 0; k < 3 * K; ++k) emit<kAdam, kParSh>(G.sh, A, sh0 + k, 0.f);
    }
    return;
  }
  const uint32_t flags = vis & 0xffu;
  // the splat's 2-D gradient, summed from its rows by the reduction that follows the backward raster (zero
  // when no pixel composited it)
  double2 g01 = make_double2(0.0, 0.0), g23 = g01, g45 = g01, g67 = g01, g89 = g01;
  double2* gp = reinterpret_cast<double2*>(V.grad2d + (int64_t)kGradStride * i);
  if (vis & kRowBit) {
    g01 = gp[0]; g23 = gp[1]; g45 = gp[2]; g67 = gp[3]; g89 = gp[4];
  } else if (V.keep_grad2d) {
#pragma unroll
    for (int k = 0; k < 5; ++k) gp[k] = make_double2(0.0, 0.0);
  }
  if (A.stat_accum) {   // densification statistic: the mean-2D gradient in NDC units
    const double su = g01.x * A.half_w, sv = g01.y * A.half_h;
    A.stat_accum[i] += (float)sqrt(su * su + sv * sv);
    A.stat_count[i] += 1.f;
  }
  const double grgb[3] = {g67.x, g67.y, g89.x};
  const double gu = g01.x, gv = g01.y, ga = g23.x, gb = g23.y, gc = g45.x, gop = g45.y;
  const double gbeta2 = g89.y;

  const float* mu = V.means + 3 * i;
  const double mx = mu[0], my = mu[1], mz = mu[2];
  const float4 qv = reinterpret_cast<const float4*>(V.quats)[i];
  const double beta = V.beta[i];
  double R[9];
  for (int k = 0; k < 9; ++k) R[k] = V.R[k];
  double p[3];
  for (int r = 0; r < 3; ++r) p[r] = R[3 * r] * mx + R[3 * r + 1] * my + R[3 * r + 2] * mz + (double)V.t[r];
  const double z = p[2];
  const double s[3] = {exp((double)V.log_scales[3 * i]), exp((double)V.log_scales[3 * i + 1]),
                       exp((double)V.log_scales[3 * i + 2])};
  const double op = 1.0 / (1.0 + exp(-(double)V.logits[i]));

  // quaternion
  const double q0 = qv.x, q1 = qv.y, q2 = qv.z, q3 = qv.w;
  const double nr = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const double qw = q0 / nr, qx = q1 / nr, qy = q2 / nr, qz = q3 / nr;
  double Q[9];
  Q[0] = 1.0 - 2.0 * (qy * qy + qz * qz); Q[1] = 2.0 * (qx * qy - qw * qz); Q[2] = 2.0 * (qx * qz + qw * qy);
  Q[3] = 2.0 * (qx * qy + qw * qz); Q[4] = 1.0 - 2.0 * (qx * qx + qz * qz); Q[5] = 2.0 * (qy * qz - qw * qx);
  Q[6] = 2.0 * (qx * qz - qw * qy); Q[7] = 2.0 * (qy * qz + qw * qx); Q[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
  double phi = 1.0;
  const double rho = V.rho;
  if (V.falloff == GES_FALLOFF_PHI) phi = 2.0 / (1.0 + exp(-(rho * beta - 2.0 * rho)));
  else if (V.falloff == GES_FALLOFF_PHI_EXACT) phi = 2.0 * exp(lgamma(3.0 / beta) - lgamma(1.0 / beta));
  const double S[3] = {phi * s[0], phi * s[1], phi * s[2]};
  double Mm[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Mm[3 * r + c] = Q[3 * r + c] * S[c];
  double Sig[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Sig[3 * r + c] = Mm[3 * r] * Mm[3 * c] + Mm[3 * r + 1] * Mm[3 * c + 1] + Mm[3 * r + 2] * Mm[3 * c + 2];

  // perspective Jacobian at p; the guard clamp of x/z, y/z is the forward's decision (record flags)
  const double fx = V.fx, fy = V.fy;
  const bool clx = (flags & 8u) != 0, cly = (flags & 16u) != 0;
  const double limx = 1.3 * (0.5 * (double)V.width / fx), limy = 1.3 * (0.5 * (double)V.height / fy);
  const double txz = clx ? copysign(limx, p[0] / z) : p[0] / z;
  const double tyz = cly ? copysign(limy, p[1] / z) : p[1] / z;
  const double xc = txz * z, yc = tyz * z;
  const double iz = 1.0 / z, iz2 = iz * iz, iz3 = iz2 * iz;
  const double J00 = fx * iz, J11 = fy * iz, J02 = -fx * xc * iz2, J12 = -fy * yc * iz2;
  double T[6];
  for (int c = 0; c < 3; ++c) {
    T[c] = J00 * R[c] + J02 * R[6 + c];
    T[3 + c] = J11 * R[3 + c] + J12 * R[6 + c];
  }
  // 2-D covariance and its inverse (the conic), recomputed in binary64
  double TS[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) TS[3 * r + c] = T[3 * r] * Sig[c] + T[3 * r + 1] * Sig[3 + c] + T[3 * r + 2] * Sig[6 + c];
  const double c00 = TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2] + 0.3;
  const double c01 = TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5];
  const double c11 = TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5] + 0.3;
  const double det = c00 * c11 - c01 * c01;
  const double ca = c11 / det, cb = -c01 / det, cc = c00 / det;

  // conic -> covariance: dL/dcov = -C G_C C with C = conic, G_C the symmetric gradient
  const double gx = -(ca * ca * ga + ca * cb * gb + cb * cb * gc);
  const double gy = -(2.0 * ca * cb * ga + (ca * cc + cb * cb) * gb + 2.0 * cb * cc * gc);
  const double gz = -(cb * cb * ga + cb * cc * gb + cc * cc * gc);
  // G2: gradient w.r.t. the full symmetric 2x2 covariance (off-diagonal split in half)
  const double G2[4] = {gx, 0.5 * gy, 0.5 * gy, gz};

  // cov = T Sigma T^T: dL/dSigma = T^T G2 T (symmetric), dL/dT = 2 G2 T Sigma
  double GT[6];   // G2 T (2x3)
  for (int c = 0; c < 3; ++c) {
    GT[c] = G2[0] * T[c] + G2[1] * T[3 + c];
    GT[3 + c] = G2[2] * T[c] + G2[3] * T[3 + c];
  }
  double GS[9];   // T^T (G2 T)
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) GS[3 * r + c] = T[r] * GT[c] + T[3 + r] * GT[3 + c];
  double gT[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      gT[3 * r + c] = 2.0 * (GT[3 * r] * Sig[c] + GT[3 * r + 1] * Sig[3 + c] + GT[3 * r + 2] * Sig[6 + c]);
  // T = J W: dL/dJ = dL/dT W^T
  const double gJ00 = gT[0] * R[0] + gT[1] * R[1] + gT[2] * R[2];
  const double gJ02 = gT[0] * R[6] + gT[1] * R[7] + gT[2] * R[8];
  const double gJ11 = gT[3] * R[3] + gT[4] * R[4] + gT[5] * R[5];
  const double gJ12 = gT[3] * R[6] + gT[4] * R[7] + gT[5] * R[8];
  double gp0 = 0.0, gp1 = 0.0, gz_ = 0.0;
  gz_ += -fx * iz2 * gJ00 + 2.0 * fx * xc * iz3 * gJ02 - fy * iz2 * gJ11 + 2.0 * fy * yc * iz3 * gJ12;
  const double gxc = -fx * iz2 * gJ02, gyc = -fy * iz2 * gJ12;
  if (clx) gz_ += gxc * txz; else gp0 += gxc;
  if (cly) gz_ += gyc * tyz; else gp1 += gyc;
  // mean2D
  gp0 += gu * fx * iz;
  gp1 += gv * fy * iz;
  gz_ += -(gu * fx * p[0] + gv * fy * p[1]) * iz2;

  // Sigma = M M^T: dL/dM = 2 GS M
  double gS[3] = {0.0, 0.0, 0.0};
  double gQ[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const double gM = 2.0 * (GS[3 * r] * Mm[c] + GS[3 * r + 1] * Mm[3 + c] + GS[3 * r + 2] * Mm[6 + c]);
      gS[c] += gM * Q[3 * r + c];
      gQ[3 * r + c] = gM * S[c];
    }
  const double gphi = gS[0] * s[0] + gS[1] * s[1] + gS[2] * s[2];
  for (int c = 0; c < 3; ++c) emit<kAdam, kParScales>(G.log_scales, A, 3 * i + c, (float)(gS[c] * phi * s[c]));
  {
    double gb_ = 0.0;
    if (V.falloff == GES_FALLOFF_PHI) gb_ = gphi * rho * phi * (1.0 - 0.5 * phi);
    else if (V.falloff == GES_FALLOFF_PHI_EXACT)   // d phi / d beta = phi (psi(1/b) - 3 psi(3/b)) / b^2
      gb_ = gphi * phi * (digamma(1.0 / beta) - 3.0 * digamma(3.0 / beta)) / (beta * beta);
    else gb_ = gbeta2;
    emit<kAdam, kParBeta>(G.beta, A, i, (float)gb_);
  }
  // rotation -> unit quaternion -> quaternion
  {
    const double w = qw, x = qx, y = qy, zq = qz;
    const double gw = 2.0 * (-zq * gQ[1] + y * gQ[2] + zq * gQ[3] - x * gQ[5] - y * gQ[6] + x * gQ[7]);
    const double gxq = 2.0 * (y * gQ[1] + zq * gQ[2] + y * gQ[3] - 2.0 * x * gQ[4] - w * gQ[5] + zq * gQ[6] + w * gQ[7] - 2.0 * x * gQ[8]);
    const double gyq = 2.0 * (-2.0 * y * gQ[0] + x * gQ[1] + w * gQ[2] + x * gQ[3] + zq * gQ[5] - w * gQ[6] + zq * gQ[7] - 2.0 * y * gQ[8]);
    const double gzq = 2.0 * (-2.0 * zq * gQ[0] - w * gQ[1] + x * gQ[2] + w * gQ[3] - 2.0 * zq * gQ[4] + y * gQ[5] + x * gQ[6] + y * gQ[7]);
    const double dot = gw * w + gxq * x + gyq * y + gzq * zq;
    emit4<kAdam, kParQuats>(G.quats, A, i,
                            make_float4((float)((gw - w * dot) / nr), (float)((gxq - x * dot) / nr),
                                        (float)((gyq - y * dot) / nr), (float)((gzq - zq * dot) / nr)));
  }
  emit<kAdam, kParOpacity>(G.opacity_logits, A, i, (float)(gop * op * (1.0 - op)));

  // colour: SH coefficients and the view direction
  double gmu[3] = {0.0, 0.0, 0.0};
  double gc3[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) gc3[ch] = (flags & (1u << ch)) ? 0.0 : grgb[ch];
  double cpos[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    cpos[j] = -(R[j] * (double)V.t[0] + R[3 + j] * (double)V.t[1] + R[6 + j] * (double)V.t[2]);
  const double e0 = mx - cpos[0], e1 = my - cpos[1], e2 = mz - cpos[2];
  const double len = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
  const double x = e0 / len, y = e1 / len, zz_ = e2 / len;
  double Y[16];
  sh_basis_f64(x, y, zz_, D, Y);
  const float* shc = V.sh + (int64_t)3 * K * i;
  // dL/dc_k,ch = Y_k gc3[ch]; dL/dY_k = sum_ch gc3[ch] c_k,ch.  Rows of 3K floats; for degrees 1 and 3
  // they are 16-byte aligned (checked on the host), so they move as float4.
  double gY[16];
#pragma unroll
  for (int k = 0; k < K; ++k) gY[k] = 0.0;
  if constexpr ((3 * K) % 4 == 0) {
    const float4* s4 = reinterpret_cast<const float4*>(shc);
    float4 xv[3 * K / 4];
#pragma unroll
    for (int m = 0; m < 3 * K / 4; ++m) xv[m] = s4[m];
#pragma unroll
    for (int m = 0; m < 3 * K / 4; ++m) {
      const float xs[4] = {xv[m].x, xv[m].y, xv[m].z, xv[m].w};
      float ys[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = (4 * m + e) / 3, ch = (4 * m + e) % 3;
        gY[k] += gc3[ch] * (double)xs[e];
        ys[e] = (float)(Y[k] * gc3[ch]);
      }
      row[m] = make_float4(ys[0], ys[1], ys[2], ys[3]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        gY[k] += gc3[ch] * (double)shc[3 * k + ch];
        emit<kAdam, kParSh>(G.sh, A, sh0 + 3 * k + ch, (float)(Y[k] * gc3[ch]));
      }
  }
  if (D > 0) {
    double gdx = 0.0, gdy = 0.0, gdz = 0.0;
    gdy += -kD1 * gY[1]; gdz += kD1 * gY[2]; gdx += -kD1 * gY[3];
    if (D > 1) {
      const double xx = x * x, yy = y * y, z2v = zz_ * zz_;
      gdx += kD2a * y * gY[4]; gdy += kD2a * x * gY[4];
      gdy += -kD2a * zz_ * gY[5]; gdz += -kD2a * y * gY[5];
      gdx += -2.0 * kD2b * x * gY[6]; gdy += -2.0 * kD2b * y * gY[6]; gdz += 4.0 * kD2b * zz_ * gY[6];
      gdx += -kD2a * zz_ * gY[7]; gdz += -kD2a * x * gY[7];
      gdx += 2.0 * kD2c * x * gY[8]; gdy += -2.0 * kD2c * y * gY[8];
      if (D > 2) {
        gdx += -kD3a * 6.0 * x * y * gY[9]; gdy += -kD3a * (3.0 * xx - 3.0 * yy) * gY[9];
        gdx += kD3b * y * zz_ * gY[10]; gdy += kD3b * x * zz_ * gY[10]; gdz += kD3b * x * y * gY[10];
        gdx += 2.0 * kD3c * x * y * gY[11]; gdy += -kD3c * (4.0 * z2v - xx - 3.0 * yy) * gY[11];
        gdz += -8.0 * kD3c * y * zz_ * gY[11];
        gdx += -6.0 * kD3d * x * zz_ * gY[12]; gdy += -6.0 * kD3d * y * zz_ * gY[12];
        gdz += kD3d * (6.0 * z2v - 3.0 * xx - 3.0 * yy) * gY[12];
        gdx += -kD3c * (4.0 * z2v - 3.0 * xx - yy) * gY[13]; gdy += 2.0 * kD3c * x * y * gY[13];
        gdz += -8.0 * kD3c * x * zz_ * gY[13];
        gdx += 2.0 * kD3e * x * zz_ * gY[14]; gdy += -2.0 * kD3e * y * zz_ * gY[14]; gdz += kD3e * (xx - yy) * gY[14];
        gdx += -kD3a * (3.0 * xx - 3.0 * yy) * gY[15]; gdy += 6.0 * kD3a * x * y * gY[15];
      }
    }
    // d = e/|e|: dL/de = (dL/dd - d (d . dL/dd)) / |e|
    const double dd = gdx * x + gdy * y + gdz * zz_;
    gmu[0] = (gdx - x * dd) / len;
    gmu[1] = (gdy - y * dd) / len;
    gmu[2] = (gdz - zz_ * dd) / len;
  }
  // p = W mu + t
  for (int c = 0; c < 3; ++c)
    emit<kAdam, kParMeans>(G.means, A, 3 * i + c, (float)(gmu[c] + R[c] * gp0 + R[3 + c] * gp1 + R[6 + c] * gz_));
}

template <int D, bool kAdam>
__device__ __forceinline__ void backward_wave(const ViewDesc& V, const ges_splat_grads& G, const AdamSplats& A,
                                              int64_t w0, float4* rows) {
  constexpr int K = (D + 1) * (D + 1);
  constexpr int F4 = 3 * K / 4;   // float4s per SH-gradient row (degrees 1 and 3)
  const int lane = threadIdx.x & 63;
  const int64_t i = w0 + lane;
  if (i < V.n) backward_splat<D, kAdam>(V, G, A, i, rows + lane * kRowPad);
  if constexpr ((3 * K) % 4 == 0) {
    if (!kAdam && !G.sh) return;
    const int cnt = (int)min<int64_t>(64, V.n - w0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the wave's rows are one contiguous block of float4s starting at splat w0
    const int64_t base4 = (int64_t)F4 * w0;
    for (int m = lane; m < cnt * F4; m += 64)
      emit4<kAdam, kParSh>(G.sh, A, base4 + m, rows[(m / F4) * kRowPad + (m % F4)]);
  }
}

template <int D, bool kAdam>
__device__ __forceinline__ void backward_views(const DeviceBatch* db, const ges_splat_grads& G, const AdamSplats& A,
                                               int64_t w0, float4* rows) {
  // the views of one scene, in order: every view before the last adds its gradients to the stored ones (the
  // first overwrites unless the caller accumulates); the last applies the update (kAdam) with the stored
  // sum as the other views' gradients, or adds its gradients like the others
  const int nv = db->nviews;
  for (int v = 0; v < nv; ++v) {
    AdamSplats a = A;
    if (v > 0) a.accumulate = 1;
    if (kAdam && v == nv - 1) {
      a.accumulate = 0;
      backward_wave<D, true>(db->views[v], G, a, w0, rows);
    } else {
      backward_wave<D, false>(db->views[v], G, a, w0, rows);
    }
    // the next view's rows reuse the LDS rows this view's SH stores read
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// One block per 256 splats of a view.  SHARED: the batch's views render the same splats and the grid
// covers them once; each thread chains its splat through every view (backward_views).
template <bool kAdam, bool SHARED>
__global__ void __launch_bounds__(256) preprocess_backward_kernel(const DeviceBatch* __restrict__ db,
                                                                   ges_splat_grads G, AdamSplats A) {
  __shared__ float4 sRows[4 * 64 * kRowPad];
  const int64_t blk = blockIdx.x;
  const int wave = threadIdx.x >> 6;
  float4* rows = sRows + wave * 64 * kRowPad;
  if constexpr (SHARED) {
    const ViewDesc& V0 = db->views[0];
    const int64_t w0 = blk * 256 + wave * 64;
    if (w0 >= V0.n) return;
    switch (V0.sh_degree) {
      case 0: backward_views<0, kAdam>(db, G, A, w0, rows); break;
      case 1: backward_views<1, kAdam>(db, G, A, w0, rows); break;
      case 2: backward_views<2, kAdam>(db, G, A, w0, rows); break;
      default: backward_views<3, kAdam>(db, G, A, w0, rows); break;
    }
    return;
  }
  const int v = view_of_block(db->pre_prefix, db->nviews, blk);
  const ViewDesc& V = db->views[v];
  const int64_t w0 = (blk - db->pre_prefix[v]) * 256 + wave * 64;
  if (w0 >= V.n) return;
  switch (V.sh_degree) {   // uniform per block: one view per block
    case 0: backward_wave<0, kAdam>(V, G, A, w0, rows); break;
    case 1: backward_wave<1, kAdam>(V, G, A, w0, rows); break;
    case 2: backward_wave<2, kAdam>(V, G, A, w0, rows); break;
    default: backward_wave<3, kAdam>(V, G, A, w0, rows); break;
  }
}

hipError_t launch_preprocess_backward(const DeviceBatch* dbatch, const Batch& b, const ges_splat_grads* grads,
                                      hipStream_t stream, const AdamSplats* args, bool fused) {
  if (b.pre_blocks == 0) return hipSuccess;
  const ges_splat_grads none{};
  const ges_splat_grads& g = grads ? *grads : none;
  const AdamSplats a = args ? *args : AdamSplats{};
  const bool shared = b.shared_scene && b.nviews > 1;
  const dim3 grid((unsigned)(shared ? b.pre_blocks / b.nviews : b.pre_blocks));
  if (shared && fused)
    hipLaunchKernelGGL((preprocess_backward_kernel<true, true>), grid, dim3(256), 0, stream, dbatch, g, a);
  else if (shared)
    hipLaunchKernelGGL((preprocess_backward_kernel<false, true>), grid, dim3(256), 0, stream, dbatch, g, a);
  else if (fused)
    hipLaunchKernelGGL((preprocess_backward_kernel<true, false>), grid, dim3(256), 0, stream, dbatch, g, a);
  else
    hipLaunchKernelGGL((preprocess_backward_kernel<false, false>), grid, dim3(256), 0, stream, dbatch, g, a);
  return hipGetLastError();
}

}  // namespace ges
