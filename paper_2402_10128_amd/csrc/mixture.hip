// mixture.hip -- the paper's 1-D mixture simulation as one batched kernel (Sec. 3.2; App. A.3).
//
// Each problem fits a mixture of n components -- Gaussian (GMM), difference of Gaussians with variance
// ratio 4 (DoG), Laplacian of Gaussian (LoG) or generalized exponential (GEF, per-component beta) -- to a
// 1-D signal sampled on m points of a linspace, by Adam on the mean squared error, for a number of epochs.
// Component i has parameters (w_raw, mu, s, beta); w = w_raw, or softplus(w_raw) for positive weights.
//
// One workgroup of 256 threads runs one problem through all its epochs: the signal, the residuals, the
// parameters, their Adam moments and gradients stay in LDS.  Per epoch:
//   1. per component, the quantities every point needs (w, dw/dw_raw, 1/(2 s^2 + eps), ...);
//   2. residuals r_j = model(x_j) - y_j, threads over points;
//   3. gradients sum_j (2/m) r_j dc_i/dtheta(x_j): the four waves take components in turn, the 64 lanes
//      split the points, and a butterfly of shuffles adds the lanes;
//   4. Adam on every parameter (the update shared with the splat optimiser).
// A component that would read past the LDS arrays (n outside 1..128), an unknown model or target row, or
// m outside 1..4096 is not run: its loss is set to NaN.
#include <cmath>

#include "ges_internal.h"

namespace ges {

constexpr int kMixThreads = 256;
constexpr int kMixMaxN = GES_MIX_MAX_COMPONENTS;
constexpr int kMixMaxM = GES_MIX_MAX_POINTS;
constexpr float kMixEps = 1e-8f;
constexpr float kMixNu = 4.f;

struct MixArgs {
  const ges_mix_problem* problems;
  const float* targets;
  int32_t ntargets, m;
  float x0, dx;
  float* params;          // [P][kMixMaxN][4]
  float* grad_out;        // [P][kMixMaxN][4] gradient at the initial parameters, or NULL
  float* final_loss;      // [P]
  const int32_t* order;   // [P] problem index per block (a permutation), or NULL for the identity
  int32_t nproblems;
  int32_t epochs;
  float lr, b1, b2, eps;
};

// Per-component constants of one epoch.
struct MixComp {
  float w, dw, mu, s, beta, inv1, inv2;   // inv1 = 1/(2 s^2 + eps); inv2 = 1/(2 s^2/nu + eps) (DoG)
};

__device__ __forceinline__ MixComp mix_prepare(const float* th, int positive) {
  MixComp c;
  const float w_raw = th[0];
  c.mu = th[1];
  c.s = th[2];
  c.beta = th[3];
  if (positive) {
    c.w = w_raw > 30.f ? w_raw : log1pf(expf(fminf(w_raw, 30.f)));
    c.dw = 1.f / (1.f + expf(-w_raw));
  } else {
    c.w = w_raw;
    c.dw = 1.f;
  }
  c.inv1 = 1.f / (2.f * c.s * c.s + kMixEps);
  c.inv2 = 1.f / (2.f * c.s * c.s / kMixNu + kMixEps);
  return c;
}

// Value of one component at x; with want_grad also its derivatives w.r.t. (w_raw, mu, s, beta).
template <bool want_grad>
__device__ __forceinline__ float mix_eval(int model, const MixComp& c, float x, float* g) {
  const float d = x - c.mu, d2 = d * d;
  float base, db_mu = 0.f, db_s = 0.f, db_beta = 0.f;
  if (model == GES_MIX_GEF) {
    const float ad = fabsf(d);
    const float a = ad == 0.f ? powf(0.f, c.beta) : expf(c.beta * logf(ad));
    base = expf(-a * c.inv1);
    if (want_grad) {
      float da_mu = 0.f, da_b = 0.f;
      if (ad != 0.f) {
        da_mu = -c.beta * expf((c.beta - 1.f) * logf(ad)) * (d > 0.f ? 1.f : -1.f);
        da_b = a * logf(ad);
      }
      db_mu = -base * da_mu * c.inv1;
      db_s = base * a * 4.f * c.s * c.inv1 * c.inv1;
      db_beta = -base * da_b * c.inv1;
    }
  } else {
    const float E1 = expf(-d2 * c.inv1);
    if (model == GES_MIX_GMM) {
      base = E1;
      if (want_grad) {
        db_mu = E1 * 2.f * d * c.inv1;
        db_s = E1 * d2 * 4.f * c.s * c.inv1 * c.inv1;
      }
    } else if (model == GES_MIX_DOG) {
      const float E2 = expf(-d2 * c.inv2);
      base = E1 - E2;
      if (want_grad) {
        db_mu = E1 * 2.f * d * c.inv1 - E2 * 2.f * d * c.inv2;
        db_s = E1 * d2 * 4.f * c.s * c.inv1 * c.inv1 - E2 * d2 * (4.f * c.s / kMixNu) * c.inv2 * c.inv2;
      }
    } else {   // LoG
      const float is2 = 1.f / (c.s * c.s);
      const float P = 1.f - d2 * is2;
      base = P * E1;
      if (want_grad) {
        db_mu = 2.f * d * is2 * E1 + P * E1 * 2.f * d * c.inv1;
        db_s = 2.f * d2 * is2 / c.s * E1 + P * E1 * d2 * 4.f * c.s * c.inv1 * c.inv1;
      }
    }
  }
  if (want_grad) {
    g[0] = c.dw * base;
    g[1] = c.w * db_mu;
    g[2] = c.w * db_s;
    g[3] = c.w * db_beta;
  }
  return c.w * base;
}

__global__ void __launch_bounds__(kMixThreads) mix_fit_kernel(const MixArgs a) {
  __shared__ float sy[kMixMaxM];
  __shared__ float sr[kMixMaxM];
  __shared__ float th[kMixMaxN][4];
  __shared__ float mo[kMixMaxN][4];
  __shared__ float ve[kMixMaxN][4];
  __shared__ float gr[kMixMaxN][4];
  __shared__ MixComp comp[kMixMaxN];
  __shared__ float lsum[kMixThreads / 64];
  // blocks take problems from the largest n down (a problem's time grows with n), so the longest ones do
  // not start last; results go to the problem's own rows
  const int p = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
  if (p < 0 || p >= a.nproblems) return;   // not a problem of this batch: nothing to do
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const ges_mix_problem pr = a.problems[p];
  const int n = pr.n, model = pr.model, positive = pr.positive;
  const int M = a.m;
  if (n < 1 || n > kMixMaxN || model < 0 || model > GES_MIX_GEF || pr.target < 0 || pr.target >= a.ntargets ||
      M < 1 || M > kMixMaxM) {
    if (t == 0) a.final_loss[p] = __int_as_float(0x7fc00000);
    return;
  }
  float* P = a.params + (size_t)p * kMixMaxN * 4;
  const float* y = a.targets + (size_t)pr.target * M;
  for (int j = t; j < M; j += kMixThreads) sy[j] = y[j];
  for (int q = t; q < n * 4; q += kMixThreads) {
    th[q >> 2][q & 3] = P[q];
    mo[q >> 2][q & 3] = 0.f;
    ve[q >> 2][q & 3] = 0.f;
  }
  __syncthreads();
  const float scale = 2.f / (float)M;
  for (int ep = 0; ep <= a.epochs; ++ep) {
    // 1. per-component constants
    for (int i = t; i < n; i += kMixThreads) comp[i] = mix_prepare(th[i], positive);
    __syncthreads();
    // 2. residuals (and, after the last update, the loss)
    float l2 = 0.f;
    for (int j = t; j < M; j += kMixThreads) {
      const float x = a.x0 + (float)j * a.dx;
      float v = 0.f;
      for (int i = 0; i < n; ++i) v += mix_eval<false>(model, comp[i], x, nullptr);
      const float r = v - sy[j];
      sr[j] = r;
      l2 = __builtin_fmaf(r, r, l2);
    }
    if (ep == a.epochs) {   // final loss: mean r^2 over the points, lanes then waves in a fixed order
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) l2 += __shfl_xor(l2, off, 64);
      if (lane == 0) lsum[wave] = l2;
      __syncthreads();
      if (t == 0) a.final_loss[p] = (((lsum[0] + lsum[1]) + lsum[2]) + lsum[3]) / (float)M;
      break;
    }
    __syncthreads();
    // 3. gradients
    for (int i = wave; i < n; i += kMixThreads / 64) {
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      const MixComp c = comp[i];
      for (int j = lane; j < M; j += 64) {
        float g[4];
        mix_eval<true>(model, c, a.x0 + (float)j * a.dx, g);
        const float r = sr[j];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = __builtin_fmaf(r, g[k], acc[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
      }
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) gr[i][k] = acc[k] * scale;
      }
    }
    __syncthreads();
    if (ep == 0 && a.grad_out) {
      float* G = a.grad_out + (size_t)p * kMixMaxN * 4;
      for (int q = t; q < n * 4; q += kMixThreads) G[q] = gr[q >> 2][q & 3];
    }
    // 4. Adam (bias corrections of step ep + 1 in binary64, as on the host for the splat optimiser)
    const int step = ep + 1;
    const double bc1 = 1.0 - pow((double)a.b1, (double)step), bc2 = 1.0 - pow((double)a.b2, (double)step);
    const float step_size = (float)((double)a.lr / bc1), inv_sqrt_bc2 = (float)(1.0 / sqrt(bc2));
    for (int q = t; q < n * 4; q += kMixThreads) {
      float& pv = th[q >> 2][q & 3];
      adam_update(pv, gr[q >> 2][q & 3], mo[q >> 2][q & 3], ve[q >> 2][q & 3], a.b1, a.b2, a.eps, step_size,
                  inv_sqrt_bc2);
    }
    __syncthreads();
  }
  for (int q = t; q < n * 4; q += kMixThreads) P[q] = th[q >> 2][q & 3];
}

hipError_t launch_mix_fit(const ges_mix_problem* problems, int nproblems, const float* targets, int ntargets, int m,
                          float x0, float dx, float* params, float* grad_out, float* final_loss, const int32_t* order,
                          int epochs, float lr, float b1, float b2, float eps, hipStream_t stream) {
  if (nproblems == 0) return hipSuccess;
  MixArgs a{problems, targets, ntargets, m, x0, dx, params, grad_out, final_loss, order, nproblems, epochs, lr, b1,
            b2, eps};
  hipLaunchKernelGGL(mix_fit_kernel, dim3((unsigned)nproblems), dim3(kMixThreads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace ges
