// optim.hip -- fused Adam step over the splat parameter groups of the GES training step (App. B.2).
//
// Adam (Kingma & Ba, 2015, Algorithm 1) with the bias corrections folded into two scalars:
//   m <- b1 m + (1 - b1) g;   v <- b2 v + (1 - b2) g^2;
//   p <- p - (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps).
// Every group (position, SH features, opacity, shape beta, rotation, scaling) carries its own learning
// rate; one launch covers all groups: block b belongs to the group whose block range holds it.
//
// Memory: each parameter reads p, g, m, v and writes p, m, v (28 B); nothing is re-read, so the kernel is
// HBM-bound.  Threads move float4 vectors when the group's four arrays are 16-byte aligned, and the
// vectors of one block are issued together so each thread has sixteen loads in flight.
#include <algorithm>
#include <cmath>

#include "ges_internal.h"

namespace ges {

constexpr int kAdamThreads = 256;
constexpr int kAdamVecPerThread = 4;                                       // float4 vectors per thread
constexpr int64_t kAdamBlockFloats = (int64_t)kAdamThreads * kAdamVecPerThread * 4;

struct AdamGroupArg {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t count;
  int64_t block0;     // first block of the group
  float step_size;    // lr / (1 - b1^t)
  int32_t vec;        // 1: p, g, m, v all 16-byte aligned
};

struct AdamArgs {
  AdamGroupArg grp[kAdamMaxGroups];
  int32_t ngroups;
  float b1, b2, eps, inv_sqrt_bc2;
};

__global__ void __launch_bounds__(kAdamThreads) adam_kernel(const AdamArgs a) {
  const int64_t b = blockIdx.x;
  // pick the group with compile-time indices only (the argument table stays in scalar registers)
  AdamGroupArg G = a.grp[0];
#pragma unroll
  for (int k = 1; k < kAdamMaxGroups; ++k)
    if (k < a.ngroups && b >= a.grp[k].block0) G = a.grp[k];
  const int64_t base = (b - G.block0) * kAdamBlockFloats;
  const int t = threadIdx.x;
  if (G.vec) {
    const int64_t nvec = G.count >> 2;
    const int64_t v0 = (base >> 2) + t;
    float4 P[kAdamVecPerThread], Gr[kAdamVecPerThread], M[kAdamVecPerThread], V[kAdamVecPerThread];
#pragma unroll
    for (int j = 0; j < kAdamVecPerThread; ++j) {
      const int64_t i = v0 + (int64_t)j * kAdamThreads;
      if (i < nvec) {
        P[j] = reinterpret_cast<const float4*>(G.p)[i];
        Gr[j] = reinterpret_cast<const float4*>(G.g)[i];
        M[j] = reinterpret_cast<const float4*>(G.m)[i];
        V[j] = reinterpret_cast<const float4*>(G.v)[i];
      }
    }
#pragma unroll
    for (int j = 0; j < kAdamVecPerThread; ++j) {
      const int64_t i = v0 + (int64_t)j * kAdamThreads;
      if (i < nvec) {
        adam_update(P[j].x, Gr[j].x, M[j].x, V[j].x, a.b1, a.b2, a.eps, G.step_size, a.inv_sqrt_bc2);
        adam_update(P[j].y, Gr[j].y, M[j].y, V[j].y, a.b1, a.b2, a.eps, G.step_size, a.inv_sqrt_bc2);
        adam_update(P[j].z, Gr[j].z, M[j].z, V[j].z, a.b1, a.b2, a.eps, G.step_size, a.inv_sqrt_bc2);
        adam_update(P[j].w, Gr[j].w, M[j].w, V[j].w, a.b1, a.b2, a.eps, G.step_size, a.inv_sqrt_bc2);
        reinterpret_cast<float4*>(G.p)[i] = P[j];
        reinterpret_cast<float4*>(G.m)[i] = M[j];
        reinterpret_cast<float4*>(G.v)[i] = V[j];
      }
    }
    // the last block also takes the (count mod 4) trailing floats
    const int64_t tail0 = nvec << 2;
    if (base + kAdamBlockFloats >= G.count && t < (int)(G.count - tail0)) {
      const int64_t i = tail0 + t;
      float p = G.p[i], m = G.m[i], v = G.v[i];
      adam_update(p, G.g[i], m, v, a.b1, a.b2, a.eps, G.step_size, a.inv_sqrt_bc2);
      G.p[i] = p;
      G.m[i] = m;
      G.v[i] = v;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4 * kAdamVecPerThread; ++j) {
      const int64_t i = base + t + (int64_t)j * kAdamThreads;
      if (i < G.count) {
        float p = G.p[i], m = G.m[i], v = G.v[i];
        adam_update(p, G.g[i], m, v, a.b1, a.b2, a.eps, G.step_size, a.inv_sqrt_bc2);
        G.p[i] = p;
        G.m[i] = m;
        G.v[i] = v;
      }
    }
  }
}

hipError_t launch_adam(const ges_adam_group* groups, int ngroups, int64_t step, float b1, float b2, float eps,
                       hipStream_t stream) {
  AdamArgs a{};
  a.ngroups = ngroups;
  a.b1 = b1;
  a.b2 = b2;
  a.eps = eps;
  const double bc1 = 1.0 - std::pow((double)b1, (double)step);
  const double bc2 = 1.0 - std::pow((double)b2, (double)step);
  a.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
  int64_t blocks = 0;
  for (int k = 0; k < kAdamMaxGroups; ++k) {
    AdamGroupArg& G = a.grp[k];
    if (k >= ngroups) {               // unused slots start past the last block, so no block selects them
      G.block0 = INT64_MAX;
      continue;
    }
    const ges_adam_group& s = groups[k];
    G.p = s.params;
    G.g = s.grads;
    G.m = s.exp_avg;
    G.v = s.exp_avg_sq;
    G.count = s.count;
    G.block0 = blocks;
    G.step_size = (float)((double)s.lr / bc1);
    const uintptr_t al = reinterpret_cast<uintptr_t>(s.params) | reinterpret_cast<uintptr_t>(s.grads) |
                         reinterpret_cast<uintptr_t>(s.exp_avg) | reinterpret_cast<uintptr_t>(s.exp_avg_sq);
    G.vec = (al & 15u) == 0 ? 1 : 0;
    blocks += (s.count + kAdamBlockFloats - 1) / kAdamBlockFloats;
  }
  if (blocks == 0) return hipSuccess;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(kAdamThreads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace ges
