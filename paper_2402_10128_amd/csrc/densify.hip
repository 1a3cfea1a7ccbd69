// densify.hip -- densification kept from Gaussian splatting (Sec. 5.2; App. B.2) and the opacity reset.
//
// Each splat is kept (0), kept and cloned (1) or split (2): selected when its mean NDC mean-2D gradient
// (accumulator / count, 0 when never visible) is at least the threshold, then cloned when its largest
// log-scale is at most ln(percent_dense * extent) and split otherwise; both tests in binary64, so the
// decision is exact.  The output holds the unsplit splats in order, then the clones in the order of their
// sources, then two children per split splat: means mu + R(q) (s * z_k) for the given normal draws, log-scales
// reduced by ln 1.6 (both in binary64), every other parameter copied.  Optimiser moments follow the kept
// splats and are zero for clones and children.
//   1. densify_count_kernel: per block, the counts of unsplit, cloned and split splats (wave ballots);
//   2. three exclusive scans of those counts (the pruning scan);
//   3. densify_scatter_kernel: per block, ranks from ballot prefixes, then the row copies.
// The opacity reset lowers every opacity above 0.01 to 0.01 (on the logit) and clears its moments.
#include <algorithm>
#include <cmath>

#include "ges_internal.h"

namespace ges {

constexpr int kDensThreads = 256;

struct DensArgs {
  const float* src[kMaxPruneArrays];
  float* dst[kMaxPruneArrays];
  int32_t rowlen[kMaxPruneArrays];
  int32_t nsets;
  const float* accum;
  const float* count;
  const float* log_scales;    // parameters' log-scales (set 0)
  const float* normals;       // [n][2][3]
  int64_t n;
  double grad_threshold, log_scale_bound, log_split_div;
  int64_t unsplit, clones;    // output sections: [0, unsplit) [unsplit, +clones) [unsplit+clones, +2 splits)
};

__device__ __forceinline__ int dens_kind(const float* accum, const float* count, const float* ls, int64_t i,
                                         double thr, double lbound) {
  const double c = (double)count[i];
  const double mean = c > 0.0 ? (double)accum[i] / c : 0.0;
  if (!(mean >= thr)) return 0;
  const double lmax = fmax(fmax((double)ls[3 * i], (double)ls[3 * i + 1]), (double)ls[3 * i + 2]);
  return lmax <= lbound ? 1 : 2;
}

// rank of this lane among the lanes of the block whose flag is set, and the block's count
__device__ __forceinline__ uint32_t block_rank(bool flag, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t ballot = __ballot(flag);
  if (lane == 0) wsum[wave] = (uint32_t)__popcll(ballot);
  __syncthreads();
  uint32_t base = 0, all = 0;
  for (int k = 0; k < kDensThreads / 64; ++k) {
    if (k < wave) base += wsum[k];
    all += wsum[k];
  }
  __syncthreads();
  *total = all;
  const uint64_t below = lane == 0 ? 0ull : (ballot & (~0ull >> (64 - lane)));
  return base + (uint32_t)__popcll(below);
}

__global__ void __launch_bounds__(kDensThreads) densify_count_kernel(const float* __restrict__ accum,
                                                                     const float* __restrict__ count,
                                                                     const float* __restrict__ ls, int64_t n, double thr,
                                                                     double lbound, uint32_t* __restrict__ counts,
                                                                     int64_t nb) {
  __shared__ uint32_t wsum[kDensThreads / 64];
  const int64_t i = (int64_t)blockIdx.x * kDensThreads + threadIdx.x;
  const int kind = i < n ? dens_kind(accum, count, ls, i, thr, lbound) : -1;
  uint32_t tu, tc, ts;
  block_rank(kind == 0 || kind == 1, wsum, &tu);
  block_rank(kind == 1, wsum, &tc);
  block_rank(kind == 2, wsum, &ts);
  if (threadIdx.x == 0) {
    counts[blockIdx.x] = tu;
    counts[nb + blockIdx.x] = tc;
    counts[2 * nb + blockIdx.x] = ts;
  }
}

__device__ __forceinline__ void copy_row(const float* s, float* d, int len) {
  for (int k = 0; k < len; ++k) d[k] = s[k];
}

__global__ void __launch_bounds__(kDensThreads) densify_scatter_kernel(const DensArgs a,
                                                                       const uint32_t* __restrict__ offsets,
                                                                       int64_t nb) {
  __shared__ uint32_t wsum[kDensThreads / 64];
  const int64_t i = (int64_t)blockIdx.x * kDensThreads + threadIdx.x;
  const int kind = i < a.n ? dens_kind(a.accum, a.count, a.log_scales, i, a.grad_threshold, a.log_scale_bound) : -1;
  uint32_t tu, tc, ts;
  const uint32_t ru = block_rank(kind == 0 || kind == 1, wsum, &tu);
  const uint32_t rc = block_rank(kind == 1, wsum, &tc);
  const uint32_t rs = block_rank(kind == 2, wsum, &ts);
  if (kind < 0) return;
  if (kind != 2) {   // the splat itself, with its moments
    const int64_t j = (int64_t)offsets[blockIdx.x] + ru;
#pragma unroll
    for (int arr = 0; arr < kMaxPruneArrays; ++arr)
      if (a.rowlen[arr]) copy_row(a.src[arr] + i * a.rowlen[arr], a.dst[arr] + j * a.rowlen[arr], a.rowlen[arr]);
  }
  if (kind == 1) {   // its clone: parameters copied, moments zero
    const int64_t j = a.unsplit + (int64_t)offsets[nb + blockIdx.x] + rc;
#pragma unroll
    for (int arr = 0; arr < kMaxPruneArrays; ++arr) {
      const int len = a.rowlen[arr];
      if (!len) continue;
      float* d = a.dst[arr] + j * len;
      if (arr < kNumPar) copy_row(a.src[arr] + i * len, d, len);
      else for (int k = 0; k < len; ++k) d[k] = 0.f;
    }
  }
  if (kind == 2) {   // two children
    const int64_t j0 = a.unsplit + a.clones + 2 * ((int64_t)offsets[2 * nb + blockIdx.x] + rs);
    const float* q = a.src[kParQuats] + 4 * i;
    const double qn = sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]);
    const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                         2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
    const float* ls = a.src[kParScales] + 3 * i;
    const double s[3] = {exp((double)ls[0]), exp((double)ls[1]), exp((double)ls[2])};
    const float* mu = a.src[kParMeans] + 3 * i;
    for (int c = 0; c < 2; ++c) {
      const int64_t j = j0 + c;
      const float* zc = a.normals + 6 * i + 3 * c;
      const double o[3] = {s[0] * (double)zc[0], s[1] * (double)zc[1], s[2] * (double)zc[2]};
#pragma unroll
      for (int arr = 0; arr < kMaxPruneArrays; ++arr) {
        const int len = a.rowlen[arr];
        if (!len) continue;
        float* d = a.dst[arr] + j * len;
        if (arr == kParMeans) {
          for (int r = 0; r < 3; ++r)
            d[r] = (float)((double)mu[r] + (R[3 * r] * o[0] + R[3 * r + 1] * o[1] + R[3 * r + 2] * o[2]));
        } else if (arr == kParScales) {
          for (int r = 0; r < 3; ++r) d[r] = (float)((double)ls[r] - a.log_split_div);
        } else if (arr < kNumPar) {
          copy_row(a.src[arr] + i * len, d, len);
        } else {
          for (int k = 0; k < len; ++k) d[k] = 0.f;
        }
      }
    }
  }
}

__global__ void opacity_reset_kernel(float* __restrict__ logits, float* __restrict__ m, float* __restrict__ v,
                                     int64_t n, double bound) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if ((double)logits[i] > bound) logits[i] = (float)bound;
    if (m) m[i] = 0.f;
    if (v) v[i] = 0.f;
  }
}

// scratch: [0, 256) the three totals; then counts[3][nb]; then offsets[3][nb]
size_t densify_scratch_bytes(int64_t n) {
  const int64_t nb = (n + kDensThreads - 1) / kDensThreads;
  return 256 + ((24 * (size_t)nb + 255) / 256) * 256;
}

hipError_t launch_densify_count(const float* accum, const float* count, const float* log_scales, int64_t n,
                                double grad_threshold, double log_scale_bound, void* scratch, hipStream_t stream) {
  const int64_t nb = (n + kDensThreads - 1) / kDensThreads;
  int64_t* totals = reinterpret_cast<int64_t*>(scratch);
  uint32_t* counts = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(scratch) + 256);
  uint32_t* offsets = counts + 3 * nb;
  if (nb > 0)
    hipLaunchKernelGGL(densify_count_kernel, dim3((unsigned)nb), dim3(kDensThreads), 0, stream, accum, count,
                       log_scales, n, grad_threshold, log_scale_bound, counts, nb);
  for (int k = 0; k < 3; ++k) {
    const hipError_t e = launch_block_scan(counts + k * nb, nb, offsets + k * nb, totals + k, stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_densify_scatter(const float* const* src, float* const* dst, const int32_t* rowlen, int nsets,
                                  const float* accum, const float* count, const float* normals, int64_t n,
                                  double grad_threshold, double log_scale_bound, double log_split_div, int64_t unsplit,
                                  int64_t clones, void* scratch, hipStream_t stream) {
  const int64_t nb = (n + kDensThreads - 1) / kDensThreads;
  if (nb == 0) return hipSuccess;
  DensArgs a{};
  for (int k = 0; k < kMaxPruneArrays; ++k) {
    a.src[k] = src[k];
    a.dst[k] = dst[k];
    a.rowlen[k] = rowlen[k];
  }
  a.nsets = nsets;
  a.accum = accum;
  a.count = count;
  a.log_scales = src[kParScales];
  a.normals = normals;
  a.n = n;
  a.grad_threshold = grad_threshold;
  a.log_scale_bound = log_scale_bound;
  a.log_split_div = log_split_div;
  a.unsplit = unsplit;
  a.clones = clones;
  const uint32_t* offsets = reinterpret_cast<const uint32_t*>(reinterpret_cast<char*>(scratch) + 256) + 3 * nb;
  hipLaunchKernelGGL(densify_scatter_kernel, dim3((unsigned)nb), dim3(kDensThreads), 0, stream, a, offsets, nb);
  return hipGetLastError();
}

hipError_t launch_opacity_reset(float* logits, float* m, float* v, int64_t n, double bound, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(opacity_reset_kernel, dim3(blocks), dim3(256), 0, stream, logits, m, v, n, bound);
  return hipGetLastError();
}

}  // namespace ges
