// prune.hip -- shape/opacity pruning and shape reset of the GES training loop (Sec. 4.4, Sec. 5.2,
// App. B.2).
//
// Pruning removes every splat whose opacity sigmoid(logit) is below a bound or whose beta is below a bound,
// and compacts the survivors, in their original order, into the caller's destination arrays: the
// parameters and, with them, the optimiser moments.  The opacity test is taken on the logit against
// ln(t / (1 - t)) in binary64, the beta test in binary64 too, so the decision is exact and fixed.
//   1. prune_count_kernel: each block counts its survivors (wave ballots);
//   2. prune_scan_kernel: one block turns the counts into exclusive block offsets and the total;
//   3. prune_scatter_kernel: each block ranks its survivors (ballot prefix + wave offsets in LDS) and copies
//      their rows of every array to offset + rank.
// Shape reset sets every beta to one value and clears beta's moments.
// Memory: the pass reads each splat's row of every array once and writes the survivors' rows once; it runs
// every 100 iterations, not every step.
#include <algorithm>

#include "ges_internal.h"

namespace ges {

constexpr int kPruneThreads = 256;
constexpr int kScanThreads = 1024;

struct PruneArgs {
  const float* src[kMaxPruneArrays];
  float* dst[kMaxPruneArrays];
  int32_t rowlen[kMaxPruneArrays];   // floats per splat (0: array absent)
  const float* opacity_logits;
  const float* beta;
  int64_t n;
  double logit_bound;                // survivors have logit >= bound
  double min_beta;                   // and beta >= min_beta
};

__device__ __forceinline__ bool survives(const PruneArgs& a, int64_t i) {
  return !((double)a.opacity_logits[i] < a.logit_bound) && !((double)a.beta[i] < a.min_beta);
}

__global__ void __launch_bounds__(kPruneThreads) prune_count_kernel(const PruneArgs a, uint32_t* __restrict__ counts) {
  __shared__ uint32_t wcount[kPruneThreads / 64];
  const int64_t i = (int64_t)blockIdx.x * kPruneThreads + threadIdx.x;
  const bool keep = i < a.n && survives(a, i);
  const uint64_t ballot = __ballot(keep);
  if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = (uint32_t)__popcll(ballot);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int k = 0; k < kPruneThreads / 64; ++k) s += wcount[k];
    counts[blockIdx.x] = s;
  }
}

// Exclusive offsets of nb block counts and the total (one block; each thread scans a contiguous chunk).
__global__ void __launch_bounds__(kScanThreads) prune_scan_kernel(const uint32_t* __restrict__ counts, int64_t nb,
                                                                 uint32_t* __restrict__ offsets,
                                                                 int64_t* __restrict__ total) {
  __shared__ uint64_t part[kScanThreads];
  const int t = threadIdx.x;
  const int64_t chunk = (nb + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = std::min<int64_t>(nb, (int64_t)t * chunk), b1 = std::min<int64_t>(nb, b0 + chunk);
  uint64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += counts[b];
  part[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the chunk sums
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint64_t run = part[t] - s;   // exclusive start of this chunk
  for (int64_t b = b0; b < b1; ++b) {
    offsets[b] = (uint32_t)run;
    run += counts[b];
  }
  if (t == kScanThreads - 1) *total = (int64_t)part[t];
}

__global__ void __launch_bounds__(kPruneThreads) prune_scatter_kernel(const PruneArgs a,
                                                                      const uint32_t* __restrict__ offsets) {
  __shared__ uint32_t wbase[kPruneThreads / 64];
  const int64_t i = (int64_t)blockIdx.x * kPruneThreads + threadIdx.x;
  const bool keep = i < a.n && survives(a, i);
  const uint64_t ballot = __ballot(keep);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wbase[wave] = (uint32_t)__popcll(ballot);
  __syncthreads();
  if (!keep) return;
  uint32_t base = offsets[blockIdx.x];
  for (int k = 0; k < wave; ++k) base += wbase[k];
  const uint64_t below = lane == 0 ? 0ull : (ballot & (~0ull >> (64 - lane)));
  const int64_t j = (int64_t)base + __popcll(below);
#pragma unroll
  for (int arr = 0; arr < kMaxPruneArrays; ++arr) {
    const int len = a.rowlen[arr];
    if (len == 0) continue;
    const float* s = a.src[arr] + i * len;
    float* d = a.dst[arr] + j * len;
    for (int k = 0; k < len; ++k) d[k] = s[k];
  }
}

__global__ void shape_reset_kernel(float* __restrict__ beta, float* __restrict__ m, float* __restrict__ v, int64_t n,
                                   float value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    beta[i] = value;
    if (m) m[i] = 0.f;
    if (v) v[i] = 0.f;
  }
}

size_t prune_scratch_bytes(int64_t n) {
  const int64_t nb = (n + kPruneThreads - 1) / kPruneThreads;
  return 256 + ((8 * (size_t)nb + 255) / 256) * 256;
}

hipError_t launch_prune(const float* const* src, float* const* dst, const int32_t* rowlen, const float* opacity_logits,
                        const float* beta, int64_t n, double logit_bound, double min_beta, void* scratch,
                        int64_t* total_dev, hipStream_t stream) {
  PruneArgs a{};
  for (int k = 0; k < kMaxPruneArrays; ++k) {
    a.src[k] = src[k];
    a.dst[k] = dst[k];
    a.rowlen[k] = rowlen[k];
  }
  a.opacity_logits = opacity_logits;
  a.beta = beta;
  a.n = n;
  a.logit_bound = logit_bound;
  a.min_beta = min_beta;
  const int64_t nb = (n + kPruneThreads - 1) / kPruneThreads;
  uint32_t* counts = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(scratch) + 256);
  uint32_t* offsets = counts + nb;
  if (nb > 0) hipLaunchKernelGGL(prune_count_kernel, dim3((unsigned)nb), dim3(kPruneThreads), 0, stream, a, counts);
  hipLaunchKernelGGL(prune_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, (const uint32_t*)counts, nb, offsets,
                     total_dev);
  if (nb > 0)
    hipLaunchKernelGGL(prune_scatter_kernel, dim3((unsigned)nb), dim3(kPruneThreads), 0, stream, a,
                       (const uint32_t*)offsets);
  return hipGetLastError();
}

hipError_t launch_block_scan(const uint32_t* counts, int64_t nb, uint32_t* offsets, int64_t* total,
                             hipStream_t stream) {
  hipLaunchKernelGGL(prune_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, counts, nb, offsets, total);
  return hipGetLastError();
}

hipError_t launch_shape_reset(float* beta, float* m, float* v, int64_t n, float value, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(shape_reset_kernel, dim3(blocks), dim3(256), 0, stream, beta, m, v, n, value);
  return hipGetLastError();
}

}  // namespace ges
