// radix.hip -- one stable LSD radix pass over (u32 key, u32 value) items with digits of up to 8 bits.
//
// Reduce-then-scan, three launches per pass:
//   upsweep:   each block counts the digits of its items in per-wave LDS histograms and writes its 256
//              counts into the digit table ([16 digit groups][nblocks][16], see radix_tidx);
//   scan:      one block per digit turns its counts into exclusive per-block offsets and writes the
//              digit's total;
//   downsweep: each block ranks its items stably -- every wave owns a contiguous quarter of the block's
//              items and ranks them 64 at a time with one ballot per digit bit (lanes holding the same
//              digit) against wave-private digit counters -- places them in LDS in digit order, and writes
//              each digit's run to its global position (exclusive digit total prefix + the block's offset),
//              so that consecutive threads write consecutive addresses.
// A tile holds 256 x ITEMS items, 8 per thread for both sorts (measured against 4, 12 and 16: more items
// leave room for fewer blocks per compute unit in LDS, fewer make the digit table longer), and a block takes
// `sub` tiles in turn when there are many (a row of the digit table per block, not per tile: the table's
// strided writes and reads, and its scan, shrink by that factor).  A filtering pass
// drops items whose key is kNoKey (compaction) and stores the kept count.  With PAIR, a value is a (u32, slot) pair whose slot is
// the item's index in the pass that makes the pairs: the pair sort carries each pair's slot in the
// candidate layout to the backward pass.
#include "ges_internal.h"

namespace ges {

__device__ __forceinline__ uint64_t radix_lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ void radix_wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Lanes of this wave holding the same digit (valid lanes only), one ballot per digit bit.
__device__ __forceinline__ uint64_t radix_peers(bool valid, uint32_t dg, int bits) {
  uint64_t peers = __ballot(valid);
  for (int bit = 0; bit < bits; ++bit) {
    const uint32_t b = (dg >> bit) & 1u;
    const uint64_t m = __ballot(b != 0u);
    const uint32_t flip = b - 1u;   // 0 if the lane's bit is set, all ones if not
    const uint32_t lo = (uint32_t)m ^ flip, hi = (uint32_t)(m >> 32) ^ flip;
    peers &= ((uint64_t)hi << 32) | lo;
  }
  return peers;
}

__device__ __forceinline__ uint32_t radix_count(const RadixPass& p) {
  return p.count_dev ? *p.count_dev : p.count_host;
}

__device__ __forceinline__ uint32_t radix_digit(const RadixPass& p, uint32_t k) {
  return (k >> p.shift) & ((1u << p.bits) - 1u);
}

// The digit table holds, per block b and digit d, the block's count of d and then its exclusive prefix over
// the blocks.  Layout [d / 16][b][d % 16]: a block's 256 entries are 16 runs of 64 contiguous bytes (its
// writes in the upsweep and reads in the downsweep are whole segments; digit-major rows of 4-byte entries
// left a partial segment per entry), and a group of 16 digits is a contiguous [blocks][16] array for the
// scan.
constexpr int kDigitGroup = 16;
__device__ __forceinline__ size_t radix_tidx(uint32_t d, uint32_t b, uint32_t nblocks) {
  return ((size_t)(d / kDigitGroup) * nblocks + b) * kDigitGroup + (d % kDigitGroup);
}

template <int ITEMS>
__global__ void __launch_bounds__(kRadixThreads) radix_upsweep_kernel(RadixPass p) {
  constexpr int kWaves = kRadixThreads / 64;
  __shared__ uint32_t hist[kWaves][256];
  const uint32_t n = radix_count(p);
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) hist[k][threadIdx.x] = 0u;
  __syncthreads();
  for (int sub = 0; sub < p.sub; ++sub) {
    const uint64_t base = ((uint64_t)blockIdx.x * p.sub + sub) * (kRadixThreads * ITEMS);
    if (base >= n) break;
    uint32_t key[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const uint64_t i = base + (uint64_t)it * kRadixThreads + threadIdx.x;
      key[it] = i < n ? p.keys_in[i] : kNoKey;
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const uint64_t i = base + (uint64_t)it * kRadixThreads + threadIdx.x;
      if (i < n && !(p.filter && key[it] == kNoKey)) atomicAdd(&hist[w][radix_digit(p, key[it])], 1u);
    }
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) c += hist[k][threadIdx.x];
  p.table[radix_tidx(threadIdx.x, blockIdx.x, p.nblocks)] = c;
}

// One block per digit: the exclusive scan of the digit's counts over the blocks (8 entries per thread per
// round, 1,024 threads: one round for up to 8,192 blocks), its total to totals[].  The 16 digits of a group
// share the table's 64-byte segments, so they are dealt to one XCD (blocks go to the XCDs round-robin) and
// each segment is fetched once into that XCD's L2.  Digits beyond the pass's width only clear their total.
constexpr int kScanThreads = 1024;
__global__ void __launch_bounds__(kScanThreads) radix_scan_kernel(RadixPass p) {
  constexpr int kPer = 8;
  __shared__ uint32_t wsum[kScanThreads / 64];
  __shared__ uint32_t carry;
  const uint32_t x = blockIdx.x & 7u, i = blockIdx.x >> 3;   // XCD, and the block's index on it
  const uint32_t d = (((i / kDigitGroup) << 3) + x) * kDigitGroup + (i % kDigitGroup);
  if (d >= (1u << p.bits)) {
    if (threadIdx.x == 0) p.totals[d] = 0u;
    return;
  }
  uint32_t* col = p.table + radix_tidx(d, 0, p.nblocks);   // entry of block b at col[16 b]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0u;
  __syncthreads();
  for (uint32_t base = 0; base < p.nblocks; base += kScanThreads * kPer) {
    const uint32_t j0 = base + threadIdx.x * kPer;
    uint32_t v[kPer];
    uint32_t local = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      v[k] = j0 + k < p.nblocks ? col[(size_t)(j0 + k) * kDigitGroup] : 0u;
      local += v[k];
    }
    uint32_t s = local;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)s, dd, 64);
      if (lane >= dd) s += y;
    }
    if (lane == 63) wsum[w] = s;
    __syncthreads();
    uint32_t run = carry + s - local;
    for (int k = 0; k < w; ++k) run += wsum[k];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (j0 + k < p.nblocks) col[(size_t)(j0 + k) * kDigitGroup] = run;
      run += v[k];
    }
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) carry = run;
    __syncthreads();
  }
  if (threadIdx.x == 0) p.totals[d] = carry;
}

template <bool PAIR>
struct RadixVal { typedef uint32_t T; };
template <>
struct RadixVal<true> { typedef uint2 T; };

template <int ITEMS, bool PAIR>
__global__ void __launch_bounds__(kRadixThreads) radix_downsweep_kernel(RadixPass p) {
  typedef typename RadixVal<PAIR>::T Val;
  constexpr int kWaves = kRadixThreads / 64;
  constexpr int kTile = kRadixThreads * ITEMS;
  constexpr int kPerWave = kTile / kWaves;   // contiguous items of one wave
  __shared__ uint32_t sk[kTile];
  __shared__ Val sv[kTile];
  __shared__ uint32_t cnt[kWaves][256];   // per-wave digit counts, then each wave's base within its digit
  __shared__ uint32_t dstart[256];        // block-local start of each digit
  __shared__ uint32_t gstart[256];        // global position of the block's first item of each digit
  __shared__ uint32_t wsum[2][kWaves];
  __shared__ uint32_t kept;
  const uint32_t n = radix_count(p);
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, t = threadIdx.x;
  if (blockIdx.x == 0 && t == 0 && p.filter && p.count_out) {
    uint32_t total = 0;
    for (int d = 0; d < 256; ++d) total += p.totals[d];
    *p.count_out = total;
  }
  if (base >= n) return;   // whole block
  for (int d = lane; d < 256; d += 64) cnt[w][d] = 0u;
  radix_wave_fence();
  uint32_t key[ITEMS], rank[ITEMS];
  Val val[ITEMS];
  uint32_t validmask = 0;
  const uint64_t wbase = base + (uint64_t)w * kPerWave;
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint64_t i = wbase + (uint64_t)r * 64 + lane;
    const bool in = i < n;
    key[r] = in ? p.keys_in[i] : kNoKey;
    if constexpr (PAIR) {
      val[r] = !in ? make_uint2(0u, 0u)
                   : (p.pvals_in ? p.pvals_in[i] : make_uint2(p.vals_in ? p.vals_in[i] : (uint32_t)i, (uint32_t)i));
    } else {
      val[r] = in ? (p.vals_in ? p.vals_in[i] : (uint32_t)i) : 0u;
    }
    validmask |= (in && !(p.filter && key[r] == kNoKey)) ? (1u << r) : 0u;
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const bool valid = (validmask >> r) & 1u;
    const uint32_t dg = radix_digit(p, key[r]);
    const uint64_t peers = radix_peers(valid, dg, p.bits);
    uint32_t rk = 0u;
    if (valid) {
      const uint32_t before = cnt[w][dg];
      rk = before + (uint32_t)__popcll(peers & radix_lanemask_lt());
      if ((peers >> lane) == 1ull) cnt[w][dg] = before + (uint32_t)__popcll(peers);   // last peer
    }
    radix_wave_fence();
    rank[r] = rk;
  }
  __syncthreads();
  // per digit: each wave's base within the digit, the block's digit counts scanned over the digits, and the
  // global start of the block's run of each digit (digit totals before it + the block's offset)
  uint32_t tot = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    const uint32_t c = cnt[k][t];
    cnt[k][t] = tot;
    tot += c;
  }
  const uint32_t gtot = p.totals[t];
  uint32_t s = tot, g = gtot;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)s, d, 64);
    const uint32_t z = (uint32_t)__shfl_up((int)g, d, 64);
    if (lane >= d) { s += y; g += z; }
  }
  if (lane == 63) { wsum[0][w] = s; wsum[1][w] = g; }
  __syncthreads();
  {
    uint32_t ls = s - tot, gs = g - gtot;
    for (int k = 0; k < w; ++k) { ls += wsum[0][k]; gs += wsum[1][k]; }
    dstart[t] = ls;
    gstart[t] = gs + p.table[radix_tidx(t, blockIdx.x, p.nblocks)];
    if (t == 255) kept = ls + tot;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    if (!((validmask >> r) & 1u)) continue;
    const uint32_t dg = radix_digit(p, key[r]);
    const uint32_t pos = dstart[dg] + cnt[w][dg] + rank[r];
    sk[pos] = key[r];
    sv[pos] = val[r];
  }
  __syncthreads();
  const uint32_t m = kept;
  for (uint32_t j = t; j < m; j += kRadixThreads) {
    const uint32_t k = sk[j];
    const uint32_t dg = radix_digit(p, k);
    const uint32_t dst = gstart[dg] + (j - dstart[dg]);
    p.keys_out[dst] = k;
    if constexpr (PAIR) p.pvals_out[dst] = sv[j];
    else p.vals_out[dst] = sv[j];
  }
}

// The same pass for blocks of several tiles (p.sub > 1): the block's tiles in turn, its global digit starts
// advancing by each tile's digit counts.
template <int ITEMS, bool PAIR>
__global__ void __launch_bounds__(kRadixThreads) radix_downsweep_multi_kernel(RadixPass p) {
  typedef typename RadixVal<PAIR>::T Val;
  constexpr int kWaves = kRadixThreads / 64;
  constexpr int kTile = kRadixThreads * ITEMS;
  constexpr int kPerWave = kTile / kWaves;   // contiguous items of one wave
  __shared__ uint32_t sk[kTile];
  __shared__ Val sv[kTile];
  __shared__ uint32_t cnt[kWaves][256];   // per-wave digit counts, then each wave's base within its digit
  __shared__ uint32_t dstart[256];        // tile-local start of each digit
  __shared__ uint32_t gstart[256];        // global position of the tile's first item of each digit
  __shared__ uint32_t wsum[2][kWaves];
  __shared__ uint32_t kept;
  const uint32_t n = radix_count(p);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, t = threadIdx.x;
  if (blockIdx.x == 0 && t == 0 && p.filter && p.count_out) {
    uint32_t total = 0;
    for (int d = 0; d < 256; ++d) total += p.totals[d];
    *p.count_out = total;
  }
  if ((uint64_t)blockIdx.x * p.sub * kTile >= n) return;   // whole block
  // the global start of the block's run of each digit: digit totals before it + the block's offset
  {
    const uint32_t gtot = p.totals[t];
    uint32_t g = gtot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t z = (uint32_t)__shfl_up((int)g, d, 64);
      if (lane >= d) g += z;
    }
    if (lane == 63) wsum[1][w] = g;
    __syncthreads();
    uint32_t gs = g - gtot;
    for (int k = 0; k < w; ++k) gs += wsum[1][k];
    gstart[t] = gs + p.table[radix_tidx(t, blockIdx.x, p.nblocks)];
  }
  // the block's tiles in turn; gstart advances by each tile's digit counts
  for (int sub = 0; sub < p.sub; ++sub) {
    const uint64_t base = ((uint64_t)blockIdx.x * p.sub + sub) * kTile;
    if (base >= n) break;
    for (int d = lane; d < 256; d += 64) cnt[w][d] = 0u;
    radix_wave_fence();
    uint32_t key[ITEMS], rank[ITEMS];
    Val val[ITEMS];
    uint32_t validmask = 0;
    const uint64_t wbase = base + (uint64_t)w * kPerWave;
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const uint64_t i = wbase + (uint64_t)r * 64 + lane;
      const bool in = i < n;
      key[r] = in ? p.keys_in[i] : kNoKey;
      if constexpr (PAIR) {
        val[r] = !in ? make_uint2(0u, 0u)
                     : (p.pvals_in ? p.pvals_in[i] : make_uint2(p.vals_in ? p.vals_in[i] : (uint32_t)i, (uint32_t)i));
      } else {
        val[r] = in ? (p.vals_in ? p.vals_in[i] : (uint32_t)i) : 0u;
      }
      validmask |= (in && !(p.filter && key[r] == kNoKey)) ? (1u << r) : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const bool valid = (validmask >> r) & 1u;
      const uint32_t dg = radix_digit(p, key[r]);
      const uint64_t peers = radix_peers(valid, dg, p.bits);
      uint32_t rk = 0u;
      if (valid) {
        const uint32_t before = cnt[w][dg];
        rk = before + (uint32_t)__popcll(peers & radix_lanemask_lt());
        if ((peers >> lane) == 1ull) cnt[w][dg] = before + (uint32_t)__popcll(peers);   // last peer
      }
      radix_wave_fence();
      rank[r] = rk;
    }
    __syncthreads();
    // per digit: each wave's base within the digit and the tile's digit counts scanned over the digits
    uint32_t tot = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      const uint32_t c = cnt[k][t];
      cnt[k][t] = tot;
      tot += c;
    }
    uint32_t s = tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)s, d, 64);
      if (lane >= d) s += y;
    }
    if (lane == 63) wsum[0][w] = s;
    __syncthreads();
    {
      uint32_t ls = s - tot;
      for (int k = 0; k < w; ++k) ls += wsum[0][k];
      dstart[t] = ls;
      if (t == 255) kept = ls + tot;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      if (!((validmask >> r) & 1u)) continue;
      const uint32_t dg = radix_digit(p, key[r]);
      const uint32_t pos = dstart[dg] + cnt[w][dg] + rank[r];
      sk[pos] = key[r];
      sv[pos] = val[r];
    }
    __syncthreads();
    const uint32_t m = kept;
    for (uint32_t j = t; j < m; j += kRadixThreads) {
      const uint32_t k = sk[j];
      const uint32_t dg = radix_digit(p, k);
      const uint32_t dst = gstart[dg] + (j - dstart[dg]);
      p.keys_out[dst] = k;
      if constexpr (PAIR) p.pvals_out[dst] = sv[j];
      else p.vals_out[dst] = sv[j];
    }
    __syncthreads();
    gstart[t] += tot;   // this tile's items of digit t precede the next tile's
    __syncthreads();
  }
}

template <int ITEMS, bool PAIR>
hipError_t launch_radix_pass_t(const RadixPass& p, hipStream_t stream) {
  hipLaunchKernelGGL(radix_upsweep_kernel<ITEMS>, dim3(p.nblocks), dim3(kRadixThreads), 0, stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(radix_scan_kernel, dim3(256), dim3(kScanThreads), 0, stream, p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.sub == 1)
    hipLaunchKernelGGL((radix_downsweep_kernel<ITEMS, PAIR>), dim3(p.nblocks), dim3(kRadixThreads), 0, stream, p);
  else
    hipLaunchKernelGGL((radix_downsweep_multi_kernel<ITEMS, PAIR>), dim3(p.nblocks), dim3(kRadixThreads), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_radix_pass(const RadixPass& p, hipStream_t stream) {
  if (p.nblocks == 0) return hipSuccess;
  if (p.bits < 1 || p.bits > 8 || p.sub < 1) return hipErrorInvalidValue;
  if (p.items == kRadixItemsPair && p.pair) return launch_radix_pass_t<kRadixItemsPair, true>(p, stream);
  if (p.items == kRadixItemsDepth && !p.pair) return launch_radix_pass_t<kRadixItemsDepth, false>(p, stream);
  return hipErrorInvalidValue;
}

}  // namespace ges
