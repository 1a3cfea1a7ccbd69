// tile_sort.hip -- per-tile ordering of the bucketed pairs by (depth, splat index).
//
// Every tile's bucket holds (depth bits, splat index) pairs in arbitrary order.  One block per tile
// sorts them ascending by depth (camera z > 0, so the IEEE bits order like the values), ties broken by
// the splat index, which makes the order unique and equal to a stable sort of the pairs in splat-index
// order.  Method: LSD radix sort with 8-bit digits, each pass a stable counting sort in which a wave
// ranks equal digits with eight ballots; digits that are constant across the tile (known from an
// AND/OR reduction) are skipped.  Runs of equal depth are then ordered by index: runs of at most 32 by
// insertion sort, longer ones (only in degenerate scenes) by extra index passes placed before the
// depth passes.
// Two LDS-resident shapes: 256 threads for lists of up to 4,096 pairs (38 KB of LDS, several blocks
// per CU) and 1,024 threads for lists of up to 16,384 pairs (146 KB: gfx950 gives a workgroup up to
// 160 KB).  Longer lists stream through global memory with the same passes.
#include "ges_internal.h"

namespace ges {

constexpr int kShortRun = 32;
constexpr int kLargeCap = 16384;

template <int CAP, int THREADS>
struct SortShared {
  static constexpr int kWaves = THREADS / 64;
  uint32_t key[CAP];
  uint32_t val[CAP];
  uint32_t hist[256];
  uint32_t run[256];
  uint32_t wcnt[kWaves][256];
  uint32_t kand, kor, vand, vor;
  uint32_t long_run;
};

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Stable rank of one element per thread within the current round: returns its destination given the
// running digit offsets; updates the offsets for the next round.  `valid` lanes participate.
template <class SS>
__device__ __forceinline__ uint32_t rank_round(SS& S, bool valid, uint32_t dg) {
  const int w = threadIdx.x >> 6;
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const bool b = (dg >> bit) & 1u;
    const uint64_t m = __ballot(valid && b);
    peers &= b ? m : ~m;
  }
  const uint32_t lrank = (uint32_t)__popcll(peers & lanemask_lt());
  const bool leader = valid && (peers & lanemask_lt()) == 0;
  if (leader) S.wcnt[w][dg] = (uint32_t)__popcll(peers);
  __syncthreads();
  uint32_t pos = 0;
  if (valid) {
    uint32_t pre = 0;
    for (int k = 0; k < w; ++k) pre += S.wcnt[k][dg];
    pos = S.run[dg] + pre + lrank;
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    const int d = threadIdx.x;
    uint32_t add = 0;
#pragma unroll
    for (int k = 0; k < SS::kWaves; ++k) { add += S.wcnt[k][d]; S.wcnt[k][d] = 0; }
    S.run[d] += add;
  }
  __syncthreads();
  return pos;
}

// Exclusive scan of S.hist into S.run (256 digits, held by threads 0..255).
template <class SS>
__device__ __forceinline__ void scan_hist(SS& S) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t x = 0, s = 0;
  if (t < 256) {
    x = S.hist[t];
    s = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(s, d, 64);
      if (lane >= d) s += y;
    }
    if (lane == 63) S.wcnt[w][0] = s;
  }
  __syncthreads();
  uint32_t pre = 0;
  if (t < 256)
    for (int k = 0; k < w; ++k) pre += S.wcnt[k][0];
  __syncthreads();
  if (t < 256) {
    S.run[t] = pre + s - x;
    S.wcnt[w][0] = 0;
  }
  __syncthreads();
}

template <class SS>
__device__ __forceinline__ void init_shared(SS& S) {
  if (threadIdx.x == 0) { S.kand = 0xffffffffu; S.kor = 0u; S.vand = 0xffffffffu; S.vor = 0u; S.long_run = 0u; }
  for (int d = threadIdx.x; d < 256; d += blockDim.x)
    for (int w = 0; w < SS::kWaves; ++w) S.wcnt[w][d] = 0;
}

// ---------------------------------------------------------------- LDS path
// Registers hold the elements in round order: element e = r * THREADS + t.
template <int CAP, int THREADS>
__device__ __forceinline__ void lds_pass(SortShared<CAP, THREADS>& S, uint32_t (&k)[CAP / THREADS],
                                         uint32_t (&vv)[CAP / THREADS], int n, bool by_key, int shift) {
  constexpr int R = CAP / THREADS;
  const int t = threadIdx.x;
  if (t < 256) S.hist[t] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = r * THREADS + t;
    if (e < n) atomicAdd(&S.hist[((by_key ? k[r] : vv[r]) >> shift) & 0xffu], 1u);
  }
  __syncthreads();
  scan_hist(S);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r * THREADS >= n) break;
    const int e = r * THREADS + t;
    const bool valid = e < n;
    const uint32_t dg = valid ? (((by_key ? k[r] : vv[r]) >> shift) & 0xffu) : 0u;
    const uint32_t pos = rank_round(S, valid, dg);
    if (valid) { S.key[pos] = k[r]; S.val[pos] = vv[r]; }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = r * THREADS + t;
    if (e < n) { k[r] = S.key[e]; vv[r] = S.val[e]; }
  }
  __syncthreads();
}

template <int CAP, int THREADS>
__device__ void sort_lds(SortShared<CAP, THREADS>& S, const uint2* __restrict__ in, uint32_t* __restrict__ out_ids,
                         int n) {
  constexpr int R = CAP / THREADS;
  const int t = threadIdx.x;
  uint32_t k[R], vv[R];
  uint32_t kand = 0xffffffffu, kor = 0u, vand = 0xffffffffu, vor = 0u;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = r * THREADS + t;
    if (e < n) {
      const uint2 p = in[e];
      k[r] = p.x; vv[r] = p.y;
      kand &= p.x; kor |= p.x; vand &= p.y; vor |= p.y;
    } else {
      k[r] = 0u; vv[r] = 0u;
    }
  }
  init_shared(S);
  __syncthreads();
  atomicAnd(&S.kand, kand); atomicOr(&S.kor, kor); atomicAnd(&S.vand, vand); atomicOr(&S.vor, vor);
  __syncthreads();
  const uint32_t kdiff = S.kand ^ S.kor, vdiff = S.vand ^ S.vor;
  for (int shift = 0; shift < 32; shift += 8)
    if ((kdiff >> shift) & 0xffu) lds_pass(S, k, vv, n, true, shift);
  // publish, then look for runs of equal depth
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = r * THREADS + t;
    if (e < n) { S.key[e] = k[r]; S.val[e] = vv[r]; }
  }
  __syncthreads();
  for (int e = t; e < n; e += THREADS) {
    if ((e == 0 || S.key[e - 1] != S.key[e]) && e + 1 < n && S.key[e + 1] == S.key[e]) {
      int len = 1;
      while (e + len < n && S.key[e + len] == S.key[e] && len <= kShortRun) ++len;
      if (len > kShortRun) {
        S.long_run = 1u;
      } else {
        for (int a = e + 1; a < e + len; ++a) {   // insertion sort of the run by index
          const uint32_t x = S.val[a];
          int b = a - 1;
          while (b >= e && S.val[b] > x) { S.val[b + 1] = S.val[b]; --b; }
          S.val[b + 1] = x;
        }
      }
    }
  }
  __syncthreads();
  if (S.long_run) {
    // composite order: stable index passes first, then the depth passes again
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = r * THREADS + t;
      if (e < n) { k[r] = S.key[e]; vv[r] = S.val[e]; }
    }
    __syncthreads();
    for (int shift = 0; shift < 32; shift += 8)
      if ((vdiff >> shift) & 0xffu) lds_pass(S, k, vv, n, false, shift);
    for (int shift = 0; shift < 32; shift += 8)
      if ((kdiff >> shift) & 0xffu) lds_pass(S, k, vv, n, true, shift);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = r * THREADS + t;
      if (e < n) S.val[e] = vv[r];
    }
    __syncthreads();
  }
  for (int e = t; e < n; e += THREADS) out_ids[e] = S.val[e];
}

// ---------------------------------------------------------------- global path (n > kLargeCap)
template <class SS>
__device__ void global_pass(SS& S, const uint2* __restrict__ src, uint2* __restrict__ dst, int64_t n, bool by_key,
                            int shift) {
  const int t = threadIdx.x;
  if (t < 256) S.hist[t] = 0;
  __syncthreads();
  for (int64_t e = t; e < n; e += blockDim.x) {
    const uint2 p = src[e];
    atomicAdd(&S.hist[((by_key ? p.x : p.y) >> shift) & 0xffu], 1u);
  }
  __syncthreads();
  scan_hist(S);
  for (int64_t base = 0; base < n; base += blockDim.x) {
    const int64_t e = base + t;
    const bool valid = e < n;
    const uint2 p = valid ? src[e] : make_uint2(0u, 0u);
    const uint32_t dg = valid ? (((by_key ? p.x : p.y) >> shift) & 0xffu) : 0u;
    const uint32_t pos = rank_round(S, valid, dg);
    if (valid) dst[pos] = p;
  }
  __syncthreads();
}

template <class SS>
__device__ void sort_global(SS& S, uint2* __restrict__ a, uint2* __restrict__ b, uint32_t* __restrict__ out_ids,
                            int64_t n) {
  const int t = threadIdx.x;
  uint32_t kand = 0xffffffffu, kor = 0u, vand = 0xffffffffu, vor = 0u;
  for (int64_t e = t; e < n; e += blockDim.x) {
    const uint2 p = a[e];
    kand &= p.x; kor |= p.x; vand &= p.y; vor |= p.y;
  }
  init_shared(S);
  __syncthreads();
  atomicAnd(&S.kand, kand); atomicOr(&S.kor, kor); atomicAnd(&S.vand, vand); atomicOr(&S.vor, vor);
  __syncthreads();
  const uint32_t kdiff = S.kand ^ S.kor, vdiff = S.vand ^ S.vor;
  uint2* src = a;
  uint2* dst = b;
  for (int shift = 0; shift < 32; shift += 8)
    if ((kdiff >> shift) & 0xffu) { global_pass(S, src, dst, n, true, shift); uint2* x = src; src = dst; dst = x; }
  for (int64_t e = t; e < n; e += blockDim.x) {
    if ((e == 0 || src[e - 1].x != src[e].x) && e + 1 < n && src[e + 1].x == src[e].x) {
      int len = 1;
      while (e + len < n && src[e + len].x == src[e].x && len <= kShortRun) ++len;
      if (len > kShortRun) {
        atomicOr(&S.long_run, 1u);
      } else {
        for (int64_t q = e + 1; q < e + len; ++q) {
          const uint2 x = src[q];
          int64_t r = q - 1;
          while (r >= e && src[r].y > x.y) { src[r + 1] = src[r]; --r; }
          src[r + 1] = x;
        }
      }
    }
  }
  __threadfence_block();
  __syncthreads();
  if (S.long_run) {
    for (int shift = 0; shift < 32; shift += 8)
      if ((vdiff >> shift) & 0xffu) { global_pass(S, src, dst, n, false, shift); uint2* x = src; src = dst; dst = x; }
    for (int shift = 0; shift < 32; shift += 8)
      if ((kdiff >> shift) & 0xffu) { global_pass(S, src, dst, n, true, shift); uint2* x = src; src = dst; dst = x; }
  }
  for (int64_t e = t; e < n; e += blockDim.x) out_ids[e] = src[e].y;
}

// LOW < n <= CAP: sort in LDS; with CAP == kLargeCap also n > CAP (global path, same block shape).
template <int CAP, int THREADS, int LOW>
__global__ void __launch_bounds__(THREADS) tile_sort_kernel(const DeviceBatch* __restrict__ db, uint2* pairs,
                                                            uint2* pairs_tmp, uint32_t* sorted_ids,
                                                            int64_t total_tiles, uint64_t capacity) {
  __shared__ SortShared<CAP, THREADS> S;
  const int64_t gt = blockIdx.x;
  if (gt >= total_tiles) return;
  const int v = view_of_block(db->tile_prefix, db->nviews, gt);
  const ViewDesc& V = db->views[v];
  const uint2 rg = V.ranges[gt - db->tile_prefix[v]];
  if (rg.y <= rg.x || (uint64_t)rg.y > capacity) return;
  const int64_t n = (int64_t)(rg.y - rg.x);
  if (n <= LOW) return;                       // handled by the smaller shape
  if (CAP != kLargeCap && n > CAP) return;    // handled by the larger shape
  if (n == 1) {
    if (threadIdx.x == 0) sorted_ids[rg.x] = pairs[rg.x].y;
    return;
  }
  if (n <= CAP) sort_lds(S, pairs + rg.x, sorted_ids + rg.x, (int)n);
  else sort_global(S, pairs + rg.x, pairs_tmp + rg.x, sorted_ids + rg.x, n);
}

hipError_t launch_tile_sort(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  if (b.total_tiles == 0 || b.key_capacity == 0) return hipSuccess;
  const dim3 grid((unsigned)b.total_tiles);
  hipLaunchKernelGGL((tile_sort_kernel<kSortCap, 256, 0>), grid, dim3(256), 0, stream, dbatch, b.pairs, b.pairs_tmp,
                     b.sorted_ids, b.total_tiles, b.key_capacity);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((tile_sort_kernel<kLargeCap, 1024, kSortCap>), grid, dim3(1024), 0, stream, dbatch, b.pairs,
                     b.pairs_tmp, b.sorted_ids, b.total_tiles, b.key_capacity);
  return hipGetLastError();
}

}  // namespace ges
