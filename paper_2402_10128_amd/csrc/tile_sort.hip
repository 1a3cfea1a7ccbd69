// tile_sort.hip -- per-tile ordering of the bucketed pairs by (depth, splat index).
//
// Every tile's bucket holds (depth bits, splat index) pairs in arbitrary order.  Each tile's list is
// sorted ascending by depth (camera z > 0, so the IEEE bits order like the values), ties broken by
// the splat index, which makes the order unique and equal to a stable sort of the pairs in splat-index
// order.  Method: LSD radix sort with 8-bit digits; digits that are constant across the tile (known from
// an AND/OR reduction) are skipped, or, when that needs fewer passes, the keys are taken relative to the
// tile's nearest depth (a tile's depths usually span less than 2^24 units in the last place, so 3 passes
// instead of 4 on the 3M-splat frame's typical tile).  Each pass is a stable counting sort ranked wave by wave: a wave owns
// a contiguous segment of the list, ranks its elements 64 at a time with eight ballots against
// wave-private digit counters in LDS, and only the scatter needs block barriers (five per pass,
// independent of the list length).  Runs of equal depth are then ordered by index: runs of at most 32
// by insertion sort, longer ones (only in degenerate scenes) by extra index passes placed before the
// depth passes.
// Shapes: lists of up to 1,024 pairs take one wave each (four tiles per 256-thread block, no block
// barriers); up to 4,096 pairs one 256-thread block per tile (37 KB of LDS); longer lists go to a persistent grid of 1,024-thread blocks (one per CU, 145 KB of LDS; gfx950
// gives a workgroup up to 160 KB) fed by a work queue, so that no CU slot is spent on a block that
// finds a short list.  Lists beyond 16,384 pairs stream through global memory in chunks of 16,384 with
// the same ranking.
#include <algorithm>

#include "ges_internal.h"

namespace ges {

constexpr int kShortRun = 32;
constexpr int kLargeCap = 16384;

template <int CAP, int THREADS>
struct SortShared {
  static constexpr int kWaves = THREADS / 64;
  static constexpr int kR = CAP / THREADS;   // elements per lane
  uint32_t key[CAP];
  uint32_t val[CAP];
  uint32_t cnt[kWaves][256];   // per-wave digit counters, then per-wave scatter bases
  uint32_t carry[256];         // streamed lists: base of every digit for the next chunk
  uint32_t wsum[kWaves];
  uint32_t kand, kor, vand, vor, kmin, kmax;
  uint32_t long_run;
};

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t digit_of(uint32_t k, uint32_t v, bool by_key, int shift, uint32_t koff = 0u) {
  return ((by_key ? k - koff : v) >> shift) & 0xffu;
}

// Digit plan of a tile's depth keys: sort the raw bits, skipping digits that are constant over the tile,
// or the keys minus the tile's smallest key (same order, since the list's keys are >= kmin), whose digits
// above the range kmax - kmin are zero.  Whichever needs fewer passes; koff is the subtrahend (0 or kmin)
// and the returned mask has the bits of the digits to sort.
__device__ __forceinline__ uint32_t key_plan(uint32_t kand, uint32_t kor, uint32_t kmin, uint32_t kmax, uint32_t& koff) {
  const uint32_t raw = kand ^ kor;
  const uint32_t range = kmax - kmin;
  const uint32_t rel = range ? (0xffffffffu >> __clz((int)range)) : 0u;
  int nraw = 0, nrel = 0;
#pragma unroll
  for (int sh = 0; sh < 32; sh += 8) {
    nraw += ((raw >> sh) & 0xffu) != 0u;
    nrel += ((rel >> sh) & 0xffu) != 0u;
  }
  koff = nrel < nraw ? kmin : 0u;
  return nrel < nraw ? rel : raw;
}

// Lanes of this wave holding the same digit (valid lanes only), from eight ballots.  The per-lane choice
// between a ballot and its complement is an XOR with the lane's sign-extended bit, so each bit costs a
// few 32-bit operations.
__device__ __forceinline__ uint64_t match_digit_ballot(bool valid, uint32_t dg) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const uint32_t b = (dg >> bit) & 1u;
    const uint64_t m = __ballot(b != 0u);
    const uint32_t flip = b - 1u;   // 0 if the lane's bit is set, all ones if not
    const uint32_t lo = (uint32_t)m ^ flip, hi = (uint32_t)(m >> 32) ^ flip;
    peers &= ((uint64_t)hi << 32) | lo;
  }
  return peers;
}

// Rank of an element among the wave's elements of the same digit seen so far (in element order);
// advances the wave's counter of that digit.
template <class SS>
__device__ __forceinline__ uint32_t wave_rank(SS& S, bool valid, uint32_t dg) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t peers = match_digit_ballot(valid, dg);
  uint32_t r = 0;
  if (valid) {
    const uint32_t before = S.cnt[w][dg];
    r = before + (uint32_t)__popcll(peers & lanemask_lt());
    if ((peers >> lane) == 1ull) S.cnt[w][dg] = before + (uint32_t)__popcll(peers);   // last peer
  }
  wave_lds_fence();
  return r;
}

// After every wave has counted: turn the per-wave counts into scatter bases, digit-major then
// wave-major, offset by `base[d]` (streamed lists) or by the exclusive digit scan (LDS lists).
// For streamed lists also advance base[d] by the chunk's count of digit d.
template <class SS>
__device__ __forceinline__ void counts_to_bases(SS& S, bool streamed) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t tot = 0;
  if (t < 256) {
#pragma unroll
    for (int k = 0; k < SS::kWaves; ++k) { const uint32_t c = S.cnt[k][t]; S.cnt[k][t] = tot; tot += c; }
  }
  uint32_t start = 0;
  if (streamed) {
    if (t < 256) { start = S.carry[t]; S.carry[t] = start + tot; }
  } else {
    uint32_t s = tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(s, d, 64);
      if (lane >= d) s += y;
    }
    if (t < 256 && lane == 63) S.wsum[w] = s;
    __syncthreads();
    if (t < 256) {
      start = s - tot;
      for (int k = 0; k < w; ++k) start += S.wsum[k];
    }
  }
  if (t < 256) {
#pragma unroll
    for (int k = 0; k < SS::kWaves; ++k) S.cnt[k][t] += start;
  }
  __syncthreads();
}

template <class SS>
__device__ __forceinline__ void zero_wave_counters(SS& S) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = lane; d < 256; d += 64) S.cnt[w][d] = 0;
  wave_lds_fence();
}

// Segment of each wave for a list of m elements: a multiple of 64, so rounds never straddle waves.
template <int THREADS>
__device__ __forceinline__ int wave_segment(int m) {
  constexpr int W = THREADS / 64;
  const int per = (m + W - 1) / W;
  return (per + 63) & ~63;
}

// ---------------------------------------------------------------- LDS-resident lists (n <= CAP)
// Element e of the list lives in the registers of wave e / seg, round (e % seg) / 64, lane e % 64.
template <int CAP, int THREADS>
__device__ __forceinline__ void lds_pass(SortShared<CAP, THREADS>& S, uint32_t (&k)[CAP / THREADS],
                                         uint32_t (&vv)[CAP / THREADS], int n, int seg, bool by_key, int shift) {
  constexpr int R = CAP / THREADS;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e0 = w * seg + lane;
  uint32_t rank[R];
  zero_wave_counters(S);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r * 64 >= seg) break;
    const bool valid = e0 + r * 64 < n;
    rank[r] = wave_rank(S, valid, valid ? digit_of(k[r], vv[r], by_key, shift) : 0u);
  }
  __syncthreads();
  counts_to_bases(S, false);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r * 64 >= seg) break;
    if (e0 + r * 64 < n) {
      const uint32_t pos = S.cnt[w][digit_of(k[r], vv[r], by_key, shift)] + rank[r];
      S.key[pos] = k[r];
      S.val[pos] = vv[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r * 64 >= seg) break;
    const int e = e0 + r * 64;
    if (e < n) { k[r] = S.key[e]; vv[r] = S.val[e]; }
  }
  __syncthreads();
}

template <class SS>
__device__ __forceinline__ void reduce_bits(SS& S, uint32_t kand, uint32_t kor, uint32_t vand, uint32_t vor,
                                            uint32_t kmin, uint32_t kmax) {
  // reduce within the wave first, so that only one lane per wave touches the shared words
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    kand &= (uint32_t)__shfl_xor((int)kand, off, 64);
    kor |= (uint32_t)__shfl_xor((int)kor, off, 64);
    vand &= (uint32_t)__shfl_xor((int)vand, off, 64);
    vor |= (uint32_t)__shfl_xor((int)vor, off, 64);
    kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off, 64));
    kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off, 64));
  }
  if (threadIdx.x == 0) {
    S.kand = 0xffffffffu; S.kor = 0u; S.vand = 0xffffffffu; S.vor = 0u; S.kmin = 0xffffffffu; S.kmax = 0u;
    S.long_run = 0u;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    atomicAnd(&S.kand, kand); atomicOr(&S.kor, kor); atomicAnd(&S.vand, vand); atomicOr(&S.vor, vor);
    atomicMin(&S.kmin, kmin); atomicMax(&S.kmax, kmax);
  }
  __syncthreads();
}

template <int CAP, int THREADS>
__device__ void sort_lds(SortShared<CAP, THREADS>& S, const uint2* __restrict__ in, uint32_t* __restrict__ out_ids,
                         int n) {
  constexpr int R = CAP / THREADS;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int seg = wave_segment<THREADS>(n);
  const int e0 = w * seg + lane;
  uint32_t k[R], vv[R];
  uint32_t kand = 0xffffffffu, kor = 0u, vand = 0xffffffffu, vor = 0u, kmin = 0xffffffffu, kmax = 0u;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    k[r] = 0u; vv[r] = 0u;
    if (r * 64 >= seg) continue;
    const int e = e0 + r * 64;
    if (e < n) {
      const uint2 p = in[e];
      k[r] = p.x; vv[r] = p.y;
      kand &= p.x; kor |= p.x; vand &= p.y; vor |= p.y;
      kmin = min(kmin, p.x); kmax = max(kmax, p.x);
    }
  }
  reduce_bits(S, kand, kor, vand, vor, kmin, kmax);
  uint32_t koff;
  const uint32_t kdiff = key_plan(S.kand, S.kor, S.kmin, S.kmax, koff), vdiff = S.vand ^ S.vor;
  // the sorted keys are k - koff (order and equality unchanged); only the ids are written out
#pragma unroll
  for (int r = 0; r < R; ++r) k[r] -= koff;
  for (int shift = 0; shift < 32; shift += 8)
    if ((kdiff >> shift) & 0xffu) lds_pass(S, k, vv, n, seg, true, shift);
  // publish, then look for runs of equal depth
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r * 64 >= seg) break;
    const int e = e0 + r * 64;
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
      if (r * 64 >= seg) break;
      const int e = e0 + r * 64;
      if (e < n) { k[r] = S.key[e]; vv[r] = S.val[e]; }
    }
    __syncthreads();
    for (int shift = 0; shift < 32; shift += 8)
      if ((vdiff >> shift) & 0xffu) lds_pass(S, k, vv, n, seg, false, shift);
    for (int shift = 0; shift < 32; shift += 8)
      if ((kdiff >> shift) & 0xffu) lds_pass(S, k, vv, n, seg, true, shift);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r * 64 >= seg) break;
      const int e = e0 + r * 64;
      if (e < n) S.val[e] = vv[r];
    }
    __syncthreads();
  }
  for (int e = t; e < n; e += THREADS) out_ids[e] = S.val[e];
}

// ---------------------------------------------------------------- streamed lists (n > CAP)
template <int CAP, int THREADS>
__device__ void stream_pass(SortShared<CAP, THREADS>& S, const uint2* __restrict__ src, uint2* __restrict__ dst,
                            int64_t n, bool by_key, int shift, uint32_t koff) {
  constexpr int R = CAP / THREADS;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // digit histogram of the whole list, scanned into the first chunk's bases
  for (int d = t; d < 256; d += THREADS) S.carry[d] = 0;
  __syncthreads();
  for (int64_t e = t; e < n; e += THREADS) {
    const uint2 p = src[e];
    atomicAdd(&S.carry[digit_of(p.x, p.y, by_key, shift, koff)], 1u);
  }
  __syncthreads();
  {
    uint32_t x = t < 256 ? S.carry[t] : 0u, s = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(s, d, 64);
      if (lane >= d) s += y;
    }
    if (t < 256 && lane == 63) S.wsum[w] = s;
    __syncthreads();
    if (t < 256) {
      uint32_t pre = s - x;
      for (int k = 0; k < w; ++k) pre += S.wsum[k];
      S.carry[t] = pre;
    }
    __syncthreads();
  }
  for (int64_t c0 = 0; c0 < n; c0 += CAP) {
    const int m = (int)min<int64_t>(CAP, n - c0);
    const int seg = wave_segment<THREADS>(m);
    const int e0 = w * seg + lane;
    uint2 p[R];
    uint32_t rank[R];
    zero_wave_counters(S);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r * 64 >= seg) break;
      const bool valid = e0 + r * 64 < m;
      p[r] = valid ? src[c0 + e0 + r * 64] : make_uint2(0u, 0u);
      rank[r] = wave_rank(S, valid, valid ? digit_of(p[r].x, p[r].y, by_key, shift, koff) : 0u);
    }
    __syncthreads();
    counts_to_bases(S, true);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r * 64 >= seg) break;
      if (e0 + r * 64 < m) dst[S.cnt[w][digit_of(p[r].x, p[r].y, by_key, shift, koff)] + rank[r]] = p[r];
    }
    __syncthreads();
  }
}

template <int CAP, int THREADS>
__device__ void sort_stream(SortShared<CAP, THREADS>& S, uint2* __restrict__ a, uint2* __restrict__ b,
                            uint32_t* __restrict__ out_ids, int64_t n) {
  const int t = threadIdx.x;
  uint32_t kand = 0xffffffffu, kor = 0u, vand = 0xffffffffu, vor = 0u, kmin = 0xffffffffu, kmax = 0u;
  for (int64_t e = t; e < n; e += THREADS) {
    const uint2 p = a[e];
    kand &= p.x; kor |= p.x; vand &= p.y; vor |= p.y;
    kmin = min(kmin, p.x); kmax = max(kmax, p.x);
  }
  reduce_bits(S, kand, kor, vand, vor, kmin, kmax);
  uint32_t koff;
  const uint32_t kdiff = key_plan(S.kand, S.kor, S.kmin, S.kmax, koff), vdiff = S.vand ^ S.vor;
  uint2* src = a;
  uint2* dst = b;
  for (int shift = 0; shift < 32; shift += 8)
    if ((kdiff >> shift) & 0xffu) { stream_pass(S, src, dst, n, true, shift, koff); uint2* x = src; src = dst; dst = x; }
  __threadfence_block();
  __syncthreads();
  for (int64_t e = t; e < n; e += THREADS) {
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
      if ((vdiff >> shift) & 0xffu) { stream_pass(S, src, dst, n, false, shift, 0u); uint2* x = src; src = dst; dst = x; }
    for (int shift = 0; shift < 32; shift += 8)
      if ((kdiff >> shift) & 0xffu) { stream_pass(S, src, dst, n, true, shift, koff); uint2* x = src; src = dst; dst = x; }
    __threadfence_block();
    __syncthreads();
  }
  for (int64_t e = t; e < n; e += THREADS) out_ids[e] = src[e].y;
}

// ---------------------------------------------------------------- one wave per tile (n <= kWaveCap)
// Short lists need no block: a wave owns a tile, holds its elements in registers (element e = r * 64 +
// lane) and a 9 KB slice of LDS, and uses wave fences only.
constexpr int kWaveCap = 1024;
constexpr int kWaveR = kWaveCap / 64;

struct WaveSortShared {
  uint32_t key[kWaveCap];
  uint32_t val[kWaveCap];
  uint32_t cnt[256];              // digit counters, then digit bases
};

__device__ __forceinline__ void wave_pass(WaveSortShared& S, uint32_t (&k)[kWaveR], uint32_t (&vv)[kWaveR], int n,
                                          bool by_key, int shift) {
  const int lane = threadIdx.x & 63;
  uint32_t rank[kWaveR];
#pragma unroll
  for (int d = 0; d < 4; ++d) S.cnt[lane * 4 + d] = 0u;
  wave_lds_fence();
#pragma unroll
  for (int r = 0; r < kWaveR; ++r) {
    if (r * 64 >= n) break;
    const bool valid = r * 64 + lane < n;
    const uint32_t dg = valid ? digit_of(k[r], vv[r], by_key, shift) : 0u;
    const uint64_t peers = match_digit_ballot(valid, dg);
    uint32_t rr = 0;
    if (valid) {
      const uint32_t before = S.cnt[dg];
      rr = before + (uint32_t)__popcll(peers & lanemask_lt());
      if ((peers >> lane) == 1ull) S.cnt[dg] = before + (uint32_t)__popcll(peers);   // last peer
    }
    wave_lds_fence();
    rank[r] = rr;
  }
  // exclusive scan of the 256 counters: lane l owns digits 4l .. 4l+3
  uint32_t c[4], sum = 0;
#pragma unroll
  for (int d = 0; d < 4; ++d) { c[d] = S.cnt[lane * 4 + d]; sum += c[d]; }
  uint32_t incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  uint32_t run = incl - sum;
#pragma unroll
  for (int d = 0; d < 4; ++d) { S.cnt[lane * 4 + d] = run; run += c[d]; }
  wave_lds_fence();
#pragma unroll
  for (int r = 0; r < kWaveR; ++r) {
    if (r * 64 >= n) break;
    if (r * 64 + lane < n) {
      const uint32_t pos = S.cnt[digit_of(k[r], vv[r], by_key, shift)] + rank[r];
      S.key[pos] = k[r];
      S.val[pos] = vv[r];
    }
  }
  wave_lds_fence();
#pragma unroll
  for (int r = 0; r < kWaveR; ++r) {
    if (r * 64 >= n) break;
    const int e = r * 64 + lane;
    if (e < n) { k[r] = S.key[e]; vv[r] = S.val[e]; }
  }
  wave_lds_fence();
}

__device__ void wave_sort(WaveSortShared& S, const uint2* __restrict__ in, uint32_t* __restrict__ out_ids, int n) {
  const int lane = threadIdx.x & 63;
  uint32_t k[kWaveR], vv[kWaveR];
  uint32_t kand = 0xffffffffu, kor = 0u, vand = 0xffffffffu, vor = 0u, kmin = 0xffffffffu, kmax = 0u;
#pragma unroll
  for (int r = 0; r < kWaveR; ++r) {
    k[r] = 0u; vv[r] = 0u;
    const int e = r * 64 + lane;
    if (e < n) {
      const uint2 p = in[e];
      k[r] = p.x; vv[r] = p.y;
      kand &= p.x; kor |= p.x; vand &= p.y; vor |= p.y;
      kmin = min(kmin, p.x); kmax = max(kmax, p.x);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    kand &= (uint32_t)__shfl_xor((int)kand, off, 64);
    kor |= (uint32_t)__shfl_xor((int)kor, off, 64);
    vand &= (uint32_t)__shfl_xor((int)vand, off, 64);
    vor |= (uint32_t)__shfl_xor((int)vor, off, 64);
    kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off, 64));
    kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off, 64));
  }
  uint32_t koff;
  const uint32_t kdiff = key_plan(kand, kor, kmin, kmax, koff), vdiff = vand ^ vor;
  // the sorted keys are k - koff (order and equality unchanged); only the ids are written out
#pragma unroll
  for (int r = 0; r < kWaveR; ++r) k[r] -= koff;
  for (int shift = 0; shift < 32; shift += 8)
    if ((kdiff >> shift) & 0xffu) wave_pass(S, k, vv, n, true, shift);
  // publish, then order runs of equal depth by index
#pragma unroll
  for (int r = 0; r < kWaveR; ++r) {
    const int e = r * 64 + lane;
    if (e < n) { S.key[e] = k[r]; S.val[e] = vv[r]; }
  }
  wave_lds_fence();
  bool long_run = false;
  for (int e = lane; e < n; e += 64) {
    if ((e == 0 || S.key[e - 1] != S.key[e]) && e + 1 < n && S.key[e + 1] == S.key[e]) {
      int len = 1;
      while (e + len < n && S.key[e + len] == S.key[e] && len <= kShortRun) ++len;
      if (len > kShortRun) {
        long_run = true;
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
  wave_lds_fence();
  if (__any(long_run)) {
    // composite order: stable index passes first, then the depth passes again
#pragma unroll
    for (int r = 0; r < kWaveR; ++r) {
      const int e = r * 64 + lane;
      if (e < n) { k[r] = S.key[e]; vv[r] = S.val[e]; }
    }
    wave_lds_fence();
    for (int shift = 0; shift < 32; shift += 8)
      if ((vdiff >> shift) & 0xffu) wave_pass(S, k, vv, n, false, shift);
    for (int shift = 0; shift < 32; shift += 8)
      if ((kdiff >> shift) & 0xffu) wave_pass(S, k, vv, n, true, shift);
#pragma unroll
    for (int r = 0; r < kWaveR; ++r) {
      const int e = r * 64 + lane;
      if (e < n) S.val[e] = vv[r];
    }
    wave_lds_fence();
  }
  for (int e = lane; e < n; e += 64) out_ids[e] = S.val[e];
}

// Lists of 1..kWaveCap pairs: four tiles per 256-thread block, one per wave.
__global__ void __launch_bounds__(256) tile_sort_wave_kernel(const DeviceBatch* __restrict__ db, const uint2* pairs,
                                                             uint32_t* sorted_ids, int64_t total_tiles,
                                                             uint64_t capacity) {
  __shared__ WaveSortShared S[4];
  const int wave = threadIdx.x >> 6;
  const int64_t gt = (int64_t)blockIdx.x * 4 + wave;
  if (gt >= total_tiles) return;
  const int v = view_of_block(db->tile_prefix, db->nviews, gt);
  const ViewDesc& V = db->views[v];
  const uint2 rg = V.ranges[gt - db->tile_prefix[v]];
  if (rg.y <= rg.x || (uint64_t)rg.y > capacity) return;
  const int n = (int)(rg.y - rg.x);
  if (n > kWaveCap) return;   // the block kernels'
  if (n == 1) {
    if ((threadIdx.x & 63) == 0) sorted_ids[rg.x] = pairs[rg.x].y;
    return;
  }
  wave_sort(S[wave], pairs + rg.x, sorted_ids + rg.x, n);
}

// Lists of kWaveCap+1..kSortCap pairs: one block per tile.  A longer list is appended to the long-list queue
// (whose counters the scatter kernel has reset).
__global__ void __launch_bounds__(256) tile_sort_short_kernel(const DeviceBatch* __restrict__ db, const uint2* pairs,
                                                              uint32_t* sorted_ids, int64_t total_tiles,
                                                              uint64_t capacity, uint32_t* queue,
                                                              uint32_t* long_list) {
  __shared__ SortShared<kSortCap, 256> S;
  const int64_t gt = blockIdx.x;
  if (gt >= total_tiles) return;
  const int v = view_of_block(db->tile_prefix, db->nviews, gt);
  const ViewDesc& V = db->views[v];
  const uint2 rg = V.ranges[gt - db->tile_prefix[v]];
  if (rg.y <= rg.x || (uint64_t)rg.y > capacity) return;
  const int n = (int)(rg.y - rg.x);
  if (n <= kWaveCap) return;   // the wave kernel's
  if (n > kSortCap) {
    if (threadIdx.x == 0) {
      const uint32_t slot = atomicAdd(&queue[0], 1u);
      if ((int64_t)slot < total_tiles) long_list[slot] = (uint32_t)gt;
    }
    return;
  }
  sort_lds(S, pairs + rg.x, sorted_ids + rg.x, n);
}

// Lists longer than kSortCap: a persistent grid (one 1,024-thread block per CU) claims the queued tiles
// one at a time and sorts them in LDS (up to kLargeCap) or streamed.  Every block leaves once the
// claims have passed the number of queued tiles.
__global__ void __launch_bounds__(1024) tile_sort_long_kernel(const DeviceBatch* __restrict__ db, uint2* pairs,
                                                              uint2* pairs_tmp, uint32_t* sorted_ids,
                                                              int64_t total_tiles, uint64_t capacity,
                                                              uint32_t* queue, const uint32_t* long_list) {
  __shared__ SortShared<kLargeCap, 1024> S;
  __shared__ uint32_t s_idx;
  const uint32_t found = (uint32_t)min<int64_t>((int64_t)queue[0], total_tiles);
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(&queue[1], 1u);
    __syncthreads();
    const uint32_t idx = s_idx;
    __syncthreads();   // every thread has read s_idx before the next claim overwrites it
    if (idx >= found) break;
    const int64_t gt = long_list[idx];
    if (gt >= total_tiles) continue;
    const int v = view_of_block(db->tile_prefix, db->nviews, gt);
    const uint2 rg = db->views[v].ranges[gt - db->tile_prefix[v]];
    if (rg.y <= rg.x || (uint64_t)rg.y > capacity) continue;
    const int64_t n = (int64_t)(rg.y - rg.x);
    if (n <= kLargeCap) sort_lds(S, pairs + rg.x, sorted_ids + rg.x, (int)n);
    else sort_stream(S, pairs + rg.x, pairs_tmp + rg.x, sorted_ids + rg.x, n);
    __syncthreads();
  }
}

hipError_t launch_tile_sort(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  if (b.total_tiles == 0 || b.key_capacity == 0) return hipSuccess;
  if (!b.sort_queue || !b.long_list) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tile_sort_wave_kernel, dim3((unsigned)((b.total_tiles + 3) / 4)), dim3(256), 0, stream, dbatch,
                     b.pairs, b.sorted_ids, b.total_tiles, b.key_capacity);
  hipError_t e0 = hipGetLastError();
  if (e0 != hipSuccess) return e0;
  hipLaunchKernelGGL(tile_sort_short_kernel, dim3((unsigned)b.total_tiles), dim3(256), 0, stream, dbatch, b.pairs,
                     b.sorted_ids, b.total_tiles, b.key_capacity, b.sort_queue, b.long_list);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t blocks = std::min<int64_t>(kLongSortBlocks, b.total_tiles);
  hipLaunchKernelGGL(tile_sort_long_kernel, dim3((unsigned)blocks), dim3(1024), 0, stream, dbatch, b.pairs,
                     b.pairs_tmp, b.sorted_ids, b.total_tiles, b.key_capacity, b.sort_queue, b.long_list);
  return hipGetLastError();
}

}  // namespace ges
