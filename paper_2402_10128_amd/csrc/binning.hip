// binning.hip -- (tile, splat) pair generation into per-tile buckets.
//
// The 3DGS lineage the paper builds on (Sec. 5.2 keeps its design choices) duplicates every splat once
// per tile it covers and sorts the pairs by (tile, depth).  Here the tile part of that order is
// established without a global sort:
//   1. bin_count:   each block owns a contiguous chunk of splats of one view and counts, in an LDS
//                   histogram, how many pairs fall into every tile; the histogram row is written to
//                   bin_counts[chunk][tile] (deterministic, no global atomics).
//   2. bin_colscan: per tile, exclusive prefix over the chunks (in place) and the tile total.
//   3. bin_tilescan: one block scans the tile totals of all views into [start,end) ranges and the
//                   number of keys per view (the only value the host reads back).
//   4. bin_scatter: each block re-walks its chunk and writes (depth bits, splat index) into its own
//                   sub-range of every tile's bucket, using LDS cursors.
// The order inside a bucket is arbitrary; the per-tile sort makes it unique.
// Load balance: each wave expands 64 splats at a time into their (splat, tile) candidates and tests
// them one per lane, so the heavy tail of near, large splats keeps every lane busy.
// HBM: 16-48 B read per splat and 8 B written per pair, plus the G x T count table.
#include "ges_internal.h"
#include "tile_geom.h"

namespace ges {

struct SplatTiles {
  int tx0, ty0, tx1, ty1, rw;    // tiles to enumerate (ELLIPSE: the rectangle cut to the ellipse's box)
  uint32_t area;                 // number of tiles to enumerate (0: none)
  bool live;                     // the record lists the splat (its rectangle is not empty)
  float u, v, a, b, c, qm, inv_a, inv_c;
  uint32_t depth_bits;
  uint32_t flags;
};

// ELLIPSE: narrow the rectangle to the tiles whose pixel-centre box can meet the accepted region of the
// exact test.  That test accepts a point when q - 1e-3 m <= q_max, with m = a dx^2 + c dy^2 + |2 b dx dy|
// <= 2 q / (1 - rho), rho = |b| / sqrt(a c) < 1; so accepted points satisfy q <= q_max / (1 - 2e-3 / (1 - rho)),
// an ellipse with half-extents X = sqrt(q' c / det), Y = sqrt(q' a / det).  Enlarged by 2.5e-3 instead
// of 2e-3, 1% and half a pixel (covering binary32 rounding here and in the test); near-degenerate
// conics (rho close to 1) keep the whole rectangle.  A superset only: the exact test decides.
__device__ __forceinline__ void narrow_to_ellipse_box(SplatTiles& s) {
  const float ac = s.a * s.c;
  const float det = ac - s.b * s.b;
  const float gap = 1.f - __builtin_fabsf(s.b) / __builtin_sqrtf(ac);
  if (!(det > 0.f) || !(gap > 0.f)) return;
  const float grow = 2.5e-3f / gap;
  if (!(grow < 0.25f)) return;
  const float q2 = s.qm / (1.f - grow);
  const float X = __builtin_sqrtf(q2 * s.c / det) * 1.01f + 0.5f;
  const float Y = __builtin_sqrtf(q2 * s.a / det) * 1.01f + 0.5f;
  if (!(X < 1e7f) || !(Y < 1e7f)) return;
  // tile tx can meet [u - X, u + X] when 16 tx + 15 >= u - X and 16 tx <= u + X
  s.tx0 = max(s.tx0, (int)__builtin_ceilf((s.u - X - 15.f) * 0.0625f));
  s.tx1 = min(s.tx1, (int)__builtin_floorf((s.u + X) * 0.0625f));
  s.ty0 = max(s.ty0, (int)__builtin_ceilf((s.v - Y - 15.f) * 0.0625f));
  s.ty1 = min(s.ty1, (int)__builtin_floorf((s.v + Y) * 0.0625f));
  if (s.tx0 > s.tx1 || s.ty0 > s.ty1) { s.area = 0u; return; }
  s.rw = s.tx1 - s.tx0 + 1;
  s.area = (uint32_t)(s.rw * (s.ty1 - s.ty0 + 1));
}

// Rectangle (and, for ELLIPSE, the conic and the narrowed rectangle) of splat i; area 0 for culled splats.
__device__ __forceinline__ void load_splat_tiles(const ViewDesc& V, int64_t i, bool ellipse, SplatTiles& s) {
  const float4 r3 = V.rec[4 * i + 3];
  const uint32_t lo = __float_as_uint(r3.y), hi = __float_as_uint(r3.z);
  s.tx0 = (int)(lo & 0xffffu); s.ty0 = (int)(lo >> 16);
  s.tx1 = (int)(hi & 0xffffu); s.ty1 = (int)(hi >> 16);
  s.rw = s.tx1 - s.tx0 + 1;
  s.flags = (uint32_t)__float_as_int(r3.x) >> 24;
  s.live = __float_as_uint(r3.w) != 0;
  s.area = s.live ? (uint32_t)(s.rw * (s.ty1 - s.ty0 + 1)) : 0u;
  s.depth_bits = __float_as_uint(V.rec[4 * i + 2].w);
  if (ellipse && s.area) {
    const float4 r0 = V.rec[4 * i + 0];
    const float4 r1 = V.rec[4 * i + 1];
    s.u = r0.x; s.v = r0.y; s.a = r0.z; s.b = r0.w; s.c = r1.x; s.qm = r1.y;
    s.inv_a = 1.0f / s.a;
    s.inv_c = 1.0f / s.c;
    narrow_to_ellipse_box(s);
  }
}

// Chunk of a view's local block index: blocks are dealt to the 8 XCDs round-robin, so with G a multiple
// of 8 the XCD of block j owns chunks (j % 8) G/8 .. (j % 8 + 1) G/8 - 1.  A tile's bucket slices of
// consecutive chunks are adjacent in memory; this way they pass through one XCD's L2, where the partial
// cache lines of neighbouring slices can merge.  Count and scatter use the same mapping.
__device__ __forceinline__ int chunk_of_block(int local, int G) {
  return (G & 7) ? local : (local & 7) * (G >> 3) + (local >> 3);
}

// Per-wave LDS staging of 64 splats for the flattened candidate walk.
struct WaveSplats {
  uint32_t excl[64];     // exclusive prefix of the rectangle areas
  uint32_t rect[64];     // tx0 | ty0 << 16
  int32_t rw[64];
  float inv_rw[64];
  float u[64], v[64], a[64], b[64], c[64], qm[64], inv_a[64], inv_c[64];
  uint32_t depth[64];
  uint32_t hits[64];
};

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Visit the (splat, tile) hits of the block's chunk [i0, i1) whose tile lies in the window [w0, w1).
// Each wave takes 64 consecutive splats at a time, scans their rectangle areas and walks the
// flattened list of (splat, rectangle tile) candidates 64 at a time, one candidate per lane, so that
// large rectangles do not serialise a wave.
// COUNT: histogram into lds; on the first window also store each splat's exact tile count (ELLIPSE).
// SCATTER: claim a slot from the tile's cursor in lds and write (depth bits, splat index).
template <bool SCATTER>
__device__ __forceinline__ void walk_chunk(const ViewDesc& V, int64_t i0, int64_t i1, int w0, int w1,
                                           uint32_t* lds, WaveSplats* wave_lds, uint2* pairs, uint64_t capacity) {
  const bool ellipse = V.tile_cull == GES_TILES_ELLIPSE;
  const bool store_count = !SCATTER && ellipse && w0 == 0;
  const int TX = V.tiles_x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  WaveSplats& W = wave_lds[wave];
  for (int64_t base = i0 + (int64_t)wave * 64; base < i1; base += (int64_t)nwaves * 64) {
    const int64_t i = base + lane;
    SplatTiles s;
    s.area = 0u;
    s.live = false;
    if (i < i1) load_splat_tiles(V, i, ellipse, s);
    // inclusive wave scan of the areas
    uint32_t incl = s.area;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    const uint32_t total = __shfl(incl, 63, 64);
    wave_lds_fence();
    W.excl[lane] = incl - s.area;
    W.hits[lane] = 0u;
    if (s.area) {
      W.rect[lane] = (uint32_t)s.tx0 | ((uint32_t)s.ty0 << 16);
      W.rw[lane] = s.rw;
      W.inv_rw[lane] = 1.0f / (float)s.rw;
      W.depth[lane] = s.depth_bits;
      if (ellipse) {
        W.u[lane] = s.u; W.v[lane] = s.v; W.a[lane] = s.a; W.b[lane] = s.b; W.c[lane] = s.c;
        W.qm[lane] = s.qm; W.inv_a[lane] = s.inv_a; W.inv_c[lane] = s.inv_c;
      }
    }
    wave_lds_fence();
    for (uint32_t c0 = 0; c0 < total; c0 += 64) {
      const uint32_t c = c0 + (uint32_t)lane;
      if (c < total) {
        // owner: the last splat whose range starts at or before c (its area is then non-zero)
        int j = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
          if (W.excl[j + step] <= c) j += step;
        const uint32_t k = c - W.excl[j];
        const int rw = W.rw[j];
        int row = (int)((float)k * W.inv_rw[j]);
        int col = (int)k - row * rw;
        if (col < 0) { --row; col += rw; }
        if (col >= rw) { ++row; col -= rw; }
        const uint32_t r0 = W.rect[j];
        const int tx = (int)(r0 & 0xffffu) + col, ty = (int)(r0 >> 16) + row;
        const int t = ty * TX + tx;
        const bool in_win = t >= w0 && t < w1;
        if (in_win || store_count) {
          const bool hit = !ellipse || ellipse_hits_tile(W.u[j], W.v[j], W.a[j], W.b[j], W.c[j], W.inv_a[j],
                                                          W.inv_c[j], W.qm[j], tx, ty, V.width, V.height);
          if (hit) {
            if (store_count) atomicAdd(&W.hits[j], 1u);
            if (in_win) {
              if (SCATTER) {
                const uint32_t pos = atomicAdd(&lds[t - w0], 1u);
                if ((uint64_t)pos < capacity) pairs[pos] = make_uint2(W.depth[j], (uint32_t)(base + j));
              } else {
                atomicAdd(&lds[t - w0], 1u);
              }
            }
          }
        }
      }
    }
    wave_lds_fence();
    if (store_count && s.live) {
      const uint32_t hits = W.hits[lane];
      reinterpret_cast<uint32_t*>(V.rec)[16 * i + R_TOUCHED] = hits;
      V.vis[i] = (hits ? kVisBit : 0u) | s.flags;
    }
  }
}

__global__ void __launch_bounds__(kBinBlockThreads) bin_count_kernel(const DeviceBatch* __restrict__ db) {
  __shared__ uint32_t hist[kBinLdsTiles];
  __shared__ WaveSplats wave_lds[kBinBlockThreads / 64];
  const int64_t blk = blockIdx.x;
  const int v = view_of_block(db->bin_prefix, db->nviews, blk);
  const ViewDesc& V = db->views[v];
  const int g = chunk_of_block((int)(blk - db->bin_prefix[v]), V.bin_blocks);
  const int64_t i0 = (int64_t)g * V.bin_chunk;
  const int64_t i1 = min<int64_t>(V.n, i0 + V.bin_chunk);
  const int T = V.tiles_x * V.tiles_y;
  for (int w0 = 0; w0 < T; w0 += kBinLdsTiles) {
    const int w1 = min(T, w0 + kBinLdsTiles);
    for (int j = threadIdx.x; j < w1 - w0; j += blockDim.x) hist[j] = 0;
    __syncthreads();
    walk_chunk<false>(V, i0, i1, w0, w1, hist, wave_lds, nullptr, 0);
    __syncthreads();
    uint32_t* out = V.bin_counts + (int64_t)g * T;
    for (int j = threadIdx.x; j < w1 - w0; j += blockDim.x) out[w0 + j] = hist[j];
    __syncthreads();
  }
}

// One thread per (view, tile): exclusive prefix over the chunk rows, 16 rows per batch of loads.
// Column scans: a block takes 64 consecutive tiles; its four waves take a quarter of every column each (the
// lanes of a wave read 64 consecutive counts per row, one coalesced 256-byte load), the quarters' sums meet
// in LDS, and each wave writes its quarter's exclusive prefix.  (One lane per whole column left it as one
// chain of 256 dependent loads.)
constexpr int kColSplit = 4;
__global__ void __launch_bounds__(256) bin_colscan_kernel(const DeviceBatch* __restrict__ db, int64_t total_tiles) {
  __shared__ uint32_t psum[kColSplit][64];
  const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
  const int64_t gt = (int64_t)blockIdx.x * 64 + lane;
  const bool live = gt < total_tiles;
  int v = 0, T = 1, G = 0, t = 0;
  uint32_t* col = nullptr;
  if (live) {
    v = view_of_block(db->tile_prefix, db->nviews, gt);
    const ViewDesc& V = db->views[v];
    T = V.tiles_x * V.tiles_y;
    t = (int)(gt - db->tile_prefix[v]);
    col = V.bin_counts + t;
    G = V.bin_blocks;
  }
  const int per = (G + kColSplit - 1) / kColSplit;
  const int g0 = min(G, part * per), g1 = min(G, g0 + per);
  uint32_t sum = 0;
  int g = g0;
  for (; g + 16 <= g1; g += 16) {   // 16 loads in flight, then their sum
    uint32_t c[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) c[k] = col[(int64_t)(g + k) * T];
#pragma unroll
    for (int k = 0; k < 16; ++k) sum += c[k];
  }
  for (; g < g1; ++g) sum += col[(int64_t)g * T];
  psum[part][lane] = sum;
  __syncthreads();
  if (!live) return;
  uint32_t acc = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kColSplit; ++k) {
    if (k < part) acc += psum[k][lane];
    total += psum[k][lane];
  }
  g = g0;
  for (; g + 16 <= g1; g += 16) {
    uint32_t c[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) c[k] = col[(int64_t)(g + k) * T];
#pragma unroll
    for (int k = 0; k < 16; ++k) { col[(int64_t)(g + k) * T] = acc; acc += c[k]; }
  }
  for (; g < g1; ++g) {
    const uint32_t c = col[(int64_t)g * T];
    col[(int64_t)g * T] = acc;
    acc += c;
  }
  if (part == kColSplit - 1) db->views[v].tile_total[t] = total;
}

// Single block: exclusive scan of every view's tile totals (views in order) into ranges; per-view
// key counts into the view headers and the batch total into keys_total (saturating at 2^32-1).
__global__ void __launch_bounds__(1024) bin_tilescan_kernel(const DeviceBatch* __restrict__ db, uint32_t* keys_total) {
  constexpr int kPer = 8;   // consecutive tiles per thread: one pass covers 8,192 tiles
  __shared__ unsigned long long wsum[16];
  __shared__ unsigned long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int v = 0; v < db->nviews; ++v) {
    const ViewDesc& V = db->views[v];
    const int T = V.tiles_x * V.tiles_y;
    const unsigned long long view_start = carry;
    for (int base = 0; base < T; base += 1024 * kPer) {
      const int t0 = base + threadIdx.x * kPer;
      uint32_t x[kPer];
      unsigned long long local = 0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        x[k] = t0 + k < T ? V.tile_total[t0 + k] : 0u;
        local += x[k];
      }
      // inclusive wave scan of the threads' sums, then the waves' sums in order
      unsigned long long s = local;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long y = __shfl_up(s, d, 64);
        if (lane >= d) s += y;
      }
      if (lane == 63) wsum[wid] = s;
      __syncthreads();
      unsigned long long wpre = 0;
      for (int k = 0; k < wid; ++k) wpre += wsum[k];
      unsigned long long run = carry + wpre + s - local;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int t = t0 + k;
        const unsigned long long e = run + x[k];
        if (t < T) {
          const uint32_t st = run > 0xffffffffull ? 0xffffffffu : (uint32_t)run;
          const uint32_t en = e > 0xffffffffull ? 0xffffffffu : (uint32_t)e;
          V.ranges[t] = x[k] == 0 ? make_uint2(0u, 0u) : make_uint2(st, en);
        }
        run = e;
      }
      __syncthreads();
      if (threadIdx.x == 1023) carry = run;
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      V.header[0] = carry - view_start;
      V.header[1] = 0ull;   // error word of the coming forward pass
      V.header[2] = 0ull;   // pair statistics of the coming forward pass
      V.header[3] = 0ull;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *keys_total = carry > 0xffffffffull ? 0xffffffffu : (uint32_t)carry;
}

__global__ void __launch_bounds__(kBinBlockThreads) bin_scatter_kernel(const DeviceBatch* __restrict__ db, uint2* pairs,
                                                                       uint64_t capacity, uint32_t* sort_queue,
                                                                       const uint32_t* keys_total) {
  __shared__ uint32_t cursor[kBinLdsTiles];
  __shared__ WaveSplats wave_lds[kBinBlockThreads / 64];
  const int64_t blk = blockIdx.x;
  if (blk == 0 && threadIdx.x < 2) sort_queue[threadIdx.x] = 0u;   // the long-list queue of the coming sort
  if (blk == 0 && threadIdx.x == 0 && (uint64_t)*keys_total > capacity)
    db->views[0].header[1] |= 1ull;   // key workspace smaller than the frame's key count
  const int v = view_of_block(db->bin_prefix, db->nviews, blk);
  const ViewDesc& V = db->views[v];
  const int g = chunk_of_block((int)(blk - db->bin_prefix[v]), V.bin_blocks);
  const int64_t i0 = (int64_t)g * V.bin_chunk;
  const int64_t i1 = min<int64_t>(V.n, i0 + V.bin_chunk);
  const int T = V.tiles_x * V.tiles_y;
  const uint32_t* row = V.bin_counts + (int64_t)g * T;
  for (int w0 = 0; w0 < T; w0 += kBinLdsTiles) {
    const int w1 = min(T, w0 + kBinLdsTiles);
    for (int j = threadIdx.x; j < w1 - w0; j += blockDim.x) cursor[j] = V.ranges[w0 + j].x + row[w0 + j];
    __syncthreads();
    walk_chunk<true>(V, i0, i1, w0, w1, cursor, wave_lds, pairs, capacity);
    __syncthreads();
  }
}

hipError_t launch_bin_count(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  if (b.bin_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(bin_count_kernel, dim3((unsigned)b.bin_blocks), dim3(kBinBlockThreads), 0, stream, dbatch);
  return hipGetLastError();
}

hipError_t launch_bin_scan(const DeviceBatch* dbatch, const Batch& b, const int32_t* /*tiles_per_view*/,
                           hipStream_t stream) {
  if (b.total_tiles > 0) {
    hipLaunchKernelGGL(bin_colscan_kernel, dim3((unsigned)((b.total_tiles + 63) / 64)), dim3(256), 0, stream, dbatch,
                       b.total_tiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(bin_tilescan_kernel, dim3(1), dim3(1024), 0, stream, dbatch, b.keys_total);
  return hipGetLastError();
}

hipError_t launch_bin_scatter(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  if (b.bin_blocks == 0 || b.key_capacity == 0) return hipSuccess;
  if (!b.sort_queue) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bin_scatter_kernel, dim3((unsigned)b.bin_blocks), dim3(kBinBlockThreads), 0, stream, dbatch,
                     b.pairs, b.key_capacity, b.sort_queue, b.keys_total);
  return hipGetLastError();
}

}  // namespace ges
