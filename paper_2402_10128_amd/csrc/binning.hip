// binning.hip -- (tile, splat) pairs of a batch, ordered by (tile, depth, splat index), and tile ranges.
//
// The 3DGS lineage the paper builds on (Sec. 5.2 keeps its design choices) duplicates every splat once
// per tile it covers and sorts the pairs by (tile, depth).  Here the depth part of that order is settled
// once per splat instead of once per pair, and only the tile part is sorted over the pairs:
//   1. depth sort (in ges_preprocess): the listed splats of every view, keyed by the depth bits the
//      preprocess writes, in four stable 8-bit LSD radix passes carrying (candidate count, item); the first
//      pass drops unlisted splats.  Stability keeps equal depths in index order.
//   2. key scan: every listed splat owns one slot per candidate tile (tile_geom.h), laid out along the
//      depth order; the offset of each 256-splat chunk and the batch's slot count (the key capacity a frame
//      needs, read back by the host).
//   3. duplicate (render): each wave takes 64 consecutive splats of the depth order, expands their
//      candidates and tests one per lane; every slot receives (batch tile, splat index) or a dropped key.
//      Slots are written in order, so the writes are contiguous.
//   4. tile sort: stable LSD radix passes on the batch tile id (two for up to 65,536 tiles); the first
//      drops the empty slots.  Pairs of one tile keep the depth order of step 3, hence (depth, index).
//   5. ranges: each tile's [start, end) from the boundaries of the sorted tile ids (empty tiles (0, 0)).
// HBM: per listed splat its record (64 B, gathered in depth order) and a few words; per slot 8 B written
// by the duplication and 12 B read and written per radix pass.
#include <algorithm>

#include "ges_internal.h"
#include "tile_geom.h"

namespace ges {

constexpr int kDepthPasses = 4;   // 31 key bits (positive binary32 depths)

__global__ void clear_cells_kernel(uint32_t* cells) {
  if (threadIdx.x < 4) cells[threadIdx.x] = 0u;
}

hipError_t launch_depth_sort(const DeviceBatch* /*dbatch*/, Batch& b, hipStream_t stream) {
  SortWs& w = b.sw;
  const int sub = radix_sub((uint64_t)b.items, kRadixItemsDepth);
  const uint32_t nb = radix_blocks((uint64_t)b.items, kRadixItemsDepth, sub);
  if (nb == 0) {   // no splat: no pass runs, so nothing else would write the listed count
    hipLaunchKernelGGL(clear_cells_kernel, dim3(1), dim3(64), 0, stream, w.cells);
    w.depth_final = 1;
    return hipGetLastError();
  }
  // the values are (candidate count, item) pairs, made by the first pass from the counts and the item
  // indices, so that the key scan and the duplication read the counts in depth order
  const uint32_t* kin = w.item_key;
  const uint2* vin = nullptr;
  int cur = 0;
  for (int pass = 0; pass < kDepthPasses; ++pass) {
    RadixPass p{};
    p.items = kRadixItemsDepth;
    p.sub = sub;
    p.bits = 8;
    p.pair = 1;
    p.keys_in = kin;
    if (pass == 0) p.vals_in = w.item_cand;
    else p.pvals_in = vin;
    p.keys_out = w.dk[cur];
    p.pvals_out = w.dv[cur];
    p.count_dev = pass == 0 ? nullptr : &w.cells[0];
    p.count_host = (uint32_t)b.items;
    p.nblocks = nb;
    p.shift = 8 * pass;
    p.filter = pass == 0;
    p.table = w.table;
    p.totals = w.totals;
    p.count_out = &w.cells[0];
    hipError_t e = launch_radix_pass(p, stream);
    if (e != hipSuccess) return e;
    kin = w.dk[cur];
    vin = w.dv[cur];
    cur ^= 1;
  }
  w.depth_final = cur ^ 1;
  return hipSuccess;
}

// Which view owns batch item j (linear scan over at most kMaxViews views).
__device__ __forceinline__ int view_of_item(const DeviceBatch* db, int64_t j) {
  return view_of_block(db->item_prefix, db->nviews, j);
}

// Candidate slots of each 256-splat chunk of the depth order (before its exclusive scan).
__global__ void __launch_bounds__(256) chunk_sum_kernel(const uint2* __restrict__ order,
                                                        const uint32_t* __restrict__ cells, uint32_t* chunk_off) {
  __shared__ uint32_t wsum[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t listed = cells[0];
  const int64_t base = (int64_t)blockIdx.x * 256;
  if (base >= (int64_t)listed) return;   // whole block
  const int64_t k = base + threadIdx.x;
  uint32_t c = k < (int64_t)listed ? order[k].x : 0u;
  for (int off = 32; off > 0; off >>= 1) c += (uint32_t)__shfl_xor((int)c, off, 64);
  if (lane == 0) wsum[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) chunk_off[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// One block: exclusive scan of the chunk sums (saturating at 2^32 - 1, which the host reports as
// capacity exceeded); the batch's slot count into cells[1]; the per-view header words and ranges cleared
// for the coming render.  Each thread scans kPer consecutive sums of a round in registers, so a round takes
// one block-wide scan of the thread totals.
__global__ void __launch_bounds__(1024) chunk_scan_kernel(const DeviceBatch* __restrict__ db, uint32_t* chunk_off,
                                                          uint32_t* cells) {
  constexpr int kPer = 8;
  __shared__ unsigned long long wsum[16];
  __shared__ unsigned long long carry;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t listed = cells[0];
  const int64_t nchunks = ((int64_t)listed + 255) / 256;
  if (threadIdx.x == 0) carry = 0ull;
  __syncthreads();
  for (int64_t base = 0; base < nchunks; base += 1024 * kPer) {
    const int64_t c0 = base + (int64_t)threadIdx.x * kPer;   // this thread's kPer consecutive entries
    uint32_t x[kPer];
    unsigned long long local = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      x[k] = c0 + k < nchunks ? chunk_off[c0 + k] : 0u;
      local += x[k];
    }
    unsigned long long s = local;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const unsigned long long y = __shfl_up(s, d, 64);
      if (lane >= d) s += y;
    }
    if (lane == 63) wsum[wid] = s;
    __syncthreads();
    unsigned long long run = carry + s - local;
    for (int q = 0; q < wid; ++q) run += wsum[q];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (c0 + k < nchunks) chunk_off[c0 + k] = run > 0xffffffffull ? 0xffffffffu : (uint32_t)run;
      run += x[k];
    }
    __syncthreads();
    if (threadIdx.x == 1023) carry = run;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cells[1] = carry >= 0xffffffffull ? 0xffffffffu : (uint32_t)carry;
    cells[2] = 0u;
    cells[3] = 0u;
  }
  for (int v = 0; v < db->nviews; ++v) {
    const ViewDesc& V = db->views[v];
    const int64_t T = (int64_t)V.tiles_x * V.tiles_y;
    for (int64_t t = threadIdx.x; t < T; t += 1024) V.ranges[t] = make_uint2(0u, 0u);
    if (threadIdx.x < 4) V.header[threadIdx.x] = 0ull;   // keys, error word, pair statistics of the render
  }
}

hipError_t launch_key_scan(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  const SortWs& w = b.sw;
  const int64_t chunks = (b.items + 255) / 256;
  if (chunks > 0) {
    hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)chunks), dim3(256), 0, stream, w.dv[w.depth_final], w.cells,
                       w.chunk_off);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(chunk_scan_kernel, dim3(1), dim3(1024), 0, stream, dbatch, w.chunk_off, w.cells);
  return hipGetLastError();
}

// Per-wave LDS staging of 64 splats and of 64 of their tile rows for the flattened candidate walk.
struct WaveSplats {
  uint32_t rexcl[64];    // exclusive prefix of the splats' tile rows
  uint32_t slots[64];    // the splat's slot count (from the key scan)
  uint32_t filled[64];   // candidates enumerated so far (checked against slots)
  int32_t tx0[64], tx1[64], ty0[64];
  uint32_t spans[64];
  float u[64], v[64], a[64], b[64], c[64], qm[64], inv_a[64], inv_c[64], q2[64], det[64], Xe[64], Y[64], ra[64];
  uint32_t id[64];       // splat index in its view
  uint32_t tbase[64];    // the view's first batch tile
  int32_t tx[64];        // the view's tiles per row
  int32_t wh[64];        // the view's width | height << 16
  uint32_t hits[64];
  // the current 64 rows: owning splat (lane), tile row, first column, exclusive prefix of their spans
  uint32_t rown[64];
  int32_t rty[64], rlo[64];
  uint32_t rexcl2[64];
};

__device__ __forceinline__ void dup_wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Last index j in [0, 64) with ex[j] <= x (ex non-decreasing, ex[0] = 0 <= x).
__device__ __forceinline__ int owner_of(const uint32_t* ex, uint32_t x) {
  int j = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1)
    if (ex[j + step] <= x) j += step;
  return j;
}

// Each wave takes 64 consecutive splats of the depth order and fills their slots: the splats' tile rows are
// flattened 64 at a time (each lane computes one row's span of candidate columns), then the candidates of
// those rows 64 at a time, one per lane; each slot receives (batch tile, splat index) when the exact test
// admits the tile (always for SQUARE), else a dropped key.  Also per splat its tile count and visibility
// bit, and per view its number of keys.
__global__ void __launch_bounds__(256) duplicate_kernel(const DeviceBatch* __restrict__ db,
                                                        const uint2* __restrict__ order,
                                                        const uint32_t* __restrict__ chunk_off, uint32_t* cells,
                                                        uint32_t* keys, uint32_t* vals, uint64_t capacity,
                                                        int ellipse) {
  __shared__ WaveSplats wave_lds[4];
  __shared__ uint32_t view_keys[kMaxViews];
  __shared__ uint32_t wave_total[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v = threadIdx.x; v < kMaxViews; v += 256) view_keys[v] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t slots = cells[1];
    cells[3] = (uint64_t)slots > capacity ? (uint32_t)capacity : slots;   // slots written below
    if ((uint64_t)slots > capacity) atomicOr(&db->views[0].header[1], 1ull);
  }
  __syncthreads();
  const uint32_t listed = cells[0];
  const int64_t chunk = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;   // 64 splats per wave
  WaveSplats& W = wave_lds[wave];
  int v = 0;
  int64_t i = 0;
  uint32_t nslots = 0u, nrows = 0u;
  bool live = false;
  uint32_t flags = 0u;
  const bool busy = chunk * 64 < (int64_t)listed;   // wave-uniform
  if (busy) {
    const int64_t k = chunk * 64 + lane;
    if (k < (int64_t)listed) {
      const uint2 cj = order[k];   // (candidate count, item)
      const uint32_t j = cj.y;
      v = view_of_item(db, j);
      const ViewDesc& V = db->views[v];
      i = (int64_t)j - db->item_prefix[v];
      const float4 r3 = V.rec[4 * i + 3];
      const uint32_t lo = __float_as_uint(r3.y), hi = __float_as_uint(r3.z);
      flags = (uint32_t)__float_as_int(r3.x) >> 24;
      const float4 r0 = V.rec[4 * i + 0];
      const float4 r1 = V.rec[4 * i + 1];
      SplatTiles s;
      candidate_tiles(r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, (int)(lo & 0xffffu), (int)(lo >> 16), (int)(hi & 0xffffu),
                      (int)(hi >> 16), ellipse != 0, s);
      live = true;
      // the splat's slots are the ones the key scan counted (the preprocess ran candidate_count on the same
      // values); its rows are enumerated until they are filled
      nslots = cj.x;
      nrows = nslots ? s.rows : 0u;
      W.slots[lane] = nslots;
      W.filled[lane] = 0u;
      W.tx0[lane] = s.tx0; W.tx1[lane] = s.tx1; W.ty0[lane] = s.ty0;
      W.spans[lane] = s.spans ? 1u : 0u;
      W.u[lane] = s.u; W.v[lane] = s.v; W.a[lane] = s.a; W.b[lane] = s.b; W.c[lane] = s.c;
      W.qm[lane] = s.qm; W.inv_a[lane] = s.inv_a; W.inv_c[lane] = s.inv_c;
      W.q2[lane] = s.q2; W.det[lane] = s.det; W.Xe[lane] = s.Xe; W.Y[lane] = s.Y; W.ra[lane] = s.ra;
      W.id[lane] = (uint32_t)i;
      W.tbase[lane] = (uint32_t)db->tile_prefix[v];
      W.tx[lane] = V.tiles_x;
      W.wh[lane] = V.width | (V.height << 16);
    }
  }
  // slots of the wave's splats: the block's offset (one 256-splat chunk) plus the earlier waves' counts
  uint32_t sincl = nslots, rincl = nrows;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)sincl, d, 64);
    const uint32_t z = (uint32_t)__shfl_up((int)rincl, d, 64);
    if (lane >= d) { sincl += y; rincl += z; }
  }
  // wave totals as scalars: the loops below then keep their control on the scalar unit
  const uint32_t total = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)sincl, 63, 64));
  const uint32_t rtotal = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)rincl, 63, 64));
  if (lane == 0) wave_total[wave] = total;
  __syncthreads();
  if (busy) {
    W.rexcl[lane] = rincl - nrows;
    W.hits[lane] = 0u;
    dup_wave_fence();
    uint64_t slot0 = chunk_off[blockIdx.x];
    for (int q = 0; q < wave; ++q) slot0 += wave_total[q];
    uint32_t done = 0;   // slots filled by the rows before this round
    for (uint32_t r0 = 0; r0 < rtotal; r0 += 64) {
      // one tile row per lane: its span of candidate columns
      const uint32_t r = r0 + (uint32_t)lane;
      uint32_t width = 0u;
      int j = 0, ty = 0, clo = 0;
      if (r < rtotal) {
        j = owner_of(W.rexcl, r);
        ty = W.ty0[j] + (int)(r - W.rexcl[j]);
        SplatTiles s;
        s.tx0 = W.tx0[j]; s.tx1 = W.tx1[j]; s.ty0 = W.ty0[j];
        s.spans = W.spans[j] != 0u;
        s.u = W.u[j]; s.v = W.v[j]; s.a = W.a[j]; s.b = W.b[j]; s.c = W.c[j]; s.qm = W.qm[j];
        s.inv_a = W.inv_a[j]; s.inv_c = W.inv_c[j]; s.q2 = W.q2[j]; s.det = W.det[j]; s.Xe = W.Xe[j]; s.Y = W.Y[j];
        s.ra = W.ra[j];
        int chi;
        row_span(s, ty, W.wh[j] >> 16, clo, chi);
        width = chi >= clo ? (uint32_t)(chi - clo + 1) : 0u;
      }
      uint32_t wincl = width;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)wincl, d, 64);
        if (lane >= d) wincl += y;
      }
      const uint32_t ctotal = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)wincl, 63, 64));
      W.rown[lane] = (uint32_t)j;
      W.rty[lane] = ty;
      W.rlo[lane] = clo;
      W.rexcl2[lane] = wincl - width;
      if (width) atomicAdd(&W.filled[j], width);
      dup_wave_fence();
      for (uint32_t c0 = 0; c0 < ctotal; c0 += 64) {
        const uint32_t c = c0 + (uint32_t)lane;
        if (c < ctotal) {
          const int q = owner_of(W.rexcl2, c);
          const int js = (int)W.rown[q];
          const int tyy = W.rty[q];
          const int txx = W.rlo[q] + (int)(c - W.rexcl2[q]);
          const int wh = W.wh[js];
          const bool hit = !ellipse || ellipse_hits_tile(W.u[js], W.v[js], W.a[js], W.b[js], W.c[js], W.inv_a[js],
                                                         W.inv_c[js], W.qm[js], txx, tyy, wh & 0xffff, wh >> 16);
          const uint32_t pos = done + c;   // position among the wave's slots
          if (pos < total) {
            if (hit) atomicAdd(&W.hits[js], 1u);
            const uint64_t slot = slot0 + pos;
            if (slot < capacity) {
              keys[slot] = hit ? W.tbase[js] + (uint32_t)(tyy * W.tx[js] + txx) : kNoKey;
              vals[slot] = W.id[js];
            }
          }
        }
      }
      done += ctotal;
      dup_wave_fence();
    }
    if (live && W.filled[lane] != nslots) atomicOr(&db->views[0].header[1], 2ull);   // never expected
    if (live) {
      // the preprocess left the candidate count in tiles_touched and the visibility bit set when it is
      // non-zero: rewrite them only where the exact count differs (scattered 4-byte stores)
      const ViewDesc& V = db->views[v];
      const uint32_t h = W.hits[lane];
      if (h != nslots) reinterpret_cast<uint32_t*>(V.rec)[16 * i + R_TOUCHED] = h;
      if (h == 0u && nslots != 0u) V.vis[i] = flags;
      const uint64_t first = slot0 + (sincl - nslots);   // the splat's first slot (its rows in the backward)
      V.slot_off[i] = first > 0xffffffffull ? 0xffffffffu : (uint32_t)first;
      if (h) atomicAdd(&view_keys[v], h);
    }
  }
  __syncthreads();
  for (int vv = threadIdx.x; vv < db->nviews; vv += 256)
    if (view_keys[vv]) atomicAdd(&db->views[vv].header[0], (unsigned long long)view_keys[vv]);
}

hipError_t launch_duplicate(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  const SortWs& w = b.sw;
  const int64_t chunks = (b.items + 255) / 256;
  if (chunks == 0 || b.key_capacity == 0) return hipSuccess;
  const int X = b.dup_buffer;
  hipLaunchKernelGGL(duplicate_kernel, dim3((unsigned)chunks), dim3(256), 0, stream, dbatch,
                     w.dv[w.depth_final], w.chunk_off, w.cells, b.kw.key[X],
                     reinterpret_cast<uint32_t*>(b.kw.pv[X]),
                     b.key_capacity, b.tile_cull == GES_TILES_ELLIPSE ? 1 : 0);
  return hipGetLastError();
}

// After the backward raster: each splat's 2-D gradient, the sum of the rows the raster stored at its
// candidate slots (one per tile in which some pixel composited it; about a tenth of the slots, as the tiles'
// walks end where their pixels saturate), added in binary64 in slot order -- the same order on every run,
// so the backward is deterministic.  A wave takes 8 words of the row marks (256 slots): it lists their marked
// slots in LDS, loads 64 rows at a time (one per lane; a row carries its splat's batch item and first
// candidate slot) and the first lane of each run of one splat's rows adds the run from LDS, carrying an
// unfinished run into the next 64 and, past the wave's words, through the rest of the splat's slot range.
// The run at the start of the range belongs to the wave holding the splat's first row if that lies before
// the range.  The splat's 2-D gradient is written and kRowBit set in its visibility word (the preprocess
// backward takes zero without it).
constexpr int kReduceWords = 8;
constexpr uint32_t kNoItem = 0xffffffffu;

struct ReduceLds {
  uint32_t slot[kReduceWords * 32];   // marked slots, in order
  Vec4 row[64][3];                    // the current 64 rows
  uint32_t owner[64];
  double carry[10];                   // sums of the run left open by the last 64 rows
  uint32_t carry_owner;
};

__device__ __forceinline__ void reduce_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void write_grad2d(const DeviceBatch* db, uint32_t item, const double* g) {
  const int v = view_of_item(db, item);
  const ViewDesc& V = db->views[v];
  const int64_t i = (int64_t)item - db->item_prefix[v];
  double2* gs = reinterpret_cast<double2*>(V.grad2d + (int64_t)kGradStride * i);
#pragma unroll
  for (int c = 0; c < 5; ++c) gs[c] = make_double2(g[2 * c], g[2 * c + 1]);
  __hip_atomic_fetch_or(V.vis + i, kRowBit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_row(double* g, const Vec4* r) {
  g[0] += r[0][0]; g[1] += r[0][1]; g[2] += r[0][2]; g[3] += r[0][3];
  g[4] += r[1][0]; g[5] += r[1][1]; g[6] += r[1][2]; g[7] += r[1][3];
  g[8] += r[2][0]; g[9] += r[2][1];
}

// The marked slots of words [w0, w0 + kReduceWords) below `end` into L.slot, in order; returns their count.
__device__ __forceinline__ uint32_t list_marks(const GlobalU32* bits, uint64_t w0, uint64_t nwords, uint64_t end,
                                               ReduceLds& L, int lane) {
  const uint64_t q = w0 + (uint64_t)lane;
  uint32_t m = 0u;
  if (lane < kReduceWords && q < nwords && q * 32 < end) {
    m = bits[q];
    if (end - q * 32 < 32) m &= (1u << (uint32_t)(end - q * 32)) - 1u;
  }
  const uint32_t cnt = (uint32_t)__builtin_popcount(m);
  uint32_t incl = cnt;
#pragma unroll
  for (int d = 1; d < kReduceWords; d <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)incl, d, 64);
    if (lane >= d) incl += y;
  }
  const uint32_t total = (uint32_t)__shfl((int)incl, kReduceWords - 1, 64);
  uint32_t p = incl - cnt;
  while (m) {
    L.slot[p++] = (uint32_t)(q * 32) + (uint32_t)__builtin_ctz(m);
    m &= m - 1u;
  }
  reduce_fence();
  return total;
}

// Lane-per-row load of rows [c0, c0 + n) of the list into LDS; returns the lane's row's item and first slot.
__device__ __forceinline__ void load_rows(const GlobalVec4* rows, ReduceLds& L, uint32_t c0, uint32_t n, int lane,
                                          uint32_t& item, uint32_t& first) {
  item = kNoItem;
  first = 0u;
  if ((uint32_t)lane < n) {
    const GlobalVec4* r = rows + (uint64_t)L.slot[c0 + lane] * (kRowFloats / 4);
    const Vec4 a0 = r[0], a1 = r[1], a2 = r[2];
    item = __float_as_uint(a2[2]);
    first = __float_as_uint(a2[3]);
    L.row[lane][0] = a0;
    L.row[lane][1] = a1;
    L.row[lane][2] = a2;
  }
  L.owner[lane] = item;
}

__global__ void __launch_bounds__(256) row_reduce_kernel(const DeviceBatch* __restrict__ db,
                                                         const float* __restrict__ rows_,
                                                         const uint32_t* __restrict__ bits_, uint64_t nslots) {
  __shared__ ReduceLds lds[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  ReduceLds& L = lds[wave];
  const uint64_t nwords = (nslots + 31) / 32;
  const uint64_t w0 = ((uint64_t)blockIdx.x * 4 + wave) * kReduceWords;
  if (w0 >= nwords) return;
  const uint64_t wend = min<uint64_t>((w0 + kReduceWords) * 32, nslots);   // first slot after the range
  const GlobalU32* bits = (const GlobalU32*)bits_;
  const GlobalVec4* rows = (const GlobalVec4*)rows_;
  const uint32_t total = list_marks(bits, w0, nwords, wend, L, lane);
  if (total == 0) return;
  if (lane == 0) L.carry_owner = kNoItem;
  uint32_t skip = kNoItem;
  for (uint32_t c0 = 0; c0 < total; c0 += 64) {
    const uint32_t n = min<uint32_t>(64u, total - c0);
    uint32_t o, lo;
    load_rows(rows, L, c0, n, lane, o, lo);
    if (c0 == 0) {
      // the first run's splat is summed by the wave of its first row: is that before this range?
      const uint32_t o0 = (uint32_t)__shfl((int)o, 0, 64);
      const uint64_t lo0 = (uint32_t)__shfl((int)lo, 0, 64);
      bool earlier = false;
      for (uint64_t q0 = lo0 >> 5; q0 < w0 && !earlier; q0 += 64) {
        const uint64_t q = q0 + (uint64_t)lane;
        uint32_t m = 0u;
        if (q < w0) {
          m = bits[q];
          if (q == lo0 >> 5) m &= ~0u << (uint32_t)(lo0 & 31u);
        }
        earlier = __ballot(m != 0u) != 0ull;
      }
      if (earlier) skip = o0;
    }
    const uint32_t co = L.carry_owner;
    double g[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) g[k] = (lane == 0 && co != kNoItem) ? L.carry[k] : 0.0;
    reduce_fence();
    // a run left open by the previous 64 rows that does not go on here ended with them
    if (lane == 0 && co != kNoItem && co != L.owner[0]) {
      write_grad2d(db, co, g);
#pragma unroll
      for (int k = 0; k < 10; ++k) g[k] = 0.0;
    }
    const bool head = (uint32_t)lane < n && (lane == 0 || L.owner[lane - 1] != o);
    bool open = false;
    if (head) {
      if (!(lane == 0 && co == o)) {
#pragma unroll
        for (int k = 0; k < 10; ++k) g[k] = 0.0;
      }
      uint32_t k = (uint32_t)lane;
      if (o != skip)
        for (; k < n && L.owner[k] == o; ++k) add_row(g, L.row[k]);
      else
        while (k < n && L.owner[k] == o) ++k;
      open = k == n;
    }
    reduce_fence();
    if (head) {
      if (open) {
#pragma unroll
        for (int c = 0; c < 10; ++c) L.carry[c] = g[c];
        L.carry_owner = o == skip ? kNoItem : o;
      } else if (o != skip) {
        write_grad2d(db, o, g);
      }
    }
    reduce_fence();
  }
  // the last run: finished here, or continued through the rest of its splat's slots
  const uint32_t co = L.carry_owner;
  if (co == kNoItem) return;
  double g[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) g[k] = L.carry[k];
  uint64_t hi;
  {
    const int v = view_of_item(db, co);
    const ViewDesc& V = db->views[v];
    const int64_t i = (int64_t)co - db->item_prefix[v];
    hi = min<uint64_t>((uint64_t)V.slot_off[i] + V.item_cand[i], nslots);
  }
  for (uint64_t q0 = w0 + kReduceWords; q0 * 32 < hi; q0 += kReduceWords) {
    reduce_fence();
    const uint32_t cnt = list_marks(bits, q0, nwords, hi, L, lane);
    for (uint32_t c0 = 0; c0 < cnt; c0 += 64) {
      const uint32_t n = min<uint32_t>(64u, cnt - c0);
      uint32_t o, lo;
      load_rows(rows, L, c0, n, lane, o, lo);
      reduce_fence();
      if (lane == 0)
        for (uint32_t k = 0; k < n; ++k) add_row(g, L.row[k]);
      reduce_fence();
    }
  }
  if (lane == 0) write_grad2d(db, co, g);
}

hipError_t launch_row_reduce(const DeviceBatch* dbatch, const Batch& b, const float* rows, const uint32_t* bits,
                             uint64_t nslots, hipStream_t stream) {
  (void)b;
  if (nslots == 0) return hipSuccess;
  const uint64_t nwords = (nslots + 31) / 32;
  const uint64_t waves = (nwords + kReduceWords - 1) / kReduceWords;
  hipLaunchKernelGGL(row_reduce_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, stream, dbatch, rows, bits,
                     nslots);
  return hipGetLastError();
}

// Tile ranges from the boundaries of the sorted tile ids (ranges were cleared by the key scan).  Each thread
// reads 4 consecutive ids as one 16-byte load; the ids either side come from the neighbouring lanes.
__global__ void __launch_bounds__(256) tile_ranges_kernel(const DeviceBatch* __restrict__ db,
                                                          const uint32_t* __restrict__ tiles,
                                                          const uint32_t* __restrict__ cells, int64_t total_tiles) {
  const uint64_t K = cells[2];
  const int lane = threadIdx.x & 63;
  const uint64_t k0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (k0 - 4 * (uint64_t)lane >= K) return;   // the whole wave lies past the keys
  uint32_t t[4] = {~0u, ~0u, ~0u, ~0u};
  if (k0 + 4 <= K) {
    const uint4 q = reinterpret_cast<const uint4*>(tiles)[k0 >> 2];
    t[0] = q.x; t[1] = q.y; t[2] = q.z; t[3] = q.w;
  } else {
    for (int e = 0; e < 4; ++e)
      if (k0 + e < K) t[e] = tiles[k0 + e];
  }
  uint32_t prev = (uint32_t)__shfl_up((int)t[3], 1, 64), next = (uint32_t)__shfl_down((int)t[0], 1, 64);
  if (lane == 0) prev = k0 > 0 && k0 <= K ? tiles[k0 - 1] : ~0u;
  if (lane == 63) next = k0 + 4 < K ? tiles[k0 + 4] : ~0u;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint64_t k = k0 + e;
    if (k >= K) break;
    const uint32_t tt = t[e];
    if ((int64_t)tt >= total_tiles) continue;   // not a tile of the batch (never written by the duplication)
    const uint32_t before = e == 0 ? prev : t[e - 1];
    const uint32_t after = e == 3 ? next : t[e + 1];
    const bool first = k == 0 || before != tt;
    const bool last = k + 1 == K || after != tt;
    if (!first && !last) continue;
    const int v = view_of_block(db->tile_prefix, db->nviews, (int64_t)tt);
    uint2* r = db->views[v].ranges + ((int64_t)tt - db->tile_prefix[v]);
    if (first) r->x = (uint32_t)k;
    if (last) r->y = (uint32_t)(k + 1);
  }
}

hipError_t launch_tile_sort(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  if (b.key_capacity == 0) return hipSuccess;
  const SortWs& w = b.sw;
  const int sub = radix_sub(b.key_capacity, kRadixItemsPair);
  const uint32_t nb = radix_blocks(b.key_capacity, kRadixItemsPair, sub);
  // the tile bits split evenly over the passes (13 bits: 7 + 6), so that no pass scatters to more digit
  // runs than it must
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) < b.total_tiles) ++bits;
  int shift = 0, cur = b.dup_buffer;
  for (int pass = 0; pass < b.tile_passes; ++pass) {
    const int left = b.tile_passes - pass;
    const int pb = (bits - shift + left - 1) / left;
    RadixPass p{};
    p.items = kRadixItemsPair;
    p.sub = sub;
    p.bits = pb;
    p.pair = 1;   // the first pass pairs each splat index with its slot
    p.keys_in = b.kw.key[cur];
    if (pass == 0) p.vals_in = reinterpret_cast<const uint32_t*>(b.kw.pv[cur]);
    else p.pvals_in = b.kw.pv[cur];
    p.keys_out = b.kw.key[cur ^ 1];
    p.pvals_out = b.kw.pv[cur ^ 1];
    p.count_dev = pass == 0 ? &w.cells[3] : &w.cells[2];
    p.nblocks = nb;
    p.shift = shift;
    p.filter = pass == 0;
    p.table = b.kw.table;
    p.totals = b.kw.totals;
    p.count_out = &w.cells[2];
    hipError_t e = launch_radix_pass(p, stream);
    if (e != hipSuccess) return e;
    shift += pb;
    cur ^= 1;
  }
  if (cur != 0) return hipErrorInvalidValue;   // the plan puts the final order in buffer 0
  const uint64_t rblocks = (b.key_capacity + 1023) / 1024;
  hipLaunchKernelGGL(tile_ranges_kernel, dim3((unsigned)rblocks), dim3(256), 0, stream, dbatch,
                     b.kw.key[0], w.cells, b.total_tiles);
  return hipGetLastError();
}

}  // namespace ges
