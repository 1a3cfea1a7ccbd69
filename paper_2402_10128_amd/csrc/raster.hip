// raster.hip -- per-tile front-to-back compositing of GES splats and its reverse-mode pass.
//
// Compositing is the discrete form of the volume-rendering integral (GES Sec. 4.2, Eq. transimttance):
// for every pixel, over its tile's splats in (depth, index) order,
//   q = a dx^2 + 2 b dx dy + c dy^2 with (dx,dy) = mean2D - pixel centre   (binary32, fixed order:
//       t = fma(a, dx, (2b) dy); q = fma(t, dx, (c dy) dy) -- identical on every machine)
//   skip unless q <= q_max (alpha >= 1/255);   falloff G = exp(-q/2) (PHI) or exp(-q^(beta/2)/2) (GEF)
//   alpha = min(0.99, o G);  t = T (1 - alpha);  stop before compositing when t < 1e-4
//   C += alpha T rgb;  T = t.
// Launch shape (gfx950): the forward pass gives a 16x16 tile two wave64s, each owning 8 rows with 2
// pixels per lane (one column, rows y and y+4): the tile's serial walk is halved, which shortens the tail
// of the heaviest tiles (3M-splat 1080p frame: 0.27 -> 0.24 ms; four waves with 1 pixel per lane: 0.30 ms).
// The backward pass, whose issue rate is saturated, keeps one wave per tile with 4 pixels per lane (rows
// y, y+4, y+8, y+12), so each splat read from LDS is used four times per lane.  Splats are staged 64 at a
// time into LDS, then every lane reads the batch back as broadcasts.  A wave stops as soon as no lane has a
// live pixel (ballot); the forward block once neither wave has.  Tiles are dealt to the 8 XCDs in groups of
// 8 neighbours (see xcd_tile).
// The backward pass walks each pixel's contributors back to front, recovering the transmittance
// before splat j as T_j = T_(j+1) / (1 - alpha_j) from the stored final T, so no per-pixel lists are
// kept.  Per splat, the 4 pixels of a lane are summed in registers and each row of 16 lanes by a DPP
// reduce-scatter; the row's lanes park the row sums in LDS, and every 32 splats each lane finishes one
// parked splat (4 row sums) and stores the tile's ten sums of the splat as a row at the pair's candidate
// slot, marking the slot; a row reduction then adds each splat's rows in binary64 in slot order (the
// cross-tile sums of a splat often cancel; binary32 accumulation would lose accuracy there), with no
// atomics, so the backward is deterministic.
// Factors of 2 common to a splat's terms (the mean2D and b gradients) are applied once per (tile, splat).
#include "ges_internal.h"

namespace ges {

constexpr float kNegHalfLog2e = -0.72134752044448170368f;   // -log2(e)/2: exp(-q/2) = 2^(kNegHalfLog2e q)

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// max(q, 0) for q that is not NaN, as one integer max of the bits (a negative q, -0 included, has a negative
// bit pattern); fmaxf costs a canonicalisation besides under IEEE mode.
__device__ __forceinline__ float clamp_q(float q) { return __int_as_float(max(__float_as_int(q), 0)); }

__device__ __forceinline__ float pair_q(float u, float v, float a, float bb, float c, float px, float py,
                                        float& dx, float& dy) {
  dx = u - px;
  dy = v - py;
  float t = bb * dy;
  t = __builtin_fmaf(a, dx, t);
  float w = c * dy;
  w = w * dy;
  return __builtin_fmaf(t, dx, w);
}

// Map a block to a global tile.  Blocks are dealt to the 8 XCDs round-robin (block index mod 8); tiles
// are dealt to them in groups of kXcdGroup horizontally adjacent tiles, group g to XCD g mod 8.  A group
// shares splats in one XCD's L2, and the dealing spreads the heavy centre of the image over all XCDs
// (contiguous bands per XCD left the busiest XCD with 1.16x the mean backward work and about 1.36x the
// mean forward work on the 3M-splat frame).  Measured on that frame: groups of 8 gave 2.25 ms per
// training step against 2.27 (groups of 4 and 16), 2.30 (bands) and 2.32 (single tiles).
constexpr int kXcdGroup = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t blk) {
  const int64_t i = blk >> 3;   // index of the block within its XCD
  return ((blk & 7) + 8 * (i / kXcdGroup)) * kXcdGroup + (i % kXcdGroup);
}

// The backward pass of a single view deals groups of kXcdGroup tiles in the order group_order gives (its
// heaviest walks first, so that the longest waves start at once and the light ones fill in behind them),
// group by group to the XCDs as xcd_tile does.  Returns -1 past the last tile.
__device__ __forceinline__ int64_t ordered_tile(int64_t blk, const uint32_t* group_order, int64_t tiles) {
  const int64_t i = blk >> 3;
  const int64_t gi = (blk & 7) + 8 * (i / kXcdGroup);
  const int64_t ngroups = (tiles + kXcdGroup - 1) / kXcdGroup;
  if (gi >= ngroups) return -1;
  const uint32_t g = group_order[gi];
  if (g >= ngroups) return -1;
  const int64_t t = (int64_t)g * kXcdGroup + (i % kXcdGroup);
  return t < tiles ? t : -1;
}

constexpr int kFwdWaves = 2;                // waves per tile in the forward pass
constexpr int kFwdPix = 4 / kFwdWaves;      // pixels per lane (one column, rows 4 apart)
static_assert(kFwdWaves == 2 || kFwdWaves == 4, "waves 0 and 1 stage the records; 16 rows split evenly");

template <int FALLOFF>
__global__ void __launch_bounds__(64 * kFwdWaves) raster_forward_kernel(const DeviceBatch* __restrict__ db,
                                                             const uint2* __restrict__ sorted_pairs,
                                                             int64_t total_tiles,
                                                             uint64_t capacity) {
  __shared__ float4 sA[64], sB[64], sC[64];
  __shared__ uint32_t live[kFwdWaves];
  __shared__ unsigned long long red[kFwdWaves][2];
  __shared__ uint32_t red_m[kFwdWaves];
  const int64_t gt = xcd_tile(blockIdx.x);
  if (gt >= total_tiles) return;   // the whole block
  const int v = view_of_block(db->tile_prefix, db->nviews, gt);
  const ViewDesc& V = db->views[v];
  const int lt = (int)(gt - db->tile_prefix[v]);
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int px = tx * kTile + (lane & 15);
  const int py0 = ty * kTile + (kTile / kFwdWaves) * w + (lane >> 4);   // the wave's rows: py0 + 4 k
  const float pxf = (float)px;
  float pyf[kFwdPix];
  uint32_t alive = 0;
#pragma unroll
  for (int k = 0; k < kFwdPix; ++k) {
    pyf[k] = (float)(py0 + 4 * k);
    if (px < V.width && py0 + 4 * k < V.height) alive |= 1u << k;
  }
  float T[kFwdPix], C[kFwdPix][3];
  uint32_t last[kFwdPix];
#pragma unroll
  for (int k = 0; k < kFwdPix; ++k) {
    T[k] = 1.f;
    C[k][0] = C[k][1] = C[k][2] = 0.f;
    last[k] = 0u;
  }
  uint32_t n_exam = 0;    // pairs examined: each terminated pixel adds 1 + its terminating position
  uint32_t n_blend = 0;   // pairs composited, for the statistics
  const uint2 rg = V.ranges[lt];
  // a range beyond the key buffer (inconsistent key count) renders as background; the list length is made
  // a scalar, so that the batch and splat loop control runs on the scalar unit
  const int n = __builtin_amdgcn_readfirstlane((uint64_t)rg.y <= capacity ? (int)(rg.y - rg.x) : 0);
  const GlobalRec* rec = (const GlobalRec*)(V.rec);
  for (int base = 0; base < n; base += 64) {
    const int cnt = min(64, n - base);
    if (lane < cnt) {   // wave 0 stages words 0-7 of the batch's records, wave 1 words 8-11
      const uint32_t id = sorted_pairs[rg.x + base + lane].x;
      if (w == 0) {
        const float4 a = rec_load(rec, 4 * (size_t)id);
        const float4 b = rec_load(rec, 4 * (size_t)id + 1);
        sA[lane] = make_float4(a.x, a.y, a.z, a.w + a.w);
        sB[lane] = b;
      } else if (w == 1) {
        sC[lane] = rec_load(rec, 4 * (size_t)id + 2);
      }
    }
    __syncthreads();
    if (__any(alive != 0)) {   // wave-uniform: a wave whose pixels have all stopped only stages
      for (int j = 0; j < cnt; ++j) {
        const float4 A = sA[j];
        const float4 B = sB[j];
        const float4 Cc = sC[j];
        const uint32_t pos1 = (uint32_t)(base + j + 1);
#pragma unroll
        for (int k = 0; k < kFwdPix; ++k) {
          if (!(alive & (1u << k))) continue;
          float dx, dy;
          float q = pair_q(A.x, A.y, A.z, A.w, B.x, pxf, pyf[k], dx, dy);
          if (!(q <= B.y)) continue;
          q = clamp_q(q);
          float G;
          if (FALLOFF == GES_FALLOFF_PHI) {
            G = fast_exp2(kNegHalfLog2e * q);
          } else {
            const float qb = fast_exp2(0.5f * B.w * fast_log2(q));
            G = fast_exp2(kNegHalfLog2e * qb);
          }
          const float alpha = fminf(kAlphaMax, B.z * G);
          const float t = T[k] * (1.f - alpha);
          if (t < kTMin) { alive &= ~(1u << k); n_exam += pos1; continue; }
          const float wgt = alpha * T[k];
          C[k][0] = __builtin_fmaf(wgt, Cc.x, C[k][0]);
          C[k][1] = __builtin_fmaf(wgt, Cc.y, C[k][1]);
          C[k][2] = __builtin_fmaf(wgt, Cc.z, C[k][2]);
          T[k] = t;
          last[k] = pos1;
          ++n_blend;
        }
        if (!__any(alive != 0)) break;
      }
    }
    // the block stops once every pixel of the tile has (the same decision in both waves, taken after the
    // barrier that also ends the reads of this batch)
    const bool wl = __any(alive != 0);
    if (lane == 0) live[w] = wl ? 1u : 0u;
    __syncthreads();
    uint32_t any_live = 0;
#pragma unroll
    for (int q = 0; q < kFwdWaves; ++q) any_live |= live[q];
    if (!any_live) break;
  }
  {
    // pair statistics of the tile: pairs examined (each pixel up to and including its terminating splat)
    // and composited, stored per tile and summed by raster_stats_kernel.  (Device-scope atomics from
    // every tile into one counter serialise across the XCDs: two per tile cost about 50 us per frame.)
    // pixels still alive examined the whole list (out-of-image pixels were never alive)
    unsigned long long e = (unsigned long long)n_exam + (unsigned long long)__popc(alive) * (uint32_t)n, b = n_blend;
    // and the length of the backward walk over the tile: its last composited position
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < kFwdPix; ++k) m = max(m, last[k]);
    for (int off = 32; off > 0; off >>= 1) {
      e += __shfl_xor(e, off, 64);
      b += __shfl_xor(b, off, 64);
      m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
    }
    if (lane == 0) { red[w][0] = e; red[w][1] = b; red_m[w] = m; }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long se = 0, sb = 0;
      uint32_t sm = 0;
#pragma unroll
      for (int q = 0; q < kFwdWaves; ++q) {
        se += red[q][0];
        sb += red[q][1];
        sm = max(sm, red_m[q]);
      }
      V.tile_stats[2 * lt] = se;
      V.tile_stats[2 * lt + 1] = sb;
      V.tile_work[lt] = sm;
    }
  }
#pragma unroll
  for (int k = 0; k < kFwdPix; ++k) {
    const int py = py0 + 4 * k;
    if (px >= V.width || py >= V.height) continue;
    const size_t pix = (size_t)py * V.width + px;
    V.out_rgb[3 * pix + 0] = __builtin_fmaf(T[k], V.bg[0], C[k][0]);
    V.out_rgb[3 * pix + 1] = __builtin_fmaf(T[k], V.bg[1], C[k][1]);
    V.out_rgb[3 * pix + 2] = __builtin_fmaf(T[k], V.bg[2], C[k][2]);
    if (V.final_T) V.final_T[pix] = T[k];
    if (V.n_contrib) V.n_contrib[pix] = last[k];
  }
}

// ---- wave64 sum with DPP: quad swaps, row rotations, then row broadcasts 15 and 31 into lane 63
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float x) {
  const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false);
  return x + __int_as_float(y);
}

// Sum over each row of 16 lanes (every lane of the row ends with its row's total).
__device__ __forceinline__ float row_sum(float x) {
  x = dpp_add<0xB1, 0xf>(x);    // quad_perm [1,0,3,2]
  x = dpp_add<0x4E, 0xf>(x);    // quad_perm [2,3,0,1]
  x = dpp_add<0x124, 0xf>(x);   // row_ror:4
  x = dpp_add<0x128, 0xf>(x);   // row_ror:8
  return x;
}

__device__ __forceinline__ float wave_sum_to_63(float x) {
  x = dpp_add<0xB1, 0xf>(x);    // quad_perm [1,0,3,2]
  x = dpp_add<0x4E, 0xf>(x);    // quad_perm [2,3,0,1]
  x = dpp_add<0x124, 0xf>(x);   // row_ror:4
  x = dpp_add<0x128, 0xf>(x);   // row_ror:8
  x = dpp_add<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x = dpp_add<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// One exchange step of a reduce-scatter inside rows of 16 lanes: the lane pairs with the lane that the
// involution CTRL maps it to (row_mirror: l^15, row_half_mirror: l^7, quad_perm [2,3,0,1]: l^2); the lane
// with the bit set keeps the second operand's partial sum and sends the first, its partner the reverse.
template <int CTRL>
__device__ __forceinline__ float xstep(float lo, float hi, bool upper) {
  const float keep = upper ? hi : lo;
  const float send = upper ? lo : hi;
  return keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), CTRL, 0xf, 0xf, false));
}

// Row sums of 8 values in 8 DPP adds and 14 selects instead of 32 DPP adds: the partner masks 15, 7, 2, 1
// span the 16 lanes of a row, and lane l ends with the sum of value (l >> 1) & 7 over its row.
__device__ __forceinline__ float row_scatter8(float a0, float a1, float a2, float a3, float a4, float a5, float a6,
                                              float a7, int lane) {
  const bool u3 = lane & 8, u2 = lane & 4, u1 = lane & 2;
  const float b0 = xstep<0x140>(a0, a4, u3), b1 = xstep<0x140>(a1, a5, u3);   // row_mirror
  const float b2 = xstep<0x140>(a2, a6, u3), b3 = xstep<0x140>(a3, a7, u3);
  const float c0 = xstep<0x141>(b0, b2, u2), c1 = xstep<0x141>(b1, b3, u2);   // row_half_mirror
  const float d0 = xstep<0x4E>(c0, c1, u1);                                    // quad_perm [2,3,0,1]
  return dpp_add<0xB1, 0xf>(d0);                                               // quad_perm [1,0,3,2]
}

constexpr int kFlush = 32;   // splats whose row partials are parked in LDS before one flush of rows

template <int FALLOFF>
__global__ void __launch_bounds__(64) raster_backward_kernel(const DeviceBatch* __restrict__ db,
                                                             const uint2* __restrict__ sorted_pairs,
                                                             int64_t total_tiles, int ordered) {
  __shared__ float4 sA[64], sB[64], sC[64];
  __shared__ float sRed[kFlush][4][10];   // [parked splat][lane row][component]
  __shared__ uint32_t sSlot[kFlush];      // the parked splat's slot: its row of this tile's sums
  __shared__ uint32_t sItem[kFlush];      // the parked splat's batch item and first candidate slot (written
  __shared__ uint32_t sFirst[kFlush];     // into its row)
  __shared__ uint32_t sIdx[64];           // batch item and first candidate slot of each staged splat
  __shared__ uint32_t sLo[64];
  const int64_t gt = ordered ? ordered_tile(blockIdx.x, db->views[0].group_order, total_tiles) : xcd_tile(blockIdx.x);
  if (gt < 0 || gt >= total_tiles) return;
  const int v = view_of_block(db->tile_prefix, db->nviews, gt);
  const ViewDesc& V = db->views[v];
  const int lt = (int)(gt - db->tile_prefix[v]);
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int lane = threadIdx.x;
  const int row = lane >> 4;
  const int px = tx * kTile + (lane & 15);
  const int py0 = ty * kTile + (lane >> 4);
  const float pxf = (float)px;
  float pyf[4], T[4], TfB[4], g[4][3], S[4][3];
  uint32_t last[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int py = py0 + 4 * k;
    pyf[k] = (float)py;
    S[k][0] = S[k][1] = S[k][2] = 0.f;
    if (px < V.width && py < V.height) {
      const size_t pix = (size_t)py * V.width + px;
      T[k] = V.final_T[pix];
      last[k] = V.n_contrib[pix];
      g[k][0] = V.dL_drgb[3 * pix];
      g[k][1] = V.dL_drgb[3 * pix + 1];
      g[k][2] = V.dL_drgb[3 * pix + 2];
    } else {
      T[k] = 1.f;
      last[k] = 0u;
      g[k][0] = g[k][1] = g[k][2] = 0.f;
    }
    // T_final (bg . g): the background's share of dL/dalpha, divided by (1 - alpha) per splat
    TfB[k] = T[k] * (V.bg[0] * g[k][0] + V.bg[1] * g[k][1] + V.bg[2] * g[k][2]);
  }
  // wave max of the last contributor position per band of 4 rows and over the tile, made scalars: the walk's
  // loop control (positions, the parked-splat count, the flush test) then runs on the scalar unit instead of
  // taking VALU issue slots, and a band skips its test of the splats behind all of its pixels' last ones
  uint32_t band_last[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t m = last[k];
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
    band_last[k] = (uint32_t)__builtin_amdgcn_readfirstlane((int)m);
  }
  const uint32_t maxlast = max(max(band_last[0], band_last[1]), max(band_last[2], band_last[3]));
  const uint2 rg = V.ranges[lt];
  const GlobalRec* rec = (const GlobalRec*)(V.rec);
  // global address space: the row stores then count only against vmcnt, and the LDS waits of the following
  // splats do not wait for them (flat stores count against lgkmcnt too)
  GlobalVec4* rows = (GlobalVec4*)(V.grad_rows);
  GlobalU32* bits = (GlobalU32*)(V.grad_bits);
  int nslot = 0;
  for (int hi = (int)maxlast; hi > 0; hi -= 64) {
    const int lo = max(0, hi - 64);
    const int cnt = hi - lo;
    if (lane < cnt) {
      const uint2 pr = sorted_pairs[rg.x + lo + lane];   // (splat index, slot)
      const float4 a = rec_load(rec, 4 * (size_t)pr.x);
      const float4 b = rec_load(rec, 4 * (size_t)pr.x + 1);
      const float4 c = rec_load(rec, 4 * (size_t)pr.x + 2);
      sA[lane] = make_float4(a.x, a.y, a.z, a.w);
      sB[lane] = b;
      sC[lane] = make_float4(c.x, c.y, c.z, __uint_as_float(pr.y));
      sIdx[lane] = (uint32_t)db->item_prefix[v] + pr.x;
      sLo[lane] = V.slot_off[pr.x];
    }
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
      const float4 A = sA[j];
      const float4 B = sB[j];
      const float4 Cc = sC[j];
      const uint32_t pos = (uint32_t)(lo + j);
      const float bb = A.w + A.w;
      // per lane: sums over its pixels of dq (a dx + b dy), dq (b dx + c dy), dq dx^2, dq dx dy, dq dy^2
      // (dq = dL/dq; halves of the mean2D and b gradients), of G dL/dalpha (opacity), of alpha T g
      // (colour) and, for GEF, of dL/dbeta
      float su = 0.f, sv = 0.f, pa = 0.f, pb = 0.f, pc = 0.f, po = 0.f, pr = 0.f, pg = 0.f, pbl = 0.f, pbeta = 0.f;
      bool entered = false;   // wave-uniform: some row band had a pixel that took the splat
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (pos >= band_last[k]) continue;   // scalar: every pixel of the band composited its last splat before
        float dx, dy;
        const float q0 = pair_q(A.x, A.y, A.z, bb, B.x, pxf, pyf[k], dx, dy);
        const bool valid = (pos < last[k]) && (q0 <= B.y);
        if (!__any(valid)) continue;   // wave-uniform: no pixel of this row band took the splat
        entered = true;
        // straight-line for every lane; a pixel that did not take the splat gets alpha = 0 (T, S and every
        // accumulated term are then unchanged: 1/(1 - 0) = 1 exactly)
        const float q = clamp_q(q0);
        float G, qb = 0.f, lq = 0.f;
        if (FALLOFF == GES_FALLOFF_PHI) {
          G = fast_exp2(kNegHalfLog2e * q);
        } else {
          lq = fast_log2(q);
          qb = fast_exp2(0.5f * B.w * lq);
          G = fast_exp2(kNegHalfLog2e * qb);
        }
        const float oG = B.z * G;
        const bool clamped = oG > kAlphaMax;
        const float alpha = valid ? (clamped ? kAlphaMax : oG) : 0.f;
        const float inv = valid ? fast_rcp(1.f - alpha) : 1.f;
        T[k] = T[k] * inv;                 // transmittance before this splat (unchanged: inv = 1 exactly)
        const float w = alpha * T[k];
        pr = __builtin_fmaf(w, g[k][0], pr);
        pg = __builtin_fmaf(w, g[k][1], pg);
        pbl = __builtin_fmaf(w, g[k][2], pbl);
        const float d0 = Cc.x - S[k][0], d1 = Cc.y - S[k][1], d2 = Cc.z - S[k][2];
        float dalpha = __builtin_fmaf(d0, g[k][0], __builtin_fmaf(d1, g[k][1], d2 * g[k][2]));
        dalpha = __builtin_fmaf(dalpha, T[k], -TfB[k] * inv);
        S[k][0] = __builtin_fmaf(alpha, d0, S[k][0]);
        S[k][1] = __builtin_fmaf(alpha, d1, S[k][1]);
        S[k][2] = __builtin_fmaf(alpha, d2, S[k][2]);
        // below the clamp: dL/do = G dL/dalpha and G dL/dG = alpha dL/dalpha = o (G dL/dalpha); above it
        // both are 0.  Per pixel only gd = G dL/dalpha is formed: the opacity o and the constant of dG/dq
        // are common to the splat's terms and multiply its row sums once (dq below is dL/dq / (o k)).
        const float gd = (valid && !clamped) ? G * dalpha : 0.f;
        po += gd;
        float dq;
        if (FALLOFF == GES_FALLOFF_PHI) {
          dq = q0 >= 0.f ? gd : 0.f;   // dG/dq = -G/2: k = -1/2
        } else {
          // dG/dq = -(beta/4) q^(beta/2 - 1) G  (q floored at 1e-12): k = -beta/4;
          // dG/dbeta = -(1/4) q^(beta/2) ln q G: the row sum of q^(beta/2) log2 q gd takes -(ln 2)/4 o
          const float qf = __int_as_float(max(__float_as_int(q), __float_as_int(1e-12f)));   // q >= +0
          const float qpow = fast_exp2((0.5f * B.w - 1.f) * fast_log2(qf));
          dq = q0 >= 0.f ? qpow * gd : 0.f;
          pbeta = __builtin_fmaf(q > 0.f ? qb * lq : 0.f, gd, pbeta);
        }
        const float dqdx = dq * dx, dqdy = dq * dy;
        su = __builtin_fmaf(dq, __builtin_fmaf(A.z, dx, A.w * dy), su);
        sv = __builtin_fmaf(dq, __builtin_fmaf(A.w, dx, B.x * dy), sv);
        pa = __builtin_fmaf(dqdx, dx, pa);
        pb = __builtin_fmaf(dqdx, dy, pb);
        pc = __builtin_fmaf(dqdy, dy, pc);
      }
      if (entered) {
        // rows of 16 lanes reduce in registers: the first 8 sums by a reduce-scatter (after it, lanes 2i and
        // 2i+1 of a row hold row sum i), the blue and beta sums by a full row sum; the row's lanes then park
        // the 10 sums in LDS, each scaled by the splat's common factor (o k for the dq sums, o for dL/dbeta)
        const float e = row_scatter8(su, sv, pa, pb, pc, po, pr, pg, lane);
        const float r8 = row_sum(pbl);
        const float r9 = FALLOFF == GES_FALLOFF_GEF ? row_sum(pbeta) : 0.f;
        const float kq = FALLOFF == GES_FALLOFF_PHI ? -0.5f * B.z : (-0.25f * B.w) * B.z;
        float* d = sRed[nslot][row];
        const int idx = (lane >> 1) & 7;
        if ((lane & 1) == 0) d[idx] = idx < 5 ? kq * e : e;
        if ((lane & 15) == 15) {
          d[8] = r8;
          d[9] = FALLOFF == GES_FALLOFF_GEF ? (-0.25f * 0.69314718055994531f * B.z) * r9 : 0.f;
        }
        if (lane == 0) {
          sSlot[nslot] = __float_as_uint(Cc.w);
          sItem[nslot] = sIdx[j];
          sFirst[nslot] = sLo[j];
        }
        ++nslot;
      }
      if (nslot == kFlush || (j == 0 && hi - 64 <= 0 && nslot > 0)) {
        // one lane per parked splat: add the four row sums and store the tile's sums of the splat, the splat's
        // batch item and its first candidate slot in the row of its slot (the row reduction adds a splat's rows
        // in slot order), marking the slot
        __syncthreads();
        if (lane < nslot) {   // entries 0 .. nslot-1 hold row partials
          const uint32_t slot = sSlot[lane];
          float val[10];
#pragma unroll
          for (int c = 0; c < 10; ++c)
            val[c] = (sRed[lane][0][c] + sRed[lane][1][c]) + (sRed[lane][2][c] + sRed[lane][3][c]);
          val[0] = 2.f * val[0];   // dL/du = 2 sum dq (a dx + b dy)
          val[1] = 2.f * val[1];   // dL/dv = 2 sum dq (b dx + c dy)
          val[3] = 2.f * val[3];   // dL/db = 2 sum dq dx dy
          if (FALLOFF != GES_FALLOFF_GEF) val[9] = 0.f;
          GlobalVec4* r = rows + (size_t)slot * (kRowFloats / 4);
          Vec4 v0, v1, v2;
          v0[0] = val[0]; v0[1] = val[1]; v0[2] = val[2]; v0[3] = val[3];
          v1[0] = val[4]; v1[1] = val[5]; v1[2] = val[6]; v1[3] = val[7];
          v2[0] = val[8]; v2[1] = val[9]; v2[2] = __uint_as_float(sItem[lane]); v2[3] = __uint_as_float(sFirst[lane]);
          r[0] = v0;
          r[1] = v1;
          r[2] = v2;
          __hip_atomic_fetch_or(bits + (slot >> 5), 1u << (slot & 31u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        nslot = 0;
      }
    }
    __syncthreads();
  }
}

// Bucket of a tile group for the backward order: 0 holds the heaviest walks (1,023 positions or more).
constexpr int kOrderBuckets = 1024;
static_assert(kXcdGroup == 8, "a tile group's work words are read as two 16-byte loads");
__device__ __forceinline__ int group_bucket(const uint32_t* work, int64_t g, int64_t tiles) {
  uint32_t w = 0;
  if ((g + 1) * kXcdGroup <= tiles) {   // a whole group (the work array is 256-byte aligned)
    const uint4 a = reinterpret_cast<const uint4*>(work)[2 * g];
    const uint4 b = reinterpret_cast<const uint4*>(work)[2 * g + 1];
    w = max(max(max(a.x, a.y), max(a.z, a.w)), max(max(b.x, b.y), max(b.z, b.w)));
  } else {
    for (int64_t t = g * kXcdGroup; t < tiles; ++t) w = max(w, work[t]);
  }
  return kOrderBuckets - 1 - (int)min(w, (uint32_t)(kOrderBuckets - 1));
}

// One block: every view's per-tile pair statistics summed into its header ([2] examined, [3] composited);
// for a single view, also the order of its tile groups for the backward pass: a counting sort on the
// group's longest walk, heaviest first (the order within a bucket is immaterial).
__global__ void __launch_bounds__(1024) raster_stats_kernel(const DeviceBatch* __restrict__ db) {
  __shared__ unsigned long long part[2][16];
  __shared__ uint32_t cursor[kOrderBuckets];
  __shared__ uint32_t wsum[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int v = 0; v < db->nviews; ++v) {
    const ViewDesc& V = db->views[v];
    const int T = V.tiles_x * V.tiles_y;
    unsigned long long e = 0, c = 0;
    for (int t = threadIdx.x; t < T; t += 1024) {
      e += V.tile_stats[2 * t];
      c += V.tile_stats[2 * t + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
      e += __shfl_xor(e, off, 64);
      c += __shfl_xor(c, off, 64);
    }
    if (lane == 0) { part[0][w] = e; part[1][w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long se = 0, sc = 0;
      for (int k = 0; k < 16; ++k) { se += part[0][k]; sc += part[1][k]; }
      V.header[2] = se;
      V.header[3] = sc;
    }
    __syncthreads();   // part[] is rewritten for the next view
  }
  if (db->nviews != 1) return;
  const ViewDesc& V = db->views[0];
  const int64_t tiles = (int64_t)V.tiles_x * V.tiles_y;
  const int64_t ngroups = (tiles + kXcdGroup - 1) / kXcdGroup;
  const int tid = threadIdx.x;
  cursor[tid] = 0u;   // one bucket per thread
  __syncthreads();
  for (int64_t g = tid; g < ngroups; g += 1024) atomicAdd(&cursor[group_bucket(V.tile_work, g, tiles)], 1u);
  __syncthreads();
  const uint32_t c = cursor[tid];   // exclusive scan of the bucket counts
  uint32_t s = c;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)s, d, 64);
    if (lane >= d) s += y;
  }
  if (lane == 63) wsum[w] = s;
  __syncthreads();
  uint32_t pre = 0;
  for (int k = 0; k < w; ++k) pre += wsum[k];
  cursor[tid] = pre + s - c;
  __syncthreads();
  for (int64_t g = tid; g < ngroups; g += 1024) {
    const uint32_t pos = atomicAdd(&cursor[group_bucket(V.tile_work, g, tiles)], 1u);
    V.group_order[pos] = (uint32_t)g;
  }
}

hipError_t launch_raster_forward(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  if (b.total_tiles == 0) return hipSuccess;
  const int64_t span = 8 * kXcdGroup;   // the grid covers whole rounds of groups
  const dim3 grid((unsigned)((b.total_tiles + span - 1) / span * span));
  // every view of a batch shares the falloff (the server fixes it per instance)
  if (b.falloff != GES_FALLOFF_GEF)   // Gaussian falloff (PHI, PHI_EXACT)
    hipLaunchKernelGGL(raster_forward_kernel<GES_FALLOFF_PHI>, grid, dim3(64 * kFwdWaves), 0, stream, dbatch, b.sorted_pairs,
                       b.total_tiles, b.key_capacity);
  else
    hipLaunchKernelGGL(raster_forward_kernel<GES_FALLOFF_GEF>, grid, dim3(64 * kFwdWaves), 0, stream, dbatch, b.sorted_pairs,
                       b.total_tiles, b.key_capacity);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(raster_stats_kernel, dim3(1), dim3(1024), 0, stream, dbatch);
  return hipGetLastError();
}

hipError_t launch_raster_backward(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream) {
  if (b.total_tiles == 0) return hipSuccess;
  const int ordered = b.nviews == 1;   // the forward's statistics pass ordered the groups of a single view
  const int64_t span = 8 * kXcdGroup;   // the grid covers whole rounds of groups
  const dim3 grid((unsigned)((b.total_tiles + span - 1) / span * span));
  if (b.falloff != GES_FALLOFF_GEF)
    hipLaunchKernelGGL(raster_backward_kernel<GES_FALLOFF_PHI>, grid, dim3(64), 0, stream, dbatch, b.sorted_pairs,
                       b.total_tiles, ordered);
  else
    hipLaunchKernelGGL(raster_backward_kernel<GES_FALLOFF_GEF>, grid, dim3(64), 0, stream, dbatch, b.sorted_pairs,
                       b.total_tiles, ordered);
  return hipGetLastError();
}

}  // namespace ges
