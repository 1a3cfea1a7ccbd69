// ges_internal.h -- device-side data layout and launchers of the GES rasterizer (gfx950).
//
// One "view" is one camera looking at one scene.  Every kernel takes an array of views so that a
// single launch can serve a batch of render requests (continuous batching); the plain render path
// is a batch of one.  All per-view buffers live in caller-provided workspaces.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stddef.h>
#include <stdint.h>

#include "../../include/ges.h"

namespace ges {

constexpr int kTile = GES_TILE;          // 16 x 16 pixel tiles
constexpr int kTilePx = kTile * kTile;   // 256 pixels, 4 per lane of one wave64
constexpr int kRecWords = 16;            // 64-byte per-splat record
constexpr int kGradStride = GES_GRAD2D_STRIDE;   // doubles per splat in the 2-D gradient accumulator
constexpr int kMaxViews = 64;
constexpr int kRadixThreads = 256;       // radix passes: blocks of 256 threads ...
constexpr int kRadixItemsDepth = 8;      // ... holding 8 items each (the depth sort of the splats) ...
constexpr int kRadixItemsPair = 8;       // ... or 8 (the pair sort: its 12-byte items need twice the LDS)
constexpr uint32_t kNoKey = 0xffffffffu; // radix key of an item that a filtering pass drops
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

// Record words (see ges.h)
constexpr uint32_t kVisBit = 0x80000000u;
constexpr uint32_t kRowBit = 0x40000000u;   // visibility word: the backward stored rows of the splat (its 2-D
                                            // gradient is the row reduction's sum; without it, zero)

enum : int {
  R_U = 0, R_V, R_A, R_B, R_C, R_QMAX, R_OPA, R_BETA, R_CR, R_CG, R_CB, R_DEPTH, R_RADFLAGS, R_RECT0, R_RECT1, R_TOUCHED
};

struct ViewDesc {
  // scene
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* logits;
  const float* sh;
  const float* beta;
  int64_t n;
  int32_t sh_degree;
  int32_t sh_coeffs;             // (D+1)^2
  // camera
  float R[9];
  float t[3];
  float campos[3];
  float fx, fy, cx, cy, near_z;
  float limx, limy;              // 1.3 * tan(half FoV) guard of the perspective Jacobian
  int32_t width, height, tiles_x, tiles_y;
  // raster parameters
  int32_t falloff, tile_cull;
  float rho;
  float bg[3];
  // workspaces (device)
  float4* rec;                   // [n] x 4 float4
  uint32_t* item_key;            // [n] depth bits of a listed splat, kNoKey otherwise (this view's part of the
  uint32_t* item_cand;           // [n]   batch's depth-sort items), and its number of candidate tiles
  uint2* ranges;                 // [tiles] [start,end) into the key arrays (global positions)
  unsigned long long* header;    // [0] keys of this view, [1] error flags, [2] [3] pair statistics
  unsigned long long* tile_stats;  // [tiles][2] pairs examined and composited per tile (forward pass)
  uint32_t* tile_work;           // [tiles] list position + 1 of the tile's last composited splat (forward pass)
  uint32_t* group_order;         // [ceil(tiles / 8)] tile groups, heaviest backward walk first
  double* grad2d;                // [n][kGradStride] binary64 2-D gradients (stored with keep_grad2d only)
  uint32_t* slot_off;            // [n] first candidate slot of a listed splat (the duplication writes it)
  const uint2* sorted_pairs;     // [keys] (splat index, slot) per sorted pair (backward)
  float* grad_rows;              // [slots][kRowFloats] per-(tile, splat) sums of the backward, at the pair's slot
  uint32_t* grad_bits;           // [slots / 32] slots whose row the backward wrote
  uint64_t grad_slots;           // slots the rows cover (the key capacity of the forward pass)
  int32_t keep_grad2d;           // store the summed 2-D gradients in grad2d
  uint32_t* vis;                 // [n] bit 31: the splat touches a tile; bits 0..4: its clamp flags
  float* final_T;                // [h*w]
  uint32_t* n_contrib;           // [h*w]
  float* out_rgb;                // [h*w*3]
  const float* dL_drgb;          // [h*w*3] (backward only)
};

// Depth-first binning of a batch.  Items are the splats of every view, view after view (item j of view v
// is splat j - item_prefix[v]).  The preprocess writes each item's depth key and candidate-tile count;
// the listed items are sorted by depth (stable: equal depths keep index order), their candidate tiles are
// laid out in that order, each candidate becomes a (tile, splat) pair or a dropped slot, and a stable sort
// by tile gives every tile's list in depth order.
struct SortWs {
  uint32_t* item_key;            // [items]
  uint32_t* item_cand;           // [items]
  uint32_t* dk[2];               // [items] depth-sort keys, ping-pong
  uint2* dv[2];                  // [items] depth-sort values (candidate count, item index), ping-pong
  uint32_t* table;               // [16][items_blocks][16] per-block digit counts of a pass, then their prefix
  uint32_t* totals;              // [256] per-digit totals of a pass
  uint32_t* chunk_off;           // [items / 256 + 1] candidate slots before each 256-item chunk of the depth order
  uint32_t* cells;               // [0] listed items, [1] candidate slots (saturating), [2] keys, [3] spare
  int depth_final;               // dv[depth_final] holds the depth order after the last pass
};

// Key workspace of a batch: [capacity] slots of (tile, splat) pairs, two buffers; the final order lands in
// buffer 0 (val[0] first in the workspace: the backward finds the sorted splat ids there).
struct KeyWs {
  uint2* pv[2];                  // (splat index, slot) values of the tile passes; the duplication writes the
                                 // splat indices as u32 into the first half of pv[dup_buffer]
  uint32_t* key[2];
  uint32_t* table;               // [16][key_blocks][16]
  uint32_t* totals;              // [256]
};
constexpr int kRowFloats = 12;   // floats per backward row (10 used; 48 bytes keep rows 16-byte aligned)

struct Batch {
  int32_t nviews;
  int32_t falloff;               // shared by every view of a batch
  int32_t tile_cull;             // shared by every view of a batch
  int32_t tile_passes;           // 8-bit digit passes of the tile sort (tile ids of the batch)
  int64_t total_tiles;
  int64_t pre_blocks;
  int64_t items;                 // splats of all views
  SortWs sw;
  KeyWs kw;
  uint32_t* keys_total;          // device: candidate slots of the batch (sw.cells + 1)
  const uint2* sorted_pairs;     // [key capacity] (splat index, slot) per sorted pair (kw.pv[0])
  uint32_t* sorted_tiles;        // [key capacity] batch tile per sorted pair (kw.key[0])
  int dup_buffer;                // buffer the duplication writes (so that the last tile pass ends in 0)
  uint64_t key_capacity;
  int32_t shared_scene;          // every view renders the same splats (the views of a training step): the
                                 // preprocess backward sums the views' gradients per splat, in view order
};

// Device view table and per-batch constants, copied to the device by the host before launches.
// The prefix tables come first so that only the views in use need to be copied.
struct DeviceBatch {
  int64_t pre_prefix[kMaxViews + 1];
  int64_t item_prefix[kMaxViews + 1];
  int64_t tile_prefix[kMaxViews + 1];
  int32_t nviews;
  int32_t pad_;
  ViewDesc views[kMaxViews];
};
inline size_t device_batch_bytes(int nviews) { return offsetof(DeviceBatch, views) + (size_t)nviews * sizeof(ViewDesc); }

constexpr int kAdamMaxGroups = GES_ADAM_MAX_GROUPS;

// One Adam update in binary32 (Kingma & Ba, Algorithm 1), the bias corrections folded into
// step_size = lr / (1 - b1^t) and inv_sqrt_bc2 = 1 / sqrt(1 - b2^t).  Shared by the stand-alone step and
// the update fused into the preprocess backward.  Every multiply-add is an explicit FMA and no product
// feeds an addition, so no compiler contraction setting can change the result: both give the same bits.
__device__ __forceinline__ void adam_update(float& p, float g, float& m, float& v, float b1, float b2, float eps,
                                            float step_size, float inv_sqrt_bc2) {
  m = __builtin_fmaf(b1, m, (1.f - b1) * g);
  v = __builtin_fmaf(b2, v, (1.f - b2) * (g * g));
  const float den = __builtin_fmaf(sqrtf(v), inv_sqrt_bc2, eps);
  p = p - (step_size * m) / den;
}

// Parameter arrays of a splat set in the order of ges_adam_splats.
enum { kParMeans = 0, kParScales = 1, kParQuats = 2, kParOpacity = 3, kParSh = 4, kParBeta = 5, kNumPar = 6 };

// Arguments of the Adam update fused into the preprocess backward (passed by value to the kernel).
struct AdamSplats {
  float* p[kNumPar];
  float* m[kNumPar];
  float* v[kNumPar];
  float step_size[kNumPar];
  float b1, b2, eps, inv_sqrt_bc2;
  float* stat_accum;        // densification statistics (NULL: off): NDC mean-2D gradient norm ...
  float* stat_count;        // ... and the number of iterations the splat was visible
  double half_w, half_h;    // pixels per NDC unit
  const float* gin[kNumPar];  // fused update: gradients of other views added first (NULL: none)
  int32_t accumulate;       // stored gradients: add to the buffers instead of overwriting them
};

// --------------------------------------------------------------------------------------------
// launchers (implemented in the .hip files); all enqueue on `stream` and return hipError_t
hipError_t launch_preprocess(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream);
// depth-first binning (binning.hip): depth order of the listed splats, candidate slots along it (with the
// batch's slot count in keys_total), then in the render: (tile, splat) pairs, the stable sort by tile and
// the tile ranges
hipError_t launch_depth_sort(const DeviceBatch* dbatch, Batch& b, hipStream_t stream);
hipError_t launch_key_scan(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream);
hipError_t launch_duplicate(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream);
hipError_t launch_tile_sort(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream);
// after the backward raster: the 2-D gradient of every splat with a row (nslots rows of kRowFloats floats,
// marked in bits), its rows added in slot order (binary64); splats without a row are left alone
hipError_t launch_row_reduce(const DeviceBatch* dbatch, const Batch& b, const float* rows, const uint32_t* bits,
                             uint64_t nslots, hipStream_t stream);
// one stable LSD radix pass over (u32 key, u32 value) items with 8-bit digits (radix.hip)
struct RadixPass {
  int32_t items;                 // per thread: kRadixItemsDepth (pair == 0) or kRadixItemsPair (pair == 1)
  int32_t bits;                  // digit width (1..8)
  int32_t pair;                  // values are (u32, slot) pairs: read from pvals_in, or made from vals_in and
                                 // the item index; written to pvals_out
  const uint32_t* keys_in;
  const uint32_t* vals_in;       // NULL: an item's value is its index
  const uint2* pvals_in;
  uint32_t* keys_out;
  uint32_t* vals_out;
  uint2* pvals_out;
  const uint32_t* count_dev;     // number of items (device), or NULL: count_host
  uint32_t count_host;
  int32_t sub;                   // tiles of 256 x items items per block
  uint32_t nblocks;              // table width: blocks of sub x 256 x items items covering the largest count
  int32_t shift;                 // digit = (key >> shift) & ((1 << bits) - 1)
  int32_t filter;                // drop items whose key is kNoKey; the kept count goes to count_out
  uint32_t* table;               // [16][nblocks][16] (digit group, block, digit in the group)
  uint32_t* totals;              // [256]
  uint32_t* count_out;
};
hipError_t launch_radix_pass(const RadixPass& p, hipStream_t stream);
// Tiles of kRadixThreads x items items that one radix block takes in turn: 1 up to 8,192 tiles (enough
// blocks to fill the device), then up to 8 (fewer, longer blocks: a shorter digit table).
inline int radix_sub(uint64_t n, int items) {
  const uint64_t tiles = (n + (uint64_t)kRadixThreads * items - 1) / ((uint64_t)kRadixThreads * items);
  return (int)std::min<uint64_t>(8, std::max<uint64_t>(1, tiles / 8192));
}
inline uint32_t radix_blocks(uint64_t n, int items, int sub = 1) {
  const uint64_t span = (uint64_t)kRadixThreads * items * sub;
  return (uint32_t)((n + span - 1) / span);
}
hipError_t launch_raster_forward(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream);
hipError_t launch_raster_backward(const DeviceBatch* dbatch, const Batch& b, hipStream_t stream);
// args (may be NULL): the fused update's arguments when `fused`; otherwise only accumulate and the
// densification statistic are read
hipError_t launch_preprocess_backward(const DeviceBatch* dbatch, const Batch& b, const ges_splat_grads* grads,
                                      hipStream_t stream, const AdamSplats* args = nullptr, bool fused = false);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream);

hipError_t launch_freq_mask(const float* target, int w, int h, float omega, void* scratch, uint8_t* mask,
                            hipStream_t stream);
size_t freq_mask_scratch_bytes(int w, int h);
// the mask with the library's per-device scratch array (GES_MASK_STATIC_SCRATCH_BYTES); allocates nothing
size_t freq_mask_static_capacity();
hipError_t launch_freq_mask_static(const float* target, int w, int h, float omega, uint8_t* mask,
                                   hipStream_t stream);
size_t loss_scratch_bytes();
hipError_t launch_loss(const float* img, const float* target, const uint8_t* mask, int w, int h, float lam_l1,
                       float lam_w, void* scratch, float* loss_out, float* dL_dimg, hipStream_t stream);

size_t ssim_scratch_bytes(int w, int h);
hipError_t launch_ssim_loss(const float* img, const float* target, int w, int h, float lam, void* scratch,
                            float* loss, float* dL, hipStream_t stream);


constexpr int kMaxPruneArrays = 18;   // parameters and two moment sets, six arrays each
size_t prune_scratch_bytes(int64_t n);
hipError_t launch_prune(const float* const* src, float* const* dst, const int32_t* rowlen, const float* opacity_logits,
                        const float* beta, int64_t n, double logit_bound, double min_beta, void* scratch,
                        int64_t* total_dev, hipStream_t stream);
hipError_t launch_shape_reset(float* beta, float* m, float* v, int64_t n, float value, hipStream_t stream);
// exclusive offsets of nb block counts and their total (one block)
hipError_t launch_block_scan(const uint32_t* counts, int64_t nb, uint32_t* offsets, int64_t* total,
                             hipStream_t stream);
size_t densify_scratch_bytes(int64_t n);
hipError_t launch_densify_count(const float* accum, const float* count, const float* log_scales, int64_t n,
                                double grad_threshold, double log_scale_bound, void* scratch, hipStream_t stream);
hipError_t launch_densify_scatter(const float* const* src, float* const* dst, const int32_t* rowlen, int nsets,
                                  const float* accum, const float* count, const float* normals, int64_t n,
                                  double grad_threshold, double log_scale_bound, double log_split_div, int64_t unsplit,
                                  int64_t clones, void* scratch, hipStream_t stream);
hipError_t launch_opacity_reset(float* logits, float* m, float* v, int64_t n, double bound, hipStream_t stream);
hipError_t launch_mix_fit(const ges_mix_problem* problems, int nproblems, const float* targets, int ntargets, int m,
                          float x0, float dx, float* params, float* grad_out, float* final_loss, const int32_t* order,
                          int epochs, float lr, float b1, float b2, float eps, hipStream_t stream);
hipError_t launch_adam(const ges_adam_group* groups, int ngroups, int64_t step, float b1, float b2, float eps,
                       hipStream_t stream);

// Workspace pointers read from the view descriptor are generic (flat).  Typed in the global address
// space, loads, stores and atomics through them become global instructions, which count only against
// vmcnt; flat ones count against lgkmcnt too, so every LDS wait would also wait for them.  Records load as
// native 4-float vectors (the float4 class cannot be copied out of another address space).
typedef float Vec4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const Vec4 GlobalRec;
typedef __attribute__((address_space(1))) double GlobalF64;
typedef __attribute__((address_space(1))) Vec4 GlobalVec4;
typedef __attribute__((address_space(1))) uint32_t GlobalU32;

__device__ __forceinline__ float4 rec_load(const GlobalRec* rec, size_t i) {
  const Vec4 v = rec[i];
  return make_float4(v[0], v[1], v[2], v[3]);
}

// Which view owns global block `blk` given a prefix table (linear scan: at most kMaxViews entries).
__device__ inline int view_of_block(const int64_t* prefix, int nviews, int64_t blk) {
  int v = 0;
  while (v + 1 < nviews && prefix[v + 1] <= blk) ++v;
  return v;
}

}  // namespace ges
