// frame.h -- host-side planning of one render frame (workspace layout, view descriptor, launches).
// Shared by the C-ABI entry points and the serving loop.
#pragma once
#include <cmath>
#include <cstring>
#include <string>

#include "ges_internal.h"

namespace ges {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Depth-first binning buffers of a batch of `items` splats (SortWs).
struct SortPlan {
  size_t off_key = 0, off_cand = 0, off_dk0 = 0, off_dv0 = 0, off_dk1 = 0, off_dv1 = 0, off_table = 0,
         off_totals = 0, off_chunks = 0, off_cells = 0, bytes = 0;
};

inline SortPlan plan_sort(int64_t items) {
  SortPlan p;
  const size_t n = (size_t)items;
  size_t o = 0;
  p.off_key = o;    o += align256(n * 4);
  p.off_cand = o;   o += align256(n * 4);
  p.off_dk0 = o;    o += align256(n * 4);
  p.off_dv0 = o;    o += align256(n * 8);
  p.off_dk1 = o;    o += align256(n * 4);
  p.off_dv1 = o;    o += align256(n * 8);
  p.off_table = o;  o += align256((size_t)256 * radix_blocks((uint64_t)n, kRadixItemsDepth) * 4);
  p.off_totals = o; o += 1024;
  p.off_chunks = o; o += align256(((n + 255) / 256 + 1) * 4);
  p.off_cells = o;  o += 256;
  p.bytes = o;
  return p;
}

inline SortWs attach_sort_ws(const SortPlan& p, void* base) {
  char* b = reinterpret_cast<char*>(base);
  SortWs w{};
  w.item_key = reinterpret_cast<uint32_t*>(b + p.off_key);
  w.item_cand = reinterpret_cast<uint32_t*>(b + p.off_cand);
  w.dk[0] = reinterpret_cast<uint32_t*>(b + p.off_dk0);
  w.dv[0] = reinterpret_cast<uint2*>(b + p.off_dv0);
  w.dk[1] = reinterpret_cast<uint32_t*>(b + p.off_dk1);
  w.dv[1] = reinterpret_cast<uint2*>(b + p.off_dv1);
  w.table = reinterpret_cast<uint32_t*>(b + p.off_table);
  w.totals = reinterpret_cast<uint32_t*>(b + p.off_totals);
  w.chunk_off = reinterpret_cast<uint32_t*>(b + p.off_chunks);
  w.cells = reinterpret_cast<uint32_t*>(b + p.off_cells);
  w.depth_final = 1;   // four passes: 0 -> 1 -> 0 -> 1 from the item keys (set again by launch_depth_sort)
  return w;
}

struct FramePlan {
  int tiles_x = 0, tiles_y = 0;
  int64_t tiles = 0;
  // splat workspace; the binning buffers of the frame's own batch come last (a server gives a batch of
  // views one such region and its views only the part before it)
  size_t off_db = 0, off_hdr = 0, off_rec = 0, off_grad = 0, off_vis = 0, off_slotoff = 0, off_ranges = 0,
         off_tstats = 0, off_twork = 0, off_gorder = 0, off_sort = 0;
  size_t view_bytes = 0, splat_bytes = 0;
  // pixel workspace
  size_t off_final_T = 0, off_n_contrib = 0, pixel_bytes = 0;
};

inline FramePlan plan_frame(int64_t n, int w, int h) {
  FramePlan p;
  p.tiles_x = (w + kTile - 1) / kTile;
  p.tiles_y = (h + kTile - 1) / kTile;
  p.tiles = (int64_t)p.tiles_x * p.tiles_y;
  size_t o = 0;
  p.off_db = o;      o += align256(sizeof(DeviceBatch));
  p.off_hdr = o;     o += 256;
  p.off_rec = o;     o += align256((size_t)n * kRecWords * 4);
  p.off_grad = o;    o += align256((size_t)n * kGradStride * 8);
  p.off_vis = o;     o += align256((size_t)n * 4);
  p.off_slotoff = o; o += align256((size_t)n * 4);
  p.off_ranges = o;  o += align256((size_t)p.tiles * 8);
  p.off_tstats = o;  o += align256((size_t)p.tiles * 16);
  p.off_twork = o;   o += align256((size_t)p.tiles * 4);
  p.off_gorder = o;  o += align256((size_t)(p.tiles + 7) / 8 * 4);
  p.view_bytes = o;
  p.off_sort = o;    o += plan_sort(n).bytes;
  p.splat_bytes = o;
  size_t q = 0;
  const size_t px = (size_t)w * h;
  p.off_final_T = q;   q += align256(px * 4);
  p.off_n_contrib = q; q += align256(px * 4);
  p.pixel_bytes = q;
  return p;
}

// Workspaces of a step over `views` views of one scene at one resolution: the view table, the per-view
// regions of the single-view layout one after another (view 0 at the single-view offsets), then the
// binning buffers of the views x n items; the views' pixel workspaces one after another.  One view gives
// exactly the single-view layout.
struct ViewsPlan {
  FramePlan fp;                  // the layout of one view
  int32_t views = 1;
  size_t view_stride = 0;        // bytes between the per-view regions
  size_t off_sort = 0, splat_bytes = 0, pixel_bytes = 0;
};

inline ViewsPlan plan_views(int64_t n, int32_t views, int w, int h) {
  ViewsPlan p;
  p.fp = plan_frame(n, w, h);
  p.views = views;
  p.view_stride = p.fp.view_bytes - p.fp.off_hdr;
  p.off_sort = p.fp.view_bytes + (size_t)(views - 1) * p.view_stride;
  p.splat_bytes = p.off_sort + plan_sort((int64_t)views * n).bytes;
  p.pixel_bytes = (size_t)views * p.fp.pixel_bytes;
  return p;
}

// Tile passes of a batch: 8-bit digits covering the largest batch tile id.
inline int tile_passes(int64_t total_tiles) {
  int bits = 1;
  while (bits < 63 && ((int64_t)1 << bits) < total_tiles) ++bits;
  return (bits + 7) / 8;
}

// Key workspace of `slots` candidate slots: two buffers of (tile; splat index, slot) pairs, the values of
// buffer 0 first (the sorted pairs the raster reads); the table of the tile passes; and, for frames that
// run the backward pass, one 48-byte row per slot for the backward's per-(tile, splat) sums with a bit per
// slot marking the written rows.
struct KeyPlan {
  size_t off_pv0 = 0, off_key0 = 0, off_pv1 = 0, off_key1 = 0, off_table = 0, off_totals = 0, off_rows = 0,
         off_bits = 0, bytes = 0;
};

inline KeyPlan plan_keys(uint64_t slots, bool backward_rows) {
  KeyPlan p;
  const size_t k = (size_t)slots;
  size_t o = 0;
  p.off_pv0 = o;    o += align256(k * 8);
  p.off_key0 = o;   o += align256(k * 4);
  p.off_pv1 = o;    o += align256(k * 8);
  p.off_key1 = o;   o += align256(k * 4);
  p.off_table = o;  o += align256((size_t)256 * radix_blocks(slots, kRadixItemsPair) * 4);
  p.off_totals = o; o += 1024;
  if (backward_rows) {
    p.off_rows = o; o += align256(k * kRowFloats * 4);
    p.off_bits = o; o += align256((k + 31) / 32 * 4);
  }
  p.bytes = o;
  return p;
}

inline KeyWs attach_key_ws(const KeyPlan& p, void* base) {
  char* b = reinterpret_cast<char*>(base);
  KeyWs w{};
  w.pv[0] = reinterpret_cast<uint2*>(b + p.off_pv0);
  w.key[0] = reinterpret_cast<uint32_t*>(b + p.off_key0);
  w.pv[1] = reinterpret_cast<uint2*>(b + p.off_pv1);
  w.key[1] = reinterpret_cast<uint32_t*>(b + p.off_key1);
  w.table = reinterpret_cast<uint32_t*>(b + p.off_table);
  w.totals = reinterpret_cast<uint32_t*>(b + p.off_totals);
  return w;
}

// Validation of the public structs; returns an empty string when valid.
inline std::string check_camera(const ges_camera* c) {
  if (!c) return "camera is NULL";
  if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384) return "width/height outside [1,16384]";
  const float vals[] = {c->fx, c->fy, c->cx, c->cy, c->near_z};
  for (float v : vals)
    if (!std::isfinite(v)) return "non-finite camera intrinsics";
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(c->R[k])) return "non-finite rotation";
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(c->t[k])) return "non-finite translation";
  if (!(c->fx > 0.f) || !(c->fy > 0.f)) return "focal lengths must be positive";
  if (!(c->near_z > 0.f)) return "near_z must be positive";
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double d = 0.0;
      for (int k = 0; k < 3; ++k) d += (double)c->R[3 * i + k] * (double)c->R[3 * j + k];
      if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-4) return "R is not orthonormal to 1e-4";
    }
  double det = (double)c->R[0] * ((double)c->R[4] * c->R[8] - (double)c->R[5] * c->R[7]) -
               (double)c->R[1] * ((double)c->R[3] * c->R[8] - (double)c->R[5] * c->R[6]) +
               (double)c->R[2] * ((double)c->R[3] * c->R[7] - (double)c->R[4] * c->R[6]);
  if (det < 0.0) return "R is a reflection";
  return "";
}

inline std::string check_splats(const ges_splats* s) {
  if (!s) return "splats is NULL";
  if (s->n < 0 || s->n >= (int64_t(1) << 31)) return "n outside [0, 2^31)";
  if (s->sh_degree < 0 || s->sh_degree > 3) return "sh_degree outside [0,3]";
  if (s->n > 0 && (!s->means || !s->log_scales || !s->quats || !s->opacity_logits || !s->sh || !s->beta))
    return "NULL splat array";
  if (s->n > 0 && (reinterpret_cast<uintptr_t>(s->quats) & 15u)) return "quats must be 16-byte aligned";
  if (s->n > 0 && (s->sh_degree == 1 || s->sh_degree == 3) && (reinterpret_cast<uintptr_t>(s->sh) & 15u))
    return "sh must be 16-byte aligned";
  return "";
}

inline std::string check_params(const ges_raster_params* p) {
  if (!p) return "params is NULL";
  if (p->falloff != GES_FALLOFF_PHI && p->falloff != GES_FALLOFF_GEF && p->falloff != GES_FALLOFF_PHI_EXACT)
    return "unknown falloff";
  if (p->tile_cull != GES_TILES_SQUARE && p->tile_cull != GES_TILES_ELLIPSE) return "unknown tile_cull";
  if (!std::isfinite(p->rho) || !std::isfinite(p->bg[0]) || !std::isfinite(p->bg[1]) || !std::isfinite(p->bg[2]))
    return "non-finite raster parameter";
  return "";
}

// Fill the camera / scene / parameter part of a view descriptor.  Derived camera values use the same
// binary32 operation order as the per-splat preprocess.
inline void fill_view(ViewDesc& V, const ges_splats* s, const ges_camera* c, const ges_raster_params* p) {
  std::memset(&V, 0, sizeof(V));
  V.means = s->means; V.log_scales = s->log_scales; V.quats = s->quats; V.logits = s->opacity_logits;
  V.sh = s->sh; V.beta = s->beta; V.n = s->n; V.sh_degree = s->sh_degree;
  V.sh_coeffs = (s->sh_degree + 1) * (s->sh_degree + 1);
  for (int k = 0; k < 9; ++k) V.R[k] = c->R[k];
  for (int k = 0; k < 3; ++k) V.t[k] = c->t[k];
  for (int j = 0; j < 3; ++j) {   // camera centre -R^T t
    volatile float acc = c->R[j] * c->t[0];
    acc = acc + c->R[3 + j] * c->t[1];
    acc = acc + c->R[6 + j] * c->t[2];
    V.campos[j] = -acc;
  }
  V.fx = c->fx; V.fy = c->fy; V.cx = c->cx; V.cy = c->cy; V.near_z = c->near_z;
  volatile float lx = 0.5f * (float)c->width;
  lx = lx / c->fx;
  lx = 1.3f * lx;
  volatile float ly = 0.5f * (float)c->height;
  ly = ly / c->fy;
  ly = 1.3f * ly;
  V.limx = lx; V.limy = ly;
  V.width = c->width; V.height = c->height;
  V.tiles_x = (c->width + kTile - 1) / kTile;
  V.tiles_y = (c->height + kTile - 1) / kTile;
  V.falloff = p->falloff; V.tile_cull = p->tile_cull; V.rho = p->rho;
  for (int k = 0; k < 3; ++k) V.bg[k] = p->bg[k];
}

// The per-view part of a splat workspace (the item arrays are attached with the batch's SortWs).
inline void attach_splat_ws(ViewDesc& V, const FramePlan& fp, void* splat_ws) {
  char* b = reinterpret_cast<char*>(splat_ws);
  V.rec = reinterpret_cast<float4*>(b + fp.off_rec);
  V.grad2d = reinterpret_cast<double*>(b + fp.off_grad);
  V.vis = reinterpret_cast<uint32_t*>(b + fp.off_vis);
  V.slot_off = reinterpret_cast<uint32_t*>(b + fp.off_slotoff);
  V.ranges = reinterpret_cast<uint2*>(b + fp.off_ranges);
  V.tile_stats = reinterpret_cast<unsigned long long*>(b + fp.off_tstats);
  V.tile_work = reinterpret_cast<uint32_t*>(b + fp.off_twork);
  V.group_order = reinterpret_cast<uint32_t*>(b + fp.off_gorder);
  V.header = reinterpret_cast<unsigned long long*>(b + fp.off_hdr);
}

}  // namespace ges
