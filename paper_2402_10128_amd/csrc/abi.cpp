// abi.cpp -- the C ABI of the GES rasterizer (include/ges.h): validation, workspace planning and
// the launch sequences of one frame.  No allocation happens here: every buffer is the caller's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "frame.h"
#include "ges_internal.h"

namespace {

thread_local std::string g_last_error;
thread_local ges::DeviceBatch g_host_batch;   // staging copy of the view table (pageable; copied per call)

// The key workspace and slot capacity each splat workspace was last rendered with: the backward pass reads
// the sorted pairs and writes its rows there (its signature carries no slot count).
std::mutex g_keys_mu;
std::unordered_map<const void*, std::pair<void*, uint64_t>> g_keys_of_frame;

ges_status fail(ges_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

ges_status device_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return GES_ERR_DEVICE;
}

#define GES_CHECK_HIP(expr, where)                 \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return device_fail(e_, where); \
  } while (0)

// ---- stage timing: event pairs recorded around launches while profiling is on
struct Profiler {
  std::mutex mu;
  bool on = false;
  uint32_t mask = ~0u;   // stages timed while on
  std::vector<hipEvent_t> free_events;
  struct Pending { int stage; hipEvent_t a, b; };
  std::vector<Pending> pending;
  double ms[GES_NUM_STAGES] = {};
  int64_t launches[GES_NUM_STAGES] = {};

  hipEvent_t get() {
    if (!free_events.empty()) { hipEvent_t e = free_events.back(); free_events.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Profiler g_prof;

template <class F>
hipError_t timed(int stage, hipStream_t stream, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (g_prof.on && ((g_prof.mask >> stage) & 1u)) { a = g_prof.get(); b = g_prof.get(); }
  }
  if (a) { hipError_t e = hipEventRecord(a, stream); if (e != hipSuccess) return e; }
  hipError_t e = launch();
  if (e != hipSuccess) return e;
  if (a && b) {
    e = hipEventRecord(b, stream);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.pending.push_back({stage, a, b});
  }
  return hipSuccess;
}

// Build the batch of a step's views (one scene, one resolution) and copy it into the splat workspace.
hipError_t upload_views(const ges_splats* s, const ges_camera* cams, int32_t nv, const ges_raster_params* p,
                        const ges::ViewsPlan& vp, void* splat_ws, void* pixel_ws, float* out_rgb,
                        const float* dL_drgb, hipStream_t stream, void* key_ws = nullptr, uint64_t key_slots = 0) {
  ges::DeviceBatch& hb = g_host_batch;
  const ges::FramePlan& fp = vp.fp;
  const int64_t pre = (s->n + 255) / 256;
  const size_t px3 = (size_t)3 * cams[0].width * cams[0].height;
  hb.nviews = nv;
  for (int32_t v = 0; v <= nv; ++v) {
    hb.pre_prefix[v] = v * pre;
    hb.item_prefix[v] = v * s->n;
    hb.tile_prefix[v] = v * fp.tiles;
  }
  char* sw_base = reinterpret_cast<char*>(splat_ws);
  const ges::SortWs sw = ges::attach_sort_ws(ges::plan_sort((int64_t)nv * s->n), sw_base + vp.off_sort);
  for (int32_t v = 0; v < nv; ++v) {
    ges::ViewDesc& V = hb.views[v];
    ges::fill_view(V, s, &cams[v], p);
    ges::attach_splat_ws(V, fp, sw_base + (size_t)v * vp.view_stride);
    V.item_key = sw.item_key + (size_t)v * s->n;
    V.item_cand = sw.item_cand + (size_t)v * s->n;
    if (pixel_ws) {
      char* pw = reinterpret_cast<char*>(pixel_ws) + (size_t)v * fp.pixel_bytes;
      V.final_T = reinterpret_cast<float*>(pw + fp.off_final_T);
      V.n_contrib = reinterpret_cast<uint32_t*>(pw + fp.off_n_contrib);
    }
    V.out_rgb = out_rgb ? out_rgb + v * px3 : nullptr;
    V.dL_drgb = dL_drgb ? dL_drgb + v * px3 : nullptr;
    if (key_ws && key_slots) {   // the backward's rows of per-(tile, splat) sums (one slot space per batch)
      const ges::KeyPlan kp = ges::plan_keys(key_slots, true);
      char* kw = reinterpret_cast<char*>(key_ws);
      V.sorted_pairs = reinterpret_cast<const uint2*>(kw + kp.off_pv0);
      V.grad_rows = reinterpret_cast<float*>(kw + kp.off_rows);
      V.grad_bits = reinterpret_cast<uint32_t*>(kw + kp.off_bits);
      V.grad_slots = key_slots;
    }
    V.keep_grad2d = (p->flags & GES_RASTER_KEEP_GRAD2D) ? 1 : 0;
  }
  return hipMemcpyAsync(sw_base + fp.off_db, &hb, ges::device_batch_bytes(nv), hipMemcpyHostToDevice, stream);
}

ges::Batch views_batch(const ges_splats* s, const ges_raster_params* p, const ges::ViewsPlan& vp, void* splat_ws) {
  ges::Batch b{};
  b.nviews = vp.views;
  b.falloff = p->falloff;
  b.total_tiles = vp.views * vp.fp.tiles;
  b.tile_cull = p->tile_cull;
  b.pre_blocks = vp.views * ((s->n + 255) / 256);
  b.items = vp.views * s->n;
  b.sw = ges::attach_sort_ws(ges::plan_sort(b.items), reinterpret_cast<char*>(splat_ws) + vp.off_sort);
  b.keys_total = &b.sw.cells[1];
  b.tile_passes = ges::tile_passes(b.total_tiles);
  b.dup_buffer = b.tile_passes & 1;
  b.shared_scene = 1;
  return b;
}

const ges::DeviceBatch* dev_batch(void* splat_ws, const ges::FramePlan& fp) {
  return reinterpret_cast<const ges::DeviceBatch*>(reinterpret_cast<char*>(splat_ws) + fp.off_db);
}

std::string check_all(const ges_splats* s, const ges_camera* c, const ges_raster_params* p) {
  std::string e = ges::check_splats(s);
  if (e.empty()) e = ges::check_camera(c);
  if (e.empty()) e = ges::check_params(p);
  return e;
}

// The views of one step: 1..kMaxViews cameras of one resolution over one scene.
std::string check_views(const ges_splats* s, const ges_camera* cams, int32_t nv, const ges_raster_params* p) {
  if (nv < 1 || nv > ges::kMaxViews) return "num_views outside [1, 64]";
  if (!cams) return "cams is NULL";
  std::string e = ges::check_splats(s);
  if (e.empty()) e = ges::check_params(p);
  for (int32_t v = 0; v < nv && e.empty(); ++v) {
    e = ges::check_camera(&cams[v]);
    if (e.empty() && (cams[v].width != cams[0].width || cams[v].height != cams[0].height))
      e = "every view of a step must have the same width and height";
  }
  if (e.empty() && (int64_t)nv * s->n >= (int64_t(1) << 31)) e = "num_views x n outside [0, 2^31)";
  return e;
}

ges_status preprocess_views(const ges_splats* splats, const ges_camera* cams, int32_t nv,
                            const ges_raster_params* params, void* splat_ws, size_t splat_ws_bytes,
                            uint64_t* num_keys_host, void* stream_) {
  const std::string e = check_views(splats, cams, nv, params);
  if (!e.empty()) return fail(GES_ERR_INVALID_ARGUMENT, e);
  if (!splat_ws) return fail(GES_ERR_INVALID_ARGUMENT, "splat_ws is NULL");
  if (reinterpret_cast<uintptr_t>(splat_ws) & 255u) return fail(GES_ERR_INVALID_ARGUMENT, "splat_ws must be 256-byte aligned");
  const ges::ViewsPlan vp = ges::plan_views(splats->n, nv, cams[0].width, cams[0].height);
  if (splat_ws_bytes < vp.splat_bytes) return fail(GES_ERR_CAPACITY, "splat workspace too small");
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  GES_CHECK_HIP(upload_views(splats, cams, nv, params, vp, splat_ws, nullptr, nullptr, nullptr, stream), "upload");
  ges::Batch b = views_batch(splats, params, vp, splat_ws);
  const ges::DeviceBatch* db = dev_batch(splat_ws, vp.fp);
  GES_CHECK_HIP(timed(GES_STAGE_PREPROCESS, stream, [&] { return ges::launch_preprocess(db, b, stream); }), "preprocess");
  GES_CHECK_HIP(timed(GES_STAGE_DEPTH_SORT, stream, [&] { return ges::launch_depth_sort(db, b, stream); }), "depth_sort");
  GES_CHECK_HIP(timed(GES_STAGE_KEY_SCAN, stream, [&] { return ges::launch_key_scan(db, b, stream); }), "key_scan");
  if (num_keys_host) {
    uint32_t k = 0;
    GES_CHECK_HIP(hipMemcpyAsync(&k, b.keys_total, 4, hipMemcpyDeviceToHost, stream), "read num_keys");
    GES_CHECK_HIP(hipStreamSynchronize(stream), "sync");
    if (k == 0xffffffffu) return fail(GES_ERR_CAPACITY, "more than 2^32-2 candidate (tile, splat) pairs in one step");
    *num_keys_host = k;
  }
  return GES_OK;
}

ges_status render_forward_views(const ges_splats* splats, const ges_camera* cams, int32_t nv,
                                const ges_raster_params* params, void* splat_ws, void* key_ws, size_t key_ws_bytes,
                                uint64_t num_keys, void* pixel_ws, float* out_rgb, void* stream_) {
  const std::string e = check_views(splats, cams, nv, params);
  if (!e.empty()) return fail(GES_ERR_INVALID_ARGUMENT, e);
  if (!splat_ws || !pixel_ws || !out_rgb) return fail(GES_ERR_INVALID_ARGUMENT, "NULL workspace or output");
  if ((reinterpret_cast<uintptr_t>(splat_ws) | reinterpret_cast<uintptr_t>(pixel_ws)) & 255u)
    return fail(GES_ERR_INVALID_ARGUMENT, "workspaces must be 256-byte aligned");
  if (num_keys >= 0xffffffffull) return fail(GES_ERR_CAPACITY, "more than 2^32-2 keys");
  const ges::ViewsPlan vp = ges::plan_views(splats->n, nv, cams[0].width, cams[0].height);
  const ges::KeyPlan kp = ges::plan_keys(num_keys, true);
  if (num_keys > 0 && (!key_ws || key_ws_bytes < kp.bytes)) return fail(GES_ERR_CAPACITY, "key workspace too small");
  if (num_keys > 0 && (reinterpret_cast<uintptr_t>(key_ws) & 255u))
    return fail(GES_ERR_INVALID_ARGUMENT, "key_ws must be 256-byte aligned");
  {
    std::lock_guard<std::mutex> lk(g_keys_mu);
    g_keys_of_frame[splat_ws] = {num_keys > 0 ? key_ws : nullptr, num_keys};
  }
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  GES_CHECK_HIP(upload_views(splats, cams, nv, params, vp, splat_ws, pixel_ws, out_rgb, nullptr, stream), "upload");
  ges::Batch b = views_batch(splats, params, vp, splat_ws);
  b.key_capacity = num_keys;
  if (num_keys > 0) {
    b.kw = ges::attach_key_ws(kp, key_ws);
    b.sorted_pairs = b.kw.pv[0];
    b.sorted_tiles = b.kw.key[0];
  }
  const ges::DeviceBatch* db = dev_batch(splat_ws, vp.fp);
  GES_CHECK_HIP(timed(GES_STAGE_DUPLICATE, stream, [&] { return ges::launch_duplicate(db, b, stream); }), "duplicate");
  GES_CHECK_HIP(timed(GES_STAGE_TILE_SORT, stream, [&] { return ges::launch_tile_sort(db, b, stream); }), "tile_sort");
  GES_CHECK_HIP(timed(GES_STAGE_RASTER_FORWARD, stream, [&] { return ges::launch_raster_forward(db, b, stream); }), "raster_forward");
  return GES_OK;
}

ges_status render_backward(const ges_splats* splats, const ges_camera* cams, int32_t nv,
                           const ges_raster_params* params, void* splat_ws, void* key_ws, void* pixel_ws,
                           const float* dL_drgb, const ges_splat_grads* grads, const ges::AdamSplats* adam,
                           bool fused, void* stream_) {
  const std::string e = check_views(splats, cams, nv, params);
  if (!e.empty()) return fail(GES_ERR_INVALID_ARGUMENT, e);
  if (!splat_ws || !pixel_ws || !dL_drgb || (!grads && !fused)) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if ((reinterpret_cast<uintptr_t>(splat_ws) | reinterpret_cast<uintptr_t>(pixel_ws)) & 255u)
    return fail(GES_ERR_INVALID_ARGUMENT, "workspaces must be 256-byte aligned");
  const ges_splat_grads none{};
  if (!grads) grads = &none;
  if (grads->quats && (reinterpret_cast<uintptr_t>(grads->quats) & 15u))
    return fail(GES_ERR_INVALID_ARGUMENT, "grads->quats must be 16-byte aligned");
  if (grads->sh && (splats->sh_degree == 1 || splats->sh_degree == 3) && (reinterpret_cast<uintptr_t>(grads->sh) & 15u))
    return fail(GES_ERR_INVALID_ARGUMENT, "grads->sh must be 16-byte aligned");
  const ges::ViewsPlan vp = ges::plan_views(splats->n, nv, cams[0].width, cams[0].height);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  uint64_t slots = 0;
  {
    std::lock_guard<std::mutex> lk(g_keys_mu);
    auto it = g_keys_of_frame.find(splat_ws);
    if (it == g_keys_of_frame.end()) return fail(GES_ERR_INVALID_ARGUMENT, "no forward pass of this splat workspace");
    if (it->second.first != (it->second.second ? key_ws : nullptr))
      return fail(GES_ERR_INVALID_ARGUMENT, "key_ws differs from the forward pass of this splat workspace");
    slots = it->second.second;
  }
  GES_CHECK_HIP(upload_views(splats, cams, nv, params, vp, splat_ws, pixel_ws, nullptr, dL_drgb, stream, key_ws,
                             slots), "upload");
  ges::Batch b = views_batch(splats, params, vp, splat_ws);
  const ges::KeyPlan kp = ges::plan_keys(slots, true);
  if (slots) b.sorted_pairs = reinterpret_cast<const uint2*>(reinterpret_cast<char*>(key_ws) + kp.off_pv0);
  const ges::DeviceBatch* db = dev_batch(splat_ws, vp.fp);
  if (slots)
    GES_CHECK_HIP(timed(GES_STAGE_ZERO, stream, [&] {
                    return ges::launch_zero(reinterpret_cast<char*>(key_ws) + kp.off_bits, (slots + 31) / 32 * 4,
                                            stream);
                  }), "clear row marks");
  GES_CHECK_HIP(timed(GES_STAGE_RASTER_BACKWARD, stream, [&] { return ges::launch_raster_backward(db, b, stream); }), "raster_backward");
  // every listed splat's row of grad2d (zero when its slots lie beyond the key capacity)
  char* kwb = reinterpret_cast<char*>(key_ws);
  GES_CHECK_HIP(timed(GES_STAGE_ROW_REDUCE, stream, [&] {
                  return ges::launch_row_reduce(db, b, slots ? reinterpret_cast<const float*>(kwb + kp.off_rows) : nullptr,
                                                slots ? reinterpret_cast<const uint32_t*>(kwb + kp.off_bits) : nullptr,
                                                slots, stream);
                }), "row_reduce");
  GES_CHECK_HIP(timed(GES_STAGE_PREPROCESS_BACKWARD, stream,
                      [&] { return ges::launch_preprocess_backward(db, b, grads, stream, adam, fused); }),
                "preprocess_backward");
  return GES_OK;
}

// The optimiser arguments of a fused backward (the Adam update of ges_adam_step).
ges_status adam_args(const ges_splats* splats, const ges_camera* cam, const ges_adam_splats* opt, ges::AdamSplats& a) {
  if (!opt || !splats) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if (opt->step < 1) return fail(GES_ERR_INVALID_ARGUMENT, "step < 1");
  if (!(opt->beta1 >= 0.f && opt->beta1 < 1.f) || !(opt->beta2 >= 0.f && opt->beta2 < 1.f))
    return fail(GES_ERR_INVALID_ARGUMENT, "beta outside [0,1)");
  if (!(opt->eps >= 0.f) || !std::isfinite(opt->eps)) return fail(GES_ERR_INVALID_ARGUMENT, "bad eps");
  a = ges::AdamSplats{};
  const float* params_in[ges::kNumPar] = {splats->means, splats->log_scales, splats->quats, splats->opacity_logits,
                                          splats->sh, splats->beta};
  const double bc1 = 1.0 - std::pow((double)opt->beta1, (double)opt->step);
  const double bc2 = 1.0 - std::pow((double)opt->beta2, (double)opt->step);
  for (int k = 0; k < ges::kNumPar; ++k) {
    if (!(opt->lr[k] >= 0.f) || !std::isfinite(opt->lr[k])) return fail(GES_ERR_INVALID_ARGUMENT, "bad lr");
    if (splats->n > 0 && (!opt->exp_avg[k] || !opt->exp_avg_sq[k]))
      return fail(GES_ERR_INVALID_ARGUMENT, "NULL moment array");
    a.p[k] = const_cast<float*>(params_in[k]);
    a.m[k] = opt->exp_avg[k];
    a.v[k] = opt->exp_avg_sq[k];
    a.step_size[k] = (float)((double)opt->lr[k] / bc1);
  }
  const bool sh_vec = splats->sh_degree == 1 || splats->sh_degree == 3;
  for (int k : {ges::kParQuats, ges::kParSh}) {
    if (k == ges::kParSh && !sh_vec) continue;
    if ((reinterpret_cast<uintptr_t>(a.m[k]) | reinterpret_cast<uintptr_t>(a.v[k])) & 15u)
      return fail(GES_ERR_INVALID_ARGUMENT, "quats/sh moments must be 16-byte aligned");
  }
  a.b1 = opt->beta1;
  a.b2 = opt->beta2;
  a.eps = opt->eps;
  a.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
  if ((opt->grad_accum == nullptr) != (opt->grad_count == nullptr))
    return fail(GES_ERR_INVALID_ARGUMENT, "grad_accum and grad_count go together");
  a.stat_accum = opt->grad_accum;
  a.stat_count = opt->grad_count;
  a.half_w = cam ? 0.5 * (double)cam->width : 0.0;
  a.half_h = cam ? 0.5 * (double)cam->height : 0.0;
  for (int k = 0; k < ges::kNumPar; ++k) a.gin[k] = opt->grads_in[k];
  if ((reinterpret_cast<uintptr_t>(a.gin[ges::kParQuats]) & 15u) ||
      (sh_vec && (reinterpret_cast<uintptr_t>(a.gin[ges::kParSh]) & 15u)))
    return fail(GES_ERR_INVALID_ARGUMENT, "grads_in quats/sh must be 16-byte aligned");
  return GES_OK;
}

ges_status backward_views_plain(const ges_splats* splats, const ges_camera* cams, int32_t nv,
                                const ges_raster_params* params, void* splat_ws, void* key_ws, void* pixel_ws,
                                const float* dL_drgb, const ges_splat_grads* grads, int32_t accumulate,
                                float* grad_accum, float* grad_count, void* stream) {
  if (!grads || !cams) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if ((grad_accum == nullptr) != (grad_count == nullptr))
    return fail(GES_ERR_INVALID_ARGUMENT, "grad_accum and grad_count go together");
  ges::AdamSplats a{};
  a.accumulate = accumulate ? 1 : 0;
  a.stat_accum = grad_accum;
  a.stat_count = grad_count;
  a.half_w = 0.5 * (double)cams[0].width;
  a.half_h = 0.5 * (double)cams[0].height;
  return render_backward(splats, cams, nv, params, splat_ws, key_ws, pixel_ws, dL_drgb, grads, &a, false, stream);
}

ges_status frame_view(int64_t n, int32_t nv, int32_t width, int32_t height, void* splat_ws, void* key_ws,
                      uint64_t num_keys, void* pixel_ws, int32_t view, ges_frame_view* out) {
  if (!out || !splat_ws) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if (n < 0 || width < 1 || height < 1 || width > 16384 || height > 16384)
    return fail(GES_ERR_INVALID_ARGUMENT, "bad sizes");
  if (nv < 1 || nv > ges::kMaxViews || view < 0 || view >= nv)
    return fail(GES_ERR_INVALID_ARGUMENT, "view outside [0, num_views)");
  const ges::ViewsPlan vp = ges::plan_views(n, nv, width, height);
  const ges::FramePlan& fp = vp.fp;
  char* sw = reinterpret_cast<char*>(splat_ws) + (size_t)view * vp.view_stride;
  std::memset(out, 0, sizeof(*out));
  out->records = reinterpret_cast<const float*>(sw + fp.off_rec);
  out->tile_ranges = reinterpret_cast<const uint32_t*>(sw + fp.off_ranges);
  out->grad2d = reinterpret_cast<const double*>(sw + fp.off_grad);
  out->stats = reinterpret_cast<const uint64_t*>(sw + fp.off_hdr);
  if (key_ws) {
    const ges::KeyPlan kp = ges::plan_keys(num_keys, true);
    char* kw = reinterpret_cast<char*>(key_ws);
    out->sorted_pairs = reinterpret_cast<const uint32_t*>(kw + kp.off_pv0);
    out->sorted_tiles = reinterpret_cast<const uint32_t*>(kw + kp.off_key0);
    out->row_marks = reinterpret_cast<const uint32_t*>(kw + kp.off_bits);
  }
  if (pixel_ws) {
    char* pw = reinterpret_cast<char*>(pixel_ws) + (size_t)view * fp.pixel_bytes;
    out->final_T = reinterpret_cast<const float*>(pw + fp.off_final_T);
    out->n_contrib = reinterpret_cast<const uint32_t*>(pw + fp.off_n_contrib);
  }
  out->tiles_x = fp.tiles_x;
  out->tiles_y = fp.tiles_y;
  out->tile_work = reinterpret_cast<const uint32_t*>(sw + fp.off_twork);
  out->group_order = reinterpret_cast<const uint32_t*>(sw + fp.off_gorder);
  return GES_OK;
}

}  // namespace

extern "C" {

uint32_t ges_abi_version(void) { return GES_ABI_VERSION; }

const char* ges_last_error(void) { return g_last_error.c_str(); }

ges_status ges_workspace_query(int64_t n, int32_t width, int32_t height, size_t* splat_ws_bytes,
                               size_t* pixel_ws_bytes) {
  return ges_views_workspace_query(n, 1, width, height, splat_ws_bytes, pixel_ws_bytes);
}

ges_status ges_views_workspace_query(int64_t n, int32_t num_views, int32_t width, int32_t height,
                                     size_t* splat_ws_bytes, size_t* pixel_ws_bytes) {
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(GES_ERR_INVALID_ARGUMENT, "n outside [0, 2^31)");
  if (width < 1 || height < 1 || width > 16384 || height > 16384)
    return fail(GES_ERR_INVALID_ARGUMENT, "width/height outside [1,16384]");
  if (num_views < 1 || num_views > ges::kMaxViews) return fail(GES_ERR_INVALID_ARGUMENT, "num_views outside [1, 64]");
  if ((int64_t)num_views * n >= (int64_t(1) << 31))
    return fail(GES_ERR_INVALID_ARGUMENT, "num_views x n outside [0, 2^31)");
  const ges::ViewsPlan vp = ges::plan_views(n, num_views, width, height);
  if (splat_ws_bytes) *splat_ws_bytes = vp.splat_bytes;
  if (pixel_ws_bytes) *pixel_ws_bytes = vp.pixel_bytes;
  return GES_OK;
}

ges_status ges_key_workspace_query(uint64_t num_keys, int64_t n, int32_t width, int32_t height, size_t* key_ws_bytes) {
  (void)n;
  if (!key_ws_bytes) return fail(GES_ERR_INVALID_ARGUMENT, "key_ws_bytes is NULL");
  if (width < 1 || height < 1 || width > 16384 || height > 16384)
    return fail(GES_ERR_INVALID_ARGUMENT, "width/height outside [1,16384]");
  if (num_keys >= 0xffffffffull) return fail(GES_ERR_CAPACITY, "more than 2^32-2 keys");
  *key_ws_bytes = ges::plan_keys(num_keys, true).bytes;
  return GES_OK;
}

ges_status ges_preprocess(const ges_splats* splats, const ges_camera* cam, const ges_raster_params* params,
                          void* splat_ws, size_t splat_ws_bytes, uint64_t* num_keys_host, void* stream) {
  if (!cam) return fail(GES_ERR_INVALID_ARGUMENT, "camera is NULL");
  return preprocess_views(splats, cam, 1, params, splat_ws, splat_ws_bytes, num_keys_host, stream);
}

ges_status ges_preprocess_views(const ges_splats* splats, const ges_camera* cams, int32_t num_views,
                                const ges_raster_params* params, void* splat_ws, size_t splat_ws_bytes,
                                uint64_t* num_keys_host, void* stream) {
  return preprocess_views(splats, cams, num_views, params, splat_ws, splat_ws_bytes, num_keys_host, stream);
}

ges_status ges_render_forward(const ges_splats* splats, const ges_camera* cam, const ges_raster_params* params,
                              void* splat_ws, void* key_ws, size_t key_ws_bytes, uint64_t num_keys, void* pixel_ws,
                              float* out_rgb, void* stream) {
  if (!cam) return fail(GES_ERR_INVALID_ARGUMENT, "camera is NULL");
  return render_forward_views(splats, cam, 1, params, splat_ws, key_ws, key_ws_bytes, num_keys, pixel_ws, out_rgb,
                              stream);
}

ges_status ges_render_forward_views(const ges_splats* splats, const ges_camera* cams, int32_t num_views,
                                    const ges_raster_params* params, void* splat_ws, void* key_ws,
                                    size_t key_ws_bytes, uint64_t num_keys, void* pixel_ws, float* out_rgb,
                                    void* stream) {
  return render_forward_views(splats, cams, num_views, params, splat_ws, key_ws, key_ws_bytes, num_keys, pixel_ws,
                              out_rgb, stream);
}

ges_status ges_render_backward(const ges_splats* splats, const ges_camera* cam, const ges_raster_params* params,
                               void* splat_ws, void* key_ws, void* pixel_ws, const float* dL_drgb,
                               const ges_splat_grads* grads, void* stream) {
  if (!grads || !cam) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  return render_backward(splats, cam, 1, params, splat_ws, key_ws, pixel_ws, dL_drgb, grads, nullptr, false, stream);
}

ges_status ges_render_backward_accumulate(const ges_splats* splats, const ges_camera* cam,
                                          const ges_raster_params* params, void* splat_ws, void* key_ws,
                                          void* pixel_ws, const float* dL_drgb, const ges_splat_grads* grads,
                                          float* grad_accum, float* grad_count, void* stream) {
  return backward_views_plain(splats, cam, 1, params, splat_ws, key_ws, pixel_ws, dL_drgb, grads, 1, grad_accum,
                              grad_count, stream);
}

ges_status ges_render_backward_views(const ges_splats* splats, const ges_camera* cams, int32_t num_views,
                                     const ges_raster_params* params, void* splat_ws, void* key_ws, void* pixel_ws,
                                     const float* dL_drgb, const ges_splat_grads* grads, int32_t accumulate,
                                     float* grad_accum, float* grad_count, void* stream) {
  return backward_views_plain(splats, cams, num_views, params, splat_ws, key_ws, pixel_ws, dL_drgb, grads, accumulate,
                              grad_accum, grad_count, stream);
}

ges_status ges_render_backward_adam(const ges_splats* splats, const ges_camera* cam, const ges_raster_params* params,
                                    void* splat_ws, void* key_ws, void* pixel_ws, const float* dL_drgb,
                                    const ges_splat_grads* grads, const ges_adam_splats* opt, void* stream) {
  if (!cam) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  ges::AdamSplats a;
  const ges_status st = adam_args(splats, cam, opt, a);
  if (st != GES_OK) return st;
  return render_backward(splats, cam, 1, params, splat_ws, key_ws, pixel_ws, dL_drgb, grads, &a, true, stream);
}

ges_status ges_render_backward_views_adam(const ges_splats* splats, const ges_camera* cams, int32_t num_views,
                                          const ges_raster_params* params, void* splat_ws, void* key_ws,
                                          void* pixel_ws, const float* dL_drgb, const ges_splat_grads* grads,
                                          const ges_adam_splats* opt, void* stream) {
  if (!cams) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  ges::AdamSplats a;
  const ges_status st = adam_args(splats, &cams[0], opt, a);
  if (st != GES_OK) return st;
  if (num_views > 1) {   // the earlier views' sum goes through `grads`, which the last view's update reads
    for (int k = 0; k < ges::kNumPar; ++k)
      if (opt->grads_in[k]) return fail(GES_ERR_INVALID_ARGUMENT, "grads_in must be NULL with more than one view");
    if (!grads || !grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits || !grads->sh ||
        !grads->beta)
      return fail(GES_ERR_INVALID_ARGUMENT, "every grads buffer is needed with more than one view");
    const float* g[ges::kNumPar] = {grads->means, grads->log_scales, grads->quats, grads->opacity_logits, grads->sh,
                                    grads->beta};
    for (int k = 0; k < ges::kNumPar; ++k) a.gin[k] = g[k];
  }
  return render_backward(splats, cams, num_views, params, splat_ws, key_ws, pixel_ws, dL_drgb, grads, &a, true,
                         stream);
}

ges_status ges_frame_view_get(int64_t n, int32_t width, int32_t height, void* splat_ws, void* key_ws, uint64_t num_keys,
                              void* pixel_ws, ges_frame_view* out) {
  return frame_view(n, 1, width, height, splat_ws, key_ws, num_keys, pixel_ws, 0, out);
}

ges_status ges_frame_view_get_views(int64_t n, int32_t num_views, int32_t width, int32_t height, void* splat_ws,
                                    void* key_ws, uint64_t num_keys, void* pixel_ws, int32_t view,
                                    ges_frame_view* out) {
  return frame_view(n, num_views, width, height, splat_ws, key_ws, num_keys, pixel_ws, view, out);
}

ges_status ges_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = on != 0;
  g_prof.mask = ~0u;
  return GES_OK;
}

ges_status ges_profile_select(uint32_t stage_mask) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = stage_mask != 0;
  g_prof.mask = stage_mask;
  return GES_OK;
}

ges_status ges_profile_read(double* ms, int64_t* launches, int32_t reset) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (auto& p : g_prof.pending) {
    GES_CHECK_HIP(hipEventSynchronize(p.b), "profile sync");
    float t = 0.f;
    GES_CHECK_HIP(hipEventElapsedTime(&t, p.a, p.b), "profile elapsed");
    g_prof.ms[p.stage] += t;
    g_prof.launches[p.stage] += 1;
    g_prof.free_events.push_back(p.a);
    g_prof.free_events.push_back(p.b);
  }
  g_prof.pending.clear();
  for (int k = 0; k < GES_NUM_STAGES; ++k) {
    if (ms) ms[k] = g_prof.ms[k];
    if (launches) launches[k] = g_prof.launches[k];
    if (reset) { g_prof.ms[k] = 0.0; g_prof.launches[k] = 0; }
  }
  return GES_OK;
}

size_t ges_mask_scratch_bytes(int32_t width, int32_t height) {
  if (width < 1 || height < 1) return 0;
  return ges::freq_mask_scratch_bytes(width, height);
}

ges_status ges_freq_mask(const float* target, int32_t width, int32_t height, float omega, void* scratch,
                         uint8_t* mask, void* stream) {
  if (!target || !scratch || !mask) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(GES_ERR_INVALID_ARGUMENT, "bad sizes");
  if (!(omega >= 0.f && omega <= 1.f)) return fail(GES_ERR_INVALID_ARGUMENT, "omega outside [0,1]");
  GES_CHECK_HIP(ges::launch_freq_mask(target, width, height, omega, scratch, mask, reinterpret_cast<hipStream_t>(stream)),
                "freq_mask");
  return GES_OK;
}

ges_status ges_freq_mask_static(const float* target, int32_t width, int32_t height, float omega, uint8_t* mask,
                                void* stream) {
  if (!target || !mask) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(GES_ERR_INVALID_ARGUMENT, "bad sizes");
  if (!(omega >= 0.f && omega <= 1.f)) return fail(GES_ERR_INVALID_ARGUMENT, "omega outside [0,1]");
  if (ges::freq_mask_scratch_bytes(width, height) > ges::freq_mask_static_capacity())
    return fail(GES_ERR_CAPACITY, "image too large for the library's mask scratch (GES_MASK_STATIC_SCRATCH_BYTES)");
  GES_CHECK_HIP(ges::launch_freq_mask_static(target, width, height, omega, mask, reinterpret_cast<hipStream_t>(stream)),
                "freq_mask_static");
  return GES_OK;
}

size_t ges_loss_scratch_bytes(void) { return ges::loss_scratch_bytes(); }

ges_status ges_loss(const float* img, const float* target, const uint8_t* mask, int32_t width, int32_t height,
                    float lam_l1, float lam_w, void* scratch, float* loss_out, float* dL_dimg, void* stream) {
  if (!img || !target || !scratch || !loss_out || !dL_dimg) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(GES_ERR_INVALID_ARGUMENT, "bad sizes");
  if (!std::isfinite(lam_l1) || !std::isfinite(lam_w)) return fail(GES_ERR_INVALID_ARGUMENT, "non-finite weight");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  GES_CHECK_HIP(timed(GES_STAGE_LOSS, st, [&] {
                  return ges::launch_loss(img, target, mask, width, height, lam_l1, mask ? lam_w : 0.f, scratch,
                                          loss_out, dL_dimg, st);
                }), "loss");
  return GES_OK;
}

size_t ges_ssim_scratch_bytes(int32_t width, int32_t height) {
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return 0;
  return ges::ssim_scratch_bytes(width, height);
}

ges_status ges_ssim_loss(const float* img, const float* target, int32_t width, int32_t height, float lam_ssim,
                         void* scratch, float* loss_inout, float* dL_dimg, void* stream) {
  if (!img || !target || !scratch || !loss_inout || !dL_dimg) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return fail(GES_ERR_INVALID_ARGUMENT, "bad sizes");
  if (!std::isfinite(lam_ssim)) return fail(GES_ERR_INVALID_ARGUMENT, "non-finite weight");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  GES_CHECK_HIP(timed(GES_STAGE_SSIM, st, [&] {
                  return ges::launch_ssim_loss(img, target, width, height, lam_ssim, scratch, loss_inout, dL_dimg, st);
                }), "ssim");
  return GES_OK;
}

ges_status ges_adam_step(const ges_adam_group* groups, int32_t ngroups, int64_t step, float beta1, float beta2,
                         float eps, void* stream) {
  if (!groups) return fail(GES_ERR_INVALID_ARGUMENT, "NULL groups");
  if (ngroups < 1 || ngroups > GES_ADAM_MAX_GROUPS) return fail(GES_ERR_INVALID_ARGUMENT, "ngroups outside 1..8");
  if (step < 1) return fail(GES_ERR_INVALID_ARGUMENT, "step < 1");
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
    return fail(GES_ERR_INVALID_ARGUMENT, "beta outside [0,1)");
  if (!(eps >= 0.f) || !std::isfinite(eps)) return fail(GES_ERR_INVALID_ARGUMENT, "bad eps");
  for (int k = 0; k < ngroups; ++k) {
    const ges_adam_group& g = groups[k];
    if (g.count < 0) return fail(GES_ERR_INVALID_ARGUMENT, "negative count");
    if (!(g.lr >= 0.f) || !std::isfinite(g.lr)) return fail(GES_ERR_INVALID_ARGUMENT, "bad lr");
    if (g.count > 0 && (!g.params || !g.grads || !g.exp_avg || !g.exp_avg_sq))
      return fail(GES_ERR_INVALID_ARGUMENT, "NULL array in a group");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  GES_CHECK_HIP(timed(GES_STAGE_ADAM, st, [&] { return ges::launch_adam(groups, ngroups, step, beta1, beta2, eps, st); }),
                "adam");
  return GES_OK;
}

size_t ges_prune_scratch_bytes(int64_t n) {
  if (n < 0 || n >= (int64_t(1) << 31)) return 0;
  return ges::prune_scratch_bytes(n);
}

ges_status ges_prune_splats(int64_t n, int32_t sh_degree, const ges_splat_set* src, const ges_splat_set* dst,
                            int32_t nsets, double min_opacity, double min_beta, void* scratch, size_t scratch_bytes,
                            int64_t* n_kept, void* stream) {
  if (!src || !dst || !scratch || !n_kept) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(GES_ERR_INVALID_ARGUMENT, "n outside [0, 2^31)");
  if (sh_degree < 0 || sh_degree > 3) return fail(GES_ERR_INVALID_ARGUMENT, "sh_degree outside 0..3");
  if (nsets < 1 || nsets > 3) return fail(GES_ERR_INVALID_ARGUMENT, "nsets outside 1..3");
  if (!(min_opacity >= 0.0 && min_opacity <= 1.0)) return fail(GES_ERR_INVALID_ARGUMENT, "min_opacity outside [0,1]");
  if (std::isnan(min_beta)) return fail(GES_ERR_INVALID_ARGUMENT, "min_beta is NaN");
  if (n > 0 && (!src[0].opacity_logits || !src[0].beta))
    return fail(GES_ERR_INVALID_ARGUMENT, "src[0] needs opacity_logits and beta");
  if (scratch_bytes < ges::prune_scratch_bytes(n)) return fail(GES_ERR_CAPACITY, "prune scratch too small");
  const int K = (sh_degree + 1) * (sh_degree + 1);
  const int32_t len[6] = {3, 3, 4, 1, 3 * K, 1};
  const float* s[ges::kMaxPruneArrays] = {};
  float* d[ges::kMaxPruneArrays] = {};
  int32_t rl[ges::kMaxPruneArrays] = {};
  for (int set = 0; set < nsets; ++set) {
    const float* sp[6] = {src[set].means, src[set].log_scales, src[set].quats, src[set].opacity_logits, src[set].sh,
                          src[set].beta};
    float* dp[6] = {dst[set].means, dst[set].log_scales, dst[set].quats, dst[set].opacity_logits, dst[set].sh,
                    dst[set].beta};
    for (int k = 0; k < 6; ++k) {
      if (!sp[k]) continue;
      if (!dp[k]) return fail(GES_ERR_INVALID_ARGUMENT, "NULL destination for a source array");
      s[6 * set + k] = sp[k];
      d[6 * set + k] = dp[k];
      rl[6 * set + k] = len[k];
    }
  }
  const double bound = min_opacity <= 0.0 ? -HUGE_VAL
                       : min_opacity >= 1.0 ? HUGE_VAL
                                            : std::log(min_opacity / (1.0 - min_opacity));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int64_t* total_dev = reinterpret_cast<int64_t*>(scratch);
  GES_CHECK_HIP(ges::launch_prune(s, d, rl, src[0].opacity_logits, src[0].beta, n, bound, min_beta, scratch, total_dev,
                                  st), "prune");
  int64_t kept = 0;
  GES_CHECK_HIP(hipMemcpyAsync(&kept, total_dev, sizeof(kept), hipMemcpyDeviceToHost, st), "read kept count");
  GES_CHECK_HIP(hipStreamSynchronize(st), "sync");
  *n_kept = kept;
  return GES_OK;
}

ges_status ges_shape_reset(float* beta, float* exp_avg, float* exp_avg_sq, int64_t n, float value, void* stream) {
  if (n < 0) return fail(GES_ERR_INVALID_ARGUMENT, "n < 0");
  if (n > 0 && !beta) return fail(GES_ERR_INVALID_ARGUMENT, "NULL beta");
  if (!std::isfinite(value)) return fail(GES_ERR_INVALID_ARGUMENT, "non-finite value");
  GES_CHECK_HIP(ges::launch_shape_reset(beta, exp_avg, exp_avg_sq, n, value, reinterpret_cast<hipStream_t>(stream)),
                "shape_reset");
  return GES_OK;
}

ges_status ges_mix_fit(const ges_mix_problem* problems, int32_t nproblems, const float* targets, int32_t ntargets,
                       int32_t m, float x0, float dx, float* params, float* grad_out, float* final_loss,
                       const int32_t* order, int32_t epochs, float lr, float beta1, float beta2, float eps,
                       void* stream) {
  if (nproblems < 0) return fail(GES_ERR_INVALID_ARGUMENT, "nproblems < 0");
  if (nproblems > 0 && (!problems || !targets || !params || !final_loss))
    return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if (m < 1 || m > GES_MIX_MAX_POINTS) return fail(GES_ERR_INVALID_ARGUMENT, "m outside 1..4096");
  if (ntargets < 1) return fail(GES_ERR_INVALID_ARGUMENT, "ntargets < 1");
  if (epochs < 0) return fail(GES_ERR_INVALID_ARGUMENT, "epochs < 0");
  if (!std::isfinite(x0) || !std::isfinite(dx) || !std::isfinite(lr) || !std::isfinite(eps) || lr < 0.f || eps < 0.f)
    return fail(GES_ERR_INVALID_ARGUMENT, "bad x0/dx/lr/eps");
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
    return fail(GES_ERR_INVALID_ARGUMENT, "beta outside [0,1)");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  GES_CHECK_HIP(timed(GES_STAGE_MIX_FIT, st, [&] {
                  return ges::launch_mix_fit(problems, nproblems, targets, ntargets, m, x0, dx, params, grad_out,
                                             final_loss, order, epochs, lr, beta1, beta2, eps, st);
                }), "mix_fit");
  return GES_OK;
}

size_t ges_densify_scratch_bytes(int64_t n) {
  if (n < 0 || n >= (int64_t(1) << 31)) return 0;
  return ges::densify_scratch_bytes(n);
}

ges_status ges_densify(int64_t n, int32_t sh_degree, const ges_splat_set* src, const ges_splat_set* dst,
                       int32_t nsets, int64_t dst_capacity, const float* grad_accum, const float* grad_count,
                       const float* normals, double grad_threshold, double scale_threshold, void* scratch,
                       size_t scratch_bytes, int64_t* n_out, void* stream) {
  if (!src || !dst || !scratch || !n_out) return fail(GES_ERR_INVALID_ARGUMENT, "NULL argument");
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(GES_ERR_INVALID_ARGUMENT, "n outside [0, 2^31)");
  if (sh_degree < 0 || sh_degree > 3) return fail(GES_ERR_INVALID_ARGUMENT, "sh_degree outside 0..3");
  if (nsets < 1 || nsets > 3) return fail(GES_ERR_INVALID_ARGUMENT, "nsets outside 1..3");
  if (!std::isfinite(grad_threshold) || !(scale_threshold > 0.0) || !std::isfinite(scale_threshold))
    return fail(GES_ERR_INVALID_ARGUMENT, "bad thresholds");
  if (n > 0 && (!grad_accum || !grad_count || !normals)) return fail(GES_ERR_INVALID_ARGUMENT, "NULL statistics");
  if (scratch_bytes < ges::densify_scratch_bytes(n)) return fail(GES_ERR_CAPACITY, "densify scratch too small");
  const int K = (sh_degree + 1) * (sh_degree + 1);
  const int32_t len[6] = {3, 3, 4, 1, 3 * K, 1};
  const float* s[ges::kMaxPruneArrays] = {};
  float* d[ges::kMaxPruneArrays] = {};
  int32_t rl[ges::kMaxPruneArrays] = {};
  for (int set = 0; set < nsets; ++set) {
    const float* sp[6] = {src[set].means, src[set].log_scales, src[set].quats, src[set].opacity_logits, src[set].sh,
                          src[set].beta};
    float* dp[6] = {dst[set].means, dst[set].log_scales, dst[set].quats, dst[set].opacity_logits, dst[set].sh,
                    dst[set].beta};
    for (int k = 0; k < 6; ++k) {
      if (!sp[k]) {
        if (set == 0 && n > 0) return fail(GES_ERR_INVALID_ARGUMENT, "set 0 needs all six parameter arrays");
        continue;
      }
      if (!dp[k]) return fail(GES_ERR_INVALID_ARGUMENT, "NULL destination for a source array");
      s[6 * set + k] = sp[k];
      d[6 * set + k] = dp[k];
      rl[6 * set + k] = len[k];
    }
  }
  const double lbound = std::log(scale_threshold);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  GES_CHECK_HIP(ges::launch_densify_count(grad_accum, grad_count, src[0].log_scales, n, grad_threshold, lbound, scratch,
                                          st), "densify count");
  int64_t tot[3] = {0, 0, 0};
  GES_CHECK_HIP(hipMemcpyAsync(tot, scratch, sizeof(tot), hipMemcpyDeviceToHost, st), "read densify counts");
  GES_CHECK_HIP(hipStreamSynchronize(st), "sync");
  *n_out = tot[0] + tot[1] + 2 * tot[2];
  if (*n_out > dst_capacity) return fail(GES_ERR_CAPACITY, "densified set exceeds dst_capacity");
  if (*n_out >= (int64_t(1) << 31)) return fail(GES_ERR_CAPACITY, "densified set exceeds 2^31 splats");
  GES_CHECK_HIP(ges::launch_densify_scatter(s, d, rl, nsets, grad_accum, grad_count, normals, n, grad_threshold, lbound,
                                            std::log(1.6), tot[0], tot[1], scratch, st), "densify scatter");
  return GES_OK;
}

ges_status ges_opacity_reset(float* opacity_logits, float* exp_avg, float* exp_avg_sq, int64_t n, double max_opacity,
                             void* stream) {
  if (n < 0) return fail(GES_ERR_INVALID_ARGUMENT, "n < 0");
  if (n > 0 && !opacity_logits) return fail(GES_ERR_INVALID_ARGUMENT, "NULL opacity_logits");
  if (!(max_opacity > 0.0 && max_opacity < 1.0)) return fail(GES_ERR_INVALID_ARGUMENT, "max_opacity outside (0,1)");
  GES_CHECK_HIP(ges::launch_opacity_reset(opacity_logits, exp_avg, exp_avg_sq, n,
                                          std::log(max_opacity / (1.0 - max_opacity)),
                                          reinterpret_cast<hipStream_t>(stream)), "opacity_reset");
  return GES_OK;
}

double ges_expon_lr(int64_t step, double lr_init, double lr_final, int64_t max_steps, int64_t delay_steps,
                    double delay_mult) {
  if (!(lr_init > 0.0) || !(lr_final > 0.0) || max_steps < 1) return std::nan("");
  const double tau = std::min(std::max((double)step / (double)max_steps, 0.0), 1.0);
  double lr = lr_init == lr_final ? lr_init : std::exp((1.0 - tau) * std::log(lr_init) + tau * std::log(lr_final));
  if (delay_steps > 0) {
    const double r = std::min(std::max((double)step / (double)delay_steps, 0.0), 1.0);
    lr *= delay_mult + (1.0 - delay_mult) * std::sin(0.5 * M_PI * r);
  }
  return lr;
}

ges_status ges_loss_schedule(int64_t iteration, int64_t total_iterations, float lam_ssim, float lam_omega,
                             float* omega, float* lam_l1) {
  if (total_iterations < 1) return fail(GES_ERR_INVALID_ARGUMENT, "total_iterations < 1");
  if (!std::isfinite(lam_ssim) || !std::isfinite(lam_omega)) return fail(GES_ERR_INVALID_ARGUMENT, "non-finite weight");
  if (omega) *omega = (float)std::min(std::max((double)iteration / (double)total_iterations, 0.0), 1.0);
  if (lam_l1) *lam_l1 = (float)(1.0 - (double)lam_ssim - (double)lam_omega);
  return GES_OK;
}

}  // extern "C"
