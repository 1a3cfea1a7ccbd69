// serve.cpp -- continuous-batching render server over resident scenes.
//
// Requests (scene, camera, caller-owned output image) are queued by ges_serve_submit and rendered by
// one server thread.  The thread repeatedly
//   1. admits queued requests in arrival order into a batch of up to max_slots views, each holding
//      an exact reservation for its per-splat and per-tile workspace carved out of the caller's pool
//      (a request is admitted only while the reservation fits the pool: the HBM budget);
//   2. enqueues, on one of two streams, the preprocess, tile histogram and tile scan of every view of
//      the batch as single launches over all views, then reads back the key count of the batch (the
//      only host synchronisation of a batch);
//   3. reserves the batch's key buffer (if it does not fit, it waits for older batches to retire and
//      finally hands back the newest views to the queue), and enqueues the scatter, per-tile sort and
//      forward raster of all views as single launches;
//   4. records a completion event and goes back to 1 without waiting, so the preprocess of batch n+1
//      overlaps the raster of batch n on the other stream; at most two batches are in flight.
// Completed batches release their reservations; requests arriving meanwhile join the next batch.
// A request's image does not depend on the other views of its batch: every stage is per view except
// the key-position scan, which only shifts where a view's keys live.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "frame.h"
#include "ges_internal.h"

namespace ges {
namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, size) with coalescing; offsets aligned to 256 bytes.
class PoolAllocator {
 public:
  explicit PoolAllocator(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(std::max<size_t>(bytes, 1));
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t id = 0;
  int32_t scene = 0;
  ges_camera cam{};
  float* out = nullptr;
  int32_t state = GES_REQ_QUEUED;
  int32_t status = GES_OK;
  uint64_t t_submit = 0, t_start = 0, t_done = 0, num_keys = 0;
  int32_t batch_size = 0;
  size_t ws_off = 0, ws_bytes = 0;
  char* inspect = nullptr;        // device buffer receiving copies of the view's frame arrays (tests)
  size_t inspect_bytes = 0;
};

struct BatchWork {
  std::vector<uint64_t> ids;
  std::vector<FramePlan> plans;
  size_t table_off = 0, table_bytes = 0;     // device view table, then the batch's binning buffers
  int64_t items = 0;                         // splats of the batch's views
  size_t key_off = 0, key_bytes = 0;
  bool has_keys = false;
  uint64_t keys = 0;
  int stream = 0;
  hipEvent_t done = nullptr;
  std::unique_ptr<DeviceBatch> host;         // kept alive until the batch retires
  std::vector<std::pair<char*, size_t>> inspect;   // per view: inspection buffer (may be null) and its size
  uint64_t sim_done_ns = 0;
};

int64_t batch_tiles(const BatchWork& b) { return b.host ? b.host->tile_prefix[b.host->nviews] : 0; }

}  // namespace

// ---- executors: the GPU one, and a simulated one for host-only tests of the scheduler ------------
struct Executor {
  virtual ~Executor() = default;
  // Enqueue preprocess + histogram + scan for every view; return the batch key count (waits).
  virtual ges_status count(BatchWork& b, char* pool, std::string& err) = 0;
  // Enqueue scatter + sort + raster and a completion marker.
  virtual ges_status render(BatchWork& b, char* pool, std::string& err) = 0;
  virtual bool done(BatchWork& b) = 0;
  virtual void wait(BatchWork& b) = 0;
  virtual void release(BatchWork& b) = 0;
};

}  // namespace ges

struct ges_server {
  ges_serve_config cfg{};
  ges_raster_params params{};
  char* pool = nullptr;
  std::unique_ptr<ges::PoolAllocator> alloc;
  std::unique_ptr<ges::Executor> exec;
  std::vector<ges_splats> scenes;
  std::mutex mu;
  std::condition_variable cv;      // wakes the worker (new work / stop)
  std::condition_variable cv_done; // wakes drain()
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, ges::Request> reqs;
  std::list<ges::BatchWork> inflight;
  uint64_t next_id = 1;
  uint64_t unfinished = 0;
  bool stop = false;
  std::thread worker;
};

namespace ges {
namespace {

bool finished_state(int32_t s) {
  return s == GES_REQ_DONE || s == GES_REQ_FAILED || s == GES_REQ_REJECTED || s == GES_REQ_CANCELLED;
}

// Inspection buffer of a served request: the view's records, tile ranges (positions in the batch's sorted
// ids), n_contrib and header, then the batch's sorted ids; every part 256-byte aligned.
struct ServeInspectLayout { size_t off_records, off_ranges, off_n_contrib, off_header, off_ids, bytes; };
ServeInspectLayout serve_inspect_layout(int64_t n, int32_t w, int32_t h, uint64_t batch_keys) {
  ServeInspectLayout L{};
  const size_t tiles = (size_t)((w + kTile - 1) / kTile) * (size_t)((h + kTile - 1) / kTile);
  L.off_records = 0;
  L.off_ranges = align256(64 * (size_t)n);
  L.off_n_contrib = L.off_ranges + align256(8 * tiles);
  L.off_header = L.off_n_contrib + align256(4 * (size_t)w * (size_t)h);
  L.off_ids = L.off_header + 256;
  L.bytes = L.off_ids + align256(8 * (size_t)batch_keys);
  return L;
}

size_t request_bytes(const ges_splats& sc, const ges_camera& c) {
  FramePlan fp = plan_frame(sc.n, c.width, c.height);
  // the view table and the binning buffers live in the batch; the per-view device batch slot is not needed
  return fp.view_bytes - align256(sizeof(DeviceBatch));
}

size_t table_bytes() { return align256(device_batch_bytes(kMaxViews)); }

// The batch's binning buffers follow its view table.
SortWs batch_sort_ws(char* pool, const BatchWork& b) {
  return attach_sort_ws(plan_sort(b.items), pool + b.table_off + table_bytes());
}

// Per-view splat workspace: the plan's layout minus the leading view-table slot.
void attach_view(ViewDesc& V, const FramePlan& fp, char* ws) {
  attach_splat_ws(V, fp, ws - align256(sizeof(DeviceBatch)));
}

class GpuExecutor : public Executor {
 public:
  GpuExecutor() {
    for (int k = 0; k < 2; ++k) {
      if (hipStreamCreateWithFlags(&streams_[k], hipStreamNonBlocking) != hipSuccess) streams_[k] = nullptr;
    }
  }
  ~GpuExecutor() override {
    for (auto s : streams_)
      if (s) (void)hipStreamDestroy(s);
  }
  bool ok() const { return streams_[0] && streams_[1]; }

  ges_status count(BatchWork& b, char* pool, std::string& err) override {
    hipStream_t st = streams_[b.stream];
    DeviceBatch* db = reinterpret_cast<DeviceBatch*>(pool + b.table_off);
    Batch bt = make_batch(b, pool);
    hipError_t e = hipMemcpyAsync(db, b.host.get(), device_batch_bytes(bt.nviews), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_preprocess(db, bt, st);
    if (e == hipSuccess) e = launch_depth_sort(db, bt, st);
    if (e == hipSuccess) e = launch_key_scan(db, bt, st);
    uint32_t k = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&k, bt.keys_total, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { err = hipGetErrorString(e); return GES_ERR_DEVICE; }
    if (k == 0xffffffffu) { err = "more than 2^32-2 candidate pairs in one batch"; return GES_ERR_CAPACITY; }
    b.keys = k;
    return GES_OK;
  }

  ges_status render(BatchWork& b, char* pool, std::string& err) override {
    hipStream_t st = streams_[b.stream];
    const DeviceBatch* db = reinterpret_cast<const DeviceBatch*>(pool + b.table_off);
    Batch bt = make_batch(b, pool);
    hipError_t e = launch_duplicate(db, bt, st);
    if (e == hipSuccess) e = launch_tile_sort(db, bt, st);
    if (e == hipSuccess) e = launch_raster_forward(db, bt, st);
    for (int v = 0; v < bt.nviews && e == hipSuccess; ++v) {
      if (!b.inspect[(size_t)v].first) continue;
      const ViewDesc& V = b.host->views[v];
      const ServeInspectLayout L = serve_inspect_layout(V.n, V.width, V.height, b.keys);
      char* dst = b.inspect[(size_t)v].first;
      const int64_t tiles = (int64_t)V.tiles_x * V.tiles_y;
      if (V.n > 0) e = hipMemcpyAsync(dst + L.off_records, V.rec, 64 * (size_t)V.n, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(dst + L.off_ranges, V.ranges, 8 * (size_t)tiles, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(dst + L.off_header, V.header, 32, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess && b.keys > 0 && L.bytes <= b.inspect[(size_t)v].second)
        e = hipMemcpyAsync(dst + L.off_ids, bt.sorted_pairs, 8 * (size_t)b.keys, hipMemcpyDeviceToDevice, st);
    }
    if (e == hipSuccess && !b.done) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(b.done, st);
    if (e != hipSuccess) { err = hipGetErrorString(e); return GES_ERR_DEVICE; }
    return GES_OK;
  }

  bool done(BatchWork& b) override { return !b.done || hipEventQuery(b.done) == hipSuccess; }
  void wait(BatchWork& b) override {
    if (b.done) (void)hipEventSynchronize(b.done);
  }
  void release(BatchWork& b) override {
    if (b.done) (void)hipEventDestroy(b.done);
    b.done = nullptr;
  }

 private:
  Batch make_batch(const BatchWork& b, char* pool) {
    Batch bt{};
    const DeviceBatch& h = *b.host;
    bt.nviews = h.nviews;
    bt.falloff = h.views[0].falloff;
    bt.tile_cull = h.views[0].tile_cull;
    bt.total_tiles = h.tile_prefix[h.nviews];
    bt.pre_blocks = h.pre_prefix[h.nviews];
    bt.items = h.item_prefix[h.nviews];
    bt.sw = batch_sort_ws(pool, b);
    bt.keys_total = &bt.sw.cells[1];
    bt.tile_passes = tile_passes(bt.total_tiles);
    bt.dup_buffer = bt.tile_passes & 1;
    if (b.has_keys && b.keys > 0) {
      bt.kw = attach_key_ws(plan_keys(b.keys, false), pool + b.key_off);
      bt.sorted_pairs = bt.kw.pv[0];
      bt.sorted_tiles = bt.kw.key[0];
      bt.key_capacity = b.keys;
    }
    return bt;
  }
  hipStream_t streams_[2] = {nullptr, nullptr};
};

// Host-only executor: key count = the sum over views of `keys_per_view`, a batch takes
// `batch_ns` plus `per_view_ns` per view; scenes whose id is `fail_scene` fail at count time.
class SimExecutor : public Executor {
 public:
  SimExecutor(uint64_t keys_per_view, uint64_t batch_ns, uint64_t per_view_ns, int32_t fail_scene,
              const std::vector<ges_splats>* scenes, std::unordered_map<uint64_t, Request>* reqs)
      : kpv_(keys_per_view), bns_(batch_ns), vns_(per_view_ns), fail_(fail_scene), reqs_(reqs) {
    (void)scenes;
  }
  ges_status count(BatchWork& b, char*, std::string& err) override {
    for (uint64_t id : b.ids)
      if (reqs_->at(id).scene == fail_) { err = "simulated executor failure"; return GES_ERR_DEVICE; }
    b.keys = kpv_ * b.ids.size();
    return GES_OK;
  }
  ges_status render(BatchWork& b, char*, std::string&) override {
    b.sim_done_ns = now_ns() + bns_ + vns_ * b.ids.size();
    return GES_OK;
  }
  bool done(BatchWork& b) override { return now_ns() >= b.sim_done_ns; }
  void wait(BatchWork& b) override {
    while (!done(b)) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  void release(BatchWork&) override {}

 private:
  uint64_t kpv_, bns_, vns_;
  int32_t fail_;
  std::unordered_map<uint64_t, Request>* reqs_;
};

void finish_request(ges_server* s, Request& r, int32_t state, int32_t status) {
  r.state = state;
  r.status = status;
  r.t_done = now_ns();
  if (r.ws_bytes) {
    s->alloc->release(r.ws_off, r.ws_bytes);
    r.ws_bytes = 0;
  }
  if (s->unfinished) --s->unfinished;
}

// Retire completed in-flight batches (lock held).  wait_oldest: block on the oldest one first.
void retire(ges_server* s, std::unique_lock<std::mutex>& lk, bool wait_oldest) {
  if (wait_oldest && !s->inflight.empty()) {
    BatchWork& b = s->inflight.front();
    lk.unlock();
    s->exec->wait(b);
    lk.lock();
  }
  bool any = false;
  for (auto it = s->inflight.begin(); it != s->inflight.end();) {
    if (!s->exec->done(*it)) { ++it; continue; }
    for (uint64_t id : it->ids) finish_request(s, s->reqs.at(id), GES_REQ_DONE, GES_OK);
    if (it->has_keys) s->alloc->release(it->key_off, it->key_bytes);
    s->alloc->release(it->table_off, it->table_bytes);
    s->exec->release(*it);
    it = s->inflight.erase(it);
    any = true;
  }
  if (any) s->cv_done.notify_all();
}

void build_views(ges_server* s, BatchWork& b) {
  b.host.reset(new DeviceBatch());
  DeviceBatch& h = *b.host;
  std::memset(&h, 0, offsetof(DeviceBatch, views));
  h.nviews = (int32_t)b.ids.size();
  b.plans.clear();
  b.inspect.clear();
  int64_t pre = 0, items = 0, tiles = 0;
  b.items = 0;
  for (uint64_t id : b.ids) b.items += s->scenes[(size_t)s->reqs.at(id).scene].n;
  const SortWs sw = batch_sort_ws(s->pool, b);
  for (size_t v = 0; v < b.ids.size(); ++v) {
    const Request& r = s->reqs.at(b.ids[v]);
    const ges_splats& sc = s->scenes[(size_t)r.scene];
    const FramePlan fp = plan_frame(sc.n, r.cam.width, r.cam.height);
    b.plans.push_back(fp);
    ViewDesc& V = h.views[v];
    fill_view(V, &sc, &r.cam, &s->params);
    attach_view(V, fp, s->pool + r.ws_off);
    V.out_rgb = r.out;
    b.inspect.emplace_back(r.inspect, r.inspect_bytes);
    // an inspected request's raster writes its n_contrib straight into the inspection buffer
    if (r.inspect)
      V.n_contrib = reinterpret_cast<uint32_t*>(
          r.inspect + serve_inspect_layout(sc.n, r.cam.width, r.cam.height, 0).off_n_contrib);
    V.item_key = sw.item_key + items;
    V.item_cand = sw.item_cand + items;
    h.pre_prefix[v] = pre;
    h.item_prefix[v] = items;
    h.tile_prefix[v] = tiles;
    pre += (sc.n + 255) / 256;
    items += sc.n;
    tiles += fp.tiles;
  }
  h.pre_prefix[b.ids.size()] = pre;
  h.item_prefix[b.ids.size()] = items;
  h.tile_prefix[b.ids.size()] = tiles;
}

void worker_loop(ges_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  int next_stream = 0;
  for (;;) {
    retire(s, lk, false);
    if (s->stop && s->queue.empty() && s->inflight.empty()) break;
    if (s->queue.empty()) {
      if (!s->inflight.empty()) {
        // poll completions while staying responsive to new arrivals
        s->cv.wait_for(lk, std::chrono::microseconds(50));
      } else {
        s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      }
      continue;
    }
    if (s->inflight.size() >= 2) { retire(s, lk, true); continue; }
    // ---- 1. admission under the pool budget
    BatchWork b;
    const int slots = s->cfg.sequential ? 1 : std::max(1, std::min(s->cfg.max_slots, (int32_t)kMaxViews));
    int64_t items = 0;
    while (!s->queue.empty() && (int)b.ids.size() < slots) {
      Request& r = s->reqs.at(s->queue.front());
      const size_t need = request_bytes(s->scenes[(size_t)r.scene], r.cam);
      size_t off = 0;
      if (!s->alloc->alloc(need, &off)) break;
      r.ws_off = off;
      r.ws_bytes = need;
      r.state = GES_REQ_RUNNING;
      r.t_start = now_ns();
      b.ids.push_back(r.id);
      items += s->scenes[(size_t)r.scene].n;
      s->queue.pop_front();
    }
    // the view table and the binning buffers of the batch; without room, give back the newest views
    while (!b.ids.empty()) {
      const size_t tb = table_bytes() + plan_sort(items).bytes;
      if (s->alloc->alloc(tb, &b.table_off)) { b.table_bytes = tb; break; }
      const uint64_t id = b.ids.back();
      b.ids.pop_back();
      Request& r = s->reqs.at(id);
      s->alloc->release(r.ws_off, r.ws_bytes);
      r.ws_bytes = 0;
      r.state = GES_REQ_QUEUED;
      items -= s->scenes[(size_t)r.scene].n;
      s->queue.push_front(id);
    }
    if (b.ids.empty()) {
      if (!s->inflight.empty()) retire(s, lk, true);
      else {   // the head request cannot fit even in an idle pool
        Request& r = s->reqs.at(s->queue.front());
        s->queue.pop_front();
        finish_request(s, r, GES_REQ_FAILED, GES_ERR_OUT_OF_MEMORY);
        s->cv_done.notify_all();
      }
      continue;
    }
    build_views(s, b);
    b.stream = next_stream;
    next_stream ^= 1;
    // ---- 2. preprocess + counts (the device work runs without the lock)
    std::string err;
    lk.unlock();
    ges_status st = s->exec->count(b, s->pool, err);
    lk.lock();
    if (st != GES_OK) {
      for (uint64_t id : b.ids) finish_request(s, s->reqs.at(id), GES_REQ_FAILED, st);
      s->alloc->release(b.table_off, b.table_bytes);
      s->cv_done.notify_all();
      continue;
    }
    // ---- 3. key buffer under the budget: wait for older batches, then give back the newest views
    bool placed = false;
    for (;;) {
      const size_t kb = plan_keys(b.keys, false).bytes;
      if (b.keys == 0 || s->alloc->alloc(kb, &b.key_off)) {
        b.key_bytes = kb;
        b.has_keys = b.keys > 0;
        placed = true;
        break;
      }
      if (!s->inflight.empty()) { retire(s, lk, true); continue; }
      if (b.ids.size() > 1) {
        // hand the newest view back to the head of the queue and recount the rest
        const uint64_t id = b.ids.back();
        b.ids.pop_back();
        Request& r = s->reqs.at(id);
        s->alloc->release(r.ws_off, r.ws_bytes);
        r.ws_bytes = 0;
        r.state = GES_REQ_QUEUED;
        s->queue.push_front(id);
        build_views(s, b);
        lk.unlock();
        st = s->exec->count(b, s->pool, err);
        lk.lock();
        if (st != GES_OK) break;
        continue;
      }
      st = GES_ERR_OUT_OF_MEMORY;
      break;
    }
    if (!placed) {
      for (uint64_t id : b.ids) finish_request(s, s->reqs.at(id), GES_REQ_FAILED, st);
      s->alloc->release(b.table_off, b.table_bytes);
      s->cv_done.notify_all();
      continue;
    }
    // ---- 4. render, record completion, keep going
    for (size_t v = 0; v < b.ids.size(); ++v) {
      Request& r = s->reqs.at(b.ids[v]);
      r.batch_size = (int32_t)b.ids.size();
    }
    lk.unlock();
    st = s->exec->render(b, s->pool, err);
    lk.lock();
    if (st != GES_OK) {
      s->exec->wait(b);
      for (uint64_t id : b.ids) finish_request(s, s->reqs.at(id), GES_REQ_FAILED, st);
      if (b.has_keys) s->alloc->release(b.key_off, b.key_bytes);
      s->alloc->release(b.table_off, b.table_bytes);
      s->exec->release(b);
      s->cv_done.notify_all();
      continue;
    }
    // per-view key counts are known on the device; record the batch total for every request
    for (uint64_t id : b.ids) s->reqs.at(id).num_keys = b.keys;
    s->inflight.push_back(std::move(b));
  }
  s->cv_done.notify_all();
}

ges_status validate_config(const ges_serve_config* c) {
  if (!c) return GES_ERR_INVALID_ARGUMENT;
  if (c->max_slots < 1 || c->max_slots > kMaxViews || c->queue_capacity < 1) return GES_ERR_INVALID_ARGUMENT;
  ges_raster_params p{c->falloff, c->tile_cull, c->rho, {c->bg[0], c->bg[1], c->bg[2]}};
  if (!check_params(&p).empty()) return GES_ERR_INVALID_ARGUMENT;
  return GES_OK;
}

ges_status start(ges_server* s, const ges_serve_config* cfg, void* pool, size_t pool_bytes) {
  s->cfg = *cfg;
  s->params = ges_raster_params{cfg->falloff, cfg->tile_cull, cfg->rho, {cfg->bg[0], cfg->bg[1], cfg->bg[2]}};
  s->pool = reinterpret_cast<char*>(pool);
  s->alloc.reset(new PoolAllocator(pool_bytes));
  s->worker = std::thread(worker_loop, s);
  return GES_OK;
}

}  // namespace
}  // namespace ges

extern "C" {

ges_status ges_serve_create(const ges_serve_config* cfg, void* pool, size_t pool_bytes, ges_server** out) {
  if (!out || !pool || pool_bytes == 0 || ges::validate_config(cfg) != GES_OK) return GES_ERR_INVALID_ARGUMENT;
  std::unique_ptr<ges_server> s(new ges_server());
  std::unique_ptr<ges::GpuExecutor> ex(new ges::GpuExecutor());
  if (!ex->ok()) return GES_ERR_DEVICE;
  s->exec = std::move(ex);
  ges::start(s.get(), cfg, pool, pool_bytes);
  *out = s.release();
  return GES_OK;
}

ges_status ges_serve_create_simulated(const ges_serve_config* cfg, size_t pool_bytes, uint64_t keys_per_view,
                                      uint64_t batch_ns, uint64_t per_view_ns, int32_t fail_scene, ges_server** out) {
  if (!out || pool_bytes == 0 || ges::validate_config(cfg) != GES_OK) return GES_ERR_INVALID_ARGUMENT;
  std::unique_ptr<ges_server> s(new ges_server());
  s->exec.reset(new ges::SimExecutor(keys_per_view, batch_ns, per_view_ns, fail_scene, &s->scenes, &s->reqs));
  // the simulated pool is never dereferenced: only offsets are handed out
  ges::start(s.get(), cfg, reinterpret_cast<void*>(uintptr_t(1) << 40), pool_bytes);
  *out = s.release();
  return GES_OK;
}

ges_status ges_serve_add_scene(ges_server* s, const ges_splats* scene, int32_t* scene_id) {
  if (!s || !scene || !scene_id) return GES_ERR_INVALID_ARGUMENT;
  if (!ges::check_splats(scene).empty()) return GES_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(s->mu);
  s->scenes.push_back(*scene);
  *scene_id = (int32_t)s->scenes.size() - 1;
  return GES_OK;
}

ges_status ges_serve_submit(ges_server* s, int32_t scene_id, const ges_camera* cam, float* out_rgb_device,
                            uint64_t* request_id) {
  return ges_serve_submit_inspect(s, scene_id, cam, out_rgb_device, nullptr, 0, request_id);
}

size_t ges_serve_inspect_bytes(int64_t n, int32_t width, int32_t height, uint64_t batch_keys) {
  if (n < 0 || width < 1 || height < 1) return 0;
  return ges::serve_inspect_layout(n, width, height, batch_keys).bytes;
}

ges_status ges_serve_submit_inspect(ges_server* s, int32_t scene_id, const ges_camera* cam, float* out_rgb_device,
                                    void* inspect_device, size_t inspect_bytes, uint64_t* request_id) {
  if (!s || !cam || !out_rgb_device || !request_id) return GES_ERR_INVALID_ARGUMENT;
  if (inspect_device && (reinterpret_cast<uintptr_t>(inspect_device) % 256 != 0)) return GES_ERR_INVALID_ARGUMENT;
  if (!ges::check_camera(cam).empty()) return GES_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return GES_ERR_INVALID_ARGUMENT;
  if (scene_id < 0 || scene_id >= (int32_t)s->scenes.size()) return GES_ERR_NOT_FOUND;
  if ((int64_t)s->queue.size() >= s->cfg.queue_capacity) return GES_ERR_BUSY;
  ges::Request r;
  r.id = s->next_id++;
  r.scene = scene_id;
  r.cam = *cam;
  r.out = out_rgb_device;
  r.t_submit = ges::now_ns();
  if (inspect_device) {
    const ges_splats& sc = s->scenes[(size_t)scene_id];
    if (inspect_bytes < ges::serve_inspect_layout(sc.n, cam->width, cam->height, 0).bytes)
      return GES_ERR_CAPACITY;
    r.inspect = reinterpret_cast<char*>(inspect_device);
    r.inspect_bytes = inspect_bytes;
  }
  const size_t need = ges::request_bytes(s->scenes[(size_t)scene_id], *cam) + ges::table_bytes() +
                      ges::plan_sort(s->scenes[(size_t)scene_id].n).bytes;
  *request_id = r.id;
  if (need > s->alloc->size()) {
    // can never be admitted: reject at once
    r.state = GES_REQ_REJECTED;
    r.status = GES_ERR_OUT_OF_MEMORY;
    r.t_done = r.t_submit;
    s->reqs.emplace(r.id, r);
    return GES_OK;
  }
  s->reqs.emplace(r.id, r);
  s->queue.push_back(r.id);
  ++s->unfinished;
  s->cv.notify_one();
  return GES_OK;
}

ges_status ges_serve_poll(ges_server* s, uint64_t request_id, ges_request_info* info) {
  if (!s || !info) return GES_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(request_id);
  if (it == s->reqs.end()) return GES_ERR_NOT_FOUND;
  const ges::Request& r = it->second;
  info->state = r.state;
  info->status = r.status;
  info->t_submit_ns = r.t_submit;
  info->t_start_ns = r.t_start;
  info->t_done_ns = r.t_done;
  info->num_keys = r.num_keys;
  info->batch_size = r.batch_size;
  return GES_OK;
}

ges_status ges_serve_drain(ges_server* s) {
  if (!s) return GES_ERR_INVALID_ARGUMENT;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.notify_one();
  s->cv_done.wait(lk, [&] { return s->unfinished == 0; });
  return GES_OK;
}

ges_status ges_serve_destroy(ges_server* s) {
  if (!s) return GES_ERR_INVALID_ARGUMENT;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // queued requests are cancelled; batches already on the device complete
    for (uint64_t id : s->queue) ges::finish_request(s, s->reqs.at(id), GES_REQ_CANCELLED, GES_OK);
    s->queue.clear();
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  delete s;
  return GES_OK;
}

}  // extern "C"
