// Serving loop for DRK rendering requests (continuous batching on one GPU).
//
// Scenes are copied once into server-owned device memory.  Requests (scene, camera, output) are
// queued by drk_serve_submit and admitted in arrival order by a scheduler thread whenever an
// in-flight slot is free and the request's workspace fits the HBM budget.  Each admitted request
// runs on its own non-blocking stream, so work of different requests (scenes, resolutions)
// overlaps on the device.  Workspaces stay resident per (scene, width, height) and are reused by
// later requests; their preprocess -> bin/sort -> raster sequence is captured once in a HIP graph
// (the camera lives in device memory written by a one-thread kernel before each replay, so the
// graph is camera-independent).  Idle workspaces are evicted least-recently-used when a new one
// does not fit.  A request whose pairs overflow its workspace is retried with a larger one.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "drk_internal.hpp"

namespace drk {
void ws_status_ptrs(drk_ws* ws, uint32_t** status, uint64_t** totals);
}

using namespace drk;

namespace {

double now_us() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec * 1e6 + ts.tv_nsec * 1e-3;
}

struct ResidentScene {
  drk_scene sc{};
  void* mem = nullptr;
  size_t bytes = 0;
};

struct WsEntry {
  drk_ws* ws = nullptr;
  int scene = -1, W = 0, H = 0;
  int64_t cap = 0;
  size_t bytes = 0;
  hipGraphExec_t exec = nullptr;
  bool busy = false;
  uint64_t last_use = 0;
};

struct Request {
  uint64_t id = 0;
  int scene = 0;
  drk_camera cam{};
  float* out = nullptr;
  double submit_us = 0, start_us = 0, done_us = 0;
  int64_t pairs = 0;
  int status = DRK_OK;
  bool done = false;
  int retries = 0;
  int bypassed = 0;                // times a later request was admitted while this one waited
  WsEntry* ws = nullptr;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  Request* req = nullptr;
  uint32_t* h_status = nullptr;   // pinned: status word and pair total copied after each request
  uint64_t* h_total = nullptr;
};

using Key = std::tuple<int, int, int>;

}  // namespace

struct drk_server {
  int device = 0;
  drk_serve_cfg cfg{};
  int64_t budget = 0;
  std::vector<ResidentScene> scenes;
  std::list<WsEntry*> pool;
  size_t ws_bytes = 0;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> reqs;
  std::vector<Slot> slots;
  std::map<Key, int64_t> learned_cap;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::thread sched;
  bool stop = false;
  uint64_t next_id = 1, tick = 0;
  int inflight = 0;
};

namespace {

int64_t initial_capacity(const drk_server* s, int scene, int W, int H) {
  auto it = s->learned_cap.find(Key(scene, W, H));
  if (it != s->learned_cap.end()) return it->second;
  if (s->cfg.initial_pairs > 0) return s->cfg.initial_pairs;
  const int64_t n = s->scenes[scene].sc.n;
  int64_t c = 4 * n + 4 * (int64_t)W * H;
  return std::max<int64_t>(c, 1 << 16);
}

size_t ws_size(const drk_server* s, int scene, int W, int H, int64_t cap) {
  size_t b = 0;
  const drk_scene& sc = s->scenes[scene].sc;
  if (drk_ws_size_query(std::max<int64_t>(sc.n, 1), sc.K, 1, W, H, cap, &b) != DRK_OK) return (size_t)-1;
  return b;
}

void drop_entry(drk_server* s, WsEntry* e) {
  if (e->exec) hipGraphExecDestroy(e->exec);
  drk_ws_destroy(e->ws);
  s->ws_bytes -= e->bytes;
  s->pool.remove(e);
  delete e;
}

// Finds an idle resident workspace for the request or creates one within the budget (evicting idle
// ones, least recently used first).  Returns null when it cannot be admitted now; *never is then set
// (with the error in *why) when it cannot be admitted at all: its workspace size is invalid or
// exceeds the whole budget, or creating it fails while no other workspace is busy (nothing that
// could free memory is running).
WsEntry* acquire(drk_server* s, Request* r, bool* never, int* why) {
  *never = false;
  const int W = r->cam.width, H = r->cam.height;
  for (WsEntry* e : s->pool)
    if (!e->busy && e->scene == r->scene && e->W == W && e->H == H) {
      e->busy = true;
      return e;
    }
  const int64_t cap = initial_capacity(s, r->scene, W, H);
  const size_t need = ws_size(s, r->scene, W, H, cap);
  if (need == (size_t)-1) {
    *never = true;
    *why = DRK_EINVAL;
    return nullptr;
  }
  if (need > (size_t)s->budget) {
    *never = true;
    *why = DRK_ENOMEM;
    return nullptr;
  }
  size_t idle = 0;
  for (WsEntry* e : s->pool)
    if (!e->busy) idle += e->bytes;
  if (s->ws_bytes - idle + need > (size_t)s->budget) return nullptr;   // not even after evicting every idle one
  while (s->ws_bytes + need > (size_t)s->budget) {
    WsEntry* victim = nullptr;
    for (WsEntry* e : s->pool)
      if (!e->busy && (!victim || e->last_use < victim->last_use)) victim = e;
    if (!victim) return nullptr;
    drop_entry(s, victim);
  }
  const drk_scene& sc = s->scenes[r->scene].sc;
  drk_ws* ws = nullptr;
  if (drk_ws_create(std::max<int64_t>(sc.n, 1), sc.K, 1, W, H, cap, &ws) != DRK_OK) {
    bool any_busy = false;
    for (WsEntry* e : s->pool) any_busy = any_busy || e->busy;
    if (!any_busy) {
      // free what is idle and try once more before giving up on the request
      while (!s->pool.empty()) drop_entry(s, s->pool.front());
      if (drk_ws_create(std::max<int64_t>(sc.n, 1), sc.K, 1, W, H, cap, &ws) != DRK_OK) {
        *never = true;
        *why = DRK_ENOMEM;
        return nullptr;
      }
    } else {
      return nullptr;
    }
  }
  WsEntry* e = new WsEntry();
  e->ws = ws;
  e->scene = r->scene; e->W = W; e->H = H; e->cap = cap;
  e->bytes = ws_bytes(ws);
  e->busy = true;
  s->ws_bytes += e->bytes;
  s->pool.push_back(e);
  return e;
}

drk_status enqueue_render(drk_server* s, Slot& slot, Request* r) {
  WsEntry* e = r->ws;
  const drk_scene& sc = s->scenes[r->scene].sc;
  hipStream_t st = slot.stream;
  drk_status rc = ws_set_cameras(e->ws, &r->cam, 1, st);
  if (rc) return rc;
  if (s->cfg.use_graphs) {
    if (!e->exec) {
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        set_error("hipStreamBeginCapture failed");
        return DRK_EDEVICE;
      }
      drk_status a = ws_preprocess_core(e->ws, &sc, &s->cfg.opts, st);
      drk_status b = a ? a : drk_bin_sort(e->ws, st);
      drk_status c = b ? b : drk_render_fwd(e->ws, ws_out_rgb(e->ws), nullptr, st);
      hipError_t ec = hipStreamEndCapture(st, &g);
      if (c) { if (g) hipGraphDestroy(g); return c; }
      if (ec != hipSuccess || !g) { set_error("hipStreamEndCapture failed"); return DRK_EDEVICE; }
      hipError_t ei = hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (ei != hipSuccess) { e->exec = nullptr; set_error("hipGraphInstantiate failed"); return DRK_EDEVICE; }
    }
    if (hipGraphLaunch(e->exec, st) != hipSuccess) { set_error("hipGraphLaunch failed"); return DRK_EDEVICE; }
  } else {
    if ((rc = ws_preprocess_core(e->ws, &sc, &s->cfg.opts, st))) return rc;
    if ((rc = drk_bin_sort(e->ws, st))) return rc;
    if ((rc = drk_render_fwd(e->ws, ws_out_rgb(e->ws), nullptr, st))) return rc;
  }
  uint32_t* d_status;
  uint64_t* d_total;
  ws_status_ptrs(e->ws, &d_status, &d_total);
  const size_t bytes = sizeof(float) * 3 * (size_t)r->cam.width * r->cam.height;
  if (hipMemcpyAsync(r->out, ws_out_rgb(e->ws), bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(slot.h_status, d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(slot.h_total, d_total, sizeof(uint64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipEventRecord(slot.ev, st) != hipSuccess) {
    set_error("enqueue copies failed");
    return DRK_EDEVICE;
  }
  return DRK_OK;
}

void complete(drk_server* s, Request* r, int status) {
  r->status = status;
  r->done_us = now_us();
  r->done = true;
  s->cv_done.notify_all();
}

void finish(drk_server* s, Slot& slot) {
  Request* r = slot.req;
  WsEntry* e = r->ws;
  slot.req = nullptr;
  --s->inflight;
  e->busy = false;
  e->last_use = ++s->tick;
  r->ws = nullptr;
  const uint32_t status = *slot.h_status;
  const int64_t total = (int64_t)*slot.h_total;
  r->pairs = total;
  if (status & ST_OVERFLOW) {
    // learn a larger capacity, drop the small workspace, run the request again first
    s->learned_cap[Key(e->scene, e->W, e->H)] = total + total / 4 + 1024;
    drop_entry(s, e);
    if (++r->retries > 3) { complete(s, r, DRK_EOVERFLOW); return; }
    s->pending.push_front(r);
    return;
  }
  complete(s, r, (status & ST_INVALID) ? DRK_EINVAL : DRK_OK);
}

// Requests behind the head that may be admitted while the head waits for memory, and how many
// times the head may be passed over before the scheduler waits for it.
constexpr int kLookahead = 16;
constexpr int kMaxBypass = 8;

void scheduler(drk_server* s) {
  hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    for (Slot& sl : s->slots)
      if (sl.req && hipEventQuery(sl.ev) == hipSuccess) finish(s, sl);
    for (Slot& sl : s->slots) {
      if (sl.req) continue;
      // the head if it fits now; else a later request that fits, while the head has been passed
      // over fewer than kMaxBypass times
      Request* r = nullptr;
      WsEntry* e = nullptr;
      Request* head = nullptr;
      int scanned = 0;
      for (auto it = s->pending.begin(); it != s->pending.end() && scanned < kLookahead;) {
        Request* q = *it;
        bool never = false;
        int why = DRK_OK;
        WsEntry* got = acquire(s, q, &never, &why);
        if (never) {
          it = s->pending.erase(it);
          q->start_us = now_us();
          complete(s, q, why);
          continue;
        }
        if (got) {
          s->pending.erase(it);
          r = q;
          e = got;
          break;
        }
        if (!head) {
          head = q;
          if (q->bypassed >= kMaxBypass) break;   // the head has waited long enough: keep arrival order
        }
        ++scanned;
        ++it;
      }
      if (r && head) ++head->bypassed;
      if (!r) break;                       // nothing fits now: wait for memory to free up
      r->ws = e;
      r->start_us = now_us();
      sl.req = r;
      ++s->inflight;
      drk_status rc = enqueue_render(s, sl, r);
      if (rc) {
        // the request fails; release its workspace (its graph may be half-built)
        sl.req = nullptr;
        --s->inflight;
        r->ws = nullptr;
        drop_entry(s, e);
        complete(s, r, rc);
      }
    }
    if (s->inflight == 0 && s->pending.empty()) {
      s->cv_sched.wait(lk);
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

}  // namespace

extern "C" {

drk_status drk_serve_create(const drk_serve_cfg* cfg, drk_server** out) {
  if (!cfg || !out) { set_error("null argument"); return DRK_EINVAL; }
  *out = nullptr;
  if (cfg->max_inflight < 1 || cfg->max_inflight > 64) { set_error("max_inflight must be in [1, 64]"); return DRK_EINVAL; }
  if (cfg->queue_capacity < 1) { set_error("queue_capacity must be >= 1"); return DRK_EINVAL; }
  if (cfg->hbm_budget_bytes < 0) { set_error("hbm_budget_bytes must be >= 0"); return DRK_EINVAL; }
  if (cfg->initial_pairs < 0) { set_error("initial_pairs must be >= 0"); return DRK_EINVAL; }
  const drk_opts& o = cfg->opts;
  if (o.cache_len < 1 || (o.cache_len > kMaxCache && o.cache_len < kExactOrder) || o.cull_mode < 0 || o.cull_mode > 2 || o.key_mode < 0 ||
      o.key_mode > 2 || o.launch_order < 0 || o.launch_order > 1 || !(o.alpha_min > 0.0f)) {
    set_error("invalid drk_opts in serve config");
    return DRK_EINVAL;
  }
  drk_server* s = new drk_server();
  s->cfg = *cfg;
  if (hipGetDevice(&s->device) != hipSuccess) { delete s; set_error("hipGetDevice failed"); return DRK_EDEVICE; }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { delete s; set_error("hipMemGetInfo failed"); return DRK_EDEVICE; }
  s->budget = cfg->hbm_budget_bytes > 0 ? cfg->hbm_budget_bytes : (int64_t)(free_b / 2);
  s->slots.resize(cfg->max_inflight);
  for (Slot& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&sl.h_status, 64, hipHostMallocDefault) != hipSuccess) {
      set_error("stream/event/pinned allocation failed");
      drk_serve_destroy(s);
      return DRK_EDEVICE;
    }
    sl.h_total = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(sl.h_status) + 8);
  }
  s->sched = std::thread(scheduler, s);
  *out = s;
  return DRK_OK;
}

drk_status drk_serve_destroy(drk_server* s) {
  if (!s) return DRK_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_sched.notify_all();
  if (s->sched.joinable()) s->sched.join();
  for (Slot& sl : s->slots) {
    if (sl.stream) hipStreamSynchronize(sl.stream);
  }
  while (!s->pool.empty()) drop_entry(s, s->pool.front());
  for (Slot& sl : s->slots) {
    if (sl.ev) hipEventDestroy(sl.ev);
    if (sl.stream) hipStreamDestroy(sl.stream);
    if (sl.h_status) hipHostFree(sl.h_status);
  }
  for (ResidentScene& r : s->scenes) hipFree(r.mem);
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
  return DRK_OK;
}

drk_status drk_serve_add_scene(drk_server* s, const drk_scene* sc, int32_t* scene_id) {
  if (!s || !sc || !scene_id) { set_error("null argument"); return DRK_EINVAL; }
  if (sc->K < 3 || sc->K > kMaxK || sc->n < 0 || (sc->color_mode != 0 && sc->color_mode != 1) ||
      (sc->color_mode == 1 && (sc->sh_degree < 0 || sc->sh_degree > 3))) {
    set_error("invalid scene");
    return DRK_EINVAL;
  }
  const int64_t n = sc->n;
  const int ncol = sc->color_mode == 1 ? 3 * (sc->sh_degree + 1) * (sc->sh_degree + 1) : 3;
  const size_t rows[8] = {3, 4, (size_t)sc->K, (size_t)sc->K, 1, 1, 1, (size_t)ncol};
  const float* src[8] = {sc->mu, sc->q, sc->scale, sc->theta, sc->eta, sc->tau, sc->opacity, sc->color};
  size_t total = 0;
  for (int i = 0; i < 8; ++i) total += rows[i] * n;
  ResidentScene rs;
  rs.bytes = total * sizeof(float);
  if (hipMalloc(&rs.mem, std::max<size_t>(rs.bytes, 256)) != hipSuccess) { set_error("scene allocation failed"); return DRK_ENOMEM; }
  float* dst = static_cast<float*>(rs.mem);
  const float* ptrs[8];
  for (int i = 0; i < 8; ++i) {
    if (n > 0 && hipMemcpy(dst, src[i], rows[i] * n * sizeof(float), hipMemcpyDeviceToDevice) != hipSuccess) {
      hipFree(rs.mem);
      set_error("scene copy failed");
      return DRK_EDEVICE;
    }
    ptrs[i] = dst;
    dst += rows[i] * n;
  }
  rs.sc = *sc;
  rs.sc.mu = ptrs[0]; rs.sc.q = ptrs[1]; rs.sc.scale = ptrs[2]; rs.sc.theta = ptrs[3];
  rs.sc.eta = ptrs[4]; rs.sc.tau = ptrs[5]; rs.sc.opacity = ptrs[6]; rs.sc.color = ptrs[7];
  std::lock_guard<std::mutex> lk(s->mu);
  s->scenes.push_back(rs);
  *scene_id = (int32_t)s->scenes.size() - 1;
  return DRK_OK;
}

drk_status drk_serve_submit(drk_server* s, int32_t scene_id, const drk_camera* cam, float* out_rgb,
                            uint64_t* request_id) {
  if (!s || !cam || !out_rgb || !request_id) { set_error("null argument"); return DRK_EINVAL; }
  std::unique_lock<std::mutex> lk(s->mu);
  if (scene_id < 0 || scene_id >= (int32_t)s->scenes.size()) { set_error("unknown scene %d", scene_id); return DRK_ENOTFOUND; }
  if (cam->width < 1 || cam->height < 1 || cam->width > 8192 || cam->height > kMaxTileRows * kTile ||
      !(cam->fx > 0.0f) || !(cam->fy > 0.0f)) {
    set_error("invalid camera");
    return DRK_EINVAL;
  }
  const size_t need = ws_size(s, scene_id, cam->width, cam->height,
                              initial_capacity(s, scene_id, cam->width, cam->height));
  if (need > (size_t)s->budget) {
    set_error("request needs %zu bytes of workspace, budget is %lld", need, (long long)s->budget);
    return DRK_ENOMEM;
  }
  if ((int32_t)s->pending.size() >= s->cfg.queue_capacity) { set_error("request queue full"); return DRK_EAGAIN; }
  Request* r = new Request();
  r->id = s->next_id++;
  r->scene = scene_id;
  r->cam = *cam;
  r->out = out_rgb;
  r->submit_us = now_us();
  s->reqs[r->id] = r;
  s->pending.push_back(r);
  *request_id = r->id;
  lk.unlock();
  s->cv_sched.notify_all();
  return DRK_OK;
}

drk_status drk_serve_poll(drk_server* s, uint64_t request_id, int32_t wait_us, drk_req_stats* out) {
  if (!s) { set_error("null server"); return DRK_EINVAL; }
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(request_id);
  if (it == s->reqs.end()) { set_error("unknown request %llu", (unsigned long long)request_id); return DRK_ENOTFOUND; }
  Request* r = it->second;
  if (!r->done && wait_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return r->done; });
  if (!r->done) return DRK_EAGAIN;
  if (out) {
    out->submit_us = r->submit_us;
    out->start_us = r->start_us;
    out->done_us = r->done_us;
    out->pairs = r->pairs;
    out->status = r->status;
    out->width = r->cam.width;
    out->height = r->cam.height;
  }
  s->reqs.erase(it);
  delete r;
  return DRK_OK;
}

}  // extern "C"
