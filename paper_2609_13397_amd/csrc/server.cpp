// Render server: continuous batching of view requests against device-resident
// scenes, admitted by an HBM budget.
//
// Requests queue in arrival order.  Each worker thread owns one HIP stream.  A free
// worker takes the oldest request if its estimated scratch memory fits the budget
// next to the requests already running (or if nothing else is running, so one
// oversized request still makes progress), then fuses further queued requests for
// the same scene into the same render call while they fit the view, pixel and memory
// caps.  Requests that arrive while others are on the device are admitted as soon as
// a worker and memory free up; the calls of different workers overlap on the GPU.
// The per-view-launch baseline is the same server with one worker and one view per
// call.  With a request time limit, requests still queued past it complete with
// CG_ERR_TIMEOUT, unrendered.  The scheduler is independent of the executor, so a CPU stand-in executor
// (a timed sleep) exercises admission, batching and cancellation without a GPU.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "fwd_state.hpp"

using namespace cg;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id;
  int32_t scene;
  cg_camera cam;
  float* out;
  double t_submit, t_admit;
  size_t est;
  int64_t px;
};

// Pairs of a view of a scene, estimated as a + b * pixels: a view of a large scene at
// low resolution has most of its Gaussians in few tiles, so the pairs do not scale with
// the pixels alone.  a and b are the least-squares fit over completed calls (k views,
// their pixels and pairs), with older calls weighted down by 0.9 per call.
struct PairModel {
  double kk = 0, kp = 0, pp = 0, ky = 0, py = 0;  // decayed sums of k^2, k px, px^2, k y, px y
  double a = 0.0, b = 4.0;                        // before any call: 4 pairs per pixel
  void add(double k, double px, double y) {
    constexpr double decay = 0.9;
    kk = decay * kk + k * k;
    kp = decay * kp + k * px;
    pp = decay * pp + px * px;
    ky = decay * ky + k * y;
    py = decay * py + px * y;
    const double det = kk * pp - kp * kp;
    double na = det > 1e-9 * kk * pp ? (ky * pp - kp * py) / det : -1.0;
    double nb = det > 1e-9 * kk * pp ? (kk * py - kp * ky) / det : -1.0;
    if (!(na >= 0.0 && nb >= 0.0)) {  // degenerate or negative: per-pixel rate only
      na = 0.0;
      nb = pp > 0.0 ? py / pp : b;
    }
    a = na;
    b = nb;
  }
  double pairs(double px) const { return a + b * px; }
};

struct SceneEntry {
  cg_gaussians g;
  cg_render_opts opts;
  PairModel model;  // running estimate used by admission and fusion
};

}  // namespace

struct cg_server {
  cg_server_config cfg;
  std::vector<SceneEntry> scenes;
  std::deque<Request> queue;
  std::vector<cg_server_completion> done;
  size_t reserved = 0, peak_reserved = 0;
  int in_flight = 0;
  int64_t next_id = 1, completed = 0, batches = 0, views = 0, max_batch_seen = 0, timed_out = 0;
  bool stopping = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<std::thread> workers;

  // Scratch estimate of one view: per (view, Gaussian) record, keys, cone, counts and
  // tile-group list;
  // per pair the tile key and value (twice, for the sort) plus slack; per tile its
  // cones and its 256 slots of the 64-byte pixel ray buffer; per pixel the output
  // staging; when the launch is small enough to take the split tile render (which one
  // decides from its longest tile list), its per-segment state (tiles + pairs / 384
  // segments, at most tiles + 16384, of 256 pixels, 20 bytes each).  The pair model is
  // refreshed from completed calls.
  static double estimate_pairs(const SceneEntry& sc, const cg_camera& cam) {
    const int64_t px = (int64_t)cam.crop_w * cam.crop_h;
    const int64_t tiles = (int64_t)((cam.crop_w + 15) / 16) * ((cam.crop_h + 15) / 16);
    return sc.model.pairs((double)px) + 64.0 * (double)tiles;
  }

  size_t estimate(const SceneEntry& sc, const cg_camera& cam) const {
    const int64_t px = (int64_t)cam.crop_w * cam.crop_h;
    const int64_t tiles = (int64_t)((cam.crop_w + 15) / 16) * ((cam.crop_h + 15) / 16);
    const double pairs = estimate_pairs(sc, cam);
    const SplitPolicy pol = split_policy();
    const double segs = tiles < pol.max_tiles
                            ? (double)tiles + std::min((double)kSegTarget, pairs / (double)kMinSegLen)
                            : 0.0;
    return (size_t)(sc.g.n * 232 + pairs * 24.0 + (double)tiles * (48.0 + 256.0 * 64.0) + (double)px * 8.0 + (1 << 20) +
                    segs * 256.0 * 20.0);
  }

  // Completes every queued request older than the time limit with CG_ERR_TIMEOUT
  // (caller holds mu).
  void expire_locked() {
    if (!(cfg.request_timeout_ms > 0.0)) return;
    const double t = now_s(), limit = cfg.request_timeout_ms * 1e-3;
    bool any = false;
    for (auto it = queue.begin(); it != queue.end();) {
      if (t - it->t_submit > limit) {
        cg_server_completion c;
        std::memset(&c, 0, sizeof(c));
        c.request_id = it->id;
        c.status = CG_ERR_TIMEOUT;
        c.scene = it->scene;
        c.t_submit = it->t_submit;
        c.t_done = t;
        done.push_back(c);
        ++completed;
        ++timed_out;
        it = queue.erase(it);
        any = true;
      } else {
        ++it;
      }
    }
    if (any) cv_done.notify_all();
  }

  bool can_admit_head() const {
    if (queue.empty()) return false;
    return in_flight == 0 || reserved + queue.front().est <= cfg.hbm_budget_bytes;
  }

  void execute(std::vector<Request>& batch, const SceneEntry& sc, int32_t* status, int64_t* pairs,
               hipStream_t stream) {
    const int n = (int)batch.size();
    if (cfg.fake_executor) {
      int64_t px = 0;
      for (auto& r : batch) px += r.px;
      const double secs = (cfg.fake_ns_per_call + cfg.fake_ns_per_pixel * (double)px) * 1e-9;
      std::this_thread::sleep_for(std::chrono::duration<double>(secs));
      *status = CG_OK;
      *pairs = 0;
      return;
    }
    std::vector<cg_camera> cams(n);
    std::vector<float*> outs(n);
    for (int i = 0; i < n; ++i) {
      cams[i] = batch[i].cam;
      outs[i] = batch[i].out;
    }
    cg_fwd_stats st;
    std::memset(&st, 0, sizeof(st));
    *status = guarded([&] {
      run_forward(&sc.g, cams.data(), n, &sc.opts, nullptr, nullptr, outs.data(), nullptr, &st, stream);
      CG_HIP(hipStreamSynchronize(stream));
    });
    *pairs = st.n_pairs;
  }

  void worker_loop(int w) {
    (void)w;
    hipStream_t stream = nullptr;
    if (!cfg.fake_executor) {
      if (hipSetDevice(cfg.device) != hipSuccess || hipStreamCreate(&stream) != hipSuccess) stream = nullptr;
    }
    for (;;) {
      std::vector<Request> batch;
      size_t est_total = 0;
      int64_t px_total = 0;
      SceneEntry scene;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          expire_locked();
          if (stopping || can_admit_head()) break;
          if (cfg.request_timeout_ms > 0.0)
            cv_work.wait_for(lk, std::chrono::duration<double, std::milli>(cfg.request_timeout_ms));
          else
            cv_work.wait(lk);
        }
        if (stopping) break;
        Request head = queue.front();
        queue.pop_front();
        scene = scenes[head.scene];
        batch.push_back(head);
        est_total = head.est;
        px_total = head.px;
        // the scene's estimate as it stands now (refreshed by completed calls)
        const auto pairs_of = [&](const Request& r) { return estimate_pairs(scene, r.cam); };
        double pairs_total = pairs_of(head);
        for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < cfg.max_batch_views;) {
          if (it->scene == head.scene && px_total + it->px <= cfg.max_batch_pixels &&
              pairs_total + pairs_of(*it) <= cfg.max_batch_pairs &&
              reserved + est_total + it->est <= cfg.hbm_budget_bytes) {
            est_total += it->est;
            px_total += it->px;
            pairs_total += pairs_of(*it);
            batch.push_back(*it);
            it = queue.erase(it);
          } else {
            ++it;
          }
        }
        reserved += est_total;
        peak_reserved = std::max(peak_reserved, reserved);
        ++in_flight;
        const double t = now_s();
        for (auto& r : batch) r.t_admit = t;
      }
      int32_t status = CG_OK;
      int64_t pairs = 0;
      const double t_start = now_s();
      execute(batch, scene, &status, &pairs, stream);
      const double t_done = now_s();
      {
        std::lock_guard<std::mutex> lk(mu);
        reserved -= est_total;
        --in_flight;
        ++batches;
        views += (int64_t)batch.size();
        max_batch_seen = std::max<int64_t>(max_batch_seen, (int64_t)batch.size());
        if (status == CG_OK && px_total > 0 && !cfg.fake_executor) {
          SceneEntry& sc = scenes[batch[0].scene];
          sc.model.add((double)batch.size(), (double)px_total, (double)pairs);
        }
        for (auto& r : batch) {
          cg_server_completion c;
          std::memset(&c, 0, sizeof(c));
          c.request_id = r.id;
          c.status = status;
          c.scene = r.scene;
          c.batch_views = (int32_t)batch.size();
          c.t_submit = r.t_submit;
          c.t_admit = r.t_admit;
          c.t_start = t_start;
          c.t_done = t_done;
          c.n_pairs = pairs;
          done.push_back(c);
          ++completed;
        }
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (stream) (void)hipStreamDestroy(stream);
  }
};

extern "C" {

void cg_server_default_config(cg_server_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->hbm_budget_bytes = (size_t)24 << 30;
  c->max_batch_views = 8;
  c->max_batch_pixels = 16 << 20;
  c->n_workers = 3;
  c->fake_executor = 0;
  c->fake_ns_per_pixel = 1.0;
  c->fake_ns_per_call = 50000.0;
  c->device = 0;
  c->request_timeout_ms = 0.0;
  c->max_batch_pairs = 12e6;
}

cg_status cg_server_create(const cg_server_config* cfg, cg_server** out) {
  return guarded([&] {
    CG_CHECK_ARG(cfg && out, "null argument");
    CG_CHECK_ARG(cfg->n_workers >= 1 && cfg->n_workers <= 16, "n_workers must be in [1, 16]");
    CG_CHECK_ARG(cfg->max_batch_views >= 1 && cfg->max_batch_views <= 256, "max_batch_views must be in [1, 256]");
    CG_CHECK_ARG(cfg->max_batch_pixels >= 1, "max_batch_pixels must be >= 1");
    CG_CHECK_ARG(cfg->hbm_budget_bytes > 0, "hbm_budget_bytes must be > 0");
    CG_CHECK_ARG(cfg->request_timeout_ms >= 0.0, "request_timeout_ms must be >= 0");
    CG_CHECK_ARG(cfg->max_batch_pairs > 0.0, "max_batch_pairs must be > 0");
    *out = nullptr;
    cg_server* s = new cg_server();
    s->cfg = *cfg;
    for (int w = 0; w < cfg->n_workers; ++w) s->workers.emplace_back([s, w] { s->worker_loop(w); });
    *out = s;
  });
}

cg_status cg_server_add_scene(cg_server* s, const cg_gaussians* g, const cg_render_opts* opts, int32_t* scene_id) {
  return guarded([&] {
    CG_CHECK_ARG(s && g && opts && scene_id, "null argument");
    (void)make_gauss(*g);
    (void)make_opts(*opts);
    std::lock_guard<std::mutex> lk(s->mu);
    s->scenes.push_back(SceneEntry{*g, *opts, PairModel{}});
    *scene_id = (int32_t)s->scenes.size() - 1;
  });
}

cg_status cg_server_submit(cg_server* s, int32_t scene, const cg_camera* cam, float* out_rgba,
                           int64_t* request_id) {
  return guarded([&] {
    CG_CHECK_ARG(s && cam, "null argument");
    check_camera(*cam, 0);
    const int64_t px = (int64_t)cam->crop_w * cam->crop_h;
    CG_CHECK_ARG(px == 0 || out_rgba, "null output");
    {
      std::lock_guard<std::mutex> lk(s->mu);
      CG_CHECK_ARG(scene >= 0 && scene < (int32_t)s->scenes.size(), "unknown scene");
      CG_CHECK_ARG(!s->stopping, "server is shutting down");
      Request r;
      r.id = s->next_id++;
      r.scene = scene;
      r.cam = *cam;
      r.out = out_rgba;
      r.t_submit = now_s();
      r.t_admit = 0.0;
      r.px = px;
      r.est = s->estimate(s->scenes[scene], *cam);
      s->queue.push_back(r);
      if (request_id) *request_id = r.id;
    }
    s->cv_work.notify_one();
  });
}

cg_status cg_server_cancel(cg_server* s, int64_t request_id, int32_t* cancelled) {
  return guarded([&] {
    CG_CHECK_ARG(s, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t found = 0;
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
      if (it->id == request_id) {
        cg_server_completion c;
        std::memset(&c, 0, sizeof(c));
        c.request_id = it->id;
        c.status = CG_ERR_STATE;
        c.scene = it->scene;
        c.t_submit = it->t_submit;
        c.t_done = now_s();
        s->done.push_back(c);
        s->queue.erase(it);
        found = 1;
        break;
      }
    }
    if (cancelled) *cancelled = found;
    s->cv_done.notify_all();
  });
}

cg_status cg_server_poll(cg_server* s, cg_server_completion* out, int32_t capacity, int32_t* n_out,
                         int32_t wait_ms) {
  return guarded([&] {
    CG_CHECK_ARG(s && n_out && (capacity == 0 || out), "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    s->expire_locked();
    if (s->done.empty() && wait_ms > 0)
      s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    const int32_t n = (int32_t)std::min<size_t>((size_t)std::max(capacity, 0), s->done.size());
    for (int32_t i = 0; i < n; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + n);
    *n_out = n;
  });
}

cg_status cg_server_drain(cg_server* s) {
  return guarded([&] {
    CG_CHECK_ARG(s, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->expire_locked();
    s->cv_done.wait(lk, [&] { return s->queue.empty() && s->in_flight == 0; });
  });
}

cg_status cg_server_get_stats(cg_server* s, cg_server_stats* out) {
  return guarded([&] {
    CG_CHECK_ARG(s && out, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->queued = (int64_t)s->queue.size();
    out->in_flight = s->in_flight;
    out->completed = s->completed;
    out->batches = s->batches;
    out->views = s->views;
    out->max_batch_views = s->max_batch_seen;
    out->reserved_bytes = (int64_t)s->reserved;
    out->peak_reserved_bytes = (int64_t)s->peak_reserved;
    out->timed_out = s->timed_out;
  });
}

void cg_server_destroy(cg_server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->queue.clear();
    s->cv_done.wait(lk, [&] { return s->in_flight == 0; });
    s->stopping = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  delete s;
}

double cg_server_now(void) { return now_s(); }

}  // extern "C"
