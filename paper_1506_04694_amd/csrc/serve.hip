// Continuous-batching request server for MLMC samples (host side).
//
// A request is one term of the estimator eq. (3.6) (or eq. (4.2) with Coarse
// Grid Variates): sample number `sample` of level `level` on the m_fine grid,
// i.e. the fine solve and its coarse companion(s) and Y = Q_f - Q_c.
//
// A server may serve several models at once (for instance 2-D and 3-D fields
// of different laws); a request names its model by index, and every batch
// holds requests of one (model, level, grid) with that model's solver options.
//
// Requests are queued as they arrive.  Each worker thread owns a context (its
// own HIP stream at default priority and its own device workspaces, which stay
// allocated between batches: fields, operators and multigrid hierarchies are
// device-resident).  A free worker takes a batch of one (model, level, grid)
// kind -- the oldest waiting requests of that kind, up to max_batch, as long
// as the estimated device memory of all running batches stays within the
// budget (a lone request always runs when nothing else is running).  The kind
// is chosen among those waiting by the age of their oldest request measured in
// units of the kind's expected service time (so short requests do not queue
// behind long ones, and a long request's priority grows until it is served),
// skipping kinds that do not fit the budget; while short requests wait, at
// most n_workers - 1 workers hold long batches, unless a long request has
// waited kStarveS.  Batches of different workers run concurrently on the
// device, so requests that arrive while others are being solved start as soon
// as a worker and memory are free.
// A sample's results do not depend on its batch (per-sample random streams and
// per-sample fixed-order reductions), so a request gives the same numbers
// alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mlmc_darcy.h"

namespace {

struct Pending {
  uint64_t id;
  mlmc_request req;
  double t_submit;
};

struct Worker {
  mlmc_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  std::thread thread;
  // device staging for one batch
  uint32_t* d_ids = nullptr;
  double* d_out = nullptr;     // q_f, q_c, y: 3 * max_batch
  int32_t* d_flags = nullptr;  // failed, iters: 2 * max_batch
  uint32_t* h_ids = nullptr;   // pinned
  double* h_out = nullptr;
  int32_t* h_flags = nullptr;
};

}  // namespace

struct mlmc_server {
  mlmc_serve_opts opts;
  int running_long = 0;  // batches of long kinds being served
  int warming = 0;       // workers still running their warm-up
  std::vector<mlmc_model> models;
  std::vector<mlmc_solver_opts> solvers;  // one per model
  std::vector<Worker> workers;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Pending> queue;
  std::vector<mlmc_result> done;
  uint64_t next_id = 1;
  uint64_t in_flight_bytes = 0;
  int running = 0;
  bool stop = false;
  std::string err;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  std::atomic<int64_t> batches{0};

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

int n_ce_for(const mlmc_server* s, int model, int m) {
  for (int q = 0; q < s->opts.n_grids; ++q)
    if (s->opts.grid_model[q] == model && s->opts.grid_m[q] == m) return s->opts.grid_n_ce[q];
  return 0;
}

// Device bytes of one request's share of a batch: k, T (d), b, p, r, z, p, q,
// z_pre and the multigrid hierarchy (about 1/3 of a level per array; in 3-D
// also the colour-split copy of the swept levels' faces, 8/7 of the finest
// level's), plus the companions on the coarse grid (1 plain, 2^d with CGV), all
// FP64, and the circulant-embedding scratch (2-D: n m; 3-D: n^2 m + n m^2
// complex values).
uint64_t request_bytes(const mlmc_server* s, const mlmc_request& r) {
  const mlmc_model& mdl = s->models[r.model];
  const int d = mdl.dim;
  const double m = (double)r.m_fine;
  const double cells = d == 3 ? m * m * m : m * m;
  const double ncomp = r.level == 0 ? 0.0 : (s->opts.cgv ? (double)(1 << d) : 1.0);
  const double per_cell = 8.0 * (10.0 + (d + 2) * 4.0 / 3.0 + (d == 3 ? 3.0 * 8.0 / 7.0 : 0.0));
  double ce = 0.0;
  const double nce = (double)n_ce_for(s, r.model, r.m_fine);
  if (mdl.field_kind == MLMC_FIELD_CORRELATED)
    ce = d == 3 ? 16.0 * (nce * nce * m + nce * m * m) : 16.0 * nce * m;
  return (uint64_t)(cells * per_cell * (1.0 + ncomp / (double)(1 << d)) + ce);
}

// Expected service time of one request (seconds): a fixed per-batch part and a
// part proportional to the cells solved (fine grid plus companions).
double est_seconds(const mlmc_server* s, const mlmc_request& r) {
  const int d = s->models[r.model].dim;
  const double m = (double)r.m_fine;
  const double cells = d == 3 ? m * m * m : m * m;
  const double ncomp = r.level == 0 ? 0.0 : (s->opts.cgv ? (double)(1 << d) : 1.0);
  return 1e-3 + cells * (1.0 + ncomp / (double)(1 << d)) * 1e-8;
}
constexpr double kLongS = 3e-3;    // kinds above this are "long"
constexpr double kStarveS = 0.05;  // a long request waiting this long is served regardless

bool same_kind(const mlmc_request& a, const mlmc_request& b) {
  return a.model == b.model && a.level == b.level && a.m_fine == b.m_fine;
}

// Under the lock: the batch for a free worker (see the file comment); false
// when no waiting kind is eligible now.
bool pick_batch(mlmc_server* s, std::vector<Pending>& batch, uint64_t& bytes, bool& is_long) {
  if (s->queue.empty()) return false;
  struct Kind {
    mlmc_request key;
    double t_oldest, est;
    uint64_t one;
  };
  std::vector<Kind> kinds;
  for (const Pending& p : s->queue) {
    bool seen = false;
    for (const Kind& k : kinds) seen = seen || same_kind(k.key, p.req);
    if (!seen) kinds.push_back({p.req, p.t_submit, est_seconds(s, p.req), request_bytes(s, p.req)});
  }
  const double now = s->now();
  bool short_waiting = false;
  for (const Kind& k : kinds) short_waiting = short_waiting || k.est <= kLongS;
  const uint64_t budget = s->opts.hbm_budget_bytes;
  int best = -1;
  double best_prio = -1.0;
  for (int q = 0; q < (int)kinds.size(); ++q) {
    const Kind& k = kinds[q];
    if (s->in_flight_bytes + k.one > budget && s->running > 0) continue;
    const double age = now - k.t_oldest;
    if (k.est > kLongS && short_waiting && s->running_long >= s->opts.n_workers - 1 &&
        age < kStarveS)
      continue;
    const double prio = age / k.est;
    if (prio > best_prio) {
      best_prio = prio;
      best = q;
    }
  }
  if (best < 0) return false;
  const Kind& k = kinds[best];
  batch.clear();
  bytes = 0;
  for (auto it = s->queue.begin(); it != s->queue.end() && (int)batch.size() < s->opts.max_batch;) {
    if (same_kind(it->req, k.key) && (batch.empty() || s->in_flight_bytes + bytes + k.one <= budget)) {
      batch.push_back(*it);
      bytes += k.one;
      it = s->queue.erase(it);
    } else {
      ++it;
    }
  }
  is_long = k.est > kLongS;
  return true;
}

// Warm-up of one worker before it takes requests: for each served grid, one
// level run of a few samples (numbers above any request's), so that the grid's
// embedding eigenvalues and the worker's workspaces exist before the first
// request of that kind arrives (computing them in the serving loop would stall
// every batch on the device: freeing device memory waits for the device).
void warm_up(mlmc_server* s, Worker& w) {
  for (int q = 0; q < s->opts.n_grids; ++q) {
    const int mi = s->opts.grid_model[q], m = s->opts.grid_m[q];
    mlmc_request rq{m % 2 == 0 ? 1 : 0, m, 0u, mi};
    const uint64_t one = request_bytes(s, rq);
    const uint64_t share = s->opts.hbm_budget_bytes / (4ull * (uint64_t)s->opts.n_workers);
    int wb = (int)std::max<uint64_t>(1, std::min<uint64_t>(share / std::max<uint64_t>(one, 1), 16));
    wb = std::min(wb, s->opts.max_batch);
    for (int t = 0; t < wb; ++t) w.h_ids[t] = 0xFFFFF000u + (uint32_t)t;
    mlmc_model mdl = s->models[mi];
    mdl.n_ce = n_ce_for(s, mi, m);
    mlmc_level_sums sums;
    std::memset(&sums, 0, sizeof sums);
    const int maxb = s->opts.max_batch;
    if (hipMemcpyAsync(w.d_ids, w.h_ids, sizeof(uint32_t) * wb, hipMemcpyHostToDevice,
                       w.stream) != hipSuccess)
      return;
    (void)mlmc_level_run_ids(w.ctx, &mdl, rq.level, m, w.d_ids, wb, s->opts.cgv, &s->solvers[mi],
                             &sums, w.d_out, w.d_out + maxb, w.d_out + 2 * maxb, w.d_flags,
                             w.d_flags + maxb);
  }
  (void)hipStreamSynchronize(w.stream);
}

void worker_loop(mlmc_server* s, int wi) {
  Worker& w = s->workers[wi];
  (void)hipSetDevice(s->opts.device);
  const int maxb = s->opts.max_batch;
  std::vector<Pending> batch;
  batch.reserve(maxb);
  warm_up(s, w);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    --s->warming;
  }
  s->cv.notify_all();
  for (;;) {
    uint64_t bytes = 0;
    bool is_long = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->stop) return;
        if (pick_batch(s, batch, bytes, is_long)) {
          s->in_flight_bytes += bytes;
          ++s->running;
          if (is_long) ++s->running_long;
          break;
        }
        // a kind held back only by the long-batch limit becomes eligible by age
        s->cv.wait_for(lk, std::chrono::milliseconds(5));
      }
    }
    const double t_start = s->now();
    const int n = (int)batch.size();
    for (int q = 0; q < n; ++q) w.h_ids[q] = batch[q].req.sample;
    const int mi = batch[0].req.model;
    mlmc_model mdl = s->models[mi];
    mdl.n_ce = n_ce_for(s, mi, batch[0].req.m_fine);
    mlmc_level_sums sums;
    std::memset(&sums, 0, sizeof sums);
    mlmc_status st = MLMC_OK;
    if (hipMemcpyAsync(w.d_ids, w.h_ids, sizeof(uint32_t) * n, hipMemcpyHostToDevice, w.stream) !=
        hipSuccess)
      st = MLMC_EDEVICE;
    if (st == MLMC_OK)
      st = mlmc_level_run_ids(w.ctx, &mdl, batch[0].req.level, batch[0].req.m_fine, w.d_ids, n,
                              s->opts.cgv, &s->solvers[mi], &sums, w.d_out, w.d_out + maxb,
                              w.d_out + 2 * maxb, w.d_flags, w.d_flags + maxb);
    if (st == MLMC_OK || st == MLMC_ENOCONV) {
      (void)hipMemcpyAsync(w.h_out, w.d_out, sizeof(double) * 3 * maxb, hipMemcpyDeviceToHost,
                           w.stream);
      (void)hipMemcpyAsync(w.h_flags, w.d_flags, sizeof(int32_t) * 2 * maxb,
                           hipMemcpyDeviceToHost, w.stream);
      (void)hipStreamSynchronize(w.stream);
    }
    const double t_done = s->now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (int q = 0; q < n; ++q) {
        mlmc_result r;
        std::memset(&r, 0, sizeof r);
        r.id = batch[q].id;
        r.level = batch[q].req.level;
        r.m_fine = batch[q].req.m_fine;
        r.sample = batch[q].req.sample;
        r.model = mi;
        r.batch_size = n;
        r.t_submit = batch[q].t_submit;
        r.t_start = t_start;
        r.t_done = t_done;
        if (st == MLMC_OK || st == MLMC_ENOCONV) {
          r.q_f = w.h_out[q];
          r.q_c = w.h_out[maxb + q];
          r.y = w.h_out[2 * maxb + q];
          r.failed = w.h_flags[q];
          r.iters = w.h_flags[maxb + q];
          r.status = MLMC_OK;
        } else {
          r.failed = 1;
          r.status = st;
        }
        s->done.push_back(r);
      }
      if (st != MLMC_OK && st != MLMC_ENOCONV) s->err = mlmc_last_error(w.ctx);
      s->in_flight_bytes -= bytes;
      --s->running;
      if (is_long) --s->running_long;
      s->batches++;
    }
    s->cv.notify_all();
  }
}

void release(mlmc_server* s) {
  for (auto& w : s->workers) {
    if (w.ctx) mlmc_ctx_destroy(w.ctx);
    if (w.stream) (void)hipStreamDestroy(w.stream);
    if (w.d_ids) (void)hipFree(w.d_ids);
    if (w.d_out) (void)hipFree(w.d_out);
    if (w.d_flags) (void)hipFree(w.d_flags);
    if (w.h_ids) (void)hipHostFree(w.h_ids);
    if (w.h_out) (void)hipHostFree(w.h_out);
    if (w.h_flags) (void)hipHostFree(w.h_flags);
  }
  delete s;
}

}  // namespace

extern "C" {

mlmc_status mlmc_serve_opts_default(mlmc_serve_opts* o) {
  if (!o) return MLMC_EINVAL;
  std::memset(o, 0, sizeof *o);
  o->device = 0;
  o->n_workers = 3;
  o->max_batch = 256;
  o->cgv = 0;
  o->hbm_budget_bytes = 64ull << 30;
  return mlmc_solver_opts_default(&o->solver);
}

mlmc_status mlmc_serve_start_models(const mlmc_model* models, const mlmc_solver_opts* solvers,
                                    int n_models, const mlmc_serve_opts* opts, mlmc_server** out) {
  if (!models || !opts || !out) return MLMC_EINVAL;
  *out = nullptr;
  if (n_models < 1 || n_models > 8 || opts->n_workers < 1 || opts->n_workers > 16 ||
      opts->max_batch < 1 || opts->n_grids < 0 || opts->n_grids > 8)
    return MLMC_EINVAL;
  for (int q = 0; q < opts->n_grids; ++q)
    if (opts->grid_model[q] < 0 || opts->grid_model[q] >= n_models) return MLMC_EINVAL;
  for (int q = 0; q < n_models; ++q)
    if (models[q].dim != 2 && models[q].dim != 3) return MLMC_EINVAL;
  mlmc_server* s = new mlmc_server();
  s->opts = *opts;
  s->models.assign(models, models + n_models);
  s->solvers.assign(n_models, opts->solver);
  if (solvers) s->solvers.assign(solvers, solvers + n_models);
  s->workers.resize(opts->n_workers);
  if (hipSetDevice(opts->device) != hipSuccess) {
    delete s;
    return MLMC_EDEVICE;
  }
  const int maxb = opts->max_batch;
  for (auto& w : s->workers) {
    bool ok = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) == hipSuccess &&
              mlmc_ctx_create(opts->device, w.stream, &w.ctx) == MLMC_OK &&
              hipMalloc(&w.d_ids, sizeof(uint32_t) * maxb) == hipSuccess &&
              hipMalloc(&w.d_out, sizeof(double) * 3 * maxb) == hipSuccess &&
              hipMalloc(&w.d_flags, sizeof(int32_t) * 2 * maxb) == hipSuccess &&
              hipHostMalloc(&w.h_ids, sizeof(uint32_t) * maxb, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&w.h_out, sizeof(double) * 3 * maxb, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&w.h_flags, sizeof(int32_t) * 2 * maxb, hipHostMallocDefault) ==
                  hipSuccess;
    if (!ok) {
      release(s);
      return MLMC_ENOMEM;
    }
  }
  s->warming = opts->n_workers;
  for (int wi = 0; wi < opts->n_workers; ++wi)
    s->workers[wi].thread = std::thread(worker_loop, s, wi);
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [s] { return s->warming == 0; });
  }
  *out = s;
  return MLMC_OK;
}

mlmc_status mlmc_serve_start(const mlmc_model* model, const mlmc_serve_opts* opts,
                             mlmc_server** out) {
  return mlmc_serve_start_models(model, nullptr, 1, opts, out);
}

mlmc_status mlmc_serve_submit(mlmc_server* s, const mlmc_request* req, uint64_t* id) {
  if (!s || !req) return MLMC_EINVAL;
  if (req->model < 0 || req->model >= (int)s->models.size()) return MLMC_EINVAL;
  if (req->level < 0 || req->m_fine < 1 || (req->level > 0 && req->m_fine % 2))
    return MLMC_EINVAL;
  if (s->models[req->model].field_kind == MLMC_FIELD_CORRELATED &&
      n_ce_for(s, req->model, req->m_fine) == 0)
    return MLMC_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return MLMC_EINVAL;
    Pending p{s->next_id++, *req, s->now()};
    if (id) *id = p.id;
    s->queue.push_back(p);
  }
  s->cv.notify_all();
  return MLMC_OK;
}

mlmc_status mlmc_serve_poll(mlmc_server* s, mlmc_result* out, int max, int* n_out,
                            int64_t* pending) {
  if (!s || !n_out || (max > 0 && !out)) return MLMC_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  const int n = std::min<int>(max, (int)s->done.size());
  for (int q = 0; q < n; ++q) out[q] = s->done[q];
  s->done.erase(s->done.begin(), s->done.begin() + n);
  *n_out = n;
  if (pending) *pending = (int64_t)s->queue.size() + (int64_t)s->done.size();
  return MLMC_OK;
}

double mlmc_serve_now(const mlmc_server* s) { return s ? s->now() : 0.0; }

mlmc_status mlmc_serve_stats(mlmc_server* s, int64_t* batches, int64_t* queued, int* running,
                             uint64_t* in_flight_bytes) {
  if (!s) return MLMC_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (batches) *batches = s->batches.load();
  if (queued) *queued = (int64_t)s->queue.size();
  if (running) *running = s->running;
  if (in_flight_bytes) *in_flight_bytes = s->in_flight_bytes;
  return MLMC_OK;
}

mlmc_status mlmc_serve_stop(mlmc_server* s) {
  if (!s) return MLMC_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& w : s->workers)
    if (w.thread.joinable()) w.thread.join();
  release(s);
  return MLMC_OK;
}

}  // extern "C"
