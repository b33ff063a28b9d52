// Continuous-batching request loop for many independent GPR solves.
//
// Each request is one solve of (K~ + eta^2 I) alpha = y (eq:gprsolve) on its own
// points and hyperparameters.  The server owns `max_slots` worker threads,
// each with its own non-blocking HIP stream.  A free slot admits a queued
// request whose plans fit in the device-byte budget next to the requests
// already in flight (oldest first, or smallest first with aging); its plan(s)
// are built, the solve runs on the slot's stream (so requests overlap on the
// device), alpha is written to the caller's buffer and the plans are released.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "gp_internal.h"

namespace gp {

struct SRequest {
  int64_t id = 0;
  int d = 0;
  int64_t n = 0;
  const double *pts = nullptr, *sigma = nullptr, *l = nullptr, *y = nullptr;
  double* alpha = nullptr;
  double nu = 0, eta = 0;
  size_t bytes = 0;
  double t_submit = 0, t_start = -1, t_ready = -1, t_done = -1;
  int status = GP_OK, iters = 0, refinements = 0, slot = -1, precision = GP_FP64;
  double rel_res = 0;
  bool done = false;
  std::string err;
  // recorded on the caller's stream at submit: the inputs are ready once it
  // has completed
  hipEvent_t ready = nullptr;
  void release_event() {
    if (ready) (void)hipEventDestroy(ready);
    ready = nullptr;
  }
  ~SRequest() { release_event(); }
};

struct Server {
  gp_server_opts o;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<SRequest*> queue;
  std::map<int64_t, std::unique_ptr<SRequest>> all;
  size_t bytes_in_use = 0, peak_bytes = 0;
  int running = 0, peak_running = 0;
  int64_t next_id = 1, completed = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  hipStream_t qstream = nullptr;  // for admission queries
  std::chrono::steady_clock::time_point t0;
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void fill_opts(const Server& S, int bulk, hipStream_t st, gp_opts* o) {
  gp_opts_init(o);
  o->precision = bulk ? GP_FP32_BULK : GP_FP64;
  o->stream = st;
}

// Device bytes the request's plan(s) will hold; decides the precision path.
size_t request_bytes(Server& S, SRequest& r) {
  gp_opts o;
  size_t b64 = 0, b32 = 0;
  fill_opts(S, 0, S.qstream, &o);
  Plan q64;
  build_plan(r.d, r.n, r.pts, r.sigma, r.l, r.nu, r.eta, S.o.plan_tol, &o, &q64, true, &b64);
  r.precision = (S.o.precision == GP_FP64 || b64 < S.o.fp64_below_bytes) ? GP_FP64 : GP_FP32_BULK;
  if (r.precision == GP_FP64) return b64;
  fill_opts(S, 1, S.qstream, &o);
  o.dw = q64.dw;
  o.M = q64.M;
  Plan q32;
  build_plan(r.d, r.n, r.pts, r.sigma, r.l, r.nu, r.eta, S.o.plan_tol_bulk, &o, &q32, true, &b32);
  return b64 + b32;
}

void run_request(Server& S, SRequest& r, hipStream_t st) {
  GP_HIP(hipStreamWaitEvent(st, r.ready, 0));
  gp_opts o;
  fill_opts(S, 0, st, &o);
  Plan P64;
  build_plan(r.d, r.n, r.pts, r.sigma, r.l, r.nu, r.eta, S.o.plan_tol, &o, &P64, false, nullptr);
  if (r.precision == GP_FP64) {
    r.t_ready = S.now();
    double* V = P64.vec.as<double>();
    gather_sorted(&P64, r.y, V + 6 * r.n);
    GP_HIP(hipMemsetAsync(V + 2 * r.n, 0, r.n * sizeof(double), st));
    int it = 0;
    double rel = 0;
    r.status = cg_solve_sorted(&P64, V + 6 * r.n, V + 2 * r.n, true, S.o.cg_tol, S.o.max_iter, 0,
                               &it, &rel);
    scatter_user(&P64, V + 2 * r.n, r.alpha);
    GP_HIP(hipStreamSynchronize(st));
    r.iters = it;
    r.rel_res = rel;
    return;
  }
  fill_opts(S, 1, st, &o);
  o.dw = P64.dw;
  o.M = P64.M;
  Plan P32;
  build_plan(r.d, r.n, r.pts, r.sigma, r.l, r.nu, r.eta, S.o.plan_tol_bulk, &o, &P32, false, nullptr);
  r.t_ready = S.now();
  int it = 0, passes = 0;
  double rel = 0;
  r.status = cg_refined_user(&P32, &P64, r.y, r.alpha, S.o.cg_tol, S.o.inner_tol, S.o.max_iter,
                             S.o.max_refine, 0, &it, &rel, &passes);
  r.iters = it;
  r.rel_res = rel;
  r.refinements = passes;
}

// Queued request to admit next (queue.end() if none may start now); called
// with the lock held.
std::deque<SRequest*>::iterator pick_next(Server* S) {
  auto best = S->queue.end();
  double best_key = 0.0;
  const double now = S->now();
  for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
    const SRequest* r = *it;
    const bool fits = S->bytes_in_use + r->bytes <= S->o.max_device_bytes || S->running == 0;
    if (S->o.policy == GP_SERVE_FIFO) return fits ? it : S->queue.end();
    if (!fits) continue;
    const double key = (double)r->bytes - S->o.aging_bytes_per_s * (now - r->t_submit);
    if (best == S->queue.end() || key < best_key) {
      best = it;
      best_key = key;
    }
  }
  return best;
}

void worker(Server* S, int slot) {
  hipStream_t st = S->streams[slot];
  while (true) {
    SRequest* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        if (S->stop && S->queue.empty()) return true;
        return pick_next(S) != S->queue.end();
      });
      if (S->queue.empty()) return;  // stop requested and nothing left
      auto it = pick_next(S);
      if (it == S->queue.end()) continue;
      r = *it;
      S->queue.erase(it);
      S->bytes_in_use += r->bytes;
      S->peak_bytes = std::max(S->peak_bytes, S->bytes_in_use);
      S->running += 1;
      S->peak_running = std::max(S->peak_running, S->running);
      r->t_start = S->now();
      r->slot = slot;
    }
    try {
      run_request(*S, *r, st);
    } catch (const Error& e) {
      r->status = e.code;
      r->err = e.msg;
    } catch (const std::exception& e) {
      r->status = GP_EDEVICE;
      r->err = e.what();
    }
    r->release_event();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->bytes_in_use -= r->bytes;
      S->running -= 1;
      S->completed += 1;
      r->t_done = S->now();
      r->done = true;
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

}  // namespace
}  // namespace gp

using namespace gp;

struct gp_server_s {
  Server S;
};

template <class F>
static int sguard(F&& f) {
  try {
    clear_error();
    return f();
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return GP_EDEVICE;
  }
}

extern "C" {

int gp_server_opts_init(gp_server_opts* o) {
  if (!o) return GP_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->max_slots = 4;
  o->max_device_bytes = (size_t)64 << 30;
  o->precision = GP_FP32_BULK;
  o->plan_tol = 1e-8;
  o->plan_tol_bulk = 1e-4;
  o->cg_tol = 1e-6;
  o->inner_tol = 3e-3;
  o->max_iter = 20000;
  o->max_refine = 10;
  o->fp64_below_bytes = (size_t)256 << 20;
  o->policy = GP_SERVE_SMALLEST;
  o->aging_bytes_per_s = (double)((size_t)1 << 30);
  return GP_OK;
}

int gp_server_create(const gp_server_opts* opts, gp_server_t* out) {
  return sguard([&] {
    if (!opts || !out) throw Error{GP_EINVAL, "null argument"};
    if (opts->max_slots < 1 || opts->max_slots > 64) throw Error{GP_EINVAL, "max_slots in 1..64"};
    if (opts->precision != GP_FP64 && opts->precision != GP_FP32_BULK)
      throw Error{GP_EINVAL, "unknown precision"};
    if (opts->policy != GP_SERVE_FIFO && opts->policy != GP_SERVE_SMALLEST)
      throw Error{GP_EINVAL, "unknown admission policy"};
    if (!(opts->aging_bytes_per_s >= 0)) throw Error{GP_EINVAL, "aging_bytes_per_s must be >= 0"};
    auto* h = new gp_server_s();
    Server& S = h->S;
    S.o = *opts;
    S.t0 = std::chrono::steady_clock::now();
    try {
      GP_HIP(hipStreamCreateWithFlags(&S.qstream, hipStreamNonBlocking));
      for (int k = 0; k < opts->max_slots; ++k) {
        hipStream_t st;
        GP_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        S.streams.push_back(st);
      }
      for (int k = 0; k < opts->max_slots; ++k) S.workers.emplace_back(worker, &S, k);
    } catch (...) {
      {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stop = true;
      }
      S.cv_work.notify_all();
      for (auto& t : S.workers) t.join();
      for (auto st : S.streams) (void)hipStreamDestroy(st);
      if (S.qstream) (void)hipStreamDestroy(S.qstream);
      delete h;
      throw;
    }
    *out = h;
    return GP_OK;
  });
}

int gp_server_submit(gp_server_t h, int d, int64_t n, const double* pts, const double* sigma,
                     const double* l, double nu, double eta, const double* y, double* alpha,
                     void* stream, int64_t* id) {
  return sguard([&] {
    if (!h || !pts || !sigma || !l || !y || !alpha || !id) throw Error{GP_EINVAL, "null argument"};
    Server& S = h->S;
    auto r = std::make_unique<SRequest>();
    r->d = d;
    r->n = n;
    r->pts = pts;
    r->sigma = sigma;
    r->l = l;
    r->y = y;
    r->alpha = alpha;
    r->nu = nu;
    r->eta = eta;
    r->t_submit = S.now();
    // the inputs may still be in production on the caller's stream: every
    // read of them (the size query here, the solve later) waits for this event
    GP_HIP(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
    GP_HIP(hipEventRecord(r->ready, static_cast<hipStream_t>(stream)));
    GP_HIP(hipStreamWaitEvent(S.qstream, r->ready, 0));
    r->bytes = request_bytes(S, *r);  // validates the inputs too
    if (r->bytes > S.o.max_device_bytes)
      throw Error{GP_ENOMEM, "request needs " + std::to_string(r->bytes) +
                                 " device bytes, more than the server budget"};
    SRequest* raw = r.get();
    {
      std::lock_guard<std::mutex> lk(S.mu);
      if (S.stop) throw Error{GP_EINVAL, "server is shutting down"};
      raw->id = S.next_id++;
      S.all[raw->id] = std::move(r);
      S.queue.push_back(raw);
    }
    S.cv_work.notify_all();
    *id = raw->id;
    return GP_OK;
  });
}

static void fill_info(const SRequest& r, gp_request_info* info) {
  info->status = r.status;
  info->iters = r.iters;
  info->refinements = r.refinements;
  info->rel_res = r.rel_res;
  info->t_submit = r.t_submit;
  info->t_start = r.t_start;
  info->t_done = r.t_done;
  info->t_ready = r.t_ready;
  info->device_bytes = r.bytes;
  info->slot = r.slot;
  info->precision = r.precision;
}

int gp_server_wait(gp_server_t h, int64_t id, gp_request_info* info) {
  return sguard([&] {
    if (!h) throw Error{GP_EINVAL, "null server"};
    Server& S = h->S;
    std::unique_lock<std::mutex> lk(S.mu);
    auto itr = S.all.find(id);
    if (itr == S.all.end()) throw Error{GP_EINVAL, "unknown request id"};
    SRequest* r = itr->second.get();
    S.cv_done.wait(lk, [&] { return r->done; });
    if (info) fill_info(*r, info);
    if (r->status != GP_OK && r->status != GP_ENOCONV) set_error(r->err);
    return r->status;
  });
}

int gp_server_poll(gp_server_t h, int64_t id, int* done) {
  return sguard([&] {
    if (!h || !done) throw Error{GP_EINVAL, "null argument"};
    Server& S = h->S;
    std::lock_guard<std::mutex> lk(S.mu);
    auto itr = S.all.find(id);
    if (itr == S.all.end()) throw Error{GP_EINVAL, "unknown request id"};
    *done = itr->second->done ? 1 : 0;
    return GP_OK;
  });
}

int gp_server_stats(gp_server_t h, gp_server_counters* st) {
  return sguard([&] {
    if (!h || !st) throw Error{GP_EINVAL, "null argument"};
    Server& S = h->S;
    std::lock_guard<std::mutex> lk(S.mu);
    st->submitted = S.next_id - 1;
    st->completed = S.completed;
    st->running = S.running;
    st->queued = (int64_t)S.queue.size();
    st->peak_running = S.peak_running;
    st->bytes_in_use = S.bytes_in_use;
    st->peak_bytes = S.peak_bytes;
    st->seconds = S.now();
    return GP_OK;
  });
}

int gp_server_destroy(gp_server_t h) {
  return sguard([&] {
    if (!h) return GP_OK;
    Server& S = h->S;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      S.stop = true;
    }
    S.cv_work.notify_all();
    for (auto& t : S.workers) t.join();
    for (auto st : S.streams) (void)hipStreamDestroy(st);
    if (S.qstream) (void)hipStreamDestroy(S.qstream);
    delete h;
    return GP_OK;
  });
}

}  // extern "C"
