// Serving loop over the operator ABI: resident operators under an HBM byte
// budget, per-operator request queues, continuous batching of the queued
// plane-wave requests of one operator into the right-hand sides of one
// ls_solve, and concurrent solves on different operators (one worker thread
// and HIP stream each).  Host-side scheduling only; every arithmetic step of
// a solve runs in the library's kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ls.h"

namespace {

struct Req {
  int64_t ticket = 0;
  uint64_t key = 0;
  double alpha = 0;
  int state = 0;                  // 0 queued, 1 running, 2 done
  ls_status status = LS_OK;
  std::vector<double> result;     // 2N doubles, operator point order
  ls_solve_stats stats{};
  double t_submit = 0, t_start = 0, t_done = 0;
  int batch = 0;
  int64_t N = 0;
};

struct SrvOp {
  ls_geometry g{};
  ls_params p{};
  ls_n2_fn n2 = nullptr;
  void* ctx = nullptr;
  double kappa = 0;
  ls_op* op = nullptr;            // null while not resident
  size_t bytes = 0;               // resident bytes (estimate until built)
  int64_t N = 0;                  // 0 until first built
  std::vector<double> xy;         // node coordinates, kept across evictions
  bool busy = false;
  size_t reserved = 0;            // solve memory reserved while busy
  uint64_t last_use = 0;
  std::deque<Req*> q;
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// unknowns of a star configuration before it is built: interior lattice
// nodes inside s < s_b plus the boundary patch grid
int64_t estimate_points(const ls_geometry& g) {
  const double area = M_PI * (1.0 + 0.5 * g.shape_a * g.shape_a);
  const int64_t np = g.n_patches > 1 ? g.n_patches : 1;
  return (int64_t)(area * g.s_b * g.s_b / (g.h * g.h)) + np * (int64_t)(g.N1 + 1) * (g.N2 + 1);
}

}  // namespace

struct ls_server {
  size_t budget = 0;
  ls_server_opts o{};
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  std::map<uint64_t, SrvOp> ops;
  std::map<int64_t, std::unique_ptr<Req>> reqs;
  int64_t next_ticket = 0;
  uint64_t clock = 0;
  int64_t evictions = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  // bytes a solve of nrhs right-hand sides needs besides the operator: its
  // workspace (exact once the operator exists, else an estimate) and the
  // right-hand sides and solutions
  size_t solve_bytes(const SrvOp& e, int64_t N, int nrhs) const {
    size_t ws = 0;
    ls_solve_opts so{};
    so.restart = o.restart;
    if (e.op && ls_solve_workspace_size(e.op, nrhs, &so, &ws) == LS_OK) return ws + (size_t)32 * N * nrhs;
    return (size_t)16 * N * nrhs * (o.restart + 9) + ((size_t)64 << 20) * nrhs;
  }
  size_t op_bytes(const SrvOp& e, int64_t n) const { return e.op || e.bytes ? e.bytes : (size_t)n * 8000; }
  // resident operators, those being built (their estimate) and the solve
  // memory reserved by running solves
  size_t resident() const {
    size_t s = 0;
    for (auto& kv : ops) {
      if (kv.second.op || kv.second.busy) s += kv.second.bytes;
      if (kv.second.busy) s += kv.second.reserved;
    }
    return s;
  }
  // lock held: make room for op `e` and a solve of *R right-hand sides
  // (lowered when only fewer fit).  1 = admitted, 0 = wait (others are busy),
  // -1 = the operator (its exact size, known once it has been built) and a
  // one-right-hand-side solve alone exceed the budget.  An operator never
  // built is admitted on its size estimate, or, when the estimate alone is
  // over the budget, once nothing else is resident or busy: its exact size
  // is checked right after the build.
  int admit(uint64_t key, SrvOp& e, int* R) {
    const bool exact = e.N != 0;
    const int64_t n = exact ? e.N : estimate_points(e.g);
    const size_t ob = op_bytes(e, n);
    if (exact && ob + solve_bytes(e, n, 1) > budget) return -1;
    while (true) {
      const size_t cur = resident() + (e.op ? 0 : ob);
      int r = *R;
      while (r > 1 && cur + solve_bytes(e, n, r) > budget) --r;
      // evict while the whole batch does not fit and something idle can go
      SrvOp* victim = nullptr;
      if (cur + solve_bytes(e, n, *R) > budget)
        for (int pass = 0; pass < 2 && !victim; ++pass)
          for (auto& kv : ops) {
            SrvOp& c = kv.second;
            if (kv.first == key || !c.op || c.busy || (pass == 0 && !c.q.empty())) continue;
            if (!victim || c.last_use < victim->last_use) victim = &c;
          }
      if (victim) {
        ls_destroy(victim->op);
        victim->op = nullptr;
        ++evictions;
        continue;
      }
      if (cur + solve_bytes(e, n, r) > budget) {
        bool alone = !e.op;
        for (auto& kv : ops)
          if (kv.first != key && (kv.second.op || kv.second.busy)) alone = false;
        if (exact || !alone) return 0;
        r = 1;                         // learn the exact size by building it
      }
      if (!e.op) e.bytes = ob;       // counted while it is being built
      *R = r;
      e.reserved = solve_bytes(e, n, r);
      return 1;
    }
  }
  // lock held, after e was built: right-hand sides of a batch of R that fit
  // with the exact sizes (0: not even one)
  int fit_after_build(uint64_t key, SrvOp& e, int R) {
    size_t others = 0;
    for (auto& kv : ops)
      if (kv.first != key) {
        if (kv.second.op || kv.second.busy) others += kv.second.bytes;
        if (kv.second.busy) others += kv.second.reserved;
      }
    int r = R;
    while (r > 0 && others + e.bytes + solve_bytes(e, e.N, r) > budget) --r;
    if (r == 0 && e.bytes + solve_bytes(e, e.N, 1) <= budget) r = 1;   // fits once the others finish
    return r;
  }
  // lock held: the idle operator whose oldest queued request is the oldest
  SrvOp* pick(uint64_t* key) {
    SrvOp* best = nullptr;
    for (auto& kv : ops) {
      SrvOp& c = kv.second;
      if (c.busy || c.q.empty()) continue;
      if (!best || c.q.front()->ticket < best->q.front()->ticket) {
        best = &c;
        *key = kv.first;
      }
    }
    return best;
  }

  void worker() {
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      uint64_t key = 0;
      SrvOp* e = nullptr;
      while (!stop && !(e = pick(&key))) cv.wait(lk);
      if (stop) break;
      int nb = std::min<int>((int)e->q.size(), o.max_batch);
      const int adm = admit(key, *e, &nb);
      if (adm == 0) {
        cv.wait_for(lk, std::chrono::milliseconds(20));
        continue;
      }
      if (adm < 0) {
        // can never fit: every queued request of this operator fails
        const double td = now_s(t0);
        for (Req* r : e->q) {
          r->status = LS_EBUDGET;
          r->state = 2;
          r->t_start = r->t_done = td;
        }
        e->q.clear();
        cv.notify_all();
        continue;
      }
      std::vector<Req*> batch;
      while (!e->q.empty() && (int)batch.size() < nb) {
        batch.push_back(e->q.front());
        e->q.pop_front();
      }
      e->busy = true;
      const double ts = now_s(t0);
      for (Req* r : batch) {
        r->state = 1;
        r->t_start = ts;
      }
      lk.unlock();
      ls_status s = LS_OK;
      if (!e->op) {
        // build outside the lock (host set-up takes seconds), publish under it
        ls_op* op = nullptr;
        s = ls_create(&e->g, e->n2, e->ctx, e->kappa, &e->p, nullptr, &op);
        if (s == LS_OK) {
          int64_t n = 0;
          (void)ls_num_points(op, &n);
          std::vector<double> xy;
          if (e->xy.empty()) {
            xy.resize(2 * (size_t)n);
            (void)ls_points(op, xy.data(), nullptr);
          }
          std::lock_guard<std::mutex> g2(mu);
          e->op = op;
          e->bytes = ls_resident_bytes(op);
          e->N = n;
          if (e->xy.empty()) e->xy.swap(xy);
          // exact sizes: drop the operator if even one right-hand side can
          // never fit, hand back the requests that do not fit now
          const int rf = fit_after_build(key, *e, (int)batch.size());
          if (rf == 0) {
            ls_destroy(e->op);
            e->op = nullptr;
            s = LS_EBUDGET;
          } else {
            while ((int)batch.size() > rf) {
              Req* back = batch.back();
              batch.pop_back();
              back->state = 0;
              e->q.push_front(back);
            }
            e->reserved = solve_bytes(*e, n, rf);
          }
        }
      }
      const int R = (int)batch.size();
      const int64_t N = e->N;
      ls_solve_stats stats{};
      std::vector<double> host;
      if (s == LS_OK) {
        // plane waves exp(i kappa (cos a, sin a) . x) at the nodes, [R][N]
        host.resize(2 * (size_t)R * N);
        for (int r = 0; r < R; ++r) {
          const double cx = std::cos(batch[r]->alpha) * e->kappa, cy = std::sin(batch[r]->alpha) * e->kappa;
          double* h = host.data() + 2 * (size_t)r * N;
          for (int64_t i = 0; i < N; ++i) {
            const double ph = cx * e->xy[2 * i] + cy * e->xy[2 * i + 1];
            h[2 * i] = std::cos(ph);
            h[2 * i + 1] = std::sin(ph);
          }
        }
        void *F = nullptr, *X = nullptr, *W = nullptr;
        const size_t bytes = 16 * (size_t)R * N;
        ls_solve_opts so{};
        so.tol = o.tol;
        so.max_iter = o.max_iter;
        so.restart = o.restart;
        so.mode = o.mode;
        so.inner_tol = o.inner_tol;
        so.max_outer = o.max_outer;
        so.ortho = o.ortho;
        size_t wsb = 0;
        if (ls_solve_workspace_size(e->op, R, &so, &wsb) != LS_OK) {
          s = LS_EINVAL;
        } else if (hipMalloc(&F, bytes) != hipSuccess || hipMalloc(&X, bytes) != hipSuccess ||
                   hipMalloc(&W, wsb) != hipSuccess) {
          s = LS_ENOMEM;
        } else if (hipMemcpyAsync(F, host.data(), bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
          s = LS_EDEVICE;
        } else {
          s = ls_solve(e->op, F, X, R, &so, &stats, W, wsb, st);
          if ((s == LS_OK || s == LS_ENOCONV) &&
              (hipMemcpyAsync(host.data(), X, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
               hipStreamSynchronize(st) != hipSuccess))
            s = LS_EDEVICE;
        }
        if (F) (void)hipFree(F);
        if (X) (void)hipFree(X);
        if (W) (void)hipFree(W);
      }
      lk.lock();
      const double td = now_s(t0);
      for (int r = 0; r < R; ++r) {
        Req* q = batch[r];
        q->status = s;
        q->stats = stats;
        q->batch = R;
        q->N = N;
        q->t_done = td;
        if (s == LS_OK || s == LS_ENOCONV)
          q->result.assign(host.begin() + 2 * (size_t)r * N, host.begin() + 2 * (size_t)(r + 1) * N);
        q->state = 2;
      }
      e->busy = false;
      e->reserved = 0;
      e->last_use = ++clock;
      cv.notify_all();
    }
    lk.unlock();
    (void)hipStreamDestroy(st);
  }
};

extern "C" {

ls_status ls_server_create(size_t budget_bytes, const ls_server_opts* opts, ls_server** out) {
  if (!out || !opts || opts->max_batch < 1 || opts->workers < 1 || opts->restart < 1 || opts->max_iter < 1 ||
      !(opts->tol > 0))
    return LS_EINVAL;
  auto* s = new ls_server();
  s->budget = budget_bytes;
  s->o = *opts;
  s->t0 = std::chrono::steady_clock::now();
  (void)hipGetDevice(&s->device);
  for (int i = 0; i < opts->workers; ++i) s->workers.emplace_back([s] { s->worker(); });
  *out = s;
  return LS_OK;
}

ls_status ls_server_add_operator(ls_server* s, uint64_t key, const ls_geometry* geom, ls_n2_fn n2, void* ctx,
                                 double kappa, const ls_params* params) {
  if (!s || !geom || !n2 || !params || !(kappa > 0)) return LS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->ops.count(key)) return LS_EINVAL;
  SrvOp& e = s->ops[key];
  e.g = *geom;
  e.p = *params;
  e.p.skip_tiles = 1;   // the server does not tune its operators, so batches use the row kernels
  e.n2 = n2;
  e.ctx = ctx;
  e.kappa = kappa;
  return LS_OK;
}

ls_status ls_server_submit(ls_server* s, uint64_t key, double alpha, int64_t* ticket) {
  if (!s || !ticket) return LS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->ops.find(key);
  if (it == s->ops.end()) return LS_EINVAL;
  auto r = std::make_unique<Req>();
  r->ticket = s->next_ticket++;
  r->key = key;
  r->alpha = alpha;
  r->t_submit = now_s(s->t0);
  it->second.q.push_back(r.get());
  *ticket = r->ticket;
  s->reqs[r->ticket] = std::move(r);
  s->cv.notify_all();
  return LS_OK;
}

ls_status ls_server_poll(ls_server* s, int64_t ticket, double* u_tot, int64_t cap, ls_request_info* info) {
  if (!s) return LS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return LS_EINVAL;
  Req& r = *it->second;
  if (r.state != 2) return LS_ENOTREADY;
  if (info) {
    info->N = r.N;
    info->batch = r.batch;
    info->stats = r.stats;
    info->t_submit = r.t_submit;
    info->t_start = r.t_start;
    info->t_done = r.t_done;
  }
  if (u_tot && !r.result.empty()) {
    if (cap < 2 * r.N) return LS_EINVAL;
    std::memcpy(u_tot, r.result.data(), r.result.size() * sizeof(double));
  }
  return r.status;
}

ls_status ls_server_release(ls_server* s, int64_t ticket) {
  if (!s) return LS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->state != 2) return LS_EINVAL;
  s->reqs.erase(it);
  return LS_OK;
}

ls_status ls_server_points(ls_server* s, uint64_t key, double* xy, int64_t cap, int64_t* N) {
  if (!s || !N) return LS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->ops.find(key);
  if (it == s->ops.end()) return LS_EINVAL;
  if (it->second.xy.empty()) return LS_ENOTREADY;
  *N = it->second.N;
  if (xy) {
    if (cap < 2 * it->second.N) return LS_EINVAL;
    std::memcpy(xy, it->second.xy.data(), it->second.xy.size() * sizeof(double));
  }
  return LS_OK;
}

ls_status ls_server_stats(ls_server* s, ls_server_info* info) {
  if (!s || !info) return LS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  info->resident_bytes = s->resident();
  info->resident_ops = 0;
  info->queued = 0;
  info->running = 0;
  for (auto& kv : s->ops) {
    if (kv.second.op) ++info->resident_ops;
    info->queued += (int64_t)kv.second.q.size();
  }
  for (auto& kv : s->reqs)
    if (kv.second->state == 1) ++info->running;
  info->evictions = s->evictions;
  return LS_OK;
}

void ls_server_destroy(ls_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->ops)
    if (kv.second.op) ls_destroy(kv.second.op);
  delete s;
}

}  // extern "C"
