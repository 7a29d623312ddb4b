// Request server: continuous batching of p-multigrid solves on one device.
//
// Classes (dim, degree, n_elem, geometry) own a set-up handle (operators and
// ILUT factors resident in HBM).  A request is queued at submit time; the
// scheduler thread admits it into a slot once its class is resident, a slot
// is free and its workspace fits the memory budget, and then advances every
// active request by one outer step per tick on the slot's own stream, polling
// completion with events.  Finished requests leave their slot at once and the
// next queued request takes it: the batch changes every tick.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "pmg_internal.hpp"

using pmgdev::fail;
using pmgdev::Workspace;

namespace {

using Key = std::tuple<int, int, int, int, int>;  // dim, degree, n_elem, geometry, pde

Key key_of(const pmg_problem& p) { return Key(p.dim, p.degree, p.n_elem, p.geometry, p.pde); }

// Closed-form estimate of a class's device footprint before it is set up:
// A_p, the ILUT factors (about twice nnz(A) under the per-part fill rule),
// both transfer matrices, FP32 copies in mixed precision, the degree-1
// hierarchy and vectors.
int64_t estimate_class_bytes(const pmg_problem& p, bool mixed) {
  const int64_t n1d = p.n_elem + p.degree - 2;
  const int64_t a1d = n1d * (2 * p.degree + 1) - (int64_t)p.degree * (p.degree + 1);
  const int64_t t1d = (int64_t)(p.n_elem - 1) * (p.degree + 2);
  int64_t nnzA = 1, nnzP = 1, n = 1, n1 = 1;
  for (int a = 0; a < p.dim; ++a) {
    nnzA *= a1d;
    nnzP *= t1d;
    n *= n1d;
    n1 *= (p.n_elem - 1);
  }
  const int64_t stencil1 = p.dim == 2 ? 9 : 27;
  int64_t b = 12 * (16 * nnzA / 5 + 2 * nnzP) + 16 * n * 4 + 12 * stencil1 * n1 * 4 / 3;
  if (mixed) b += 4 * (3 * nnzA + 2 * nnzP);
  return b;
}

struct Request {
  int64_t ticket = 0;
  pmg_problem prob{};
  std::vector<double> b, x;
  bool done = false;
  pmg_request_info info{};
};

struct ClassEntry {
  Key key;
  pmg_handle h = nullptr;
  bool ready = false, failed = false, setting_up = false;
  pmg_status setup_status = PMG_OK;
  int64_t bytes = 0;          // operators (estimate until set up)
  int active = 0, queued = 0; // requests using / waiting for the class
  double last_use = 0;
  std::vector<std::unique_ptr<Workspace>> free_ws;
  int64_t ws_bytes = 0;       // bytes of allocated workspaces of this class
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  std::shared_ptr<Request> req;
  ClassEntry* cls = nullptr;
  std::unique_ptr<Workspace> ws;
  int phase = 0;  // 0 idle, 1 initial residual in flight, 2 step in flight
  double r0 = 0;
  int it = 0;
};

}  // namespace

struct pmg_server_s {
  pmg_server_options opt{};
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_done, cv_setup, cv_idle;
  std::map<Key, std::unique_ptr<ClassEntry>> classes;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<int64_t, std::shared_ptr<Request>> requests;
  std::deque<ClassEntry*> setup_jobs;
  std::vector<Slot> slots;
  int max_slots = 1;
  int precision = PMG_FP32_IN_FP64;
  int64_t next_ticket = 1;
  int64_t bytes_in_use = 0;
  pmg_server_stats stats{};
  bool stop = false;
  std::thread sched, setup;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

  // Frees memory by destroying least recently used classes that no request
  // uses or waits for, until `need` bytes fit.  Caller holds mu.
  bool make_room(int64_t need, const ClassEntry* keep) {
    while (bytes_in_use + need > opt.budget_bytes) {
      ClassEntry* victim = nullptr;
      for (auto& kv : classes) {
        ClassEntry* c = kv.second.get();
        if (c == keep || !c->ready || c->active || c->queued || c->setting_up) continue;
        if (!victim || c->last_use < victim->last_use) victim = c;
      }
      if (!victim) return false;
      bytes_in_use -= victim->bytes + victim->ws_bytes;
      victim->free_ws.clear();
      pmg_destroy(victim->h);
      classes.erase(victim->key);
      stats.evictions++;
    }
    return true;
  }

  pmg_status setup_class(ClassEntry* c, std::unique_lock<std::mutex>& lk) {
    // runs with mu held on entry and exit; releases it around the host setup
    pmg_problem pr{};
    std::tie(pr.dim, pr.degree, pr.n_elem, pr.geometry, pr.pde) = c->key;
    pr.rhs_kind = PMG_RHS_SINE;
    pr.freq[0] = pr.freq[1] = pr.freq[2] = 1;
    pmg_options o;
    pmg_default_options(&o);
    o.precision = PMG_FP32_IN_FP64;  // handles carry FP64 and FP32 values
    o.device = opt.device;
    o.setup_threads = opt.setup_threads;
    o.max_iter = opt.max_iter;
    o.tri_waves_per_cu = opt.tri_waves_per_cu;
    c->setting_up = true;
    lk.unlock();
    auto t = std::chrono::steady_clock::now();
    pmg_handle h = nullptr;
    pmg_status st = pmg_setup(&pr, &o, &h);
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t).count();
    lk.lock();
    c->setting_up = false;
    stats.setup_seconds += secs;
    if (st != PMG_OK) {
      c->failed = true;
      c->setup_status = st;
      bytes_in_use -= c->bytes;
      c->bytes = 0;
      cv_setup.notify_all();
      return st;
    }
    pmg_info info;
    pmg_get_info(h, &info);
    bytes_in_use += info.device_bytes - c->bytes;
    c->bytes = info.device_bytes;
    c->h = h;
    c->ready = true;
    c->last_use = now();
    cv_setup.notify_all();
    return PMG_OK;
  }

  // Finds or creates the class of p, reserving its estimated bytes.  Caller
  // holds mu.  Returns EBUDGET if the class can never fit or does not fit now.
  pmg_status get_class(const pmg_problem& p, ClassEntry** out, bool& created) {
    created = false;
    auto it = classes.find(key_of(p));
    if (it != classes.end()) {
      *out = it->second.get();
      return it->second->failed ? it->second->setup_status : PMG_OK;
    }
    const int64_t est = estimate_class_bytes(p, true);
    if (est > opt.max_class_bytes || est > opt.budget_bytes)
      return fail(PMG_EBUDGET, "class estimated at " + std::to_string(est) + " bytes exceeds the class limit");
    if (!make_room(est, nullptr)) return fail(PMG_EBUDGET, "no room for the class in the device budget now");
    auto c = std::make_unique<ClassEntry>();
    c->key = key_of(p);
    c->bytes = est;
    bytes_in_use += est;
    *out = c.get();
    classes[c->key] = std::move(c);
    created = true;
    return PMG_OK;
  }

  void setup_loop() {
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
      if (setup_jobs.empty()) {
        cv_setup.wait_for(lk, std::chrono::milliseconds(20));
        continue;
      }
      ClassEntry* c = setup_jobs.front();
      setup_jobs.pop_front();
      if (c->ready || c->failed) continue;
      setup_class(c, lk);
    }
  }

  // Retires the request of slot s (its stream is idle).  Takes mu itself.
  void finish(Slot& s, pmg_status st, double rel) {
    Request& r = *s.req;
    hipMemcpyAsync(r.x.data(), s.ws->x, sizeof(double) * r.x.size(), hipMemcpyDeviceToHost, s.stream);
    hipStreamSynchronize(s.stream);
    std::lock_guard<std::mutex> lk(mu);
    r.info.status = st;
    r.info.iterations = s.it;
    r.info.relres = rel;
    r.info.t_finish = now();
    r.done = true;
    if (st == PMG_OK) stats.completed++; else stats.failed++;
    s.cls->active--;
    s.cls->last_use = now();
    s.cls->free_ws.push_back(std::move(s.ws));
    s.req.reset();
    s.cls = nullptr;
    s.phase = 0;
    cv_done.notify_all();
    cv_idle.notify_all();
  }

  void launch_step(Slot& s) {
    pmg_handle h = s.cls->h;
    pmgdev::outer_step(h, *s.ws, precision == PMG_FP32_IN_FP64, s.ws->b, s.ws->x, s.ws->r, true, s.stream);
    pmgdev::enqueue_norm_readback(*s.ws, s.stream);
    hipEventRecord(s.ev, s.stream);
    s.phase = 2;
  }

  // Moves queued requests into free slots (caller holds mu).  Returns the
  // slots that were filled; their device work is started by the caller.
  std::vector<int> admit() {
    std::vector<int> filled;
    for (auto qi = queue.begin(); qi != queue.end();) {
      auto req = *qi;
      auto ci = classes.find(key_of(req->prob));
      ClassEntry* c = ci == classes.end() ? nullptr : ci->second.get();
      if (!c || c->failed) {
        req->info.status = c ? c->setup_status : PMG_EBUDGET;
        req->info.t_finish = now();
        req->done = true;
        if (c) c->queued--;
        stats.failed++;
        qi = queue.erase(qi);
        cv_done.notify_all();
        cv_idle.notify_all();
        continue;
      }
      if (!c->ready) {
        ++qi;
        continue;
      }
      int free_slot = -1;
      for (int i = 0; i < max_slots; ++i)
        if (!slots[i].req) {
          free_slot = i;
          break;
        }
      if (free_slot < 0) break;
      Slot& s = slots[free_slot];
      std::unique_ptr<Workspace> ws;
      if (!c->free_ws.empty()) {
        ws = std::move(c->free_ws.back());
        c->free_ws.pop_back();
      } else {
        const int64_t wb = (int64_t)pmgdev::workspace_bytes(c->h, true, true);
        if (!make_room(wb, c)) {
          ++qi;
          continue;
        }
        ws.reset(new Workspace());
        if (pmgdev::alloc_workspace(c->h, *ws, true, true, s.stream) != PMG_OK) {
          ++qi;
          continue;
        }
        c->ws_bytes += (int64_t)ws->mem.bytes;
        bytes_in_use += (int64_t)ws->mem.bytes;
      }
      s.req = req;
      s.cls = c;
      s.ws = std::move(ws);
      s.it = 0;
      s.phase = 1;
      c->queued--;
      c->active++;
      req->info.t_admit = now();
      qi = queue.erase(qi);
      filled.push_back(free_slot);
    }
    return filled;
  }

  void sched_loop() {
    hipSetDevice(opt.device);
    for (;;) {
      std::vector<int> filled;
      int nslots;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (stop) break;
        filled = admit();
        nslots = max_slots;
      }
      bool progressed = !filled.empty();
      // start admitted requests: upload b, x = 0, initial residual and norm
      for (int i : filled) {
        Slot& s = slots[i];
        const Request& r = *s.req;
        hipMemcpyAsync(s.ws->b, r.b.data(), sizeof(double) * r.b.size(), hipMemcpyHostToDevice, s.stream);
        pmgdev::zero(s.ws->x, (int64_t)r.b.size(), s.stream);
        pmgdev::residual64(s.cls->h, *s.ws, s.ws->b, s.ws->x, s.ws->r, true, s.stream);
        pmgdev::enqueue_norm_readback(*s.ws, s.stream);
        hipEventRecord(s.ev, s.stream);
      }
      // advance active requests whose previous step has completed
      for (int i = 0; i < nslots; ++i) {
        Slot& s = slots[i];
        if (!s.req || hipEventQuery(s.ev) != hipSuccess) continue;
        progressed = true;
        if (pmgdev::take_fault(*s.ws, s.stream) != PMG_OK) { finish(s, PMG_EDEVICE, 1.0); continue; }
        const double nrm = std::sqrt(s.ws->host_scalar[0]);
        if (s.phase == 1) {
          s.r0 = nrm;
          if (!std::isfinite(nrm)) { finish(s, PMG_ENAN, 1.0); continue; }
          if (nrm == 0.0) { finish(s, PMG_OK, 0.0); continue; }
          launch_step(s);
          continue;
        }
        s.it++;
        const double rel = nrm / s.r0;
        if (!std::isfinite(rel) || rel > opt.diverge_ratio) { finish(s, PMG_EDIVERGED, rel); continue; }
        if (rel <= opt.tol) { finish(s, PMG_OK, rel); continue; }
        if (s.it >= opt.max_iter) { finish(s, PMG_EMAXIT, rel); continue; }
        launch_step(s);
      }
      if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
};

extern "C" {

pmg_status pmg_server_default_options(pmg_server_options* o) {
  if (!o) return fail(PMG_EINVAL, "NULL options");
  std::memset(o, 0, sizeof(*o));
  o->budget_bytes = 0;  // 70 % of the device's memory, taken at pmg_server_create
  o->max_class_bytes = 0;
  o->max_slots = 16;
  o->precision = PMG_FP32_IN_FP64;
  o->tol = 1e-10;
  o->max_iter = 100;
  o->device = 0;
  o->setup_threads = 0;
  o->diverge_ratio = 1e10;
  o->tri_waves_per_cu = 1;
  return PMG_OK;
}

pmg_status pmg_server_create(const pmg_server_options* o, pmg_server* out) {
  if (!out) return fail(PMG_EINVAL, "NULL out");
  *out = nullptr;
  pmg_server_options op;
  if (o) op = *o; else pmg_server_default_options(&op);
  if (op.budget_bytes < 0 || op.max_slots < 1 || op.max_slots > 256 || !(op.tol > 0) || op.max_iter < 1 ||
      !(op.diverge_ratio > 0) || (op.precision != PMG_FP64 && op.precision != PMG_FP32_IN_FP64) ||
      op.tri_waves_per_cu < 0)
    return fail(PMG_EINVAL, "invalid server options");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= op.device)
    return fail(PMG_EDEVICE, "no HIP device " + std::to_string(op.device));
  PMG_HIP_OK(hipSetDevice(op.device));
  if (op.budget_bytes == 0) {
    hipDeviceProp_t prop;
    PMG_HIP_OK(hipGetDeviceProperties(&prop, op.device));
    op.budget_bytes = (int64_t)((double)prop.totalGlobalMem * 0.7);
  }
  if (op.max_class_bytes <= 0) op.max_class_bytes = op.budget_bytes / 4;
  std::unique_ptr<pmg_server_s> s(new pmg_server_s());
  s->opt = op;
  s->t0 = std::chrono::steady_clock::now();
  s->max_slots = op.max_slots;
  s->precision = op.precision;
  s->slots.resize(256);
  for (int i = 0; i < op.max_slots; ++i) {
    PMG_HIP_OK(hipStreamCreateWithFlags(&s->slots[i].stream, hipStreamNonBlocking));
    PMG_HIP_OK(hipEventCreateWithFlags(&s->slots[i].ev, hipEventDisableTiming));
  }
  pmg_server_s* raw = s.get();
  s->sched = std::thread([raw] { raw->sched_loop(); });
  s->setup = std::thread([raw] { raw->setup_loop(); });
  *out = s.release();
  return PMG_OK;
}

pmg_status pmg_server_prepare(pmg_server s, const pmg_problem* prob) {
  if (!s || !prob) return fail(PMG_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  ClassEntry* c = nullptr;
  bool created = false;
  pmg_status st = s->get_class(*prob, &c, created);
  if (st != PMG_OK) return st;
  if (c->ready) return PMG_OK;
  if (created) return s->setup_class(c, lk);
  s->cv_setup.wait(lk, [&] { return c->ready || c->failed; });
  return c->ready ? PMG_OK : c->setup_status;
}

pmg_status pmg_server_submit(pmg_server s, const pmg_problem* prob, const double* b_host, int64_t* ticket) {
  if (!s || !prob || !ticket) return fail(PMG_EINVAL, "NULL argument");
  *ticket = -1;
  {
    std::string msg;
    if (!pmgdev::valid_problem(prob, msg)) return fail(PMG_EINVAL, msg);
  }
  const double submit_t = s->now();
  auto req = std::make_shared<Request>();
  req->prob = *prob;
  int64_t n = 1;
  for (int a = 0; a < prob->dim; ++a) n *= (prob->n_elem + prob->degree - 2);
  {
    std::unique_lock<std::mutex> lk(s->mu);
    ClassEntry* c = nullptr;
    bool created = false;
    pmg_status st = s->get_class(*prob, &c, created);
    if (st != PMG_OK) {
      s->stats.rejected++;
      return st;
    }
    if (created) {
      s->setup_jobs.push_back(c);
      s->cv_setup.notify_all();
    }
    c->queued++;
  }
  if (b_host) {
    req->b.assign(b_host, b_host + n);
  } else {
    pmg::SetupParams sp;
    sp.dim = prob->dim;
    sp.p = prob->degree;
    sp.nel = prob->n_elem;
    sp.geom = prob->geometry;
    sp.rhs = prob->rhs_kind;
    sp.pde = prob->pde;
    sp.fn = prob->f;
    sp.fn_ctx = prob->f_ctx;
    for (int a = 0; a < 3; ++a) sp.freq[a] = prob->freq[a] > 0 ? prob->freq[a] : 1;
    std::string msg;
    if (pmg::load_vector(sp, req->b, msg)) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->classes[key_of(*prob)]->queued--;
      return fail(PMG_EINVAL, msg);
    }
  }
  req->x.assign(n, 0.0);
  req->info.n = n;
  req->info.t_submit = submit_t;
  std::lock_guard<std::mutex> lk(s->mu);
  req->ticket = s->next_ticket++;
  s->requests[req->ticket] = req;
  s->queue.push_back(req);
  s->stats.submitted++;
  *ticket = req->ticket;
  return PMG_OK;
}

pmg_status pmg_server_wait(pmg_server s, int64_t ticket, double* x_host, pmg_request_info* info) {
  if (!s) return fail(PMG_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return fail(PMG_EINVAL, "unknown ticket");
  auto req = it->second;
  s->cv_done.wait(lk, [&] { return req->done; });
  if (x_host) std::memcpy(x_host, req->x.data(), sizeof(double) * req->x.size());
  if (info) *info = req->info;
  s->requests.erase(it);
  return (pmg_status)req->info.status;
}

pmg_status pmg_server_poll(pmg_server s, int64_t ticket, int32_t* done, double* x_host, pmg_request_info* info) {
  if (!s || !done) return fail(PMG_EINVAL, "NULL argument");
  *done = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return fail(PMG_EINVAL, "unknown ticket");
  auto req = it->second;
  if (!req->done) return PMG_OK;
  *done = 1;
  if (x_host) std::memcpy(x_host, req->x.data(), sizeof(double) * req->x.size());
  if (info) *info = req->info;
  s->requests.erase(it);
  return (pmg_status)req->info.status;
}

pmg_status pmg_server_configure(pmg_server s, int32_t max_slots, int32_t precision) {
  if (!s || max_slots < 1 || max_slots > 256 || (precision != PMG_FP64 && precision != PMG_FP32_IN_FP64))
    return fail(PMG_EINVAL, "invalid configuration");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_idle.wait(lk, [&] {
    if (!s->queue.empty()) return false;
    for (auto& sl : s->slots)
      if (sl.req) return false;
    return true;
  });
  for (int i = 0; i < max_slots; ++i) {
    if (!s->slots[i].stream) {
      PMG_HIP_OK(hipStreamCreateWithFlags(&s->slots[i].stream, hipStreamNonBlocking));
      PMG_HIP_OK(hipEventCreateWithFlags(&s->slots[i].ev, hipEventDisableTiming));
    }
  }
  s->max_slots = max_slots;
  s->precision = precision;
  return PMG_OK;
}

pmg_status pmg_server_get_stats(pmg_server s, pmg_server_stats* st) {
  if (!s || !st) return fail(PMG_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->stats;
  st->classes_resident = 0;
  for (auto& kv : s->classes) st->classes_resident += kv.second->ready ? 1 : 0;
  st->slots_active = 0;
  for (auto& sl : s->slots) st->slots_active += sl.req ? 1 : 0;
  st->queued = (int32_t)s->queue.size();
  st->bytes_in_use = s->bytes_in_use;
  return PMG_OK;
}

pmg_status pmg_server_get_options(pmg_server s, pmg_server_options* o) {
  if (!s || !o) return fail(PMG_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *o = s->opt;
  o->max_slots = s->max_slots;
  o->precision = s->precision;
  return PMG_OK;
}

double pmg_server_clock(pmg_server s) { return s ? s->now() : 0.0; }

pmg_status pmg_server_destroy(pmg_server s) {
  if (!s) return PMG_OK;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_idle.wait(lk, [&] {
      for (auto& sl : s->slots)
        if (sl.req) return false;
      return true;
    });
    s->stop = true;
    s->cv_setup.notify_all();
  }
  s->sched.join();
  s->setup.join();
  hipSetDevice(s->opt.device);
  hipDeviceSynchronize();
  for (auto& sl : s->slots) {
    if (sl.stream) hipStreamDestroy(sl.stream);
    if (sl.ev) hipEventDestroy(sl.ev);
  }
  for (auto& kv : s->classes) {
    kv.second->free_ws.clear();
    if (kv.second->h) pmg_destroy(kv.second->h);
  }
  delete s;
  return PMG_OK;
}

}  // extern "C"
