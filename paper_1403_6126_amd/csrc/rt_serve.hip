// Serving runtime declared in include/rt_serve.h: an HBM arena with
// first-fit allocation, an IO thread (admission by footprint, uploads,
// result downloads) and a scheduler thread (packed persistent launches of
// small requests, chunked per-step launches of the others, completion by
// event polling).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rt.h"
#include "rt_internal.hpp"
#include "rt_serve.h"

using namespace rtk;

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over one device block; free ranges kept sorted by
// offset and merged with their neighbours on release.
class Arena {
 public:
  bool init(size_t bytes) {
    size_ = bytes & ~(size_t)255;
    if (hipMalloc(&base_, size_) != hipSuccess) {
      base_ = nullptr;
      return false;
    }
    free_[0] = size_;
    return true;
  }
  void destroy() {
    if (base_) hipFree(base_);
    base_ = nullptr;
  }
  char *alloc(size_t n) {
    n = a256(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, rem = it->second - n;
      free_.erase(it);
      if (rem) free_[off + n] = rem;
      used_ += n;
      peak_ = std::max(peak_, used_);
      return base_ + off;
    }
    return nullptr;
  }
  void release(char *p, size_t n) {
    n = a256(n);
    size_t off = (size_t)(p - base_);
    used_ -= n;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        off = prev->first;
        n += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      free_.erase(next);
    }
    free_[off] = n;
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  char *base_ = nullptr;
  size_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

enum State { kQueued, kAdmitted, kRunning, kRetiring, kDone };

struct Request {
  long long id = 0;
  rt_request r{};
  std::vector<double> mu, w, ghost;
  rt_ctx ctx;
  size_t footprint = 0;
  char *block = nullptr;
  double *d_sa = nullptr, *d_ss = nullptr, *d_rho = nullptr, *d_T = nullptr, *d_v = nullptr;
  double *d_E = nullptr, *d_F = nullptr, *d_tot = nullptr;
  void *d_I[2] = {nullptr, nullptr};
  rt_fields fields{};
  rt_out out{};
  bool packed = false;
  bool large = false;
  int steps_issued = 0;
  int chunk = 1;
  hipEvent_t ev_ready = nullptr;
  hipEvent_t ev_chunk[2] = {nullptr, nullptr};
  int n_inflight = 0;
  int head = 0;  // oldest chunk event in flight
  hipEvent_t ev_done = nullptr;  // what retirement waits for
  std::atomic<int> state{kQueued};
  int status = RT_OK;
  double t_submit = 0, t_admit = 0, t_done = 0;
  double work = 0;
};

struct Batch {
  std::vector<Request *> reqs;
  hipEvent_t ev = nullptr;
  int slot = -1;
};

constexpr int kStageSlots = 8;
constexpr int kMaxBatch = 512;

}  // namespace

struct rt_server {
  rt_serve_config cfg{};
  int device = 0;
  Arena arena;
  hipStream_t s_io = nullptr, s_pack = nullptr, s_small = nullptr, s_large = nullptr;
  PackedJob *h_stage = nullptr;  // pinned [kStageSlots][kMaxBatch]
  PackedJob *d_stage = nullptr;
  bool slot_busy[kStageSlots] = {};
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;                  // guards the queues and the request map
  std::condition_variable cv_io;  // IO thread: new submissions or retirements
  std::condition_variable cv_sched;
  std::condition_variable cv_done;
  std::deque<Request *> pending;  // submitted, not admitted
  std::deque<Request *> ready;    // admitted, uploads queued
  std::deque<Request *> retire;   // finished on the device
  std::unordered_map<long long, std::unique_ptr<Request>> reqs;
  long long next_id = 1;
  bool stop = false;
  bool admit_blocked = false;  // the queue head did not fit; wait for a release
  std::thread io_thread, sched_thread;
  // counters
  long long submitted = 0, completed = 0, active = 0, peak_active = 0;
  long long packed_launches = 0, packed_requests = 0, chunk_launches = 0;
  double updates = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void io_loop();
  void sched_loop();
  bool admit_one(Request *q);
  void retire_one(Request *q);
};

namespace {

// Completion test of an event.  hipEventQuery reports "not ready" as an
// error that would otherwise be returned by the next hipGetLastError of
// this thread (the launch checks), so it is cleared here.
bool event_done(hipEvent_t e) {
  const hipError_t r = hipEventQuery(e);
  if (r == hipErrorNotReady) {
    (void)hipGetLastError();
    return false;
  }
  return r == hipSuccess;
}

hipEvent_t new_event() {
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Device footprint of a request: fields, outputs, intensities, context scratch.
size_t footprint_of(const rt_ctx &c) {
  const size_t nc = c.ncell, sb = ctx_storage_bytes(&c);
  size_t b = 0;
  b += 4 * a256(sizeof(double) * nc);          // sigma_a, sigma_s, rho, T
  b += a256(sizeof(double) * 3 * nc);          // v
  b += a256(sizeof(double) * nc);              // E_r
  b += a256(sizeof(double) * 3 * nc);          // F_r
  b += a256(sizeof(double) * kNtot);           // totals
  b += 2 * a256(sb * c.nang * nc);             // intensities
  b += ctx_scratch_bytes(&c);
  return b;
}

}  // namespace

// Carves the request's arrays from its arena block and queues the uploads
// and the preparation kernels on the IO stream.
bool rt_server::admit_one(Request *q) {
  rt_ctx &c = q->ctx;
  const size_t nc = c.ncell, sb = ctx_storage_bytes(&c);
  char *p = q->block;
  auto take = [&](size_t bytes) {
    char *at = p;
    p += a256(bytes);
    return at;
  };
  q->d_sa = (double *)take(sizeof(double) * nc);
  q->d_ss = (double *)take(sizeof(double) * nc);
  q->d_rho = (double *)take(sizeof(double) * nc);
  q->d_T = (double *)take(sizeof(double) * nc);
  q->d_v = (double *)take(sizeof(double) * 3 * nc);
  q->d_E = (double *)take(sizeof(double) * nc);
  q->d_F = (double *)take(sizeof(double) * 3 * nc);
  q->d_tot = (double *)take(sizeof(double) * kNtot);
  q->d_I[0] = take(sb * c.nang * nc);
  q->d_I[1] = take(sb * c.nang * nc);
  char *scratch = take(ctx_scratch_bytes(&c));
  const rt_request &r = q->r;
  hipStream_t s = s_io;
  bool ok = ctx_attach_scratch(&c, scratch, s) == RT_OK;
  auto up = [&](void *dst, const void *src, size_t bytes) {
    ok = ok && hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  up(q->d_sa, r.sigma_a, sizeof(double) * nc);
  up(q->d_ss, r.sigma_s, sizeof(double) * nc);
  up(q->d_rho, r.rho, sizeof(double) * nc);
  up(q->d_T, r.T, sizeof(double) * nc);
  up(q->d_v, r.v, sizeof(double) * 3 * nc);
  if (r.I0)
    up(q->d_I[0], r.I0, sb * c.nang * nc);
  else
    ok = ok && ctx_init_equilibrium(&c, q->d_T, q->d_I[0], s) == RT_OK;
  c.I[0] = q->d_I[0];
  c.I[1] = q->d_I[1];
  c.cur = 0;
  c.mom_cur = 0;
  q->fields.sigma_a = q->d_sa;
  q->fields.sigma_s = q->d_ss;
  q->fields.rho = q->d_rho;
  q->fields.T = q->d_T;
  q->fields.v = q->d_v;
  q->out.Er = q->d_E;
  q->out.Fr = q->d_F;
  q->out.totals = q->d_tot;
  ok = ok && ctx_moments(&c, s) == RT_OK;
  ok = ok && ctx_prepare_call(&c, r.dt, &q->fields, s) == RT_OK;
  q->ev_ready = new_event();
  q->ev_chunk[0] = new_event();
  q->ev_chunk[1] = new_event();
  ok = ok && q->ev_ready && q->ev_chunk[0] && q->ev_chunk[1];
  ok = ok && hipEventRecord(q->ev_ready, s) == hipSuccess;
  return ok;
}

// Copies the results to the caller's buffers (after the request's last
// kernel), reads the device status and releases the arena block.
void rt_server::retire_one(Request *q) {
  rt_ctx &c = q->ctx;
  const size_t nc = c.ncell, sb = ctx_storage_bytes(&c);
  hipStream_t s = s_io;
  bool ok = true;
  if (q->ev_done) ok = hipStreamWaitEvent(s, q->ev_done, 0) == hipSuccess;
  int dev_status = 0;
  auto down = [&](void *dst, const void *src, size_t bytes) {
    if (dst) ok = ok && hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) == hipSuccess;
  };
  if (q->block) {
    const int final_buf = q->packed ? (q->r.nsteps & 1) : c.cur;
    down(q->r.T_out, q->d_T, sizeof(double) * nc);
    down(q->r.Er, q->d_E, sizeof(double) * nc);
    down(q->r.Fr, q->d_F, sizeof(double) * 3 * nc);
    down(q->r.totals, q->d_tot, sizeof(double) * kNtot);
    down(q->r.I_out, q->d_I[final_buf], sb * c.nang * nc);
    down(&dev_status, c.status, sizeof(int));
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
  }
  if (q->status == RT_OK) {
    if (!ok)
      q->status = RT_EDEVICE;
    else if (dev_status)
      q->status = RT_ENOCONV;
  }
  for (hipEvent_t e : {q->ev_ready, q->ev_chunk[0], q->ev_chunk[1]})
    if (e) hipEventDestroy(e);
  q->ev_ready = q->ev_chunk[0] = q->ev_chunk[1] = nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (q->block) arena.release(q->block, q->footprint);
  q->block = nullptr;
  admit_blocked = false;
  q->t_done = now();
  q->ctx.h_mu.clear();
  q->ctx.h_w.clear();
  q->ctx.h_muf.clear();
  q->ctx.h_wf.clear();
  q->ctx.h_ghost.clear();
  q->state = kDone;
  completed += 1;
  active -= 1;
  if (q->status == RT_OK) updates += q->work;
}

void rt_server::io_loop() {
  hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_io.wait(lk, [&] {
      return stop || !retire.empty() ||
             (!pending.empty() && active < cfg.max_active && !admit_blocked);
    });
    if (!retire.empty()) {
      Request *q = retire.front();
      retire.pop_front();
      lk.unlock();
      retire_one(q);
      lk.lock();
      cv_done.notify_all();
      continue;
    }
    if (stop && pending.empty()) break;
    // admission in submission order: the head waits until it fits
    while (!pending.empty() && active < cfg.max_active) {
      Request *q = pending.front();
      char *blk = arena.alloc(q->footprint);
      if (!blk) {
        admit_blocked = true;
        break;
      }
      pending.pop_front();
      q->block = blk;
      active += 1;
      peak_active = std::max(peak_active, active);
      q->t_admit = now();
      q->state = kAdmitted;
      lk.unlock();
      const bool ok = admit_one(q);
      lk.lock();
      if (!ok) {
        q->status = RT_EDEVICE;
        q->ev_done = nullptr;
        retire.push_back(q);
        continue;
      }
      ready.push_back(q);
      cv_sched.notify_all();
      if (!retire.empty()) break;  // finished work first: it frees memory
    }
    if (stop && pending.empty() && retire.empty() && active == 0) break;
  }
}

void rt_server::sched_loop() {
  hipSetDevice(device);
  std::vector<Request *> running;  // chunked requests
  std::vector<Batch> batches;
  std::vector<Request *> to_pack;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      if (ready.empty() && running.empty() && batches.empty() && to_pack.empty()) {
        cv_sched.wait(lk, [&] { return stop || !ready.empty(); });
        if (stop && ready.empty()) break;
      }
      while (!ready.empty()) {
        Request *q = ready.front();
        ready.pop_front();
        q->state = kRunning;
        if (q->packed)
          to_pack.push_back(q);
        else
          running.push_back(q);
      }
    }
    bool progress = false;
    // packed launches: one per angle-group class and boundary class
    while (!to_pack.empty()) {
      int slot = -1;
      for (int i = 0; i < kStageSlots; ++i)
        if (!slot_busy[i]) {
          slot = i;
          break;
        }
      if (slot < 0) break;
      const int groups = to_pack.front()->ctx.shape.groups;
      const int waves = to_pack.front()->ctx.shape.waves;
      const bool per = to_pack.front()->ctx.all_periodic;
      Batch b;
      b.slot = slot;
      std::vector<Request *> rest;
      for (Request *q : to_pack) {
        if ((int)b.reqs.size() < kMaxBatch && q->ctx.shape.groups == groups &&
            q->ctx.shape.waves == waves && q->ctx.all_periodic == per)
          b.reqs.push_back(q);
        else
          rest.push_back(q);
      }
      to_pack.swap(rest);
      PackedJob *hj = h_stage + (size_t)slot * kMaxBatch;
      PackedJob *dj = d_stage + (size_t)slot * kMaxBatch;
      for (size_t i = 0; i < b.reqs.size(); ++i) {
        Request *q = b.reqs[i];
        rt_ctx &c = q->ctx;
        PackedJob &j = hj[i];
        std::memset(&j, 0, sizeof(j));
        ctx_fill_args(&c, q->r.dt, &q->fields, j.a);
        j.a.I_in = c.I[0];
        j.a.I_out = c.I[1];
        j.a.mom_in = c.mom[0];
        j.a.mom_out = c.mom[1];
        j.a.oE = q->d_E;
        j.a.oF = q->d_F;
        j.nsteps = q->r.nsteps;
        j.totals = q->d_tot;
        hipStreamWaitEvent(s_pack, q->ev_ready, 0);
      }
      bool ok = hipMemcpyAsync(dj, hj, sizeof(PackedJob) * b.reqs.size(), hipMemcpyHostToDevice,
                               s_pack) == hipSuccess;
      ok = ok && launch_packed_f32(dj, (int)b.reqs.size(), waves, groups, per, s_pack) == hipSuccess;
      b.ev = new_event();
      ok = ok && b.ev && hipEventRecord(b.ev, s_pack) == hipSuccess;
      slot_busy[slot] = true;
      for (Request *q : b.reqs) {
        q->ev_done = b.ev;
        if (!ok) q->status = RT_EDEVICE;
      }
      packed_launches += 1;
      packed_requests += (long long)b.reqs.size();
      batches.push_back(std::move(b));
      progress = true;
    }
    // chunked requests: keep up to two chunks in flight each.  Large
    // requests go one at a time in submission order (the oldest unfinished
    // one issues), the others round-robin, so that small and medium work
    // overlaps the large request on the device instead of queueing behind it
    // and the large ones keep their stand-alone service time.
    long long large_head = -1;
    for (Request *q : running)
      if (q->large && q->steps_issued < q->r.nsteps && q->status == RT_OK &&
          (large_head < 0 || q->id < large_head))
        large_head = q->id;
    std::vector<Request *> finished;
    for (size_t i = 0; i < running.size();) {
      Request *q = running[i];
      while (q->n_inflight > 0 && event_done(q->ev_chunk[q->head])) {
        q->head ^= 1;
        q->n_inflight -= 1;
        progress = true;
      }
      const int nsteps = q->r.nsteps;
      if (q->steps_issued >= nsteps || q->status != RT_OK) {
        if (q->n_inflight == 0) {
          finished.push_back(q);
          running[i] = running.back();
          running.pop_back();
          continue;
        }
      } else if (q->n_inflight < 2 && (!q->large || q->id == large_head)) {
        hipStream_t s = q->large ? s_large : s_small;
        if (q->steps_issued == 0) hipStreamWaitEvent(s, q->ev_ready, 0);
        const int k0 = q->steps_issued, k1 = std::min(nsteps, k0 + q->chunk);
        int st = ctx_step_range(&q->ctx, q->r.dt, &q->fields, &q->out, k0, k1, nsteps, s);
        const int slot = (q->head + q->n_inflight) & 1;
        if (st == RT_OK && hipEventRecord(q->ev_chunk[slot], s) != hipSuccess) st = RT_EDEVICE;
        if (st != RT_OK) {
          q->status = st;
        } else {
          q->ev_done = q->ev_chunk[slot];
          q->n_inflight += 1;
          q->steps_issued = k1;
          chunk_launches += 1;
        }
        progress = true;
      }
      ++i;
    }
    for (size_t i = 0; i < batches.size();) {
      if (event_done(batches[i].ev)) {
        for (Request *q : batches[i].reqs) finished.push_back(q);
        slot_busy[batches[i].slot] = false;
        // the IO thread waits on the event before it is destroyed below
        hipEventSynchronize(batches[i].ev);
        for (Request *q : batches[i].reqs) q->ev_done = nullptr;
        hipEventDestroy(batches[i].ev);
        batches[i] = std::move(batches.back());
        batches.pop_back();
        progress = true;
        continue;
      }
      ++i;
    }
    if (!finished.empty()) {
      std::lock_guard<std::mutex> lk(mu);
      for (Request *q : finished) {
        q->state = kRetiring;
        retire.push_back(q);
      }
      cv_io.notify_all();
    }
    if (!progress) {
      std::unique_lock<std::mutex> lk(mu);
      cv_sched.wait_for(lk, std::chrono::microseconds(50), [&] { return !ready.empty(); });
    }
  }
}

extern "C" {

int rt_serve_create(const rt_serve_config *cfg, rt_server **out) {
  if (!out) return RT_EINVAL;
  *out = nullptr;
  if (!cfg || cfg->pool_bytes < 4096 || cfg->max_active < 1 || cfg->packed_cells < 0 ||
      cfg->chunk_work < 1 || cfg->large_work < 1)
    return RT_EINVAL;
  rt_server *s = new (std::nothrow) rt_server();
  if (!s) return RT_ENOMEM;
  s->cfg = *cfg;
  hipGetDevice(&s->device);
  s->t0 = std::chrono::steady_clock::now();
  bool ok = s->arena.init(cfg->pool_bytes);
  ok = ok && hipStreamCreateWithFlags(&s->s_io, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&s->s_pack, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&s->s_small, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&s->s_large, hipStreamNonBlocking) == hipSuccess;
  const size_t stage = sizeof(PackedJob) * kStageSlots * kMaxBatch;
  ok = ok && hipHostMalloc((void **)&s->h_stage, stage, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMalloc((void **)&s->d_stage, stage) == hipSuccess;
  if (!ok) {
    if (s->h_stage) hipHostFree(s->h_stage);
    if (s->d_stage) hipFree(s->d_stage);
    for (hipStream_t st : {s->s_io, s->s_pack, s->s_small, s->s_large})
      if (st) hipStreamDestroy(st);
    s->arena.destroy();
    delete s;
    return RT_ENOMEM;
  }
  s->io_thread = std::thread([s] { s->io_loop(); });
  s->sched_thread = std::thread([s] { s->sched_loop(); });
  *out = s;
  return RT_OK;
}

int rt_serve_submit(rt_server *s, const rt_request *r, long long *id) {
  if (!s || !r || !id) return RT_EINVAL;
  *id = 0;
  if (r->nsteps < 1 || !r->sigma_a || !r->sigma_s || !r->rho || !r->T || !r->v)
    return RT_EINVAL;
  if (r->params.flags & RT_GAS_FEEDBACK) return RT_EUNSUPPORTED;
  std::unique_ptr<Request> q(new (std::nothrow) Request());
  if (!q) return RT_ENOMEM;
  q->r = *r;
  const int N = r->angles.n;
  if (N < 1 || N > RT_MAX_ANGLES || !r->angles.mu || !r->angles.w) return RT_EINVAL;
  q->mu.assign(r->angles.mu, r->angles.mu + 3 * (size_t)N);
  q->w.assign(r->angles.w, r->angles.w + N);
  rt_angles an{N, q->mu.data(), q->w.data()};
  int st = ctx_init_host(&r->grid, &an, &r->params, &q->ctx);
  if (st != RT_OK) return st;
  st = ctx_check_dt(&q->ctx, r->dt);
  if (st != RT_OK) return st;
  if (r->ghost) std::memcpy(q->ctx.h_ghost.data(), r->ghost, sizeof(double) * 6 * (size_t)N);
  q->r.angles = an;
  q->r.ghost = nullptr;
  q->ctx.owns_device = false;
  q->ctx.device = s->device;
  q->footprint = a256(footprint_of(q->ctx));
  if (q->footprint > s->arena.size()) return RT_ENOMEM;
  const double per_step = (double)q->ctx.ncell * (double)N;
  q->work = per_step * r->nsteps;
  q->packed = r->params.precision == RT_FP32_MIXED && q->ctx.ncell <= s->cfg.packed_cells &&
              q->ctx.shape.waves > 0 && !q->ctx.shape.second;
  q->large = per_step >= (double)s->cfg.large_work;
  q->chunk = (int)std::max(1.0, std::min((double)r->nsteps, (double)s->cfg.chunk_work / per_step));
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return RT_ESTATE;
  q->id = s->next_id++;
  q->t_submit = s->now();
  *id = q->id;
  s->pending.push_back(q.get());
  s->reqs.emplace(q->id, std::move(q));
  s->submitted += 1;
  s->cv_io.notify_all();
  return RT_OK;
}

static void fill_result(const Request *q, rt_serve_result *res) {
  if (!res) return;
  res->status = q->status;
  res->packed = q->packed ? 1 : 0;
  res->t_submit = q->t_submit;
  res->t_admit = q->t_admit;
  res->t_done = q->t_done;
}

int rt_serve_poll(rt_server *s, long long id, rt_serve_result *res) {
  if (!s) return RT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return RT_EINVAL;
  if (it->second->state != kDone) return RT_PENDING;
  fill_result(it->second.get(), res);
  return RT_OK;
}

int rt_serve_wait(rt_server *s, long long id, rt_serve_result *res) {
  if (!s) return RT_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return RT_EINVAL;
  Request *q = it->second.get();
  s->cv_done.wait(lk, [&] { return q->state == kDone; });
  fill_result(q, res);
  return RT_OK;
}

double rt_serve_now(rt_server *s) { return s ? s->now() : 0.0; }

int rt_serve_get_counters(rt_server *s, rt_serve_counters *c) {
  if (!s || !c) return RT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  c->submitted = s->submitted;
  c->completed = s->completed;
  c->active = s->active;
  c->peak_active = s->peak_active;
  c->pool_bytes = s->arena.size();
  c->pool_used = s->arena.used();
  c->peak_pool_used = s->arena.peak();
  c->packed_launches = s->packed_launches;
  c->packed_requests = s->packed_requests;
  c->chunk_launches = s->chunk_launches;
  c->cell_angle_updates = s->updates;
  return RT_OK;
}

int rt_serve_destroy(rt_server *s) {
  if (!s) return RT_EINVAL;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->completed == s->submitted; });
    s->stop = true;
    s->cv_io.notify_all();
    s->cv_sched.notify_all();
  }
  s->io_thread.join();
  s->sched_thread.join();
  hipDeviceSynchronize();
  hipHostFree(s->h_stage);
  hipFree(s->d_stage);
  for (hipStream_t st : {s->s_io, s->s_pack, s->s_small, s->s_large}) hipStreamDestroy(st);
  s->arena.destroy();
  delete s;
  return RT_OK;
}

}  // extern "C"
