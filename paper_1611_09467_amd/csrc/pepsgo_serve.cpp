// Request loop with continuous batching over device streams (the serving
// form of the per-sample evaluation).  One scheduler thread per server owns
// the streams, the device pool and every request in flight; callers only
// touch the incoming and completed queues.
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
#include <thread>
#include <vector>

#include "pepsgo.h"
#include "pepsgo_internal.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxStreams = 16;
constexpr int kMaxParts = 64;         // requests gathered into one launch at most
constexpr size_t kLatWindow = 65536;  // latencies kept for the percentiles
constexpr uint32_t kWarnFlags = PEPSGO_F_ZERO_PSI | PEPSGO_F_NONFINITE | PEPSGO_F_NEAR_TIE;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device region; offsets only.
class Pool {
 public:
  explicit Pool(size_t bytes) : size_(bytes) { free_[0] = bytes; }
  bool alloc(size_t n, size_t* off) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, at = it->first + n;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += n;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }

 private:
  size_t size_, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Req {
  uint64_t id;
  pepsgo_peps P;
  pepsgo_eval_params prm;
  int batch;
  const uint8_t* cfg;
  double* logabs;
  int8_t* sign;
  double* eloc;
  uint32_t* flags;
  double* grad;
  int nm;          // sites per configuration
  int64_t gel;     // gradient values per sample (0 without gradients)
  size_t per_ws;   // workspace bytes per sample
  int next = 0;    // first sample not yet handed to a chunk
  int inflight = 0;
  int status = PEPSGO_OK;
  uint32_t flag_or = 0;  // OR of the flags of its completed chunks
  int64_t t_submit = 0, t_start = 0;
};

struct Part {
  Req* r;
  int off, n;
};

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  std::vector<Part> parts;
  size_t off = 0, bytes = 0;
  uint32_t* d_or = nullptr;  // device: OR of each part's flags
  uint32_t* h_or = nullptr;  // pinned host copy, valid once ev has completed
};

bool same_work(const Req& a, const Req& b) {
  return a.P == b.P && a.prm.Dc == b.prm.Dc && a.prm.J1 == b.prm.J1 && a.prm.J2 == b.prm.J2 &&
         a.prm.precision == b.prm.precision && a.prm.grad_mode == b.prm.grad_mode &&
         a.prm.want_eloc == b.prm.want_eloc;
}

}  // namespace

struct pepsgo_server_ {
  int device;
  pepsgo_serve_config cfg;
  char* base = nullptr;  // device pool
  std::unique_ptr<Pool> pool;
  std::vector<Slot> slots;
  std::thread th;

  std::mutex mu;  // guards incoming, done, stop, outstanding
  std::condition_variable cv_done, cv_work;
  std::deque<std::unique_ptr<Req>> incoming;
  std::deque<pepsgo_serve_done> done;
  bool stop = false;
  int outstanding = 0;
  uint64_t next_id = 1;
  // service figures (guarded by mu)
  int64_t st_requests = 0, st_samples = 0, st_first = 0, st_last = 0;
  std::deque<double> st_lat_ms;

  // scheduler-thread state
  std::vector<std::unique_ptr<Req>> active;  // arrival order

  void run();
  bool launch(Slot& sl);
  void finish(Slot& sl, int status);
  void retire();
};

void pepsgo_server_::finish(Slot& sl, int status) {
  for (size_t k = 0; k < sl.parts.size(); ++k) {
    const Part& p = sl.parts[k];
    p.r->inflight -= 1;
    if (status != PEPSGO_OK && p.r->status == PEPSGO_OK) p.r->status = status;
    if (status == PEPSGO_OK) p.r->flag_or |= sl.h_or[k];
  }
  if (sl.bytes) pool->release(sl.off, sl.bytes);
  sl.parts.clear();
  sl.bytes = 0;
  sl.busy = false;
}

// Move finished requests (nothing left to hand out, nothing in flight) to
// the completed queue.
void pepsgo_server_::retire() {
  std::vector<pepsgo_serve_done> out;
  for (auto it = active.begin(); it != active.end();) {
    Req& r = **it;
    if (r.status != PEPSGO_OK) r.next = r.batch;  // stop handing out an erroneous request
    if (r.next == r.batch && r.inflight == 0) {
      pepsgo_serve_done d;
      d.id = r.id;
      d.status = r.status == PEPSGO_OK && (r.flag_or & kWarnFlags) ? PEPSGO_WARN_SAMPLES : r.status;
      d.batch = r.batch;
      d.t_submit_ns = r.t_submit;
      d.t_start_ns = r.t_start;
      d.t_done_ns = now_ns();
      out.push_back(d);
      it = active.erase(it);
    } else {
      ++it;
    }
  }
  if (!out.empty()) {
    std::lock_guard<std::mutex> g(mu);
    for (auto& d : out) {
      done.push_back(d);
      st_requests += 1;
      st_samples += d.batch;
      st_last = d.t_done_ns;
      st_lat_ms.push_back((double)(d.t_done_ns - d.t_submit_ns) * 1e-6);
      if (st_lat_ms.size() > kLatWindow) st_lat_ms.pop_front();
    }
    outstanding -= (int)out.size();
    cv_done.notify_all();
  }
}

bool pepsgo_server_::launch(Slot& sl) {
  // the pending request with the fewest chunks in flight, earliest first
  Req* r = nullptr;
  for (auto& q : active)
    if (q->next < q->batch && (!r || q->inflight < r->inflight)) r = q.get();
  if (!r) return false;
  bool idle = true;
  for (const Slot& o : slots) idle = idle && !o.busy;
  const int floor_n = idle ? 1 : std::max(1, cfg.min_chunk);

  int n = std::min(cfg.max_chunk, r->batch - r->next);
  std::vector<Part> parts;
  parts.push_back({r, r->next, n});
  int total = n;
  // fill the launch with samples of later requests doing the same work
  for (auto& q : active) {
    if (total >= cfg.max_chunk || (int)parts.size() >= kMaxParts) break;
    if (q.get() == r || q->next >= q->batch || !same_work(*q, *r)) continue;
    const int m = std::min(cfg.max_chunk - total, q->batch - q->next);
    parts.push_back({q.get(), q->next, m});
    total += m;
  }
  const size_t io = (size_t)r->nm + 8 + 1 + 8 + 4 + (size_t)r->gel * 8;
  size_t off = 0, bytes = 0;
  for (;;) {
    const bool staged = parts.size() > 1;
    bytes = align_up(r->per_ws * total) + (staged ? align_up(io * total) + 5 * kAlign : 0);
    if (pool->alloc(bytes, &off)) break;
    // short of memory: serve the first request alone, in a smaller chunk
    if (parts.size() > 1) {
      parts.resize(1);
      total = parts[0].n;
      continue;
    }
    if (total <= floor_n) return false;  // wait for memory to free up
    total = std::max(floor_n, total / 2);
    parts[0].n = total;
  }
  const bool staged = parts.size() > 1;
  const int64_t t = now_ns();
  for (const Part& p : parts) {
    p.r->next += p.n;
    p.r->inflight += 1;
    if (!p.r->t_start) p.r->t_start = t;
  }
  sl.parts = parts;
  sl.off = off;
  sl.bytes = bytes;
  sl.busy = true;

  char* blk = base + off;
  const size_t wsb = r->per_ws * total;
  const uint8_t* cfg_p;
  double *la, *el, *gr;
  int8_t* sg;
  uint32_t* fl;
  int rc = PEPSGO_OK;
  hipError_t e = hipSuccess;
  if (!staged) {
    const Part& p = parts[0];
    cfg_p = r->cfg + (int64_t)p.off * r->nm;
    la = r->logabs + p.off;
    sg = r->sign + p.off;
    el = r->eloc + p.off;
    fl = r->flags + p.off;
    gr = r->gel ? r->grad + (int64_t)p.off * r->gel : nullptr;
  } else {
    char* io_p = blk + align_up(wsb);
    la = reinterpret_cast<double*>(io_p);
    el = reinterpret_cast<double*>(io_p + align_up((size_t)total * 8));
    fl = reinterpret_cast<uint32_t*>(io_p + 2 * align_up((size_t)total * 8));
    sg = reinterpret_cast<int8_t*>(io_p + 2 * align_up((size_t)total * 8) + align_up((size_t)total * 4));
    uint8_t* c = reinterpret_cast<uint8_t*>(io_p + 2 * align_up((size_t)total * 8) +
                                            align_up((size_t)total * 4) + align_up((size_t)total));
    gr = r->gel ? reinterpret_cast<double*>(c + align_up((size_t)total * r->nm)) : nullptr;
    cfg_p = c;
    int at = 0;
    for (const Part& p : parts) {
      if (e == hipSuccess)
        e = hipMemcpyAsync(c + (int64_t)at * r->nm, p.r->cfg + (int64_t)p.off * r->nm,
                           (size_t)p.n * r->nm, hipMemcpyDeviceToDevice, sl.s);
      at += p.n;
    }
  }
  if (e == hipSuccess)
    rc = pepsgo_evaluate(r->P, &r->prm, total, cfg_p, la, sg, el, fl, gr, blk, wsb, sl.s);
  if (e == hipSuccess && rc == PEPSGO_OK && staged) {
    int at = 0;
    for (const Part& p : parts) {
      Req& q = *p.r;
      const size_t n8 = (size_t)p.n * 8;
      if (e == hipSuccess) e = hipMemcpyAsync(q.logabs + p.off, la + at, n8, hipMemcpyDeviceToDevice, sl.s);
      if (e == hipSuccess) e = hipMemcpyAsync(q.eloc + p.off, el + at, n8, hipMemcpyDeviceToDevice, sl.s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(q.flags + p.off, fl + at, (size_t)p.n * 4, hipMemcpyDeviceToDevice, sl.s);
      if (e == hipSuccess) e = hipMemcpyAsync(q.sign + p.off, sg + at, p.n, hipMemcpyDeviceToDevice, sl.s);
      if (e == hipSuccess && q.gel)
        e = hipMemcpyAsync(q.grad + (int64_t)p.off * q.gel, gr + (int64_t)at * q.gel, n8 * q.gel,
                           hipMemcpyDeviceToDevice, sl.s);
      at += p.n;
    }
  }
  if (e == hipSuccess && rc == PEPSGO_OK) {
    // OR of each part's flags, for the completion status
    int at = 0;
    for (size_t k = 0; k < parts.size() && e == hipSuccess; ++k) {
      const Part& p = parts[k];
      const uint32_t* f = staged ? fl + at : p.r->flags + p.off;
      e = pg::launch_flags_or(f, p.n, sl.d_or + k, sl.s);
      at += p.n;
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(sl.h_or, sl.d_or, parts.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                         sl.s);
  }
  if (e == hipSuccess && rc == PEPSGO_OK) e = hipEventRecord(sl.ev, sl.s);
  if (e != hipSuccess) rc = PEPSGO_EDEVICE;
  if (rc != PEPSGO_OK) {
    // nothing was recorded for this chunk: wait for what may have been queued, then fail it
    (void)hipStreamSynchronize(sl.s);
    finish(sl, rc);
  }
  return true;
}

void pepsgo_server_::run() {
  (void)hipSetDevice(device);
  for (;;) {
    bool stopping;
    {
      std::unique_lock<std::mutex> g(mu);
      bool busy = false;
      for (const Slot& s : slots) busy = busy || s.busy;
      if (incoming.empty() && active.empty() && !stop)
        cv_work.wait(g, [&] { return stop || !incoming.empty(); });
      while (!incoming.empty()) {
        active.push_back(std::move(incoming.front()));
        incoming.pop_front();
      }
      stopping = stop;
      (void)busy;
    }
    bool progressed = false;
    for (Slot& sl : slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipErrorNotReady) continue;
      finish(sl, q == hipSuccess ? PEPSGO_OK : PEPSGO_EDEVICE);
      progressed = true;
    }
    retire();
    for (Slot& sl : slots)
      if (!sl.busy && launch(sl)) progressed = true;
    retire();
    bool busy = false;
    for (const Slot& s : slots) busy = busy || s.busy;
    if (stopping && active.empty() && !busy) {
      std::lock_guard<std::mutex> g(mu);
      if (incoming.empty()) break;
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

extern "C" {

int pepsgo_serve_create(pepsgo_ctx ctx, const pepsgo_serve_config* cfg, pepsgo_server* out) {
  if (!ctx || !out) return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_create: NULL argument");
  pepsgo_serve_config c{};
  if (cfg) c = *cfg;
  if (c.pool_bytes == 0) c.pool_bytes = (size_t)4 << 30;
  if (c.streams == 0) c.streams = 4;
  if (c.max_chunk == 0) c.max_chunk = 2048;
  if (c.min_chunk == 0) c.min_chunk = 32;
  if (c.streams < 1 || c.streams > kMaxStreams || c.max_chunk < 1 || c.min_chunk < 1)
    return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_create: streams %d (1..%d), max_chunk %d, min_chunk %d",
                        c.streams, kMaxStreams, c.max_chunk, c.min_chunk);
  auto srv = std::make_unique<pepsgo_server_>();
  srv->device = pg::ctx_device(ctx);
  srv->cfg = c;
  if (hipSetDevice(srv->device) != hipSuccess)
    return pg::api_fail(PEPSGO_EDEVICE, "pepsgo_serve_create: hipSetDevice failed");
  if (hipMalloc(&srv->base, c.pool_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return pg::api_fail(PEPSGO_ENOMEM, "pepsgo_serve_create: cannot reserve a %zu-byte pool", c.pool_bytes);
  }
  srv->pool = std::make_unique<Pool>(c.pool_bytes);
  srv->slots.resize(c.streams);
  for (Slot& s : srv->slots) {
    if (hipStreamCreateWithFlags(&s.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&s.d_or, kMaxParts * sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc(&s.h_or, kMaxParts * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      for (Slot& t : srv->slots) {
        if (t.ev) (void)hipEventDestroy(t.ev);
        if (t.s) (void)hipStreamDestroy(t.s);
        if (t.d_or) (void)hipFree(t.d_or);
        if (t.h_or) (void)hipHostFree(t.h_or);
      }
      (void)hipFree(srv->base);
      return pg::api_fail(PEPSGO_EDEVICE, "pepsgo_serve_create: stream or event creation failed");
    }
  }
  pepsgo_server_* p = srv.release();
  p->th = std::thread([p] { p->run(); });
  *out = p;
  return PEPSGO_OK;
}

int pepsgo_serve_submit(pepsgo_server srv, pepsgo_peps peps, const pepsgo_eval_params* params,
                        int batch, const uint8_t* configs, double* logabs, int8_t* sign,
                        double* eloc, uint32_t* flags, double* grad, uint64_t* id) {
  if (!srv || !peps || !params || !id)
    return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_submit: NULL argument");
  if (batch < 0) return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_submit: batch %d < 0", batch);
  if (batch > 0 && (!configs || !logabs || !sign || !eloc || !flags))
    return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_submit: NULL buffer");
  if (params->grad_mode == PEPSGO_GRAD_PER_SAMPLE && batch > 0 && !grad)
    return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_submit: grad_mode PER_SAMPLE needs a grad buffer");
  size_t per = 0;
  int rc = pepsgo_workspace_bytes(peps, params, 1, &per);
  if (rc) return rc;
  int64_t gel = 0;
  rc = pepsgo_grad_layout(peps, &gel, nullptr);
  if (rc) return rc;
  auto r = std::make_unique<Req>();
  int N = 0, M = 0;
  pg::peps_shape(peps, &N, &M);
  r->P = peps;
  r->prm = *params;
  r->batch = batch;
  r->cfg = configs;
  r->logabs = logabs;
  r->sign = sign;
  r->eloc = eloc;
  r->flags = flags;
  r->grad = grad;
  r->nm = N * M;
  r->gel = params->grad_mode == PEPSGO_GRAD_PER_SAMPLE ? gel : 0;
  r->per_ws = per;
  if (align_up(per) > srv->pool->size())
    return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_submit: one sample needs %zu bytes, pool holds %zu",
                        per, srv->pool->size());
  r->t_submit = now_ns();
  std::lock_guard<std::mutex> g(srv->mu);
  if (srv->stop) return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_submit: server is stopping");
  if (srv->cfg.max_pending > 0 && srv->outstanding >= srv->cfg.max_pending)
    return pg::api_fail(PEPSGO_EBUSY, "pepsgo_serve_submit: %d requests pending (max_pending %d)",
                        srv->outstanding, srv->cfg.max_pending);
  if (srv->st_first == 0) srv->st_first = r->t_submit;
  r->id = srv->next_id++;
  *id = r->id;
  srv->outstanding += 1;
  srv->incoming.push_back(std::move(r));
  srv->cv_work.notify_one();
  return PEPSGO_OK;
}

int pepsgo_serve_poll(pepsgo_server srv, pepsgo_serve_done* out, int max, int64_t timeout_us) {
  if (!srv || (!out && max > 0) || max < 0)
    return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_poll: bad argument");
  std::unique_lock<std::mutex> g(srv->mu);
  if (srv->done.empty() && timeout_us > 0)
    srv->cv_done.wait_for(g, std::chrono::microseconds(timeout_us), [&] { return !srv->done.empty(); });
  int n = 0;
  while (n < max && !srv->done.empty()) {
    out[n++] = srv->done.front();
    srv->done.pop_front();
  }
  return n;
}

int pepsgo_serve_pending(pepsgo_server srv, int* requests) {
  if (!srv || !requests) return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_pending: NULL argument");
  std::lock_guard<std::mutex> g(srv->mu);
  *requests = srv->outstanding;
  return PEPSGO_OK;
}

int pepsgo_serve_stats(pepsgo_server srv, pepsgo_serve_stats_t* out, int reset) {
  if (!srv || !out) return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_stats: NULL argument");
  std::lock_guard<std::mutex> g(srv->mu);
  out->requests = srv->st_requests;
  out->samples = srv->st_samples;
  out->pending = srv->outstanding;
  std::vector<double> lat(srv->st_lat_ms.begin(), srv->st_lat_ms.end());
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double q) {
    if (lat.empty()) return 0.0;
    const size_t k = (size_t)std::min<double>((double)lat.size() - 1, q * (double)(lat.size() - 1) + 0.5);
    return lat[k];
  };
  out->p50_ms = pct(0.50);
  out->p99_ms = pct(0.99);
  const double span = (double)(srv->st_last - srv->st_first) * 1e-9;
  out->samples_per_s = span > 0.0 ? (double)srv->st_samples / span : 0.0;
  if (reset) {
    srv->st_requests = srv->st_samples = 0;
    srv->st_first = srv->st_last = 0;
    srv->st_lat_ms.clear();
  }
  return PEPSGO_OK;
}

int pepsgo_serve_destroy(pepsgo_server srv) {
  if (!srv) return pg::api_fail(PEPSGO_EINVAL, "pepsgo_serve_destroy: NULL server");
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  if (srv->th.joinable()) srv->th.join();
  (void)hipSetDevice(srv->device);
  for (Slot& s : srv->slots) {
    (void)hipStreamSynchronize(s.s);
    (void)hipEventDestroy(s.ev);
    (void)hipStreamDestroy(s.s);
    (void)hipFree(s.d_or);
    (void)hipHostFree(s.h_or);
  }
  (void)hipFree(srv->base);
  delete srv;
  return PEPSGO_OK;
}

}  // extern "C"
