// Serving loop (include/ckks.h, ckks_server_*): continuous batching of
// key-switching jobs under an HBM budget.
//
// Requests are queued by ckks_server_submit from any host thread.  One worker
// thread repeatedly (1) retires finished batches (their HIP event has
// completed), releasing the jobs' scratch and marking their tickets done, and
// (2) admits queued jobs in arrival order, as long as fewer than max_slots
// jobs are on the device and each job's scratch fits in the arena (a device
// buffer of hbm_budget bytes allocated at creation), then launches the
// admitted group as one batch through the job-table pipeline on the next of
// several streams.  A request that arrives while earlier batches run is
// admitted as soon as slots and memory free up, and its batch overlaps with
// the ones already on the device.  Each job has private scratch and the
// arithmetic is exact, so a job's result does not depend on what it was
// batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "ctx.h"
#include "keyswitch.h"

using namespace ckks;

namespace ckks {
int api_fail(int code, const std::string& msg);
uint32_t api_galois(const Ctx& c, int rot);
}  // namespace ckks

namespace {

constexpr int kStreams = 3;
constexpr int kRing = 16;  // batches that may be in flight at once
constexpr size_t kAlignB = 256;

size_t align_up(size_t b) { return (b + kAlignB - 1) / kAlignB * kAlignB; }

double now_us(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
}

// First-fit allocator over [0, size) of the device arena.
struct Arena {
  size_t size = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t n) {
    size = n;
    free_.clear();
    if (n) free_[0] = n;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t o = it->first;
        free_.erase(it);
        if (rest) free_[o + n] = rest;
        used += n;
        peak = std::max(peak, used);
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    used -= n;
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
};

struct Req {
  uint64_t ticket;
  int ctx;
  ckks_job job;
  size_t bytes;      // scratch (from the arena)
  size_t io_bytes;   // inputs and output
  size_t key_bytes;  // the key array (0 for rescale)
  hipEvent_t ready;  // recorded on the submitter's stream: the job's inputs are written
  void* src;         // that stream
};

struct Flight {
  int ring;
  int stream;
  hipEvent_t ev;
  std::vector<uint64_t> tickets;
  // the jobs' submit events and streams (until the waits are enqueued)
  std::vector<std::pair<void*, hipEvent_t>> ready;
  std::vector<std::pair<size_t, size_t>> allocs;
  size_t io_bytes = 0;                // whole-footprint mode: inputs and outputs
  std::vector<const void*> keys;      // whole-footprint mode: key references
  int ks_jobs;
};

}  // namespace

struct ckks_server {
  std::vector<const Ctx*> ctxs;
  int device = 0;
  size_t budget = 0;
  int max_slots = 0;
  void* d_arena = nullptr;
  Arena arena;
  hipStream_t streams[kStreams] = {};
  int next_stream = 0;
  // per ring slot: device and pinned host job tables of max_slots entries
  KsJob* d_ks[kRing] = {};
  RsJob* d_rs[kRing] = {};
  KsJob* h_ks[kRing] = {};
  RsJob* h_rs[kRing] = {};
  bool ring_busy[kRing] = {};
  hipEvent_t events[kRing] = {};

  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  int error = 0;
  std::string error_msg;

  std::deque<Req> pending;
  std::deque<Flight> inflight;
  // Events that order a job after the work its submitter queued before it
  // (recorded by ckks_server_submit on the submitter's stream, waited on by
  // the batch's stream before the job-table copy).  Returned to the pool once
  // the wait is enqueued: a later record does not affect an enqueued wait.
  std::vector<hipEvent_t> event_pool;
  std::vector<hipEvent_t> all_events;
  int jobs_on_device = 0;
  // whole-footprint accounting (ckks_server_set_accounting): the budget also
  // covers the in-flight jobs' inputs and outputs and each distinct key once
  int whole = 0;
  size_t io_used = 0, key_used = 0, total_peak = 0;
  std::map<const void*, std::pair<int, size_t>> key_refs;  // key -> (in-flight jobs, bytes)
  uint64_t next_ticket = 0;
  std::vector<double> t_submit, t_done;  // by ticket; t_done < 0 while pending
  std::vector<uint8_t> is_ks;
  uint64_t completed = 0, completed_ks = 0, rejected = 0, batches = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  size_t job_bytes(const Ctx& c, const ckks_job& j) const {
    return align_up((j.op == CKKS_JOB_RESCALE ? rs_ws_words(c, j.L) : ks_ws_words(c, j.L)) * 4);
  }
  // Inputs and output of a job (limbs of N words): ct [2][L] in (d [L] for a
  // plain key-switch, a second ct for HMult), [2][L] out ([2][L-1] rescale).
  static size_t io_bytes_of(const Ctx& c, const ckks_job& j) {
    const size_t limb = (size_t)c.N * 4, L = (size_t)j.L;
    switch (j.op) {
      case CKKS_JOB_KEYSWITCH: return (L + 2 * L) * limb;
      case CKKS_JOB_HMULT: return (4 * L + 2 * L) * limb;
      case CKKS_JOB_RESCALE: return (2 * L + 2 * (L - 1)) * limb;
      default: return (2 * L + 2 * L) * limb;
    }
  }
  // The whole key array the job names: [beta_max][2][L_max + k] limbs.
  static size_t key_bytes_of(const Ctx& c, const ckks_job& j) {
    return j.op == CKKS_JOB_RESCALE ? 0 : (size_t)c.beta_max() * 2 * (c.L_max + c.k) * c.N * 4;
  }
  size_t total_used() const { return arena.used + io_used + key_used; }

  void retire_locked() {
    while (!inflight.empty()) {
      Flight& f = inflight.front();
      const hipError_t q = hipEventQuery(f.ev);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess && !error) {
        error = CKKS_EHIP;
        error_msg = std::string("batch failed: ") + hipGetErrorString(q);
      }
      const double t = now_us(t0);
      for (uint64_t tk : f.tickets) {
        t_done[tk] = t;
        ++completed;
        completed_ks += is_ks[tk];
      }
      for (auto& a : f.allocs) arena.release(a.first, a.second);
      io_used -= f.io_bytes;
      for (const void* k : f.keys) {
        auto it = key_refs.find(k);
        if (it != key_refs.end() && --it->second.first == 0) {
          key_used -= it->second.second;
          key_refs.erase(it);
        }
      }
      jobs_on_device -= (int)f.tickets.size();
      ring_busy[f.ring] = false;
      inflight.pop_front();
      cv_done.notify_all();
    }
  }

  // Admit the longest FIFO prefix of one context's jobs that fits; launch it.
  bool admit_locked() {
    if (pending.empty() || error) return false;
    int ring = -1;
    for (int i = 0; i < kRing; ++i)
      if (!ring_busy[i]) {
        ring = i;
        break;
      }
    if (ring < 0) return false;
    const int ci = pending.front().ctx;
    const Ctx& c = *ctxs[ci];
    Flight f;
    f.ring = ring;
    f.ks_jobs = 0;
    int nks = 0, nrs = 0, Lks = 0, Lrs = 0;
    while (!pending.empty() && pending.front().ctx == ci && jobs_on_device + nks + nrs < max_slots) {
      Req& r = pending.front();
      if (whole) {
        const bool new_key = r.key_bytes && key_refs.find(r.job.key) == key_refs.end();
        if (total_used() + r.bytes + r.io_bytes + (new_key ? r.key_bytes : 0) > budget) break;
      }
      size_t off;
      if (!arena.alloc(r.bytes, &off)) break;
      if (whole) {
        io_used += r.io_bytes;
        f.io_bytes += r.io_bytes;
        if (r.key_bytes) {
          auto& ref = key_refs[r.job.key];
          if (ref.first++ == 0) {
            ref.second = r.key_bytes;
            key_used += r.key_bytes;
          }
          f.keys.push_back(r.job.key);
        }
        total_peak = std::max(total_peak, total_used());
      }
      uint32_t* ws = (uint32_t*)((char*)d_arena + off);
      const ckks_job& j = r.job;
      if (j.op == CKKS_JOB_RESCALE) {
        h_rs[ring][nrs++] = RsJob{j.L, {0, 0, 0}, j.in0, j.out, ws, nullptr};
        Lrs = std::max(Lrs, j.L);
      } else {
        const int kind = j.op == CKKS_JOB_KEYSWITCH ? KS_PLAIN : j.op == CKKS_JOB_HMULT ? KS_HMULT : KS_HROT;
        h_ks[ring][nks++] = KsJob{kind, j.L, j.op == CKKS_JOB_HROT ? api_galois(c, j.rot) : 0u, 0, j.in0,
                                  j.op == CKKS_JOB_HMULT ? j.in1 : nullptr, j.key, j.out, ws};
        Lks = std::max(Lks, j.L);
      }
      f.tickets.push_back(r.ticket);
      f.allocs.emplace_back(off, r.bytes);
      f.ready.emplace_back(r.src, r.ready);
      pending.pop_front();
    }
    if (f.tickets.empty()) return false;
    const hipStream_t st = streams[next_stream];
    f.stream = next_stream;
    next_stream = (next_stream + 1) % kStreams;
    hipError_t e = hipSuccess;
    // per submitting stream, the event of its last job in the batch covers the
    // earlier ones (recorded in submit order on that stream)
    for (size_t i = 0; i < f.ready.size() && e == hipSuccess; ++i) {
      bool later = false;
      for (size_t k = i + 1; k < f.ready.size(); ++k) later = later || f.ready[k].first == f.ready[i].first;
      if (!later) e = hipStreamWaitEvent(st, f.ready[i].second, 0);
    }
    for (auto& rv : f.ready) event_pool.push_back(rv.second);
    f.ready.clear();
    // up to kInlineJobs jobs travel in the kernel arguments; larger groups
    // through the ring slot's device table
    if (e == hipSuccess && nks > kInlineJobs)
      e = hipMemcpyAsync(d_ks[ring], h_ks[ring], sizeof(KsJob) * nks, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nrs > kInlineJobs)
      e = hipMemcpyAsync(d_rs[ring], h_rs[ring], sizeof(RsJob) * nrs, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nks) {
      JobArg<KsJob> ka{};
      ka.table = nks > kInlineJobs ? d_ks[ring] : nullptr;
      if (!ka.table)
        for (int t = 0; t < nks; ++t) ka.inl[t] = h_ks[ring][t];
      e = ks_launch(c, c.sched, ka, nks, Lks, true, false, st);
    }
    if (e == hipSuccess && nrs) {
      JobArg<RsJob> ra{};
      ra.table = nrs > kInlineJobs ? d_rs[ring] : nullptr;
      if (!ra.table)
        for (int t = 0; t < nrs; ++t) ra.inl[t] = h_rs[ring][t];
      e = rs_launch(c, ra, nrs, Lrs, st);
    }
    f.ev = events[ring];
    if (e == hipSuccess) e = hipEventRecord(f.ev, st);
    if (e != hipSuccess) {
      error = CKKS_EHIP;
      error_msg = std::string("batch launch failed: ") + hipGetErrorString(e);
    }
    ring_busy[ring] = true;
    jobs_on_device += (int)f.tickets.size();
    ++batches;
    inflight.push_back(std::move(f));
    return true;
  }

  void run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      retire_locked();
      bool launched = false;
      while (admit_locked()) launched = true;
      if (stop && pending.empty() && inflight.empty()) break;
      if (error && inflight.empty()) {
        // nothing can complete any more: fail the queue
        for (Req& r : pending) {
          t_done[r.ticket] = now_us(t0);
          event_pool.push_back(r.ready);
        }
        pending.clear();
        cv_done.notify_all();
        if (stop) break;
      }
      if (!launched) {
        if (inflight.empty())
          cv_work.wait_for(lk, std::chrono::milliseconds(5));
        else {
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(10));
          lk.lock();
        }
      }
    }
  }
};

namespace {

void server_free(ckks_server* s) {
  for (int i = 0; i < kRing; ++i) {
    if (s->d_ks[i]) (void)hipFree(s->d_ks[i]);
    if (s->d_rs[i]) (void)hipFree(s->d_rs[i]);
    if (s->h_ks[i]) (void)hipHostFree(s->h_ks[i]);
    if (s->h_rs[i]) (void)hipHostFree(s->h_rs[i]);
    if (s->events[i]) (void)hipEventDestroy(s->events[i]);
  }
  for (hipStream_t st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : s->all_events) (void)hipEventDestroy(ev);
  if (s->d_arena) (void)hipFree(s->d_arena);
  delete s;
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double idx = p / 100.0 * (double)(v.size() - 1);
  const size_t lo = (size_t)idx, hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (v[hi] - v[lo]) * (idx - (double)lo);
}

}  // namespace

extern "C" {

int ckks_server_create(const ckks_ctx* const* ctxs, int nctx, size_t hbm_budget, int max_slots,
                       ckks_server** out) {
  if (!ctxs || nctx < 1 || !out || max_slots < 1 || hbm_budget == 0)
    return api_fail(CKKS_EINVAL, "bad server arguments");
  *out = nullptr;
  for (int i = 0; i < nctx; ++i) {
    if (!ctxs[i]) return api_fail(CKKS_EINVAL, "null context");
    if (ctxs[i]->c.device != ctxs[0]->c.device)
      return api_fail(CKKS_EINVAL, "all contexts of a server must be on one device");
  }
  ckks_server* s = new (std::nothrow) ckks_server;
  if (!s) return api_fail(CKKS_ENOMEM, "host allocation failed");
  for (int i = 0; i < nctx; ++i) s->ctxs.push_back(&ctxs[i]->c);
  s->device = ctxs[0]->c.device;
  s->budget = hbm_budget;
  s->max_slots = max_slots;
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(s->device) != hipSuccess) {
    delete s;
    return api_fail(CKKS_EHIP, "hipSetDevice failed");
  }
  bool ok = hipMalloc(&s->d_arena, hbm_budget) == hipSuccess;
  for (int i = 0; ok && i < kStreams; ++i)
    ok = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < kRing; ++i) {
    ok = hipMalloc(&s->d_ks[i], sizeof(KsJob) * max_slots) == hipSuccess &&
         hipMalloc(&s->d_rs[i], sizeof(RsJob) * max_slots) == hipSuccess &&
         hipHostMalloc((void**)&s->h_ks[i], sizeof(KsJob) * max_slots, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void**)&s->h_rs[i], sizeof(RsJob) * max_slots, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming) == hipSuccess;
  }
  (void)hipSetDevice(prev);
  if (!ok) {
    server_free(s);
    return api_fail(CKKS_ENOMEM, "server allocation (arena, streams, tables) failed");
  }
  s->arena.init(hbm_budget);
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return CKKS_OK;
}

int ckks_server_submit(ckks_server* s, int ctx_index, const ckks_job* job, void* stream, uint64_t* ticket) {
  if (!s || !job || !ticket) return api_fail(CKKS_EINVAL, "null argument");
  if (ctx_index < 0 || ctx_index >= (int)s->ctxs.size()) return api_fail(CKKS_EINVAL, "bad context index");
  const Ctx& c = *s->ctxs[ctx_index];
  const ckks_job& j = *job;
  const int lo = j.op == CKKS_JOB_RESCALE ? 2 : 1;
  if (j.op < CKKS_JOB_KEYSWITCH || j.op > CKKS_JOB_RESCALE) return api_fail(CKKS_EINVAL, "unknown op");
  if (j.L < lo || j.L > c.L_max || !j.in0 || !j.out) return api_fail(CKKS_EINVAL, "bad level or null pointer");
  if (j.op != CKKS_JOB_RESCALE && (!j.key || (j.op == CKKS_JOB_HMULT && !j.in1)))
    return api_fail(CKKS_EINVAL, "null key or second input");
  const size_t bytes = s->job_bytes(c, j);
  const size_t io = ckks_server::io_bytes_of(c, j), keyb = ckks_server::key_bytes_of(c, j);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error) return api_fail(s->error, s->error_msg);
  if (bytes > s->budget || (s->whole && bytes + io + keyb > s->budget)) {
    ++s->rejected;
    return api_fail(CKKS_ENOMEM, s->whole ? "job footprint exceeds the server's HBM budget"
                                          : "job scratch exceeds the server's HBM budget");
  }
  // order the job after the work queued so far on the submitter's stream
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (prev != s->device && hipSetDevice(s->device) != hipSuccess)
    return api_fail(CKKS_EHIP, "hipSetDevice failed");
  hipEvent_t ready = nullptr;
  hipError_t e = hipSuccess;
  if (!s->event_pool.empty()) {
    ready = s->event_pool.back();
    s->event_pool.pop_back();
  } else if ((e = hipEventCreateWithFlags(&ready, hipEventDisableTiming)) == hipSuccess) {
    s->all_events.push_back(ready);
  }
  if (e == hipSuccess) e = hipEventRecord(ready, (hipStream_t)stream);
  if (prev != s->device) (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    if (ready) s->event_pool.push_back(ready);
    return api_fail(CKKS_EHIP, std::string("recording the submit event: ") + hipGetErrorString(e));
  }
  const uint64_t tk = s->next_ticket++;
  s->t_submit.push_back(now_us(s->t0));
  s->t_done.push_back(-1.0);
  s->is_ks.push_back(j.op != CKKS_JOB_RESCALE);
  s->pending.push_back(Req{tk, ctx_index, j, bytes, io, keyb, ready, stream});
  s->cv_work.notify_one();
  *ticket = tk;
  return CKKS_OK;
}

int ckks_server_poll(ckks_server* s, uint64_t ticket, int* done) {
  if (!s || !done) return api_fail(CKKS_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket >= s->next_ticket) return api_fail(CKKS_EINVAL, "unknown ticket");
  *done = s->t_done[ticket] >= 0.0;
  return s->error ? api_fail(s->error, s->error_msg) : CKKS_OK;
}

int ckks_server_drain(ckks_server* s) {
  if (!s) return api_fail(CKKS_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [s] { return (s->pending.empty() && s->inflight.empty()) || (s->error && s->inflight.empty()); });
  return s->error ? api_fail(s->error, s->error_msg) : CKKS_OK;
}

int ckks_server_stats(ckks_server* s, ckks_stats* st) {
  if (!s || !st) return api_fail(CKKS_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<double> lat;
  double first = -1, last = 0;
  for (uint64_t t = 0; t < s->next_ticket; ++t)
    if (s->t_done[t] >= 0.0) {
      lat.push_back(s->t_done[t] - s->t_submit[t]);
      first = first < 0 ? s->t_submit[t] : std::min(first, s->t_submit[t]);
      last = std::max(last, s->t_done[t]);
    }
  st->submitted = s->next_ticket;
  st->completed = s->completed;
  st->rejected = s->rejected;
  st->pending = s->pending.size();
  st->in_flight = (uint64_t)s->jobs_on_device;
  st->batches = s->batches;
  st->p50_us = percentile(lat, 50.0);
  st->p99_us = percentile(lat, 99.0);
  st->mean_us = lat.empty() ? 0.0 : [&] { double a = 0; for (double v : lat) a += v; return a / lat.size(); }();
  st->max_us = lat.empty() ? 0.0 : *std::max_element(lat.begin(), lat.end());
  st->ks_per_s = (last > first && first >= 0) ? (double)s->completed_ks / ((last - first) * 1e-6) : 0.0;
  st->budget_bytes = s->budget;
  st->peak_bytes = s->whole ? s->total_peak : s->arena.peak;
  return CKKS_OK;
}

int ckks_server_set_accounting(ckks_server* s, int whole_footprint) {
  if (!s) return api_fail(CKKS_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->next_ticket) return api_fail(CKKS_EINVAL, "accounting must be chosen before the first submit");
  s->whole = whole_footprint != 0;
  return CKKS_OK;
}

int ckks_server_times(ckks_server* s, uint64_t first, int n, double* h_submit_us, double* h_done_us) {
  if (!s || n < 0 || (n && (!h_submit_us || !h_done_us))) return api_fail(CKKS_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  if (first + (uint64_t)n > s->next_ticket) return api_fail(CKKS_EINVAL, "ticket range out of bounds");
  for (int i = 0; i < n; ++i) {
    h_submit_us[i] = s->t_submit[first + i];
    h_done_us[i] = s->t_done[first + i];
  }
  return CKKS_OK;
}

int ckks_server_destroy(ckks_server* s) {
  if (!s) return CKKS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  for (hipStream_t st : s->streams)
    if (st) (void)hipStreamSynchronize(st);
  server_free(s);
  (void)hipSetDevice(prev);
  return CKKS_OK;
}

}  // extern "C"
