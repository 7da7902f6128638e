// Projection server: continuous batching of Z = X V requests (the map of
// eq. (dim_reduction_maps)) with V resident on the device.
//
// Host side: submit() appends to a FIFO queue; admission and launches
// happen under the server's lock, in submit() itself when a launch slot is
// free and otherwise in a scheduler thread that also retires finished
// launches. Queued requests are admitted while fewer than max_inflight are
// unfinished and, for requests in host memory, while the staging arena has
// room; admitted requests (up to kProjMaxReq) are packed into the request
// table of a free launch slot. The table travels by value in the kernel
// arguments (no upload before the kernels), and a launch starts only the
// persistent batch kernel of each tile class that has tiles; slots rotate
// over several streams, so a launch made while others run overlaps them on
// the device. Completion is seen by polling each slot's event.
#include "common.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace lspca {
namespace {

using Clock = std::chrono::steady_clock;

constexpr int kSlots = 8, kStreams = 4;
constexpr size_t kAlign = 256;

size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

struct Request {
  uint64_t ticket = 0;
  const void *X = nullptr;
  void *Z = nullptr;
  int64_t rows = 0;
  bool host = false;
  size_t off = 0, bx = 0, bz = 0;      // arena block of a host request: X then Z
  int64_t tiles = 0;
  bool small = false;                  // small-tile class (few rows, 16-bit data)
  Clock::time_point t_submit, t_launch, t_done;
  int64_t enqueue_ns = 0;
  int status = 1;                      // 1 while pending; then LSPCA_OK or an error
};

// First-fit allocator over [0, size) with coalescing free list.
class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
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
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

struct Slot {
  ProjTable tab{};                     // copied into the kernel arguments at launch
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  Clock::time_point t_enqueued;
  std::vector<Request *> reqs;
};

}  // namespace
}  // namespace lspca

struct lspca_server {
  int dev = 0;
  lspca_dtype xdt = LSPCA_BF16;
  int64_t n = 0;
  int k = 0;
  size_t esz = 0, zsz = 0;
  void *VTh = nullptr, *VTl = nullptr;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  lspca::Arena alloc;
  int max_inflight = 1, queue_cap = 16;
  int BM = 128, BN = 128, ntn = 1, grid = 256;
  int64_t small_rows = 0;              // requests of at most this many rows: small tiles
  int ntn_s = 1, grid_s = 0;
  bool vec = false;
  hipStream_t streams[lspca::kStreams] = {};
  lspca::Slot slots[lspca::kSlots];

  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<lspca::Request *> pending;  // submitted, not admitted
  std::deque<lspca::Request *> ready;    // admitted, not launched
  std::unordered_map<uint64_t, lspca::Request *> live;
  uint64_t next_ticket = 1;
  int inflight = 0;                      // admitted, unfinished
  bool stop = false, paused = false;
  std::thread th;
  lspca_server_stats st{};
};

namespace lspca {
namespace {

int busy_slots(const lspca_server *S) {
  int b = 0;
  for (const Slot &sl : S->slots) b += sl.busy;
  return b;
}

void finish(lspca_server *S, Request *r, int status, Clock::time_point now) {
  r->status = status;
  r->t_done = now;
  if (r->host && r->bx + r->bz) S->alloc.release(r->off, r->bx + r->bz);
  --S->inflight;
  ++S->st.completed;
  S->st.rows_completed += (uint64_t)r->rows;
  using ns = std::chrono::nanoseconds;
  S->st.queue_ns += (uint64_t)std::chrono::duration_cast<ns>(r->t_launch - r->t_submit).count();
  S->st.enqueue_ns += (uint64_t)r->enqueue_ns;
  S->st.device_ns += (uint64_t)std::chrono::duration_cast<ns>(now - r->t_launch).count();
}

// Enqueue one launch on a free slot with the requests at the front of
// `ready`. Returns false when no slot is free.
bool launch_one(lspca_server *S) {
  Slot *sl = nullptr;
  for (Slot &x : S->slots)
    if (!x.busy) {
      sl = &x;
      break;
    }
  if (!sl) return false;
  ProjTable *t = &sl->tab;
  // take requests in FIFO order; small-tile ones go first in the table
  int64_t tiles[2] = {0, 0};
  while (!S->ready.empty() && (int)sl->reqs.size() < kProjMaxReq) {
    Request *r = S->ready.front();
    if (!sl->reqs.empty() && tiles[r->small] + r->tiles > (int64_t)1 << 30) break;
    S->ready.pop_front();
    tiles[r->small] += r->tiles;
    sl->reqs.push_back(r);
  }
  int nreq = 0;
  int64_t t0[2] = {0, 0};
  for (int cls = 1; cls >= 0; --cls)
    for (Request *r : sl->reqs) {
      if ((int)r->small != cls) continue;
      ProjReq &q = t->req[nreq++];
      q.X = r->host ? (const void *)(S->arena + r->off) : r->X;
      q.Z = r->host ? (void *)(S->arena + r->off + r->bx) : r->Z;
      q.ldx = S->n;
      q.ldz = S->k;
      q.rows = r->rows;
      q.tile0 = (int32_t)t0[cls];
      q.pad = 0;
      t0[cls] += r->tiles;
    }
  t->nreq = nreq;
  t->ntiles = (int32_t)tiles[0];
  t->ntn = S->ntn;
  t->ntiles_s = (int32_t)tiles[1];
  t->ntn_s = S->ntn_s;
  t->nreq_s = 0;
  for (Request *r : sl->reqs) t->nreq_s += r->small ? 1 : 0;
  t->pad0 = t->pad1 = 0;
  const auto t_start = Clock::now();
  hipError_t e = hipSuccess;
  for (Request *r : sl->reqs)
    if (r->host && e == hipSuccess)
      e = hipMemcpyAsync(S->arena + r->off, r->X, (size_t)r->rows * S->n * S->esz, hipMemcpyHostToDevice,
                         sl->stream);
  // the small-tile kernel first (the latency-bound requests), then the
  // standard one; a class without tiles is not launched, and a class with
  // fewer tiles than the persistent grid gets one workgroup per tile
  int rc = LSPCA_OK;
  if (e == hipSuccess && tiles[1] > 0)
    rc = launch_proj_batch_small(S->xdt, t, S->VTh, S->VTl, S->n, S->k, (int)S->n, S->vec,
                                 (int)std::min<int64_t>(S->grid_s, tiles[1]), sl->stream);
  if (e == hipSuccess && rc == LSPCA_OK && tiles[0] > 0)
    rc = launch_proj_batch(S->xdt, t, S->VTh, S->VTl, S->n, S->k, (int)S->n, S->vec,
                           (int)std::min<int64_t>(S->grid, tiles[0]), sl->stream);
  if (e == hipSuccess && rc != LSPCA_OK) e = hipErrorLaunchFailure;
  for (Request *r : sl->reqs)
    if (r->host && e == hipSuccess)
      e = hipMemcpyAsync(r->Z, S->arena + r->off + r->bx, (size_t)r->rows * S->k * S->zsz,
                         hipMemcpyDeviceToHost, sl->stream);
  if (e == hipSuccess) e = hipEventRecord(sl->done, sl->stream);
  const auto t_end = Clock::now();
  for (Request *r : sl->reqs) {
    r->t_launch = t_end;
    r->enqueue_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(t_end - t_start).count();
  }
  if (e != hipSuccess) {
    const auto now = Clock::now();
    for (Request *r : sl->reqs) finish(S, r, LSPCA_EHIP, now);
    sl->reqs.clear();
    S->cv_done.notify_all();
    return true;
  }
  sl->busy = true;
  ++S->st.launches;
  if ((uint32_t)nreq > S->st.max_requests_per_launch) S->st.max_requests_per_launch = nreq;
  const uint32_t b = (uint32_t)busy_slots(S);
  if (b > S->st.max_concurrent_launches) S->st.max_concurrent_launches = b;
  return true;
}

// Admit queued requests in FIFO order and launch what is admitted (called
// with S->mu held, by the scheduler and by submit). Returns whether
// anything moved.
bool pump(lspca_server *S) {
  bool progressed = false;
  while (!S->pending.empty() && S->inflight < S->max_inflight) {
    Request *r = S->pending.front();
    if (r->host) {
      if (!S->alloc.alloc(r->bx + r->bz, &r->off)) break;
      if (S->alloc.used() > S->st.arena_peak_bytes) S->st.arena_peak_bytes = S->alloc.used();
    }
    S->pending.pop_front();
    ++S->inflight;
    S->ready.push_back(r);
    progressed = true;
  }
  if (!S->paused)
    while (!S->ready.empty() && launch_one(S)) progressed = true;
  return progressed;
}

void scheduler(lspca_server *S) {
  (void)hipSetDevice(S->dev);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool progressed = false;
    // retire finished launches
    for (Slot &sl : S->slots) {
      if (!sl.busy) continue;
      const hipError_t e = hipEventQuery(sl.done);
      if (e == hipErrorNotReady) continue;
      const auto now = Clock::now();
      for (Request *r : sl.reqs) finish(S, r, e == hipSuccess ? LSPCA_OK : LSPCA_EHIP, now);
      sl.reqs.clear();
      sl.busy = false;
      progressed = true;
    }
    if (progressed) S->cv_done.notify_all();
    // admit in FIFO order and launch
    if (pump(S)) progressed = true;
    if (S->stop && S->pending.empty() && S->ready.empty() && busy_slots(S) == 0) break;
    if (progressed) continue;
    if (busy_slots(S) > 0) {
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else {
      S->cv_sched.wait(lk);
    }
  }
}

bool is_host_pointer(const void *p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return true;                         // unknown to HIP: pageable host memory
  }
  return a.type == hipMemoryTypeHost || a.type == hipMemoryTypeUnregistered;
}

void release_resources(lspca_server *S) {
  for (Slot &sl : S->slots)
    if (sl.done) (void)hipEventDestroy(sl.done);
  for (hipStream_t s : S->streams)
    if (s) (void)hipStreamDestroy(s);
  if (S->VTh) (void)hipFree(S->VTh);
  if (S->VTl) (void)hipFree(S->VTl);
  if (S->arena) (void)hipFree(S->arena);
}

int create_resources(lspca_server *S, const double *V) {
  const size_t vbytes = S->esz * (size_t)S->n * S->k;
  LSPCA_HIP(hipMalloc(&S->VTh, vbytes));
  if (S->xdt == LSPCA_BF16 || S->xdt == LSPCA_F16) LSPCA_HIP(hipMalloc(&S->VTl, vbytes));
  if (S->arena_bytes) LSPCA_HIP(hipMalloc((void **)&S->arena, S->arena_bytes));
  for (hipStream_t &s : S->streams) LSPCA_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  LSPCA_TRY(launch_convert_vt(V, S->n, S->k, S->xdt, S->VTh, S->VTl, S->streams[0]));
  LSPCA_HIP(hipStreamSynchronize(S->streams[0]));
  for (int i = 0; i < kSlots; ++i) {
    Slot &sl = S->slots[i];
    sl.stream = S->streams[i % kStreams];
    LSPCA_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
  }
  return LSPCA_OK;
}

}  // namespace
}  // namespace lspca

using lspca::Clock;
using lspca::set_error;

extern "C" {

int lspca_server_create(const double *V, int64_t n, int32_t k, lspca_dtype xdt, size_t arena_bytes,
                        int32_t max_inflight, lspca_server **out) {
  if (!out || !V) { set_error("V and out must not be NULL"); return LSPCA_EINVAL; }
  *out = nullptr;
  if (n < 1 || k < 1 || n > (1 << 30) || k > 4096) { set_error("bad sizes (n=%lld k=%d)", (long long)n, k); return LSPCA_EINVAL; }
  if ((int)xdt < 0 || (int)xdt > 3) { set_error("unknown dtype %d", (int)xdt); return LSPCA_EINVAL; }
  if (max_inflight < 1) { set_error("max_inflight must be >= 1"); return LSPCA_EINVAL; }
  lspca_server *S = new (std::nothrow) lspca_server();
  if (!S) { set_error("out of host memory"); return LSPCA_ENOMEM; }
  int rc = LSPCA_OK;
  do {
    if (hipGetDevice(&S->dev) != hipSuccess) { set_error("hipGetDevice failed"); rc = LSPCA_EHIP; break; }
    S->xdt = xdt;
    S->n = n;
    S->k = k;
    S->esz = lspca::dtype_size(xdt);
    S->zsz = xdt == LSPCA_F64 ? 8 : 4;
    S->arena_bytes = lspca::round_up(arena_bytes);
    S->alloc.init(S->arena_bytes);
    S->max_inflight = max_inflight;
    S->queue_cap = 16 * max_inflight;
    lspca::proj_tile_shape(xdt, k, &S->BM, &S->BN);
    S->ntn = (k + S->BN - 1) / S->BN;
    S->vec = (n * (int64_t)S->esz) % 16 == 0;
    rc = lspca::proj_batch_grid(xdt, k, S->vec, &S->grid);
    if (rc != LSPCA_OK) break;
    S->small_rows = lspca::proj_small_rows(xdt);
    if (S->small_rows > 0) {
      S->ntn_s = (k + lspca::kProjSmallBN - 1) / lspca::kProjSmallBN;
      rc = lspca::proj_small_grid(xdt, S->vec, &S->grid_s);
      if (rc != LSPCA_OK) break;
    }
    rc = lspca::create_resources(S, V);
  } while (false);
  if (rc != LSPCA_OK) {
    lspca::release_resources(S);
    delete S;
    return rc;
  }
  S->st.struct_size = sizeof(lspca_server_stats);
  S->th = std::thread(lspca::scheduler, S);
  *out = S;
  return LSPCA_OK;
}

int lspca_server_submit(lspca_server *S, const void *X, int64_t r, void *Z, uint64_t *ticket) {
  if (!S || !ticket) { set_error("server and ticket must not be NULL"); return LSPCA_EINVAL; }
  if (r < 0 || r > 0x7fffffffLL) { set_error("bad row count %lld", (long long)r); return LSPCA_EINVAL; }
  auto *q = new (std::nothrow) lspca::Request();
  if (!q) { set_error("out of host memory"); return LSPCA_ENOMEM; }
  q->rows = r;
  q->X = X;
  q->Z = Z;
  if (r > 0) {
    if (!X || !Z) { delete q; set_error("X and Z must not be NULL"); return LSPCA_EINVAL; }
    const bool hx = lspca::is_host_pointer(X), hz = lspca::is_host_pointer(Z);
    if (hx != hz) { delete q; set_error("X and Z must both be device or both be host memory"); return LSPCA_EINVAL; }
    q->host = hx;
    if (!hx && S->vec && (uintptr_t)X % 16 != 0) { delete q; set_error("device X must be 16-byte aligned"); return LSPCA_EINVAL; }
    if (!hx && (uintptr_t)Z % S->zsz != 0) { delete q; set_error("Z misaligned"); return LSPCA_EINVAL; }
    q->small = r <= S->small_rows;
    q->tiles = q->small ? (r + lspca::kProjSmallBM - 1) / lspca::kProjSmallBM * S->ntn_s
                        : (r + S->BM - 1) / S->BM * S->ntn;
    if (hx) {
      q->bx = lspca::round_up((size_t)r * S->n * S->esz);
      q->bz = lspca::round_up((size_t)r * S->k * S->zsz);
      if (q->bx + q->bz > S->arena_bytes) {
        const size_t need = q->bx + q->bz;
        delete q;
        set_error("host request needs %zu staging bytes, arena has %zu", need, S->arena_bytes);
        return LSPCA_E2BIG;
      }
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if ((int)S->pending.size() >= S->queue_cap) {
    delete q;
    set_error("queue full (%d requests waiting)", S->queue_cap);
    return LSPCA_EAGAIN;
  }
  q->ticket = S->next_ticket++;
  q->t_submit = Clock::now();
  ++S->st.submitted;
  S->live[q->ticket] = q;
  *ticket = q->ticket;
  if (r == 0) {
    q->status = LSPCA_OK;
    q->t_done = q->t_submit;
    ++S->st.completed;
    return LSPCA_OK;
  }
  S->pending.push_back(q);
  // admit and launch from the submitting thread when a slot is free (no
  // wake-up of the scheduler on the request's path); the scheduler is woken
  // to retire it
  if (S->th.joinable() && !S->stop) (void)lspca::pump(S);
  S->cv_sched.notify_one();
  return LSPCA_OK;
}

int lspca_server_wait(lspca_server *S, uint64_t ticket, int64_t timeout_us, double *latency_ms) {
  if (!S) { set_error("server must not be NULL"); return LSPCA_EINVAL; }
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->live.find(ticket);
  if (it == S->live.end()) { set_error("unknown ticket %llu", (unsigned long long)ticket); return LSPCA_ENOTFOUND; }
  lspca::Request *q = it->second;
  auto done = [&] { return q->status != 1; };
  if (timeout_us < 0) S->cv_done.wait(lk, done);
  else if (!done()) S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done);
  if (!done()) { set_error("request %llu still running", (unsigned long long)ticket); return LSPCA_ETIMEDOUT; }
  const int status = q->status;
  if (latency_ms) latency_ms[0] = std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count();
  S->live.erase(it);
  delete q;
  if (status != LSPCA_OK) set_error("request %llu failed on the device", (unsigned long long)ticket);
  return status;
}

int lspca_server_pause(lspca_server *S, int paused) {
  if (!S) { set_error("server must not be NULL"); return LSPCA_EINVAL; }
  std::lock_guard<std::mutex> lk(S->mu);
  S->paused = paused != 0;
  S->cv_sched.notify_one();
  return LSPCA_OK;
}

int lspca_server_get_stats(lspca_server *S, lspca_server_stats *out) {
  if (!S || !out) { set_error("server and out must not be NULL"); return LSPCA_EINVAL; }
  if (out->struct_size < sizeof(lspca_server_stats)) { set_error("stats struct_size too small"); return LSPCA_EINVAL; }
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  out->struct_size = sizeof(lspca_server_stats);
  return LSPCA_OK;
}

int lspca_server_destroy(lspca_server *S) {
  if (!S) return LSPCA_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->paused = false;
    S->cv_sched.notify_one();
  }
  if (S->th.joinable()) S->th.join();
  for (auto &kv : S->live) delete kv.second;
  S->live.clear();
  lspca::release_resources(S);
  delete S;
  return LSPCA_OK;
}

}  // extern "C"
