// Continuous-batching server over a resident scene.
//
// Memory: one device arena of mem_budget_bytes is allocated at creation and
// carved by a first-fit allocator (no hipMalloc after creation).  The
// scene's render records live in it for the server's lifetime.
//
// Scheduling: requests queue in FIFO order.  Each of max_slots worker
// threads owns a HIP stream; when idle it forms a batch from the head of the
// queue (the head request, then more while the batch stays within
// max_batch_cams cameras and its memory reservation fits the free arena),
// runs project -> count (one read-back) -> sort -> persistent render on its
// own stream, then releases the memory and completes the requests.  Batches
// of different workers run concurrently on the device; requests that arrive
// while others are in flight are admitted as soon as a slot and memory free
// up.  A request whose entry-phase memory alone exceeds the budget is
// rejected at submission (GUT_E_ADMISSION).
//
// Results are bitwise identical to rendering a request alone: a camera's tile
// lists, sort order (depth, then particle) and per-tile arithmetic do not
// depend on the other cameras of its batch.
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
#include <unordered_map>
#include <vector>

#include "common.h"

namespace gut {

using Clock = std::chrono::steady_clock;

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit allocator over [0, size) with coalescing free blocks.
class Arena {
 public:
  void init(size_t size) {
    size_ = size;
    free_.clear();
    free_[0] = size;
    used_ = peak_ = 0;
  }
  // returns offset or SIZE_MAX
  size_t alloc(size_t bytes) {
    bytes = al256(bytes ? bytes : 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        sizes_[off] = bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off) {
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return;
    size_t bytes = s->second;
    sizes_.erase(s);
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
  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t peak() const { return peak_; }

 private:
  size_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
  std::map<size_t, size_t> sizes_;
};

struct Request {
  uint64_t id;
  std::vector<gut_camera> cams;
  std::vector<float*> out;
  Clock::time_point t_submit, t_done;
  int state = 0;  // 0 queued, 1 running, 2 done
  gut_status status = GUT_OK;
};

struct Worker {
  hipStream_t stream = nullptr;
  std::thread th;
  void* pinned = nullptr;  // staging for camera tables and lists
};

}  // namespace gut

struct gut_server {
  gut_scene scene;
  gut_params params;
  int device = 0;
  int max_slots = 1, max_batch_cams = 8, n_blocks = 1024;
  char* base = nullptr;
  size_t budget = 0;
  gut::Arena arena;
  size_t record_off = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<gut::Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<gut::Request>> reqs;
  std::vector<gut::Worker> workers;
  bool stop = false;
  int busy = 0;
  uint64_t next_id = 1;
  double pairs_per_entry = 4.0;  // running estimate used to reserve pair memory
  // statistics window
  gut::Clock::time_point t0;
  std::vector<double> lat_ms;
  int64_t submitted = 0, completed = 0, rejected = 0, batches = 0, cameras = 0;
  gut_status fatal = GUT_OK;
};

namespace gut {

constexpr size_t kStage = 64 * 1024;

// Device memory one batch needs before its pair count is known.
static size_t batch_entry_bytes(int64_t n, const std::vector<DevCam>& dc, int64_t T) {
  const int64_t E = n * (int64_t)dc.size();
  return al256(E * 8) + al256(E * 4) * 2 + al256(E * 12) + al256(bin_entry_bytes(E)) +
         al256(T * 12) + al256(dc.size() * sizeof(DevCam)) + al256(dc.size() * sizeof(float*)) +
         al256(2 * (2 * kMaxCams + 1) * sizeof(int)) + al256(16 * sizeof(unsigned)) + 4096;
}

static size_t batch_pair_bytes(int64_t P) { return al256(P * 4) + al256(bin_pair_bytes(P)); }

struct Batch {
  std::vector<Request*> reqs;
  size_t off_entry = SIZE_MAX, off_pair = SIZE_MAX;
  int64_t P_reserved = 0;
};

static gut_status run_batch(gut_server* S, Worker& W, Batch& B) {
  std::vector<Request*>& batch = B.reqs;
  hipStream_t s = W.stream;
  std::vector<gut_camera> cams;
  std::vector<float*> outs;
  for (auto* r : batch)
    for (size_t c = 0; c < r->cams.size(); c++) { cams.push_back(r->cams[c]); outs.push_back(r->out[c]); }
  const int nc = (int)cams.size();
  std::vector<DevCam> dc(nc);
  int64_t T = 0;
  gut_status st = prepare_cams(cams.data(), nc, S->params, dc.data(), &T, nullptr);
  if (st != GUT_OK) return st;
  const int64_t n = S->scene.n, E = n * nc;
  // memory reserved by the scheduler when it formed the batch
  size_t off_entry = B.off_entry, off_pair = B.off_pair;
  const int64_t P_reserved = B.P_reserved;
  char* b = S->base + off_entry;
  auto take = [&](size_t bytes) { char* p = b; b += al256(bytes); return p; };
  gut_projected proj = {};
  proj.rect = (int16_t*)take(E * 8);
  proj.tiles = (uint32_t*)take(E * 4);
  proj.depth = (float*)take(E * 4);
  proj.rgb = (float*)take(E * 12);
  proj.record = (float*)(S->base + S->record_off);
  char* ews = take(bin_entry_bytes(E));
  uint32_t* ranges = (uint32_t*)take(T * 12);  // [T,2] ranges, then the render order
  DevCam* d_cams = (DevCam*)take(nc * sizeof(DevCam));
  float** d_outs = (float**)take(nc * sizeof(float*));
  int* d_lists = (int*)take(2 * (2 * kMaxCams + 1) * sizeof(int));
  unsigned* d_counters = (unsigned*)take(16 * sizeof(unsigned));

  auto release = [&]() {
    // queued work may still use the memory (bin_count returns while the
    // depth sort runs)
    (void)hipStreamSynchronize(s);
    std::lock_guard<std::mutex> lk(S->mu);
    S->arena.release(off_entry);
    if (off_pair != SIZE_MAX) S->arena.release(off_pair);
    S->cv.notify_all();
  };
  // camera and output tables through the worker's pinned staging area
  char* stage = (char*)W.pinned;
  std::memcpy(stage, dc.data(), nc * sizeof(DevCam));
  std::memcpy(stage + 32768, outs.data(), nc * sizeof(float*));
  if ((st = hipMemcpyAsync(d_cams, stage, nc * sizeof(DevCam), hipMemcpyHostToDevice, s) == hipSuccess
                ? GUT_OK : GUT_E_HIP) != GUT_OK ||
      (st = hipMemcpyAsync(d_outs, stage + 32768, nc * sizeof(float*), hipMemcpyHostToDevice, s) ==
                    hipSuccess ? GUT_OK : GUT_E_HIP) != GUT_OK) {
    release();
    return st;
  }
  UTConst ut = make_ut(S->params);
  Thresholds th = make_thresholds(S->params);
  uint32_t nvis = 0;
  uint64_t P = 0;
  if ((st = project_launch(&S->scene, dc.data(), nc, ut, th, &proj, false, s)) != GUT_OK ||
      (st = bin_count(&proj, (int)n, dc.data(), nc, T, ews, ranges, &nvis, &P, s)) != GUT_OK) {
    release();
    return st;
  }
  if (P >= (uint64_t(1) << 32)) {  // pair offsets are 32-bit
    release();
    set_error("batch needs %llu pairs, more than 2^32 - 1", (unsigned long long)P);
    return GUT_E_CAPACITY;
  }
  if ((int64_t)P > P_reserved) {  // grow the pair buffers, waiting for memory if needed
    std::unique_lock<std::mutex> lk(S->mu);
    if (off_pair != SIZE_MAX) { S->arena.release(off_pair); off_pair = SIZE_MAX; }
    while (true) {
      off_pair = S->arena.alloc(batch_pair_bytes((int64_t)P));
      if (off_pair != SIZE_MAX) break;
      if (S->busy <= 1) {  // nothing else in flight will free memory
        lk.unlock();
        release();
        set_error("batch needs %llu pairs, more than the server budget holds", (unsigned long long)P);
        return GUT_E_CAPACITY;
      }
      S->cv.wait(lk);
    }
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (E > 0) S->pairs_per_entry = 0.8 * S->pairs_per_entry + 0.2 * ((double)P / (double)E);
  }
  char* pb = S->base + off_pair;
  uint32_t* ids = (uint32_t*)pb;
  char* pws = pb + al256((P > 0 ? P : 1) * 4);
  int* h_lists = (int*)(stage + 49152);
  if ((st = bin_sort(&proj, (int)n, dc.data(), nc, T, E, ews, nvis, P, pws, ranges, ids, s)) != GUT_OK ||
      (st = bin_order(dc.data(), nc, T, ranges, s)) != GUT_OK ||
      (st = render_batch_launch(d_cams, dc.data(), nc, th, (int)n, ranges, ranges + 2 * T, ids,
                                proj.record, proj.rgb, d_outs, d_counters, d_lists, h_lists,
                                S->n_blocks, s)) != GUT_OK) {
    release();
    return st;
  }
  hipError_t he = hipStreamSynchronize(s);
  release();
  if (he != hipSuccess) {
    set_error("batch failed: %s", hipGetErrorString(he));
    return GUT_E_HIP;
  }
  return GUT_OK;
}

// Pick the next batch from the queue head and reserve its memory (caller
// holds the lock).  The head request is always taken if its entry-phase
// memory fits now; further requests join while the batch stays within
// max_batch_cams cameras and its entry memory plus estimated pair memory
// fits the free arena.
static Batch take_batch(gut_server* S) {
  Batch B;
  std::vector<gut_camera> all;
  int64_t best_entry = 0, best_pairs = 0;
  const size_t free_bytes = S->arena.largest_free();
  size_t taken = 0;
  for (size_t qi = 0; qi < S->queue.size(); qi++) {
    Request* r = S->queue[qi];
    int rc = (int)r->cams.size();
    if (!B.reqs.empty() && (int)all.size() + rc > S->max_batch_cams) break;
    if ((int)all.size() + rc > kMaxCams) break;
    std::vector<gut_camera> trial = all;
    trial.insert(trial.end(), r->cams.begin(), r->cams.end());
    std::vector<DevCam> dc(trial.size());
    int64_t T = 0;
    if (prepare_cams(trial.data(), (int)trial.size(), S->params, dc.data(), &T, nullptr) != GUT_OK) break;
    const int64_t E = S->scene.n * (int64_t)trial.size();
    const size_t entry = batch_entry_bytes(S->scene.n, dc, T);
    const int64_t pairs = (int64_t)(S->pairs_per_entry * 1.25 * (double)E) + 1024;
    if (entry + batch_pair_bytes(pairs) > free_bytes) {
      if (B.reqs.empty() && entry <= free_bytes) {  // head alone: pairs grow later
        all = trial;
        best_entry = (int64_t)entry;
        best_pairs = 0;
        taken = 1;
      }
      break;
    }
    all = trial;
    best_entry = (int64_t)entry;
    best_pairs = pairs;
    taken = qi + 1;
    B.reqs.push_back(r);
  }
  if (taken == 1 && B.reqs.empty()) B.reqs.push_back(S->queue.front());
  if (B.reqs.empty()) return B;
  B.off_entry = S->arena.alloc((size_t)best_entry);
  if (B.off_entry == SIZE_MAX) { B.reqs.clear(); return B; }
  if (best_pairs > 0) {
    B.off_pair = S->arena.alloc(batch_pair_bytes(best_pairs));
    B.P_reserved = B.off_pair == SIZE_MAX ? 0 : best_pairs;
  }
  for (size_t k = 0; k < B.reqs.size(); k++) S->queue.pop_front();
  return B;
}

static void worker_main(gut_server* S, int wi) {
  Worker& W = S->workers[wi];
  (void)hipSetDevice(S->device);
  while (true) {
    Batch B;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      while (true) {
        if (!S->queue.empty()) {
          B = take_batch(S);
          if (!B.reqs.empty()) break;
        } else if (S->stop) {
          return;
        }
        S->cv.wait(lk);
      }
      S->busy++;
      for (auto* r : B.reqs) r->state = 1;
    }
    gut_status st = run_batch(S, W, B);
    std::vector<Request*>& batch = B.reqs;
    auto now = Clock::now();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->busy--;
      S->batches++;
      for (auto* r : batch) {
        r->status = st;
        r->state = 2;
        r->t_done = now;
        if (st == GUT_OK) {
          S->completed++;
          S->cameras += (int64_t)r->cams.size();
          S->lat_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
        }
      }
      if (st != GUT_OK && st != GUT_E_CAPACITY) S->fatal = st;
    }
    S->cv.notify_all();
  }
}

}  // namespace gut

using namespace gut;

extern "C" gut_status gut_serve_create(const gut_scene* scene, const gut_params* p,
                                       size_t mem_budget_bytes, int32_t max_slots,
                                       int32_t max_batch_cams, gut_server** out) {
  gut_status st = check_params(p);
  if (st != GUT_OK) return st;
  if (p->kbuffer > 0) {
    set_error("gut_serve_create: the server renders in tile order (kbuffer must be 0)");
    return GUT_E_UNSUPPORTED;
  }
  if ((st = check_scene(scene, true)) != GUT_OK) return st;
  if (!out || max_slots < 1 || max_slots > 16 || max_batch_cams < 1 || max_batch_cams > kMaxCams) {
    set_error("max_slots must be in [1, 16] and max_batch_cams in [1, %d]", kMaxCams);
    return GUT_E_INVALID;
  }
  size_t rec = al256((size_t)scene->n * 64);
  if (mem_budget_bytes < rec + (1 << 20)) {
    set_error("budget %zu too small for the scene's render records (%zu bytes)", mem_budget_bytes, rec);
    return GUT_E_ADMISSION;
  }
  auto S = std::make_unique<gut_server>();
  S->scene = *scene;
  S->params = *p;
  S->max_slots = max_slots;
  S->max_batch_cams = max_batch_cams;
  GUT_HIP(hipGetDevice(&S->device));
  hipDeviceProp_t prop;
  GUT_HIP(hipGetDeviceProperties(&prop, S->device));
  S->n_blocks = prop.multiProcessorCount * 8;
  GUT_HIP(hipMalloc((void**)&S->base, mem_budget_bytes));
  S->budget = mem_budget_bytes;
  S->arena.init(mem_budget_bytes);
  S->record_off = S->arena.alloc(rec);
  hipStream_t s0;
  GUT_HIP(hipStreamCreateWithFlags(&s0, hipStreamNonBlocking));
  st = record_launch(scene, (float*)(S->base + S->record_off), s0);
  hipError_t he = hipStreamSynchronize(s0);
  (void)hipStreamDestroy(s0);
  if (st != GUT_OK || he != hipSuccess) {
    (void)hipFree(S->base);
    return st != GUT_OK ? st : GUT_E_HIP;
  }
  S->workers.resize(max_slots);
  for (int w = 0; w < max_slots; w++) {
    GUT_HIP(hipStreamCreateWithFlags(&S->workers[w].stream, hipStreamNonBlocking));
    GUT_HIP(hipHostMalloc(&S->workers[w].pinned, kStage, hipHostMallocDefault));
  }
  S->t0 = Clock::now();
  gut_server* raw = S.release();
  for (int w = 0; w < max_slots; w++) raw->workers[w].th = std::thread(worker_main, raw, w);
  *out = raw;
  return GUT_OK;
}

extern "C" gut_status gut_serve_submit(gut_server* S, const gut_camera* cams, int32_t n_cams,
                                       float* const* out_rgb, uint64_t* request_id) {
  if (!S || !cams || !out_rgb || !request_id || n_cams < 1 || n_cams > kMaxCams) {
    set_error("bad gut_serve_submit arguments");
    return GUT_E_INVALID;
  }
  std::vector<DevCam> dc(n_cams);
  int64_t T = 0;
  gut_status st = prepare_cams(cams, n_cams, S->params, dc.data(), &T, nullptr);
  if (st != GUT_OK) return st;
  for (int c = 0; c < n_cams; c++)
    if (!out_rgb[c]) { set_error("out_rgb[%d] is NULL", c); return GUT_E_INVALID; }
  auto r = std::make_unique<Request>();
  r->cams.assign(cams, cams + n_cams);
  r->out.assign(out_rgb, out_rgb + n_cams);
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(S->mu);
  if (batch_entry_bytes(S->scene.n, dc, T) > S->budget - al256((size_t)S->scene.n * 64)) {
    S->rejected++;
    set_error("request needs more device memory than the server budget");
    return GUT_E_ADMISSION;
  }
  r->id = S->next_id++;
  *request_id = r->id;
  S->queue.push_back(r.get());
  S->reqs[r->id] = std::move(r);
  S->submitted++;
  S->cv.notify_all();
  return GUT_OK;
}

extern "C" gut_status gut_serve_poll(gut_server* S, uint64_t id, int32_t* done) {
  if (!S || !done) return GUT_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) { set_error("unknown request %llu", (unsigned long long)id); return GUT_E_NOT_FOUND; }
  *done = it->second->state == 2;
  return it->second->state == 2 ? it->second->status : GUT_OK;
}

extern "C" gut_status gut_serve_wait(gut_server* S, uint64_t id) {
  if (!S) return GUT_E_INVALID;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) { set_error("unknown request %llu", (unsigned long long)id); return GUT_E_NOT_FOUND; }
  Request* r = it->second.get();
  S->cv.wait(lk, [&] { return r->state == 2; });
  return r->status;
}

extern "C" gut_status gut_serve_latency(gut_server* S, uint64_t id, double* ms) {
  if (!S || !ms) return GUT_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return GUT_E_NOT_FOUND;
  Request* r = it->second.get();
  if (r->state != 2) { *ms = -1.0; return GUT_OK; }
  *ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  return r->status;
}

extern "C" gut_status gut_serve_stats(gut_server* S, gut_serve_metrics* m) {
  if (!S || !m) return GUT_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  std::vector<double> v = S->lat_ms;
  std::sort(v.begin(), v.end());
  auto pct = [&](double q) {
    if (v.empty()) return 0.0;
    double k = q * (v.size() - 1);
    size_t i = (size_t)k;
    double f = k - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
  };
  double sum = 0;
  for (double x : v) sum += x;
  m->wall_s = std::chrono::duration<double>(Clock::now() - S->t0).count();
  m->frames_per_s = m->wall_s > 0 ? S->cameras / m->wall_s : 0.0;
  m->p50_ms = pct(0.5);
  m->p99_ms = pct(0.99);
  m->mean_ms = v.empty() ? 0.0 : sum / v.size();
  m->max_ms = v.empty() ? 0.0 : v.back();
  m->submitted = S->submitted;
  m->completed = S->completed;
  m->rejected = S->rejected;
  m->batches = S->batches;
  m->cameras = S->cameras;
  m->peak_bytes = (int64_t)S->arena.peak();
  return S->fatal;
}

extern "C" gut_status gut_serve_reset_stats(gut_server* S) {
  if (!S) return GUT_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  S->lat_ms.clear();
  S->submitted = S->completed = S->rejected = S->batches = S->cameras = 0;
  S->t0 = Clock::now();
  // completed requests are forgotten; queued and running ones stay
  for (auto it = S->reqs.begin(); it != S->reqs.end();) {
    if (it->second->state == 2) it = S->reqs.erase(it);
    else ++it;
  }
  return GUT_OK;
}

extern "C" gut_status gut_serve_destroy(gut_server* S) {
  if (!S) return GUT_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;  // workers drain the queue, then leave
  }
  S->cv.notify_all();
  for (auto& w : S->workers)
    if (w.th.joinable()) w.th.join();
  for (auto& w : S->workers) {
    if (w.stream) (void)hipStreamDestroy(w.stream);
    if (w.pinned) (void)hipHostFree(w.pinned);
  }
  if (S->base) (void)hipFree(S->base);
  delete S;
  return GUT_OK;
}
