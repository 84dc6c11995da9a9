// Continuous-batching scheduler of gut_server, independent of the device.
//
// The scheduler owns the request queue, the memory arena (offsets into one
// device allocation made by the backend), the worker threads and the latency
// statistics.  A Backend supplies what touches the device:
//
//   gut_status plan(const gut_camera* cams, int n_cams, size_t* entry_bytes) const
//       checks the cameras; memory a batch of them needs before its pair
//       count P is known
//   int64_t entries(int n_cams) const      (camera, particle) entries, E
//   size_t pair_bytes(int64_t P) const     memory of P pairs
//   size_t resident_bytes() const          arena bytes held for the scene
//   gut_status count(int slot, const std::vector<gut_camera>&, const std::vector<float*>&,
//                    size_t off_entry, uint64_t* P)
//       phase 1 on the slot's stream: project and count the pairs
//   gut_status finish(int slot, const std::vector<gut_camera>&, const std::vector<float*>&,
//                     size_t off_entry, size_t off_pair, uint64_t P)
//       phase 2: sort and render, then wait for the slot's stream
//   void quiesce(int slot)                 wait for the slot's queued work
//
// Requests queue in FIFO order.  An idle worker forms a batch from the head
// of the queue (the head request, then more while the batch stays within
// max_batch_cams cameras and its entry memory plus estimated pair memory fits
// the largest free block), runs phase 1, grows the pair reservation if P
// exceeds it, runs phase 2, releases the memory and completes the requests.
//
// Pair growth under memory pressure: a worker whose pairs do not fit waits
// for memory that running workers will free.  While any worker waits, no new
// batch starts.  When every busy worker is waiting (no one will free
// memory), the last to notice gives way: it releases its entry memory and
// puts its requests back at the head of the queue.  A single request goes
// back marked to run alone with its known pair count reserved up front; a
// merged batch that gives way with no other batch in flight is split (its
// head request is retried alone).  A single request whose entry and pair
// memory exceed the whole arena fails with GUT_E_CAPACITY.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gut.h"

namespace gut {

using Clock = std::chrono::steady_clock;

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit allocator over [0, size) with coalescing free blocks.
class Arena {
 public:
  static constexpr size_t kNone = SIZE_MAX;
  void init(size_t size) {
    size_ = size;
    free_.clear();
    sizes_.clear();
    if (size) free_[0] = size;
    used_ = peak_ = 0;
  }
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
    return kNone;
  }
  // Returns false for an offset that is not allocated (nothing changes).
  bool release(size_t off) {
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return false;
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
    return true;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }
  size_t free_blocks() const { return free_.size(); }

 private:
  size_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
  std::map<size_t, size_t> sizes_;
};

struct Request {
  uint64_t id = 0;
  std::vector<gut_camera> cams;
  std::vector<float*> out;
  Clock::time_point t_submit, t_done;
  int state = 0;       // 0 queued, 1 running, 2 done
  bool solo = false;   // never merged with other requests (set when it gave way)
  int64_t hint_pairs = 0;  // pairs it needed when it gave way, reserved up front
  gut_status status = GUT_OK;
};

struct SchedStats {
  int64_t submitted = 0, completed = 0, rejected = 0, batches = 0, cameras = 0;
  int64_t requeued = 0, splits = 0;
};

template <class Backend>
class Scheduler {
 public:
  // The backend must outlive the scheduler.  arena_bytes: the device
  // allocation the offsets refer to; the backend's resident bytes are taken
  // from it first.
  Scheduler(Backend* be, size_t arena_bytes, int max_slots, int max_batch_cams, int max_cams)
      : be_(be), max_slots_(max_slots), max_batch_cams_(max_batch_cams), max_cams_(max_cams) {
    arena_.init(arena_bytes);
    resident_off_ = arena_.alloc(be_->resident_bytes());
    t0_ = Clock::now();
  }
  ~Scheduler() { stop(); }

  size_t resident_offset() const { return resident_off_; }
  bool resident_ok() const { return resident_off_ != Arena::kNone; }

  void start() {
    for (int w = 0; w < max_slots_; w++) threads_.emplace_back(&Scheduler::worker_main, this, w);
  }

  // Workers drain the queue, then leave.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : threads_)
      if (t.joinable()) t.join();
    threads_.clear();
  }

  gut_status submit(const gut_camera* cams, int n_cams, float* const* out, uint64_t* id,
                    const char** why) {
    size_t entry = 0;
    gut_status st = be_->plan(cams, n_cams, &entry);
    if (st != GUT_OK) return st;
    auto r = std::make_unique<Request>();
    r->cams.assign(cams, cams + n_cams);
    r->out.assign(out, out + n_cams);
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(mu_);
    const size_t room = arena_.size() - al256(be_->resident_bytes());
    if (entry > room) {
      stats_.rejected++;
      if (why) *why = "request needs more device memory than the server budget";
      return GUT_E_ADMISSION;
    }
    r->id = next_id_++;
    *id = r->id;
    queue_.push_back(r.get());
    reqs_[r->id] = std::move(r);
    stats_.submitted++;
    cv_.notify_all();
    return GUT_OK;
  }

  gut_status poll(uint64_t id, int32_t* done) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end()) return GUT_E_NOT_FOUND;
    *done = it->second->state == 2;
    return it->second->state == 2 ? it->second->status : GUT_OK;
  }

  gut_status wait(uint64_t id) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end()) return GUT_E_NOT_FOUND;
    Request* r = it->second.get();
    cv_.wait(lk, [&] { return r->state == 2; });
    return r->status;
  }

  // Waits at most `ms` milliseconds; *done tells whether the request ended.
  gut_status wait_for(uint64_t id, double ms, int32_t* done) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end()) return GUT_E_NOT_FOUND;
    Request* r = it->second.get();
    // system_clock: its timed wait is the one thread checkers understand
    const auto until = std::chrono::system_clock::now() +
                       std::chrono::duration_cast<std::chrono::system_clock::duration>(
                           std::chrono::duration<double, std::milli>(ms));
    *done = cv_.wait_until(lk, until, [&] { return r->state == 2; });
    return *done ? r->status : GUT_OK;
  }

  gut_status latency(uint64_t id, double* ms) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end()) return GUT_E_NOT_FOUND;
    Request* r = it->second.get();
    if (r->state != 2) { *ms = -1.0; return GUT_OK; }
    *ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    return r->status;
  }

  // Latency percentiles over the window, the counters and the sticky status
  // of the first device failure (GUT_OK if none).
  gut_status metrics(gut_serve_metrics* m) {
    std::lock_guard<std::mutex> lk(mu_);
    std::vector<double> v = lat_ms_;
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
    m->wall_s = std::chrono::duration<double>(Clock::now() - t0_).count();
    m->frames_per_s = m->wall_s > 0 ? stats_.cameras / m->wall_s : 0.0;
    m->p50_ms = pct(0.5);
    m->p99_ms = pct(0.99);
    m->mean_ms = v.empty() ? 0.0 : sum / v.size();
    m->max_ms = v.empty() ? 0.0 : v.back();
    m->submitted = stats_.submitted;
    m->completed = stats_.completed;
    m->rejected = stats_.rejected;
    m->batches = stats_.batches;
    m->cameras = stats_.cameras;
    m->peak_bytes = (int64_t)arena_.peak();
    return fatal_;
  }

  void reset_stats() {
    std::lock_guard<std::mutex> lk(mu_);
    lat_ms_.clear();
    stats_ = SchedStats();
    t0_ = Clock::now();
    for (auto it = reqs_.begin(); it != reqs_.end();) {  // completed requests are forgotten
      if (it->second->state == 2) it = reqs_.erase(it);
      else ++it;
    }
  }

  // For tests: counters and arena state under the lock.
  SchedStats counters() {
    std::lock_guard<std::mutex> lk(mu_);
    return stats_;
  }
  size_t arena_used() {
    std::lock_guard<std::mutex> lk(mu_);
    return arena_.used();
  }
  size_t arena_free_blocks() {
    std::lock_guard<std::mutex> lk(mu_);
    return arena_.free_blocks();
  }

 private:
  struct Batch {
    std::vector<Request*> reqs;
    size_t off_entry = Arena::kNone, off_pair = Arena::kNone, entry_bytes = 0;
    int64_t P_reserved = 0;
  };
  enum class Outcome { Done, Requeued };

  // Pick the next batch from the queue head and reserve its memory (caller
  // holds the lock).  No batch starts while a worker waits for pair memory.
  Batch take_batch() {
    Batch B;
    if (growing_ > 0 || queue_.empty()) return B;
    std::vector<gut_camera> all;
    size_t best_entry = 0;
    int64_t best_pairs = 0;
    const size_t free_bytes = arena_.largest_free();
    for (size_t qi = 0; qi < queue_.size(); qi++) {
      Request* r = queue_[qi];
      const int rc = (int)r->cams.size();
      if (!B.reqs.empty() && (r->solo || B.reqs.front()->solo)) break;
      if (!B.reqs.empty() && (int)all.size() + rc > max_batch_cams_) break;
      if ((int)all.size() + rc > max_cams_) break;
      std::vector<gut_camera> trial = all;
      trial.insert(trial.end(), r->cams.begin(), r->cams.end());
      size_t entry = 0;
      if (be_->plan(trial.data(), (int)trial.size(), &entry) != GUT_OK) break;
      const int64_t E = be_->entries((int)trial.size());
      int64_t pairs = (int64_t)(pairs_per_entry_ * 1.25 * (double)E) + 1024;
      if (B.reqs.empty()) pairs = std::max(pairs, r->hint_pairs);
      if (entry + be_->pair_bytes(pairs) > free_bytes) {
        if (B.reqs.empty() && entry <= free_bytes && r->hint_pairs == 0) {  // the head alone: its pairs grow later
          all = trial;
          best_entry = entry;
          best_pairs = 0;
          B.reqs.push_back(r);
        }
        break;
      }
      all = trial;
      best_entry = entry;
      best_pairs = pairs;
      B.reqs.push_back(r);
    }
    if (B.reqs.empty()) return B;
    B.entry_bytes = best_entry;
    B.off_entry = arena_.alloc(best_entry);
    if (B.off_entry == Arena::kNone) { B.reqs.clear(); return B; }
    if (best_pairs > 0) {
      B.off_pair = arena_.alloc(be_->pair_bytes(best_pairs));
      B.P_reserved = B.off_pair == Arena::kNone ? 0 : best_pairs;
    }
    for (size_t k = 0; k < B.reqs.size(); k++) queue_.pop_front();
    return B;
  }

  // Release a batch's memory once its queued device work has ended.
  void release_batch(int slot, Batch& B) {
    be_->quiesce(slot);
    std::lock_guard<std::mutex> lk(mu_);
    if (B.off_entry != Arena::kNone) arena_.release(B.off_entry);
    if (B.off_pair != Arena::kNone) arena_.release(B.off_pair);
    B.off_entry = B.off_pair = Arena::kNone;
    cv_.notify_all();
  }

  Outcome run_batch(int slot, Batch& B, gut_status* out) {
    std::vector<gut_camera> cams;
    std::vector<float*> outs;
    for (auto* r : B.reqs)
      for (size_t c = 0; c < r->cams.size(); c++) { cams.push_back(r->cams[c]); outs.push_back(r->out[c]); }
    uint64_t P = 0;
    gut_status st = be_->count(slot, cams, outs, B.off_entry, &P);
    if (st != GUT_OK) { release_batch(slot, B); *out = st; return Outcome::Done; }
    if (P >= (uint64_t(1) << 32)) {  // pair offsets are 32-bit
      release_batch(slot, B);
      *out = GUT_E_CAPACITY;
      return Outcome::Done;
    }
    if ((int64_t)P > B.P_reserved) {
      std::unique_lock<std::mutex> lk(mu_);
      if (B.off_pair != Arena::kNone) {
        arena_.release(B.off_pair);
        B.off_pair = Arena::kNone;
        cv_.notify_all();
      }
      growing_++;
      while (true) {
        B.off_pair = arena_.alloc(be_->pair_bytes((int64_t)P));
        if (B.off_pair != Arena::kNone) break;
        if (busy_ - growing_ == 0) {  // every busy worker waits for memory: give way
          growing_--;
          const bool alone = busy_ == 1;
          const size_t need = al256(B.entry_bytes) + al256(be_->pair_bytes((int64_t)P));
          const size_t room = arena_.size() - al256(be_->resident_bytes());
          lk.unlock();
          release_batch(slot, B);
          lk.lock();
          if (B.reqs.size() == 1 && need > room) {  // cannot fit even in an empty arena
            *out = GUT_E_CAPACITY;
            return Outcome::Done;
          }
          for (size_t k = B.reqs.size(); k-- > 0;) { B.reqs[k]->state = 0; queue_.push_front(B.reqs[k]); }
          if (B.reqs.size() == 1) {
            B.reqs.front()->solo = true;
            B.reqs.front()->hint_pairs = (int64_t)P;
          } else if (alone) {  // split: the head request is retried alone, then the rest
            B.reqs.front()->solo = true;
            stats_.splits++;
          }
          stats_.requeued++;
          return Outcome::Requeued;
        }
        cv_.wait(lk);
      }
      growing_--;
      cv_.notify_all();  // new batches may start again
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      const int64_t E = be_->entries((int)cams.size());
      if (E > 0) pairs_per_entry_ = 0.8 * pairs_per_entry_ + 0.2 * ((double)P / (double)E);
    }
    st = be_->finish(slot, cams, outs, B.off_entry, B.off_pair, P);
    release_batch(slot, B);
    *out = st;
    return Outcome::Done;
  }

  void worker_main(int slot) {
    while (true) {
      Batch B;
      {
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
          if (!queue_.empty()) {
            B = take_batch();
            if (!B.reqs.empty()) break;
          } else if (stop_) {
            return;
          }
          cv_.wait(lk);
        }
        busy_++;
        for (auto* r : B.reqs) r->state = 1;
      }
      gut_status st = GUT_OK;
      const Outcome oc = run_batch(slot, B, &st);
      const auto now = Clock::now();
      {
        std::lock_guard<std::mutex> lk(mu_);
        busy_--;
        if (oc == Outcome::Done) {
          stats_.batches++;
          for (auto* r : B.reqs) {
            r->status = st;
            r->state = 2;
            r->t_done = now;
            if (st == GUT_OK) {
              stats_.completed++;
              stats_.cameras += (int64_t)r->cams.size();
              lat_ms_.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
            }
          }
          if (st != GUT_OK && st != GUT_E_CAPACITY && fatal_ == GUT_OK) fatal_ = st;
        }
      }
      cv_.notify_all();
    }
  }

  Backend* be_;
  const int max_slots_, max_batch_cams_, max_cams_;
  Arena arena_;
  size_t resident_off_ = Arena::kNone;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Request*> queue_;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs_;
  std::vector<std::thread> threads_;
  bool stop_ = false;
  int busy_ = 0, growing_ = 0;
  uint64_t next_id_ = 1;
  double pairs_per_entry_ = 4.0;  // running estimate used to reserve pair memory
  Clock::time_point t0_;
  std::vector<double> lat_ms_;
  SchedStats stats_;
  gut_status fatal_ = GUT_OK;
};

}  // namespace gut
