// Host-only tests of the serving scheduler (serve_core.h) with a fake device
// backend: arena, admission, batch formation, pair-buffer growth under
// contention, batch splitting, error paths and statistics.  Built with g++
// (optionally under AddressSanitizer/UBSan or ThreadSanitizer) by
// tests/test_serve_core_host.py; exits non-zero on the first failure.
//
// The fake backend reads a camera's pair count from its fx, fails a batch
// whose camera has cx < 0, and keeps a shadow of the arena regions each slot
// is using, so that two batches sharing memory is caught.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "serve_core.h"

using namespace gut;

#define CHECK(cond)                                                            \
  do {                                                                         \
    if (!(cond)) {                                                             \
      std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);     \
      std::exit(1);                                                            \
    }                                                                          \
  } while (0)

struct Region { size_t off, bytes; };

struct FakeBackend {
  int64_t n = 10;
  size_t entry_per_cam = 200000;
  size_t pair_unit = 16;
  int sleep_us = 200;
  // the first `barrier` calls of count() wait until that many have arrived
  int barrier = 0;
  std::mutex mu;
  std::condition_variable cv;
  int arrived = 0;
  std::vector<std::vector<Region>> live;  // per slot
  std::vector<int> finished_tags;          // out[0] tag of each finished batch, in order
  std::atomic<int> counts{0}, finishes{0};

  explicit FakeBackend(int slots) : live(slots) {}

  gut_status plan(const gut_camera* cams, int n_cams, size_t* entry) const {
    for (int c = 0; c < n_cams; c++)
      if (cams[c].width <= 0 || cams[c].height <= 0) return GUT_E_INVALID;
    *entry = entry_per_cam * (size_t)n_cams;
    return GUT_OK;
  }
  int64_t entries(int n_cams) const { return n * n_cams; }
  size_t pair_bytes(int64_t P) const { return (size_t)P * pair_unit; }
  size_t resident_bytes() const { return (size_t)n * 64; }

  void claim(int slot, size_t off, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    for (size_t s = 0; s < live.size(); s++)
      for (auto& r : live[s])
        CHECK(off + bytes <= r.off || r.off + r.bytes <= off);  // no two batches share memory
    live[slot].push_back({off, bytes});
  }

  gut_status count(int slot, const std::vector<gut_camera>& cams, const std::vector<float*>&,
                   size_t off_entry, uint64_t* P) {
    claim(slot, off_entry, entry_per_cam * cams.size());
    counts++;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (arrived < barrier) {
        arrived++;
        cv.notify_all();
        // system_clock: its timed wait is the one thread checkers understand
        CHECK(cv.wait_until(lk, std::chrono::system_clock::now() + std::chrono::seconds(10),
                            [&] { return arrived >= barrier; }));
      }
    }
    std::this_thread::sleep_for(std::chrono::microseconds(sleep_us));
    uint64_t p = 0;
    for (auto& c : cams) {
      if (c.cx < 0) return GUT_E_HIP;
      p += (uint64_t)c.fx;
    }
    *P = p;
    return GUT_OK;
  }

  gut_status finish(int slot, const std::vector<gut_camera>& cams, const std::vector<float*>& outs,
                    size_t, size_t off_pair, uint64_t P) {
    if (P > 0) claim(slot, off_pair, pair_bytes((int64_t)P));
    std::this_thread::sleep_for(std::chrono::microseconds(sleep_us));
    for (size_t c = 0; c < cams.size(); c++) outs[c][0] = (float)cams[c].fy;  // "render"
    std::lock_guard<std::mutex> lk(mu);
    finished_tags.push_back((int)cams[0].fy);
    finishes++;
    return GUT_OK;
  }

  void quiesce(int slot) {
    std::lock_guard<std::mutex> lk(mu);
    live[slot].clear();
  }
};

static gut_camera cam(double pairs, int tag, bool fail = false) {
  gut_camera c;
  std::memset(&c, 0, sizeof(c));
  c.width = 64;
  c.height = 48;
  c.fx = pairs;
  c.fy = tag;
  c.cx = fail ? -1.0 : 1.0;
  return c;
}

using Sched = Scheduler<FakeBackend>;

static void wait_all(Sched& S, const std::vector<uint64_t>& ids, std::vector<gut_status>* st) {
  for (uint64_t id : ids) {
    int32_t done = 0;
    gut_status s = S.wait_for(id, 20000.0, &done);
    CHECK(done == 1);  // a hang fails here instead of blocking the test
    if (st) st->push_back(s);
  }
}

static void test_arena() {
  Arena A;
  A.init(4096);
  size_t a = A.alloc(100), b = A.alloc(256), c = A.alloc(1000);
  CHECK(a == 0 && b == 256 && c == 512);
  CHECK(A.used() == 256 + 256 + 1024);
  CHECK(A.alloc(4096) == Arena::kNone);
  CHECK(A.release(b));
  CHECK(!A.release(b));
  CHECK(!A.release(12345));
  CHECK(A.alloc(200) == 256);  // first fit reuses the hole
  CHECK(A.release(256));
  CHECK(A.release(a));          // merges with the hole after it
  CHECK(A.largest_free() == 4096 - 1536);
  CHECK(A.alloc(512) == 0);
  CHECK(A.release(0));
  CHECK(A.release(c));          // everything coalesces
  CHECK(A.free_blocks() == 1 && A.largest_free() == 4096 && A.used() == 0);
  CHECK(A.peak() == 1536);
  CHECK(A.alloc(0) == 0);       // zero bytes still get a distinct block
  std::printf("arena ok\n");
}

static void test_admission_and_errors() {
  FakeBackend be(1);
  Sched S(&be, 640 + 300000, 1, 4, 64);
  S.start();
  std::vector<gut_camera> two = {cam(10, 1), cam(10, 2)};
  std::vector<float> o(2);
  float* outs[2] = {&o[0], &o[1]};
  uint64_t id = 0;
  const char* why = nullptr;
  CHECK(S.submit(two.data(), 2, outs, &id, &why) == GUT_E_ADMISSION);  // 400000 > budget
  CHECK(why != nullptr);
  gut_camera bad = cam(10, 1);
  bad.width = 0;
  CHECK(S.submit(&bad, 1, outs, &id, nullptr) == GUT_E_INVALID);
  int32_t done = 0;
  CHECK(S.poll(999, &done) == GUT_E_NOT_FOUND);
  CHECK(S.wait(999) == GUT_E_NOT_FOUND);
  double ms = 0;
  CHECK(S.latency(999, &ms) == GUT_E_NOT_FOUND);
  // a device failure: the batch's requests fail, the status is sticky, and
  // later requests still run
  gut_camera f = cam(10, 3, true);
  uint64_t idf = 0, idg = 0;
  CHECK(S.submit(&f, 1, outs, &idf, nullptr) == GUT_OK);
  std::vector<gut_status> st;
  wait_all(S, {idf}, &st);
  CHECK(st[0] == GUT_E_HIP);
  gut_camera g = cam(10, 4);
  CHECK(S.submit(&g, 1, outs, &idg, nullptr) == GUT_OK);
  st.clear();
  wait_all(S, {idg}, &st);
  CHECK(st[0] == GUT_OK && o[0] == 4.0f);
  gut_serve_metrics m;
  CHECK(S.metrics(&m) == GUT_E_HIP);
  CHECK(m.rejected == 1 && m.completed == 1 && m.submitted == 2);
  S.stop();
  CHECK(S.arena_used() == al256(640));
  std::printf("admission and errors ok\n");
}

static void test_batching_fifo() {
  FakeBackend be(1);
  Sched S(&be, 640 + 4000000, 1, 2, 64);
  std::vector<float> o(5);
  std::vector<uint64_t> ids;
  for (int r = 0; r < 5; r++) {  // queued before any worker runs: batching is deterministic
    gut_camera c = cam(100, r + 1);
    float* out = &o[r];
    uint64_t id = 0;
    CHECK(S.submit(&c, 1, &out, &id, nullptr) == GUT_OK);
    ids.push_back(id);
  }
  S.start();
  std::vector<gut_status> st;
  wait_all(S, ids, &st);
  for (int r = 0; r < 5; r++) CHECK(st[r] == GUT_OK && o[r] == (float)(r + 1));
  CHECK(S.counters().batches == 3);  // [1,2], [3,4], [5]
  CHECK((be.finished_tags == std::vector<int>{1, 3, 5}));
  gut_serve_metrics m;
  CHECK(S.metrics(&m) == GUT_OK);
  CHECK(m.completed == 5 && m.cameras == 5 && m.p50_ms <= m.p99_ms && m.p99_ms <= m.max_ms);
  S.reset_stats();
  CHECK(S.metrics(&m) == GUT_OK && m.completed == 0);
  int32_t done = 0;
  CHECK(S.poll(ids[0], &done) == GUT_E_NOT_FOUND);  // completed requests were forgotten
  S.stop();
  std::printf("batching ok\n");
}

// Two slots, each batch's entry memory fits, but after counting both need
// more pair memory than is free while the other holds its entry memory: one
// gives way (requeues), the other grows, and both complete.
static void test_growth_contention() {
  for (int rep = 0; rep < 20; rep++) {
    FakeBackend be(2);
    be.barrier = 2;
    be.sleep_us = 50;
    const size_t res = al256(640), entry = 200000, reserve = al256((4 * 10 * 5 / 4 + 1024) * 16);
    const size_t budget = res + 2 * (entry + reserve) + 100000;
    Sched S(&be, budget, 2, 1, 64);
    std::vector<float> o(2);
    std::vector<uint64_t> ids;
    for (int r = 0; r < 2; r++) {
      gut_camera c = cam(210000 / 16, r + 1);
      float* out = &o[r];
      uint64_t id = 0;
      CHECK(S.submit(&c, 1, &out, &id, nullptr) == GUT_OK);
      ids.push_back(id);
    }
    S.start();
    std::vector<gut_status> st;
    wait_all(S, ids, &st);
    CHECK(st[0] == GUT_OK && st[1] == GUT_OK);
    CHECK(o[0] == 1.0f && o[1] == 2.0f);
    CHECK(S.counters().requeued >= 1);
    S.stop();
    CHECK(S.arena_used() == res && S.arena_free_blocks() == 1);
  }
  std::printf("growth under contention ok\n");
}

// A merged batch whose pairs cannot fit even alone is split; each request
// then runs alone.  A single request that cannot fit fails with
// GUT_E_CAPACITY, which is not sticky.
static void test_split_and_capacity() {
  FakeBackend be(1);
  const size_t res = al256(640);
  Sched S(&be, res + 534368 - 640, 1, 2, 64);
  std::vector<float> o(3);
  std::vector<uint64_t> ids;
  for (int r = 0; r < 2; r++) {
    gut_camera c = cam(10000, r + 1);  // 160000 bytes of pairs each
    float* out = &o[r];
    uint64_t id = 0;
    CHECK(S.submit(&c, 1, &out, &id, nullptr) == GUT_OK);
    ids.push_back(id);
  }
  gut_camera big = cam(1000000, 3);  // 16 MB of pairs: never fits
  float* out = &o[2];
  uint64_t idb = 0;
  CHECK(S.submit(&big, 1, &out, &idb, nullptr) == GUT_OK);
  ids.push_back(idb);
  S.start();
  std::vector<gut_status> st;
  wait_all(S, ids, &st);
  CHECK(st[0] == GUT_OK && st[1] == GUT_OK && st[2] == GUT_E_CAPACITY);
  CHECK(o[0] == 1.0f && o[1] == 2.0f);
  CHECK(S.counters().splits >= 1);
  gut_serve_metrics m;
  CHECK(S.metrics(&m) == GUT_OK);  // capacity failures are not device failures
  S.stop();
  CHECK(S.arena_used() == res);
  std::printf("split and capacity ok\n");
}

// Many requests from several client threads over four slots: all complete,
// memory is never shared, and the arena ends with the resident block only.
static void test_stress() {
  FakeBackend be(4);
  be.sleep_us = 20;
  const size_t res = al256(640);
  Sched S(&be, res + 3000000, 4, 3, 64);
  S.start();
  std::vector<float> o(400);
  std::vector<std::vector<uint64_t>> ids(4);
  std::vector<std::thread> th;
  for (int t = 0; t < 4; t++)
    th.emplace_back([&, t] {
      unsigned x = 12345u + t;
      for (int r = 0; r < 100; r++) {
        x = x * 1103515245u + 12345u;
        const int nc = 1 + (int)((x >> 16) % 3);
        std::vector<gut_camera> cs;
        std::vector<float*> outs;
        for (int c = 0; c < nc; c++) {
          x = x * 1103515245u + 12345u;
          cs.push_back(cam(1000 + (x >> 16) % 40000, t * 100 + r));
          outs.push_back(&o[t * 100 + r]);
        }
        uint64_t id = 0;
        CHECK(S.submit(cs.data(), nc, outs.data(), &id, nullptr) == GUT_OK);
        ids[t].push_back(id);
      }
    });
  for (auto& t : th) t.join();
  for (int t = 0; t < 4; t++) {
    std::vector<gut_status> st;
    wait_all(S, ids[t], &st);
    for (auto s : st) {
      if (s != GUT_OK) std::fprintf(stderr, "status %d\n", (int)s);
      CHECK(s == GUT_OK);
    }
  }
  for (int k = 0; k < 400; k++) CHECK(o[k] == (float)k);
  gut_serve_metrics m;
  CHECK(S.metrics(&m) == GUT_OK && m.completed == 400);
  S.stop();
  CHECK(S.arena_used() == res && S.arena_free_blocks() == 1);
  std::printf("stress ok (%lld batches, %lld requeued)\n", (long long)m.batches,
              (long long)S.counters().requeued);
}

// Stopping drains the queue first.
static void test_stop_drains() {
  FakeBackend be(2);
  Sched S(&be, al256(640) + 2000000, 2, 1, 64);
  std::vector<float> o(6);
  std::vector<uint64_t> ids;
  for (int r = 0; r < 6; r++) {
    gut_camera c = cam(500, r + 1);
    float* out = &o[r];
    uint64_t id = 0;
    CHECK(S.submit(&c, 1, &out, &id, nullptr) == GUT_OK);
    ids.push_back(id);
  }
  S.start();
  S.stop();
  for (int r = 0; r < 6; r++) CHECK(o[r] == (float)(r + 1));
  CHECK(be.finishes.load() == 6);
  std::printf("stop drains ok\n");
}

int main() {
  test_arena();
  test_admission_and_errors();
  test_batching_fifo();
  test_growth_contention();
  test_split_and_capacity();
  test_stress();
  test_stop_drains();
  std::printf("ALL OK\n");
  return 0;
}
