// Continuous-batching server over a resident scene (gut_serve_*).
//
// The scheduling -- FIFO queue, memory arena, batch formation, pair-buffer
// growth, worker threads, latency statistics -- is the device-independent
// Scheduler of serve_core.h.  This file is its HIP backend: one device arena
// of mem_budget_bytes allocated at creation (no hipMalloc after it), the
// scene's render records resident in it for the server's lifetime, and one
// stream plus a pinned staging area per execution slot.  A batch runs
// project -> count (one read-back) on the slot's stream, then, once its pair
// memory is reserved, sort -> persistent render.  Batches of different slots
// run concurrently on the device.
//
// Results are bitwise identical to rendering a request alone: a camera's tile
// lists, sort order (depth, then particle) and per-tile arithmetic do not
// depend on the other cameras of its batch.
#include <cstring>
#include <memory>
#include <vector>

#include "common.h"
#include "serve_core.h"

namespace gut {

constexpr size_t kStage = 64 * 1024;

// Device memory one batch needs before its pair count is known: the
// projection (rect, tiles, depth, rgb, mean, extent ellipse), the count
// phase's workspace, ranges and render order, and the launch tables.
static size_t batch_entry_bytes(int64_t n, int n_cams, int64_t T) {
  const int64_t E = n * (int64_t)n_cams;
  return al256(E * 8) + al256(E * 4) * 2 + al256(E * 12) + al256(E * 8) + al256(E * 16) +
         al256(bin_count_bytes(n, T)) + al256(T * 12) + al256(n_cams * sizeof(DevCam)) +
         al256(n_cams * sizeof(float*)) + al256(2 * (2 * kMaxCams + 1) * sizeof(int)) +
         al256(16 * sizeof(unsigned)) + 4096;
}

static size_t batch_pair_bytes(int64_t P) { return al256(P * 4) + al256(bin_pair_bytes(P)); }

class HipBackend {
 public:
  gut_scene scene;
  gut_params params;
  int device = 0, n_blocks = 1024;
  char* base = nullptr;
  size_t record_off = 0;

  struct Slot {
    hipStream_t stream = nullptr;
    void* pinned = nullptr;  // staging for camera tables and lists
    // state of the batch between count() and finish()
    std::vector<DevCam> dc;
    int64_t T = 0;
  };
  std::vector<Slot> slots;

  gut_status plan(const gut_camera* cams, int n_cams, size_t* entry_bytes) const {
    if (n_cams < 1 || n_cams > kMaxCams) {
      set_error("n_cams must be in [1, %d]", kMaxCams);
      return GUT_E_INVALID;
    }
    std::vector<DevCam> dc(n_cams);
    int64_t T = 0;
    gut_status st = prepare_cams(cams, n_cams, params, dc.data(), &T, nullptr);
    if (st != GUT_OK) return st;
    *entry_bytes = batch_entry_bytes(scene.n, n_cams, T);
    return GUT_OK;
  }
  int64_t entries(int n_cams) const { return scene.n * (int64_t)n_cams; }
  size_t pair_bytes(int64_t P) const { return batch_pair_bytes(P); }
  size_t resident_bytes() const { return al256((size_t)scene.n * 64); }

  struct EntryMem {
    gut_projected proj;
    char* cws;
    uint32_t* ranges;  // [T,2] ranges, then the render order
    DevCam* d_cams;
    float** d_outs;
    int* d_lists;
    unsigned* d_counters;
  };
  EntryMem carve(size_t off_entry, int nc, int64_t T) const {
    const int64_t E = scene.n * (int64_t)nc;
    char* b = base + off_entry;
    auto take = [&](size_t bytes) { char* p = b; b += al256(bytes); return p; };
    EntryMem m;
    m.proj = gut_projected{};
    m.proj.rect = (int16_t*)take(E * 8);
    m.proj.tiles = (uint32_t*)take(E * 4);
    m.proj.depth = (float*)take(E * 4);
    m.proj.rgb = (float*)take(E * 12);
    m.proj.mean2d = (float*)take(E * 8);
    m.proj.extent = (float*)take(E * 16);
    m.proj.record = (float*)(base + record_off);
    m.cws = take(bin_count_bytes(scene.n, T));
    m.ranges = (uint32_t*)take(T * 12);
    m.d_cams = (DevCam*)take(nc * sizeof(DevCam));
    m.d_outs = (float**)take(nc * sizeof(float*));
    m.d_lists = (int*)take(2 * (2 * kMaxCams + 1) * sizeof(int));
    m.d_counters = (unsigned*)take(16 * sizeof(unsigned));
    return m;
  }

  gut_status count(int slot, const std::vector<gut_camera>& cams, const std::vector<float*>& outs,
                   size_t off_entry, uint64_t* P) {
    Slot& W = slots[slot];
    const int nc = (int)cams.size();
    W.dc.assign(nc, DevCam{});
    gut_status st = prepare_cams(cams.data(), nc, params, W.dc.data(), &W.T, nullptr);
    if (st != GUT_OK) return st;
    EntryMem m = carve(off_entry, nc, W.T);
    hipStream_t s = W.stream;
    // camera and output tables through the slot's pinned staging area
    char* stage = (char*)W.pinned;
    std::memcpy(stage, W.dc.data(), nc * sizeof(DevCam));
    std::memcpy(stage + 32768, outs.data(), nc * sizeof(float*));
    GUT_HIP(hipMemcpyAsync(m.d_cams, stage, nc * sizeof(DevCam), hipMemcpyHostToDevice, s));
    GUT_HIP(hipMemcpyAsync(m.d_outs, stage + 32768, nc * sizeof(float*), hipMemcpyHostToDevice, s));
    if ((st = project_launch(&scene, W.dc.data(), nc, make_ut(params), make_thresholds(params), &m.proj,
                             false, s)) != GUT_OK)
      return st;
    if ((st = bin_count_launch(&m.proj, (int)scene.n, W.dc.data(), nc, W.T, params.tile_cull != 0, m.cws,
                               m.ranges, s)) != GUT_OK)
      return st;
    return bin_count_wait(P);
  }

  gut_status finish(int slot, const std::vector<gut_camera>& cams, const std::vector<float*>&,
                    size_t off_entry, size_t off_pair, uint64_t P) {
    Slot& W = slots[slot];
    const int nc = (int)cams.size();
    EntryMem m = carve(off_entry, nc, W.T);
    hipStream_t s = W.stream;
    char* pb = base + off_pair;
    uint32_t* ids = (uint32_t*)pb;
    char* pws = pb + al256((P > 0 ? P : 1) * 4);
    int* h_lists = (int*)((char*)W.pinned + 49152);
    gut_status st;
    if ((st = bin_sort_launch(&m.proj, (int)scene.n, W.dc.data(), nc, W.T, params.tile_cull != 0, m.cws,
                              (int64_t)P, pws, m.ranges, ids, s)) != GUT_OK ||
        (st = render_batch_launch(m.d_cams, W.dc.data(), nc, make_thresholds(params), (int)scene.n, m.ranges,
                                  m.ranges + 2 * W.T, ids, m.proj.record, m.proj.rgb, m.d_outs,
                                  m.d_counters, m.d_lists, h_lists, n_blocks, s)) != GUT_OK)
      return st;
    hipError_t he = hipStreamSynchronize(s);
    if (he != hipSuccess) {
      set_error("batch failed: %s", hipGetErrorString(he));
      return GUT_E_HIP;
    }
    return GUT_OK;
  }

  // queued work may still use the memory
  void quiesce(int slot) { (void)hipStreamSynchronize(slots[slot].stream); }
};

}  // namespace gut

struct gut_server {
  gut::HipBackend be;
  std::unique_ptr<gut::Scheduler<gut::HipBackend>> sched;
};

using namespace gut;

static void free_backend(HipBackend& be) {
  for (auto& w : be.slots) {
    if (w.stream) (void)hipStreamDestroy(w.stream);
    if (w.pinned) (void)hipHostFree(w.pinned);
  }
  be.slots.clear();
  if (be.base) (void)hipFree(be.base);
  be.base = nullptr;
}

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
  HipBackend& be = S->be;
  be.scene = *scene;
  be.params = *p;
  GUT_HIP(hipGetDevice(&be.device));
  hipDeviceProp_t prop;
  GUT_HIP(hipGetDeviceProperties(&prop, be.device));
  be.n_blocks = prop.multiProcessorCount * 8;
  GUT_HIP(hipMalloc((void**)&be.base, mem_budget_bytes));
  S->sched.reset(new Scheduler<HipBackend>(&be, mem_budget_bytes, max_slots, max_batch_cams, kMaxCams));
  be.record_off = S->sched->resident_offset();
  be.slots.resize(max_slots);
  hipStream_t s0 = nullptr;
  hipError_t he = hipStreamCreateWithFlags(&s0, hipStreamNonBlocking);
  st = he == hipSuccess ? record_launch(scene, (float*)(be.base + be.record_off), s0) : GUT_E_HIP;
  if (he == hipSuccess) he = hipStreamSynchronize(s0);
  if (s0) (void)hipStreamDestroy(s0);
  for (int w = 0; w < max_slots && st == GUT_OK && he == hipSuccess; w++) {
    he = hipStreamCreateWithFlags(&be.slots[w].stream, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipHostMalloc(&be.slots[w].pinned, kStage, hipHostMallocDefault);
  }
  if (st != GUT_OK || he != hipSuccess) {
    if (he != hipSuccess) set_error("gut_serve_create: %s", hipGetErrorString(he));
    S->sched.reset();
    free_backend(be);
    return st != GUT_OK ? st : GUT_E_HIP;
  }
  S->sched->start();
  *out = S.release();
  return GUT_OK;
}

extern "C" gut_status gut_serve_submit(gut_server* S, const gut_camera* cams, int32_t n_cams,
                                       float* const* out_rgb, uint64_t* request_id) {
  if (!S || !cams || !out_rgb || !request_id || n_cams < 1 || n_cams > kMaxCams) {
    set_error("bad gut_serve_submit arguments");
    return GUT_E_INVALID;
  }
  for (int c = 0; c < n_cams; c++)
    if (!out_rgb[c]) { set_error("out_rgb[%d] is NULL", c); return GUT_E_INVALID; }
  const char* why = nullptr;
  gut_status st = S->sched->submit(cams, n_cams, out_rgb, request_id, &why);
  if (why) set_error("%s", why);
  return st;
}

extern "C" gut_status gut_serve_poll(gut_server* S, uint64_t id, int32_t* done) {
  if (!S || !done) return GUT_E_INVALID;
  gut_status st = S->sched->poll(id, done);
  if (st == GUT_E_NOT_FOUND) set_error("unknown request %llu", (unsigned long long)id);
  return st;
}

extern "C" gut_status gut_serve_wait(gut_server* S, uint64_t id) {
  if (!S) return GUT_E_INVALID;
  gut_status st = S->sched->wait(id);
  if (st == GUT_E_NOT_FOUND) set_error("unknown request %llu", (unsigned long long)id);
  return st;
}

extern "C" gut_status gut_serve_latency(gut_server* S, uint64_t id, double* ms) {
  if (!S || !ms) return GUT_E_INVALID;
  return S->sched->latency(id, ms);
}

extern "C" gut_status gut_serve_stats(gut_server* S, gut_serve_metrics* m) {
  if (!S || !m) return GUT_E_INVALID;
  return S->sched->metrics(m);
}

extern "C" gut_status gut_serve_reset_stats(gut_server* S) {
  if (!S) return GUT_E_INVALID;
  S->sched->reset_stats();
  return GUT_OK;
}

extern "C" gut_status gut_serve_destroy(gut_server* S) {
  if (!S) return GUT_E_INVALID;
  S->sched->stop();  // workers drain the queue, then leave
  S->sched.reset();
  free_backend(S->be);
  delete S;
  return GUT_OK;
}
