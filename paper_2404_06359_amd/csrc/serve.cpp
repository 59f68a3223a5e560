// Decode-request server: continuous batching of mesh decodes over a
// device-resident pool of encoded meshes (host code, HIP runtime API).
//
// Requests name a mesh of the pool.  A scheduler thread admits pending
// requests in arrival order while their decoded output (3 bytes per strip
// triangle) fits into the caller's output arena -- the HBM budget for
// in-flight outputs -- and a launch slot is free.  Each slot owns a HIP stream
// (default priority) and one batch's mesh table and work list in pinned,
// coherent host memory that the kernel reads directly (no copy: a
// host-to-device copy call blocked the scheduler for milliseconds now and
// then).  The requests admitted together go out as one
// decode_meshlets_batched launch on that slot's stream, so up to
// `max_inflight` batches run on the device at once, and requests that arrive
// while others decode are admitted as soon as a slot and arena space free up.
// A finished request's output stays in the arena until the caller releases
// it.  Admission is strictly first-come first-served: a request that does not
// fit blocks the ones behind it (no starvation of large meshes).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"

using namespace gtsr;

namespace {

constexpr uint64_t kArenaAlign = 256;

// Arena bytes an output of `bytes` occupies (whole 256-byte units, at least one).
uint64_t arena_span(uint64_t bytes) {
  return std::max<uint64_t>(kArenaAlign, (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign);
}

uint64_t now_ns() {
  return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                      std::chrono::steady_clock::now().time_since_epoch())
                      .count());
}

// First-fit allocator over [0, size) with coalescing free list.
class Arena {
 public:
  explicit Arena(uint64_t size) : size_(size) {
    if (size) free_[0] = size;
  }
  bool alloc(uint64_t bytes, uint64_t& off) {
    bytes = arena_span(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const uint64_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = arena_span(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t used() const { return used_; }
  uint64_t size() const { return size_; }

 private:
  uint64_t size_, used_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

struct Request {
  uint64_t tag;
  uint32_t mesh;
  uint64_t off = 0, bytes = 0;
  uint64_t t_submit = 0, t_admit = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  gtsr_mesh_entry* h_table = nullptr;   // pinned, coherent host memory
  gtsr_work_item* h_work = nullptr;
  gtsr_mesh_entry* d_table = nullptr;   // the same memory, as the device addresses it
  gtsr_work_item* d_work = nullptr;
  std::vector<Request> reqs;
  bool busy = false;
};

struct MeshInfo {
  gtsr_mesh_entry entry;
  std::vector<uint32_t> cuts;   // work-item boundaries: meshlet indices, first 0, last meshlet_count
  uint64_t out_bytes;
};

}  // namespace

struct gtsr_server {
  gtsr_server_params p{};
  int device = 0;
  std::vector<MeshInfo> meshes;
  Arena arena{0};
  std::vector<Slot> slots;
  std::deque<Request> pending;
  std::unordered_map<uint64_t, std::pair<uint64_t, uint64_t>> live;   // tag -> arena range (admitted, unreleased)
  std::unordered_map<uint64_t, bool> known;                           // tags submitted and not yet released
  std::deque<gtsr_completion> done;
  std::mutex mu;
  std::condition_variable cv_done;
  std::atomic<bool> stop{false};
  std::atomic<uint64_t> wake{0};   // bumped by submit and release
  std::mutex wake_mu;
  std::condition_variable cv_wake;
  std::thread thread;
  std::string thread_error;
  gtsr_server_stats stats{};

  explicit gtsr_server(uint64_t arena_bytes) : arena(arena_bytes) {}
  void loop();
  bool retire();
  bool admit_and_launch();
};

namespace {

// Splits mesh m's meshlets into items of about target strip triangles, coarser
// if that would need more than max_items items.
void make_cuts(const gtsr_meshlet* ml, uint32_t count, uint32_t target, uint32_t max_items,
               std::vector<uint32_t>& cuts) {
  uint64_t total = 0;
  for (uint32_t i = 0; i < count; ++i) total += ml[i].tri_count;
  for (;;) {
    cuts.assign(1, 0);
    uint32_t m = 0;
    while (m < count) {
      uint64_t tris = 0;
      uint32_t end = m;
      while (end < count && (end == m || tris + ml[end].tri_count <= target)) tris += ml[end++].tri_count;
      cuts.push_back(end);
      m = end;
    }
    if (cuts.size() - 1 <= max_items) return;
    target = uint32_t(std::min<uint64_t>(0xFFFFFFFFull, std::max<uint64_t>(2ull * target, total / max_items + 256)));
  }
}

int hip_fail(const char* who, const char* what, hipError_t e) {
  return fail(GTSR_EHIP, std::string(who) + ": " + what + ": " + hipGetErrorString(e));
}

void free_slot(Slot& s) {
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  if (s.h_table) (void)hipHostFree(s.h_table);
  if (s.h_work) (void)hipHostFree(s.h_work);
  s = Slot{};
}

}  // namespace

// Moves finished batches' requests to the completion queue.
bool gtsr_server::retire() {
  bool any = false;
  for (Slot& s : slots) {
    if (!s.busy) continue;
    const hipError_t e = hipEventQuery(s.done);
    if (e == hipErrorNotReady) continue;
    const uint64_t t = now_ns();
    std::lock_guard<std::mutex> lk(mu);
    for (const Request& r : s.reqs) {
      gtsr_completion c{};
      c.tag = r.tag;
      c.mesh = r.mesh;
      c.status = e == hipSuccess ? GTSR_OK : GTSR_EHIP;
      c.out_offset = r.off;
      c.out_bytes = meshes[r.mesh].out_bytes;
      c.t_submit_ns = r.t_submit;
      c.t_admit_ns = r.t_admit;
      c.t_done_ns = t;
      done.push_back(c);
      stats.completed += 1;
      stats.strip_triangles += meshes[r.mesh].entry.strip_triangles;
    }
    s.reqs.clear();
    s.busy = false;
    any = true;
  }
  if (any) cv_done.notify_all();
  return any;
}

// Admits pending requests into a free slot and launches them as one batch.
bool gtsr_server::admit_and_launch() {
  Slot* slot = nullptr;
  for (Slot& s : slots)
    if (!s.busy) {
      slot = &s;
      break;
    }
  if (!slot) return false;
  uint32_t items = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    const uint64_t t = now_ns();
    while (!pending.empty() && slot->reqs.size() < p.max_batch) {
      Request& r = pending.front();
      const MeshInfo& mi = meshes[r.mesh];
      const uint32_t need = uint32_t(mi.cuts.size() - 1);
      if (items + need > p.max_items) break;
      uint64_t off = 0;
      if (mi.out_bytes && !arena.alloc(mi.out_bytes, off)) break;
      r.off = off;
      r.bytes = mi.out_bytes;
      r.t_admit = t;
      live[r.tag] = {off, mi.out_bytes};
      const uint32_t row = uint32_t(slot->reqs.size());
      gtsr_mesh_entry e = mi.entry;
      e.out = p.arena + off;
      slot->h_table[row] = e;
      for (size_t k = 0; k + 1 < mi.cuts.size(); ++k)
        slot->h_work[items++] = gtsr_work_item{row, mi.cuts[k], mi.cuts[k + 1], 0};
      slot->reqs.push_back(r);
      pending.pop_front();
    }
    if (slot->reqs.empty()) return false;
    stats.batches += 1;
    stats.max_batch_seen = std::max<uint64_t>(stats.max_batch_seen, slot->reqs.size());
    stats.max_arena_used = std::max<uint64_t>(stats.max_arena_used, arena.used());
  }
  // The table and work list were written above, before the launch: the kernel
  // reads them from host memory.
  const uint32_t rows = uint32_t(slot->reqs.size());
  hipError_t e = hipSuccess;
  int rc = decode_meshlets_batched(slot->d_table, rows, slot->d_work, items, nullptr, 0, &p.cfg, slot->stream);
  if (rc == GTSR_OK) {
    e = hipEventRecord(slot->done, slot->stream);
    if (e != hipSuccess) rc = GTSR_EHIP;
  }
  if (rc != GTSR_OK) {
    // The batch never reached the device: report its requests as failed.
    std::lock_guard<std::mutex> lk(mu);
    const uint64_t t = now_ns();
    for (const Request& r : slot->reqs) {
      gtsr_completion c{};
      c.tag = r.tag;
      c.mesh = r.mesh;
      c.status = rc;
      c.out_offset = r.off;
      c.out_bytes = r.bytes;
      c.t_submit_ns = r.t_submit;
      c.t_admit_ns = r.t_admit;
      c.t_done_ns = t;
      done.push_back(c);
    }
    slot->reqs.clear();
    cv_done.notify_all();
    return true;
  }
  slot->busy = true;
  return true;
}

void gtsr_server::loop() {
  if (hipSetDevice(device) != hipSuccess) {
    thread_error = "gtsr_server: cannot select the device";
    return;
  }
  while (!stop.load(std::memory_order_acquire)) {
    const uint64_t seen = wake.load(std::memory_order_acquire);
    bool progress = retire();
    while (admit_and_launch()) progress = true;
    if (progress || wake.load(std::memory_order_acquire) != seen) continue;
    bool inflight = false;
    for (const Slot& sl : slots) inflight = inflight || sl.busy;
    if (inflight) {
      // batches on the device: poll their events closely
      std::this_thread::yield();
      continue;
    }
    // nothing on the device: sleep until a submit or a release
    std::unique_lock<std::mutex> lk(wake_mu);
    cv_wake.wait_for(lk, std::chrono::milliseconds(1), [this, seen] {
      return wake.load(std::memory_order_acquire) != seen || stop.load(std::memory_order_acquire);
    });
  }
}

namespace {

void bump(gtsr_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->wake_mu);
    s->wake.fetch_add(1, std::memory_order_release);
  }
  s->cv_wake.notify_one();
}

}  // namespace

extern "C" int gtsr_server_create(const gtsr_mesh_entry* host_table, const gtsr_meshlet* const* host_meshlets,
                                  uint32_t mesh_count, const gtsr_server_params* params, gtsr_server** out) {
  const char* who = "gtsr_server_create";
  if (!out || !params || (mesh_count && (!host_table || !host_meshlets)))
    return fail(GTSR_EINVAL, std::string(who) + ": null argument");
  *out = nullptr;
  gtsr_server_params p = *params;
  if (!p.arena && p.arena_bytes) return fail(GTSR_EINVAL, std::string(who) + ": null arena");
  if (reinterpret_cast<uintptr_t>(p.arena) % kArenaAlign)
    return fail(GTSR_EINVAL, std::string(who) + ": arena must be 256-byte aligned");
  if (p.max_inflight == 0) p.max_inflight = 4;
  if (p.max_batch == 0) p.max_batch = 256;
  if (p.target_tris == 0) p.target_tris = 768;
  if (p.max_items == 0) p.max_items = 1u << 20;
  if (p.max_inflight > 8 || p.max_batch > 65536 || p.max_items > (1u << 26) || p.reserved || p.reserved2 ||
      (p.cfg.run_tris != 0 && p.cfg.run_tris != 1024 && p.cfg.run_tris != 1280) || p.cfg.waves_per_group > 16 ||
      p.cfg.groups_per_cu > 1024)
    return fail(GTSR_EINVAL, std::string(who) + ": parameter out of range");
  auto* s = new (std::nothrow) gtsr_server(p.arena_bytes);
  if (!s) return fail(GTSR_ENOMEM, std::string(who) + ": out of memory");
  s->p = p;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(GTSR_EHIP, std::string(who) + ": no device");
  }
  s->meshes.resize(mesh_count);
  for (uint32_t i = 0; i < mesh_count; ++i) {
    MeshInfo& mi = s->meshes[i];
    mi.entry = host_table[i];
    mi.entry.out = nullptr;
    mi.out_bytes = 3 * host_table[i].strip_triangles;
    if (host_table[i].meshlet_count && !host_meshlets[i]) {
      delete s;
      return fail(GTSR_EINVAL, std::string(who) + ": null meshlet array");
    }
    make_cuts(host_meshlets[i], host_table[i].meshlet_count, p.target_tris, p.max_items, mi.cuts);
  }
  s->slots.resize(p.max_inflight);
  int rc = GTSR_OK;
  for (Slot& sl : s->slots) {
    hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    const unsigned host_flags = hipHostMallocMapped | hipHostMallocCoherent;
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_table), p.max_batch * sizeof(gtsr_mesh_entry), host_flags);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_work), p.max_items * sizeof(gtsr_work_item), host_flags);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&sl.d_table), sl.h_table, 0);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&sl.d_work), sl.h_work, 0);
    if (e != hipSuccess) {
      rc = hip_fail(who, "slot resources", e);
      break;
    }
  }
  if (rc != GTSR_OK) {
    for (Slot& sl : s->slots) free_slot(sl);
    delete s;
    return rc;
  }
  s->thread = std::thread([s] { s->loop(); });
  *out = s;
  return ok();
}

extern "C" int gtsr_server_submit(gtsr_server* s, uint32_t mesh, uint64_t tag) {
  if (!s) return fail(GTSR_EINVAL, "gtsr_server_submit: null server");
  if (mesh >= s->meshes.size()) return fail(GTSR_EINVAL, "gtsr_server_submit: mesh out of range");
  const MeshInfo& mi = s->meshes[mesh];
  // (checked in the arena's 256-byte units: an output that fits only unrounded
  // could never be admitted and would block every request behind it)
  if (mi.out_bytes && arena_span(mi.out_bytes) > s->arena.size())
    return fail(GTSR_ELIMIT, "gtsr_server_submit: the mesh's output is larger than the arena");
  if (mi.cuts.size() - 1 > s->p.max_items)
    return fail(GTSR_ELIMIT, "gtsr_server_submit: the mesh needs more work items than a batch holds");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->known.emplace(tag, true).second) return fail(GTSR_EINVAL, "gtsr_server_submit: tag already in use");
    Request r;
    r.tag = tag;
    r.mesh = mesh;
    r.t_submit = now_ns();
    s->pending.push_back(r);
    s->stats.submitted += 1;
  }
  bump(s);
  return ok();
}

extern "C" int gtsr_server_poll(gtsr_server* s, gtsr_completion* out, uint32_t capacity, uint32_t* count,
                                uint32_t timeout_us) {
  if (!s || !count || (capacity && !out)) return fail(GTSR_EINVAL, "gtsr_server_poll: null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_us)
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [s] { return !s->done.empty(); });
  uint32_t n = 0;
  while (n < capacity && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  *count = n;
  if (!s->thread_error.empty()) return fail(GTSR_EHIP, s->thread_error);
  return ok();
}

extern "C" int gtsr_server_release(gtsr_server* s, uint64_t tag) {
  if (!s) return fail(GTSR_EINVAL, "gtsr_server_release: null server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->live.find(tag);
    if (it == s->live.end()) return fail(GTSR_EINVAL, "gtsr_server_release: no admitted request with this tag");
    for (const Slot& sl : s->slots)
      for (const Request& r : sl.reqs)
        if (r.tag == tag) return fail(GTSR_EINVAL, "gtsr_server_release: the request is still decoding");
    if (it->second.second) s->arena.release(it->second.first, it->second.second);
    s->live.erase(it);
    s->known.erase(tag);
  }
  bump(s);
  return ok();
}

extern "C" int gtsr_server_get_stats(gtsr_server* s, gtsr_server_stats* st) {
  if (!s || !st) return fail(GTSR_EINVAL, "gtsr_server_get_stats: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->stats;
  st->pending = s->pending.size();
  st->arena_used = s->arena.used();
  return ok();
}

extern "C" int gtsr_server_replay(gtsr_server* s, const uint64_t* arrival_ns, const uint32_t* meshes, uint32_t n,
                                  uint64_t tag_base, gtsr_completion* out, uint64_t* start_ns) {
  const char* who = "gtsr_server_replay";
  if (!s || (n && (!arrival_ns || !meshes || !out))) return fail(GTSR_EINVAL, std::string(who) + ": null argument");
  for (uint32_t i = 1; i < n; ++i)
    if (arrival_ns[i] < arrival_ns[i - 1]) return fail(GTSR_EINVAL, std::string(who) + ": arrivals not sorted");
  const uint64_t t0 = now_ns();
  if (start_ns) *start_ns = t0;
  uint32_t next = 0, finished = 0;
  std::vector<gtsr_completion> buf(256);
  while (finished < n) {
    const uint64_t t = now_ns() - t0;
    while (next < n && arrival_ns[next] <= t) {
      if (int rc = gtsr_server_submit(s, meshes[next], tag_base + next)) return rc;
      ++next;
    }
    uint32_t got = 0;
    if (int rc = gtsr_server_poll(s, buf.data(), uint32_t(buf.size()), &got, 0)) return rc;
    for (uint32_t k = 0; k < got; ++k) {
      const gtsr_completion& c = buf[k];
      if (c.tag < tag_base || c.tag - tag_base >= n) return fail(GTSR_EINVAL, std::string(who) + ": foreign completion");
      out[c.tag - tag_base] = c;
      if (c.status != GTSR_OK) return fail(c.status, std::string(who) + ": a decode failed");
      if (int rc = gtsr_server_release(s, c.tag)) return rc;
      ++finished;
    }
    if (!got) std::this_thread::yield();
  }
  return ok();
}

extern "C" void gtsr_server_destroy(gtsr_server* s) {
  if (!s) return;
  s->stop.store(true, std::memory_order_release);
  bump(s);
  if (s->thread.joinable()) s->thread.join();
  for (Slot& sl : s->slots) {
    if (sl.busy) (void)hipEventSynchronize(sl.done);
    free_slot(sl);
  }
  delete s;
}
