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
// fit blocks the ones behind it (no starvation of large meshes) until it is
// admitted or withdrawn.  The admission policy itself lives in admission.h,
// free of device calls; this file adds the slots' device resources and the
// scheduler thread.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "admission.h"

using namespace gtsr;
using serve::Scheduler;

namespace {

uint64_t now_ns() {
  return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                      std::chrono::steady_clock::now().time_since_epoch())
                      .count());
}

// A launch slot's device resources; which requests its batch holds is the
// scheduler's business.
struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  gtsr_mesh_entry* h_table = nullptr;   // pinned, coherent host memory
  gtsr_work_item* h_work = nullptr;
  gtsr_mesh_entry* d_table = nullptr;   // the same memory, as the device addresses it
  gtsr_work_item* d_work = nullptr;
};

}  // namespace

struct gtsr_server {
  gtsr_server_params p{};
  int device = 0;
  Scheduler sched;
  std::vector<Slot> slots;
  std::mutex mu;                         // guards sched
  std::condition_variable cv_done;
  std::atomic<bool> stop{false};
  std::atomic<uint64_t> wake{0};   // bumped by submit, cancel and release
  std::mutex wake_mu;
  std::condition_variable cv_wake;
  std::thread thread;
  std::string thread_error;              // set by the scheduler thread under mu

  explicit gtsr_server(const gtsr_server_params& prm)
      : p(prm), sched(prm.arena, prm.arena_bytes, prm.max_inflight, prm.max_batch, prm.max_items) {}
  void loop();
  bool retire();
  bool admit_and_launch();
};

namespace {

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

// Completes the batches the device has finished.  (Only this thread changes
// which slots are busy, so reading that without the lock is safe.)
bool gtsr_server::retire() {
  bool any = false;
  for (uint32_t i = 0; i < slots.size(); ++i) {
    if (!sched.busy(i)) continue;
    const hipError_t e = hipEventQuery(slots[i].done);
    if (e == hipErrorNotReady) continue;
    const uint64_t t = now_ns();
    std::lock_guard<std::mutex> lk(mu);
    sched.finish(i, e == hipSuccess ? GTSR_OK : GTSR_EHIP, t);
    any = true;
  }
  if (any) cv_done.notify_all();
  return any;
}

// Admits queued requests into a free slot and launches them as one batch.
bool gtsr_server::admit_and_launch() {
  const int k = sched.free_slot();
  if (k < 0) return false;
  Slot& slot = slots[k];
  uint32_t rows = 0, items = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    items = sched.admit(uint32_t(k), slot.h_table, slot.h_work, now_ns(), &rows);
  }
  if (!rows) return false;
  // The table and work list were written above, before the launch: the kernel
  // reads them from host memory.
  int rc = decode_meshlets_batched(slot.d_table, rows, slot.d_work, items, nullptr, 0, &p.cfg, slot.stream);
  if (rc == GTSR_OK && hipEventRecord(slot.done, slot.stream) != hipSuccess) {
    // The launch is queued but cannot be tracked: wait for it, so that no
    // arena range is handed out again while the kernel may still write it.
    (void)hipStreamSynchronize(slot.stream);
    rc = GTSR_EHIP;
  }
  if (rc != GTSR_OK) {
    // The batch did not complete as tracked work: report its requests as failed.
    {
      std::lock_guard<std::mutex> lk(mu);
      sched.finish(uint32_t(k), rc, now_ns());
    }
    cv_done.notify_all();
  }
  return true;
}

void gtsr_server::loop() {
  if (hipSetDevice(device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(mu);
    thread_error = "gtsr_server: cannot select the device";
    return;
  }
  while (!stop.load(std::memory_order_acquire)) {
    const uint64_t seen = wake.load(std::memory_order_acquire);
    bool progress = retire();
    while (admit_and_launch()) progress = true;
    if (progress || wake.load(std::memory_order_acquire) != seen) continue;
    if (sched.any_busy()) {
      // batches on the device: poll their events closely
      std::this_thread::yield();
      continue;
    }
    // nothing on the device: sleep until a submit, a cancel or a release
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
  if (reinterpret_cast<uintptr_t>(p.arena) % serve::kArenaAlign)
    return fail(GTSR_EINVAL, std::string(who) + ": arena must be 256-byte aligned");
  if (p.max_inflight == 0) p.max_inflight = 4;
  if (p.max_batch == 0) p.max_batch = 256;
  if (p.target_tris == 0) p.target_tris = 768;
  if (p.max_items == 0) p.max_items = 1u << 20;
  if (p.max_inflight > 8 || p.max_batch > 65536 || p.max_items > (1u << 26) || p.reserved || p.reserved2 ||
      (p.cfg.run_tris != 0 && p.cfg.run_tris != 1024 && p.cfg.run_tris != 1280) || p.cfg.waves_per_group > 16 ||
      p.cfg.groups_per_cu > 1024)
    return fail(GTSR_EINVAL, std::string(who) + ": parameter out of range");
  for (uint32_t i = 0; i < mesh_count; ++i)
    if (host_table[i].meshlet_count && !host_meshlets[i])
      return fail(GTSR_EINVAL, std::string(who) + ": null meshlet array");
  auto* s = new (std::nothrow) gtsr_server(p);
  if (!s) return fail(GTSR_ENOMEM, std::string(who) + ": out of memory");
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(GTSR_EHIP, std::string(who) + ": no device");
  }
  s->sched.meshes.resize(mesh_count);
  for (uint32_t i = 0; i < mesh_count; ++i) {
    serve::MeshInfo& mi = s->sched.meshes[i];
    mi.entry = host_table[i];
    mi.entry.out = nullptr;
    mi.out_bytes = 3 * host_table[i].strip_triangles;
    serve::make_cuts(host_meshlets[i], host_table[i].meshlet_count, p.target_tris, p.max_items, mi.cuts);
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
  const char* why = "";
  int rc;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    rc = s->sched.submit(mesh, tag, now_ns(), &why);
  }
  if (rc != GTSR_OK) return fail(rc, std::string("gtsr_server_submit: ") + why);
  bump(s);
  return ok();
}

extern "C" int gtsr_server_cancel(gtsr_server* s, uint64_t tag) {
  if (!s) return fail(GTSR_EINVAL, "gtsr_server_cancel: null server");
  const char* why = "";
  int rc;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    rc = s->sched.cancel(tag, now_ns(), &why);
  }
  if (rc != GTSR_OK) return fail(rc, std::string("gtsr_server_cancel: ") + why);
  s->cv_done.notify_all();
  bump(s);
  return ok();
}

extern "C" int gtsr_server_poll(gtsr_server* s, gtsr_completion* out, uint32_t capacity, uint32_t* count,
                                uint32_t timeout_us) {
  if (!s || !count || (capacity && !out)) return fail(GTSR_EINVAL, "gtsr_server_poll: null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->sched.has_completions() && timeout_us)
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [s] { return s->sched.has_completions(); });
  *count = s->sched.poll(out, capacity);
  if (!s->thread_error.empty()) return fail(GTSR_EHIP, s->thread_error);
  return ok();
}

extern "C" int gtsr_server_release(gtsr_server* s, uint64_t tag) {
  if (!s) return fail(GTSR_EINVAL, "gtsr_server_release: null server");
  const char* why = "";
  int rc;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    rc = s->sched.release(tag, &why);
  }
  if (rc != GTSR_OK) return fail(rc, std::string("gtsr_server_release: ") + why);
  bump(s);
  return ok();
}

extern "C" int gtsr_server_get_stats(gtsr_server* s, gtsr_server_stats* st) {
  if (!s || !st) return fail(GTSR_EINVAL, "gtsr_server_get_stats: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->sched.stats();
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
  for (uint32_t i = 0; i < s->slots.size(); ++i) {
    if (s->sched.busy(i)) (void)hipEventSynchronize(s->slots[i].done);
    free_slot(s->slots[i]);
  }
  delete s;
}
