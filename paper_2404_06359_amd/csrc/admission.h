// Admission and batching state of the decode-request server, with no device
// calls: the arena allocator, the first-come first-served queue, the batches
// of the launch slots and the completion queue.  The server's scheduler
// thread drives it under the server's lock and does the device work (the
// slots' streams, launches and completion events) itself, so the policy can
// be exercised on the host alone.  Not thread-safe by itself.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "gtsr.h"

namespace gtsr {
namespace serve {

constexpr uint64_t kArenaAlign = 256;

// Arena bytes an output of `bytes` occupies (whole 256-byte units, at least one).
inline uint64_t arena_span(uint64_t bytes) {
  return std::max<uint64_t>(kArenaAlign, (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign);
}

// First-fit allocator over [0, size) with a coalescing free list.
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
  size_t free_ranges() const { return free_.size(); }

 private:
  uint64_t size_, used_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

// A pool mesh as the scheduler sees it: its table row (device stream
// pointers), its work-item boundaries and its output size.
struct MeshInfo {
  gtsr_mesh_entry entry;
  std::vector<uint32_t> cuts;   // work-item boundaries: meshlet indices, first 0, last meshlet_count
  uint64_t out_bytes;
};

// Splits a mesh's meshlets into items of about `target` strip triangles,
// coarser if that would need more than max_items items.  A mesh that needs
// more even at the largest target keeps that split; submit refuses it.
inline void make_cuts(const gtsr_meshlet* ml, uint32_t count, uint32_t target, uint32_t max_items,
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
    if (cuts.size() - 1 <= max_items || target == 0xFFFFFFFFu) return;
    target = uint32_t(std::min<uint64_t>(0xFFFFFFFFull, std::max<uint64_t>(2ull * target, total / max_items + 256)));
  }
}

struct Request {
  uint64_t tag;
  uint32_t mesh;
  uint64_t off = 0, bytes = 0;
  uint64_t t_submit = 0, t_admit = 0;
};

class Scheduler {
 public:
  // arena_base: the device address of arena offset 0 (written into the
  // table rows); slots: launch slots; max_batch / max_items: requests and
  // work items one batch may hold.
  Scheduler(uint8_t* arena_base, uint64_t arena_bytes, uint32_t slots, uint32_t max_batch, uint32_t max_items)
      : base_(arena_base), arena_(arena_bytes), slots_(slots), max_batch_(max_batch), max_items_(max_items) {}

  std::vector<MeshInfo> meshes;

  // Queues a request.  GTSR_EINVAL: mesh out of range or tag in use;
  // GTSR_ELIMIT: the output can never fit the arena (checked in its 256-byte
  // units: an output that fits only unrounded would block every request
  // behind it forever), or the mesh needs more work items than a batch holds.
  int submit(uint32_t mesh, uint64_t tag, uint64_t now, const char** why) {
    if (mesh >= meshes.size()) return say(why, "mesh out of range", GTSR_EINVAL);
    const MeshInfo& mi = meshes[mesh];
    if (mi.out_bytes && arena_span(mi.out_bytes) > arena_.size())
      return say(why, "the mesh's output is larger than the arena", GTSR_ELIMIT);
    if (mi.cuts.size() - 1 > max_items_)
      return say(why, "the mesh needs more work items than a batch holds", GTSR_ELIMIT);
    if (!known_.insert(tag).second) return say(why, "tag already in use", GTSR_EINVAL);
    Request r;
    r.tag = tag;
    r.mesh = mesh;
    r.t_submit = now;
    pending_.push_back(r);
    stats_.submitted += 1;
    return GTSR_OK;
  }

  // Withdraws a request that has not been admitted: it leaves the queue (so
  // the requests behind it may be admitted), its completion carries
  // GTSR_ECANCELED and no output, and its tag is free at once.
  // GTSR_EBUSY: already admitted (it completes normally and must be
  // released); GTSR_EINVAL: no such tag.
  int cancel(uint64_t tag, uint64_t now, const char** why) {
    for (auto it = pending_.begin(); it != pending_.end(); ++it) {
      if (it->tag != tag) continue;
      gtsr_completion c{};
      c.tag = tag;
      c.mesh = it->mesh;
      c.status = GTSR_ECANCELED;
      c.t_submit_ns = it->t_submit;
      c.t_done_ns = now;
      done_.push_back(c);
      pending_.erase(it);
      known_.erase(tag);
      stats_.cancelled += 1;
      return GTSR_OK;
    }
    if (known_.count(tag)) return say(why, "the request was already admitted", GTSR_EBUSY);
    return say(why, "no request with this tag", GTSR_EINVAL);
  }

  // Gives a finished request's arena range back.  GTSR_EINVAL: no admitted
  // request with this tag, or it is still in a batch that has not finished.
  int release(uint64_t tag, const char** why) {
    auto it = live_.find(tag);
    if (it == live_.end()) return say(why, "no admitted request with this tag", GTSR_EINVAL);
    for (const Slot& s : slots_)
      for (const Request& r : s.reqs)
        if (r.tag == tag) return say(why, "the request is still decoding", GTSR_EINVAL);
    if (it->second.second) arena_.release(it->second.first, it->second.second);
    live_.erase(it);
    known_.erase(tag);
    return GTSR_OK;
  }

  // Index of a slot with no batch, or -1.
  int free_slot() const {
    for (size_t i = 0; i < slots_.size(); ++i)
      if (!slots_[i].busy) return int(i);
    return -1;
  }
  bool busy(uint32_t slot) const { return slots_[slot].busy; }
  bool any_busy() const {
    for (const Slot& s : slots_)
      if (s.busy) return true;
    return false;
  }

  // Admits queued requests in arrival order into free slot `slot` while the
  // batch has room (max_batch requests, max_items work items) and each
  // output fits the arena; the first that does not fit stops admission (no
  // request overtakes another).  Writes the batch's mesh table (row i =
  // request i, its out field pointing into the arena) and work list, and
  // marks the slot busy when it admitted any.  Returns the work-item count
  // (0 = nothing admitted); *rows receives the request count.
  uint32_t admit(uint32_t slot, gtsr_mesh_entry* table, gtsr_work_item* work, uint64_t now, uint32_t* rows) {
    Slot& s = slots_[slot];
    uint32_t items = 0;
    *rows = 0;
    if (s.busy) return 0;
    while (!pending_.empty() && s.reqs.size() < max_batch_) {
      Request& r = pending_.front();
      const MeshInfo& mi = meshes[r.mesh];
      const uint32_t need = uint32_t(mi.cuts.size() - 1);
      if (items + need > max_items_) break;
      uint64_t off = 0;
      if (mi.out_bytes && !arena_.alloc(mi.out_bytes, off)) break;
      r.off = off;
      r.bytes = mi.out_bytes;
      r.t_admit = now;
      live_[r.tag] = {off, mi.out_bytes};
      const uint32_t row = uint32_t(s.reqs.size());
      gtsr_mesh_entry e = mi.entry;
      e.out = base_ + off;
      table[row] = e;
      for (size_t k = 0; k + 1 < mi.cuts.size(); ++k) work[items++] = gtsr_work_item{row, mi.cuts[k], mi.cuts[k + 1], 0};
      s.reqs.push_back(r);
      pending_.pop_front();
    }
    if (s.reqs.empty()) return 0;
    s.busy = true;
    *rows = uint32_t(s.reqs.size());
    stats_.batches += 1;
    stats_.max_batch_seen = std::max<uint64_t>(stats_.max_batch_seen, s.reqs.size());
    stats_.max_arena_used = std::max<uint64_t>(stats_.max_arena_used, arena_.used());
    return items;
  }

  // The batch of `slot` is over: its requests complete with `status`
  // (GTSR_OK when the device finished it; otherwise the error that kept it
  // from the device or failed it there) and the slot is free again.  Their
  // arena ranges stay allocated until each is released.
  void finish(uint32_t slot, int status, uint64_t now) {
    Slot& s = slots_[slot];
    for (const Request& r : s.reqs) {
      gtsr_completion c{};
      c.tag = r.tag;
      c.mesh = r.mesh;
      c.status = status;
      c.out_offset = r.off;
      c.out_bytes = r.bytes;
      c.t_submit_ns = r.t_submit;
      c.t_admit_ns = r.t_admit;
      c.t_done_ns = now;
      done_.push_back(c);
      if (status == GTSR_OK) {
        stats_.completed += 1;
        stats_.strip_triangles += meshes[r.mesh].entry.strip_triangles;
      } else {
        stats_.failed += 1;
      }
    }
    s.reqs.clear();
    s.busy = false;
  }

  // Moves up to capacity completions, oldest first, to out.
  uint32_t poll(gtsr_completion* out, uint32_t capacity) {
    uint32_t n = 0;
    while (n < capacity && !done_.empty()) {
      out[n++] = done_.front();
      done_.pop_front();
    }
    return n;
  }
  bool has_completions() const { return !done_.empty(); }

  gtsr_server_stats stats() const {
    gtsr_server_stats st = stats_;
    st.pending = pending_.size();
    st.arena_used = arena_.used();
    return st;
  }
  uint64_t arena_size() const { return arena_.size(); }
  size_t arena_free_ranges() const { return arena_.free_ranges(); }

 private:
  struct Slot {
    std::vector<Request> reqs;
    bool busy = false;
  };
  static int say(const char** why, const char* msg, int code) {
    if (why) *why = msg;
    return code;
  }

  uint8_t* base_;
  Arena arena_;
  std::vector<Slot> slots_;
  uint32_t max_batch_, max_items_;
  std::deque<Request> pending_;
  std::unordered_map<uint64_t, std::pair<uint64_t, uint64_t>> live_;   // tag -> arena range (admitted, unreleased)
  std::unordered_set<uint64_t> known_;                                 // tags submitted and not yet released
  std::deque<gtsr_completion> done_;
  gtsr_server_stats stats_{};
};

}  // namespace serve
}  // namespace gtsr
