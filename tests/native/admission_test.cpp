// Host-only tests of the decode-request server's admission policy
// (paper_2404_06359_amd/csrc/admission.h), driven by a fake executor: batches
// "finish" when the test says so, with the status the test chooses, and no
// device is involved.  Built and run by tests/test_serving_cpu.py, with and
// without AddressSanitizer/UndefinedBehaviorSanitizer.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "admission.h"

using gtsr::serve::Arena;
using gtsr::serve::arena_span;
using gtsr::serve::make_cuts;
using gtsr::serve::MeshInfo;
using gtsr::serve::Scheduler;

namespace {

int g_checks = 0;

#define CHECK(cond)                                                                   \
  do {                                                                                \
    ++g_checks;                                                                       \
    if (!(cond)) {                                                                    \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      std::exit(1);                                                                   \
    }                                                                                 \
  } while (0)

uint8_t* const kBase = reinterpret_cast<uint8_t*>(uintptr_t(1) << 40);   // never dereferenced

// A mesh whose output is `tris` strip triangles (3 bytes each), cut into
// `items` work items of one meshlet each.
MeshInfo mesh(uint64_t tris, uint32_t items = 1) {
  MeshInfo m{};
  m.entry.meshlet_count = items;
  m.entry.strip_triangles = tris;
  m.entry.meshlets = reinterpret_cast<const gtsr_meshlet*>(uintptr_t(0x1000) * (tris + 1));
  m.out_bytes = 3 * tris;
  for (uint32_t k = 0; k <= items; ++k) m.cuts.push_back(k);
  return m;
}

struct Fake {
  Scheduler s;
  std::vector<std::vector<gtsr_mesh_entry>> table;
  std::vector<std::vector<gtsr_work_item>> work;
  uint64_t clock = 1000;
  Fake(uint64_t arena, uint32_t slots, uint32_t max_batch, uint32_t max_items)
      : s(kBase, arena, slots, max_batch, max_items), table(slots), work(slots) {
    for (uint32_t i = 0; i < slots; ++i) {
      table[i].resize(max_batch);
      work[i].resize(max_items);
    }
  }
  // Admits into the first free slot; returns {slot, rows} (slot -1 if none free).
  std::pair<int, uint32_t> admit() {
    const int k = s.free_slot();
    if (k < 0) return {-1, 0};
    uint32_t rows = 0;
    s.admit(uint32_t(k), table[k].data(), work[k].data(), ++clock, &rows);
    return {k, rows};
  }
  std::vector<gtsr_completion> drain() {
    std::vector<gtsr_completion> out(64);
    out.resize(s.poll(out.data(), uint32_t(out.size())));
    return out;
  }
};

void test_first_come_first_served_batches() {
  Fake f(1 << 20, 2, 2, 16);
  f.s.meshes = {mesh(100, 2), mesh(200, 3), mesh(300, 1)};
  for (uint64_t t = 0; t < 5; ++t) CHECK(f.s.submit(uint32_t(t % 3), 10 + t, t, nullptr) == GTSR_OK);
  // slot 0 takes requests 10, 11 (max_batch 2): rows in arrival order, work
  // items row-major over each mesh's cuts, outputs at increasing arena offsets
  auto [k0, r0] = f.admit();
  CHECK(k0 == 0 && r0 == 2);
  CHECK(f.table[0][0].out == kBase + 0 && f.table[0][0].strip_triangles == 100);
  CHECK(f.table[0][1].out == kBase + arena_span(300) && f.table[0][1].strip_triangles == 200);
  const gtsr_work_item want0[] = {{0, 0, 1, 0}, {0, 1, 2, 0}, {1, 0, 1, 0}, {1, 1, 2, 0}, {1, 2, 3, 0}};
  for (int i = 0; i < 5; ++i)
    CHECK(f.work[0][i].mesh == want0[i].mesh && f.work[0][i].first == want0[i].first &&
          f.work[0][i].end == want0[i].end);
  auto [k1, r1] = f.admit();
  CHECK(k1 == 1 && r1 == 2 && f.table[1][0].strip_triangles == 300 && f.table[1][1].strip_triangles == 100);
  CHECK(f.admit().first == -1);   // both slots busy
  CHECK(f.s.stats().pending == 1 && f.s.stats().batches == 2 && f.s.stats().max_batch_seen == 2);
  // slot 1 finishes first: its requests complete first, slot 1 is reused
  f.s.finish(1, GTSR_OK, ++f.clock);
  auto done = f.drain();
  CHECK(done.size() == 2 && done[0].tag == 12 && done[1].tag == 13 && done[0].status == GTSR_OK);
  CHECK(done[0].out_bytes == 900 && done[0].t_submit_ns == 2 && done[0].t_admit_ns < done[0].t_done_ns);
  auto [k2, r2] = f.admit();
  CHECK(k2 == 1 && r2 == 1 && f.table[1][0].strip_triangles == 200);   // request 14 (mesh 1)
  CHECK(f.s.stats().completed == 2 && f.s.stats().strip_triangles == 400);
}

void test_head_of_line_blocking_and_release() {
  // arena of 4 units: a 3-unit output, then a 2-unit one that does not fit
  // while the first is held, then a 1-unit one that would fit but must wait
  Fake f(4 * 256, 4, 8, 64);
  f.s.meshes = {mesh(256), mesh(170), mesh(10)};   // 768 B = 3 units, 510 B = 2 units, 30 B = 1 unit
  CHECK(f.s.submit(0, 1, 0, nullptr) == GTSR_OK);
  CHECK(f.s.submit(1, 2, 0, nullptr) == GTSR_OK);
  CHECK(f.s.submit(2, 3, 0, nullptr) == GTSR_OK);
  auto [k, rows] = f.admit();
  CHECK(k == 0 && rows == 1);                 // only the first: the second blocks the third
  CHECK(f.admit().second == 0);               // nothing admissible, no batch formed
  CHECK(f.s.stats().batches == 1 && f.s.stats().pending == 2 && f.s.stats().arena_used == 768);
  const char* why = nullptr;
  CHECK(f.s.release(1, &why) == GTSR_EINVAL);   // still decoding
  f.s.finish(0, GTSR_OK, ++f.clock);
  CHECK(f.admit().second == 0);               // finished but unreleased: the arena is still held
  CHECK(f.s.release(1, &why) == GTSR_OK);
  CHECK(f.s.release(1, &why) == GTSR_EINVAL);   // twice
  auto [k2, rows2] = f.admit();
  CHECK(rows2 == 2 && f.table[k2][0].strip_triangles == 170 && f.table[k2][1].strip_triangles == 10);
  CHECK(f.s.stats().arena_used == 768 && f.s.stats().max_arena_used == 768);
}

void test_batch_limits() {
  Fake f(1 << 20, 1, 3, 5);
  f.s.meshes = {mesh(10, 2), mesh(10, 4)};
  const char* why = nullptr;
  CHECK(f.s.submit(0, 1, 0, &why) == GTSR_OK);
  CHECK(f.s.submit(1, 2, 0, &why) == GTSR_OK);   // 2 + 4 items > 5: a batch of its own
  CHECK(f.s.submit(0, 3, 0, &why) == GTSR_OK);
  auto [k, rows] = f.admit();
  CHECK(rows == 1);
  f.s.finish(uint32_t(k), GTSR_OK, ++f.clock);
  CHECK(f.admit().second == 1);   // 4 items, then 4 + 2 > 5 stops
  f.s.finish(0, GTSR_OK, ++f.clock);
  CHECK(f.admit().second == 1);
  // max_batch: 3 requests of one item each
  for (uint64_t t = 10; t < 15; ++t) CHECK(f.s.submit(0, t, 0, &why) == GTSR_OK);
  f.s.finish(0, GTSR_OK, ++f.clock);
  CHECK(f.admit().second == 2);   // 2 + 2 items, the third would make 6
  Fake g(1 << 20, 1, 3, 64);
  g.s.meshes = {mesh(10, 1)};
  for (uint64_t t = 0; t < 5; ++t) CHECK(g.s.submit(0, t, 0, &why) == GTSR_OK);
  CHECK(g.admit().second == 3);
}

void test_submit_errors() {
  Fake f(1024, 1, 4, 4);
  f.s.meshes = {mesh(341), mesh(342), mesh(1, 5), mesh(0)};   // 1023 B fits 4 units; 1026 B does not
  const char* why = nullptr;
  CHECK(f.s.submit(4, 1, 0, &why) == GTSR_EINVAL);
  CHECK(f.s.submit(1, 1, 0, &why) == GTSR_ELIMIT);
  CHECK(f.s.submit(2, 1, 0, &why) == GTSR_ELIMIT);   // 5 items > max_items 4
  CHECK(f.s.submit(0, 1, 0, &why) == GTSR_OK);
  CHECK(f.s.submit(3, 1, 0, &why) == GTSR_EINVAL);   // tag in use
  CHECK(f.s.submit(3, 2, 0, &why) == GTSR_OK);       // an empty output takes no arena
  CHECK(f.admit().second == 2);
  CHECK(f.s.stats().arena_used == 1024 && f.s.stats().submitted == 2);
  f.s.finish(0, GTSR_OK, ++f.clock);
  auto done = f.drain();
  CHECK(done.size() == 2 && done[1].out_bytes == 0);
  CHECK(f.s.release(2, &why) == GTSR_OK && f.s.release(1, &why) == GTSR_OK);
  CHECK(f.s.stats().arena_used == 0 && f.s.arena_free_ranges() == 1);
  CHECK(f.s.submit(0, 1, 0, &why) == GTSR_OK);   // a released tag may be used again
}

void test_error_propagation() {
  Fake f(1 << 20, 2, 4, 16);
  f.s.meshes = {mesh(100)};
  const char* why = nullptr;
  for (uint64_t t = 0; t < 3; ++t) CHECK(f.s.submit(0, t, 0, &why) == GTSR_OK);
  auto [k, rows] = f.admit();
  CHECK(rows == 3);
  f.s.finish(uint32_t(k), GTSR_EHIP, ++f.clock);   // the launch or the device failed the batch
  auto done = f.drain();
  CHECK(done.size() == 3);
  for (const auto& c : done) CHECK(c.status == GTSR_EHIP);
  CHECK(f.s.stats().failed == 3 && f.s.stats().completed == 0 && f.s.stats().strip_triangles == 0);
  // the failed requests' ranges are released like any other, and the slot is free again
  for (uint64_t t = 0; t < 3; ++t) CHECK(f.s.release(t, &why) == GTSR_OK);
  CHECK(f.s.stats().arena_used == 0 && f.s.free_slot() == 0);
}

void test_cancel() {
  Fake f(2 * 256, 2, 4, 16);
  f.s.meshes = {mesh(80), mesh(170)};   // 1 unit, 2 units
  const char* why = nullptr;
  CHECK(f.s.submit(0, 1, 5, &why) == GTSR_OK);
  CHECK(f.s.submit(1, 2, 6, &why) == GTSR_OK);   // blocked behind request 1's unit
  CHECK(f.s.submit(0, 3, 7, &why) == GTSR_OK);
  CHECK(f.admit().second == 1);
  CHECK(f.s.cancel(1, ++f.clock, &why) == GTSR_EBUSY);   // in flight
  CHECK(f.s.cancel(99, ++f.clock, &why) == GTSR_EINVAL);
  // withdrawing the blocked head lets the request behind it go ahead
  CHECK(f.s.cancel(2, ++f.clock, &why) == GTSR_OK);
  auto done = f.drain();
  CHECK(done.size() == 1 && done[0].tag == 2 && done[0].status == GTSR_ECANCELED && done[0].out_bytes == 0 &&
        done[0].t_submit_ns == 6 && done[0].t_admit_ns == 0);
  CHECK(f.s.cancel(2, ++f.clock, &why) == GTSR_EINVAL);   // its tag is free at once
  CHECK(f.s.submit(0, 2, 8, &why) == GTSR_OK);
  auto [k, rows] = f.admit();
  CHECK(k == 1 && rows == 1 && f.table[1][0].strip_triangles == 80);   // request 3
  f.s.finish(0, GTSR_OK, ++f.clock);
  CHECK(f.s.cancel(1, ++f.clock, &why) == GTSR_EBUSY);    // finished, not yet released
  CHECK(f.s.stats().cancelled == 1 && f.s.stats().pending == 1);
}

void test_arena() {
  CHECK(arena_span(0) == 256 && arena_span(1) == 256 && arena_span(256) == 256 && arena_span(257) == 512);
  Arena a(4 * 256);
  uint64_t off[4];
  for (int i = 0; i < 4; ++i) CHECK(a.alloc(100, off[i]) && off[i] == uint64_t(256 * i));   // first fit, in order
  uint64_t x = 0;
  CHECK(!a.alloc(1, x) && a.used() == 1024);
  a.release(off[1], 100);
  a.release(off[2], 100);   // merges with the range before it
  CHECK(a.free_ranges() == 1 && a.used() == 512);
  CHECK(a.alloc(512, x) && x == 256);
  a.release(x, 512);
  a.release(off[3], 100);   // merges with the range before it
  a.release(off[0], 100);   // and with the one after it
  CHECK(a.free_ranges() == 1 && a.used() == 0);
  CHECK(a.alloc(1024, x) && x == 0);
  CHECK(!a.alloc(1, x));
  a.release(0, 1024);
  // a hole too small for the request is skipped (first fit by address)
  CHECK(a.alloc(256, off[0]) && a.alloc(512, off[1]) && a.alloc(256, off[2]));
  a.release(off[0], 256);
  a.release(off[2], 256);
  CHECK(a.free_ranges() == 2);
  CHECK(!a.alloc(512, x));
  CHECK(a.alloc(200, x) && x == 0);
}

void test_make_cuts() {
  std::vector<gtsr_meshlet> ml(10);
  for (int i = 0; i < 10; ++i) ml[i].tri_count = uint16_t(100 + 10 * i);
  std::vector<uint32_t> cuts;
  make_cuts(ml.data(), 10, 300, 100, cuts);
  // greedy: add meshlets while the item stays within 300 triangles (one at least)
  CHECK((cuts == std::vector<uint32_t>{0, 2, 4, 6, 7, 8, 9, 10}));
  make_cuts(ml.data(), 10, 300, 3, cuts);   // too many items: coarser target until <= 3
  CHECK(cuts.size() - 1 <= 3 && cuts.front() == 0 && cuts.back() == 10);
  for (size_t i = 1; i < cuts.size(); ++i) CHECK(cuts[i] > cuts[i - 1]);
  make_cuts(ml.data(), 0, 300, 3, cuts);
  CHECK((cuts == std::vector<uint32_t>{0}));
  make_cuts(ml.data(), 10, 1, 100, cuts);   // a meshlet larger than the target is one item
  CHECK(cuts.size() == 11);
  // more triangles than the largest target holds, one item allowed: the split
  // stops at that target (two items), which submit then refuses
  std::vector<gtsr_meshlet> big(65540);
  for (gtsr_meshlet& m : big) m.tri_count = 65535;
  make_cuts(big.data(), uint32_t(big.size()), 1u << 31, 1, cuts);
  CHECK(cuts.size() == 3 && cuts.front() == 0 && cuts.back() == big.size());
}

// Random operations against a plain model of the policy: every admitted
// batch is the longest prefix of the queue that fits; live ranges never
// overlap and stay inside the arena; the arena's use equals the live spans;
// each request completes exactly once; admission follows submission order.
void test_random_against_model() {
  std::mt19937_64 rng(20240406);
  for (int round = 0; round < 40; ++round) {
    const uint64_t arena = 256 * (4 + rng() % 60);
    const uint32_t slots = 1 + uint32_t(rng() % 4), max_batch = 1 + uint32_t(rng() % 6),
                   max_items = 4 + uint32_t(rng() % 12);
    Fake f(arena, slots, max_batch, max_items);
    for (int m = 0; m < 8; ++m) f.s.meshes.push_back(mesh(rng() % (arena / 3 + 1), 1 + uint32_t(rng() % 4)));
    std::map<uint64_t, std::pair<uint64_t, uint64_t>> live;   // tag -> [off, off + span)
    std::set<uint64_t> pending_model, inflight, finished, cancelled;
    std::vector<uint64_t> order, admitted_order;
    std::map<int, std::vector<uint64_t>> batch;   // slot -> tags
    std::map<uint64_t, uint32_t> tag_mesh;
    uint64_t next_tag = 0;
    for (int op = 0; op < 600; ++op) {
      const int what = int(rng() % 6);
      const char* why = nullptr;
      if (what == 0 || what == 1) {
        const uint32_t m = uint32_t(rng() % f.s.meshes.size());
        const int rc = f.s.submit(m, next_tag, ++f.clock, &why);
        const MeshInfo& mi = f.s.meshes[m];
        const bool ok = !(mi.out_bytes && arena_span(mi.out_bytes) > arena) && mi.cuts.size() - 1 <= max_items;
        CHECK((rc == GTSR_OK) == ok);
        if (ok) {
          tag_mesh[next_tag] = m;
          pending_model.insert(next_tag);
          order.push_back(next_tag);
        }
        ++next_tag;
      } else if (what == 2) {
        auto [k, rows] = f.admit();
        if (k >= 0 && rows) {
          auto st = f.s.stats();
          CHECK(st.pending == pending_model.size() - rows);
          std::vector<uint64_t> tags;
          for (uint64_t t : order)
            if (pending_model.count(t) && tags.size() < rows) tags.push_back(t);
          // the rows are the oldest pending requests, in order
          for (uint32_t r = 0; r < rows; ++r) {
            const MeshInfo& mi = f.s.meshes[tag_mesh[tags[r]]];
            CHECK(f.table[k][r].strip_triangles == mi.entry.strip_triangles &&
                  f.table[k][r].meshlets == mi.entry.meshlets);
            CHECK(f.table[k][r].out >= kBase && f.table[k][r].out + mi.out_bytes <= kBase + arena);
          }
          for (uint64_t t : tags) {
            pending_model.erase(t);
            inflight.insert(t);
            admitted_order.push_back(t);
          }
          batch[k] = tags;
        }
      } else if (what == 3) {
        for (int k = 0; k < int(slots); ++k)
          if (f.s.busy(uint32_t(k)) && rng() % 2) {
            f.s.finish(uint32_t(k), rng() % 8 ? GTSR_OK : GTSR_EHIP, ++f.clock);
            for (uint64_t t : batch[k]) {
              inflight.erase(t);
              finished.insert(t);
            }
            batch[k].clear();
          }
        for (const gtsr_completion& c : f.drain()) {
          if (c.status == GTSR_ECANCELED) {
            CHECK(cancelled.count(c.tag) == 1);
            continue;
          }
          CHECK(finished.count(c.tag) == 1 && !live.count(c.tag));
          const uint64_t end = c.out_offset + (c.out_bytes ? arena_span(c.out_bytes) : 0);
          CHECK(end <= arena);
          for (const auto& kv : live)
            if (c.out_bytes && kv.second.second > kv.second.first)
              CHECK(end <= kv.second.first || c.out_offset >= kv.second.second);   // no overlap
          live[c.tag] = {c.out_offset, end};
        }
      } else if (what == 4) {
        if (!live.empty()) {
          auto it = live.begin();
          std::advance(it, rng() % live.size());
          CHECK(f.s.release(it->first, &why) == GTSR_OK);
          finished.erase(it->first);
          live.erase(it);
        }
        if (!inflight.empty()) CHECK(f.s.release(*inflight.begin(), &why) == GTSR_EINVAL);
      } else {
        if (!pending_model.empty() && rng() % 2) {
          const uint64_t t = *pending_model.begin();
          CHECK(f.s.cancel(t, ++f.clock, &why) == GTSR_OK);
          pending_model.erase(t);
          cancelled.insert(t);
        } else if (!inflight.empty()) {
          CHECK(f.s.cancel(*inflight.begin(), ++f.clock, &why) == GTSR_EBUSY);
        }
      }
      uint64_t used = 0;
      for (const auto& kv : live) used += kv.second.second - kv.second.first;
      // the model sees ranges once polled; in-flight and unpolled ones also hold arena
      CHECK(f.s.stats().arena_used >= used);
    }
    // admission order is submission order (cancelled requests skipped)
    std::vector<uint64_t> expect;
    for (uint64_t t : order)
      if (!cancelled.count(t) && std::find(admitted_order.begin(), admitted_order.end(), t) != admitted_order.end())
        expect.push_back(t);
    CHECK(expect == admitted_order);
  }
}

}  // namespace

int main() {
  test_first_come_first_served_batches();
  test_head_of_line_blocking_and_release();
  test_batch_limits();
  test_submit_errors();
  test_error_propagation();
  test_cancel();
  test_arena();
  test_make_cuts();
  test_random_against_model();
  std::printf("admission_test: %d checks passed\n", g_checks);
  return 0;
}
