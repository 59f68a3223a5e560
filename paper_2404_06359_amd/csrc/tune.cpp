// Launch-shape autotuner for the batched decoders (host code, HIP runtime API).
//
// The batched decoders' speed depends on four knobs the stream format leaves
// open: how many strip triangles one work item holds (gtsr_plan_batch's
// target, i.e. how many meshlets a wavefront takes per item), how many
// wavefronts share a workgroup, how many workgroups the grid holds per CU,
// and the LDS tile (the longest run of strip triangles a wavefront stages at
// once).  gtsr_autotune_batched measures every combination of the caller's
// work lists (one per target, already on the device) and launch shapes on
// the caller's own meshes and returns the fastest; the caller keeps the
// winning list, so nothing is re-planned between tuning and use.
//
// Measurement protocol.  The decode is used as back-to-back graph launches,
// and a device that has sat idle runs the first launches after it slower
// than the steady state, so the tuner never lets the device idle while it
// measures: after a warm-up of back-to-back launches, each round enqueues
// every shape in turn, kLaunchesPerSample launches each, with one event
// between shapes, and all rounds of a stage are enqueued before the host
// waits for the first (one synchronisation per stage).  A shape's
// sample is its event interval over those launches; its figure is the
// median over rounds.  The fastest shapes of that first stage (at least
// kMinFinalists, and every other one within kFinalBand of the fastest, up to
// kMaxFinalists) are then measured again, alone, over three times as many
// rounds, and among the finalists the earliest in the candidate order within
// kTieFraction of the fastest median wins, so that shapes the measurement
// cannot tell apart do not make the choice flip from run to run.  Every candidate decodes the
// whole table into its outputs, so the outputs hold the decoded meshes
// afterwards, exactly as after one batched decode.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "common.h"

using namespace gtsr;

namespace {

// Static-split grids of 32 waves per CU and grids 4, 8 and 16 times larger
// (the dispatcher refills freed slots as groups finish), each with both LDS
// tiles (1280- and 1024-triangle runs; plain GTS streams take the second
// only), and persistent claiming grids.
const gtsr_launch_cfg kDefaultCfgs[] = {
    {1, 0, 32, 1280, 0},  {2, 0, 16, 1280, 0},  {1, 0, 128, 1280, 0}, {1, 0, 256, 1280, 0}, {2, 0, 64, 1280, 0},
    {2, 0, 128, 1280, 0}, {4, 0, 32, 1280, 0},  {1, 0, 512, 1280, 0}, {2, 0, 256, 1280, 0}, {1, 0, 32, 1024, 0},
    {2, 0, 16, 1024, 0},  {1, 0, 128, 1024, 0}, {1, 0, 256, 1024, 0}, {2, 0, 64, 1024, 0},  {2, 0, 128, 1024, 0},
    {4, 0, 32, 1024, 0},  {1, 0, 512, 1024, 0}, {2, 0, 256, 1024, 0},
    // persistent grids claiming work from per-XCD counters (need a workspace)
    {1, 0, 32, 0, 1},     {1, 0, 32, 0, 2},     {1, 0, 32, 0, 4},
};
constexpr uint32_t kLaunchesPerSample = 4;
constexpr uint32_t kMinFinalists = 4;
constexpr uint32_t kMaxFinalists = 16;
constexpr float kFinalBand = 0.015f;      // stage-1 medians this close to the fastest go to stage 2
constexpr float kTieFraction = 0.01f;
constexpr float kWarmMs = 60.0f;          // device time of back-to-back launches before measuring
constexpr uint32_t kMaxWarmLaunches = 400;

struct EventSet {
  std::vector<hipEvent_t> ev;
  ~EventSet() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

int hip_fail(const char* what, hipError_t e) {
  return fail(GTSR_EHIP, std::string("gtsr_autotune_batched: ") + what + ": " + hipGetErrorString(e));
}

struct Candidate {
  uint32_t target;        // index of its work list
  gtsr_launch_cfg cfg;
  std::vector<float> samples;
  float median = 0.0f, min = 0.0f;
};

float median_of(std::vector<float> v) {
  if (v.empty()) return 0.0f;
  std::sort(v.begin(), v.end());
  const size_t n = v.size();
  return n % 2 ? v[n / 2] : 0.5f * (v[n / 2 - 1] + v[n / 2]);
}

}  // namespace

extern "C" int gtsr_autotune_batched(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count, uint32_t format,
                                     const gtsr_work_item* const* dev_works, const uint32_t* work_counts,
                                     uint32_t n_works, void* dev_workspace, uint64_t workspace_bytes,
                                     const gtsr_launch_cfg* cfgs, uint32_t n_cfgs, uint32_t reps,
                                     gtsr_tune_point* points, uint32_t capacity, uint32_t* point_count,
                                     gtsr_tune_point* best, void* hip_stream) {
  if (!best || (n_works && (!dev_works || !work_counts)) || (mesh_count && !dev_mesh_table))
    return fail(GTSR_EINVAL, "gtsr_autotune_batched: null argument");
  if (format != GTSR_FORMAT_REUSE && format != GTSR_FORMAT_GTS)
    return fail(GTSR_EINVAL, "gtsr_autotune_batched: bad format");
  std::vector<gtsr_launch_cfg> shapes;
  if (!cfgs || !n_cfgs) {
    for (const gtsr_launch_cfg& c : kDefaultCfgs)
      if ((format == GTSR_FORMAT_REUSE || c.run_tris != 1280) && (!c.items_per_claim || dev_workspace))
        shapes.push_back(c);
  } else {
    shapes.assign(cfgs, cfgs + n_cfgs);
  }
  if (reps == 0) reps = 5;
  if (reps > 1000) return fail(GTSR_EINVAL, "gtsr_autotune_batched: reps > 1000");
  for (uint32_t i = 0; i < n_works; ++i)
    if (work_counts[i] && !dev_works[i]) return fail(GTSR_EINVAL, "gtsr_autotune_batched: null work list");
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  auto enqueue = [&](const gtsr_work_item* work, uint32_t items, const gtsr_launch_cfg& cfg) {
    return format == GTSR_FORMAT_GTS
               ? gtsr_decode_gts_batched(dev_mesh_table, mesh_count, work, items, dev_workspace, workspace_bytes,
                                         &cfg, hip_stream)
               : decode_meshlets_batched(dev_mesh_table, mesh_count, work, items, dev_workspace, workspace_bytes,
                                         &cfg, hip_stream);
  };

  std::vector<Candidate> cand;
  for (uint32_t i = 0; i < n_works; ++i)
    for (const gtsr_launch_cfg& c : shapes) cand.push_back(Candidate{i, c, {}, 0.0f, 0.0f});
  if (cand.empty()) {
    if (point_count) *point_count = 0;
    return fail(GTSR_EINVAL, "gtsr_autotune_batched: no shapes to measure");
  }
  const uint32_t n_cand = uint32_t(cand.size());
  auto launch = [&](const Candidate& c) { return enqueue(dev_works[c.target], work_counts[c.target], c.cfg); };

  // Events of one stage: (candidates + 1) per round, every round enqueued
  // before the first is read, so the device never waits for the host.
  EventSet ev;
  auto events = [&](size_t n) -> int {
    for (hipEvent_t& e : ev.ev)
      if (e) (void)hipEventDestroy(e);
    ev.ev.assign(n, nullptr);
    for (hipEvent_t& e : ev.ev)
      if (hipError_t r = hipEventCreate(&e)) return hip_fail("event", r);
    return GTSR_OK;
  };
  if (int rc = events(2)) return rc;

  // Every shape once, untimed (rejects a bad cfg before anything is timed),
  // then one timed launch of the first to size the warm-up.
  for (const Candidate& c : cand)
    if (int rc = launch(c)) return rc;
  if (hipError_t e = hipEventRecord(ev.ev[0], stream)) return hip_fail("event record", e);
  if (int rc = launch(cand[0])) return rc;
  if (hipError_t e = hipEventRecord(ev.ev[1], stream)) return hip_fail("event record", e);
  if (hipError_t e = hipEventSynchronize(ev.ev[1])) return hip_fail("event wait", e);
  float one = 0.0f;
  if (hipError_t e = hipEventElapsedTime(&one, ev.ev[0], ev.ev[1])) return hip_fail("elapsed time", e);
  const uint32_t warm = uint32_t(std::min<float>(kMaxWarmLaunches, std::ceil(kWarmMs / std::max(one, 1e-3f))));

  // A stage: `rounds` rounds over the candidates `set`, the starting shape
  // rotating per round; warm-up launches in front when asked.
  auto stage = [&](const std::vector<uint32_t>& set, uint32_t rounds, uint32_t warm_launches) -> int {
    const size_t n = set.size(), per = n + 1;
    if (int rc = events(per * rounds)) return rc;
    for (uint32_t k = 0; k < warm_launches; ++k)
      if (int rc = launch(cand[set[0]])) return rc;
    for (uint32_t r = 0; r < rounds; ++r) {
      hipEvent_t* e = ev.ev.data() + per * r;
      if (hipError_t x = hipEventRecord(e[0], stream)) return hip_fail("event record", x);
      for (size_t k = 0; k < n; ++k) {
        for (uint32_t l = 0; l < kLaunchesPerSample; ++l)
          if (int rc = launch(cand[set[(k + r) % n]])) return rc;
        if (hipError_t x = hipEventRecord(e[k + 1], stream)) return hip_fail("event record", x);
      }
    }
    if (hipError_t x = hipEventSynchronize(ev.ev.back())) return hip_fail("event wait", x);
    for (uint32_t r = 0; r < rounds; ++r) {
      hipEvent_t* e = ev.ev.data() + per * r;
      for (size_t k = 0; k < n; ++k) {
        float ms = 0.0f;
        if (hipError_t x = hipEventElapsedTime(&ms, e[k], e[k + 1])) return hip_fail("elapsed time", x);
        cand[set[(k + r) % n]].samples.push_back(ms / kLaunchesPerSample);
      }
    }
    for (uint32_t k : set) {
      Candidate& c = cand[k];
      c.median = median_of(c.samples);
      c.min = c.samples.empty() ? 0.0f : *std::min_element(c.samples.begin(), c.samples.end());
    }
    return GTSR_OK;
  };

  // Stage 1: every shape, reps rounds, after the warm-up.
  std::vector<uint32_t> all(n_cand);
  for (uint32_t k = 0; k < n_cand; ++k) all[k] = k;
  if (int rc = stage(all, reps, warm)) return rc;

  // Stage 2: the fastest again, alone, three times as many rounds (a few
  // launches in front cover the host's turnaround after stage 1).  A shape
  // within the band of the fastest goes on even when it ranks below the
  // minimum count, so that stage-1 noise among near-equal shapes does not
  // decide which of them can win.
  std::vector<uint32_t> rank = all;
  std::stable_sort(rank.begin(), rank.end(), [&](uint32_t a, uint32_t b) { return cand[a].median < cand[b].median; });
  uint32_t n_fin = std::min<uint32_t>(kMinFinalists, n_cand);
  while (n_fin < std::min<uint32_t>(kMaxFinalists, n_cand) &&
         cand[rank[n_fin]].median <= cand[rank[0]].median * (1.0f + kFinalBand))
    ++n_fin;
  std::vector<uint32_t> fin(rank.begin(), rank.begin() + n_fin);
  std::sort(fin.begin(), fin.end());
  if (fin.size() > 1) {
    for (uint32_t f : fin) cand[f].samples.clear();
    if (int rc = stage(fin, 3 * reps, 8)) return rc;
  }
  float fastest = cand[fin[0]].median;
  for (uint32_t f : fin) fastest = std::min(fastest, cand[f].median);
  uint32_t pick = fin[0];
  for (uint32_t f : fin)
    if (cand[f].median <= fastest * (1.0f + kTieFraction)) {
      pick = f;   // fin is in candidate order: the first within the tie band
      break;
    }

  uint32_t written = 0;
  for (uint32_t k = 0; k < n_cand; ++k) {
    const Candidate& c = cand[k];
    const bool finalist = fin.size() > 1 && std::find(fin.begin(), fin.end(), k) != fin.end();
    gtsr_tune_point pt{c.target, work_counts[c.target], c.cfg, c.median, c.min, finalist ? 2u : 1u, 0u};
    if (points && written < capacity) points[written] = pt;
    ++written;
    if (k == pick) *best = pt;
  }
  if (point_count) *point_count = written;
  return ok();
}
