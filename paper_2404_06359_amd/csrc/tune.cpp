// Launch-shape autotuner for the batched decoder (host code, HIP runtime API).
//
// The batched decoder's speed depends on four knobs the stream format leaves
// open: how many strip triangles one work item holds (gtsr_plan_batch's
// target, i.e. how many meshlets a wavefront takes per item), how many
// wavefronts share a workgroup, how many workgroups the grid holds per CU,
// and the LDS tile (the longest run of strip triangles a wavefront stages at
// once).  gtsr_autotune_batched measures every requested
// combination on the caller's own meshes and returns the fastest.  Every
// candidate decodes the whole table into its outputs, so the outputs hold the
// decoded meshes afterwards, exactly as after one decode_meshlets_batched.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <string>
#include <vector>

#include "common.h"

using namespace gtsr;

namespace {

const uint32_t kDefaultTargets[] = {384, 768, 1536, 3072};
// Grids of 32 waves per CU and grids 4, 8 and 16 times larger (the
// dispatcher refills freed slots as groups finish), each with both LDS tiles
// (1280- and 1024-triangle runs).
const gtsr_launch_cfg kDefaultCfgs[] = {
    {1, 0, 32, 1280},  {2, 0, 16, 1280},  {1, 0, 128, 1280}, {1, 0, 256, 1280}, {2, 0, 64, 1280},
    {2, 0, 128, 1280}, {4, 0, 32, 1280},  {1, 0, 512, 1280}, {2, 0, 256, 1280}, {1, 0, 32, 1024},
    {2, 0, 16, 1024},  {1, 0, 128, 1024}, {1, 0, 256, 1024}, {2, 0, 64, 1024},  {2, 0, 128, 1024},
    {4, 0, 32, 1024},  {1, 0, 512, 1024}, {2, 0, 256, 1024},
};

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

struct DeviceBuffer {
  void* p = nullptr;
  ~DeviceBuffer() {
    if (p) (void)hipFree(p);
  }
};

int hip_fail(const char* what, hipError_t e) {
  return fail(GTSR_EHIP, std::string("gtsr_autotune_batched: ") + what + ": " + hipGetErrorString(e));
}

}  // namespace

extern "C" int gtsr_autotune_batched(const gtsr_meshlet* const* host_meshlets, const uint32_t* meshlet_counts,
                                     const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                                     const uint32_t* targets, uint32_t n_targets, const gtsr_launch_cfg* cfgs,
                                     uint32_t n_cfgs, uint32_t reps, gtsr_tune_point* points, uint32_t capacity,
                                     uint32_t* point_count, gtsr_tune_point* best, void* hip_stream) {
  if (!best || (mesh_count && (!host_meshlets || !meshlet_counts || !dev_mesh_table)))
    return fail(GTSR_EINVAL, "gtsr_autotune_batched: null argument");
  if (!targets || !n_targets) {
    targets = kDefaultTargets;
    n_targets = sizeof(kDefaultTargets) / sizeof(kDefaultTargets[0]);
  }
  if (!cfgs || !n_cfgs) {
    cfgs = kDefaultCfgs;
    n_cfgs = sizeof(kDefaultCfgs) / sizeof(kDefaultCfgs[0]);
  }
  if (reps == 0) reps = 5;
  if (reps > 1000) return fail(GTSR_EINVAL, "gtsr_autotune_batched: reps > 1000");
  for (uint32_t i = 0; i < n_targets; ++i)
    if (targets[i] == 0) return fail(GTSR_EINVAL, "gtsr_autotune_batched: target_tris must be > 0");
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);

  // Plans for every target, sized first so that one device buffer holds any.
  std::vector<std::vector<gtsr_work_item>> plans(n_targets);
  size_t max_items = 1;
  for (uint32_t i = 0; i < n_targets; ++i) {
    uint32_t n = 0;
    if (int rc = gtsr_plan_batch(host_meshlets, meshlet_counts, mesh_count, targets[i], nullptr, 0, &n)) return rc;
    plans[i].resize(n);
    if (n) {
      if (int rc = gtsr_plan_batch(host_meshlets, meshlet_counts, mesh_count, targets[i], plans[i].data(), n, &n))
        return rc;
    }
    max_items = std::max<size_t>(max_items, n);
  }
  DeviceBuffer work;
  if (hipError_t e = hipMalloc(&work.p, max_items * sizeof(gtsr_work_item)))
    return hip_fail("work list allocation", e);
  Events ev;
  if (hipError_t e = hipEventCreate(&ev.a)) return hip_fail("event", e);
  if (hipError_t e = hipEventCreate(&ev.b)) return hip_fail("event", e);

  uint32_t written = 0;
  bool have_best = false;
  std::vector<float> ms(reps);
  for (uint32_t i = 0; i < n_targets; ++i) {
    const uint32_t items = uint32_t(plans[i].size());
    if (items) {
      if (hipError_t e = hipMemcpyAsync(work.p, plans[i].data(), items * sizeof(gtsr_work_item),
                                        hipMemcpyHostToDevice, stream))
        return hip_fail("work list upload", e);
    }
    const auto* dev_work = static_cast<const gtsr_work_item*>(work.p);
    for (uint32_t j = 0; j < n_cfgs; ++j) {
      const gtsr_launch_cfg& cfg = cfgs[j];
      // warm-up launch (also rejects a bad cfg before anything is timed)
      if (int rc = decode_meshlets_batched(dev_mesh_table, mesh_count, dev_work, items, &cfg, stream)) return rc;
      for (uint32_t r = 0; r < reps; ++r) {
        if (hipError_t e = hipEventRecord(ev.a, stream)) return hip_fail("event record", e);
        if (int rc = decode_meshlets_batched(dev_mesh_table, mesh_count, dev_work, items, &cfg, stream)) return rc;
        if (hipError_t e = hipEventRecord(ev.b, stream)) return hip_fail("event record", e);
        if (hipError_t e = hipEventSynchronize(ev.b)) return hip_fail("event wait", e);
        if (hipError_t e = hipEventElapsedTime(&ms[r], ev.a, ev.b)) return hip_fail("elapsed time", e);
      }
      std::sort(ms.begin(), ms.end());
      gtsr_tune_point pt{targets[i], items, cfg, ms[reps / 2], ms[0]};
      if (points && written < capacity) points[written] = pt;
      ++written;
      if (!have_best || pt.median_ms < best->median_ms) {
        *best = pt;
        have_best = true;
      }
    }
  }
  if (point_count) *point_count = written;
  return ok();
}
