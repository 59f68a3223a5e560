// Achievable-bandwidth calibration for the decoders' HBM access pattern on
// CDNA4 (gfx950).
//
// The connectivity decode moves about 0.24 of its algorithmic bytes as reads
// (descriptors, flag chunks, reuse bytes) and 0.76 as writes (3 bytes per
// strip triangle, Sec. 3's 8-bit local index triples); every access is a
// 16-byte buffer load or a non-temporal 16-byte buffer store, and each
// wavefront walks contiguous blocks of its arrays.  k_stream_calib does the
// same memory work with no decode: every wavefront streams one contiguous
// block of src with kLoads 16-byte loads per lane per step and one
// contiguous block of dst with kStores non-temporal 16-byte stores per lane
// per step (13 to 4: 0.235 read, 0.765 written).  A step's loads are issued
// one step ahead of the stores that use them, as the decoders prefetch one
// run ahead, and every stored value depends on the loads, so nothing can be
// dropped.  Its bytes per second bound what any decoder with this traffic
// mix reaches on the device at hand.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace gtsr {
namespace {

constexpr uint32_t kWave = 64;
constexpr uint32_t kXcds = 8;
constexpr uint32_t kLoads = 4;    // 1 KiB units read per step (64 lanes x 16 bytes)
constexpr uint32_t kStores = 13;  // 1 KiB units written per step
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kNonTemporal = 2;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), kRsrcWord3);
}

// Steps [q0, q1) of `steps`, one contiguous block per wavefront, XCD-major
// (workgroups go round-robin over the 8 XCDs), as the plain decoder splits
// its meshlets.  Every step costs the same, so these blocks are balanced
// across the XCDs as they are; the batched decoder deals its work list to
// the XCDs in stripes only because its items differ in cost.
__device__ __forceinline__ void calib_block(uint32_t steps, uint32_t& q0, uint32_t& q1) {
  const uint32_t waves = blockDim.x / kWave;
  const uint32_t wave = uint32_t(__builtin_amdgcn_readfirstlane(threadIdx.x / kWave));
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint32_t wx = gridDim.x / kXcds * waves;
  const uint32_t q = blockIdx.x / kXcds * waves + wave;
  const uint32_t x0 = uint32_t(uint64_t(steps) * xcd / kXcds), x1 = uint32_t(uint64_t(steps) * (xcd + 1) / kXcds);
  const uint32_t len = x1 - x0, share = len / wx, extra = len % wx;
  q0 = std::min(x0 + q * share + std::min(q, extra), x1);
  q1 = std::min(q0 + share + (q < extra ? 1u : 0u), x1);
}

__global__ __launch_bounds__(kWave * 16) void k_stream_calib(const uint8_t* __restrict__ src,
                                                             uint8_t* __restrict__ dst, uint32_t steps) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t q0, q1;
  calib_block(steps, q0, q1);
  if (q0 >= q1) return;
  // one resource per wave block; offsets stay below 2^31 per block
  const uint64_t sbytes = uint64_t(q1 - q0) * kLoads * 1024, dbytes = uint64_t(q1 - q0) * kStores * 1024;
  const __amdgpu_buffer_rsrc_t s = rsrc(src + uint64_t(q0) * kLoads * 1024, uint32_t(std::min<uint64_t>(sbytes, 0x7FFFFFFFu)));
  const __amdgpu_buffer_rsrc_t d = rsrc(dst + uint64_t(q0) * kStores * 1024, uint32_t(std::min<uint64_t>(dbytes, 0x7FFFFFFFu)));
  u32x4 v[kLoads];
#pragma unroll
  for (uint32_t j = 0; j < kLoads; ++j)
    v[j] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(s, int(1024 * j + 16 * lane), 0, 0));
  for (uint32_t q = 0; q < q1 - q0; ++q) {
    // next step's loads (past the block: out of range, they read zero)
    u32x4 n[kLoads];
    const uint32_t nb = (q + 1) * kLoads * 1024;
#pragma unroll
    for (uint32_t j = 0; j < kLoads; ++j)
      n[j] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(s, int(nb + 1024 * j + 16 * lane), 0, 0));
    u32x4 x = v[0];
#pragma unroll
    for (uint32_t j = 1; j < kLoads; ++j) x ^= v[j];
    const uint32_t db = q * kStores * 1024;
#pragma unroll
    for (uint32_t j = 0; j < kStores; ++j) {
      u32x4 w = x;
      w.x ^= j;
      __builtin_amdgcn_raw_buffer_store_b128(w, d, int(db + 1024 * j + 16 * lane), 0, kNonTemporal);
    }
#pragma unroll
    for (uint32_t j = 0; j < kLoads; ++j) v[j] = n[j];
  }
}

}  // namespace
}  // namespace gtsr

using namespace gtsr;

extern "C" int gtsr_stream_calib(const uint8_t* dev_src, uint64_t src_bytes, uint8_t* dev_dst, uint64_t dst_bytes,
                                 const gtsr_launch_cfg* cfg, uint64_t* steps_out, void* hip_stream) {
  const char* who = "gtsr_stream_calib";
  if (cfg && (cfg->meshlets_per_wave || cfg->run_tris))
    return fail(GTSR_EINVAL, std::string(who) + ": cfg.meshlets_per_wave and cfg.run_tris must be 0");
  const uint32_t waves = cfg && cfg->waves_per_group ? cfg->waves_per_group : 1;
  const uint32_t gpc = cfg && cfg->groups_per_cu ? cfg->groups_per_cu : 256;
  if (waves > 16) return fail(GTSR_EINVAL, std::string(who) + ": waves_per_group > 16");
  if (gpc > 1024) return fail(GTSR_EINVAL, std::string(who) + ": groups_per_cu > 1024");
  const uint64_t steps = std::min(src_bytes / (kLoads * 1024), dst_bytes / (kStores * 1024));
  if (steps_out) *steps_out = steps;
  if (steps > 0xFFFFFFFFull) return fail(GTSR_ELIMIT, std::string(who) + ": more than 2^32-1 steps");
  if (steps == 0) return ok();
  if (!dev_src || !dev_dst) return fail(GTSR_EINVAL, std::string(who) + ": null device pointer");
  int devno = 0, cus = 0;
  if (hipGetDevice(&devno) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, devno) != hipSuccess || cus <= 0)
    return fail(GTSR_EHIP, std::string(who) + ": cannot query the device");
  const uint64_t want = (steps + waves - 1) / waves;
  uint64_t groups = std::min<uint64_t>(uint64_t(cus) * gpc, want);
  groups = (groups + kXcds - 1) / kXcds * kXcds;
  // a wavefront's block of dst stays addressable by 32-bit buffer offsets
  const uint64_t per_wave = steps / (groups * waves / kXcds) / kXcds + 2;
  if (per_wave * kStores * 1024 > 0x7FFFFFFFull)
    return fail(GTSR_ELIMIT, std::string(who) + ": more than 2 GiB per wavefront; use a larger grid");
  hipLaunchKernelGGL(k_stream_calib, dim3(uint32_t(groups)), dim3(kWave * waves), 0,
                     static_cast<hipStream_t>(hip_stream), dev_src, dev_dst, uint32_t(steps));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GTSR_EHIP, std::string(who) + ": " + hipGetErrorString(e));
  return ok();
}
