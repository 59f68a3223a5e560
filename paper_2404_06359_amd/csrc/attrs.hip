// Dequantization of crack-free fixed-point vertex attributes (Sec. 4.4) on
// CDNA4 (gfx950).
//
// Every meshlet-local vertex's channel value is its meshlet's lowest grid
// value plus a 16-bit offset -- the vertex's index on the channel's global
// grid -- mapped back as (L + q) * delta + origin with one float64 fused
// multiply-add rounded to float32.  The result depends on the grid value only,
// so every copy of a vertex in different meshlets gets the same bits.
//
// One wavefront takes a contiguous block of meshlets (XCD-major, as the
// decoders); a meshlet's offsets and outputs are contiguous (vertex-major,
// channel-minor), so its lanes read and write consecutive elements.  The
// kernel is bound by HBM traffic: 2 bytes read and 4 written per element,
// plus 4 bytes of L per channel and meshlet.
#include <hip/hip_runtime.h>

#include "common.h"

namespace gtsr {
namespace {

constexpr uint32_t kWave = 64;
constexpr uint32_t kXcds = 8;

__global__ __launch_bounds__(256) void k_dequantize(const int32_t* __restrict__ lowest,
                                                    const uint16_t* __restrict__ offsets,
                                                    const uint64_t* __restrict__ vert_off,
                                                    const float* __restrict__ origin,
                                                    const float* __restrict__ delta, float* __restrict__ out,
                                                    uint32_t meshlet_count, uint32_t channels, uint64_t out_count,
                                                    uint64_t offset_count) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t waves = blockDim.x / kWave;
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint64_t wx = uint64_t(gridDim.x / kXcds) * waves;
  const uint64_t qi = uint64_t(blockIdx.x / kXcds) * waves + wave;
  const uint64_t x0 = uint64_t(meshlet_count) * xcd / kXcds, x1 = uint64_t(meshlet_count) * (xcd + 1) / kXcds;
  const uint32_t m0 = uint32_t(x0 + (x1 - x0) * qi / wx), m1 = uint32_t(x0 + (x1 - x0) * (qi + 1) / wx);
  const uint32_t step = kWave % channels;
  // vertex offsets past this bound address elements neither array holds (and
  // bounding them first keeps the products below from overflowing)
  const uint64_t v_limit = (out_count < offset_count ? out_count : offset_count) / channels;
  for (uint32_t m = m0; m < m1; ++m) {
    const uint64_t v0 = vert_off[m], v1 = vert_off[m + 1];
    if (v1 < v0 || v1 > v_limit) continue;   // corrupt offsets: the meshlet is skipped
    const uint64_t e0 = v0 * channels, e1 = v1 * channels;
    const int32_t* Lm = lowest + uint64_t(m) * channels;
    uint32_t ch = lane % channels;
    for (uint64_t e = e0 + lane; e < e1; e += kWave) {
      const int64_t g = int64_t(Lm[ch]) + offsets[e];
      out[e] = float(__builtin_fma(double(g), double(delta[ch]), double(origin[ch])));
      ch += step;
      if (ch >= channels) ch -= channels;
    }
  }
}

}  // namespace
}  // namespace gtsr

using namespace gtsr;

extern "C" int gtsr_dequantize(const gtsr_attr_stream* dev, float* dev_out, uint64_t out_count,
                               const gtsr_launch_cfg* cfg, void* hip_stream) {
  const char* who = "gtsr_dequantize";
  if (!dev) return fail(GTSR_EINVAL, std::string(who) + ": null stream");
  if (dev->channels == 0 || dev->channels > 64) return fail(GTSR_EINVAL, std::string(who) + ": channels must be 1..64");
  if (cfg && cfg->run_tris) return fail(GTSR_EINVAL, std::string(who) + ": cfg.run_tris must be 0");
  if (dev->meshlet_count == 0) return ok();
  if (!dev->lowest || !dev->offsets || !dev->vert_off || !dev->origin || !dev->delta || !dev_out)
    return fail(GTSR_EINVAL, std::string(who) + ": null device pointer");
  uint32_t waves = cfg && cfg->waves_per_group ? cfg->waves_per_group : 4;
  uint32_t mpw = cfg && cfg->meshlets_per_wave ? cfg->meshlets_per_wave : 4;
  if (waves > 4) return fail(GTSR_EINVAL, std::string(who) + ": waves_per_group > 4");
  int devno = 0, cus = 0;
  if (hipGetDevice(&devno) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, devno) != hipSuccess || cus <= 0)
    return fail(GTSR_EHIP, std::string(who) + ": cannot query the device");
  uint64_t groups = (uint64_t(dev->meshlet_count) + uint64_t(mpw) * waves - 1) / (uint64_t(mpw) * waves);
  groups = std::min<uint64_t>(groups, uint64_t(cus) * 16);
  groups = (groups + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL(k_dequantize, dim3(uint32_t(groups)), dim3(kWave * waves), 0,
                     static_cast<hipStream_t>(hip_stream), dev->lowest, dev->offsets, dev->vert_off, dev->origin,
                     dev->delta, dev_out, dev->meshlet_count, dev->channels, out_count, dev->offset_count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GTSR_EHIP, std::string(who) + ": " + hipGetErrorString(e));
  return ok();
}
