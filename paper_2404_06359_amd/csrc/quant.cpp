// Crack-free fixed-point vertex attribute quantization, host side (Sec. 4.4).
//
// Per attribute channel the global grid spacing comes from the widest
// meshlet: delta = w / (2^b - 1), kept as the smallest float32 not below that
// (1 for a flat channel).  A value's grid index is floor((A - origin) /
// delta) with origin the channel minimum, so every meshlet that holds a
// vertex stores the same grid value for it; a meshlet keeps its lowest grid
// value and b-bit offsets from it.  If float64 rounding would let a meshlet
// span more than 2^b - 1 grid steps, delta grows by 2^-20 relative steps
// until none does.
#include <cmath>
#include <limits>
#include <vector>

#include "common.h"

using namespace gtsr;

namespace {

inline double grid_index(float a, float lo, float d) {
  return std::floor((static_cast<double>(a) - static_cast<double>(lo)) / static_cast<double>(d));
}

}  // namespace

extern "C" int gtsr_quantize_attributes(const float* attrs, uint32_t vertex_count, uint32_t channels,
                                        const uint32_t* verts, const uint64_t* vert_off, uint32_t meshlet_count,
                                        uint32_t bits, float* origin, float* delta, int32_t* lowest,
                                        uint16_t* offsets) {
  const char* who = "gtsr_quantize_attributes";
  if (bits < 1 || bits > 16 || channels == 0 || channels > 64)
    return fail(GTSR_EINVAL, std::string(who) + ": bits must be 1..16, channels 1..64");
  if (!origin || !delta || (vertex_count && !attrs) || (meshlet_count && (!vert_off || !lowest)))
    return fail(GTSR_EINVAL, std::string(who) + ": null argument");
  const uint64_t total = meshlet_count ? vert_off[meshlet_count] : 0;
  if (total && (!verts || !offsets)) return fail(GTSR_EINVAL, std::string(who) + ": null argument");
  for (uint32_t m = 0; m < meshlet_count; ++m)
    if (vert_off[m + 1] < vert_off[m]) return fail(GTSR_EINVAL, std::string(who) + ": vert_off decreasing");
  for (uint64_t k = 0; k < total; ++k)
    if (verts[k] >= vertex_count) return fail(GTSR_EINVAL, std::string(who) + ": vertex id out of range");
  const double top = static_cast<double>((1u << bits) - 1);
  const float inf = std::numeric_limits<float>::infinity();
  std::vector<double> g(total);
  for (uint32_t i = 0; i < channels; ++i) {
    auto at = [&](uint64_t v) { return attrs[v * channels + i]; };
    float lo = vertex_count ? inf : 0.0f;
    for (uint32_t v = 0; v < vertex_count; ++v) lo = std::min(lo, at(v));
    double w = 0.0;
    for (uint32_t m = 0; m < meshlet_count; ++m) {
      if (vert_off[m + 1] == vert_off[m]) continue;
      float a = inf, z = -inf;
      for (uint64_t k = vert_off[m]; k < vert_off[m + 1]; ++k) {
        a = std::min(a, at(verts[k]));
        z = std::max(z, at(verts[k]));
      }
      w = std::max(w, static_cast<double>(z) - static_cast<double>(a));
    }
    float d = 1.0f;
    if (w > 0.0) {
      d = static_cast<float>(w / top);
      if (static_cast<double>(d) < w / top) d = std::nextafter(d, inf);
    }
    for (;;) {
      bool fits = true;
      for (uint64_t k = 0; k < total; ++k) {
        g[k] = grid_index(at(verts[k]), lo, d);
        if (g[k] >= 2147483647.0) return fail(GTSR_ELIMIT, std::string(who) + ": grid value exceeds 31 bits");
      }
      for (uint32_t m = 0; m < meshlet_count && fits; ++m) {
        double gmin = std::numeric_limits<double>::infinity(), gmax = -gmin;
        for (uint64_t k = vert_off[m]; k < vert_off[m + 1]; ++k) {
          gmin = std::min(gmin, g[k]);
          gmax = std::max(gmax, g[k]);
        }
        if (vert_off[m + 1] > vert_off[m] && gmax - gmin > top) fits = false;
      }
      if (fits) break;
      d = static_cast<float>(static_cast<double>(d) * (1.0 + 1.0 / 1048576.0));
    }
    origin[i] = lo;
    delta[i] = d;
    for (uint32_t m = 0; m < meshlet_count; ++m) {
      double gmin = std::numeric_limits<double>::infinity();
      for (uint64_t k = vert_off[m]; k < vert_off[m + 1]; ++k) gmin = std::min(gmin, g[k]);
      const int32_t L = vert_off[m + 1] > vert_off[m] ? static_cast<int32_t>(gmin) : 0;
      lowest[uint64_t(m) * channels + i] = L;
      for (uint64_t k = vert_off[m]; k < vert_off[m + 1]; ++k)
        offsets[k * channels + i] = static_cast<uint16_t>(static_cast<int64_t>(g[k]) - L);
    }
  }
  return ok();
}
