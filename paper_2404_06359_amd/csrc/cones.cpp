// Per-meshlet normal cones for culling whole meshlets before decode (Sec. 3:
// the amplification shader tests a cone of the meshlet's triangle normals and
// drops meshlets that face entirely away).  Host side, offline.
//
// Cone of a meshlet: axis = the normalised sum, in strip order, of its
// triangles' unit normals ((p1 - p0) x (p2 - p0) in float64, each triangle
// rotated -- orientation kept -- to start at its smallest vertex id, so that
// every construction from the same triangles in the same order rounds the
// same way; zero-area triangles ignored); the opening
// half-angle theta is the largest angle between the axis and a normal.  For a
// view direction d (unit, from the eye into the scene), a triangle with
// normal n faces away when dot(n, d) > 0; every triangle of the cone does
// when the axis is within 90 degrees - theta of d, i.e. dot(axis, d) >
// sin(theta).  Stored: axis (float32 x3) and cutoff = sin(theta) + 1e-5 (a
// margin for the float32 rounding of axis and test), or 2 (never culled)
// when theta >= 90 degrees or the normals cancel.
#include <cmath>

#include "common.h"

using namespace gtsr;

extern "C" int gtsr_meshlet_cones(const uint32_t* indices, uint64_t triangle_count, const float* positions,
                                  uint32_t vertex_count, const uint32_t* tri_ids, const uint32_t* kept_off,
                                  uint32_t meshlet_count, float* cones) {
  const char* who = "gtsr_meshlet_cones";
  if (meshlet_count && (!indices || !positions || !kept_off || !cones))
    return fail(GTSR_EINVAL, std::string(who) + ": null argument");
  if (meshlet_count && kept_off[meshlet_count] && !tri_ids) return fail(GTSR_EINVAL, std::string(who) + ": null tri_ids");
  for (uint32_t m = 0; m < meshlet_count; ++m) {
    if (kept_off[m + 1] < kept_off[m] || kept_off[m + 1] > triangle_count)
      return fail(GTSR_EINVAL, std::string(who) + ": kept_off out of range");
    if (kept_off[m + 1] - kept_off[m] > kMaxStripTris)   // a meshlet holds at most 256 triangles
      return fail(GTSR_EINVAL, std::string(who) + ": kept_off gives a meshlet more than 256 triangles");
    double u[256][3];
    uint32_t nu = 0;
    double sx = 0, sy = 0, sz = 0;
    for (uint32_t k = kept_off[m]; k < kept_off[m + 1]; ++k) {
      const uint32_t t = tri_ids[k];
      if (t >= triangle_count) return fail(GTSR_EINVAL, std::string(who) + ": triangle id out of range");
      uint32_t g[3];
      for (int c = 0; c < 3; ++c) {
        g[c] = indices[3ull * t + c];
        if (g[c] >= vertex_count) return fail(GTSR_EINVAL, std::string(who) + ": vertex id out of range");
      }
      const int r = g[1] < g[0] ? (g[2] < g[1] ? 2 : 1) : (g[2] < g[0] ? 2 : 0);   // smallest id first
      double p[3][3];
      for (int c = 0; c < 3; ++c)
        for (int j = 0; j < 3; ++j) p[c][j] = positions[3ull * g[(c + r) % 3] + j];
      const double ax = p[1][0] - p[0][0], ay = p[1][1] - p[0][1], az = p[1][2] - p[0][2];
      const double bx = p[2][0] - p[0][0], by = p[2][1] - p[0][1], bz = p[2][2] - p[0][2];
      const double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
      const double len = std::sqrt(nx * nx + ny * ny + nz * nz);
      if (len == 0.0) continue;
      u[nu][0] = nx / len; u[nu][1] = ny / len; u[nu][2] = nz / len;
      sx += u[nu][0]; sy += u[nu][1]; sz += u[nu][2];
      ++nu;
    }
    float* out = cones + 4ull * m;
    const double sl = std::sqrt(sx * sx + sy * sy + sz * sz);
    if (nu == 0 || sl == 0.0) {
      out[0] = out[1] = out[2] = 0.0f;
      out[3] = 2.0f;
      continue;
    }
    const double a[3] = {sx / sl, sy / sl, sz / sl};
    double cmin = 1.0;
    for (uint32_t i = 0; i < nu; ++i) cmin = std::min(cmin, a[0] * u[i][0] + a[1] * u[i][1] + a[2] * u[i][2]);
    out[0] = static_cast<float>(a[0]);
    out[1] = static_cast<float>(a[1]);
    out[2] = static_cast<float>(a[2]);
    out[3] = cmin <= 0.0 ? 2.0f : static_cast<float>(std::sqrt(std::max(0.0, 1.0 - cmin * cmin)) + 1e-5);
  }
  return ok();
}
