// Host-side C ABI: error state, stream validation, batch planning.
#include <cstring>
#include <string>

#include "common.h"

namespace gtsr {

namespace {
thread_local std::string g_last_error;
}

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int ok() {
  g_last_error.clear();
  return GTSR_OK;
}

}  // namespace gtsr

using namespace gtsr;

extern "C" const char* gtsr_last_error(void) { return g_last_error.c_str(); }

namespace {

inline uint64_t load_u64(const uint8_t* p) {
  uint64_t v;
  std::memcpy(&v, p, 8);
  return v;
}

}  // namespace

// Structural validity of a host stream (the decoders' memory-safety checks are
// weaker: they only keep every access inside the given sizes).
extern "C" int gtsr_validate(const gtsr_stream* s) {
  if (!s) return fail(GTSR_EINVAL, "gtsr_validate: null stream");
  if (s->meshlet_count && !s->meshlets) return fail(GTSR_EINVAL, "gtsr_validate: null meshlets");
  if (s->bits_bytes && !s->bits) return fail(GTSR_EINVAL, "gtsr_validate: null bits");
  if (s->reuse_bytes && !s->reuse) return fail(GTSR_EINVAL, "gtsr_validate: null reuse");
  if (s->bits_bytes % kChunkBytes) return fail(GTSR_ECORRUPT, "gtsr_validate: bits_bytes not a multiple of 16");
  uint64_t chunk = 0, rpos = 0, opos = 0;
  const uint64_t total_chunks = s->bits_bytes / kChunkBytes;
  for (uint32_t m = 0; m < s->meshlet_count; ++m) {
    const gtsr_meshlet& d = s->meshlets[m];
    const uint32_t T = d.tri_count, V = d.vert_count;
    auto bad = [&](const char* what) {
      return fail(GTSR_ECORRUPT, "gtsr_validate: meshlet " + std::to_string(m) + ": " + what);
    };
    if (T < 1 || T > kMaxStripTris) return bad("tri_count out of 1..256");
    if (V < 3 || V > 256) return bad("vert_count out of 3..256");
    if (V > T + 2) return bad("more vertices than index slots");
    if (d.chunk_off != chunk || d.reuse_off != rpos || d.out_off != opos) return bad("offsets not contiguous");
    const uint32_t nch = chunks_of(T);
    const uint32_t n_ru = T + 2 - V;
    if (chunk + nch > total_chunks) return bad("flag chunks past the end");
    if (rpos + n_ru > s->reuse_bytes) return bad("reuse bytes past the end");
    const uint8_t* cb = s->bits + chunk * kChunkBytes;
    uint32_t newest = 2, used = 0;
    for (uint32_t c = 0; c < nch; ++c) {
      uint64_t lr = load_u64(cb + 16 * c), inc = load_u64(cb + 16 * c + 8);
      uint32_t valid = (c + 1 < nch || T % 64 == 0) ? 64 : T % 64;
      uint64_t mask = valid == 64 ? ~0ull : ((1ull << valid) - 1);
      if ((lr & ~mask) || (inc & ~mask)) return bad("bits set past tri_count");
      if (c == 0 && (inc & 1)) return bad("increment bit on triangle 0");
      for (uint32_t i = 0; i < valid; ++i) {
        uint32_t t = 64 * c + i;
        if (t == 0) continue;
        if ((inc >> i) & 1) {
          ++newest;
        } else {
          if (used >= n_ru) return bad("more reuse slots than reuse bytes");
          if (s->reuse[rpos + used] > newest) return bad("reuse byte names a vertex not yet introduced");
          ++used;
        }
      }
    }
    if (newest + 1 != V) return bad("increment count does not match vert_count");
    if (used != n_ru) return bad("reuse slot count does not match");
    chunk += nch;
    rpos += n_ru;
    opos += T;
  }
  if (chunk != total_chunks) return fail(GTSR_ECORRUPT, "gtsr_validate: bits_bytes does not match the chunks");
  if (rpos != s->reuse_bytes) return fail(GTSR_ECORRUPT, "gtsr_validate: reuse_bytes does not match");
  if (opos != s->strip_triangles) return fail(GTSR_ECORRUPT, "gtsr_validate: strip_triangles does not match");
  return ok();
}

// Plain GTS from GTS-Reuse: the L/R word of every chunk, and per meshlet the
// index stream after the first triangle -- the next new vertex (3, 4, ...)
// where the increment flag is set, else the next reuse byte (Sec. 4.3).
extern "C" int gtsr_gts_from_reuse(const gtsr_stream* s, gtsr_meshlet* gdesc, uint8_t* words, uint64_t words_bytes,
                                   uint8_t* index, uint64_t index_bytes) {
  if (!s) return fail(GTSR_EINVAL, "gtsr_gts_from_reuse: null stream");
  if (int rc = gtsr_validate(s)) return rc;
  if (s->meshlet_count && (!gdesc || !words || (s->strip_triangles > s->meshlet_count && !index)))
    return fail(GTSR_EINVAL, "gtsr_gts_from_reuse: null output");
  if (words_bytes < s->bits_bytes / 2 || index_bytes < s->strip_triangles - s->meshlet_count)
    return fail(GTSR_EINVAL, "gtsr_gts_from_reuse: output too small");
  uint64_t ipos = 0;
  for (uint32_t m = 0; m < s->meshlet_count; ++m) {
    const gtsr_meshlet& d = s->meshlets[m];
    const uint32_t T = d.tri_count, nch = chunks_of(T);
    const uint8_t* cb = s->bits + uint64_t(d.chunk_off) * kChunkBytes;
    for (uint32_t c = 0; c < nch; ++c) std::memcpy(words + 8ull * (d.chunk_off + c), cb + 16 * c, 8);
    gtsr_meshlet g = d;
    g.reuse_off = static_cast<uint32_t>(ipos);
    gdesc[m] = g;
    uint32_t next_new = 3;
    uint64_t r = d.reuse_off;
    for (uint32_t t = 1; t < T; ++t) {
      const uint64_t inc = load_u64(cb + 16 * (t / 64) + 8);
      index[ipos++] = ((inc >> (t % 64)) & 1) ? static_cast<uint8_t>(next_new++) : s->reuse[r++];
    }
  }
  return ok();
}

// Consecutive meshlets of one mesh are grouped until they reach target_tris
// strip triangles; an item never crosses a mesh boundary.
extern "C" int gtsr_plan_batch(const gtsr_meshlet* const* host_meshlets, const uint32_t* meshlet_counts,
                               uint32_t mesh_count, uint32_t target_tris, gtsr_work_item* items,
                               uint32_t capacity, uint32_t* count) {
  if (!count || (mesh_count && (!host_meshlets || !meshlet_counts)))
    return fail(GTSR_EINVAL, "gtsr_plan_batch: null argument");
  if (target_tris == 0) return fail(GTSR_EINVAL, "gtsr_plan_batch: target_tris must be > 0");
  uint64_t n = 0;
  for (uint32_t i = 0; i < mesh_count; ++i) {
    const uint32_t M = meshlet_counts[i];
    if (M && !host_meshlets[i]) return fail(GTSR_EINVAL, "gtsr_plan_batch: null meshlet array");
    uint32_t first = 0;
    while (first < M) {
      uint32_t end = first;
      uint64_t tris = 0;
      while (end < M && (end == first || tris + host_meshlets[i][end].tri_count <= target_tris)) {
        tris += host_meshlets[i][end].tri_count;
        ++end;
      }
      if (items && n < capacity) items[n] = gtsr_work_item{i, first, end, 0};
      ++n;
      first = end;
    }
  }
  if (n > 0xFFFFFFFFull) return fail(GTSR_ELIMIT, "gtsr_plan_batch: too many work items");
  *count = static_cast<uint32_t>(n);
  return ok();
}
