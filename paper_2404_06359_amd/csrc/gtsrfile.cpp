// .gtsr files: a versioned container of encoded meshes, so that a pool is
// encoded once (offline, Sec. 1: encoding belongs to the asset pipeline) and
// reloaded for decoding.  Host code.
//
// Layout, little-endian:
//   header (64 bytes): magic "GTSRFILE", version, mesh count, the offsets of
//     the mesh table and of the data, the total size, and a 64-bit FNV-1a
//     hash of everything after the header;
//   mesh table: one 128-byte record per mesh (format, counts, sizes and the
//     file offset of each array);
//   data: the arrays, each starting on a 16-byte boundary (zero padding).
// A reader trusts nothing: every size and offset is checked against the file
// and against the others, the hash is checked, and every stream is checked
// against its format's invariants (gtsr_validate for GTS-Reuse) before any
// pointer is handed out.
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"

using namespace gtsr;

namespace {

constexpr char kMagic[8] = {'G', 'T', 'S', 'R', 'F', 'I', 'L', 'E'};
constexpr uint32_t kVersion = 1;
constexpr uint64_t kHeaderBytes = 64;
constexpr uint64_t kRecordBytes = 128;
constexpr uint32_t kArrays = 7;   // meshlets, bits, reuse, vertices, vert_off, kept_off, tri_ids
constexpr uint32_t kHasKept = 1, kHasTriIds = 2;

struct Header {
  char magic[8];
  uint32_t version, mesh_count;
  uint64_t table_offset, data_offset, total_bytes, hash;
  uint64_t reserved[2];
};
static_assert(sizeof(Header) == kHeaderBytes, "header layout");

struct Record {
  uint32_t format, meshlet_count;
  uint64_t strip_triangles, input_triangles, restarts;
  uint64_t bits_bytes, reuse_bytes, vertex_count;
  uint32_t flags, reserved;
  uint64_t offset[kArrays];
};
static_assert(sizeof(Record) == 120, "record layout");

uint64_t fnv1a(const uint8_t* p, uint64_t n, uint64_t h = 0xcbf29ce484222325ull) {
  for (uint64_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

uint64_t align16(uint64_t x) { return (x + 15) & ~uint64_t(15); }

// Byte sizes of mesh m's arrays, in the order of Record::offset.
void array_bytes(const Record& r, uint64_t out[kArrays]) {
  out[0] = 16ull * r.meshlet_count;
  out[1] = r.bits_bytes;
  out[2] = r.reuse_bytes;
  out[3] = 4ull * r.vertex_count;
  out[4] = 8ull * (uint64_t(r.meshlet_count) + 1);
  out[5] = (r.flags & kHasKept) ? 4ull * (uint64_t(r.meshlet_count) + 1) : 0;
  out[6] = (r.flags & kHasTriIds) ? 4ull * r.input_triangles : 0;
}

uint64_t load_u64(const uint8_t* p) {
  uint64_t v;
  std::memcpy(&v, p, 8);
  return v;
}

// Plain GTS invariants (the stream gtsr_gts_from_reuse writes): per meshlet
// one 8-byte L/R word per 64 strip triangles with no bit past T_s, and T_s - 1
// index bytes, each naming a vertex at most one past the newest so far
// (first appearance order), the newest ending at V - 1.
int validate_plain(const gtsr_meshlet* d, uint32_t M, const uint8_t* words, uint64_t words_bytes,
                   const uint8_t* index, uint64_t index_bytes, uint64_t strip_triangles, const std::string& who) {
  if (words_bytes % 8) return fail(GTSR_ECORRUPT, who + ": L/R words not a multiple of 8 bytes");
  uint64_t w = 0, ip = 0, op = 0;
  for (uint32_t m = 0; m < M; ++m) {
    const uint32_t T = d[m].tri_count, V = d[m].vert_count;
    auto bad = [&](const char* what) {
      return fail(GTSR_ECORRUPT, who + ": meshlet " + std::to_string(m) + ": " + what);
    };
    if (T < 1 || T > kMaxStripTris) return bad("tri_count out of 1..256");
    if (V < 3 || V > 256 || V > T + 2) return bad("vert_count out of range");
    if (d[m].chunk_off != w || d[m].reuse_off != ip || d[m].out_off != op) return bad("offsets not contiguous");
    const uint32_t nw = chunks_of(T);
    if (8 * (w + nw) > words_bytes || ip + (T - 1) > index_bytes) return bad("arrays past the end");
    for (uint32_t c = 0; c < nw; ++c) {
      const uint32_t valid = (c + 1 < nw || T % 64 == 0) ? 64 : T % 64;
      const uint64_t mask = valid == 64 ? ~0ull : ((1ull << valid) - 1);
      if (load_u64(words + 8 * (w + c)) & ~mask) return bad("bits set past tri_count");
    }
    uint32_t newest = 2;
    for (uint32_t t = 1; t < T; ++t) {
      const uint32_t x = index[ip + t - 1];
      if (x > newest + 1) return bad("index names a vertex out of first-appearance order");
      if (x == newest + 1) ++newest;
    }
    if (newest + 1 != V) return bad("vertex count does not match");
    w += nw;
    ip += T - 1;
    op += T;
  }
  if (8 * w != words_bytes || ip != index_bytes || op != strip_triangles)
    return fail(GTSR_ECORRUPT, who + ": array sizes do not match the descriptors");
  return GTSR_OK;
}

}  // namespace

struct gtsr_file {
  uint8_t* data = nullptr;   // the whole file, 16-byte aligned
  uint64_t bytes = 0;
  uint32_t mesh_count = 0;
  ~gtsr_file() { std::free(data); }
};

extern "C" int gtsr_file_write(const char* path, const gtsr_file_mesh* meshes, uint32_t mesh_count) {
  const std::string who = "gtsr_file_write";
  if (!path || (mesh_count && !meshes)) return fail(GTSR_EINVAL, who + ": null argument");
  std::vector<Record> recs(mesh_count);
  uint64_t pos = align16(kHeaderBytes + kRecordBytes * uint64_t(mesh_count));
  const uint64_t data_offset = pos;
  for (uint32_t i = 0; i < mesh_count; ++i) {
    const gtsr_file_mesh& g = meshes[i];
    if (g.format != GTSR_FORMAT_REUSE && g.format != GTSR_FORMAT_GTS)
      return fail(GTSR_EINVAL, who + ": mesh " + std::to_string(i) + ": bad format");
    Record& r = recs[i];
    std::memset(&r, 0, sizeof(r));
    r.format = g.format;
    r.meshlet_count = g.meshlet_count;
    r.strip_triangles = g.strip_triangles;
    r.input_triangles = g.input_triangles;
    r.restarts = g.restarts;
    r.bits_bytes = g.bits_bytes;
    r.reuse_bytes = g.reuse_bytes;
    r.vertex_count = g.vertex_count;
    r.flags = (g.kept_off ? kHasKept : 0) | (g.tri_ids ? kHasTriIds : 0);
    const void* src[kArrays] = {g.meshlets, g.bits, g.reuse, g.vertices, g.vert_off, g.kept_off, g.tri_ids};
    uint64_t sz[kArrays];
    array_bytes(r, sz);
    for (uint32_t a = 0; a < kArrays; ++a) {
      if (sz[a] && !src[a]) return fail(GTSR_EINVAL, who + ": mesh " + std::to_string(i) + ": null array");
      r.offset[a] = pos;
      pos = align16(pos + sz[a]);
    }
  }
  const uint64_t total = pos;
  std::vector<uint8_t> buf;
  try {
    buf.assign(total, 0);
  } catch (const std::bad_alloc&) {
    return fail(GTSR_ENOMEM, who + ": out of memory");
  }
  for (uint32_t i = 0; i < mesh_count; ++i) {
    const gtsr_file_mesh& g = meshes[i];
    const Record& r = recs[i];
    std::memcpy(buf.data() + kHeaderBytes + kRecordBytes * i, &r, sizeof(r));
    const void* src[kArrays] = {g.meshlets, g.bits, g.reuse, g.vertices, g.vert_off, g.kept_off, g.tri_ids};
    uint64_t sz[kArrays];
    array_bytes(r, sz);
    for (uint32_t a = 0; a < kArrays; ++a)
      if (sz[a]) std::memcpy(buf.data() + r.offset[a], src[a], sz[a]);
  }
  Header h{};
  std::memcpy(h.magic, kMagic, 8);
  h.version = kVersion;
  h.mesh_count = mesh_count;
  h.table_offset = kHeaderBytes;
  h.data_offset = data_offset;
  h.total_bytes = total;
  h.hash = fnv1a(buf.data() + kHeaderBytes, total - kHeaderBytes);
  std::memcpy(buf.data(), &h, sizeof(h));
  // write to a temporary name, then rename: a reader never sees half a file
  const std::string tmp = std::string(path) + ".partial";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(GTSR_EIO, who + ": cannot create " + tmp + ": " + std::strerror(errno));
  const bool written = std::fwrite(buf.data(), 1, total, f) == total;
  const bool closed = std::fclose(f) == 0;
  if (!written || !closed) {
    std::remove(tmp.c_str());
    return fail(GTSR_EIO, who + ": cannot write " + tmp);
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(GTSR_EIO, who + ": cannot rename to " + std::string(path) + ": " + std::strerror(errno));
  }
  return ok();
}

extern "C" int gtsr_file_open(const char* path, gtsr_file** out) {
  const std::string who = "gtsr_file_open";
  if (!path || !out) return fail(GTSR_EINVAL, who + ": null argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(GTSR_EIO, who + ": cannot open " + std::string(path) + ": " + std::strerror(errno));
  uint64_t size = 0;
  if (std::fseek(f, 0, SEEK_END) == 0) {
    const long n = std::ftell(f);
    size = n > 0 ? uint64_t(n) : 0;
  }
  std::rewind(f);
  auto* file = new (std::nothrow) gtsr_file();
  if (!file) {
    std::fclose(f);
    return fail(GTSR_ENOMEM, who + ": out of memory");
  }
  if (size) file->data = static_cast<uint8_t*>(std::aligned_alloc(16, align16(size)));
  if (size && !file->data) {
    std::fclose(f);
    delete file;
    return fail(GTSR_ENOMEM, who + ": out of memory");
  }
  const bool read = size == 0 || std::fread(file->data, 1, size, f) == size;
  std::fclose(f);
  file->bytes = size;
  auto corrupt = [&](const std::string& what) {
    delete file;
    return fail(GTSR_ECORRUPT, who + ": " + std::string(path) + ": " + what);
  };
  if (!read) {
    delete file;
    return fail(GTSR_EIO, who + ": cannot read " + std::string(path));
  }
  if (size < kHeaderBytes) return corrupt("shorter than the header");
  Header h;
  std::memcpy(&h, file->data, sizeof(h));
  if (std::memcmp(h.magic, kMagic, 8) != 0) return corrupt("not a .gtsr file");
  if (h.version != kVersion) return corrupt("unsupported version " + std::to_string(h.version));
  if (h.total_bytes != size) return corrupt("size does not match the header (truncated or extended)");
  if (h.table_offset != kHeaderBytes || h.mesh_count > (size - kHeaderBytes) / kRecordBytes ||
      h.data_offset < kHeaderBytes + kRecordBytes * uint64_t(h.mesh_count) || h.data_offset > size ||
      h.data_offset % 16)
    return corrupt("bad table or data offset");
  if (fnv1a(file->data + kHeaderBytes, size - kHeaderBytes) != h.hash) return corrupt("hash mismatch");
  file->mesh_count = h.mesh_count;
  for (uint32_t i = 0; i < h.mesh_count; ++i) {
    Record r;
    std::memcpy(&r, file->data + kHeaderBytes + kRecordBytes * i, sizeof(r));
    const std::string mesh = "mesh " + std::to_string(i) + ": ";
    if (r.format != GTSR_FORMAT_REUSE && r.format != GTSR_FORMAT_GTS) return corrupt(mesh + "bad format");
    if (r.flags & ~(kHasKept | kHasTriIds)) return corrupt(mesh + "unknown flags");
    if (r.meshlet_count > (1u << 30) || r.input_triangles > (uint64_t(1) << 40) ||
        r.vertex_count > (uint64_t(1) << 40))
      return corrupt(mesh + "counts out of range");
    uint64_t sz[kArrays];
    array_bytes(r, sz);
    for (uint32_t a = 0; a < kArrays; ++a)
      if (r.offset[a] % 16 || r.offset[a] < h.data_offset || r.offset[a] > size || sz[a] > size - r.offset[a])
        return corrupt(mesh + "array " + std::to_string(a) + " outside the file");
    gtsr_file_mesh g;
    if (int rc = gtsr_file_mesh_get(file, i, &g)) {
      delete file;
      return rc;
    }
    // vertex lists: offsets from 0, non-decreasing, V per meshlet, ending at the count
    uint64_t vpos = 0;
    for (uint32_t m = 0; m < r.meshlet_count; ++m) {
      if (g.vert_off[m] != vpos) return corrupt(mesh + "vertex offsets not contiguous");
      vpos += g.meshlets[m].vert_count;
    }
    if (g.vert_off[r.meshlet_count] != vpos || vpos != r.vertex_count) return corrupt(mesh + "vertex count");
    if (g.kept_off) {
      if (g.kept_off[0] != 0 || g.kept_off[r.meshlet_count] != r.input_triangles)
        return corrupt(mesh + "kept offsets do not span the input triangles");
      for (uint32_t m = 0; m < r.meshlet_count; ++m)
        if (g.kept_off[m + 1] < g.kept_off[m] || g.kept_off[m + 1] - g.kept_off[m] > g.meshlets[m].tri_count)
          return corrupt(mesh + "kept offsets out of order");
    }
    int rc;
    if (r.format == GTSR_FORMAT_REUSE) {
      const gtsr_stream s{g.meshlets, g.bits, g.reuse, g.meshlet_count, 0, g.bits_bytes, g.reuse_bytes,
                          g.strip_triangles};
      rc = gtsr_validate(&s);
    } else {
      rc = validate_plain(g.meshlets, g.meshlet_count, g.bits, g.bits_bytes, g.reuse, g.reuse_bytes,
                          g.strip_triangles, who + ": " + mesh);
    }
    if (rc != GTSR_OK) {
      const std::string why = gtsr_last_error();
      return corrupt(mesh + why);
    }
  }
  *out = file;
  return ok();
}

extern "C" int gtsr_file_mesh_count(const gtsr_file* file, uint32_t* count) {
  if (!file || !count) return fail(GTSR_EINVAL, "gtsr_file_mesh_count: null argument");
  *count = file->mesh_count;
  return ok();
}

extern "C" int gtsr_file_mesh_get(const gtsr_file* file, uint32_t i, gtsr_file_mesh* mesh) {
  if (!file || !mesh) return fail(GTSR_EINVAL, "gtsr_file_mesh_get: null argument");
  Header h;
  std::memcpy(&h, file->data, sizeof(h));
  if (i >= h.mesh_count) return fail(GTSR_EINVAL, "gtsr_file_mesh_get: mesh index out of range");
  Record r;
  std::memcpy(&r, file->data + kHeaderBytes + kRecordBytes * i, sizeof(r));
  uint64_t sz[kArrays];
  array_bytes(r, sz);
  const uint8_t* base = file->data;
  auto at = [&](uint32_t a) -> const uint8_t* { return sz[a] ? base + r.offset[a] : nullptr; };
  std::memset(mesh, 0, sizeof(*mesh));
  mesh->format = r.format;
  mesh->meshlet_count = r.meshlet_count;
  mesh->strip_triangles = r.strip_triangles;
  mesh->input_triangles = r.input_triangles;
  mesh->restarts = r.restarts;
  mesh->meshlets = reinterpret_cast<const gtsr_meshlet*>(at(0));
  mesh->bits = at(1);
  mesh->bits_bytes = r.bits_bytes;
  mesh->reuse = at(2);
  mesh->reuse_bytes = r.reuse_bytes;
  mesh->vertices = reinterpret_cast<const uint32_t*>(at(3));
  mesh->vertex_count = r.vertex_count;
  mesh->vert_off = reinterpret_cast<const uint64_t*>(base + r.offset[4]);
  mesh->kept_off = reinterpret_cast<const uint32_t*>(at(5));
  mesh->tri_ids = reinterpret_cast<const uint32_t*>(at(6));
  return ok();
}

extern "C" void gtsr_file_close(gtsr_file* file) { delete file; }
