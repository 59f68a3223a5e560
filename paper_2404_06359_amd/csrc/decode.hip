// GPU decoders for GTS-Reuse meshlet connectivity, written for CDNA4 (gfx950).
//
// Kuth et al., "Towards Practical Meshlet Compression", Sec. 4.2 / 4.3: every
// triangle of a strip is produced on its own, without the triangle before it.
// Per strip triangle t (one lane each, 64 per chunk):
//
//   index stream  I[0..2] = 0,1,2;  for t >= 1 with increment flag g[t] set,
//                 I[t+2] = s_t = 2 + sum_{u=1..t} g[u]  (prefix count, mbcnt);
//                 with g[t] clear, I[t+2] = reuse[t + 1 - s_t], where
//                 t + 1 - s_t is the number of clear flags before t: the rank
//                 of t among the reuse slots, i.e. mbcnt of the complemented
//                 increment word plus a carried count.
//   pivot         the last L/R flip at or before t: with the change word
//                 ch[j] = f[j] xor f[j-1] (ch[0] = 0), j_t = max{j <= t: ch[j]}
//                 (0 if none) and X_t = I[j_t] -- the same vertex as I[k+1]
//                 for the last k < t with f[k] != f[t]; a count-leading-zeros
//                 of ch shifted so that bit t is the top bit, else the last
//                 change carried from earlier chunks (fans longer than a word).
//   triangle      f[t] = L: (X_t, I[t+1], I[t+2]);  R: (I[t+1], X_t, I[t+2]).
//
// Data movement.  A wavefront decodes a run of consecutive meshlets of one
// mesh: it loads up to 32 descriptors with one vector load, stages the run's
// flag chunks and reuse bytes in LDS with coalesced loads, decodes each
// meshlet from LDS into an LDS output tile, then writes the run's output
// bytes (contiguous in the stream layout) with dword stores.  The chunk loop
// touches no global memory.  A run holds at most kRunTris strip triangles so
// that the tile fits LDS at full occupancy.
//
// Memory safety on corrupted input: a meshlet whose descriptor points
// outside the given sizes (or outside the run's LDS tile) ends the run and is
// skipped; every LDS index is bounded by the tile sizes whatever the flag
// bits say.

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "common.h"

namespace gtsr {
namespace {

constexpr uint32_t kWave = 64;
constexpr uint32_t kMaxWavesPerGroup = 16;
constexpr uint32_t kXcds = 8;                // workgroups go round-robin over 8 XCDs
constexpr uint64_t kWorkspaceBytes = 256;
constexpr uint32_t kRunTris = 768;           // strip triangles per run (LDS tile)
constexpr uint32_t kRunMeshlets = 32;        // meshlets per run (one descriptor per lane)

// One wavefront's LDS tile.
struct RunTile {
  static constexpr uint32_t kChunks = kRunTris / 64 + kRunMeshlets;
  uint4 bits[kChunks];                       // LR lo/hi, INC lo/hi per chunk
  uint32_t out[(3 * kRunTris + 3 * 64 + 8) / 4];   // + a partial chunk past the end, + shift
  uint8_t reuse[kRunTris + 256 + 64];        // + reads by lanes whose flags say "new"
  uint8_t idx[272];                          // I[0 .. T_s+1] of the current meshlet
};
constexpr uint32_t kTileBytes = sizeof(RunTile);

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Orders this wavefront's LDS writes before its later LDS reads of other
// lanes' values; LDS operations of one wavefront complete in issue order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t mbcnt64(uint64_t mask, uint32_t base) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), base));
}

struct Stream {
  const gtsr_meshlet* meshlets;
  const uint8_t* bits;
  const uint8_t* reuse;
  uint8_t* out;
  uint64_t chunks;
  uint64_t reuse_bytes;
  uint64_t out_tris;
};

// Per-meshlet state carried from chunk to chunk (all wave-uniform).
struct ChunkCarry {
  uint32_t inc_base;      // 1 + increments before this chunk (triangle 0 counted as one)
  uint32_t reuse_pos;     // reuse slots before this chunk, plus the meshlet's tile offset
  uint32_t last_change;   // last L/R flip position in earlier chunks (0: none)
  uint64_t prev_top;      // flag of the previous chunk's last triangle
};

// Chunk C (strip triangles 64C .. 64C+63) of the meshlet whose flag chunks
// start at tile.bits + co and whose output starts at tile byte ob.
template <uint32_t C>
__device__ __forceinline__ void decode_chunk(RunTile& tile, uint32_t co, uint32_t ob, uint32_t lane,
                                             ChunkCarry& k) {
  uint8_t* I = tile.idx;
  const uint4 w = tile.bits[co + C];
  const uint64_t lr = (uint64_t(uniform(w.y)) << 32) | uniform(w.x);
  uint64_t inc = (uint64_t(uniform(w.w)) << 32) | uniform(w.z);
  uint64_t ch = lr ^ ((lr << 1) | k.prev_top);
  if (C == 0) {
    inc |= 1;    // triangle 0 counts as introducing vertex 2 (I[2] = 2)
    ch &= ~1ull;
  }
  const uint32_t t = 64 * C + lane;
  // new slot I[t+2]: the next vertex number, or the reuse byte whose rank is
  // the number of reuse slots before t (lanes below minus increments below)
  const uint32_t ones = __builtin_amdgcn_mbcnt_hi(uint32_t(inc >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(inc), 0u));
  const uint32_t fresh = ones + k.inc_base + 1;
  const uint32_t r = tile.reuse[(k.reuse_pos + lane) - ones];
  const uint32_t N = __builtin_amdgcn_inverse_ballot_w64(inc) ? fresh : r;
  I[t + 2] = uint8_t(N);
  // pivot: the last flip at or before t
  const uint64_t upto = ch << (63 - lane);
  const uint32_t piv = upto ? t - uint32_t(__builtin_clzll(upto)) : k.last_change;

  if (ch) k.last_change = 64 * C + 63 - uint32_t(__builtin_clzll(ch));
  k.prev_top = lr >> 63;
  const uint32_t news = uint32_t(__builtin_popcountll(inc));
  k.inc_base += news;
  k.reuse_pos += 64 - news;

  wave_lds_sync();
  const uint32_t P = I[t + 1];
  const uint32_t X = I[piv];
  const bool right = __builtin_amdgcn_inverse_ballot_w64(lr);
  uint8_t* o = reinterpret_cast<uint8_t*>(tile.out) + ob + 3 * t;
  o[0] = uint8_t(right ? P : X);
  o[1] = uint8_t(right ? X : P);
  o[2] = uint8_t(N);
}

// Decodes one meshlet whose flag chunks start at tile.bits[co], reuse bytes
// at tile.reuse[ro], output at tile byte ob.  T: strip triangles (1..256).
// Lanes past T compute garbage that lands past the meshlet's output (the next
// meshlet overwrites it, or it lies past the run and is never stored).
__device__ __forceinline__ void decode_meshlet(RunTile& tile, uint32_t co, uint32_t ro, uint32_t ob, uint32_t T,
                                               uint32_t lane) {
  ChunkCarry k{1, ro, 0, 0};
  decode_chunk<0>(tile, co, ob, lane, k);
  if (T > 64) decode_chunk<1>(tile, co, ob, lane, k);
  if (T > 128) decode_chunk<2>(tile, co, ob, lane, k);
  if (T > 192) decode_chunk<3>(tile, co, ob, lane, k);
  wave_lds_sync();
}

// Writes tile bytes [shift, shift + bytes) to dst - shift + [shift, ...):
// whole dwords where the dword lies inside the span, single bytes at its two
// ragged ends.  dst is 4-byte aligned minus shift.
__device__ __forceinline__ void store_span(uint8_t* dst_run, uint32_t bytes, const RunTile& tile, uint32_t lane) {
  const uint32_t shift = uint32_t(reinterpret_cast<uintptr_t>(dst_run)) & 3u;
  uint32_t* g = reinterpret_cast<uint32_t*>(dst_run - shift);
  const uint32_t end = shift + bytes;
  const uint32_t nd = (end + 3) >> 2;
  for (uint32_t j = lane; j < nd; j += kWave) {
    const uint32_t w = tile.out[j];
    const uint32_t lo = 4 * j;
    if (lo >= shift && lo + 4 <= end) {
      g[j] = w;
    } else {
      uint8_t* gb = reinterpret_cast<uint8_t*>(g + j);
      for (uint32_t b = 0; b < 4; ++b)
        if (lo + b >= shift && lo + b < end) gb[b] = uint8_t(w >> (8 * b));
    }
  }
}

// Decodes meshlets [m, m_end) of stream s with the calling wavefront, run by
// run.  tile.idx[0..2] must hold 0,1,2.
__device__ __forceinline__ void decode_range(const Stream& s, uint32_t m, uint32_t m_end, RunTile& tile,
                                          uint32_t lane) {
  while (m < m_end) {
    const uint32_t cnt = min(m_end - m, kRunMeshlets);
    uint4 d = make_uint4(0, 0, 0, 0);
    if (lane < cnt) d = *reinterpret_cast<const uint4*>(s.meshlets + m + lane);
    const uint32_t T = d.w & 0xFFFFu, V = d.w >> 16;
    const uint32_t nch = (T + 63) >> 6;
    const uint32_t nru = T + 2 - V;
    const uint32_t c0 = uniform(d.x), r0 = uniform(d.y), o0 = uniform(d.z);
    const uint32_t ra = r0 & ~3u;   // reuse bytes are staged from a dword boundary
    bool ok = lane < cnt && T - 1u < kMaxStripTris && V >= 3 && V <= 256 && V <= T + 2;
    ok = ok && uint64_t(d.x) + nch <= s.chunks && uint64_t(d.y) + nru <= s.reuse_bytes &&
         uint64_t(d.z) + T <= s.out_tris;
    ok = ok && d.x - c0 + nch <= RunTile::kChunks && d.y - ra + nru <= kRunTris + 3 &&
         d.z - o0 + T <= kRunTris && d.x >= c0 && d.y >= r0 && d.z >= o0;
    const uint64_t okm = __builtin_amdgcn_ballot_w64(ok);
    const uint32_t k = uint32_t(__builtin_ctzll(~okm));   // leading run of usable meshlets
    if (k == 0) {   // the first meshlet is unusable: skip it
      ++m;
      continue;
    }
    const uint32_t c_end = __builtin_amdgcn_readlane(d.x + nch, k - 1);
    const uint32_t r_end = __builtin_amdgcn_readlane(d.y + nru, k - 1);
    const uint32_t o_end = __builtin_amdgcn_readlane(d.z + T, k - 1);

    // stage flag chunks and reuse bytes
    const uint4* gbits = reinterpret_cast<const uint4*>(s.bits) + c0;
    for (uint32_t j = lane; j < c_end - c0; j += kWave) tile.bits[j] = gbits[j];
    const uint32_t nrd = (r_end - ra + 3) >> 2;
    uint32_t* treuse = reinterpret_cast<uint32_t*>(tile.reuse);
    for (uint32_t j = lane; j < nrd; j += kWave) {
      const uint64_t gofs = uint64_t(ra) + 4 * j;
      uint32_t v;
      if (gofs + 4 <= s.reuse_bytes) {
        v = *reinterpret_cast<const uint32_t*>(s.reuse + gofs);
      } else {   // the array ends inside this dword
        v = 0;
        for (uint32_t b = 0; b < 4; ++b)
          if (gofs + b < s.reuse_bytes) v |= uint32_t(s.reuse[gofs + b]) << (8 * b);
      }
      treuse[j] = v;
    }
    wave_lds_sync();

    uint8_t* dst = s.out + 3ull * o0;
    const uint32_t shift = uint32_t(reinterpret_cast<uintptr_t>(dst)) & 3u;
    for (uint32_t i = 0; i < k; ++i) {
      const uint32_t co = __builtin_amdgcn_readlane(d.x, i) - c0;
      const uint32_t ro = __builtin_amdgcn_readlane(d.y, i) - ra;
      const uint32_t oo = __builtin_amdgcn_readlane(d.z, i) - o0;
      const uint32_t Ti = __builtin_amdgcn_readlane(T, i);
      decode_meshlet(tile, co, ro, shift + 3 * oo, Ti, lane);
    }
    store_span(dst, 3 * (o_end - o0), tile, lane);
    wave_lds_sync();
    m += k;
  }
}

__device__ __forceinline__ RunTile& wave_tile(uint32_t wave, uint32_t lane) {
  extern __shared__ uint4 lds_tiles[];
  RunTile& tile = reinterpret_cast<RunTile*>(lds_tiles)[wave];
  if (lane < 3) tile.idx[lane] = uint8_t(lane);
  return tile;
}

// Plain decoder: workgroup b covers waves_per_group * mpw consecutive
// meshlets; wave w of it the w-th run of mpw.  Consecutive workgroups go to
// different XCDs, so tiles are handed out XCD-major: each XCD decodes one
// contiguous stretch of the mesh and its L2 sees whole output lines.
__global__ __launch_bounds__(kWave * kMaxWavesPerGroup) void k_decode_plain(
    const gtsr_meshlet* __restrict__ meshlets, const uint8_t* __restrict__ bits,
    const uint8_t* __restrict__ reuse, uint8_t* __restrict__ out, uint32_t meshlet_count,
    uint64_t chunks, uint64_t reuse_bytes, uint64_t out_tris, uint32_t mpw) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = uniform(threadIdx.x / kWave);
  const uint32_t waves = blockDim.x / kWave;
  RunTile& tile = wave_tile(wave, lane);
  const uint32_t per_xcd = gridDim.x / kXcds;
  const uint32_t group = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  const uint64_t m0 = (uint64_t(group) * waves + wave) * mpw;
  if (m0 >= meshlet_count) return;
  const uint32_t m1 = uint32_t(min(m0 + mpw, uint64_t(meshlet_count)));
  const Stream s{meshlets, bits, reuse, out, chunks, reuse_bytes, out_tris};
  decode_range(s, uint32_t(m0), m1, tile, lane);
}

// Persistent batched decoder: every wavefront takes work items (a run of
// meshlets of one mesh) from a shared counter until none are left.
__global__ __launch_bounds__(kWave * kMaxWavesPerGroup) void k_decode_batched(
    const gtsr_mesh_entry* __restrict__ table, uint32_t mesh_count,
    const gtsr_work_item* __restrict__ work, uint32_t work_items, uint32_t* __restrict__ counter) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = uniform(threadIdx.x / kWave);
  RunTile& tile = wave_tile(wave, lane);
  for (;;) {
    uint32_t item = 0;
    if (lane == 0) item = atomicAdd(counter, 1u);
    item = uniform(item);
    if (item >= work_items) break;
    const gtsr_work_item wi = work[item];
    const uint32_t mesh = uniform(wi.mesh);
    if (mesh >= mesh_count) continue;
    const gtsr_mesh_entry& e = table[mesh];
    Stream s;
    s.meshlets = e.meshlets;
    s.bits = e.bits;
    s.reuse = e.reuse;
    s.out = e.out;
    s.chunks = e.bits_bytes / 16;
    s.reuse_bytes = e.reuse_bytes;
    s.out_tris = e.strip_triangles;
    const uint32_t mcount = e.meshlet_count;
    const uint32_t first = uniform(wi.first);
    const uint32_t end = min(uniform(wi.end), mcount);
    if (first < end) decode_range(s, first, end, tile, lane);
  }
}

__global__ void k_fill_zero(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

struct Defaults {
  uint32_t waves = 4, mpw = 16, gpc = 8;
};

int resolve_cfg(const gtsr_launch_cfg* cfg, Defaults& d, const char* who) {
  if (!cfg) return GTSR_OK;
  if (cfg->reserved) return fail(GTSR_EINVAL, std::string(who) + ": cfg.reserved must be 0");
  if (cfg->waves_per_group) {
    if (cfg->waves_per_group > kMaxWavesPerGroup) return fail(GTSR_EINVAL, std::string(who) + ": waves_per_group > 16");
    d.waves = cfg->waves_per_group;
  }
  if (cfg->meshlets_per_wave) {
    if (cfg->meshlets_per_wave > 64) return fail(GTSR_EINVAL, std::string(who) + ": meshlets_per_wave > 64");
    d.mpw = cfg->meshlets_per_wave;
  }
  if (cfg->groups_per_cu) {
    if (cfg->groups_per_cu > 32) return fail(GTSR_EINVAL, std::string(who) + ": groups_per_cu > 32");
    d.gpc = cfg->groups_per_cu;
  }
  return GTSR_OK;
}

std::mutex g_cu_mutex;
std::vector<uint32_t> g_cu_count;   // per device, 0 = not queried yet

uint32_t cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  std::lock_guard<std::mutex> lk(g_cu_mutex);
  if (g_cu_count.size() <= size_t(dev)) g_cu_count.resize(dev + 1, 0);
  if (!g_cu_count[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 0;
    g_cu_count[dev] = uint32_t(n);
  }
  return g_cu_count[dev];
}

int check_launch(const char* who) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GTSR_EHIP, std::string(who) + ": " + hipGetErrorString(e));
  return ok();
}

int enqueue_batched(const gtsr_mesh_entry* table, uint32_t mesh_count, const gtsr_work_item* work,
                    uint32_t work_items, void* workspace, uint64_t workspace_bytes,
                    const gtsr_launch_cfg* cfg, hipStream_t stream, const char* who) {
  if ((mesh_count && !table) || (work_items && !work) || !workspace)
    return fail(GTSR_EINVAL, std::string(who) + ": null pointer");
  if (workspace_bytes < kWorkspaceBytes || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return fail(GTSR_EINVAL, std::string(who) + ": workspace must be >= 256 bytes, 256-byte aligned");
  if ((reinterpret_cast<uintptr_t>(table) & 15) || (reinterpret_cast<uintptr_t>(work) & 15))
    return fail(GTSR_EINVAL, std::string(who) + ": tables must be 16-byte aligned");
  Defaults d;
  if (int rc = resolve_cfg(cfg, d, who)) return rc;
  const uint32_t cus = cu_count();
  if (!cus) return fail(GTSR_EHIP, std::string(who) + ": cannot query the device");
  uint32_t* counter = static_cast<uint32_t*>(workspace);
  hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(64), 0, stream, counter, uint32_t(kWorkspaceBytes / 4));
  if (int rc = check_launch(who)) return rc;
  uint32_t groups = cus * d.gpc;
  groups = (groups + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL(k_decode_batched, dim3(groups), dim3(kWave * d.waves), d.waves * kTileBytes, stream,
                     table, mesh_count, work, work_items, counter);
  return check_launch(who);
}

}  // namespace
}  // namespace gtsr

using namespace gtsr;

namespace gtsr {
namespace {

int check_plain_args(const gtsr_stream* dev, const uint8_t* dev_out, uint64_t out_bytes) {
  if (!dev) return fail(GTSR_EINVAL, "decode_meshlets: null stream");
  if (dev->meshlet_count == 0) return GTSR_OK;
  if (!dev->meshlets || !dev->bits || !dev_out || (dev->reuse_bytes && !dev->reuse))
    return fail(GTSR_EINVAL, "decode_meshlets: null device pointer");
  if (out_bytes / 3 < dev->strip_triangles)
    return fail(GTSR_EINVAL, "decode_meshlets: out_bytes < 3 * strip_triangles");
  if ((reinterpret_cast<uintptr_t>(dev->meshlets) & 15) || (reinterpret_cast<uintptr_t>(dev->bits) & 15))
    return fail(GTSR_EINVAL, "decode_meshlets: meshlets and bits must be 16-byte aligned");
  const uint64_t groups = (uint64_t(dev->meshlet_count) + 15) / 16 * 16;
  if (groups > 0x7FFFFFFFull) return fail(GTSR_ELIMIT, "decode_meshlets: grid too large");
  return GTSR_OK;
}

void launch_plain(const gtsr_stream* dev, uint8_t* dev_out, uint64_t out_bytes, const Defaults& d,
                  hipStream_t stream) {
  if (dev->meshlet_count == 0) return;
  const uint64_t per_group = uint64_t(d.waves) * d.mpw;
  uint64_t groups = (dev->meshlet_count + per_group - 1) / per_group;
  groups = (groups + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL(k_decode_plain, dim3(uint32_t(groups)), dim3(kWave * d.waves), d.waves * kTileBytes,
                     stream, dev->meshlets, dev->bits, dev->reuse, dev_out, dev->meshlet_count,
                     dev->bits_bytes / 16, dev->reuse_bytes, out_bytes / 3, d.mpw);
}

}  // namespace
}  // namespace gtsr

extern "C" int gtsr_decode_meshlets_cfg(const gtsr_stream* dev, uint8_t* dev_out, uint64_t out_bytes,
                                        const gtsr_launch_cfg* cfg, void* hip_stream) {
  if (int rc = check_plain_args(dev, dev_out, out_bytes)) return rc;
  Defaults d;
  if (int rc = resolve_cfg(cfg, d, "decode_meshlets")) return rc;
  launch_plain(dev, dev_out, out_bytes, d, static_cast<hipStream_t>(hip_stream));
  return check_launch("decode_meshlets");
}

extern "C" int gtsr_decode_meshlets_many(const gtsr_stream* streams, uint8_t* const* dev_outs,
                                         const uint64_t* out_bytes, uint32_t n, const gtsr_launch_cfg* cfg,
                                         void* hip_stream) {
  if (n && (!streams || !dev_outs || !out_bytes))
    return fail(GTSR_EINVAL, "gtsr_decode_meshlets_many: null argument");
  Defaults d;
  if (int rc = resolve_cfg(cfg, d, "gtsr_decode_meshlets_many")) return rc;
  for (uint32_t i = 0; i < n; ++i)
    if (int rc = check_plain_args(&streams[i], dev_outs[i], out_bytes[i])) return rc;
  for (uint32_t i = 0; i < n; ++i)
    launch_plain(&streams[i], dev_outs[i], out_bytes[i], d, static_cast<hipStream_t>(hip_stream));
  return check_launch("gtsr_decode_meshlets_many");
}

extern "C" int decode_meshlets(const gtsr_stream* dev, uint8_t* dev_out, uint64_t out_bytes, void* hip_stream) {
  return gtsr_decode_meshlets_cfg(dev, dev_out, out_bytes, nullptr, hip_stream);
}

extern "C" uint64_t gtsr_batched_workspace_bytes(void) { return kWorkspaceBytes; }

extern "C" int decode_meshlets_batched(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                                       const gtsr_work_item* dev_work, uint32_t work_items,
                                       void* dev_workspace, uint64_t workspace_bytes,
                                       const gtsr_launch_cfg* cfg, void* hip_stream) {
  return enqueue_batched(dev_mesh_table, mesh_count, dev_work, work_items, dev_workspace, workspace_bytes,
                         cfg, static_cast<hipStream_t>(hip_stream), "decode_meshlets_batched");
}

extern "C" int gtsr_batched_graph_create(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                                         const gtsr_work_item* dev_work, uint32_t work_items,
                                         void* dev_workspace, uint64_t workspace_bytes,
                                         const gtsr_launch_cfg* cfg, void** graph_exec) {
  const char* who = "gtsr_batched_graph_create";
  if (!graph_exec) return fail(GTSR_EINVAL, "gtsr_batched_graph_create: null graph_exec");
  *graph_exec = nullptr;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
    return fail(GTSR_EHIP, "gtsr_batched_graph_create: stream creation failed");
  hipGraph_t graph = nullptr;
  int rc = GTSR_OK;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = fail(GTSR_EHIP, "gtsr_batched_graph_create: begin capture failed");
  } else {
    rc = enqueue_batched(dev_mesh_table, mesh_count, dev_work, work_items, dev_workspace, workspace_bytes,
                         cfg, s, who);
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc == GTSR_OK && e != hipSuccess)
      rc = fail(GTSR_EHIP, std::string(who) + ": end capture: " + hipGetErrorString(e));
  }
  if (rc == GTSR_OK) {
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = fail(GTSR_EHIP, std::string(who) + ": instantiate: " + hipGetErrorString(e));
    else *graph_exec = exec;
  }
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(s);
  return rc == GTSR_OK ? ok() : rc;
}

extern "C" int gtsr_graph_launch(void* graph_exec, void* hip_stream) {
  if (!graph_exec) return fail(GTSR_EINVAL, "gtsr_graph_launch: null graph");
  hipError_t e = hipGraphLaunch(static_cast<hipGraphExec_t>(graph_exec), static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(GTSR_EHIP, std::string("gtsr_graph_launch: ") + hipGetErrorString(e));
  return ok();
}

extern "C" void gtsr_graph_destroy(void* graph_exec) {
  if (graph_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph_exec));
}

extern "C" uint32_t gtsr_device_cu_count(void) { return cu_count(); }
