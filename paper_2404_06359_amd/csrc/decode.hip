// GPU decoders for GTS-Reuse meshlet connectivity, written for CDNA4 (gfx950).
//
// Kuth et al., "Towards Practical Meshlet Compression", Sec. 4.2 / 4.3: the
// decoder must produce every triangle independently, without the triangle
// before it.  Per strip triangle t (one lane each, 64 per chunk):
//
//   index stream  I[0..2] = 0,1,2;  for t >= 1:  s_t = 2 + sum_{u=1..t} g[u]
//                 I[t+2] = g[t] ? s_t : reuse[t + 1 - s_t]
//   pivot         the last flip of the L/R flags at or before t: with the
//                 change mask  ch[j] = f[j] xor f[j-1]  (ch[0] = 0),
//                 j_t = max{ j <= t : ch[j] = 1 }  (0 if none) and X_t = I[j_t]
//                 (equivalently I[k+1] for the last k < t with f[k] != f[t])
//   triangle      f[t] = L: (X_t, I[t+1], I[t+2]);  R: (I[t+1], X_t, I[t+2])
//
// The flag words are uniform across the wave and sit in scalar registers;
// s_t is the wave's popcount prefix (mbcnt) of the increment word plus a
// carried base; j_t is a count-leading-zeros on the change word shifted so
// that lane t's bit is the top bit, else the last change carried from earlier
// chunks (fans longer than one word, Sec. 4.2).  I[] lives in LDS, one array
// per wavefront; each lane writes I[t+2] and reads I[t+1] and I[j_t].
//
// Memory safety on corrupted input: a meshlet whose descriptor points outside
// the given array sizes is skipped, reuse reads are clamped into the
// meshlet's own reuse bytes, and all LDS indices stay below T_s + 2.

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "common.h"

namespace gtsr {
namespace {

constexpr uint32_t kWave = 64;
constexpr uint32_t kIdxBytes = 272;          // I[0 .. T_s+1] for T_s <= 256, padded
constexpr uint32_t kMaxWavesPerGroup = 16;
constexpr uint32_t kXcds = 8;                // workgroups go round-robin over 8 XCDs
constexpr uint64_t kWorkspaceBytes = 256;

// Loads through the constant address space: a wave-uniform address becomes a
// scalar load into SGPRs.  Only used for data the kernels never write.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) u32x4 const_u32x4;

__device__ __forceinline__ uint4 load_uniform16(const void* p) {
  const u32x4 v = *reinterpret_cast<const_u32x4*>(reinterpret_cast<uintptr_t>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Orders this wavefront's LDS writes before its later LDS reads (other lanes'
// values); LDS operations of one wavefront complete in issue order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// Decodes meshlet m of stream s with the calling wavefront.  I: this wave's
// LDS index array with I[0..2] = 0,1,2 already in place.
__device__ __forceinline__ void decode_meshlet(const Stream& s, uint32_t m, uint8_t* I, uint32_t lane) {
  const uint4 d = load_uniform16(s.meshlets + m);
  const uint32_t chunk_off = d.x, reuse_off = d.y, out_off = d.z;
  const uint32_t T = d.w & 0xFFFFu, V = d.w >> 16;
  const uint32_t nch = (T + 63) >> 6;
  const int32_t n_ru = int32_t(T) + 2 - int32_t(V);
  if (T - 1u >= kMaxStripTris || V < 3 || V > 256 || n_ru < 0) return;
  if (uint64_t(chunk_off) + nch > s.chunks || uint64_t(reuse_off) + uint32_t(n_ru) > s.reuse_bytes ||
      uint64_t(out_off) + T > s.out_tris)
    return;
  const uint8_t* cb = s.bits + 16ull * chunk_off;
  const uint8_t* rb = s.reuse + reuse_off;
  uint8_t* ob = s.out + 3ull * out_off;

  uint32_t inc_base = 2;      // 2 + increments in earlier chunks
  uint32_t last_change = 0;   // last L/R change position in earlier chunks (0: none)
  uint64_t prev_top = 0;      // flag of the last triangle of the previous chunk
  for (uint32_t c = 0; c < nch; ++c) {
    const uint4 w = load_uniform16(cb + 16ull * c);
    const uint64_t lr = (uint64_t(w.y) << 32) | w.x;
    uint64_t inc = (uint64_t(w.w) << 32) | w.z;
    uint64_t ch = lr ^ ((lr << 1) | prev_top);
    if (c == 0) { inc &= ~1ull; ch &= ~1ull; }

    const uint32_t t = 64 * c + lane;
    const bool active = t < T;
    const uint32_t f = uint32_t(lr >> lane) & 1u;
    const uint32_t g = uint32_t(inc >> lane) & 1u;
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(uint32_t(inc >> 32),
                                                     __builtin_amdgcn_mbcnt_lo(uint32_t(inc), 0u));
    const uint32_t s_t = inc_base + below + g;
    uint32_t N = s_t;
    if (active && !g) {
      if (t == 0) {
        N = 2;
      } else {
        int32_t r = int32_t(t + 1 - s_t);
        r = r < n_ru - 1 ? r : n_ru - 1;
        N = r >= 0 ? rb[r] : 0u;
      }
    }
    if (active && t > 0) I[t + 2] = uint8_t(N);

    const uint64_t upto = ch << (63 - lane);   // change bits at or below lane t, lane t on top
    const uint32_t piv = upto ? (t - uint32_t(__builtin_clzll(upto))) : last_change;

    if (ch) last_change = 64 * c + 63 - uint32_t(__builtin_clzll(ch));
    prev_top = lr >> 63;
    inc_base += uint32_t(__builtin_popcountll(inc));

    wave_lds_sync();
    if (active) {
      const uint32_t P = I[t + 1];
      const uint32_t X = I[piv];
      uint8_t* o = ob + 3ull * t;
      o[0] = uint8_t(f ? P : X);
      o[1] = uint8_t(f ? X : P);
      o[2] = uint8_t(N);
    }
  }
  wave_lds_sync();
}

__device__ __forceinline__ uint8_t* wave_index_array(uint8_t* lds, uint32_t wave, uint32_t lane) {
  uint8_t* I = lds + wave * kIdxBytes;
  if (lane < 3) I[lane] = uint8_t(lane);
  return I;
}

// Plain decoder: workgroup b covers waves_per_group * mpw consecutive
// meshlets; wave w of it the w-th run of mpw.  Consecutive workgroups go to
// different XCDs, so tiles are handed out XCD-major: each XCD decodes one
// contiguous stretch of the mesh and its L2 sees whole output lines.
__global__ __launch_bounds__(kWave * kMaxWavesPerGroup) void k_decode_plain(
    const gtsr_meshlet* __restrict__ meshlets, const uint8_t* __restrict__ bits,
    const uint8_t* __restrict__ reuse, uint8_t* __restrict__ out, uint32_t meshlet_count,
    uint64_t chunks, uint64_t reuse_bytes, uint64_t out_tris, uint32_t mpw) {
  extern __shared__ uint8_t lds[];
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = uniform(threadIdx.x / kWave);
  const uint32_t waves = blockDim.x / kWave;
  uint8_t* I = wave_index_array(lds, wave, lane);
  const uint32_t per_xcd = gridDim.x / kXcds;
  const uint32_t tile = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  const uint64_t m0 = (uint64_t(tile) * waves + wave) * mpw;
  const Stream s{meshlets, bits, reuse, out, chunks, reuse_bytes, out_tris};
  for (uint32_t k = 0; k < mpw; ++k) {
    const uint64_t m = m0 + k;
    if (m >= meshlet_count) break;
    decode_meshlet(s, uint32_t(m), I, lane);
  }
}

// Persistent batched decoder: every wavefront takes work items (a run of
// meshlets of one mesh) from a shared counter until none are left.
__global__ __launch_bounds__(kWave * kMaxWavesPerGroup) void k_decode_batched(
    const gtsr_mesh_entry* __restrict__ table, uint32_t mesh_count,
    const gtsr_work_item* __restrict__ work, uint32_t work_items, uint32_t* __restrict__ counter) {
  extern __shared__ uint8_t lds[];
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = uniform(threadIdx.x / kWave);
  uint8_t* I = wave_index_array(lds, wave, lane);
  for (;;) {
    uint32_t item = 0;
    if (lane == 0) item = atomicAdd(counter, 1u);
    item = uniform(item);
    if (item >= work_items) break;
    const uint4 wi = load_uniform16(work + item);
    if (wi.x >= mesh_count) continue;
    const gtsr_mesh_entry* e = table + wi.x;
    const uint4 e0 = load_uniform16(reinterpret_cast<const uint8_t*>(e));
    const uint4 e1 = load_uniform16(reinterpret_cast<const uint8_t*>(e) + 16);
    const uint4 e2 = load_uniform16(reinterpret_cast<const uint8_t*>(e) + 32);
    const uint4 e3 = load_uniform16(reinterpret_cast<const uint8_t*>(e) + 48);
    Stream s;
    s.meshlets = reinterpret_cast<const gtsr_meshlet*>((uint64_t(e0.y) << 32) | e0.x);
    s.bits = reinterpret_cast<const uint8_t*>((uint64_t(e0.w) << 32) | e0.z);
    s.reuse = reinterpret_cast<const uint8_t*>((uint64_t(e1.y) << 32) | e1.x);
    s.out = reinterpret_cast<uint8_t*>((uint64_t(e1.w) << 32) | e1.z);
    const uint32_t mcount = e2.x;
    s.chunks = ((uint64_t(e2.w) << 32) | e2.z) / 16;
    s.reuse_bytes = (uint64_t(e3.y) << 32) | e3.x;
    s.out_tris = (uint64_t(e3.w) << 32) | e3.z;
    const uint32_t end = wi.z < mcount ? wi.z : mcount;
    for (uint32_t m = wi.y; m < end; ++m) decode_meshlet(s, m, I, lane);
  }
}

__global__ void k_fill_zero(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

struct Defaults {
  uint32_t waves = 4, mpw = 4, gpc = 8;
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
  hipLaunchKernelGGL(k_decode_batched, dim3(groups), dim3(kWave * d.waves), d.waves * kIdxBytes, stream,
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
  hipLaunchKernelGGL(k_decode_plain, dim3(uint32_t(groups)), dim3(kWave * d.waves), d.waves * kIdxBytes,
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
