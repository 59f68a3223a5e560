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
// Data movement.  A wavefront decodes a contiguous block of meshlets of one
// mesh, run by run (a run: at most 32 meshlets and Shape::kTris strip
// triangles, contiguous in all three stream arrays and in the output).  Per
// run it loads the descriptors with one vector load, the flag chunks with one
// vector load that brings them into L2 (the decode reads each chunk into
// SGPRs by scalar loads) and the reuse bytes into LDS, decodes every meshlet
// from LDS into an LDS output tile, and writes the run's output span with
// 16-byte stores.  The runs are software-pipelined: while run j is
// decoded, the flag chunks and reuse bytes of run j+1 and the descriptors of
// run j+2 are already in flight.  All global loads and stores are raw buffer
// operations whose inactive lanes carry an out-of-range offset (reads return
// zero, writes are dropped), so every run issues the same instructions and
// waiting for the prefetched loads never waits for the previous run's stores.
//
// Memory safety on corrupted input: a meshlet whose descriptor points outside
// the given sizes, does not continue its predecessor contiguously, or does
// not fit the run's tile ends the run and is skipped; buffer ranges bound
// every global access but the scalar flag loads, which those checks keep
// inside the stream's flag array; every LDS index is bounded by the tile
// sizes whatever the flag bits say.

#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"

namespace gtsr {
namespace {

constexpr uint32_t kWave = 64;
constexpr uint32_t kMaxWavesPerGroup = 16;
constexpr uint32_t kXcds = 8;                // workgroups go round-robin over 8 XCDs
// Grids may hold more groups than stay resident: the dispatcher refills freed
// slots, which keeps every SIMD full until the work runs out (a SIMD issues
// its oldest waves first, so equal static shares finish far apart).
constexpr uint32_t kMaxGroupsPerCu = 1024;
constexpr uint32_t kRunMeshlets = 32;        // meshlets per run (one descriptor per lane)
// LDS per wavefront: 160 KB per CU over 32 resident wavefronts (8 per SIMD).
constexpr uint32_t kTileBudget = 160 * 1024 / 32;

// Run shape per stream format and tile choice.  The tile holds the run's
// output (3 bytes per strip triangle) and its staged reuse bytes.  GTS-Reuse
// needs about half a reuse byte per strip triangle, so its default tile
// (kTile 0) takes longer runs (fewer runs, less per-run work) with a smaller
// stage; kTile 1 is the 1024-triangle run with a 1024-byte stage, which plain
// GTS always uses (one index byte per strip triangle).  A run also ends when
// its reuse bytes outgrow the stage.
template <bool kPlain, uint32_t kTile = 0>
struct Shape {
  static constexpr bool kShort = kPlain || kTile == 1;
  static constexpr uint32_t kTris = kShort ? 1024 : 1280;        // strip triangles per run
  static constexpr uint32_t kStage = kShort ? 1024 : 640;        // reuse / index bytes staged per run
  static constexpr uint32_t kChunks = kTris / 64 + kRunMeshlets; // flag chunks per run (one per lane)
  static constexpr uint32_t kOutBlocks = (3 * kTris + 3 * 64 + 16 + 15) / 16;
};

// One wavefront's LDS tile.
template <bool kPlain, uint32_t kTile = 0>
struct RunTile {
  uint4 out[Shape<kPlain, kTile>::kOutBlocks];          // + a partial chunk past the run, + 16-byte shift
  uint8_t reuse[Shape<kPlain, kTile>::kStage + 64];     // + reads by lanes whose flags say "new"
  uint8_t idx[272];                                     // I[0 .. T_s+1] of the current meshlet
};
template <bool kPlain, uint32_t kTile = 0>
constexpr uint32_t kTileBytes = sizeof(RunTile<kPlain, kTile>);

template <bool kPlain, uint32_t kTile>
constexpr bool shape_fits() {
  using S = Shape<kPlain, kTile>;
  return S::kChunks <= kWave                          // one flag chunk per lane
         && S::kStage % 16 == 0 && S::kStage <= 16 * kWave   // the stage: one 16-byte block per lane at most
         && S::kOutBlocks <= 4 * kWave                // four 16-byte stores per lane cover the output tile
         && 3 * (kWave - 1) + 3 * S::kTris + 18 < 16 * S::kOutBlocks   // dropped compacted lanes stay in the tile
         && S::kStage + 64 <= 2048 && 15 + 3 * (S::kTris - 1) < 4096   // layout word fields
         && kTileBytes<kPlain, kTile> <= kTileBudget;
}
static_assert(shape_fits<false, 0>() && shape_fits<false, 1>() && shape_fits<true, 0>(),
              "run shapes fit the tile, the layout word and the LDS budget");

// The lane builtins return int; these keep every value unsigned (a signed
// value widened into a 64-bit flag word would smear its sign bit upward).
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return uint32_t(__builtin_amdgcn_readfirstlane(v)); }
__device__ __forceinline__ uint32_t lane_value(uint32_t v, uint32_t lane) {
  return uint32_t(__builtin_amdgcn_readlane(v, lane));
}

// Value of the lane below (lane 0 gets 0): DPP wavefront shift right by one.
__device__ __forceinline__ uint32_t from_lane_below(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x138, 0xF, 0xF, false));
}

// Orders this wavefront's LDS writes before its later LDS reads of other
// lanes' values; LDS operations of one wavefront complete in issue order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Raw buffer resources: base + byte range; accesses at offsets past the range
// read zero / write nothing.
constexpr int kRsrcWord3 = 0x00020000;
constexpr uint32_t kOutOfRange = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), kRsrcWord3);
}

__device__ __forceinline__ uint4 load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, int(off), 0, 0));
  return make_uint4(v.x, v.y, v.z, v.w);
}

// Cache policy of the output stores: non-temporal (the nt bit of gfx950's
// cache-policy field).  The kernel writes its output once and never reads it,
// so the stores should not displace from L2 the flag chunks that each run
// prefetches for the scalar loads of its decode.
constexpr int kOutputPolicy = 2;

__device__ __forceinline__ void store16(__amdgpu_buffer_rsrc_t r, uint32_t off, const uint4& w) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = {w.x, w.y, w.z, w.w};
  __builtin_amdgcn_raw_buffer_store_b128(v, r, int(off), 0, kOutputPolicy);
}

// One mesh's stream.  GTS-Reuse: `bits` holds 16-byte chunks {LR, INC},
// `reuse` the reuse bytes.  Plain GTS: `bits` holds one 8-byte L/R word per
// chunk, `reuse` one index byte per strip triangle after the first.  With a
// compacted output, `kept` holds the M + 1 per-meshlet offsets among the
// non-degenerate triangles and `out_tris` counts output triangles of that
// output.  With culling, `cones` holds a float4 {axis, cutoff} per meshlet and
// `view` the view direction.
struct Stream {
  const uint8_t* meshlets;
  const uint8_t* bits;
  const uint8_t* reuse;
  uint8_t* out;
  const uint32_t* kept;
  uint32_t chunks;        // the array sizes, clipped to 32 bits (offsets are 32-bit)
  uint32_t reuse_bytes;
  uint32_t out_tris;
  uint32_t meshlet_count;
  const float* cones = nullptr;
  float view[3] = {0.0f, 0.0f, 0.0f};
};

__device__ __forceinline__ uint32_t clip32(uint64_t v) { return v > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(v); }

// ---------------------------------------------------------------- one meshlet

// Flag words of one chunk, wave-uniform (SGPRs).
struct Flags {
  uint64_t lr, inc;
};

// Chunk idx of a run whose first flag chunk is at g, fetched by scalar loads
// straight into SGPRs (the constant address space marks the words uniform and
// unchanged during the kernel).  A scalar load is not bounds-checked: every
// chunk read lies inside the range the run's plan validated against the
// stream's size.  The run loop has already pulled the run's chunks into L2
// with one vector load, so these hit the cache; fetching them this way
// instead of moving them out of that load's VGPRs with v_readlane saves four
// VALU instructions per chunk.
typedef __attribute__((address_space(4))) const unsigned long long ConstU64;
template <bool kPlain>
__device__ __forceinline__ Flags chunk_flags(const uint8_t* g, uint32_t idx) {
  if constexpr (kPlain) {
    ConstU64* q = (ConstU64*)(g + 8ull * idx);
    return Flags{q[0], 0ull};
  }
  ConstU64* q = (ConstU64*)(g + 16ull * idx);
  return Flags{q[0], q[1]};
}

// Per-lane LDS pointers, fixed for the kernel.
struct LanePtrs {
  const uint8_t* reuse;   // tile.reuse + lane
  uint8_t* idx;           // tile.idx + lane
  uint8_t* out;           // tile.out + 3 * lane
  uint32_t lane0;         // 1 in lane 0, else 0
};

// Phase 1 for chunk C: the new slot I[t+2] -- the next vertex number, or the
// reuse byte whose rank is the number of reuse slots before t (lanes below
// minus increments below).  inc_base: 2 + increments before this chunk,
// triangle 0 counted as introducing vertex 2; reuse_pos: reuse slots before
// this chunk plus the meshlet's tile offset.
//
// Plain GTS stores that slot directly: index byte t - 1 of the meshlet (its
// tile offset is reuse_pos), triangle 0's slot being the implicit 2.
template <bool kPlain, uint32_t C>
__device__ __forceinline__ uint32_t new_index(const LanePtrs& lp, const Flags& f, uint32_t& inc_base,
                                              uint32_t& reuse_pos, uint32_t lane) {
  if constexpr (kPlain) {
    const uint32_t b = lp.reuse[reuse_pos + 64 * C - 1];   // lane 0 of chunk 0 reads a byte it ignores
    return (C == 0 && lane == 0) ? 2u : b;
  }
  const uint64_t inc = C == 0 ? (f.inc | 1) : f.inc;
  uint32_t fresh, r;
  if constexpr (C == 0) {
    // inc_base is the constant 2 here: mbcnt adds it, and the reuse rank
    // follows from the sum (reuse_pos + 2 - fresh = reuse_pos - ones)
    fresh = __builtin_amdgcn_mbcnt_hi(uint32_t(inc >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(inc), 2u));
    r = lp.reuse[reuse_pos + 2 - fresh];
  } else {
    const uint32_t ones = __builtin_amdgcn_mbcnt_hi(uint32_t(inc >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(inc), 0u));
    fresh = ones + inc_base;
    r = lp.reuse[reuse_pos - ones];
  }
  const uint32_t N = __builtin_amdgcn_inverse_ballot_w64(inc) ? fresh : r;
  const uint32_t news = uint32_t(__builtin_popcountll(inc));
  inc_base += news;
  reuse_pos += 64 - news;
  return N;
}

// Phase 2, reads: I[t+1] and the pivot.
struct Pivot {
  uint32_t P, X;
};
template <uint32_t C>
__device__ __forceinline__ Pivot pivot_of(const LanePtrs& lp, const uint8_t* idx0, const Flags& f, uint32_t N,
                                          uint32_t lane, uint32_t& last_change, uint64_t& prev_top) {
  uint64_t ch = f.lr ^ ((f.lr << 1) | prev_top);
  if (C == 0) ch |= 1;
  const uint64_t upto = ch << (63 - lane);
  const uint8_t* at_t = lp.idx + 64 * C;                  // &I[t]
  const uint8_t* px = at_t - __builtin_clzll(upto);       // &I[last flip <= t] when upto != 0
  if (C != 0 && !upto) px = idx0 + last_change;
  if (C == 0 || ch) last_change = 64 * C + 63 - uint32_t(__builtin_clzll(ch));   // else: no flip in this chunk
  prev_top = f.lr >> 63;
  // I[t+1]: the new slot of the lane below.  In a meshlet's first chunk lane 0
  // takes I[1] = 1, so a DPP shift (lane 0 gets 0, plus lane0) replaces the
  // LDS read; later chunks read the slot their lane 0 needs from the chunk
  // before.
  const uint32_t P =
      C == 0 ? uint32_t(__builtin_amdgcn_update_dpp(0, int(N), 0x138, 0xF, 0xF, true)) + lp.lane0 : at_t[1];
  return Pivot{P, *px};
}

// Phase 2, writes: the oriented triple at out_m + 3t.
//
// Compacted output: only the lanes whose triple names three different
// vertices (every triangle but the four degenerates of each restart) and
// that lie inside the meshlet write, packed in order from kept_pos; the
// others write to the tile's spare bytes past the longest shifted run.
template <uint32_t C, bool kCompact, bool kPlain, uint32_t kTile>
__device__ __forceinline__ void put_triangle(const LanePtrs& lp, uint8_t* out_m, const Flags& f, uint32_t N,
                                             const Pivot& pv, uint32_t lane, uint32_t T, uint32_t& kept_pos) {
  const uint32_t P = pv.P, X = pv.X;
  const bool right = __builtin_amdgcn_inverse_ballot_w64(f.lr);
  uint8_t* o;
  if constexpr (kCompact) {
    const bool keep = 64 * C + lane < T && X != P && P != N && X != N;
    const uint64_t km = __builtin_amdgcn_ballot_w64(keep);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(uint32_t(km >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(km), 0u));
    o = keep ? out_m + 3 * (kept_pos + below) : lp.out + 3 * Shape<kPlain, kTile>::kTris + 16;   // past any shifted run
    kept_pos += uint32_t(__builtin_popcountll(km));
  } else {
    o = out_m + 192 * C;
  }
  o[0] = uint8_t(right ? P : X);
  o[1] = uint8_t(right ? X : P);
  o[2] = uint8_t(N);
}

// Phase 2 for chunk C: the pivot (the last L/R flip at or before t; in chunk 0
// the change word gets bit 0 set, so "no flip so far" lands on position 0,
// whose vertex I[0] is the right pivot) and the oriented triple.
template <uint32_t C, bool kCompact, bool kPlain, uint32_t kTile>
__device__ __forceinline__ void emit_triangle(const LanePtrs& lp, const uint8_t* idx0, uint8_t* out_m,
                                              const Flags& f, uint32_t N, uint32_t lane, uint32_t& last_change,
                                              uint64_t& prev_top, uint32_t T, uint32_t& kept_pos) {
  const Pivot pv = pivot_of<C>(lp, idx0, f, N, lane, last_change, prev_top);
  put_triangle<C, kCompact, kPlain, kTile>(lp, out_m, f, N, pv, lane, T, kept_pos);
}

// Decodes one meshlet of NCH flag chunks (chunks co.. of the run at gb), reuse bytes
// at tile.reuse[ro], output at tile byte ob.  Phase 1 writes the index slots
// of all chunks, phase 2 reads them back, so each meshlet waits for LDS twice
// whatever its size.  Lanes past T_s compute garbage that lands past the
// meshlet's output (the next meshlet overwrites it, or it lies past the run
// and is never stored).
//
// Compacted output: ob addresses the meshlet's first kept triangle and T
// (its strip triangles) bounds the lanes that may write.
template <uint32_t NCH, bool kPlain, bool kCompact, uint32_t kTile>
__device__ __forceinline__ void decode_meshlet(RunTile<kPlain, kTile>& tile, const LanePtrs& lp, const uint8_t* gb, uint32_t co,
                                               uint32_t ro, uint32_t ob, uint32_t lane, uint32_t T) {
  Flags f0 = chunk_flags<kPlain>(gb, co), f1{0, 0}, f2{0, 0}, f3{0, 0};
  if constexpr (NCH > 1) f1 = chunk_flags<kPlain>(gb, co + 1);
  if constexpr (NCH > 2) f2 = chunk_flags<kPlain>(gb, co + 2);
  if constexpr (NCH > 3) f3 = chunk_flags<kPlain>(gb, co + 3);
  uint32_t inc_base = 2, reuse_pos = ro;
  const uint32_t n0 = new_index<kPlain, 0>(lp, f0, inc_base, reuse_pos, lane);
  uint32_t n1 = 0, n2 = 0, n3 = 0;
  if constexpr (NCH > 1) n1 = new_index<kPlain, 1>(lp, f1, inc_base, reuse_pos, lane);
  if constexpr (NCH > 2) n2 = new_index<kPlain, 2>(lp, f2, inc_base, reuse_pos, lane);
  if constexpr (NCH > 3) n3 = new_index<kPlain, 3>(lp, f3, inc_base, reuse_pos, lane);
  lp.idx[2] = uint8_t(n0);
  if constexpr (NCH > 1) lp.idx[66] = uint8_t(n1);
  if constexpr (NCH > 2) lp.idx[130] = uint8_t(n2);
  if constexpr (NCH > 3) lp.idx[194] = uint8_t(n3);
  wave_lds_sync();
  // lane-relative output (lp.out = tile + 3 * lane), or the tile base when compacting
  uint8_t* out_m = kCompact ? reinterpret_cast<uint8_t*>(tile.out) + ob : lp.out + ob;
  uint32_t last_change = 0, kept_pos = 0;
  uint64_t prev_top = 0;
  emit_triangle<0, kCompact, kPlain, kTile>(lp, tile.idx, out_m, f0, n0, lane, last_change, prev_top, T, kept_pos);
  if constexpr (NCH > 1) emit_triangle<1, kCompact, kPlain, kTile>(lp, tile.idx, out_m, f1, n1, lane, last_change, prev_top, T, kept_pos);
  if constexpr (NCH > 2) emit_triangle<2, kCompact, kPlain, kTile>(lp, tile.idx, out_m, f2, n2, lane, last_change, prev_top, T, kept_pos);
  if constexpr (NCH > 3) emit_triangle<3, kCompact, kPlain, kTile>(lp, tile.idx, out_m, f3, n3, lane, last_change, prev_top, T, kept_pos);
  wave_lds_sync();
}

// Index slots of the second meshlet of a pair start this far up the index
// area: past the 130 slots a two-chunk meshlet uses, and with room for its
// own 130 below the area's end.
constexpr uint32_t kPairIdx = 136;

// Two meshlets of NCH (1 or 2) chunks decoded together, so that the LDS and
// scalar-load waits of one overlap the work of the other: the reads of both
// phases are issued for both meshlets before either's writes.  a's chunks
// start at run chunk co, b's at co + NCH; wa, wb: their layout words.  b's
// index slots start kPairIdx bytes up, where the caller has set I[0] = 0 and
// I[1] = 1.  a's triples are written before b's, so b overwrites the garbage
// of a's lanes past its T_s.
template <uint32_t NCH, bool kPlain, bool kCompact, uint32_t kTile>
__device__ __forceinline__ void decode_pair(RunTile<kPlain, kTile>& tile, const LanePtrs& lp, const uint8_t* gb, uint32_t co,
                                            uint32_t wa, uint32_t wb, uint32_t lane, uint32_t Ta, uint32_t Tb) {
  static_assert(NCH == 1 || NCH == 2, "pairs of one- or two-chunk meshlets");
  static_assert(kPairIdx >= 64 * NCH + 2 && kPairIdx + 64 * NCH + 2 <= sizeof(RunTile<kPlain, kTile>::idx), "index area");
  LanePtrs lq = lp;
  lq.idx += kPairIdx;
  const Flags fa0 = chunk_flags<kPlain>(gb, co), fb0 = chunk_flags<kPlain>(gb, co + NCH);
  Flags fa1{0, 0}, fb1{0, 0};
  if constexpr (NCH > 1) {
    fa1 = chunk_flags<kPlain>(gb, co + 1);
    fb1 = chunk_flags<kPlain>(gb, co + 3);
  }
  uint32_t ia = 2, ib = 2, ra = (wa >> 6) & 2047u, rb = (wb >> 6) & 2047u;
  const uint32_t na0 = new_index<kPlain, 0>(lp, fa0, ia, ra, lane);
  const uint32_t nb0 = new_index<kPlain, 0>(lq, fb0, ib, rb, lane);
  uint32_t na1 = 0, nb1 = 0;
  if constexpr (NCH > 1) {
    na1 = new_index<kPlain, 1>(lp, fa1, ia, ra, lane);
    nb1 = new_index<kPlain, 1>(lq, fb1, ib, rb, lane);
  }
  lp.idx[2] = uint8_t(na0);
  lq.idx[2] = uint8_t(nb0);
  if constexpr (NCH > 1) {
    lp.idx[66] = uint8_t(na1);
    lq.idx[66] = uint8_t(nb1);
  }
  wave_lds_sync();
  uint32_t lca = 0, lcb = 0, ka = 0, kb = 0;
  uint64_t pta = 0, ptb = 0;
  const Pivot pa0 = pivot_of<0>(lp, tile.idx, fa0, na0, lane, lca, pta);
  const Pivot pb0 = pivot_of<0>(lq, tile.idx + kPairIdx, fb0, nb0, lane, lcb, ptb);
  Pivot pa1{0, 0}, pb1{0, 0};
  if constexpr (NCH > 1) {
    pa1 = pivot_of<1>(lp, tile.idx, fa1, na1, lane, lca, pta);
    pb1 = pivot_of<1>(lq, tile.idx + kPairIdx, fb1, nb1, lane, lcb, ptb);
  }
  uint8_t* const base = kCompact ? reinterpret_cast<uint8_t*>(tile.out) : lp.out;
  uint8_t* const out_a = base + ((wa >> 17) & 4095u);
  uint8_t* const out_b = base + ((wb >> 17) & 4095u);
  put_triangle<0, kCompact, kPlain, kTile>(lp, out_a, fa0, na0, pa0, lane, Ta, ka);
  if constexpr (NCH > 1) put_triangle<1, kCompact, kPlain, kTile>(lp, out_a, fa1, na1, pa1, lane, Ta, ka);
  put_triangle<0, kCompact, kPlain, kTile>(lp, out_b, fb0, nb0, pb0, lane, Tb, kb);
  if constexpr (NCH > 1) put_triangle<1, kCompact, kPlain, kTile>(lp, out_b, fb1, nb1, pb1, lane, Tb, kb);
  wave_lds_sync();
}

// --------------------------------------------------------------------- runs

// A run: the first k meshlets of a descriptor batch (k = 0: the batch's first
// meshlet is unusable and is skipped).  All fields wave-uniform.
struct Plan {
  uint32_t k;
  uint32_t c0, r0, o0;    // first flag chunk, reuse byte, output triangle
  uint32_t nch;           // flag chunks
  uint32_t ra, nrb;       // reuse staging start (16-byte aligned) and 16-byte blocks
  uint32_t tris;          // output triangles (strip triangles, or kept ones when compacting)
  uint32_t shift;         // output start modulo 16 bytes: the tile byte of the first triangle
  uint32_t same_nch;      // the chunk count shared by all k meshlets, else 0
};

// Per-lane layout of meshlet `lane` in the run's tile, one word:
// bits 0..5 first flag chunk, 6..16 reuse offset, 17..28 output byte offset
// in the tile (shift + 3 * output triangle offset, < 4096), 29..30 chunk
// count - 1.
__device__ __forceinline__ uint32_t pack_layout(uint32_t co, uint32_t ro, uint32_t ob, uint32_t nch) {
  return co | (ro << 6) | (ob << 17) | ((nch - 1) << 29);
}

// Descriptors of meshlets [m, min(m + 32, m_end)), one per lane (zero past).
__device__ __forceinline__ uint4 load_descriptors(const Stream& s, uint32_t m, uint32_t m_end, uint32_t lane) {
  const uint32_t cnt = m < m_end ? min(m_end - m, kRunMeshlets) : 0u;
  return load16(buffer(s.meshlets + 16ull * m, 16 * cnt), 16 * lane);
}

// Kept offsets of the same meshlets and of the one after each (compacted
// output): lane i gets kept[m + i] and kept[m + i + 1]; m_end <= M, so both
// stay inside the M + 1 entries.
__device__ __forceinline__ uint2 load_kept(const Stream& s, uint32_t m, uint32_t m_end, uint32_t lane) {
  const uint32_t cnt = m < m_end ? min(m_end - m, kRunMeshlets) : 0u;
  const __amdgpu_buffer_rsrc_t r = buffer(s.kept + m, 4 * (cnt + (cnt ? 1 : 0)));
  const uint32_t a = uint32_t(__builtin_amdgcn_raw_buffer_load_b32(r, int(4 * lane), 0, 0));
  const uint32_t b = uint32_t(__builtin_amdgcn_raw_buffer_load_b32(r, int(4 * lane + 4), 0, 0));
  return make_uint2(a, b);
}

// Validates the descriptors (and kept offsets kd) and takes the leading run of
// usable meshlets.  layout: the per-lane word above; with a compacted output
// its output field is the kept offset inside the run, and o0 names the run's
// first kept triangle.
//
// Culling: a meshlet whose normal cone faces away from the view direction
// (dot(axis, view) > cutoff, in this float32 order) is not usable either,
// so it is skipped and its output left untouched.
template <bool kPlain, bool kCompact, bool kCull, uint32_t kTile>
__device__ __forceinline__ Plan make_plan(const Stream& s, const uint4& d, const uint2& kd, uint32_t m,
                                          uint32_t m_end, uint32_t lane, uint32_t& layout,
                                          const uint4& cone = make_uint4(0, 0, 0, 0)) {
  const uint32_t cnt = m < m_end ? min(m_end - m, kRunMeshlets) : 0u;
  const uint32_t T = d.w & 0xFFFFu, V = d.w >> 16;
  const uint32_t nch = (T + 63) >> 6;
  const uint32_t nru = kPlain ? T - 1 : T + 2 - V;   // reuse bytes, or index bytes
  Plan p;
  p.c0 = uniform(d.x);
  p.r0 = uniform(d.y);
  p.o0 = uniform(d.z);
  p.ra = p.r0 & ~15u;
  // Every test below is evaluated whatever the others give (bitwise &, no
  // short circuit), so the checks stay straight-line mask arithmetic.
  // Counts in range (V >= 3 and V <= T + 2 as one unsigned compare, T >= 1),
  // arrays not overrun (overflow-free forms):
  bool ok = (lane < cnt) & (T - 1u < kMaxStripTris) & (V - 3u <= T - 1u) & (V <= 256);
  ok &= (d.x <= s.chunks) & (nch <= s.chunks - d.x) & (d.y <= s.reuse_bytes) & (nru <= s.reuse_bytes - d.y);
  // contiguous with the meshlet before it (lane 0 starts the run)
  const uint32_t ex = d.x + nch, ey = d.y + nru, ez = d.z + T;
  const uint32_t px = from_lane_below(ex), py = from_lane_below(ey), pz = from_lane_below(ez);
  ok &= (lane == 0) | ((d.x == px) & (d.y == py) & (d.z == pz));
  // the run still fits the tile
  using S = Shape<kPlain, kTile>;
  ok &= (ex - p.c0 <= S::kChunks) & (ey - p.ra <= S::kStage) & (ez - p.o0 <= S::kTris);
  uint32_t ot = d.z - p.o0;
  if constexpr (kCull) {
    const float ax = __uint_as_float(cone.x), ay = __uint_as_float(cone.y), az = __uint_as_float(cone.z);
    const float dot = __builtin_fmaf(az, s.view[2], __builtin_fmaf(ay, s.view[1], ax * s.view[0]));
    ok &= !(dot > __uint_as_float(cone.w));
  }
  if constexpr (kCompact) {
    // kept triangles: no more than the strip triangles, so kept positions stay
    // at or before the strip positions inside the tile; the output holds them
    const uint32_t kf = uniform(kd.x);
    ok &= (kd.y >= kd.x) & (kd.y - kd.x <= T) & (kd.x - kf <= d.z - p.o0) & (kd.y <= s.out_tris);
    ot = kd.x - kf;
    p.o0 = kf;
  } else {
    ok &= (d.z <= s.out_tris) & (T <= s.out_tris - d.z);
  }
  const uint64_t okm = __builtin_amdgcn_ballot_w64(ok);
  p.k = uint32_t(__builtin_ctzll(~okm));   // leading run of usable meshlets (okm has no bit past lane 31)
  p.shift = uint32_t(reinterpret_cast<uintptr_t>(s.out) + 3 * p.o0) & 15u;
  layout = pack_layout(d.x - p.c0, d.y - p.ra, p.shift + 3 * ot, nch);
  const uint32_t nch0 = uniform(nch);
  p.same_nch = p.k && !__builtin_amdgcn_ballot_w64((lane < p.k) & (nch != nch0)) ? nch0 : 0u;
  if (p.k) {
    p.nch = lane_value(ex, p.k - 1) - p.c0;
    p.nrb = (lane_value(ey, p.k - 1) - p.ra + 15) >> 4;
    p.tris = (kCompact ? lane_value(kd.y, p.k - 1) : lane_value(ez, p.k - 1)) - p.o0;
  } else {
    p.nch = p.nrb = p.tris = 0;
  }
  return p;
}

// The run's flag chunks, one per lane (GTS-Reuse: 16-byte chunks; plain GTS:
// 8-byte L/R words).  Issued one run ahead, this load brings them into L2
// for the scalar loads of the decode.
template <bool kPlain>
__device__ __forceinline__ uint4 load_bits(const Stream& s, const Plan& p, uint32_t lane) {
  if constexpr (kPlain) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 v = __builtin_bit_cast(
        u32x2, __builtin_amdgcn_raw_buffer_load_b64(buffer(s.bits + 8ull * p.c0, 8 * p.nch), int(8 * lane), 0, 0));
    return make_uint4(v.x, v.y, 0, 0);
  }
  // one dword per 16-byte chunk brings its cache line in and keeps three
  // VGPRs per pipeline stage free
  const uint32_t w = uint32_t(__builtin_amdgcn_raw_buffer_load_b32(buffer(s.bits + 16ull * p.c0, 16 * p.nch),
                                                                   int(16 * lane), 0, 0));
  return make_uint4(w, 0, 0, 0);
}

// The reuse allocation extends to a multiple of 16 bytes, so whole blocks can
// be read up to the block holding the run's last reuse byte.
__device__ __forceinline__ uint4 load_reuse(const Stream& s, const Plan& p, uint32_t lane) {
  return load16(buffer(s.reuse + p.ra, 16 * p.nrb), 16 * lane);
}

// A run whose k meshlets all have NCH chunks: meshlet i's chunks start at
// chunk NCH * i of the run, and no meshlet needs a size dispatch.  Meshlets
// of up to kPairMaxChunks chunks are decoded in pairs (a run's odd last one
// alone).
constexpr uint32_t kPairMaxChunks = 2;
template <uint32_t NCH, bool kPlain, bool kCompact, uint32_t kTile>
__device__ __forceinline__ void decode_run_same(RunTile<kPlain, kTile>& tile, const LanePtrs& lp, uint32_t k, uint32_t layout,
                                                uint32_t tri_counts, const uint8_t* gb, uint32_t lane) {
  if constexpr (NCH <= kPairMaxChunks) {
    if (lane < 2) tile.idx[kPairIdx + lane] = uint8_t(lane);
    uint32_t i = 0;
    for (; i + 1 < k; i += 2) {
      const uint32_t wa = lane_value(layout, i), wb = lane_value(layout, i + 1);
      const uint32_t Ta = kCompact ? lane_value(tri_counts, i) : 0u;
      const uint32_t Tb = kCompact ? lane_value(tri_counts, i + 1) : 0u;
      decode_pair<NCH, kPlain, kCompact, kTile>(tile, lp, gb, NCH * i, wa, wb, lane, Ta, Tb);
    }
    if (i < k) {
      const uint32_t w = lane_value(layout, i);
      const uint32_t T = kCompact ? lane_value(tri_counts, i) : 0u;
      decode_meshlet<NCH, kPlain, kCompact, kTile>(tile, lp, gb, NCH * i, (w >> 6) & 2047u, (w >> 17) & 4095u, lane, T);
    }
    return;
  }
  for (uint32_t i = 0; i < k; ++i) {
    const uint32_t w = lane_value(layout, i);
    const uint32_t T = kCompact ? lane_value(tri_counts, i) : 0u;
    decode_meshlet<NCH, kPlain, kCompact, kTile>(tile, lp, gb, NCH * i, (w >> 6) & 2047u, (w >> 17) & 4095u, lane, T);
  }
}

// Decodes the run's meshlets from the tile.  gb: the run's first flag chunk
// in global memory; tri_counts: lane i holds meshlet i's T_s (read only when
// compacting).  Runs of one chunk count (most runs:
// a mesh's meshlets mostly share one size class) take a loop specialised to
// it; the others dispatch per meshlet.
template <bool kPlain, bool kCompact, uint32_t kTile>
__device__ __forceinline__ void decode_run(RunTile<kPlain, kTile>& tile, const LanePtrs& lp, const Plan& p, uint32_t layout,
                                           uint32_t tri_counts, const uint8_t* gb, uint32_t lane) {
  if (p.same_nch == 1) return decode_run_same<1, kPlain, kCompact, kTile>(tile, lp, p.k, layout, tri_counts, gb, lane);
  if (p.same_nch == 2) return decode_run_same<2, kPlain, kCompact, kTile>(tile, lp, p.k, layout, tri_counts, gb, lane);
  if (p.same_nch == 4) return decode_run_same<4, kPlain, kCompact, kTile>(tile, lp, p.k, layout, tri_counts, gb, lane);
  for (uint32_t i = 0; i < p.k; ++i) {
    const uint32_t w = lane_value(layout, i);
    const uint32_t co = w & 63u, ro = (w >> 6) & 2047u, ob = (w >> 17) & 4095u;
    const uint32_t nch = (w >> 29) + 1;
    const uint32_t T = kCompact ? lane_value(tri_counts, i) : 0u;
    if (nch > 2) {
      if (nch > 3) decode_meshlet<4, kPlain, kCompact, kTile>(tile, lp, gb, co, ro, ob, lane, T);
      else decode_meshlet<3, kPlain, kCompact, kTile>(tile, lp, gb, co, ro, ob, lane, T);
    } else {
      if (nch > 1) decode_meshlet<2, kPlain, kCompact, kTile>(tile, lp, gb, co, ro, ob, lane, T);
      else decode_meshlet<1, kPlain, kCompact, kTile>(tile, lp, gb, co, ro, ob, lane, T);
    }
  }
}

// Writes the run's tile bytes [shift, shift + 3 * tris) to dst .. dst + 3 *
// tris (shift = dst mod 16): the 16-byte blocks inside the span with four
// stores per lane, then the ragged bytes at the two ends (at most 15 each)
// with one byte store per lane.
template <bool kPlain, uint32_t kTile>
__device__ __forceinline__ void store_run(uint8_t* dst, uint32_t shift, uint32_t tris, const RunTile<kPlain, kTile>& tile,
                                          uint32_t lane) {
  uint8_t* base = dst - shift;                      // 16-byte aligned, tile byte 0
  const uint32_t end = shift + 3 * tris;
  const uint32_t full0 = (shift + 15) >> 4;         // first block inside the span
  const uint32_t full1 = end >> 4;                  // one past the last block inside
  const __amdgpu_buffer_rsrc_t blocks = buffer(base, 16 * full1);
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    const uint32_t j = full0 + lane + kWave * q;
    constexpr uint32_t kOutBlocks = Shape<kPlain, kTile>::kOutBlocks;
    const uint32_t jt = j < kOutBlocks ? j : kOutBlocks - 1;
    store16(blocks, 16 * j, tile.out[jt]);   // blocks at or past full1 lie outside `blocks`: dropped
  }
  const uint32_t head_end = min(16 * full0, end);
  const uint32_t head = head_end - shift;
  const uint32_t tail_start = max(16 * full1, head_end);
  const uint32_t tail = end - tail_start;
  const uint32_t pos = lane < head ? shift + lane : tail_start + (lane - head);
  const uint32_t byte = reinterpret_cast<const uint8_t*>(tile.out)[pos < sizeof(tile.out) ? pos : 0];
  __builtin_amdgcn_raw_buffer_store_b8(uint8_t(byte), buffer(base, end), int(lane < head + tail ? pos : kOutOfRange),
                                       0, kOutputPolicy);
}

// As many stores as store_run issues (five), all out of range: they write
// nothing.  Issued after the prologue's loads so that both ways into the run
// loop have five stores after the prefetched loads, which lets the compiler
// wait for those loads alone.  Their data is a register already live (v):
// constant store data costs registers the decode needs.
__device__ __forceinline__ void store_nothing(uint8_t* any, uint32_t v) {
  const __amdgpu_buffer_rsrc_t none = buffer(any, 0);
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q)
    __builtin_amdgcn_raw_buffer_store_b32(v, none, int(kOutOfRange + 16 * q), 0, kOutputPolicy);
  __builtin_amdgcn_raw_buffer_store_b8(uint8_t(v), none, int(kOutOfRange), 0, kOutputPolicy);
}

// Cones of meshlets [m, min(m + 32, m_end)), one float4 per lane (culling).
__device__ __forceinline__ uint4 load_cones(const Stream& s, uint32_t m, uint32_t m_end, uint32_t lane) {
  const uint32_t cnt = m < m_end ? min(m_end - m, kRunMeshlets) : 0u;
  return load16(buffer(s.cones + 4ull * m, 16 * cnt), 16 * lane);
}

// Decodes meshlets [m, m_end) of stream s with the calling wavefront.
template <bool kPlain, bool kCompact, bool kCull, uint32_t kTile>
__device__ __forceinline__ void decode_range(const Stream& s, uint32_t m, uint32_t m_end, RunTile<kPlain, kTile>& tile,
                                             const LanePtrs& lp, uint32_t lane) {
  if (m >= m_end) return;
  const uint4 zero4 = make_uint4(0, 0, 0, 0);
  uint4 d = load_descriptors(s, m, m_end, lane);
  uint2 kd = kCompact ? load_kept(s, m, m_end, lane) : make_uint2(0, 0);
  uint4 cd = kCull ? load_cones(s, m, m_end, lane) : zero4;
  uint32_t layout;
  Plan p = make_plan<kPlain, kCompact, kCull, kTile>(s, d, kd, m, m_end, lane, layout, cd);
  uint32_t mn = m + (p.k ? p.k : 1);
  uint4 dn = load_descriptors(s, mn, m_end, lane);
  uint2 kdn = kCompact ? load_kept(s, mn, m_end, lane) : make_uint2(0, 0);
  uint4 cdn = kCull ? load_cones(s, mn, m_end, lane) : zero4;
  uint4 bv = load_bits<kPlain>(s, p, lane);
  uint4 rv = load_reuse(s, p, lane);
  store_nothing(s.out, lane);
  for (;;) {
    // the tile is free: stage this run's reuse bytes
    if (lane < Shape<kPlain, kTile>::kStage / 16) reinterpret_cast<uint4*>(tile.reuse)[lane] = rv;
    // plan the next run, if the range has one, and start its loads; they
    // overlap this run's decode
    const bool last = mn >= m_end;
    uint32_t layout_n = 0, mnn = mn;
    Plan pn = {};
    uint4 dnn = zero4, cdnn = zero4, bvn = zero4, rvn = zero4;
    uint2 kdnn = make_uint2(0, 0);
    if (!last) {
      pn = make_plan<kPlain, kCompact, kCull, kTile>(s, dn, kdn, mn, m_end, lane, layout_n, cdn);
      mnn = mn + (pn.k ? pn.k : 1);
      dnn = load_descriptors(s, mnn, m_end, lane);
      kdnn = kCompact ? load_kept(s, mnn, m_end, lane) : make_uint2(0, 0);
      cdnn = kCull ? load_cones(s, mnn, m_end, lane) : zero4;
      bvn = load_bits<kPlain>(s, pn, lane);
      rvn = load_reuse(s, pn, lane);
    }
    const uint32_t tri_counts = d.w & 0xFFFFu;
    wave_lds_sync();
    // the run's flag chunks have arrived in L2 (their values are not used:
    // the decode reads them again by scalar loads)
    if constexpr (kPlain)
      asm volatile("" ::"v"(bv.x), "v"(bv.y));
    else
      asm volatile("" ::"v"(bv.x));
    decode_run<kPlain, kCompact, kTile>(tile, lp, p, layout, tri_counts, s.bits + (kPlain ? 8ull : 16ull) * p.c0, lane);
    store_run<kPlain, kTile>(s.out + 3ull * p.o0, p.shift, p.tris, tile, lane);
    wave_lds_sync();
    if (last) break;
    p = pn;
    layout = layout_n;
    d = dn;
    dn = dnn;
    kdn = kdnn;
    cdn = cdnn;
    bv = bvn;
    rv = rvn;
    mn = mnn;
  }
}

template <bool kPlain, uint32_t kTile>
__device__ __forceinline__ RunTile<kPlain, kTile>& wave_tile(uint32_t wave, uint32_t lane, LanePtrs& lp) {
  extern __shared__ uint4 lds_tiles[];
  RunTile<kPlain, kTile>& tile = reinterpret_cast<RunTile<kPlain, kTile>*>(lds_tiles)[wave];
  if (lane < 3) tile.idx[lane] = uint8_t(lane);
  lp.reuse = tile.reuse + lane;
  lp.idx = tile.idx + lane;
  lp.out = reinterpret_cast<uint8_t*>(tile.out) + 3 * lane;
  lp.lane0 = lane == 0 ? 1u : 0u;
  return tile;
}

// Splits [0, n) into one contiguous block per wavefront of the grid, XCD-major:
// workgroups are dispatched round-robin over the 8 XCDs, so the blocks of one
// XCD's waves are adjacent and its L2 sees whole output lines.
__device__ __forceinline__ void wave_block(uint32_t n, uint32_t wave, uint32_t waves, uint32_t& b0, uint32_t& b1) {
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint32_t wx = gridDim.x / kXcds * waves;            // waves of this XCD (the grid is a multiple of 8)
  const uint32_t q = blockIdx.x / kXcds * waves + wave;     // this wave's rank among them
  const uint32_t x0 = uint32_t(uint64_t(n) * xcd / kXcds), x1 = uint32_t(uint64_t(n) * (xcd + 1) / kXcds);
  // equal shares, one more for the first (x1 - x0) mod wx waves: one 32-bit
  // division (two 64-bit ones cost every wave of the grid ~230 scalar
  // instructions); q < wx, so the clamps only guard
  const uint32_t len = x1 - x0, share = len / wx, extra = len % wx;
  b0 = min(x0 + q * share + min(q, extra), x1);
  b1 = min(b0 + share + (q < extra ? 1u : 0u), x1);
}

// The batched decoder deals the work list to the XCDs in stripes of
// kStripe items, round-robin (stripe j to XCD j mod 8), and splits each XCD's
// stripes evenly over its wavefronts.  A list in mesh order mixes meshes of
// different cost per item; an eighth of it per XCD left the XCDs finishing up
// to 24 us apart in a 0.55 ms launch, while stripes give each XCD the same
// mix.  256-item stripes keep each wavefront's block inside one stripe almost
// always (blocks are a few items), so consecutive items of a mesh still merge.
constexpr uint32_t kStripe = 256;

// Work items of XCD x: stripes x, x + 8, ... (the list's last stripe may be partial).
__device__ __forceinline__ uint32_t xcd_items(uint32_t n, uint32_t xcd) {
  const uint32_t F = n / kStripe, rem = n % kStripe;
  const uint32_t full = F > xcd ? (F - 1 - xcd) / kXcds + 1 : 0u;
  return full * kStripe + (F % kXcds == xcd ? rem : 0u);
}

// The v-th work item of XCD x (v < xcd_items(n, x), so the result is < n).
__device__ __forceinline__ uint32_t xcd_item(uint32_t v, uint32_t xcd) {
  return ((v / kStripe) * kXcds + xcd) * kStripe + v % kStripe;
}

// This wavefront's block [b0, b1) of its XCD's items (indices for xcd_item):
// equal shares, one more for the first (items mod waves) wavefronts.
__device__ __forceinline__ void item_block(uint32_t n, uint32_t wave, uint32_t waves, uint32_t& b0, uint32_t& b1,
                                          uint32_t& xcd) {
  xcd = blockIdx.x % kXcds;
  const uint32_t wx = gridDim.x / kXcds * waves;            // waves of this XCD (the grid is a multiple of 8)
  const uint32_t q = blockIdx.x / kXcds * waves + wave;     // this wave's rank among them
  const uint32_t len = xcd_items(n, xcd), share = len / wx, extra = len % wx;
  b0 = min(q * share + min(q, extra), len);
  b1 = min(b0 + share + (q < extra ? 1u : 0u), len);
}

// Plain decoder: every wavefront decodes one contiguous block of meshlets.
// kPlain: plain GTS stream; kCompact: degenerate triangles dropped, kept
// offsets in `kept`, out_tris counting output triangles.
// kCull: meshlets whose normal cone faces away from (vx, vy, vz) are skipped.
template <bool kPlain, bool kCompact, bool kCull = false, uint32_t kTile = 0>
__global__ __launch_bounds__(kWave * kMaxWavesPerGroup) void k_decode_plain(
    const gtsr_meshlet* __restrict__ meshlets, const uint8_t* __restrict__ bits,
    const uint8_t* __restrict__ reuse, uint8_t* __restrict__ out, const uint32_t* __restrict__ kept,
    uint32_t meshlet_count, uint64_t chunks, uint64_t reuse_bytes, uint64_t out_tris,
    const float* __restrict__ cones = nullptr, float vx = 0.0f, float vy = 0.0f, float vz = 0.0f) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = uniform(threadIdx.x / kWave);
  LanePtrs lp;
  RunTile<kPlain, kTile>& tile = wave_tile<kPlain, kTile>(wave, lane, lp);
  uint32_t b0, b1;
  wave_block(meshlet_count, wave, blockDim.x / kWave, b0, b1);
  if (b0 >= b1) return;
  const Stream s{reinterpret_cast<const uint8_t*>(meshlets), bits, reuse, out, kept,
                 clip32(chunks), clip32(reuse_bytes), clip32(out_tris), meshlet_count, cones, {vx, vy, vz}};
  decode_range<kPlain, kCompact, kCull, kTile>(s, b0, b1, tile, lp, lane);
}

// Decodes work items [b0, b1) of the batched work list with the calling
// wavefront: 64 items at a time, one per lane, merging consecutive items that
// continue the same mesh into one meshlet range.  [b0, b1) are list positions,
// or with kStriped positions among XCD xcd's stripes (xcd_item).
template <bool kPlain, uint32_t kTile, bool kStriped = false>
__device__ __forceinline__ void decode_items(const gtsr_mesh_entry* __restrict__ table, uint32_t mesh_count,
                                             const gtsr_work_item* __restrict__ work, uint32_t b0, uint32_t b1,
                                             RunTile<kPlain, kTile>& tile, const LanePtrs& lp, uint32_t lane,
                                             uint32_t xcd = 0) {
  for (uint64_t base = b0; base < b1; base += kWave) {
    const uint32_t cnt = uint32_t(min(b1 - base, uint64_t(kWave)));
    uint4 wi = make_uint4(0xFFFFFFFFu, 0, 0, 0);
    const uint32_t v = uint32_t(base) + lane;
    if (lane < cnt) wi = *reinterpret_cast<const uint4*>(work + (kStriped ? xcd_item(v, xcd) : v));
    const uint32_t prev_mesh = __shfl_up(wi.x, 1);
    const uint32_t prev_end = __shfl_up(wi.z, 1);
    // lane continues the item before it: same mesh, starts where it ended
    const uint64_t cont = __builtin_amdgcn_ballot_w64(lane > 0 && lane < cnt && wi.x == prev_mesh &&
                                                      wi.y == prev_end);
    uint32_t p = 0;
    while (p < cnt) {
      const uint64_t rest = p + 1 < 64 ? (cont >> (p + 1)) : 0ull;
      const uint32_t more = uint32_t(__builtin_ctzll(~rest));   // items continuing this one
      const uint32_t last = p + more;
      const uint32_t mesh = lane_value(wi.x, p);
      const uint32_t first = lane_value(wi.y, p);
      const uint32_t end = lane_value(wi.z, last);
      p = last + 1;
      if (mesh >= mesh_count) continue;
      const gtsr_mesh_entry& e = table[mesh];
      if ((reinterpret_cast<uintptr_t>(e.meshlets) | reinterpret_cast<uintptr_t>(e.bits) |
           reinterpret_cast<uintptr_t>(e.reuse)) & 15)
        continue;   // misaligned arrays: the entry is skipped
      const Stream s{reinterpret_cast<const uint8_t*>(e.meshlets), e.bits, e.reuse, e.out, nullptr,
                     clip32(e.bits_bytes / (kPlain ? 8 : 16)), clip32(e.reuse_bytes), clip32(e.strip_triangles),
                     e.meshlet_count};
      const uint32_t stop = min(end, e.meshlet_count);
      if (first < stop) decode_range<kPlain, false, false, kTile>(s, first, stop, tile, lp, lane);
    }
  }
}

// Batched decoder, static split: every wavefront of an over-subscribed grid
// takes one block of its XCD's stripes of the work list (items are balanced
// by strip triangles) and exits; the dispatcher refills freed slots with the
// next groups, so each XCD decodes its stripes roughly in order.
// kPlain: every entry holds a plain GTS stream; kTile: the LDS tile (Shape).
// Eight wavefronts per SIMD, as many as the LDS tiles admit (47 VGPRs, no
// scratch; the attribute keeps the compiler within 64).
template <bool kPlain, uint32_t kTile>
__global__ __launch_bounds__(kWave * kMaxWavesPerGroup) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_decode_batched(
    const gtsr_mesh_entry* __restrict__ table, uint32_t mesh_count,
    const gtsr_work_item* __restrict__ work, uint32_t work_items) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = uniform(threadIdx.x / kWave);
  LanePtrs lp;
  RunTile<kPlain, kTile>& tile = wave_tile<kPlain, kTile>(wave, lane, lp);
  uint32_t b0, b1, xcd;
  item_block(work_items, wave, blockDim.x / kWave, b0, b1, xcd);
  decode_items<kPlain, kTile, true>(table, mesh_count, work, b0, b1, tile, lp, lane, xcd);
}

// Batched decoder, persistent with claimed work: a grid of about the
// resident wavefront count, whose waves claim per_claim consecutive items at
// a time from a counter of their XCD's share of the list (its stripes, as
// in the static split; workgroups go
// round-robin over the 8 XCDs, so each XCD's waves claim from their own
// counter, in their own cache lines) until the share runs out.  Each claim's
// atomic is issued one claim ahead, so its return is in by the time the
// items before it are decoded.  The counters must be zero at the launch
// (k_claim_reset in front, in the same stream); a claim past the share ends
// the wave, so every wave exits.
constexpr uint32_t kClaimStride = 32;                    // 32-bit words between counters: one per 128-byte line
constexpr uint32_t kClaimWords = kXcds * kClaimStride;   // 1 KiB of workspace

__device__ __forceinline__ uint32_t claim_issue(uint32_t* ctr, uint32_t per_claim, uint32_t lane) {
  uint32_t v = 0;
  if (lane == 0) v = __hip_atomic_fetch_add(ctr, per_claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;   // lane 0's value; read with uniform() only when it is needed
}

template <bool kPlain, uint32_t kTile>
__global__ __launch_bounds__(kWave * kMaxWavesPerGroup) void k_decode_batched_claim(
    const gtsr_mesh_entry* __restrict__ table, uint32_t mesh_count,
    const gtsr_work_item* __restrict__ work, uint32_t work_items, uint32_t* __restrict__ counters,
    uint32_t per_claim) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = uniform(threadIdx.x / kWave);
  LanePtrs lp;
  RunTile<kPlain, kTile>& tile = wave_tile<kPlain, kTile>(wave, lane, lp);
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint32_t len = xcd_items(work_items, xcd);   // this XCD's stripes, as in the static split
  uint32_t* ctr = counters + xcd * kClaimStride;
  uint32_t c = uniform(claim_issue(ctr, per_claim, lane));
  while (c < len) {
    const uint32_t next = claim_issue(ctr, per_claim, lane);
    decode_items<kPlain, kTile, true>(table, mesh_count, work, c, min(c + per_claim, len), tile, lp, lane, xcd);
    c = uniform(next);
  }
}

// Zeroes the claim counters in front of a claiming launch (a kernel, so that
// a captured graph holds no memset node).
__global__ void k_claim_reset(uint32_t* __restrict__ counters) {
  if (threadIdx.x < kClaimWords) counters[threadIdx.x] = 0;
}

struct Defaults {
  uint32_t waves = 4, mpw = 8, gpc = 8;
  uint32_t tile = 0;   // Shape tile index; GTS-Reuse: 0 = 1280-triangle runs, 1 = 1024
  uint32_t claim = 0;  // batched: work items per claim (0 = static split)
};

// run_tris (batched decoders only): 0 = the default tile, else the run
// length of a compiled tile (1280 or 1024 for GTS-Reuse, 1024 for plain GTS).
int resolve_cfg(const gtsr_launch_cfg* cfg, Defaults& d, const char* who, bool batched = false,
                bool plain = false) {
  if (!cfg) return GTSR_OK;
  if (cfg->run_tris) {
    if (!batched) return fail(GTSR_EINVAL, std::string(who) + ": cfg.run_tris must be 0 (batched decoders only)");
    if (cfg->run_tris == Shape<false, 1>::kTris) d.tile = 1;
    else if (plain || cfg->run_tris != Shape<false, 0>::kTris)
      return fail(GTSR_EINVAL, std::string(who) + ": cfg.run_tris must be 0, 1024 or (GTS-Reuse) 1280");
  }
  if (cfg->waves_per_group) {
    if (cfg->waves_per_group > kMaxWavesPerGroup) return fail(GTSR_EINVAL, std::string(who) + ": waves_per_group > 16");
    d.waves = cfg->waves_per_group;
  }
  if (cfg->meshlets_per_wave) {
    if (cfg->meshlets_per_wave > 1024) return fail(GTSR_EINVAL, std::string(who) + ": meshlets_per_wave > 1024");
    d.mpw = cfg->meshlets_per_wave;
  }
  if (cfg->groups_per_cu) {
    if (cfg->groups_per_cu > kMaxGroupsPerCu)
      return fail(GTSR_EINVAL, std::string(who) + ": groups_per_cu > 1024");
    d.gpc = cfg->groups_per_cu;
  }
  if (cfg->items_per_claim) {
    if (!batched) return fail(GTSR_EINVAL, std::string(who) + ": cfg.items_per_claim must be 0 (batched decoders only)");
    if (cfg->items_per_claim > 1024) return fail(GTSR_EINVAL, std::string(who) + ": items_per_claim > 1024");
    d.claim = cfg->items_per_claim;
  }
  return GTSR_OK;
}

// Per-device caches, fixed-size so that no call after the first allocates.
constexpr int kMaxDevices = 64;
std::mutex g_cu_mutex;
uint32_t g_cu_count[kMaxDevices];   // 0 = not queried yet

uint32_t cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
  std::lock_guard<std::mutex> lk(g_cu_mutex);
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

inline uint32_t round_up8(uint64_t g) { return uint32_t((g + kXcds - 1) / kXcds * kXcds); }

int enqueue_batched(const gtsr_mesh_entry* table, uint32_t mesh_count, const gtsr_work_item* work,
                    uint32_t work_items, void* workspace, uint64_t workspace_bytes, const gtsr_launch_cfg* cfg,
                    hipStream_t stream, const char* who, bool plain = false) {
  if ((mesh_count && !table) || (work_items && !work)) return fail(GTSR_EINVAL, std::string(who) + ": null pointer");
  if ((reinterpret_cast<uintptr_t>(table) & 15) || (reinterpret_cast<uintptr_t>(work) & 15))
    return fail(GTSR_EINVAL, std::string(who) + ": tables must be 16-byte aligned");
  if (work_items > 0x80000000u) return fail(GTSR_EINVAL, std::string(who) + ": more than 2^31 work items");
  Defaults d;
  // measured best on the batched 2000-mesh workload: one-wave groups, 256 per
  // CU (about 9 times the resident count, so freed slots are refilled until
  // the end)
  d.waves = 1;
  d.gpc = 256;
  if (int rc = resolve_cfg(cfg, d, who, true, plain)) return rc;
  if (d.claim) {
    if (!workspace || workspace_bytes < GTSR_BATCHED_WORKSPACE_BYTES)
      return fail(GTSR_EINVAL, std::string(who) + ": claiming needs a workspace of GTSR_BATCHED_WORKSPACE_BYTES");
    if (reinterpret_cast<uintptr_t>(workspace) & 3)
      return fail(GTSR_EINVAL, std::string(who) + ": workspace must be 4-byte aligned");
    if (!cfg->groups_per_cu) d.gpc = 32 / d.waves ? 32 / d.waves : 1;   // about the resident count
  }
  const uint32_t cus = cu_count();
  if (!cus) return fail(GTSR_EHIP, std::string(who) + ": cannot query the device");
  if (work_items == 0) return ok();
  // the configured grid, or fewer groups when the list has fewer items (or
  // claims) than that grid has wavefronts
  const uint64_t units = d.claim ? (uint64_t(work_items) + d.claim - 1) / d.claim : work_items;
  const uint64_t want = (units + d.waves - 1) / d.waves;
  const uint32_t groups = round_up8(std::min<uint64_t>(uint64_t(cus) * d.gpc, want));
  const dim3 grid(groups), block(kWave * d.waves);
  const uint32_t lds = d.waves * (plain ? kTileBytes<true, 0> : d.tile == 1 ? kTileBytes<false, 1> : kTileBytes<false, 0>);
  if (d.claim) {
    uint32_t* ctr = static_cast<uint32_t*>(workspace);
    hipLaunchKernelGGL(k_claim_reset, dim3(1), dim3(kClaimWords), 0, stream, ctr);
    if (plain)
      hipLaunchKernelGGL((k_decode_batched_claim<true, 0>), grid, block, lds, stream, table, mesh_count, work,
                         work_items, ctr, d.claim);
    else if (d.tile == 1)
      hipLaunchKernelGGL((k_decode_batched_claim<false, 1>), grid, block, lds, stream, table, mesh_count, work,
                         work_items, ctr, d.claim);
    else
      hipLaunchKernelGGL((k_decode_batched_claim<false, 0>), grid, block, lds, stream, table, mesh_count, work,
                         work_items, ctr, d.claim);
    return check_launch(who);
  }
  if (plain)
    hipLaunchKernelGGL((k_decode_batched<true, 0>), grid, block, lds, stream, table, mesh_count, work, work_items);
  else if (d.tile == 1)
    hipLaunchKernelGGL((k_decode_batched<false, 1>), grid, block, lds, stream, table, mesh_count, work, work_items);
  else
    hipLaunchKernelGGL((k_decode_batched<false, 0>), grid, block, lds, stream, table, mesh_count, work, work_items);
  return check_launch(who);
}

int check_plain_args(const gtsr_stream* dev, const uint8_t* dev_out, uint64_t out_bytes, bool compact = false) {
  if (!dev) return fail(GTSR_EINVAL, "decode_meshlets: null stream");
  if (dev->meshlet_count == 0) return GTSR_OK;
  if (!dev->meshlets || !dev->bits || !dev_out || (dev->reuse_bytes && !dev->reuse))
    return fail(GTSR_EINVAL, "decode_meshlets: null device pointer");
  if (!compact && out_bytes / 3 < dev->strip_triangles)
    return fail(GTSR_EINVAL, "decode_meshlets: out_bytes < 3 * strip_triangles");
  if ((reinterpret_cast<uintptr_t>(dev->meshlets) | reinterpret_cast<uintptr_t>(dev->bits) |
       reinterpret_cast<uintptr_t>(dev->reuse)) & 15)
    return fail(GTSR_EINVAL, "decode_meshlets: meshlets, bits and reuse must be 16-byte aligned");
  return GTSR_OK;
}

// Grid: one wave per mpw meshlets, capped at groups_per_cu resident groups
// per CU (each wave then takes a larger contiguous block).
// plain: plain GTS stream (8-byte L/R words); kept: compacted output.
int launch_plain(const gtsr_stream* dev, uint8_t* dev_out, uint64_t out_bytes, const Defaults& d,
                 uint32_t cus, hipStream_t stream, bool plain = false, const uint32_t* kept = nullptr) {
  if (dev->meshlet_count == 0) return GTSR_OK;
  const uint64_t waves = (uint64_t(dev->meshlet_count) + d.mpw - 1) / d.mpw;
  uint64_t groups = (waves + d.waves - 1) / d.waves;
  groups = std::min<uint64_t>(groups, uint64_t(cus) * d.gpc);
  const dim3 grid(round_up8(groups)), block(kWave * d.waves);
  const uint32_t lds = d.waves * (plain ? kTileBytes<true> : kTileBytes<false>);
  const uint64_t chunks = dev->bits_bytes / (plain ? 8 : 16);
#define GTSR_LAUNCH_PLAIN(P, K)                                                                                   \
  hipLaunchKernelGGL((k_decode_plain<P, K>), grid, block, lds, stream, dev->meshlets, dev->bits, dev->reuse, dev_out, \
                     kept, dev->meshlet_count, chunks, dev->reuse_bytes, out_bytes / 3)
  if (plain) {
    if (kept) GTSR_LAUNCH_PLAIN(true, true);
    else GTSR_LAUNCH_PLAIN(true, false);
  } else {
    if (kept) GTSR_LAUNCH_PLAIN(false, true);
    else GTSR_LAUNCH_PLAIN(false, false);
  }
#undef GTSR_LAUNCH_PLAIN
  return GTSR_OK;
}

}  // namespace
}  // namespace gtsr

using namespace gtsr;

extern "C" int gtsr_decode_meshlets_cfg(const gtsr_stream* dev, uint8_t* dev_out, uint64_t out_bytes,
                                        const gtsr_launch_cfg* cfg, void* hip_stream) {
  if (int rc = check_plain_args(dev, dev_out, out_bytes)) return rc;
  Defaults d;
  if (int rc = resolve_cfg(cfg, d, "decode_meshlets")) return rc;
  const uint32_t cus = cu_count();
  if (!cus) return fail(GTSR_EHIP, "decode_meshlets: cannot query the device");
  launch_plain(dev, dev_out, out_bytes, d, cus, static_cast<hipStream_t>(hip_stream));
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
  const uint32_t cus = cu_count();
  if (!cus) return fail(GTSR_EHIP, "gtsr_decode_meshlets_many: cannot query the device");
  for (uint32_t i = 0; i < n; ++i)
    launch_plain(&streams[i], dev_outs[i], out_bytes[i], d, cus, static_cast<hipStream_t>(hip_stream));
  return check_launch("gtsr_decode_meshlets_many");
}

extern "C" int decode_meshlets(const gtsr_stream* dev, uint8_t* dev_out, uint64_t out_bytes, void* hip_stream) {
  return gtsr_decode_meshlets_cfg(dev, dev_out, out_bytes, nullptr, hip_stream);
}

extern "C" int gtsr_decode_gts(const gtsr_stream* dev, uint8_t* dev_out, uint64_t out_bytes, const gtsr_launch_cfg* cfg,
                               void* hip_stream) {
  if (int rc = check_plain_args(dev, dev_out, out_bytes)) return rc;
  if (dev->bits_bytes % 8) return fail(GTSR_EINVAL, "gtsr_decode_gts: bits_bytes must be a multiple of 8");
  Defaults d;
  if (int rc = resolve_cfg(cfg, d, "gtsr_decode_gts")) return rc;
  const uint32_t cus = cu_count();
  if (!cus) return fail(GTSR_EHIP, "gtsr_decode_gts: cannot query the device");
  launch_plain(dev, dev_out, out_bytes, d, cus, static_cast<hipStream_t>(hip_stream), true);
  return check_launch("gtsr_decode_gts");
}

extern "C" int gtsr_decode_compact(const gtsr_stream* dev, uint32_t format, const uint32_t* dev_kept_off,
                                   uint8_t* dev_out, uint64_t out_bytes, const gtsr_launch_cfg* cfg,
                                   void* hip_stream) {
  const char* who = "gtsr_decode_compact";
  if (format != GTSR_FORMAT_REUSE && format != GTSR_FORMAT_GTS) return fail(GTSR_EINVAL, std::string(who) + ": bad format");
  if (int rc = check_plain_args(dev, dev_out, out_bytes, true)) return rc;
  if (dev->meshlet_count && !dev_kept_off) return fail(GTSR_EINVAL, std::string(who) + ": null kept offsets");
  if (reinterpret_cast<uintptr_t>(dev_kept_off) & 3)
    return fail(GTSR_EINVAL, std::string(who) + ": kept offsets must be 4-byte aligned");
  if (format == GTSR_FORMAT_GTS && dev->bits_bytes % 8)
    return fail(GTSR_EINVAL, std::string(who) + ": bits_bytes must be a multiple of 8");
  Defaults d;
  if (int rc = resolve_cfg(cfg, d, who)) return rc;
  const uint32_t cus = cu_count();
  if (!cus) return fail(GTSR_EHIP, std::string(who) + ": cannot query the device");
  launch_plain(dev, dev_out, out_bytes, d, cus, static_cast<hipStream_t>(hip_stream), format == GTSR_FORMAT_GTS,
               dev_kept_off);
  return check_launch(who);
}

extern "C" int gtsr_decode_culled(const gtsr_stream* dev, const float* dev_cones, float view_x, float view_y,
                                  float view_z, uint8_t* dev_out, uint64_t out_bytes, const gtsr_launch_cfg* cfg,
                                  void* hip_stream) {
  const char* who = "gtsr_decode_culled";
  if (int rc = check_plain_args(dev, dev_out, out_bytes)) return rc;
  if (dev->meshlet_count && !dev_cones) return fail(GTSR_EINVAL, std::string(who) + ": null cones");
  if (reinterpret_cast<uintptr_t>(dev_cones) & 15) return fail(GTSR_EINVAL, std::string(who) + ": cones must be 16-byte aligned");
  Defaults d;
  if (int rc = resolve_cfg(cfg, d, who)) return rc;
  const uint32_t cus = cu_count();
  if (!cus) return fail(GTSR_EHIP, std::string(who) + ": cannot query the device");
  if (dev->meshlet_count == 0) return ok();
  const uint64_t waves = (uint64_t(dev->meshlet_count) + d.mpw - 1) / d.mpw;
  uint64_t groups = (waves + d.waves - 1) / d.waves;
  groups = std::min<uint64_t>(groups, uint64_t(cus) * d.gpc);
  hipLaunchKernelGGL((k_decode_plain<false, false, true>), dim3(round_up8(groups)), dim3(kWave * d.waves),
                     d.waves * kTileBytes<false>, static_cast<hipStream_t>(hip_stream), dev->meshlets, dev->bits,
                     dev->reuse, dev_out, nullptr, dev->meshlet_count, dev->bits_bytes / 16, dev->reuse_bytes,
                     out_bytes / 3, dev_cones, view_x, view_y, view_z);
  return check_launch(who);
}

extern "C" int gtsr_decode_gts_batched(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                                       const gtsr_work_item* dev_work, uint32_t work_items, void* dev_workspace,
                                       uint64_t workspace_bytes, const gtsr_launch_cfg* cfg, void* hip_stream) {
  return enqueue_batched(dev_mesh_table, mesh_count, dev_work, work_items, dev_workspace, workspace_bytes, cfg,
                         static_cast<hipStream_t>(hip_stream), "gtsr_decode_gts_batched", true);
}

extern "C" int decode_meshlets_batched(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                                       const gtsr_work_item* dev_work, uint32_t work_items, void* dev_workspace,
                                       uint64_t workspace_bytes, const gtsr_launch_cfg* cfg, void* hip_stream) {
  return enqueue_batched(dev_mesh_table, mesh_count, dev_work, work_items, dev_workspace, workspace_bytes, cfg,
                         static_cast<hipStream_t>(hip_stream), "decode_meshlets_batched");
}

extern "C" int gtsr_batched_graph_create(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                                         const gtsr_work_item* dev_work, uint32_t work_items, void* dev_workspace,
                                         uint64_t workspace_bytes, uint32_t format, const gtsr_launch_cfg* cfg,
                                         void** graph_exec) {
  const char* who = "gtsr_batched_graph_create";
  if (!graph_exec) return fail(GTSR_EINVAL, "gtsr_batched_graph_create: null graph_exec");
  *graph_exec = nullptr;
  if (format != GTSR_FORMAT_REUSE && format != GTSR_FORMAT_GTS)
    return fail(GTSR_EINVAL, "gtsr_batched_graph_create: bad format");
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
    return fail(GTSR_EHIP, "gtsr_batched_graph_create: stream creation failed");
  hipGraph_t graph = nullptr;
  int rc = GTSR_OK;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = fail(GTSR_EHIP, "gtsr_batched_graph_create: begin capture failed");
  } else {
    rc = enqueue_batched(dev_mesh_table, mesh_count, dev_work, work_items, dev_workspace, workspace_bytes, cfg, s,
                         who, format == GTSR_FORMAT_GTS);
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc == GTSR_OK && e != hipSuccess)
      rc = fail(GTSR_EHIP, std::string(who) + ": end capture: " + hipGetErrorString(e));
  }
  if (rc == GTSR_OK && graph) {
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

// ------------------------------------------------- allocation-free entry point

// The claim counters of gtsr_decode_batched_noalloc: a file-scope device
// array, one copy per device the library runs on, kept until the process
// ends.  In host code its name is not a device address; each device's
// address comes from hipGetSymbolAddress on that call's first use of the
// device, with the device current, and is kept per device.
static __device__ __align__(256) uint32_t scratch[GTSR_BATCHED_WORKSPACE_BYTES / 4];

namespace gtsr {
namespace {
constexpr uint32_t kScratchBytes = GTSR_BATCHED_WORKSPACE_BYTES;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices];

int scratch_ptr(void** out, const char* who) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(GTSR_EHIP, std::string(who) + ": cannot query the device");
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GTSR_EHIP, std::string(who) + ": scratch address: " + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GTSR_OK;
}
}  // namespace
}  // namespace gtsr

extern "C" int gtsr_decode_batched_noalloc(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                                           const gtsr_work_item* dev_work, uint32_t work_items, uint32_t format,
                                           const gtsr_launch_cfg* cfg, void* hip_stream) {
  const char* who = "gtsr_decode_batched_noalloc";
  if (format != GTSR_FORMAT_REUSE && format != GTSR_FORMAT_GTS) return fail(GTSR_EINVAL, std::string(who) + ": bad format");
  gtsr_launch_cfg c{};
  if (cfg) c = *cfg;
  if (!c.items_per_claim) c.items_per_claim = 2;
  void* ws = nullptr;
  if (int rc = scratch_ptr(&ws, who)) return rc;
  return enqueue_batched(dev_mesh_table, mesh_count, dev_work, work_items, ws, kScratchBytes, &c,
                         static_cast<hipStream_t>(hip_stream), who, format == GTSR_FORMAT_GTS);
}
