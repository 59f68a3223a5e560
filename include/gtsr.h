/*
 * gtsr.h -- GTS-Reuse meshlet connectivity codec for MI355X (gfx950).
 *
 * Kuth et al., "Towards Practical Meshlet Compression" (VMV 2024):
 *   - Sec. 3: a mesh is split into meshlets of at most max_vertices vertices
 *     and max_triangles triangles; each meshlet indexes its own vertices with
 *     8-bit local indices (3 bytes per triangle, "basic mesh shading").
 *   - Sec. 4.2: each meshlet's triangles are stored as a generalized triangle
 *     strip, one L/R flag per triangle; a strip restart costs four degenerate
 *     triangles; a meshlet whose strip outgrows the triangle limit is split.
 *   - Sec. 4.3: vertices are renumbered by first appearance in the strip, so
 *     the strip starts with 0,1,2 and every first appearance is one set
 *     increment flag; only reused local indices are stored, one byte each.
 *   - Sec. 1 / Sec. 4: compression happens offline on the CPU, decompression
 *     on the GPU back to 8-bit local index triples.
 *
 * encode_meshlets is the CPU side; decode_meshlets (one mesh) and
 * decode_meshlets_batched (many meshes, one launch) are the GPU
 * side.  Every call returns an int status (GTSR_OK or a negative code); no
 * exception crosses this interface.  gtsr_last_error() describes the last
 * failure on the calling thread.  All calls are reentrant.
 *
 * Stream layout (little-endian; the encoder writes it, the decoders read it)
 *   meshlets  gtsr_meshlet[meshlet_count], 16 bytes each.
 *   bits      16 bytes per 64 strip triangles of a meshlet: u64 LR, u64 INC.
 *             Bit i of chunk c belongs to strip triangle 64c+i.  LR bit 1 = R
 *             (the strip continues across the right edge of the previous
 *             triangle), 0 = L (left edge); for triangle 0 the flag gives its
 *             orientation (L: 0,1,2; R: 1,0,2).  INC bit 1 = the triangle's new
 *             index is the next new vertex, 0 = the next reuse byte.  Triangle
 *             0 has no INC bit (stored 0).  Bits at positions >= T_s are 0.
 *   reuse     one byte per reused local index, meshlet after meshlet.
 *   Offsets are contiguous: meshlet m+1 starts where meshlet m ends in all
 *   three arrays and in the output; the first meshlet starts at 0.
 *   output    uint8[strip_triangles][3]: meshlet m's T_s triples start at
 *             triangle out_off.  Degenerate (restart) triples are included.
 */
#ifndef GTSR_H
#define GTSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GTSR_OK = 0,
  GTSR_EINVAL = -1,       /* null pointer, index >= vertex_count, buffer too small, bad config */
  GTSR_ENOMEM = -2,       /* host allocation failed */
  GTSR_EDEGENERATE = -3,  /* an input triangle repeats a vertex */
  GTSR_ELIMIT = -4,       /* caps out of range, or counts overflow 32-bit offsets */
  GTSR_ECORRUPT = -5,     /* gtsr_validate found a violated stream invariant */
  GTSR_EHIP = -6,         /* a HIP runtime call failed */
  GTSR_ECANCELED = -7,    /* serving: the request was withdrawn before admission */
  GTSR_EBUSY = -8,        /* serving: too late to withdraw, the request was already admitted */
  GTSR_EIO = -9           /* a file could not be opened, read or written */
};

/* Stream formats (Sec. 4.2 / 4.3; Fig. "Strip Encoding" (c) and (d)). */
enum {
  GTSR_FORMAT_REUSE = 0,  /* GTS-Reuse: 16-byte chunks {LR, INC} + reuse bytes (the layout above) */
  GTSR_FORMAT_GTS = 1     /* plain GTS: one 8-byte L/R word per 64 strip triangles + one index
                             byte per strip triangle after the first (the vertex it adds; the
                             first triangle's 0,1,2 are implicit).  Descriptors keep their
                             layout: chunk_off counts 8-byte words, reuse_off index bytes. */
};

/* Per-meshlet descriptor, 16 bytes.  tri_count = T_s (strip triangles,
 * degenerates included, 1..256); vert_count = V (3..256); the meshlet holds
 * T_s + 2 - V reuse bytes and ceil(T_s/64) flag chunks. */
typedef struct gtsr_meshlet {
  uint32_t chunk_off;   /* first 16-byte flag chunk */
  uint32_t reuse_off;   /* first reuse byte */
  uint32_t out_off;     /* first output triangle */
  uint16_t tri_count;
  uint16_t vert_count;
} gtsr_meshlet;

/* gtsr_encode_params.flags */
enum {
  /* After the greedy strips of a meshlet, search for fewer strips (the
   * optimal GTS of Sec. 3.1; the paper solves a MILP): branch and bound over
   * chains of neighbouring triangles, 200000 search nodes per meshlet, kept
   * when it beats the greedy count.  Streams then differ from the greedy
   * encoder's; decoding is unchanged. */
  GTSR_ENCODE_EXACT_STRIPS = 1
};

typedef struct gtsr_encode_params {
  uint32_t max_vertices;    /* 3..256 */
  uint32_t max_triangles;   /* 1..256; bounds T_s (restart degenerates count) */
  uint32_t threads;         /* 0 = all hardware threads */
  uint32_t flags;           /* GTSR_ENCODE_* bits; others must be 0 */
} gtsr_encode_params;

typedef struct gtsr_encoded gtsr_encoded;   /* opaque, host memory, library-owned */

/* Read-only view into a gtsr_encoded (host pointers, valid until
 * gtsr_encoded_free).  vertices[vert_off[m] .. vert_off[m+1]) maps meshlet
 * m's local vertex ids to the input's vertex ids (host-side only; the
 * decoders never read it).  payload_bits = sum over meshlets of
 * T_s + (T_s - 1) + 8 * reuse bytes; stored_bytes = sum of
 * 16 + 16 * chunks + reuse bytes. */
typedef struct gtsr_encoded_view {
  uint32_t meshlet_count;
  uint32_t reserved;
  uint64_t input_triangles, strip_triangles, restarts, reuse_count, split_meshlets;
  const gtsr_meshlet* meshlets;
  const uint8_t* bits;
  uint64_t bits_bytes;
  const uint8_t* reuse;
  uint64_t reuse_bytes;
  const uint32_t* vertices;
  const uint64_t* vert_off;     /* meshlet_count + 1 entries */
  uint64_t payload_bits, stored_bytes;
  const uint32_t* kept_off;     /* meshlet_count + 1 entries: input triangles before meshlet m
                                   (strip triangles minus restart degenerates); the offsets of a
                                   compacted output (gtsr_decode_compact) */
  const uint32_t* tri_ids;      /* input_triangles entries: the input triangles of meshlet m at
                                   [kept_off[m], kept_off[m+1]), in strip (= compacted output) order */
  uint64_t exact_tried;         /* GTSR_ENCODE_EXACT_STRIPS: meshlets searched */
  uint64_t exact_proven;        /* ... of which the search finished (optimal strips) */
} gtsr_encoded_view;

/* One encoded mesh.  For decode_meshlets the three pointers are device
 * pointers; for gtsr_validate they are host pointers. */
typedef struct gtsr_stream {
  const gtsr_meshlet* meshlets;
  const uint8_t* bits;
  const uint8_t* reuse;
  uint32_t meshlet_count;
  uint32_t reserved;
  uint64_t bits_bytes;        /* 16 * total chunks */
  uint64_t reuse_bytes;
  uint64_t strip_triangles;   /* sum of T_s = output triangles */
} gtsr_stream;

/* Launch shape for the decoders; NULL selects the built-in defaults. */
typedef struct gtsr_launch_cfg {
  uint32_t waves_per_group;     /* 1..16: workgroup of 64*waves threads */
  uint32_t meshlets_per_wave;   /* decode_meshlets: meshlets per wavefront at least, 1..1024 */
  uint32_t groups_per_cu;       /* groups per CU the grid is capped at, 1..1024 (above the
                                   resident count, the dispatcher refills freed slots) */
  uint32_t run_tris;            /* batched decoders: the LDS tile, as strip triangles per run:
                                   0 = default, 1280 or 1024 (GTS-Reuse), 1024 (plain GTS);
                                   every other decoder: must be 0 */
  uint32_t items_per_claim;     /* batched decoders: 0 = static split (each wavefront of an
                                   over-subscribed grid decodes one block of its XCD's
                                   256-item stripes of the work list);
                                   1..1024 = persistent grid (groups_per_cu groups per CU, at
                                   most one wavefront per claim) whose wavefronts claim this
                                   many work items at a time from per-XCD counters kept in
                                   the caller's workspace; every other decoder: must be 0 */
} gtsr_launch_cfg;

/* Workspace bytes a batched decode with cfg.items_per_claim > 0 needs: eight
 * 32-bit counters, one per 128-byte line. */
#define GTSR_BATCHED_WORKSPACE_BYTES 1024u

/* One row of the batched decoder's mesh table (device memory, 64 bytes):
 * a gtsr_stream's device pointers plus where its output goes. */
typedef struct gtsr_mesh_entry {
  const gtsr_meshlet* meshlets;
  const uint8_t* bits;
  const uint8_t* reuse;
  uint8_t* out;               /* device, >= 3 * strip_triangles bytes */
  uint32_t meshlet_count;
  uint32_t reserved0;
  uint64_t bits_bytes;
  uint64_t reuse_bytes;
  uint64_t strip_triangles;
} gtsr_mesh_entry;

/* One work item of the batched decoder: meshlets [first, end) of one mesh.
 * An item past the mesh's meshlet count is clipped to it, one with
 * first >= end decodes nothing, and overlapping items decode the shared
 * meshlets again (the same bytes).  Consecutive items of one mesh where the
 * second starts at the first's end are decoded as one range [first of the
 * first, end of the last). */
typedef struct gtsr_work_item {
  uint32_t mesh;
  uint32_t first;
  uint32_t end;
  uint32_t reserved;
} gtsr_work_item;

/* ---------------------------------------------------------------- CPU side */

/* Split a CCW triangle list into meshlets and encode each (Sec. 3, 4.2, 4.3).
 * indices: host uint32[triangle_count][3], each < vertex_count, no repeated
 * vertex in a triangle.  Meshlets are built greedily (the paper uses a
 * third-party builder and MILP-optimal strips; the greedy rules are stated in
 * the implementation).  On success *out owns host memory until
 * gtsr_encoded_free.  An empty mesh gives 0 meshlets.
 * Errors: EINVAL (null pointer, index >= vertex_count), EDEGENERATE, ELIMIT
 * (caps out of range, reserved != 0, more than 2^32-1 strip triangles),
 * ENOMEM. */
int encode_meshlets(const uint32_t* indices, uint64_t triangle_count, uint32_t vertex_count,
                    const gtsr_encode_params* params, gtsr_encoded** out);

/* Fewest strips that cover a triangle set of at most 256 CCW triangles (the
 * optimal GTS of Sec. 3.1), by the branch and bound of
 * GTSR_ENCODE_EXACT_STRIPS from no incumbent, stopped after node_limit
 * search nodes: *strips gets the best count found, *proven 1 if the search
 * finished (the count is optimal).  Neighbours are as for the encoder
 * (edges shared by exactly two triangles in opposite directions).  Errors:
 * EINVAL, ELIMIT (more than 256 triangles), ENOMEM. */
int gtsr_min_strips(const uint32_t* indices, uint32_t triangle_count, uint64_t node_limit, uint32_t* strips,
                    uint32_t* proven);

/* Fill *view with pointers into e: the meshlets of Sec. 3 (descriptors,
 * local-to-global vertex lists), the GTS-Reuse streams of Sec. 4.2 / 4.3
 * (flag chunks, reuse bytes) and the encoder's counters (restarts: Sec. 4.2's
 * four degenerates each; payload bits as in Table 2).  Errors: EINVAL on
 * null. */
int gtsr_encoded_view_get(const gtsr_encoded* e, gtsr_encoded_view* view);

void gtsr_encoded_free(gtsr_encoded* e);

/* Full structural check of a host-resident stream against the invariants of
 * Sec. 4.3 (vertices renumbered by first appearance: the strip starts with
 * 0, 1, 2, every increment flag introduces the next vertex, every reuse byte
 * names one already introduced) and of the layout above: counts in range
 * (Sec. 3's caps, T_s <= 256), contiguous offsets from 0, array sizes equal
 * to the totals, triangle 0's INC bit and all bits past T_s clear,
 * increments = V - 3.  Returns OK or ECORRUPT (EINVAL on null). */
int gtsr_validate(const gtsr_stream* host_stream);

/* Re-encode a valid host GTS-Reuse stream as plain GTS (same strips, same
 * flags; each strip triangle after the first stores the vertex it adds).
 * Caller-owned host outputs: gdesc[meshlet_count]; words, 8 bytes per
 * 16-byte chunk of the input (words_bytes = bits_bytes / 2); index,
 * strip_triangles - meshlet_count bytes.  Errors: EINVAL (null pointer,
 * capacity too small), ECORRUPT (the input fails gtsr_validate). */
int gtsr_gts_from_reuse(const gtsr_stream* host_reuse_stream, gtsr_meshlet* gdesc, uint8_t* words,
                        uint64_t words_bytes, uint8_t* index, uint64_t index_bytes);

/* Build a triangle-balanced work list for decode_meshlets_batched (not in
 * the paper, which dispatches one thread group per meshlet (Sec. 3); the
 * batched decoders hand a wavefront a run of consecutive meshlets instead).
 * host_meshlets[i] points at mesh i's host descriptor array of
 * meshlet_counts[i] entries.  Items never span two meshes and hold
 * consecutive meshlets totalling about target_tris strip triangles (at
 * least one meshlet).  Writes at most capacity items to items (may be NULL
 * to count) and the number needed to *count.  Errors: EINVAL. */
int gtsr_plan_batch(const gtsr_meshlet* const* host_meshlets, const uint32_t* meshlet_counts,
                    uint32_t mesh_count, uint32_t target_tris, gtsr_work_item* items,
                    uint32_t capacity, uint32_t* count);

/* ---------------------------------------------------------------- GPU side */

/* Decode one mesh on the GPU (Sec. 4.2 / 4.3): each wavefront decodes a
 * contiguous block of meshlets, one lane per strip triangle.  dev: host struct
 * holding device pointers.  dev_out: device, out_bytes >= 3 *
 * strip_triangles.  dev->meshlets, dev->bits and dev->reuse must be 16-byte
 * aligned, and the reuse allocation must extend to the next multiple of 16
 * bytes past reuse_bytes (it is read in whole 16-byte blocks); the output may
 * have any alignment.  bits_bytes and reuse_bytes must not exceed the
 * allocations behind dev->bits and dev->reuse: flag chunks are fetched with
 * scalar loads, which only the descriptor checks against bits_bytes keep in
 * bounds.
 * Enqueued on hip_stream (a hipStream_t; NULL = the null stream); returns
 * before the work finishes; allocates nothing, never synchronizes.  Meshlets whose descriptor points outside the given sizes
 * are skipped (their output bytes are left untouched); gtsr_validate reports
 * such streams.  Errors: EINVAL (null pointer, out_bytes too small, bad
 * cfg), EHIP (launch failed). */
int decode_meshlets(const gtsr_stream* dev, uint8_t* dev_out, uint64_t out_bytes, void* hip_stream);

/* decode_meshlets with an explicit launch shape (cfg may be NULL). */
int gtsr_decode_meshlets_cfg(const gtsr_stream* dev, uint8_t* dev_out, uint64_t out_bytes,
                             const gtsr_launch_cfg* cfg, void* hip_stream);

/* decode_meshlets for a plain GTS stream (GTSR_FORMAT_GTS): dev->bits holds
 * the 8-byte L/R words (bits_bytes a multiple of 8), dev->reuse the index
 * bytes (reuse_bytes of them, allocation padded to 16 bytes).  Same output,
 * alignment, skipping and error rules as decode_meshlets. */
int gtsr_decode_gts(const gtsr_stream* dev, uint8_t* dev_out, uint64_t out_bytes, const gtsr_launch_cfg* cfg,
                    void* hip_stream);

/* Decode one mesh (format GTSR_FORMAT_REUSE or GTSR_FORMAT_GTS) into a
 * compacted output without the restart degenerates (Sec. 4.2: four per
 * restart, the only triangles with a repeated index): meshlet m's kept
 * triangles land in order at triangle dev_kept_off[m].  dev_kept_off: device
 * uint32[meshlet_count + 1], 4-byte aligned (gtsr_encoded_view.kept_off);
 * out_bytes should be >= 3 * dev_kept_off[meshlet_count].  A meshlet whose
 * kept range is decreasing, longer than its strip or past out_bytes is
 * skipped.  Errors: EINVAL, EHIP. */
int gtsr_decode_compact(const gtsr_stream* dev, uint32_t format, const uint32_t* dev_kept_off, uint8_t* dev_out,
                        uint64_t out_bytes, const gtsr_launch_cfg* cfg, void* hip_stream);

/* Per-meshlet normal cones for culling (Sec. 3: the amplification shader
 * drops meshlets whose triangles all face away).  Host side: for meshlet m
 * the input triangles tri_ids[kept_off[m] .. kept_off[m+1]) of indices
 * (gtsr_encoded_view), vertex positions float32[vertex_count][3].  Writes
 * cones float32[meshlet_count][4] = {axis x, y, z, cutoff}: axis = the
 * normalised sum, in tri_ids order, of the unit triangle normals
 * (p1-p0) x (p2-p0), each triangle first rotated (orientation kept) to start
 * at its smallest vertex id (zero-area triangles ignored), cutoff =
 * sin(largest angle between axis and a normal) + 1e-5, or 2 when that angle
 * is 90 degrees or more (never culled); float64 arithmetic, rounded once to
 * float32, so the result depends only on the triangles and their order.
 * Errors: EINVAL (a kept range decreasing, past triangle_count or longer
 * than 256 triangles; a triangle or vertex id out of range). */
int gtsr_meshlet_cones(const uint32_t* indices, uint64_t triangle_count, const float* positions,
                       uint32_t vertex_count, const uint32_t* tri_ids, const uint32_t* kept_off,
                       uint32_t meshlet_count, float* cones);

/* decode_meshlets with cone culling in front (GTS-Reuse format): a meshlet
 * whose cone satisfies fmaf(az, vz, fmaf(ay, vy, ax * vx)) > cutoff (every
 * triangle faces away from the unit view direction v) is not decoded and its
 * output bytes are left untouched; every other meshlet decodes as in
 * decode_meshlets.  dev_cones: device float32[meshlet_count][4], 16-byte
 * aligned (gtsr_meshlet_cones).  Errors: EINVAL, EHIP. */
int gtsr_decode_culled(const gtsr_stream* dev, const float* dev_cones, float view_x, float view_y, float view_z,
                       uint8_t* dev_out, uint64_t out_bytes, const gtsr_launch_cfg* cfg, void* hip_stream);

/* One plain decode launch per mesh, back to back on hip_stream: streams[i]
 * (host array of structs holding device pointers) into dev_outs[i] (host
 * array of device pointers) of out_bytes[i] bytes.  Arguments of every mesh
 * are checked before the first launch; then it behaves as n calls of
 * gtsr_decode_meshlets_cfg.  Errors: EINVAL, EHIP. */
int gtsr_decode_meshlets_many(const gtsr_stream* streams, uint8_t* const* dev_outs,
                              const uint64_t* out_bytes, uint32_t n, const gtsr_launch_cfg* cfg,
                              void* hip_stream);

/* Decode many meshes in one launch.  dev_mesh_table: device
 * gtsr_mesh_entry[mesh_count]; dev_work: device gtsr_work_item[work_items]
 * (gtsr_plan_batch); both 16-byte aligned, as must be every entry's
 * meshlets, bits and reuse pointer (entries that are not are skipped); each
 * reuse allocation must extend to a multiple of 16 bytes, and no entry's
 * sizes may exceed its allocations (as for decode_meshlets).  Two launch
 * modes (cfg->items_per_claim):
 *   0 (default): static split.  The grid holds groups_per_cu groups per CU
 *     (default: 256 one-wavefront groups, about nine times what stays
 *     resident, so the dispatcher refills freed slots until the work runs
 *     out; fewer groups when the list has fewer items than that grid has
 *     wavefronts).  The list is dealt to the 8 XCDs in stripes of 256 items,
 *     round-robin, so that every XCD gets the same mix of meshes; each
 *     wavefront decodes one contiguous block of its XCD's stripes and exits.
 *     No atomics; dev_workspace may be NULL.
 *   k > 0: persistent.  The grid holds groups_per_cu groups per CU (meant
 *     to be about the resident count, e.g. 32 one-wavefront groups), and
 *     each wavefront claims k consecutive items at a time from a counter of
 *     its XCD's share of the list (the same stripes) until the share runs
 *     out.  The counters
 *     live in dev_workspace (device, 4-byte aligned, at least
 *     GTSR_BATCHED_WORKSPACE_BYTES bytes, caller-owned) and are zeroed by a
 *     small kernel enqueued in front of the decode, so calls that share a
 *     workspace must not overlap (one stream, or ordered streams).
 * The list should be balanced by strip triangles (gtsr_plan_batch) and have
 * many more items than the grid has wavefronts.  Same skipping rule as
 * decode_meshlets; items naming a mesh >= mesh_count are skipped.  Enqueued
 * on hip_stream; allocates nothing.  Errors: EINVAL (null or misaligned
 * pointer, bad cfg, workspace missing or too small for claiming, more than
 * 2^31 work items), EHIP. */
int decode_meshlets_batched(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                            const gtsr_work_item* dev_work, uint32_t work_items, void* dev_workspace,
                            uint64_t workspace_bytes, const gtsr_launch_cfg* cfg, void* hip_stream);

/* decode_meshlets_batched for a table whose entries all hold plain GTS
 * streams (bits = L/R words, bits_bytes a multiple of 8; reuse = index
 * bytes). */
int gtsr_decode_gts_batched(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                            const gtsr_work_item* dev_work, uint32_t work_items, void* dev_workspace,
                            uint64_t workspace_bytes, const gtsr_launch_cfg* cfg, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * decode_meshlets_batched in its claiming mode with the claim counters in a
 * static device array of the library's own instead of a caller workspace.
 * The array is GTSR_BATCHED_WORKSPACE_BYTES (1 KiB: one 32-bit counter per
 * XCD, one per 128-byte line), its size fixed whatever the input (the input
 * limits are those of decode_meshlets_batched: at most 2^31 work items), and
 * each device holds one copy until the process ends.  Its address is looked
 * up once per device, on the first call with that device current.  A small
 * kernel enqueued in front of the decode zeroes the counters, so each call
 * starts clean; calls that overlap on one device share the array and race,
 * so enqueue them on one stream (or ordered streams).  format:
 * GTSR_FORMAT_REUSE or GTSR_FORMAT_GTS; cfg as for decode_meshlets_batched
 * (NULL or items_per_claim 0 = 2 items per claim; groups_per_cu 0 = 32 /
 * waves_per_group).  Calls no hipMalloc, hipFree or other allocating
 * routine; enqueued on hip_stream.  Errors: as decode_meshlets_batched, and
 * EHIP if the array's address cannot be found. */
int gtsr_decode_batched_noalloc(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                                const gtsr_work_item* dev_work, uint32_t work_items, uint32_t format,
                                const gtsr_launch_cfg* cfg, void* hip_stream);

/* Capture one batched decode into an executable HIP graph once (its kernel
 * node, and with cfg->items_per_claim > 0 the counter-zeroing kernel node in
 * front of it); *graph_exec receives the handle.  format: GTSR_FORMAT_REUSE
 * (decode_meshlets_batched) or GTSR_FORMAT_GTS (gtsr_decode_gts_batched);
 * workspace as for those.  Captured on a stream of the library's own, so
 * the graph has no upstream dependency on the caller's stream: the launch
 * takes its stream in gtsr_graph_launch instead of here.  The tables and
 * the workspace must stay valid while the graph is used; their contents may
 * change between launches, their addresses and sizes may not.  Errors:
 * EINVAL, EHIP. */
int gtsr_batched_graph_create(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count,
                              const gtsr_work_item* dev_work, uint32_t work_items, void* dev_workspace,
                              uint64_t workspace_bytes, uint32_t format, const gtsr_launch_cfg* cfg,
                              void** graph_exec);

/* One measured launch shape of gtsr_autotune_batched (44 bytes). */
typedef struct gtsr_tune_point {
  uint32_t target_tris;       /* gtsr_autotune_batched: index of the candidate work list */
  uint32_t work_items;        /* items in that work list */
  gtsr_launch_cfg cfg;        /* waves_per_group, groups_per_cu, run_tris, items_per_claim */
  float median_ms, min_ms;    /* per launch, over the rounds of the last stage that measured it */
  uint32_t stage;             /* 1, or 2 for a finalist (measured again alone) */
  uint32_t reserved;
} gtsr_tune_point;

/* Pick the batched decoder's launch shape, LDS tile, launch mode and
 * work-list granularity by measurement (the paper decodes one meshlet per
 * workgroup and has no such knob).  format: GTSR_FORMAT_REUSE
 * (decode_meshlets_batched) or GTSR_FORMAT_GTS (gtsr_decode_gts_batched).
 * The caller passes n_works candidate work lists for the table, already on
 * the device (dev_works[i] of work_counts[i] items, typically
 * gtsr_plan_batch at different targets), and the candidates are every list
 * times every shape in cfgs[n_cfgs] (NULL or 0 = the built-in shapes:
 * static-split grids of 32 wavefronts per CU and 4, 8 and 16 times that,
 * each with run_tris 1280 and 1024, the 1280 ones for GTS-Reuse only; and,
 * when a workspace is given, persistent grids of 32 one-wavefront groups
 * per CU claiming 1, 2 or 4 items at a time with the default tile).
 * dev_workspace / workspace_bytes: as for decode_meshlets_batched, needed
 * by claiming shapes (may be NULL when no shape claims).  Protocol: every
 * candidate once untimed; a warm-up of back-to-back launches (about 60 ms
 * of device time); then reps rounds (0 = 5, at most 1000), each enqueuing
 * every candidate in turn, 4 launches each, with HIP events between
 * candidates and no host wait inside a stage, so the device never idles
 * while measuring; a candidate's figure is the median over rounds of its
 * per-launch time.  The finalists -- the 4 fastest, and any others within
 * 1.5 % of the fastest, at most 16 in all -- are measured again alone over
 * 3 * reps rounds; among them the first in candidate order (list-major) whose
 * median is within 1 % of the fastest is *best (target_tris holds its list
 * index).
 * points (may be NULL) receives up to capacity points, one per candidate in
 * candidate order (the finalists' figures from the second stage), and
 * *point_count (may be NULL) the number of candidates.  Synchronous:
 * returns after the last timed launch.  Allocates no device memory.  Every
 * launch decodes the whole table, so the table's outputs hold the decoded
 * meshes on return.  Errors: EINVAL (null argument, bad format, bad cfg),
 * EHIP. */
int gtsr_autotune_batched(const gtsr_mesh_entry* dev_mesh_table, uint32_t mesh_count, uint32_t format,
                          const gtsr_work_item* const* dev_works, const uint32_t* work_counts, uint32_t n_works,
                          void* dev_workspace, uint64_t workspace_bytes, const gtsr_launch_cfg* cfgs,
                          uint32_t n_cfgs, uint32_t reps, gtsr_tune_point* points, uint32_t capacity,
                          uint32_t* point_count, gtsr_tune_point* best, void* hip_stream);

/* ------------------------------------------------------------ serving */

/* A decode-request server over a device-resident pool of encoded meshes
 * (continuous batching; not in the paper, which decodes inside a renderer).
 * A scheduler thread admits requests first-come first-served while each one's
 * output (3 * strip_triangles bytes) fits into the output arena and a launch
 * slot is free; the requests admitted together go to the device as one
 * decode_meshlets_batched launch on the slot's own HIP stream, so up to
 * max_inflight batches decode at once and new requests join as slots and
 * arena space free up.  A request that does not fit blocks those behind it.
 * Outputs stay in the arena until gtsr_server_release. */
typedef struct gtsr_server gtsr_server;   /* opaque */

typedef struct gtsr_server_params {
  uint8_t* arena;            /* device memory for decoded outputs, caller-owned, 256-byte aligned */
  uint64_t arena_bytes;      /* the admission budget for outputs in flight or unreleased; each
                                output takes whole 256-byte units of it */
  uint32_t max_inflight;     /* batches on the device at once, 1..8 (0 = 4) */
  uint32_t max_batch;        /* requests per batch, 1..65536 (0 = 256) */
  uint32_t target_tris;      /* strip triangles per work item (0 = 768) */
  uint32_t max_items;        /* work items per batch, 1..2^26 (0 = 2^20); a mesh that
                                would need more is split into coarser items */
  gtsr_launch_cfg cfg;       /* launch shape of every batch (zeros = defaults) */
  uint32_t reserved;         /* must be 0 */
  uint32_t reserved2;
} gtsr_server_params;

/* One finished request.  Times are steady-clock nanoseconds: submitted,
 * admitted (arena space granted, batch formed), seen finished by the
 * scheduler. */
typedef struct gtsr_completion {
  uint64_t tag;              /* the caller's tag from gtsr_server_submit */
  uint32_t mesh;
  int32_t status;            /* GTSR_OK, or the error that failed the batch */
  uint64_t out_offset;       /* the output's byte offset in the arena */
  uint64_t out_bytes;        /* 3 * strip_triangles of the mesh */
  uint64_t t_submit_ns, t_admit_ns, t_done_ns;
} gtsr_completion;

typedef struct gtsr_server_stats {
  uint64_t submitted, completed, batches, max_batch_seen;
  uint64_t strip_triangles;  /* decoded by completed requests */
  uint64_t max_arena_used, arena_used, pending;
  uint64_t cancelled;        /* withdrawn by gtsr_server_cancel */
  uint64_t failed;           /* completed with an error status */
} gtsr_server_stats;

/* host_table: host copy of the pool's mesh table (device stream pointers;
 * the out field is ignored, outputs go to the arena); host_meshlets[i]: mesh
 * i's host descriptors (read during this call only, to plan its work items).
 * The pool's device arrays must outlive the server.  Creates max_inflight HIP
 * streams (default priority), pinned coherent host memory for max_batch table
 * rows and max_items work items per slot (the decode kernel reads a batch's
 * table and work list from there, with no copy), and the scheduler thread,
 * all on the current device.  Errors: EINVAL, ENOMEM, EHIP. */
int gtsr_server_create(const gtsr_mesh_entry* host_table, const gtsr_meshlet* const* host_meshlets,
                       uint32_t mesh_count, const gtsr_server_params* params, gtsr_server** server);

/* Queue a decode of mesh under a caller-chosen tag, unique among the
 * requests not yet released.  Thread-safe, returns at once.  Errors: EINVAL
 * (mesh out of range, tag in use), ELIMIT (the output, rounded up to whole
 * 256-byte units, can never fit the arena). */
int gtsr_server_submit(gtsr_server* server, uint32_t mesh, uint64_t tag);

/* Move up to capacity finished requests to out (oldest first) and their number
 * to *count; waits up to timeout_us microseconds for the first one.
 * Errors: EINVAL, EHIP (the scheduler thread could not start). */
int gtsr_server_poll(gtsr_server* server, gtsr_completion* out, uint32_t capacity, uint32_t* count,
                     uint32_t timeout_us);

/* Give a finished request's arena range back to the budget; the output may
 * be overwritten afterwards.  Errors: EINVAL (unknown tag, still decoding). */
int gtsr_server_release(gtsr_server* server, uint64_t tag);

/* Withdraw a request that has not been admitted yet: it leaves the queue, so
 * the requests behind it (which first-come first-served admission holds
 * back while it does not fit) may go ahead; poll reports it with status
 * ECANCELED and no output; its tag is free at once (no release).
 * Thread-safe.  Errors: EBUSY (already admitted: it completes normally and
 * is released as usual), EINVAL (no request with this tag). */
int gtsr_server_cancel(gtsr_server* server, uint64_t tag);

int gtsr_server_get_stats(gtsr_server* server, gtsr_server_stats* stats);

/* Client loop for open-loop measurement: submits request i (mesh meshes[i],
 * tag tag_base + i) at arrival_ns[i] nanoseconds (non-decreasing) after the
 * call starts (*start_ns receives the start, steady clock; may be NULL),
 * releases each output as soon as it finishes, and stores request i's
 * completion in out[i].  Returns when all n have finished.  Errors: those of
 * submit, poll and release; a failed decode returns its status. */
int gtsr_server_replay(gtsr_server* server, const uint64_t* arrival_ns, const uint32_t* meshes, uint32_t n,
                       uint64_t tag_base, gtsr_completion* out, uint64_t* start_ns);

/* Stop the scheduler, wait for batches on the device, free everything the
 * server allocated (not the arena). */
void gtsr_server_destroy(gtsr_server* server);

/* ------------------------------------------------------- .gtsr files */

/* A versioned container of encoded meshes, so that a pool is encoded once,
 * offline, and reloaded for decoding (the paper encodes in the asset
 * pipeline and decodes at run time, Sec. 1).  Layout (little-endian): a
 * 64-byte header (magic "GTSRFILE", version 1, mesh count, table and data
 * offsets, total size, 64-bit FNV-1a hash of everything after the header), a
 * 128-byte record per mesh (format, counts, sizes, the offset of each
 * array), then the arrays, each on a 16-byte boundary. */
typedef struct gtsr_file gtsr_file;   /* opaque: an opened, checked file in host memory */

/* One mesh as written to or read from a file: the encoder's host arrays.
 * Plain GTS (format GTSR_FORMAT_GTS) keeps its L/R words in bits and its
 * index bytes in reuse, as gtsr_gts_from_reuse writes them. */
typedef struct gtsr_file_mesh {
  uint32_t format;              /* GTSR_FORMAT_REUSE or GTSR_FORMAT_GTS */
  uint32_t meshlet_count;
  uint64_t strip_triangles, input_triangles, restarts;
  const gtsr_meshlet* meshlets; /* meshlet_count descriptors */
  const uint8_t* bits;
  uint64_t bits_bytes;
  const uint8_t* reuse;
  uint64_t reuse_bytes;
  const uint32_t* vertices;     /* local -> global vertex ids, meshlet after meshlet */
  uint64_t vertex_count;
  const uint64_t* vert_off;     /* meshlet_count + 1 entries */
  const uint32_t* kept_off;     /* meshlet_count + 1 entries, or NULL (not stored) */
  const uint32_t* tri_ids;      /* input_triangles entries, or NULL (not stored) */
} gtsr_file_mesh;

/* Write mesh_count meshes to path (host arrays, read during the call only;
 * kept_off and tri_ids may be NULL).  Each array must hold the entries its
 * field's comment names (sizes follow from the counts; the writer cannot
 * check them).  The streams themselves are written as given: gtsr_file_open
 * is where they are validated.  The file appears whole or not at all
 * (written under path + ".partial", then renamed).  Errors: EINVAL (null
 * argument or array, bad format), ENOMEM, EIO. */
int gtsr_file_write(const char* path, const gtsr_file_mesh* meshes, uint32_t mesh_count);

/* Read a whole file into host memory and check it: header, sizes and offsets
 * against the file, the hash, and every mesh against its format's stream
 * invariants (gtsr_validate for GTS-Reuse, Sec. 4.3) and its vertex and kept
 * offsets.  *file is set only on success.  Errors: EINVAL, ENOMEM, EIO (cannot
 * open or read), ECORRUPT (anything that does not check out). */
int gtsr_file_open(const char* path, gtsr_file** file);

int gtsr_file_mesh_count(const gtsr_file* file, uint32_t* count);

/* Mesh i of an opened file; the pointers point into the file's memory and stay
 * valid until gtsr_file_close.  Errors: EINVAL (null, index out of range). */
int gtsr_file_mesh_get(const gtsr_file* file, uint32_t i, gtsr_file_mesh* mesh);

void gtsr_file_close(gtsr_file* file);

/* ------------------------------------------------- vertex attributes */

/* Crack-free fixed-point quantization of per-vertex attributes (Sec. 4.4),
 * host side.  attrs: float32[vertex_count][channels]; the meshlets' vertex
 * lists verts[vert_off[m] .. vert_off[m+1]) (gtsr_encoded_view).  Per channel
 * the global grid spacing is w / (2^bits - 1), w the widest meshlet extent,
 * kept as the smallest float32 not below it (1 for a flat channel, widened
 * in 2^-20 relative steps if float64 rounding would let a meshlet span more
 * than 2^bits - 1 steps); origin = the channel minimum; a value's grid index
 * is floor((A - origin) / delta) in float64.  Outputs (caller-owned, host):
 * origin[channels], delta[channels], lowest int32[meshlet_count][channels]
 * (each meshlet's lowest grid value), offsets uint16[vert_off[M]][channels]
 * (grid value - lowest).  Errors: EINVAL (bits not 1..16, channels not
 * 1..64, null pointer, bad ids), ELIMIT (a grid value past 31 bits). */
int gtsr_quantize_attributes(const float* attrs, uint32_t vertex_count, uint32_t channels, const uint32_t* verts,
                             const uint64_t* vert_off, uint32_t meshlet_count, uint32_t bits, float* origin,
                             float* delta, int32_t* lowest, uint16_t* offsets);

/* Quantized attributes in device memory (gtsr_quantize_attributes' outputs
 * and the meshlets' vert_off, uint64[meshlet_count + 1]). */
typedef struct gtsr_attr_stream {
  const int32_t* lowest;
  const uint16_t* offsets;
  const uint64_t* vert_off;
  const float* origin;
  const float* delta;
  uint32_t meshlet_count;
  uint32_t channels;          /* 1..64 */
  uint64_t offset_count;      /* elements the offsets array holds (vert_off[M] * channels for a
                                 well-formed stream); no offset at or past it is read */
} gtsr_attr_stream;

/* Dequantize on the GPU: dev_out float32[vert_off[M]][channels] receives
 * (lowest + offset) * delta + origin per meshlet-local vertex and channel,
 * computed as one float64 fused multiply-add rounded to float32, so copies of
 * a vertex in different meshlets get identical bits.  out_count: elements the
 * output holds; meshlets whose range passes it or dev->offset_count (or whose
 * vert_off entries decrease) are skipped.  cfg (may be
 * NULL): waves_per_group 1..4, meshlets_per_wave.  Enqueued on hip_stream,
 * allocates nothing.  Errors: EINVAL, EHIP. */
int gtsr_dequantize(const gtsr_attr_stream* dev, float* dev_out, uint64_t out_count, const gtsr_launch_cfg* cfg,
                    void* hip_stream);

/* ------------------------------------------- bandwidth calibration */

/* Achievable HBM bandwidth for the decoders' traffic mix (not in the paper:
 * the yardstick the batched decode is measured against, beside the 8 TB/s
 * peak).  The decode reads about 0.24 of its bytes (descriptors, flag chunks,
 * reuse bytes; Sec. 4.2 / 4.3's streams) and writes 0.76 (Sec. 3's 3-byte
 * triples) with 16-byte loads and non-temporal 16-byte stores, each
 * wavefront walking contiguous blocks.  This kernel does that memory work
 * alone: *steps_out = min(src_bytes / 4096, dst_bytes / 13312) steps, each
 * reading 4 KiB of dev_src and writing 13 KiB of dev_dst (contiguous per
 * wavefront, XCD-major, loads one step ahead of the stores that use them).
 * Bytes moved per launch = 17408 * steps.  dev_dst receives values derived
 * from dev_src (no meaning).  cfg (may be NULL): waves_per_group 1..16 (0 =
 * 1), groups_per_cu 1..1024 (0 = 256); meshlets_per_wave and run_tris must
 * be 0.  Both buffers 16-byte aligned, device memory.  Enqueued on
 * hip_stream, allocates nothing.  Errors: EINVAL, ELIMIT (more than 2^32-1
 * steps, or over 2 GiB of dst per wavefront), EHIP. */
int gtsr_stream_calib(const uint8_t* dev_src, uint64_t src_bytes, uint8_t* dev_dst, uint64_t dst_bytes,
                      const gtsr_launch_cfg* cfg, uint64_t* steps_out, void* hip_stream);

/* Enqueue a captured graph on hip_stream.  Errors: EINVAL, EHIP. */
int gtsr_graph_launch(void* graph_exec, void* hip_stream);

void gtsr_graph_destroy(void* graph_exec);

/* Compute units of the current device, as the decoders size their
 * grids.  Returns 0 on error. */
uint32_t gtsr_device_cu_count(void);

/* Message for the last non-OK return on the calling thread ("" if none). */
const char* gtsr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GTSR_H */
