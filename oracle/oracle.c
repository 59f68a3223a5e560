/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU reference for the GTS-Reuse meshlet
 * connectivity codec of "Towards Practical Meshlet Compression" (Kuth et al.,
 * VMV 2024).  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load this file's library.  The product library never links it, and
 * this file includes none of the product's headers: it parses the stream
 * layout from bytes on its own.
 *
 * What it computes (paper section / equation it follows):
 *
 *   oracle_decode        Sec. 4.2 "Strip Encoding" and Sec. 2 (definition of a
 *                        generalized triangle strip: a path enters a triangle
 *                        (A,B,C) through (A,B) and leaves across the right edge
 *                        (B,C) or the left edge (C,A), chosen by one L/R flag
 *                        per triangle), plus Sec. 4.3 "Index Reuse Packing"
 *                        (new vertices appear in ascending order starting with
 *                        0,1,2; a set increment flag means "next new vertex",
 *                        a clear one means "next entry of the reuse array").
 *                        Implemented as the sequential strip walk, one
 *                        triangle after the other.  The data-parallel closed
 *                        form (flip search + prefix count, reuse read at
 *                        t+1-s) is NOT used here; the tests pin this walk
 *                        against that closed form, written separately.
 *
 *   oracle_encode        Sec. 3 (meshlets bounded by max vertices / max
 *                        triangles), Sec. 4.2 (strips, restarts as four
 *                        degenerate triangles, split of a meshlet whose strip
 *                        exceeds the triangle limit), Sec. 4.3 (vertex
 *                        renumbering by first appearance).  The paper builds
 *                        meshlets with a third-party library and optimal
 *                        strips with a MILP; here both are replaced by a
 *                        documented greedy rule (the same rule the product
 *                        encoder implements, so the two streams can be
 *                        compared byte for byte).  Meshlet and restart counts
 *                        versus the paper's meshes: parity unpinned.
 *
 *   oracle_check_stream  Structural validity of a stream (counts, contiguous
 *                        offsets, zero padding bits, increment total, reuse
 *                        entries referring to already-introduced vertices).
 *
 *   oracle_gts_decode    The plain GTS variant of Sec. 4.2 / Fig. "Strip
 *                        Encoding" (c): the same L/R flags, but every strip
 *                        triangle t >= 1 stores the local index it adds as
 *                        one byte (0,1,2 of the first triangle implicit).
 *                        Same sequential walk as oracle_decode.
 *   oracle_gts_from_reuse  Re-encodes a GTS-Reuse stream as plain GTS: walks
 *                        each meshlet's index stream and writes it out.
 *   oracle_quantize      Sec. 4.4 "Crack-Free Fixed-Point Vertex Attribute
 *   oracle_dequantize    Quantization": per channel, the largest meshlet extent
 *                        w sets the global grid spacing w / (2^b - 1); every
 *                        value is put on that grid, each meshlet stores its
 *                        lowest grid value L and b-bit offsets from it;
 *                        decoding adds L back and maps the grid value to
 *                        floating point.
 *   oracle_min_strips    The fewest strips (restarts + 1) that cover a small
 *                        triangle set (Sec. 3.1, the optimal GTS): any
 *                        simple path of neighbouring triangles is a strip,
 *                        so the answer is T minus the most neighbour pairs
 *                        that can be chained with no triangle in three pairs
 *                        (no fork) and no cycle; found by trying every subset
 *                        of pairs (brute force, tiny inputs only).
 *   oracle_cones         Sec. 3 (cone culling in the amplification shader):
 *   oracle_cull          per meshlet, the cone around the normalised sum of
 *                        its triangles' unit normals that holds all of them;
 *                        a meshlet is culled for view direction d when the
 *                        whole cone faces away from d.  The paper fixes no
 *                        rounding; this one takes the triangles in strip
 *                        order, each rotated to start at its smallest vertex
 *                        id, in float64, rounded once to float32.
 *   oracle_compact       Drops the degenerate triangles of the restarts
 *                        (Sec. 4.2: four per restart; they are the only
 *                        triangles with a repeated index) from decoded
 *                        triples, keeping order; reports each meshlet's
 *                        offset among the kept triangles.
 *
 * Stream layout parsed here (all little-endian):
 *   descriptor, 16 bytes per meshlet:
 *     u32 chunk_off   first 16-byte flag chunk of the meshlet
 *     u32 reuse_off   first reuse byte of the meshlet
 *     u32 out_off     first output triangle of the meshlet
 *     u16 tri_count   strip triangles T_s (degenerates included), 1..256
 *     u16 vert_count  meshlet vertices V, 3..256
 *   flag chunk, 16 bytes per 64 strip triangles: u64 LR, u64 INC;
 *     bit i of chunk c belongs to strip triangle 64c+i; LR bit 1 = R, 0 = L;
 *     INC bit 1 = new vertex.  Triangle 0 has no INC bit (stored 0).
 *   reuse: one byte per reused index, meshlet by meshlet.
 *   output: 3 bytes per strip triangle at byte 3*(out_off + t).
 * Plain GTS stream layout:
 *   descriptor, 16 bytes: u32 word_off (first 8-byte L/R word), u32 index_off
 *     (first index byte), u32 out_off, u16 tri_count, u16 vert_count;
 *   L/R words, 8 bytes per 64 strip triangles (bit i of word w belongs to
 *     strip triangle 64w+i, 1 = R); bits past T_s are 0;
 *   index bytes, T_s - 1 per meshlet: the vertex each triangle t >= 1 adds.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_EDEGENERATE (-3)
#define OR_ELIMIT (-4)
#define OR_ECORRUPT (-5)

#define FLAG_L 0
#define FLAG_R 1

/* ------------------------------------------------------------------ bytes */

static uint32_t rd_u16(const uint8_t* p) { return (uint32_t)p[0] | ((uint32_t)p[1] << 8); }
static uint32_t rd_u32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static uint64_t rd_u64(const uint8_t* p) {
  return (uint64_t)rd_u32(p) | ((uint64_t)rd_u32(p + 4) << 32);
}
static void wr_u16(uint8_t* p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void wr_u32(uint8_t* p, uint32_t v) {
  p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}

/* One strip triangle's L/R flag and increment flag, read bit by bit. */
static int flag_lr(const uint8_t* bits, uint32_t chunk_off, uint32_t t) {
  uint64_t w = rd_u64(bits + 16ull * (chunk_off + t / 64));
  return (int)((w >> (t % 64)) & 1u);
}
static int flag_inc(const uint8_t* bits, uint32_t chunk_off, uint32_t t) {
  uint64_t w = rd_u64(bits + 16ull * (chunk_off + t / 64) + 8);
  return (int)((w >> (t % 64)) & 1u);
}

/* ----------------------------------------------------------------- decode */

/*
 * Decode one meshlet by walking its strip (Sec. 2 and Sec. 4.2 / 4.3).
 *
 * The first triangle is the implicit (0,1,2) of Sec. 4.3; its own flag picks
 * its orientation: L keeps (0,1,2), R gives (1,0,2).  Every later triangle
 * enters across an edge of its predecessor (A,B,C): flag R = across the right
 * edge (B,C), so it starts (C,B,...); flag L = across the left edge (C,A), so
 * it starts (A,C,...).  Its third vertex is the next new vertex (counting up
 * from 3) when its increment flag is set, otherwise the next reuse byte.
 */
int oracle_decode_meshlet(const uint8_t* desc16, const uint8_t* bits, uint64_t bits_bytes,
                          const uint8_t* reuse, uint64_t reuse_bytes,
                          uint8_t* out, uint64_t out_bytes) {
  uint32_t chunk_off = rd_u32(desc16 + 0);
  uint32_t reuse_off = rd_u32(desc16 + 4);
  uint32_t out_off = rd_u32(desc16 + 8);
  uint32_t T = rd_u16(desc16 + 12);
  uint32_t V = rd_u16(desc16 + 14);
  if (T < 1 || T > 256 || V < 3 || V > 256) return OR_ECORRUPT;
  uint64_t nchunks = (T + 63) / 64;
  if (16ull * (chunk_off + nchunks) > bits_bytes) return OR_ECORRUPT;
  if (3ull * ((uint64_t)out_off + T) > out_bytes) return OR_EINVAL;

  uint32_t A, B, C;
  if (flag_lr(bits, chunk_off, 0) == FLAG_L) { A = 0; B = 1; } else { A = 1; B = 0; }
  C = 2;
  uint8_t* o = out + 3ull * out_off;
  o[0] = (uint8_t)A; o[1] = (uint8_t)B; o[2] = (uint8_t)C;

  uint32_t next_new = 3;      /* id the next incremented vertex receives */
  uint64_t next_reuse = reuse_off;
  for (uint32_t t = 1; t < T; ++t) {
    uint32_t D;
    if (flag_inc(bits, chunk_off, t)) {
      D = next_new++;
    } else {
      if (next_reuse >= reuse_bytes) return OR_ECORRUPT;
      D = reuse[next_reuse++];
    }
    if (flag_lr(bits, chunk_off, t) == FLAG_R) { A = C; /* B stays */ }
    else { /* A stays */ B = C; }
    C = D;
    o[3 * t + 0] = (uint8_t)A; o[3 * t + 1] = (uint8_t)B; o[3 * t + 2] = (uint8_t)C;
  }
  return OR_OK;
}

/* Decode meshlets [m0, m1) of a stream.  Returns the first error, else OK. */
int oracle_decode_range(const uint8_t* desc, uint32_t m0, uint32_t m1,
                        const uint8_t* bits, uint64_t bits_bytes,
                        const uint8_t* reuse, uint64_t reuse_bytes,
                        uint8_t* out, uint64_t out_bytes) {
  for (uint32_t m = m0; m < m1; ++m) {
    int rc = oracle_decode_meshlet(desc + 16ull * m, bits, bits_bytes, reuse, reuse_bytes, out, out_bytes);
    if (rc != OR_OK) return rc;
  }
  return OR_OK;
}

int oracle_decode(const uint8_t* desc, uint32_t meshlet_count,
                  const uint8_t* bits, uint64_t bits_bytes,
                  const uint8_t* reuse, uint64_t reuse_bytes,
                  uint8_t* out, uint64_t out_bytes) {
  return oracle_decode_range(desc, 0, meshlet_count, bits, bits_bytes, reuse, reuse_bytes, out, out_bytes);
}

/* ------------------------------------------------------------ stream check */

/*
 * Structural validity of a stream: per-meshlet counts in range, offsets
 * contiguous from 0 in meshlet order, array sizes equal to the totals,
 * triangle 0's increment bit and every bit past T_s clear, the increment
 * total equal to V-3 (vertices 0,1,2 are implicit, Sec. 4.3), and every reuse
 * byte naming a vertex already introduced at that point of the strip.
 */
int oracle_check_stream(const uint8_t* desc, uint32_t meshlet_count,
                        const uint8_t* bits, uint64_t bits_bytes,
                        const uint8_t* reuse, uint64_t reuse_bytes,
                        uint64_t strip_triangles) {
  uint64_t chunk = 0, rpos = 0, opos = 0;
  for (uint32_t m = 0; m < meshlet_count; ++m) {
    const uint8_t* d = desc + 16ull * m;
    uint32_t chunk_off = rd_u32(d), reuse_off = rd_u32(d + 4), out_off = rd_u32(d + 8);
    uint32_t T = rd_u16(d + 12), V = rd_u16(d + 14);
    if (T < 1 || T > 256 || V < 3 || V > 256 || V > T + 2) return OR_ECORRUPT;
    if (chunk_off != chunk || reuse_off != rpos || out_off != opos) return OR_ECORRUPT;
    uint32_t nch = (T + 63) / 64;
    if (16ull * (chunk + nch) > bits_bytes) return OR_ECORRUPT;
    uint32_t n_ru = T + 2 - V;
    if (rpos + n_ru > reuse_bytes) return OR_ECORRUPT;
    for (uint32_t t = T; t < 64 * nch; ++t)
      if (flag_lr(bits, chunk_off, t) || flag_inc(bits, chunk_off, t)) return OR_ECORRUPT;
    if (flag_inc(bits, chunk_off, 0)) return OR_ECORRUPT;
    uint32_t newest = 2, used = 0;
    for (uint32_t t = 1; t < T; ++t) {
      if (flag_inc(bits, chunk_off, t)) {
        ++newest;
      } else {
        if (used >= n_ru) return OR_ECORRUPT;
        if (reuse[rpos + used] > newest) return OR_ECORRUPT;
        ++used;
      }
    }
    if (newest + 1 != V || used != n_ru) return OR_ECORRUPT;
    chunk += nch; rpos += n_ru; opos += T;
  }
  if (16ull * chunk != bits_bytes || rpos != reuse_bytes || opos != strip_triangles) return OR_ECORRUPT;
  return OR_OK;
}

/* -------------------------------------------------------------- plain GTS */

static int gts_flag(const uint8_t* words, uint32_t word_off, uint32_t t) {
  uint64_t w = rd_u64(words + 8ull * (word_off + t / 64));
  return (int)((w >> (t % 64)) & 1u);
}

/*
 * Decode a plain GTS stream by the strip walk of Sec. 2 / 4.2: the first
 * triangle is (0,1,2) oriented by its flag; every later one keeps the edge
 * its flag names and adds the vertex its index byte gives.
 */
int oracle_gts_decode(const uint8_t* desc, uint32_t meshlet_count,
                      const uint8_t* words, uint64_t words_bytes,
                      const uint8_t* index, uint64_t index_bytes,
                      uint8_t* out, uint64_t out_bytes) {
  for (uint32_t m = 0; m < meshlet_count; ++m) {
    const uint8_t* d = desc + 16ull * m;
    uint32_t word_off = rd_u32(d), index_off = rd_u32(d + 4), out_off = rd_u32(d + 8);
    uint32_t T = rd_u16(d + 12), V = rd_u16(d + 14);
    if (T < 1 || T > 256 || V < 3 || V > 256) return OR_ECORRUPT;
    if (8ull * (word_off + (T + 63) / 64) > words_bytes) return OR_ECORRUPT;
    if ((uint64_t)index_off + T - 1 > index_bytes) return OR_ECORRUPT;
    if (3ull * ((uint64_t)out_off + T) > out_bytes) return OR_EINVAL;
    uint32_t A, B, C;
    if (gts_flag(words, word_off, 0) == FLAG_L) { A = 0; B = 1; } else { A = 1; B = 0; }
    C = 2;
    uint8_t* o = out + 3ull * out_off;
    o[0] = (uint8_t)A; o[1] = (uint8_t)B; o[2] = (uint8_t)C;
    for (uint32_t t = 1; t < T; ++t) {
      uint32_t D = index[index_off + t - 1];
      if (gts_flag(words, word_off, t) == FLAG_R) { A = C; } else { B = C; }
      C = D;
      o[3 * t + 0] = (uint8_t)A; o[3 * t + 1] = (uint8_t)B; o[3 * t + 2] = (uint8_t)C;
    }
  }
  return OR_OK;
}

/*
 * Plain GTS from GTS-Reuse: the same flags (the L/R word of every 16-byte
 * chunk) and, per meshlet, the index stream I[3..T_s+1] that the reuse walk
 * produces (next new vertex for a set increment flag, else the next reuse
 * byte).  gdesc: 16 * meshlet_count bytes; words: 8 * chunks bytes; index:
 * sum of (T_s - 1) bytes; each capacity is checked.
 */
int oracle_gts_from_reuse(const uint8_t* desc, uint32_t meshlet_count,
                          const uint8_t* bits, uint64_t bits_bytes,
                          const uint8_t* reuse, uint64_t reuse_bytes,
                          uint8_t* gdesc, uint8_t* words, uint64_t words_cap,
                          uint8_t* index, uint64_t index_cap) {
  uint64_t ipos = 0;
  for (uint32_t m = 0; m < meshlet_count; ++m) {
    const uint8_t* d = desc + 16ull * m;
    uint32_t chunk_off = rd_u32(d), reuse_off = rd_u32(d + 4), out_off = rd_u32(d + 8);
    uint32_t T = rd_u16(d + 12), V = rd_u16(d + 14);
    if (T < 1 || T > 256 || V < 3 || V > 256) return OR_ECORRUPT;
    uint32_t nch = (T + 63) / 64;
    if (16ull * (chunk_off + nch) > bits_bytes) return OR_ECORRUPT;
    if (8ull * (chunk_off + nch) > words_cap || ipos + T - 1 > index_cap) return OR_EINVAL;
    for (uint32_t c = 0; c < nch; ++c)
      memcpy(words + 8ull * (chunk_off + c), bits + 16ull * (chunk_off + c), 8);
    uint8_t* g = gdesc + 16ull * m;
    wr_u32(g, chunk_off); wr_u32(g + 4, (uint32_t)ipos); wr_u32(g + 8, out_off);
    wr_u16(g + 12, T); wr_u16(g + 14, V);
    uint32_t next_new = 3;
    uint64_t next_reuse = reuse_off;
    for (uint32_t t = 1; t < T; ++t) {
      uint32_t D;
      if (flag_inc(bits, chunk_off, t)) {
        D = next_new++;
      } else {
        if (next_reuse >= reuse_bytes) return OR_ECORRUPT;
        D = reuse[next_reuse++];
      }
      index[ipos++] = (uint8_t)D;
    }
  }
  return OR_OK;
}

/*
 * Keep the triples of `tris` (n of them) that name three different
 * vertices, in order, at out (capacity out_cap triples); *kept receives their
 * number.  If desc is not NULL, offsets[m] (m = 0..meshlet_count) receives
 * the number of kept triples before meshlet m's first output triangle.
 */
int oracle_compact(const uint8_t* tris, uint64_t n, uint8_t* out, uint64_t out_cap, uint64_t* kept,
                   const uint8_t* desc, uint32_t meshlet_count, uint64_t* offsets) {
  uint64_t k = 0;
  uint32_t m = 0;
  for (uint64_t t = 0; t < n; ++t) {
    while (desc && m < meshlet_count && rd_u32(desc + 16ull * m + 8) == t) offsets[m++] = k;
    const uint8_t* a = tris + 3 * t;
    if (a[0] == a[1] || a[1] == a[2] || a[0] == a[2]) continue;
    if (k >= out_cap) return OR_EINVAL;
    memcpy(out + 3 * k, a, 3);
    ++k;
  }
  while (desc && m < meshlet_count) offsets[m++] = k;
  if (desc) offsets[meshlet_count] = k;
  *kept = k;
  return OR_OK;
}

/* ----------------------------------------------------- attribute quantization */

#include <math.h>

/*
 * Crack-free fixed-point quantization (Sec. 4.4), channel by channel:
 *   w      = largest extent (max - min) of the channel over any one meshlet;
 *   delta  = w / (2^b - 1), taken as the smallest float32 not below it (1 if
 *            w = 0), widened by 2^-20 relative steps while some meshlet's
 *            grid values would still span more than 2^b - 1;
 *   origin = the channel's minimum over all vertices (a float32 value);
 *   G(v)   = floor((A(v) - origin) / delta), in float64: the vertex's value
 *            on the global grid, the same in every meshlet that holds it;
 *   L      = the lowest G in a meshlet; q = G - L in [0, 2^b - 1].
 * Inputs: attrs float32[nverts][n]; the meshlets' local vertex lists
 * verts[vert_off[m] .. vert_off[m+1]).  Outputs: origin[n], delta[n],
 * L int32[M][n], q uint16[sum V][n] (b <= 16).  ELIMIT if a grid value does
 * not fit 31 bits.
 */
int oracle_quantize(const float* attrs, uint32_t nverts, uint32_t n, const uint32_t* verts,
                    const uint64_t* vert_off, uint32_t M, uint32_t b,
                    float* origin, float* delta, int32_t* L, uint16_t* q) {
  if (b < 1 || b > 16 || n == 0) return OR_EINVAL;
  const double top = (double)((1u << b) - 1);
  for (uint32_t i = 0; i < n; ++i) {
    float lo = INFINITY;
    for (uint32_t v = 0; v < nverts; ++v) if (attrs[(uint64_t)v * n + i] < lo) lo = attrs[(uint64_t)v * n + i];
    if (nverts == 0) lo = 0.0f;
    double w = 0.0;
    for (uint32_t m = 0; m < M; ++m) {
      float a = INFINITY, z = -INFINITY;
      for (uint64_t k = vert_off[m]; k < vert_off[m + 1]; ++k) {
        float x = attrs[(uint64_t)verts[k] * n + i];
        if (x < a) a = x;
        if (x > z) z = x;
      }
      if (vert_off[m + 1] > vert_off[m] && (double)z - (double)a > w) w = (double)z - (double)a;
    }
    float d = 1.0f;
    if (w > 0.0) {
      d = (float)(w / top);
      if ((double)d < w / top) d = nextafterf(d, INFINITY);
    }
    for (;;) {
      int fits = 1;
      for (uint32_t m = 0; m < M && fits; ++m) {
        double gmin = INFINITY, gmax = -INFINITY;
        for (uint64_t k = vert_off[m]; k < vert_off[m + 1]; ++k) {
          double g = floor(((double)attrs[(uint64_t)verts[k] * n + i] - (double)lo) / (double)d);
          if (g < gmin) gmin = g;
          if (g > gmax) gmax = g;
        }
        if (gmax >= 2147483647.0) return OR_ELIMIT;
        if (vert_off[m + 1] > vert_off[m] && gmax - gmin > top) fits = 0;
      }
      if (fits) break;
      d = (float)((double)d * (1.0 + 1.0 / 1048576.0));
    }
    origin[i] = lo;
    delta[i] = d;
    for (uint32_t m = 0; m < M; ++m) {
      double gmin = INFINITY;
      for (uint64_t k = vert_off[m]; k < vert_off[m + 1]; ++k) {
        double g = floor(((double)attrs[(uint64_t)verts[k] * n + i] - (double)lo) / (double)d);
        if (g < gmin) gmin = g;
      }
      int32_t Lm = vert_off[m + 1] > vert_off[m] ? (int32_t)gmin : 0;
      L[(uint64_t)m * n + i] = Lm;
      for (uint64_t k = vert_off[m]; k < vert_off[m + 1]; ++k) {
        double g = floor(((double)attrs[(uint64_t)verts[k] * n + i] - (double)lo) / (double)d);
        q[k * n + i] = (uint16_t)((int64_t)g - Lm);
      }
    }
  }
  return OR_OK;
}

/*
 * Decode: the grid value L + q of every meshlet-local vertex, mapped back as
 * (L + q) * delta + origin with one float64 fused multiply-add, rounded to
 * float32 (a function of the grid value alone, so every copy of a vertex
 * gets the same bits).  out float32[sum V][n].
 */
int oracle_dequantize(const int32_t* L, const uint16_t* q, const uint64_t* vert_off, uint32_t M, uint32_t n,
                      const float* origin, const float* delta, float* out) {
  for (uint32_t m = 0; m < M; ++m)
    for (uint64_t k = vert_off[m]; k < vert_off[m + 1]; ++k)
      for (uint32_t i = 0; i < n; ++i) {
        int64_t g = (int64_t)L[(uint64_t)m * n + i] + q[k * n + i];
        out[k * n + i] = (float)fma((double)g, (double)delta[i], (double)origin[i]);
      }
  return OR_OK;
}

/* ------------------------------------------------------------ cone culling */

/*
 * Cones from decoded meshlets: the triangles of meshlet m are its decoded
 * triples (restart degenerates, which repeat a vertex, dropped) mapped through
 * its vertex list to global vertex ids, in strip order.  Each triangle is
 * rotated (orientation kept) to start at its smallest global id, and its unit
 * normal is (p1-p0) x (p2-p0) normalised (zero-area triangles ignored), with
 * positions float32[nverts][3] and float64 arithmetic; axis = the normalised
 * sum of the unit normals in strip order; cos_min = the smallest
 * dot(axis, n).  Output per meshlet {axis x, y, z, cutoff} in float32 with
 * cutoff = sqrt(max(0, 1 - cos_min^2)) + 1e-5 (sin of the half-angle plus a
 * rounding margin), or 2 when cos_min <= 0 or the normals cancel (the cone
 * is a half-space or more: never culled).  The rotation fixes the rounding of
 * each normal, so any construction that takes the same triangles in the same
 * order gets the same bits.
 */
int oracle_cones(const uint8_t* desc, uint32_t meshlet_count, const uint8_t* decoded,
                 const uint32_t* verts, const uint64_t* vert_off, const float* pos, uint32_t nverts,
                 float* cones) {
  for (uint32_t m = 0; m < meshlet_count; ++m) {
    const uint8_t* d = desc + 16ull * m;
    uint32_t out_off = rd_u32(d + 8), T = rd_u16(d + 12);
    double sum[3] = {0, 0, 0};
    double* un = (double*)malloc(sizeof(double) * 3 * (T ? T : 1));
    if (!un) return OR_ENOMEM;
    uint32_t nu = 0;
    for (uint32_t t = 0; t < T; ++t) {
      const uint8_t* x = decoded + 3ull * (out_off + t);
      if (x[0] == x[1] || x[1] == x[2] || x[0] == x[2]) continue;
      uint32_t g[3];
      for (int c = 0; c < 3; ++c) {
        uint64_t k = vert_off[m] + x[c];
        if (k >= vert_off[m + 1]) { free(un); return OR_ECORRUPT; }
        g[c] = verts[k];
        if (g[c] >= nverts) { free(un); return OR_EINVAL; }
      }
      /* start at the smallest id, same cyclic order */
      int r = g[1] < g[0] ? (g[2] < g[1] ? 2 : 1) : (g[2] < g[0] ? 2 : 0);
      double p[3][3];
      for (int c = 0; c < 3; ++c)
        for (int j = 0; j < 3; ++j) p[c][j] = pos[3ull * g[(c + r) % 3] + j];
      double a[3] = {p[1][0] - p[0][0], p[1][1] - p[0][1], p[1][2] - p[0][2]};
      double b[3] = {p[2][0] - p[0][0], p[2][1] - p[0][1], p[2][2] - p[0][2]};
      double n[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
      double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      if (len == 0.0) continue;
      for (int j = 0; j < 3; ++j) { un[3 * nu + j] = n[j] / len; sum[j] += n[j] / len; }
      ++nu;
    }
    double sl = sqrt(sum[0] * sum[0] + sum[1] * sum[1] + sum[2] * sum[2]);
    float* o = cones + 4ull * m;
    if (nu == 0 || sl == 0.0) {
      o[0] = o[1] = o[2] = 0.0f; o[3] = 2.0f;
    } else {
      double ax[3] = {sum[0] / sl, sum[1] / sl, sum[2] / sl};
      double cmin = 1.0;
      for (uint32_t i = 0; i < nu; ++i) {
        double c = ax[0] * un[3 * i] + ax[1] * un[3 * i + 1] + ax[2] * un[3 * i + 2];
        if (c < cmin) cmin = c;
      }
      o[0] = (float)ax[0]; o[1] = (float)ax[1]; o[2] = (float)ax[2];
      o[3] = cmin <= 0.0 ? 2.0f : (float)(sqrt(fmax(0.0, 1.0 - cmin * cmin)) + 1e-5);
    }
    free(un);
  }
  return OR_OK;
}

/* Culling decision for view direction v: culled[m] = 1 when
 * fmaf(az, vz, fmaf(ay, vy, ax * vx)) > cutoff, computed in float32. */
int oracle_cull(const float* cones, uint32_t meshlet_count, float vx, float vy, float vz, uint8_t* culled) {
  for (uint32_t m = 0; m < meshlet_count; ++m) {
    const float* c = cones + 4ull * m;
    float dot = fmaf(c[2], vz, fmaf(c[1], vy, c[0] * vx));
    culled[m] = dot > c[3];
  }
  return OR_OK;
}

/* ----------------------------------------------------------------- encode */

typedef struct {
  uint32_t meshlets;
  uint8_t* desc;   uint64_t desc_cap;
  uint8_t* bits;   uint64_t bits_bytes, bits_cap;
  uint8_t* reuse;  uint64_t reuse_bytes, reuse_cap;
  uint32_t* verts; uint64_t verts_len, verts_cap;
  uint64_t* vert_off; uint64_t vert_off_cap;
  uint64_t input_triangles, strip_triangles, restarts, reuse_count, split_meshlets;
  uint64_t payload_bits, stored_bytes;
} oracle_enc;

static int grow(void** p, uint64_t* cap, uint64_t need, uint64_t elem) {
  if (need <= *cap) return 0;
  uint64_t nc = *cap ? *cap : 64;
  while (nc < need) nc *= 2;
  void* q = realloc(*p, nc * elem);
  if (!q) return -1;
  memset((uint8_t*)q + *cap * elem, 0, (nc - *cap) * elem);
  *p = q; *cap = nc;
  return 0;
}

void oracle_enc_free(oracle_enc* e) {
  if (!e) return;
  free(e->desc); free(e->bits); free(e->reuse); free(e->verts); free(e->vert_off);
  free(e);
}

/* Half-edge record used to find each triangle's neighbour across each edge. */
typedef struct { uint32_t lo, hi, tri; uint8_t edge, forward; } half_edge;

static int he_cmp(const void* a, const void* b) {
  const half_edge* x = (const half_edge*)a; const half_edge* y = (const half_edge*)b;
  if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
  if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
  if (x->tri != y->tri) return x->tri < y->tri ? -1 : 1;
  return (int)x->edge - (int)y->edge;
}

/*
 * Edge e of triangle (v0,v1,v2) runs from v_e to v_{e+1 mod 3}.  Two triangles
 * are neighbours across an edge only when exactly two triangles use that edge
 * and they traverse it in opposite directions (a consistently oriented
 * 2-manifold edge, the situation Sec. 3 assumes for meshlets).  nbr[3t+e] is
 * the neighbouring triangle or -1, nbr_edge[3t+e] the neighbour's own index of
 * that edge.
 */
static int build_adjacency(const uint32_t* tri, uint64_t T, int64_t* nbr, uint8_t* nbr_edge) {
  half_edge* he = (half_edge*)malloc(sizeof(half_edge) * 3 * (T ? T : 1));
  if (!he) return OR_ENOMEM;
  for (uint64_t t = 0; t < T; ++t)
    for (int e = 0; e < 3; ++e) {
      uint32_t a = tri[3 * t + e], b = tri[3 * t + (e + 1) % 3];
      half_edge* h = &he[3 * t + e];
      h->lo = a < b ? a : b; h->hi = a < b ? b : a;
      h->tri = (uint32_t)t; h->edge = (uint8_t)e; h->forward = a < b;
      nbr[3 * t + e] = -1; nbr_edge[3 * t + e] = 0;
    }
  qsort(he, 3 * T, sizeof(half_edge), he_cmp);
  uint64_t i = 0;
  while (i < 3 * T) {
    uint64_t j = i;
    while (j < 3 * T && he[j].lo == he[i].lo && he[j].hi == he[i].hi) ++j;
    if (j - i == 2 && he[i].forward != he[i + 1].forward) {
      half_edge* x = &he[i]; half_edge* y = &he[i + 1];
      nbr[3ull * x->tri + x->edge] = y->tri; nbr_edge[3ull * x->tri + x->edge] = y->edge;
      nbr[3ull * y->tri + y->edge] = x->tri; nbr_edge[3ull * y->tri + y->edge] = x->edge;
    }
    i = j;
  }
  free(he);
  return OR_OK;
}

/*
 * Brute-force optimum for tiny inputs (T <= 16, at most 24 neighbour pairs):
 * every subset of neighbour pairs is tried; a subset is a set of strips when
 * no triangle is in more than two of its pairs and it closes no cycle; the
 * fewest strips is T minus the largest such subset.
 */
int oracle_min_strips(const uint32_t* tri, uint32_t T, uint32_t* min_strips) {
  if (T > 16) return OR_ELIMIT;
  if (T == 0) { *min_strips = 0; return OR_OK; }
  int64_t nbr[48];
  uint8_t nbr_edge[48];
  int rc = build_adjacency(tri, T, nbr, nbr_edge);
  if (rc != OR_OK) return rc;
  uint32_t ea[24], eb[24], E = 0;
  for (uint32_t t = 0; t < T; ++t)
    for (int e = 0; e < 3; ++e)
      if (nbr[3 * t + e] > (int64_t)t) {
        if (E == 24) return OR_ELIMIT;
        ea[E] = t; eb[E] = (uint32_t)nbr[3 * t + e]; ++E;
      }
  uint32_t best = 0;
  for (uint32_t mask = 0; mask < (1u << E); ++mask) {
    uint32_t cnt = (uint32_t)__builtin_popcount(mask);
    if (cnt <= best) continue;
    uint32_t deg[16] = {0}, parent[16];
    for (uint32_t t = 0; t < T; ++t) parent[t] = t;
    int ok = 1;
    for (uint32_t k = 0; k < E && ok; ++k) {
      if (!(mask >> k & 1u)) continue;
      if (++deg[ea[k]] > 2 || ++deg[eb[k]] > 2) { ok = 0; break; }
      uint32_t a = ea[k], b = eb[k];
      while (parent[a] != a) a = parent[a];
      while (parent[b] != b) b = parent[b];
      if (a == b) ok = 0;          /* would close a cycle */
      else parent[a] = b;
    }
    if (ok) best = cnt;
  }
  *min_strips = T - best;
  return OR_OK;
}

/*
 * A strip is a path through the mesh's neighbour relation: triangles tri[0..len)
 * (global numbers) and, for each but the last, the edge index (0..2, in that
 * triangle's own vertex order) through which the path leaves it.  Any simple
 * path is a valid generalized strip (Sec. 2): each triangle is entered
 * through one edge and left through one of the two others.
 */
typedef struct { uint32_t* tri; uint8_t* exit; uint32_t len; } strip;

/* Appends one meshlet made of strips s[0..n) to the stream. */
static int emit_part(oracle_enc* E, const uint32_t* tri, const uint8_t* nbr_edge,
                     const strip* s, uint32_t n) {
  /* Strip-triangle count: every strip after the first costs 4 degenerates. */
  uint32_t T = 0;
  for (uint32_t k = 0; k < n; ++k) T += s[k].len;
  T += 4 * (n - 1);

  /* Index slots I[0..T+1] and flags f[0..T-1], in global vertex numbers. */
  uint32_t* I = (uint32_t*)malloc(sizeof(uint32_t) * (T + 2));
  uint8_t* f = (uint8_t*)malloc(T);
  uint32_t* seen = (uint32_t*)malloc(sizeof(uint32_t) * (T + 2));
  if (!I || !f || !seen) { free(I); free(f); free(seen); return OR_ENOMEM; }
  uint32_t slot = 0, ti = 0;
  for (uint32_t k = 0; k < n; ++k) {
    const strip* S = &s[k];
    const uint32_t* v = &tri[3ull * S->tri[0]];
    uint32_t a, b, c;
    if (S->len == 1) { a = v[0]; b = v[1]; c = v[2]; }
    else {  /* rotate the first triangle so that its exit is the right edge (B,C) */
      int e = S->exit[0];
      a = v[(e + 2) % 3]; b = v[e]; c = v[(e + 1) % 3];
    }
    if (k == 0) {
      I[slot++] = a; I[slot++] = b; I[slot++] = c;
      f[ti++] = FLAG_L;
    } else {
      /* restart (four degenerate triangles, Sec. 4.2): slots c_prev, a, a, b
       * with flags L,R,L,R, then slot c with flag L yields (a,b,c) */
      uint32_t cp = I[slot - 1];
      I[slot++] = cp; f[ti++] = FLAG_L;
      I[slot++] = a;  f[ti++] = FLAG_R;
      I[slot++] = a;  f[ti++] = FLAG_L;
      I[slot++] = b;  f[ti++] = FLAG_R;
      I[slot++] = c;  f[ti++] = FLAG_L;
    }
    /* each following triangle adds the vertex opposite its entry edge; its
     * flag says whether its predecessor left through its right edge (entry+1)
     * or its left edge (entry+2); the first triangle leaves through its right
     * edge by the rotation above */
    int prev_in = -1;
    for (uint32_t q = 1; q < S->len; ++q) {
      int prev_exit = S->exit[q - 1];
      int fl = (q == 1) ? FLAG_R : (prev_exit == (prev_in + 1) % 3 ? FLAG_R : FLAG_L);
      int in_edge = nbr_edge[3ull * S->tri[q - 1] + (uint32_t)prev_exit];
      I[slot++] = tri[3ull * S->tri[q] + (uint32_t)(in_edge + 2) % 3];
      f[ti++] = (uint8_t)fl;
      prev_in = in_edge;
    }
  }

  /* Renumber by first appearance (Sec. 4.3): increments and reuse bytes. */
  uint32_t V = 0;
  uint32_t nch = (T + 63) / 64;
  uint64_t chunk_off = E->bits_bytes / 16;
  uint64_t reuse_off = E->reuse_bytes;
  if (grow((void**)&E->bits, &E->bits_cap, E->bits_bytes + 16ull * nch, 1)) goto nomem;
  for (uint32_t i = 0; i < T + 2; ++i) {
    int32_t found = -1;
    for (uint32_t q = 0; q < V; ++q) if (seen[q] == I[i]) { found = (int32_t)q; break; }
    if (found < 0) seen[V++] = I[i];
    if (i >= 3) {
      uint32_t t = i - 2;
      if (found < 0) {
        E->bits[16ull * (chunk_off + t / 64) + 8 + (t % 64) / 8] |= (uint8_t)(1u << (t % 8));
      } else {
        if (grow((void**)&E->reuse, &E->reuse_cap, E->reuse_bytes + 1, 1)) goto nomem;
        E->reuse[E->reuse_bytes++] = (uint8_t)found;
      }
    }
  }
  for (uint32_t t = 0; t < T; ++t)
    if (f[t] == FLAG_R) E->bits[16ull * (chunk_off + t / 64) + (t % 64) / 8] |= (uint8_t)(1u << (t % 8));
  E->bits_bytes += 16ull * nch;

  /* descriptor */
  if (grow((void**)&E->desc, &E->desc_cap, 16ull * (E->meshlets + 1), 1)) goto nomem;
  uint8_t* d = E->desc + 16ull * E->meshlets;
  wr_u32(d, (uint32_t)chunk_off); wr_u32(d + 4, (uint32_t)reuse_off);
  wr_u32(d + 8, (uint32_t)E->strip_triangles); wr_u16(d + 12, T); wr_u16(d + 14, V);

  /* local -> global vertex list */
  if (grow((void**)&E->verts, &E->verts_cap, E->verts_len + V, sizeof(uint32_t))) goto nomem;
  memcpy(E->verts + E->verts_len, seen, sizeof(uint32_t) * V);
  E->verts_len += V;
  if (grow((void**)&E->vert_off, &E->vert_off_cap, (uint64_t)E->meshlets + 2, sizeof(uint64_t))) goto nomem;
  E->vert_off[E->meshlets + 1] = E->verts_len;

  E->meshlets += 1;
  E->strip_triangles += T;
  E->restarts += n - 1;
  E->reuse_count += T + 2 - V;
  E->payload_bits += (uint64_t)T + (T - 1) + 8ull * (T + 2 - V);
  E->stored_bytes += 16 + 16ull * nch + (T + 2 - V);
  free(I); free(f); free(seen);
  return OR_OK;
nomem:
  free(I); free(f); free(seen);
  return OR_ENOMEM;
}

/*
 * Greedy strips over one meshlet of n triangles (the paper solves for optimal
 * strips with a MILP, Sec. 4.1; this is a plain greedy stand-in).  Triangles
 * are referred to by their position 0..n-1 in the meshlet; "free" neighbours
 * are in-meshlet neighbours not yet in a strip.
 *   1. The strip starts at the triangle with the fewest free neighbours
 *      (ties: lowest position).
 *   2. It leaves toward the free neighbour with the fewest free neighbours
 *      (ties: lowest position, then lowest edge index).
 *   3. From a triangle entered through edge i, the right edge is i+1 and the
 *      left edge i+2 (mod 3).  The walk continues to whichever of the two
 *      neighbours is free and has fewer free neighbours; on a tie it takes the
 *      direction opposite to the one it came from (alternating); it stops when
 *      neither is free.
 *   4. Then, from the start triangle, it walks the other way: to the free
 *      neighbour (not through the edge of step 2) with the fewest free
 *      neighbours (ties: lowest position, then edge), then on by rule 3, the
 *      start's edge of step 2 counting as the edge it was entered through.
 *   5. The strip is the backward walk reversed, the start, the forward walk.
 * The strips are then packed, in order, into parts whose strip-triangle count
 * (4 degenerates per restart) stays within max_tris (Sec. 4.2's split).
 */
static int encode_meshlet(oracle_enc* E, const uint32_t* tri, const int64_t* nbr, const uint8_t* nbr_edge,
                          const uint32_t* mt, uint32_t n, const int64_t* owner, int64_t mid,
                          const uint32_t* pos_in, uint32_t max_tris) {
  uint8_t* used = (uint8_t*)calloc(n, 1);
  int32_t* lnbr = (int32_t*)malloc(sizeof(int32_t) * 3 * n);
  int32_t* fw = (int32_t*)malloc(sizeof(int32_t) * n);   /* forward walk */
  uint8_t* fw_exit = (uint8_t*)malloc(n);                /* exit edge of the triangle before fw[j] */
  int32_t* bw = (int32_t*)malloc(sizeof(int32_t) * n);   /* backward walk */
  uint8_t* bw_in = (uint8_t*)malloc(n);                  /* edge bw[j] was entered through */
  strip* S = (strip*)calloc(n, sizeof(strip));
  uint32_t ns = 0;
  int rc = OR_OK;
  if (!used || !lnbr || !fw || !fw_exit || !bw || !bw_in || !S) { rc = OR_ENOMEM; goto done; }
  for (uint32_t i = 0; i < n; ++i)
    for (int e = 0; e < 3; ++e) {
      int64_t g = nbr[3ull * mt[i] + e];
      lnbr[3 * i + e] = (g >= 0 && owner[g] == mid) ? (int32_t)pos_in[g] : -1;
    }
#define FREE_NBRS(p, out) do { uint32_t c_ = 0; \
    for (int k_ = 0; k_ < 3; ++k_) if (lnbr[3 * (p) + k_] >= 0 && !used[lnbr[3 * (p) + k_]]) ++c_; \
    (out) = c_; } while (0)

  for (;;) {
    /* 1. start */
    int32_t s = -1; uint32_t sc = 4;
    for (uint32_t i = 0; i < n; ++i) {
      if (used[i]) continue;
      uint32_t c; FREE_NBRS(i, c);
      if (c < sc) { sc = c; s = (int32_t)i; }
    }
    if (s < 0) break;
    used[s] = 1;
    uint32_t nf = 0, nb = 0;
    /* 2. forward exit */
    int ef = -1; uint32_t bc = 4; int32_t bp = 0;
    for (int e = 0; e < 3; ++e) {
      int32_t p = lnbr[3 * s + e];
      if (p < 0 || used[p]) continue;
      uint32_t c; FREE_NBRS(p, c);
      if (ef < 0 || c < bc || (c == bc && p < bp)) { ef = e; bc = c; bp = p; }
    }
    for (int dir = 0; dir < 2 && ef >= 0; ++dir) {
      int e0 = -1;
      if (dir == 0) e0 = ef;
      else {   /* 4. backward exit */
        bc = 4; bp = 0;
        for (int e = 0; e < 3; ++e) {
          if (e == ef) continue;
          int32_t p = lnbr[3 * s + e];
          if (p < 0 || used[p]) continue;
          uint32_t c; FREE_NBRS(p, c);
          if (e0 < 0 || c < bc || (c == bc && p < bp)) { e0 = e; bc = c; bp = p; }
        }
        if (e0 < 0) break;
      }
      int s_in = (dir == 0) ? (ef + 2) % 3 : ef;     /* edge the start counts as entered through */
      int came = (e0 == (s_in + 1) % 3) ? FLAG_R : FLAG_L;
      int32_t cur = lnbr[3 * s + e0];
      int in_edge = nbr_edge[3ull * mt[s] + e0];
      used[cur] = 1;
      if (dir == 0) { fw[nf] = cur; fw_exit[nf] = (uint8_t)e0; ++nf; }
      else { bw[nb] = cur; bw_in[nb] = (uint8_t)in_edge; ++nb; }
      for (;;) {   /* 3. walk */
        int er = (in_edge + 1) % 3, el = (in_edge + 2) % 3;
        int32_t pr = lnbr[3 * cur + er], pl = lnbr[3 * cur + el];
        if (pr >= 0 && used[pr]) pr = -1;
        if (pl >= 0 && used[pl]) pl = -1;
        if (pr < 0 && pl < 0) break;
        int go;
        if (pr >= 0 && pl >= 0) {
          uint32_t cr, cl; FREE_NBRS(pr, cr); FREE_NBRS(pl, cl);
          if (cr < cl) go = FLAG_R;
          else if (cl < cr) go = FLAG_L;
          else go = (came == FLAG_R) ? FLAG_L : FLAG_R;
        } else {
          go = pr >= 0 ? FLAG_R : FLAG_L;
        }
        int eo = go == FLAG_R ? er : el;
        int32_t nx = go == FLAG_R ? pr : pl;
        in_edge = nbr_edge[3ull * mt[cur] + eo];
        cur = nx; came = go; used[cur] = 1;
        if (dir == 0) { fw[nf] = cur; fw_exit[nf] = (uint8_t)eo; ++nf; }
        else { bw[nb] = cur; bw_in[nb] = (uint8_t)in_edge; ++nb; }
      }
    }
    /* 5. assemble: reversed backward walk, start, forward walk */
    strip* st = &S[ns++];
    st->len = nb + 1 + nf;
    st->tri = (uint32_t*)malloc(sizeof(uint32_t) * st->len);
    st->exit = (uint8_t*)malloc(st->len);
    if (!st->tri || !st->exit) { rc = OR_ENOMEM; goto done; }
    uint32_t L = 0;
    for (uint32_t j = nb; j-- > 0;) { st->tri[L] = mt[bw[j]]; st->exit[L] = bw_in[j]; ++L; }
    st->tri[L] = mt[s]; st->exit[L] = (uint8_t)(nf ? ef : 0); ++L;
    for (uint32_t j = 0; j < nf; ++j) {
      st->tri[L] = mt[fw[j]];
      st->exit[L] = (j + 1 < nf) ? fw_exit[j + 1] : 0;
      ++L;
    }
  }
#undef FREE_NBRS

  /* pack strips into parts of at most max_tris strip triangles */
  {
    uint32_t k = 0;
    int first_part = 1;
    while (k < ns) {
      uint32_t T = S[k].len, end = k + 1;
      while (end < ns && T + 4 + S[end].len <= max_tris) { T += 4 + S[end].len; ++end; }
      rc = emit_part(E, tri, nbr_edge, &S[k], end - k);
      if (rc != OR_OK) goto done;
      if (!first_part) E->split_meshlets += 1;
      first_part = 0;
      k = end;
    }
  }
done:
  if (S) for (uint32_t i = 0; i < ns; ++i) { free(S[i].tri); free(S[i].exit); }
  free(S); free(used); free(lnbr); free(fw); free(fw_exit); free(bw); free(bw_in);
  return rc;
}

/*
 * Greedy meshlets (the paper uses a third-party meshlet builder, Sec. 5; this
 * is a plain stand-in).  "Unassigned" means in no meshlet yet.
 *   - Seed: among the candidates the previous meshlet was left with, the one
 *     with the fewest unassigned neighbours (ties: lowest number); if there
 *     are none, the lowest-numbered unassigned triangle.  The seed has level 0.
 *   - Candidates: unassigned triangles that are neighbours of a meshlet
 *     triangle; each keeps the level of its first discovery, one more than
 *     the level of the meshlet triangle that found it.
 *   - Growth: add the candidate with the fewest new vertices, then the fewest
 *     unassigned neighbours, then the lowest level, then the lowest number,
 *     among those that keep the meshlet within max_vertices vertices; stop at
 *     max_triangles triangles or when no candidate fits.
 */
int oracle_encode(const uint32_t* tri, uint64_t T, uint32_t V, uint32_t max_vertices,
                  uint32_t max_triangles, oracle_enc** out) {
  if (!out) return OR_EINVAL;
  *out = NULL;
  if (!tri && T) return OR_EINVAL;
  if (max_vertices < 3 || max_vertices > 256 || max_triangles < 1 || max_triangles > 256) return OR_ELIMIT;
  if (T > 0xFFFFFFFFull / 5) return OR_ELIMIT;
  for (uint64_t t = 0; t < T; ++t) {
    uint32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    if (a >= V || b >= V || c >= V) return OR_EINVAL;
    if (a == b || b == c || a == c) return OR_EDEGENERATE;
  }
  oracle_enc* E = (oracle_enc*)calloc(1, sizeof(oracle_enc));
  if (!E) return OR_ENOMEM;
  E->input_triangles = T;
  if (grow((void**)&E->vert_off, &E->vert_off_cap, 1, sizeof(uint64_t))) { oracle_enc_free(E); return OR_ENOMEM; }
  E->vert_off[0] = 0;
  if (T == 0) { *out = E; return OR_OK; }

  int64_t* nbr = (int64_t*)malloc(sizeof(int64_t) * 3 * T);
  uint8_t* nbr_edge = (uint8_t*)malloc(3 * T);
  int64_t* owner = (int64_t*)malloc(sizeof(int64_t) * T);
  int64_t* vstamp = (int64_t*)malloc(sizeof(int64_t) * (V ? V : 1));
  int64_t* cstamp = (int64_t*)malloc(sizeof(int64_t) * T);
  uint32_t* mt = (uint32_t*)malloc(sizeof(uint32_t) * max_triangles);
  uint32_t* cand = (uint32_t*)malloc(sizeof(uint32_t) * T);
  uint32_t* cand_level = (uint32_t*)malloc(sizeof(uint32_t) * T);
  uint32_t* pos_in = (uint32_t*)malloc(sizeof(uint32_t) * T);
  int rc = OR_OK;
  if (!nbr || !nbr_edge || !owner || !vstamp || !cstamp || !mt || !cand || !cand_level || !pos_in) {
    rc = OR_ENOMEM; goto fail;
  }
  rc = build_adjacency(tri, T, nbr, nbr_edge);
  if (rc != OR_OK) goto fail;
  for (uint64_t t = 0; t < T; ++t) { owner[t] = -1; cstamp[t] = -1; }
  for (uint32_t v = 0; v < V; ++v) vstamp[v] = -1;

#define UNASSIGNED_NBRS(g, out) do { uint32_t c_ = 0; \
    for (int e_ = 0; e_ < 3; ++e_) { int64_t h_ = nbr[3ull * (g) + e_]; if (h_ >= 0 && owner[h_] < 0) ++c_; } \
    (out) = c_; } while (0)

  uint64_t scan = 0;
  uint32_t nc = 0;
  for (int64_t mid = 0;; ++mid) {
    /* seed */
    int64_t seed = -1; uint32_t seed_free = 4;
    for (uint32_t q = 0; q < nc; ++q) {
      uint32_t c; UNASSIGNED_NBRS(cand[q], c);
      if (seed < 0 || c < seed_free || (c == seed_free && cand[q] < (uint32_t)seed)) { seed = cand[q]; seed_free = c; }
    }
    if (seed < 0) {
      while (scan < T && owner[scan] >= 0) ++scan;
      if (scan >= T) break;
      seed = (int64_t)scan;
    }
    uint32_t n = 0, nv = 0;
    nc = 0;
    uint32_t pick = (uint32_t)seed, pick_level = 0;
    for (;;) {
      owner[pick] = mid;
      mt[n++] = pick;
      for (int k = 0; k < 3; ++k) {
        uint32_t v = tri[3ull * pick + k];
        if (vstamp[v] != mid) { vstamp[v] = mid; ++nv; }
      }
      /* drop it from the candidates, then add its undiscovered neighbours */
      for (uint32_t q = 0; q < nc; ++q)
        if (cand[q] == pick) { cand[q] = cand[nc - 1]; cand_level[q] = cand_level[nc - 1]; --nc; break; }
      for (int e = 0; e < 3; ++e) {
        int64_t g = nbr[3ull * pick + e];
        if (g >= 0 && owner[g] < 0 && cstamp[g] != mid) {
          cstamp[g] = mid; cand[nc] = (uint32_t)g; cand_level[nc] = pick_level + 1; ++nc;
        }
      }
      if (n >= max_triangles) break;
      /* next: fewest new vertices, fewest unassigned neighbours, lowest level, lowest number */
      int64_t best = -1; uint32_t bcost = 0, bfree = 0, blevel = 0;
      for (uint32_t q = 0; q < nc; ++q) {
        uint32_t g = cand[q], cost = 0, fr;
        for (int k = 0; k < 3; ++k) if (vstamp[tri[3ull * g + k]] != mid) ++cost;
        if (nv + cost > max_vertices) continue;
        UNASSIGNED_NBRS(g, fr);
        int better;
        if (best < 0) better = 1;
        else if (cost != bcost) better = cost < bcost;
        else if (fr != bfree) better = fr < bfree;
        else if (cand_level[q] != blevel) better = cand_level[q] < blevel;
        else better = g < (uint32_t)best;
        if (better) { best = g; bcost = cost; bfree = fr; blevel = cand_level[q]; }
      }
      if (best < 0) break;
      pick = (uint32_t)best; pick_level = blevel;
    }
    for (uint32_t i = 0; i < n; ++i) pos_in[mt[i]] = i;
    rc = encode_meshlet(E, tri, nbr, nbr_edge, mt, n, owner, mid, pos_in, max_triangles);
    if (rc != OR_OK) goto fail;
  }
#undef UNASSIGNED_NBRS
  if (E->strip_triangles > 0xFFFFFFFFull) { rc = OR_ELIMIT; goto fail; }
  free(nbr); free(nbr_edge); free(owner); free(vstamp); free(cstamp); free(mt);
  free(cand); free(cand_level); free(pos_in);
  *out = E;
  return OR_OK;
fail:
  free(nbr); free(nbr_edge); free(owner); free(vstamp); free(cstamp); free(mt);
  free(cand); free(cand_level); free(pos_in);
  oracle_enc_free(E);
  return rc;
}

/* --------------------------------------------------------------- accessors */

uint32_t oracle_enc_meshlets(const oracle_enc* e) { return e->meshlets; }
const uint8_t* oracle_enc_desc(const oracle_enc* e) { return e->desc; }
const uint8_t* oracle_enc_bits(const oracle_enc* e) { return e->bits; }
uint64_t oracle_enc_bits_bytes(const oracle_enc* e) { return e->bits_bytes; }
const uint8_t* oracle_enc_reuse(const oracle_enc* e) { return e->reuse; }
uint64_t oracle_enc_reuse_bytes(const oracle_enc* e) { return e->reuse_bytes; }
const uint32_t* oracle_enc_verts(const oracle_enc* e) { return e->verts; }
const uint64_t* oracle_enc_vert_off(const oracle_enc* e) { return e->vert_off; }
/* stats: 0 input triangles, 1 strip triangles, 2 restarts, 3 reuse count,
 * 4 split meshlets, 5 payload bits, 6 stored bytes */
uint64_t oracle_enc_stat(const oracle_enc* e, int which) {
  switch (which) {
    case 0: return e->input_triangles;
    case 1: return e->strip_triangles;
    case 2: return e->restarts;
    case 3: return e->reuse_count;
    case 4: return e->split_meshlets;
    case 5: return e->payload_bits;
    case 6: return e->stored_bytes;
    default: return 0;
  }
}
