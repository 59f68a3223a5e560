// CPU encoder: triangle list -> meshlets -> GTS-Reuse streams.
//
// Kuth et al., "Towards Practical Meshlet Compression": meshlets bounded by
// max vertices / max triangles (Sec. 3), each stored as a generalized strip
// with one L/R flag per triangle and four degenerate triangles per restart,
// split when the strip outgrows the triangle limit (Sec. 4.2), vertices
// renumbered by first appearance so that new vertices cost one increment bit
// and only reused indices are stored as bytes (Sec. 4.3).
//
// The paper builds meshlets with a third-party library and finds optimal
// strips with a MILP (Sec. 4.1, Sec. 5).  This encoder uses deterministic
// greedy rules instead (stated at build_meshlets and make_strips); a
// sequential reference implementation of the same rules exists, so streams
// from the two can be compared byte for byte.
//
// Work split: adjacency and meshlet growth are sequential over the mesh;
// strips, renumbering and packing run on `threads` threads over contiguous
// meshlet ranges, whose outputs are concatenated in meshlet order.

#include <algorithm>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "common.h"

struct gtsr_encoded {
  std::vector<gtsr_meshlet> meshlets;
  std::vector<uint8_t> bits;
  std::vector<uint8_t> reuse;
  std::vector<uint32_t> verts;
  std::vector<uint64_t> vert_off;
  std::vector<uint32_t> kept_off;   // input triangles before each meshlet
  std::vector<uint32_t> tri_ids;    // input triangle ids, meshlet by meshlet, in strip order
  uint64_t input_triangles = 0, strip_triangles = 0, restarts = 0, reuse_count = 0;
  uint64_t split_meshlets = 0, payload_bits = 0, stored_bytes = 0;
  uint64_t exact_tried = 0, exact_proven = 0;
};

namespace gtsr {
namespace {

constexpr uint8_t kFlagL = 0;
constexpr uint8_t kFlagR = 1;

inline uint32_t corner(const uint32_t* idx, uint32_t t, uint32_t k) { return idx[3ull * t + k]; }

// Neighbour across edge e of triangle t (edge e runs from corner e to corner
// e+1 mod 3) and that neighbour's own index of the shared edge.  An edge links
// two triangles only when exactly two triangles use it, in opposite
// directions.
struct Adjacency {
  std::vector<uint32_t> nbr;   // 3T, kNone when there is no neighbour
  std::vector<uint8_t> twin;   // 3T
};

void build_adjacency(const uint32_t* idx, uint32_t T, uint32_t V, Adjacency& A) {
  const uint64_t H = 3ull * T;
  A.nbr.assign(H, kNone);
  A.twin.assign(H, 0);
  // bucket half-edges by their smaller endpoint (counting sort)
  std::vector<uint32_t> head(static_cast<size_t>(V) + 1, 0);
  for (uint64_t h = 0; h < H; ++h) {
    uint32_t t = static_cast<uint32_t>(h / 3), e = static_cast<uint32_t>(h % 3);
    uint32_t a = corner(idx, t, e), b = corner(idx, t, (e + 1) % 3);
    ++head[std::min(a, b) + 1];
  }
  for (uint32_t v = 0; v < V; ++v) head[v + 1] += head[v];
  std::vector<uint32_t> fill(head.begin(), head.end() - 1);
  std::vector<uint32_t> he(H);
  for (uint64_t h = 0; h < H; ++h) {
    uint32_t t = static_cast<uint32_t>(h / 3), e = static_cast<uint32_t>(h % 3);
    uint32_t a = corner(idx, t, e), b = corner(idx, t, (e + 1) % 3);
    he[fill[std::min(a, b)]++] = static_cast<uint32_t>(h);
  }
  auto other_end = [&](uint32_t h) {
    uint32_t t = h / 3, e = h % 3;
    uint32_t a = corner(idx, t, e), b = corner(idx, t, (e + 1) % 3);
    return std::max(a, b);
  };
  auto forward = [&](uint32_t h) {
    uint32_t t = h / 3, e = h % 3;
    return corner(idx, t, e) < corner(idx, t, (e + 1) % 3);
  };
  for (uint32_t v = 0; v < V; ++v) {
    uint32_t* b = he.data() + head[v];
    uint32_t* e = he.data() + head[v + 1];
    // buckets are small (about the vertex valence): insertion sort by far end
    for (uint32_t* p = b + 1; p < e; ++p) {
      uint32_t x = *p, kx = other_end(x);
      uint32_t* q = p;
      while (q > b && other_end(q[-1]) > kx) { *q = q[-1]; --q; }
      *q = x;
    }
    for (uint32_t* p = b; p < e;) {
      uint32_t* r = p + 1;
      uint32_t key = other_end(*p);
      while (r < e && other_end(*r) == key) ++r;
      if (r - p == 2 && forward(p[0]) != forward(p[1])) {
        uint32_t x = p[0], y = p[1];
        A.nbr[x] = y / 3; A.twin[x] = static_cast<uint8_t>(y % 3);
        A.nbr[y] = x / 3; A.twin[y] = static_cast<uint8_t>(x % 3);
      }
      p = r;
    }
  }
}

// ---------------------------------------------------------------- meshlets

struct Meshlets {
  std::vector<uint32_t> tris;    // triangles, meshlet after meshlet, in growth order
  std::vector<uint32_t> start;   // meshlet m = tris[start[m] .. start[m+1])
  std::vector<uint32_t> owner;   // meshlet of each triangle
  std::vector<uint32_t> pos;     // position of each triangle inside its meshlet
};

// Greedy meshlet growth.  "Free" = not in any meshlet yet.
//  * Seed: among the candidates the previous meshlet ended with, the one with
//    the fewest free neighbours (ties: lowest triangle number); if there are
//    none, the lowest-numbered free triangle.  The seed sits at level 0.
//  * Candidates: free triangles adjacent to the growing meshlet; each keeps
//    the level of its first discovery (one more than its discoverer's).
//  * Growth: take the candidate with the fewest new vertices, then the fewest
//    free neighbours, then the lowest level, then the lowest number, among
//    those that keep the vertex count within max_v; stop at max_t triangles
//    or when none fits.
// New-vertex and free-neighbour counts are kept per candidate and decremented
// as vertices join and triangles are taken, so one step costs one pass over
// the (short) candidate list.
void build_meshlets(const uint32_t* idx, uint32_t T, uint32_t V, const Adjacency& A,
                    uint32_t max_v, uint32_t max_t, Meshlets& M) {
  // vertex -> incident triangles
  std::vector<uint32_t> vt_head(static_cast<size_t>(V) + 1, 0);
  for (uint64_t i = 0; i < 3ull * T; ++i) ++vt_head[idx[i] + 1];
  for (uint32_t v = 0; v < V; ++v) vt_head[v + 1] += vt_head[v];
  std::vector<uint32_t> vt(3ull * T);
  {
    std::vector<uint32_t> f(vt_head.begin(), vt_head.end() - 1);
    for (uint64_t i = 0; i < 3ull * T; ++i) vt[f[idx[i]]++] = static_cast<uint32_t>(i / 3);
  }
  M.owner.assign(T, kNone);
  M.pos.assign(T, 0);
  M.tris.clear();
  M.tris.reserve(T);
  M.start.clear();
  std::vector<uint32_t> vstamp(V, 0), cstamp(T, 0), cslot(T, 0);

  struct Cand { uint32_t tri; uint32_t level; uint8_t cost, free; };
  std::vector<Cand> cand;
  cand.reserve(1024);

  auto free_nbrs = [&](uint32_t g) {
    uint32_t c = 0;
    for (int e = 0; e < 3; ++e) {
      uint32_t h = A.nbr[3ull * g + e];
      if (h != kNone && M.owner[h] == kNone) ++c;
    }
    return c;
  };

  uint32_t scan = 0;
  for (uint32_t serial = 0;; ++serial) {
    uint32_t seed = kNone, seed_free = 0;
    for (const Cand& c : cand)
      if (seed == kNone || c.free < seed_free || (c.free == seed_free && c.tri < seed)) {
        seed = c.tri; seed_free = c.free;
      }
    if (seed == kNone) {
      while (scan < T && M.owner[scan] != kNone) ++scan;
      if (scan >= T) break;
      seed = scan;
    }
    cand.clear();
    const uint32_t stamp = serial + 1;
    M.start.push_back(static_cast<uint32_t>(M.tris.size()));
    uint32_t n = 0, nv = 0;
    uint32_t pick = seed, pick_level = 0;
    for (;;) {
      M.owner[pick] = serial;
      M.pos[pick] = n++;
      M.tris.push_back(pick);
      if (cstamp[pick] == stamp) {   // leaves the candidate list
        uint32_t s = cslot[pick];
        cand[s] = cand.back();
        cslot[cand[s].tri] = s;
        cand.pop_back();
        cstamp[pick] = 0;
      }
      for (int k = 0; k < 3; ++k) {
        uint32_t v = corner(idx, pick, k);
        if (vstamp[v] == stamp) continue;
        vstamp[v] = stamp;
        ++nv;
        for (uint32_t q = vt_head[v]; q < vt_head[v + 1]; ++q)
          if (cstamp[vt[q]] == stamp) --cand[cslot[vt[q]]].cost;
      }
      for (int e = 0; e < 3; ++e) {
        uint32_t g = A.nbr[3ull * pick + e];
        if (g == kNone) continue;
        if (cstamp[g] == stamp) {
          --cand[cslot[g]].free;        // pick was one of its free neighbours
        } else if (M.owner[g] == kNone) {
          uint8_t cost = 0;
          for (int k = 0; k < 3; ++k) cost += vstamp[corner(idx, g, k)] != stamp;
          cstamp[g] = stamp;
          cslot[g] = static_cast<uint32_t>(cand.size());
          cand.push_back({g, pick_level + 1, cost, static_cast<uint8_t>(free_nbrs(g))});
        }
      }
      if (n >= max_t) break;
      const bool room = nv < max_v;
      uint64_t best_key = ~0ull;
      uint32_t best = kNone, best_level = 0;
      for (const Cand& c : cand) {
        if (c.cost && !room) continue;
        uint64_t key = (uint64_t(c.cost) << 44) | (uint64_t(c.free) << 42) |
                       (uint64_t(c.level) << 32) | c.tri;
        if (key < best_key) { best_key = key; best = c.tri; best_level = c.level; }
      }
      if (best == kNone) break;
      pick = best;
      pick_level = best_level;
    }
  }
  M.start.push_back(static_cast<uint32_t>(M.tris.size()));
}

// ------------------------------------------------------------------ strips

// A strip is a path of triangles (global numbers) with, for each but the
// last, the edge (0..2, in that triangle's own corner order) it leaves by.
struct Strip { uint32_t first, len; };   // into a per-meshlet path buffer

// Greedy strips over one meshlet of n triangles; "free" = in the meshlet and
// not yet in a strip; positions are growth order.
//  1. Start at the triangle with the fewest free neighbours (ties: lowest
//     position).
//  2. Leave toward the free neighbour with the fewest free neighbours (ties:
//     lowest position, then lowest edge).
//  3. From a triangle entered through edge i, the right edge is i+1 and the
//     left edge i+2 (mod 3); go to whichever side is free with fewer free
//     neighbours; on a tie, turn opposite to the last turn (alternate); stop
//     when neither side is free.
//  4. Walk backward from the start: to the free neighbour (not across the
//     edge of step 2) with the fewest free neighbours (ties: position, then
//     edge), then by rule 3, counting the edge of step 2 as the start's entry.
//  5. The strip is the backward walk reversed, the start, the forward walk.
class Stripper {
 public:
  void run(const uint32_t* mt, uint32_t n, uint32_t serial, const Adjacency& A, const Meshlets& M) {
    n_ = n;
    for (uint32_t i = 0; i < n; ++i) {
      used_[i] = 0;
      for (int e = 0; e < 3; ++e) {
        uint32_t g = A.nbr[3ull * mt[i] + e];
        lnbr_[3 * i + e] = (g != kNone && M.owner[g] == serial) ? static_cast<int16_t>(M.pos[g]) : int16_t(-1);
      }
    }
    strips.clear();
    path_len = 0;
    for (;;) {
      int s = -1;
      uint32_t sc = 4;
      for (uint32_t i = 0; i < n; ++i) {
        if (used_[i]) continue;
        uint32_t c = free_nbrs(static_cast<int>(i));
        if (c < sc) { sc = c; s = static_cast<int>(i); if (c == 0) break; }
      }
      if (s < 0) break;
      used_[s] = 1;
      int ef = best_exit(s, -1);
      uint32_t nf = 0, nb = 0;
      if (ef >= 0) {
        nf = walk(s, ef, (ef + 2) % 3, A, mt, fw_, fw_edge_, /*record_exit=*/true);
        int eb = best_exit(s, ef);
        if (eb >= 0) nb = walk(s, eb, ef, A, mt, bw_, bw_edge_, /*record_exit=*/false);
      }
      Strip st{path_len, nb + 1 + nf};
      for (uint32_t j = nb; j-- > 0;) push(mt[bw_[j]], bw_edge_[j]);
      push(mt[s], static_cast<uint8_t>(nf ? ef : 0));
      for (uint32_t j = 0; j < nf; ++j) push(mt[fw_[j]], j + 1 < nf ? fw_edge_[j + 1] : 0);
      strips.push_back(st);
    }
  }

  std::vector<Strip> strips;
  uint32_t path_tri[kMaxStripTris];
  uint8_t path_exit[kMaxStripTris];
  uint32_t path_len = 0;

  const int16_t* local_nbrs() const { return lnbr_; }
  uint32_t size() const { return n_; }
  // Replaces the strips by the paths given as per-triangle chosen links
  // (link[3p+e]: the pair across edge e of position p is chained): a path
  // starts at its lowest-positioned end, paths in order of that position.
  void set_paths(const uint8_t* link, const uint32_t* mt) {
    strips.clear();
    path_len = 0;
    for (uint32_t i = 0; i < n_; ++i) used_[i] = 0;
    for (uint32_t i = 0; i < n_; ++i) {
      if (used_[i]) continue;
      uint32_t d = link[3 * i] + link[3 * i + 1] + link[3 * i + 2];
      if (d > 1) continue;   // not an end: reached from one
      Strip st{path_len, 0};
      int cur = static_cast<int>(i), prev = -1;
      for (;;) {
        used_[cur] = 1;
        int next = -1, ne = 0;
        for (int e = 0; e < 3; ++e)
          if (link[3 * cur + e] && lnbr_[3 * cur + e] != prev) { next = lnbr_[3 * cur + e]; ne = e; }
        push(mt[cur], static_cast<uint8_t>(next >= 0 ? ne : 0));
        ++st.len;
        if (next < 0) break;
        prev = cur;
        cur = next;
      }
      strips.push_back(st);
    }
  }

 private:
  uint32_t free_nbrs(int p) const {
    uint32_t c = 0;
    for (int e = 0; e < 3; ++e) {
      int q = lnbr_[3 * p + e];
      c += (q >= 0 && !used_[q]);
    }
    return c;
  }
  int best_exit(int s, int skip_edge) const {
    int be = -1, bp = 0;
    uint32_t bc = 4;
    for (int e = 0; e < 3; ++e) {
      if (e == skip_edge) continue;
      int p = lnbr_[3 * s + e];
      if (p < 0 || used_[p]) continue;
      uint32_t c = free_nbrs(p);
      if (be < 0 || c < bc || (c == bc && p < bp)) { be = e; bc = c; bp = p; }
    }
    return be;
  }
  // Walks from s across edge e0, s counting as entered through s_in.  Stores
  // visited positions in out[]; edge[j] is, with record_exit, the edge its
  // predecessor was left by, otherwise the edge out[j] was entered through.
  uint32_t walk(int s, int e0, int s_in, const Adjacency& A, const uint32_t* mt,
                int16_t* out, uint8_t* edge, bool record_exit) {
    uint32_t cnt = 0;
    uint8_t came = (e0 == (s_in + 1) % 3) ? kFlagR : kFlagL;
    int cur = lnbr_[3 * s + e0];
    int in = A.twin[3ull * mt[s] + e0];
    used_[cur] = 1;
    out[cnt] = static_cast<int16_t>(cur);
    edge[cnt++] = static_cast<uint8_t>(record_exit ? e0 : in);
    for (;;) {
      int er = (in + 1) % 3, el = (in + 2) % 3;
      int pr = lnbr_[3 * cur + er], pl = lnbr_[3 * cur + el];
      if (pr >= 0 && used_[pr]) pr = -1;
      if (pl >= 0 && used_[pl]) pl = -1;
      if (pr < 0 && pl < 0) break;
      uint8_t go;
      if (pr >= 0 && pl >= 0) {
        uint32_t cr = free_nbrs(pr), cl = free_nbrs(pl);
        go = cr < cl ? kFlagR : cl < cr ? kFlagL : (came == kFlagR ? kFlagL : kFlagR);
      } else {
        go = pr >= 0 ? kFlagR : kFlagL;
      }
      int eo = go == kFlagR ? er : el;
      int nx = go == kFlagR ? pr : pl;
      in = A.twin[3ull * mt[cur] + eo];
      cur = nx;
      came = go;
      used_[cur] = 1;
      out[cnt] = static_cast<int16_t>(cur);
      edge[cnt++] = static_cast<uint8_t>(record_exit ? eo : in);
    }
    return cnt;
  }
  void push(uint32_t tri, uint8_t exit) { path_tri[path_len] = tri; path_exit[path_len] = exit; ++path_len; }

  uint32_t n_ = 0;
  uint8_t used_[kMaxStripTris];
  int16_t lnbr_[3 * kMaxStripTris];
  int16_t fw_[kMaxStripTris], bw_[kMaxStripTris];
  uint8_t fw_edge_[kMaxStripTris], bw_edge_[kMaxStripTris];
};

// ---------------------------------------------------------------- emission

struct Piece {   // encoder output of a contiguous meshlet range
  std::vector<gtsr_meshlet> desc;   // offsets relative to the piece
  std::vector<uint64_t> bits;       // LR, INC per chunk
  std::vector<uint8_t> reuse;
  std::vector<uint32_t> verts;
  std::vector<uint32_t> vcount;
  std::vector<uint32_t> kept;       // input triangles per meshlet
  std::vector<uint32_t> tri_ids;    // their ids, in strip order
  uint64_t strip_tris = 0, restarts = 0, splits = 0, payload = 0, stored = 0;
  uint64_t exact_tried = 0, exact_proven = 0;
};

// Small map from global vertex number to local id for one meshlet part.
class LocalIds {
 public:
  void reset() { ++gen_; if (gen_ == 0) { std::memset(stamp_, 0, sizeof(stamp_)); gen_ = 1; } }
  // returns the local id and whether it is new
  uint32_t lookup(uint32_t v, uint32_t next_id, bool* is_new) {
    uint32_t h = (v * 2654435761u) >> (32 - kBits);
    for (;;) {
      if (stamp_[h] != gen_) {
        stamp_[h] = gen_; key_[h] = v; val_[h] = next_id;
        *is_new = true;
        return next_id;
      }
      if (key_[h] == v) { *is_new = false; return val_[h]; }
      h = (h + 1) & (kSize - 1);
    }
  }
 private:
  static constexpr uint32_t kBits = 10, kSize = 1u << kBits;
  uint32_t stamp_[kSize] = {};
  uint32_t key_[kSize];
  uint32_t val_[kSize];
  uint32_t gen_ = 0;
};

// Emits one meshlet part made of strips [k0, k1) of `st`: slot sequence with
// restarts (Sec. 4.2), first-appearance renumbering (Sec. 4.3), packing.
void emit_part(const uint32_t* idx, const Adjacency& A, const Stripper& st, size_t k0, size_t k1,
               LocalIds& ids, Piece& P) {
  uint32_t slots[kMaxStripTris + 2];
  uint8_t flags[kMaxStripTris];
  uint32_t ns = 0, nt = 0;
  for (size_t k = k0; k < k1; ++k) {
    const Strip& S = st.strips[k];
    const uint32_t* tri = st.path_tri + S.first;
    const uint8_t* ex = st.path_exit + S.first;
    P.tri_ids.insert(P.tri_ids.end(), tri, tri + S.len);
    uint32_t a, b, c;
    if (S.len == 1) {
      a = corner(idx, tri[0], 0); b = corner(idx, tri[0], 1); c = corner(idx, tri[0], 2);
    } else {   // rotate so the exit edge is the right edge (B,C)
      uint32_t e = ex[0];
      a = corner(idx, tri[0], (e + 2) % 3); b = corner(idx, tri[0], e); c = corner(idx, tri[0], (e + 1) % 3);
    }
    if (k == k0) {
      slots[ns++] = a; slots[ns++] = b; slots[ns++] = c;
      flags[nt++] = kFlagL;
    } else {       // four degenerates: c_prev, a, a, b (L,R,L,R), then c (L)
      uint32_t cp = slots[ns - 1];
      slots[ns++] = cp; flags[nt++] = kFlagL;
      slots[ns++] = a;  flags[nt++] = kFlagR;
      slots[ns++] = a;  flags[nt++] = kFlagL;
      slots[ns++] = b;  flags[nt++] = kFlagR;
      slots[ns++] = c;  flags[nt++] = kFlagL;
    }
    int prev_in = -1;
    for (uint32_t q = 1; q < S.len; ++q) {
      int px = ex[q - 1];
      uint8_t fl = q == 1 ? kFlagR : (px == (prev_in + 1) % 3 ? kFlagR : kFlagL);
      int in = A.twin[3ull * tri[q - 1] + px];
      slots[ns++] = corner(idx, tri[q], static_cast<uint32_t>(in + 2) % 3);
      flags[nt++] = fl;
      prev_in = in;
    }
  }
  const uint32_t T = nt;
  const uint32_t nch = chunks_of(T);
  gtsr_meshlet d;
  d.chunk_off = static_cast<uint32_t>(P.bits.size() / 2);
  d.reuse_off = static_cast<uint32_t>(P.reuse.size());
  d.out_off = static_cast<uint32_t>(P.strip_tris);
  size_t b0 = P.bits.size();
  P.bits.resize(b0 + 2 * nch, 0);
  uint64_t* bw = P.bits.data() + b0;
  ids.reset();
  uint32_t V = 0;
  for (uint32_t i = 0; i < ns; ++i) {
    bool fresh;
    uint32_t id = ids.lookup(slots[i], V, &fresh);
    if (fresh) { P.verts.push_back(slots[i]); ++V; }
    if (i >= 3) {
      uint32_t t = i - 2;
      if (fresh) bw[2 * (t / 64) + 1] |= 1ull << (t % 64);
      else P.reuse.push_back(static_cast<uint8_t>(id));
    }
  }
  for (uint32_t t = 0; t < T; ++t)
    if (flags[t] == kFlagR) bw[2 * (t / 64)] |= 1ull << (t % 64);
  d.tri_count = static_cast<uint16_t>(T);
  d.vert_count = static_cast<uint16_t>(V);
  P.desc.push_back(d);
  P.vcount.push_back(V);
  P.kept.push_back(T - 4 * static_cast<uint32_t>(k1 - k0 - 1));
  const uint32_t n_ru = T + 2 - V;
  P.strip_tris += T;
  P.restarts += (k1 - k0) - 1;
  P.payload += uint64_t(T) + (T - 1) + 8ull * n_ru;
  P.stored += 16 + 16ull * nch + n_ru;
}

// ------------------------------------------------------------ exact strips

// Fewest strips over one triangle set by branch and bound (the optimal GTS of
// Sec. 3.1, which the paper finds with a MILP).  Any simple path of
// neighbouring triangles is a strip, so the task is to chain as many
// neighbour pairs as possible such that no triangle is in more than two
// chained pairs (no fork) and no chained pairs close a cycle; strips = n -
// chained.  Depth-first over the pairs in order (include before exclude),
// with the bound chained + floor(sum over triangles of min(2 - degree,
// undecided pairs at it) / 2), and an incumbent to beat.  Stops after
// node_limit nodes; `proven` tells whether the search space was exhausted.
class ExactStrips {
 public:
  uint32_t solve(const int16_t* lnbr, uint32_t n, uint32_t incumbent_strips, uint64_t node_limit, bool* proven) {
    n_ = n;
    pa_.clear(); pb_.clear(); ea_.clear(); eb_.clear();
    for (uint32_t t = 0; t < n; ++t)
      for (int e = 0; e < 3; ++e) {
        const int q = lnbr[3 * t + e];
        if (q > static_cast<int>(t)) {
          int eq = 0;
          for (int f = 0; f < 3; ++f) if (lnbr[3 * q + f] == static_cast<int>(t)) eq = f;
          pa_.push_back(t); pb_.push_back(static_cast<uint32_t>(q)); ea_.push_back(e); eb_.push_back(eq);
        }
      }
    const size_t E = pa_.size();
    deg_.assign(n, 0); und_.assign(n, 0); parent_.resize(n); chosen_.assign(E, 0);
    for (uint32_t t = 0; t < n; ++t) parent_[t] = t;
    for (size_t k = 0; k < E; ++k) { ++und_[pa_[k]]; ++und_[pb_[k]]; }
    pot_ = 0;
    for (uint32_t t = 0; t < n; ++t) pot_ += contrib(t);
    best_ = n >= incumbent_strips ? n - incumbent_strips : 0;   // chained pairs to beat
    have_best_ = false;
    nodes_ = 0; limit_ = node_limit; aborted_ = false;
    dfs(0, 0);
    *proven = !aborted_;
    return n - best_;
  }
  bool improved() const { return have_best_; }
  // per-triangle chained links of the best solution (valid when improved())
  void links(uint8_t* link) const {
    std::memset(link, 0, 3 * n_);
    for (size_t k = 0; k < pa_.size(); ++k)
      if (best_sel_[k]) { link[3 * pa_[k] + ea_[k]] = 1; link[3 * pb_[k] + eb_[k]] = 1; }
  }

 private:
  uint32_t contrib(uint32_t t) const { return std::min<uint32_t>(2 - deg_[t], und_[t]); }
  uint32_t find(uint32_t x) const { while (parent_[x] != x) x = parent_[x]; return x; }
  void dfs(size_t k, uint32_t chained) {
    if (aborted_) return;
    if (++nodes_ > limit_) { aborted_ = true; return; }
    if (chained > best_) {
      best_ = chained;
      best_sel_ = chosen_;
      have_best_ = true;
    }
    if (k == pa_.size() || chained + pot_ / 2 <= best_) return;
    const uint32_t a = pa_[k], b = pb_[k];
    const uint32_t before = contrib(a) + contrib(b);
    --und_[a]; --und_[b];
    // include
    if (deg_[a] < 2 && deg_[b] < 2) {
      const uint32_t ra = find(a), rb = find(b);
      if (ra != rb) {
        ++deg_[a]; ++deg_[b];
        parent_[ra] = rb;
        chosen_[k] = 1;
        pot_ = pot_ - before + contrib(a) + contrib(b);
        dfs(k + 1, chained + 1);
        pot_ = pot_ - contrib(a) - contrib(b) + before;
        chosen_[k] = 0;
        parent_[ra] = ra;
        --deg_[a]; --deg_[b];
      }
    }
    // exclude
    pot_ = pot_ - before + contrib(a) + contrib(b);
    dfs(k + 1, chained);
    pot_ = pot_ - contrib(a) - contrib(b) + before;
    ++und_[a]; ++und_[b];
  }

  uint32_t n_ = 0;
  std::vector<uint32_t> pa_, pb_;
  std::vector<int> ea_, eb_;
  std::vector<uint32_t> deg_, und_, parent_;
  std::vector<uint8_t> chosen_, best_sel_;
  uint64_t pot_ = 0, nodes_ = 0, limit_ = 0;
  uint32_t best_ = 0;
  bool have_best_ = false, aborted_ = false;
};

constexpr uint64_t kExactNodeLimit = 200000;   // search nodes per meshlet

void encode_range(const uint32_t* idx, const Adjacency& A, const Meshlets& M, uint32_t m0, uint32_t m1,
                  uint32_t max_t, bool exact, Piece& P) {
  Stripper* st = new Stripper();
  LocalIds* ids = new LocalIds();
  ExactStrips* ex = exact ? new ExactStrips() : nullptr;
  uint8_t link[3 * kMaxStripTris];
  for (uint32_t m = m0; m < m1; ++m) {
    const uint32_t* mt = M.tris.data() + M.start[m];
    const uint32_t n = M.start[m + 1] - M.start[m];
    st->run(mt, n, m, A, M);
    if (ex && st->strips.size() > 1) {
      bool proven = false;
      ex->solve(st->local_nbrs(), n, static_cast<uint32_t>(st->strips.size()), kExactNodeLimit, &proven);
      if (ex->improved()) {
        ex->links(link);
        st->set_paths(link, mt);
      }
      P.exact_proven += proven;
      P.exact_tried += 1;
    }
    // pack strips, in order, into parts of at most max_t strip triangles
    size_t k = 0;
    bool first = true;
    while (k < st->strips.size()) {
      uint32_t T = st->strips[k].len;
      size_t end = k + 1;
      while (end < st->strips.size() && T + 4 + st->strips[end].len <= max_t) {
        T += 4 + st->strips[end].len;
        ++end;
      }
      emit_part(idx, A, *st, k, end, *ids, P);
      if (!first) ++P.splits;
      first = false;
      k = end;
    }
  }
  delete st;
  delete ids;
  delete ex;
}

}  // namespace
}  // namespace gtsr

using namespace gtsr;

extern "C" int encode_meshlets(const uint32_t* indices, uint64_t triangle_count, uint32_t vertex_count,
                               const gtsr_encode_params* params, gtsr_encoded** out) {
  if (!out || !params) return fail(GTSR_EINVAL, "encode_meshlets: null params/out");
  *out = nullptr;
  if (!indices && triangle_count) return fail(GTSR_EINVAL, "encode_meshlets: null indices");
  const uint32_t max_v = params->max_vertices, max_t = params->max_triangles;
  if (max_v < 3 || max_v > 256 || max_t < 1 || max_t > 256)
    return fail(GTSR_ELIMIT, "encode_meshlets: max_vertices must be 3..256, max_triangles 1..256");
  if (params->flags & ~uint32_t(GTSR_ENCODE_EXACT_STRIPS))
    return fail(GTSR_EINVAL, "encode_meshlets: unknown flags");
  const bool exact = params->flags & GTSR_ENCODE_EXACT_STRIPS;
  if (triangle_count > 0xFFFFFFFFull / 5)
    return fail(GTSR_ELIMIT, "encode_meshlets: too many triangles for 32-bit offsets");
  const uint32_t T = static_cast<uint32_t>(triangle_count);
  for (uint64_t t = 0; t < triangle_count; ++t) {
    uint32_t a = indices[3 * t], b = indices[3 * t + 1], c = indices[3 * t + 2];
    if (a >= vertex_count || b >= vertex_count || c >= vertex_count)
      return fail(GTSR_EINVAL, "encode_meshlets: index >= vertex_count at triangle " + std::to_string(t));
    if (a == b || b == c || a == c)
      return fail(GTSR_EDEGENERATE, "encode_meshlets: repeated vertex in triangle " + std::to_string(t));
  }
  gtsr_encoded* E = new (std::nothrow) gtsr_encoded();
  if (!E) return fail(GTSR_ENOMEM, "encode_meshlets: out of memory");
  try {
    E->input_triangles = T;
    E->vert_off.push_back(0);
    E->kept_off.push_back(0);
    if (T == 0) { *out = E; return ok(); }
    // Vertex ids in order of first appearance in the triangle list.  No rule
    // below compares vertex ids: ties go by triangle number, the edge
    // direction test compares the two ends of one edge (a relabelling flips it
    // for both of that edge's half-edges alike), and each meshlet renumbers
    // its vertices by first appearance.  So the streams are the same, but
    // triangles near each other in the list, which share vertices, get nearby
    // ids, and the per-vertex arrays are walked with locality instead of at
    // random.  The vertex lists are mapped back to the caller's ids at the end.
    std::vector<uint32_t> rel(3ull * T), orig;
    {
      std::vector<uint32_t> first(vertex_count, kNone);
      for (uint64_t i = 0; i < 3ull * T; ++i) {
        uint32_t& f = first[indices[i]];
        if (f == kNone) {
          f = static_cast<uint32_t>(orig.size());
          orig.push_back(indices[i]);
        }
        rel[i] = f;
      }
    }
    const uint32_t* idx = rel.data();
    const uint32_t V = static_cast<uint32_t>(orig.size());
    Adjacency A;
    build_adjacency(idx, T, V, A);
    Meshlets M;
    build_meshlets(idx, T, V, A, max_v, max_t, M);
    const uint32_t nm = static_cast<uint32_t>(M.start.size() - 1);

    uint32_t threads = params->threads ? params->threads : std::max(1u, std::thread::hardware_concurrency());
    threads = std::max(1u, std::min(threads, (nm + 63) / 64));
    std::vector<Piece> pieces(threads);
    std::vector<std::thread> pool;
    for (uint32_t i = 0; i < threads; ++i) {
      uint32_t m0 = static_cast<uint32_t>(uint64_t(nm) * i / threads);
      uint32_t m1 = static_cast<uint32_t>(uint64_t(nm) * (i + 1) / threads);
      if (threads == 1) encode_range(idx, A, M, m0, m1, max_t, exact, pieces[i]);
      else pool.emplace_back(encode_range, idx, std::cref(A), std::cref(M), m0, m1, max_t, exact,
                             std::ref(pieces[i]));
    }
    for (auto& th : pool) th.join();

    uint64_t n_desc = 0, n_bits = 0, n_reuse = 0, n_verts = 0, n_tris = 0;
    for (const Piece& P : pieces) {
      n_desc += P.desc.size(); n_bits += P.bits.size(); n_reuse += P.reuse.size();
      n_verts += P.verts.size(); n_tris += P.strip_tris;
    }
    if (n_tris > 0xFFFFFFFFull || n_reuse > 0xFFFFFFFFull || n_bits / 2 > 0xFFFFFFFFull) {
      delete E;
      return fail(GTSR_ELIMIT, "encode_meshlets: stream exceeds 32-bit offsets");
    }
    E->meshlets.reserve(n_desc);
    E->bits.resize(n_bits * 8);
    E->reuse.reserve(n_reuse);
    E->verts.reserve(n_verts);
    E->vert_off.reserve(n_desc + 1);
    E->kept_off.reserve(n_desc + 1);
    uint64_t ko = 0;
    uint64_t chunk0 = 0, reuse0 = 0, out0 = 0, vo = 0;
    for (const Piece& P : pieces) {
      for (gtsr_meshlet d : P.desc) {
        d.chunk_off += static_cast<uint32_t>(chunk0);
        d.reuse_off += static_cast<uint32_t>(reuse0);
        d.out_off += static_cast<uint32_t>(out0);
        E->meshlets.push_back(d);
      }
      if (!P.bits.empty()) std::memcpy(E->bits.data() + chunk0 * 16, P.bits.data(), P.bits.size() * 8);
      E->reuse.insert(E->reuse.end(), P.reuse.begin(), P.reuse.end());
      for (uint32_t v : P.verts) E->verts.push_back(orig[v]);   // back to the caller's vertex ids
      E->tri_ids.insert(E->tri_ids.end(), P.tri_ids.begin(), P.tri_ids.end());
      for (uint32_t v : P.vcount) { vo += v; E->vert_off.push_back(vo); }
      for (uint32_t k : P.kept) { ko += k; E->kept_off.push_back(static_cast<uint32_t>(ko)); }
      chunk0 += P.bits.size() / 2;
      reuse0 += P.reuse.size();
      out0 += P.strip_tris;
      E->restarts += P.restarts;
      E->split_meshlets += P.splits;
      E->payload_bits += P.payload;
      E->stored_bytes += P.stored;
      E->exact_tried += P.exact_tried;
      E->exact_proven += P.exact_proven;
    }
    E->strip_triangles = out0;
    E->reuse_count = reuse0;
  } catch (const std::bad_alloc&) {
    delete E;
    return fail(GTSR_ENOMEM, "encode_meshlets: out of memory");
  }
  *out = E;
  return ok();
}

extern "C" int gtsr_encoded_view_get(const gtsr_encoded* e, gtsr_encoded_view* v) {
  if (!e || !v) return fail(GTSR_EINVAL, "gtsr_encoded_view_get: null argument");
  std::memset(v, 0, sizeof(*v));
  v->meshlet_count = static_cast<uint32_t>(e->meshlets.size());
  v->input_triangles = e->input_triangles;
  v->strip_triangles = e->strip_triangles;
  v->restarts = e->restarts;
  v->reuse_count = e->reuse_count;
  v->split_meshlets = e->split_meshlets;
  v->meshlets = e->meshlets.data();
  v->bits = e->bits.data();
  v->bits_bytes = e->bits.size();
  v->reuse = e->reuse.data();
  v->reuse_bytes = e->reuse.size();
  v->vertices = e->verts.data();
  v->vert_off = e->vert_off.data();
  v->payload_bits = e->payload_bits;
  v->stored_bytes = e->stored_bytes;
  v->kept_off = e->kept_off.data();
  v->tri_ids = e->tri_ids.data();
  v->exact_tried = e->exact_tried;
  v->exact_proven = e->exact_proven;
  return ok();
}

extern "C" void gtsr_encoded_free(gtsr_encoded* e) { delete e; }

extern "C" int gtsr_min_strips(const uint32_t* indices, uint32_t triangle_count, uint64_t node_limit,
                               uint32_t* strips, uint32_t* proven) {
  if (!strips || !proven || (triangle_count && !indices)) return fail(GTSR_EINVAL, "gtsr_min_strips: null argument");
  if (triangle_count > kMaxStripTris) return fail(GTSR_ELIMIT, "gtsr_min_strips: more than 256 triangles");
  uint32_t V = 0;
  for (uint64_t k = 0; k < 3ull * triangle_count; ++k) V = std::max(V, indices[k] + 1);
  try {
    Adjacency A;
    build_adjacency(indices, triangle_count, V, A);
    int16_t lnbr[3 * kMaxStripTris];
    for (uint64_t h = 0; h < 3ull * triangle_count; ++h)
      lnbr[h] = A.nbr[h] == kNone ? int16_t(-1) : static_cast<int16_t>(A.nbr[h]);
    ExactStrips ex;
    bool done = false;
    *strips = triangle_count ? ex.solve(lnbr, triangle_count, triangle_count, node_limit, &done) : 0;
    *proven = done ? 1u : 0u;
  } catch (const std::bad_alloc&) {
    return fail(GTSR_ENOMEM, "gtsr_min_strips: out of memory");
  }
  return ok();
}
