/*
 * meshgen.c -- construction of synthetic CCW triangle meshes (input data
 * only; nothing here knows about meshlets, strips or the codec).
 *
 *   mg_grid          nx*ny quads, each split along a given diagonal
 *   mg_icosphere     unit icosphere after `level` 1-to-4 subdivisions
 *   mg_sphere_patch  the n faces of a sphere whose centroids score highest
 *                    along a direction (a spherical cap), vertices compacted
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* tri: uint32[2*nx*ny][3]; diag[q] picks quad q's diagonal; perm (may be
 * NULL) renames vertices. */
void mg_grid(uint32_t nx, uint32_t ny, const uint8_t* diag, const uint32_t* perm, uint32_t* tri) {
  const uint64_t w = (uint64_t)nx + 1, nq = (uint64_t)nx * ny;
  for (uint64_t q = 0; q < nq; ++q) {
    uint64_t i = q % nx, j = q / nx;
    uint32_t a = (uint32_t)(j * w + i), b = a + 1, c = (uint32_t)(a + w + 1), d = (uint32_t)(a + w);
    uint32_t t[6];
    if (diag[q] == 0) { t[0] = a; t[1] = b; t[2] = c; t[3] = a; t[4] = c; t[5] = d; }
    else { t[0] = a; t[1] = b; t[2] = d; t[3] = b; t[4] = c; t[5] = d; }
    for (int k = 0; k < 6; ++k) tri[6 * q + k] = perm ? perm[t[k]] : t[k];
  }
}

static const double kIcoV[12][3] = {
    {-1, 1.6180339887498949, 0}, {1, 1.6180339887498949, 0}, {-1, -1.6180339887498949, 0},
    {1, -1.6180339887498949, 0}, {0, -1, 1.6180339887498949}, {0, 1, 1.6180339887498949},
    {0, -1, -1.6180339887498949}, {0, 1, -1.6180339887498949}, {1.6180339887498949, 0, -1},
    {1.6180339887498949, 0, 1}, {-1.6180339887498949, 0, -1}, {-1.6180339887498949, 0, 1}};
static const uint32_t kIcoF[20][3] = {
    {0, 11, 5}, {0, 5, 1}, {0, 1, 7}, {0, 7, 10}, {0, 10, 11}, {1, 5, 9}, {5, 11, 4},
    {11, 10, 2}, {10, 7, 6}, {7, 1, 8}, {3, 9, 4}, {3, 4, 2}, {3, 2, 6}, {3, 6, 8},
    {3, 8, 9}, {4, 9, 5}, {2, 4, 11}, {6, 2, 10}, {8, 6, 7}, {9, 8, 1}};

static void normalize(double* p) {
  double n = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  p[0] /= n; p[1] /= n; p[2] /= n;
}

/* v: double[10*4^level+2][3], f: uint32[20*4^level][3].  Returns 0 or -2. */
int mg_icosphere(uint32_t level, double* v, uint32_t* f) {
  uint64_t nv = 12, nf = 20;
  for (int i = 0; i < 12; ++i) { memcpy(v + 3 * i, kIcoV[i], sizeof(kIcoV[i])); normalize(v + 3 * i); }
  memcpy(f, kIcoF, sizeof(kIcoF));
  uint64_t fmax = 20ull << (2 * level);
  uint32_t* nf_buf = (uint32_t*)malloc(sizeof(uint32_t) * 3 * (fmax ? fmax : 1));
  if (!nf_buf) return -2;
  for (uint32_t L = 0; L < level; ++L) {
    uint64_t ne = nf * 3 / 2, cap = 1;
    while (cap < 2 * ne) cap <<= 1;
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * cap);
    uint32_t* val = (uint32_t*)malloc(sizeof(uint32_t) * cap);
    if (!key || !val) { free(key); free(val); free(nf_buf); return -2; }
    memset(key, 0xFF, sizeof(uint64_t) * cap);
    for (uint64_t q = 0; q < nf; ++q) {
      uint32_t m[3];
      for (int e = 0; e < 3; ++e) {
        uint32_t a = f[3 * q + e], b = f[3 * q + (e + 1) % 3];
        uint64_t lo = a < b ? a : b, hi = a < b ? b : a, k = lo << 32 | hi;
        uint64_t h = (k * 0x9E3779B97F4A7C15ull) >> 20;
        for (;;) {
          h &= cap - 1;
          if (key[h] == k) { m[e] = val[h]; break; }
          if (key[h] == ~0ull) {
            key[h] = k; val[h] = (uint32_t)nv; m[e] = (uint32_t)nv;
            double* p = v + 3 * nv;
            for (int c = 0; c < 3; ++c) p[c] = 0.5 * (v[3 * a + c] + v[3 * b + c]);
            normalize(p);
            ++nv;
            break;
          }
          ++h;
        }
      }
      uint32_t a = f[3 * q], b = f[3 * q + 1], c = f[3 * q + 2];
      uint32_t ab = m[0], bc = m[1], ca = m[2];
      uint32_t* o = nf_buf + 12 * q;
      o[0] = a;  o[1] = ab; o[2] = ca;
      o[3] = ab; o[4] = b;  o[5] = bc;
      o[6] = ca; o[7] = bc; o[8] = c;
      o[9] = ab; o[10] = bc; o[11] = ca;
    }
    free(key); free(val);
    nf *= 4;
    memcpy(f, nf_buf, sizeof(uint32_t) * 3 * nf);
  }
  free(nf_buf);
  return 0;
}

/* Order: higher score first, then lower face number. */
static int better(const double* s, uint32_t x, uint32_t y) {
  return s[x] > s[y] || (s[x] == s[y] && x < y);
}

/* Moves the n best faces (by `better`) to idx[0..n) in O(F) expected time. */
static void select_best(const double* s, uint32_t* idx, uint64_t F, uint64_t n, uint64_t seed) {
  uint64_t lo = 0, hi = F;   /* the boundary n lies in [lo, hi) */
  uint64_t x = seed | 1;
  while (hi - lo > 1) {
    x ^= x << 13; x ^= x >> 7; x ^= x << 17;
    uint64_t p = lo + x % (hi - lo);
    uint32_t piv = idx[p];
    /* three-way partition around piv: better | piv | worse */
    uint64_t i = lo, lt = lo, gt = hi;
    while (i < gt) {
      uint32_t y = idx[i];
      if (y == piv) { ++i; continue; }
      if (better(s, y, piv)) { idx[i] = idx[lt]; idx[lt] = y; ++lt; ++i; }
      else { --gt; idx[i] = idx[gt]; idx[gt] = y; }
    }
    /* [lo,lt) better, [lt,gt) == piv (one face), [gt,hi) worse */
    if (n < lt) hi = lt;
    else if (n >= gt) lo = gt;
    else return;
  }
}

/* The n faces of (v, f) whose centroids have the largest dot product with
 * dir; out_tri receives them in face order with vertices renumbered
 * 0..nverts-1 in increasing original order.  Returns 0, -1 (n > F) or -2. */
int mg_sphere_patch(const double* v, uint64_t V, const uint32_t* f, uint64_t F, uint64_t n,
                    const double* dir, uint32_t* out_tri, uint32_t* out_nverts) {
  if (n > F) return -1;
  double* s = (double*)malloc(sizeof(double) * F);
  uint32_t* idx = (uint32_t*)malloc(sizeof(uint32_t) * F);
  uint8_t* take = (uint8_t*)calloc(F, 1);
  uint32_t* remap = (uint32_t*)malloc(sizeof(uint32_t) * V);
  if (!s || !idx || !take || !remap) { free(s); free(idx); free(take); free(remap); return -2; }
  for (uint64_t q = 0; q < F; ++q) {
    const uint32_t* t = f + 3 * q;
    double c0 = v[3 * t[0]] + v[3 * t[1]] + v[3 * t[2]];
    double c1 = v[3 * t[0] + 1] + v[3 * t[1] + 1] + v[3 * t[2] + 1];
    double c2 = v[3 * t[0] + 2] + v[3 * t[1] + 2] + v[3 * t[2] + 2];
    s[q] = c0 * dir[0] + c1 * dir[1] + c2 * dir[2];
    idx[q] = (uint32_t)q;
  }
  if (n < F) select_best(s, idx, F, n, 0x2404635900000001ull ^ F);
  for (uint64_t i = 0; i < n; ++i) take[idx[i]] = 1;
  for (uint64_t i = 0; i < V; ++i) remap[i] = 0;
  for (uint64_t q = 0; q < F; ++q)
    if (take[q]) for (int k = 0; k < 3; ++k) remap[f[3 * q + k]] = 1;
  uint32_t nv = 0;
  for (uint64_t i = 0; i < V; ++i) remap[i] = remap[i] ? nv++ : 0xFFFFFFFFu;
  uint64_t o = 0;
  for (uint64_t q = 0; q < F; ++q)
    if (take[q]) { for (int k = 0; k < 3; ++k) out_tri[3 * o + k] = remap[f[3 * q + k]]; ++o; }
  *out_nverts = nv;
  free(s); free(idx); free(take); free(remap);
  return 0;
}
