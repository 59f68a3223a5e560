/* The C ABI used from plain C99, host calls only (no device is needed):
 * encode a 16x16 grid, validate its stream, plan a batch, convert it to
 * plain GTS, write both to a .gtsr file, read them back, and check every
 * error path's status code and message.  Built with gcc against libgtsr.so
 * and run by tests/test_abi_c_cpu.py. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gtsr.h"

static int checks = 0;

#define CHECK(cond)                                                              \
  do {                                                                           \
    ++checks;                                                                    \
    if (!(cond)) {                                                               \
      fprintf(stderr, "%s:%d: check failed: %s (last error: %s)\n", __FILE__, \
              __LINE__, #cond, gtsr_last_error());                               \
      exit(1);                                                                   \
    }                                                                            \
  } while (0)

int main(int argc, char** argv) {
  const char* path = argc > 1 ? argv[1] : "abi_host_test.gtsr";
  /* a 16x16 quad grid, two CCW triangles per quad */
  enum { N = 16, V = (N + 1) * (N + 1), T = 2 * N * N };
  static uint32_t tri[3 * T];
  uint32_t t = 0;
  for (uint32_t y = 0; y < N; ++y)
    for (uint32_t x = 0; x < N; ++x) {
      const uint32_t a = y * (N + 1) + x, b = a + 1, c = a + N + 1, d = c + 1;
      const uint32_t q[6] = {a, b, d, a, d, c};
      memcpy(tri + 3 * t, q, sizeof q);
      t += 2;
    }

  gtsr_encode_params prm = {64, 126, 1, 0};
  gtsr_encoded* enc = NULL;
  CHECK(encode_meshlets(tri, T, V, &prm, &enc) == GTSR_OK && enc);
  gtsr_encoded_view v;
  CHECK(gtsr_encoded_view_get(enc, &v) == GTSR_OK);
  CHECK(v.input_triangles == T && v.strip_triangles == T + 4 * v.restarts);
  CHECK(v.meshlet_count > 0 && v.vert_off[v.meshlet_count] > 0);

  gtsr_stream s = {v.meshlets, v.bits, v.reuse, v.meshlet_count, 0, v.bits_bytes, v.reuse_bytes,
                   v.strip_triangles};
  CHECK(gtsr_validate(&s) == GTSR_OK);

  /* a batch plan over two copies of the mesh: items cover every meshlet once */
  const gtsr_meshlet* ms[2] = {v.meshlets, v.meshlets};
  const uint32_t counts[2] = {v.meshlet_count, v.meshlet_count};
  uint32_t need = 0;
  CHECK(gtsr_plan_batch(ms, counts, 2, 200, NULL, 0, &need) == GTSR_OK && need >= 2);
  gtsr_work_item* items = calloc(need, sizeof *items);
  uint32_t got = 0;
  CHECK(items && gtsr_plan_batch(ms, counts, 2, 200, items, need, &got) == GTSR_OK && got == need);
  uint32_t covered[2] = {0, 0};
  for (uint32_t i = 0; i < got; ++i) {
    CHECK(items[i].mesh < 2 && items[i].first == covered[items[i].mesh] && items[i].end > items[i].first);
    covered[items[i].mesh] = items[i].end;
  }
  CHECK(covered[0] == v.meshlet_count && covered[1] == v.meshlet_count);

  /* plain GTS: one 8-byte word per chunk, T_s - 1 index bytes per meshlet */
  gtsr_meshlet* gd = calloc(v.meshlet_count, sizeof *gd);
  uint8_t* words = calloc(v.bits_bytes / 2 + 1, 1);
  uint8_t* index = calloc(v.strip_triangles, 1);
  CHECK(gd && words && index);
  CHECK(gtsr_gts_from_reuse(&s, gd, words, v.bits_bytes / 2, index, v.strip_triangles - v.meshlet_count) ==
        GTSR_OK);

  gtsr_file_mesh fm[2];
  memset(fm, 0, sizeof fm);
  fm[0].format = GTSR_FORMAT_REUSE;
  fm[0].meshlet_count = v.meshlet_count;
  fm[0].strip_triangles = v.strip_triangles;
  fm[0].input_triangles = v.input_triangles;
  fm[0].restarts = v.restarts;
  fm[0].meshlets = v.meshlets;
  fm[0].bits = v.bits;
  fm[0].bits_bytes = v.bits_bytes;
  fm[0].reuse = v.reuse;
  fm[0].reuse_bytes = v.reuse_bytes;
  fm[0].vertices = v.vertices;
  fm[0].vertex_count = v.vert_off[v.meshlet_count];
  fm[0].vert_off = v.vert_off;
  fm[0].kept_off = v.kept_off;
  fm[0].tri_ids = v.tri_ids;
  fm[1] = fm[0];
  fm[1].format = GTSR_FORMAT_GTS;
  fm[1].meshlets = gd;
  fm[1].bits = words;
  fm[1].bits_bytes = v.bits_bytes / 2;
  fm[1].reuse = index;
  fm[1].reuse_bytes = v.strip_triangles - v.meshlet_count;
  fm[1].kept_off = NULL;
  fm[1].tri_ids = NULL;
  CHECK(gtsr_file_write(path, fm, 2) == GTSR_OK);

  gtsr_file* f = NULL;
  CHECK(gtsr_file_open(path, &f) == GTSR_OK && f);
  uint32_t n = 0;
  CHECK(gtsr_file_mesh_count(f, &n) == GTSR_OK && n == 2);
  for (uint32_t i = 0; i < 2; ++i) {
    gtsr_file_mesh g;
    CHECK(gtsr_file_mesh_get(f, i, &g) == GTSR_OK);
    CHECK(g.format == fm[i].format && g.meshlet_count == fm[i].meshlet_count);
    CHECK(g.strip_triangles == fm[i].strip_triangles && g.restarts == fm[i].restarts);
    CHECK(memcmp(g.meshlets, fm[i].meshlets, 16ull * g.meshlet_count) == 0);
    CHECK(g.bits_bytes == fm[i].bits_bytes && memcmp(g.bits, fm[i].bits, g.bits_bytes) == 0);
    CHECK(g.reuse_bytes == fm[i].reuse_bytes && memcmp(g.reuse, fm[i].reuse, g.reuse_bytes) == 0);
    CHECK(memcmp(g.vert_off, fm[i].vert_off, 8ull * (g.meshlet_count + 1)) == 0);
    CHECK((g.kept_off != NULL) == (fm[i].kept_off != NULL) && (g.tri_ids != NULL) == (fm[i].tri_ids != NULL));
  }
  gtsr_file_mesh none;
  CHECK(gtsr_file_mesh_get(f, 2, &none) == GTSR_EINVAL && strstr(gtsr_last_error(), "out of range"));
  gtsr_file_close(f);

  /* error paths: status codes and messages */
  gtsr_encoded* bad = NULL;
  CHECK(encode_meshlets(tri, T, 3, &prm, &bad) != GTSR_OK && bad == NULL);   /* vertex ids past the count */
  CHECK(strlen(gtsr_last_error()) > 0);
  CHECK(gtsr_validate(NULL) == GTSR_EINVAL);
  gtsr_meshlet broken = v.meshlets[0];
  broken.vert_count = 2;
  gtsr_stream bs = s;
  bs.meshlets = &broken;
  bs.meshlet_count = 1;
  CHECK(gtsr_validate(&bs) == GTSR_ECORRUPT && strstr(gtsr_last_error(), "vert_count"));
  CHECK(gtsr_file_open("/nonexistent/dir/x.gtsr", &f) == GTSR_EIO);
  CHECK(gtsr_file_write(NULL, fm, 1) == GTSR_EINVAL);

  free(items);
  free(gd);
  free(words);
  free(index);
  gtsr_encoded_free(enc);
  printf("abi_host_test: %d checks passed\n", checks);
  return 0;
}
