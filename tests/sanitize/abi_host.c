/*
 * abi_host.c -- drives the library's host code without a GPU, for a build of
 * that code under AddressSanitizer and UndefinedBehaviorSanitizer: the
 * argument checks every entry point makes before touching the device, the
 * status strings, context creation without a device, and the tune store with
 * its JSON reader (valid files, every truncation of one, seeded byte
 * mutations, hostile nesting and numbers, report buffers of every small
 * size).  Prints "abi_host ok" and exits 0 when every check holds; a failed
 * check exits 1, a sanitizer report aborts.
 *
 * Usage: abi_host <scratch directory>
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dgal.h"

#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);          \
      exit(1);                                                              \
    }                                                                       \
  } while (0)

static char dir[4096];

static void path_of(char *out, size_t n, const char *name) {
  snprintf(out, n, "%s/%s", dir, name);
}

static void write_file(const char *path, const char *data, size_t len) {
  FILE *f = fopen(path, "wb");
  CHECK(f != NULL);
  CHECK(fwrite(data, 1, len, f) == len);
  CHECK(fclose(f) == 0);
}

static void null_context(void) {
  dgal_polys p;
  memset(&p, 0, sizeof(p));
  p.kmax = 4;
  dgal_saved s;
  memset(&s, 0, sizeof(s));
  dgal_boxes bx;
  memset(&bx, 0, sizeof(bx));
  bx.dim = 5;
  int64_t a = 0, b = 0, t = 0;
  char buf[64];
  CHECK(dgal_iou_pairs(NULL, p, p, NULL, NULL, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_iou_matrix(NULL, p, p, NULL, NULL, NULL, 0, 0, NULL, 0, &s, NULL) == DGAL_EINVAL);
  CHECK(dgal_iou_matrix(NULL, p, p, NULL, NULL, NULL, 0, 0, NULL, 0, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_iou_matrix_noalloc(NULL, p, p, NULL, NULL, NULL, 0, 0, NULL, 0, NULL) ==
        DGAL_EINVAL);
  CHECK(dgal_iou_backward(NULL, DGAL_PAIRS, p, p, NULL, NULL, NULL, 0, 0, NULL, 0, NULL, NULL,
                          NULL, NULL, NULL, NULL, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_iou_backward(NULL, DGAL_MATRIX, p, p, NULL, NULL, NULL, 0, 0, NULL, 0, NULL, NULL,
                          &s, NULL, NULL, NULL, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_intersect(NULL, p, p, NULL, NULL, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_intersect_backward(NULL, p, p, NULL, NULL, NULL, NULL, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_area(NULL, p, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_area_backward(NULL, p, NULL, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_iou_boxes(NULL, bx, bx, NULL, NULL, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_iou_boxes_backward(NULL, bx, bx, NULL, NULL, NULL, NULL, NULL, NULL) ==
        DGAL_EINVAL);
  CHECK(dgal_iou_simple_pairs(NULL, p, p, NULL, NULL, NULL, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_iou_simple_backward(NULL, p, p, NULL, NULL, NULL, NULL, NULL, NULL, NULL) ==
        DGAL_EINVAL);
  CHECK(dgal_validate(NULL, p, NULL, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_validate_simple(NULL, p, NULL, NULL, NULL) == DGAL_EINVAL);
  CHECK(dgal_set_validate(NULL, 1) == DGAL_EINVAL);
  CHECK(dgal_set_autotune(NULL, 1) == DGAL_EINVAL);
  CHECK(dgal_autotune_report(NULL, buf, sizeof(buf)) == DGAL_EINVAL);
  CHECK(dgal_set_profiling(NULL, 1) == DGAL_EINVAL);
  CHECK(dgal_profile_report(NULL, buf, sizeof(buf)) == DGAL_EINVAL);
  CHECK(dgal_set_path_stats(NULL, 1) == DGAL_EINVAL);
  CHECK(dgal_path_stats(NULL, &a, &b, &t, NULL) == DGAL_EINVAL);
  CHECK(dgal_check(NULL, NULL) == DGAL_EINVAL);
  dgal_destroy(NULL);
  CHECK(dgal_create(NULL, 0) == DGAL_EINVAL);
  /* no device here: creation fails cleanly and leaves NULL */
  dgal_ctx *c = (dgal_ctx *)&s;
  const int st = dgal_create(&c, 0);
  CHECK(st == DGAL_EHIP || st == DGAL_EINVAL);
  CHECK(c == NULL);
  for (int k = -8; k <= 8; ++k) CHECK(dgal_status_string(k) != NULL);
}

static const char *valid_cache =
    "{\"format\": \"dgal-tune-cache\", \"version\": 1, \"note\": [true, false, null, -1.5e3],\n"
    " \"entries\": [\n"
    "  {\"key\": \"gfx950/matrix_fwd/K4/fixed1/z1/seg1/b17.7\", \"grid\": 0, \"cull_mult\": 16,"
    " \"exact_mult\": 8, \"bwd_mult\": 0, \"tile_rows\": 4, \"ms\": 0.25},\n"
    "  {\"key\": \"gfx950/pairs_fwd/K8/fixed0/z0/seg1/b19\", \"grid\": 4096, \"x\": {\"y\": []}},\n"
    "  {\"key\": \"gfx950/matrix_bwd/K4/fixed1/z1/seg1/b17.7\", \"bwd_mult\": 16,"
    " \"s\": \"\\\"\\\\\\/\\b\\f\\n\\r\\t\\u0041\"}\n"
    " ]}\n";

static void tune_cache(void) {
  char p1[4200], p2[4200], p3[4200];
  path_of(p1, sizeof(p1), "valid.json");
  path_of(p2, sizeof(p2), "saved.json");
  path_of(p3, sizeof(p3), "fuzz.json");
  const size_t len = strlen(valid_cache);
  write_file(p1, valid_cache, len);
  CHECK(dgal_tune_cache_clear() == DGAL_OK);
  CHECK(dgal_tune_cache_load(p1) == 3);
  /* reports into every small buffer size: truncated, always terminated */
  char rep[2048];
  for (int64_t n = 0; n < (int64_t)sizeof(rep); ++n) {
    memset(rep, 'Z', sizeof(rep));
    CHECK(dgal_tune_cache_report(n ? rep : NULL, n) == 3);
    if (n > 0) CHECK(memchr(rep, '\0', (size_t)n) != NULL);
  }
  CHECK(dgal_tune_cache_report(NULL, -1) == DGAL_EINVAL);
  CHECK(dgal_tune_cache_save(p2) == DGAL_OK);
  CHECK(dgal_tune_cache_clear() == DGAL_OK);
  CHECK(dgal_tune_cache_load(p2) == 3);
  CHECK(dgal_tune_cache_load(NULL) == DGAL_EINVAL);
  CHECK(dgal_tune_cache_load("") == DGAL_EINVAL);
  CHECK(dgal_tune_cache_save(NULL) == DGAL_EINVAL);
  {
    char missing[4200];
    path_of(missing, sizeof(missing), "no/such/file.json");
    CHECK(dgal_tune_cache_load(missing) == DGAL_EIO);
    CHECK(dgal_tune_cache_save(missing) == DGAL_EIO);
  }
  /* every truncation of a valid file loads whole or is refused */
  for (size_t n = 0; n < len; ++n) {
    write_file(p3, valid_cache, n);
    const int r = dgal_tune_cache_load(p3);
    CHECK(r == DGAL_EINVAL || r == 3);
  }
  /* seeded byte mutations: whatever the result, no sanitizer report */
  char *m = (char *)malloc(len + 1);
  CHECK(m != NULL);
  uint64_t x = 0x9E3779B97F4A7C15ull;
  const char alphabet[] = "{}[]\",:0123456789.eE+-truefalsnl \\u\n\x01\xff";
  for (int it = 0; it < 4000; ++it) {
    memcpy(m, valid_cache, len + 1);
    const int edits = 1 + (int)(x % 4);
    for (int e = 0; e < edits; ++e) {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      m[x % len] = alphabet[(x >> 20) % (sizeof(alphabet) - 1)];
    }
    write_file(p3, m, len);
    const int r = dgal_tune_cache_load(p3);
    CHECK(r == DGAL_EINVAL || (r >= 0 && r <= 3));
  }
  free(m);
  /* hostile shapes: deep nesting, long keys, extreme numbers */
  {
    static char deep[20100];
    size_t k = 0;
    k += (size_t)snprintf(deep, sizeof(deep), "{\"format\": \"dgal-tune-cache\", \"version\": 1, \"entries\": ");
    for (int i = 0; i < 10000; ++i) deep[k++] = '[';
    for (int i = 0; i < 10; ++i) deep[k++] = ']';
    deep[k] = '\0';
    write_file(p3, deep, k);
    CHECK(dgal_tune_cache_load(p3) == DGAL_EINVAL);
  }
  const char *bad[] = {
      "{\"format\": \"dgal-tune-cache\", \"version\": 1, \"entries\": [{\"key\": \"k\", \"grid\": 1e999}]}",
      "{\"format\": \"dgal-tune-cache\", \"version\": 1, \"entries\": [{\"key\": \"k\", \"grid\": -0.5}]}",
      "{\"format\": \"dgal-tune-cache\", \"version\": 1, \"entries\": [{\"key\": \"k\", \"grid\": 1e}]}",
      "{\"format\": \"dgal-tune-cache\", \"version\": 1, \"entries\": [{\"key\": \"\\u00e9\"}]}",
      "{\"format\": \"dgal-tune-cache\", \"version\": 1, \"entries\": [{\"key\": \"\\uZZZZ\"}]}",
      "{\"format\": \"dgal-tune-cache\", \"version\": 1, \"entries\": [{\"key\": \"k\", \"ms\": 1e300}]}",
      "\"dgal-tune-cache\"",
      "-",
  };
  for (size_t i = 0; i < sizeof(bad) / sizeof(bad[0]); ++i) {
    write_file(p3, bad[i], strlen(bad[i]));
    CHECK(dgal_tune_cache_load(p3) == DGAL_EINVAL);
  }
  {
    char longkey[700];
    char key[400];
    memset(key, 'a', sizeof(key) - 1);
    key[sizeof(key) - 1] = '\0';
    snprintf(longkey, sizeof(longkey),
             "{\"format\": \"dgal-tune-cache\", \"version\": 1, \"entries\": [{\"key\": \"%s\"}]}",
             key);
    write_file(p3, longkey, strlen(longkey));
    CHECK(dgal_tune_cache_load(p3) == DGAL_EINVAL);
  }
  CHECK(dgal_tune_cache_clear() == DGAL_OK);
  CHECK(dgal_tune_cache_report(NULL, 0) == 0);
}

int main(int argc, char **argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: abi_host <scratch directory>\n");
    return 2;
  }
  snprintf(dir, sizeof(dir), "%s", argv[1]);
  null_context();
  tune_cache();
  printf("abi_host ok\n");
  return 0;
}
