/* Host-side paths of the C ABI that run without a GPU: status strings,
 * defaults, argument checks, and the degree-predictor file reader on valid
 * and damaged files. Built with AddressSanitizer and UndefinedBehaviorSanitizer
 * over a host-only build of the library (no device code), so every host
 * access and integer operation of these paths is checked. Exit status 0 when
 * every call returns what it should; the sanitizers abort on any error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "bernnn.h"

static int fails = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "failed: %s (line %d)\n", #cond, __LINE__); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

static void put_u32(FILE *f, uint32_t v) { fwrite(&v, 4, 1, f); }

/* a predictor file: magic, version, count, `np` floats (only `nwrite` of
 * them written), metadata length `ml` (only `mwrite` bytes written) */
static void write_pred(const char *path, const char *magic, uint32_t ver, uint32_t np, uint32_t nwrite, uint32_t ml,
                       uint32_t mwrite) {
  FILE *f = fopen(path, "wb");
  fwrite(magic, 1, 8, f);
  put_u32(f, ver);
  put_u32(f, np);
  float z = 0.25f;
  for (uint32_t i = 0; i < nwrite; ++i) fwrite(&z, 4, 1, f);
  put_u32(f, ml);
  for (uint32_t i = 0; i < mwrite; ++i) fputc('m', f);
  fclose(f);
}

int main(int argc, char **argv) {
  const char *dir = argc > 1 ? argv[1] : ".";
  char path[4096];
  EXPECT(strcmp(bern_status_str(BERN_OK), "BERN_OK") == 0);
  EXPECT(strcmp(bern_status_str(12345), "BERN_UNKNOWN") == 0);
  bern_opts o;
  bern_opts_default(&o);
  EXPECT(o.L == 2 && o.graph == 0 && o.lin == 0);
  bern_train_opts t;
  bern_train_opts_default(&t);
  EXPECT(t.epochs > 0 && t.batch > 0);

  /* networks rejected before any device call */
  const int32_t widths[3] = {2, 3, 1};
  double W[9] = {0}, b[4] = {0};
  bern_net *net = NULL;
  EXPECT(bern_net_create(0, widths, W, b, &net) == BERN_E_ARG);
  EXPECT(bern_net_create(2, NULL, W, b, &net) == BERN_E_ARG);
  const int32_t zero_in[3] = {0, 3, 1};
  EXPECT(bern_net_create(2, zero_in, W, b, &net) == BERN_E_ARG);
  W[1] = INFINITY;
  EXPECT(bern_net_create(2, widths, W, b, &net) == BERN_E_NUMERIC);
  EXPECT(strlen(bern_last_error()) > 0);
  W[1] = 0.0;
  EXPECT(bern_net_create(2, widths, W, b, NULL) == BERN_E_ARG);
  size_t sz = 0;
  EXPECT(bern_workspace_size(NULL, &o, 1, &sz, NULL) == BERN_E_ARG);
  EXPECT(bern_bounds(NULL, &o, 1, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, NULL) == BERN_E_ARG);
  EXPECT(bern_relu_poly(1, 9, NULL, NULL, NULL, NULL, NULL) == BERN_E_ARG);
  EXPECT(bern_tune_variants(-1) <= 0);
  EXPECT(bern_tune_variants(1 << 20) <= 0);
  EXPECT(bern_prof_name(-1) != NULL && bern_prof_name(1 << 20) != NULL);

  /* predictor files: every damaged form is refused by the reader */
  const uint32_t np = (uint32_t)bern_pred_params();
  bern_pred *p = NULL;
  EXPECT(bern_pred_load(NULL, &p) == BERN_E_ARG);
  snprintf(path, sizeof path, "%s/missing.bin", dir);
  EXPECT(bern_pred_load(path, &p) == BERN_E_ARG && p == NULL);
  snprintf(path, sizeof path, "%s/badmagic.bin", dir);
  write_pred(path, "BERNPREX", 1, np, np, 0, 0);
  EXPECT(bern_pred_load(path, &p) != BERN_OK && p == NULL);
  snprintf(path, sizeof path, "%s/badver.bin", dir);
  write_pred(path, "BERNPRED", 7, np, np, 0, 0);
  EXPECT(bern_pred_load(path, &p) != BERN_OK && p == NULL);
  snprintf(path, sizeof path, "%s/badcount.bin", dir);
  write_pred(path, "BERNPRED", 1, np + 1, np + 1, 0, 0);
  EXPECT(bern_pred_load(path, &p) != BERN_OK && p == NULL);
  snprintf(path, sizeof path, "%s/short.bin", dir);
  write_pred(path, "BERNPRED", 1, np, np / 2, 0, 0);
  EXPECT(bern_pred_load(path, &p) != BERN_OK && p == NULL);
  snprintf(path, sizeof path, "%s/hugemeta.bin", dir);
  write_pred(path, "BERNPRED", 1, np, np, 0xFFFFFFF0u, 3);
  EXPECT(bern_pred_load(path, &p) != BERN_OK && p == NULL);
  snprintf(path, sizeof path, "%s/empty.bin", dir);
  fclose(fopen(path, "wb"));
  EXPECT(bern_pred_load(path, &p) != BERN_OK && p == NULL);
  /* training rejects bad sizes and options before any device call */
  EXPECT(bern_pred_train(NULL, NULL, 0, &t, path, NULL, &p) == BERN_E_ARG);
  bern_train_opts bad = t;
  bad.batch = 0;
  float X[8] = {0};
  int8_t y[1] = {0};
  EXPECT(bern_pred_train(X, y, 1, &bad, path, NULL, &p) == BERN_E_ARG);
  int8_t ybad[1] = {4};
  EXPECT(bern_pred_train(X, ybad, 1, &t, path, NULL, &p) == BERN_E_ARG);
  X[3] = NAN;
  EXPECT(bern_pred_train(X, y, 1, &t, path, NULL, &p) == BERN_E_NUMERIC);
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("host driver: all calls clean\n");
  return 0;
}
