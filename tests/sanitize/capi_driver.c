/*
 * Driver for the host-sanitized build of the C-ABI library (host code built
 * with AddressSanitizer + UndefinedBehaviorSanitizer, no device code): calls
 * every entry point that needs no GPU -- version, default options, the chi^2
 * quantile over its domain and outside it, context creation without a
 * device, and every entry point with NULL or invalid arguments, which must
 * return an error code and not touch memory.  Prints the quantiles for the
 * test to compare.  Test infrastructure only.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "vfisv.h"

static int fails = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "line %d: expected %s\n", __LINE__, #cond); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

int main(void) {
  EXPECT(vfisv_version() != NULL && strlen(vfisv_version()) > 0);
  vfisv_options o;
  memset(&o, 0x5A, sizeof o);
  vfisv_options_default(&o);
  EXPECT(o.max_iter == 50);
  vfisv_options_default(NULL);

  /* chi^2 quantile: in the domain (printed), outside it (errors) */
  const int dofs[] = {1, 2, 3, 7, 24, 100, 448, 4096, 1000000};
  const double qs[] = {1e-6, 0.01, 0.5, 0.99, 1.0 - 1e-9};
  for (unsigned i = 0; i < sizeof dofs / sizeof dofs[0]; ++i)
    for (unsigned j = 0; j < sizeof qs / sizeof qs[0]; ++j) {
      double x = -1.0;
      EXPECT(vfisv_chi2_quantile(dofs[i], qs[j], &x) == VFISV_OK);
      printf("quantile %d %.17g %.17g\n", dofs[i], qs[j], x);
    }
  double x;
  EXPECT(vfisv_chi2_quantile(0, 0.5, &x) == VFISV_E_INVALID);
  EXPECT(vfisv_chi2_quantile(1000001, 0.5, &x) == VFISV_E_INVALID);
  EXPECT(vfisv_chi2_quantile(10, 0.0, &x) == VFISV_E_INVALID);
  EXPECT(vfisv_chi2_quantile(10, 1.0, &x) == VFISV_E_INVALID);
  EXPECT(vfisv_chi2_quantile(10, NAN, &x) == VFISV_E_INVALID);
  EXPECT(vfisv_chi2_quantile(10, 0.5, NULL) == VFISV_E_INVALID);

  /* no device here: creation fails cleanly and says why */
  vfisv_ctx *ctx = (vfisv_ctx *)&o;
  EXPECT(vfisv_create(&ctx, 0) != VFISV_OK && ctx == NULL);
  EXPECT(strlen(vfisv_last_error(NULL)) > 0);
  EXPECT(vfisv_create(&ctx, -1) != VFISV_OK && ctx == NULL);
  EXPECT(vfisv_create(NULL, 0) == VFISV_E_INVALID);
  EXPECT(vfisv_destroy(NULL) == VFISV_OK);

  /* NULL context / objects / arguments */
  float f[64];
  double d[64];
  int32_t i32[64];
  int64_t i64[64];
  vfisv_instrument *inst = NULL;
  vfisv_instrument_info info;
  vfisv_counters cnt;
  vfisv_tuning tun;
  vfisv_mlp *mlp = NULL;
  vfisv_learned_phases ph;
  EXPECT(vfisv_instrument_create(NULL, NULL, &inst) == VFISV_E_INVALID);
  EXPECT(vfisv_instrument_info_get(NULL, &info) == VFISV_E_INVALID);
  EXPECT(vfisv_instrument_destroy(NULL) == VFISV_OK);
  EXPECT(vfisv_synthesize(NULL, NULL, 1, f, NULL, f, NULL, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_synthesize_voigt(NULL, NULL, 1, f, NULL, f, NULL, 2, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_invert(NULL, NULL, 1, f, f, 0, NULL, NULL, f, d, i32, i32, NULL) ==
         VFISV_E_INVALID);
  EXPECT(vfisv_invert_batches(NULL, NULL, 1, NULL, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_autotune(NULL, NULL, 1, f, f, 0, NULL, 1, &tun, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_init_classical(NULL, NULL, 1, f, f, f, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_init_combined(NULL, NULL, 1, f, f, 0.06f, f, f, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_stokes_weights(NULL, NULL, 1, f, f, f, f, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_get_counters(NULL, &cnt) == VFISV_E_INVALID);
  EXPECT(vfisv_iter_histogram(NULL, 1, i32, 4, i64, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_solve(NULL, 1, f, f, d, 0x3FF, d, i32, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_create(NULL, 24, f, f, f, f, 1, &mlp) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_destroy(NULL) == VFISV_OK);
  EXPECT(vfisv_mlp_num_params(NULL) < 0);
  EXPECT(vfisv_mlp_num_inputs(NULL) < 0);
  EXPECT(vfisv_mlp_get_params(NULL, f, 1) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_set_params(NULL, f, 1) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_forward(NULL, NULL, 1, f, f, f, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_gradient(NULL, NULL, 1, f, f, f, d, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_train_step(NULL, NULL, f, f, i32, 1, 1e-3f, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_take_loss(NULL, d) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_stats(NULL, 1, 24, f, f, f, f, f, f, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_train(NULL, NULL, NULL, NULL, d, d, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_save(NULL, "/nonexistent/net.bin") == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_load(NULL, "/nonexistent/net.bin", &mlp) == VFISV_E_INVALID);
  EXPECT(vfisv_mlp_get_norm(NULL, f, f, f, f) == VFISV_E_INVALID);
  EXPECT(vfisv_invert_learned(NULL, NULL, NULL, 1, f, f, 0, NULL, 15, 0.0, f, d, i32, i32,
                              NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_invert_learned_noalloc(NULL, NULL, NULL, 1, f, f, 0, NULL, 15, 0.0, f, d, i32,
                                      i32, NULL) == VFISV_E_INVALID);
  EXPECT(vfisv_learned_phase_timing(NULL, 1) == VFISV_E_INVALID);
  EXPECT(vfisv_learned_phases_get(NULL, &ph) == VFISV_E_INVALID);
  printf("capi driver: %s\n", fails ? "FAILED" : "ok");
  return fails != 0;
}
