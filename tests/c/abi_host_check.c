/* Host-only use of the library through its C header, compiled as C99: the
 * declarations must be plain C, and the calls that need no GPU (parameter
 * map, workspace sizing, argument validation before any device work) must
 * behave as documented. Prints "ok" and exits 0 on success. */
#include <stdio.h>
#include <string.h>

#include "mclbm.h"

static int fails = 0;

static void expect(int cond, const char* what) {
  if (!cond) {
    printf("FAILED: %s\n", what);
    ++fails;
  }
}

int main(void) {
  mclbm_sample_desc d[2];
  memset(d, 0, sizeof(d));
  d[0].n = 32; d[0].u0 = 0.05; d[0].re = 100.0; d[0].amp = 0.05; d[0].project = 1; d[0].stride = 1;
  d[1] = d[0];
  d[1].n = 64; d[1].stride = 4;

  const double om = mclbm_omega(32, 0.05, 100.0);
  expect(om > 1.96 && om < 1.98, "omega of 32^3, U0 0.05, Re 100");
  expect(mclbm_omega(0, 0.05, 100.0) == 0.0, "omega rejects n = 0");

  const size_t b27 = mclbm_workspace_bytes(2, d, MCLBM_FP32_SHIFTED, MCLBM_D3Q27);
  const size_t b19 = mclbm_workspace_bytes(2, d, MCLBM_FP32_SHIFTED, MCLBM_D3Q19);
  const size_t b64 = mclbm_workspace_bytes(2, d, MCLBM_FP64, MCLBM_D3Q27);
  expect(b27 >= (size_t)27 * (32 * 32 * 32 + 64 * 64 * 64) * 4, "D3Q27 FP32 workspace holds the populations");
  expect(b19 < b27 && b64 > b27, "workspace ordering D3Q19 < D3Q27 FP32 < D3Q27 FP64");
  expect(mclbm_workspace_bytes(2, d, MCLBM_FP32_SHIFTED, 15) == 0, "unknown lattice");

  mclbm_ctx* ctx = NULL;
  mclbm_status st = mclbm_create(&ctx, 2, d, MCLBM_FP32_SHIFTED, MCLBM_D3Q27, NULL, b27, NULL);
  expect(st == MCLBM_ERR_ARG && ctx == NULL, "create without a workspace fails before any device work");
  expect(strstr(mclbm_last_error(), "workspace") != NULL, "the error message names the workspace");
  st = mclbm_create(&ctx, 2, d, MCLBM_FP32_SHIFTED, MCLBM_D3Q27, (void*)256, 16, NULL);
  expect(st == MCLBM_ERR_OOM, "create with a too small workspace");
  expect(mclbm_ticks(NULL) == -1, "ticks of a NULL context");
  expect(mclbm_stream_copy(NULL, NULL, 16, NULL) == MCLBM_ERR_ARG, "stream copy of NULL buffers");

  /* host-only arithmetic and argument checks of the statistics entry points */
  {
    const double ns[3] = {64.0, 128.0, 256.0}, ds[3] = {0.4, 0.2, 0.1};
    double slope = 0.0;
    expect(mclbm_eoc_slope(ns, ds, 3, &slope) == MCLBM_OK && slope > -1.0000001 && slope < -0.9999999,
           "slope of d ~ 1/n is -1");
    expect(mclbm_eoc_slope(ns, ds, 1, &slope) == MCLBM_ERR_ARG, "one point has no slope");
    expect(mclbm_eoc_slope(NULL, ds, 3, &slope) == MCLBM_ERR_ARG, "slope without resolutions");
  }
  expect(mclbm_ensemble_moments(NULL, 4, 1, 1, NULL, NULL, NULL) == MCLBM_ERR_ARG, "moments of NULL");
  expect(mclbm_ensemble_moments((const double*)256, 1, 1, 1, (double*)256, (double*)512, NULL) == MCLBM_ERR_ARG,
         "a spread of one sample");
  expect(mclbm_sample_error(NULL, NULL, 1, 8, NULL, NULL, 0, NULL) == MCLBM_ERR_ARG, "sample error of NULL");
  expect(mclbm_w1_1pt(NULL, NULL, 1, 8, NULL, NULL, 0, NULL) == MCLBM_ERR_ARG, "W1 of NULL");
  expect(mclbm_sample_error_work_bytes(0) == 0 && mclbm_w1_work_bytes(0) == 0, "work of nothing");
  expect(mclbm_compensate(NULL, 0, 1, NULL, NULL, NULL, NULL, NULL) == MCLBM_ERR_ARG, "compensate without a context");
  expect(mclbm_dissipation(NULL, NULL, 2, 0, 1, NULL, NULL) == MCLBM_ERR_ARG, "dissipation without a context");
  expect(mclbm_checkpoint_bytes(NULL) == 0 && mclbm_ckpt_bytes(NULL, 10, 5) == 0, "checkpoint sizes without a context");
  expect(mclbm_observables_range_work_bytes(NULL, 0, 1) == 0, "observables work without a context");

  if (fails == 0) printf("ok\n");
  return fails == 0 ? 0 : 1;
}
