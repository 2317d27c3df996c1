/*
 * A plain C consumer of the libclue C ABI (no Python, no torch), used by the
 * GPU test of the boundary. It reads one event from a binary file, clusters it
 * on HIP device 0 with clue_run and with clue_run_batch (one event), again
 * after a retuning through clue_set_tuning (the tuning struct as a C compiler
 * lays it out), checks that all runs agree, checks two argument errors, and
 * writes the cluster ids and seed flags.
 *
 * Input file:  int64 n; float dc, rho_c, delta_c, delta_o, x_min, y_min, x_max,
 *              y_max; int32 n_layers; float x[n]; float y[n]; int32 layer[n];
 *              float energy[n].
 * Output file: int32 cluster_id[n]; uint8 is_seed[n].
 * Exit status: 0 on success, 1 on a usage or I/O error, 2 on a library or
 * HIP error, 3 when the plain and batched forms disagree.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "clue.h"

#define CHECK_HIP(expr)                                                      \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      fprintf(stderr, "%s: %s\n", #expr, hipGetErrorString(e_));             \
      return 2;                                                              \
    }                                                                        \
  } while (0)

#define CHECK_CLUE(c, expr)                                                  \
  do {                                                                       \
    int r_ = (expr);                                                         \
    if (r_ != CLUE_OK) {                                                     \
      fprintf(stderr, "%s: %d (%s)\n", #expr, r_, clue_last_error(c));       \
      return 2;                                                              \
    }                                                                        \
  } while (0)

static int read_all(FILE *f, void *dst, size_t bytes) { return fread(dst, 1, bytes, f) == bytes ? 0 : -1; }

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s <event.bin> <out.bin>\n", argv[0]);
    return 1;
  }
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 1;
  int64_t n = 0;
  float par[8];
  int32_t n_layers = 0;
  if (read_all(f, &n, sizeof n) || read_all(f, par, sizeof par) || read_all(f, &n_layers, sizeof n_layers) || n < 1) {
    fclose(f);
    return 1;
  }
  const size_t n4 = (size_t)n * 4;
  float *x = malloc(n4), *y = malloc(n4), *e = malloc(n4);
  int32_t *layer = malloc(n4), *cid = malloc(n4), *cid2 = malloc(n4);
  uint8_t *seed = malloc((size_t)n), *seed2 = malloc((size_t)n);
  if (!x || !y || !e || !layer || !cid || !cid2 || !seed || !seed2 || read_all(f, x, n4) || read_all(f, y, n4) ||
      read_all(f, layer, n4) || read_all(f, e, n4)) {
    fclose(f);
    return 1;
  }
  fclose(f);

  clue_params p;
  memset(&p, 0, sizeof p);
  p.dc = par[0];
  p.rho_c = par[1];
  p.delta_c = par[2];
  p.delta_o = par[3];
  p.x_min = par[4];
  p.y_min = par[5];
  p.x_max = par[6];
  p.y_max = par[7];
  p.n_layers = n_layers;
  p.kernel = CLUE_KERNEL_FLAT;
  clue_ctx *c = NULL;
  CHECK_CLUE(NULL, clue_create(&c, &p, 0, n, 1, 0));

  float *dx, *dy, *de;
  int32_t *dl, *dcid, *dev_ids;
  uint8_t *dseed;
  CHECK_HIP(hipMalloc((void **)&dx, n4));
  CHECK_HIP(hipMalloc((void **)&dy, n4));
  CHECK_HIP(hipMalloc((void **)&de, n4));
  CHECK_HIP(hipMalloc((void **)&dl, n4));
  CHECK_HIP(hipMalloc((void **)&dcid, n4));
  CHECK_HIP(hipMalloc((void **)&dev_ids, n4));
  CHECK_HIP(hipMalloc((void **)&dseed, (size_t)n));
  CHECK_HIP(hipMemcpy(dx, x, n4, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dy, y, n4, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(de, e, n4, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dl, layer, n4, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemset(dev_ids, 0, n4));

  /* plain form on the default stream */
  CHECK_CLUE(c, clue_run(c, n, dx, dy, dl, de, dcid, dseed, NULL));
  CHECK_CLUE(c, clue_status(c, NULL));
  CHECK_HIP(hipMemcpy(cid, dcid, n4, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(seed, dseed, (size_t)n, hipMemcpyDeviceToHost));

  /* batched form (one event) on a stream of our own */
  hipStream_t s;
  CHECK_HIP(hipStreamCreate(&s));
  CHECK_HIP(hipMemset(dcid, 0xff, n4));
  CHECK_CLUE(c, clue_run_batch(c, n, 1, dev_ids, dx, dy, dl, de, dcid, dseed, (void *)s));
  CHECK_CLUE(c, clue_status(c, (void *)s));
  CHECK_HIP(hipMemcpy(cid2, dcid, n4, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(seed2, dseed, (size_t)n, hipMemcpyDeviceToHost));
  if (memcmp(cid, cid2, n4) || memcmp(seed, seed2, (size_t)n)) {
    fprintf(stderr, "plain and batched forms disagree\n");
    return 3;
  }

  /* retune from C (small LDS caps force the fallback paths, k-way expansion)
   * and run both forms again: the output must not change */
  clue_tuning t;
  int32_t halo = 0;
  CHECK_CLUE(c, clue_get_tuning(c, &t, &halo));
  if (t.lds_cap < 64 || t.block_x < 1 || halo < 1) return 2;
  t.lds_cap = 96;
  t.plain_lds_cap = 64;
  t.expansion = 2;
  t.nh_first_radius = -1.0f; /* keep */
  CHECK_CLUE(c, clue_set_tuning(c, &t));
  clue_tuning t2;
  CHECK_CLUE(c, clue_get_tuning(c, &t2, &halo));
  if (t2.lds_cap != 96 || t2.plain_lds_cap != 64 || t2.expansion != 2) return 2;
  for (int form = 0; form < 2; ++form) {
    CHECK_HIP(hipMemset(dcid, 0xff, n4));
    if (form == 0)
      CHECK_CLUE(c, clue_run(c, n, dx, dy, dl, de, dcid, dseed, NULL));
    else
      CHECK_CLUE(c, clue_run_batch(c, n, 1, dev_ids, dx, dy, dl, de, dcid, dseed, NULL));
    CHECK_CLUE(c, clue_status(c, NULL));
    CHECK_HIP(hipMemcpy(cid2, dcid, n4, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(seed2, dseed, (size_t)n, hipMemcpyDeviceToHost));
    if (memcmp(cid, cid2, n4) || memcmp(seed, seed2, (size_t)n)) {
      fprintf(stderr, "the retuned %s form disagrees\n", form ? "batched" : "plain");
      return 3;
    }
  }

  /* argument errors come back as codes with a message, nothing is launched */
  if (clue_run(c, -1, dx, dy, dl, de, dcid, dseed, NULL) != CLUE_ERR_ARG || !clue_last_error(c)[0]) return 2;
  if (clue_run(c, n + 1, dx, dy, dl, de, dcid, dseed, NULL) != CLUE_ERR_CAPACITY) return 2;

  CHECK_HIP(hipStreamDestroy(s));
  CHECK_HIP(hipFree(dx));
  CHECK_HIP(hipFree(dy));
  CHECK_HIP(hipFree(de));
  CHECK_HIP(hipFree(dl));
  CHECK_HIP(hipFree(dcid));
  CHECK_HIP(hipFree(dev_ids));
  CHECK_HIP(hipFree(dseed));
  clue_destroy(c);

  FILE *o = fopen(argv[2], "wb");
  if (!o) return 1;
  const int bad = fwrite(cid, 1, n4, o) != n4 || fwrite(seed, 1, (size_t)n, o) != (size_t)n;
  fclose(o);
  free(x); free(y); free(e); free(layer); free(cid); free(cid2); free(seed); free(seed2);
  return bad ? 1 : 0;
}
