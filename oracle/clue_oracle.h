/*
 * CLUE oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of CLUE's per-layer
 * clustering (Rovere et al., arXiv:2001.09761). Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the GPU library
 * shares no source, header or helper with it.
 *
 * It follows the paper step by step:
 *   fixed-grid index      Sec. 2.1, Eq. 1 (Omega_d) and Eq. 2 (N_d)
 *   local density rho     Eq. 3, Algorithm 1 (kernel chi flat, Gaussian or
 *                         exponential; see oracle_exp32)
 *   nearest-higher/delta  Eq. 4, Algorithm 2, d_m = max(delta_o, delta_c)
 *   seeds/outliers        Sec. 2.2 thresholds, first loop of Algorithm 3
 *   followers F_i         Eq. 5, first loop of Algorithm 3
 *   cluster expansion     second loop of Algorithm 3 (stack DFS from seeds)
 *
 * Readings where the paper is silent or ambiguous (all documented in the
 * design notes):
 *   - neighbours live on the same (event, layer) only;
 *   - distances are compared squared in float32: d2 = fl(fl(dx*dx)+fl(dy*dy)),
 *     dx = fl(xi-xj), no fused multiply-add, thresholds squared once in float32,
 *     strict '<' for dc and dm, strict '>' for delta_c and delta_o;
 *   - rho sums float32 weights sequentially in ascending hit index, the hit
 *     itself included; rho64 sums the same set in double;
 *   - "higher density" is the strict total order (rho, index): j is higher
 *     than i when rho_j > rho_i, or rho_j == rho_i and j > i
 *     (paper_strict = 1 keeps Eq. 4 literally: rho_j > rho_i only);
 *   - the argmin of Eq. 4 keeps the smallest index among equal d2;
 *   - a seed is never a follower; a hit that is neither seed nor outlier and
 *     has nh = -1 (possible only when rho == rho_c) is an orphan root;
 *   - cluster ids are numbered per event by ascending seed index (the loop
 *     order of Algorithm 3); noise (outliers, orphans and their descendants)
 *     gets cluster id -1;
 *   - hit indices reported in nh and in the follower lists are event-local.
 */
#ifndef CLUE_ORACLE_H
#define CLUE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORACLE_OK = 0,
  ORACLE_ERR_ARG = -1,
  ORACLE_ERR_NOMEM = -3,
  ORACLE_ERR_INPUT = -5
};

typedef struct {
  float dc, rho_c, delta_c, delta_o;     /* the four CLUE parameters (Sec. 2.2) */
  float x_min, y_min, x_max, y_max;      /* extent of the fixed grid; outside -> edge bin */
  int32_t n_layers;                      /* layer ids in [0, n_layers) */
  float bin_size;                        /* oracle grid bin (cm); <= 0 -> max(dc, d_m) */
  int32_t paper_strict;                  /* 1: higher <=> rho_j > rho_i only */
  int32_t brute_force;                   /* 1: Omega = every hit of the same layer */
  int32_t kernel;                        /* chi of Eq. 3: 0 flat, 1 Gaussian, 2 exponential */
  float kernel_scale;                    /* s (cm): exp(-d^2 / (2 s^2)) or exp(-d / s) */
} oracle_params;

/*
 * Cluster n hits grouped into n_events events (event ids non-decreasing in
 * [0, n_events); event == NULL means a single event). All pointers are HOST
 * pointers. Required outputs: cluster_id[n], is_seed[n]. Optional (NULL to
 * skip): rho[n], rho64[n], nh[n] (event-local), delta2[n] (+inf when nh = -1),
 * fstart[n+1] and flist[n] (follower lists per hit in caller order, entries
 * event-local and ascending), n_clusters[n_events].
 * n_threads >= 1 parallelises density and nearest-higher over (event, layer)
 * units; results do not depend on it.
 * Returns ORACLE_OK or a negative error (bad argument, allocation failure,
 * non-finite or out-of-range input).
 */
int oracle_run(const oracle_params *p, int64_t n, int32_t n_events, const int32_t *event,
               const float *x, const float *y, const int32_t *layer, const float *energy,
               int32_t *cluster_id, uint8_t *is_seed,
               float *rho, double *rho64, int32_t *nh, float *delta2,
               int32_t *fstart, int32_t *flist, int32_t *n_clusters, int n_threads);

const char *oracle_last_error(void);

/* The binary32 exponential the Gaussian and exponential kernels use, for
 * x <= 0 (definition in clue_oracle.c); out[i] = exp32(x[i]). */
void oracle_exp32(const float *x, float *out, int64_t n);

#ifdef __cplusplus
}
#endif
#endif
