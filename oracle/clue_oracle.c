/*
 * CLUE oracle: TEST INFRASTRUCTURE ONLY (see clue_oracle.h for the contract
 * and the readings of the paper it implements).
 *
 * Build: gcc -std=c99 -O2 -ffp-contract=off -fno-fast-math -fPIC -shared
 *        -pthread. x86-64 evaluates float arithmetic in SSE single precision,
 *        so every float operation below is one IEEE binary32 rounding.
 */
#define _POSIX_C_SOURCE 200809L
#include "clue_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static __thread char g_err[256];

const char *oracle_last_error(void) { return g_err; }

static int fail(int code, const char *msg) {
  snprintf(g_err, sizeof g_err, "%s", msg);
  return code;
}

/* Squared distance in float32, two products and one sum, each rounded. */
static float dist2(float xi, float yi, float xj, float yj) {
  float dx = xi - xj;
  float dy = yi - yj;
  float dx2 = dx * dx;
  float dy2 = dy * dy;
  return dx2 + dy2;
}

/*
 * exp(x) for x <= 0 in binary32 arithmetic, used by the Gaussian and
 * exponential kernels of Eq. 3. Range reduction after Cody and Waite
 * (Software Manual for the Elementary Functions, 1980): x = k ln2 + r with
 * k = floor(x / ln2 + 1/2), ln2 split into a part with trailing zero bits
 * (so k * hi is exact) and the remainder; exp(r) by its degree-7 Taylor
 * polynomial in Horner form; the result scaled by 2^k. Every operation is
 * one binary32 rounding, so the value is a fixed function of x. Results
 * below 2^-125 (k < -125) are defined as 0.
 */
static float exp32(float x) {
  const float inv_ln2 = (float)(1.0 / 0.69314718055994530942);
  const float ln2_hi = 0.693145751953125f;
  const float ln2_lo = (float)(0.69314718055994530942 - 0.693145751953125);
  const float t = x * inv_ln2;
  const float kf = floorf(t + 0.5f);
  if (!(kf >= -125.0f)) return 0.0f;
  const float r = (x - kf * ln2_hi) - kf * ln2_lo;
  float p = (float)(1.0 / 5040.0);
  p = p * r + (float)(1.0 / 720.0);
  p = p * r + (float)(1.0 / 120.0);
  p = p * r + (float)(1.0 / 24.0);
  p = p * r + (float)(1.0 / 6.0);
  p = p * r + 0.5f;
  p = p * r + 1.0f;
  p = p * r + 1.0f;
  union { uint32_t u; float f; } two_k;
  two_k.u = (uint32_t)((int32_t)kf + 127) << 23;
  return p * two_k.f;
}

void oracle_exp32(const float *x, float *out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = exp32(x[i]);
}

/* Kernel weight chi(d) of Eq. 3 for a pair at float32 squared distance d2:
 * 1 (flat), exp(-d^2 / (2 s^2)) (Gaussian) or exp(-d / s) (exponential);
 * a = fl(1 / (2 s^2)) or fl(1 / s); d = sqrtf(d2), correctly rounded. */
static float kernel_weight(int kernel, float a, float d2) {
  if (kernel == 1) return exp32(-(d2 * a));
  if (kernel == 2) return exp32(-(sqrtf(d2) * a));
  return 1.0f;
}

static double kernel_weight64(int kernel, double s, double d2) {
  if (kernel == 1) return exp(-d2 / (2.0 * s * s));
  if (kernel == 2) return exp(-sqrt(d2) / s);
  return 1.0;
}

/* One (event, layer) unit with its own fixed grid (Sec. 2.1). */
typedef struct {
  const float *x, *y, *e;  /* event-local base pointers */
  int32_t *ids;            /* hits of this layer, ascending event-local index */
  int32_t count;
  int32_t nbx, nby;
  int32_t *bin_start;      /* nbx*nby + 1 */
  int32_t *bin_items;      /* count, ascending index within each bin */
  float *rho;              /* event-local outputs */
  double *rho64;
  int32_t *nh;
  float *delta2;
} unit_t;

typedef struct {
  const oracle_params *p;
  double bin;
  float dc2, dm2;
  float dm;
  float ka;  /* kernel constant: fl(1 / (2 s^2)) or fl(1 / s) */
} ctx_t;

/* Bin coordinate of a position: floor((v - lo) / bin) clamped to the grid. */
static int32_t bin_coord(double v, double lo, double bin, int32_t nb) {
  double t = floor((v - lo) / bin);
  if (!(t >= 0.0)) return 0;
  if (t > (double)(nb - 1)) return nb - 1;
  return (int32_t)t;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
  return (u > v) - (u < v);
}

/*
 * Omega_d(i) (Eq. 1): every hit in the bins touched by the window
 * [x_i - d, x_i + d] x [y_i - d, y_i + d], padded by one bin on each side so
 * that float rounding of the window edges can never drop a neighbour. The
 * padding only adds candidates that the distance test then rejects. With
 * brute_force set, Omega_d(i) is the whole layer.
 */
static int32_t gather_window(const ctx_t *c, const unit_t *u, int32_t i, float d, int32_t *out) {
  if (c->p->brute_force) {
    memcpy(out, u->ids, (size_t)u->count * sizeof(int32_t));
    return u->count;
  }
  const oracle_params *p = c->p;
  double xi = u->x[i], yi = u->y[i];
  int32_t bx0 = bin_coord(xi - d, p->x_min, c->bin, u->nbx) - 1;
  int32_t bx1 = bin_coord(xi + d, p->x_min, c->bin, u->nbx) + 1;
  int32_t by0 = bin_coord(yi - d, p->y_min, c->bin, u->nby) - 1;
  int32_t by1 = bin_coord(yi + d, p->y_min, c->bin, u->nby) + 1;
  if (bx0 < 0) bx0 = 0;
  if (by0 < 0) by0 = 0;
  if (bx1 > u->nbx - 1) bx1 = u->nbx - 1;
  if (by1 > u->nby - 1) by1 = u->nby - 1;
  int32_t m = 0;
  for (int32_t by = by0; by <= by1; ++by)
    for (int32_t bx = bx0; bx <= bx1; ++bx) {
      int32_t b = by * u->nbx + bx;
      for (int32_t k = u->bin_start[b]; k < u->bin_start[b + 1]; ++k) out[m++] = u->bin_items[k];
    }
  return m;
}

/* Algorithm 1 / Eq. 3: rho_i = sum of fl(chi(d_ij) * w_j) over N_dc(i), added
 * in ascending j (chi = 1 for the flat kernel: the weights themselves). */
static void unit_density(const ctx_t *c, unit_t *u, int32_t *scratch) {
  for (int32_t a = 0; a < u->count; ++a) {
    int32_t i = u->ids[a];
    int32_t m = gather_window(c, u, i, c->p->dc, scratch);
    qsort(scratch, (size_t)m, sizeof(int32_t), cmp_i32);
    float acc = 0.0f;
    double acc64 = 0.0;
    for (int32_t k = 0; k < m; ++k) {
      int32_t j = scratch[k];
      const float d2 = dist2(u->x[i], u->y[i], u->x[j], u->y[j]);
      if (d2 < c->dc2) {
        const int kern = c->p->kernel;
        const float w = kern ? kernel_weight(kern, c->ka, d2) * u->e[j] : u->e[j];
        acc = acc + w;
        acc64 = acc64 + kernel_weight64(kern, (double)c->p->kernel_scale, (double)d2) * (double)u->e[j];
      }
    }
    u->rho[i] = acc;
    if (u->rho64) u->rho64[i] = acc64;
  }
}

static int higher(const ctx_t *c, const float *rho, int32_t j, int32_t i) {
  if (rho[j] > rho[i]) return 1;
  if (c->p->paper_strict) return 0;
  return rho[j] == rho[i] && j > i;
}

/* Algorithm 2 / Eq. 4: nh_i = argmin over N'_dm(i) of d_ij (smallest index on
 * equal distance), delta_i = d_{i,nh_i}, or nh_i = -1 and delta_i = +inf. */
static void unit_nearest_higher(const ctx_t *c, unit_t *u, int32_t *scratch) {
  for (int32_t a = 0; a < u->count; ++a) {
    int32_t i = u->ids[a];
    int32_t m = gather_window(c, u, i, c->dm, scratch);
    int32_t best = -1;
    float bd = INFINITY;
    for (int32_t k = 0; k < m; ++k) {
      int32_t j = scratch[k];
      float d2 = dist2(u->x[i], u->y[i], u->x[j], u->y[j]);
      if (!(d2 < c->dm2)) continue;
      if (!higher(c, u->rho, j, i)) continue;
      if (d2 < bd || (d2 == bd && j < best)) {
        bd = d2;
        best = j;
      }
    }
    u->nh[i] = best;
    u->delta2[i] = bd;
  }
}

typedef struct {
  const ctx_t *c;
  unit_t *units;
  int32_t n_units;
  int32_t tid, nthreads;
  int32_t max_count;
  int stage; /* 0: density, 1: nearest-higher */
  int status;
} worker_t;

static void *worker_main(void *arg) {
  worker_t *w = (worker_t *)arg;
  int32_t *scratch = (int32_t *)malloc(((size_t)w->max_count + 1) * sizeof(int32_t));
  if (!scratch) {
    w->status = ORACLE_ERR_NOMEM;
    return NULL;
  }
  for (int32_t k = w->tid; k < w->n_units; k += w->nthreads) {
    if (w->units[k].count == 0) continue;
    if (w->stage == 0)
      unit_density(w->c, &w->units[k], scratch);
    else
      unit_nearest_higher(w->c, &w->units[k], scratch);
  }
  free(scratch);
  w->status = ORACLE_OK;
  return NULL;
}

static int run_stage(const ctx_t *c, unit_t *units, int32_t n_units, int32_t max_count, int stage,
                     int n_threads) {
  if (n_threads < 1) n_threads = 1;
  if (n_threads > n_units) n_threads = n_units > 0 ? n_units : 1;
  worker_t *ws = (worker_t *)calloc((size_t)n_threads, sizeof(worker_t));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  if (!ws || !th) {
    free(ws);
    free(th);
    return ORACLE_ERR_NOMEM;
  }
  for (int t = 0; t < n_threads; ++t) {
    ws[t] = (worker_t){c, units, n_units, t, n_threads, max_count, stage, ORACLE_OK};
  }
  int rc = ORACLE_OK;
  if (n_threads == 1) {
    worker_main(&ws[0]);
  } else {
    char *created = (char *)calloc((size_t)n_threads, 1);
    if (!created) {
      free(ws);
      free(th);
      return ORACLE_ERR_NOMEM;
    }
    for (int t = 0; t < n_threads; ++t) {
      if (pthread_create(&th[t], NULL, worker_main, &ws[t]) == 0)
        created[t] = 1;
      else
        worker_main(&ws[t]); /* no thread available: run that share here */
    }
    for (int t = 0; t < n_threads; ++t)
      if (created[t]) pthread_join(th[t], NULL);
    free(created);
  }
  for (int t = 0; t < n_threads; ++t)
    if (ws[t].status != ORACLE_OK) rc = ws[t].status;
  free(ws);
  free(th);
  return rc;
}

static int finite_f(float v) { return isfinite(v) != 0; }

int oracle_run(const oracle_params *p, int64_t n, int32_t n_events, const int32_t *event,
               const float *x, const float *y, const int32_t *layer, const float *energy,
               int32_t *cluster_id, uint8_t *is_seed,
               float *rho, double *rho64, int32_t *nh, float *delta2,
               int32_t *fstart, int32_t *flist, int32_t *n_clusters, int n_threads) {
  g_err[0] = 0;
  if (!p) return fail(ORACLE_ERR_ARG, "null params");
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(ORACLE_ERR_ARG, "n out of range");
  if (n_events < 1) return fail(ORACLE_ERR_ARG, "n_events < 1");
  if (!finite_f(p->dc) || !(p->dc > 0.0f) || !finite_f(p->rho_c) || !finite_f(p->delta_c) ||
      !finite_f(p->delta_o) || p->delta_c < 0.0f || p->delta_o < 0.0f)
    return fail(ORACLE_ERR_ARG, "bad clustering parameters");
  if (!finite_f(p->x_min) || !finite_f(p->x_max) || !finite_f(p->y_min) || !finite_f(p->y_max) ||
      !(p->x_max > p->x_min) || !(p->y_max > p->y_min))
    return fail(ORACLE_ERR_ARG, "bad grid extent");
  if (p->n_layers < 1) return fail(ORACLE_ERR_ARG, "n_layers < 1");
  if (p->kernel < 0 || p->kernel > 2) return fail(ORACLE_ERR_ARG, "unknown kernel");
  if (p->kernel != 0 && !(p->kernel_scale > 0.0f && finite_f(p->kernel_scale)))
    return fail(ORACLE_ERR_ARG, "kernel_scale must be positive");
  if (n == 0) {
    if (fstart) fstart[0] = 0;
    if (n_clusters)
      for (int32_t e = 0; e < n_events; ++e) n_clusters[e] = 0;
    return ORACLE_OK;
  }
  if (!x || !y || !layer || !energy || !cluster_id || !is_seed)
    return fail(ORACLE_ERR_ARG, "null input or output pointer");
  if (n_events > 1 && !event) return fail(ORACLE_ERR_ARG, "event ids required for n_events > 1");

  for (int64_t h = 0; h < n; ++h) {
    if (!finite_f(x[h]) || !finite_f(y[h]) || !finite_f(energy[h]))
      return fail(ORACLE_ERR_INPUT, "non-finite x, y or energy");
    if (layer[h] < 0 || layer[h] >= p->n_layers) return fail(ORACLE_ERR_INPUT, "layer out of range");
    if (event) {
      if (event[h] < 0 || event[h] >= n_events) return fail(ORACLE_ERR_INPUT, "event out of range");
      if (h > 0 && event[h] < event[h - 1]) return fail(ORACLE_ERR_INPUT, "event ids decrease");
    }
  }

  ctx_t c;
  c.p = p;
  c.dm = p->delta_o > p->delta_c ? p->delta_o : p->delta_c;
  c.dc2 = p->dc * p->dc;
  c.dm2 = c.dm * c.dm;
  c.ka = 0.0f;
  if (p->kernel == 1) c.ka = (float)(1.0 / (2.0 * (double)p->kernel_scale * (double)p->kernel_scale));
  if (p->kernel == 2) c.ka = (float)(1.0 / (double)p->kernel_scale);
  {
    double b = p->bin_size > 0.0f ? (double)p->bin_size : (double)(p->dc > c.dm ? p->dc : c.dm);
    double dmax = (double)(p->dc > c.dm ? p->dc : c.dm);
    if (b < 1e-3 * dmax) return fail(ORACLE_ERR_ARG, "oracle bin too small for the search radius");
    c.bin = b;
  }
  const float dc2_seed = p->delta_c * p->delta_c;
  const float do2 = p->delta_o * p->delta_o;
  int32_t nbx = (int32_t)ceil(((double)p->x_max - p->x_min) / c.bin);
  int32_t nby = (int32_t)ceil(((double)p->y_max - p->y_min) / c.bin);
  if (nbx < 1) nbx = 1;
  if (nby < 1) nby = 1;
  if ((int64_t)nbx * nby > (1 << 26)) return fail(ORACLE_ERR_ARG, "oracle grid too fine");

  /* Event ranges in caller order. */
  int64_t *ev_start = (int64_t *)calloc((size_t)n_events + 1, sizeof(int64_t));
  if (!ev_start) return fail(ORACLE_ERR_NOMEM, "alloc");
  for (int64_t h = 0; h < n; ++h) ev_start[(event ? event[h] : 0) + 1]++;
  for (int32_t e = 0; e < n_events; ++e) ev_start[e + 1] += ev_start[e];

  const int32_t L = p->n_layers;
  const int64_t n_units64 = (int64_t)n_events * L;
  if (n_units64 > (1 << 28)) {
    free(ev_start);
    return fail(ORACLE_ERR_ARG, "too many (event, layer) units");
  }
  const int32_t n_units = (int32_t)n_units64;

  unit_t *units = (unit_t *)calloc((size_t)n_units, sizeof(unit_t));
  int32_t *ids = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *bin_items = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *nh_loc = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  float *rho_loc = (float *)malloc((size_t)n * sizeof(float));
  float *d2_loc = (float *)malloc((size_t)n * sizeof(float));
  double *rho64_loc = rho64 ? rho64 : NULL;
  if (!units || !ids || !bin_items || !nh_loc || !rho_loc || !d2_loc) {
    free(units); free(ids); free(bin_items); free(nh_loc); free(rho_loc); free(d2_loc); free(ev_start);
    return fail(ORACLE_ERR_NOMEM, "alloc");
  }

  /* Partition every event's hits by layer, ascending index within a layer. */
  int32_t max_count = 0;
  int rc = ORACLE_OK;
  for (int32_t e = 0; e < n_events && rc == ORACLE_OK; ++e) {
    int64_t s = ev_start[e], ne = ev_start[e + 1] - s;
    int32_t *cnt = (int32_t *)calloc((size_t)L + 1, sizeof(int32_t));
    if (!cnt) { rc = ORACLE_ERR_NOMEM; break; }
    for (int64_t a = 0; a < ne; ++a) cnt[layer[s + a] + 1]++;
    for (int32_t l = 0; l < L; ++l) cnt[l + 1] += cnt[l];
    for (int32_t l = 0; l < L; ++l) {
      unit_t *u = &units[(int64_t)e * L + l];
      u->x = x + s;
      u->y = y + s;
      u->e = energy + s;
      u->ids = ids + s + cnt[l];
      u->count = 0;
      u->rho = rho_loc + s;
      u->rho64 = rho64_loc ? rho64_loc + s : NULL;
      u->nh = nh_loc + s;
      u->delta2 = d2_loc + s;
    }
    for (int64_t a = 0; a < ne; ++a) {
      unit_t *u = &units[(int64_t)e * L + layer[s + a]];
      u->ids[u->count++] = (int32_t)a;
    }
    free(cnt);
  }
  /* One fixed grid per unit: register each hit index in its bin. */
  for (int32_t k = 0; k < n_units && rc == ORACLE_OK; ++k) {
    unit_t *u = &units[k];
    if (u->count > max_count) max_count = u->count;
    if (u->count == 0 || p->brute_force) continue;
    u->nbx = nbx;
    u->nby = nby;
    u->bin_start = (int32_t *)calloc((size_t)nbx * nby + 1, sizeof(int32_t));
    if (!u->bin_start) { rc = ORACLE_ERR_NOMEM; break; }
    u->bin_items = bin_items + (u->ids - ids);
    int32_t *bin_of = (int32_t *)malloc((size_t)u->count * sizeof(int32_t));
    if (!bin_of) { rc = ORACLE_ERR_NOMEM; break; }
    for (int32_t a = 0; a < u->count; ++a) {
      int32_t i = u->ids[a];
      int32_t bx = bin_coord(u->x[i], p->x_min, c.bin, nbx);
      int32_t by = bin_coord(u->y[i], p->y_min, c.bin, nby);
      bin_of[a] = by * nbx + bx;
      u->bin_start[bin_of[a] + 1]++;
    }
    for (int32_t b = 0; b < nbx * nby; ++b) u->bin_start[b + 1] += u->bin_start[b];
    int32_t *fill = (int32_t *)malloc((size_t)nbx * nby * sizeof(int32_t));
    if (!fill) { free(bin_of); rc = ORACLE_ERR_NOMEM; break; }
    memcpy(fill, u->bin_start, (size_t)nbx * nby * sizeof(int32_t));
    for (int32_t a = 0; a < u->count; ++a) u->bin_items[fill[bin_of[a]]++] = u->ids[a];
    free(fill);
    free(bin_of);
  }

  if (rc == ORACLE_OK) rc = run_stage(&c, units, n_units, max_count, 0, n_threads);
  if (rc == ORACLE_OK) rc = run_stage(&c, units, n_units, max_count, 1, n_threads);

  /* Algorithm 3, per event in ascending index: promote seeds (numbered in
   * loop order), demote outliers, register every other hit that has a
   * nearest-higher as a follower of it; then expand from the seeds with a
   * stack. */
  int32_t *fcount = NULL, *fpos = NULL, *flocal = NULL, *stack = NULL;
  if (rc == ORACLE_OK) {
    fcount = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    fpos = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    flocal = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    stack = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!fcount || !fpos || !flocal || !stack) rc = ORACLE_ERR_NOMEM;
  }
  if (rc == ORACLE_OK) {
    for (int32_t e = 0; e < n_events; ++e) {
      int64_t s = ev_start[e];
      int32_t ne = (int32_t)(ev_start[e + 1] - s);
      int32_t k = 0, top = 0;
      int32_t *fc = fcount + s; /* fc[i+1] counts followers of i */
      for (int32_t i = 0; i < ne; ++i) {
        int seed = rho_loc[s + i] > p->rho_c && d2_loc[s + i] > dc2_seed;
        int outlier = rho_loc[s + i] < p->rho_c && d2_loc[s + i] > do2;
        is_seed[s + i] = (uint8_t)seed;
        cluster_id[s + i] = -1;
        if (seed) {
          cluster_id[s + i] = k++;
        } else if (!outlier && nh_loc[s + i] >= 0) {
          fc[nh_loc[s + i] + 1]++;
        }
      }
      /* follower lists as CSR, filled in ascending follower index */
      int32_t *fs = fpos + s;
      fs[0] = 0;
      for (int32_t i = 0; i + 1 < ne; ++i) fs[i + 1] = fs[i] + fc[i + 1];
      int32_t *fill = (int32_t *)malloc(((size_t)ne + 1) * sizeof(int32_t));
      if (!fill) { rc = ORACLE_ERR_NOMEM; break; }
      if (ne > 0) memcpy(fill, fs, (size_t)ne * sizeof(int32_t));
      for (int32_t i = 0; i < ne; ++i) {
        int seed = is_seed[s + i];
        int outlier = rho_loc[s + i] < p->rho_c && d2_loc[s + i] > do2;
        if (!seed && !outlier && nh_loc[s + i] >= 0) flocal[s + fill[nh_loc[s + i]]++] = i;
      }
      free(fill);
      for (int32_t i = 0; i < ne; ++i)
        if (is_seed[s + i]) stack[top++] = i;
      while (top > 0) {
        int32_t i = stack[--top];
        int32_t b = fs[i], end = fs[i] + fc[i + 1];
        for (int32_t q = b; q < end; ++q) {
          int32_t j = flocal[s + q];
          cluster_id[s + j] = cluster_id[s + i];
          stack[top++] = j;
        }
      }
      if (n_clusters) n_clusters[e] = k;
      if (fstart) {
        for (int32_t i = 0; i < ne; ++i) fstart[s + i] = (int32_t)s + fs[i];
      }
    }
    if (rc == ORACLE_OK) {
      if (fstart) fstart[n] = 0;
      if (fstart || flist) {
        /* total followers, and flist in global CSR order */
        int64_t tot = 0;
        for (int32_t e = 0; e < n_events; ++e) {
          int64_t s = ev_start[e];
          int32_t ne = (int32_t)(ev_start[e + 1] - s);
          int32_t cnt = 0;
          for (int32_t i = 0; i < ne; ++i) cnt += fcount[s + i + 1];
          if (fstart)
            for (int32_t i = 0; i < ne; ++i) fstart[s + i] = (int32_t)(tot + fpos[s + i]);
          if (flist)
            for (int32_t q = 0; q < cnt; ++q) flist[tot + q] = flocal[s + q];
          tot += cnt;
        }
        if (fstart) fstart[n] = (int32_t)tot;
      }
    }
  }

  if (rc == ORACLE_OK) {
    if (rho) memcpy(rho, rho_loc, (size_t)n * sizeof(float));
    if (nh) memcpy(nh, nh_loc, (size_t)n * sizeof(int32_t));
    if (delta2) memcpy(delta2, d2_loc, (size_t)n * sizeof(float));
  }
  for (int32_t k = 0; k < n_units; ++k) free(units[k].bin_start);
  free(units); free(ids); free(bin_items); free(nh_loc); free(rho_loc); free(d2_loc);
  free(ev_start); free(fcount); free(fpos); free(flocal); free(stack);
  if (rc != ORACLE_OK && !g_err[0]) fail(rc, "oracle failure");
  return rc;
}
