// libclue host runtime: contexts, the scratch arena, geometry planning, HIP
// graph capture of the batched form, and the C ABI declared in clue.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "clue.h"
#include "clue_internal.h"

using namespace clue;

struct clue_ctx {
  int device = 0;
  clue_params params{};
  Geom g{};
  Arena a{};
  void* arena_base = nullptr;
  size_t arena_bytes = 0;
  uint64_t budget = 0;
  int n_cu = 1;
  float tile = 0.0f;
  int tpq = 1, bx = 8, by = 8, lds_cap = kDefaultLdsCap;
  int plain_cap = 0;  // LDS cap of the plain form (clue_run); 0: lds_cap
  Geom g_plain{};     // g with the plain form's LDS cap
  float r1 = -1.0f;  // nearest-higher first radius; negative: default d_m / 4
  int quads = 1;      // density strategy (1 quads by search, 2 per-query merge, 3 quads by merge)
  int expansion = 1;  // labels: 1 pointer jumping, 2 depth-first walk per seed
  LaunchCfg cfg{};
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool timing = false;
  bool timed_valid = false;
  hipEvent_t ev[S_COUNT + 1] = {};
  int64_t last_n = -1;
  int32_t last_events = 0;
  // host-resident form: two device staging chunks and their streams/events
  void* stage_base = nullptr;
  int64_t stage_hits = 0;
  hipStream_t h2d = nullptr, comp = nullptr, d2h = nullptr;
  hipEvent_t in_ready[2] = {}, done[2] = {}, out_done[2] = {};
  bool last_followers_valid = false;
  std::string err;
};

static thread_local std::string g_create_err;

static int set_err(clue_ctx* c, int code, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_create_err = msg;
  return code;
}

static int hip_fail(clue_ctx* c, hipError_t e, const char* what) {
  return set_err(c, CLUE_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                                    \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return hip_fail((c), _e, #expr);  \
  } while (0)

static inline bool finite(float v) { return std::isfinite(v); }

// ---------------------------------------------------------------------------
// Geometry: tile size, halo and window bounds.
// ---------------------------------------------------------------------------
static int plan_geom(const clue_params& p, float tile, int tpq, int bx, int by, int lds_cap, float r1, int quads,
                     int expansion, Geom& g, std::string& msg) {
  if (!finite(p.dc) || !(p.dc > 0.0f) || !finite(p.rho_c) || !finite(p.delta_c) || !finite(p.delta_o) ||
      p.delta_c < 0.0f || p.delta_o < 0.0f) {
    msg = "invalid clustering parameters (need finite dc > 0, rho_c, delta_c >= 0, delta_o >= 0)";
    return CLUE_ERR_ARG;
  }
  if (!finite(p.x_min) || !finite(p.x_max) || !finite(p.y_min) || !finite(p.y_max) || !(p.x_max > p.x_min) ||
      !(p.y_max > p.y_min)) {
    msg = "invalid grid extent";
    return CLUE_ERR_ARG;
  }
  if (p.n_layers < 1) {
    msg = "n_layers must be >= 1";
    return CLUE_ERR_ARG;
  }
  if (p.kernel < CLUE_KERNEL_FLAT || p.kernel > CLUE_KERNEL_EXPONENTIAL ||
      (p.kernel != CLUE_KERNEL_FLAT && !(finite(p.kernel_scale) && p.kernel_scale > 0.0f))) {
    msg = "kernel must be flat, Gaussian or exponential, with kernel_scale > 0 for the latter two";
    return CLUE_ERR_ARG;
  }
  if (tpq != 1 && tpq != 2 && tpq != 4 && tpq != 8) {
    msg = "threads_per_query must be 1, 2, 4 or 8";
    return CLUE_ERR_ARG;
  }
  if (bx < 1 || by < 1 || bx > 16 || by > 16) {
    msg = "tile block must be within 1..16 tiles per side";
    return CLUE_ERR_ARG;
  }
  if (expansion != 1 && expansion != 2) {
    msg = "expansion must be 1 (pointer jumping) or 2 (depth-first per seed)";
    return CLUE_ERR_ARG;
  }
  if (lds_cap < 64 || lds_cap > kMaxLdsCap) {
    msg = "lds_cap must be within 64..2048 hits";
    return CLUE_ERR_ARG;
  }
  const float dm = std::max(p.delta_o, p.delta_c);
  const double dmax = std::max((double)dm, (double)p.dc);
  double t = tile > 0.0f ? (double)tile : std::max((double)dm, 2.0 * p.dc) * (1.0 + 1.0 / 128.0);
  if (!(t > 0.0) || !std::isfinite(t)) {
    msg = "invalid tile size";
    return CLUE_ERR_ARG;
  }
  const float inv_t = (float)(1.0 / t);
  const double t_eff = 1.0 / (double)inv_t;
  const double wx = (double)p.x_max - p.x_min, wy = (double)p.y_max - p.y_min;
  const double nxd = std::ceil(wx / t_eff), nyd = std::ceil(wy / t_eff);
  if (nxd * nyd > (double)(1 << 26)) {
    msg = "grid too fine: extent / tile_size gives more than 2^26 tiles per layer";
    return CLUE_ERR_ARG;
  }
  g.x0 = p.x_min;
  g.y0 = p.y_min;
  g.inv_t = inv_t;
  g.nx = std::max(1, (int)nxd);
  g.ny = std::max(1, (int)nyd);
  g.tpl = g.nx * g.ny;
  g.L = p.n_layers;
  g.dc2 = p.dc * p.dc;
  g.kernel = p.kernel;
  g.ka = p.kernel == CLUE_KERNEL_GAUSSIAN
             ? (float)(1.0 / (2.0 * (double)p.kernel_scale * (double)p.kernel_scale))
             : (p.kernel == CLUE_KERNEL_EXPONENTIAL ? (float)(1.0 / (double)p.kernel_scale) : 0.0f);
  g.dm2 = dm * dm;
  g.dcs2 = p.delta_c * p.delta_c;
  g.do2 = p.delta_o * p.delta_o;
  g.rho_c = p.rho_c;
  g.win_dc = (float)((double)p.dc * (1.0 + 1.0 / 1024.0));
  g.win_dm = (float)((double)dm * (1.0 + 1.0 / 1024.0));
  g.flags = p.flags;
  g.density_quads = quads == 2 ? 0 : (quads == 3 ? 2 : 1);
  g.expand = expansion == 2 ? 1 : 0;
  // First nearest-higher pass: radius r1 (default d_m / 4); off when r1 <= 0
  // or r1 >= d_m.
  const float r1v = r1 < 0.0f ? 0.25f * dm : r1;
  g.nh_phase1 = (r1v > 0.0f && r1v < dm && std::isfinite(r1v)) ? 1 : 0;
  g.r1sq = g.nh_phase1 ? r1v * r1v : 0.0f;
  g.win_r1 = g.nh_phase1 ? (float)((double)r1v * (1.0 + 1.0 / 1024.0)) : 0.0f;
  // Bound on how many tiles a query window reaches from its own tile:
  // tile_coord is floor((v - x0) * inv_t) with at most a few float32
  // roundings; the half width of a window is win + 2^-20 |v|.
  const double amax = std::max({std::fabs((double)p.x_min), std::fabs((double)p.x_max),
                                std::fabs((double)p.y_min), std::fabs((double)p.y_max)}) +
                      2.0 * dmax + 1.0;
  const double eps = (amax + std::max(std::fabs((double)p.x_min), std::fabs((double)p.y_min))) * inv_t *
                         std::ldexp(1.0, -20) +
                     std::ldexp(1.0, -16);
  auto reach = [&](double w) { return (w * (1.0 + std::ldexp(1.0, -20)) + amax * std::ldexp(1.0, -20)) * inv_t; };
  const double rc = reach(g.win_dc), rm = reach(g.win_dm);
  const int halo = (int)std::floor(std::max(rc, rm) + eps) + 1;
  const int maxl = (int)std::floor(2.0 * rc + eps) + 2;
  if (maxl > 3) {
    msg = "tile_size too small for dc: the density window must span at most 3 tiles per side "
          "(tile_size > dc * 1.002)";
    return CLUE_ERR_ARG;
  }
  const int rw = std::min(bx + 2 * halo, g.nx), rh = std::min(by + 2 * halo, g.ny);
  if (rh > kMaxRegionRows || rh * (rw + 1) > kMaxRegionTiles) {
    msg = "tile block plus halo exceeds the staged-region limit; use a larger tile_size or smaller block";
    return CLUE_ERR_ARG;
  }
  g.bx = bx;
  g.by = by;
  g.nbx = (g.nx + bx - 1) / bx;
  g.nby = (g.ny + by - 1) / by;
  g.bpu = g.nbx * g.nby;
  g.halo = halo;
  g.maxl = maxl;
  g.tpq = tpq;
  g.lds_cap = lds_cap;
  g.ts_ints = rh * (rw + 1) + 1;
  g.q_ints = (bx + 1) * (by + 1) + 1;
  return CLUE_OK;
}

// ---------------------------------------------------------------------------
// Arena layout.
// ---------------------------------------------------------------------------
struct ArenaPlan {
  size_t off[32];
  size_t total;
  int64_t tiles, chunks;
};

enum {
  A_KEY, A_RANK, A_TS, A_XS, A_YS, A_ES, A_HS, A_RHO, A_PARENT, A_FLAGS, A_SEEDBITS, A_SEEDW, A_EVSTART, A_FSTART,
  A_FRANK, A_FLIST, A_RHO_OUT, A_NH_OUT, A_D2_OUT, A_STATUS, A_COUNTERS, A_ERR, A_DESC, A_NUM
};

static bool plan_arena(const Geom& g, int64_t N, int32_t E, ArenaPlan& P) {
  const int64_t tiles = (int64_t)E * g.L * g.tpl + 1;
  if (tiles >= ((int64_t)1 << 31) || N >= ((int64_t)1 << 31) - 1) return false;
  const int64_t chunks = std::max<int64_t>((tiles + kScanChunk - 1) / kScanChunk, (N + 1 + kScanChunk - 1) / kScanChunk);
  const bool fol = builds_lists(g);
  const bool keep = g.flags & CLUE_KEEP_INTERMEDIATES;
  size_t sz[A_NUM];
  const size_t n = (size_t)std::max<int64_t>(N, 1);
  sz[A_KEY] = 4 * n;
  sz[A_RANK] = 4 * n;
  sz[A_TS] = 4 * (size_t)tiles + 64;
  sz[A_XS] = sz[A_YS] = sz[A_ES] = sz[A_HS] = 4 * n;
  sz[A_RHO] = 4 * n;
  sz[A_PARENT] = 4 * n;
  sz[A_FLAGS] = n;
  sz[A_SEEDBITS] = sz[A_SEEDW] = 4 * (n / 32 + 2) + 64;
  sz[A_EVSTART] = 4 * ((size_t)E + 1);
  sz[A_FSTART] = fol ? 4 * (n + 1) + 64 : 0;
  sz[A_FRANK] = fol ? 4 * n : 0;
  sz[A_FLIST] = fol ? 4 * n : 0;
  sz[A_RHO_OUT] = sz[A_NH_OUT] = sz[A_D2_OUT] = keep ? 4 * n : 0;
  sz[A_STATUS] = 8 * 2 * (size_t)chunks;
  sz[A_COUNTERS] = 4 * C_COUNT;
  sz[A_ERR] = 4;
  sz[A_DESC] = sizeof(RunDesc);
  size_t o = 0;
  for (int i = 0; i < A_NUM; ++i) {
    P.off[i] = o;
    o += (sz[i] + 255) & ~(size_t)255;
  }
  P.total = o;
  P.tiles = tiles;
  P.chunks = chunks;
  return true;
}

// Sub-buffers of an arena that starts at `b`, laid out by `P`.
static Arena arena_at(char* b, const Geom& g, const ArenaPlan& P, int64_t N, int32_t E) {
  Arena a{};
  const bool fol = builds_lists(g);
  const bool keep = g.flags & CLUE_KEEP_INTERMEDIATES;
  a.key = (int32_t*)(b + P.off[A_KEY]);
  a.rank = (int32_t*)(b + P.off[A_RANK]);
  a.tile_start = (int32_t*)(b + P.off[A_TS]);
  a.xs = (float*)(b + P.off[A_XS]);
  a.ys = (float*)(b + P.off[A_YS]);
  a.es = (float*)(b + P.off[A_ES]);
  a.hs = (int32_t*)(b + P.off[A_HS]);
  a.rho = (float*)(b + P.off[A_RHO]);
  a.parent = (int32_t*)(b + P.off[A_PARENT]);
  a.flags = (uint8_t*)(b + P.off[A_FLAGS]);
  a.seedbits = (uint32_t*)(b + P.off[A_SEEDBITS]);
  a.seed_wrank = (int32_t*)(b + P.off[A_SEEDW]);
  a.ev_start = (int32_t*)(b + P.off[A_EVSTART]);
  a.fstart = fol ? (int32_t*)(b + P.off[A_FSTART]) : nullptr;
  a.frank = fol ? (int32_t*)(b + P.off[A_FRANK]) : nullptr;
  a.flist = fol ? (int32_t*)(b + P.off[A_FLIST]) : nullptr;
  a.rho_out = keep ? (float*)(b + P.off[A_RHO_OUT]) : nullptr;
  a.nh_out = keep ? (int32_t*)(b + P.off[A_NH_OUT]) : nullptr;
  a.d2_out = keep ? (float*)(b + P.off[A_D2_OUT]) : nullptr;
  a.scan_status = (unsigned long long*)(b + P.off[A_STATUS]);
  a.counters = (int32_t*)(b + P.off[A_COUNTERS]);
  a.err = (uint32_t*)(b + P.off[A_ERR]);
  a.desc = (RunDesc*)(b + P.off[A_DESC]);
  a.cap_hits = N;
  a.cap_events = E;
  a.cap_tiles = P.tiles;
  a.cap_chunks = P.chunks;
  return a;
}

static void bind_arena(clue_ctx* c, const ArenaPlan& P, int64_t N, int32_t E) {
  c->a = arena_at((char*)c->arena_base, c->g, P, N, E);
}

static void drop_graph(clue_ctx* c) {
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->exec = nullptr;
  c->graph = nullptr;
}

static void compute_cfg(clue_ctx* c) {
  const int lds = lds_bytes_for(c->g);
  // a multiple of kQueues: streaming kernels give each XCD one run of chunks
  c->cfg.persist_blocks_stream = (c->n_cu * std::min(occupancy_blocks_per_cu(0, 0), 8) + kQueues - 1) / kQueues * kQueues;
  c->cfg.persist_blocks_scatter = (c->n_cu * kScatterBlocksPerCU + kQueues - 1) / kQueues * kQueues;
  c->cfg.persist_blocks_rho = c->n_cu * occupancy_blocks_per_cu(1, lds);
  c->cfg.persist_blocks_nh = c->n_cu * occupancy_blocks_per_cu(3, lds_bytes_nh(c->g));
  if (std::getenv("CLUE_VERBOSE"))
    std::fprintf(stderr, "clue: persistent grids stream=%d rho=%d nh=%d scan=%d (cu=%d, lds rho=%d nh=%d)\n",
                 c->cfg.persist_blocks_stream, c->cfg.persist_blocks_rho, c->cfg.persist_blocks_nh,
                 c->cfg.persist_blocks_scan, c->n_cu, lds, lds_bytes_nh(c->g));
  c->cfg.persist_blocks_scan = c->n_cu * std::min(occupancy_blocks_per_cu(2, 0), 4);
}

// (Re)allocates the arena for (N, E) under the current geometry.
static int alloc_arena(clue_ctx* c, int64_t N, int32_t E) {
  ArenaPlan P;
  if (!plan_arena(c->g, N, E, P))
    return set_err(c, CLUE_ERR_CAPACITY, "capacity exceeds 32-bit index limits (hits or tiles)");
  if (c->budget && P.total > c->budget)
    return set_err(c, CLUE_ERR_BUDGET, "arena of " + std::to_string(P.total) + " bytes exceeds the HBM budget");
  HIP_TRY(c, hipSetDevice(c->device));
  if (c->arena_base) {
    HIP_TRY(c, hipDeviceSynchronize());
    drop_graph(c);
    void* old = c->arena_base;
    c->arena_base = nullptr;
    // until the new arena is bound the context holds nothing: a run that
    // follows a failed allocation is refused for capacity
    c->a = Arena{};
    c->arena_bytes = 0;
    c->last_n = -1;
    HIP_TRY(c, hipFree(old));
  }
  hipError_t e = hipMalloc(&c->arena_base, P.total);
  if (e != hipSuccess) {
    c->arena_base = nullptr;
    return set_err(c, CLUE_ERR_NOMEM, "hipMalloc of " + std::to_string(P.total) + " bytes failed");
  }
  c->arena_bytes = P.total;
  HIP_TRY(c, hipMemset(c->arena_base, 0, P.total));
  bind_arena(c, P, N, E);
  c->last_n = -1;
  return CLUE_OK;
}

static int ensure_graph(clue_ctx* c) {
  if (c->exec) return CLUE_OK;
  if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  RunDesc d{};
  d.n = (int32_t)c->a.cap_hits;
  d.n_events = c->a.cap_events;
  LaunchCfg cfg = c->cfg;
  cfg.graph_mode = true;
  HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = launch_pipeline(c->g, c->a, d, cfg, c->cap_stream, nullptr);
  hipGraph_t graph = nullptr;
  hipError_t ce = hipStreamEndCapture(c->cap_stream, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);  // the launch error is the one reported
    return hip_fail(c, le, "launch during capture");
  }
  if (ce != hipSuccess) return hip_fail(c, ce, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(graph);  // the instantiation error is the one reported
    return hip_fail(c, ie, "hipGraphInstantiate");
  }
  c->graph = graph;
  c->exec = exec;
  return CLUE_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int clue_footprint_bytes(const clue_params* p, int64_t max_hits, int32_t max_events, uint64_t* bytes_out) {
  if (!p || !bytes_out || max_hits < 0 || max_events < 1) return CLUE_ERR_ARG;
  Geom g{};
  std::string msg;
  const int tpq = p->threads_per_query > 0 ? p->threads_per_query : 1;
  int rc = plan_geom(*p, p->tile_size, tpq, 8, 8, kDefaultLdsCap, -1.0f, 1, 1, g, msg);
  if (rc != CLUE_OK) return rc;
  ArenaPlan P;
  if (!plan_arena(g, max_hits, max_events, P)) return CLUE_ERR_CAPACITY;
  *bytes_out = P.total;
  return CLUE_OK;
}

int clue_create(clue_ctx** out, const clue_params* p, int hip_device, int64_t max_hits, int32_t max_events,
                uint64_t hbm_budget_bytes) {
  if (!out) return set_err(nullptr, CLUE_ERR_ARG, "null output pointer");
  *out = nullptr;
  if (!p) return set_err(nullptr, CLUE_ERR_ARG, "null params");
  if (max_hits < 0 || max_hits >= ((int64_t)1 << 31) - 1 || max_events < 1)
    return set_err(nullptr, CLUE_ERR_ARG, "capacity out of range (0 <= max_hits < 2^31-1, max_events >= 1)");
  clue_ctx* c = new (std::nothrow) clue_ctx();
  if (!c) return set_err(nullptr, CLUE_ERR_NOMEM, "host allocation failed");
  c->device = hip_device;
  c->params = *p;
  c->budget = hbm_budget_bytes;
  c->tpq = p->threads_per_query > 0 ? p->threads_per_query : 1;
  c->tile = p->tile_size;
  std::string msg;
  int rc = plan_geom(c->params, c->tile, c->tpq, c->bx, c->by, c->lds_cap, c->r1, c->quads, c->expansion, c->g,
                     msg);
  if (rc != CLUE_OK) {
    set_err(nullptr, rc, msg);
    delete c;
    return rc;
  }
  hipError_t e = hipSetDevice(hip_device);
  if (e == hipSuccess) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, hip_device);
    if (e == hipSuccess) c->n_cu = prop.multiProcessorCount;
  }
  if (e != hipSuccess) {
    set_err(nullptr, CLUE_ERR_HIP, std::string("HIP device unavailable: ") + hipGetErrorString(e));
    delete c;
    return CLUE_ERR_HIP;
  }
  for (int i = 0; i <= S_COUNT; ++i) {
    e = hipEventCreate(&c->ev[i]);
    if (e != hipSuccess) {
      set_err(nullptr, CLUE_ERR_HIP, "hipEventCreate failed");
      clue_destroy(c);
      return CLUE_ERR_HIP;
    }
  }
  compute_cfg(c);
  rc = alloc_arena(c, max_hits, max_events);
  if (rc != CLUE_OK) {
    g_create_err = c->err;
    clue_destroy(c);
    return rc;
  }
  *out = c;
  return CLUE_OK;
}

int clue_reserve(clue_ctx* c, int64_t max_hits, int32_t max_events) {
  if (!c) return CLUE_ERR_ARG;
  if (max_hits < 0 || max_hits >= ((int64_t)1 << 31) - 1 || max_events < 1)
    return set_err(c, CLUE_ERR_ARG, "capacity out of range");
  if (max_hits <= c->a.cap_hits && max_events <= c->a.cap_events) return CLUE_OK;
  return alloc_arena(c, std::max<int64_t>(max_hits, c->a.cap_hits), std::max(max_events, c->a.cap_events));
}

static int check_run_args(clue_ctx* c, int64_t n, int32_t n_events, const void* x, const void* y, const void* layer,
                          const void* energy, const void* cid, const void* seed) {
  if (!c) return CLUE_ERR_ARG;
  if (n < 0 || n >= ((int64_t)1 << 31) - 1) return set_err(c, CLUE_ERR_ARG, "n out of range");
  if (n_events < 1) return set_err(c, CLUE_ERR_ARG, "n_events must be >= 1");
  if (n > 0 && (!x || !y || !layer || !energy || !cid || !seed))
    return set_err(c, CLUE_ERR_ARG, "null input or output pointer");
  if (n > c->a.cap_hits || n_events > c->a.cap_events)
    return set_err(c, CLUE_ERR_CAPACITY,
                   "run of " + std::to_string(n) + " hits / " + std::to_string(n_events) +
                       " events exceeds the reserved capacity (" + std::to_string(c->a.cap_hits) + " / " +
                       std::to_string(c->a.cap_events) + "); call clue_reserve");
  return CLUE_OK;
}

static int validate_inputs(clue_ctx* c, const RunDesc& d, hipStream_t s) {
  HIP_TRY(c, launch_validate(c->g, c->a, d, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  uint32_t err = 0;
  HIP_TRY(c, hipMemcpy(&err, c->a.err, sizeof err, hipMemcpyDeviceToHost));
  if (err & E_INPUT) {
    uint32_t z = 0;
    HIP_TRY(c, hipMemcpy(c->a.err, &z, sizeof z, hipMemcpyHostToDevice));
    return set_err(c, CLUE_ERR_INPUT, "invalid hit data: non-finite x/y/energy, layer out of range, "
                                      "or event ids out of range / decreasing");
  }
  return CLUE_OK;
}

static int run_common(clue_ctx* c, int64_t n, int32_t n_events, int32_t event_base, const int32_t* event,
                      const float* x, const float* y, const int32_t* layer, const float* energy, int32_t* cid,
                      uint8_t* seed, void* stream, bool batched) {
  int rc = check_run_args(c, n, n_events, x, y, layer, energy, cid, seed);
  if (rc != CLUE_OK) return rc;
  if (batched && n_events > 1 && n > 0 && !event) return set_err(c, CLUE_ERR_ARG, "null event ids");
  c->timed_valid = false;
  if (n == 0) {
    c->last_n = 0;
    c->last_events = n_events;
    return CLUE_OK;
  }
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  RunDesc d{};
  // the plain form may stage a different number of hits per work item
  c->g_plain = c->g;
  if (c->plain_cap > 0) c->g_plain.lds_cap = c->plain_cap;
  d.n = (int32_t)n;
  d.n_events = n_events;
  d.x = x;
  d.y = y;
  d.e = energy;
  d.layer = layer;
  d.event = batched ? event : nullptr;
  d.event_base = batched ? event_base : 0;
  d.cluster_id = cid;
  d.is_seed = seed;
  if (c->params.flags & CLUE_VALIDATE) {
    rc = validate_inputs(c, d, s);
    if (rc != CLUE_OK) return rc;
  }
  hipEvent_t* ev = c->timing ? c->ev : nullptr;
  if (!batched) {
    LaunchCfg cfg = c->cfg;
    cfg.graph_mode = false;
    HIP_TRY(c, launch_pipeline(c->g_plain, c->a, d, cfg, s, ev));
  } else {
    HIP_TRY(c, launch_set_desc(d, c->a.desc, s));
    if (ev) {
      LaunchCfg cfg = c->cfg;
      cfg.graph_mode = true;
      HIP_TRY(c, launch_pipeline(c->g, c->a, d, cfg, s, ev));
    } else {
      rc = ensure_graph(c);
      if (rc != CLUE_OK) return rc;
      HIP_TRY(c, hipGraphLaunch(c->exec, s));
    }
  }
  c->timed_valid = ev != nullptr;
  c->last_n = n;
  c->last_events = n_events;
  return CLUE_OK;
}

int clue_run(clue_ctx* c, int64_t n, const float* x, const float* y, const int32_t* layer, const float* energy,
             int32_t* cluster_id, uint8_t* is_seed, void* stream) {
  return run_common(c, n, 1, 0, nullptr, x, y, layer, energy, cluster_id, is_seed, stream, false);
}

int clue_run_batch(clue_ctx* c, int64_t n, int32_t n_events, const int32_t* event, const float* x, const float* y,
                   const int32_t* layer, const float* energy, int32_t* cluster_id, uint8_t* is_seed, void* stream) {
  return run_common(c, n, n_events, 0, event, x, y, layer, energy, cluster_id, is_seed, stream, true);
}

int clue_run_batch_range(clue_ctx* c, int64_t n, int32_t first_event, int32_t n_events, const int32_t* event,
                         const float* x, const float* y, const int32_t* layer, const float* energy,
                         int32_t* cluster_id, uint8_t* is_seed, void* stream) {
  if (first_event < 0) return set_err(c, CLUE_ERR_ARG, "first_event must be >= 0");
  return run_common(c, n, n_events, first_event, event, x, y, layer, energy, cluster_id, is_seed, stream, true);
}

// Device staging of the host-resident form: per chunk x, y, E, layer, event
// (4 bytes each) and cluster_id (4) + is_seed (1) for stage_hits hits.
struct StageChunk {
  float *x, *y, *e;
  int32_t *layer, *event, *cid;
  uint8_t* seed;
};

static StageChunk stage_chunk(clue_ctx* c, int k) {
  const size_t n = (size_t)c->stage_hits;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t per = al(4 * n) * 6 + al(n);
  char* b = (char*)c->stage_base + (size_t)k * per;
  StageChunk s;
  s.x = (float*)b;
  s.y = (float*)(b + al(4 * n));
  s.e = (float*)(b + 2 * al(4 * n));
  s.layer = (int32_t*)(b + 3 * al(4 * n));
  s.event = (int32_t*)(b + 4 * al(4 * n));
  s.cid = (int32_t*)(b + 5 * al(4 * n));
  s.seed = (uint8_t*)(b + 6 * al(4 * n));
  return s;
}

static int ensure_staging(clue_ctx* c) {
  if (c->stage_base && c->stage_hits == c->a.cap_hits) return CLUE_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  if (c->stage_base) {
    HIP_TRY(c, hipDeviceSynchronize());
    void* old = c->stage_base;
    c->stage_base = nullptr;
    HIP_TRY(c, hipFree(old));
  }
  const size_t n = (size_t)c->a.cap_hits;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t bytes = 2 * (al(4 * n) * 6 + al(n));
  if (c->budget && c->arena_bytes + bytes > c->budget)
    return set_err(c, CLUE_ERR_BUDGET, "host-form staging of " + std::to_string(bytes) + " bytes exceeds the HBM budget");
  hipError_t e = hipMalloc(&c->stage_base, bytes);
  if (e != hipSuccess) {
    c->stage_base = nullptr;
    return set_err(c, CLUE_ERR_NOMEM, "hipMalloc of the host-form staging failed");
  }
  c->stage_hits = (int64_t)n;
  for (hipStream_t* st : {&c->h2d, &c->comp, &c->d2h})
    if (!*st) HIP_TRY(c, hipStreamCreateWithFlags(st, hipStreamNonBlocking));
  for (int i = 0; i < 2; ++i)
    for (hipEvent_t* ev : {&c->in_ready[i], &c->done[i], &c->out_done[i]})
      if (!*ev) HIP_TRY(c, hipEventCreateWithFlags(ev, hipEventDisableTiming));
  return CLUE_OK;
}

int clue_run_batch_host(clue_ctx* c, int64_t n, int32_t n_events, const int32_t* event, const float* x,
                        const float* y, const int32_t* layer, const float* energy, int32_t* cluster_id,
                        uint8_t* is_seed) {
  if (!c) return CLUE_ERR_ARG;
  if (n < 0 || n >= ((int64_t)1 << 31) - 1) return set_err(c, CLUE_ERR_ARG, "n out of range");
  if (n_events < 1) return set_err(c, CLUE_ERR_ARG, "n_events must be >= 1");
  if (n > 0 && (!x || !y || !layer || !energy || !cluster_id || !is_seed))
    return set_err(c, CLUE_ERR_ARG, "null input or output pointer");
  if (n > 0 && n_events > 1 && !event) return set_err(c, CLUE_ERR_ARG, "null event ids");
  c->timed_valid = false;
  if (n == 0) {
    c->last_n = 0;
    c->last_events = n_events;
    return CLUE_OK;
  }
  // first hit of every event (ids non-decreasing; clamped so that the
  // chunks always tile [0, n))
  std::vector<int64_t> start((size_t)n_events + 1, 0);
  for (int32_t e = 0; e <= n_events; ++e) {
    int64_t lo = 0, hi = n;
    if (e == n_events || !event) {
      lo = e == 0 ? 0 : n;
    } else {
      while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (event[mid] < e)
          lo = mid + 1;
        else
          hi = mid;
      }
    }
    start[e] = e == 0 ? 0 : std::max(lo, start[e - 1]);
  }
  start[n_events] = n;
  // chunks of whole events within the capacity
  std::vector<std::pair<int32_t, int32_t>> chunks;  // (first event, count)
  for (int32_t e0 = 0; e0 < n_events;) {
    int32_t e1 = e0;
    while (e1 < n_events && e1 - e0 < c->a.cap_events && start[e1 + 1] - start[e0] <= c->a.cap_hits) ++e1;
    if (e1 == e0)
      return set_err(c, CLUE_ERR_CAPACITY, "event " + std::to_string(e0) + " has " +
                                               std::to_string(start[e0 + 1] - start[e0]) +
                                               " hits, more than the context capacity");
    chunks.emplace_back(e0, e1 - e0);
    e0 = e1;
  }
  int rc = ensure_staging(c);
  if (rc != CLUE_OK) return rc;
  for (size_t k = 0; k < chunks.size(); ++k) {
    const int slot = (int)(k & 1);
    const StageChunk sc = stage_chunk(c, slot);
    const int32_t e0 = chunks[k].first, ne = chunks[k].second;
    const int64_t h0 = start[e0], nh = start[e0 + ne] - h0;
    if (k >= 2) HIP_TRY(c, hipStreamWaitEvent(c->h2d, c->done[slot], 0));  // inputs of chunk k - 2 consumed
    HIP_TRY(c, hipMemcpyAsync(sc.x, x + h0, nh * 4, hipMemcpyHostToDevice, c->h2d));
    HIP_TRY(c, hipMemcpyAsync(sc.y, y + h0, nh * 4, hipMemcpyHostToDevice, c->h2d));
    HIP_TRY(c, hipMemcpyAsync(sc.e, energy + h0, nh * 4, hipMemcpyHostToDevice, c->h2d));
    HIP_TRY(c, hipMemcpyAsync(sc.layer, layer + h0, nh * 4, hipMemcpyHostToDevice, c->h2d));
    if (event) HIP_TRY(c, hipMemcpyAsync(sc.event, event + h0, nh * 4, hipMemcpyHostToDevice, c->h2d));
    HIP_TRY(c, hipEventRecord(c->in_ready[slot], c->h2d));
    HIP_TRY(c, hipStreamWaitEvent(c->comp, c->in_ready[slot], 0));
    if (k >= 2) HIP_TRY(c, hipStreamWaitEvent(c->comp, c->out_done[slot], 0));  // outputs of chunk k - 2 copied
    if (event)
      rc = run_common(c, nh, ne, e0, sc.event, sc.x, sc.y, sc.layer, sc.e, sc.cid, sc.seed, c->comp, true);
    else
      rc = run_common(c, nh, 1, 0, nullptr, sc.x, sc.y, sc.layer, sc.e, sc.cid, sc.seed, c->comp, true);
    if (rc != CLUE_OK) {
      (void)hipDeviceSynchronize();  // drain the copies in flight; rc is the error reported
      return rc;
    }
    HIP_TRY(c, hipEventRecord(c->done[slot], c->comp));
    HIP_TRY(c, hipStreamWaitEvent(c->d2h, c->done[slot], 0));
    HIP_TRY(c, hipMemcpyAsync(cluster_id + h0, sc.cid, nh * 4, hipMemcpyDeviceToHost, c->d2h));
    HIP_TRY(c, hipMemcpyAsync(is_seed + h0, sc.seed, nh, hipMemcpyDeviceToHost, c->d2h));
    HIP_TRY(c, hipEventRecord(c->out_done[slot], c->d2h));
  }
  HIP_TRY(c, hipStreamSynchronize(c->d2h));
  HIP_TRY(c, hipStreamSynchronize(c->comp));
  return clue_status(c, c->comp);
}

int clue_get_intermediates(clue_ctx* c, float* rho, int32_t* nh, float* delta2, void* stream) {
  if (!c) return CLUE_ERR_ARG;
  if (!(c->params.flags & CLUE_KEEP_INTERMEDIATES))
    return set_err(c, CLUE_ERR_STATE, "context created without CLUE_KEEP_INTERMEDIATES");
  if (c->last_n < 0) return set_err(c, CLUE_ERR_STATE, "no run yet");
  const size_t b = (size_t)c->last_n * 4;
  hipStream_t s = (hipStream_t)stream;
  if (b == 0) return CLUE_OK;
  if (rho) HIP_TRY(c, hipMemcpyAsync(rho, c->a.rho_out, b, hipMemcpyDeviceToDevice, s));
  if (nh) HIP_TRY(c, hipMemcpyAsync(nh, c->a.nh_out, b, hipMemcpyDeviceToDevice, s));
  if (delta2) HIP_TRY(c, hipMemcpyAsync(delta2, c->a.d2_out, b, hipMemcpyDeviceToDevice, s));
  return CLUE_OK;
}

int clue_get_followers(clue_ctx* c, int32_t* fstart, int32_t* flist, int64_t* n_followers_out, void* stream) {
  if (!c) return CLUE_ERR_ARG;
  if (c->params.flags & CLUE_NO_FOLLOWERS) return set_err(c, CLUE_ERR_STATE, "context built without follower lists");
  if (c->last_n < 0) return set_err(c, CLUE_ERR_STATE, "no run yet");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = c->last_n;
  if (n == 0) {
    if (fstart) {
      const int32_t z = 0;
      HIP_TRY(c, hipMemcpyAsync(fstart, &z, 4, hipMemcpyHostToDevice, s));
      HIP_TRY(c, hipStreamSynchronize(s));
    }
    if (n_followers_out) *n_followers_out = 0;
    return CLUE_OK;
  }
  if (fstart) HIP_TRY(c, hipMemcpyAsync(fstart, c->a.fstart, (size_t)(n + 1) * 4, hipMemcpyDeviceToDevice, s));
  if (flist) HIP_TRY(c, hipMemcpyAsync(flist, c->a.flist, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  if (n_followers_out) {
    int32_t tot = 0;
    HIP_TRY(c, hipStreamSynchronize(s));
    HIP_TRY(c, hipMemcpy(&tot, c->a.fstart + n, 4, hipMemcpyDeviceToHost));
    *n_followers_out = tot;
  }
  return CLUE_OK;
}

int clue_status(clue_ctx* c, void* stream) {
  if (!c) return CLUE_ERR_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize((hipStream_t)stream));
  if (!c->a.err) return CLUE_OK;  // no arena bound (a failed reallocation)
  uint32_t err = 0;
  HIP_TRY(c, hipMemcpy(&err, c->a.err, sizeof err, hipMemcpyDeviceToHost));
  if (err) {
    uint32_t z = 0;
    HIP_TRY(c, hipMemcpy(c->a.err, &z, sizeof z, hipMemcpyHostToDevice));
  }
  if (err & E_INPUT) return set_err(c, CLUE_ERR_INPUT, "invalid hit data");
  if (err & E_WINDOW) return set_err(c, CLUE_ERR_DEVICE, "a query window left its staged halo");
  if (err & E_WALK) return set_err(c, CLUE_ERR_DEVICE, "a cluster expansion walk exceeded its step bound");
  return CLUE_OK;
}

int clue_set_tuning(clue_ctx* c, const clue_tuning* t) {
  if (!c || !t) return CLUE_ERR_ARG;
  Geom g{};
  std::string msg;
  const float tile = t->tile_size > 0.0f ? t->tile_size : c->tile;
  const int tpq = t->threads_per_query > 0 ? t->threads_per_query : c->tpq;
  const int bx = t->block_x > 0 ? t->block_x : c->bx, by = t->block_y > 0 ? t->block_y : c->by;
  const int cap = t->lds_cap > 0 ? t->lds_cap : c->lds_cap;
  const int plain_cap = t->plain_lds_cap > 0 ? t->plain_lds_cap : c->plain_cap;
  if (plain_cap != 0 && (plain_cap < 64 || plain_cap > kMaxLdsCap))
    return set_err(c, CLUE_ERR_ARG, "plain_lds_cap must be within 64..2048 hits");
  const float r1 = t->nh_first_radius >= 0.0f ? t->nh_first_radius : c->r1;
  const int quads = t->density_quads > 0 ? t->density_quads : c->quads;
  const int expansion = t->expansion > 0 ? t->expansion : c->expansion;
  int rc = plan_geom(c->params, tile, tpq, bx, by, cap, r1, quads, expansion, g, msg);
  if (rc != CLUE_OK) return set_err(c, rc, msg);
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  const bool regrow =
      (int64_t)c->a.cap_events * g.L * g.tpl + 1 > c->a.cap_tiles || (builds_lists(g) && !c->a.flist);
  const Geom old = c->g;
  c->g = g;
  drop_graph(c);
  compute_cfg(c);
  if (regrow) {
    rc = alloc_arena(c, c->a.cap_hits, c->a.cap_events);
    if (rc != CLUE_OK) {
      c->g = old;
      compute_cfg(c);
      return rc;
    }
  }
  c->tile = tile;
  c->tpq = tpq;
  c->bx = bx;
  c->by = by;
  c->lds_cap = cap;
  c->plain_cap = plain_cap;
  c->r1 = r1;
  c->quads = quads;
  c->expansion = expansion;
  return CLUE_OK;
}

int clue_get_tuning(const clue_ctx* c, clue_tuning* t, int32_t* halo) {
  if (!c) return CLUE_ERR_ARG;
  if (t) {
    t->tile_size = (float)(1.0 / (double)c->g.inv_t);
    t->threads_per_query = c->g.tpq;
    t->block_x = c->g.bx;
    t->block_y = c->g.by;
    t->lds_cap = c->g.lds_cap;
    t->plain_lds_cap = c->plain_cap > 0 ? c->plain_cap : c->g.lds_cap;
    t->nh_first_radius = c->g.nh_phase1 ? std::sqrt(c->g.r1sq) : 0.0f;
    t->density_quads = c->g.density_quads == 0 ? 2 : (c->g.density_quads == 2 ? 3 : 1);
    t->expansion = c->g.expand ? 2 : 1;
  }
  if (halo) *halo = c->g.halo;
  return CLUE_OK;
}

int clue_enable_stage_timing(clue_ctx* c, int enable) {
  if (!c) return CLUE_ERR_ARG;
  c->timing = enable != 0;
  c->timed_valid = false;
  return CLUE_OK;
}

int clue_stage_times(clue_ctx* c, float* ms, const char** names, int cap) {
  if (!c) return CLUE_ERR_ARG;
  if (!c->timed_valid) return set_err(c, CLUE_ERR_STATE, "no timed run since timing was enabled");
  HIP_TRY(c, hipEventSynchronize(c->ev[S_COUNT]));
  int k = 0;
  for (; k < S_COUNT && k < cap; ++k) {
    float t = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&t, c->ev[k], c->ev[k + 1]));
    if (ms) ms[k] = t;
    if (names) names[k] = kStageNames[k];
  }
  return S_COUNT;
}

// ---------------------------------------------------------------------------
// The no-allocation form: the plain one-event pipeline over a fixed scratch
// array in device memory. The array is a module global, so each device that
// loads this library holds its own copy until the process ends; its device
// address is looked up once per device (the name itself is only a host-side
// stand-in) and every run on that device shares it.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;  // CLUE_NOALLOC_SCRATCH_BYTES
static_assert(kNoAllocScratchBytes == (size_t)CLUE_NOALLOC_SCRATCH_BYTES, "header and library agree on the size");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device `dev`, looked up on the
// first call there.
static int scratch_on_device(int dev, void** out) {
  if (dev < 0 || dev >= kMaxScratchDevices)
    return set_err(nullptr, CLUE_ERR_ARG, "device index beyond the no-allocation form's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_err(nullptr, CLUE_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CLUE_OK;
}

int clue_run_noalloc(const clue_params* p, const clue_tuning* t, int64_t n, const float* x, const float* y,
                     const int32_t* layer, const float* energy, int32_t* cluster_id, uint8_t* is_seed,
                     void* stream) {
  if (!p) return set_err(nullptr, CLUE_ERR_ARG, "null params");
  if (n < 0 || n >= ((int64_t)1 << 31) - 1) return set_err(nullptr, CLUE_ERR_ARG, "n out of range");
  if (n > 0 && (!x || !y || !layer || !energy || !cluster_id || !is_seed))
    return set_err(nullptr, CLUE_ERR_ARG, "null input or output pointer");
  if (p->flags & (CLUE_VALIDATE | CLUE_KEEP_INTERMEDIATES))
    return set_err(nullptr, CLUE_ERR_ARG,
                   "CLUE_VALIDATE and CLUE_KEEP_INTERMEDIATES need a context: the no-allocation form "
                   "neither synchronises nor keeps results past the call");
  // the tuning of a fresh context, with any positive field of *t in its place
  const clue_ctx defaults{};
  float tile = p->tile_size;
  int tpq = p->threads_per_query > 0 ? p->threads_per_query : 1;
  int bx = defaults.bx, by = defaults.by, cap = defaults.lds_cap, quads = defaults.quads;
  float r1 = defaults.r1;
  int expansion = defaults.expansion;
  if (t) {
    if (t->tile_size > 0.0f) tile = t->tile_size;
    if (t->threads_per_query > 0) tpq = t->threads_per_query;
    if (t->block_x > 0) bx = t->block_x;
    if (t->block_y > 0) by = t->block_y;
    // a single event runs as the plain form: its own cap when set
    if (t->plain_lds_cap > 0)
      cap = t->plain_lds_cap;
    else if (t->lds_cap > 0)
      cap = t->lds_cap;
    if (t->nh_first_radius >= 0.0f) r1 = t->nh_first_radius;
    if (t->density_quads > 0) quads = t->density_quads;
    if (t->expansion > 0) expansion = t->expansion;
  }
  Geom g{};
  std::string msg;
  int rc = plan_geom(*p, tile, tpq, bx, by, cap, r1, quads, expansion, g, msg);
  if (rc != CLUE_OK) return set_err(nullptr, rc, msg);
  ArenaPlan P;
  if (!plan_arena(g, std::max<int64_t>(n, 1), 1, P) || P.total > kNoAllocScratchBytes)
    return set_err(nullptr, CLUE_ERR_CAPACITY,
                   "the no-allocation form holds " + std::to_string(kNoAllocScratchBytes) +
                       " bytes of scratch per device; this run of " + std::to_string(n) + " hits needs " +
                       std::to_string(P.total) + " (use a context)");
  if (n == 0) return CLUE_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_err(nullptr, CLUE_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  void* base = nullptr;
  rc = scratch_on_device(dev, &base);
  if (rc != CLUE_OK) return rc;
  const Arena a = arena_at((char*)base, g, P, n, 1);
  RunDesc d{};
  d.n = (int32_t)n;
  d.n_events = 1;
  d.x = x;
  d.y = y;
  d.e = energy;
  d.layer = layer;
  d.event = nullptr;
  d.event_base = 0;
  d.cluster_id = cluster_id;
  d.is_seed = is_seed;
  // plain launches, sized to the run; the first kernel clears every counter,
  // tile count and scan status the run reads, so the previous call's
  // contents do not matter
  LaunchCfg cfg{};
  cfg.graph_mode = false;
  if (g.expand) {  // the k-way walk's grid: one run of workgroups per XCD
    int ncu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return set_err(nullptr, CLUE_ERR_HIP, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(e));
    cfg.persist_blocks_stream = std::max(1, ncu) * 8;
  }
  e = launch_pipeline(g, a, d, cfg, (hipStream_t)stream, nullptr);
  if (e != hipSuccess) return set_err(nullptr, CLUE_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return CLUE_OK;
}

const char* clue_last_error(const clue_ctx* c) {
  if (!c) return g_create_err.c_str();
  return c->err.c_str();
}

// Teardown has no caller to report to: every release is attempted, and their
// status codes are deliberately dropped.
void clue_destroy(clue_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipStream_t st : {c->h2d, c->comp, c->d2h})
    if (st) (void)hipStreamDestroy(st);
  for (int i = 0; i < 2; ++i)
    for (hipEvent_t e : {c->in_ready[i], c->done[i], c->out_done[i]})
      if (e) (void)hipEventDestroy(e);
  if (c->stage_base) (void)hipFree(c->stage_base);
  for (int i = 0; i <= S_COUNT; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->arena_base) (void)hipFree(c->arena_base);
  delete c;
}

}  // extern "C"
