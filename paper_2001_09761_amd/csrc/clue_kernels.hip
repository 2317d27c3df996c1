// HIP kernels of libclue for gfx950 (MI355X).
//
// Stage map (arXiv:2001.09761):
//   k_clear            clears counters, tile counts and scan status
//   k_hist             fixed grid, part 1: atomic per-tile histogram (Sec. 2.1)
//   k_scan<TILES>      exclusive prefix scan of the tile counts (decoupled look-back)
//   k_scatter          fixed grid, part 2: hit ids into the tile CSR (arrival order)
//   k_place            fixed grid, part 3: each tile's records in ascending hit index
//   k_density          rho (Eq. 3, Algorithm 1) over LDS-staged tile windows,
//                      summed in ascending hit index along merged 2x2-tile
//                      lists of the index-ordered tiles
//   k_density_spill    rho of the queries in tiles too dense for LDS, queued by
//                      k_density and spread over the whole GPU
//   k_nearest_higher   nh / delta (Eq. 4, Algorithm 2) fused with the seed /
//                      outlier / follower decision (Sec. 2.2, Algorithm 3)
//   k_nh_spill         the same for the queries that k_nearest_higher queued
//   k_scan<SEEDS>      seed numbering by prefix scan over the seed bitmap (and
//                      follower list offsets); writes the caller-order seed flags
//   k_label            cluster ids: each hit follows nearest-higher links of
//                      followers to its root (pointer jumping with path
//                      compression); registers follower-list entries
//   k_expand_init      the k-way alternative to k_label (Algorithm 3): follower
//   k_expand_dfs       lists, seed list, then one depth-first walk per seed
//   k_follow_sort      sorts each follower list by hit index, event-local ids
//
// Every float operation that decides a result is an explicit round-to-nearest
// intrinsic (no contraction), so results match a plain IEEE binary32
// evaluation of the same expressions.
#include "clue_internal.h"

#include <algorithm>
#include <climits>

namespace clue {

const char* const kStageNames[S_COUNT] = {"clear",        "grid_hist",  "grid_scan",
                                          "grid_scatter", "grid_place", "density",
                                          "nearest_higher", "seed_scan", "labels",
                                          "follower_lists"};

// ---------------------------------------------------------------------------
// Run descriptor: by value (plain launches) or from device memory (graph).
// ---------------------------------------------------------------------------
template <bool G>
struct DescArg;
template <>
struct DescArg<false> {
  RunDesc d;
  __device__ __forceinline__ RunDesc get() const { return d; }
};
template <>
struct DescArg<true> {
  const RunDesc* p;
  __device__ __forceinline__ RunDesc get() const { return *p; }
};

// ---------------------------------------------------------------------------
// Geometry helpers.
// ---------------------------------------------------------------------------

// Tile coordinate of a position: floor((v - origin) / T) clamped to the grid.
// Monotone non-decreasing in v, which is what makes the query windows below
// supersets of the true neighbourhoods.
__device__ __forceinline__ int tile_coord(float v, float origin, float inv_t, int n) {
  float t = floorf(__fmul_rn(__fsub_rn(v, origin), inv_t));
  t = fminf(fmaxf(t, 0.0f), (float)(n - 1));
  return (int)t;
}

__device__ __forceinline__ float dist2(float xi, float yi, float xj, float yj) {
  float dx = __fsub_rn(xi, xj);
  float dy = __fsub_rn(yi, yj);
  return __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
}

// Half width of a query window: the radius inflated by 2^-10 relative plus
// 2^-20 |v|, so that rounding of v +- w can never exclude a hit whose float32
// squared distance passes the strict threshold.
__device__ __forceinline__ float window_half(float w, float v) {
  return __fadd_rn(w, __fmul_rn(fabsf(v), 0x1p-20f));
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ int ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int32_t* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// First caller-order hit of event e, clamped to [0, n] (memory safety for
// unvalidated event ids).
__device__ __forceinline__ int event_first_hit(const Arena& a, const RunDesc& d, int e) {
  return clampi(a.ev_start[e], 0, d.n);
}

// Seeds are marked by one bit per hit in caller order; the seed scan gives
// the count before each 32-bit word. Words cover hits 0..n, so the rank of
// n (the seed total) is defined too.
__host__ __device__ __forceinline__ int64_t seed_words(int64_t n) { return n / 32 + 1; }
// Seeds among caller hits 0..h-1 (h in [0, n]).
__device__ __forceinline__ int seed_rank(const Arena& a, int h) {
  return a.seed_wrank[h >> 5] + __popc(a.seedbits[h >> 5] & ((1u << (h & 31)) - 1u));
}

// Event of tile-CSR slot s: slots are ordered by (event, layer, tile), so the
// event is the last e whose first tile starts at or before s.
__device__ __forceinline__ int event_of_slot(const Geom& g, const Arena& a, const RunDesc& d, int s) {
  const int64_t per = (int64_t)g.L * g.tpl;
  int lo = 0, hi = d.n_events - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.tile_start[mid * per] <= s)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Streaming kernels cut their index range into chunks of `chunk` consecutive
// indices and give each XCD one contiguous run of chunks (workgroups are
// dispatched to the XCDs round-robin by id; the grid is a multiple of
// kQueues). Neighbouring indices share lines in the gathers and scattered
// writes that follow, so they are fetched into, and completed in, one L2.
// ---------------------------------------------------------------------------
struct ChunkRun {
  int c, end, step;
};
__device__ __forceinline__ ChunkRun xcd_run(int n, int chunk) {
  const int nch = (int)(((int64_t)n + chunk - 1) / chunk);
  const int x = (int)blockIdx.x % kQueues, i = (int)blockIdx.x / kQueues;
  return {(int)((int64_t)nch * x / kQueues) + i, (int)((int64_t)nch * (x + 1) / kQueues),
          (int)gridDim.x / kQueues};
}

// ---------------------------------------------------------------------------
// k_clear
// ---------------------------------------------------------------------------
template <bool G>
__global__ __launch_bounds__(kWG) void k_clear(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  const int64_t tt = (int64_t)d.n_events * g.L * g.tpl + 1;
  const int64_t n1 = (int64_t)d.n + 1;
  const bool fol = builds_lists(g);
  const int64_t stride = (int64_t)gridDim.x * kWG;
  const int64_t i0 = (int64_t)blockIdx.x * kWG + threadIdx.x;
  for (int64_t i = i0; i < tt; i += stride) a.tile_start[i] = 0;
  if (fol)
    for (int64_t i = i0; i < n1; i += stride) a.fstart[i] = 0;
  constexpr int64_t SC = (int64_t)kWG * scan_items(G);
  const int64_t nchunk_t = (tt + SC - 1) / SC;
  const int64_t nchunk_s = (n1 + SC - 1) / SC;
  for (int64_t i = i0; i < nchunk_t && i < a.cap_chunks; i += stride) a.scan_status[i] = 0ull;
  for (int64_t i = i0; i < nchunk_s && i < a.cap_chunks; i += stride) a.scan_status[a.cap_chunks + i] = 0ull;
  for (int64_t i = i0; i < C_COUNT; i += stride) a.counters[i] = 0;
  for (int64_t i = i0; i <= d.n_events; i += stride) a.ev_start[i] = 0;
  for (int64_t i = i0; i < seed_words(d.n); i += stride) a.seedbits[i] = 0u;
}

// ---------------------------------------------------------------------------
// k_hist: tile of every hit, atomic count per tile, arrival rank kept.
// Lanes of a wave that share a tile are grouped first, so each distinct tile
// costs one atomic per wave (hits of a cluster tend to be adjacent in input
// order); ranks within a group follow lane order. Each lane takes kPlaceU
// hits per step so that their atomics are in flight together.
// ---------------------------------------------------------------------------
template <bool G>
__global__ __launch_bounds__(kWG) void k_hist(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  constexpr int U = kPlaceU;  // sub-batches per step; their atomics overlap
  const int lane = threadIdx.x & 63;
  for (ChunkRun r = xcd_run(d.n, kWG * U); r.c < r.end; r.c += r.step) {
    const int h0 = r.c * kWG * U;  // uniform per workgroup
    // every load of a lane is issued before its first store (the event
    // starts below could alias the inputs as far as the compiler knows)
    int t[U], ev[U], evp[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int h = h0 + j * kWG + (int)threadIdx.x;
      t[j] = -1;
      ev[j] = evp[j] = 0;
      if (h < d.n) {
        if (d.event) {
          ev[j] = clampi(d.event[h] - d.event_base, 0, d.n_events - 1);
          evp[j] = h == 0 ? -1 : clampi(d.event[h - 1] - d.event_base, 0, d.n_events - 1);
        }
        const int l = clampi(d.layer[h], 0, g.L - 1);
        const int tx = tile_coord(d.x[h], g.x0, g.inv_t, g.nx);
        const int ty = tile_coord(d.y[h], g.y0, g.inv_t, g.ny);
        t[j] = l * g.tpl + ty * g.nx + tx;  // the event's part is added below
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int h = h0 + j * kWG + (int)threadIdx.x;
      if (h >= d.n) continue;
      const int e = ev[j];
      t[j] += e * g.L * g.tpl;
      if (d.event) {
        for (int k = evp[j] + 1; k <= e; ++k) a.ev_start[k] = h;
        if (h == d.n - 1)
          for (int k = e + 1; k <= d.n_events; ++k) a.ev_start[k] = d.n;
      } else if (h == 0) {
        a.ev_start[0] = 0;
        a.ev_start[1] = d.n;
      }
    }
    int base[U], off[U], leader[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const bool valid = t[j] >= 0;
      unsigned long long todo = __ballot(valid);
      int ld = lane, o = 0, cnt = 0;
      while (todo) {  // wave-uniform: one pass per distinct tile in the wave
        // the lowest unmatched lane leads; its tile is read into a scalar
        // register, and a lane's offset is the count of its peers below it
        const int l = __ffsll((long long)todo) - 1;
        const int lt = __builtin_amdgcn_readlane(t[j], l);
        const bool mine = t[j] == lt;  // invalid lanes (-1) never match a tile
        const unsigned long long peers = __ballot(mine);
        if (mine) {
          ld = l;
          o = __builtin_amdgcn_mbcnt_hi((unsigned)(peers >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)peers, 0u));
          cnt = __popcll(peers);
        }
        todo &= ~peers;
      }
      base[j] = 0;
      if (valid && lane == ld) base[j] = atomicAdd(&a.tile_start[t[j]], cnt);
      off[j] = o;
      leader[j] = ld;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int bs = __shfl(base[j], leader[j], 64);
      const int h = h0 + j * kWG + (int)threadIdx.x;
      if (t[j] >= 0) {
        a.key[h] = t[j];
        a.rank[h] = bs + off[j];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// k_scatter: hit h's id and tile go to slot tile_start[tile] + rank (arrival
// order within a tile), kept in the rho and parent buffers, which are free
// until the density stage.
// k_place: slot by slot, each hit counts the ids of its tile that are smaller
// than its own and writes its record at that position, so every tile of the
// CSR lists its hits in ascending hit index. Neighbouring slots share their
// tile, so the counting loads are broadcasts from lines just read.
// ---------------------------------------------------------------------------
template <bool G>
__global__ __launch_bounds__(kWG) void k_scatter(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  int* ids = reinterpret_cast<int*>(a.rho);
  constexpr int U = G ? kBatchU : kPlaceU;
  for (ChunkRun rn = xcd_run(d.n, kWG * U); rn.c < rn.end; rn.c += rn.step) {
    const int h0 = rn.c * kWG * U + (int)threadIdx.x;
    int t[U], r[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int h = h0 + j * kWG;
      t[j] = -1;
      if (h < d.n) {
        t[j] = a.key[h];
        r[j] = a.rank[h];
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (t[j] >= 0) {
        const int s = a.tile_start[t[j]] + r[j];
        ids[s] = h0 + j * kWG;
        a.parent[s] = t[j];
      }
    }
  }
}

template <bool G>
__global__ __launch_bounds__(kWG) void k_place(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  const int* ids = reinterpret_cast<const int*>(a.rho);
  constexpr int U = G ? kBatchU : kPlaceU;
  constexpr int C = kWG * U;  // slots per chunk
  // the chunk's arrival-order ids in LDS: a hit's tile mostly lies inside
  // the chunk, so most of its counting reads are LDS reads
  __shared__ int s_ids[C];
  for (ChunkRun rn = xcd_run(d.n, C); rn.c < rn.end; rn.c += rn.step) {
    const int c0 = rn.c * C;
    const int c1 = min(c0 + C, d.n);
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int sl = c0 + (int)threadIdx.x + j * kWG;
      s_ids[sl - c0] = sl < d.n ? ids[sl] : 0;
    }
    __syncthreads();
    // slots in groups of four: a group's loads are all issued before its
    // first store (which could alias them as far as the compiler knows)
    constexpr int V = 4;
#pragma unroll
    for (int j0 = 0; j0 < U; j0 += V) {
      int hv[V], s0v[V], s1v[V];
      float xv[V], yv[V], ev[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int sl = c0 + (int)threadIdx.x + (j0 + k) * kWG;
        hv[k] = -1;
        if (sl < d.n) {
          const int h = s_ids[sl - c0];
          const int t = a.parent[sl];
          hv[k] = h;
          xv[k] = d.x[h];
          yv[k] = d.y[h];
          ev[k] = d.e[h];
          s0v[k] = a.tile_start[t];
          s1v[k] = a.tile_start[t + 1];
        }
      }
#pragma unroll
      for (int k = 0; k < V; ++k) {
        if (hv[k] < 0) continue;
        const int h = hv[k], s0 = s0v[k], s1 = s1v[k];
        // the tile [s0, s1) in three parts: before the chunk, in it, after it
        const int m0 = min(max(s0, c0), s1), m1 = max(min(s1, c1), m0);
        int rk = 0;
        for (int c = s0; c < m0; ++c) rk += ids[c] < h;
        int c = m0;
        for (; c + 3 < m1; c += 4)
          rk += (s_ids[c - c0] < h) + (s_ids[c + 1 - c0] < h) + (s_ids[c + 2 - c0] < h) + (s_ids[c + 3 - c0] < h);
        for (; c < m1; ++c) rk += s_ids[c - c0] < h;
        for (c = m1; c < s1; ++c) rk += ids[c] < h;
        const int slot = s0 + rk;
        a.xs[slot] = xv[k];
        a.ys[slot] = yv[k];
        a.es[slot] = ev[k];
        a.hs[slot] = h;
      }
    }
    __syncthreads();  // the next chunk overwrites the staged ids
  }
}

// ---------------------------------------------------------------------------
// Decoupled look-back exclusive scan, one or two channels.
// Status word: [63:62] flag (1 aggregate, 2 inclusive prefix), [61:31]
// channel 1, [30:0] channel 0. Every value is a count below 2^31.
// Chunk ids come from an atomic ticket, so every chunk a workgroup waits on
// was taken by a running workgroup that publishes without waiting: each wait
// ends.
// ---------------------------------------------------------------------------
enum ScanKind { SCAN_TILES = 0, SCAN_SEEDS = 1, SCAN_SEEDS_FOLLOW = 2 };

__device__ __forceinline__ unsigned long long st_pack(int flag, int v0, int v1) {
  return ((unsigned long long)flag << 62) | ((unsigned long long)(unsigned)(v1 & 0x7fffffff) << 31) |
         (unsigned long long)(unsigned)(v0 & 0x7fffffff);
}
__device__ __forceinline__ int st_flag(unsigned long long w) { return (int)(w >> 62); }
__device__ __forceinline__ int st_v0(unsigned long long w) { return (int)(w & 0x7fffffffull); }
__device__ __forceinline__ int st_v1(unsigned long long w) { return (int)((w >> 31) & 0x7fffffffull); }

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <bool G, int KIND>
__global__ __launch_bounds__(kWG) void k_scan(DescArg<G> dg, Geom g, Arena a) {
  constexpr int NCH = KIND == SCAN_SEEDS_FOLLOW ? 2 : 1;
  constexpr int SI = scan_items(G), SC = kWG * SI;
  const RunDesc d = dg.get();
  const int64_t nel = KIND == SCAN_TILES ? (int64_t)d.n_events * g.L * g.tpl : (int64_t)d.n;
  const int64_t nout = nel + 1;  // the last output is the total
  const int64_t nchunks = (nout + SC - 1) / SC;
  unsigned long long* status = a.scan_status + (KIND == SCAN_TILES ? 0 : a.cap_chunks);
  int* ticket = &a.counters[KIND == SCAN_TILES ? C_TICKET_TILES : C_TICKET_SEEDS];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  __shared__ int s_chunk;
  __shared__ int s_wsum[NCH][kWG / 64];
  __shared__ int s_prefix[NCH];

  for (;;) {
    if (threadIdx.x == 0) s_chunk = atomicAdd(ticket, 1);
    __syncthreads();
    const int64_t chunk = s_chunk;
    __syncthreads();
    if (chunk >= nchunks) break;
    const int64_t base = chunk * SC + (int64_t)threadIdx.x * SI;

    int v[NCH][SI];
    if constexpr (KIND == SCAN_TILES) {
      if (base + SI <= nel) {
        const int4* p = reinterpret_cast<const int4*>(a.tile_start + base);
#pragma unroll
        for (int q = 0; q < SI / 4; ++q) {
          int4 w = p[q];
          v[0][4 * q] = w.x; v[0][4 * q + 1] = w.y; v[0][4 * q + 2] = w.z; v[0][4 * q + 3] = w.w;
        }
      } else {
#pragma unroll
        for (int i = 0; i < SI; ++i) v[0][i] = base + i < nel ? a.tile_start[base + i] : 0;
      }
    } else {
      // channel 0: the seeds of bitmap word w at element 32 w, zero elsewhere,
      // so that the prefix at 32 w counts the seeds before word w
      static_assert(SI % 32 == 0 || 32 % SI == 0, "a thread's elements hold whole words or none");
      const int64_t nw = seed_words(d.n);
      // the bitmap words of this thread's elements, loaded once
      constexpr int NW = (SI + 31) / 32;
      unsigned wv[NW];
#pragma unroll
      for (int k = 0; k < NW; ++k) wv[k] = (base >> 5) + k < nw ? a.seedbits[(base >> 5) + k] : 0u;
#pragma unroll
      for (int i = 0; i < SI; ++i) {
        const int64_t e = base + i;
        v[0][i] = (e & 31) == 0 ? __popc(wv[(e >> 5) - (base >> 5)]) : 0;
      }
      // the follower counts are loaded before the flag stores below, which
      // could alias them as far as the compiler knows
      if constexpr (NCH == 2) {
        if (base + SI <= nel) {
          const int4* p = reinterpret_cast<const int4*>(a.fstart + base);
#pragma unroll
          for (int q = 0; q < SI / 4; ++q) {
            int4 w = p[q];
            v[1][4 * q] = w.x; v[1][4 * q + 1] = w.y; v[1][4 * q + 2] = w.z; v[1][4 * q + 3] = w.w;
          }
        } else {
#pragma unroll
          for (int i = 0; i < SI; ++i) v[1][i] = base + i < nel ? a.fstart[base + i] : 0;
        }
      }
      // the caller-order seed flags, expanded from the bitmap 16 at a time
      // (one bit per hit -> one byte per hit), in coalesced stores
      static_assert(SI % 16 == 0, "flags are written 16 at a time");
#pragma unroll
      for (int q = 0; q < SI; q += 16) {
        const int64_t e0 = base + q;
        if (e0 >= nel) break;
        const unsigned w = (wv[(e0 >> 5) - (base >> 5)] >> (e0 & 31)) & 0xffffu;
        unsigned b4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) b4[k] = (((w >> (4 * k)) & 0xfu) * 0x00204081u) & 0x01010101u;
        uint8_t* dst = d.is_seed + e0;
        if (e0 + 16 <= nel && ((uintptr_t)dst & 15u) == 0) {
          *reinterpret_cast<uint4*>(dst) = make_uint4(b4[0], b4[1], b4[2], b4[3]);
        } else {
          for (int k = 0; k < 16 && e0 + k < nel; ++k) dst[k] = (uint8_t)((w >> k) & 1u);
        }
      }
    }
    // thread-local exclusive prefix
    int tsum[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      int acc = 0;
#pragma unroll
      for (int i = 0; i < SI; ++i) {
        int t = v[c][i];
        v[c][i] = acc;
        acc += t;
      }
      tsum[c] = acc;
    }
    int texcl[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      int incl = wave_incl_scan(tsum[c], lane);
      texcl[c] = incl - tsum[c];
      if (lane == 63) s_wsum[c][wave] = incl;
    }
    __syncthreads();
    int agg[NCH];
    int wbase[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      int acc = 0;
      wbase[c] = 0;
#pragma unroll
      for (int w = 0; w < kWG / 64; ++w) {
        if (w == wave) wbase[c] = acc;
        acc += s_wsum[c][w];
      }
      agg[c] = acc;
    }
    // look-back by wave 0
    if (wave == 0) {
      int run[NCH];
#pragma unroll
      for (int c = 0; c < NCH; ++c) run[c] = 0;
      if (chunk == 0) {
        if (lane == 0)
          __hip_atomic_store(&status[0], st_pack(2, agg[0], NCH == 2 ? agg[NCH - 1] : 0), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      } else {
        if (lane == 0)
          __hip_atomic_store(&status[chunk], st_pack(1, agg[0], NCH == 2 ? agg[NCH - 1] : 0), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        int64_t look = chunk - 1;
        for (;;) {
          const int64_t j = look - lane;
          unsigned long long w = j >= 0 ? __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                        : st_pack(2, 0, 0);
          while (__any(st_flag(w) == 0)) {
            if (st_flag(w) == 0)
              w = __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          const unsigned long long incl_mask = __ballot(st_flag(w) == 2);
          const int stop = incl_mask ? __ffsll((long long)incl_mask) - 1 : 64;
          const bool take = lane <= stop;
          run[0] += wave_sum(take ? st_v0(w) : 0);
          if constexpr (NCH == 2) run[1] += wave_sum(take ? st_v1(w) : 0);
          if (incl_mask) break;
          look -= 64;
        }
        if (lane == 0)
          __hip_atomic_store(&status[chunk],
                             st_pack(2, run[0] + agg[0], NCH == 2 ? run[NCH - 1] + agg[NCH - 1] : 0),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (lane == 0) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) s_prefix[c] = run[c];
      }
    }
    __syncthreads();
    // outputs
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int off = s_prefix[c] + wbase[c] + texcl[c];
      if (KIND != SCAN_TILES && c == 0) {  // one count per bitmap word
#pragma unroll
        for (int i = 0; i < SI; i += 32)
          if (base + i < nout && ((base + i) & 31) == 0) a.seed_wrank[(base + i) >> 5] = off + v[c][i];
        continue;
      }
      int* out = KIND == SCAN_TILES ? a.tile_start : a.fstart;
      if (base + SI <= nout) {
        int4* p = reinterpret_cast<int4*>(out + base);
#pragma unroll
        for (int q = 0; q < SI / 4; ++q)
          p[q] = make_int4(off + v[c][4 * q], off + v[c][4 * q + 1], off + v[c][4 * q + 2], off + v[c][4 * q + 3]);
      } else {
#pragma unroll
        for (int i = 0; i < SI; ++i)
          if (base + i < nout) out[base + i] = off + v[c][i];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Tile-block work items. An item is one (event, layer) unit and a block of
// bx*by tiles (the core); its staged region adds `halo` tiles around the core
// (clamped to the grid). Dense blocks whose region does not fit in LDS are
// processed as four quarter blocks, a quarter that still does not fit one
// core tile at a time, and a tile whose own region does not fit is queued
// for the stage's spill kernel, which searches global memory.
// ---------------------------------------------------------------------------
struct Region {
  int unit;       // event * L + layer
  int e;          // event
  int rx0, ry0;   // region origin (tile coordinates)
  int rw, rh;     // region size in tiles
  int cx0, cy0;   // core origin relative to the region
  int cw, ch;     // core size in tiles
  int total;      // hits in the region
};

// Region metadata in LDS (pointers into the workgroup's shared memory; ts and
// qoff live in the dynamic part, sized for the configured block and halo):
//   ts[r*(rw+1) + c]  LDS offset of region tile (r, c); c = rw is the row end,
//                     and ts[rh*(rw+1)] repeats the last row's end
//   row_gs[r]         global slot of the first hit of region row r
//   row_lo[r]         LDS offset of region row r (row_lo[rh] = total)
//   core_lo[r]        prefix of core-hit counts over core rows
//   qoff[q]           density: offsets of the merged 2x2-tile lists
struct RegionLds {
  int* ts;
  int* row_gs;
  int* row_lo;
  int* core_lo;
  int* qoff;
  int* qtotal;
};
constexpr int kRowMetaInts = kMaxRegionRows + 2 * (kMaxRegionRows + 1) + 1;

__device__ __forceinline__ RegionLds region_lds(int* row_meta, int* ts, int* qoff) {
  RegionLds L;
  L.ts = ts;
  L.row_gs = row_meta;
  L.row_lo = row_meta + kMaxRegionRows;
  L.core_lo = row_meta + 2 * kMaxRegionRows + 1;
  L.qtotal = row_meta + 3 * kMaxRegionRows + 2;
  L.qoff = qoff;
  return L;
}

__device__ __forceinline__ void item_block(const Geom& g, int item, int& unit, int& tx0, int& ty0, int& tx1,
                                           int& ty1) {
  unit = item / g.bpu;
  const int b = item - unit * g.bpu;
  const int bj = b / g.nbx;
  const int bi = b - bj * g.nbx;
  tx0 = bi * g.bx;
  ty0 = bj * g.by;
  tx1 = min(tx0 + g.bx, g.nx) - 1;
  ty1 = min(ty0 + g.by, g.ny) - 1;
}

__device__ __forceinline__ void make_region(const Geom& g, int unit, int tx0, int ty0, int tx1, int ty1, Region& R) {
  R.unit = unit;
  R.e = unit / g.L;
  R.rx0 = max(tx0 - g.halo, 0);
  R.ry0 = max(ty0 - g.halo, 0);
  const int rx1 = min(tx1 + g.halo, g.nx - 1), ry1 = min(ty1 + g.halo, g.ny - 1);
  R.rw = rx1 - R.rx0 + 1;
  R.rh = ry1 - R.ry0 + 1;
  R.cx0 = tx0 - R.rx0;
  R.cy0 = ty0 - R.ry0;
  R.cw = tx1 - tx0 + 1;
  R.ch = ty1 - ty0 + 1;
}

// Loads the region's tile offsets and builds the LDS layout. Starts and ends
// with a barrier; R.total and the core counts are then valid everywhere.
__device__ __forceinline__ void region_setup(const Geom& g, const Arena& a, Region& R, RegionLds& L) {
  __syncthreads();
  const int64_t ubase = (int64_t)R.unit * g.tpl;
  const int per_row = R.rw + 1;
  const int ntile = R.rh * per_row;
  for (int k = threadIdx.x; k < ntile; k += kWG) {
    const int r = k / per_row, c = k - r * per_row;
    L.ts[k] = a.tile_start[ubase + (int64_t)(R.ry0 + r) * g.nx + R.rx0 + c];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int r = threadIdx.x;
    const int len = r < R.rh ? L.ts[r * per_row + R.rw] - L.ts[r * per_row] : 0;
    const int incl = wave_incl_scan(len, r);
    if (r < R.rh) {
      L.row_gs[r] = L.ts[r * per_row];
      L.row_lo[r] = incl - len;
    }
    if (r == 63) L.row_lo[R.rh] = incl;
    const int cr = (R.cy0 + r) * per_row + R.cx0;
    const int clen = r < R.ch ? L.ts[cr + R.cw] - L.ts[cr] : 0;
    const int cincl = wave_incl_scan(clen, r);
    if (r < R.ch) L.core_lo[r] = cincl - clen;
    if (r == 63) L.core_lo[R.ch] = cincl;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ntile; k += kWG) {
    const int r = k / per_row;
    L.ts[k] = L.row_lo[r] + (L.ts[k] - L.row_gs[r]);
  }
  // one entry past the last row's end, equal to it: (ntile - 1, ntile) is an
  // empty tile that searches may read in place of a tile they do not need
  if (threadIdx.x == 0) L.ts[ntile] = L.row_lo[R.rh];
  __syncthreads();
  R.total = L.row_lo[R.rh];
}

// Core query q -> (region row, LDS position). `cr` is a core row at or
// before q's, and is left at q's: a lane walking its queries in increasing
// order keeps it between calls.
__device__ __forceinline__ void core_query(const RegionLds& L, const Region& R, int q, int& cr, int& row, int& p) {
  while (cr + 1 < R.ch && L.core_lo[cr + 1] <= q) ++cr;
  row = R.cy0 + cr;
  p = L.ts[row * (R.rw + 1) + R.cx0] + (q - L.core_lo[cr]);
}

__device__ __forceinline__ int slot_of(const RegionLds& L, int row, int p) { return L.row_gs[row] + (p - L.row_lo[row]); }

// Work-item scheduling. Items are (event, layer, tile block) triples in
// row-major block order, so consecutive items are spatially adjacent and
// share halo tiles. Plain launches take item = workgroup id: the dispatcher
// issues workgroups in order, so the items in flight stay adjacent.
// Persistent launches split the items into one contiguous run per XCD (each
// XCD has its own L2) and pop them from that XCD's queue head; an XCD whose
// run is exhausted steals from the others. The XCD comes from the hardware
// XCC_ID register.
__device__ __forceinline__ int xcc_id() {
  // s_getreg_b32 hwreg(HW_REG_XCC_ID = 20, offset 0, 4 bits)
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kQueues - 1);
}

__device__ __forceinline__ void queue_range(int n, int x, int& lo, int& cnt) {
  const int q = n / kQueues, r = n - q * kQueues;
  lo = x * q + min(x, r);
  cnt = q + (x < r ? 1 : 0);
}

struct ItemSched {
  int v;     // queues visited so far (persistent) / item taken (plain)
  int home;  // this workgroup's XCD
};

// Next work item, or -1 when none is left; uniform across the workgroup.
template <bool G>
__device__ __forceinline__ int next_item(ItemSched& st, int n_items, int* heads, int* s_item) {
  if constexpr (!G) {
    if (st.v++ > 0) return -1;
    return (int)blockIdx.x < n_items ? (int)blockIdx.x : -1;
  } else {
    while (st.v < kQueues) {  // own XCD's queue first, then steal
      const int x = (st.home + st.v) & (kQueues - 1);
      int lo, cnt;
      queue_range(n_items, x, lo, cnt);
      __syncthreads();
      if (threadIdx.x == 0) *s_item = atomicAdd(&heads[x * kCounterStride], 1);
      __syncthreads();
      const int k = *s_item;
      if (k < cnt) return lo + k;
      ++st.v;
    }
    return -1;
  }
}

// Query window [v - w', v + w'] in tile coordinates (w' from window_half).
struct Window {
  int x0, x1, y0, y1;
};
__device__ __forceinline__ Window query_window(const Geom& g, float w, float xi, float yi) {
  const float wx = window_half(w, xi), wy = window_half(w, yi);
  Window W;
  W.x0 = tile_coord(__fsub_rn(xi, wx), g.x0, g.inv_t, g.nx);
  W.x1 = tile_coord(__fadd_rn(xi, wx), g.x0, g.inv_t, g.nx);
  W.y0 = tile_coord(__fsub_rn(yi, wy), g.y0, g.inv_t, g.ny);
  W.y1 = tile_coord(__fadd_rn(yi, wy), g.y0, g.inv_t, g.ny);
  return W;
}

// ---------------------------------------------------------------------------
// Density (Eq. 3): rho_i = sum of E_j over same-layer j with d2 < dc2, added
// in ascending j. Tiles list their hits in ascending index; a query first marks
// the passing hits of each window tile in a 64-bit mask, then merges only the
// passing hits of the (at most MAXL x MAXL) sorted tile lists.
// Staged records: (x, y, E) and the hit index, laid out per instance (Staged).
// ---------------------------------------------------------------------------
// exp(x) for x <= 0 as one fixed binary32 evaluation, after Cody and Waite's
// range reduction: x = k ln2 + r with k = floor(x / ln2 + 1/2) and ln2 split
// into a high part with trailing zero bits (k * hi exact) and the remainder;
// exp(r) by its degree-7 Taylor polynomial in Horner form; then the scale by
// 2^k. Every step is an explicit binary32 rounding, so any IEEE evaluation of
// the same steps gives the same bits. 0 when k < -125.
__device__ __forceinline__ float exp32(float x) {
  constexpr float inv_ln2 = (float)(1.0 / 0.69314718055994530942);
  constexpr float ln2_hi = 0.693145751953125f;
  constexpr float ln2_lo = (float)(0.69314718055994530942 - 0.693145751953125);
  const float kf = floorf(__fadd_rn(__fmul_rn(x, inv_ln2), 0.5f));
  if (!(kf >= -125.0f)) return 0.0f;
  const float r = __fsub_rn(__fsub_rn(x, __fmul_rn(kf, ln2_hi)), __fmul_rn(kf, ln2_lo));
  float p = (float)(1.0 / 5040.0);
  p = __fadd_rn(__fmul_rn(p, r), (float)(1.0 / 720.0));
  p = __fadd_rn(__fmul_rn(p, r), (float)(1.0 / 120.0));
  p = __fadd_rn(__fmul_rn(p, r), (float)(1.0 / 24.0));
  p = __fadd_rn(__fmul_rn(p, r), (float)(1.0 / 6.0));
  p = __fadd_rn(__fmul_rn(p, r), 0.5f);
  p = __fadd_rn(__fmul_rn(p, r), 1.0f);
  p = __fadd_rn(__fmul_rn(p, r), 1.0f);
  return __fmul_rn(p, __uint_as_float((unsigned)((int)kf + 127) << 23));
}

// Correctly rounded binary32 square root of x >= 0: the hardware estimate
// (within an ulp) is corrected by comparing x with the squares of the
// midpoints to its neighbours, which are exact in binary64. Subnormal x is
// scaled by 2^64 first (exact, and exactly undone by 2^-32).
__device__ __forceinline__ float sqrt_rn(float x) {
  if (!(x > 0.0f) || x == __int_as_float(0x7f800000)) return x;
  const bool tiny = x < 1.17549435e-38f;
  const float xs = tiny ? __fmul_rn(x, 18446744073709551616.0f) : x;
  float s = __builtin_sqrtf(xs);
  const double xd = (double)xs;
  const float up = __uint_as_float(__float_as_uint(s) + 1u);
  const double mh = 0.5 * ((double)s + (double)up);
  if (mh * mh < xd) {
    s = up;
  } else {
    const float dn = __uint_as_float(__float_as_uint(s) - 1u);
    const double ml = 0.5 * ((double)dn + (double)s);
    if (ml * ml > xd) s = dn;
  }
  return tiny ? __fmul_rn(s, 2.3283064365386963e-10f) : s;
}

// One term of Eq. 3 for a neighbour at squared distance d2 with energy e:
// e (flat kernel), fl(exp(-fl(d2 a)) e) (Gaussian, a = 1 / (2 s^2)) or
// fl(exp(-fl(sqrt(d2) a)) e) (exponential, a = 1 / s).
template <int K>
__device__ __forceinline__ float kernel_term(float d2, float ka, float e) {
  if constexpr (K == 0) {
    return e;
  } else if constexpr (K == 1) {
    return __fmul_rn(exp32(-__fmul_rn(d2, ka)), e);
  } else {
    return __fmul_rn(exp32(-__fmul_rn(sqrt_rn(d2), ka)), e);
  }
}

// A staged record's position and energy.
struct Rec3 {
  float x, y, e;
};

// Staged density records, 16 bytes per hit in both layouts:
// * the two-tile instance keeps 12-byte records (x, y, E) with the hit
//   indices (the sort keys) in an array of their own, so that the records one
//   wave reads at once, and the keys the quad-list build probes, spread over
//   more LDS banks than 16-byte records would;
// * the three-tile instance keeps 16-byte records (x, y, E, hit index), whose
//   mask loop reads the (x, y) of two records in one 64-bit pair load.
template <int MAXL>
struct Staged {
  static constexpr bool kSplit = MAXL == 2;
  static constexpr int kRecBytes = kSplit ? 12 : 16;
  static constexpr int kKeyShift = kSplit ? 2 : 4;  // log2 of the LDS stride between keys
  unsigned char* base;
  int cap;
  __device__ __forceinline__ const float* rec(int j) const {
    return reinterpret_cast<const float*>(base + kRecBytes * j);
  }
  __device__ __forceinline__ float2 xy(int j) const {
    if constexpr (kSplit) {
      const float* r = rec(j);
      return make_float2(r[0], r[1]);
    } else {
      return *reinterpret_cast<const float2*>(rec(j));
    }
  }
  __device__ __forceinline__ const int* key_ptr(int j) const {
    if constexpr (kSplit) return reinterpret_cast<const int*>(base + 12 * cap) + j;
    else return reinterpret_cast<const int*>(base + 16 * j + 12);
  }
  __device__ __forceinline__ int key(int j) const { return *key_ptr(j); }
  __device__ __forceinline__ void put(int j, float x, float y, float en, int h) const {
    if constexpr (kSplit) {
      *reinterpret_cast<Rec3*>(base + 12 * j) = Rec3{x, y, en};
      *const_cast<int*>(key_ptr(j)) = h;
    } else {
      *reinterpret_cast<float4*>(base + 16 * j) = make_float4(x, y, en, __int_as_float(h));
    }
  }
  // The record at a quad-list entry (its byte offset). As one three- or
  // four-float vector; at the density kernel's occupancy bound the compiler
  // issues the split layout's as a two-word and a one-word LDS load from the
  // same address.
  __device__ __forceinline__ Rec3 at(int byte_off) const {
    if constexpr (kSplit) {
      typedef float Float3 __attribute__((ext_vector_type(3)));
      typedef Float3 Float3A4 __attribute__((aligned(4)));
      const Float3 v = *reinterpret_cast<const Float3A4*>(base + byte_off);
      return Rec3{v.x, v.y, v.z};
    } else {
      const float4 v = *reinterpret_cast<const float4*>(base + byte_off);
      return Rec3{v.x, v.y, v.z};
    }
  }
};

// Energy and hit index of a staged record, for both layouts (a 16-byte
// record carries its index in the fourth word; a 12-byte record's index is in
// the array beside the records).
__device__ __forceinline__ float rec_e(const float4& r) { return r.z; }
__device__ __forceinline__ float rec_e(const Rec3& r) { return r.e; }
__device__ __forceinline__ int rec_key(const float4* rec, const int*, int j) { return __float_as_int(rec[j].w); }
__device__ __forceinline__ int rec_key(const Rec3*, const int* keys, int j) { return keys[j]; }

template <int MAXL, int K, typename T>
__device__ __forceinline__ float density_merge_full(const T* __restrict__ rec, const int* __restrict__ keys, const int* lo,
                                                   const int* hi, float xi, float yi, float dc2, float ka) {
  constexpr int NL = MAXL * MAXL;
  int cur[NL], head[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    cur[k] = lo[k];
    head[k] = cur[k] < hi[k] ? rec_key(rec, keys, cur[k]) : INT_MAX;
  }
  float acc = 0.0f;
  for (;;) {
    int m = head[0];
#pragma unroll
    for (int k = 1; k < NL; ++k) m = min(m, head[k]);
    if (m == INT_MAX) break;
    int p = 0;
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (head[k] == m) p = cur[k];
    const T r = rec[p];
    const float d2 = dist2(xi, yi, r.x, r.y);
    if (d2 < dc2) acc = __fadd_rn(acc, kernel_term<K>(d2, ka, rec_e(r)));
    const int np = p + 1;
    int nh = INT_MAX;
    bool more = false;
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (head[k] == m) more = np < hi[k];
    if (more) nh = rec_key(rec, keys, np);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      if (head[k] == m) {
        cur[k] = np;
        head[k] = nh;
      }
    }
  }
  return acc;
}

// Lowest set bit of a 64-bit mask kept as two 32-bit halves.
__device__ __forceinline__ int lowbit64(unsigned lo, unsigned hi) {
  return lo ? __builtin_ctz(lo) : 32 + __builtin_ctz(hi);
}

template <int MAXL, int K, typename T>
__device__ __forceinline__ float density_two_pass(const T* __restrict__ rec, const int* __restrict__ keys, const int* lo,
                                                  const int* hi, float xi, float yi, float dc2, float ka) {
  constexpr int NL = MAXL * MAXL;
  unsigned mlo[NL], mhi[NL];
  bool big = false;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    mlo[k] = 0u;
    mhi[k] = 0u;
    const int len = hi[k] - lo[k];
    big |= len > 64;
    const T* base = rec + lo[k];
    const int n0 = min(len, 32);
    int c = 0;
    for (; c + 3 < n0; c += 4) {
      const float2 q0 = *reinterpret_cast<const float2*>(base + c);
      const float2 q1 = *reinterpret_cast<const float2*>(base + c + 1);
      const float2 q2 = *reinterpret_cast<const float2*>(base + c + 2);
      const float2 q3 = *reinterpret_cast<const float2*>(base + c + 3);
      const unsigned m4 = (dist2(xi, yi, q0.x, q0.y) < dc2 ? 1u : 0u) | (dist2(xi, yi, q1.x, q1.y) < dc2 ? 2u : 0u) |
                          (dist2(xi, yi, q2.x, q2.y) < dc2 ? 4u : 0u) | (dist2(xi, yi, q3.x, q3.y) < dc2 ? 8u : 0u);
      mlo[k] |= m4 << c;
    }
    for (; c < n0; ++c) {
      const float2 q = *reinterpret_cast<const float2*>(base + c);
      mlo[k] |= (dist2(xi, yi, q.x, q.y) < dc2 ? 1u : 0u) << c;
    }
    const int n1 = min(len, 64);
#pragma unroll 4
    for (int c = 32; c < n1; ++c) {
      const float2 q = *reinterpret_cast<const float2*>(base + c);
      mhi[k] |= (dist2(xi, yi, q.x, q.y) < dc2 ? 1u : 0u) << (c - 32);
    }
  }
  if (big) return density_merge_full<MAXL, K>(rec, keys, lo, hi, xi, yi, dc2, ka);
  // heads of the lists; with the flat kernel the head's energy is kept,
  // otherwise the selected head is re-read from LDS when it is added
  int hh[NL];
  float ee[K == 0 ? NL : 1];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    hh[k] = INT_MAX;
    if constexpr (K == 0) ee[k] = 0.0f;
    if (mlo[k] | mhi[k]) {
      const int j = lo[k] + lowbit64(mlo[k], mhi[k]);
      hh[k] = rec_key(rec, keys, j);
      if constexpr (K == 0) ee[k] = rec_e(rec[j]);
    }
  }
  float acc = 0.0f;
  for (;;) {
    int m = hh[0];
#pragma unroll
    for (int k = 1; k < NL; ++k) m = min(m, hh[k]);
    if (m == INT_MAX) break;
    // the selected list: take its head, drop its lowest passing bit
    float e = 0.0f;
    if constexpr (K == 0) e = ee[0];
    unsigned ml = mlo[0], mh = mhi[0];
    int base = lo[0];
#pragma unroll
    for (int k = 1; k < NL; ++k) {
      if (hh[k] == m) {
        if constexpr (K == 0) e = ee[k];
        ml = mlo[k];
        mh = mhi[k];
        base = lo[k];
      }
    }
    if constexpr (K == 0) {
      acc = __fadd_rn(acc, e);
    } else {
      const T rs = rec[base + lowbit64(ml, mh)];
      acc = __fadd_rn(acc, kernel_term<K>(dist2(xi, yi, rs.x, rs.y), ka, rec_e(rs)));
    }
    if (ml)
      ml &= ml - 1u;
    else
      mh &= mh - 1u;
    const bool more = (ml | mh) != 0u;
    int nk = INT_MAX;
    float ne = 0.0f;
    if (more) {
      const int j = base + lowbit64(ml, mh);
      nk = rec_key(rec, keys, j);
      ne = rec_e(rec[j]);
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      if (hh[k] == m) {
        mlo[k] = ml;
        mhi[k] = mh;
        hh[k] = nk;
        if constexpr (K == 0) ee[k] = ne;
      }
    }
  }
  return acc;
}

// Global-memory density (tiles too dense to stage): the window's tile lists,
// each in ascending hit index in the CSR, are merged on the fly (cursors and
// head indices in registers), so each query passes over its window once.
template <int K>
__device__ __forceinline__ float density_global(const Geom& g, const Arena& a, int64_t ubase, float xi, float yi) {
  const Window W = query_window(g, g.win_dc, xi, yi);
  constexpr int NL = 9;  // the density window spans at most 3 x 3 tiles
  int cur[NL], end[NL], head[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int ty = W.y0 + k / 3, tx = W.x0 + k % 3;
    cur[k] = end[k] = 0;
    if (ty <= W.y1 && tx <= W.x1) {
      const int64_t t = ubase + (int64_t)ty * g.nx + tx;
      cur[k] = a.tile_start[t];
      end[k] = a.tile_start[t + 1];
    }
    head[k] = cur[k] < end[k] ? a.hs[cur[k]] : INT_MAX;
  }
  float acc = 0.0f;
  for (;;) {
    int m = head[0];
#pragma unroll
    for (int k = 1; k < NL; ++k) m = min(m, head[k]);
    if (m == INT_MAX) break;
    int s = 0;
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (head[k] == m) s = cur[k];
    const float d2 = dist2(xi, yi, a.xs[s], a.ys[s]);
    if (d2 < g.dc2) acc = __fadd_rn(acc, kernel_term<K>(d2, g.ka, a.es[s]));
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      if (head[k] == m) {
        ++cur[k];
        head[k] = cur[k] < end[k] ? a.hs[cur[k]] : INT_MAX;
      }
    }
  }
  return acc;
}

// Quad-list entries are byte offsets of records (a staged position times the
// record size, below 2^15 for every LDS cap), so a scan adds no index scaling.
static_assert(kMaxLdsCap * 16 <= 65536, "quad-list byte offsets are 16-bit");
// Byte address of a shared-memory object in the workgroup's LDS, and a load
// from such an address: loops that step through LDS by byte address then need
// no base register added per access.
__device__ __forceinline__ unsigned lds_address(const void* p) {
  return (unsigned)(size_t)(const __attribute__((address_space(3))) void*)p;
}
__device__ __forceinline__ int lds_load_int(unsigned addr) {
  return *(const __attribute__((address_space(3))) int*)(size_t)addr;
}
static_assert(kMaxRegionRows <= 64 && kMaxRegionTiles <= 1024, "a staged tile id is (row << 10) | column in 16 bits");

// Density over a staged region (records x, y, E and their hit indices; each
// tile in ascending hit index). With MAXL == 2 every query window lies inside the
// 2x2 tile quad anchored at its lower-left window tile; the quads a core
// query can use are merged once per region into index-ordered lists (byte
// offsets of the records), so each query is one linear scan in ascending
// hit index. Otherwise (or if the quads do not fit) a query merges its
// window's tile lists itself.
template <int MAXL, int K>
__device__ __forceinline__ void density_staged(const Geom& g, const Arena& a, const Region& R, RegionLds& L,
                                               const Staged<MAXL>& S, unsigned short* stile, unsigned short* qidx,
                                               unsigned short sent, bool keep) {
  const int per_row = R.rw + 1;
  const int64_t ubase = (int64_t)R.unit * g.tpl;
  const int ntl = R.rh * per_row;
  // region tile of every staged position as (row << 10) | column (rows
  // < 64, columns < 1024), two lanes per tile
  for (int k = threadIdx.x; k < 2 * ntl; k += kWG) {
    const int tl = k >> 1;
    const int tr = tl / per_row, tc = tl - tr * per_row;
    if (tc == R.rw) continue;  // row-end entry
    const unsigned short code = (unsigned short)((tr << 10) | tc);
    const int end = L.ts[tl + 1];
    for (int p = L.ts[tl] + (k & 1); p < end; p += 2) stile[p] = code;
  }
  __syncthreads();
  // copy the records (tiles are already in ascending hit index); every
  // global load of a lane is issued before its first LDS store
  for (int base = 0; base < R.total; base += kStagePer * kWG) {
    Rec3 v[kStagePer];
    int h[kStagePer];
#pragma unroll
    for (int k = 0; k < kStagePer; ++k) {
      const int p = base + (int)threadIdx.x + k * kWG;
      if (p < R.total) {
        const int sl = slot_of(L, stile[p] >> 10, p);
        v[k] = Rec3{a.xs[sl], a.ys[sl], a.es[sl]};
        h[k] = a.hs[sl];
      }
    }
#pragma unroll
    for (int k = 0; k < kStagePer; ++k) {
      const int p = base + (int)threadIdx.x + k * kWG;
      if (p < R.total) S.put(p, v[k].x, v[k].y, v[k].e, h[k]);
    }
  }
  // quads anchored at region tiles [qx0, qx1] x [qy0, qy1]
  const int qx0 = max(R.cx0 - 1, 0), qx1 = min(R.cx0 + R.cw - 1, R.rw - 1);
  const int qy0 = max(R.cy0 - 1, 0), qy1 = min(R.cy0 + R.ch - 1, R.rh - 1);
  const int qw = qx1 - qx0 + 1;
  const int nquad = qw * (qy1 - qy0 + 1);
  bool use_quads = MAXL == 2 && g.density_quads && nquad < g.q_ints;
  if (use_quads) {
    if (threadIdx.x < 64) {
      // quad sizes -> offsets, 64 quads per wave step. Each list is padded
      // with the sentinel to a multiple of four entries, so the queries read
      // their lists four entries at a time with no remainder loop (pads past
      // the array are not written: the quads are then not used).
      int run = 0;
      for (int q0 = 0; q0 < nquad; q0 += 64) {
        const int q = q0 + (int)threadIdx.x;
        int len = 0;
        if (q < nquad) {
          const int ax = qx0 + q % qw, ay = qy0 + q / qw;
          const int bx1 = min(ax + 1, R.rw - 1), by1 = min(ay + 1, R.rh - 1);
          for (int ty = ay; ty <= by1; ++ty) len += L.ts[ty * per_row + bx1 + 1] - L.ts[ty * per_row + ax];
        }
        const int plen = (len + 3) & ~3;
        const int incl = wave_incl_scan(plen, threadIdx.x);
        if (q < nquad) {
          const int o = run + incl - plen;
          L.qoff[q] = o;
          for (int i = o + len; i < o + plen && i < 4 * g.lds_cap; ++i) qidx[i] = sent;
        }
        run += __builtin_amdgcn_readlane(incl, 63);
      }
      if (threadIdx.x == 0) {
        L.qoff[nquad] = run;
        *L.qtotal = run;
      }
    }
  }
  __syncthreads();
  if (use_quads && *L.qtotal <= 4 * g.lds_cap && g.density_quads == 2) {
    // one lane per quad: a sequential merge of its (up to four) index-sorted
    // tile lists
    for (int q = threadIdx.x; q < nquad; q += kWG) {
      const int ax = qx0 + q % qw, ay = qy0 + q / qw;
      const int bx1 = min(ax + 1, R.rw - 1), by1 = min(ay + 1, R.rh - 1);
      int cur[4], end[4], key[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int tx = (k & 1) ? bx1 : ax, ty = (k & 2) ? by1 : ay;
        const bool dup = ((k & 1) && bx1 == ax) || ((k & 2) && by1 == ay);
        const int t = ty * per_row + tx;
        cur[k] = dup ? 0 : L.ts[t];
        end[k] = dup ? 0 : L.ts[t + 1];
        key[k] = cur[k] < end[k] ? S.key(cur[k]) : INT_MAX;
      }
      const int out = L.qoff[q], n = (end[0] - cur[0]) + (end[1] - cur[1]) + (end[2] - cur[2]) + (end[3] - cur[3]);
      for (int i = 0; i < n; ++i) {
        const int m = min(min(key[0], key[1]), min(key[2], key[3]));
        const bool s0 = key[0] == m, s1 = !s0 && key[1] == m, s2 = !s0 && !s1 && key[2] == m;
        const int pk = s0 ? cur[0] : (s1 ? cur[1] : (s2 ? cur[2] : cur[3]));
        const int ek = s0 ? end[0] : (s1 ? end[1] : (s2 ? end[2] : end[3]));
        qidx[out + i] = (unsigned short)(pk * S.kRecBytes);
        const int np = pk + 1;
        const int nk = np < ek ? S.key(np) : INT_MAX;
        const bool s3 = !s0 && !s1 && !s2;
        cur[0] = s0 ? np : cur[0];
        key[0] = s0 ? nk : key[0];
        cur[1] = s1 ? np : cur[1];
        key[1] = s1 ? nk : key[1];
        cur[2] = s2 ? np : cur[2];
        key[2] = s2 ? nk : key[2];
        cur[3] = s3 ? np : cur[3];
        key[3] = s3 ? nk : key[3];
      }
    }
    __syncthreads();
  } else if (use_quads && *L.qtotal <= 4 * g.lds_cap) {
    // place every sorted record into each quad that holds its tile: its
    // position there is its rank in its own tile plus, for each other tile
    // of the quad, the entries with a smaller hit index (each of the up to
    // eight neighbour tiles is counted once and shared by the quads)
    for (int p = threadIdx.x; p < R.total; p += kWG) {
      const int tr = stile[p] >> 10, tc = stile[p] & 1023;
      const int tl = tr * per_row + tc;
      const int hp = S.key(p);
      const int own = p - L.ts[tl];
      bool qv[2][2];
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const int ax = tc - dx, ay = tr - dy;
          qv[dy][dx] = ax >= qx0 && ax <= qx1 && ay >= qy0 && ay <= qy1;
        }
      // lower bounds in the needed neighbour tiles. The tile offsets are read
      // without a branch: a neighbour that is not needed (or lies outside the
      // region) reads the empty pair after the last row's end.
      const int rm = max(tr - 1, 0) * per_row, r0 = tl - tc, rp = min(tr + 1, R.rh - 1) * per_row;
      const int cm = max(tc - 1, 0), cp = min(tc + 1, R.rw - 1);
      const int empty = R.rh * per_row - 1;
      int lo[9], len[9];
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
          const int k = (oy + 1) * 3 + ox + 1;
          lo[k] = 0;
          len[k] = 0;
          if (k == 4) continue;  // the hit's own tile
          bool need = false;
#pragma unroll
          for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx)
              need |= qv[dy][dx] && (ox == -dx || ox == 1 - dx) && (oy == -dy || oy == 1 - dy);
          const int nx = tc + ox, ny = tr + oy;
          need &= nx >= 0 && nx < R.rw && ny >= 0 && ny < R.rh;
          const int nt = need ? (oy < 0 ? rm : oy > 0 ? rp : r0) + (ox < 0 ? cm : ox > 0 ? cp : tc) : empty;
          lo[k] = L.ts[nt];
          len[k] = L.ts[nt + 1] - lo[k];
        }
      // The searches share one power-of-two step sequence, from the largest
      // of the tiles down to one record. Each holds the LDS address of its
      // last counted key (at first, the key before its tile); a step probes
      // the key `step` records further on, clamped to the tile's last key. A
      // clamped probe is taken only when every key of the tile is smaller,
      // which is then the count. So no search branches, and all loads of a
      // step are issued before its compares. An empty tile starts and ends
      // at record 0's key, so every probe reads a staged key.
      int maxlen = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) maxlen = max(maxlen, len[k]);
      constexpr int ks = Staged<MAXL>::kKeyShift;
      const unsigned key0 = lds_address(S.key_ptr(0));  // LDS address of record 0's key
      unsigned at[9], end[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        at[k] = len[k] > 0 ? key0 + (((unsigned)lo[k] - 1u) << ks) : key0;
        end[k] = at[k] + ((unsigned)len[k] << ks);
      }
      // per quad, the sum of its three searches' starting addresses
      unsigned start3[2][2];
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          start3[dy][dx] = 0u;
#pragma unroll
          for (int oy = -dy; oy <= 1 - dy; ++oy)
#pragma unroll
            for (int ox = -dx; ox <= 1 - dx; ++ox)
              if (ox != 0 || oy != 0) start3[dy][dx] += at[(oy + 1) * 3 + ox + 1];
        }
      // at least one step (one key): with every tile empty it changes nothing
      unsigned step = (1u << ks) << max(31 - __clz(maxlen), 0);
      do {
        unsigned pr[9];
        int kv[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          if (k == 4) continue;
          pr[k] = min(at[k] + step, end[k]);
          kv[k] = lds_load_int(pr[k]);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k)
          if (k != 4) at[k] = kv[k] < hp ? pr[k] : at[k];
        step >>= 1;
      } while (step >= (1u << ks));
      // each quad: the own rank plus the three neighbour counts (one key
      // stride of address per counted key)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          if (!qv[dy][dx]) continue;
          unsigned below = 0u - start3[dy][dx];
#pragma unroll
          for (int oy = -dy; oy <= 1 - dy; ++oy)
#pragma unroll
            for (int ox = -dx; ox <= 1 - dx; ++ox)
              if (ox != 0 || oy != 0) below += at[(oy + 1) * 3 + ox + 1];
          qidx[L.qoff[(tr - dy - qy0) * qw + (tc - dx - qx0)] + own + (int)(below >> ks)] =
              (unsigned short)(p * S.kRecBytes);
        }
    }
    __syncthreads();
  } else {
    use_quads = false;
  }
  const int nq = L.core_lo[R.ch];
  int cr = 0;
  for (int q = threadIdx.x; q < nq; q += kWG) {
    int row, p;
    core_query(L, R, q, cr, row, p);
    const int slot = slot_of(L, row, p);
    const float2 me = S.xy(p);
    const float xi = me.x, yi = me.y;
    const Window W = query_window(g, g.win_dc, xi, yi);
    const int tx0 = W.x0 - R.rx0, tx1 = W.x1 - R.rx0, ty0 = W.y0 - R.ry0, ty1 = W.y1 - R.ry0;
    const bool ok = tx0 >= 0 && ty0 >= 0 && tx1 < R.rw && ty1 < R.rh && tx1 - tx0 < MAXL && ty1 - ty0 < MAXL;
    float rho = 0.0f;
    if (ok && use_quads) {
      const int qq = (ty0 - qy0) * qw + (tx0 - qx0);
      const unsigned short* qp = qidx + L.qoff[qq];
      const unsigned short* const qe = qidx + L.qoff[qq + 1];
      // four entries at a time (the lists are padded to a multiple of four);
      // additions stay in ascending index order
      for (; qp < qe; qp += 4) {
        const int i0 = qp[0], i1 = qp[1], i2 = qp[2], i3 = qp[3];
        const Rec3 r0 = S.at(i0), r1 = S.at(i1), r2 = S.at(i2), r3 = S.at(i3);
        const float d0 = dist2(xi, yi, r0.x, r0.y), d1 = dist2(xi, yi, r1.x, r1.y);
        const float d2 = dist2(xi, yi, r2.x, r2.y), d3 = dist2(xi, yi, r3.x, r3.y);
        const float a0 = __fadd_rn(rho, kernel_term<K>(d0, g.ka, r0.e));
        rho = d0 < g.dc2 ? a0 : rho;
        const float a1 = __fadd_rn(rho, kernel_term<K>(d1, g.ka, r1.e));
        rho = d1 < g.dc2 ? a1 : rho;
        const float a2 = __fadd_rn(rho, kernel_term<K>(d2, g.ka, r2.e));
        rho = d2 < g.dc2 ? a2 : rho;
        const float a3 = __fadd_rn(rho, kernel_term<K>(d3, g.ka, r3.e));
        rho = d3 < g.dc2 ? a3 : rho;
      }
    } else if (ok) {
      int lo[MAXL * MAXL], hi[MAXL * MAXL];
#pragma unroll
      for (int jy = 0; jy < MAXL; ++jy)
#pragma unroll
        for (int jx = 0; jx < MAXL; ++jx) {
          const int k = jy * MAXL + jx;
          const int ty = ty0 + jy, tx = tx0 + jx;
          if (ty <= ty1 && tx <= tx1) {
            lo[k] = L.ts[ty * per_row + tx];
            hi[k] = L.ts[ty * per_row + tx + 1];
          } else {
            lo[k] = 0;
            hi[k] = 0;
          }
        }
      if constexpr (Staged<MAXL>::kSplit)
        rho = density_two_pass<MAXL, K>(reinterpret_cast<const Rec3*>(S.base), S.key_ptr(0), lo, hi, xi, yi, g.dc2, g.ka);
      else
        rho = density_two_pass<MAXL, K>(reinterpret_cast<const float4*>(S.base), nullptr, lo, hi, xi, yi, g.dc2, g.ka);
    } else {
      atomicOr(a.err, (uint32_t)E_WINDOW);
      rho = density_global<K>(g, a, ubase, xi, yi);
    }
    a.rho[slot] = rho;
    if (keep) a.rho_out[S.key(p)] = rho;
  }
}

// Regions whose tiles are too dense for LDS are not searched by the workgroup
// that meets them: their core queries are queued, tile by tile in chunks of
// `per` consecutive slots (the tile and the chunk's first slot, in the key and
// rank buffers, which are free after the grid build), and a spill kernel after
// the stage spreads the chunks over every workgroup of the GPU. Each tile is a
// core tile of one region, and a chunk holds at least one hit, so there are at
// most n chunks.
__device__ __forceinline__ void spill_region(const Geom& g, const Arena& a, const Region& R, int counter, int per) {
  const int64_t ubase = (int64_t)R.unit * g.tpl;
  for (int k = threadIdx.x; k < R.cw * R.ch; k += kWG) {
    const int cy = k / R.cw, cx = k - cy * R.cw;
    const int64_t t = ubase + (int64_t)(R.ry0 + R.cy0 + cy) * g.nx + R.rx0 + R.cx0 + cx;
    const int s0 = a.tile_start[t], s1 = a.tile_start[t + 1];
    const int nch = (s1 - s0 + per - 1) / per;
    if (nch == 0) continue;
    const int i0 = atomicAdd(&a.counters[counter], nch);
    for (int c = 0; c < nch; ++c) {
      a.key[i0 + c] = (int)t;
      a.rank[i0 + c] = s0 + c * per;
    }
  }
}

// Density of the spilled queries, one lane per query, from global memory.
template <bool G, int K>
__global__ __launch_bounds__(kWG) void k_density_spill(DescArg<G> dg, Geom g, Arena a) {
  const int nch = a.counters[C_SPILL_RHO];
  const bool keep = g.flags & 2u;
  for (int i = blockIdx.x; i < nch; i += gridDim.x) {
    const int64_t t = a.key[i];
    const int slot = a.rank[i] + (int)threadIdx.x;
    if (slot >= a.tile_start[t + 1]) continue;
    const float rho = density_global<K>(g, a, t - t % g.tpl, a.xs[slot], a.ys[slot]);
    a.rho[slot] = rho;
    if (keep) a.rho_out[a.hs[slot]] = rho;
  }
}

// The flat-kernel quad path is built for seven waves per SIMD (72 VGPRs), so
// that an LDS cap of up to 768 staged hits fits seven workgroups per CU; the
// compiler then keeps one item-level value in scratch, reloaded once per work
// item. The other instances keep their registers (they would spill in loops).
constexpr int density_min_waves(int maxl, int k) { return maxl == 2 && k == 0 ? 7 : 1; }

template <bool G, int MAXL, int K>
__global__ __launch_bounds__(kWG, density_min_waves(MAXL, K)) void k_density(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_rows[kRowMetaInts];
  __shared__ int s_item;
  const Staged<MAXL> S{smem, g.lds_cap};
  unsigned short* stile = reinterpret_cast<unsigned short*>(smem + 16 * g.lds_cap);  // both layouts: 16 B per hit
  unsigned short* qidx = reinterpret_cast<unsigned short*>(smem + density_qidx_offset(g.lds_cap));
  // the record every quad list is padded with, to a multiple of four entries:
  // x = +inf puts it at an infinite squared distance from every query
  const unsigned short sent = (unsigned short)density_sentinel_offset(g.lds_cap);
  if (threadIdx.x == 0)
    *reinterpret_cast<float4*>(smem + sent) = make_float4(__int_as_float(0x7f800000), 0.0f, 0.0f, 0.0f);
  int* meta = reinterpret_cast<int*>(smem + lds_records_density(g.lds_cap));
  RegionLds L = region_lds(s_rows, meta, meta + g.ts_ints);
  const int n_items = d.n_events * g.L * g.bpu;
  const bool keep = g.flags & 2u;
  ItemSched st{0, G ? xcc_id() : 0};
  for (int item; (item = next_item<G>(st, n_items, &a.counters[C_QUEUE_RHO], &s_item)) >= 0;) {
    int unit, tx0, ty0, tx1, ty1;
    item_block(g, item, unit, tx0, ty0, tx1, ty1);
    Region R;
    make_region(g, unit, tx0, ty0, tx1, ty1, R);
    region_setup(g, a, R, L);
    if (L.core_lo[R.ch] == 0) continue;
    if (R.total <= g.lds_cap) {
      density_staged<MAXL, K>(g, a, R, L, S, stile, qidx, sent, keep);
      continue;
    }
    // too dense: the four quarter blocks, then single tiles
    const int hx = (tx1 - tx0 + 2) >> 1, hy = (ty1 - ty0 + 2) >> 1;
    for (int sy = ty0; sy <= ty1; sy += hy)
      for (int sx = tx0; sx <= tx1; sx += hx) {
        const int ex = min(sx + hx - 1, tx1), ey = min(sy + hy - 1, ty1);
        make_region(g, unit, sx, sy, ex, ey, R);
        region_setup(g, a, R, L);
        if (L.core_lo[R.ch] == 0) continue;
        if (R.total <= g.lds_cap) {
          density_staged<MAXL, K>(g, a, R, L, S, stile, qidx, sent, keep);
          continue;
        }
        for (int ty = sy; ty <= ey; ++ty)
          for (int tx = sx; tx <= ex; ++tx) {
            make_region(g, unit, tx, ty, tx, ty, R);
            region_setup(g, a, R, L);
            if (L.core_lo[R.ch] == 0) continue;
            if (R.total <= g.lds_cap)
              density_staged<MAXL, K>(g, a, R, L, S, stile, qidx, sent, keep);
            else
              spill_region(g, a, R, C_SPILL_RHO, kWG);
          }
      }
  }
}

// ---------------------------------------------------------------------------
// Nearest-higher (Eq. 4) and the decision (Sec. 2.2, Algorithm 3).
// Phase 1 searches a small window of radius r1 <= d_m; when its best
// higher hit lies strictly within r1, no hit outside that window can be
// closer, so the query is done. Other queries are queued in LDS and searched
// over the full d_m window with `tpq` lanes each (phase 2).
// Records: (x, y, hit index as bits, ord(rho)); the last two halves form
// the 64-bit (ord(rho), index) key in register order.
// ---------------------------------------------------------------------------
// Order-preserving map of a float to uint32 (-0 folds onto +0), so that
// (rho, index) compares as one 64-bit unsigned key.
__device__ __forceinline__ unsigned ord_f32(float v) {
  const unsigned u = __float_as_uint(__fadd_rn(v, 0.0f));
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
// Inverse of ord_f32 (gives +0 for a folded -0, which compares the same).
__device__ __forceinline__ float ord_inv(unsigned o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}
__device__ __forceinline__ unsigned long long key64(unsigned hi, unsigned lo) {
  return ((unsigned long long)hi << 32) | lo;
}

struct NhBest {
  unsigned long long k;  // (d2 bits, caller index) of the best so far
  int p;                 // LDS position >= 0, or global slot s encoded as -2 - s; -1 none
  __device__ __forceinline__ float d2() const { return __uint_as_float((unsigned)(k >> 32)); }
  __device__ __forceinline__ int h() const { return (int)(unsigned)(k & 0xffffffffu); }
};

// Search state before any candidate, for the squared radius thr: the key
// (thr, 0) is beaten exactly by the keys (d2, index) with d2 < thr, so the
// radius test needs no comparison of its own.
__device__ __forceinline__ NhBest nh_start(float thr) { return NhBest{key64(__float_as_uint(thr), 0u), -1}; }

// One candidate j for query i: eligible when j is higher (ord/index keys);
// keeps the lexicographic minimum of (d2, index), which starts at
// nh_start(thr), and the candidate's position pq. d2 >= 0, so its bit
// pattern orders like its value.
template <bool STRICT>
__device__ __forceinline__ void nh_consider(NhBest& b, float d2, unsigned ordj, unsigned hj, int pq, unsigned ordi,
                                            unsigned hi) {
  const bool higher = STRICT ? ordj > ordi : key64(ordj, hj) > key64(ordi, hi);
  const unsigned long long ck = key64(__float_as_uint(d2), hj);
  const bool take = higher & (ck < b.k);  // branch-free select
  b.k = take ? ck : b.k;
  b.p = take ? pq : b.p;
}

// Staged records carry, in place of the caller index, the word
// (event-local index << kPosBits) | LDS position. Within one event it orders
// like the caller index, so the (rho, index) and (d2, index) keys compare as
// before, and the winner's LDS position comes back out of its key: the scan
// tracks no position of its own.
constexpr int kPosBits = 11;
constexpr unsigned kPosMask = (1u << kPosBits) - 1u;
constexpr int kPackedEventMax = 1 << (32 - kPosBits);  // hits per event
static_assert(kMaxLdsCap <= (1 << kPosBits), "an LDS position must fit the packed index word");
__device__ __forceinline__ unsigned nh_pack(int h, int ev_first, int p) {
  return ((unsigned)(h - ev_first) << kPosBits) | (unsigned)p;
}
__device__ __forceinline__ int nh_unpack_h(unsigned z, int ev_first) { return ev_first + (int)(z >> kPosBits); }
// After a staged scan from key k0: a found winner gets its LDS position in
// b.p and its caller index back in the key's low word.
__device__ __forceinline__ void nh_unpack(NhBest& b, unsigned long long k0, int ev_first) {
  if (b.p == -1 && b.k < k0) {
    const unsigned z = (unsigned)(b.k & 0xffffffffu);
    b.p = (int)(z & kPosMask);
    b.k = key64((unsigned)(b.k >> 32), (unsigned)nh_unpack_h(z, ev_first));
  }
}

__device__ __forceinline__ void nh_reduce(NhBest& b, int tpq) {
  for (int o = 1; o < tpq; o <<= 1) {
    const unsigned long long ok = __shfl_xor(b.k, o, 64);
    const int op = __shfl_xor(b.p, o, 64);
    if (ok < b.k) {
      b.k = ok;
      b.p = op;
    }
  }
}

// Writes the decision for the hit in `slot` with nearest-higher `b` (b.p
// already converted to a slot index, or -1).
__device__ __forceinline__ void decide_and_store(const Geom& g, const Arena& a, const RunDesc& d, int slot, int hi,
                                                 float ri, const NhBest& b, int ev_first) {
  const bool has = b.p >= 0;
  const float d2 = has ? b.d2() : __int_as_float(0x7f800000);
  const bool seed = ri > g.rho_c && d2 > g.dcs2;
  const bool outlier = ri < g.rho_c && d2 > g.do2;
  const bool follower = !seed && !outlier && has;
  a.parent[slot] = follower ? b.p : slot;
  a.flags[slot] = (uint8_t)((seed ? F_SEED : 0) | (outlier ? F_OUTLIER : 0) | (follower ? F_FOLLOWER : 0));
  if (seed) atomicOr(&a.seedbits[hi >> 5], 1u << (hi & 31));
  if (follower && builds_lists(g)) a.frank[slot] = atomicAdd(&a.fstart[b.h()], 1);
  if (g.flags & 2u) {
    a.nh_out[hi] = has ? b.h() - ev_first : -1;
    a.d2_out[hi] = d2;
  }
}

// One staged record r for query i, as nh_consider but tracking no position:
// the record's index word carries it (nh_pack). The eligibility test comes
// first, and the scheduling barrier keeps the distance arithmetic after it:
// the record's rho word is then dead when d2 is formed, so d2 takes its
// register and (index word, d2) is already the register pair of the key.
template <bool STRICT>
__device__ __forceinline__ void nh_consider_rec(NhBest& b, float4 r, float xi, float yi, unsigned ordi, unsigned hi) {
  const unsigned ordj = __float_as_uint(r.w), hj = __float_as_uint(r.z);
  const bool higher = STRICT ? ordj > ordi : key64(ordj, hj) > key64(ordi, hi);
  __builtin_amdgcn_sched_barrier(0);
  const unsigned long long ck = key64(__float_as_uint(dist2(xi, yi, r.x, r.y)), hj);
  const bool take = higher & (ck < b.k);
  b.k = take ? ck : b.k;
}

// Scans window tiles [tx0..tx1] x [ty0..ty1] (region coordinates) of the
// staged records (x, y, index, ord(rho)) with lanes sub, sub + step, ...
template <bool STRICT>
__device__ __forceinline__ void nh_scan_staged(const float4* __restrict__ rec, const int* ts, int per_row,
                                               int tx0, int tx1, int ty0, int ty1, int sub, int step, float xi,
                                               float yi, unsigned ordi, unsigned hi, NhBest& b) {
  for (int ty = ty0; ty <= ty1; ++ty) {
    const int q0 = ts[ty * per_row + tx0];
    const int q1 = ts[ty * per_row + tx1 + 1];
    int c = q0 + sub;
    const int c4 = q1 - 3 * step;
    // four independent LDS loads in flight per step
    for (; c < c4; c += 4 * step) {
      const float4 r0 = rec[c], r1 = rec[c + step], r2 = rec[c + 2 * step], r3 = rec[c + 3 * step];
      nh_consider_rec<STRICT>(b, r0, xi, yi, ordi, hi);
      nh_consider_rec<STRICT>(b, r1, xi, yi, ordi, hi);
      nh_consider_rec<STRICT>(b, r2, xi, yi, ordi, hi);
      nh_consider_rec<STRICT>(b, r3, xi, yi, ordi, hi);
    }
    for (; c < q1; c += step) nh_consider_rec<STRICT>(b, rec[c], xi, yi, ordi, hi);
  }
}

template <bool STRICT>
__device__ __forceinline__ void nh_global_scan(const Geom& g, const Arena& a, int64_t ubase, const Window& W, int sub, int step,
                               float xi, float yi, unsigned ordi, unsigned hi, NhBest& b) {
  for (int ty = W.y0; ty <= W.y1; ++ty) {
    const int64_t t = ubase + (int64_t)ty * g.nx;
    const int s0 = a.tile_start[t + W.x0], s1 = a.tile_start[t + W.x1 + 1];
    for (int c = s0 + sub; c < s1; c += step)
      nh_consider<STRICT>(b, dist2(xi, yi, a.xs[c], a.ys[c]), ord_f32(a.rho[c]), (unsigned)a.hs[c], -2 - c, ordi,
                          hi);
  }
}

// Returns false, having written nothing, when a staged hit's event-local
// index does not fit the packed word; the caller then searches the region in
// global memory.
template <bool STRICT>
__device__ __forceinline__ bool nh_staged(const Geom& g, const Arena& a, const RunDesc& d, const Region& R, const RegionLds& L,
                          float4* rec, unsigned short* queue, unsigned char* prow, unsigned short* coreq, int* s_qn,
                          int ev_first) {
  const int per_row = R.rw + 1;
  const int64_t ubase = (int64_t)R.unit * g.tpl;
  // the region row of every staged position (it gives the staging loads
  // their slots and the winners theirs), and the LDS position of every core
  // query, 16 lanes per row
  for (int k = threadIdx.x; k < 16 * R.rh; k += kWG) {
    const int r = k >> 4;
    const int end = L.row_lo[r + 1];
    for (int p = L.row_lo[r] + (k & 15); p < end; p += 16) prow[p] = (unsigned char)r;
    const int cr = r - R.cy0;
    if (cr >= 0 && cr < R.ch) {
      const int p0 = L.ts[r * per_row + R.cx0];
      const int q1 = L.core_lo[cr + 1];
      for (int q = L.core_lo[cr] + (k & 15); q < q1; q += 16) coreq[q] = (unsigned short)(p0 + q - L.core_lo[cr]);
    }
  }
  __syncthreads();
  // every global load of a lane is issued before its first LDS store
  bool outside = false;  // a hit whose event-local index does not fit the packed word
  for (int base = 0; base < R.total; base += kStagePer * kWG) {
    float4 v[kStagePer];
#pragma unroll
    for (int k = 0; k < kStagePer; ++k) {
      const int p = base + (int)threadIdx.x + k * kWG;
      if (p < R.total) {
        const int s = slot_of(L, prow[p], p);
        v[k] = make_float4(a.xs[s], a.ys[s], a.rho[s], __int_as_float(a.hs[s]));
      }
    }
#pragma unroll
    for (int k = 0; k < kStagePer; ++k) {
      const int p = base + (int)threadIdx.x + k * kWG;
      if (p < R.total) {
        outside |= (unsigned)(__float_as_int(v[k].w) - ev_first) >= (unsigned)kPackedEventMax;
        rec[p] = make_float4(v[k].x, v[k].y, __uint_as_float(nh_pack(__float_as_int(v[k].w), ev_first, p)),
                             __uint_as_float(ord_f32(v[k].z)));
      }
    }
  }
  if (threadIdx.x == 0) *s_qn = 0;
  // Event ids that decrease (unvalidated input) can leave hits of this unit
  // before its event's first hit; their packed index would wrap. Such a
  // region is searched in global memory, where records carry caller indices.
  if (__syncthreads_or(outside)) return false;
  const int nq = L.core_lo[R.ch];
  // phase 1: radius r1; only hits strictly within r1 can settle a query here
  for (int q = threadIdx.x; q < nq; q += kWG) {
    const int p = coreq[q];
    const int row = prow[p];
    bool done = false;
    if (g.nh_phase1) {
      const float4 me = rec[p];
      const unsigned ordi = __float_as_uint(me.w), zi = __float_as_uint(me.z);
      const Window W = query_window(g, g.win_r1, me.x, me.y);
      const int tx0 = W.x0 - R.rx0, tx1 = W.x1 - R.rx0, ty0 = W.y0 - R.ry0, ty1 = W.y1 - R.ry0;
      if (tx0 >= 0 && ty0 >= 0 && tx1 < R.rw && ty1 < R.rh) {
        NhBest b = nh_start(g.r1sq);
        const unsigned long long k0 = b.k;
        nh_scan_staged<STRICT>(rec, L.ts, per_row, tx0, tx1, ty0, ty1, 0, 1, me.x, me.y, ordi, zi, b);
        nh_unpack(b, k0, ev_first);
        if (b.p >= 0) {
          b.p = slot_of(L, prow[b.p], b.p);
          decide_and_store(g, a, d, slot_of(L, row, p), nh_unpack_h(zi, ev_first), ord_inv(ordi), b, ev_first);
          done = true;
        }
      }
    }
    if (!done) queue[atomicAdd(s_qn, 1)] = (unsigned short)p;  // its LDS position
  }
  __syncthreads();
  // phase 2: full d_m window, tpq lanes per query
  const int nu = *s_qn;
  const int tpq = g.tpq;
  const int sub = threadIdx.x & (tpq - 1);
  const int qpp = kWG / tpq;
  for (int base = 0; base < nu; base += qpp) {  // uniform trip count
    const int qi = base + threadIdx.x / tpq;
    const bool active = qi < nu;
    NhBest b = nh_start(g.dm2);
    const unsigned long long k0 = b.k;
    int slot = 0;
    unsigned hi = 0, ordi = 0;
    if (active) {
      const int p = queue[qi];
      slot = slot_of(L, prow[p], p);
      const float4 me = rec[p];
      ordi = __float_as_uint(me.w);
      const unsigned zi = __float_as_uint(me.z);
      hi = (unsigned)nh_unpack_h(zi, ev_first);
      const Window W = query_window(g, g.win_dm, me.x, me.y);
      const int tx0 = W.x0 - R.rx0, tx1 = W.x1 - R.rx0, ty0 = W.y0 - R.ry0, ty1 = W.y1 - R.ry0;
      if (tx0 >= 0 && ty0 >= 0 && tx1 < R.rw && ty1 < R.rh) {
        nh_scan_staged<STRICT>(rec, L.ts, per_row, tx0, tx1, ty0, ty1, sub, tpq, me.x, me.y, ordi, zi, b);
      } else {
        // global records carry the caller index itself, and the found slot as -2 - s
        atomicOr(a.err, (uint32_t)E_WINDOW);
        nh_global_scan<STRICT>(g, a, ubase, W, sub, tpq, me.x, me.y, ordi, hi, b);
      }
    }
    nh_reduce(b, tpq);  // the lanes of one query all took the same branch
    nh_unpack(b, k0, ev_first);
    if (active && sub == 0) {
      if (b.p >= 0)
        b.p = slot_of(L, prow[b.p], b.p);
      else if (b.p <= -2)
        b.p = -2 - b.p;
      decide_and_store(g, a, d, slot, (int)hi, ord_inv(ordi), b, ev_first);
    }
  }
  return true;
}

template <bool STRICT>
__device__ __forceinline__ void nh_global_region(const Geom& g, const Arena& a, const RunDesc& d, const Region& R,
                                 const RegionLds& L, int ev_first) {
  const int64_t ubase = (int64_t)R.unit * g.tpl;
  const int nq = L.core_lo[R.ch];
  const int tpq = g.tpq;
  const int sub = threadIdx.x & (tpq - 1);
  const int qpp = kWG / tpq;
  int cr = 0;
  for (int base = 0; base < nq; base += qpp) {
    const int q = base + threadIdx.x / tpq;
    const bool active = q < nq;
    NhBest b = nh_start(g.dm2);
    int slot = 0;
    unsigned hi = 0;
    if (active) {
      int row, p;
      core_query(L, R, q, cr, row, p);
      slot = slot_of(L, row, p);
      const float xi = a.xs[slot], yi = a.ys[slot];
      hi = (unsigned)a.hs[slot];
      const Window W = query_window(g, g.win_dm, xi, yi);
      nh_global_scan<STRICT>(g, a, ubase, W, sub, tpq, xi, yi, ord_f32(a.rho[slot]), hi, b);
    }
    nh_reduce(b, tpq);
    if (active && sub == 0) {
      if (b.p <= -2) b.p = -2 - b.p;
      decide_and_store(g, a, d, slot, (int)hi, a.rho[slot], b, ev_first);
    }
  }
}

template <bool STRICT>
__device__ __forceinline__ void nh_item(const Geom& g, const Arena& a, const RunDesc& d, int item, RegionLds& L,
                                        float4* rec, unsigned short* queue, unsigned char* prow, unsigned short* coreq,
                                        int* s_qn) {
  int unit, tx0, ty0, tx1, ty1;
  item_block(g, item, unit, tx0, ty0, tx1, ty1);
  Region R;
  make_region(g, unit, tx0, ty0, tx1, ty1, R);
  region_setup(g, a, R, L);
  if (L.core_lo[R.ch] == 0) return;
  const int ev_first = event_first_hit(a, d, R.e);
  if (event_first_hit(a, d, R.e + 1) - ev_first > kPackedEventMax) {
    // an event too large for the packed index word: the spill kernel searches
    // global memory, where records carry caller indices
    spill_region(g, a, R, C_SPILL_NH, kWG / g.tpq);
    return;
  }
  if (R.total <= g.lds_cap) {
    if (!nh_staged<STRICT>(g, a, d, R, L, rec, queue, prow, coreq, s_qn, ev_first)) nh_global_region<STRICT>(g, a, d, R, L, ev_first);
    return;
  }
  // too dense: the four quarter blocks, then single tiles
  const int hx = (tx1 - tx0 + 2) >> 1, hy = (ty1 - ty0 + 2) >> 1;
  for (int sy = ty0; sy <= ty1; sy += hy)
    for (int sx = tx0; sx <= tx1; sx += hx) {
      const int ex = min(sx + hx - 1, tx1), ey = min(sy + hy - 1, ty1);
      make_region(g, unit, sx, sy, ex, ey, R);
      region_setup(g, a, R, L);
      if (L.core_lo[R.ch] == 0) continue;
      if (R.total <= g.lds_cap && nh_staged<STRICT>(g, a, d, R, L, rec, queue, prow, coreq, s_qn, ev_first)) continue;
      if (R.total <= g.lds_cap) {
        nh_global_region<STRICT>(g, a, d, R, L, ev_first);
        continue;
      }
      for (int ty = sy; ty <= ey; ++ty)
        for (int tx = sx; tx <= ex; ++tx) {
          make_region(g, unit, tx, ty, tx, ty, R);
          region_setup(g, a, R, L);
          if (L.core_lo[R.ch] == 0) continue;
          if (R.total > g.lds_cap)
            spill_region(g, a, R, C_SPILL_NH, kWG / g.tpq);
          else if (!nh_staged<STRICT>(g, a, d, R, L, rec, queue, prow, coreq, s_qn, ev_first))
            nh_global_region<STRICT>(g, a, d, R, L, ev_first);
        }
    }
}

// Nearest-higher of the spilled queries, tpq lanes per query, from global
// memory, with the decision.
template <bool G, bool STRICT>
__global__ __launch_bounds__(kWG) void k_nh_spill(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  const int nch = a.counters[C_SPILL_NH];
  const int tpq = g.tpq;
  const int sub = threadIdx.x & (tpq - 1);
  for (int i = blockIdx.x; i < nch; i += gridDim.x) {  // uniform per workgroup: the shuffles below
    const int64_t t = a.key[i];
    const int slot = a.rank[i] + (int)threadIdx.x / tpq;
    const bool active = slot < a.tile_start[t + 1];
    const int64_t ubase = t - t % g.tpl;
    const int ev_first = event_first_hit(a, d, (int)(t / ((int64_t)g.L * g.tpl)));
    NhBest b = nh_start(g.dm2);
    unsigned hi = 0;
    if (active) {
      const float xi = a.xs[slot], yi = a.ys[slot];
      hi = (unsigned)a.hs[slot];
      const Window W = query_window(g, g.win_dm, xi, yi);
      nh_global_scan<STRICT>(g, a, ubase, W, sub, tpq, xi, yi, ord_f32(a.rho[slot]), hi, b);
    }
    nh_reduce(b, tpq);
    if (active && sub == 0) {
      if (b.p <= -2) b.p = -2 - b.p;
      decide_and_store(g, a, d, slot, (int)hi, a.rho[slot], b, ev_first);
    }
  }
}

// Built for eight waves per SIMD (64 VGPRs): the compiler then keeps one
// item-level value in scratch, reloaded once per work item, and the kernel
// runs 11% faster than at seven waves.
template <bool G, bool STRICT>
__global__ __launch_bounds__(kWG, 8) void k_nearest_higher(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_rows[kRowMetaInts];
  __shared__ int s_qn;
  __shared__ int s_item;
  float4* rec = reinterpret_cast<float4*>(smem);
  unsigned short* queue = reinterpret_cast<unsigned short*>(rec + g.lds_cap);
  unsigned short* coreq = queue + g.lds_cap;
  unsigned char* prow = reinterpret_cast<unsigned char*>(coreq + g.lds_cap);
  RegionLds L = region_lds(s_rows, reinterpret_cast<int*>(smem + lds_records_nh(g.lds_cap)), nullptr);
  const int n_items = d.n_events * g.L * g.bpu;
  ItemSched st{0, G ? xcc_id() : 0};
  for (int item; (item = next_item<G>(st, n_items, &a.counters[C_QUEUE_NH], &s_item)) >= 0;)
    nh_item<STRICT>(g, a, d, item, L, rec, queue, prow, coreq, &s_qn);
}

// ---------------------------------------------------------------------------
// Labels: follow the follower -> nearest-higher links to the root (pointer
// jumping with path compression; concurrent updates only ever store an
// ancestor, so every read is an ancestor and every chase ends at the root).
// A root that is a seed gives its seed number within the event; any other
// root (outlier, orphan) gives -1. Also places follower-list entries.
// ---------------------------------------------------------------------------
template <bool G>
__global__ __launch_bounds__(kWG) void k_label(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  const bool fol = builds_lists(g);
  constexpr int U = G ? kBatchU : kPlaceU;  // hits per lane per step, their chases interleaved
  constexpr int C = kWG * U;  // slots per chunk
  // the chunk's parent, caller index and flags, staged in LDS: a nearest-higher
  // lies within d_m, so most links stay inside the chunk. A staged parent may
  // be older than a compression stored since; it is still an ancestor.
  __shared__ int s_par[C];
  __shared__ int s_hs[C];
  __shared__ unsigned char s_fl[C];
  __shared__ int s_ev[2];  // the chunk's event when it holds one event (else -1), its first hit
  for (ChunkRun rn = xcd_run(d.n, C); rn.c < rn.end; rn.c += rn.step) {
    const int c0 = rn.c * C;
    if (threadIdx.x == 0) {
      const int e0 = event_of_slot(g, a, d, c0);
      const int e1 = event_of_slot(g, a, d, min(c0 + C, d.n) - 1);
      s_ev[0] = e0 == e1 ? e0 : -1;
      s_ev[1] = event_first_hit(a, d, e0);
    }
    const int sb = c0 + (int)threadIdx.x;
    int s[U], p0[U], hsj[U], r[U], p[U];
    unsigned f[U];
    bool v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      s[j] = sb + j * kWG;
      v[j] = s[j] < d.n;
      p0[j] = s[j];
      hsj[j] = 0;
      f[j] = 0;
      if (v[j]) {
        p0[j] = a.parent[s[j]];
        f[j] = a.flags[s[j]];
        hsj[j] = a.hs[s[j]];
      }
      s_par[s[j] - c0] = p0[j];
      s_hs[s[j] - c0] = hsj[j];
      s_fl[s[j] - c0] = (unsigned char)f[j];
    }
    __syncthreads();
    auto staged = [&](int x) { return (unsigned)(x - c0) < (unsigned)C; };
    // first hit of each hit's event, from its slot
    const int ev1 = s_ev[0], first1 = s_ev[1];
    int first[U];
#pragma unroll
    for (int j = 0; j < U; ++j)
      first[j] = ev1 >= 0 || !v[j] ? first1 : event_first_hit(a, d, event_of_slot(g, a, d, s[j]));
    if (fol) {
      // entries are event-local already: the list sort then leaves lists of
      // one entry alone. Every load of a lane comes before its first store
      // (the stores could alias them as far as the compiler knows).
      int at[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        at[j] = -1;
        if (v[j] && (f[j] & F_FOLLOWER)) {
          const int owner = staged(p0[j]) ? s_hs[p0[j] - c0] : a.hs[p0[j]];
          at[j] = a.fstart[owner] + a.frank[s[j]];
        }
      }
#pragma unroll
      for (int j = 0; j < U; ++j)
        if (at[j] >= 0) a.flist[at[j]] = hsj[j] - first[j];
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      r[j] = s[j];
      p[j] = p0[j];
    }
    for (;;) {
      bool more = false;
#pragma unroll
      for (int j = 0; j < U; ++j) {
        if (p[j] != r[j]) {
          r[j] = p[j];
          p[j] = staged(r[j]) ? s_par[r[j] - c0] : ld_relaxed(&a.parent[r[j]]);
          more = true;
        }
      }
      if (!more) break;
    }
    int lab[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      lab[j] = -1;
      if (!v[j]) continue;
      const bool in = staged(r[j]);
      if ((in ? s_fl[r[j] - c0] : a.flags[r[j]]) & F_SEED)
        lab[j] = seed_rank(a, in ? s_hs[r[j] - c0] : a.hs[r[j]]) - seed_rank(a, first[j]);
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (!v[j]) continue;
      if (r[j] != s[j] && r[j] != p0[j]) st_relaxed(&a.parent[s[j]], r[j]);
      d.cluster_id[hsj[j]] = lab[j];
    }
    __syncthreads();  // the next chunk overwrites the staged arrays
  }
}

// ---------------------------------------------------------------------------
// Labels by k-way expansion (Sec. 2.2, Algorithm 3): one thread per seed walks
// the seed's follower tree depth first and gives every hit in it the seed's
// cluster id. The walk keeps no stack: each follower's owner and its position
// in the owner's list (key / rank, free after the grid build) lead back up to
// the next unvisited sibling, so a thread holds O(1) state whatever the tree's
// depth.
// ---------------------------------------------------------------------------

// Part 1: places follower-list entries (as k_label does), records owner and
// position per follower, labels seeds with their number within the event and
// every other hit -1, and lists the seeds by rank.
template <bool G>
__global__ __launch_bounds__(kWG) void k_expand_init(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  int* const seeds = reinterpret_cast<int*>(a.xs);
  constexpr int U = kPlaceU;
  for (ChunkRun rn = xcd_run(d.n, kWG * U); rn.c < rn.end; rn.c += rn.step) {
    const int sb = rn.c * kWG * U + (int)threadIdx.x;
    int p[U], h[U];
    unsigned f[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int s = sb + j * kWG;
      f[j] = 0;
      p[j] = 0;
      h[j] = 0;
      if (s < d.n) {
        f[j] = a.flags[s] | 0x100u;
        p[j] = a.parent[s];
        h[j] = a.hs[s];
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (!(f[j] & 0x100u)) continue;
      const int s = sb + j * kWG;
      int lab = -1;
      if (f[j] & F_FOLLOWER) {
        const int owner = a.hs[p[j]];
        const int r = a.frank[s];
        a.flist[a.fstart[owner] + r] = h[j];
        a.key[h[j]] = owner;
        a.rank[h[j]] = r;
      } else if (f[j] & F_SEED) {
        const int e = d.event ? clampi(d.event[h[j]] - d.event_base, 0, d.n_events - 1) : 0;
        const int rk = seed_rank(a, h[j]);
        lab = rk - seed_rank(a, event_first_hit(a, d, e));
        seeds[rk] = h[j];
      }
      d.cluster_id[h[j]] = lab;
    }
  }
}

// Part 2: the walks. Each visits its tree in preorder: down to a node's first
// follower, else up through owners to the first one with a next sibling. A
// walk takes at most 2 (n + 1) steps (each edge down once and up once); a walk
// that reached that bound would mean corrupt lists, so it stops and flags the
// run instead of looping.
template <bool G>
__global__ __launch_bounds__(kWG) void k_expand_dfs(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  const int* const seeds = reinterpret_cast<const int*>(a.xs);
  const int ns = seed_rank(a, d.n);
  const int64_t max_steps = 2 * ((int64_t)d.n + 1);
  for (int t = blockIdx.x * kWG + (int)threadIdx.x; t < ns; t += gridDim.x * kWG) {
    const int root = seeds[t];
    const int lab = d.cluster_id[root];
    int u = root;
    int b = a.fstart[u], e = a.fstart[u + 1];
    int64_t steps = 0;
    for (;;) {
      if (++steps > max_steps) {
        atomicOr(a.err, (uint32_t)E_WALK);
        break;
      }
      if (b < e) {
        u = a.flist[b];  // first follower
      } else {
        // climb to the nearest node (u or an ancestor) that has a next sibling
        bool found = false;
        while (u != root && steps <= max_steps) {
          ++steps;
          const int p = a.key[u];
          const int nx = a.fstart[p] + a.rank[u] + 1;
          if (nx < a.fstart[p + 1]) {
            u = a.flist[nx];
            found = true;
            break;
          }
          u = p;
        }
        if (!found) break;
      }
      d.cluster_id[u] = lab;
      b = a.fstart[u];
      e = a.fstart[u + 1];
    }
  }
}

// Follower lists: sort each list by hit index. k_label writes event-local
// entries, so lists of one entry are already final; after the depth-first
// expansion (which walks caller indices) every entry is made event-local
// here. Lists of up to kShortList entries are sorted in registers (odd-even
// transposition networks of four entries, when every list of the wave fits,
// or eight); longer ones by insertion in place.
constexpr int kShortList = 8;

template <bool G>
__global__ __launch_bounds__(kWG) void k_follow_sort(DescArg<G> dg, Geom g, Arena a) {
  const RunDesc d = dg.get();
  constexpr int U = kPlaceU;
  for (ChunkRun rn = xcd_run(d.n, kWG * U); rn.c < rn.end; rn.c += rn.step) {
    const int hb = rn.c * kWG * U + (int)threadIdx.x;
    int b[U], end[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int h = hb + j * kWG;
      b[j] = 0;
      end[j] = 0;
      if (h < d.n) {
        b[j] = a.fstart[h];
        end[j] = a.fstart[h + 1];
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int len = end[j] - b[j];
      // nearly every wave holds only lists of up to four entries: then the
      // whole wave takes the shorter network (a wave-uniform choice)
      const bool four = __all(len <= 4);
      if (len < (g.expand ? 1 : 2)) continue;
      int off = 0;
      if (g.expand) {
        const int h = hb + j * kWG;
        off = event_first_hit(a, d, d.event ? clampi(d.event[h] - d.event_base, 0, d.n_events - 1) : 0);
      }
      if (four) {
        int v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = i < len ? a.flist[b[j] + i] : INT_MAX;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int i = r & 1; i + 1 < 4; i += 2) {
            const int lo = min(v[i], v[i + 1]), hi = max(v[i], v[i + 1]);
            v[i] = lo;
            v[i + 1] = hi;
          }
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i < len) a.flist[b[j] + i] = v[i] - off;
        continue;
      }
      if (len <= kShortList) {
        int v[kShortList];
#pragma unroll
        for (int i = 0; i < kShortList; ++i) v[i] = i < len ? a.flist[b[j] + i] : INT_MAX;
#pragma unroll
        for (int r = 0; r < kShortList; ++r)
#pragma unroll
          for (int i = r & 1; i + 1 < kShortList; i += 2) {
            const int lo = min(v[i], v[i + 1]), hi = max(v[i], v[i + 1]);
            v[i] = lo;
            v[i + 1] = hi;
          }
#pragma unroll
        for (int i = 0; i < kShortList; ++i)
          if (i < len) a.flist[b[j] + i] = v[i] - off;
        continue;
      }
      for (int i = b[j] + 1; i < end[j]; ++i) {
        const int v = a.flist[i];
        int k = i - 1;
        while (k >= b[j] && a.flist[k] > v) {
          a.flist[k + 1] = a.flist[k];
          --k;
        }
        a.flist[k + 1] = v;
      }
      for (int i = b[j]; i < end[j]; ++i) a.flist[i] -= off;
    }
  }
}

// ---------------------------------------------------------------------------
// Input validation (CLUE_VALIDATE).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_validate(RunDesc d, int L, uint32_t* err) {
  const int stride = gridDim.x * kWG;
  bool bad = false;
  for (int h = blockIdx.x * kWG + threadIdx.x; h < d.n; h += stride) {
    bad |= !isfinite(d.x[h]) || !isfinite(d.y[h]) || !isfinite(d.e[h]);
    bad |= d.layer[h] < 0 || d.layer[h] >= L;
    if (d.event) {
      bad |= d.event[h] < d.event_base || d.event[h] - d.event_base >= d.n_events;
      if (h > 0) bad |= d.event[h] < d.event[h - 1];
    }
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(err, (uint32_t)E_INPUT);
}

__global__ void k_set_desc(RunDesc d, RunDesc* dd) {
  if (threadIdx.x == 0) *dd = d;
}

// ---------------------------------------------------------------------------
// Host launches.
// ---------------------------------------------------------------------------
// Dynamic LDS of the density kernel: per staged hit 16 bytes of record and
// hit index, a 16-bit tile id and four 16-bit quad-list entries, then the
// region's tile offsets and quad-list offsets.
int lds_bytes_for(const Geom& g) { return lds_records_density(g.lds_cap) + 4 * (g.ts_ints + g.q_ints); }
// Nearest-higher: per staged hit a float4 record, a 16-bit queue entry, a
// 16-bit core-query position and its region row (a byte), then the region's
// tile offsets.
int lds_bytes_nh(const Geom& g) { return lds_records_nh(g.lds_cap) + 4 * g.ts_ints; }

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

template <bool G>
static hipError_t launch_all(const Geom& g, const Arena& a, DescArg<G> dg, const RunDesc& host_d,
                             const LaunchCfg& cfg, hipStream_t s, hipEvent_t* ev) {
  // Grid sizes: plain launches are sized to the run; graph launches use
  // persistent grids (sizes are read from the descriptor on the device).
  const int64_t n = host_d.n;
  const int64_t tt = (int64_t)host_d.n_events * g.L * g.tpl + 1;
  const int64_t items = (int64_t)host_d.n_events * g.L * g.bpu;
  // streaming grids are a multiple of kQueues (one run of chunks per XCD)
  auto stream_grid = [&](int64_t work) {
    if (G) return cfg.persist_blocks_stream;
    const int64_t b = std::max<int64_t>(1, std::min<int64_t>(cdiv(work, kWG), 1 << 20));
    return (int)((b + kQueues - 1) / kQueues * kQueues);
  };
  const int g_clear = G ? cfg.persist_blocks_stream
                        : (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(std::max(tt, n + 1), kWG), 1 << 16));
  const int g_rho = G ? cfg.persist_blocks_rho : (int)std::max<int64_t>(1, items);
  const int g_nh = G ? cfg.persist_blocks_nh : (int)std::max<int64_t>(1, items);
  const int g_scan_t = G ? cfg.persist_blocks_scan : cdiv(tt, kScanChunk);
  // spill kernels: one workgroup per CU in single launches (an empty queue
  // costs one counter read per workgroup)
  const int g_spill = G ? cfg.persist_blocks_stream : 256;
  const int g_scan_s = G ? cfg.persist_blocks_scan : cdiv(n + 1, kScanChunk);
  const bool fol = !(g.flags & 8u);
  int k = 0;
  auto mark = [&]() {
    if (ev) (void)hipEventRecord(ev[k++], s);
  };
  mark();
  k_clear<G><<<g_clear, kWG, 0, s>>>(dg, g, a);
  mark();
  k_hist<G><<<stream_grid(cdiv(n, kPlaceU)), kWG, 0, s>>>(dg, g, a);
  mark();
  k_scan<G, SCAN_TILES><<<g_scan_t, kWG, 0, s>>>(dg, g, a);
  mark();
  k_scatter<G><<<G ? cfg.persist_blocks_scatter : stream_grid(cdiv(n, kPlaceU)), kWG, 0, s>>>(dg, g, a);
  mark();
  k_place<G><<<stream_grid(cdiv(n, G ? kBatchU : kPlaceU)), kWG, 0, s>>>(dg, g, a);
  mark();
  const int lds = lds_bytes_for(g);
  if (g.kernel == 0) {
    if (g.maxl == 2)
      k_density<G, 2, 0><<<g_rho, kWG, lds, s>>>(dg, g, a);
    else
      k_density<G, 3, 0><<<g_rho, kWG, lds, s>>>(dg, g, a);
    k_density_spill<G, 0><<<g_spill, kWG, 0, s>>>(dg, g, a);
  } else if (g.kernel == 1) {
    if (g.maxl == 2)
      k_density<G, 2, 1><<<g_rho, kWG, lds, s>>>(dg, g, a);
    else
      k_density<G, 3, 1><<<g_rho, kWG, lds, s>>>(dg, g, a);
    k_density_spill<G, 1><<<g_spill, kWG, 0, s>>>(dg, g, a);
  } else {
    if (g.maxl == 2)
      k_density<G, 2, 2><<<g_rho, kWG, lds, s>>>(dg, g, a);
    else
      k_density<G, 3, 2><<<g_rho, kWG, lds, s>>>(dg, g, a);
    k_density_spill<G, 2><<<g_spill, kWG, 0, s>>>(dg, g, a);
  }
  mark();
  if (g.flags & 4u) {
    k_nearest_higher<G, true><<<g_nh, kWG, lds_bytes_nh(g), s>>>(dg, g, a);
    k_nh_spill<G, true><<<g_spill, kWG, 0, s>>>(dg, g, a);
  } else {
    k_nearest_higher<G, false><<<g_nh, kWG, lds_bytes_nh(g), s>>>(dg, g, a);
    k_nh_spill<G, false><<<g_spill, kWG, 0, s>>>(dg, g, a);
  }
  mark();
  if (builds_lists(g))
    k_scan<G, SCAN_SEEDS_FOLLOW><<<g_scan_s, kWG, 0, s>>>(dg, g, a);
  else
    k_scan<G, SCAN_SEEDS><<<g_scan_s, kWG, 0, s>>>(dg, g, a);
  mark();
  if (g.expand) {
    k_expand_init<G><<<stream_grid(cdiv(n, kPlaceU)), kWG, 0, s>>>(dg, g, a);
    const int g_dfs = G ? cfg.persist_blocks_stream : std::min(stream_grid(n), std::max(1, cfg.persist_blocks_stream));
    k_expand_dfs<G><<<g_dfs, kWG, 0, s>>>(dg, g, a);
  } else {
    k_label<G><<<stream_grid(cdiv(n, G ? kBatchU : kPlaceU)), kWG, 0, s>>>(dg, g, a);
  }
  mark();
  if (fol) k_follow_sort<G><<<stream_grid(cdiv(n, kPlaceU)), kWG, 0, s>>>(dg, g, a);
  mark();
  return hipGetLastError();
}

hipError_t launch_pipeline(const Geom& g, const Arena& a, const RunDesc& d, const LaunchCfg& cfg, hipStream_t s,
                           hipEvent_t* ev) {
  if (cfg.graph_mode) {
    DescArg<true> dg{a.desc};
    return launch_all<true>(g, a, dg, d, cfg, s, ev);
  }
  DescArg<false> dg{d};
  return launch_all<false>(g, a, dg, d, cfg, s, ev);
}

hipError_t launch_set_desc(const RunDesc& d, RunDesc* dd, hipStream_t s) {
  k_set_desc<<<1, 64, 0, s>>>(d, dd);
  return hipGetLastError();
}

hipError_t launch_validate(const Geom& g, const Arena& a, const RunDesc& d, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(d.n, kWG), 4096));
  k_validate<<<grid, kWG, 0, s>>>(d, g.L, a.err);
  return hipGetLastError();
}

int occupancy_blocks_per_cu(int which, int lds_bytes) {
  int nb = 0;
  hipError_t e = hipSuccess;
  switch (which) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_hist<true>, kWG, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_density<true, 2, 0>, kWG, lds_bytes); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_scan<true, SCAN_SEEDS_FOLLOW>, kWG, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_nearest_higher<true, false>, kWG, lds_bytes); break;
    default: break;
  }
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

}  // namespace clue
