// Internal declarations shared by the HIP kernels and the host runtime of
// libclue. Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clue {

constexpr int kWG = 256;            // threads per workgroup, every kernel
constexpr int kScanItems = 16;      // elements per thread in the prefix scans of single launches
constexpr int kScanItemsBatch = 64; // ... and of the persistent batched form, whose fewer, larger
                                    // chunks shorten the look-back chains
constexpr int kScanChunk = kWG * kScanItems;  // the smaller chunk, which sizes the status array
__host__ __device__ constexpr int scan_items(bool graph) { return graph ? kScanItemsBatch : kScanItems; }
constexpr int kMaxRegionTiles = 640;   // staged region tiles, rows x (cols + 1), per workgroup
constexpr int kMaxRegionRows = 64;
constexpr int kDefaultLdsCap = 960;    // staged hits per workgroup (fast path)
constexpr int kMaxLdsCap = 2048;
// The density kernel's LDS arrays: per staged hit 16 bytes of record and hit
// index, then a 16-bit tile id per hit, then four 16-bit quad-list entries per
// hit (from an 8-byte boundary), then one 16-byte sentinel record, rounded up
// to 16 bytes.
__host__ __device__ constexpr int density_qidx_offset(int lds_cap) { return (lds_cap * (16 + 2) + 7) & ~7; }
__host__ __device__ constexpr int density_sentinel_offset(int lds_cap) {
  return (density_qidx_offset(lds_cap) + lds_cap * 8 + 15) & ~15;
}
__host__ __device__ constexpr int lds_records_density(int lds_cap) { return density_sentinel_offset(lds_cap) + 16; }
static_assert(density_sentinel_offset(2048) + 16 <= 65536, "quad-list entries are 16-bit LDS byte offsets");
// ... and of the nearest-higher kernel's (float4 record, 16-bit queue entry,
// 16-bit core-query position, 8-bit region row).
__host__ __device__ constexpr int lds_records_nh(int lds_cap) { return (lds_cap * (16 + 2 + 2 + 1) + 15) & ~15; }
static_assert(kMaxLdsCap <= 65536, "nearest-higher queue entries are 16-bit");
constexpr int kStagePer = 4;       // staged hits per lane per round (loads in flight)
constexpr int kPlaceU = 4;         // hits per lane per step of the streaming grid-build and list kernels
constexpr int kBatchU = 8;         // ... and of the batched k_scatter, k_place and k_label: longer runs
                                   // per workgroup, and 2048-slot LDS chunks that keep more of a tile
                                   // or a parent chain on chip (single launches keep kPlaceU, for more
                                   // workgroups per event)
constexpr int kScatterBlocksPerCU = 2;  // persistent k_scatter workgroups per CU

// Counters in device memory, cleared at the start of every run. Each sits on
// its own 256-byte line so that atomics on different counters do not
// contend; the tile-block stages have one queue head per XCD.
constexpr int kCounterStride = 64;  // ints
constexpr int kQueues = 8;          // one per XCD
enum Counter {
  C_TICKET_TILES = 0,                           // chunk tickets of the tile-count scan
  C_TICKET_SEEDS = 1 * kCounterStride,          // chunk tickets of the seed / follower scan
  C_QUEUE_RHO = 2 * kCounterStride,             // kQueues heads for the density stage
  C_QUEUE_NH = (2 + kQueues) * kCounterStride,  // kQueues heads for the nearest-higher stage
  C_SPILL_RHO = (2 + 2 * kQueues) * kCounterStride,      // density query chunks left to the spill kernel
  C_SPILL_NH = (2 + 2 * kQueues + 1) * kCounterStride,   // ... and nearest-higher query chunks
  C_COUNT = (2 + 2 * kQueues + 2) * kCounterStride
};

// Device error word bits (read and cleared by clue_status).
enum ErrBits : uint32_t {
  E_INPUT = 1u,    // non-finite coordinate/energy, bad layer or event id
  E_WINDOW = 2u,   // a query window left the staged halo (never expected)
  E_WALK = 4u,     // an expansion walk exceeded its step bound (never expected)
};

// Per-run descriptor: sizes and the caller's buffers.
struct RunDesc {
  int32_t n;
  int32_t n_events;
  const float* x;
  const float* y;
  const float* e;
  const int32_t* layer;
  const int32_t* event;  // nullptr: single event
  int32_t event_base;    // event ids are event_base + [0, n_events)
  int32_t* cluster_id;
  uint8_t* is_seed;
};

// Geometry and thresholds, fixed between re-tunings.
struct Geom {
  float x0, y0;     // grid origin (x_min, y_min)
  float inv_t;      // 1 / tile size, float32
  int32_t nx, ny;   // tiles per dimension
  int32_t tpl;      // tiles per layer = nx * ny
  int32_t L;        // layers
  int32_t bx, by;   // tile block (work item) shape
  int32_t nbx, nby; // blocks per dimension
  int32_t bpu;      // blocks per (event, layer) unit
  int32_t halo;     // staged halo in tiles around a block
  int32_t maxl;     // density window tiles per dimension (2 or 3)
  int32_t tpq;      // lanes per nearest-higher query
  int32_t lds_cap;  // staged hits per workgroup
  int32_t ts_ints;  // LDS ints for a region's tile offsets: rows * (cols + 1) + 1
  int32_t q_ints;   // LDS ints for the quad-list offsets: (bx + 1) * (by + 1) + 1
  float dc2;        // fl(dc*dc)
  int32_t kernel;   // density kernel: 0 flat, 1 Gaussian, 2 exponential
  float ka;         // its constant: fl(1 / (2 s^2)) or fl(1 / s)
  float dm2;        // fl(dm*dm), dm = max(delta_o, delta_c)
  float dcs2;       // fl(delta_c*delta_c)
  float do2;        // fl(delta_o*delta_o)
  float rho_c;
  float win_dc;     // dc (1 + 2^-10): density window half width before the |x| margin
  float win_dm;     // dm (1 + 2^-10)
  int32_t density_quads;  // 1: per-item quad lists by search; 2: by sequential merge; 0: per-query merge
  int32_t nh_phase1;  // nearest-higher first searches radius r1 < dm
  float r1sq;       // fl(r1*r1)
  float win_r1;     // r1 (1 + 2^-10)
  int32_t expand;   // cluster expansion: 0 pointer jumping, 1 depth-first from each seed
  uint32_t flags;   // CLUE_* flags
};

// Follower lists (counts, ranks, CSR) are built when the caller asks for them
// or when the depth-first expansion walks them.
__host__ __device__ inline bool builds_lists(const Geom& g) { return !(g.flags & 8u) || g.expand != 0; }

// Arena: device scratch owned by a context.
struct Arena {
  int32_t* key;          // [N]   caller order: global tile id of each hit
  int32_t* rank;         // [N]   caller order: arrival rank within its tile
                         //       (free after the grid build: the spill queues of the
                         //       density and nearest-higher stages, tile and first slot
                         //       of each query chunk)
                         //       (the depth-first expansion reuses both for each
                         //       follower's owner and its position in the owner's list)
                         //       (the grid build keeps arrival-order hit ids and tiles
                         //       in the rho and parent buffers until each tile is
                         //       ordered by hit index)
  int32_t* tile_start;   // [TT+1] tile counts, scanned in place into CSR offsets
  float* xs;             // [N]   slot order (tile CSR; hit index ascending within a tile);
                         //       after the nearest-higher stage, the depth-first
                         //       expansion's seed list
  float* ys;
  float* es;
  int32_t* hs;           // [N]   slot -> caller (batch-global) hit index
  float* rho;            // [N]   slot order
  int32_t* parent;       // [N]   slot order: nearest-higher slot of a follower, else itself
  uint8_t* flags;        // [N]   slot order: F_SEED | F_OUTLIER | F_FOLLOWER
  uint32_t* seedbits;    // [N/32+2] caller order: one bit per hit, set for seeds
  int32_t* seed_wrank;   // [N/32+2] seeds in the words before each word of seedbits
  int32_t* ev_start;     // [E+1] caller-order first hit of each event
  int32_t* fstart;       // [N+1] caller order: follower counts, scanned into CSR offsets
  int32_t* frank;        // [N]   slot order: rank of a follower within its owner's list
  int32_t* flist;        // [N]   follower lists (caller-global indices until finalised)
  float* rho_out;        // [N]   caller order, with CLUE_KEEP_INTERMEDIATES
  int32_t* nh_out;
  float* d2_out;
  unsigned long long* scan_status;  // [max chunks of either scan]
  int32_t* counters;     // [C_COUNT]
  uint32_t* err;         // [1]
  RunDesc* desc;         // device copy of the run descriptor (graph replays)
  int64_t cap_hits;
  int32_t cap_events;
  int64_t cap_tiles;     // TT capacity
  int64_t cap_chunks;
};

enum HitFlags : uint8_t { F_SEED = 1, F_OUTLIER = 2, F_FOLLOWER = 4 };

enum Stage {
  S_CLEAR = 0, S_HIST, S_SCAN_TILES, S_SCATTER, S_PLACE, S_RHO, S_NH, S_SCAN_SEEDS, S_LABEL, S_FOLLOW,
  S_COUNT
};
extern const char* const kStageNames[S_COUNT];

struct LaunchCfg {
  bool graph_mode;   // persistent kernels reading the descriptor from device memory
  int persist_blocks_stream;  // persistent grid of the streaming kernels
  int persist_blocks_scatter; // persistent grid of k_scatter (fewer workgroups: its
                              // scattered writes complete lines in L2 more often)
  int persist_blocks_rho;     // persistent grid of the density kernel
  int persist_blocks_nh;      // persistent grid of the nearest-higher kernel
  int persist_blocks_scan;    // persistent grid of the scans
};

// Host-side launches (implemented in clue_kernels.hip). `d` is the run
// descriptor by value (plain mode) and `dd` its device copy (graph mode).
// `ev` receives a HIP event after each stage when non-null.
hipError_t launch_pipeline(const Geom& g, const Arena& a, const RunDesc& d, const LaunchCfg& cfg,
                           hipStream_t s, hipEvent_t* ev);
hipError_t launch_set_desc(const RunDesc& d, RunDesc* dd, hipStream_t s);
hipError_t launch_validate(const Geom& g, const Arena& a, const RunDesc& d, hipStream_t s);
int occupancy_blocks_per_cu(int which, int lds_bytes);
int lds_bytes_for(const Geom& g);
int lds_bytes_nh(const Geom& g);

}  // namespace clue
