// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace scan {

// Per-vertex role during the run (Table 1 of the paper: ?, C, !C).
enum : uint8_t { ROLE_UNK = 0, ROLE_CORE = 1, ROLE_NONCORE = 2,
                 ROLE_HUB = 3 };  // ROLE_HUB: in no cluster, neighbours in two or more (Def 2.7)
// Per-edge similarity state (Table 1: ?, S, !S).
enum : uint8_t { SIM_UNK = 0, SIM_YES = 1, SIM_NO = 2 };

// Degree buckets of the oriented edge list, keyed by the smaller degree d_s
// and the larger degree d_l:
//   0: d_s <= 4, 1: <= 8, 2: <= 16, 3: <= 32, 4: <= 64   (groups of 4..64 lanes per edge)
//   5: d_s > 64, d_l <= kHubMinDegree                     (one wave per edge, tiled)
//   6: d_s > 64, d_l >  kHubMinDegree                     (LDS-hash kernel, by larger side)
constexpr int kNumBuckets = 7;
constexpr int kHubMinDegree = 512;

__host__ __device__ inline int bucket_of(int64_t ds) {
  return ds <= 4 ? 0 : ds <= 8 ? 1 : ds <= 16 ? 2 : ds <= 32 ? 3 : ds <= 64 ? 4 : 5;
}

// What a pass over the oriented edges does with each edge.
enum Mode : int {
  MODE_CORES = 0,   // identifyCore (Alg. 2): similarity test + lower/upper bound counting
  MODE_MERGE = 1,   // progressive core-core merge (Alg. 3, second loop)
  MODE_ATTACH = 2,  // border attachment (Alg. 3, last loop), minimum label
  MODE_COUNTS = 3   // exact closed counts of every edge (no pruning)
};

// Stats slots (int64 counters on the device).
enum : int {
  ST_EVAL = 0,      // + phase: edges intersected
  ST_BOUND = 4,     // + phase: decided by the degree bound
  ST_PROBES = 8,    // + phase: smaller-list elements consumed
  ST_BUCKET_EVAL = 12,   // + bucket (cores phase only)
  ST_BUCKET_PROBES = 19, // + bucket
  ST_GROUP_SPLIT = 26,   // LDS-hash kernel: lanes of a group that claimed a different chunk than the group's first lane
  ST_COUNT = 27
};
// Mode -> stats phase slot (0..3).
__host__ __device__ inline int mode_slot(int mode) { return mode; }

// Smallest closed count c with (c q)^2 >= p^2 a b.  Requires q*max(a,b) < 2^32
// so that p^2 a b <= q^2 a b < 2^64 and every product below fits in 64 bits.
__host__ __device__ inline uint32_t closed_needed(uint64_t p, uint64_t q, uint64_t a, uint64_t b) {
  const uint64_t X = (p * p) * (a * b);
  uint64_t r = (uint64_t)sqrt((double)X);
  if (r > 0xFFFFFFFFull) r = 0xFFFFFFFFull;
  while (r * r > X) --r;
  while (r < 0xFFFFFFFFull && (r + 1) * (r + 1) <= X) ++r;
  const uint64_t s = (r * r == X) ? r : r + 1;  // ceil(sqrt(X))
  return (uint32_t)((s + q - 1) / q);           // (c q)^2 >= X  <=>  c q >= ceil(sqrt(X))
}

// LDS-hash kernel of the last bucket (d_u > 64): one job = up to kHubJobEdges
// in-edges (u, v) of one larger side v, consecutive in the edge list.
constexpr int kHubJobEdges = 2048; // in-edges per job
constexpr int64_t kHubJobWork = 1 << 24;  // smaller-list elements per job (bound on probes)
constexpr int kHubBlock = 512;     // threads per block of the LDS-hash kernel
constexpr int kHubBlocksPerCU = 2; // blocks resident per compute unit (each holds its own table)
constexpr int kHubWavesPerSimd = kHubBlocksPerCU * kHubBlock / 256;  // 4 SIMDs of wave64 per CU
constexpr int kHubBatch = 256;     // survivors per table fill
constexpr int kHubPerThread = kHubJobEdges / kHubBlock;  // in-edges classified per thread and round
constexpr int kHubInsertBatch = 4; // table inserts per thread with their loads issued together
constexpr int kHubGroup = 8;      // lanes streaming one survivor
constexpr int kHubUnroll = 8;      // elements per lane per step
constexpr int kHubChunk = 1024;    // elements of one survivor handed to a group at a time
// col_idx is allocated with this many spare elements after its end, so that the
// LDS-hash kernel's step loads (up to one step past a chunk's end, values
// beyond the end ignored) need no clamping
constexpr int64_t kColPad = 2 * kHubGroup * kHubUnroll;
constexpr int kHubLog2Slots = 14;  // LDS table per block: 16384 int32 slots = 64 KiB
constexpr int kHubSlots = 1 << kHubLog2Slots;
constexpr int kHubWindow = kHubSlots / 2;  // elements of nbr(v) per table fill (load <= 1/2)
// The same LDS array read as a bitmap covers kHubBitmapBits consecutive ids;
// a window of nbr(v) is taken as a bitmap when that many ids from its first
// element on hold at least kHubBitmapMin elements of nbr(v).
constexpr int kHubBitmapBits = kHubSlots * 32;
constexpr int kHubBitmapMin = 4096;
// A hash window of at most this many elements (a quarter of the slots) uses
// first-fit placement, so that most probes read a single bucket.
constexpr int kHubSparseMax = kHubSlots / 4;
// windows of a job that its later batches take from LDS instead of finding again
constexpr int kHubMaxWindows = 64;
struct HubJob {
  int64_t begin;  // first edge of the job
  int32_t v;      // common larger side
  int32_t count;  // edges in the job (<= kHubJobEdges)
  int32_t wbeg;   // v's windows: entries wbeg .. wbeg + wcnt - 1 of the window table
  int32_t wcnt;   // (0: none computed, the kernel finds them)
};
// Window table entry: (end of the window in v's row) << 1 | (1 if a bitmap window).
// The windows of a row depend only on the row, so they are computed once per
// hub vertex when the graph is created (hub_windows) rather than by the kernel.
int64_t hub_windows(const int32_t* row, int64_t dv, std::vector<uint32_t>& out);
// Fills wbeg / wcnt of every job from the rows the kernel reads (row of v at
// rows + rp[v]) and returns the window table.
void assign_hub_windows(std::vector<HubJob>& jobs, const int64_t* rp, const int32_t* rows,
                        std::vector<uint32_t>& table);

struct EdgeArgs {
  const int64_t* rp;
  const int32_t* ci;
  const int32_t* hci;  // rows read by the LDS-hash kernel: ci, or ci renamed by degree rank
  const int2* edges;  // oriented: x = smaller side (deg, id), y = larger side
  const uint32_t* wtab;  // LDS-hash windows of the jobs' larger sides (HubJob::wbeg)
  const int2* edeg;   // degrees of both sides per oriented edge (null: read from rp)
  const int32_t* hsamp;  // hsamp[k] = hci[32 k], the first id of every 128-byte line of hci
                         // (null: the LDS-hash kernel searches the rows themselves)
  int64_t e_begin, e_end;
  uint8_t* state;     // per oriented edge
  int32_t* lower;     // confirmed |N_eps| lower bound (starts at 1)
  int32_t* upper;     // |N_eps| upper bound (starts at deg + 1)
  uint8_t* role;
  int32_t* parent;
  int32_t* label;
  int32_t* counts;       // MODE_COUNTS: per arc output (optional)
  int32_t* edge_counts;  // MODE_COUNTS: per oriented edge output (optional)
  unsigned long long* stats;
  uint64_t p, q;
  int32_t mu;
  int32_t pruning;
  int32_t bucket;
  // Row placement: row of x starts at ci + rp[x] - delta, with delta_a for
  // a_lo <= x < a_hi and delta_b otherwise (0 and 0 when the graph is resident).
  int32_t a_lo, a_hi;
  int64_t delta_a, delta_b;
  // Batch of graphs: graph id of every vertex and per-graph eps = gp/gq, mu
  // (null for a single graph, which uses p, q, mu above).
  const int32_t* gid;
  const uint64_t* gp;
  const uint64_t* gq;
  const int32_t* gmu;
  // Number of cores after the cores pass (null: unknown); the merge and attach
  // kernels return at once when it is zero.
  const unsigned long long* ncores;
};

// Launchers (kernels.hip)
void launch_init(hipStream_t s, int32_t n, const int64_t* rp, int32_t mu, int32_t* lower,
                 int32_t* upper, uint8_t* role, int32_t* parent, const int32_t* gid = nullptr,
                 const int32_t* gmu = nullptr);
void launch_edges(hipStream_t s, int mode, int bucket, const EdgeArgs& a);
// Same with an explicit lane-group width (4, 8, 16, 32 or 64), any bucket.
void launch_edges_lanes(hipStream_t s, int mode, int lanes, const EdgeArgs& a);
// Last bucket through the LDS-hash kernel; counter must be zero on entry,
// worklist holds one int32 per edge of the bucket.
void launch_hub(hipStream_t s, int mode, const EdgeArgs& a, const HubJob* jobs, int64_t njobs,
                unsigned long long* counter, int32_t* worklist);
// Blocks of the LDS-hash kernel's grid (compute units of the device); queried
// once, before any launch is captured into a HIP graph.
int hub_grid_blocks();
void launch_zero_u64(hipStream_t s, unsigned long long* p, int n);
void launch_copy16(hipStream_t s, const void* src, void* dst, int64_t n16);
// Read-only stream of n16 16-byte words; sink holds read16_sink_words() words.
void launch_read16(hipStream_t s, const void* src, int64_t n16, uint32_t* sink);
int read16_sink_words();
void launch_fill_u8(hipStream_t s, uint8_t* p, int64_t n, uint8_t v);
// ncores (optional): incremented by the number of cores after the pass.
void launch_finalize_roles(hipStream_t s, int32_t n, int32_t mu, const int32_t* lower, uint8_t* role,
                           const int32_t* gid = nullptr, const int32_t* gmu = nullptr,
                           unsigned long long* ncores = nullptr);
void launch_hook(hipStream_t s, int64_t m, const int2* edges, const uint8_t* state,
                 const uint8_t* role, int32_t* parent);
void launch_flatten(hipStream_t s, int32_t n, const uint8_t* role, int32_t* parent, int32_t* label);
// split = 1: vertices in no cluster are output as hub (3) or outlier (4).
void launch_output(hipStream_t s, int32_t n, const uint8_t* role, const int32_t* label,
                   int32_t* out_labels, uint8_t* out_roles, int32_t split, const int32_t* gid = nullptr,
                   const int32_t* gbase = nullptr);
void launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v);
// Hub marking over m oriented edges (after attach): first[] must hold -1.
void launch_hub_outlier_edges(hipStream_t s, int64_t m, const int2* edges, const int32_t* label, int32_t* first,
                              uint8_t* role);

// Serving: |N[u]| |N[v]| per oriented edge (once per graph), then one query
// from cached per-edge closed counts and those products (no intersections).
void launch_closed_products(hipStream_t s, int64_t m, const int64_t* rp, const int2* edges, uint64_t* ab);
void launch_rethreshold(hipStream_t s, int32_t n, int64_t m, const int2* edges, const int32_t* ecount,
                        const uint64_t* ab, uint64_t p, uint64_t q, int32_t mu, int32_t* lower,
                        uint8_t* role, int32_t* parent, int32_t* label, uint8_t* state,
                        int32_t* out_labels, uint8_t* out_roles, int32_t split);

// ---------------------------------------------------------------------------
// Batched clustering in one persistent launch (many graphs packed as one
// disjoint union).  Every graph goes through the phases below in order; a
// phase is cut into tiles (vertex tiles or edge tiles per degree bucket), and
// blocks of the persistent kernel take (graph, phase, tile) items from a
// device queue.  The block that finishes the last tile of a graph's phase
// publishes the tiles of its next phase.
enum BatchPhase : int {
  BP_INIT = 0,  // bounds, roles, parents (vertex tiles)
  BP_CORES,     // similarity test + core counting (edge tiles)
  BP_FINAL,     // role finalize, cores counted per graph (vertex tiles)
  BP_HOOK,      // union along known-similar core-core edges (edge tiles)
  BP_MERGE,     // progressive core-core merge (edge tiles)
  BP_FLAT,      // labels = roots (vertex tiles)
  BP_ATTACH,    // border attachment (edge tiles)
  BP_HUBOUT,    // hub / outlier marks, only with split roles (edge tiles)
  BP_OUTPUT,    // graph-local labels and roles (vertex tiles)
  BP_DONE
};
// Phases that have nothing to do for a graph without cores: their tiles are
// never queued.
__host__ __device__ inline bool batch_phase_needs_cores(int ph) {
  return ph == BP_HOOK || ph == BP_MERGE || ph == BP_ATTACH || ph == BP_HUBOUT;
}
__host__ __device__ inline bool batch_vertex_phase(int ph) {
  return ph == BP_INIT || ph == BP_FINAL || ph == BP_FLAT || ph == BP_OUTPUT;
}
// Tiles of phase ph for a graph of n vertices with ek[k] edges in bucket k.
// An edge tile is tile_edges consecutive edges of the graph's bucket ranges
// taken one after the other (so a tile may span several buckets).
__host__ __device__ inline int64_t batch_phase_tiles(int ph, int64_t n, const int64_t* ek, int64_t tile_edges,
                                                     int64_t tile_vertices, int split) {
  if (ph == BP_HUBOUT && !split) return 0;
  if (batch_vertex_phase(ph)) return (n + tile_vertices - 1) / tile_vertices;
  int64_t m = 0;
  for (int k = 0; k < kNumBuckets; ++k) m += ek[k];
  return (m + tile_edges - 1) / tile_edges;
}

struct BatchArgs {
  EdgeArgs A;                    // graph arrays, per-vertex graph ids and per-graph eps/mu
  int32_t G;
  const int64_t* vtx_off;        // [G + 1] first vertex of each graph in the union
  const int64_t* eoff;           // [kNumBuckets * (G + 1)]: first edge of graph g in bucket k
  uint32_t lanes_code;           // lane-group width of bucket k: 4 << ((lanes_code >> 3k) & 7)
                                 // (a scalar, so that no kernel argument is indexed at run time)
  int32_t tile_edges;            // edges per edge tile (a multiple of 64)
  int32_t tile_vertices;         // vertices per vertex tile
  int32_t split;                 // hub / outlier roles
  int32_t* out_labels;           // graph-local labels
  uint8_t* out_roles;
  unsigned long long* queue;     // items of every phase after BP_INIT (empty slots hold ~0)
  const int64_t* init_prefix;    // [G + 1]: prefix of the graphs' BP_INIT tiles
  int32_t* remaining;            // [G]: tiles of the graph's current phase not finished
  unsigned long long* ncores;    // [G]
  unsigned long long* ctl;       // [0] slots taken, [1] queue slots filled, [2] error, [3] items skipped
  int64_t total;                 // items of the whole run if no phase is skipped
  int64_t init_items;            // BP_INIT items (init_prefix[G])
  int64_t queue_cap;             // queue slots
  uint64_t watchdog_ticks;       // wall-clock ticks a block waits for an item before giving up
};
// Resets the queue and counters, then runs the whole batch (two kernels,
// capturable).  grid = blocks of the persistent kernel.
void launch_batch(hipStream_t s, const BatchArgs& B, int grid);
// eoff for graphs with vertex offsets vtx_off over the bucketed edge list
// (edges of each bucket in increasing order of their larger side).
void launch_batch_edge_offsets(hipStream_t s, int32_t G, const int64_t* vtx_off, const int2* edges,
                               const int64_t* bucket_off_host, int64_t* eoff);
// Blocks of the persistent kernel that fit on the device at once.
int batch_grid_blocks();

// Lines of 32 ids (128 bytes) that hold nnz ids.
inline int64_t sample_lines(int64_t nnz) { return (nnz + 31) >> 5; }

// samp[k] = rows[32 k] for k < nlines (rows holds at least 32 (nlines - 1) + 1 ids).
void launch_line_samples(hipStream_t s, int64_t nlines, const int32_t* rows, int32_t* samp);

// deg[e] = (degree of edges[e].x, degree of edges[e].y) for m oriented edges.
void launch_edge_degrees(hipStream_t s, int64_t m, const int64_t* rp, const int2* edges, int2* deg);

// Layout (layout.hip)
struct LayoutResult {
  int64_t bucket_off[kNumBuckets + 1];
  int64_t hub_jobs;
  int32_t max_degree;
  int32_t error;  // 0 or bit mask of validation failures
};
// Validates the CSR and builds the oriented, bucketed edge list and the job
// table of the last bucket, both allocated here (caller frees):
//   *d_edges: bucket_off[kNumBuckets] entries, *d_jobs: hub_jobs entries.
// The job table is returned on the host (jobs), to be completed with the
// windows and uploaded by the caller.
hipError_t build_layout(hipStream_t s, int32_t n, int64_t nnz, const int64_t* h_rp,
                        const int32_t* h_ci, const int64_t* d_rp, const int32_t* d_ci, int validate,
                        int2** d_edges, std::vector<HubJob>* jobs, LayoutResult* out);
// Fills d_hci (nnz entries) with the rows of the CSR with every vertex renamed
// to its rank in order of increasing degree (ties by id), each row sorted
// again (also returned in h_hci).  Intersection sizes do not depend on the names.  The top
// kHubBitmapBits ranks hold most arc endpoints of a skewed graph, so the
// LDS-hash kernel covers most of a long row with one bitmap window, and a
// survivor's low-degree neighbours, the likely misses, come first, which
// settles dissimilar edges earlier.  Built on the host threads and copied;
// synchronous.
hipError_t build_ranked_rows(hipStream_t s, int32_t n, int64_t nnz, const int64_t* h_rp,
                             const int32_t* h_ci, int32_t* d_hci, std::vector<int32_t>* h_hci);

}  // namespace scan
