// Internal: the graph object behind the opaque scan_graph handle, error
// reporting, and entry points shared by the C-ABI translation units.
#pragma once

#include "scan_internal.h"
#include "../../include/scan.h"

#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

using namespace scan;

namespace scan {

// Device buffers one clustering run works in: the graph's own (graph_state),
// a set of the graph's pool for calls that overlap (ExtraRun), or a
// caller-provided region of the same sizes.
struct RunState {
  int32_t* lower;
  int32_t* upper;
  uint8_t* role;
  int32_t* parent;
  int32_t* label;
  uint8_t* state;                // one per oriented edge
  unsigned long long* stats;     // ST_COUNT
  unsigned long long* counters;  // kCounters
  int32_t* worklist;             // one per edge of the last bucket
};

// Per-run buffers, stream and events of a call that overlaps another call on
// the same in-memory graph; allocated at the first overlap and kept, for the
// next one, until the graph is destroyed.
struct ExtraRun {
  RunState R{};
  int32_t* d_out_labels = nullptr;  // staging for host outputs
  uint8_t* d_out_roles = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev[SCAN_NUM_PHASES + kNumBuckets + 2] = {};
  uint64_t bytes = 0;  // device bytes it holds
  bool busy = false;
};

}  // namespace scan

// Partitioned (out-of-core) layout: GPUSCAN++ Section 5 (Def. 5.1, Lemma 5.1,
// Alg. 5).  The CSR stays in pinned host memory; vertex ranges ("units") are
// sized so that a block (two consecutive units) fits half of the device row
// buffer and a unit one of the two slots of its other half, and every edge
// belongs to the pair of its lower endpoint's block with the other endpoint's
// unit (or to the block's own pair).  A chunk is a run of one pair's edges
// (grouped by degree bucket) small enough for the device edge buffer.
struct PartChunk {
  int32_t bi, bj;                          // block bi with unit bj of a later block (-1: edges inside bi)
  int64_t begin, end;                      // range of the pinned edge array
  int64_t bucket_off[kNumBuckets + 1];     // bucket sub-ranges, clipped to [begin, end)
  int64_t job_off = 0, job_cnt = 0;        // LDS-hash jobs of the last bucket (chunk-relative edges)
};

struct PartPlan {
  std::vector<int32_t> block_lo;  // K+1 vertex boundaries of the blocks
  std::vector<int32_t> unit_lo;   // U+1 vertex boundaries of the units (a block is upb units)
  int32_t upb = 1;                // units per block
  int32_t nslots = 1;             // device slots for units (2: the next unit uploads while one is read)
  int64_t jcap = 0;               // ints per unit slot (slots follow the block's half of the row buffer)
  std::vector<int64_t> h_rp;      // host copy of row_ptr
  std::vector<PartChunk> chunks;
  int32_t* h_ci = nullptr;        // pinned copy of col_idx
  int2* h_edges = nullptr;        // pinned: oriented edges ordered by (pair, bucket, arc)
  uint8_t* h_state = nullptr;     // pinned: edge states, streamed with the edges
  int32_t* h_ecount = nullptr;    // pinned: per-edge closed counts (scan_similarity)
  int64_t row_cap = 0;            // ints of the device row buffer (a block, then the unit slots)
  int64_t chunk_cap = 0;          // edges per chunk
  int32_t* d_rows = nullptr;
  int2* d_edges = nullptr;        // two chunk buffers (edges, states): the next chunk is
  uint8_t* d_state = nullptr;     // uploaded on the copy stream while kernels run on the other
  int2* d_edges2 = nullptr;
  uint8_t* d_state2 = nullptr;
  int32_t* d_ecount = nullptr;
  HubJob* d_jobs = nullptr;       // every chunk's LDS-hash jobs (resident)
  uint32_t* d_wtab = nullptr;     // their windows
  int32_t* d_worklist = nullptr;  // one slot per edge of a chunk
  unsigned long long* d_jobctr = nullptr;
  hipStream_t copy = nullptr;     // upload stream of edges and states (default priority)
  hipEvent_t up[2] = {}, done[2] = {};
  hipStream_t rowcopy = nullptr;  // upload stream of unit rows (default priority)
  hipEvent_t rready[2] = {}, rfree[2] = {};  // per unit slot: rows uploaded / last reader done
  uint64_t h2d_bytes = 0;         // bytes sent to the device by the last call
  int64_t chunks_streamed = 0;    // chunks sent by the last call (passes that skip chunks send fewer)
};

struct scan_graph {
  bool partitioned = false;
  PartPlan part;
  int32_t n = 0;
  int64_t nnz = 0, m = 0;
  int32_t max_degree = 0;
  int64_t bucket_off[kNumBuckets + 1] = {0};
  scan_opts opts{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  // graph (read-only after create)
  int64_t* d_rp = nullptr;
  int32_t* d_ci = nullptr;
  int32_t* d_hci = nullptr;  // rows renamed by degree rank (LDS-hash kernel), or null
  int32_t* d_hsamp = nullptr;  // first id of every 128-byte line of the rows the LDS-hash kernel reads
  int2* d_edges = nullptr;
  HubJob* d_jobs = nullptr;
  int64_t hub_jobs = 0;
  uint32_t* d_wtab = nullptr;     // LDS-hash windows of the jobs' larger sides
  int2* d_edeg = nullptr;         // degrees of both sides per oriented edge
  int64_t wtab_entries = 0;
  int32_t* d_worklist = nullptr;  // one slot per edge of the last bucket
  // per-run state
  int32_t* d_lower = nullptr;
  int32_t* d_upper = nullptr;
  uint8_t* d_role = nullptr;
  int32_t* d_parent = nullptr;
  int32_t* d_label = nullptr;
  uint8_t* d_state = nullptr;
  unsigned long long* d_stats = nullptr;
  unsigned long long* d_counters = nullptr;  // job counters of the LDS-hash kernel, one per pass
  int32_t* d_out_labels = nullptr;  // staging for the host-output entry points
  uint8_t* d_out_roles = nullptr;
  int32_t* d_counts = nullptr;      // staging for scan_similarity
  hipEvent_t ev[SCAN_NUM_PHASES + kNumBuckets + 2] = {};
  std::mutex lock;  // the graph's own per-run buffers, staging and events (one call at a time)
  // buffer sets of calls that find the graph's own ones in use
  std::mutex pool_lock;  // extra and the sets' busy flags
  std::vector<std::unique_ptr<ExtraRun>> extra;
  std::atomic<uint64_t> extra_bytes{0};
  mutable std::mutex stats_lock;  // last
  scan_stats last{};
};

namespace scan {

// Job counters of the LDS-hash kernel (one per pass), then the number of cores.
constexpr int kCounters = 5;

RunState graph_state(scan_graph* g);
// Publishes the statistics of a finished call (scan_last_stats reads them).
void set_last(scan_graph* g, const scan_stats& L);

// Per-bucket kernel choice for one run: lanes[k] = lane-group width of the
// group kernel for bucket k (0 = the bucket's default), hub = LDS-hash kernel
// for the last bucket.
struct RunConfig {
  int lanes[kNumBuckets];
  bool hub;
};

void launch_bucket(scan_graph* g, hipStream_t s, int mode, int k, EdgeArgs& A, const RunState& R,
                   const RunConfig* cfg = nullptr);
// Kernel launches of one clustering run (capturable); A carries eps/mu (or
// per-graph arrays); gbase (batch) turns labels into graph-local ids.  The run
// works in R, or in the graph's own buffers when R is null, and marks its
// phases (timing) with the events ev, or the graph's own when ev is null.
void enqueue_clustering(scan_graph* g, EdgeArgs& A, int32_t* d_labels, uint8_t* d_roles,
                        const int32_t* gbase, hipStream_t s, bool timing, const RunConfig* cfg,
                        const RunState* R = nullptr, hipEvent_t* ev = nullptr);
// Checks eps = p/q and mu against the graph (Def 2.3, Def 2.4, the 64-bit
// range of the test) and reduces p/q; SCAN_OK or the error code.
int check_params(const scan_graph* g, int64_t& p, int64_t& q, int32_t mu);
// Waits for the run enqueued on s and publishes its statistics, read from R's
// counters and the events ev (the graph's own buffers and events by default).
int collect_stats(scan_graph* g, hipStream_t s, bool timing);
int collect_stats(scan_graph* g, hipStream_t s, bool timing, const RunState& R, hipEvent_t* ev);

// Sets the thread-local message returned by scan_last_error; returns code.
int fail(int code, const char* fmt, ...);
int fail_hip(hipError_t e, const char* what);

// Exact closed counts of every edge of g on stream s, written per arc
// (d_counts_arc, CSR order) and/or per oriented edge (d_counts_edge); either
// may be null.
int run_counts(scan_graph* g, int32_t* d_counts_arc, int32_t* d_counts_edge, hipStream_t s);

// Partitioned path (partition.hip).  device bytes the in-memory layout needs
// (an upper bound of what scan_graph_create allocates):
uint64_t inmemory_footprint(int32_t n, int64_t nnz, bool ranked);
// Device bytes an in-memory graph holds now (its buffers as allocated).
uint64_t graph_device_bytes(const scan_graph* g);
// The part of them fixed at creation (layout and the graph's own per-run
// state, without the staging allocated on first use).
uint64_t graph_layout_bytes(const scan_graph* g);
// Plans blocks and chunks for `budget` device bytes, copies the CSR to pinned
// memory and allocates the resident state and streaming buffers.
int part_validate(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx, bool full);
int part_create(scan_graph* g, const int64_t* row_ptr, const int32_t* col_idx, uint64_t budget);
void part_release(scan_graph* g);
int part_run(scan_graph* g, uint64_t p, uint64_t q, int32_t mu, int32_t* d_labels, uint8_t* d_roles,
             hipStream_t s);
// Exact per-arc closed counts into host memory (CSR order).
int part_counts(scan_graph* g, int32_t* h_counts, hipStream_t s);

}  // namespace scan

#define HIP_TRY(call, what)                             \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return scan::fail_hip(_e, what); \
  } while (0)
