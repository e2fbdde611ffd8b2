// scan_run_device_noalloc: the in-memory clustering run of scan_run_device
// without any device allocation on the call.  Every per-run buffer (bounds,
// roles, union-find parents, labels, edge states, statistics and job
// counters, the LDS-hash kernel's worklist) is carved out of one file-scope
// device array, `scratch`, of kScratchBytes bytes.  Each device the library
// runs on holds its own copy of the array for the life of the process.
//
// Host code never passes `scratch` itself to a kernel: in host code that name
// is only a stand-in for the symbol.  The device address of each device's copy
// is looked up once, with hipGetSymbolAddress while that device is current,
// and kept per device; kernels receive that address.
//
// Every call on one device shares that device's array, which keeps the last
// call's contents; a run clears and initialises every part it reads (the
// counters by kernels at its start), so no state leaks from one call to the
// next.  Calls that overlap on one device race on the array.
#include "graph.h"

#include <mutex>

namespace {

constexpr uint64_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up once
// per device).  SCAN_OK or an error code.
int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(SCAN_E_DEVICE, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SCAN_E_DEVICE, "hipGetSymbolAddress(scratch) returned no address");
    g_scratch_ptr[device] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return SCAN_OK;
}

constexpr uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Bytes of the scratch a run on g needs, and the run state laid out from base
// (base may be null to size only).
uint64_t layout_state(const scan_graph* g, unsigned char* base, RunState* R) {
  const uint64_t n = (uint64_t)(g->n > 0 ? g->n : 1);
  const uint64_t m = (uint64_t)(g->m > 0 ? g->m : 1);
  const int64_t w = g->bucket_off[kNumBuckets] - g->bucket_off[kNumBuckets - 1];
  const uint64_t wl = (uint64_t)(w > 0 ? w : 1);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    unsigned char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  RunState r{};
  r.stats = reinterpret_cast<unsigned long long*>(take(8ull * ST_COUNT));
  r.counters = reinterpret_cast<unsigned long long*>(take(8ull * kCounters));
  r.lower = reinterpret_cast<int32_t*>(take(4 * n));
  r.upper = reinterpret_cast<int32_t*>(take(4 * n));
  r.parent = reinterpret_cast<int32_t*>(take(4 * n));
  r.label = reinterpret_cast<int32_t*>(take(4 * n));
  r.role = take(n);
  r.state = take(m);
  r.worklist = reinterpret_cast<int32_t*>(take(4 * wl));
  if (R) *R = r;
  return off;
}

}  // namespace

extern "C" {

int scan_run_device_noalloc(scan_graph* g, int64_t eps_num, int64_t eps_den, int32_t mu, int32_t* d_labels,
                            uint8_t* d_roles, void* stream) {
  if (!g) return fail(SCAN_E_INVAL, "graph is NULL");
  if (g->n > 0 && (!d_labels || !d_roles)) return fail(SCAN_E_INVAL, "output pointer is NULL");
  if (g->partitioned) return fail(SCAN_E_INVAL, "scan_run_device_noalloc serves in-memory graphs only");
  int64_t p = eps_num, q = eps_den;
  int rc = check_params(g, p, q, mu);
  if (rc != SCAN_OK) return rc;
  const uint64_t need = layout_state(g, nullptr, nullptr);
  if (need > kScratchBytes)
    return fail(SCAN_E_NOMEM, "scan_run_device_noalloc: the run needs %llu bytes of scratch, the static scratch "
                "holds %llu (n = %d, m = %lld)", (unsigned long long)need, (unsigned long long)kScratchBytes,
                g->n, (long long)g->m);
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (dev != g->device)
    return fail(SCAN_E_INVAL, "the graph lives on device %d, the current device is %d", g->device, dev);
  unsigned char* base = nullptr;
  rc = scratch_address(dev, &base);
  if (rc != SCAN_OK) return rc;
  RunState R{};
  layout_state(g, base, &R);
  EdgeArgs A{};
  A.p = (uint64_t)p;
  A.q = (uint64_t)q;
  A.mu = mu;
  A.pruning = g->opts.pruning;
  hipStream_t s = stream ? (hipStream_t)stream : g->stream;
  enqueue_clustering(g, A, d_labels, d_roles, nullptr, s, false, nullptr, &R);
  HIP_TRY(hipGetLastError(), "kernel launch");
  // on the caller's stream the run stays stream-ordered (the caller
  // synchronises); on the graph's own stream the outputs are ready on return
  if (!stream) HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return SCAN_OK;
}

}  // extern "C"
