// hesp_noalloc.hip -- hesp_simulate_batch_noalloc: the batched simulation of
// hesp_simulate_batch with every scratch buffer carved from one fixed device
// array, for callers that cannot allocate device memory.
//
// The pipeline is the one of hesp_simulate_batch in a single chunk, on the
// caller's stream only: exact task and edge counts, their prefix sums (plus the
// byte size of each candidate's block), preparation and the persistent event
// loop.  Each candidate's arrays lie together in its own block of the region
// part of the array, blocks in candidate order; a candidate whose block would
// end past the region gets HESP_ECAPACITY.  No candidate ordering by size and
// no autotuning (lanes per candidate are an argument).
#include <hip/hip_runtime.h>

#include <mutex>

#include "hesp.h"
#include "hesp_internal.h"

using namespace hesp;

extern "C" int hesp_internal_fail(int code, const char* msg);
extern "C" int hesp_internal_batch_setup(const hesp_platform* pf, hesp_policy policy, const hesp_batch* batch,
                                         const hesp_tree_batch* tree, const hesp_outputs* out, SimTables& tb,
                                         BatchView& bv);

namespace {

// The whole scratch of the entry point.  Every call on one device shares it.
static __device__ __align__(256) uint8_t scratch[HESP_NOALLOC_BYTES];

constexpr int kMaxDevices = 64;
constexpr int64_t kN = HESP_NOALLOC_MAX_CAND;

constexpr int64_t up256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// byte offsets of the parts of the array
constexpr int64_t kCounter = 0;
constexpr int64_t kCntTasks = 256;
constexpr int64_t kCntEdges = kCntTasks + up256(4 * kN);
constexpr int64_t kOffT = kCntEdges + up256(8 * kN);
constexpr int64_t kOffE = kOffT + up256(8 * (kN + 1));
constexpr int64_t kOffV = kOffE + up256(8 * (kN + 1));
constexpr int64_t kOffTop = kOffV + up256(8 * (kN + 1));
constexpr int64_t kOffB = kOffTop + up256(8 * (kN + 1));
constexpr int64_t kNsrc = kOffB + up256(8 * (kN + 1));
constexpr int64_t kRegion = kNsrc + up256(4 * kN);

static_assert(HESP_NOALLOC_BYTES - kRegion == HESP_NOALLOC_REGION, "region size of the public header");

// device address of the array and compute-unit count, per device, taken once
// with that device current
struct DevInfo {
  uint8_t* ptr = nullptr;
  int cus = 0;
};
DevInfo g_dev[kMaxDevices];
std::mutex g_mu;

int fail(int code, const char* msg) { return hesp_internal_fail(code, msg); }

int device_info(DevInfo& out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(HESP_EHIP, "hesp_simulate_batch_noalloc: no usable current device");
  std::lock_guard<std::mutex> lk(g_mu);
  DevInfo& d = g_dev[dev];
  if (!d.ptr) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(HESP_EHIP, "hesp_simulate_batch_noalloc: hipGetSymbolAddress failed");
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cus <= 0) return fail(HESP_EHIP, "hesp_simulate_batch_noalloc: no compute-unit count");
    d.cus = cus;
    d.ptr = (uint8_t*)p;
  }
  out = d;
  return HESP_OK;
}

}  // namespace

extern "C" int hesp_simulate_batch_noalloc(const hesp_platform* pf, hesp_policy policy, const hesp_batch* batch,
                                           const hesp_outputs* out, int32_t group, void* stream) {
  static_assert(HESP_NOALLOC_BYTES % 256 == 0, "scratch size");
  if (!batch) return fail(HESP_EINVAL, "hesp_simulate_batch_noalloc: null batch");
  if (batch->n_cand > kN)
    return fail(HESP_EINVAL, "hesp_simulate_batch_noalloc: more than HESP_NOALLOC_MAX_CAND (16384) candidates");
  if (group != 0 && group != 16 && group != 32 && group != 64)
    return fail(HESP_EINVAL, "hesp_simulate_batch_noalloc: group must be 0, 16, 32 or 64");
  SimTables tb;
  BatchView bv;
  if (int r = hesp_internal_batch_setup(pf, policy, batch, nullptr, out, tb, bv)) return r;
  if (tb.capped) return fail(HESP_EUNSUPPORTED, "hesp_simulate_batch_noalloc: no finite memory spaces");
  if (tb.max_level > kXferLevels)
    return fail(HESP_EUNSUPPORTED, "hesp_simulate_batch_noalloc: platform tables of at most 3 levels");
  if (group == 0) group = tb.n_procs <= 16 ? 16 : (tb.n_procs <= 32 ? 32 : 64);
  if (group < tb.n_procs) return fail(HESP_EINVAL, "hesp_simulate_batch_noalloc: group below the processor count");
  if (bv.dmax > kMaxWaveLevel && group == kWave)
    return fail(HESP_EUNSUPPORTED, "hesp_simulate_batch_noalloc: depths above 3 take 16 or 32 lanes per candidate");
  const int n = bv.n_cand;
  if (n == 0) return HESP_OK;
  DevInfo d;
  if (int r = device_info(d)) return r;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* base = d.ptr;
  int32_t* cnt_t = (int32_t*)(base + kCntTasks);
  int64_t* cnt_e = (int64_t*)(base + kCntEdges);
  int64_t* off_t = (int64_t*)(base + kOffT);
  int64_t* off_e = (int64_t*)(base + kOffE);
  int64_t* off_v = (int64_t*)(base + kOffV);
  int64_t* off_top = (int64_t*)(base + kOffTop);
  int64_t* off_b = (int64_t*)(base + kOffB);

  auto hip_fail = [](hipError_t e) {
    return fail(HESP_EHIP, e == hipSuccess ? "hesp_simulate_batch_noalloc" : hipGetErrorString(e));
  };
  hipError_t e = launch_count(bv, cnt_t, cnt_e, s);
  if (e != hipSuccess) return hip_fail(e);
  e = launch_layout(bv, tb.n_mem, cnt_t, cnt_e, 0, 0, off_t, off_e, off_v, off_top, off_b, s);
  if (e != hipSuccess) return hip_fail(e);

  ChunkView cv{};
  cv.task_off = off_t;
  cv.edge_off = off_e;
  cv.vf_off = off_v;
  cv.top_off = off_top;
  cv.c0 = 0;
  cv.nc = n;
  cv.cnt_tasks = cnt_t;
  cv.cnt_edges = cnt_e;
  cv.nsrc = (int32_t*)(base + kNsrc);
  cv.byte_off = off_b;
  cv.region = base + kRegion;
  cv.region_cap = (int64_t)HESP_NOALLOC_BYTES - kRegion;
  const OutView ov{out->d_makespan, out->d_status, out->d_n_tasks, out->d_sched_off,
                   out->d_proc,     out->d_start,  out->d_finish};
  e = launch_prepare(tb, bv, cv, ov, s);
  if (e != hipSuccess) return hip_fail(e);
  e = launch_sim(tb, bv, cv, ov, 32 * d.cus, group, (uint32_t*)(base + kCounter), s);
  if (e != hipSuccess) return hip_fail(e);
  return HESP_OK;
}
