// Batched filtering: plans, the job table in the caller's workspace, and the
// persistent per-class launches (one HIP graph per plan when asked for).
//
// A plan resolves every job on the host (arguments, W, the Algorithm 2 fit,
// the unit-sum spatial profile), picks each job's kernel family and tile
// geometry, and cuts every image into output tiles ("work items").  Items are
// grouped into classes that share one kernel (window class NT and family);
// each class has its own tile height and grid mode, which bf_plan_tune can
// measure and remember for later plans; inside a class the jobs are ordered by decreasing
// number of planes 4K+1, so a persistent grid that takes items round-robin
// gives every workgroup a similar load.  The descriptor table and the items
// are copied once into the caller's workspace:
//
//   [ JobDesc x n_jobs | pad to 256 B | int4 items (job, x0, y0, 0) ]
//
// The copy is staged through library-owned pinned host memory.  A staging
// buffer is reused only after the event recorded behind its copy has
// completed; one whose copy was recorded into a stream capture is never
// reused (the captured copy node keeps reading it).  The pool is never freed
// before process exit, which avoids calling into the HIP runtime from static
// destructors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <tuple>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bf_internal.h"

namespace bf {
namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct ClassLaunch {
  int nt = 0;                 // window class: 16-row tiles spanned by 16 rows + 2W halo
  int family = 0;             // 1 wave kernel, 2 shared-plane staged, 0 general
  TileChoice tc{};            // current tile geometry (tc.th is tunable)
  int grid = 0;               // 0: occupancy-sized persistent grid; -1: one workgroup per item; > 0: fixed
  int t_max = 0;              // largest T among the class's jobs (sizes the dynamic LDS)
  int f_max = 0;              // largest gray-level table extent F among them
  std::vector<int> jobs;      // ordered by decreasing K
  std::vector<int> th_options;  // tile heights every job of the class supports
  size_t item_off = 0;        // first item of the class
  int n_items = 0;
  double px = 0.0;            // pixels of the class
  double cost = 0.0;          // sum over items of (4K+1) x tile area, for ordering
  bool tuned = false;         // geometry taken from the tuner (or its cache)
};

struct PlanData {
  bf_planes prec = BF_PLANES_FP32;
  std::vector<JobDesc> descs;
  std::vector<int4> items;
  std::vector<ClassLaunch> classes;
  int status = BF_OK;      // BF_OK or BF_FIT_NOT_CONVERGED
  size_t items_off = 0;    // byte offset of the items in the workspace
  size_t ws_bytes = 0;     // sized for the smallest tile height of every class
};

// Workgroups per class launch.  BF_BATCH_GRID=items gives one workgroup per
// item (the hardware dispatcher balances the load); a positive number fixes
// the grid; the default sizes a persistent grid from the occupancy.
int grid_mode_from_env() {
  const char* s = std::getenv("BF_BATCH_GRID");
  if (!s || !*s) return 0;
  if (std::strcmp(s, "items") == 0) return -1;
  const int v = std::atoi(s);
  return v > 0 ? v : 0;
}

bool valid_tile_rows(int v) { return v == 32 || v == 64 || v == 96 || v == 128 || v == 144; }

// Preferred output-tile height (32, 64, 96, 128 or 144 rows) from BF_TILE_ROWS; 0 = default.
int tile_rows_from_env() {
  const char* s = std::getenv("BF_TILE_ROWS");
  if (!s || !*s) return 0;
  const int v = std::atoi(s);
  return valid_tile_rows(v) ? v : 0;
}

int valid_prec(bf_planes prec) {
  return prec == BF_PLANES_FP32 || prec == BF_PLANES_FP16 || prec == BF_PLANES_BF16;
}

// ---- tuned geometry, shared by every plan of the process ------------------
// Key: plane format, window class, kernel family and the class size
// (round(log2(pixels))); value: tile rows and grid mode measured fastest.
struct TuneKey {
  int prec, nt, family, size_log2;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, nt, family, size_log2) < std::tie(o.prec, o.nt, o.family, o.size_log2);
  }
};
struct TuneVal {
  int th, grid;
};
std::mutex g_tune_mutex;
std::map<TuneKey, TuneVal>* g_tune = new std::map<TuneKey, TuneVal>();  // never freed

TuneKey tune_key(bf_planes prec, const ClassLaunch& c) {
  return TuneKey{static_cast<int>(prec), c.nt, c.family, static_cast<int>(std::lround(std::log2(std::max(c.px, 1.0))))};
}

int items_of(const JobDesc& d, int th, int cols) {
  return ((d.height + th - 1) / th) * ((d.width + cols - 1) / cols);
}

// Lays the items of every class out in class order (classes already sorted).
void emit_items(PlanData& p) {
  p.items.clear();
  for (ClassLaunch& c : p.classes) {
    c.item_off = p.items.size();
    c.cost = 0.0;
    for (int j : c.jobs) {
      const JobDesc& d = p.descs[j];
      for (int y0 = 0; y0 < d.height; y0 += c.tc.th)
        for (int x0 = 0; x0 < d.width; x0 += c.tc.cols) {
          p.items.push_back(make_int4(j, x0, y0, 0));
          c.cost += (4.0 * d.K + 1.0) * c.tc.th * c.tc.cols;
        }
    }
    c.n_items = static_cast<int>(p.items.size() - c.item_off);
  }
}

int build_plan(const bf_job* jobs, int n_jobs, bf_planes prec, PlanData& p) {
  if (!jobs || n_jobs < 1) return fail(BF_E_INVALID, "jobs must be non-NULL and n_jobs >= 1");
  if (!valid_prec(prec)) return fail(BF_E_INVALID, "unknown plane precision");
  p = PlanData{};
  p.prec = prec;
  const int grid_env = grid_mode_from_env();
  const int th_env = tile_rows_from_env();
  p.descs.resize(n_jobs);
  std::map<long, ClassLaunch> by_class;  // key (nt, family)
  for (int i = 0; i < n_jobs; ++i) {
    Resolved r;
    const int rc = resolve_job(&jobs[i], &r);
    if (rc < 0) {
      set_error("job " + std::to_string(i) + ": " + bf_last_error());
      return rc;
    }
    if (r.status > p.status) p.status = r.status;
    p.descs[i] = r.desc;
    const int nt = window_tiles(r.desc.W);
    // the family is the one the shortest tile gets; taller tiles are options
    // when every job of the class supports them with the same family
    const TileChoice base = choose_tile(r.desc, prec, 32);
    ClassLaunch& c = by_class[(long)nt * 10 + base.family];
    if (c.jobs.empty()) {
      c.nt = nt;
      c.family = base.family;
      c.tc = base;
      c.tc.offsets16 = false;
      for (int th : {32, 64, 96, 128, 144}) {
        const TileChoice t = choose_tile(r.desc, prec, th);
        if (t.th == th && t.family == base.family) c.th_options.push_back(th);
      }
    } else {
      std::vector<int> keep;
      for (int th : c.th_options) {
        const TileChoice t = choose_tile(r.desc, prec, th);
        if (t.th == th && t.family == base.family) keep.push_back(th);
      }
      c.th_options = keep;
    }
    c.jobs.push_back(i);
    c.tc.offsets16 = c.tc.offsets16 || base.offsets16;
    c.t_max = std::max(c.t_max, r.desc.T);
    c.f_max = std::max(c.f_max, r.desc.F);
    c.px += (double)r.desc.height * r.desc.width;
  }
  size_t max_items = 0;
  for (auto& kv : by_class) {
    ClassLaunch c = kv.second;
    if (c.th_options.empty()) c.th_options.push_back(32);
    std::stable_sort(c.jobs.begin(), c.jobs.end(), [&](int a, int b) { return p.descs[a].K > p.descs[b].K; });
    // default geometry: the tallest tile the class supports (for fp32 planes
    // 32 rows with windows wider than 6 row tiles, which spill registers at
    // taller tiles), unless the environment or an earlier tuning run says
    // otherwise
    int th = th_env ? th_env : prec != BF_PLANES_FP32 ? 128 : c.nt >= 7 ? 32 : 128;
    int grid = grid_env;
    if (!th_env && !grid_env) {
      std::lock_guard<std::mutex> lock(g_tune_mutex);
      auto it = g_tune->find(tune_key(prec, c));
      if (it != g_tune->end()) {
        th = it->second.th;
        grid = it->second.grid;
        c.tuned = true;
      }
    }
    int pick = c.th_options.front();
    for (int o : c.th_options)
      if (o <= th) pick = o;
    c.tc.th = pick;
    c.grid = grid;
    size_t most = 0;
    for (int j : c.jobs) most += items_of(p.descs[j], c.th_options.front(), c.tc.cols);
    max_items += most;
    p.classes.push_back(std::move(c));
  }
  if (max_items > (size_t)INT32_MAX) return fail(BF_E_UNSUPPORTED, "too many tiles in one batch");
  // every job's output must be disjoint from every other job's input and
  // output: the launches write all images concurrently
  {
    struct Span {
      uintptr_t lo, hi;
      int job;
      bool out;
    };
    std::vector<Span> spans;
    spans.reserve(2 * (size_t)n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
      const JobDesc& d = p.descs[i];
      const uintptr_t s0 = reinterpret_cast<uintptr_t>(d.src), d0 = reinterpret_cast<uintptr_t>(d.dst);
      spans.push_back({s0, s0 + sizeof(float) * ((size_t)(d.height - 1) * d.src_pitch + d.width), i, false});
      spans.push_back({d0, d0 + sizeof(float) * ((size_t)(d.height - 1) * d.dst_pitch + d.width), i, true});
    }
    std::sort(spans.begin(), spans.end(), [](const Span& a, const Span& b) { return a.lo < b.lo; });
    // sweep: an output span may not intersect any other span (inputs may
    // share memory with inputs).  Tracking only the farthest-reaching open
    // span suffices because resolve_job has already rejected a job whose own
    // src and dst hulls meet: an open span of the current span's own job
    // cannot reach past its start, so the farthest one, when it does, is
    // another job's.
    size_t best_out = SIZE_MAX;  // index of the open output span reaching farthest
    uintptr_t reach_any = 0, reach_out = 0;
    int job_any = -1;
    for (size_t k = 0; k < spans.size(); ++k) {
      const Span& sp = spans[k];
      const bool hits_out = best_out != SIZE_MAX && sp.lo < reach_out && spans[best_out].job != sp.job;
      const bool out_hits_any = sp.out && sp.lo < reach_any && job_any != sp.job;
      if (hits_out || out_hits_any)
        return fail(BF_E_INVALID, "job " + std::to_string(sp.job) + ": an output overlaps another job's image");
      if (sp.hi > reach_any) {
        reach_any = sp.hi;
        job_any = sp.job;
      }
      if (sp.out && sp.hi > reach_out) {
        reach_out = sp.hi;
        best_out = k;
      }
    }
  }
  emit_items(p);
  // most expensive class first: when launched one after another its tail is
  // followed by cheaper work
  std::stable_sort(p.classes.begin(), p.classes.end(),
                   [](const ClassLaunch& a, const ClassLaunch& b) { return a.cost > b.cost; });
  emit_items(p);
  p.items_off = align_up(sizeof(JobDesc) * (size_t)n_jobs, 256);
  p.ws_bytes = p.items_off + sizeof(int4) * max_items;
  return BF_OK;
}

// ---- pinned staging of the job table --------------------------------------
struct StagingSlot {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  int device = -1;
  bool recorded = false;  // ev recorded behind the last copy
  bool retired = false;   // read by a captured copy node: never reused
};

std::mutex g_staging_mutex;
std::vector<StagingSlot*>* g_staging = new std::vector<StagingSlot*>();  // never freed (see top)

int stream_device(hipStream_t s, int* dev) {
  hipError_t e = s ? hipStreamGetDevice(s, dev) : hipGetDevice(dev);
  if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("cannot query the stream's device: ") + hipGetErrorString(e));
  return BF_OK;
}

struct DeviceGuard {
  int saved = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&saved) != hipSuccess) saved = -1;
    if (saved != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (saved >= 0 && hipGetDevice(&cur) == hipSuccess && cur != saved) (void)hipSetDevice(saved);
  }
};

// Copies the plan's table into `workspace` on `stream` (asynchronously);
// *device_out receives the stream's device.  Arguments are checked before any
// HIP call.
int upload_table(const PlanData& p, void* workspace, size_t ws_bytes, hipStream_t stream, int* device_out) {
  if (!workspace) return fail(BF_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < p.ws_bytes)
    return fail(BF_E_WORKSPACE, "workspace smaller than bf_workspace_bytes() = " + std::to_string(p.ws_bytes));
  if (reinterpret_cast<uintptr_t>(workspace) % 16 != 0)
    return fail(BF_E_WORKSPACE, "workspace must be 16-byte aligned");
  int dev = 0;
  int rc = stream_device(stream, &dev);
  if (rc != BF_OK) return rc;
  if (device_out) *device_out = dev;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (stream && hipStreamIsCapturing(stream, &cs) != hipSuccess) cs = hipStreamCaptureStatusNone;

  std::lock_guard<std::mutex> lock(g_staging_mutex);
  StagingSlot* slot = nullptr;
  for (StagingSlot* s : *g_staging) {
    if (s->retired || s->device != dev || s->cap < p.ws_bytes) continue;
    if (s->recorded) {
      const hipError_t q = hipEventQuery(s->ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) continue;  // leave a slot with a failed event alone
    }
    slot = s;
    break;
  }
  if (!slot) {
    DeviceGuard g(dev);
    slot = new StagingSlot();
    slot->device = dev;
    slot->cap = align_up(std::max<size_t>(p.ws_bytes, 64 << 10), 4096);
    hipError_t e = hipHostMalloc(&slot->host, slot->cap, hipHostMallocPortable);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&slot->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (slot->host) (void)hipHostFree(slot->host);
      delete slot;
      return fail(BF_E_DEVICE, std::string("pinned staging allocation failed: ") + hipGetErrorString(e));
    }
    g_staging->push_back(slot);
  }
  unsigned char* h = static_cast<unsigned char*>(slot->host);
  std::memcpy(h, p.descs.data(), sizeof(JobDesc) * p.descs.size());
  std::memset(h + sizeof(JobDesc) * p.descs.size(), 0, p.items_off - sizeof(JobDesc) * p.descs.size());
  std::memcpy(h + p.items_off, p.items.data(), sizeof(int4) * p.items.size());
  const size_t used = p.items_off + sizeof(int4) * p.items.size();
  hipError_t e = hipMemcpyAsync(workspace, h, used, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("job table copy failed: ") + hipGetErrorString(e));
  if (cs != hipStreamCaptureStatusNone) {
    slot->retired = true;
    slot->recorded = false;
  } else {
    e = hipEventRecord(slot->ev, stream);
    if (e != hipSuccess) {
      slot->retired = true;  // cannot tell when the copy ends
      return fail(BF_E_DEVICE, std::string("event record failed: ") + hipGetErrorString(e));
    }
    slot->recorded = true;
  }
  return BF_OK;
}

int launch_class(const PlanData& p, const ClassLaunch& c, const void* workspace, hipStream_t stream) {
  const unsigned char* ws = static_cast<const unsigned char*>(workspace);
  const JobDesc* jobs = reinterpret_cast<const JobDesc*>(ws);
  const int4* items = reinterpret_cast<const int4*>(ws + p.items_off) + c.item_off;
  const int grid = c.grid < 0 ? c.n_items : c.grid;
  hipError_t e = launch_batched(jobs, items, c.n_items, c.t_max, c.f_max, p.prec, c.nt, c.tc, grid, stream);
  if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("batched kernel launch failed: ") + hipGetErrorString(e));
  return BF_OK;
}

int launch_all(const PlanData& p, const void* workspace, hipStream_t stream) {
  for (const ClassLaunch& c : p.classes) {
    int rc = launch_class(p, c, workspace, stream);
    if (rc != BF_OK) return rc;
  }
  return BF_OK;
}

}  // namespace
}  // namespace bf

using namespace bf;

struct bf_plan {
  PlanData p;
  void* ws = nullptr;   // device workspace of the last upload
  size_t ws_cap = 0;    // its size
  int device = -1;
  // graph form: classes as independent kernel nodes of one graph
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipEvent_t done = nullptr;
  bool launched = false;

  void drop_graph() {
    if (exec) {
      if (launched && done) (void)hipEventSynchronize(done);
      (void)hipGraphExecDestroy(exec);
      exec = nullptr;
    }
    launched = false;
  }
  ~bf_plan() {
    drop_graph();
    for (hipStream_t s : side) (void)hipStreamDestroy(s);
    for (hipEvent_t e : join) (void)hipEventDestroy(e);
    if (capture) (void)hipStreamDestroy(capture);
    if (fork) (void)hipEventDestroy(fork);
    if (done) (void)hipEventDestroy(done);
  }

  // Captures the class launches on library streams: class 0 on the capture
  // stream, every other class on a side stream forked from it and joined back,
  // so the graph holds them as independent nodes that may run concurrently.
  int build_graph() {
    DeviceGuard g(device);
    hipError_t e = hipSuccess;
    if (!capture) e = hipStreamCreateWithFlags(&capture, hipStreamNonBlocking);
    if (e == hipSuccess && !fork) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess && !done) e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    while (e == hipSuccess && side.size() + 1 < p.classes.size()) {
      hipStream_t s = nullptr;
      hipEvent_t ev = nullptr;
      e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
      if (e != hipSuccess) break;
      side.push_back(s);
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) break;
      join.push_back(ev);
    }
    if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("graph resources: ") + hipGetErrorString(e));
    e = hipStreamBeginCapture(capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("stream capture: ") + hipGetErrorString(e));
    int rc = BF_OK;
    if (p.classes.size() > 1) {
      e = hipEventRecord(fork, capture);
      if (e != hipSuccess) rc = fail(BF_E_DEVICE, std::string("capture fork: ") + hipGetErrorString(e));
    }
    for (size_t c = 0; rc == BF_OK && c < p.classes.size(); ++c) {
      hipStream_t s = c == 0 ? capture : side[c - 1];
      if (c > 0 && (e = hipStreamWaitEvent(s, fork, 0)) != hipSuccess) {
        rc = fail(BF_E_DEVICE, std::string("capture fork: ") + hipGetErrorString(e));
        break;
      }
      rc = launch_class(p, p.classes[c], ws, s);
      if (rc == BF_OK && c > 0) {
        e = hipEventRecord(join[c - 1], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(capture, join[c - 1], 0);
        if (e != hipSuccess) rc = fail(BF_E_DEVICE, std::string("capture join: ") + hipGetErrorString(e));
      }
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(capture, &graph);
    if (rc == BF_OK && e != hipSuccess) rc = fail(BF_E_DEVICE, std::string("end capture: ") + hipGetErrorString(e));
    if (rc == BF_OK) {
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        exec = nullptr;
        rc = fail(BF_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
      }
    }
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
};

extern "C" size_t bf_workspace_bytes(const bf_job* jobs, int n_jobs, bf_planes prec) {
  PlanData p;
  if (build_plan(jobs, n_jobs, prec, p) < 0) return (size_t)-1;
  return p.ws_bytes;
}

extern "C" int bf_filter_batched(const bf_job* jobs, int n_jobs, bf_planes prec, void* workspace,
                                 size_t ws_bytes, void* hip_stream) {
  PlanData p;
  int rc = build_plan(jobs, n_jobs, prec, p);
  if (rc < 0) return rc;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  rc = upload_table(p, workspace, ws_bytes, stream, nullptr);
  if (rc < 0) return rc;
  rc = launch_all(p, workspace, stream);
  if (rc < 0) return rc;
  if (p.status != BF_OK) set_error("a fit stopped at K_max with ||b - A d|| > eps");
  return p.status;
}

namespace bf {
int filter_batched_pageable(const bf_job* jobs, int n_jobs, bf_planes prec, size_t table_cap, const char* cap_name,
                            int (*table_of)(hipStream_t, void**), hipStream_t stream) {
  PlanData p;
  int rc = build_plan(jobs, n_jobs, prec, p);
  if (rc < 0) return rc;
  if (p.ws_bytes > table_cap)
    return fail(BF_E_UNSUPPORTED, "the job table and tiles need " + std::to_string(p.ws_bytes) +
                                      " bytes, more than " + cap_name + " = " + std::to_string(table_cap));
  void* table_dev = nullptr;
  rc = table_of(stream, &table_dev);
  if (rc != BF_OK) return rc;
  // the table in ordinary host memory; a copy from pageable memory has been
  // read out of it by the time hipMemcpyAsync returns
  std::vector<unsigned char> host(p.items_off + sizeof(int4) * p.items.size(), 0);
  std::memcpy(host.data(), p.descs.data(), sizeof(JobDesc) * p.descs.size());
  std::memcpy(host.data() + p.items_off, p.items.data(), sizeof(int4) * p.items.size());
  hipError_t e = hipMemcpyAsync(table_dev, host.data(), host.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("job table copy failed: ") + hipGetErrorString(e));
  rc = launch_all(p, table_dev, stream);
  if (rc < 0) return rc;
  if (p.status != BF_OK) set_error("a fit stopped at K_max with ||b - A d|| > eps");
  return p.status;
}
}  // namespace bf

extern "C" int bf_plan_create(const bf_job* jobs, int n_jobs, bf_planes prec, bf_plan** plan) {
  if (!plan) return fail(BF_E_INVALID, "plan must be non-NULL");
  *plan = nullptr;
  bf_plan* pl = new bf_plan();
  int rc = build_plan(jobs, n_jobs, prec, pl->p);
  if (rc < 0) {
    delete pl;
    return rc;
  }
  *plan = pl;
  if (pl->p.status != BF_OK) set_error("a fit stopped at K_max with ||b - A d|| > eps");
  return pl->p.status;
}

extern "C" size_t bf_plan_workspace_bytes(const bf_plan* plan) { return plan ? plan->p.ws_bytes : (size_t)-1; }

extern "C" int bf_plan_upload(bf_plan* plan, void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!plan) return fail(BF_E_INVALID, "plan is NULL");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int dev = -1;
  const int rc = upload_table(plan->p, workspace, ws_bytes, stream, &dev);
  if (rc != BF_OK) return rc;
  plan->drop_graph();  // the table may have changed
  plan->ws = workspace;
  plan->ws_cap = ws_bytes;
  plan->device = dev;
  return BF_OK;
}

extern "C" int bf_plan_launch(bf_plan* plan, void* hip_stream, int use_graph) {
  if (!plan) return fail(BF_E_INVALID, "plan is NULL");
  if (!plan->ws) return fail(BF_E_INVALID, "bf_plan_upload must precede bf_plan_launch");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  int rc = stream_device(stream, &dev);
  if (rc != BF_OK) return rc;
  if (dev != plan->device) return fail(BF_E_INVALID, "stream belongs to another device than the uploaded table");
  if (!use_graph) return launch_all(plan->p, plan->ws, stream);
  if (!plan->exec) {
    rc = plan->build_graph();
    if (rc != BF_OK) return rc;
  }
  hipError_t e = hipGraphLaunch(plan->exec, stream);
  if (e == hipSuccess) e = hipEventRecord(plan->done, stream);
  if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("graph launch failed: ") + hipGetErrorString(e));
  plan->launched = true;
  return BF_OK;
}

extern "C" void bf_plan_destroy(bf_plan* plan) { delete plan; }

extern "C" int bf_plan_tune(bf_plan* plan, void* hip_stream, int reps) {
  if (!plan) return fail(BF_E_INVALID, "plan is NULL");
  if (!plan->ws) return fail(BF_E_INVALID, "bf_plan_upload must precede bf_plan_tune");
  if (reps < 1 || reps > 1000) return fail(BF_E_INVALID, "reps must satisfy 1 <= reps <= 1000");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  int rc = stream_device(stream, &dev);
  if (rc != BF_OK) return rc;
  if (dev != plan->device) return fail(BF_E_INVALID, "stream belongs to another device than the uploaded table");
  PlanData& p = plan->p;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  {
    DeviceGuard g(dev);
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return fail(BF_E_DEVICE, std::string("event create: ") + hipGetErrorString(e));
    }
  }
  auto time_class = [&](const ClassLaunch& c, float* ms) -> int {
    int r = upload_table(p, plan->ws, plan->ws_cap, stream, nullptr);
    if (r == BF_OK) r = launch_class(p, c, plan->ws, stream);  // warm-up
    if (r != BF_OK) return r;
    hipError_t e = hipEventRecord(e0, stream);
    for (int i = 0; e == hipSuccess && i < reps; ++i) {
      r = launch_class(p, c, plan->ws, stream);
      if (r != BF_OK) return r;
    }
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("tuning run failed: ") + hipGetErrorString(e));
    return BF_OK;
  };
  for (ClassLaunch& c : p.classes) {
    float best = 0.f;
    int best_th = c.tc.th, best_grid = c.grid;
    bool have = false;
    for (int th : c.th_options) {
      for (int grid : {0, -1}) {
        c.tc.th = th;
        c.grid = grid;
        emit_items(p);
        float ms = 0.f;
        rc = time_class(c, &ms);
        if (rc != BF_OK) break;
        if (!have || ms < best) {
          best = ms;
          best_th = th;
          best_grid = grid;
          have = true;
        }
      }
      if (rc != BF_OK) break;
    }
    c.tc.th = best_th;
    c.grid = best_grid;
    if (rc != BF_OK) break;
    c.tuned = true;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    (*g_tune)[tune_key(p.prec, c)] = TuneVal{best_th, best_grid};
  }
  emit_items(p);
  const int rc2 = upload_table(p, plan->ws, plan->ws_cap, stream, nullptr);
  plan->drop_graph();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc != BF_OK ? rc : rc2;
}

extern "C" int bf_plan_describe(const bf_plan* plan, char* buf, size_t len) {
  if (!plan) return fail(BF_E_INVALID, "plan is NULL");
  std::string out = "{\"planes\": " + std::to_string(static_cast<int>(plan->p.prec)) +
                    ", \"jobs\": " + std::to_string(plan->p.descs.size()) +
                    ", \"workspace_bytes\": " + std::to_string(plan->p.ws_bytes) + ", \"classes\": [";
  for (size_t i = 0; i < plan->p.classes.size(); ++i) {
    const ClassLaunch& c = plan->p.classes[i];
    out += (i ? ", " : "");
    out += "{\"nt\": " + std::to_string(c.nt) + ", \"family\": " + std::to_string(c.family) +
           ", \"tile_rows\": " + std::to_string(c.tc.th) + ", \"tile_cols\": " + std::to_string(c.tc.cols) +
           ", \"grid\": " + std::to_string(c.grid) + ", \"items\": " + std::to_string(c.n_items) +
           ", \"jobs\": " + std::to_string(c.jobs.size()) + ", \"t_max\": " + std::to_string(c.t_max) +
           ", \"f_max\": " + std::to_string(c.f_max) +
           ", \"tuned\": " + (c.tuned ? "true" : "false") + "}";
  }
  out += "]}";
  if (buf && len > 0) {
    const size_t n = std::min(len - 1, out.size());
    std::memcpy(buf, out.data(), n);
    buf[n] = '\0';
  }
  return static_cast<int>(out.size());
}

// ---- persistence of the tuned geometry -------------------------------------
// Text file: a header line "bf-tune 1", then one line per entry:
//   planes window_class family round(log2(pixels)) tile_rows grid
extern "C" int bf_tune_save(const char* path) {
  if (!path) return fail(BF_E_INVALID, "path is NULL");
  std::ofstream out(path, std::ios::trunc);
  if (!out) return fail(BF_E_INVALID, std::string("cannot write ") + path);
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  out << "bf-tune 1\n";
  for (const auto& kv : *g_tune)
    out << kv.first.prec << ' ' << kv.first.nt << ' ' << kv.first.family << ' ' << kv.first.size_log2 << ' '
        << kv.second.th << ' ' << kv.second.grid << '\n';
  if (!out) return fail(BF_E_INVALID, std::string("write failed: ") + path);
  return BF_OK;
}

extern "C" int bf_tune_load(const char* path) {
  if (!path) return fail(BF_E_INVALID, "path is NULL");
  std::ifstream in(path);
  if (!in) return fail(BF_E_INVALID, std::string("cannot read ") + path);
  std::string line;
  if (!std::getline(in, line) || line != "bf-tune 1") return fail(BF_E_INVALID, "not a bf-tune 1 file");
  std::map<TuneKey, TuneVal> entries;
  int lineno = 1;
  while (std::getline(in, line)) {
    ++lineno;
    if (line.empty()) continue;
    std::istringstream ls(line);
    TuneKey k{};
    TuneVal v{};
    std::string rest;
    if (!(ls >> k.prec >> k.nt >> k.family >> k.size_log2 >> v.th >> v.grid) || (ls >> rest) ||
        k.prec < 0 || k.prec > 2 || k.nt < 2 || k.nt > 9 || k.family < 0 || k.family > 2 ||
        !valid_tile_rows(v.th) || v.grid < -1)
      return fail(BF_E_INVALID, std::string("bad entry on line ") + std::to_string(lineno) + " of " + path);
    entries[k] = v;
  }
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  for (const auto& kv : entries) (*g_tune)[kv.first] = kv.second;
  return static_cast<int>(entries.size());
}

extern "C" void bf_tune_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  g_tune->clear();
}
