// Batched reconstruction of independent slices (the slices of a volume or a
// multi-slice protocol are independent problems that the paper solves in
// parallel, Section 3.4): one plan per slice, any mix of geometries.
//
// A CG iteration of every slice is captured once into one HIP graph and the
// graph is replayed for every iteration.  The per-iteration state (the
// iteration count that selects the residual slot and the history entry) is
// device-resident, so the same graph serves every iteration.  Slices are
// dealt to a few streams (longest first onto the least-loaded stream) so that
// the operator kernels of different slices overlap inside the graph; the CG
// vector steps of all slices then run as work-list kernels, one launch per
// step for the whole batch, whose items are (slice, block) pairs.  Set-up
// (E'^H y, the first residual) and the copy-out run eagerly on the lanes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "../../include/gpjc.h"
#include "plan.h"


struct gpjc_batch {
  std::vector<gpjc_plan*> plans;
  std::vector<int> lane_of;
  std::vector<hipStream_t> lanes;
  hipStream_t origin = nullptr;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  struct Graph {
    hipGraphExec_t exec = nullptr;
    long gen = -1;
  };
  Graph graphs[3][2];  // [precision][refresh iteration]
  std::vector<gpjc::CgSlice> h_list;  // the slices' CG vectors, for the work-list kernels
  gpjc::CgSlice* d_list = nullptr;
  int list_grid = 1024;  // persistent grid of the work-list kernels
};

namespace gpjc {

namespace {

void destroy_batch(gpjc_batch* b) {
  for (auto& row : b->graphs)
    for (auto& g : row)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
  for (hipEvent_t e : b->join)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipStream_t s : b->lanes)
    if (s) (void)hipStreamDestroy(s);
  if (b->origin) (void)hipStreamDestroy(b->origin);
  if (b->d_list) (void)hipFree(b->d_list);
  delete b;
}

long config_generation(const gpjc_batch& b) {
  long g = 0;
  for (const gpjc_plan* p : b.plans) g += p->config_gen;
  return g;
}

// Plans run on their lane streams (and without stage timing) while the batch
// works; the caller's settings come back when this goes out of scope.
struct LaneBinding {
  gpjc_batch& b;
  std::vector<hipStream_t> streams;
  std::vector<char> timing;
  explicit LaneBinding(gpjc_batch& bb) : b(bb) {
    for (size_t i = 0; i < b.plans.size(); ++i) {
      streams.push_back(b.plans[i]->stream);
      timing.push_back(b.plans[i]->timing.on);
      b.plans[i]->stream = b.lanes[b.lane_of[i]];
      b.plans[i]->timing.on = false;
    }
  }
  ~LaneBinding() {
    for (size_t i = 0; i < b.plans.size(); ++i) {
      b.plans[i]->stream = streams[i];
      b.plans[i]->timing.on = timing[i];
    }
  }
};

// origin -> every lane
int fork_lanes(gpjc_batch& b) {
  GPJC_HIP(hipEventRecord(b.fork, b.origin));
  for (hipStream_t s : b.lanes) GPJC_HIP(hipStreamWaitEvent(s, b.fork, 0));
  return GPJC_OK;
}
// every lane -> origin
int join_lanes(gpjc_batch& b) {
  for (size_t l = 0; l < b.lanes.size(); ++l) {
    GPJC_HIP(hipEventRecord(b.join[l], b.lanes[l]));
    GPJC_HIP(hipStreamWaitEvent(b.origin, b.join[l], 0));
  }
  return GPJC_OK;
}

// The operator part of every slice on the lanes, then back on origin.
int lanes_op_part(gpjc_batch& b, Store st, int phase) {
  int status = fork_lanes(b);
  for (size_t i = 0; status == GPJC_OK && i < b.plans.size(); ++i) status = cg_op_part(*b.plans[i], st, phase);
  if (status == GPJC_OK) status = join_lanes(b);
  return status;
}

int list_step(gpjc_batch& b, int op) {
  return launch_cg_list(b.d_list, (int)b.plans.size(), op, b.list_grid, b.origin);
}

int capture_iteration(gpjc_batch& b, Store st, bool refresh, hipGraphExec_t* exec) {
  GPJC_HIP(hipStreamBeginCapture(b.origin, hipStreamCaptureModeThreadLocal));
  int status = lanes_op_part(b, st, 0);
  if (status == GPJC_OK) status = list_step(b, kCgListQ);
  if (status == GPJC_OK) status = list_step(b, kCgListUpdate);
  if (refresh) {
    if (status == GPJC_OK) status = lanes_op_part(b, st, 1);
    if (status == GPJC_OK) status = list_step(b, kCgListStart);
    if (status == GPJC_OK) status = list_step(b, kCgListNorm);
  } else if (status == GPJC_OK) {
    status = list_step(b, kCgListDir);
  }
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(b.origin, &graph);
  if (status == GPJC_OK && e != hipSuccess) status = fail(GPJC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  if (status == GPJC_OK) {
    const hipError_t ei = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) status = fail(GPJC_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
  }
  if (graph) (void)hipGraphDestroy(graph);
  return status;
}

int get_graph(gpjc_batch& b, Store st, bool refresh, hipGraphExec_t* exec) {
  gpjc_batch::Graph& g = b.graphs[static_cast<int>(st)][refresh ? 1 : 0];
  const long gen = config_generation(b);
  if (g.exec && g.gen != gen) {
    GPJC_HIP(hipGraphExecDestroy(g.exec));
    g.exec = nullptr;
  }
  if (!g.exec) {
    GPJC_TRY(capture_iteration(b, st, refresh, &g.exec));
    g.gen = gen;
  }
  *exec = g.exec;
  return GPJC_OK;
}

}  // namespace
}  // namespace gpjc

using namespace gpjc;

extern "C" {

int gpjc_batch_create(gpjc_plan* const* plans, int n, int lanes, gpjc_batch** out) {
  if (!out) return fail(GPJC_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!plans || n < 1) return fail(GPJC_E_INVAL, "a batch needs at least one plan");
  if (lanes < 0) return fail(GPJC_E_INVAL, "lanes must be >= 0");
  std::set<const gpjc_plan*> seen;
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return fail(GPJC_E_INVAL, "plan " + std::to_string(i) + " is NULL");
    if (!seen.insert(plans[i]).second) return fail(GPJC_E_INVAL, "plan " + std::to_string(i) + " appears twice");
  }
  const int nl = std::max(1, std::min(lanes == 0 ? 4 : lanes, std::min(n, 16)));
  gpjc_batch* b = new gpjc_batch();
  b->plans.assign(plans, plans + n);
  // longest slice first onto the least-loaded lane
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  auto work = [&](int i) {
    const Plan& p = *plans[i];
    return (double)p.B * p.nc * p.ny * p.nt;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work(a) > work(c); });
  std::vector<double> load(nl, 0.0);
  b->lane_of.assign(n, 0);
  for (int i : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->lane_of[i] = l;
    load[l] += work(i);
  }
  hipError_t e = hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking);
  for (int l = 0; e == hipSuccess && l < nl; ++l) {
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    b->lanes.push_back(s);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int l = 0; e == hipSuccess && l < nl; ++l) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    b->join.push_back(ev);
  }
  if (e == hipSuccess) e = hipMalloc(&b->d_list, sizeof(CgSlice) * n);
  int cus = 0;
  if (e == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0) == hipSuccess && cus > 0)
    b->list_grid = 4 * cus;
  if (e != hipSuccess) {
    destroy_batch(b);
    return fail(GPJC_E_DEVICE, std::string("batch streams: ") + hipGetErrorString(e));
  }
  *out = b;
  return GPJC_OK;
}

int gpjc_batch_destroy(gpjc_batch* batch) {
  if (!batch) return fail(GPJC_E_INVAL, "batch is NULL");
  (void)hipStreamSynchronize(batch->origin);
  destroy_batch(batch);
  return GPJC_OK;
}

int gpjc_batch_lanes(const gpjc_batch* batch, int* h_lane_of) {
  if (!batch) return fail(GPJC_E_INVAL, "batch is NULL");
  if (h_lane_of) std::copy(batch->lane_of.begin(), batch->lane_of.end(), h_lane_of);
  return (int)batch->lanes.size();
}

int gpjc_batch_recon_cg(gpjc_batch* batch, gpjc_prec prec, const gpjc_c64* const* d_y, gpjc_c64* const* d_x,
                        int iters, int refine_every, double* h_resid) {
  TraceRange trace("gpjc_batch_recon_cg");
  if (!batch) return fail(GPJC_E_INVAL, "batch is NULL");
  if (!d_y || !d_x) return fail(GPJC_E_INVAL, "pointer arrays are NULL");
  if (refine_every < 0) return fail(GPJC_E_INVAL, "refine_every must be >= 0");
  gpjc_batch& b = *batch;
  const int n = (int)b.plans.size();
  Store st = Store::F32;
  for (int i = 0; i < n; ++i) {
    const Plan& pl = *b.plans[i];
    GPJC_TRY(check_prec(pl, prec, &st));
    GPJC_TRY(check_bank(pl));
    if (iters < 0 || iters + 1 > pl.hist_cap) return fail(GPJC_E_INVAL, "iters out of range");
    if (!d_y[i] || !d_x[i]) return fail(GPJC_E_INVAL, "slice " + std::to_string(i) + ": NULL buffer");
    if (reinterpret_cast<uintptr_t>(d_y[i]) % 8 || reinterpret_cast<uintptr_t>(d_x[i]) % 8)
      return fail(GPJC_E_INVAL, "slice " + std::to_string(i) + ": buffers must be 8-byte aligned");
  }
  const bool refine = refine_every > 0 && is_16bit(st);
  // Work queued by the caller on the plans' own streams comes first.
  for (int i = 0; i < n; ++i) GPJC_HIP(hipStreamSynchronize(b.plans[i]->stream));
  std::vector<int> flags(n, 0);
  int status = GPJC_OK;
  {
    LaneBinding bind(b);
    // the slices' vectors for the work-list kernels (the graphs read the list
    // when they run)
    b.h_list.resize(n);
    for (int i = 0; i < n; ++i) b.h_list[i] = cg_slice_of(*b.plans[i]);
    const hipError_t ec =
        hipMemcpyAsync(b.d_list, b.h_list.data(), sizeof(CgSlice) * n, hipMemcpyHostToDevice, b.origin);
    if (ec != hipSuccess) return fail(GPJC_E_DEVICE, std::string("batch list: ") + hipGetErrorString(ec));
    status = fork_lanes(b);
    for (int i = 0; status == GPJC_OK && i < n; ++i)
      status = cg_setup(*b.plans[i], st, refine, reinterpret_cast<const float2*>(d_y[i]),
                        reinterpret_cast<const float2*>(d_x[i]));
    if (status == GPJC_OK) status = join_lanes(b);
    hipGraphExec_t g_plain = nullptr, g_refresh = nullptr;
    if (status == GPJC_OK && iters > 0) status = get_graph(b, st, false, &g_plain);
    if (status == GPJC_OK && refine && iters > refine_every) status = get_graph(b, st, true, &g_refresh);
    for (int it = 0; status == GPJC_OK && it < iters; ++it) {
      const hipError_t e = hipGraphLaunch(cg_refresh_at(it, iters, refine_every, st) ? g_refresh : g_plain, b.origin);
      if (e != hipSuccess) status = fail(GPJC_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
    }
    if (status == GPJC_OK) status = fork_lanes(b);
    for (int i = 0; status == GPJC_OK && i < n; ++i)
      status = cg_finish(*b.plans[i], reinterpret_cast<float2*>(d_x[i]), iters,
                         h_resid ? h_resid + (size_t)i * (iters + 1) : nullptr, &flags[i]);
    if (status == GPJC_OK) status = join_lanes(b);
    const hipError_t e = hipStreamSynchronize(b.origin);
    if (status == GPJC_OK && e != hipSuccess) status = fail(GPJC_E_DEVICE, hipGetErrorString(e));
  }
  if (status != GPJC_OK) return status;
  for (int i = 0; i < n; ++i)
    if (flags[i]) return fail(GPJC_E_NUMERIC, "CG: non-finite residual or curvature in slice " + std::to_string(i));
  return GPJC_OK;
}

int gpjc_autotune(gpjc_plan* plan, gpjc_prec prec, const char* cache_path, int* h_choice) {
  TraceRange trace("gpjc_autotune");
  if (!plan) return fail(GPJC_E_INVAL, "plan is NULL");
  if (plan->general) return fail(GPJC_E_UNSUPPORTED, "modulation-map plans have no group contraction to tune");
  Store st = Store::F32;
  GPJC_TRY(check_prec(*plan, prec, &st));
  GPJC_TRY(check_bank(*plan));
  return autotune(*plan, st, cache_path, h_choice);
}

int gpjc_batch_autotune(gpjc_batch* batch, gpjc_prec prec, const char* cache_path) {
  TraceRange trace("gpjc_batch_autotune");
  if (!batch) return fail(GPJC_E_INVAL, "batch is NULL");
  for (gpjc_plan* p : batch->plans) GPJC_TRY(gpjc_autotune(p, prec, cache_path, nullptr));
  return GPJC_OK;
}

}  // extern "C"
