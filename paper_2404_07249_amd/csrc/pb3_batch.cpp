// Batched execution: many fields through one or more plans.
//
// Jobs that share a plan object are launched together, up to kMaxJobs per
// kernel launch (grid dimension z = job, each job with its own slice of
// one workspace allocation).  Groups of different plans are spread over a
// few internal streams (longest-first onto the least-loaded stream), forked
// from and joined back into the caller's stream.  With PB3_BATCH_GRAPH the
// fork, every group's launch sequence and the join are captured once into
// a HIP graph that later runs replay; a run with different pointers or
// precision captures again and updates the executable graph in place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "pb3_internal.h"

namespace {

constexpr int kBatchStreams = 4;

struct Group {
  pb3_plan* plan = nullptr;
  std::vector<int> jobs;   // indices into the batch's job list
  size_t stride = 0;       // workspace bytes per job
  size_t offset = 0;       // byte offset of job 0's workspace in the batch allocation
  int stream = 0;          // internal stream index
  double cost = 0;         // relative cost estimate
};

}  // namespace

struct pb3_batch {
  unsigned flags = 0;
  int device_id = 0;
  int n_jobs = 0;
  std::vector<Group> groups;
  int n_streams = 0;
  std::vector<hipStream_t> streams;  // group streams
  hipStream_t cap = nullptr;         // capture origin
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  size_t ws_bytes = 0;
  void* ws_base = nullptr;
  bool ws_owned = false;
  // captured graph and the arguments it was captured with
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;
};

namespace pb3 {

static double plan_cost(const pb3_plan& p) {
  const double n3 = (double)npix(p), m3 = (double)mpix(p);
  const double pairs = (double)p.nb_pad * (p.nb_pad + 1) / 2;
  // forward FFT bytes plus the contraction's pair x bin products
  return 40.0 * n3 + pairs * p.nb_pad * m3 / 64.0;
}

static void release(pb3_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  for (hipStream_t s : b->streams)
    if (s) hipStreamDestroy(s);
  if (b->cap) hipStreamDestroy(b->cap);
  if (b->fork) hipEventDestroy(b->fork);
  for (hipEvent_t e : b->join)
    if (e) hipEventDestroy(e);
  if (b->ws_owned && b->ws_base) hipFree(b->ws_base);
}

static void set_workspace(pb3_batch* b, void* base, bool owned) {
  if (b->ws_owned && b->ws_base) hipFree(b->ws_base);
  b->ws_base = base;
  b->ws_owned = owned;
  // the captured graph holds the old addresses
  if (b->exec) {
    hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->key.clear();
  }
}

// Fork from `origin`, every group's launch sequence on its stream, join
// back into `origin`.
static pb3_status enqueue_batch(pb3_batch* b, const float* const* deltas, double* const* pk, double* const* bk,
                                pb3_precision prec, hipStream_t origin) {
  hipError_t e = hipEventRecord(b->fork, origin);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  for (int i = 0; i < b->n_streams; ++i) {
    e = hipStreamWaitEvent(b->streams[i], b->fork, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  for (const Group& g : b->groups) {
    Exec x;
    x.ws = carve(g.plan, (char*)b->ws_base + g.offset, g.stride);
    x.wstride = g.stride;
    x.n_jobs = (int)g.jobs.size();
    for (int k = 0; k < x.n_jobs; ++k) {
      const int j = g.jobs[k];
      x.io.delta[k] = deltas[j];
      x.io.pk[k] = pk ? pk[j] : nullptr;
      x.io.bk[k] = bk ? bk[j] : nullptr;
    }
    pb3_status st = enqueue(*g.plan, x, pk != nullptr, bk != nullptr, prec, b->streams[g.stream]);
    if (st != PB3_OK) return st;
  }
  for (int i = 0; i < b->n_streams; ++i) {
    e = hipEventRecord(b->join[i], b->streams[i]);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    e = hipStreamWaitEvent(origin, b->join[i], 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  return PB3_OK;
}

static pb3_status run_graph(pb3_batch* b, const float* const* deltas, double* const* pk, double* const* bk,
                            pb3_precision prec, hipStream_t s) {
  std::vector<const void*> key;
  key.reserve(3 * b->n_jobs + 3);
  key.push_back((const void*)(uintptr_t)(prec + 1));
  key.push_back(pk ? (const void*)1 : nullptr);
  key.push_back(bk ? (const void*)1 : nullptr);
  for (int j = 0; j < b->n_jobs; ++j) {
    key.push_back(deltas[j]);
    key.push_back(pk ? pk[j] : nullptr);
    key.push_back(bk ? bk[j] : nullptr);
  }
  if (!b->exec || key != b->key) {
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    pb3_status st = enqueue_batch(b, deltas, pk, bk, prec, b->cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->cap, &graph);
    if (st != PB3_OK) {
      if (graph) hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    bool updated = false;
    if (b->exec) {
      hipGraphNode_t err_node = nullptr;
      hipGraphExecUpdateResult res;
      updated = hipGraphExecUpdate(b->exec, graph, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
      if (!updated) {
        // a refused update (e.g. a kernel node whose block size changed with
        // the precision) is not an error: instantiate anew.  The refusal
        // leaves a sticky last error that the next launch check would
        // report, so clear it here.
        (void)hipGetLastError();
        hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
      }
    }
    if (!updated) {
      e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        b->exec = nullptr;
        hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
      }
    }
    hipGraphDestroy(graph);
    b->key.swap(key);
  }
  hipError_t e = hipGraphLaunch(b->exec, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return PB3_OK;
}

}  // namespace pb3

using namespace pb3;

extern "C" {

pb3_status pb3_batch_create(pb3_plan* const* plans, int n_jobs, unsigned flags, pb3_batch** out) {
  if (!out) {
    set_error("null output pointer");
    return PB3_EINVAL;
  }
  *out = nullptr;
  if (!plans || n_jobs <= 0) {
    set_error("a batch needs at least one job");
    return PB3_EINVAL;
  }
  if (flags & ~(PB3_BATCH_GRAPH | PB3_BATCH_EXT_WORKSPACE)) {
    set_error("unknown batch flag");
    return PB3_EINVAL;
  }
  for (int j = 0; j < n_jobs; ++j) {
    if (!plans[j]) {
      set_error("null plan in batch");
      return PB3_EINVAL;
    }
    if (!plans[j]->device) {
      set_error("batch plans must be device plans (not PB3_FLAG_HOST_ONLY)");
      return PB3_EINVAL;
    }
    if (plans[j]->flags & PB3_FLAG_POWER_ONLY) {
      set_error("batch plans must carry bispectrum tables (not PB3_FLAG_POWER_ONLY)");
      return PB3_EINVAL;
    }
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  for (int j = 0; j < n_jobs; ++j) {
    if (plans[j]->device_id != dev) {
      set_error("batch plans must live on the current device");
      return PB3_EINVAL;
    }
  }
  pb3_batch* b = new (std::nothrow) pb3_batch();
  if (!b) {
    set_error("host allocation failed");
    return PB3_ENOMEM;
  }
  b->flags = flags;
  b->device_id = dev;
  b->n_jobs = n_jobs;
  // group by plan object, in order of first appearance, kMaxJobs per group
  std::vector<pb3_plan*> seen;
  for (int j = 0; j < n_jobs; ++j)
    if (std::find(seen.begin(), seen.end(), plans[j]) == seen.end()) seen.push_back(plans[j]);
  for (pb3_plan* p : seen) {
    std::vector<int> js;
    for (int j = 0; j < n_jobs; ++j)
      if (plans[j] == p) js.push_back(j);
    for (size_t k = 0; k < js.size(); k += kMaxJobs) {
      Group g;
      g.plan = p;
      g.jobs.assign(js.begin() + k, js.begin() + std::min(js.size(), k + kMaxJobs));
      g.stride = workspace_bytes(p);
      g.cost = plan_cost(*p) * g.jobs.size();
      b->groups.push_back(std::move(g));
    }
  }
  // longest group first onto the least-loaded stream
  b->n_streams = std::min<int>(kBatchStreams, (int)b->groups.size());
  std::vector<int> order(b->groups.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return b->groups[a].cost > b->groups[c].cost; });
  std::vector<double> load(b->n_streams, 0.0);
  for (int gi : order) {
    int best = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->groups[gi].stream = best;
    load[best] += b->groups[gi].cost;
  }
  size_t off = 0;
  for (Group& g : b->groups) {
    g.offset = off;
    off += g.stride * g.jobs.size();
  }
  b->ws_bytes = off;
  pb3_status st = PB3_OK;
  b->streams.assign(b->n_streams, nullptr);
  b->join.assign(b->n_streams, nullptr);
  for (int i = 0; i < b->n_streams && st == PB3_OK; ++i) {
    if ((e = hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking)) != hipSuccess)
      st = hip_fail(e, "hipStreamCreateWithFlags");
    else if ((e = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming)) != hipSuccess)
      st = hip_fail(e, "hipEventCreateWithFlags");
  }
  if (st == PB3_OK && (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess)
    st = hip_fail(e, "hipStreamCreateWithFlags");
  if (st == PB3_OK && (e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess)
    st = hip_fail(e, "hipEventCreateWithFlags");
  if (st == PB3_OK && !(flags & PB3_BATCH_EXT_WORKSPACE)) {
    void* base = nullptr;
    e = dev_malloc(&base, b->ws_bytes);
    if (e != hipSuccess) {
      set_error("batch workspace hipMalloc of " + std::to_string(b->ws_bytes) + " bytes: " + hipGetErrorString(e));
      st = PB3_ENOMEM;
    } else {
      set_workspace(b, base, true);
    }
  }
  if (st != PB3_OK) {
    release(b);
    delete b;
    return st;
  }
  *out = b;
  return PB3_OK;
}

size_t pb3_batch_workspace_bytes(const pb3_batch* batch) { return batch ? batch->ws_bytes : 0; }

pb3_status pb3_batch_bind_workspace(pb3_batch* batch, void* dev, size_t bytes) {
  if (!batch || !dev) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  if (bytes < batch->ws_bytes) {
    set_error("batch workspace too small: need " + std::to_string(batch->ws_bytes) + " bytes");
    return PB3_ENOMEM;
  }
  if (((uintptr_t)dev) % 256) {
    set_error("workspace must be 256-byte aligned");
    return PB3_EINVAL;
  }
  set_workspace(batch, dev, false);
  return PB3_OK;
}

pb3_status pb3_batch_run(pb3_batch* batch, const float* const* deltas, double* const* pk, double* const* bk,
                         pb3_precision prec, void* stream) {
  if (!batch || !deltas || (!pk && !bk)) {
    set_error("null argument");
    return PB3_EINVAL;
  }
  pb3_status st = check_prec(prec);
  if (st != PB3_OK) return st;
  if (!batch->ws_base) {
    set_error("batch has no workspace (PB3_BATCH_EXT_WORKSPACE without a bound workspace)");
    return PB3_EINVAL;
  }
  int dev = -1;
  hipGetDevice(&dev);
  if (dev != batch->device_id) {
    set_error("batch was created on another device");
    return PB3_EINVAL;
  }
  for (int j = 0; j < batch->n_jobs; ++j) {
    if (!deltas[j] || (pk && !pk[j]) || (bk && !bk[j]) || ((uintptr_t)deltas[j] & 7u) != 0) {
      set_error("null (or not 8-byte aligned) device pointer for job " + std::to_string(j));
      return PB3_EINVAL;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  if (batch->flags & PB3_BATCH_GRAPH) return run_graph(batch, deltas, pk, bk, prec, s);
  return enqueue_batch(batch, deltas, pk, bk, prec, s);
}

int pb3_batch_launches(const pb3_batch* batch, int with_pk, int with_bk) {
  if (!batch) return 0;
  int n = 0;
  for (const Group& g : batch->groups) n += launches_per_sequence(*g.plan, with_pk != 0, with_bk != 0);
  return n;
}

int pb3_batch_groups(const pb3_batch* batch) { return batch ? (int)batch->groups.size() : 0; }

pb3_status pb3_batch_destroy(pb3_batch* batch) {
  if (!batch) return PB3_OK;
  release(batch);
  delete batch;
  return PB3_OK;
}

pb3_status pb3_bispectrum_batched(pb3_plan* const* plans, const float* const* deltas, double* const* bk_outs,
                                  int n_jobs, pb3_precision prec, void* stream) {
  if (!bk_outs) {
    set_error("null output array");
    return PB3_EINVAL;
  }
  pb3_batch* b = nullptr;
  pb3_status st = pb3_batch_create(plans, n_jobs, 0, &b);
  if (st != PB3_OK) return st;
  st = pb3_batch_run(b, deltas, nullptr, bk_outs, prec, stream);
  if (st == PB3_OK) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
  }
  pb3_batch_destroy(b);
  return st;
}

}  // extern "C"
