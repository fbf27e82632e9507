// muca_context.h -- the library-side state behind a muca_ctx handle
// (internal; the public interface is include/muca.h).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/muca.h"
#include "muca_device.h"

using muca::GroupDesc;
using muca::SweepTask;

namespace muca_detail {
// Records the thread-local error text returned by mucaLastError; returns code.
int fail(int code, const char* fmt, ...);
}  // namespace muca_detail

constexpr int64_t kLdsBytes = 160 * 1024;  // LDS per CU of gfx950
// Default cap of the walker state in flight when it lives in device memory:
// below the 256 MB last-level (Infinity) cache of MI355X.
constexpr size_t kResidentBytes = size_t(224) << 20;

struct muca_context {
  int device = 0;
  uint32_t seed32 = 0, first_id = 0;
  std::vector<GroupDesc> g;
  GroupDesc* d_groups = nullptr;
  int ngroups = 0, nwalkers = 0, total_bins = 0, thr_entries = 0;
  int64_t total_words = 0, total_pos = 0;
  uint32_t* d_bits = nullptr;
  uint32_t* d_pos = nullptr;
  int32_t* d_E = nullptr;
  uint64_t* d_T = nullptr;
  uint32_t* d_tun = nullptr;  // per walker: last window end (bits 0-1), trips (bits 2-31)
  int32_t* d_wgroup = nullptr;
  uint32_t* d_thr = nullptr;
  double* d_slope = nullptr;
  int32_t* d_status = nullptr;  // bit 0: non-finite weight read; bit 1: produced
  int32_t* d_ones = nullptr;
  int32_t* d_active = nullptr;
  int32_t* d_flat = nullptr;
  int32_t* d_iters = nullptr;
  int32_t* d_counter = nullptr;  // [0] iteration index, [1] groups still active
  int32_t* h_pinned = nullptr;   // host-pinned readback of the counters
  int tunnel_target = 30;        // trips per group that end a MUCA_STOP_TUNNEL run
  int layout = MUCA_LAYOUT_AUTO;  // requested
  int tuned = 0;                  // layout picked by mucaAutotune (0 = none yet)
  hipStream_t last_stream = nullptr;
  // cooperative layouts: one task table per lanes-per-walker choice.  A task
  // is one set of walkers (one block's worth of one group); block b runs
  // tasks [first[b], first[b+1]) one after the other.
  struct Coop {
    SweepTask* d_tasks = nullptr;
    int32_t* d_first = nullptr;
    int ntasks = 0, nblocks = 0;
    size_t need = 0;       // LDS bytes for the walker state of the largest set
  } coop[6];  // lanes per walker / walkers per wavefront: [0] 16/4, [1] 64/1, [2] 16/2,
              // [3] 16/1, [4] 64/1 with one set per block (LOOK4), [5] 16/2 or 16/4
              // per group (SUB16MIX)
  int num_cu = 256;        // compute units of the device
  size_t tbl_bytes = 0;    // largest threshold table of one group
  size_t hist_bytes = 0;   // largest histogram of one group
  // captured iteration of mucaRun (replayed once per iteration)
  bool use_graph = true;
  bool bricked = false;  // some group keeps bricked bits (always device-memory state)
  bool run_started = false;  // a mucaRun has initialised the loop state
  hipStream_t run_stream = nullptr;  // default priority
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  struct GraphKey {
    const void *lnW, *P, *H;
    int sweeps, rule, stop, layout, tunnel_target;
    size_t lds_limit;
    bool operator==(const GraphKey& o) const {
      return lnW == o.lnW && P == o.P && H == o.H && sweeps == o.sweeps && rule == o.rule &&
             stop == o.stop && layout == o.layout && tunnel_target == o.tunnel_target &&
             lds_limit == o.lds_limit;
    }
  } graph_key{};
  size_t lds_limit = kLdsBytes;  // LDS a cooperative block may use
  // walker state (bytes) a device-memory-state launch keeps in flight
  size_t resident_limit = kResidentBytes;
  size_t lds_device = 64 * 1024;  // device maximum per block

  // Forget the cooperative task tables (rebuilt on the next launch) and the
  // captured iteration, e.g. after a change of the LDS or resident limit.
  void drop_tables() {
    (void)hipDeviceSynchronize();
    for (auto& q : coop) {
      (void)hipFree(q.d_tasks);
      (void)hipFree(q.d_first);
      q = Coop{};
    }
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }

  ~muca_context() {
    (void)hipFree(d_groups);
    (void)hipFree(d_bits);
    (void)hipFree(d_pos);
    (void)hipFree(d_E);
    (void)hipFree(d_T);
    (void)hipFree(d_tun);
    (void)hipFree(d_wgroup);
    (void)hipFree(d_thr);
    (void)hipFree(d_slope);
    (void)hipFree(d_status);
    (void)hipFree(d_ones);
    (void)hipFree(d_active);
    (void)hipFree(d_flat);
    (void)hipFree(d_iters);
    (void)hipFree(d_counter);
    for (auto& q : coop) {
      (void)hipFree(q.d_tasks);
      (void)hipFree(q.d_first);
    }
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (run_stream) (void)hipStreamDestroy(run_stream);
    if (h_pinned) (void)hipHostFree(h_pinned);
  }
};
