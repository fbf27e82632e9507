// muca_runtime.hip -- host runtime and C ABI of libmuca (see include/muca.h).
//
// Owns the device state of all walkers (occupation bits, particle sites,
// energies, attempt counters), the per-group descriptors and the acceptance
// threshold table; launches the kernels of the MUCA iteration (paper Sec. 2)
// on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/muca.h"
#include "muca_context.h"
#include "muca_kernels.h"

using muca::GroupDesc;
using muca::SweepTask;

namespace muca_detail {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace muca_detail

using muca_detail::fail;
using muca_detail::g_last_error;

namespace {

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(e_ == hipErrorOutOfMemory ? MUCA_ENOMEM : MUCA_EHIP, "%s: %s (%s:%d)",    \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                        \
  } while (0)

#define HIP_TRY_DEL(expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      delete c;                                                                             \
      return fail(MUCA_EHIP, "%s: %s", #expr, hipGetErrorString(e_));                       \
    }                                                                                       \
  } while (0)

#define LAUNCH_CHECK()                                                                      \
  do {                                                                                      \
    hipError_t e_ = hipGetLastError();                                                      \
    if (e_ != hipSuccess)                                                                   \
      return fail(MUCA_EHIP, "kernel launch: %s (%s:%d)", hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                \
  } while (0)

// Default lower window edge: the energy of a compact cluster.  In 2D a
// w-wide block of N sites filled row by row has 2N - w - ceil(N/w) bonds;
// in 3D full x*y layers stacked z high (3xyz - xy - yz - zx bonds) carry a
// partial layer of m sites filled in the same way, each with one bond down.
// No extent reaches L, so no bond wraps round the torus.
int64_t block_bonds(int64_t m, int64_t wmax, int64_t hmax) {
  if (m == 0) return 0;
  int64_t best = -1;
  for (int64_t w = 1; w <= wmax && w <= m; ++w) {
    const int64_t rows = (m + w - 1) / w;
    if (rows > hmax) continue;
    best = std::max(best, 2 * m - w - rows);
  }
  return best;
}

int32_t energy_floor(int d, int L, int N) {
  const int64_t e = L - 1;
  if (d == 2) return (int32_t)(-std::max<int64_t>(0, block_bonds(N, e, e)));
  int64_t best = 0;
  for (int64_t x = 1; x <= e; ++x)
    for (int64_t y = 1; y <= e; ++y) {
      const int64_t layer = x * y, z = N / layer, m = N - layer * z;
      if (z + (m ? 1 : 0) > e) continue;
      const int64_t top = block_bonds(m, x, y);
      if (top < 0) continue;
      const int64_t box = z ? 3 * layer * z - layer - y * z - z * x : 0;
      best = std::max(best, box + top + (z ? m : 0));
    }
  return (int32_t)(-best);
}

template <typename T>
int dev_alloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  HIP_TRY(hipMalloc((void**)p, n * sizeof(T)));
  return MUCA_OK;
}

}  // namespace


// ---------------------------------------------------------------- static workspace
// Device memory of the allocation-free sweep (mucaSweepNoAlloc): the
// threshold table, then the task table of the cooperative layouts.  One copy
// per device, held until the process ends; every call on a device shares it.
constexpr size_t kStaticBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices];  // device address of `scratch`, per device

// Looks up the device address of the workspace on the current device (once
// per device).  In host code `scratch` names a host-side stand-in, never the
// device memory, so kernels and copies use only the address found here.
int static_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(MUCA_EHIP, "device %d beyond the %d supported", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static_ptr[device]) return MUCA_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(MUCA_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_static_ptr[device] = ptr;
  return MUCA_OK;
}

// The plain task table of a cooperative layout: set i is walkers
// [f, f + count) of one group, sets in group order, one set per block.
// spread > 0: every group's walkers in every spread-th row; spread = 0: two
// walkers per wavefront for the groups with V = vmax, four for the others.
__global__ void k_plain_tasks(const GroupDesc* __restrict__ groups, int ngroups, int lanes,
                              int spread, int vmax, SweepTask* __restrict__ tasks,
                              int32_t* __restrict__ first, int nsets) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) first[nsets] = nsets;
  if (i >= nsets) return;
  int base = 0;
  for (int gi = 0; gi < ngroups; ++gi) {
    const GroupDesc g = groups[gi];
    const int sp = spread > 0 ? spread : (g.V == vmax ? 2 : 1);
    const int wpb = 256 / lanes / sp;
    const int n = (g.walkers + wpb - 1) / wpb;
    if (i < base + n) {
      const int f = (i - base) * wpb;
      tasks[i] = SweepTask{gi, g.first_walker + f, min(wpb, g.walkers - f), sp};
      first[i] = i;
      return;
    }
    base += n;
  }
}

}  // namespace

namespace {

int check_ctx(muca_ctx c) {
  if (!c) return fail(MUCA_EINVAL, "null context");
  return MUCA_OK;
}

// Acceptance thresholds of every group into thr (the context's table, or
// the static workspace of the allocation-free sweep).
int enqueue_thresholds_to(muca_ctx c, const double* lnW, uint32_t* thr, hipStream_t s) {
  int maxe = 0;
  for (const auto& q : c->g) maxe = std::max(maxe, q.nbins * q.nd);
  dim3 grid((unsigned)std::min(1024, (maxe + 255) / 256), (unsigned)c->ngroups);
  hipLaunchKernelGGL(muca::k_thresholds, grid, dim3(256), 0, s, c->d_groups, lnW, thr,
                     c->d_status);
  LAUNCH_CHECK();
  return MUCA_OK;
}

int enqueue_thresholds(muca_ctx c, const double* lnW, hipStream_t s) {
  return enqueue_thresholds_to(c, lnW, c->d_thr, s);
}

int resolved_layout(muca_ctx c) {
  if (c->layout != MUCA_LAYOUT_AUTO) return c->layout;
  return c->tuned ? c->tuned : MUCA_LAYOUT_SUB16;
}

// A set is up to 256/G/spread walkers of one group (one block's worth).
// When the sets outnumber the CUs, they are packed longest first (V per
// sweep) into a whole number of blocks per CU, a block running its sets one
// after the other: otherwise the few blocks beyond a full round share SIMDs
// with the long chains and stretch the launch (258 sets of 16 walkers on 256
// CUs cost 30 % in the batched 2D workload).  Otherwise one set per block,
// the groups interleaved so that every CU receives a mix of lattice sizes.
constexpr int kCoops = 6;
constexpr int kCoopLanes[kCoops] = {16, 64, 16, 16, 64, 16};  // lanes per walker
// 16-lane rows per walker row used; 0: per group (SUB16MIX, see group_spread)
constexpr int kCoopSpread[kCoops] = {1, 1, 2, 4, 1, 0};
constexpr bool kCoopPacked[kCoops] = {true, true, true, true, false, true};

// Rows per walker of group g in cooperative table `which`.  SUB16MIX: the
// groups with the context's largest lattice get two walkers per wavefront
// (their chains bound the launch, and fewer walkers per wavefront take the
// rare paths less often), the others four.
int group_spread(const muca_context* c, int which, const GroupDesc& g) {
  if (kCoopSpread[which] > 0) return kCoopSpread[which];
  int vmax = 0;
  for (const auto& h : c->g) vmax = std::max(vmax, h.V);
  return g.V == vmax ? 2 : 1;
}

int group_wpb(const muca_context* c, int which, const GroupDesc& g) {
  return 256 / kCoopLanes[which] / group_spread(c, which, g);
}

// Task table (coop index) of a cooperative layout, -1 for the one-walker-per-
// lane layout.
int coop_index(int layout) {
  switch (layout) {
    case MUCA_LAYOUT_SUB16: return 0;
    case MUCA_LAYOUT_SUB64: return 1;
    case MUCA_LAYOUT_SUB16X2: return 2;
    case MUCA_LAYOUT_SUB16X1: return 3;
    case MUCA_LAYOUT_LOOK4: return 4;
    case MUCA_LAYOUT_SUB16MIX: return 5;
    default: return -1;
  }
}

// Host-side sizes of a cooperative layout: LDS bytes for the walker state of
// the largest set (need), and the context's largest histogram and threshold
// table of one group (hist_bytes, tbl_bytes).  No device work.
size_t coop_sizes(muca_ctx c, int which) {
  size_t need = 0;
  c->hist_bytes = 0;
  c->tbl_bytes = 0;
  for (const auto& g : c->g) {
    const int wpb = group_wpb(c, which, g);
    // per walker: (site, coordinates) pairs, bits rounded up to whole pairs;
    // one word of alignment slack before the first slot
    need = std::max(need, (size_t)wpb * (size_t)(2 * g.N + ((g.words + 1) & ~1)) *
                              sizeof(uint32_t) + sizeof(uint32_t));
    c->hist_bytes = std::max(c->hist_bytes, (size_t)g.nbins * sizeof(int32_t));
    c->tbl_bytes = std::max(c->tbl_bytes, (size_t)g.nbins * (size_t)g.nd * sizeof(uint32_t));
  }
  return need;
}

int build_coop(muca_ctx c, int which) {
  auto& q = c->coop[which];
  if (q.d_tasks) return MUCA_OK;
  std::vector<std::vector<SweepTask>> per(c->ngroups);
  const size_t need = coop_sizes(c, which);
  for (int i = 0; i < c->ngroups; ++i) {
    const GroupDesc& g = c->g[i];
    const int wpb = group_wpb(c, which, g), sp = group_spread(c, which, g);
    for (int f = 0; f < g.walkers; f += wpb)
      per[i].push_back(SweepTask{i, g.first_walker + f, std::min(wpb, g.walkers - f), sp});
  }
  std::vector<SweepTask> sets;
  for (size_t r = 0;; ++r) {
    bool any = false;
    for (auto& v : per)
      if (r < v.size()) {
        sets.push_back(v[r]);
        any = true;
      }
    if (!any) break;
  }
  const int n = (int)sets.size(), C = std::max(1, c->num_cu);
  std::vector<SweepTask> tasks;
  std::vector<int32_t> first;
  // With walker state in device memory, cap the state in flight at once
  // (resident_limit bytes): a population whose state exceeds the device's
  // last-level cache runs faster in rounds that fit it.
  const size_t cap = std::min(c->lds_limit, c->lds_device);
  const bool state_lds = !c->bricked && need + c->hist_bytes <= cap;
  int Bmax = n;
  if (!state_lds && c->resident_limit > 0) {
    size_t set_bytes = 1;
    for (const auto& t : sets)
      set_bytes = std::max(set_bytes, (size_t)t.count *
                                          ((size_t)c->g[t.group].words + c->g[t.group].N) *
                                          sizeof(uint32_t));
    Bmax = std::max(C, (int)(c->resident_limit / set_bytes / (size_t)C) * C);
  }
  if (!kCoopPacked[which] || (n <= C && n <= Bmax)) {
    tasks = sets;
    for (int b = 0; b <= n; ++b) first.push_back(b);
  } else {
    const int B = std::min((n / C) * C, Bmax);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return c->g[sets[a].group].V > c->g[sets[b].group].V;
    });
    std::vector<std::vector<int>> blk(B);
    std::vector<int64_t> load(B, 0);
    for (int i : order) {  // longest first onto the least loaded block (lowest index on ties)
      const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      blk[b].push_back(i);
      load[b] += c->g[sets[i].group].V;
    }
    // B / C rounds of blocks share the CUs.  Blocks sorted by load, with
    // every other round in reverse order, so that a CU's longest block gets
    // the shortest partners (the dispatcher hands out each round across the
    // CUs in order).
    std::vector<int> bo(B);
    for (int b = 0; b < B; ++b) bo[b] = b;
    std::stable_sort(bo.begin(), bo.end(), [&](int a, int b) { return load[a] > load[b]; });
    for (int r = 1; r < B / C; r += 2) std::reverse(bo.begin() + r * C, bo.begin() + (r + 1) * C);
    for (int b : bo) {
      first.push_back((int32_t)tasks.size());
      for (int i : blk[b]) tasks.push_back(sets[i]);
    }
    first.push_back((int32_t)tasks.size());
  }
  q.ntasks = (int)tasks.size();
  q.nblocks = (int)first.size() - 1;
  q.need = need;
  if (int r = dev_alloc(&q.d_tasks, tasks.size())) return r;
  if (int r = dev_alloc(&q.d_first, first.size())) return r;
  HIP_TRY(hipMemcpy(q.d_tasks, tasks.data(), sizeof(SweepTask) * tasks.size(),
                    hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(q.d_first, first.data(), sizeof(int32_t) * first.size(),
                    hipMemcpyHostToDevice));
  return MUCA_OK;
}

// Where a cooperative launch finds its tables: block b runs tasks
// [first[b], first[b + 1]); need = LDS bytes of the largest set's state.
struct CoopTables {
  const SweepTask* tasks;
  const int32_t* first;
  int nblocks;
  size_t need;
  const uint32_t* thr;
};

template <int G>
int launch_coop_tables(muca_ctx c, int which, const CoopTables& q, int sweeps, int32_t* H,
                       const int32_t* active, hipStream_t s) {
  const size_t cap = std::min(c->lds_limit, c->lds_device);
  // LDS-resident walker state comes with a block histogram in LDS
  const bool state_lds = !c->bricked && q.need + c->hist_bytes <= cap;
  const size_t state = state_lds ? q.need + c->hist_bytes : 0;
  const bool tbl_lds = c->lds_limit > 0 && state + c->tbl_bytes <= cap;
  const size_t dyn = state + (tbl_lds ? c->tbl_bytes : 0);
  const int tbl_words = tbl_lds ? (int)(c->tbl_bytes / sizeof(uint32_t)) : 0;
  // With state in device memory the 16-lane layouts issue the gathers of the
  // next attempts before deciding the current one: two ahead when every
  // group's V is a multiple of 16 (full batches), else one; the 64-lane
  // layout does not pipeline (pipelined, it ran slower on the large 3D
  // lattices).
  const bool pipe = G == 16;
  bool full16 = true;
  for (const auto& g : c->g) full16 = full16 && g.V % 16 == 0;
  auto kern = state_lds ? (tbl_lds ? muca::k_sweep_sub<G, true, true, 0>
                                   : muca::k_sweep_sub<G, true, false, 0>)
            : pipe      ? (full16 ? (tbl_lds ? muca::k_sweep_sub<16, false, true, 2>
                                             : muca::k_sweep_sub<16, false, false, 2>)
                                  : (tbl_lds ? muca::k_sweep_sub<16, false, true, 1>
                                             : muca::k_sweep_sub<16, false, false, 1>))
                        : (tbl_lds ? muca::k_sweep_sub<64, false, true, 0>
                                   : muca::k_sweep_sub<64, false, false, 0>);
  hipLaunchKernelGGL(kern, dim3((unsigned)q.nblocks), dim3(256), dyn, s, c->d_groups, q.tasks,
                     q.first, c->d_bits, c->d_pos, c->d_E, c->d_T, c->d_tun, q.thr, H, active,
                     sweeps, c->first_id, c->seed32, tbl_words,
                     state_lds ? (int)(c->hist_bytes / sizeof(int32_t)) : 0);
  LAUNCH_CHECK();
  return MUCA_OK;
}

template <int G>
int launch_coop(muca_ctx c, int which, int sweeps, int32_t* H, const int32_t* active,
                hipStream_t s) {
  if (int r = build_coop(c, which)) return r;
  const auto& q = c->coop[which];
  return launch_coop_tables<G>(c, which, CoopTables{q.d_tasks, q.d_first, q.nblocks, q.need,
                                                    c->d_thr},
                               sweeps, H, active, s);
}

// Lookahead layout: blocks of four walkers (one per wavefront), walker state
// and block histogram in LDS; the caller falls back to SUB64 when they do not
// fit (look_fits).  One task per block.
bool look_fits(muca_ctx c, size_t need) {
  const size_t cap = std::min(c->lds_limit, c->lds_device);
  return !c->bricked && need + c->hist_bytes <= cap;
}

void launch_look_tables(muca_ctx c, const SweepTask* tasks, int ntasks, size_t need,
                        const uint32_t* thr, int sweeps, int32_t* H, const int32_t* active,
                        hipStream_t s) {
  const size_t cap = std::min(c->lds_limit, c->lds_device);
  const size_t state = need + c->hist_bytes;
  const bool tbl_lds = state + c->tbl_bytes <= cap;
  const size_t dyn = state + (tbl_lds ? c->tbl_bytes : 0);
  auto kern = tbl_lds ? muca::k_sweep_look<true> : muca::k_sweep_look<false>;
  hipLaunchKernelGGL(kern, dim3((unsigned)ntasks), dim3(256), dyn, s, c->d_groups, tasks,
                     c->d_bits, c->d_pos, c->d_E, c->d_T, c->d_tun, thr, H, active, sweeps,
                     c->first_id, c->seed32, tbl_lds ? (int)(c->tbl_bytes / sizeof(uint32_t)) : 0,
                     (int)(c->hist_bytes / sizeof(int32_t)));
}

int launch_look(muca_ctx c, int sweeps, int32_t* H, const int32_t* active, hipStream_t s) {
  if (int r = build_coop(c, 4)) return r;
  const auto& q = c->coop[4];
  if (!look_fits(c, q.need)) return launch_coop<64>(c, 1, sweeps, H, active, s);
  launch_look_tables(c, q.d_tasks, q.ntasks, q.need, c->d_thr, sweeps, H, active, s);
  LAUNCH_CHECK();
  return MUCA_OK;
}

int enqueue_sweep_kernel(muca_ctx c, int layout, int sweeps, int32_t* H, const int32_t* active,
                         hipStream_t s) {
  switch (layout) {
    case MUCA_LAYOUT_LANE:
      hipLaunchKernelGGL(muca::k_sweep_lane, dim3((unsigned)((c->nwalkers + 63) / 64)), dim3(64),
                         0, s, c->d_groups, c->d_wgroup, c->d_bits, c->d_pos, c->d_E, c->d_T,
                         c->d_tun, c->d_thr, H, active, c->nwalkers, sweeps, c->first_id,
                         c->seed32);
      LAUNCH_CHECK();
      return MUCA_OK;
    case MUCA_LAYOUT_SUB16:
      return launch_coop<16>(c, 0, sweeps, H, active, s);
    case MUCA_LAYOUT_SUB64:
      return launch_coop<64>(c, 1, sweeps, H, active, s);
    case MUCA_LAYOUT_LOOK4:
      return launch_look(c, sweeps, H, active, s);
    case MUCA_LAYOUT_SUB16X2:
      return launch_coop<16>(c, 2, sweeps, H, active, s);
    case MUCA_LAYOUT_SUB16X1:
      return launch_coop<16>(c, 3, sweeps, H, active, s);
    case MUCA_LAYOUT_SUB16MIX:
      return launch_coop<16>(c, 5, sweeps, H, active, s);
    default:
      return fail(MUCA_EINVAL, "unknown layout %d", layout);
  }
}

int enqueue_zero_hist(muca_ctx c, int32_t* H, const int32_t* active, hipStream_t s) {
  int maxb = 0;
  for (const auto& q : c->g) maxb = std::max(maxb, q.nbins);
  hipLaunchKernelGGL(muca::k_zero_hist, dim3((unsigned)((maxb + 255) / 256), (unsigned)c->ngroups),
                     dim3(256), 0, s, c->d_groups, active, H);
  LAUNCH_CHECK();
  return MUCA_OK;
}

int enqueue_sweep(muca_ctx c, const double* lnW, int sweeps, int32_t* H, const int32_t* active,
                  hipStream_t s) {
  if (int rc = enqueue_thresholds(c, lnW, s)) return rc;
  if (int rc = enqueue_zero_hist(c, H, active, s)) return rc;
  return enqueue_sweep_kernel(c, resolved_layout(c), sweeps, H, active, s);
}

int check_sweeps(muca_ctx c, int sweeps) {
  if (sweeps < 1) return fail(MUCA_EINVAL, "sweeps must be >= 1 (got %d)", sweeps);
  for (size_t i = 0; i < c->g.size(); ++i)
    if ((int64_t)c->g[i].walkers * (int64_t)sweeps > 2147483647LL)
      return fail(MUCA_EOVERFLOW, "group %zu: walkers x sweeps exceeds INT32_MAX", i);
  return MUCA_OK;
}

}  // namespace

extern "C" {

const char* mucaLastError(void) { return g_last_error.c_str(); }

int mucaInitGroups(muca_ctx* out, const muca_group* groups, int ngroups, uint64_t seed,
                   uint32_t first_id) {
  if (!out) return fail(MUCA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!groups || ngroups < 1) return fail(MUCA_EINVAL, "need at least one group");
  auto* c = new (std::nothrow) muca_context();
  if (!c) return fail(MUCA_ENOMEM, "host allocation failed");
  c->seed32 = (uint32_t)seed;
  c->first_id = first_id;
  c->ngroups = ngroups;
  int64_t walkers = 0, bins = 0, thr = 0, words = 0, pos = 0;
  for (int i = 0; i < ngroups; ++i) {
    const muca_group q = groups[i];
    auto bad = [&](const char* why) {
      delete c;
      return fail(MUCA_EINVAL, "group %d (d=%d L=%d N=%d walkers=%d window=[%d,%d]): %s", i, q.d,
                  q.L, q.N, q.walkers, q.e_lo, q.e_hi, why);
    };
    if (q.d != 2 && q.d != 3) return bad("d must be 2 or 3");
    if (q.L < 3 || q.L > 1024) return bad("L must be in [3, 1024]");
    const int64_t V = (q.d == 2) ? (int64_t)q.L * q.L : (int64_t)q.L * q.L * q.L;
    if (V > (1 << 24)) return bad("V = L^d must not exceed 2^24");
    if (q.walkers < 1) return bad("walkers must be >= 1");
    if (q.N < 1 || q.N > V - 1) return bad("N must be in [1, V-1]");
    GroupDesc d{};
    d.d = q.d;
    d.L = q.L;
    d.N = q.N;
    d.V = (int32_t)V;
    if (q.e_lo == 0 && q.e_hi == 0) {
      if (2 * (int64_t)q.N > V) return bad("default window needs N <= V/2");
      d.e_lo = energy_floor(q.d, q.L, q.N);
      d.e_hi = 0;
    } else {
      if (q.e_lo > q.e_hi || q.e_hi > 0 || (int64_t)q.e_lo < -(int64_t)q.d * q.N)
        return bad("window must satisfy -dN <= e_lo <= e_hi <= 0");
      d.e_lo = q.e_lo;
      d.e_hi = q.e_hi;
    }
    d.nbins = d.e_hi - d.e_lo + 1;
    if (d.nbins > (1 << 24)) return bad("the window must hold at most 2^24 bins");
    d.nd = 4 * q.d + 1;
    d.bin_off = (int32_t)bins;
    d.thr_off = (int32_t)thr;
    d.first_walker = (int32_t)walkers;
    d.walkers = q.walkers;
    d.words = (int32_t)((V + 31) / 32);
    d.LL = q.L * q.L;
    d.invL = 1.0f / (float)q.L;
    // 3D lattices whose walker state cannot sit in LDS (16 walkers of a
    // block: bits + two words per particle) keep bricked bits in device
    // memory (fewer lines per neighbourhood gather; bit_ref on the device).
    const int64_t state16 = 16 * ((int64_t)d.words + 2 * (int64_t)q.N) * 4;
    d.brick8 = (q.d == 3 && q.L % 8 == 0 && state16 > kLdsBytes) ? q.L / 8 : 0;
    d.bits_off = words;
    d.pos_off = pos;
    walkers += q.walkers;
    bins += d.nbins;
    thr += (int64_t)d.nbins * d.nd;
    words += (int64_t)q.walkers * d.words;
    pos += (int64_t)q.walkers * q.N;
    if (walkers > 0x7FFFFFFF || thr > 0x7FFFFFFF) {
      delete c;
      return fail(MUCA_EINVAL, "too many walkers or bins");
    }
    c->g.push_back(d);
    c->bricked = c->bricked || d.brick8 != 0;
  }
  c->nwalkers = (int)walkers;
  c->total_bins = (int)bins;
  c->thr_entries = (int)thr;
  c->total_words = words;
  c->total_pos = pos;
  HIP_TRY_DEL(hipGetDevice(&c->device));
  if (int r = static_setup(c->device)) {
    delete c;
    return r;
  }
  {
    int v = 0;
    HIP_TRY_DEL(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    c->lds_device = (size_t)v;
    int cus = 0;
    HIP_TRY_DEL(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    c->num_cu = std::max(1, cus);
    // allow every cooperative kernel the device's full LDS per block (set
    // once here, outside any stream capture)
    const void* kernels[] = {
        (const void*)muca::k_sweep_sub<16, true, true, 0>,
        (const void*)muca::k_sweep_sub<16, true, false, 0>,
        (const void*)muca::k_sweep_sub<16, false, true, 1>,
        (const void*)muca::k_sweep_sub<16, false, false, 1>,
        (const void*)muca::k_sweep_sub<16, false, true, 2>,
        (const void*)muca::k_sweep_sub<16, false, false, 2>,
        (const void*)muca::k_sweep_sub<64, true, true, 0>,
        (const void*)muca::k_sweep_sub<64, true, false, 0>,
        (const void*)muca::k_sweep_sub<64, false, true, 0>,
        (const void*)muca::k_sweep_sub<64, false, false, 0>,
        (const void*)muca::k_sweep_look<true>, (const void*)muca::k_sweep_look<false>};
    for (const void* k : kernels)
      HIP_TRY_DEL(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, v));
  }

  std::vector<int32_t> wg((size_t)walkers);
  for (int i = 0; i < ngroups; ++i)
    for (int j = 0; j < c->g[i].walkers; ++j) wg[(size_t)c->g[i].first_walker + j] = i;

  int rc = MUCA_OK;
  auto run = [&]() -> int {
    int r;
    if ((r = dev_alloc(&c->d_groups, (size_t)ngroups))) return r;
    if ((r = dev_alloc(&c->d_bits, (size_t)words))) return r;
    if ((r = dev_alloc(&c->d_pos, (size_t)pos))) return r;
    if ((r = dev_alloc(&c->d_E, (size_t)walkers))) return r;
    if ((r = dev_alloc(&c->d_T, (size_t)walkers))) return r;
    if ((r = dev_alloc(&c->d_tun, (size_t)walkers))) return r;
    if ((r = dev_alloc(&c->d_wgroup, (size_t)walkers))) return r;
    if ((r = dev_alloc(&c->d_thr, (size_t)thr))) return r;
    if ((r = dev_alloc(&c->d_slope, (size_t)bins))) return r;
    if ((r = dev_alloc(&c->d_status, 1))) return r;
    if ((r = dev_alloc(&c->d_ones, (size_t)ngroups))) return r;
    if ((r = dev_alloc(&c->d_active, (size_t)ngroups))) return r;
    if ((r = dev_alloc(&c->d_flat, (size_t)ngroups))) return r;
    if ((r = dev_alloc(&c->d_iters, (size_t)ngroups))) return r;
    if ((r = dev_alloc(&c->d_counter, 2))) return r;
    HIP_TRY(hipHostMalloc((void**)&c->h_pinned, 4 * sizeof(int32_t), hipHostMallocDefault));
    HIP_TRY(hipMemcpy(c->d_groups, c->g.data(), sizeof(GroupDesc) * (size_t)ngroups,
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_wgroup, wg.data(), sizeof(int32_t) * wg.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(c->d_status, 0, sizeof(int32_t)));
    HIP_TRY(hipMemset(c->d_tun, 0, sizeof(uint32_t) * (size_t)walkers));
    hipLaunchKernelGGL(muca::k_fill_i32, dim3(1), dim3(256), 0, nullptr, c->d_ones, 1, ngroups);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(muca::k_init_place, dim3((unsigned)((walkers + 63) / 64)), dim3(64), 0,
                       nullptr, c->d_groups, c->d_wgroup, c->d_bits, c->d_pos, c->d_E, c->d_T,
                       (int)walkers, first_id, c->seed32);
    LAUNCH_CHECK();
    HIP_TRY(hipDeviceSynchronize());
    std::vector<int32_t> E((size_t)walkers);
    HIP_TRY(hipMemcpy(E.data(), c->d_E, sizeof(int32_t) * E.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < ngroups; ++i)
      for (int j = 0; j < c->g[i].walkers; ++j) {
        const int32_t e = E[(size_t)c->g[i].first_walker + j];
        if (e < c->g[i].e_lo || e > c->g[i].e_hi)
          return fail(MUCA_EINVAL, "group %d walker %d: initial energy %d outside window [%d,%d]",
                      i, j, e, c->g[i].e_lo, c->g[i].e_hi);
      }
    return MUCA_OK;
  };
  rc = run();
  if (rc != MUCA_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return MUCA_OK;
}

int mucaDefaultWindow(int d, int L, int N, int32_t* e_lo, int32_t* e_hi) {
  if (!e_lo || !e_hi) return fail(MUCA_EINVAL, "null output");
  if (d != 2 && d != 3) return fail(MUCA_EINVAL, "d must be 2 or 3");
  if (L < 3 || L > 1024) return fail(MUCA_EINVAL, "L must be in [3, 1024]");
  const int64_t V = (d == 2) ? (int64_t)L * L : (int64_t)L * L * L;
  if (V > (1 << 24)) return fail(MUCA_EINVAL, "V = L^d must not exceed 2^24");
  if (N < 1 || 2 * (int64_t)N > V) return fail(MUCA_EINVAL, "default window needs 1 <= N <= V/2");
  *e_lo = energy_floor(d, L, N);
  *e_hi = 0;
  return MUCA_OK;
}

int mucaInit(muca_ctx* out, int d, int L, int N, int walkers, uint64_t seed) {
  muca_group q{d, L, N, walkers, 0, 0};
  return mucaInitGroups(out, &q, 1, seed, 0u);
}

int mucaDestroy(muca_ctx ctx) {
  if (!ctx) return MUCA_OK;
  (void)hipDeviceSynchronize();
  delete ctx;
  return MUCA_OK;
}

int mucaNumGroups(muca_ctx c, int* n) {
  if (int r = check_ctx(c)) return r;
  if (!n) return fail(MUCA_EINVAL, "null output");
  *n = c->ngroups;
  return MUCA_OK;
}

int mucaNumWalkers(muca_ctx c, int* n) {
  if (int r = check_ctx(c)) return r;
  if (!n) return fail(MUCA_EINVAL, "null output");
  *n = c->nwalkers;
  return MUCA_OK;
}

int mucaTotalBins(muca_ctx c, int* n) {
  if (int r = check_ctx(c)) return r;
  if (!n) return fail(MUCA_EINVAL, "null output");
  *n = c->total_bins;
  return MUCA_OK;
}

int mucaGetWindow(muca_ctx c, int group, int32_t* e_lo, int32_t* e_hi, int32_t* bin_offset) {
  if (int r = check_ctx(c)) return r;
  if (group < 0 || group >= c->ngroups) return fail(MUCA_EINVAL, "group %d out of range", group);
  if (e_lo) *e_lo = c->g[group].e_lo;
  if (e_hi) *e_hi = c->g[group].e_hi;
  if (bin_offset) *bin_offset = c->g[group].bin_off;
  return MUCA_OK;
}

int mucaSetLayout(muca_ctx c, int layout) {
  if (int r = check_ctx(c)) return r;
  if (layout < MUCA_LAYOUT_AUTO || layout >= MUCA_NUM_LAYOUTS)
    return fail(MUCA_EINVAL, "unknown layout %d", layout);
  c->layout = layout;
  return MUCA_OK;
}

int mucaGetLayout(muca_ctx c, int* layout) {
  if (int r = check_ctx(c)) return r;
  if (!layout) return fail(MUCA_EINVAL, "null output");
  *layout = resolved_layout(c);
  return MUCA_OK;
}

int mucaAutotune(muca_ctx c, const double* lnW, int probe_sweeps, int* chosen, double* ms,
                 void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!lnW) return fail(MUCA_EINVAL, "lnW is NULL");
  if (int r = check_sweeps(c, probe_sweeps)) return r;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  // save walker state
  uint32_t *b0 = nullptr, *p0 = nullptr;
  int32_t *e0 = nullptr, *h = nullptr;
  uint64_t* t0 = nullptr;
  uint32_t* u0 = nullptr;
  int rc = MUCA_OK;
  double best = 1e300;
  int pick = MUCA_LAYOUT_SUB16;
  const size_t resident0 = c->resident_limit;
  size_t pick_rl = resident0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  auto save = [&](bool back) -> int {
    const auto k = hipMemcpyDeviceToDevice;
    HIP_TRY(hipMemcpyAsync(back ? c->d_bits : b0, back ? b0 : c->d_bits,
                           sizeof(uint32_t) * (size_t)c->total_words, k, s));
    HIP_TRY(hipMemcpyAsync(back ? c->d_pos : p0, back ? p0 : c->d_pos,
                           sizeof(uint32_t) * (size_t)c->total_pos, k, s));
    HIP_TRY(hipMemcpyAsync(back ? c->d_E : e0, back ? e0 : c->d_E,
                           sizeof(int32_t) * (size_t)c->nwalkers, k, s));
    HIP_TRY(hipMemcpyAsync(back ? c->d_T : t0, back ? t0 : c->d_T,
                           sizeof(uint64_t) * (size_t)c->nwalkers, k, s));
    HIP_TRY(hipMemcpyAsync(back ? c->d_tun : u0, back ? u0 : c->d_tun,
                           sizeof(uint32_t) * (size_t)c->nwalkers, k, s));
    return MUCA_OK;
  };
  auto body = [&]() -> int {
    int r;
    if ((r = dev_alloc(&b0, (size_t)c->total_words))) return r;
    if ((r = dev_alloc(&p0, (size_t)c->total_pos))) return r;
    if ((r = dev_alloc(&e0, (size_t)c->nwalkers))) return r;
    if ((r = dev_alloc(&t0, (size_t)c->nwalkers))) return r;
    if ((r = dev_alloc(&u0, (size_t)c->nwalkers))) return r;
    if ((r = dev_alloc(&h, (size_t)c->total_bins))) return r;
    HIP_TRY(hipEventCreate(&ev0));
    HIP_TRY(hipEventCreate(&ev1));
    if ((r = save(false))) return r;
    if ((r = enqueue_thresholds(c, lnW, s))) return r;
    for (int lay = MUCA_LAYOUT_LANE; lay < MUCA_NUM_LAYOUTS; ++lay) {
      // cooperative layouts with walker state in device memory: with the
      // resident cap and without it
      const int which = coop_index(lay);
      const size_t capb = std::min(c->lds_limit, c->lds_device);
      const bool dev_state =
          which >= 0 && (c->bricked || coop_sizes(c, which) + c->hist_bytes > capb);
      const int nres = dev_state && resident0 > 0 ? 2 : 1;
      for (int v = 0; v < nres; ++v) {
        const size_t rl = v == 0 ? resident0 : 0;
        if (rl != c->resident_limit) {
          c->resident_limit = rl;
          c->drop_tables();
        }
        if ((r = enqueue_zero_hist(c, h, c->d_ones, s))) return r;
        HIP_TRY(hipEventRecord(ev0, s));
        if ((r = enqueue_sweep_kernel(c, lay, probe_sweeps, h, c->d_ones, s))) return r;
        HIP_TRY(hipEventRecord(ev1, s));
        HIP_TRY(hipEventSynchronize(ev1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, ev0, ev1));
        if (ms && (v == 0 || t < ms[lay])) ms[lay] = t;
        if (t < best) {
          best = t;
          pick = lay;
          pick_rl = rl;
        }
        if ((r = save(true))) return r;
      }
    }
    HIP_TRY(hipStreamSynchronize(s));
    return MUCA_OK;
  };
  if (ms)
    for (int i = 0; i < MUCA_NUM_LAYOUTS; ++i) ms[i] = 0.0;
  rc = body();
  (void)hipFree(b0);
  (void)hipFree(p0);
  (void)hipFree(e0);
  (void)hipFree(t0);
  (void)hipFree(u0);
  (void)hipFree(h);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (c->resident_limit != pick_rl) {
    c->resident_limit = pick_rl;
    c->drop_tables();
  }
  if (rc) return rc;
  c->tuned = pick;
  if (chosen) *chosen = pick;
  return MUCA_OK;
}

int mucaGetPlacement(muca_ctx c, int* state_in_lds, int* table_in_lds) {
  if (int r = check_ctx(c)) return r;
  const int which = coop_index(resolved_layout(c));
  int st = 0, tb = 0;
  if (which >= 0) {
    const size_t need = coop_sizes(c, which);
    const size_t cap = std::min(c->lds_limit, c->lds_device);
    st = (!c->bricked && need + c->hist_bytes <= cap) ? 1 : 0;
    const size_t state = st ? need + c->hist_bytes : 0;
    tb = (c->lds_limit > 0 && state + c->tbl_bytes <= cap) ? 1 : 0;
  }
  if (state_in_lds) *state_in_lds = st;
  if (table_in_lds) *table_in_lds = tb;
  return MUCA_OK;
}

int mucaSetGraph(muca_ctx c, int enable) {
  if (int r = check_ctx(c)) return r;
  c->use_graph = enable != 0;
  return MUCA_OK;
}

int mucaSetLdsLimit(muca_ctx c, int64_t bytes) {
  if (int r = check_ctx(c)) return r;
  if (bytes < 0 || bytes > kLdsBytes) return fail(MUCA_EINVAL, "LDS limit must be in [0, 163840]");
  if ((size_t)bytes != c->lds_limit) {
    c->lds_limit = (size_t)bytes;
    c->drop_tables();
  }
  return MUCA_OK;
}

int mucaGetResidentLimit(muca_ctx c, int64_t* bytes) {
  if (int r = check_ctx(c)) return r;
  if (!bytes) return fail(MUCA_EINVAL, "null output");
  *bytes = (int64_t)c->resident_limit;
  return MUCA_OK;
}

int mucaSetResidentLimit(muca_ctx c, int64_t bytes) {
  if (int r = check_ctx(c)) return r;
  if (bytes < 0) return fail(MUCA_EINVAL, "resident limit must be >= 0");
  if ((size_t)bytes != c->resident_limit) {
    c->resident_limit = (size_t)bytes;
    c->drop_tables();
  }
  return MUCA_OK;
}

int mucaThresholdEntries(muca_ctx c, int* entries) {
  if (int r = check_ctx(c)) return r;
  if (!entries) return fail(MUCA_EINVAL, "null output");
  *entries = c->thr_entries;
  return MUCA_OK;
}

int mucaBuildThresholds(muca_ctx c, const double* lnW, uint32_t* thr_out, void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!lnW) return fail(MUCA_EINVAL, "lnW is NULL");
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  if (int r = enqueue_thresholds(c, lnW, s)) return r;
  if (thr_out)
    HIP_TRY(hipMemcpyAsync(thr_out, c->d_thr, sizeof(uint32_t) * (size_t)c->thr_entries,
                           hipMemcpyDeviceToDevice, s));
  return MUCA_OK;
}

int mucaSweepActive(muca_ctx c, const double* lnW, int sweeps, int32_t* H, const int32_t* active,
                    void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!lnW || !H) return fail(MUCA_EINVAL, "lnW and H must not be NULL");
  if (int r = check_sweeps(c, sweeps)) return r;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  return enqueue_sweep(c, lnW, sweeps, H, active ? active : c->d_ones, s);
}

int mucaSweep(muca_ctx c, const double* lnW, int sweeps, int32_t* H, void* stream) {
  return mucaSweepActive(c, lnW, sweeps, H, nullptr, stream);
}

int mucaSweepNoAlloc(muca_ctx c, const double* lnW, int sweeps, int32_t* H, void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!lnW || !H) return fail(MUCA_EINVAL, "lnW and H must not be NULL");
  if (int r = check_sweeps(c, sweeps)) return r;
  unsigned char* ws = (unsigned char*)g_static_ptr[c->device];
  if (!ws) return fail(MUCA_EHIP, "static workspace of device %d not set up", c->device);
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  const int layout = resolved_layout(c);
  // workspace: [thresholds][tasks][first], each 256-byte aligned
  auto up = [](size_t n) { return (n + 255) & ~(size_t)255; };
  const size_t thr_bytes = up((size_t)c->thr_entries * sizeof(uint32_t));
  const int which = coop_index(layout);  // -1: one walker per lane, no task table
  const int G = which >= 0 ? kCoopLanes[which] : 0;
  int nsets = 0, vmax = 0;
  if (which >= 0)
    for (const auto& g : c->g) {
      const int wpb = group_wpb(c, which, g);
      nsets += (g.walkers + wpb - 1) / wpb;
      vmax = std::max(vmax, g.V);
    }
  const size_t task_bytes = which >= 0 ? up((size_t)nsets * sizeof(SweepTask)) : 0;
  const size_t first_bytes = which >= 0 ? up(((size_t)nsets + 1) * sizeof(int32_t)) : 0;
  if (thr_bytes + task_bytes + first_bytes > kStaticBytes)
    return fail(MUCA_EINVAL,
                "mucaSweepNoAlloc: this context needs %zu bytes of workspace (threshold table "
                "%zu, tasks %zu), more than the static %zu",
                thr_bytes + task_bytes + first_bytes, thr_bytes, task_bytes + first_bytes,
                kStaticBytes);
  uint32_t* thr = (uint32_t*)ws;
  SweepTask* tasks = (SweepTask*)(ws + thr_bytes);
  int32_t* first = (int32_t*)(ws + thr_bytes + task_bytes);
  if (int r = enqueue_thresholds_to(c, lnW, thr, s)) return r;
  if (int r = enqueue_zero_hist(c, H, c->d_ones, s)) return r;
  if (which < 0) {
    hipLaunchKernelGGL(muca::k_sweep_lane, dim3((unsigned)((c->nwalkers + 63) / 64)), dim3(64),
                       0, s, c->d_groups, c->d_wgroup, c->d_bits, c->d_pos, c->d_E, c->d_T,
                       c->d_tun, thr, H, c->d_ones, c->nwalkers, sweeps, c->first_id,
                       c->seed32);
    LAUNCH_CHECK();
    return MUCA_OK;
  }
  hipLaunchKernelGGL(k_plain_tasks, dim3((unsigned)((nsets + 255) / 256)), dim3(256), 0, s,
                     c->d_groups, c->ngroups, kCoopLanes[which], kCoopSpread[which], vmax, tasks,
                     first, nsets);
  LAUNCH_CHECK();
  const size_t need = coop_sizes(c, which);
  const CoopTables q{tasks, first, nsets, need, thr};
  if (which == 4) {
    if (look_fits(c, need)) {
      launch_look_tables(c, tasks, nsets, need, thr, sweeps, H, c->d_ones, s);
      LAUNCH_CHECK();
      return MUCA_OK;
    }
    return launch_coop_tables<64>(c, 1, q, sweeps, H, c->d_ones, s);  // as SUB64
  }
  return G == 16 ? launch_coop_tables<16>(c, which, q, sweeps, H, c->d_ones, s)
                 : launch_coop_tables<64>(c, which, q, sweeps, H, c->d_ones, s);
}

int mucaUpdateWeights(muca_ctx c, const int32_t* H, double* lnW, double* P, int rule,
                      void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!H || !lnW || !P) return fail(MUCA_EINVAL, "H, lnW and P must not be NULL");
  if (rule != MUCA_RULE_BERG && rule != MUCA_RULE_SIMPLE)
    return fail(MUCA_EINVAL, "unknown rule %d", rule);
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  hipLaunchKernelGGL(muca::k_update, dim3((unsigned)c->ngroups), dim3(256), 0, s, c->d_groups, H,
                     lnW, P, c->d_slope, rule, c->d_ones, c->d_status);
  LAUNCH_CHECK();
  return MUCA_OK;
}

int mucaIsFlat(muca_ctx c, const int32_t* H, int32_t* flags, void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!H || !flags) return fail(MUCA_EINVAL, "H and flags must not be NULL");
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  hipLaunchKernelGGL(muca::k_flat, dim3((unsigned)c->ngroups), dim3(256), 0, s, c->d_groups, H,
                     flags);
  LAUNCH_CHECK();
  return MUCA_OK;
}

int mucaStatus(muca_ctx c, void* stream) {
  if (int r = check_ctx(c)) return r;
  hipStream_t s = stream ? (hipStream_t)stream : c->last_stream;
  HIP_TRY(hipStreamSynchronize(s));
  int32_t st = 0;
  HIP_TRY(hipMemcpy(&st, c->d_status, sizeof st, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(c->d_status, 0, sizeof st));
  if (st & 1) return fail(MUCA_ENONFINITE, "non-finite weight passed to a sweep");
  if (st & 2) return fail(MUCA_ENONFINITE, "weight update produced a non-finite weight");
  return MUCA_OK;
}

int mucaRun(muca_ctx c, double* lnW, double* P, int32_t* H, int sweeps_per_iter, int max_iters,
            int rule, int stop, int resume, int32_t* iters, int32_t* flat, void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!lnW || !P || !H || !iters || !flat)
    return fail(MUCA_EINVAL, "lnW, P, H, iters and flat must not be NULL");
  if (max_iters < 1) return fail(MUCA_EINVAL, "max_iters must be >= 1");
  if (rule != MUCA_RULE_BERG && rule != MUCA_RULE_SIMPLE)
    return fail(MUCA_EINVAL, "unknown rule %d", rule);
  if (stop != MUCA_STOP_NONE && stop != MUCA_STOP_FLAT && stop != MUCA_STOP_TUNNEL)
    return fail(MUCA_EINVAL, "unknown stop criterion %d", stop);
  if (int r = check_sweeps(c, sweeps_per_iter)) return r;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  const int G = c->ngroups;
  if (resume && !c->run_started)
    return fail(MUCA_EINVAL, "resume without a previous mucaRun on this context");
  if (!resume) {
    hipLaunchKernelGGL(muca::k_fill_f64,
                       dim3((unsigned)std::min(1024, (c->total_bins + 255) / 256)), dim3(256), 0,
                       s, P, 0.0, c->total_bins);
    hipLaunchKernelGGL(muca::k_fill_i32, dim3(1), dim3(256), 0, s, c->d_active, 1, G);
    hipLaunchKernelGGL(muca::k_fill_i32, dim3(1), dim3(256), 0, s, c->d_flat, 0, G);
    hipLaunchKernelGGL(muca::k_fill_i32, dim3(1), dim3(256), 0, s, c->d_iters, 0, G);
    hipLaunchKernelGGL(muca::k_fill_i32, dim3(1), dim3(64), 0, s, c->d_counter, 0, 1);
    hipLaunchKernelGGL(muca::k_fill_i32, dim3(1), dim3(64), 0, s, c->d_counter + 1, G, 1);
    LAUNCH_CHECK();
    c->run_started = true;
  }
  // one iteration: thresholds, sweep, loop control, recursion, counter
  auto enqueue_iteration = [&](hipStream_t st) -> int {
    if (int r = enqueue_sweep(c, lnW, sweeps_per_iter, H, c->d_active, st)) return r;
    hipLaunchKernelGGL(muca::k_control, dim3((unsigned)G), dim3(256), 0, st, c->d_groups, H,
                       c->d_active, c->d_flat, c->d_iters, c->d_counter, c->d_counter + 1,
                       c->d_tun, stop, c->tunnel_target);
    hipLaunchKernelGGL(muca::k_update, dim3((unsigned)G), dim3(256), 0, st, c->d_groups, H, lnW, P,
                       c->d_slope, rule, c->d_active, c->d_status);
    hipLaunchKernelGGL(muca::k_bump, dim3(1), dim3(64), 0, st, c->d_counter);
    LAUNCH_CHECK();
    return MUCA_OK;
  };
  hipStream_t rs = s;
  if (c->use_graph) {
    if (!c->run_stream) HIP_TRY(hipStreamCreateWithFlags(&c->run_stream, hipStreamNonBlocking));
    rs = c->run_stream;
    const muca_context::GraphKey key{lnW, P, H, sweeps_per_iter, rule, stop, resolved_layout(c),
                                     c->tunnel_target, c->lds_limit};
    if (!c->graph_exec || !(key == c->graph_key)) {
      if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
      if (c->graph) (void)hipGraphDestroy(c->graph);
      c->graph_exec = nullptr;
      c->graph = nullptr;
      // task tables and kernel attributes are set up outside the capture
      for (int which = 0; which < kCoops; ++which)
        if (int r = build_coop(c, which)) return r;
      HIP_TRY(hipStreamBeginCapture(rs, hipStreamCaptureModeThreadLocal));
      const int r = enqueue_iteration(rs);
      hipGraph_t gr = nullptr;
      const hipError_t e = hipStreamEndCapture(rs, &gr);
      if (r) {
        if (gr) (void)hipGraphDestroy(gr);
        return r;
      }
      HIP_TRY(e);
      c->graph = gr;
      HIP_TRY(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
      c->graph_key = key;
    }
    // order the internal stream after the caller's work
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ev, s));
    HIP_TRY(hipStreamWaitEvent(rs, ev, 0));
    HIP_TRY(hipEventDestroy(ev));
  }
  int remaining = G;
  if (resume) {  // groups already flat stay finished
    HIP_TRY(hipMemcpyAsync(c->h_pinned, c->d_counter, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipStreamSynchronize(s));
    remaining = c->h_pinned[1];
  }
  for (int i = 0; i < max_iters && remaining > 0; ++i) {
    if (c->use_graph) {
      HIP_TRY(hipGraphLaunch(c->graph_exec, rs));
    } else if (int r = enqueue_iteration(rs)) {
      return r;
    }
    if (stop != MUCA_STOP_NONE) {
      HIP_TRY(hipMemcpyAsync(c->h_pinned, c->d_counter, 2 * sizeof(int32_t),
                             hipMemcpyDeviceToHost, rs));
      HIP_TRY(hipStreamSynchronize(rs));
      remaining = c->h_pinned[1];
      if (remaining == 0) break;
    }
  }
  if (rs != s) {
    hipEvent_t ev;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ev, rs));
    HIP_TRY(hipStreamWaitEvent(s, ev, 0));
    HIP_TRY(hipEventDestroy(ev));
  }
  HIP_TRY(hipMemcpyAsync(iters, c->d_iters, sizeof(int32_t) * (size_t)G, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(flat, c->d_flat, sizeof(int32_t) * (size_t)G, hipMemcpyDeviceToHost, s));
  if (int r = mucaStatus(c, s)) return r;
  return (stop != MUCA_STOP_NONE && remaining > 0) ? MUCA_NOT_CONVERGED : MUCA_OK;
}

int mucaReweight(muca_ctx c, const double* lnW, const int32_t* H, const double* beta, int nbeta,
                 double* out, void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!lnW || !H || !beta || !out)
    return fail(MUCA_EINVAL, "lnW, H, beta and out must not be NULL");
  if (nbeta < 1) return fail(MUCA_EINVAL, "nbeta must be >= 1, got %d", nbeta);
  if ((int64_t)nbeta * c->ngroups > 0x7FFFFFFFLL)
    return fail(MUCA_EINVAL, "ngroups x nbeta exceeds the grid limit");
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  hipLaunchKernelGGL(muca::k_reweight, dim3((unsigned)(c->ngroups * nbeta)), dim3(256), 0, s,
                     c->d_groups, lnW, H, beta, nbeta, out);
  LAUNCH_CHECK();
  return MUCA_OK;
}

}  // extern "C"

namespace {

// LDS bytes of the droplet kernel for this context (two flags, the sorted
// sites padded to a power of two, the union-find parents), or 0 with the
// error set when a group does not fit.
size_t droplet_lds(muca_ctx c) {
  size_t need = 0;
  for (int i = 0; i < c->ngroups; ++i) {
    size_t npad = 1;
    while (npad < (size_t)c->g[i].N) npad <<= 1;
    need = std::max(need, 2 * sizeof(int32_t) + 4 * npad + 4 * (size_t)c->g[i].N);
  }
  if (need > c->lds_device) {
    fail(MUCA_EINVAL, "droplet measurement needs %zu bytes of LDS per block (device: %zu)",
         need, c->lds_device);
    return 0;
  }
  return need;
}

int enqueue_droplets(muca_ctx c, int32_t* out, long long* osum, int32_t* ocount, size_t need,
                     hipStream_t s) {
  hipLaunchKernelGGL(muca::k_largest_cluster, dim3((unsigned)c->nwalkers), dim3(256), need, s,
                     c->d_groups, c->d_wgroup, c->d_pos, c->d_E, out, osum, ocount);
  LAUNCH_CHECK();
  return MUCA_OK;
}

// The droplet kernel's dynamic LDS limit, raised to what the context needs
// (outside any stream capture: a host-side attribute).
int droplet_attr(size_t need) {
  HIP_TRY(hipFuncSetAttribute((const void*)muca::k_largest_cluster,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)need));
  return MUCA_OK;
}

// ---------------------------------------------------------------- checkpoint
// State image of mucaSaveState / mucaLoadState: a header, one muca_group
// record per group (window resolved), then the device arrays below, in this
// order.  It holds everything that later iterations read from library
// memory: the walker state (whose random streams are counter-based, so the
// attempt counters resume them exactly) and the loop state of mucaRun.
struct CkptHeader {
  char magic[8];
  uint32_t version, ngroups, seed32, first_id;
  int32_t nwalkers, tunnel_target, run_started, reserved;
  int64_t total_words, total_pos;
  uint64_t payload_bytes;  // bytes after the header
  uint64_t checksum;       // FNV-1a (64 bit) of those bytes
};
constexpr char kCkptMagic[8] = {'M', 'U', 'C', 'A', 'S', 'T', 'A', 'T'};
constexpr uint32_t kCkptVersion = 1;

struct CkptSection {
  void* dev;
  size_t bytes;
};

std::vector<CkptSection> ckpt_sections(muca_ctx c) {
  const size_t W = (size_t)c->nwalkers, G = (size_t)c->ngroups;
  return {{c->d_bits, sizeof(uint32_t) * (size_t)c->total_words},
          {c->d_pos, sizeof(uint32_t) * (size_t)c->total_pos},
          {c->d_E, sizeof(int32_t) * W},
          {c->d_T, sizeof(uint64_t) * W},
          {c->d_tun, sizeof(uint32_t) * W},
          {c->d_active, sizeof(int32_t) * G},
          {c->d_flat, sizeof(int32_t) * G},
          {c->d_iters, sizeof(int32_t) * G},
          {c->d_counter, sizeof(int32_t) * 2}};
}

size_t ckpt_payload(muca_ctx c) {
  size_t n = sizeof(muca_group) * (size_t)c->ngroups;
  for (const auto& q : ckpt_sections(c)) n += q.bytes;
  return n;
}

muca_group ckpt_group(const GroupDesc& g) {
  return muca_group{g.d, g.L, g.N, g.walkers, g.e_lo, g.e_hi};
}

// Fowler-Noll-Vo FNV-1a, 64-bit offset basis and prime.
uint64_t fnv1a64(const unsigned char* p, size_t n) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

}  // namespace

extern "C" {

int mucaLargestCluster(muca_ctx c, int32_t* out, void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!out) return fail(MUCA_EINVAL, "out must not be NULL");
  const size_t need = droplet_lds(c);
  if (!need) return MUCA_EINVAL;
  if (int r = droplet_attr(need)) return r;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  return enqueue_droplets(c, out, nullptr, nullptr, need, s);
}

int mucaMeasureDroplets(muca_ctx c, long long* osum, int32_t* ocount, int32_t* out,
                        void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!osum || !ocount) return fail(MUCA_EINVAL, "osum and ocount must not be NULL");
  const size_t need = droplet_lds(c);
  if (!need) return MUCA_EINVAL;
  if (int r = droplet_attr(need)) return r;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  return enqueue_droplets(c, out, osum, ocount, need, s);
}

int mucaProduction(muca_ctx c, const double* lnW, int sweeps_between, int measurements,
                   int32_t* H, long long* osum, int32_t* ocount, void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!lnW || !H || !osum || !ocount)
    return fail(MUCA_EINVAL, "lnW, H, osum and ocount must not be NULL");
  if (measurements < 1) return fail(MUCA_EINVAL, "measurements must be >= 1");
  if (int r = check_sweeps(c, sweeps_between)) return r;
  if ((int64_t)sweeps_between * measurements > 2147483647LL)
    return fail(MUCA_EOVERFLOW, "sweeps_between x measurements exceeds INT32_MAX");
  if (int r = check_sweeps(c, sweeps_between * measurements)) return r;
  const size_t need = droplet_lds(c);
  if (!need) return MUCA_EINVAL;
  if (int r = droplet_attr(need)) return r;
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  const unsigned fill = (unsigned)std::min(1024, (c->total_bins + 255) / 256);
  hipLaunchKernelGGL(muca::k_fill_i64, dim3(fill), dim3(256), 0, s, osum, 0LL, c->total_bins);
  hipLaunchKernelGGL(muca::k_fill_i32, dim3(fill), dim3(256), 0, s, ocount, 0, c->total_bins);
  LAUNCH_CHECK();
  if (int r = enqueue_thresholds(c, lnW, s)) return r;
  if (int r = enqueue_zero_hist(c, H, c->d_ones, s)) return r;
  const int layout = resolved_layout(c);
  for (int m = 0; m < measurements; ++m) {
    if (int r = enqueue_sweep_kernel(c, layout, sweeps_between, H, c->d_ones, s)) return r;
    if (int r = enqueue_droplets(c, nullptr, osum, ocount, need, s)) return r;
  }
  return MUCA_OK;
}

int mucaReweightObservable(muca_ctx c, const double* lnW, const int32_t* ocount,
                           const long long* osum, const double* beta, int nbeta, double* out,
                           void* stream) {
  if (int r = check_ctx(c)) return r;
  if (!lnW || !ocount || !osum || !beta || !out)
    return fail(MUCA_EINVAL, "lnW, ocount, osum, beta and out must not be NULL");
  if (nbeta < 1) return fail(MUCA_EINVAL, "nbeta must be >= 1, got %d", nbeta);
  if ((int64_t)nbeta * c->ngroups > 0x7FFFFFFFLL)
    return fail(MUCA_EINVAL, "ngroups x nbeta exceeds the grid limit");
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  hipLaunchKernelGGL(muca::k_reweight_obs, dim3((unsigned)(c->ngroups * nbeta)), dim3(256), 0, s,
                     c->d_groups, lnW, ocount, osum, beta, nbeta, out);
  LAUNCH_CHECK();
  return MUCA_OK;
}

int mucaCalibrateRandomLines(const uint32_t* table, int64_t table_bytes, uint32_t* sink,
                             int64_t sink_words, int rounds, double* lines_read, double* seconds,
                             void* stream) {
  if (!table || !sink || !lines_read || !seconds)
    return fail(MUCA_EINVAL, "table, sink, lines_read and seconds must not be NULL");
  const int64_t lines = table_bytes / 128;
  if (lines < 1 || lines > 0xFFFFFFFFLL)
    return fail(MUCA_EINVAL, "table must hold 1 .. 2^32 - 1 lines of 128 bytes");
  if (rounds < 1) return fail(MUCA_EINVAL, "rounds must be >= 1");
  if (sink_words < 256) return fail(MUCA_EINVAL, "sink must hold at least 256 words");
  const int64_t blocks = std::min<int64_t>(sink_words / 256, 1 << 20);
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  auto run = [&]() -> int {
    // one untimed launch, then the timed one
    for (int k = 0; k < 2; ++k) {
      if (k == 1) HIP_TRY(hipEventRecord(a, s));
      hipLaunchKernelGGL(muca::k_random_lines, dim3((unsigned)blocks), dim3(256), 0, s, table,
                         (uint32_t)lines, rounds, (uint32_t)(k * 7919), sink);
      LAUNCH_CHECK();
    }
    HIP_TRY(hipEventRecord(b, s));
    HIP_TRY(hipEventSynchronize(b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    *seconds = ms * 1e-3;
    *lines_read = (double)blocks * 256.0 * 8.0 * (double)rounds;
    return MUCA_OK;
  };
  const int rc = run();
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

int mucaSetTunnelTarget(muca_ctx c, int target) {
  if (int r = check_ctx(c)) return r;
  if (target < 1) return fail(MUCA_EINVAL, "tunnelling target must be >= 1, got %d", target);
  c->tunnel_target = target;
  return MUCA_OK;
}

int mucaGetTunnel(muca_ctx c, uint32_t* last_end, uint32_t* trips) {
  if (int r = check_ctx(c)) return r;
  HIP_TRY(hipDeviceSynchronize());
  std::vector<uint32_t> st((size_t)c->nwalkers);
  HIP_TRY(hipMemcpy(st.data(), c->d_tun, sizeof(uint32_t) * st.size(), hipMemcpyDeviceToHost));
  for (size_t i = 0; i < st.size(); ++i) {
    if (last_end) last_end[i] = st[i] & 3u;
    if (trips) trips[i] = st[i] >> 2;
  }
  return MUCA_OK;
}

int mucaStateBytes(muca_ctx c, int64_t* bytes) {
  if (int r = check_ctx(c)) return r;
  if (!bytes) return fail(MUCA_EINVAL, "bytes must not be NULL");
  *bytes = (int64_t)(sizeof(CkptHeader) + ckpt_payload(c));
  return MUCA_OK;
}

int mucaSaveState(muca_ctx c, void* image, int64_t bytes) {
  if (int r = check_ctx(c)) return r;
  const size_t payload = ckpt_payload(c), need = sizeof(CkptHeader) + payload;
  if (!image) return fail(MUCA_EINVAL, "image must not be NULL");
  if (bytes < (int64_t)need)
    return fail(MUCA_EINVAL, "state image needs %zu bytes, got %lld", need, (long long)bytes);
  HIP_TRY(hipDeviceSynchronize());
  unsigned char* out = static_cast<unsigned char*>(image);
  unsigned char* p = out + sizeof(CkptHeader);
  for (const auto& g : c->g) {
    const muca_group r = ckpt_group(g);
    std::memcpy(p, &r, sizeof r);
    p += sizeof r;
  }
  for (const auto& q : ckpt_sections(c)) {
    HIP_TRY(hipMemcpy(p, q.dev, q.bytes, hipMemcpyDeviceToHost));
    p += q.bytes;
  }
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, sizeof h.magic);
  h.version = kCkptVersion;
  h.ngroups = (uint32_t)c->ngroups;
  h.seed32 = c->seed32;
  h.first_id = c->first_id;
  h.nwalkers = c->nwalkers;
  h.tunnel_target = c->tunnel_target;
  h.run_started = c->run_started ? 1 : 0;
  h.total_words = c->total_words;
  h.total_pos = c->total_pos;
  h.payload_bytes = payload;
  h.checksum = fnv1a64(out + sizeof(CkptHeader), payload);
  std::memcpy(out, &h, sizeof h);
  return MUCA_OK;
}

int mucaLoadState(muca_ctx c, const void* image, int64_t bytes) {
  if (int r = check_ctx(c)) return r;
  if (!image) return fail(MUCA_EINVAL, "image must not be NULL");
  const size_t payload = ckpt_payload(c), need = sizeof(CkptHeader) + payload;
  if (bytes < (int64_t)sizeof(CkptHeader))
    return fail(MUCA_EINVAL, "state image of %lld bytes has no header", (long long)bytes);
  const unsigned char* in = static_cast<const unsigned char*>(image);
  CkptHeader h;
  std::memcpy(&h, in, sizeof h);
  if (std::memcmp(h.magic, kCkptMagic, sizeof h.magic) != 0 || h.version != kCkptVersion)
    return fail(MUCA_EINVAL, "not a state image of this library (magic or version)");
  if (h.ngroups != (uint32_t)c->ngroups || h.nwalkers != c->nwalkers ||
      h.total_words != c->total_words || h.total_pos != c->total_pos ||
      h.payload_bytes != payload)
    return fail(MUCA_EINVAL, "state image was saved from a context of other groups");
  if (bytes < (int64_t)need)
    return fail(MUCA_EINVAL, "state image truncated: %lld of %zu bytes", (long long)bytes, need);
  if (h.seed32 != c->seed32 || h.first_id != c->first_id)
    return fail(MUCA_EINVAL, "state image was saved with seed %u, first id %u (context: %u, %u)",
                h.seed32, h.first_id, c->seed32, c->first_id);
  if (h.tunnel_target < 1 || (h.run_started != 0 && h.run_started != 1))
    return fail(MUCA_EINVAL, "state image header is corrupt");
  const unsigned char* p = in + sizeof(CkptHeader);
  if (fnv1a64(p, payload) != h.checksum)
    return fail(MUCA_EINVAL, "state image checksum mismatch (corrupt image)");
  for (const auto& g : c->g) {
    muca_group r;
    std::memcpy(&r, p, sizeof r);
    const muca_group m = ckpt_group(g);
    if (std::memcmp(&r, &m, sizeof r) != 0)
      return fail(MUCA_EINVAL, "state image was saved from a context of other groups");
    p += sizeof r;
  }
  HIP_TRY(hipDeviceSynchronize());
  for (const auto& q : ckpt_sections(c)) {
    HIP_TRY(hipMemcpy(q.dev, p, q.bytes, hipMemcpyHostToDevice));
    p += q.bytes;
  }
  c->tunnel_target = h.tunnel_target;
  c->run_started = h.run_started != 0;
  return MUCA_OK;
}

int mucaReadWalker(muca_ctx c, int walker, uint32_t* bits, uint32_t* pos, int32_t* E,
                   uint64_t* t) {
  if (int r = check_ctx(c)) return r;
  if (walker < 0 || walker >= c->nwalkers) return fail(MUCA_EINVAL, "walker %d out of range", walker);
  HIP_TRY(hipDeviceSynchronize());
  int gi = 0;
  while (gi + 1 < c->ngroups && walker >= c->g[gi + 1].first_walker) ++gi;
  const GroupDesc& g = c->g[gi];
  const int64_t j = walker - g.first_walker;
  if (bits) {
    HIP_TRY(hipMemcpy(bits, c->d_bits + g.bits_off + j * g.words, sizeof(uint32_t) * g.words,
                      hipMemcpyDeviceToHost));
    if (g.brick8) {  // bricked (see bit_ref) -> linear
      std::vector<uint32_t> raw(bits, bits + g.words);
      std::fill(bits, bits + g.words, 0u);
      const uint32_t L = (uint32_t)g.L, nb = (uint32_t)g.brick8;
      for (uint32_t z = 0, s = 0; z < L; ++z)
        for (uint32_t y = 0; y < L; ++y)
          for (uint32_t x = 0; x < L; ++x, ++s) {
            const uint32_t b = ((z >> 3) * nb + (y >> 3)) * nb + (x >> 3);
            const uint32_t w = (b << 4) | ((z & 7u) << 1) | ((y & 7u) >> 2);
            const uint32_t k = (x & 7u) | ((y & 3u) << 3);
            if ((raw[w] >> k) & 1u) bits[s >> 5] |= 1u << (s & 31u);
          }
    }
  }
  if (pos)
    HIP_TRY(hipMemcpy(pos, c->d_pos + g.pos_off + j * g.N, sizeof(uint32_t) * g.N,
                      hipMemcpyDeviceToHost));
  if (E) HIP_TRY(hipMemcpy(E, c->d_E + walker, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (t) HIP_TRY(hipMemcpy(t, c->d_T + walker, sizeof(uint64_t), hipMemcpyDeviceToHost));
  return MUCA_OK;
}

}  // extern "C"
