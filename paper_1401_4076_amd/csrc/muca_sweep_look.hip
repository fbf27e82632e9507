// muca_sweep_look.hip -- equilibrium sweep, one walker per wavefront, four
// attempts looked at per step (paper Sec. 2: fixed weights, acceptance
// min(1, W(E_n)/W(E_o)); Sec. 4: a sweep is L^d attempts).
//
// Each 16-lane row of the wavefront gathers the neighbourhood of one of the
// next four attempts in the same instruction; the four decisions are then
// taken in order on the scalar unit:
//  * a decision reads the threshold of (E, dE) from a window of threshold
//    rows E - 2d .. E + 2d held in registers (reloaded after each step in
//    which E changed; a decision outside the window reads the table);
//  * an accepted move is written to the walker state in LDS, patched into
//    the prefetched particle sites of later attempts of the batch, and marks
//    every later row of the step whose gathered sites contain the move's
//    sites or whose particle is the moved one;
//  * a marked row, a row whose first candidate is occupied (and, in 3D, whose
//    second candidate's neighbourhood was not gathered), is redone exactly by
//    a single-attempt path on the current state.
// Hence every decision sees exactly the state the sequential chain would
// see, and random numbers, candidate order and decisions equal those of the
// other layouts.  Walker state, the threshold table (when it fits) and the
// block histogram live in LDS; the batch of 64 attempts is laid out so that
// lane 16q + s holds attempt 4s + q, which row q reads at step s.
#include "muca_kernels.h"

#pragma clang fp contract(off)

namespace muca {

namespace {

struct Role {
  uint32_t shift, edge;
  int32_t step, wrap;
};

__device__ __forceinline__ Role role_of(const GroupDesc& g, int dir) {
  Role r{0u, 0xFFFFFFFFu, 0, 0};
  if (dir < 0) return r;
  const int axis = dir >> 1;
  const int32_t stride = axis == 0 ? 1 : (axis == 1 ? g.L : g.LL);
  r.shift = kXyzBits * (uint32_t)axis;
  if ((dir & 1) == 0) {
    r.edge = (uint32_t)(g.L - 1);
    r.step = stride;
    r.wrap = -(g.L - 1) * stride;
  } else {
    r.edge = 0u;
    r.step = -stride;
    r.wrap = (g.L - 1) * stride;
  }
  return r;
}

__device__ __forceinline__ uint32_t at_role(const Role& r, uint32_t lin, uint32_t xyz) {
  const uint32_t c = (xyz >> r.shift) & kXyzMask;
  return lin + (uint32_t)((c == r.edge) ? r.wrap : r.step);
}

// Value of lane `src` (per-lane source, through the LDS crossbar).
__device__ __forceinline__ uint32_t from_lane(uint32_t v, int src) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

__device__ __forceinline__ uint32_t rl(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Marks a wave-uniform value as such (keeps it in a scalar register).
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

struct Look {
  const GroupDesc* g;
  uint32_t* bits;
  uint32_t* plin;
  uint32_t* pxyz;
  const uint32_t* th;
  int32_t* hist;
  int lane, ls, d2, nd, full;
  uint32_t V, N, key0, seed32, in_sweep;
  int32_t E, Ew;  // current energy, energy at which the window was loaded
  uint64_t t;
  uint32_t tun;  // tunnelling state (see tunnel_step)
  // roles of the fast gather (per row): [0,2d) nbr(s_o), 2d: c2, 2d+1: c3,
  // [2d+2, 4d+2) nbr(c2), [4d+2, 6d+2) nbr(c3) when full
  Role role;
  bool on, r_so, r_c3;
  Role role2;  // second gather: lanes [0, 2d) of each row, nbr of s_n
  // threshold window entries (r, c) -> r nd + c, lanes of three registers
  uint32_t tw0, tw1, tw2;
  int32_t wr0, wc0, wr1, wc1, wr2, wc2;
  // batch of 64 attempts: lane 16q + s holds attempt 4s + q
  uint32_t b_k, b_u, b_c2, b_c2x, b_c3, b_c3x, b_so, b_sox;
};

__device__ __forceinline__ uint32_t window_entry(const Look& W, int32_t r, int32_t c) {
  const GroupDesc& g = *W.g;
  if (r < 0) return 0u;
  const int32_t E = W.E + r - W.d2;
  if (E < g.e_lo || E > g.e_hi || c < 0) return 0u;
  return W.th[(E - g.e_lo) * W.nd + c];
}

__device__ __forceinline__ void load_window(Look& W) {
  W.Ew = W.E;
  W.tw0 = window_entry(W, W.wr0, W.wc0);
  W.tw1 = window_entry(W, W.wr1, W.wc1);
  W.tw2 = window_entry(W, W.wr2, W.wc2);
}

// Threshold of (E, dE) for the current E.
__device__ __forceinline__ uint32_t threshold_of(const Look& W, int dE) {
  const int dr = uni(W.E - W.Ew);
  if (dr >= -W.d2 && dr <= W.d2) {
    const int idx = (dr + W.d2) * W.nd + dE + W.d2;
    if (idx < 64) return rl(W.tw0, idx);
    if (idx < 128) return rl(W.tw1, idx - 64);
    return rl(W.tw2, idx - 128);
  }
  const GroupDesc& g = *W.g;
  return W.th[(W.E - g.e_lo) * W.nd + dE + W.d2];  // uniform address
}

// One attempt on the current state with all rows doing the same work; used
// for marked rows and rare cases.  Returns dE, sets sn / snx.
__device__ __forceinline__ int exact_attempt(Look& W, uint32_t so, uint32_t sox, uint32_t c2, uint32_t c2x,
                             uint32_t c3, uint32_t c3x, uint64_t ta, uint32_t* sn_out,
                             uint32_t* snx_out) {
  const GroupDesc& g = *W.g;
  const int d2 = W.d2;
  const uint32_t dmask = (1u << d2) - 1u;
  const uint32_t blin = W.r_so ? so : (W.r_c3 ? c3 : c2);
  const uint32_t bxyz = W.r_so ? sox : (W.r_c3 ? c3x : c2x);
  const uint32_t site = at_role(W.role, blin, bxyz);
  uint32_t v = 0;
  if (W.on) v = W.bits[site >> 5];
  const bool occ = W.on && ((v >> (site & 31u)) & 1u);
  const bool isso = W.on && (site == so);
  const uint32_t m = (uint32_t)__ballot(occ) & 0xFFFFu;  // row 0 (all rows identical)
  const uint32_t mx = (uint32_t)__ballot(isso) & 0xFFFFu;
  const uint32_t nm = m & ~mx;
  const int ko = __popc(m & dmask);
  const bool c2free = !((m >> d2) & 1u), c3free = !((m >> (d2 + 1)) & 1u);
  if (c2free) {
    *sn_out = c2;
    *snx_out = c2x;
    return ko - __popc((nm >> (d2 + 2)) & dmask);
  }
  if (W.full && c3free) {
    *sn_out = c3;
    *snx_out = c3x;
    return ko - __popc((nm >> (2 * d2 + 2)) & dmask);
  }
  uint32_t sn = c3, snx = c3x;
  if (!c3free) {
    uint32_t blk = 0;
    for (;;) {
      blk += 1;
      const U4 q = philox((uint32_t)ta, (uint32_t)(ta >> 32), blk, 0u, W.key0, W.seed32);
      const int l4 = W.ls & 3;
      const uint32_t word = (l4 == 0) ? q.x : (l4 == 1) ? q.y : (l4 == 2) ? q.z : q.w;
      const uint32_t cand = draw(word, W.V);
      uint32_t vv = 0;
      if (W.ls < 4) vv = W.bits[cand >> 5];
      const bool fr = (W.ls < 4) && !((vv >> (cand & 31u)) & 1u);
      const uint32_t fm = (uint32_t)__ballot(fr) & 0xFu;
      if (fm) {
        const int first = __ffs(fm) - 1;
        const uint32_t pick = first == 0 ? q.x : first == 1 ? q.y : first == 2 ? q.z : q.w;
        sn = draw(pick, W.V);
        snx = site_xyz(g, sn);
        break;
      }
    }
  }
  const uint32_t s3 = at_role(W.role2, sn, snx);
  uint32_t v3 = 0;
  const bool on3 = W.ls < d2;
  if (on3) v3 = W.bits[s3 >> 5];
  const bool occ3 = on3 && ((v3 >> (s3 & 31u)) & 1u) && (s3 != so);
  *sn_out = sn;
  *snx_out = snx;
  return ko - __popc((uint32_t)__ballot(occ3) & 0xFFFFu);
}

__device__ __forceinline__ void batch(Look& W) {
  const GroupDesc& g = *W.g;
  const int q = W.lane >> 4, s = W.lane & 15;
  const uint64_t tl = W.t + (uint64_t)(4 * s + q);
  const U4 r = philox((uint32_t)tl, (uint32_t)(tl >> 32), 0u, 0u, W.key0, W.seed32);
  W.b_k = draw(r.x, W.N);
  W.b_u = r.y;
  W.b_c2 = draw(r.z, W.V);
  W.b_c3 = draw(r.w, W.V);
  W.b_c2x = site_xyz(g, W.b_c2);
  W.b_c3x = site_xyz(g, W.b_c3);
  W.b_so = W.plin[W.b_k];
  W.b_sox = W.pxyz[W.b_k];
}

// Step S of the batch: attempts 4S .. 4S+3 (those below nb).
__device__ __forceinline__ void step(Look& W, int S, int nb) {
  const GroupDesc& g = *W.g;
  const int d2 = W.d2;
  const uint32_t dmask = (1u << d2) - 1u;
  // fast gather: row q takes attempt 4S + q, held by batch lane 16q + S
  const int src = (W.lane & 48) + S;
  const uint32_t so = from_lane(W.b_so, src), sox = from_lane(W.b_sox, src);
  const uint32_t c2 = from_lane(W.b_c2, src), c2x = from_lane(W.b_c2x, src);
  const uint32_t c3 = from_lane(W.b_c3, src), c3x = from_lane(W.b_c3x, src);
  const uint32_t k_row = from_lane(W.b_k, src);
  const uint32_t blin = W.r_so ? so : (W.r_c3 ? c3 : c2);
  const uint32_t bxyz = W.r_so ? sox : (W.r_c3 ? c3x : c2x);
  const uint32_t site = at_role(W.role, blin, bxyz);
  uint32_t v = 0;
  if (W.on) v = W.bits[site >> 5];
  const uint64_t OCC = __ballot(W.on && ((v >> (site & 31u)) & 1u));
  const uint64_t SO = __ballot(W.on && (site == so));
  const int E0 = W.E;
  uint32_t dirty = 0;  // rows whose gathered view is stale
  for (int q = 0; q < 4; ++q) {
    const int a = 4 * S + q;
    if (a < nb) {
      const int bl = 16 * q + S;  // batch lane of this attempt
      const uint32_t m = uni((uint32_t)(OCC >> (16 * q)) & 0xFFFFu);
      const uint32_t nm = uni(m & ~((uint32_t)(SO >> (16 * q)) & 0xFFFFu));
      const bool c2free = !((m >> d2) & 1u), c3free = !((m >> (d2 + 1)) & 1u);
      const uint32_t k = rl(W.b_k, bl);
      int dE;
      uint32_t sn, snx;
      dirty = uni(dirty);
      if (!((dirty >> q) & 1u) && (c2free || (W.full && c3free))) {
        dE = __popc(m & dmask) - __popc((nm >> (c2free ? d2 + 2 : 2 * d2 + 2)) & dmask);
        sn = rl(c2free ? W.b_c2 : W.b_c3, bl);
        snx = rl(c2free ? W.b_c2x : W.b_c3x, bl);
      } else {
        dE = exact_attempt(W, rl(W.b_so, bl), rl(W.b_sox, bl), rl(W.b_c2, bl), rl(W.b_c2x, bl),
                           rl(W.b_c3, bl), rl(W.b_c3x, bl), W.t + (uint64_t)a, &sn, &snx);
      }
      dE = uni(dE);
      sn = uni(sn);
      snx = uni(snx);
      const uint32_t T = uni(threshold_of(W, dE));
      const uint32_t u = rl(W.b_u, bl);
      if (accepts(T, u)) {
        const uint32_t so_a = rl(W.b_so, bl);
        if (W.lane == 0) {
          W.plin[k] = sn;
          W.pxyz[k] = snx;
          atomicAnd(&W.bits[so_a >> 5], ~(1u << (so_a & 31u)));
          atomicOr(&W.bits[sn >> 5], 1u << (sn & 31u));
        }
        // later attempts of the batch that chose the same particle
        const bool same = W.b_k == k;
        W.b_so = same ? sn : W.b_so;
        W.b_sox = same ? snx : W.b_sox;
        W.E += dE;
        // rows of this step whose gathered view the move touched
        const bool hit = (W.on && (site == so_a || site == sn)) || (k_row == k);
        const uint64_t HB = __ballot(hit);
        for (int r = q + 1; r < 4; ++r)
          if ((HB >> (16 * r)) & 0xFFFFull) dirty |= 1u << r;
        dirty = uni(dirty);
      }
      W.in_sweep += 1;
      if (W.in_sweep == W.V) {
        W.in_sweep = 0;
        if (W.lane == 0) atomicAdd(&W.hist[W.E - g.e_lo], 1);
        W.tun = tunnel_step(W.tun, W.E - g.e_lo, g.nbins - 1);
      }
    }
  }
  if (W.E != E0) load_window(W);
}

}  // namespace

template <bool kTbl>
__global__ void __launch_bounds__(256) k_sweep_look(
    const GroupDesc* __restrict__ groups, const SweepTask* __restrict__ tasks,
    uint32_t* __restrict__ gbits, uint32_t* __restrict__ gpos, int32_t* __restrict__ gE,
    uint64_t* __restrict__ gT, uint32_t* __restrict__ gtun, const uint32_t* __restrict__ thr,
    int32_t* __restrict__ H, const int32_t* __restrict__ active, int sweeps, uint32_t first_id,
    uint32_t seed32, int tbl_words, int hist_words) {
  // LDS: [threshold table (tbl_words)] [block histogram (hist_words)] [walker slots]
  extern __shared__ uint32_t smem[];
  const SweepTask task = tasks[blockIdx.x];
  if (active && !active[task.group]) return;  // uniform per block
  const GroupDesc g = groups[task.group];
  Look W;
  W.g = &g;
  W.lane = threadIdx.x & 63;
  W.ls = W.lane & 15;
  const int slot = threadIdx.x >> 6;
  const bool has = slot < task.count;
  const int w = task.first + slot;
  const int64_t j = w - g.first_walker;
  uint32_t* sb = gbits + g.bits_off + j * g.words;
  uint32_t* sp = gpos + g.pos_off + j * g.N;
  if constexpr (kTbl) {
    const uint32_t* src = thr + g.thr_off;
    const int n = g.nbins * g.nd;
    for (int i = threadIdx.x; i < n; i += blockDim.x) smem[i] = src[i];
  }
  int32_t* lhist = reinterpret_cast<int32_t*>(smem + tbl_words);
  for (int i = threadIdx.x; i < g.nbins; i += blockDim.x) lhist[i] = 0;
  W.bits = smem + (size_t)tbl_words + (size_t)hist_words +
           (size_t)slot * (size_t)(g.words + 2 * g.N);
  W.plin = W.bits + g.words;
  W.pxyz = W.plin + g.N;
  if (has) {
    for (int i = W.lane; i < g.words; i += 64) W.bits[i] = sb[i];
    for (int i = W.lane; i < g.N; i += 64) {
      const uint32_t s = sp[i];
      W.plin[i] = s;
      W.pxyz[i] = site_xyz(g, s);
    }
  }
  __syncthreads();

  if (has) {
    const int d2 = 2 * g.d, ls = W.ls;
    W.d2 = d2;
    W.nd = g.nd;
    W.V = (uint32_t)g.V;
    W.N = (uint32_t)g.N;
    W.full = (3 * d2 + 2 <= 16) ? 1 : 0;
    const int nroles = W.full ? 3 * d2 + 2 : 2 * d2 + 2;
    W.on = ls < nroles;
    W.r_so = ls < d2;
    W.r_c3 = (ls == d2 + 1) || (ls >= 2 * d2 + 2 && ls < nroles);
    int dir = -1;
    if (ls < d2) dir = ls;
    else if (ls >= d2 + 2 && ls < 2 * d2 + 2) dir = ls - d2 - 2;
    else if (ls >= 2 * d2 + 2 && ls < nroles) dir = ls - 2 * d2 - 2;
    W.role = role_of(g, dir);
    W.role2 = role_of(g, ls < d2 ? ls : -1);
    if constexpr (kTbl) W.th = smem;
    else W.th = thr + g.thr_off;
    W.hist = lhist;
    W.key0 = first_id + (uint32_t)w;
    W.seed32 = seed32;
    W.E = gE[w];
    W.t = gT[w];
    W.tun = gtun[w];
    W.in_sweep = 0;
    const int nd = W.nd, nw = nd * nd;
    const int i0 = W.lane, i1 = W.lane + 64, i2 = W.lane + 128;
    W.wr0 = i0 < nw ? i0 / nd : -1;
    W.wc0 = i0 < nw ? i0 % nd : -1;
    W.wr1 = i1 < nw ? i1 / nd : -1;
    W.wc1 = i1 < nw ? i1 % nd : -1;
    W.wr2 = i2 < nw ? i2 / nd : -1;
    W.wc2 = i2 < nw ? i2 % nd : -1;
    load_window(W);
    const int64_t total = (int64_t)sweeps * (int64_t)W.V;
    for (int64_t done = 0; done < total; done += 64) {
      const int nb = (int)((total - done) < 64 ? (total - done) : 64);
      batch(W);
      for (int S = 0; 4 * S < nb; ++S) step(W, S, nb);
      W.t += (uint64_t)nb;
    }
    if (W.lane == 0) {
      gE[w] = W.E;
      gT[w] = W.t;
      gtun[w] = W.tun;
    }
  }
  __syncthreads();
  if (has) {
    for (int i = W.lane; i < g.words; i += 64) sb[i] = W.bits[i];
    for (int i = W.lane; i < g.N; i += 64) sp[i] = W.plin[i];
  }
  for (int i = threadIdx.x; i < g.nbins; i += blockDim.x)
    if (lhist[i]) atomicAdd(&H[g.bin_off + i], lhist[i]);
}

template __global__ void k_sweep_look<true>(const GroupDesc*, const SweepTask*, uint32_t*,
                                            uint32_t*, int32_t*, uint64_t*, uint32_t*,
                                            const uint32_t*, int32_t*, const int32_t*, int,
                                            uint32_t, uint32_t, int, int);
template __global__ void k_sweep_look<false>(const GroupDesc*, const SweepTask*, uint32_t*,
                                             uint32_t*, int32_t*, uint64_t*, uint32_t*,
                                             const uint32_t*, int32_t*, const int32_t*, int,
                                             uint32_t, uint32_t, int, int);

}  // namespace muca
