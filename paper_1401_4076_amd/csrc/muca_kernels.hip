// muca_kernels.hip -- HIP kernels of the parallel multicanonical iteration
// for gfx950: initial placement, acceptance thresholds, the equilibrium
// sweep (one walker per lane), histogram clearing, the binary64 weight
// recursion and the flatness test.  Each kernel cites the step of the
// method it implements (paper Sec. 2-4).
#include "muca_kernels.h"

#pragma clang fp contract(off)

namespace muca {

// ---------------------------------------------------------------- placement
// Fixed particle number (Sec. 3): N distinct uniform random sites per walker,
// drawn from the placement stream (counters (i_lo, i_hi, 0, 1)); an occupied
// candidate is skipped.  E is then counted once per occupied pair.
__global__ void k_init_place(const GroupDesc* __restrict__ groups,
                             const int32_t* __restrict__ wgroup, uint32_t* __restrict__ bits,
                             uint32_t* __restrict__ pos, int32_t* __restrict__ E,
                             uint64_t* __restrict__ T, int nwalkers, uint32_t first_id,
                             uint32_t seed32) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwalkers) return;
  const GroupDesc g = groups[wgroup[w]];
  const int64_t j = w - g.first_walker;
  uint32_t* wb = bits + g.bits_off + j * g.words;
  uint32_t* wp = pos + g.pos_off + j * g.N;
  for (int i = 0; i < g.words; ++i) wb[i] = 0u;
  const uint32_t key0 = first_id + (uint32_t)w;
  int placed = 0;
  for (uint64_t i = 0; placed < g.N; ++i) {
    const U4 r = philox((uint32_t)i, (uint32_t)(i >> 32), 0u, 1u, key0, seed32);
    const uint32_t cand[4] = {r.x, r.y, r.z, r.w};
    for (int c = 0; c < 4 && placed < g.N; ++c) {
      const uint32_t s = draw(cand[c], (uint32_t)g.V);
      if (!occupied(g, wb, s)) {
        set_site(g, wb, s);
        wp[placed++] = s;
      }
    }
  }
  int pairs = 0;
  for (int k = 0; k < g.N; ++k) {
    uint32_t nb[6];
    neighbours(g, wp[k], nb);
    for (int a = 0; a < g.d; ++a) {  // + direction of each axis: each pair once
      const uint32_t q = nb[2 * a];
      pairs += occupied(g, wb, q);
    }
  }
  E[w] = -pairs;
  T[w] = 0;
}

// ---------------------------------------------------------------- thresholds
// Acceptance min(1, W(E_n)/W(E_o)) of Sec. 2 tabulated per (b_o, dE) from
// binary64 lnW; window exits are "never".  grid.y = group.
__global__ void k_thresholds(const GroupDesc* __restrict__ groups, const double* __restrict__ lnW,
                             uint32_t* __restrict__ thr, int32_t* __restrict__ status) {
  const GroupDesc g = groups[blockIdx.y];
  const int n = g.nbins * g.nd;
  const double* lw = lnW + g.bin_off;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int bo = i / g.nd;
    const int dE = i - bo * g.nd - 2 * g.d;
    const int bn = bo + dE;
    uint32_t T = 0u;
    if (bn >= 0 && bn < g.nbins) {
      const double a = lw[bn], b = lw[bo];
      if (!isfinite(a) || !isfinite(b)) {
        atomicOr(status, 1);
      } else {
        T = threshold(a - b);
      }
    }
    thr[g.thr_off + i] = T;
  }
}

// ---------------------------------------------------------------- histograms
__global__ void k_zero_hist(const GroupDesc* __restrict__ groups, const int32_t* __restrict__ active,
                            int32_t* __restrict__ H) {
  const int gi = blockIdx.y;
  if (active && !active[gi]) return;
  const GroupDesc g = groups[gi];
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < g.nbins; b += gridDim.x * blockDim.x)
    H[g.bin_off + b] = 0;
}

// ---------------------------------------------------------------- sweep (lane)
// Equilibrium run with fixed weights (Sec. 2), one walker per lane, walker
// state in device memory.  One attempt t: Philox block (t_lo, t_hi, 0, 0) =
// (x0, x1, x2, x3); particle k = draw(x0, N) at s_o; the first empty site
// among draw(x2, V), draw(x3, V), then the words of blocks r = 1, 2, ... is
// s_n; dE = k_o - k_n with k_n not counting s_o; accept iff the threshold of
// (E_o, dE) admits x1.  After each sweep of V attempts (Sec. 4) the walker
// adds one entry at its energy (eq. (2)).
__global__ void __launch_bounds__(64) k_sweep_lane(
    const GroupDesc* __restrict__ groups, const int32_t* __restrict__ wgroup,
    uint32_t* __restrict__ bits, uint32_t* __restrict__ pos, int32_t* __restrict__ E,
    uint64_t* __restrict__ T, uint32_t* __restrict__ tun, const uint32_t* __restrict__ thr,
    int32_t* __restrict__ H, const int32_t* __restrict__ active, int nwalkers, int sweeps,
    uint32_t first_id, uint32_t seed32) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwalkers) return;
  const int gi = wgroup[w];
  if (active && !active[gi]) return;
  const GroupDesc g = groups[gi];
  const int64_t j = w - g.first_walker;
  uint32_t* wb = bits + g.bits_off + j * g.words;
  uint32_t* wp = pos + g.pos_off + j * g.N;
  const uint32_t* th = thr + g.thr_off;
  int32_t* hg = H + g.bin_off;
  const uint32_t key0 = first_id + (uint32_t)w;
  int32_t e = E[w];
  uint64_t t = T[w];
  uint32_t tn = tun[w];
  const uint32_t V = (uint32_t)g.V, N = (uint32_t)g.N;
  for (int sw = 0; sw < sweeps; ++sw) {
    for (uint32_t a = 0; a < V; ++a, ++t) {
      const uint32_t tl = (uint32_t)t, th_ = (uint32_t)(t >> 32);
      U4 r = philox(tl, th_, 0u, 0u, key0, seed32);
      const uint32_t u = r.y;
      const uint32_t k = draw(r.x, N);
      const uint32_t so = wp[k];
      uint32_t sn = draw(r.z, V);
      if (occupied(g, wb, sn)) {
        sn = draw(r.w, V);
        uint32_t blk = 0;
        while (occupied(g, wb, sn)) {
          blk += 1;
          r = philox(tl, th_, blk, 0u, key0, seed32);
          sn = draw(r.x, V);
          if (!occupied(g, wb, sn)) break;
          sn = draw(r.y, V);
          if (!occupied(g, wb, sn)) break;
          sn = draw(r.z, V);
          if (!occupied(g, wb, sn)) break;
          sn = draw(r.w, V);
        }
      }
      uint32_t nb[6];
      int ko = 0, kn = 0;
      neighbours(g, so, nb);
      for (int q = 0; q < 2 * g.d; ++q) ko += occupied(g, wb, nb[q]);
      neighbours(g, sn, nb);
      for (int q = 0; q < 2 * g.d; ++q)
        kn += (nb[q] != so) ? occupied(g, wb, nb[q]) : 0u;
      const int dE = ko - kn;
      const uint32_t Tacc = th[(e - g.e_lo) * g.nd + dE + 2 * g.d];
      if (accepts(Tacc, u)) {
        clear_site(g, wb, so);
        set_site(g, wb, sn);
        wp[k] = sn;
        e += dE;
      }
    }
    atomicAdd(&hg[e - g.e_lo], 1);
    tn = tunnel_step(tn, e - g.e_lo, g.nbins - 1);
  }
  E[w] = e;
  T[w] = t;
  tun[w] = tn;
}

// ---------------------------------------------------------------- recursion
// Next weights from lnW and the summed histogram (Sec. 2).  One block per
// active group.  The Berg rule first computes every slope in parallel, then
// one lane rebuilds lnW from lnW(e_hi) = 0 downward in a fixed order.
__global__ void __launch_bounds__(256) k_update(const GroupDesc* __restrict__ groups,
                                                const int32_t* __restrict__ H,
                                                double* __restrict__ lnW, double* __restrict__ P,
                                                double* __restrict__ slope, int rule,
                                                const int32_t* __restrict__ active,
                                                int32_t* __restrict__ status) {
  const int gi = blockIdx.x;
  if (active && !active[gi]) return;
  const GroupDesc g = groups[gi];
  const int nb = g.nbins;
  const int32_t* h = H + g.bin_off;
  double* lw = lnW + g.bin_off;
  double* pp = P + g.bin_off;
  double* d = slope + g.bin_off;
  __shared__ int lo_s, hi_s, bad_s;
  if (threadIdx.x == 0) {
    lo_s = nb;
    hi_s = -1;
    bad_s = 0;
  }
  __syncthreads();
  if (rule == 1) {
    // W^{i+1}(E) = W^i(E) / H^i(E); an empty bin keeps its weight.
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      const int32_t hb = h[b] > 0 ? h[b] : 1;
      d[b] = lw[b] - log_ieee(hb);
    }
    __syncthreads();
    const double top = d[nb - 1];
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      const double v = d[b] - top;
      lw[b] = v;
      if (!isfinite(v)) bad_s = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && bad_s) atomicOr(status, 2);
    return;
  }
  // Berg: p-weighted mean of the slope estimates of all iterations.
  int lo = nb, hi = -1;
  for (int b = threadIdx.x; b + 1 < nb; b += blockDim.x) {
    const double slope_old = lw[b + 1] - lw[b];
    if (h[b] > 0 && h[b + 1] > 0) {
      const double h0 = (double)h[b], h1 = (double)h[b + 1];
      const double p = h0 * h1 / (h0 + h1);
      const double acc = pp[b] + p;
      pp[b] = acc;
      const double kappa = p / acc;
      d[b] = slope_old + kappa * (log_ieee(h[b]) - log_ieee(h[b + 1]));
    } else {
      d[b] = slope_old;
    }
    if (pp[b] > 0.0) {
      lo = min(lo, b);
      hi = max(hi, b);
    }
  }
  atomicMin(&lo_s, lo);
  atomicMax(&hi_s, hi);
  __syncthreads();
  const int elo = lo_s, ehi = hi_s;
  if (ehi >= 0) {  // frontier: copy the nearest estimated slope outward
    const double dl = d[elo], dh = d[ehi];
    __syncthreads();
    for (int b = threadIdx.x; b + 1 < nb; b += blockDim.x) {
      if (b < elo) d[b] = dl;
      if (b > ehi) d[b] = dh;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    lw[nb - 1] = v;
    int bad = 0;
    for (int b = nb - 2; b >= 0; --b) {
      v = v - d[b];
      lw[b] = v;
      bad |= !isfinite(v);
    }
    if (bad) atomicOr(status, 2);
  }
}

// ---------------------------------------------------------------- flatness
// flat <=> both window ends visited and 2 min_{H>0} H > max H.
__device__ __forceinline__ int group_flat(const int32_t* h, int nb, int* mn_s, int* mx_s) {
  int mn = 0x7FFFFFFF, mx = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const int v = h[b];
    if (v > 0) mn = min(mn, v);
    mx = max(mx, v);
  }
  atomicMin(mn_s, mn);
  atomicMax(mx_s, mx);
  __syncthreads();
  return (h[0] > 0 && h[nb - 1] > 0 && 2LL * (long long)(*mn_s) > (long long)(*mx_s)) ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_flat(const GroupDesc* __restrict__ groups,
                                              const int32_t* __restrict__ H,
                                              int32_t* __restrict__ flags) {
  const GroupDesc g = groups[blockIdx.x];
  __shared__ int mn_s, mx_s;
  if (threadIdx.x == 0) {
    mn_s = 0x7FFFFFFF;
    mx_s = 0;
  }
  __syncthreads();
  const int f = group_flat(H + g.bin_off, g.nbins, &mn_s, &mx_s);
  if (threadIdx.x == 0) flags[blockIdx.x] = f;
}

// Loop control of the iteration: for each active group record the flatness
// of H^i and the iteration count.  stop = 1: a flat group becomes inactive
// (keeps lnW^i, H^i); stop = 2: so does a group whose walkers have made
// tunnel_target tunnelling events in total (Sec. 4).  remaining = number of
// groups still active.
__global__ void __launch_bounds__(256) k_control(const GroupDesc* __restrict__ groups,
                                                 const int32_t* __restrict__ H,
                                                 int32_t* __restrict__ active,
                                                 int32_t* __restrict__ flat,
                                                 int32_t* __restrict__ iters,
                                                 int32_t* __restrict__ iter_counter,
                                                 int32_t* __restrict__ remaining,
                                                 const uint32_t* __restrict__ tun, int stop,
                                                 int tunnel_target) {
  const int gi = blockIdx.x;
  if (!active[gi]) return;
  const GroupDesc g = groups[gi];
  __shared__ int mn_s, mx_s;
  __shared__ unsigned long long trips_s;
  if (threadIdx.x == 0) {
    mn_s = 0x7FFFFFFF;
    mx_s = 0;
    trips_s = 0ull;
  }
  __syncthreads();
  const int f = group_flat(H + g.bin_off, g.nbins, &mn_s, &mx_s);
  if (stop == 2) {
    unsigned long long n = 0ull;
    for (int j = threadIdx.x; j < g.walkers; j += blockDim.x) n += tun[g.first_walker + j] >> 2;
    atomicAdd(&trips_s, n);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    flat[gi] = f;
    iters[gi] = *iter_counter + 1;
    if ((stop == 1 && f) || (stop == 2 && trips_s >= (unsigned long long)tunnel_target)) {
      active[gi] = 0;
      atomicSub(remaining, 1);
    }
  }
}

// ---------------------------------------------------------------- reweighting
// Canonical averages from a multicanonical histogram (Sec. 3: the data are
// reweighted to the temperatures of interest).  A run with weights W visits E
// with probability ~ Omega(E) W(E), so ln Omega(E) = ln H(E) - ln W(E) on the
// visited bins, up to a constant.  At inverse temperature beta (J = 1) the
// canonical weight of E is exp(ln Omega(E) - beta E); with a(E) that exponent
// and m its largest value over the visited bins:
//   ln Z = m + ln sum exp(a - m),  <E>, <E^2> the weighted means,
//   C = beta^2 sum w (E - <E>)^2 / sum w  (taken about the mean).
// One block per (group, beta); reductions in a fixed order.
namespace {
template <typename Op>
__device__ __forceinline__ double block_reduce(double v, double* red, Op op) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = op(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}
}  // namespace

__global__ void __launch_bounds__(256) k_reweight(const GroupDesc* __restrict__ groups,
                                                  const double* __restrict__ lnW,
                                                  const int32_t* __restrict__ H,
                                                  const double* __restrict__ beta, int nbeta,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  const int gi = blockIdx.x / nbeta, k = blockIdx.x - gi * nbeta;
  const GroupDesc g = groups[gi];
  const double b = beta[k];
  const int32_t* h = H + g.bin_off;
  const double* lw = lnW + g.bin_off;
  auto expo = [&](int i) { return log((double)h[i]) - lw[i] - b * (double)(g.e_lo + i); };
  double m = -INFINITY;
  for (int i = threadIdx.x; i < g.nbins; i += blockDim.x)
    if (h[i] > 0) m = fmax(m, expo(i));
  m = block_reduce(m, red, [](double x, double y) { return fmax(x, y); });
  double* o = out + 4 * ((size_t)gi * (size_t)nbeta + (size_t)k);
  if (m == -INFINITY) {  // no visited bin (uniform over the block)
    if (threadIdx.x < 4) o[threadIdx.x] = NAN;
    return;
  }
  const auto add = [](double x, double y) { return x + y; };
  double z = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < g.nbins; i += blockDim.x)
    if (h[i] > 0) {
      const double w = exp(expo(i) - m);
      z += w;
      s1 += w * (double)(g.e_lo + i);
    }
  z = block_reduce(z, red, add);
  s1 = block_reduce(s1, red, add);
  const double mean = s1 / z;
  double s2 = 0.0, sc = 0.0;
  for (int i = threadIdx.x; i < g.nbins; i += blockDim.x)
    if (h[i] > 0) {
      const double w = exp(expo(i) - m);
      const double e = (double)(g.e_lo + i);
      s2 += w * e * e;
      sc += w * (e - mean) * (e - mean);
    }
  s2 = block_reduce(s2, red, add);
  sc = block_reduce(sc, red, add);
  if (threadIdx.x == 0) {
    o[0] = m + log(z);
    o[1] = mean;
    o[2] = s2 / z;
    o[3] = b * b * sc / z;
  }
}

// ---------------------------------------------------------------- droplets
// Size of the largest cluster of nearest-neighbour-bonded particles of each
// walker (Sec. 3 follows condensation through the largest droplet).  One
// block per walker.  LDS: the walker's particle sites, sorted (bitonic), so
// that a neighbour site is found among the occupied ones by binary search for
// any lattice size; then a union-find forest over the positions of the sorted
// array (the clusters do not depend on how particles are numbered).  A link
// is one compare-and-swap that points a root at a smaller root, so parent
// chains strictly decrease: every walk up a chain ends within N steps and
// every union retries at most N times (a retry means another link took the
// root; at most N - 1 links exist).  The loops are bounded by those counts; a
// bound that is ever reached reports -1.
//
// With osum != nullptr the size is also added, at the walker's current
// energy bin, to osum (int64, exact) and ocount counts the measurement: the
// energy-binned measurement of a production run.
namespace {
__device__ __forceinline__ int root_of(const int32_t* parent, int x, int n) {
  for (int k = 0; k <= n; ++k) {
    const int px = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (px == x) return x;
    x = px;
  }
  return -1;
}

// Index of site t in the ascending array S[0, n), or -1.
__device__ __forceinline__ int find_site(const uint32_t* S, int n, uint32_t t) {
  int lo = 0, hi = n;  // first index with S[i] >= t lies in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (S[mid] < t) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && S[lo] == t) ? lo : -1;
}
}  // namespace

__global__ void __launch_bounds__(256) k_largest_cluster(
    const GroupDesc* __restrict__ groups, const int32_t* __restrict__ wgroup,
    const uint32_t* __restrict__ pos, const int32_t* __restrict__ E, int32_t* __restrict__ out,
    long long* __restrict__ osum, int32_t* __restrict__ ocount) {
  // LDS (dynamic only): [best, error flag] [S: npad sorted sites, later the
  // cluster sizes] [parent: N]
  extern __shared__ uint32_t smem[];
  const int w = blockIdx.x;
  const GroupDesc g = groups[wgroup[w]];
  const int N = g.N, L = g.L;
  int npad = 1;
  while (npad < N) npad <<= 1;
  int32_t* flags = reinterpret_cast<int32_t*>(smem);
  uint32_t* S = smem + 2;
  int32_t* cnt = reinterpret_cast<int32_t*>(S);
  int32_t* parent = reinterpret_cast<int32_t*>(S + npad);
  const uint32_t* p = pos + g.pos_off + (int64_t)(w - g.first_walker) * N;
  for (int i = threadIdx.x; i < npad; i += blockDim.x) S[i] = i < N ? p[i] : 0xFFFFFFFFu;
  for (int i = threadIdx.x; i < N; i += blockDim.x) parent[i] = i;
  if (threadIdx.x == 0) {
    flags[0] = 0;
    flags[1] = 0;
  }
  __syncthreads();
  // bitonic sort, ascending (the padding sorts to the end)
  for (int k = 2; k <= npad; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < npad; i += blockDim.x) {
        const int ij = i ^ j;
        if (ij > i) {
          const uint32_t a = S[i], b = S[ij];
          if ((a > b) == ((i & k) == 0)) {
            S[i] = b;
            S[ij] = a;
          }
        }
      }
      __syncthreads();
    }
  bool bad = false;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int s = (int)S[i];
    const int x = s % L, y = (s / L) % L, z = s / g.LL;
    for (int dir = 0; dir < 2 * g.d; ++dir) {
      const int axis = dir >> 1;
      const int c = axis == 0 ? x : (axis == 1 ? y : z);
      const int stride = axis == 0 ? 1 : (axis == 1 ? L : g.LL);
      const int t = (dir & 1) == 0 ? (c == L - 1 ? s - (L - 1) * stride : s + stride)
                                   : (c == 0 ? s + (L - 1) * stride : s - stride);
      const int j = find_site(S, N, (uint32_t)t);
      if (j < 0 || j >= i) continue;  // each bond once, from its higher index
      int tries = 0;
      for (; tries <= N; ++tries) {
        const int a = root_of(parent, i, N), b = root_of(parent, j, N);
        if (a < 0 || b < 0) {
          tries = N + 1;
          break;
        }
        if (a == b) break;
        const int hi = a > b ? a : b, lo = a > b ? b : a;
        if (atomicCAS(&parent[hi], hi, lo) == hi) break;
      }
      if (tries > N) bad = true;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) cnt[i] = 0;  // the sites are done
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int r = root_of(parent, i, N);
    if (r < 0) bad = true;
    else atomicAdd(&cnt[r], 1);
  }
  __syncthreads();
  int m = 0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) m = cnt[i] > m ? cnt[i] : m;
  atomicMax(&flags[0], m);
  if (bad) atomicOr(&flags[1], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int size = flags[1] ? -1 : flags[0];
    if (out) out[w] = size;
    if (osum) {
      const int b = E[w] - g.e_lo;  // the walker's energy lies in its window
      atomicAdd(reinterpret_cast<unsigned long long*>(&osum[g.bin_off + b]),
                (unsigned long long)(long long)size);
      atomicAdd(&ocount[g.bin_off + b], 1);
    }
  }
}

// Canonical average of an observable measured during a production run
// (Sec. 3: the data are reweighted to the temperatures of interest): osum[b]
// is the sum of the observable over the cnt[b] measurements taken at bin b,
// so (osum / cnt)(E) is its microcanonical mean, and
//   <O>_beta = sum_E (osum / cnt)(E) Omega(E) exp(-beta E) / sum_E Omega(E) exp(-beta E)
// with ln Omega(E) = ln cnt(E) - ln W(E) over the bins with cnt > 0.  One block
// per (group, beta); the sums are shifted by the largest exponent and reduced
// in a fixed order.  NaN for a group without a measurement.
__global__ void __launch_bounds__(256) k_reweight_obs(const GroupDesc* __restrict__ groups,
                                                      const double* __restrict__ lnW,
                                                      const int32_t* __restrict__ cnt,
                                                      const long long* __restrict__ osum,
                                                      const double* __restrict__ beta, int nbeta,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  const int gi = blockIdx.x / nbeta, k = blockIdx.x - gi * nbeta;
  const GroupDesc g = groups[gi];
  const double b = beta[k];
  const int32_t* h = cnt + g.bin_off;
  const long long* o = osum + g.bin_off;
  const double* lw = lnW + g.bin_off;
  auto expo = [&](int i) { return log((double)h[i]) - lw[i] - b * (double)(g.e_lo + i); };
  double m = -INFINITY;
  for (int i = threadIdx.x; i < g.nbins; i += blockDim.x)
    if (h[i] > 0) m = fmax(m, expo(i));
  m = block_reduce(m, red, [](double x, double y) { return fmax(x, y); });
  if (m == -INFINITY) {  // no measurement (uniform over the block)
    if (threadIdx.x == 0) out[(size_t)gi * nbeta + k] = NAN;
    return;
  }
  const auto add = [](double x, double y) { return x + y; };
  double z = 0.0, so = 0.0;
  for (int i = threadIdx.x; i < g.nbins; i += blockDim.x)
    if (h[i] > 0) {
      const double w = exp(expo(i) - m);
      z += w;
      so += w * ((double)o[i] / (double)h[i]);
    }
  z = block_reduce(z, red, add);
  so = block_reduce(so, red, add);
  if (threadIdx.x == 0) out[(size_t)gi * nbeta + k] = so / z;
}

// ---------------------------------------------------------------- calibration
// Random-line read rate of the device: every lane follows 8 independent
// streams of uniformly random 128-byte lines of the table (one 4-byte load
// per line, so each miss moves a whole line) and folds the values into one
// word per lane.  Streams are xorshift32 generators; a line index is
// floor(x lines / 2^32).
__global__ void __launch_bounds__(256) k_random_lines(const uint32_t* __restrict__ table,
                                                      uint32_t lines, int rounds, uint32_t seed,
                                                      uint32_t* __restrict__ sink) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = (tid * 8u + (uint32_t)j) * 0x9E3779B9u + seed + 1u;
  uint32_t acc = 0u;
  for (int r = 0; r < rounds; ++r) {
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      x[j] ^= x[j] << 13;
      x[j] ^= x[j] >> 17;
      x[j] ^= x[j] << 5;
      const uint32_t line = __umulhi(x[j], lines);
      v[j] = table[(size_t)line * 32u];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += v[j];
  }
  sink[tid] = acc;
}

__global__ void k_bump(int32_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter += 1;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_i64(long long* __restrict__ p, long long v, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_f64(double* __restrict__ p, double v, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace muca
