/*
 * muca_ref.c -- CPU oracle of the parallel multicanonical (MUCA) iteration.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE: a plain, slow, single-threaded
 * definition of what the GPU library computes, written from the paper
 * (Zierenberg, Wiedenmann, Janke, arXiv:1401.4076) and the pinned readings
 * below.  It is loaded only by tests/, the smoke check and the CPU-baseline
 * leg of bench.py.  It shares no code with paper_1401_4076_amd/.
 *
 * Compile with -ffp-contract=off and without fast-math: the acceptance
 * thresholds and the weight recursion are reproduced bit for bit on the GPU,
 * so every floating-point operation below is a single IEEE-754 binary64
 * operation in the order written.  No libm exp/log is used; floor, ldexp and
 * frexp are exact operations.
 *
 * Readings where the paper is silent (each is restated where it is used):
 *   move      pick a uniform random particle, jump to a uniform random empty
 *             site (symmetric proposal, so min(1, W_n/W_o) is exact balance)
 *   RNG       Philox4x32-10, key = (global walker id, low 32 bits of seed),
 *             attempt t uses counters (t_lo, t_hi, r, 0), r = 0, 1, ...;
 *             initial placement uses counters (i_lo, i_hi, 0, 1)
 *   uniform   uniform(u, n) = (u * n) >> 32 in 64-bit arithmetic
 *   accept    x = lnW(E_n) - lnW(E_o); accept always if x >= 0, never if
 *             x < -23, else iff u < floor(exp(x) * 2^32), where a value of
 *             2^32 - 1 or more also means always
 *   histogram one entry per walker after each sweep of V = L^d attempts
 *   window    [e_lo, e_hi]; moves leaving it are rejected
 *   recursion Berg's error-weighted recursion on adjacent bins (default)
 *             or the simple rule W^{i+1} = W^i / H^i of Sec. 2
 *   flatness  both window ends visited and 2 * min_{H>0} H > max H
 */
#include "muca_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#pragma GCC optimize("fp-contract=off")

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).       */
/* ------------------------------------------------------------------------ */

void ref_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u; /* Weyl sequence key schedule */
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Map a 32-bit word to {0, ..., n-1} by multiply-shift. */
static uint32_t uniform(uint32_t u, uint32_t n) {
  return (uint32_t)(((uint64_t)u * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------------ */
/* exp and log from IEEE operations only.                                    */
/* ------------------------------------------------------------------------ */

/* ln 2 split so that k * LN2_HI is exact for |k| < 2^20 (Cody-Waite). */
static const double LN2_HI = 0x1.62e42ff000000p-1;
static const double LN2_LO = -0x1.718432a1b0e26p-35;
static const double INV_LN2 = 0x1.71547652b82fep+0;
static const double SQRT_HALF = 0x1.6a09e667f3bcdp-1;

/* exp(x) for -23 <= x < 0: x = k ln2 + r with |r| <= ln2/2, exp(r) by the
 * Taylor polynomial of degree 13 (truncation below 2^-56), scaled by 2^k. */
double ref_exp(double x) {
  static double c[14]; /* c_n = 1/n!, n! exact in binary64 for n <= 13 */
  static int ready = 0;
  if (!ready) {
    double fact = 1.0;
    for (int n = 0; n <= 13; ++n) {
      if (n > 1) fact = fact * (double)n;
      c[n] = 1.0 / fact;
    }
    ready = 1;
  }
  double k = floor(x * INV_LN2 + 0.5);
  double r = (x - k * LN2_HI) - k * LN2_LO;
  double q = c[13];
  for (int n = 12; n >= 0; --n) q = q * r + c[n];
  return ldexp(q, (int)k);
}

/* ln(h) for integer h >= 1: h = m 2^e with m in [sqrt(1/2), sqrt(2)),
 * ln m = 2 atanh(s) with s = (m-1)/(m+1), series through s^21. */
double ref_log(int64_t h) {
  int e;
  double m = frexp((double)h, &e);
  if (m < SQRT_HALF) {
    m = m * 2.0;
    e = e - 1;
  }
  double f = m - 1.0;
  double s = f / (2.0 + f);
  double z = s * s;
  double q = 1.0 / 21.0;
  for (int j = 9; j >= 0; --j) q = q * z + 1.0 / (double)(2 * j + 1);
  double lnm = (2.0 * s) * q;
  return (double)e * LN2_HI + ((double)e * LN2_LO + lnm);
}

/* Sec. 2: a proposed state E_n is accepted with probability
 * min(1, W(E_n)/W(E_o)) = min(1, exp(x)), x = lnW(E_n) - lnW(E_o).
 * Realised with one 32-bit uniform u: P(accept) = floor(exp(x) 2^32) / 2^32. */
int ref_accept(double x, uint32_t u) {
  if (x >= 0.0) return 1;
  if (x < -23.0) return 0; /* exp(x) 2^32 < 1 */
  double v = floor(ldexp(ref_exp(x), 32));
  if (v >= 4294967295.0) return 1;
  return (double)u < v;
}

/* ------------------------------------------------------------------------ */
/* Lattice: sites s = x + L y (+ L^2 z), periodic, 2d nearest neighbours.   */
/* ------------------------------------------------------------------------ */

static int64_t ipow(int L, int d) {
  int64_t v = 1;
  for (int i = 0; i < d; ++i) v *= L;
  return v;
}

/* Neighbour of site s in direction dir (axis dir/2, +1 for even dir, -1 for odd). */
static uint32_t neighbour(int d, int L, uint32_t s, int dir) {
  uint32_t coord[3];
  uint32_t rest = s;
  for (int a = 0; a < d; ++a) {
    coord[a] = rest % (uint32_t)L;
    rest /= (uint32_t)L;
  }
  int a = dir / 2;
  if (dir % 2 == 0)
    coord[a] = (coord[a] + 1) % (uint32_t)L;
  else
    coord[a] = (coord[a] + (uint32_t)L - 1) % (uint32_t)L;
  uint32_t out = 0;
  for (int b = d - 1; b >= 0; --b) out = out * (uint32_t)L + coord[b];
  return out;
}

/* Number of occupied nearest neighbours of site s, not counting `skip`. */
static int occupied_neighbours(int d, int L, const uint8_t* n, uint32_t s, int64_t skip) {
  int k = 0;
  for (int dir = 0; dir < 2 * d; ++dir) {
    uint32_t q = neighbour(d, L, s, dir);
    if ((int64_t)q != skip && n[q]) ++k;
  }
  return k;
}

/* Sec. 3, eq. (5) with J = 1: E = -(number of occupied nearest-neighbour pairs). */
static int32_t energy(int d, int L, const uint8_t* n) {
  int64_t V = ipow(L, d);
  int32_t pairs = 0;
  for (int64_t s = 0; s < V; ++s) {
    if (!n[s]) continue;
    for (int dir = 0; dir < 2 * d; dir += 2) /* each pair once: + directions */
      if (n[neighbour(d, L, (uint32_t)s, dir)]) ++pairs;
  }
  return -pairs;
}

/* ------------------------------------------------------------------------ */
/* Default energy window [E_floor, 0].  The paper takes the range from short */
/* parallel-tempering runs (Sec. 3); the reading here is the energy of a     */
/* compact, non-wrapping cluster built by filling rows and layers.           */
/* ------------------------------------------------------------------------ */

/* Bonds of m sites filled row by row with rows of width w (open boundaries). */
static int64_t row_fill_bonds(int64_t m, int64_t w) {
  int64_t q = m / w, r = m % w, b = 0;
  b += q * (w - 1);               /* bonds inside full rows */
  if (r > 0) b += r - 1;          /* inside the partial row */
  if (q > 1) b += (q - 1) * w;    /* between full rows */
  if (q > 0) b += r;              /* partial row onto the last full row */
  return b;
}

/* Best row filling of m sites inside a w_max x h_max rectangle; -1 if none fits. */
static int64_t best_rect_bonds(int64_t m, int64_t w_max, int64_t h_max) {
  if (m == 0) return 0;
  int64_t best = -1;
  for (int64_t w = 1; w <= w_max; ++w) {
    int64_t rows = (m + w - 1) / w;
    if (rows > h_max) continue;
    int64_t b = row_fill_bonds(m, w);
    if (b > best) best = b;
  }
  return best;
}

int32_t ref_energy_floor(int d, int L, int N) {
  int64_t lim = L - 1; /* extents below L: no bond wraps round the torus */
  int64_t best = 0;
  if (d == 2) {
    int64_t b = best_rect_bonds(N, lim, lim);
    if (b > best) best = b;
  } else {
    for (int64_t x = 1; x <= lim; ++x)
      for (int64_t y = 1; y <= lim; ++y) {
        int64_t z = N / (x * y), m = N - x * y * z;
        if (z + (m > 0 ? 1 : 0) > lim) continue;
        int64_t box = 0;
        if (z > 0) box = (x - 1) * y * z + x * (y - 1) * z + x * y * (z - 1);
        int64_t top = best_rect_bonds(m, x, y);
        if (top < 0) continue;
        int64_t b = box + top + (z > 0 ? m : 0); /* partial layer sits on the box */
        if (b > best) best = b;
      }
  }
  return (int32_t)(-best);
}

/* ------------------------------------------------------------------------ */
/* Exact density of states by enumeration (test pin for the sampler).       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int d, L, N;
  int64_t V;
  uint8_t* n;
  int64_t* omega;
} dos_walk;

static void dos_rec(dos_walk* w, int64_t first, int placed, int bonds) {
  if (placed == w->N) {
    w->omega[bonds] += 1;
    return;
  }
  for (int64_t s = first; s <= w->V - (w->N - placed); ++s) {
    int add = occupied_neighbours(w->d, w->L, w->n, (uint32_t)s, -1);
    w->n[s] = 1;
    dos_rec(w, s + 1, placed + 1, bonds + add);
    w->n[s] = 0;
  }
}

int ref_brute_dos(int d, int L, int N, int64_t* omega) {
  if ((d != 2 && d != 3) || L < 3 || N < 0) return -1;
  int64_t V = ipow(L, d);
  if (N > V) return -1;
  dos_walk w;
  w.d = d; w.L = L; w.N = N; w.V = V;
  w.n = (uint8_t*)calloc((size_t)V, 1);
  w.omega = omega;
  memset(omega, 0, sizeof(int64_t) * (size_t)(d * N + 1));
  dos_rec(&w, 0, 0, 0);
  free(w.n);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Walkers and groups.                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int group;
  uint32_t id;    /* global walker id = Philox key word 0 */
  uint8_t* n;     /* occupation n_i of every site */
  uint32_t* pos;  /* site of every particle */
  int32_t E;
  uint64_t t;     /* attempts made so far */
  uint32_t last_end;  /* window end visited last: 0 none yet, 1 bottom, 2 top */
  uint32_t trips;     /* tunnelling events completed (see tunnel_visit) */
} walker;

struct ref_ctx {
  int ngroups;
  ref_group* g;   /* with resolved windows */
  int* first_walker;
  int* bin_off;
  int total_bins;
  int nwalkers;
  walker* w;
  uint32_t seed32;
};

int ref_num_groups(const ref_ctx* c) { return c->ngroups; }
int ref_total_bins(const ref_ctx* c) { return c->total_bins; }
int ref_num_walkers(const ref_ctx* c) { return c->nwalkers; }
int ref_bin_offset(const ref_ctx* c, int g) {
  return (g < 0 || g >= c->ngroups) ? -1 : c->bin_off[g];
}
int ref_window(const ref_ctx* c, int g, int32_t* e_lo, int32_t* e_hi) {
  if (g < 0 || g >= c->ngroups) return -1;
  *e_lo = c->g[g].e_lo;
  *e_hi = c->g[g].e_hi;
  return 0;
}

/* Uniform random placement of N particles (fixed particle number, Sec. 3):
 * candidate sites uniform(word, V) in stream order, an occupied candidate is
 * skipped. */
static void place(walker* w, const ref_group* g, uint32_t seed32) {
  int64_t V = ipow(g->L, g->d);
  memset(w->n, 0, (size_t)V);
  uint32_t key[2] = {w->id, seed32};
  int count = 0;
  for (uint64_t i = 0; count < g->N; ++i) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0, 1};
    uint32_t x[4];
    ref_philox(ctr, key, x);
    for (int j = 0; j < 4 && count < g->N; ++j) {
      uint32_t s = uniform(x[j], (uint32_t)V);
      if (!w->n[s]) {
        w->n[s] = 1;
        w->pos[count++] = s;
      }
    }
  }
  w->E = energy(g->d, g->L, w->n);
  w->t = 0;
}

void ref_destroy(ref_ctx* c) {
  if (!c) return;
  for (int i = 0; i < c->nwalkers; ++i) {
    free(c->w[i].n);
    free(c->w[i].pos);
  }
  free(c->w);
  free(c->g);
  free(c->first_walker);
  free(c->bin_off);
  free(c);
}

ref_ctx* ref_create(const ref_group* g, int ngroups, uint64_t seed, uint32_t first_id) {
  if (ngroups < 1) return NULL;
  ref_ctx* c = (ref_ctx*)calloc(1, sizeof(ref_ctx));
  c->ngroups = ngroups;
  c->g = (ref_group*)malloc(sizeof(ref_group) * (size_t)ngroups);
  c->first_walker = (int*)malloc(sizeof(int) * (size_t)ngroups);
  c->bin_off = (int*)malloc(sizeof(int) * (size_t)ngroups);
  c->seed32 = (uint32_t)seed;
  int64_t total_w = 0, total_b = 0;
  for (int i = 0; i < ngroups; ++i) {
    ref_group q = g[i];
    if ((q.d != 2 && q.d != 3) || q.L < 3 || q.L > 1024 || q.N < 1 || q.walkers < 1) goto fail;
    int64_t V = ipow(q.L, q.d);
    if (q.N > V - 1) goto fail;
    if (q.e_lo == 0 && q.e_hi == 0) {
      if (2 * (int64_t)q.N > V) goto fail; /* E = 0 needs N <= V/2 */
      q.e_lo = ref_energy_floor(q.d, q.L, q.N);
      q.e_hi = 0;
    }
    if (q.e_lo > q.e_hi || q.e_hi > 0 || q.e_lo < -q.d * q.N) goto fail;
    c->g[i] = q;
    c->first_walker[i] = (int)total_w;
    c->bin_off[i] = (int)total_b;
    total_w += q.walkers;
    total_b += q.e_hi - q.e_lo + 1;
  }
  c->nwalkers = (int)total_w;
  c->total_bins = (int)total_b;
  c->w = (walker*)calloc((size_t)total_w, sizeof(walker));
  for (int i = 0; i < ngroups; ++i) {
    const ref_group* q = &c->g[i];
    int64_t V = ipow(q->L, q->d);
    for (int j = 0; j < q->walkers; ++j) {
      walker* w = &c->w[c->first_walker[i] + j];
      w->group = i;
      w->id = first_id + (uint32_t)(c->first_walker[i] + j);
      w->n = (uint8_t*)malloc((size_t)V);
      w->pos = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)q->N);
      place(w, q, c->seed32);
      if (w->E < q->e_lo || w->E > q->e_hi) goto fail; /* start outside window */
    }
  }
  return c;
fail:
  if (!c->w) c->nwalkers = 0;
  ref_destroy(c);
  return NULL;
}

int ref_get_walker(const ref_ctx* c, int wi, uint8_t* n, uint32_t* pos, int32_t* E,
                   uint64_t* t) {
  if (wi < 0 || wi >= c->nwalkers) return -1;
  const walker* w = &c->w[wi];
  const ref_group* g = &c->g[w->group];
  if (n) memcpy(n, w->n, (size_t)ipow(g->L, g->d));
  if (pos) memcpy(pos, w->pos, sizeof(uint32_t) * (size_t)g->N);
  if (E) *E = w->E;
  if (t) *t = w->t;
  return 0;
}

int ref_get_tunnel(const ref_ctx* c, uint32_t* last_end, uint32_t* trips) {
  for (int i = 0; i < c->nwalkers; ++i) {
    if (last_end) last_end[i] = c->w[i].last_end;
    if (trips) trips[i] = c->w[i].trips;
  }
  return 0;
}

int ref_set_walker(ref_ctx* c, int wi, const uint8_t* n, const uint32_t* pos, int32_t E,
                   uint64_t t) {
  if (wi < 0 || wi >= c->nwalkers) return -1;
  walker* w = &c->w[wi];
  const ref_group* g = &c->g[w->group];
  memcpy(w->n, n, (size_t)ipow(g->L, g->d));
  memcpy(w->pos, pos, sizeof(uint32_t) * (size_t)g->N);
  w->E = E;
  w->t = t;
  return 0;
}

int32_t ref_recount(const ref_ctx* c, int wi) {
  const walker* w = &c->w[wi];
  const ref_group* g = &c->g[w->group];
  return energy(g->d, g->L, w->n);
}

/* ------------------------------------------------------------------------ */
/* Equilibrium run of one walker with fixed weights (Sec. 2).                */
/* ------------------------------------------------------------------------ */

/* One update: propose moving a uniform random particle k from s_o to a
 * uniform random empty site s_n; E_n = E_o + k_o - k_n where k_o counts the
 * occupied neighbours of s_o and k_n those of s_n other than s_o. */
static void attempt(walker* w, const ref_group* g, const double* lnW, uint32_t seed32) {
  uint32_t V = (uint32_t)ipow(g->L, g->d);
  uint32_t key[2] = {w->id, seed32};
  uint32_t ctr[4] = {(uint32_t)w->t, (uint32_t)(w->t >> 32), 0, 0};
  uint32_t x[4];
  ref_philox(ctr, key, x);
  uint32_t u = x[1];
  uint32_t k = uniform(x[0], (uint32_t)g->N);
  uint32_t s_o = w->pos[k];
  /* candidates: words 2 and 3 of block 0, then words 0..3 of blocks 1, 2, ... */
  uint32_t s_n = 0;
  int j = 2;
  for (;;) {
    if (j == 4) {
      ctr[2] += 1;
      ref_philox(ctr, key, x);
      j = 0;
    }
    uint32_t s = uniform(x[j++], V);
    if (!w->n[s]) {
      s_n = s;
      break;
    }
  }
  int k_o = occupied_neighbours(g->d, g->L, w->n, s_o, -1);
  int k_n = occupied_neighbours(g->d, g->L, w->n, s_n, (int64_t)s_o);
  int32_t E_o = w->E;
  int32_t E_n = E_o + k_o - k_n;
  int acc = 0;
  if (E_n >= g->e_lo && E_n <= g->e_hi)
    acc = ref_accept(lnW[E_n - g->e_lo] - lnW[E_o - g->e_lo], u);
  if (acc) {
    w->n[s_o] = 0;
    w->n[s_n] = 1;
    w->pos[k] = s_n;
    w->E = E_n;
  }
  w->t += 1;
}

/* Sec. 4: the paper counts convergence in tunnelling events, a walker
 * travelling from the top of the energy range to its bottom or back.  The
 * walker's energy is looked at once per sweep, where its histogram entry is
 * taken: standing at the window's bottom (e_lo) or top (e_hi) after last
 * touching the other end completes one trip.  (A window of one bin has
 * no trips.) */
static void tunnel_visit(walker* w, const ref_group* g) {
  int end = 0;
  if (w->E == g->e_lo) end = 1;
  else if (w->E == g->e_hi) end = 2;
  if (end == 0 || (uint32_t)end == w->last_end) return;
  if (w->last_end != 0) w->trips += 1;
  w->last_end = (uint32_t)end;
}

/* Sec. 2, eq. (2): every process j samples H^i_j(E) with the same weights
 * W^i; the histograms are summed, H^i(E) = sum_j H^i_j(E).  Here each walker
 * plays the role of one process.  A sweep is L^d updates (Sec. 4); the
 * histogram takes one entry per walker after every sweep. */
int ref_sweep(ref_ctx* c, const double* lnW, int sweeps, int32_t* H, const int32_t* active) {
  if (sweeps < 1) return -1;
  for (int gi = 0; gi < c->ngroups; ++gi) {
    if (active && !active[gi]) continue;
    const ref_group* g = &c->g[gi];
    int nb = g->e_hi - g->e_lo + 1;
    if ((int64_t)g->walkers * sweeps > 2147483647LL) return -2;
    int32_t* Hg = H + c->bin_off[gi];
    const double* lw = lnW + c->bin_off[gi];
    memset(Hg, 0, sizeof(int32_t) * (size_t)nb);
    int64_t V = ipow(g->L, g->d);
    for (int j = 0; j < g->walkers; ++j) {
      walker* w = &c->w[c->first_walker[gi] + j];
      for (int s = 0; s < sweeps; ++s) {
        for (int64_t a = 0; a < V; ++a) attempt(w, g, lw, c->seed32);
        Hg[w->E - g->e_lo] += 1;
        tunnel_visit(w, g);
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Weight recursion (Sec. 2).                                                */
/* ------------------------------------------------------------------------ */

/* Simple rule of Sec. 2, W^{i+1}(E) = W^i(E) / H^i(E), in logarithms; an
 * unvisited bin keeps its weight; normalised so that lnW at e_hi is 0. */
static void update_simple(int nb, const int32_t* H, double* lnW) {
  for (int b = 0; b < nb; ++b) lnW[b] = lnW[b] - ref_log(H[b] > 0 ? H[b] : 1);
  double top = lnW[nb - 1];
  for (int b = 0; b < nb; ++b) lnW[b] = lnW[b] - top;
}

/* Recursive scheme (Sec. 2; reading: Berg's error-weighted recursion).
 * With the weight slope d(b) = lnW(b+1) - lnW(b), each iteration gives the
 * estimate d(b) + ln H(b) - ln H(b+1) for every pair of visited neighbouring
 * bins, with statistical weight p = H(b) H(b+1) / (H(b) + H(b+1)); the new
 * slope is the p-weighted mean of all estimates so far, accumulated as
 * P(b) += p, d(b) += (p / P(b)) (ln H(b) - ln H(b+1)).  Slopes of pairs
 * never estimated beyond the lowest / highest estimated pair are copied from
 * that pair; lnW is rebuilt downward from lnW(e_hi) = 0. */
static void update_berg(int nb, const int32_t* H, double* lnW, double* P) {
  double* d = (double*)malloc(sizeof(double) * (size_t)(nb > 1 ? nb - 1 : 1));
  for (int b = 0; b + 1 < nb; ++b) {
    if (H[b] > 0 && H[b + 1] > 0) {
      double h0 = (double)H[b], h1 = (double)H[b + 1];
      double p = h0 * h1 / (h0 + h1);
      P[b] = P[b] + p;
      double kappa = p / P[b];
      d[b] = (lnW[b + 1] - lnW[b]) + kappa * (ref_log(H[b]) - ref_log(H[b + 1]));
    } else {
      d[b] = lnW[b + 1] - lnW[b];
    }
  }
  int lo = -1, hi = -1;
  for (int b = 0; b + 1 < nb; ++b)
    if (P[b] > 0.0) {
      if (lo < 0) lo = b;
      hi = b;
    }
  if (lo >= 0) {
    for (int b = 0; b < lo; ++b) d[b] = d[lo];
    for (int b = hi + 1; b + 1 < nb; ++b) d[b] = d[hi];
  }
  lnW[nb - 1] = 0.0;
  for (int b = nb - 2; b >= 0; --b) lnW[b] = lnW[b + 1] - d[b];
  free(d);
}

int ref_update(ref_ctx* c, const int32_t* H, double* lnW, double* P, int rule,
               const int32_t* active) {
  if (rule != 0 && rule != 1) return -1;
  for (int gi = 0; gi < c->ngroups; ++gi) {
    if (active && !active[gi]) continue;
    const ref_group* g = &c->g[gi];
    int nb = g->e_hi - g->e_lo + 1, off = c->bin_off[gi];
    if (rule == 1)
      update_simple(nb, H + off, lnW + off);
    else
      update_berg(nb, H + off, lnW + off, P + off);
  }
  return 0;
}

/* Flatness (reading of "max/min of H over the energy range"): both window
 * ends visited and 2 * min over visited bins > max. */
int ref_flat(const ref_ctx* c, const int32_t* H, int32_t* flags) {
  for (int gi = 0; gi < c->ngroups; ++gi) {
    const ref_group* g = &c->g[gi];
    int nb = g->e_hi - g->e_lo + 1;
    const int32_t* h = H + c->bin_off[gi];
    int64_t mn = -1, mx = 0;
    for (int b = 0; b < nb; ++b) {
      if (h[b] <= 0) continue;
      if (mn < 0 || h[b] < mn) mn = h[b];
      if (h[b] > mx) mx = h[b];
    }
    flags[gi] = (h[0] > 0 && h[nb - 1] > 0 && 2 * mn > mx) ? 1 : 0;
  }
  return 0;
}

/* Tunnelling events of group gi so far: the sum of its walkers' trips. */
static int64_t group_trips(const ref_ctx* c, int gi) {
  int64_t n = 0;
  for (int j = 0; j < c->g[gi].walkers; ++j) n += c->w[c->first_walker[gi] + j].trips;
  return n;
}

/* The iteration of Sec. 2: equilibrium runs with fixed weights W^i, summed
 * histogram H^i, new weights W^{i+1}; repeated until converged.
 * stop = 0: exactly max_iters iterations of (sweep, update); returns
 *   lnW^K, H^{K-1}; flat[g] reports the last histogram.
 * stop = 1: a group stops at its first flat H^i; it keeps lnW^i and H^i and
 *   iters[g] = i + 1.  Groups still running after max_iters hold
 *   lnW^{max_iters}, H^{max_iters-1}; the return value is then 1.
 * stop = 2 (Sec. 4): as 1, but a group stops once its walkers have made
 *   tunnel_target tunnelling events in total (counted since the walkers
 *   were created, at the end of each iteration's sweeps). */
int ref_run(ref_ctx* c, double* lnW, double* P, int32_t* H, int sweeps, int max_iters,
            int rule, int stop, int tunnel_target, int32_t* iters, int32_t* flat) {
  int G = c->ngroups;
  int32_t* active = (int32_t*)malloc(sizeof(int32_t) * (size_t)G);
  int32_t* f = (int32_t*)malloc(sizeof(int32_t) * (size_t)G);
  int status = 0, remaining = G;
  for (int g = 0; g < G; ++g) {
    active[g] = 1;
    iters[g] = 0;
    flat[g] = 0;
  }
  for (int i = 0; i < max_iters && remaining > 0; ++i) {
    int rc = ref_sweep(c, lnW, sweeps, H, active);
    if (rc) { status = rc; goto done; }
    ref_flat(c, H, f);
    for (int g = 0; g < G; ++g) {
      if (!active[g]) continue;
      iters[g] = i + 1;
      flat[g] = f[g];
      if ((stop == 1 && f[g]) || (stop == 2 && group_trips(c, g) >= tunnel_target)) {
        active[g] = 0;
        --remaining;
      }
    }
    if (remaining == 0) break;
    rc = ref_update(c, H, lnW, P, rule, active);
    if (rc) { status = rc; goto done; }
  }
  if (stop && remaining > 0) status = 1;
done:
  free(active);
  free(f);
  return status;
}
