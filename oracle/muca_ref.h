/*
 * muca_ref.h -- CPU oracle of the parallel multicanonical (MUCA) iteration.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  This is the plain, slow,
 * single-threaded reference that the GPU library is checked against.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source with the GPU library (paper_1401_4076_amd/).
 *
 * Paper: J. Zierenberg, M. Wiedenmann, W. Janke, "Application of the parallel
 * multicanonical method to lattice gas condensation" (arXiv:1401.4076).
 *   - Lattice gas, n_i in {0,1}, H = -J sum_<ij> n_i n_j, fixed N:  Sec. 3, eq. (5).
 *   - Metropolis with weights, accept with min(1, W(E_n)/W(E_o)):  Sec. 2.
 *   - p independent equilibrium runs with identical weights, summed
 *     histograms H^i(E) = sum_j H^i_j(E):                         Sec. 2, eq. (2).
 *   - consecutive weights from the previous weights and H^i by a
 *     recursive scheme; the simple example W^{i+1} = W^i / H^i:   Sec. 2.
 *   - one sweep = L^d updates:                                    Sec. 4.
 * Where the paper is silent the oracle follows the readings listed at the
 * top of the corresponding function in muca_ref.c.
 *
 * Parity unpinned against the paper (only pinned against the GPU path, bit
 * for bit): the frontier extrapolation of the Berg recursion and the
 * flatness criterion.  Everything else has an independent pin in tests/.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -shared -fPIC (no fast-math).
 */
#ifndef MUCA_REF_H
#define MUCA_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t d, L, N, walkers, e_lo, e_hi; /* e_lo = e_hi = 0 -> default window */
} ref_group;

typedef struct ref_ctx ref_ctx;

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void ref_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* exp(x) for -23 <= x < 0 using only IEEE +,-,*,/,floor,ldexp. */
double ref_exp(double x);
/* ln(h) for an integer h >= 1 using only IEEE +,-,*,/,frexp. */
double ref_log(int64_t h);
/* Acceptance decision for the difference x = lnW(E_n) - lnW(E_o) and the
 * 32-bit uniform u.  Returns 1 to accept. */
int ref_accept(double x, uint32_t u);
/* Lowest energy of the constructed compact cluster (default window edge). */
int32_t ref_energy_floor(int d, int L, int N);
/* Exact density of states by enumeration of all C(V,N) configurations.
 * omega has d*N+1 entries, omega[k] = #configurations with E = -k. */
int ref_brute_dos(int d, int L, int N, int64_t* omega);

/* Create walkers for ngroups groups; walker ids are first_id, first_id+1, ...
 * assigned group by group.  Returns NULL on invalid input. */
ref_ctx* ref_create(const ref_group* g, int ngroups, uint64_t seed, uint32_t first_id);
void ref_destroy(ref_ctx* c);
int ref_num_groups(const ref_ctx* c);
int ref_window(const ref_ctx* c, int group, int32_t* e_lo, int32_t* e_hi);
int ref_total_bins(const ref_ctx* c);
int ref_bin_offset(const ref_ctx* c, int group);
int ref_num_walkers(const ref_ctx* c);

/* Each walker of each active group (active == NULL: all) performs `sweeps`
 * sweeps with weights lnW; H (total bins, concatenated over groups) is
 * overwritten with the summed histogram (inactive groups: left untouched). */
int ref_sweep(ref_ctx* c, const double* lnW, int sweeps, int32_t* H, const int32_t* active);
/* Weight recursion on each active group.  rule 0 = Berg error-weighted
 * recursion, rule 1 = simple W/H.  P has the layout of lnW: P[off_g + b] is
 * the accumulator of the bin pair (b, b+1); the entry of each group's last
 * bin is unused.  P is zero at the start of a run. */
int ref_update(ref_ctx* c, const int32_t* H, double* lnW, double* P, int rule,
               const int32_t* active);
/* flags[g] = 1 if the histogram of group g is flat. */
int ref_flat(const ref_ctx* c, const int32_t* H, int32_t* flags);
/* Whole iteration loop (see muca_ref.c).  stop: 0 fixed count, 1 until
 * flat, 2 until tunnel_target tunnelling events per group.  Returns 0 when
 * every group has stopped or the fixed count is done, 1 when max_iters is
 * hit first, <0 on error. */
int ref_run(ref_ctx* c, double* lnW, double* P, int32_t* H, int sweeps, int max_iters,
            int rule, int stop, int tunnel_target, int32_t* iters, int32_t* flat);
/* Per walker: the window end visited last (0 none, 1 bottom, 2 top, looked at
 * after every sweep) and the tunnelling events (trips from one end to the
 * other) completed since creation.  Either array may be NULL. */
int ref_get_tunnel(const ref_ctx* c, uint32_t* last_end, uint32_t* trips);

/* Walker state access (occupation bytes n[V], particle sites pos[N]). */
int ref_get_walker(const ref_ctx* c, int w, uint8_t* n, uint32_t* pos, int32_t* E,
                   uint64_t* t);
int ref_set_walker(ref_ctx* c, int w, const uint8_t* n, const uint32_t* pos, int32_t E,
                   uint64_t t);
/* Recount E of walker w from its occupations (for invariant checks). */
int32_t ref_recount(const ref_ctx* c, int w);

#ifdef __cplusplus
}
#endif
#endif
