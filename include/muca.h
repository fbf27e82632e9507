/*
 * muca.h -- C ABI of libmuca, the MI355X (gfx950) implementation of the
 * equilibrium parallel multicanonical (MUCA) iteration of
 * J. Zierenberg, M. Wiedenmann, W. Janke, "Application of the parallel
 * multicanonical method to lattice gas condensation" (arXiv:1401.4076).
 *
 * The method (paper Sec. 2): p independent equilibrium runs share identical
 * weights W^i(E); each run fills a histogram H^i_j(E); the histograms are
 * summed, H^i(E) = sum_j H^i_j(E) (eq. (2)); the next weights W^{i+1} are
 * computed from W^i and H^i by a recursive scheme and given back to every
 * run; this repeats until the weights are converged.  Here each of many
 * lattice-gas walkers on one GPU plays the role of one process.
 *
 * Model (Sec. 3, eq. (5)): lattice gas on a periodic square (d = 2) or
 * simple-cubic (d = 3) lattice of V = L^d sites, occupations n_i in {0,1},
 * fixed particle number N, E = -(number of occupied nearest-neighbour
 * pairs) (J = 1).  A sweep is V update attempts (Sec. 4).  An attempt moves
 * a uniform random particle to a uniform random empty site and is accepted
 * with min(1, W(E_n)/W(E_o)) (Sec. 2).
 *
 * Reproducibility: results are a pure function of (groups, seed,
 * first walker id, initial lnW, sweep schedule, rule).  They do not depend on
 * the kernel layout, on graph or eager execution, or on how walkers are
 * spread over devices.  Random numbers are Philox4x32-10 with key
 * (global walker id, low 32 bits of seed); attempt t of a walker uses
 * counters (t_lo, t_hi, r, 0), r = 0, 1, ...; the initial placement uses
 * counters (i_lo, i_hi, 0, 1).
 *
 * Memory: the library owns walker state (allocated by mucaInit*, freed by
 * mucaDestroy).  The caller owns lnW (double), P (double) and H (int32):
 * device pointers of total_bins entries each, concatenated over groups in
 * group order (group g starts at its bin offset, bin b <-> E = e_lo + b).
 * Calls taking a `stream` (a hipStream_t; NULL = the null stream) are
 * asynchronous on it unless stated otherwise.  A context is not
 * thread-safe; use one context per stream.
 *
 * Errors: every call returns MUCA_OK (0), the positive status
 * MUCA_NOT_CONVERGED, or a negative code; mucaLastError() returns a
 * thread-local description of the last failure.  No C++ exception crosses
 * this interface.
 */
#ifndef MUCA_H
#define MUCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MUCA_OK 0
#define MUCA_NOT_CONVERGED 1  /* mucaRun: max_iters reached before every group stopped */
#define MUCA_EINVAL (-1)      /* invalid argument */
#define MUCA_EOVERFLOW (-2)   /* walkers x sweeps of a group exceeds INT32_MAX */
#define MUCA_ENOMEM (-3)      /* device allocation failed */
#define MUCA_EHIP (-4)        /* HIP runtime error */
#define MUCA_ENONFINITE (-5)  /* non-finite weight met by the sweep or produced by an update */

#define MUCA_RULE_BERG 0   /* recursive scheme of Sec. 2, read as Berg's error-weighted recursion */
#define MUCA_RULE_SIMPLE 1 /* W^{i+1}(E) = W^i(E) / H^i(E), Sec. 2 */

#define MUCA_STOP_NONE 0    /* mucaRun: a fixed number of iterations */
#define MUCA_STOP_FLAT 1    /* mucaRun: a group stops at its first flat histogram */
#define MUCA_STOP_TUNNEL 2  /* mucaRun: a group stops once its walkers made the
                               tunnelling target (mucaSetTunnelTarget), Sec. 4 */

#define MUCA_LAYOUT_AUTO 0  /* chosen per context (see mucaAutotune) */
#define MUCA_LAYOUT_LANE 1  /* one walker per lane, walker state in device memory */
#define MUCA_LAYOUT_SUB16 2 /* 16 lanes per walker (4 walkers per wavefront) */
#define MUCA_LAYOUT_SUB64 3 /* 64 lanes (one wavefront) per walker */
#define MUCA_LAYOUT_LOOK4 4 /* one wavefront per walker, four attempts gathered per step
                               (walker state in LDS; else runs as SUB64) */
#define MUCA_LAYOUT_SUB16X2 5 /* 16 lanes per walker, 2 walkers per wavefront (more
                                 wavefronts per SIMD for small populations); with
                                 state in device memory the next attempt's gather
                                 is issued before the current one is decided */
#define MUCA_LAYOUT_SUB16X1 6 /* as SUB16X2 with 1 walker per wavefront */
#define MUCA_LAYOUT_SUB16MIX 7 /* 16 lanes per walker, per group: 2 walkers per
                                  wavefront for the groups with the context's
                                  largest lattice, 4 for the others */
#define MUCA_NUM_LAYOUTS 8    /* layout indices 0 .. MUCA_NUM_LAYOUTS - 1 */

typedef struct muca_context* muca_ctx;

/* One group of walkers with its own lattice, weights and histogram.
 * e_lo = e_hi = 0 selects the default window [E_floor(d,L,N), 0], where
 * E_floor is the energy of a compact cluster built from full layers and
 * rows (the paper takes the range from short parallel-tempering runs,
 * Sec. 3).  Moves whose new energy leaves [e_lo, e_hi] are rejected. */
typedef struct {
  int32_t d;       /* 2 or 3 */
  int32_t L;       /* 3 <= L <= 1024, V = L^d <= 2^24 */
  int32_t N;       /* 1 <= N <= V-1; N <= V/2 for the default window */
  int32_t walkers; /* >= 1 */
  int32_t e_lo, e_hi; /* -d N <= e_lo <= e_hi <= 0 with at most 2^24 bins, or both 0 */
} muca_group;

/* Create a context of one group; equivalent to mucaInitGroups with one
 * group, default window and first walker id 0.  Runs the uniform random
 * initial placement on the current device and waits for it. */
int mucaInit(muca_ctx* out, int d, int L, int N, int walkers, uint64_t seed);

/* Create a context of ngroups groups.  Walkers get global ids
 * first_id, first_id + 1, ... group by group in array order (first_id lets
 * several devices each own a disjoint range of one walker population).
 * Allocates all device state on the current device, places the particles
 * (N distinct uniform random sites per walker) and waits.  Fails with
 * MUCA_EINVAL if an initial energy lies outside its group's window. */
int mucaInitGroups(muca_ctx* out, const muca_group* groups, int ngroups, uint64_t seed,
                   uint32_t first_id);

/* Default window [e_lo, e_hi] = [E_floor(d, L, N), 0] of a group, computed
 * on the host (no device work).  Same validation as mucaInitGroups. */
int mucaDefaultWindow(int d, int L, int N, int32_t* e_lo, int32_t* e_hi);

/* Free all device state of the context.  NULL is accepted. */
int mucaDestroy(muca_ctx ctx);

/* Thread-local text of the last error ("" if none). */
const char* mucaLastError(void);

/* Sizes.  bin_offset is the index of bin 0 of group g in lnW, H and P. */
int mucaNumGroups(muca_ctx ctx, int* ngroups);
int mucaNumWalkers(muca_ctx ctx, int* nwalkers);
int mucaTotalBins(muca_ctx ctx, int* total_bins);
int mucaGetWindow(muca_ctx ctx, int group, int32_t* e_lo, int32_t* e_hi, int32_t* bin_offset);

/* Kernel layout used by the sweep (MUCA_LAYOUT_*).  Results are the same
 * for every layout; only the speed differs.  In the cooperative layouts the
 * walker state sits in LDS for the whole launch when the block's walkers fit
 * (mucaGetLayout reports the resolved layout; AUTO resolves to SUB16 until
 * mucaAutotune has run). */
int mucaSetLayout(muca_ctx ctx, int layout);
int mucaGetLayout(muca_ctx ctx, int* layout);

/* Where the resolved layout's sweep keeps the walker state and the threshold
 * table: 1 = LDS for the whole launch, 0 = device memory (the one-walker-
 * per-lane layout keeps both in device memory).  Host-side; no device work.
 * Either output may be NULL. */
int mucaGetPlacement(muca_ctx ctx, int* state_in_lds, int* table_in_lds);

/* Largest LDS allocation (bytes per block of 256 lanes) the cooperative
 * layouts may use, capped by the device limit.  Walker state (occupation
 * bits and particle sites of the block's walkers) goes to LDS when it fits,
 * then the group's threshold table when it fits beside it; what does not
 * fit stays in device memory.  Default 163840; 0 keeps everything in device
 * memory.  A context with a 3D group of L % 8 == 0 whose 16-walker state
 * exceeds 163840 bytes keeps that group's bits in 8x8x8 bricks (fewer memory
 * lines per neighbourhood) and walker state in device memory in every
 * layout (LOOK4 then runs as SUB64); results are unchanged. */
int mucaSetLdsLimit(muca_ctx ctx, int64_t bytes);

/* Largest walker state (bytes of occupation bits and particle sites) that a
 * cooperative launch keeps in flight at once when the state lives in device
 * memory: the walker sets then run in rounds of whole blocks per compute
 * unit, at least one block per compute unit.  The random accesses of the
 * sweep are cheapest while the state in flight fits the device's last-level
 * cache (256 MB on MI355X).  Default 224 MiB; 0 = no cap; mucaAutotune may
 * change it (see there).  Results are unchanged; only the speed differs.
 * Changing this limit or the LDS limit waits for the device and rebuilds the
 * context's task tables and captured iteration on their next use. */
int mucaSetResidentLimit(muca_ctx ctx, int64_t bytes);
int mucaGetResidentLimit(muca_ctx ctx, int64_t* bytes);

/* Time every layout on `probe_sweeps` sweeps with weights lnW (device) and
 * keep the fastest; a cooperative layout whose walker state lives in device
 * memory is timed with the context's resident limit (mucaSetResidentLimit)
 * and without a limit, and the faster of the two is kept; synchronous.  Walker state is saved before and restored
 * after the probes, so the call does not change any later result.  chosen
 * (host, may be NULL) receives the layout, ms (host, may be NULL,
 * MUCA_NUM_LAYOUTS doubles) the probe time per layout index (0 where not
 * run). */
int mucaAutotune(muca_ctx ctx, const double* lnW, int probe_sweeps, int* chosen, double* ms,
                 void* stream);

/* Acceptance thresholds from the weights (Sec. 2, min(1, W(E_n)/W(E_o))):
 * for every group, bin b_o and energy change dE in [-2d, 2d],
 *   x = lnW[b_o + dE] - lnW[b_o],
 *   T = 0xFFFFFFFF ("always") if x >= 0 or floor(exp(x) 2^32) >= 2^32 - 1,
 *   T = 0 ("never") if x < -23 or b_o + dE is outside the window,
 *   T = floor(exp(x) 2^32) otherwise (accept iff the attempt's 32-bit
 *   uniform u < T),
 * with exp evaluated by IEEE-754 binary64 operations only.  The table of
 * group g holds bins_g x (4 d_g + 1) uint32, row b_o, column dE + 2 d_g;
 * groups follow each other in order.  thr_out (device, may be NULL)
 * receives a copy of the whole table; mucaThresholdEntries gives its size.
 * lnW is a device pointer.  Non-finite weights give MUCA_ENONFINITE from
 * the next synchronising call (mucaRun, mucaStatus). */
int mucaThresholdEntries(muca_ctx ctx, int* entries);
int mucaBuildThresholds(muca_ctx ctx, const double* lnW, uint32_t* thr_out, void* stream);

/* Equilibrium runs with fixed weights (Sec. 2, eq. (2)): every walker of
 * every group makes `sweeps` sweeps of V attempts with weights lnW
 * (device, total_bins doubles), adding one histogram entry at its energy
 * after each sweep.  H (device, total_bins int32) is overwritten with the
 * summed histograms H^i(E) = sum_j H^i_j(E).  mucaSweepActive sweeps only
 * groups with active[g] != 0 (device, ngroups int32) and leaves the H
 * entries of the other groups untouched.  Walker state carries over from
 * call to call.  Fails with MUCA_EOVERFLOW if walkers_g x sweeps > INT32_MAX. */
int mucaSweep(muca_ctx ctx, const double* lnW, int sweeps, int32_t* H, void* stream);
int mucaSweepActive(muca_ctx ctx, const double* lnW, int sweeps, int32_t* H,
                    const int32_t* active, void* stream);

/* mucaSweep for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same sweep, with the same results and arguments, that calls no allocating
 * routine.  Its threshold table and block task table live in a static device
 * workspace of 4 MiB (MUCA_NOALLOC_WORKSPACE_BYTES) per device, set up when
 * the first context is created on that device; the task table is the plain
 * one (one set of walkers per block, sets in group order), written by a
 * kernel on `stream`.  Fails with MUCA_EINVAL, before any device work, when
 * the context's threshold table plus task table exceed the workspace (the
 * threshold table holds total bins x (4d+1) 32-bit entries).  Every call on
 * a device shares that device's workspace: calls that overlap in time on one
 * device (different streams or host threads) race and must be serialised by
 * the caller. */
#define MUCA_NOALLOC_WORKSPACE_BYTES 4194304
int mucaSweepNoAlloc(muca_ctx ctx, const double* lnW, int sweeps, int32_t* H, void* stream);

/* Next weights from the previous weights and the summed histogram
 * (Sec. 2), in place on lnW and P (device pointers).  rule:
 *   MUCA_RULE_SIMPLE: lnW(b) -= ln max(H(b), 1), then lnW -= lnW(e_hi);
 *   MUCA_RULE_BERG: for each pair of neighbouring bins (b, b+1) both
 *     visited, p = H(b) H(b+1) / (H(b) + H(b+1)), P(b) += p, and the slope
 *     d(b) = lnW(b+1) - lnW(b) becomes d(b) + (p / P(b)) (ln H(b) - ln H(b+1));
 *     other slopes are kept, except that never-estimated pairs (P = 0) below
 *     the lowest or above the highest estimated pair take that pair's slope;
 *     lnW(e_hi) = 0 and lnW is rebuilt downward, one bin after the other.
 * P[off_g + b] belongs to pair (b, b+1); the last entry of each group is
 * unused; P must be zero at the start of a run.  ln is evaluated by
 * IEEE-754 binary64 operations only. */
int mucaUpdateWeights(muca_ctx ctx, const int32_t* H, double* lnW, double* P, int rule,
                      void* stream);

/* flags[g] (device, ngroups int32) = 1 if H of group g is flat: both window
 * ends visited and 2 min_{b: H(b) > 0} H(b) > max_b H(b); else 0. */
int mucaIsFlat(muca_ctx ctx, const int32_t* H, int32_t* flags, void* stream);

/* The whole iteration (Sec. 2), synchronous.  lnW, P, H are device
 * pointers; lnW holds the initial weights on entry (flat or learned), P is
 * zeroed by the call (resume = 0).  resume = 1 continues the previous
 * mucaRun of this context exactly where it stopped (same P, same finished
 * groups, iteration count continued), so a long run can be split into
 * several calls; max_iters then counts the iterations of this call.
 * iters and flat are host arrays of ngroups int32.
 *   stop = MUCA_STOP_NONE: exactly max_iters iterations of (sweep, update):
 *     lnW = lnW^K, H = H^{K-1}, flat[g] = flatness of H^{K-1}, iters[g] = K.
 *   stop = MUCA_STOP_FLAT: group g stops at its first flat H^i: lnW keeps
 *     lnW^i, H keeps H^i, iters[g] = i + 1, flat[g] = 1.  Groups not flat
 *     after max_iters keep lnW^{max_iters}, H^{max_iters - 1}, flat[g] = 0,
 *     and the call returns MUCA_NOT_CONVERGED.
 *   stop = MUCA_STOP_TUNNEL (the criterion of Sec. 4): as MUCA_STOP_FLAT, but
 *     group g stops after the first iteration i at whose end its walkers
 *     have made the tunnelling target in total (see mucaGetTunnel; counted
 *     since the context was created); flat[g] reports H^i.
 * Any other stop value is MUCA_EINVAL.
 * The per-iteration work (thresholds, sweep, loop control, recursion) is
 * captured once as a HIP graph on an internal stream, ordered after the
 * caller's stream, and replayed; the graph is kept for later calls with the
 * same pointers and parameters. */
int mucaRun(muca_ctx ctx, double* lnW, double* P, int32_t* H, int sweeps_per_iter,
            int max_iters, int rule, int stop, int resume, int32_t* iters,
            int32_t* flat, void* stream);

/* Tunnelling events (Sec. 4 measures convergence by them: trips of a walker
 * from the top of its group's energy window to the bottom or back).  A
 * walker's energy is looked at after every sweep, where its histogram entry
 * is taken: at e_lo or e_hi after last visiting the other end it completes
 * a trip.  A window of one bin has no trips.  The counts run from the
 * context's creation, through every mucaSweep and mucaRun (mucaAutotune
 * restores them).
 * mucaSetTunnelTarget: trips per group that end a MUCA_STOP_TUNNEL run
 *   (target >= 1; 30 when never set, as in Sec. 4).
 * mucaGetTunnel: per walker (host arrays of nwalkers uint32, either may be
 *   NULL; waits for the device) the end visited last (0 none yet, 1 e_lo,
 *   2 e_hi) and the trips completed. */
int mucaSetTunnelTarget(muca_ctx ctx, int target);
int mucaGetTunnel(muca_ctx ctx, uint32_t* last_end, uint32_t* trips);

/* Canonical reweighting (Sec. 3: the multicanonical data are reweighted to
 * the temperatures of interest).  H is a histogram taken with weights lnW
 * (normally a production mucaSweep with the converged weights); both device
 * arrays in the concatenated bin layout.  beta: device array of nbeta
 * inverse temperatures (J = 1, k_B = 1).  out: device array of
 * ngroups x nbeta x 4 doubles, out[(g * nbeta + k) * 4 + j] =
 *   j = 0: ln Z(beta) = ln sum_E exp(ln Omega(E) - beta E), with
 *          ln Omega(E) = ln H(E) - lnW(E) over the visited bins (H > 0), so
 *          up to the same additive constant as ln Omega;
 *   j = 1: <E>;  j = 2: <E^2>;
 *   j = 3: C = beta^2 <(E - <E>)^2> (specific heat of the whole lattice).
 * A group without a visited bin gets NaN.  Sums are shifted by the largest
 * exponent; binary64 throughout (exp and log of the device math library).
 * nbeta >= 1, else MUCA_EINVAL; asynchronous on stream. */
int mucaReweight(muca_ctx ctx, const double* lnW, const int32_t* H, const double* beta,
                 int nbeta, double* out, void* stream);

/* Largest droplet (Sec. 3 follows condensation through the largest cluster
 * of particles): out[w] (device, nwalkers int32) = number of particles in
 * the largest set connected through nearest-neighbour bonds (periodic) in
 * walker w's current configuration.  Any lattice size; the walker's sorted
 * particle sites and a union-find forest sit in LDS, so a group may hold at
 * most as many particles as fit (8 + 4 P + 4 N bytes per block, P the power
 * of two >= N; N <= 16384 on MI355X), else MUCA_EINVAL.  Asynchronous on
 * stream; -1 marks an internal bound reached (not expected: the union-find
 * loops are bounded by N). */
int mucaLargestCluster(muca_ctx ctx, int32_t* out, void* stream);

/* The energy-binned droplet measurement of a production run: for every
 * walker, its largest droplet (as mucaLargestCluster) is added to osum at
 * the bin of the walker's current energy and ocount counts the measurement
 * there (device arrays of total_bins int64 and int32, concatenated bin
 * layout; accumulated, not cleared).  out (device, nwalkers int32) may be
 * NULL, else it also receives the sizes.  Integer sums: exact and
 * independent of the order of the walkers. */
int mucaMeasureDroplets(muca_ctx ctx, long long* osum, int32_t* ocount, int32_t* out,
                        void* stream);

/* A production run with fixed weights lnW (Sec. 3: after the iteration the
 * system is simulated with the converged weights and the measurements are
 * reweighted): `measurements` rounds of (sweeps_between sweeps of every
 * walker, then mucaMeasureDroplets).  H (device, total_bins int32) receives
 * the histogram of all sweeps; osum and ocount are cleared first and receive
 * the droplet sums and counts per bin at the measurement sweeps.  Same
 * walker-state carry-over and overflow checks as mucaSweep (over the total
 * sweeps).  Asynchronous on stream. */
int mucaProduction(muca_ctx ctx, const double* lnW, int sweeps_between, int measurements,
                   int32_t* H, long long* osum, int32_t* ocount, void* stream);

/* Canonical average of an observable measured during a production run
 * (Sec. 3): osum[b] is its sum over the ocount[b] measurements at bin b (as
 * mucaProduction or mucaMeasureDroplets leave them), taken with weights lnW.
 * out[g * nbeta + k] (device, ngroups x nbeta doubles) =
 *   sum_E (osum / ocount)(E) Omega(E) exp(-beta_k E) / sum_E Omega(E) exp(-beta_k E),
 * ln Omega(E) = ln ocount(E) - lnW(E) over the bins with ocount > 0 (NaN for
 * a group without one).  Shifted by the largest exponent, binary64, fixed
 * reduction order; asynchronous on stream. */
int mucaReweightObservable(muca_ctx ctx, const double* lnW, const int32_t* ocount,
                           const long long* osum, const double* beta, int nbeta, double* out,
                           void* stream);

/* Calibration of the memory-bound roofline of the sweeps with walker state in
 * device memory, whose attempts read a few random 128-byte lines each: the
 * device's rate of random whole-line reads.  sink_words / 256 blocks of 256
 * lanes (at most 2^20 blocks) each follow 8 independent xorshift32 streams
 * of uniformly random lines of `table` (device, table_bytes bytes, at least
 * one 128-byte line, at most 2^32 - 1) for `rounds` rounds, one 4-byte load
 * per line, and store one word per lane into sink (device).  One untimed
 * launch, then a timed one (HIP events on stream); lines_read and seconds
 * (host) describe the timed launch.  Synchronous.  A table larger than the
 * last-level cache measures HBM, a smaller one the caches. */
int mucaCalibrateRandomLines(const uint32_t* table, int64_t table_bytes, uint32_t* sink,
                             int64_t sink_words, int rounds, double* lines_read, double* seconds,
                             void* stream);

/* enable = 0 makes mucaRun enqueue every iteration eagerly on the caller's
 * stream instead of replaying the captured graph (same results). */
int mucaSetGraph(muca_ctx ctx, int enable);

/* Copy one walker's state to host memory (waits for the device):
 * occupation bits (ceil(V/32) words, site s = x + L y + L^2 z is bit s%32 of
 * word s/32), particle sites pos[N], energy and attempt counter.  Any of
 * the output pointers may be NULL. */
int mucaReadWalker(muca_ctx ctx, int walker, uint32_t* bits, uint32_t* pos, int32_t* E,
                   uint64_t* t);

/* Checkpoint and resume (not part of the paper's method; lets one run of
 * the iteration of Sec. 2 span several processes or sessions).
 * mucaStateBytes: size in bytes of the context's state image.
 * mucaSaveState: waits for the device and writes the image into the host
 *   buffer image (bytes >= mucaStateBytes, else MUCA_EINVAL): a header, the
 *   group list, every walker's occupation bits (in the context's own bit
 *   layout), particle sites, energy, attempt counter and tunnelling state,
 *   and the loop state of mucaRun (finished groups, iteration counts) and
 *   the tunnelling target.  The caller-owned lnW, P and H are not in it:
 *   the caller keeps copies taken at the same point.
 * mucaLoadState: overwrites the context's state with an image saved from a
 *   context created with the same groups, seed and first walker id (else
 *   MUCA_EINVAL, as for a truncated image, another format or a checksum
 *   mismatch; the context is then unchanged); waits for the device.
 *   Afterwards mucaSweep and mucaRun(resume = 1) with the saved lnW and P
 *   continue bit-identically to the run the image was saved from, since
 *   the random streams are counter-based.
 * The image is host-endian and meant for the same library build. */
int mucaStateBytes(muca_ctx ctx, int64_t* bytes);
int mucaSaveState(muca_ctx ctx, void* image, int64_t bytes);
int mucaLoadState(muca_ctx ctx, const void* image, int64_t bytes);

/* Synchronise the context's last stream and report a pending device-side
 * error (MUCA_ENONFINITE) or MUCA_OK.  Clears the pending error. */
int mucaStatus(muca_ctx ctx, void* stream);

/* ------------------------------------------------------------------------
 * Learned initial weights (not part of the paper's method; the recursion
 * from flat weights is its fallback).  A network maps the features
 * (2(d - 2.5), L / 64, 10 N / L^d, E / e_lo) of a bin to
 * y = (lnW(E) - lnW(e_lo)) / N; it is trained on converged weight tables the
 * iteration produced and proposes lnW for a new lattice.
 * Architecture 4 -> 128 -> 128 -> 128 -> 1 with SiLU; hidden layers use BF16
 * weights (round-to-nearest-even copies of FP32 master weights) and BF16
 * activations with FP32 accumulation; the first layer reads FP32 inputs; the
 * output layer has FP32 weights.  Loss: mean squared error over the rows;
 * optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the master weights;
 * gradients pass straight through the BF16 rounding of activations.
 * Parameters (FP32, flat, mucaMlpParamCount() of them): W1[128][4] b1[128]
 * W2[128][128] b2[128] W3[128][128] b3[128] W4[128] b4.
 * X is rows x 4 FP32 (row-major), T and Y rows FP32; all device pointers.
 * ------------------------------------------------------------------------ */
typedef struct muca_mlp* muca_mlp_t;

int mucaMlpParamCount(void);
/* Allocate a network for up to max_rows rows (parameters unset). */
int mucaMlpCreate(muca_mlp_t* out, int max_rows);
int mucaMlpDestroy(muca_mlp_t net);
/* Host copies of the FP32 master parameters; setting them also clears the
 * Adam state and refreshes the BF16 copy (synchronous). */
int mucaMlpSetParams(muca_mlp_t net, const float* params, int n);
int mucaMlpGetParams(muca_mlp_t net, float* params, int n);
/* Y = net(X). */
int mucaMlpForward(muca_mlp_t net, const float* X, int rows, float* Y, void* stream);
/* Gradient of the loss w.r.t. every parameter (grad: device, ParamCount
 * floats) and the loss (device float, may be NULL); parameters unchanged. */
int mucaMlpGradient(muca_mlp_t net, const float* X, const float* T, int rows, float* grad,
                    float* loss, void* stream);
/* One full-batch Adam step with learning rate lr; loss (device, may be
 * NULL) receives the loss before the step. */
int mucaMlpTrainStep(muca_mlp_t net, const float* X, const float* T, int rows, float lr,
                     float* loss, void* stream);
/* Training rows of one group of a context: features X (bins x 4) and, if T
 * is not NULL, targets T = (lnW(E) - lnW(e_lo)) / N from its weights lnW
 * (the context's concatenated layout). */
int mucaMlpTableRows(muca_ctx ctx, int group, const double* lnW, float* X, float* T,
                     void* stream);
/* Initial weights of one group from the network: lnW(E) = N y(E) shifted so
 * that lnW(e_hi) = 0, written into the context's concatenated layout. */
int mucaMlpPredictWeights(muca_mlp_t net, muca_ctx ctx, int group, double* lnW, void* stream);

#ifdef __cplusplus
}
#endif
#endif
