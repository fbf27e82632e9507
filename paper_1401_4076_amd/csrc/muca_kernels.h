// muca_kernels.h -- kernel declarations shared by the kernel and runtime
// translation units of libmuca.
#pragma once

#include "muca_device.h"

namespace muca {

__global__ void k_init_place(const GroupDesc* groups, const int32_t* wgroup, uint32_t* bits,
                             uint32_t* pos, int32_t* E, uint64_t* T, int nwalkers,
                             uint32_t first_id, uint32_t seed32);
__global__ void k_thresholds(const GroupDesc* groups, const double* lnW, uint32_t* thr,
                             int32_t* status);
__global__ void k_zero_hist(const GroupDesc* groups, const int32_t* active, int32_t* H);
__global__ void k_sweep_lane(const GroupDesc* groups, const int32_t* wgroup, uint32_t* bits,
                             uint32_t* pos, int32_t* E, uint64_t* T, uint32_t* tun,
                             const uint32_t* thr,
                             int32_t* H, const int32_t* active, int nwalkers, int sweeps,
                             uint32_t first_id, uint32_t seed32);
template <int G, bool kLds, bool kTbl, int kPipe>
__global__ void k_sweep_sub(const GroupDesc* groups, const SweepTask* tasks, const int32_t* first,
                            uint32_t* gbits, uint32_t* gpos, int32_t* gE, uint64_t* gT,
                            uint32_t* gtun, const uint32_t* thr, int32_t* H,
                            const int32_t* active, int sweeps,
                            uint32_t first_id, uint32_t seed32, int tbl_words, int hist_words);
template <bool kTbl>
__global__ void k_sweep_look(const GroupDesc* groups, const SweepTask* tasks, uint32_t* gbits,
                             uint32_t* gpos, int32_t* gE, uint64_t* gT, uint32_t* gtun,
                             const uint32_t* thr, int32_t* H, const int32_t* active, int sweeps,
                             uint32_t first_id,
                             uint32_t seed32, int tbl_words, int hist_words);
__global__ void k_update(const GroupDesc* groups, const int32_t* H, double* lnW, double* P,
                         double* slope, int rule, const int32_t* active, int32_t* status);
__global__ void k_flat(const GroupDesc* groups, const int32_t* H, int32_t* flags);
__global__ void k_control(const GroupDesc* groups, const int32_t* H, int32_t* active,
                          int32_t* flat, int32_t* iters, int32_t* iter_counter,
                          int32_t* remaining, const uint32_t* tun, int stop, int tunnel_target);
__global__ void k_reweight(const GroupDesc* groups, const double* lnW, const int32_t* H,
                           const double* beta, int nbeta, double* out);
__global__ void k_largest_cluster(const GroupDesc* groups, const int32_t* wgroup,
                                  const uint32_t* pos, const int32_t* E, int32_t* out,
                                  long long* osum, int32_t* ocount);
__global__ void k_reweight_obs(const GroupDesc* groups, const double* lnW, const int32_t* cnt,
                               const long long* osum, const double* beta, int nbeta,
                               double* out);
__global__ void k_random_lines(const uint32_t* table, uint32_t lines, int rounds, uint32_t seed,
                               uint32_t* sink);
__global__ void k_bump(int32_t* counter);
__global__ void k_fill_i32(int32_t* p, int32_t v, int n);
__global__ void k_fill_f64(double* p, double v, int n);
__global__ void k_fill_i64(long long* p, long long v, int n);

}  // namespace muca
