// launch.h -- host entry points of the kernels, one overload per precision.
#pragma once

#include <hip/hip_runtime.h>

#include "mcx_internal.h"

namespace mcx {

// one iteration of the event loop: source, flight, knock, e+- steps, advance;
// if ev is not null, ev[0..4] are recorded before the source kernel and after
// each of the four transport kernels (per-kernel durations)
constexpr int kTimedKernels = 4;
hipError_t launch_iteration(const KArgs<double>& a, int par, uint32_t target, int grid, int block, hipStream_t s,
                            hipEvent_t* ev);
hipError_t launch_iteration(const KArgs<float>& a, int par, uint32_t target, int grid, int block, hipStream_t s,
                            hipEvent_t* ev);
hipError_t launch_chunk_init(Counters* c, uint64_t first, uint64_t end, uint64_t run_first, uint32_t adm,
                             hipStream_t s);
// the chunk flush of the tally table, and the clearing of a table
hipError_t launch_clear_table(TSlot* tab, uint64_t nslot, hipStream_t s);
hipError_t launch_flush(TSlot* tab, uint64_t nslot, double* sum_q, double* sum_q2, Counters* cnt,
                        int test_mode, double* hist_led, uint64_t n_run, hipStream_t s);
hipError_t launch_dose(const double* sum_q, const double* sum_q2, const double* rho, uint64_t nvox, double vol,
                       double nhist, double* dose, double* sigma, hipStream_t s);
hipError_t launch_dose(const double* sum_q, const double* sum_q2, const float* rho, uint64_t nvox, double vol,
                       double nhist, double* dose, double* sigma, hipStream_t s);
// density gradient helpers
hipError_t launch_adjoint_weights(const double* dl_ddose, const double* rho, uint64_t nvox, double vol, double* w,
                                  hipStream_t s);
hipError_t launch_adjoint_weights(const double* dl_ddose, const float* rho, uint64_t nvox, double vol, double* w,
                                  hipStream_t s);
hipError_t launch_adjoint_finalize(const double* grad_acc, const double* dl_ddose, const double* sum_q,
                                   const double* rho, uint64_t nvox, double vol, double nhist, double* out,
                                   hipStream_t s);
hipError_t launch_adjoint_finalize(const double* grad_acc, const double* dl_ddose, const double* sum_q,
                                   const float* rho, uint64_t nvox, double vol, double nhist, double* out,
                                   hipStream_t s);
hipError_t launch_sum(const double* q, uint64_t n, double* out, hipStream_t s);
// per-source dose influence: the chunk flush that also adds every score to
// the (source, voxel) table, and the table's compaction into arrays
hipError_t launch_flush_influence(TSlot* tab, uint64_t nslot, double* sum_q2, Counters* cnt,
                                  int test_mode, double* hist_led, uint64_t n_run, const SourceDev* src, int nsrc,
                                  uint64_t* ikeys, double* iq, double* iq2, uint64_t imask, uint32_t* iovf,
                                  hipStream_t s);
hipError_t launch_influence_compact(const uint64_t* ikeys, const double* iq, const double* iq2, uint64_t nslot,
                                    uint32_t* osrc, uint32_t* ovox, double* oq, double* oq2, uint64_t cap,
                                    unsigned long long* count, hipStream_t s);
// same-density cube half-widths of every voxel into `out` (tmp: nvox bytes)
// (mat, when not null: a cube also has one material throughout)
hipError_t launch_cube_map(const double* rho, const uint8_t* mat, int nx, int ny, int nz, uint8_t* out, uint8_t* tmp,
                           hipStream_t s);
hipError_t launch_cube_map(const float* rho, const uint8_t* mat, int nx, int ny, int nz, uint8_t* out, uint8_t* tmp,
                           hipStream_t s);
// LDS bytes the e+- kernel stages for a grid of n nodes
size_t estep_lds_bytes(int n, bool fp64);
hipError_t configure_kernels(int n_grid, bool fp64);

}  // namespace mcx
