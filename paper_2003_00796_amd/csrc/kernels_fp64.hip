// kernels_fp64.hip -- FP64 instantiation of the transport kernels.  Built with
// -ffp-contract=off: no multiply-add fusion, so the arithmetic follows the
// order of the source expressions.
// the FP64 step kernel needs up to 256 registers: bound it to 2 waves per
// SIMD, so that no flavour's register count (with the accumulation registers
// it may borrow) drops it to one
#ifndef MCX_ESTEP_WAVES
#define MCX_ESTEP_WAVES 2
#endif
// blocks of the tally flush, which loops over the table's span
#ifndef MCX_FLUSH_GRID
#define MCX_FLUSH_GRID 2048
#endif
#include <algorithm>

#include "transport_kernels.h"

namespace mcx {

template <int F>
static hipError_t launch_flavor(const KArgs<double>& a, int par, uint32_t target, int grid, int block, hipStream_t s,
                                hipEvent_t* ev) {
  const size_t sm_f = size_t(T_PHOTON_END) * a.tb.n * sizeof(double);
  const size_t sm_e = (size_t(T_NCH) * a.tb.n + kSoftN) * sizeof(double);
  if (ev) (void)hipEventRecord(ev[0], s);
  // the optional physics changes the e+- step only; weights reach every kernel
  hipLaunchKernelGGL((k_source<double, source_flavor(F)>), dim3(grid), dim3(block), 0, s, a, par);
  if (ev) (void)hipEventRecord(ev[1], s);
  constexpr int PF = photon_flavor(F);
  hipLaunchKernelGGL((k_flight<double, PF>), dim3(grid), dim3(block), several(F) ? sm_f * size_t(a.tb.nmat) : sm_f, s, a, par);
  if (ev) (void)hipEventRecord(ev[2], s);
  hipLaunchKernelGGL((k_knock<double, PF>), dim3(grid), dim3(block), several(F) ? sm_f * size_t(a.tb.nmat) : sm_f, s, a, par);
  if (ev) (void)hipEventRecord(ev[3], s);
  hipLaunchKernelGGL((k_estep<double, F>), dim3(grid), dim3(block), several(F) ? size_t(kSoftN) * sizeof(double) : sm_e, s,
                     a, par);
  if (ev) (void)hipEventRecord(ev[4], s);
  hipLaunchKernelGGL(k_advance<double>, dim3(1), dim3(64), 0, s, a.cnt, par, target, a.cap);
  return hipGetLastError();
}

hipError_t launch_iteration(const KArgs<double>& a, int par, uint32_t target, int grid, int block, hipStream_t s,
                            hipEvent_t* ev) {
  // replays never write the test outputs
  if (a.mode == 1 && a.mm && a.vr) return launch_flavor<FL_MMVR_ADJ_A>(a, par, target, grid, block, s, ev);
  if (a.mode == 2 && a.mm && a.vr) return launch_flavor<FL_MMVR_ADJ_B>(a, par, target, grid, block, s, ev);
  if (a.mode == 0 && a.mm && a.vr)
    return a.test_mode ? launch_flavor<FL_MMVR_TEST>(a, par, target, grid, block, s, ev)
                       : launch_flavor<FL_MMVR>(a, par, target, grid, block, s, ev);
  if (a.mode == 1)
    return a.mm ? launch_flavor<FL_MM_ADJ_A>(a, par, target, grid, block, s, ev)
                : (a.vr ? launch_flavor<FL_VR_ADJ_A>(a, par, target, grid, block, s, ev)
                        : (a.annih ? launch_flavor<FL_EXT_ADJ_A>(a, par, target, grid, block, s, ev)
                                   : launch_flavor<FL_ADJ_A>(a, par, target, grid, block, s, ev)));
  if (a.mode == 2)
    return a.mm ? launch_flavor<FL_MM_ADJ_B>(a, par, target, grid, block, s, ev)
                : (a.vr ? launch_flavor<FL_VR_ADJ_B>(a, par, target, grid, block, s, ev)
                        : (a.annih ? launch_flavor<FL_EXT_ADJ_B>(a, par, target, grid, block, s, ev)
                                   : launch_flavor<FL_ADJ_B>(a, par, target, grid, block, s, ev)));
  if (a.vr)
    return a.test_mode ? launch_flavor<FL_VR_TEST>(a, par, target, grid, block, s, ev)
                       : launch_flavor<FL_VR>(a, par, target, grid, block, s, ev);
  if (a.mm)
    return a.test_mode ? launch_flavor<FL_MM_TEST>(a, par, target, grid, block, s, ev)
                       : launch_flavor<FL_MM>(a, par, target, grid, block, s, ev);
  if (a.straggle || a.annih)
    return a.test_mode ? launch_flavor<FL_EXT_TEST>(a, par, target, grid, block, s, ev)
                       : launch_flavor<FL_EXT>(a, par, target, grid, block, s, ev);
  if (a.test_mode) return launch_flavor<FL_TEST>(a, par, target, grid, block, s, ev);
  return launch_flavor<FL_FWD>(a, par, target, grid, block, s, ev);
}

hipError_t launch_chunk_init(Counters* c, uint64_t first, uint64_t end, uint64_t run_first, uint32_t adm,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_chunk_init<double>, dim3(1), dim3(64), 0, s, c, first, end, run_first, adm);
  return hipGetLastError();
}

hipError_t launch_clear_table(TSlot* tab, uint64_t nslot, hipStream_t s) {
  const unsigned g = unsigned(std::min<uint64_t>((nslot + 255) / 256, 8192));
  hipLaunchKernelGGL(k_clear_table<double>, dim3(g), dim3(256), 0, s, tab, nslot);
  return hipGetLastError();
}

hipError_t launch_flush(TSlot* tab, uint64_t nslot, double* sum_q, double* sum_q2, Counters* cnt,
                        int test_mode, double* hist_led, uint64_t n_run, hipStream_t s) {
  hipLaunchKernelGGL(k_flush<double>, dim3(MCX_FLUSH_GRID), dim3(256), 0, s, tab, nslot, sum_q, sum_q2, cnt, test_mode,
                     hist_led, n_run);
  return hipGetLastError();
}

hipError_t launch_dose(const double* sum_q, const double* sum_q2, const double* rho, uint64_t nvox, double vol,
                       double nhist, double* dose, double* sigma, hipStream_t s) {
  const int block = 256;
  uint64_t g = (nvox + block - 1) / block;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_dose<double>, dim3(unsigned(g)), dim3(block), 0, s, sum_q, sum_q2, rho, nvox, vol, nhist,
                     dose, sigma);
  return hipGetLastError();
}

size_t estep_lds_bytes(int n, bool fp64) {
  return (size_t(T_NCH) * n + kSoftN) * (fp64 ? sizeof(double) : sizeof(float));
}

hipError_t configure_fp64(int n_grid) {
  const int bytes = int(estep_lds_bytes(n_grid, true));
  const void* k[kFlavors] = {reinterpret_cast<const void*>(&k_estep<double, FL_FWD>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_TEST>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_ADJ_A>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_ADJ_B>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_EXT>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_EXT_TEST>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_MM>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_MM_TEST>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_VR>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_VR_TEST>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_MM_ADJ_A>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_MM_ADJ_B>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_VR_ADJ_A>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_VR_ADJ_B>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_EXT_ADJ_A>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_EXT_ADJ_B>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_MMVR>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_MMVR_TEST>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_MMVR_ADJ_A>),
                             reinterpret_cast<const void*>(&k_estep<double, FL_MMVR_ADJ_B>)};
  for (const void* f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cube_map(const double* rho, const uint8_t* mat, int nx, int ny, int nz, uint8_t* out, uint8_t* tmp,
                           hipStream_t s) {
  const uint64_t nv = uint64_t(nx) * ny * nz;
  const unsigned g = unsigned(std::min<uint64_t>((nv + 255) / 256, 65536));
  // seed, then the x, y and z passes: tmp -> out -> tmp -> out
  hipLaunchKernelGGL(k_cube_seed<double>, dim3(g), dim3(256), 0, s, rho, mat, nx, ny, nz, tmp);
  hipLaunchKernelGGL(k_cube_pass<double>, dim3(g), dim3(256), 0, s, tmp, out, nx, ny, nz, 0);
  hipLaunchKernelGGL(k_cube_pass<double>, dim3(g), dim3(256), 0, s, out, tmp, nx, ny, nz, 1);
  hipLaunchKernelGGL(k_cube_pass<double>, dim3(g), dim3(256), 0, s, tmp, out, nx, ny, nz, 2);
  return hipGetLastError();
}

hipError_t launch_adjoint_weights(const double* dl_ddose, const double* rho, uint64_t nvox, double vol, double* w,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_adj_weights<double>, dim3(2048), dim3(256), 0, s, dl_ddose, rho, nvox, vol, w);
  return hipGetLastError();
}

hipError_t launch_adjoint_finalize(const double* grad_acc, const double* dl_ddose, const double* sum_q,
                                   const double* rho, uint64_t nvox, double vol, double nhist, double* out,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_adj_finalize<double>, dim3(2048), dim3(256), 0, s, grad_acc, dl_ddose, sum_q, rho, nvox, vol,
                     nhist, out);
  return hipGetLastError();
}

hipError_t launch_sum(const double* q, uint64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_sum<double>, dim3(1024), dim3(256), 0, s, q, n, out);
  return hipGetLastError();
}

}  // namespace mcx
