// kernels_mixed.hip -- FP32-physics instantiation of the transport kernels
// (positions, boundary distances, remaining mass thickness and tallies stay
// FP64).  Multiply-add contraction is allowed here.
// the FP32 step and photon-walk kernels fit 128 registers: bound them to 4
// waves per SIMD
#ifndef MCX_ESTEP_WAVES
#define MCX_ESTEP_WAVES 4
#endif
#ifndef MCX_FLIGHT_WAVES
#define MCX_FLIGHT_WAVES 4
#endif
#include <algorithm>

#include "transport_kernels.h"

namespace mcx {

template <int F>
static hipError_t launch_flavor(const KArgs<float>& a, int par, uint32_t target, int grid, int block, hipStream_t s,
                                hipEvent_t* ev) {
  const size_t sm_f = size_t(T_PHOTON_END) * a.tb.n * sizeof(float);
  const size_t sm_e = (size_t(T_NCH) * a.tb.n + kSoftN) * sizeof(float);
  if (ev) (void)hipEventRecord(ev[0], s);
  // the optional physics changes the e+- step only; weights reach every kernel
  hipLaunchKernelGGL((k_source<float, source_flavor(F)>), dim3(grid), dim3(block), 0, s, a, par);
  if (ev) (void)hipEventRecord(ev[1], s);
  constexpr int PF = photon_flavor(F);
  hipLaunchKernelGGL((k_flight<float, PF>), dim3(grid), dim3(block), several(F) ? sm_f * size_t(a.tb.nmat) : sm_f, s, a, par);
  if (ev) (void)hipEventRecord(ev[2], s);
  hipLaunchKernelGGL((k_knock<float, PF>), dim3(grid), dim3(block), several(F) ? sm_f * size_t(a.tb.nmat) : sm_f, s, a, par);
  if (ev) (void)hipEventRecord(ev[3], s);
  hipLaunchKernelGGL((k_estep<float, F>), dim3(grid), dim3(block), several(F) ? size_t(kSoftN) * sizeof(float) : sm_e, s,
                     a, par);
  if (ev) (void)hipEventRecord(ev[4], s);
  hipLaunchKernelGGL(k_advance<float>, dim3(1), dim3(64), 0, s, a.cnt, par, target, a.cap);
  return hipGetLastError();
}

hipError_t launch_iteration(const KArgs<float>& a, int par, uint32_t target, int grid, int block, hipStream_t s,
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

hipError_t launch_dose(const double* sum_q, const double* sum_q2, const float* rho, uint64_t nvox, double vol,
                       double nhist, double* dose, double* sigma, hipStream_t s) {
  const int block = 256;
  uint64_t g = (nvox + block - 1) / block;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_dose<float>, dim3(unsigned(g)), dim3(block), 0, s, sum_q, sum_q2, rho, nvox, vol, nhist,
                     dose, sigma);
  return hipGetLastError();
}

hipError_t configure_fp64(int n_grid);

hipError_t configure_kernels(int n_grid, bool fp64) {
  if (fp64) return configure_fp64(n_grid);
  const int bytes = int(estep_lds_bytes(n_grid, false));
  const void* k[kFlavors] = {reinterpret_cast<const void*>(&k_estep<float, FL_FWD>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_TEST>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_ADJ_A>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_ADJ_B>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_EXT>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_EXT_TEST>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_MM>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_MM_TEST>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_VR>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_VR_TEST>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_MM_ADJ_A>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_MM_ADJ_B>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_VR_ADJ_A>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_VR_ADJ_B>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_EXT_ADJ_A>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_EXT_ADJ_B>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_MMVR>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_MMVR_TEST>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_MMVR_ADJ_A>),
                             reinterpret_cast<const void*>(&k_estep<float, FL_MMVR_ADJ_B>)};
  for (const void* f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cube_map(const float* rho, const uint8_t* mat, int nx, int ny, int nz, uint8_t* out, uint8_t* tmp,
                           hipStream_t s) {
  const uint64_t nv = uint64_t(nx) * ny * nz;
  const unsigned g = unsigned(std::min<uint64_t>((nv + 255) / 256, 65536));
  // seed, then the x, y and z passes: tmp -> out -> tmp -> out
  hipLaunchKernelGGL(k_cube_seed<float>, dim3(g), dim3(256), 0, s, rho, mat, nx, ny, nz, tmp);
  hipLaunchKernelGGL(k_cube_pass<float>, dim3(g), dim3(256), 0, s, tmp, out, nx, ny, nz, 0);
  hipLaunchKernelGGL(k_cube_pass<float>, dim3(g), dim3(256), 0, s, out, tmp, nx, ny, nz, 1);
  hipLaunchKernelGGL(k_cube_pass<float>, dim3(g), dim3(256), 0, s, tmp, out, nx, ny, nz, 2);
  return hipGetLastError();
}

hipError_t launch_adjoint_weights(const double* dl_ddose, const float* rho, uint64_t nvox, double vol, double* w,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_adj_weights<float>, dim3(2048), dim3(256), 0, s, dl_ddose, rho, nvox, vol, w);
  return hipGetLastError();
}

hipError_t launch_adjoint_finalize(const double* grad_acc, const double* dl_ddose, const double* sum_q,
                                   const float* rho, uint64_t nvox, double vol, double nhist, double* out,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_adj_finalize<float>, dim3(2048), dim3(256), 0, s, grad_acc, dl_ddose, sum_q, rho, nvox, vol,
                     nhist, out);
  return hipGetLastError();
}

}  // namespace mcx
