// influence.hip -- per-source (beamlet) dose-influence tally.
//
// Treatment planning with many beamlets needs, besides the summed dose, the
// dose each beamlet delivers to each voxel.  The per-history tally already
// holds every (history, voxel) score q of a chunk until the chunk's flush
// (the estimator of Eq. (1)-(3) of the paper needs each history's score
// complete before it is squared); when influence output is on, the flush
// also adds q and q^2 to a second open-addressing table keyed by
// (source index, voxel).  The source of a history is found by binary search
// over the sources' cumulative history counts.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "mcx_internal.h"
#include "transport_device.h"

namespace mcx {

namespace {

// index of the source owning history h: the first s with h < src[s].end
__device__ __forceinline__ uint32_t source_of(const SourceDev* src, int nsrc, uint64_t h) {
  int lo = 0, hi = nsrc - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (h < src[mid].end) hi = mid;
    else lo = mid + 1;
  }
  return uint32_t(lo);
}

// the chunk flush of k_flush (Sum q^2, run statistics, test ledger, slots
// cleared), and each score also added to the (source, voxel) table
__global__ void k_flush_influence(TSlot* tab, uint64_t nslot, double* sum_q2, Counters* cnt,
                                  int test_mode, double* hist_led, uint64_t n_run, const SourceDev* src, int nsrc,
                                  uint64_t* ikeys, double* iq, double* iq2, uint64_t imask, uint32_t* iovf) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  uint32_t occ = 0;
  double dep = 0.0;
  for (uint64_t s = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < nslot; s += stride) {
    const TSlot t = tab[s];
    const uint64_t k = t.key;
    if (k == kEmptyKey) continue;
    const double q = t.q;
    dep += q;
    const uint32_t v = uint32_t(k & 0xFFFFFFFFull);
    unsafeAtomicAdd(&sum_q2[v], q * q);
    if (test_mode) {
      const uint64_t h = (k >> 32) - cnt->run_first;
      if (h < n_run) unsafeAtomicAdd(&hist_led[3 * h], q);
    }
    const uint64_t ik = (uint64_t(source_of(src, nsrc, k >> 32)) << 32) | v;
    uint64_t slot = mix64(ik) & imask;
    int probe = 0;
    for (; probe < 4096; ++probe) {
      const uint64_t o =
          atomicCAS((unsigned long long*)&ikeys[slot], (unsigned long long)kEmptyKey, (unsigned long long)ik);
      if (o == kEmptyKey || o == ik) {
        unsafeAtomicAdd(&iq[slot], q);
        unsafeAtomicAdd(&iq2[slot], q * q);
        break;
      }
      slot = (slot + 1) & imask;
    }
    if (probe == 4096) atomicOr(iovf, 1u);
    tab[s] = TSlot{kEmptyKey, 0.0};
    ++occ;
  }
  occ = wave_sum(occ);
  dep = wave_sum(dep);
  if (__lane_id() == 0 && occ) atomicAdd((unsigned long long*)&cnt->occupied, (unsigned long long)occ);
  if (__lane_id() == 0 && dep != 0.0) unsafeAtomicAdd(&cnt->e_dep, dep);
}

// occupied entries of the (source, voxel) table, in slot order of arrival;
// entries beyond cap are counted, not written
__global__ void k_influence_compact(const uint64_t* ikeys, const double* iq, const double* iq2, uint64_t nslot,
                                    uint32_t* osrc, uint32_t* ovox, double* oq, double* oq2, uint64_t cap,
                                    unsigned long long* count) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t s = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < nslot; s += stride) {
    const uint64_t k = ikeys[s];
    if (k == kEmptyKey) continue;
    const unsigned long long i = atomicAdd(count, 1ull);
    if (i < cap) {
      osrc[i] = uint32_t(k >> 32);
      ovox[i] = uint32_t(k & 0xFFFFFFFFull);
      oq[i] = iq[s];
      oq2[i] = iq2[s];
    }
  }
}

}  // namespace

hipError_t launch_flush_influence(TSlot* tab, uint64_t nslot, double* sum_q2, Counters* cnt,
                                  int test_mode, double* hist_led, uint64_t n_run, const SourceDev* src, int nsrc,
                                  uint64_t* ikeys, double* iq, double* iq2, uint64_t imask, uint32_t* iovf,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_flush_influence, dim3(8192), dim3(256), 0, s, tab, nslot, sum_q2, cnt, test_mode,
                     hist_led, n_run, src, nsrc, ikeys, iq, iq2, imask, iovf);
  return hipGetLastError();
}

hipError_t launch_influence_compact(const uint64_t* ikeys, const double* iq, const double* iq2, uint64_t nslot,
                                    uint32_t* osrc, uint32_t* ovox, double* oq, double* oq2, uint64_t cap,
                                    unsigned long long* count, hipStream_t s) {
  hipLaunchKernelGGL(k_influence_compact, dim3(4096), dim3(256), 0, s, ikeys, iq, iq2, nslot, osrc, ovox, oq, oq2,
                     cap, count);
  return hipGetLastError();
}

}  // namespace mcx
