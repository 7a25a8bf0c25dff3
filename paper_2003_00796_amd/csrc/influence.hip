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
      // a key stays in its slot until the table is cleared, so a load that
      // finds one (this entry's or another's) needs no compare-and-swap; only
      // a slot seen empty is claimed, and the swap returns what is there now
      uint64_t o = __hip_atomic_load(&ikeys[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (o == kEmptyKey)
        o = atomicCAS((unsigned long long*)&ikeys[slot], (unsigned long long)kEmptyKey, (unsigned long long)ik);
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

// occupied entries of the (source, voxel) table, in no fixed order; entries
// beyond cap are counted, not written.  The places are handed out by one
// counter, which serialises every atomic taken on it (~1e8 per second), so a
// block reserves them once per tile of kCompactBlock x kCompactPer slots:
// each thread holds its kCompactPer keys in registers, the block sums the
// threads' counts (shuffles within a wavefront, LDS across them), thread 0
// takes the tile's places, and each thread writes its entries from its
// prefix on
constexpr int kCompactBlock = 256;
constexpr int kCompactPer = 16;

__global__ __launch_bounds__(kCompactBlock) void k_influence_compact(const uint64_t* ikeys, const double* iq,
                                                                     const double* iq2, uint64_t nslot, uint32_t* osrc,
                                                                     uint32_t* ovox, double* oq, double* oq2,
                                                                     uint64_t cap, unsigned long long* count) {
  constexpr int kWaves = kCompactBlock / 64;
  __shared__ uint32_t wave_total[kWaves];
  __shared__ unsigned long long tile_base;
  const uint32_t lane = __lane_id(), wave = threadIdx.x / 64;
  const uint64_t tile = uint64_t(kCompactBlock) * kCompactPer;
  // t0 depends on the block only: every thread runs the same tiles
  for (uint64_t t0 = uint64_t(blockIdx.x) * tile; t0 < nslot; t0 += uint64_t(gridDim.x) * tile) {
    uint64_t k[kCompactPer];
    uint32_t mine = 0;
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) {
      const uint64_t s = t0 + uint64_t(j) * kCompactBlock + threadIdx.x;
      k[j] = s < nslot ? ikeys[s] : kEmptyKey;
      mine += k[j] != kEmptyKey ? 1u : 0u;
    }
    uint32_t incl = mine;  // inclusive prefix of the counts within the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane >= uint32_t(o)) incl += y;
    }
    if (lane == 63) wave_total[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wave_total[w];
      before += uint32_t(w) < wave ? c : 0u;
      total += c;
    }
    if (threadIdx.x == 0) tile_base = total ? atomicAdd(count, (unsigned long long)total) : 0ull;
    __syncthreads();
    unsigned long long i = tile_base + before + (incl - mine);
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) {
      if (k[j] == kEmptyKey) continue;
      if (i < cap) {
        const uint64_t s = t0 + uint64_t(j) * kCompactBlock + threadIdx.x;
        osrc[i] = uint32_t(k[j] >> 32);
        ovox[i] = uint32_t(k[j] & 0xFFFFFFFFull);
        oq[i] = iq[s];
        oq2[i] = iq2[s];
      }
      ++i;
    }
    __syncthreads();  // wave_total and tile_base are written again by the next tile
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
  hipLaunchKernelGGL(k_influence_compact, dim3(4096), dim3(kCompactBlock), 0, s, ikeys, iq, iq2, nslot, osrc, ovox, oq, oq2,
                     cap, count);
  return hipGetLastError();
}

}  // namespace mcx
