// transport_device.h -- device side of the particle-history loop, templated
// on the compute type T (double: FP64 path; float: mixed path with FP64
// positions, boundary distances and tallies).
//
// Event-based organisation of the loop of Sec. 4.1 of the paper (JUMP, STEP,
// KNOCK): particles live in structure-of-arrays queues, one queue per event
// type, so that each wavefront runs one kind of event:
//   k_source  new primaries for history ids taken from a global cursor
//   k_flight  photon JUMP + STEP (free path in mass thickness, voxel DDA);
//             sorts each photon into the queue of its interaction
//   k_knock   photon KNOCK, one interaction type per queue
//   k_estep   electron/positron Class II steps (up to `steps` per visit),
//             hard events inline
//   k_advance queue bookkeeping and admission of the next histories
// Energy deposits are coalesced per particle and voxel in registers and added
// to an open-addressing (history, voxel) table; k_flush turns each history's
// per-voxel score q into Sum q and Sum q^2 (Eq. (1)-(3)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mcx_internal.h"

namespace mcx {

// ---------------------------------------------------------------------------
// math in the compute type
// ---------------------------------------------------------------------------
template <typename T>
struct M;

template <>
struct M<double> {
  static __device__ __forceinline__ double log(double x) { return ::log(x); }
  static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
  static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ double pow(double a, double b) { return ::exp(b * ::log(a)); }
  static __device__ __forceinline__ double log1p(double x) { return ::log1p(x); }
  static __device__ __forceinline__ double expm1(double x) { return ::expm1(x); }
  static __device__ __forceinline__ double floor(double x) { return ::floor(x); }
  static __device__ __forceinline__ void sincos(double x, double* s, double* c) { ::sincos(x, s, c); }
  static __device__ __forceinline__ double cos(double x) { return ::cos(x); }
  static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
};

template <>
struct M<float> {
  static __device__ __forceinline__ float log(float x) { return __logf(x); }
  static __device__ __forceinline__ float exp(float x) { return __expf(x); }
  static __device__ __forceinline__ float sqrt(float x) { return ::sqrtf(x); }
  static __device__ __forceinline__ float pow(float a, float b) { return __expf(b * __logf(a)); }
  // log(1 + x) accurate for small x: log(u) x / (u - 1) with u = 1 + x
  // (the rounding of u cancels in the ratio)
  static __device__ __forceinline__ float log1p(float x) {
    const float u = 1.0f + x;
    return u == 1.0f ? x : __logf(u) * (x / (u - 1.0f));
  }
  // exp(x) - 1 accurate for small x: (u - 1) x / log(u) with u = exp(x)
  static __device__ __forceinline__ float expm1(float x) {
    const float u = __expf(x);
    return u == 1.0f ? x : (u - 1.0f) * (x / __logf(u));
  }
  static __device__ __forceinline__ float floor(float x) { return ::floorf(x); }
  static __device__ __forceinline__ void sincos(float x, float* s, float* c) { __sincosf(x, s, c); }
  static __device__ __forceinline__ float cos(float x) { return __cosf(x); }
  static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
};

template <typename T>
constexpr bool is_fp64() { return std::is_same<T, double>::value; }

// ---------------------------------------------------------------------------
// counter-based random numbers: Philox4x32-10 (Salmon et al., SC'11)
// key = (seed, history id); counter = (draw / 2, uid_lo, uid_hi, 0);
// draw d is 64-bit word d % 2 of the call.
//
// A particle holds the draws [base, base + nw) in w[].  The e+- step refills
// them at the start of a step (`rng_refill`): the rng_pairs<T>() calls from
// the one holding draw ctr on, aligned so that w[0] is draw ctr.  The step's
// draws then sit at offsets the compiler knows along its straight-line path,
// and the one inlined Philox site runs with every live lane.  A draw that is
// not held computes its own call (the rest of the kernels draw only this
// way).  FP32 paths keep only the upper 32 bits of each 64-bit draw word:
// their uniforms use its top 23 bits.  The seed is the same for every
// particle of a launch, so its key schedule runs on the scalar unit.
// ---------------------------------------------------------------------------
#ifndef MCX_RNG_PAIRS
#define MCX_RNG_PAIRS 4
#endif
#ifndef MCX_RNG_PAIRS_FP64
#define MCX_RNG_PAIRS_FP64 4
#endif
// calls held per particle (eight draws cover a typical hard-event step; the
// FP64 words take twice the registers, which the FP64 kernels' 256 hold)
template <typename T>
constexpr int rng_pairs() { return std::is_same<T, double>::value ? MCX_RNG_PAIRS_FP64 : MCX_RNG_PAIRS; }

template <typename T>
struct RngWord {
  using type = uint64_t;
};
template <>
struct RngWord<float> {
  using type = uint32_t;
};

template <typename T>
struct Rng {
  using W = typename RngWord<T>::type;
  uint32_t k0, k1, u0, u1;
  uint32_t ctr;   // next draw index
  uint32_t base;  // draw index of w[0]
  uint32_t nw;    // draws held in w[]
  W w[2 * rng_pairs<T>()];
};

__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                         uint32_t k1, uint32_t* o) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32 x 32 -> 64-bit product is one v_mad_u64_u32 (a separate high
    // and low multiply costs about a third more)
    const uint64_t p0 = uint64_t(0xD2511F53u) * c0, p1 = uint64_t(0xCD9E8D57u) * c2;
    const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  o[0] = c0; o[1] = c1; o[2] = c2; o[3] = c3;
}

// the two draw words of one call
__device__ __forceinline__ void pair_words(const uint32_t* o, uint64_t* w0, uint64_t* w1) {
  *w0 = (uint64_t(o[1]) << 32) | o[0];
  *w1 = (uint64_t(o[3]) << 32) | o[2];
}
__device__ __forceinline__ void pair_words(const uint32_t* o, uint32_t* w0, uint32_t* w1) {
  *w0 = o[1];
  *w1 = o[3];
}

template <typename T>
__device__ __forceinline__ void rng_init(Rng<T>& r, uint32_t seed, uint32_t hist, uint64_t uid, uint32_t ctr) {
  r.k0 = seed; r.k1 = hist;
  r.u0 = uint32_t(uid); r.u1 = uint32_t(uid >> 32);
  r.ctr = ctr;
  r.base = ctr;
  r.nw = 0u;
}

// one Philox call of the particle's stream (the seed is wave-uniform)
template <typename T>
__device__ __forceinline__ void rng_call(const Rng<T>& r, uint32_t pair, uint32_t* o) {
  philox10(pair, r.u0, r.u1, 0u, __builtin_amdgcn_readfirstlane(r.k0), r.k1, o);
}

// hold the draws from ctr on: rng_pairs<T>() calls from the one holding draw
// ctr; when ctr is odd the first word of that call is already used
template <typename T>
__device__ __forceinline__ void rng_refill(Rng<T>& r) {
  using W = typename RngWord<T>::type;
  constexpr int kW = 2 * rng_pairs<T>();
  const uint32_t pair = r.ctr >> 1;
  W raw[kW];
#pragma unroll
  for (int j = 0; j < rng_pairs<T>(); ++j) {
    uint32_t o[4];
    rng_call(r, pair + uint32_t(j), o);
    pair_words(o, &raw[2 * j], &raw[2 * j + 1]);
  }
  // shift by one word when ctr is odd, as a bitwise blend: written as a
  // select, the compiler turns the shift into an indexed load from a stack
  // copy of raw[] (a scratch round trip per step); the bit-field extract
  // keeps the mask opaque to that rewrite
  const uint32_t odd = __builtin_amdgcn_ubfe(r.ctr, 0u, 1u);
  const W m = W(0) - W(odd);
#pragma unroll
  for (int j = 0; j < kW - 1; ++j) r.w[j] = (raw[j] & ~m) | (raw[j + 1] & m);
  r.w[kW - 1] = raw[kW - 1];
  r.base = r.ctr;
  r.nw = uint32_t(kW) - odd;
}

// next draw word (unrolled selects: no runtime-indexed private array)
template <typename T>
__device__ __forceinline__ typename RngWord<T>::type rng_next(Rng<T>& r) {
  uint32_t off = r.ctr - r.base;
  if (!(off < r.nw)) {
    uint32_t o[4];
    rng_call(r, r.ctr >> 1, o);
    typename RngWord<T>::type w0, w1;
    pair_words(o, &w0, &w1);
    const bool odd = (r.ctr & 1u) != 0u;
    r.w[0] = odd ? w1 : w0;
    r.w[1] = w1;
    r.base = r.ctr;
    r.nw = odd ? 1u : 2u;
    off = 0u;
  }
  typename RngWord<T>::type v = r.w[0];
#pragma unroll
  for (int j = 1; j < 2 * rng_pairs<T>(); ++j) v = off == uint32_t(j) ? r.w[j] : v;
  r.ctr++;
  return v;
}

template <typename T>
__device__ __forceinline__ T uni(Rng<T>& r);
template <>
__device__ __forceinline__ double uni<double>(Rng<double>& r) {
  return (double(rng_next(r) >> 11) + 0.5) * 0x1.0p-53;
}
// FP32: top 23 bits of the same 64-bit word, ((w >> 41) + 1/2) 2^-23, exact in FP32
template <>
__device__ __forceinline__ float uni<float>(Rng<float>& r) {
  return (float(rng_next(r) >> 9) + 0.5f) * 0x1.0p-23f;
}

// SplitMix64 finaliser (Steele et al., OOPSLA'14)
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// uid of the k-th secondary of a particle
__device__ __forceinline__ uint64_t child_uid(uint64_t parent, uint32_t k) {
  return mix64((parent ^ (uint64_t(k + 1u) * 0x9E3779B97F4A7C15ull)) + 0x9E3779B97F4A7C15ull);
}

// ---------------------------------------------------------------------------
// particle state in registers
// ---------------------------------------------------------------------------
template <typename T>
struct Part {
  double x[3];
  T d[3];
  T e;
  int ix[3];
  uint32_t type, nchild;
  uint32_t hist;
  uint64_t uid;
  uint64_t hash;
  double w;  // statistical weight (1 without interaction forcing)
  T clk;     // e+-: majorant optical depth left before the next hard or delta event, 0 if none pending
  Rng<T> rng;
};

__device__ __forceinline__ uint64_t join64(uint32_t lo, uint32_t hi) { return uint64_t(lo) | (uint64_t(hi) << 32); }
__device__ __forceinline__ double join_f64(uint32_t lo, uint32_t hi) {
  return __longlong_as_double(static_cast<long long>(join64(lo, hi)));
}
__device__ __forceinline__ void split64(uint64_t v, uint32_t& lo, uint32_t& hi) {
  lo = uint32_t(v);
  hi = uint32_t(v >> 32);
}
__device__ __forceinline__ void split_f64(double d, uint32_t& lo, uint32_t& hi) {
  split64(static_cast<uint64_t>(__double_as_longlong(d)), lo, hi);
}
__device__ __forceinline__ uint32_t pack_vox(const int ix[3]) {
  return uint32_t(ix[0]) | (uint32_t(ix[1]) << 10) | (uint32_t(ix[2]) << 20);
}

// write a record: position and voxel of `p`, then direction, energy, uid,
// draw counter and type/children given
template <typename T>
__device__ __forceinline__ void store_record(const KArgs<T>& a, const Bank<T>& b, uint32_t i, const Part<T>& p,
                                             const T d[3], T e, uint64_t uid, uint32_t ctr, uint32_t flags,
                                             uint64_t hash, double w, T clk) {
  Chunk c0, c1, cm;
  split_f64(p.x[0], c0.x, c0.y);
  split_f64(p.x[1], c0.z, c0.w);
  split_f64(p.x[2], c1.x, c1.y);
  split64(uid, c1.z, c1.w);
  cm.x = p.hist;
  cm.y = ctr;
  cm.z = pack_vox(p.ix);
  cm.w = flags;
  b.c[0][i] = c0;
  b.c[1][i] = c1;
  if constexpr (sizeof(T) == 8) {
    Chunk c2, c3;
    split_f64(double(d[0]), c2.x, c2.y);
    split_f64(double(d[1]), c2.z, c2.w);
    split_f64(double(d[2]), c3.x, c3.y);
    split_f64(double(e), c3.z, c3.w);
    b.c[2][i] = c2;
    b.c[3][i] = c3;
    b.c[4][i] = cm;
  } else {
    Chunk c2;
    c2.x = __float_as_uint(float(d[0]));
    c2.y = __float_as_uint(float(d[1]));
    c2.z = __float_as_uint(float(d[2]));
    c2.w = __float_as_uint(float(e));
    b.c[2][i] = c2;
    b.c[3][i] = cm;
  }
  if (a.test_mode) b.hash[i] = hash;
  if (a.vr) b.w[i] = w;
  if (b.clk) b.clk[i] = clk;  // the e+- queues
}

template <typename T>
__device__ __forceinline__ void load_part(const KArgs<T>& a, const Bank<T>& b, uint32_t i, Part<T>& p) {
  const Chunk c0 = b.c[0][i], c1 = b.c[1][i];
  Chunk cm;
  p.x[0] = join_f64(c0.x, c0.y);
  p.x[1] = join_f64(c0.z, c0.w);
  p.x[2] = join_f64(c1.x, c1.y);
  p.uid = join64(c1.z, c1.w);
  if constexpr (sizeof(T) == 8) {
    const Chunk c2 = b.c[2][i], c3 = b.c[3][i];
    cm = b.c[4][i];
    p.d[0] = T(join_f64(c2.x, c2.y));
    p.d[1] = T(join_f64(c2.z, c2.w));
    p.d[2] = T(join_f64(c3.x, c3.y));
    p.e = T(join_f64(c3.z, c3.w));
  } else {
    const Chunk c2 = b.c[2][i];
    cm = b.c[3][i];
    p.d[0] = T(__uint_as_float(c2.x));
    p.d[1] = T(__uint_as_float(c2.y));
    p.d[2] = T(__uint_as_float(c2.z));
    p.e = T(__uint_as_float(c2.w));
  }
  p.hist = cm.x;
  p.ix[0] = int(cm.z & 1023u); p.ix[1] = int((cm.z >> 10) & 1023u); p.ix[2] = int(cm.z >> 20);
  p.type = cm.w & 3u;
  p.nchild = cm.w >> 2;
  p.hash = a.test_mode ? b.hash[i] : 0ull;
  p.w = a.vr ? b.w[i] : 1.0;
  p.clk = b.clk ? b.clk[i] : T(0);
  rng_init(p.rng, a.seed, p.hist, p.uid, cm.y);
}

template <typename T>
__device__ __forceinline__ void store_part(const KArgs<T>& a, const Bank<T>& b, uint32_t i, const Part<T>& p) {
  store_record(a, b, i, p, p.d, p.e, p.uid, p.rng.ctr, p.type | (p.nchild << 2), p.hash, p.w, p.clk);
}

// a secondary waiting to be appended: shares position/voxel/history with its parent
template <typename T>
struct Child {
  T d[3];
  T e;
  uint32_t type;
  uint64_t uid;
  double w;
  bool on;
};

template <typename T>
__device__ __forceinline__ void store_child(const KArgs<T>& a, const Bank<T>& b, uint32_t i, const Part<T>& p,
                                            const Child<T>& c) {
  store_record(a, b, i, p, c.d, c.e, c.uid, 0u, c.type, 0ull, c.w, T(0));
}

// ---------------------------------------------------------------------------
// wavefront-aggregated append: one atomic per wave and destination queue
// (all active lanes of the wave must call it)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool pred) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0ull) return ~0u;
  const uint32_t lane = __lane_id();
  const uint32_t leader = uint32_t(__ffsll((unsigned long long)mask) - 1);
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, uint32_t(__popcll(mask)));
  base = __shfl(base, int(leader));
  const uint32_t below = uint32_t(__popcll(mask & ((1ull << lane) - 1ull)));
  return pred ? base + below : ~0u;
}

// ---------------------------------------------------------------------------
// statistics: frequent events counted in registers per lane and reduced per
// wave at the end of a kernel; rare ones through LDS; one global atomic per
// counter per block
// ---------------------------------------------------------------------------
struct BlockStats {
  unsigned long long c[S_NSTAT];
  double e_esc;
};

// per-lane registers for the counters of every step or flight; the rest go
// through LDS (stat_add), and the deposited energy is summed by the flush
struct LaneStats {
  uint32_t esteps, deposits, flights, crossings, inserts;
};

__device__ __forceinline__ void stats_init(BlockStats* s, LaneStats& l) {
  for (int i = threadIdx.x; i < S_NSTAT; i += blockDim.x) s->c[i] = 0ull;
  if (threadIdx.x == 0) s->e_esc = 0.0;
  l.esteps = l.deposits = l.flights = l.crossings = l.inserts = 0u;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// every thread of the block must call this (after its last event)
__device__ __forceinline__ void stats_flush(BlockStats* s, const LaneStats& l, Counters* cnt) {
  const uint32_t es = wave_sum(l.esteps), de = wave_sum(l.deposits);
  const uint32_t fl = wave_sum(l.flights), cr = wave_sum(l.crossings), in = wave_sum(l.inserts);
  if (__lane_id() == 0) {
    if (in) atomicAdd(&s->c[S_INSERTS], (unsigned long long)in);
    if (es) atomicAdd(&s->c[S_ESTEPS], (unsigned long long)es);
    if (de) atomicAdd(&s->c[S_DEPOSITS], (unsigned long long)de);
    if (fl) atomicAdd(&s->c[S_FLIGHTS], (unsigned long long)fl);
    if (cr) atomicAdd(&s->c[S_CROSSINGS], (unsigned long long)cr);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < S_NSTAT; i += blockDim.x)
    if (s->c[i]) atomicAdd((unsigned long long*)&cnt->stat[i], s->c[i]);
  if (threadIdx.x == 0 && s->e_esc != 0.0) unsafeAtomicAdd(&cnt->e_esc, s->e_esc);
}

__device__ __forceinline__ void stat_add(BlockStats* s, int k, unsigned long long v = 1ull) {
  atomicAdd(&s->c[k], v);
}

// ---------------------------------------------------------------------------
// tally: (history, voxel) -> score, open addressing with linear probing
// ---------------------------------------------------------------------------
// An insertion is a compare-and-swap of the key into its slot (an empty slot
// is claimed, a slot holding this key is found), then an add of the score
// that nobody waits for.  The score is added to the voxel's Sum q at once
// (Eq. (1) needs no per-history total); the flush scans the table for the
// per-history totals that Sum q^2 needs and clears it.
template <typename T>
__device__ __forceinline__ void tally_probe(const KArgs<T>& a, uint64_t key, double q, uint64_t slot, uint64_t k) {
  for (int probe = 0; probe < 4096; ++probe) {
    if (k == kEmptyKey || k == key) {
      unsafeAtomicAdd(&a.htab[slot].q, q);
      return;
    }
    slot = (slot + 1) & a.hmask;
    k = atomicCAS((unsigned long long*)&a.htab[slot].key, (unsigned long long)kEmptyKey, (unsigned long long)key);
  }
  atomicOr(&a.cnt->overflow, uint32_t(OVF_TALLY));
}

template <typename T>
__device__ __forceinline__ uint64_t tally_slot(const KArgs<T>& a, uint64_t key) {
  return mix64(key) & a.hmask;
}

template <typename T>
__device__ __forceinline__ void tally_insert(const KArgs<T>& a, uint64_t key, double q, LaneStats& ls) {
  ls.inserts++;
  unsafeAtomicAdd(&a.sum_q[uint32_t(key & 0xFFFFFFFFull)], q);
  const uint64_t slot = tally_slot(a, key);
  const uint64_t k = atomicCAS((unsigned long long*)&a.htab[slot].key, (unsigned long long)kEmptyKey,
                               (unsigned long long)key);
  tally_probe(a, key, q, slot, k);
}

// Deposits of one particle are summed in registers while they stay in one
// voxel; when the voxel (or history) changes, the finished sum becomes
// `pending`.  In the e+- kernel the pending entry's compare-and-swap is
// issued at the end of a step and its result examined at the start of the
// next one, so the round trip overlaps the rest of the iteration; the other
// kernels insert at their end.  All deposits of one Class II step or one
// photon interaction fall in the same voxel.
constexpr uint32_t kNotIssued = ~0u;

struct DepAcc {
  uint64_t key;
  double q;
  uint64_t pkey;   // pending (finished) entry
  double pq;
  uint64_t fres;   // result of the pending entry's compare-and-swap
  uint32_t fslot;  // its slot, or kNotIssued
};

__device__ __forceinline__ DepAcc dep_init() { return DepAcc{kEmptyKey, 0.0, kEmptyKey, 0.0, kEmptyKey, kNotIssued}; }

template <typename T>
__device__ __forceinline__ void dep_insert(const KArgs<T>& a, uint64_t key, double q, LaneStats& ls) {
  if (key == kEmptyKey || q == 0.0) return;
  if (a.mode == 0) {
    tally_insert(a, key, q, ls);
  } else if (a.mode == 1) {
    const uint32_t v = uint32_t(key & 0xFFFFFFFFull);
    const uint64_t h = (key >> 32) - a.cnt->run_first;
    unsafeAtomicAdd(&a.adj_q[h], a.adj_w[v] * q);
  }
}

// complete the pending entry whose compare-and-swap is in flight
template <typename T>
__device__ __forceinline__ void dep_resolve(const KArgs<T>& a, DepAcc& acc) {
  if (acc.fslot == kNotIssued) return;
  tally_probe(a, acc.pkey, acc.pq, uint64_t(acc.fslot), acc.fres);
  acc.pkey = kEmptyKey;
  acc.pq = 0.0;
  acc.fslot = kNotIssued;
}

// start the insertion of the pending entry (call at one convergent point per
// step, after dep_resolve earlier in the same step)
template <typename T>
__device__ __forceinline__ void dep_flush_pending(const KArgs<T>& a, DepAcc& acc, LaneStats& ls) {
  if (acc.pkey == kEmptyKey) return;
  if (a.mode != 0 || acc.pq == 0.0) {
    dep_insert(a, acc.pkey, acc.pq, ls);
    acc.pkey = kEmptyKey;
    acc.pq = 0.0;
    return;
  }
  ls.inserts++;
  unsafeAtomicAdd(&a.sum_q[uint32_t(acc.pkey & 0xFFFFFFFFull)], acc.pq);
  const uint64_t slot = tally_slot(a, acc.pkey);
  acc.fslot = uint32_t(slot);
  acc.fres = atomicCAS((unsigned long long*)&a.htab[slot].key, (unsigned long long)kEmptyKey,
                       (unsigned long long)acc.pkey);
}

// insert everything (end of a kernel)
template <typename T>
__device__ __forceinline__ void dep_flush(const KArgs<T>& a, DepAcc& acc, LaneStats& ls) {
  dep_resolve(a, acc);
  dep_insert(a, acc.pkey, acc.pq, ls);
  acc.pkey = kEmptyKey;
  acc.pq = 0.0;
  dep_insert(a, acc.key, acc.q, ls);
  acc.key = kEmptyKey;
  acc.q = 0.0;
}

template <typename T>
__device__ __forceinline__ uint32_t vlin(const KArgs<T>& a, const int ix[3]) {
  return (uint32_t(ix[2]) * uint32_t(a.ny) + uint32_t(ix[1])) * uint32_t(a.nx) + uint32_t(ix[0]);
}

template <typename T>
__device__ __forceinline__ void deposit(const KArgs<T>& a, DepAcc& acc, LaneStats& ls, const Part<T>& p, T e) {
  if (e == T(0)) return;
  const uint64_t key = (uint64_t(p.hist) << 32) | vlin(a, p.ix);
  if (key != acc.key) {
    if (acc.pkey != kEmptyKey) {
      // a second voxel change before the caller flushed: insert now
      if (acc.fslot != kNotIssued) {
        dep_resolve(a, acc);
      } else {
        dep_insert(a, acc.pkey, acc.pq, ls);
      }
    }
    acc.pkey = acc.key;
    acc.pq = acc.q;
    acc.key = key;
    acc.q = 0.0;
  }
  acc.q += a.vr ? double(e) * p.w : double(e);  // weighted under interaction forcing
  ls.deposits++;
}

// ---------------------------------------------------------------------------
// event hash (order independent per history)
// ---------------------------------------------------------------------------
enum Ev : uint32_t {
  EV_COMPTON = 1, EV_PHOTO = 2, EV_RAYLEIGH = 3, EV_PAIR = 4, EV_PH_ESCAPE = 5,
  EV_CROSS = 6, EV_STEP = 7, EV_HARD_EL = 8, EV_HARD_IN = 9, EV_HARD_BR = 10,
  EV_ABSORB = 11, EV_E_ESCAPE = 12, EV_ANNIH_FLIGHT = 13
};

template <typename T>
__device__ __forceinline__ void event(const KArgs<T>& a, Part<T>& p, uint32_t code, uint32_t v) {
  if (!a.test_mode) return;
  const uint64_t word = uint64_t(code) | (uint64_t(v) << 8) | (uint64_t(p.nchild & 0xFFFFFFu) << 40);
  p.hash = mix64(p.hash + word);
}

template <typename T>
__device__ __forceinline__ void finish(const KArgs<T>& a, const Part<T>& p) {
  if (!a.test_mode) return;
  atomicAdd((unsigned long long*)&a.hist_hash[p.hist - a.cnt->run_first],
            (unsigned long long)mix64(p.hash ^ p.uid));
}

template <typename T>
__device__ __forceinline__ void ledger_escape(const KArgs<T>& a, BlockStats* st, const Part<T>& p) {
  stat_add(st, S_ESCAPED);
  const double ew = a.vr ? double(p.e) * p.w : double(p.e);
  atomicAdd(&st->e_esc, ew);
  if (p.type == POSITRON) stat_add(st, S_POSESC);
  if (!a.test_mode) return;
  const uint64_t h = p.hist - a.cnt->run_first;
  unsafeAtomicAdd(&a.hist_led[3 * h + 1], ew);
  if (p.type == POSITRON) unsafeAtomicAdd(&a.hist_led[3 * h + 2], a.vr ? p.w : 1.0);
}

// ---------------------------------------------------------------------------
// geometry: constant LOCATE / STEP on the voxel grid
// ---------------------------------------------------------------------------
// distance to the exit face of the current voxel; ties go to x, then y, z
template <typename T>
__device__ __forceinline__ double face_dist(const KArgs<T>& a, const Part<T>& p, int* axis) {
  const double o[3] = {a.ox, a.oy, a.oz};
  const double dd[3] = {a.dx, a.dy, a.dz};
  double best = __builtin_huge_val();
  int ax = -1;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T dk = p.d[k];
    if (dk == T(0)) continue;
    const double face = dk > T(0) ? o[k] + double(p.ix[k] + 1) * dd[k] : o[k] + double(p.ix[k]) * dd[k];
    // FP64 path: exact FP64 division; mixed path: the FP64 offset to the face
    // (a few millimetres at most) divided in FP32
    double s = is_fp64<T>() ? (face - p.x[k]) / double(dk) : double(T(face - p.x[k]) / dk);
    if (s < 0.0) s = 0.0;
    if (s < best) { best = s; ax = k; }
  }
  *axis = ax;
  return best;
}

template <typename T>
__device__ __forceinline__ void move(Part<T>& p, double s) {
#pragma unroll
  for (int k = 0; k < 3; ++k) p.x[k] = p.x[k] + s * double(p.d[k]);
}

// move to the face on `ax`, snap onto it and step the voxel index;
// true if the particle left the grid
template <typename T>
__device__ __forceinline__ bool cross(const KArgs<T>& a, Part<T>& p, double s, int ax, LaneStats& ls) {
  const double o[3] = {a.ox, a.oy, a.oz};
  const double dd[3] = {a.dx, a.dy, a.dz};
  const int n[3] = {a.nx, a.ny, a.nz};
  move(p, s);
  bool out = false;
  // unrolled so that every array index is a constant (no scratch memory)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k == ax) {
      const bool up = p.d[k] > T(0);
      p.x[k] = up ? o[k] + double(p.ix[k] + 1) * dd[k] : o[k] + double(p.ix[k]) * dd[k];
      p.ix[k] += up ? 1 : -1;
      out = p.ix[k] < 0 || p.ix[k] >= n[k];
    }
  }
  ls.crossings++;
  return out;
}

// polar deflection by cos_t and azimuth phi, then renormalise
template <typename T>
__device__ __forceinline__ void rotate(T d[3], T cost, T phi) {
  const T s2t = T(1) - cost * cost;
  const T sint = s2t > T(0) ? M<T>::sqrt(s2t) : T(0);
  T sp, cp;
  M<T>::sincos(phi, &sp, &cp);
  const T u = d[0], v = d[1], w = d[2];
  const T s2 = T(1) - w * w;
  T nu, nv, nw;
  if (s2 > T(1e-10)) {
    const T s = M<T>::sqrt(s2);
    nu = u * cost + sint * (u * w * cp - v * sp) / s;
    nv = v * cost + sint * (v * w * cp + u * sp) / s;
    nw = w * cost - s * sint * cp;
  } else {
    nu = sint * cp;
    nv = sint * sp;
    nw = w > T(0) ? cost : -cost;
  }
  const T nn = M<T>::sqrt(nu * nu + nv * nv + nw * nw);
  d[0] = nu / nn;
  d[1] = nv / nn;
  d[2] = nw / nn;
}

// ---------------------------------------------------------------------------
// table interpolation (tables in LDS, channel-major)
// ---------------------------------------------------------------------------
template <typename T>
struct Grid {
  int i;
  T f;
};

template <typename T>
__device__ __forceinline__ Grid<T> grid_at(const Tab<T>& tb, T le) {
  const T x = (le - tb.lemin) * tb.inv_dl;
  const T fl = M<T>::floor(x);
  int i;
  if (!(fl >= T(0))) i = 0;  // also catches NaN
  else if (fl > T(tb.n - 2)) i = tb.n - 2;
  else i = int(fl);
  return Grid<T>{i, x - T(i)};
}

// piecewise power law between positive nodes; linear in E from the
// threshold on a segment whose lower node is zero
template <typename T>
__device__ __forceinline__ T interp(const T* s, int n, int ch, const Grid<T>& g, T e, T thr) {
  if (thr > T(0) && !(e > thr)) return T(0);
  const T l0 = s[ch * n + g.i], l1 = s[ch * n + g.i + 1];
  if (!(l1 > -M<T>::inf())) return T(0);
  if (!(l0 > -M<T>::inf())) {
    const T ei = s[T_ENODE * n + g.i], ej = s[T_ENODE * n + g.i + 1];
    const T lo = thr > ei ? thr : ei;
    return M<T>::exp(l1) * (e - lo) / (ej - lo);
  }
  return M<T>::exp(l0 + g.f * (l1 - l0));
}

// range R(E): R_i + Int_{E_i}^{E} dE/S on the power-law segment; `le` is ln E
template <typename T>
__device__ __forceinline__ T range_at(const T* s, int n, int base, const Grid<T>& g, T e, T le, T lemin, T dl) {
  const T ei = s[T_ENODE * n + g.i];
  const T si = s[(base + O_S) * n + g.i];
  const T q = s[(base + O_Q) * n + g.i];
  const T ri = s[(base + O_R) * n + g.i];
  // (E_i/S_i) ((E/E_i)^q - 1)/q, written with expm1 of q ln(E/E_i): no
  // power function and no cancellation near the node
  const T lr = le - (lemin + T(g.i) * dl);  // ln(E/E_i)
  const T seg = (ei / si) * ((q > T(-1e-10) && q < T(1e-10)) ? lr : M<T>::expm1(q * lr) / q);
  return ri + seg;
}

// inverse range: the energy whose range is r (E_min if r <= 0).  The segment
// i with R_i <= r < R_{i+1} is found by walking from the node `hint` (the
// node of the energy before the loss, which lies at most a few nodes away)
template <typename T>
__device__ __forceinline__ T range_inv(const T* s, int n, int base, T r, int hint) {
  if (!(r > T(0))) return s[T_ENODE * n];
  const T* rr = s + (base + O_R) * n;
  int lo = hint < 0 ? 0 : (hint > n - 2 ? n - 2 : hint);
  while (lo > 0 && rr[lo] > r) --lo;
  while (lo < n - 2 && rr[lo + 1] <= r) ++lo;
  const T ei = s[T_ENODE * n + lo];
  const T si = s[(base + O_S) * n + lo];
  const T q = s[(base + O_Q) * n + lo];
  const T d = r - rr[lo];
  // E_i (1 + d q S_i/E_i)^(1/q), as exp(log1p(.)/q)
  if (q > T(-1e-10) && q < T(1e-10)) return ei * M<T>::exp(d * si / ei);
  return ei * M<T>::exp(M<T>::log1p(d * q * si / ei) / q);
}

template <typename T>
__device__ __forceinline__ T hard_sum(const Tab<T>& tb, const T* s, int base, int lep, const Grid<T>& g, T e) {
  const int n = tb.n;
  return interp(s, n, base + O_LEL, g, e, T(0)) + interp(s, n, base + O_LIN, g, e, tb.thr_in[lep]) +
         interp(s, n, base + O_LBR, g, e, tb.thr_br);
}

// upper bound of the hard cross section at e: on a segment without a
// channel threshold, exp of the log-log chord of the node sums (ln of a sum
// of power laws is convex in ln E and lies below its chord); elsewhere the
// sum of the channels
template <typename T>
__device__ __forceinline__ T hard_bound(const Tab<T>& tb, const T* s, int base, int lep, const Grid<T>& g, T e) {
  const int n = tb.n;
  const T l0 = s[(base + O_LHC) * n + g.i];
  if (l0 > -M<T>::inf()) return M<T>::exp(l0 + g.f * (s[(base + O_LH) * n + g.i + 1] - l0));
  return hard_sum(tb, s, base, lep, g, e);
}

// majorant over [elo, e]: the bound above is monotone on each segment (or
// convex in ln E on a threshold segment, as every channel is), so its
// maximum sits at elo, e or a node between
template <typename T>
__device__ __forceinline__ T majorant(const Tab<T>& tb, const T* s, int base, int lep, T elo, const Grid<T>& ge,
                                      T e) {
  const int n = tb.n;
  T m = hard_bound(tb, s, base, lep, ge, e);
  const Grid<T> gl = grid_at(tb, M<T>::log(elo));
  const T a = hard_bound(tb, s, base, lep, gl, elo);
  if (a > m) m = a;
  for (int j = gl.i; j <= ge.i + 1 && j < n; ++j) {
    const T ej = s[T_ENODE * n + j];
    if (ej > elo && ej < e) {
      const T v = s[(base + O_HSUM) * n + j];
      if (v > m) m = v;
    }
  }
  return m;
}

// A of the soft angular law p(mu) ~ (mu + A)^-2 on [0,1] whose mean
// A (1 + A) ln(1 + 1/A) - A equals mbar (clamped to 0.49).  Start from the
// tabulated ln A (linear in y = ln(mbar / (1/2 - mbar)), within 6e-6 of the
// root on 1024 nodes) or, below the table, from the small-A expansion
// A (ln(1/A) - 1) = mbar; then Newton steps on ln A: none in FP32, one in
// FP64 (quadratic convergence: relative error below 6e-12).
template <typename T>
__device__ __forceinline__ T soft_a(T mbar, const T* soft) {
  if (!(mbar > T(0))) return T(0);
  if (mbar > T(kSoftMHi)) mbar = T(kSoftMHi);
  T s;
  if (mbar < T(kSoftMLo)) {
    const T lm = M<T>::log(mbar);
    const T a0 = mbar / (-lm);
    s = M<T>::log(mbar / (-M<T>::log(a0) - T(1)));
  } else {
    const T y0 = T(-20.030118654386467);  // y(1e-9)
    const T inv_dy = T(double(kSoftN - 1) / (3.8918202981106256 + 20.030118654386467));  // y(0.49) = 3.89...
    const T x = (M<T>::log(mbar / (T(0.5) - mbar)) - y0) * inv_dy;
    int j = int(x);
    j = j < 0 ? 0 : (j > kSoftN - 2 ? kSoftN - 2 : j);
    const T f = x - T(j);
    s = soft[j] + f * (soft[j + 1] - soft[j]);
  }
  const int steps = is_fp64<T>() ? 1 : 0;
  for (int it = 0; it < steps; ++it) {
    const T A = M<T>::exp(s);
    const T L = M<T>::log1p(T(1) / A);
    const T g = A * ((T(1) + A) * L - T(1)) - mbar;
    const T dg = A * ((T(1) + T(2) * A) * L - T(2));  // d g / d ln A
    if (dg > T(0)) s -= g / dg;
  }
  return M<T>::exp(s);
}

// cos theta from p(cos) ~ (1 - beta cos)^-2 on [-1, 1] by inversion
template <typename T>
__device__ __forceinline__ T leading_angle(T beta, T xi) {
  return (T(2) * xi - T(1) + beta) / (T(2) * beta * xi + T(1) - beta);
}

template <typename T>
__device__ __forceinline__ T beta_of(T t) {
  return M<T>::sqrt(t * (t + T(2) * T(kMc2))) / (t + T(kMc2));
}

// ---------------------------------------------------------------------------
// LDS staging of table channels [c0, c1)
// ---------------------------------------------------------------------------
// channels [0, c1) of the table block into LDS, plus `extra` values after them
template <typename T>
__device__ __forceinline__ void stage(const Tab<T>& tb, T* lds, int c1, int extra = 0) {
  const int total = c1 * tb.n + extra;
  for (int k = threadIdx.x; k < total; k += blockDim.x) lds[k] = tb.t[k];
}

}  // namespace mcx
