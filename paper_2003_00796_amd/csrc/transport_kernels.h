// transport_kernels.h -- the kernels of one iteration of the event loop and
// of the tally, templated on the compute type.  Included by exactly one
// translation unit per precision (kernels_fp64.hip, kernels_mixed.hip), which
// are compiled with different floating-point contraction settings.
#pragma once

#include "launch.h"
#include "transport_device.h"

// minimum waves per SIMD the e+- step kernel is compiled for (bounds its
// registers); 1 lets the compiler use as many registers as it wants
#ifndef MCX_ESTEP_WAVES
#define MCX_ESTEP_WAVES 1
#endif
// photons waiting for an interaction at or below which the interaction
// kernel follows each photon to its end (see k_knock)
#ifndef MCX_CHAIN_PHOTONS
#define MCX_CHAIN_PHOTONS 131072
#endif
#ifndef MCX_CHAIN_DIV
#define MCX_CHAIN_DIV 8
#endif
// the interaction kernel, with the photon flight inlined for the chains,
// needs about 250 registers in FP64: bound it to 2 waves per SIMD
#ifndef MCX_KNOCK_WAVES
#define MCX_KNOCK_WAVES 2
#endif
// tail of the e+- kernel: once the input queue is empty, a wavefront keeps
// stepping its particles for at least MCX_TAIL_MIN more steps, then writes
// them all back as soon as fewer than MCX_TAIL_ALIVE of its lanes hold one
// (64: as soon as one lane is idle)
#ifndef MCX_TAIL_MIN
#define MCX_TAIL_MIN 16
#endif
#ifndef MCX_TAIL_ALIVE
#define MCX_TAIL_ALIVE 64
#endif

namespace mcx {

// queue roles of an iteration with parity `par`
__device__ __forceinline__ int q_gin(int par) { return Q_G0 + par; }
__device__ __forceinline__ int q_gout(int par) { return Q_G0 + 1 - par; }
__device__ __forceinline__ int q_ein(int par) { return Q_E0 + par; }
__device__ __forceinline__ int q_eout(int par) { return Q_E0 + 1 - par; }

// Kernel flavours: the transport kernels are compiled once per flavour, and
// each tells the compiler the values of the run-time switches of its
// argument block (the host launches the flavour that matches them), so the
// forward kernels carry no test-output or replay code (nor its registers).
enum Flavor : int {
  FL_FWD = 0,         // forward transport
  FL_TEST = 1,        // forward transport with the per-history test outputs
  FL_ADJ_A = 2,       // first density-gradient replay (per-history weighted score)
  FL_ADJ_B = 3,       // second replay (likelihood-ratio scores of photon flights)
  FL_EXT = 4,         // forward transport with the optional physics: soft energy-loss
                      // straggling, positron annihilation in flight (run-time switches)
  FL_EXT_TEST = 5,    // the same with the per-history test outputs
  FL_MM = 6,          // several materials (per-voxel index), with the optional physics
  FL_MM_TEST = 7,     // the same with the per-history test outputs
  FL_VR = 8,          // interaction forcing: weighted particles, with the optional physics
  FL_VR_TEST = 9,     // the same with the per-history test outputs
  FL_MM_ADJ_A = 10,   // the density-gradient replays on several-material phantoms
  FL_MM_ADJ_B = 11,
  FL_VR_ADJ_A = 12,   // the density-gradient replays with weighted particles
  FL_VR_ADJ_B = 13,
  FL_EXT_ADJ_A = 14,  // the density-gradient replays with annihilation in flight
  FL_EXT_ADJ_B = 15,
  FL_MMVR = 16,       // several materials and weighted particles, with the optional physics
  FL_MMVR_TEST = 17,  // the same with the per-history test outputs
  FL_MMVR_ADJ_A = 18, // the density-gradient replays on several materials with weights
  FL_MMVR_ADJ_B = 19
};
constexpr int kFlavors = 20;

// the optional physics changes the e+- step only: the other kernels of an
// extended flavour are those of the flavour without it; several materials
// change the photon flight and interactions too
constexpr int base_flavor(int f) {
  return (f == FL_EXT || f == FL_MM || f == FL_VR || f == FL_MMVR)
             ? FL_FWD
             : ((f == FL_EXT_TEST || f == FL_MM_TEST || f == FL_VR_TEST || f == FL_MMVR_TEST)
                    ? FL_TEST
                    : ((f == FL_MM_ADJ_A || f == FL_VR_ADJ_A || f == FL_EXT_ADJ_A || f == FL_MMVR_ADJ_A)
                           ? FL_ADJ_A
                           : ((f == FL_MM_ADJ_B || f == FL_VR_ADJ_B || f == FL_EXT_ADJ_B || f == FL_MMVR_ADJ_B)
                                  ? FL_ADJ_B
                                  : f)));
}
constexpr bool extended(int f) { return f >= FL_EXT; }
constexpr bool several(int f) {
  return f == FL_MM || f == FL_MM_TEST || f == FL_MM_ADJ_A || f == FL_MM_ADJ_B || f >= FL_MMVR;
}
// weighted particles: every kernel carries the weights
constexpr bool weighted(int f) {
  return f == FL_VR || f == FL_VR_TEST || f == FL_VR_ADJ_A || f == FL_VR_ADJ_B || f >= FL_MMVR;
}
constexpr int photon_flavor(int f) { return several(f) || weighted(f) ? f : base_flavor(f); }
constexpr int source_flavor(int f) { return weighted(f) ? f : base_flavor(f); }

// constants of material m (selects over the kMaxMat entries: no indexing of
// the argument block by a run-time value)
template <typename T>
__device__ __forceinline__ MatConst<T> mat_const(const Tab<T>& tb, uint32_t m) {
  return m == 0u ? tb.mc[0] : (m == 1u ? tb.mc[1] : (m == 2u ? tb.mc[2] : tb.mc[3]));
}

// the table constants of material m (several-material kernels)
template <typename T>
__device__ __forceinline__ Tab<T> mat_tab(const Tab<T>& tb, uint32_t m) {
  const MatConst<T> mc = mat_const(tb, m);
  Tab<T> t = tb;
  t.k_coef = mc.k_coef;
  t.eta_a = mc.eta_a;
  t.eta_b = mc.eta_b;
  t.strag_k = mc.strag_k;
  t.strag_b = mc.strag_b;
  t.annih_k = mc.annih_k;
  return t;
}

template <int F, typename T>
__device__ __forceinline__ void set_flavor(const KArgs<T>& a) {
  constexpr int B = base_flavor(F);
  __builtin_assume(a.test_mode == (B == FL_TEST ? 1 : 0));
  __builtin_assume(a.mode == (B == FL_ADJ_A ? 1 : (B == FL_ADJ_B ? 2 : 0)));
  constexpr int W = weighted(F) ? 1 : 0;
  __builtin_assume(a.vr == W);
}

// striped queues: this block's stripe, the records of a stripe, the prefix
// sums of the stripe occupancies (wave-uniform) and the record of the i-th
// queued particle
__device__ __forceinline__ uint32_t my_stripe() { return blockIdx.x & uint32_t(kStripes - 1); }

template <typename T>
__device__ __forceinline__ uint32_t stripe_cap(const KArgs<T>& a) {
  return a.cap / uint32_t(kStripes);
}

struct StripeSums {
  uint32_t pre[kStripes + 1];
};

__device__ __forceinline__ StripeSums stripe_sums(const Counters* c, int q, uint32_t cs) {
  StripeSums t;
  t.pre[0] = 0u;
#pragma unroll
  for (int k = 0; k < kStripes; ++k) t.pre[k + 1] = t.pre[k] + min(c->ns[q][k].v, cs);
  return t;
}

__device__ __forceinline__ uint32_t striped_record(const StripeSums& t, uint32_t i, uint32_t cs) {
  uint32_t s = 0u, base = 0u;
#pragma unroll
  for (int k = 1; k < kStripes; ++k) {
    const bool in = i >= t.pre[k];
    s = in ? uint32_t(k) : s;
    base = in ? t.pre[k] : base;
  }
  return s * cs + (i - base);
}

// wavefront-aggregated append; returns the record index, ~0u on overflow
template <typename T>
__device__ __forceinline__ uint32_t append(const KArgs<T>& a, int q, bool pred) {
  const bool striped = q < kStripedQueues;
  const uint32_t st = my_stripe();
  const uint32_t cap = striped ? stripe_cap(a) : a.cap;
  const uint32_t slot = wave_append(striped ? &a.cnt->ns[q][st].v : &a.cnt->n[q].v, pred);
  if (pred && slot >= cap) {
    atomicOr(&a.cnt->overflow, uint32_t(OVF_QUEUE));
    return ~0u;
  }
  return striped ? st * cap + slot : slot;
}

// ---------------------------------------------------------------------------
// source: primaries for history ids [cursor, cursor + adm)
// ---------------------------------------------------------------------------
template <typename T, int F>
__global__ __launch_bounds__(kMaxBlock) void k_source(KArgs<T> a, int par) {
  set_flavor<F>(a);
  const uint32_t adm = a.cnt->adm;
  const uint64_t first = a.cnt->cursor;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < adm; base += stride) {
    const uint32_t i = base + threadIdx.x;
    const bool act = i < adm;
    Part<T> p;
    bool ok = false;
    if (act) {
      const uint64_t h = first + i;
      int lo = 0, hi = a.nsrc - 1;  // first source whose end exceeds h
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.src[mid].end > h) hi = mid;
        else lo = mid + 1;
      }
      const SourceDev& s = a.src[lo];
      p.type = uint32_t(s.particle);
      p.e = T(s.energy);
      p.hist = uint32_t(h);
      p.uid = 1ull;
      p.nchild = 0u;
      p.hash = 0ull;
      p.w = 1.0;
      p.clk = T(0);
      rng_init(p.rng, a.seed, p.hist, 1ull, 0u);
      p.x[0] = s.pos[0]; p.x[1] = s.pos[1]; p.x[2] = s.pos[2];
      p.d[0] = T(s.dir[0]); p.d[1] = T(s.dir[1]); p.d[2] = T(s.dir[2]);
      if (s.kind == 1) {
        // rectangle: both offsets use the FP64 words of draws 0 and 1 so that
        // the start point is the same in both precisions
        uint32_t o[4];
        philox10(0u, 1u, 0u, 0u, a.seed, p.hist, o);
        uint64_t w0, w1;
        pair_words(o, &w0, &w1);
        const double ux = (double(w0 >> 11) + 0.5) * 0x1.0p-53;
        const double uy = (double(w1 >> 11) + 0.5) * 0x1.0p-53;
        p.rng.ctr = 2u;
        p.x[0] = s.pos[0] + (ux - 0.5) * s.width[0];
        p.x[1] = s.pos[1] + (uy - 0.5) * s.width[1];
      }
      const double o[3] = {a.ox, a.oy, a.oz};
      const double dd[3] = {a.dx, a.dy, a.dz};
      const int n[3] = {a.nx, a.ny, a.nz};
      ok = true;
      for (int k = 0; k < 3; ++k) {
        const double f = floor((p.x[k] - o[k]) / dd[k]);
        if (!(f >= 0.0) || !(f < double(n[k]))) ok = false;
        else p.ix[k] = int(f);
      }
      if (!ok) atomicOr(&a.cnt->overflow, uint32_t(OVF_SOURCE));
    }
    const bool is_g = ok && p.type == PHOTON;
    const bool is_e = ok && p.type != PHOTON;
    const uint32_t sg = append(a, q_gin(par), is_g);
    const uint32_t se = append(a, q_ein(par), is_e);
    if (is_g && sg != ~0u) store_part(a, a.q[q_gin(par)], sg, p);
    if (is_e && se != ~0u) store_part(a, a.q[q_ein(par)], se, p);
  }
}

// ---------------------------------------------------------------------------
// photon JUMP + STEP: free path in mass thickness, DDA through the voxels;
// escaped photons end here, the others are sorted by interaction type
// ---------------------------------------------------------------------------
// voxels the photon walk computes ahead of the mass-thickness sum
#ifndef MCX_WALK
#define MCX_WALK 2
#endif
constexpr int kWalk = MCX_WALK;

// Same-density cubes.  cube[v] is the largest r <= kCubeMax such that every
// voxel within Chebyshev distance r of v lies in the grid and has v's density:
// the L-infinity distance from v to the nearest boundary voxel (one with a
// face, edge or corner neighbour of another density or outside the grid).
// Inside such a cube the mass thickness along a ray is the density times the
// length, so the walk crosses the cube's inner faces in one step.
#ifndef MCX_CUBE_MAX
#define MCX_CUBE_MAX 31
#endif
constexpr int kCubeMax = MCX_CUBE_MAX;  // stored in a byte
static_assert(kCubeMax >= 1 && kCubeMax <= 255, "cube half-width must fit a byte");
// smallest half-width for which the walk takes the one-step crossing
#ifndef MCX_CUBE_MIN
#define MCX_CUBE_MIN 1
#endif
constexpr uint32_t kCubeMin = MCX_CUBE_MIN;

template <typename T>
__global__ void k_cube_seed(const T* rho, const uint8_t* mat, int nx, int ny, int nz, uint8_t* out) {
  const uint64_t nv = uint64_t(nx) * ny * nz;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nv; v += stride) {
    const int x = int(v % uint64_t(nx)), y = int((v / uint64_t(nx)) % uint64_t(ny)), z = int(v / (uint64_t(nx) * ny));
    bool edge = x == 0 || y == 0 || z == 0 || x == nx - 1 || y == ny - 1 || z == nz - 1;
    const T r0 = rho[v];
    for (int dz = -1; dz <= 1 && !edge; ++dz)
      for (int dy = -1; dy <= 1 && !edge; ++dy)
        for (int dx = -1; dx <= 1 && !edge; ++dx)
          edge = rho[(uint64_t(z + dz) * ny + uint64_t(y + dy)) * nx + uint64_t(x + dx)] != r0 ||
                 (mat && mat[(uint64_t(z + dz) * ny + uint64_t(y + dy)) * nx + uint64_t(x + dx)] != mat[v]);
    out[v] = edge ? uint8_t(0) : uint8_t(kCubeMax);
  }
}

// one separable pass of the L-infinity distance along axis ax:
// out[v] = min over |d| <= kCubeMax of max(|d|, in[v + d e_ax])
template <typename T>
__global__ void k_cube_pass(const uint8_t* in, uint8_t* out, int nx, int ny, int nz, int ax) {
  const uint64_t nv = uint64_t(nx) * ny * nz;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const int n = ax == 0 ? nx : (ax == 1 ? ny : nz);
  const uint64_t step = ax == 0 ? 1ull : (ax == 1 ? uint64_t(nx) : uint64_t(nx) * ny);
  for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nv; v += stride) {
    const int c = int((v / step) % uint64_t(n));
    int best = in[v];
    for (int d = 1; d < best; ++d) {  // a term at offset d is at least d
      if (c - d >= 0) best = min(best, max(d, int(in[v - uint64_t(d) * step])));
      if (c + d < n) best = min(best, max(d, int(in[v + uint64_t(d) * step])));
    }
    out[v] = uint8_t(best);
  }
}

#ifndef MCX_FLIGHT_WAVES
#define MCX_FLIGHT_WAVES 1
#endif
// One photon flight (JUMP and STEP through the voxels): from the photon's
// position to its next interaction, whose channel it returns (0 Compton,
// 1 photoabsorption, 2 Rayleigh, 3 pair production), or out of the phantom
// (-1: the escape is recorded and the photon's history record finished).  In
// the second gradient replay it also scores the flight's density derivatives.
// `tab` holds the photon channels in LDS (of every material with several).
template <typename T, int F>
__device__ __forceinline__ int photon_flight(const KArgs<T>& a, const T* tab, Part<T>& p, LaneStats& ls,
                                             BlockStats* bs) {
  constexpr bool MMF = several(F);
  const int nt = a.tb.n;
  int ch = -1;
  const T e = p.e;
  const Grid<T> g = grid_at(a.tb, M<T>::log(e));
  T mu[4];
  T mt = T(0);
  // several materials: the attenuation rho mu_m(E) of each voxel's
  // material; the flight is measured in optical depth
  T mtm[kMaxMat];
  if constexpr (MMF) {
#pragma unroll
    for (int m = 0; m < kMaxMat; ++m) {
      const T* tm = tab + m * T_PHOTON_END * nt;
      mtm[m] = m < a.tb.nmat ? interp(tm, nt, T_LMU_C, g, e, T(0)) + interp(tm, nt, T_LMU_PE, g, e, T(0)) +
                                   interp(tm, nt, T_LMU_R, g, e, T(0)) +
                                   interp(tm, nt, T_LMU_PP, g, e, a.tb.thr_pp)
                             : T(0);
    }
  } else {
    mu[0] = interp(tab, nt, T_LMU_C, g, e, T(0));
    mu[1] = interp(tab, nt, T_LMU_PE, g, e, T(0));
    mu[2] = interp(tab, nt, T_LMU_R, g, e, T(0));
    mu[3] = interp(tab, nt, T_LMU_PP, g, e, a.tb.thr_pp);
    mt = mu[0] + mu[1] + mu[2] + mu[3];
  }
  // replay B: mu of voxel vv's material (several materials), else mu
  auto mu_of = [&](uint32_t vv) -> double {
    if constexpr (MMF) {
      const uint32_t m = a.mat[vv];
      return double(m == 0u ? mtm[0] : (m == 1u ? mtm[1] : (m == 2u ? mtm[2] : mtm[3])));
    } else {
      return double(mt);
    }
  };
  auto att = [&](uint32_t vv) -> double {
    if constexpr (MMF) {
      const uint32_t m = a.mat[vv];
      const T mm = m == 0u ? mtm[0] : (m == 1u ? mtm[1] : (m == 2u ? mtm[2] : mtm[3]));
      return double(a.rho[vv]) * double(mm);
    } else {
      return double(a.rho[vv]);
    }
  };
  ls.flights++;
  double tau = MMF ? double(-M<T>::log(uni<T>(p.rng))) : double(-M<T>::log(uni<T>(p.rng)) / mt);
  // incremental DDA: tn[k] = distance along the ray to the next face
  // normal to axis k, advanced by the voxel pitch over |d_k| per crossing
  const double o[3] = {a.ox, a.oy, a.oz};
  const double dd[3] = {a.dx, a.dy, a.dz};
  const int nn[3] = {a.nx, a.ny, a.nz};
  double tn[3], dt[3];
  int stp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double dk = double(p.d[k]);
    if (dk > 0.0) {
      stp[k] = 1;
      tn[k] = (o[k] + double(p.ix[k] + 1) * dd[k] - p.x[k]) / dk;
      dt[k] = dd[k] / dk;
    } else if (dk < 0.0) {
      stp[k] = -1;
      tn[k] = (o[k] + double(p.ix[k]) * dd[k] - p.x[k]) / dk;
      dt[k] = -dd[k] / dk;
    } else {
      stp[k] = 0;
      tn[k] = __builtin_huge_val();
      dt[k] = 0.0;
    }
    if (tn[k] < 0.0) tn[k] = 0.0;
  }
  if (!(tn[0] < __builtin_huge_val()) && !(tn[1] < __builtin_huge_val()) &&
      !(tn[2] < __builtin_huge_val())) {
    atomicOr(&a.cnt->overflow, uint32_t(OVF_LOST));
    tau = 0.0;
  }
  double t = 0.0;
  bool escaped = false;
  uint32_t v = vlin(a, p.ix);
  double t0 = tn[0], t1 = tn[1], t2 = tn[2];
  // faces per unit length along each axis (|d_k| / pitch), for counting
  // the faces a cube crossing passes
  const double it[3] = {fabs(double(p.d[0])) * a.idx, fabs(double(p.d[1])) * a.idy, fabs(double(p.d[2])) * a.idz};
  double rho_v = att(v);
  uint32_t cube_v = a.cube[v];
  // replay B: the history's centred weighted score times d ln p / d rho_j
  // of this free flight (-mu l_j per voxel, +1/rho at the interaction)
  const double cq = a.mode == 2 ? a.adj_q[p.hist - a.cnt->run_first] - a.adj_qbar : 0.0;
  const double mud = double(mt);
  // The walk runs kWalk voxels ahead of the mass-thickness sum: the
  // geometry of the next kWalk segments needs no density, so their
  // densities are requested together and their latencies overlap.
  bool ended = false;
  uint32_t esc_v = v;
  while (!ended) {
    if (cube_v >= kCubeMin) {
      // one step to the first of: the interaction, were the cube's density
      // to continue, and the cube's boundary; it crosses every face strictly
      // before that point (at most cube_v per axis, all inside the cube) and
      // leaves the decision at the point to the walk below
      const double r = double(cube_v);
      const double te = fmin(fmin(t0 + r * dt[0], t1 + r * dt[1]), t2 + r * dt[2]);
      const double tt = fmin(te, t + tau / rho_v);
      const int lim = int(cube_v);
      const int n0 = tt > t0 ? min(lim, int(ceil((tt - t0) * it[0]))) : 0;
      const int n1 = tt > t1 ? min(lim, int(ceil((tt - t1) * it[1]))) : 0;
      const int n2 = tt > t2 ? min(lim, int(ceil((tt - t2) * it[2]))) : 0;
      if (n0 + n1 + n2 > 0) {
        double tl = t;  // the last face crossed
        if (n0 > 0) tl = fmax(tl, t0 + double(n0 - 1) * dt[0]);
        if (n1 > 0) tl = fmax(tl, t1 + double(n1 - 1) * dt[1]);
        if (n2 > 0) tl = fmax(tl, t2 + double(n2 - 1) * dt[2]);
        if (cq != 0.0) {
          // replay B: the same faces one by one, for each voxel's length
          double u0 = t0, u1 = t1, u2 = t2, tc = t;
          int m0 = n0, m1 = n1, m2 = n2;
          int jx[3] = {p.ix[0], p.ix[1], p.ix[2]};
          for (int left = n0 + n1 + n2; left > 0; --left) {
            // next face among the axes with faces left; ties in x, y, z order
            const bool a0 = m0 > 0 && (m1 <= 0 || u0 <= u1) && (m2 <= 0 || u0 <= u2);
            const bool a1 = !a0 && m1 > 0 && (m2 <= 0 || u1 <= u2);
            const bool a2 = !a0 && !a1;
            const double uk = a0 ? u0 : (a1 ? u1 : u2);
            unsafeAtomicAdd(&a.adj_grad[vlin(a, jx)], cq * (-(MMF ? mu_of(v) : mud) * (uk - tc)));
            tc = uk;
            u0 = a0 ? u0 + dt[0] : u0;
            u1 = a1 ? u1 + dt[1] : u1;
            u2 = a2 ? u2 + dt[2] : u2;
            jx[0] += a0 ? stp[0] : 0;
            jx[1] += a1 ? stp[1] : 0;
            jx[2] += a2 ? stp[2] : 0;
            m0 -= a0 ? 1 : 0;
            m1 -= a1 ? 1 : 0;
            m2 -= a2 ? 1 : 0;
          }
        }
        tau = fmax(tau - rho_v * (tl - t), 0.0);
        t = tl;
        p.ix[0] += stp[0] * n0;
        p.ix[1] += stp[1] * n1;
        p.ix[2] += stp[2] * n2;
        t0 += double(n0) * dt[0];
        t1 += double(n1) * dt[1];
        t2 += double(n2) * dt[2];
        ls.crossings += uint32_t(n0 + n1 + n2);
        v = vlin(a, p.ix);
      }
    }
    // branch-free: the lanes of a wavefront walk different axes
    double seg[kWalk], tend[kWalk];
    uint32_t vs[kWalk + 1];
    int axs[kWalk];
    bool outs[kWalk];
    {
      double u0 = t0, u1 = t1, u2 = t2, tc = t;
      int j0 = p.ix[0], j1 = p.ix[1], j2 = p.ix[2];
      uint32_t vc = v;
      bool gone = false;  // an earlier segment of this batch leaves the phantom
#pragma unroll
      for (int j = 0; j < kWalk; ++j) {
        const bool a0 = (u0 <= u1) & (u0 <= u2);
        const bool a1 = !a0 & (u1 <= u2);
        const bool a2 = !a0 & !a1;
        const double tf = a0 ? u0 : (a1 ? u1 : u2);
        seg[j] = tf - tc;
        tend[j] = tf;
        vs[j] = vc;
        axs[j] = a0 ? 0 : (a1 ? 1 : 2);
        j0 += a0 ? stp[0] : 0;
        j1 += a1 ? stp[1] : 0;
        j2 += a2 ? stp[2] : 0;
        u0 = a0 ? u0 + dt[0] : u0;
        u1 = a1 ? u1 + dt[1] : u1;
        u2 = a2 ? u2 + dt[2] : u2;
        const bool out = (j0 < 0) | (j0 >= nn[0]) | (j1 < 0) | (j1 >= nn[1]) | (j2 < 0) | (j2 >= nn[2]);
        outs[j] = out;
        gone = gone | out;
        const int jx[3] = {j0, j1, j2};
        vc = gone ? vc : vlin(a, jx);
        tc = tf;
      }
      vs[kWalk] = vc;
    }
    double rr[kWalk];
#pragma unroll
    for (int j = 0; j < kWalk; ++j) rr[j] = att(vs[j]);
    // the voxel after the last segment: where the next pass starts
    const double rho_n = att(vs[kWalk]);
    const uint32_t cube_n = a.cube[vs[kWalk]];
#pragma unroll
    for (int j = 0; j < kWalk; ++j) {
      const double rho = rr[j], sj = seg[j];
      const bool act = !ended;
      const bool hit = act & (rho * sj >= tau);
      const bool pass = act & !hit;
      if (cq != 0.0 && act) {
        // several materials: rho here is rho mu_m, tau an optical depth
        const double muj = MMF ? mu_of(vs[j]) : mud;
        const double rj = MMF ? double(a.rho[vs[j]]) : rho;
        unsafeAtomicAdd(&a.adj_grad[vs[j]], hit ? cq * (-muj * (tau / rho) + 1.0 / rj) : cq * (-muj * sj));
      }
      t = hit ? t + tau / rho : (pass ? tend[j] : t);
      tau = pass ? tau - rho * sj : tau;
      p.ix[0] += (pass & (axs[j] == 0)) ? stp[0] : 0;
      p.ix[1] += (pass & (axs[j] == 1)) ? stp[1] : 0;
      p.ix[2] += (pass & (axs[j] == 2)) ? stp[2] : 0;
      t0 = (pass & (axs[j] == 0)) ? t0 + dt[0] : t0;
      t1 = (pass & (axs[j] == 1)) ? t1 + dt[1] : t1;
      t2 = (pass & (axs[j] == 2)) ? t2 + dt[2] : t2;
      ls.crossings += pass ? 1u : 0u;
      const bool esc = pass & outs[j];
      esc_v = esc ? vs[j] : esc_v;
      escaped = escaped | esc;
      v = (pass & !outs[j]) ? vs[j + 1] : v;
      ended = ended | hit | esc;
    }
    rho_v = rho_n;
    cube_v = cube_n;
  }
  if (escaped) {
    ledger_escape(a, bs, p);
    event(a, p, EV_PH_ESCAPE, esc_v);
    finish(a, p);
  }
  move(p, t);
  if (!escaped) {
    if constexpr (MMF) {
      // the interaction by the tables of the voxel the photon stops in
      const T* tm = tab + int(a.mat[v]) * T_PHOTON_END * nt;
      mu[0] = interp(tm, nt, T_LMU_C, g, e, T(0));
      mu[1] = interp(tm, nt, T_LMU_PE, g, e, T(0));
      mu[2] = interp(tm, nt, T_LMU_R, g, e, T(0));
      mu[3] = interp(tm, nt, T_LMU_PP, g, e, a.tb.thr_pp);
      mt = mu[0] + mu[1] + mu[2] + mu[3];
    }
    const T u = uni<T>(p.rng) * mt;
    T cum = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cum += mu[k];
      if (ch < 0 && u < cum) ch = k;
    }
    if (ch < 0) {
#pragma unroll
      for (int k = 3; k >= 0; --k)
        if (ch < 0 && mu[k] > T(0)) ch = k;
    }
  }
  return ch;
}

// the photon channels into LDS: those of every material with several
template <typename T, int F>
__device__ __forceinline__ void stage_photon(const KArgs<T>& a, T* tab) {
  const int nt = a.tb.n;
  if constexpr (several(F)) {
    // the photon channels of every material, T_PHOTON_END x n each
    const int per = T_PHOTON_END * nt;
    for (int k = threadIdx.x; k < per * a.tb.nmat; k += blockDim.x) {
      const int m = k / per;
      tab[k] = a.tb.t[mat_block(m, nt) + uint32_t(k - m * per)];
    }
  } else {
    stage(a.tb, tab, T_PHOTON_END);
  }
}

template <typename T, int F>
__global__ __launch_bounds__(kMaxBlock, MCX_FLIGHT_WAVES) void k_flight(KArgs<T> a, int par) {
  set_flavor<F>(a);
  const uint32_t cs = stripe_cap(a);
  const StripeSums sums = stripe_sums(a.cnt, q_gin(par), cs);
  const uint32_t n = sums.pre[kStripes];
  if (blockIdx.x * blockDim.x >= n) return;
  extern __shared__ __align__(16) unsigned char smem[];
  T* tab = reinterpret_cast<T*>(smem);
  __shared__ BlockStats bs;
  LaneStats ls;
  stats_init(&bs, ls);
  stage_photon<T, F>(a, tab);
  __syncthreads();
  const Bank<T>& in = a.q[q_gin(par)];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
    const uint32_t i = base + threadIdx.x;
    int ch = -1;
    Part<T> p;
    if (i < n) {
      load_part(a, in, striped_record(sums, i, cs), p);
      ch = photon_flight<T, F>(a, tab, p, ls, &bs);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t slot = append(a, Q_KC + c, ch == c);
      if (ch == c && slot != ~0u) store_part(a, a.q[Q_KC + c], slot, p);
    }
  }
  stats_flush(&bs, ls, a.cnt);
}

// ---------------------------------------------------------------------------
// photon KNOCK: the four interaction queues are processed as one index space,
// so that (except at the three boundaries) each wavefront runs one type
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T sample_kn(Rng<T>& r, T e, T* cost) {
  const T k = e / T(kMc2);
  const T kmin = T(1) / (T(1) + T(2) * k);
  const T a1 = M<T>::log(T(1) + T(2) * k);
  const T a2 = T(0.5) * (T(1) - kmin * kmin);
  T kap = T(1), ct = T(1);
  for (int tries = 0; tries < kMaxTries; ++tries) {
    const T ub = uni<T>(r), ux = uni<T>(r), ua = uni<T>(r);
    if (ub * (a1 + a2) < a1) kap = M<T>::exp(-ux * a1);
    else kap = M<T>::sqrt(kmin * kmin + ux * (T(1) - kmin * kmin));
    ct = T(1) - (T(1) - kap) / (k * kap);
    ct = ct < T(-1) ? T(-1) : (ct > T(1) ? T(1) : ct);
    const T g = T(1) - kap * (T(1) - ct * ct) / (T(1) + kap * kap);
    if (ua <= g) break;
  }
  *cost = ct;
  return kap;
}

template <typename T>
__device__ __forceinline__ T sample_rayleigh(Rng<T>& r, T e, T ray_a) {
  const T U = (e / T(kHc)) * (e / T(kHc));
  const T c3 = -M<T>::expm1(T(-3) * M<T>::log1p(ray_a * U));
  T ct = T(1);
  for (int tries = 0; tries < kMaxTries; ++tries) {
    const T xi = uni<T>(r), ua = uni<T>(r);
    const T u = M<T>::expm1(-M<T>::log1p(-xi * c3) / T(3)) / ray_a;
    ct = T(1) - T(2) * u / U;
    if (ct < T(-1)) ct = T(-1);
    if (ua <= T(0.5) * (T(1) + ct * ct)) break;
  }
  return ct;
}

// a new secondary of p: takes the next ordinal; kept if above its absorption
// energy (positrons always, so that they annihilate), else deposited here
template <typename T>
__device__ __forceinline__ void make_child(const KArgs<T>& a, Part<T>& p, Child<T>& c, uint32_t type, T e,
                                           const T d[3], DepAcc& acc, LaneStats& ls, BlockStats* bs) {
  const uint32_t k = p.nchild++;
  stat_add(bs, S_SECONDARIES);
  c.on = false;
  if (type != POSITRON && !(e > a.eabs[type])) {
    deposit(a, acc, ls, p, e);
    return;
  }
  c.on = true;
  c.type = type;
  c.w = p.w;
  c.e = e;
  c.d[0] = d[0]; c.d[1] = d[1]; c.d[2] = d[2];
  c.uid = child_uid(p.uid, k);
}

// One photon interaction of channel q at the photon's position (KNOCK):
// secondaries in c1 (and c2 for pair production); returns whether the photon
// goes on (Compton above Eabs, Rayleigh), else its history record is finished.
template <typename T, int F>
__device__ __forceinline__ bool photon_interact(const KArgs<T>& a, int q, Part<T>& p, Child<T>& c1, Child<T>& c2,
                                                DepAcc& acc, LaneStats& ls, BlockStats* bs) {
  bool keep = false;
  const uint32_t v = vlin(a, p.ix);
  if (q == 0) {
    stat_add(bs, S_COMPTON);
    T cost;
    const T kap = sample_kn(p.rng, p.e, &cost);
    const T phi = T(2.0 * kPi) * uni<T>(p.rng);
    const T d0[3] = {p.d[0], p.d[1], p.d[2]};
    rotate(p.d, cost, phi);
    const T ep = kap * p.e;
    const T te = p.e - ep;
    T pe[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) pe[k] = p.e * d0[k] - ep * p.d[k];
    const T nn = M<T>::sqrt(pe[0] * pe[0] + pe[1] * pe[1] + pe[2] * pe[2]);
    if (nn > T(0)) { pe[0] /= nn; pe[1] /= nn; pe[2] /= nn; }
    else { pe[0] = d0[0]; pe[1] = d0[1]; pe[2] = d0[2]; }
    make_child(a, p, c1, ELECTRON, te, pe, acc, ls, bs);
    if (ep > a.eabs[PHOTON]) {
      p.e = ep;
      keep = true;
    } else {
      deposit(a, acc, ls, p, ep);
      stat_add(bs, S_ABSORBED);
    }
    event(a, p, EV_COMPTON, v);
  } else if (q == 1) {
    stat_add(bs, S_PHOTO);
    make_child(a, p, c1, ELECTRON, p.e, p.d, acc, ls, bs);
    stat_add(bs, S_ABSORBED);
    event(a, p, EV_PHOTO, v);
  } else if (q == 2) {
    stat_add(bs, S_RAYLEIGH);
    const T ct = sample_rayleigh(p.rng, p.e, several(F) ? mat_const(a.tb, a.mat[v]).ray_a : a.tb.ray_a);
    const T phi = T(2.0 * kPi) * uni<T>(p.rng);
    rotate(p.d, ct, phi);
    keep = true;
    event(a, p, EV_RAYLEIGH, v);
  } else {
    stat_add(bs, S_PAIR);
    const T avail = p.e - T(2.0 * kMc2);
    const T eps = uni<T>(p.rng);
    const T tm = eps * avail, tp = (T(1) - eps) * avail;
    T dm[3] = {p.d[0], p.d[1], p.d[2]};
    T dp[3] = {p.d[0], p.d[1], p.d[2]};
    const T cm = leading_angle(beta_of(tm), uni<T>(p.rng));
    const T fm = T(2.0 * kPi) * uni<T>(p.rng);
    const T cp = leading_angle(beta_of(tp), uni<T>(p.rng));
    const T fp = T(2.0 * kPi) * uni<T>(p.rng);
    rotate(dm, cm, fm);
    rotate(dp, cp, fp);
    make_child(a, p, c1, ELECTRON, tm, dm, acc, ls, bs);
    make_child(a, p, c2, POSITRON, tp, dp, acc, ls, bs);
    stat_add(bs, S_ABSORBED);
    event(a, p, EV_PAIR, v);
  }
  if (!keep) finish(a, p);
  return keep;
}

// Photon interactions.  While many photons are in flight, a launch performs
// one interaction per photon and hands the scattered photon to the next
// iteration's flight kernel.  In the tail of a chunk (at most
// MCX_CHAIN_PHOTONS photons wait for an interaction, and at most
// 1/MCX_CHAIN_DIV of the chunk's largest interaction launch) each lane
// follows its photon through every further flight and interaction to its
// end (the secondaries go to the e+- queue as they are made), so that the
// last photons of long scattering chains do not each cost an iteration of
// every kernel.  The relative bound keeps small runs, whose photons would
// all be chained from the start, on the flight kernel, which walks the
// voxels at a higher occupancy.  Each particle draws from its own random
// stream, so the result does not depend on which kernel runs a flight.
template <typename T, int F>
__global__ __launch_bounds__(kMaxBlock, MCX_KNOCK_WAVES) void k_knock(KArgs<T> a, int par) {
  set_flavor<F>(a);
  Counters* C = a.cnt;
  const uint32_t n0 = min(C->n[Q_KC].v, a.cap), n1 = min(C->n[Q_KP].v, a.cap);
  const uint32_t n2 = min(C->n[Q_KR].v, a.cap), n3 = min(C->n[Q_KX].v, a.cap);
  const uint32_t e1 = n0 + n1, e2 = e1 + n2, ntot = e2 + n3;
  if (blockIdx.x * blockDim.x >= ntot) return;
  extern __shared__ __align__(16) unsigned char smem[];
  T* tab = reinterpret_cast<T*>(smem);
  __shared__ BlockStats bs;
  LaneStats ls;
  stats_init(&bs, ls);
  // the peak of earlier launches (this launch raises it only when it takes
  // more photons than any before, and then chains nothing either way)
  const uint32_t peak = C->knock_peak;
  const bool chain = ntot <= uint32_t(MCX_CHAIN_PHOTONS) && uint64_t(ntot) * MCX_CHAIN_DIV <= peak;
  if (blockIdx.x == 0 && threadIdx.x == 0 && ntot > peak) atomicMax(&C->knock_peak, ntot);
  if (chain) stage_photon<T, F>(a, tab);
  __syncthreads();
  const int eo = q_eout(par);
  const uint32_t cs = stripe_cap(a);
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < ntot; base += stride) {
    const uint32_t i = base + threadIdx.x;
    Part<T> p;
    Child<T> c1, c2;
    c1.on = false;
    c2.on = false;
    bool keep = false;
    DepAcc acc = dep_init();
    if (i < ntot) {
      int q = i < n0 ? 0 : (i < e1 ? 1 : (i < e2 ? 2 : 3));
      const uint32_t j = i - (q == 0 ? 0u : (q == 1 ? n0 : (q == 2 ? e1 : e2)));
      load_part(a, a.q[Q_KC + q], j, p);
      keep = photon_interact<T, F>(a, q, p, c1, c2, acc, ls, &bs);
      while (chain && keep) {
        // this interaction's secondaries (made where the photon is now), then
        // the photon's next flight and interaction; a chain stops (its photon
        // goes on in the next iteration) once the secondaries fill half of an
        // e+- queue stripe, so that long chains cannot overflow a small bank
        const uint32_t t1 = append(a, eo, c1.on);
        if (c1.on && t1 != ~0u) store_child(a, a.q[eo], t1, p, c1);
        const uint32_t t2 = append(a, eo, c2.on);
        if (c2.on && t2 != ~0u) store_child(a, a.q[eo], t2, p, c2);
        const bool half = (c1.on && t1 != ~0u && t1 % cs >= cs / 2) || (c2.on && t2 != ~0u && t2 % cs >= cs / 2);
        c1.on = false;
        c2.on = false;
        if (half) break;
        q = photon_flight<T, F>(a, tab, p, ls, &bs);
        keep = q >= 0 && photon_interact<T, F>(a, q, p, c1, c2, acc, ls, &bs);
      }
      dep_flush(a, acc, ls);
    }
    const uint32_t sg = append(a, q_gout(par), keep);
    if (keep && sg != ~0u) store_part(a, a.q[q_gout(par)], sg, p);
    const uint32_t s1 = append(a, eo, c1.on);
    if (c1.on && s1 != ~0u) store_child(a, a.q[eo], s1, p, c1);
    const uint32_t s2 = append(a, eo, c2.on);
    if (c2.on && s2 != ~0u) store_child(a, a.q[eo], s2, p, c2);
  }
  stats_flush(&bs, ls, a.cnt);
}

// ---------------------------------------------------------------------------
// electron / positron Class II transport
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void e_absorb(const KArgs<T>& a, Part<T>& p, Child<T>& c1, Child<T>& c2, DepAcc& acc,
                                         LaneStats& ls, BlockStats* bs) {
  const uint32_t v = vlin(a, p.ix);
  deposit(a, acc, ls, p, p.e);
  stat_add(bs, S_ABSORBED);
  if (p.type == POSITRON) {
    // annihilation at rest: two back-to-back photons, isotropic
    stat_add(bs, S_ANNIH);
    const T ct = T(2) * uni<T>(p.rng) - T(1);
    const T phi = T(2.0 * kPi) * uni<T>(p.rng);
    const T s2 = T(1) - ct * ct;
    const T st = M<T>::sqrt(s2 > T(0) ? s2 : T(0));
    T sp, cp;
    M<T>::sincos(phi, &sp, &cp);
    const T d1[3] = {st * cp, st * sp, ct};
    const T d2[3] = {-d1[0], -d1[1], -d1[2]};
    make_child(a, p, c1, PHOTON, T(kMc2), d1, acc, ls, bs);
    make_child(a, p, c2, PHOTON, T(kMc2), d2, acc, ls, bs);
  }
  p.e = T(0);
  event(a, p, EV_ABSORB, v);
  finish(a, p);
}

template <typename T>
__device__ __forceinline__ void e_escape(const KArgs<T>& a, Part<T>& p, uint32_t v, BlockStats* bs) {
  ledger_escape(a, bs, p);
  event(a, p, EV_E_ESCAPE, v);
  p.e = T(0);
  finish(a, p);
}

template <typename T>
__device__ __forceinline__ T binary_cos(T e, T w, bool primary) {
  const T m2 = T(2.0 * kMc2);
  T c2 = primary ? (e - w) * (e + m2) / (e * (e - w + m2)) : w * (e + m2) / (e * (w + m2));
  if (c2 > T(1)) c2 = T(1);
  return M<T>::sqrt(c2);
}

// Straggling of the soft energy loss over a step: a loss of mean m (the CSDA
// loss over the step's mass path) and variance om2 = mass path x the soft
// second moment at the step's initial energy.  Gaussian (Box-Muller, cosine
// branch) truncated symmetrically to (0, 2m) when m > 3 sd; uniform on
// m -/+ sqrt(3) sd when sqrt(3) sd < m <= 3 sd; else 0 with probability
// a = 1 - 4 m^2 / (3 s2) and uniform on (0, 3 s2 / (2m)) otherwise, with
// s2 = om2 + m^2 (the same mean and second moment).  The draws depend on
// the mass path, not on m: a zero path (a particle on a face) draws nothing,
// although its CSDA loss may be a rounding residue rather than 0; m = 0 on a
// positive path takes the two-mode branch, which returns 0.
template <typename T>
__device__ __forceinline__ T soft_omega2(const Tab<T>& tb, int lep, T e) {
  const T p2 = e * (e + T(2.0 * kMc2));
  const T et = e + T(kMc2);
  const T beta2 = p2 / (et * et);
  const T wmax = lep ? e : T(0.5) * e;
  const T wc = tb.wcc_soft < wmax ? tb.wcc_soft : wmax;
  const T wr = tb.wcr_soft < e ? tb.wcr_soft : e;
  return tb.strag_k * wc / beta2 + T(0.5) * tb.strag_b * wr * wr;
}

template <typename T>
__device__ __forceinline__ T soft_straggle(const Tab<T>& tb, int lep, T e, T m, double mass_path, Rng<T>& rng) {
  if (!(mass_path > 0.0)) return m;
  const T om2 = T(mass_path) * soft_omega2(tb, lep, e);
  const T m2 = m * m;
  if (m2 > T(9) * om2) {
    const T om = M<T>::sqrt(om2);
    for (int tries = 0; tries < kMaxTries; ++tries) {
      const T r = M<T>::sqrt(T(-2) * M<T>::log(uni<T>(rng)));
      const T w = m + om * r * M<T>::cos(T(2.0 * kPi) * uni<T>(rng));
      if (w > T(0) && w < T(2) * m) return w;
    }
    return m;
  }
  if (m2 > T(3) * om2) return m + M<T>::sqrt(T(3) * om2) * (T(2) * uni<T>(rng) - T(1));
  const T s2 = om2 + m2;
  const T aa = T(1) - T(4) * m2 / (T(3) * s2);
  const T u = uni<T>(rng);
  return u < aa ? T(0) : T(1.5) * s2 / m * (u - aa) / (T(1) - aa);
}

// Heitler's cross section per gram of two-photon annihilation in flight of a
// positron of kinetic energy e (g = 1 + e/mc^2, p = sqrt(g^2 - 1)):
// pi r_e^2 n_e [(g^2 + 4g + 1) ln(g + p) - (g + 3) p] / ((g + 1)(g^2 - 1)).
// It falls with energy.
template <typename T>
__device__ __forceinline__ T sigma_annih(const Tab<T>& tb, T e) {
  const T g = T(1) + e / T(kMc2);
  const T p = M<T>::sqrt(g * g - T(1));
  return tb.annih_k * ((g * g + T(4) * g + T(1)) * M<T>::log(g + p) - (g + T(3)) * p) / ((g + T(1)) * (g * g - T(1)));
}

// Per-step data of the density gradient (second replay): the step's voxel,
// its likelihood-ratio scores (majorant free path and soft deflection), its
// pathwise soft-loss coefficient l S(E1) at fixed geometric length, the CSDA
// chain factor r = S(E1)/S(E) and the loss weight d = weight x w_v; at the
// particle's end, lam_end = d of the voxel where it is absorbed, else 0.
struct EGrad {
  uint32_t v;
  double score, coef, r, d, lam_end;
  double se;  // d ln p(mu) / dE of the hinge's soft deflection (term E), 0 without a hinge
  bool end;
};

// d ln p(mu) / d rho of the soft angular law p(mu) = A (1 + A) / (mu + A)^2
// on [0, 1], whose mean m(A) = A (1 + A) ln(1 + 1/A) - A is matched to
// <mu> = (1 - exp(-rho len t1s))/2 at the step's geometric length len:
// [1/A + 1/(1 + A) - 2/(mu + A)] len t1s (1/2 - <mu>) / m'(A),
// m'(A) = (1 + 2A) ln(1 + 1/A) - 2; 0 where A is held at its bound
__device__ __forceinline__ double soft_score(double A, double mu, double mbar, double len, double t1s) {
  if (!(A > 0.0) || mbar > kSoftMHi) return 0.0;
  const double dm_da = (1.0 + 2.0 * A) * log1p(1.0 / A) - 2.0;
  return (1.0 / A + 1.0 / (1.0 + A) - 2.0 / (mu + A)) * (len * t1s * (0.5 - mbar)) / dm_da;
}

// one Class II step; returns false when the particle is gone.  EXT compiles
// in the optional physics (straggling, annihilation in flight), each behind
// its run-time switch.  G = 1 also fills eg with the step's gradient data;
// with `look` set it moves the particle without any other effect (no deposit,
// secondary, statistic or event): the look-ahead pass of the second replay.
template <typename T, bool EXT, int G = 0>
__device__ __forceinline__ bool e_step(const KArgs<T>& a, const Tab<T>& tb, const T* tab, const T* soft, Part<T>& p, Child<T>& c1,
                       Child<T>& c2, DepAcc& acc, LaneStats& ls, BlockStats* bs, EGrad& eg, bool look = false) {
  const bool DRY = G != 0 && look;
  const int nt = tb.n;
  const int lep = p.type == POSITRON ? 1 : 0;
  const int base = T_E + lep * T_ES;
  const T eabs = a.eabs[p.type];
  if constexpr (G != 0) {
    eg.v = vlin(a, p.ix);
    eg.score = 0.0;
    eg.coef = 0.0;
    eg.r = 1.0;
    eg.d = a.adj_w[eg.v] * (a.vr ? p.w : 1.0);
    eg.lam_end = 0.0;
    eg.se = 0.0;
    eg.end = false;
  }
  if (!(p.e > eabs)) {
    if constexpr (G != 0) {
      eg.end = true;
      eg.lam_end = eg.d;
    }
    if (!DRY) e_absorb(a, p, c1, c2, acc, ls, bs);
    return false;
  }
  if (!DRY) ls.esteps++;
  rng_refill(p.rng);
  const T e = p.e;
  const uint32_t v = vlin(a, p.ix);
  const T rho = a.rho[v];
  // step control: maximum mass step and hard-event majorant over [elo, e]
  const T le = M<T>::log(e);
  const Grid<T> g = grid_at(tb, le);
  const T ss = interp(tab, nt, base + O_LS, g, e, T(0));
  const T tau_max = a.c2 * e / ss;
  const T r0 = range_at(tab, nt, base, g, e, le, tb.lemin, tb.dl);
  T elo = r0 - tau_max > T(0) ? range_inv(tab, nt, base, r0 - tau_max, g.i) : tb.emin;
  if (elo > e) elo = e;
  if (EXT && a.straggle) {
    // a straggled loss can exceed the step's CSDA loss: by at most twice the
    // CSDA mean (Gaussian and uniform laws) and by at most 6 Omega^2(E)/S
    // (two-mode law; 8 here, for the stopping power's change over the step):
    // the hard-event majorant covers every energy the step can end at
    const T d2 = T(2) * (e - elo);
    const T dw = T(8) * soft_omega2(tb, lep, e) / ss;
    const T dmax = dw > d2 ? dw : d2;
    elo = e - dmax > tb.emin ? e - dmax : tb.emin;
  }
  T smaj = majorant(tb, tab, base, lep, elo, g, e);
  if constexpr (EXT) {
    // annihilation in flight: its cross section falls with energy, so its
    // value at the interval's low end bounds it over the step
    if (a.annih && lep) smaj += sigma_annih(tb, elo);
  }
  // the hard-event clock: a pending free path runs on across steps, so where
  // faces cut a track does not change where its hard events fall
  if (!(p.clk > T(0))) p.clk = -M<T>::log(uni<T>(p.rng));
  const T tau_h = smaj > T(0) ? p.clk / smaj : M<T>::inf();
  const bool capped = !(tau_h <= tau_max);
  const T tau_s = capped ? tau_max : tau_h;
  const double len = double(tau_s / rho);
  const double th = double(uni<T>(p.rng)) * len;
  int ax;
  const double db = face_dist(a, p, &ax);
  if (ax < 0) {
    atomicOr(&a.cnt->overflow, uint32_t(OVF_LOST));
    if constexpr (G != 0) eg.end = true;
    return false;
  }
  // the step ends at the first face on its path or at its full length; a
  // reached hinge deflects the particle by the soft angular law of the whole
  // step.  The soft loss is charged where the step ends, over the geometric
  // length s travelled, so the energy along a track is the CSDA energy of
  // the path travelled whatever the voxel size.
  bool face_end = db <= th;
  double s = db, after = db;
  if (!face_end) {
    move(p, th);
    const T t1s = interp(tab, nt, base + O_LT1S, g, e, T(0));
    const T mbar = T(0.5) * (T(1) - M<T>::exp(-T(double(rho) * len) * t1s));
    const T A = soft_a(mbar, soft);
    const T u3 = uni<T>(p.rng);
    const T mu = A * u3 / (T(1) + A - u3);
    if constexpr (G != 0) {
      const double sc = soft_score(double(A), double(mu), double(mbar), len, double(t1s));
      eg.score += sc;
      if (a.grad_e) {
        // the same law's score with respect to the energy: <mu> moves with E
        // through t1s, a power law between nodes (stored as logarithms)
        const T l0 = tab[(base + O_LT1S) * nt + g.i], l1 = tab[(base + O_LT1S) * nt + g.i + 1];
        if (l0 > -M<T>::inf() && l1 > -M<T>::inf())
          eg.se = sc * double(rho) * double(l1 - l0) * double(tb.inv_dl) / double(e);
      }
    }
    const T phi = T(2.0 * kPi) * uni<T>(p.rng);
    rotate(p.d, T(1) - T(2) * mu, phi);
    const double rem = len - th;
    const double db2 = face_dist(a, p, &ax);
    if (ax < 0) {
      atomicOr(&a.cnt->overflow, uint32_t(OVF_LOST));
      if constexpr (G != 0) eg.end = true;
      return false;
    }
    face_end = db2 <= rem;
    after = face_end ? db2 : rem;
    s = face_end ? th + db2 : len;
  }
  const double mass_path = double(rho) * s;
  // the clock runs down by the majorant optical depth of the path; a step
  // that ends uncapped at its full length ends at an event (below)
  const bool event_end = !face_end && !capped;
  p.clk = event_end ? T(0) : p.clk - smaj * T(mass_path);
  // gradient: the candidate events of the majorant process along the path
  // are a Poisson process of rate rho smaj per unit length: -smaj s over the
  // path, +1/rho at an event
  if constexpr (G != 0) eg.score += -double(smaj) * s + (event_end ? 1.0 / double(rho) : 0.0);
  T e1 = range_inv(tab, nt, base, T(r0 - T(mass_path)), g.i);
  if (!(e1 < e)) e1 = e;
  if (EXT && a.straggle) {
    // the loss keeps its CSDA mean and fluctuates about it (drawn after the
    // soft deflection)
    e1 = e - soft_straggle(tb, lep, e, e - e1, mass_path, p.rng);
    if (!(e1 > T(0))) e1 = T(0);
  }
  if (!DRY) deposit(a, acc, ls, p, e - e1);
  p.e = e1;
  if constexpr (G != 0) {
    // d(loss)/d rho at fixed geometric length s = s S(E1); dE1/dE = S(E1)/S(E)
    const Grid<T> g1 = grid_at(tb, M<T>::log(e1));
    const double s1 = double(interp(tab, nt, base + O_LS, g1, e1, T(0)));
    eg.coef = s * s1;
    eg.r = s1 / double(ss);
  }
  if (face_end) {
    // an energy at or below Eabs is absorbed at the next step's start, in
    // the voxel entered
    if (!DRY) event(a, p, EV_CROSS, v);
    if (cross(a, p, after, ax, ls)) {
      if constexpr (G != 0) eg.end = true;
      if (!DRY) e_escape(a, p, v, bs);
      return false;
    }
    return true;
  }
  move(p, after);
  if (!(e1 > eabs)) {
    if constexpr (G != 0) {
      eg.end = true;
      eg.lam_end = eg.d;
    }
    if (!DRY) e_absorb(a, p, c1, c2, acc, ls, bs);
    return false;
  }
  if (capped) {
    if (!DRY) event(a, p, EV_STEP, v);
    return true;
  }
  // hard event or delta: elastic, inelastic, bremsstrahlung in this order.
  // Each kind samples its own variables, then all share the azimuth draw,
  // the rotations and the secondary (one inlined copy each).
  const T u = uni<T>(p.rng) * smaj;
  const Grid<T> g1 = grid_at(tb, M<T>::log(e1));
  const T s_el = interp(tab, nt, base + O_LEL, g1, e1, T(0));
  const T s_in = interp(tab, nt, base + O_LIN, g1, e1, tb.thr_in[lep]);
  const T s_br = interp(tab, nt, base + O_LBR, g1, e1, tb.thr_br);
  int kind = u < s_el ? 1 : (u < s_el + s_in ? 2 : (u < s_el + s_in + s_br ? 3 : 0));
  if constexpr (EXT) {
    if (kind == 0 && a.annih && lep && u < s_el + s_in + s_br + sigma_annih(tb, e1)) kind = 4;
  }
  if (kind == 0) {
    if (!DRY) {
      stat_add(bs, S_DELTA);
      event(a, p, EV_STEP, v);
    }
    return true;
  }
  if constexpr (EXT) {
    if (kind == 4) {
      // the photons take the positron's energy away: no energy adjoint beyond
      if constexpr (G != 0) eg.end = true;
      if (DRY) return false;
      // two-photon annihilation with an electron at rest: the softer photon
      // takes the share z of E + 2mc^2, z in [zmin, 1/2], from Heitler's DCS
      // S(z) + S(1-z), S(x) = -(g+1)^2 + (g^2+4g+1)/x - 1/x^2: proposal 1/z
      // (log-uniform), acceptance z (S(z) + S(1-z)) / (2 (g^2+4g+1)) <= 1;
      // polar cosines (g + 1 - 1/z)/p from energy-momentum conservation, the
      // photons on opposite azimuths
      stat_add(bs, S_ANNIH);
      stat_add(bs, S_ANNIH_FLIGHT);
      const T gm = T(1) + e1 / T(kMc2);
      const T pm = M<T>::sqrt(gm * gm - T(1));
      const T zmin = T(1) / (gm + T(1) + pm);
      const T cc = gm * gm + T(4) * gm + T(1);
      const T g1 = (gm + T(1)) * (gm + T(1));
      T z = T(0.5);
      for (int tries = 0; tries < kMaxTries; ++tries) {
        z = zmin * M<T>::pow(T(0.5) / zmin, uni<T>(p.rng));
        const T y = T(1) - z;
        const T f = -g1 + cc / z - T(1) / (z * z) - g1 + cc / y - T(1) / (y * y);
        if (uni<T>(p.rng) * T(2) * cc <= z * f) break;
      }
      const T ph = T(2.0 * kPi) * uni<T>(p.rng);
      const T etot = e1 + T(2.0 * kMc2);
      const T ka = z * etot, kb = etot - ka;
      T ca = (gm + T(1) - T(1) / z) / pm, cb = (gm + T(1) - T(1) / (T(1) - z)) / pm;
      ca = ca > T(1) ? T(1) : (ca < T(-1) ? T(-1) : ca);
      cb = cb > T(1) ? T(1) : (cb < T(-1) ? T(-1) : cb);
      T da[3] = {p.d[0], p.d[1], p.d[2]}, dv[3] = {p.d[0], p.d[1], p.d[2]};
      rotate(da, ca, ph);
      rotate(dv, cb, ph + T(kPi));
      make_child(a, p, c1, PHOTON, ka, da, acc, ls, bs);
      make_child(a, p, c2, PHOTON, kb, dv, acc, ls, bs);
      p.e = T(0);
      event(a, p, EV_ANNIH_FLIGHT, v);
      finish(a, p);
      return false;
    }
  }
  T cos_p = T(1), cos_c = T(1), w = T(0);  // primary and secondary polar cosines, energy lost
  if (kind == 1) {
    if (!DRY) stat_add(bs, S_HARD_EL);
    // screened Rutherford restricted to [mu_c, 1]
    const T p2 = e1 * (e1 + T(2.0 * kMc2));
    const T et = e1 + T(kMc2);
    const T pv = p2 / et;
    const T beta2 = p2 / (et * et);
    const T kk = tb.k_coef * (T(kMc2) / pv) * (T(kMc2) / pv);
    const T eta = tb.eta_a * (T(kMc2) * T(kMc2) / p2) * (T(1.13) + tb.eta_b / beta2);
    T muc = T(1) / (s_el / kk + T(1) / (T(1) + eta)) - eta;
    muc = muc < T(0) ? T(0) : (muc > T(1) ? T(1) : muc);
    const T ia = T(1) / (muc + eta), ib = T(1) / (T(1) + eta);
    T m = T(1) / (ia - uni<T>(p.rng) * (ia - ib)) - eta;
    m = m < T(0) ? T(0) : (m > T(1) ? T(1) : m);
    cos_p = T(1) - T(2) * m;
  } else if (kind == 2) {
    if (!DRY) stat_add(bs, S_HARD_IN);
    // Moller (e-) or Bhabha (e+) energy transfer k = W/E above kc = Wcc/E:
    // proposal ~ 1/k^2 on [kc, 1/2] (e-) or [kc, 1] (e+), then rejection
    const T kc = a.wcc / e1;
    const T gm = T(1) + e1 / T(kMc2);
    const T aa = ((gm - T(1)) / gm) * ((gm - T(1)) / gm);
    T b1 = T(0), b2 = T(0), b3 = T(0), b4 = T(0);
    if (lep) {
      const T gp = gm + T(1);
      b1 = aa * (T(2) * gp * gp - T(1)) / (gm * gm - T(1));
      b2 = aa * (T(3) * gp * gp + T(1)) / (gp * gp);
      b3 = aa * T(2) * (gm - T(1)) * gm / (gp * gp);
      b4 = aa * (gm - T(1)) * (gm - T(1)) / (gp * gp);
    }
    const T span = lep == 0 ? T(1) - T(2) * kc : T(1) - kc;
    // e-: k^2 times the bracket, f = 1 + r^2 + a k^2 - (1 - a) r with
    // r = k/(1-k), is at most 1 + 5 a k^2 on (0, 1/2]: the proposal is
    // 1/k^2 (weight w1 = 1/kc - 2, by inversion) plus a flat part (weight
    // w2 = 5a (1/2 - kc)), one uniform choosing the part and sampling it
    const T w1 = T(1) / kc - T(2), w2 = T(5) * aa * (T(0.5) - kc);
    const T wt = lep == 0 ? w1 + w2 : T(1);
    T k = kc;
    for (int tries = 0; tries < kMaxTries; ++tries) {
      const T uu = uni<T>(p.rng) * wt, ua = uni<T>(p.rng);
      bool ok;
      if (lep == 0) {
        k = uu < w1 ? kc / (T(1) - (uu / w1) * span) : kc + (uu - w1) / w2 * (T(0.5) - kc);
        const T r = k / (T(1) - k);
        ok = ua * (T(1) + T(5) * aa * k * k) <= T(1) + r * r + aa * k * k - (T(1) - aa) * r;
      } else {
        k = kc / (T(1) - uu * span);
        const T gg = T(1) - b1 * k + b2 * k * k - b3 * k * k * k + b4 * k * k * k * k;
        ok = ua <= gg;
      }
      if (ok) break;
    }
    w = k * e1;
    cos_p = binary_cos(e1, w, true);
    cos_c = binary_cos(e1, w, false);
  } else {
    if (!DRY) stat_add(bs, S_HARD_BR);
    w = a.wcr * M<T>::pow(e1 / a.wcr, uni<T>(p.rng));
    cos_c = leading_angle(beta_of(e1), uni<T>(p.rng));
  }
  const T ph = T(2.0 * kPi) * uni<T>(p.rng);
  bool turn = kind == 1;
  if (kind != 1) {
    // the secondary leaves from the direction before the event: the knock-on
    // electron on the opposite azimuth, the photon on the drawn one
    T dc[3] = {p.d[0], p.d[1], p.d[2]};
    if (!DRY) rotate(dc, cos_c, kind == 2 ? ph + T(kPi) : ph);
    // interaction forcing: the channel's cross section is F times the
    // analog one; the event changes the primary with probability 1/F (a draw
    // after the azimuth's) and its secondary carries weight w/F
    bool apply = true;
    double fw = 1.0;
    if (a.vr) {
      const double f = kind == 2 ? a.f_in : a.f_br;
      if (f > 1.0) {
        apply = double(uni<T>(p.rng)) * f < 1.0;
        fw = f;
      }
    }
    // bremsstrahlung splitting: a second photon of the same energy with its
    // own polar cosine and azimuth (drawn after the above), each of the two
    // with half the weight; it takes the second child slot
    const bool split = a.vr && kind == 3 && a.split_br == 2;
    T d2[3] = {p.d[0], p.d[1], p.d[2]};
    if (split) {
      const T c2c = leading_angle(beta_of(e1), uni<T>(p.rng));
      const T ph2 = T(2.0 * kPi) * uni<T>(p.rng);
      if (!DRY) rotate(d2, c2c, ph2);
      fw *= 2.0;
    }
    if (apply) p.e = e1 - w;
    if (!DRY) {
      const double w0 = p.w;
      p.w = w0 / fw;
      make_child(a, p, c1, kind == 2 ? ELECTRON : PHOTON, w, dc, acc, ls, bs);
      if (split) make_child(a, p, c2, PHOTON, w, d2, acc, ls, bs);
      p.w = w0;
    }
    turn = kind == 2 && apply;
  }
  // one rotation of the primary serves the elastic and the inelastic events
  // (the children above take the direction before the event)
  if (turn) rotate(p.d, cos_p, ph);
  if (!DRY) event(a, p, kind == 1 ? EV_HARD_EL : (kind == 2 ? EV_HARD_IN : EV_HARD_BR), v);
  return true;
}

// The e+- kernel keeps its lanes busy: a lane whose particle is gone (or has
// used its step budget and is written back to the output queue) takes the
// next record of the input queue, until the queue is exhausted.  A wavefront
// reserves input records kTakeBatch at a time and hands them to its lanes
// over the following iterations.  Track lengths are long-tailed, so a
// wavefront whose queue has run dry would otherwise run its few longest tracks
// to the end with most lanes idle: after a short tail it writes them back
// instead, and they continue, among full wavefronts, in the next iteration.
constexpr uint32_t kTakeBatch = 32;

template <typename T, int F>
__global__ __launch_bounds__(kMaxBlock, MCX_ESTEP_WAVES) void k_estep(KArgs<T> a, int par) {
  set_flavor<F>(a);
  const uint32_t cs = stripe_cap(a);
  const StripeSums sums = stripe_sums(a.cnt, q_ein(par), cs);
  const uint32_t n = sums.pre[kStripes];
  if (blockIdx.x * blockDim.x >= n) return;
  extern __shared__ __align__(16) unsigned char smem[];
  T* tab = reinterpret_cast<T*>(smem);
  __shared__ BlockStats bs;
  LaneStats ls;
  stats_init(&bs, ls);
  constexpr bool MMF = several(F);
  const int ntab = a.tb.n;
  if constexpr (MMF) {
    // several materials: the soft-law table (after material 0's block) in
    // LDS; each step reads its material's channels from the table block
    for (int k = threadIdx.x; k < kSoftN; k += blockDim.x) tab[k] = a.tb.t[T_NCH * ntab + k];
  } else {
    stage(a.tb, tab, T_NCH, kSoftN);
  }
  __syncthreads();
  const Bank<T>& in = a.q[q_ein(par)];
  const int ge = q_eout(par), gg = q_gout(par);
  const uint32_t lane = __lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  Part<T> p;
  DepAcc acc = dep_init();
  bool alive = false, taking = true;
  constexpr bool ADJB = base_flavor(F) == FL_ADJ_B;
  // second replay: the look-ahead phase, the particle's input record and its
  // energy-adjoint sums
  bool ahead = false;
  uint32_t rec = 0;
  double lam_tot = 0.0, lam_pre = 0.0, lam_p = 1.0;
  double psi_tot = 0.0, psi_pre = 0.0;  // term E: the same sums of the hinges' energy scores
  uint32_t used = 0, dry = 0;
  uint32_t rbase = 0, rleft = 0;  // the wavefront's reserved input records [rbase, rbase + rleft)
  for (;;) {
    if (taking) {
      const uint64_t needm = __ballot(!alive);
      const uint32_t cnt = uint32_t(__popcll(needm));
      const uint32_t rank = uint32_t(__popcll(needm & below));
      uint32_t idx = rbase + rank;
      if (cnt > rleft) {  // wave-uniform: reserve more
        const uint32_t r = max(cnt - rleft, kTakeBatch);
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(&a.cnt->take_e.v, r);
        b = __shfl(b, 0);
        if (rank >= rleft) idx = b + (rank - rleft);
        rbase = b + (cnt - rleft);
        rleft = r - (cnt - rleft);
      } else {
        rbase += cnt;
        rleft -= cnt;
      }
      const bool need = !alive;
      if (__ballot(need && idx >= n) != 0ull) taking = false;  // wave-uniform
      const uint64_t got = __ballot(need && idx < n);
      if (lane == 0 && got) atomicAdd(&bs.c[S_EVISITS], (unsigned long long)__popcll(got));
      if (need && idx < n) {
        load_part(a, in, striped_record(sums, idx, cs), p);
        alive = true;
        used = 0;
        if constexpr (ADJB) {
          // second replay: first follow the particle's whole remaining track
          // without effects (the look-ahead), then again from its record
          ahead = true;
          rec = striped_record(sums, idx, cs);
          lam_tot = 0.0;
          psi_tot = 0.0;
          lam_p = 1.0;
        }
      }
    } else {
      ++dry;
    }
    if (!__any(alive)) break;
    dep_resolve(a, acc);  // the insertion issued in the previous step
    Child<T> c1, c2;
    c1.on = false;
    c2.on = false;
    if (alive) {
      EGrad eg;
      constexpr int G = ADJB ? 1 : 0;
      const bool look = ADJB && ahead;
      if constexpr (MMF) {
        // the step stays in its voxel, so in one material
        const uint32_t m = a.mat[vlin(a, p.ix)];
        alive = e_step<T, true, G>(a, mat_tab(a.tb, m), a.tb.t + mat_block(int(m), ntab), tab, p, c1, c2, acc, ls,
                                   &bs, eg, look);
      } else {
        alive = e_step<T, extended(F), G>(a, a.tb, tab, tab + T_NCH * ntab, p, c1, c2, acc, ls, &bs, eg, look);
      }
      if constexpr (ADJB) {
        if (look) {
          // lam_tot = sum_k d_k (1 - r_k) P_k + lam_end P_K, P_k the product of
          // the chain factors before step k: every later step's energy
          // adjoint follows from it and the sums before that step
          lam_tot += eg.d * (1.0 - eg.r) * lam_p;
          psi_tot += eg.se * lam_p;
          lam_p *= eg.r;
          if (!alive) {
            lam_tot += eg.lam_end * lam_p;
            load_part(a, in, rec, p);  // back to the record for the second pass
            alive = true;
            ahead = false;
            lam_pre = 0.0;
            psi_pre = 0.0;
            lam_p = 1.0;
          }
        } else {
          // the history's centred score times the step's scores, and the soft
          // loss it deposits here minus what the particle then lacks downstream
          lam_pre += eg.d * (1.0 - eg.r) * lam_p;
          psi_pre += eg.se * lam_p;
          lam_p *= eg.r;
          const double lam_after = eg.end ? eg.lam_end : (lam_tot - lam_pre) / lam_p;
          // term E: the later hinges' energy scores, chained back to this
          // step's end, times d(E1)/d rho = -s S(E1)
          const double psi_after = eg.end ? 0.0 : (psi_tot - psi_pre) / lam_p;
          const double cq = a.adj_q[p.hist - a.cnt->run_first] - a.adj_qbar;
          const double gv = cq * (eg.score - eg.coef * psi_after) + eg.coef * (eg.d - lam_after);
          if (gv != 0.0) unsafeAtomicAdd(&a.adj_grad[eg.v], gv);
        }
      }
      ++used;
    }
    dep_flush_pending(a, acc, ls);
    // secondaries of this step and particles written back: one atomic per
    // output queue and wavefront, both in flight together
    const bool tail = dry >= MCX_TAIL_MIN && __popcll(__ballot(alive)) < MCX_TAIL_ALIVE;  // wave-uniform
    // (the second replay follows each particle to its end: its look-ahead
    // covers the whole remaining track)
    const bool park = !ADJB && alive && (used >= a.steps || tail);
    const bool c1e = c1.on && c1.type != PHOTON, c1g = c1.on && c1.type == PHOTON;
    const uint64_t me1 = __ballot(c1e), mep = __ballot(park), mg1 = __ballot(c1g), mg2 = __ballot(c2.on);
    const uint32_t ne1 = uint32_t(__popcll(me1)), ng1 = uint32_t(__popcll(mg1));
    const uint32_t ne = ne1 + uint32_t(__popcll(mep)), ng = ng1 + uint32_t(__popcll(mg2));
    if (ne + ng != 0u) {  // wave-uniform
      uint32_t be = 0, bg = 0;
      const uint32_t st = my_stripe();
      if (lane == 0) {
        atomicAdd(&bs.c[S_EWRITES], (unsigned long long)(ne + ng));
        if (ne) be = atomicAdd(&a.cnt->ns[ge][st].v, ne);
        if (ng) bg = atomicAdd(&a.cnt->ns[gg][st].v, ng);
      }
      be = __shfl(be, 0);
      bg = __shfl(bg, 0);
      // slots within this block's stripe of each output queue
      const uint32_t s1 = c1e ? be + uint32_t(__popcll(me1 & below)) : bg + uint32_t(__popcll(mg1 & below));
      const uint32_t s2 = bg + ng1 + uint32_t(__popcll(mg2 & below));
      const uint32_t so = be + ne1 + uint32_t(__popcll(mep & below));
      const bool ov = (c1.on && s1 >= cs) || (c2.on && s2 >= cs) || (park && so >= cs);
      if (ov) atomicOr(&a.cnt->overflow, uint32_t(OVF_QUEUE));
      if (c1.on && s1 < cs) store_child(a, a.q[c1e ? ge : gg], st * cs + s1, p, c1);
      if (c2.on && s2 < cs) store_child(a, a.q[gg], st * cs + s2, p, c2);
      if (park && so < cs) store_part(a, a.q[ge], st * cs + so, p);
    }
    if (park) alive = false;
  }
  dep_flush(a, acc, ls);
  stats_flush(&bs, ls, a.cnt);
}

// ---------------------------------------------------------------------------
// bookkeeping between iterations (one thread)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_advance(Counters* c, int par, uint32_t target, uint32_t cap) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t cs = cap / uint32_t(kStripes);
  uint32_t pop = 0u;
  for (int k = 0; k < kStripes; ++k) {
    pop += min(c->ns[Q_G0 + 1 - par][k].v, cs) + min(c->ns[Q_E0 + 1 - par][k].v, cs);
    c->ns[Q_G0 + par][k].v = 0u;
    c->ns[Q_E0 + par][k].v = 0u;
  }
  c->n[Q_KC].v = c->n[Q_KP].v = c->n[Q_KR].v = c->n[Q_KX].v = 0u;
  c->take_e.v = 0u;
  c->cursor += c->adm;
  const uint64_t rem = c->chunk_end - c->cursor;
  uint64_t adm = target > pop ? uint64_t(target - pop) : 0ull;
  if (adm > rem) adm = rem;
  c->adm = uint32_t(adm);
  c->done = (pop == 0u && rem == 0ull) ? 1u : 0u;
  c->iter++;
}

// start of a chunk of histories [first, end)
template <typename T>
__global__ void k_chunk_init(Counters* c, uint64_t first, uint64_t end, uint64_t run_first, uint32_t adm) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int q = 0; q < Q_NQ; ++q) c->n[q].v = 0u;
  for (int q = 0; q < kStripedQueues; ++q)
    for (int k = 0; k < kStripes; ++k) c->ns[q][k].v = 0u;
  c->overflow = 0u;
  c->done = 0u;
  c->iter = 0u;
  c->cursor = first;
  c->chunk_end = end;
  c->run_first = run_first;
  c->adm = adm;
  c->occupied = 0ull;
  c->knock_peak = 0u;
  c->take_e.v = 0u;
}

// ---------------------------------------------------------------------------
// tally flush: each (history, voxel) score q, complete now that its history
// is, adds q^2 to Sum q^2 (Eq. (1)-(3); Sum q was formed at insertion);
// slots are cleared for the next chunk
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_flush(TSlot* tab, uint64_t nslot, double* sum_q, double* sum_q2, Counters* cnt, int test_mode,
                        double* hist_led, uint64_t n_run) {
  // the table is a stream of 16-byte slots: each thread loads kFlushUnroll
  // of them (a wavefront's loads coalesce) before it examines any, so that
  // several loads are in flight per thread; occupied slots add q^2 and are
  // emptied
  constexpr int kFlushUnroll = 4;
  const uint64_t lanes = uint64_t(gridDim.x) * blockDim.x;
  uint32_t occ = 0;
  double dep = 0.0;  // deposited energy, for the run statistics
  for (uint64_t s0 = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; s0 < nslot; s0 += kFlushUnroll * lanes) {
    TSlot t[kFlushUnroll];
#pragma unroll
    for (int j = 0; j < kFlushUnroll; ++j) {
      const uint64_t s = s0 + uint64_t(j) * lanes;
      t[j] = s < nslot ? tab[s] : TSlot{kEmptyKey, 0.0};
    }
#pragma unroll
    for (int j = 0; j < kFlushUnroll; ++j) {
      const uint64_t k = t[j].key;
      if (k == kEmptyKey) continue;
      const double q = t[j].q;
      dep += q;
      const uint32_t v = uint32_t(k & 0xFFFFFFFFull);
      unsafeAtomicAdd(&sum_q2[v], q * q);  // Sum q was formed at insertion
      if (test_mode) {
        const uint64_t h = (k >> 32) - cnt->run_first;
        if (h < n_run) unsafeAtomicAdd(&hist_led[3 * h], q);
      }
      tab[s0 + uint64_t(j) * lanes] = TSlot{kEmptyKey, 0.0};
      ++occ;
    }
  }
  occ = wave_sum(occ);
  dep = wave_sum(dep);
  if (__lane_id() == 0 && occ) atomicAdd((unsigned long long*)&cnt->occupied, (unsigned long long)occ);
  if (__lane_id() == 0 && dep != 0.0) unsafeAtomicAdd(&cnt->e_dep, dep);
}

// an empty table: every key empty, every score 0
template <typename T>
__global__ void k_clear_table(TSlot* tab, uint64_t nslot) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t s = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < nslot; s += stride) tab[s] = TSlot{kEmptyKey, 0.0};
}

// density gradient helpers: loss weights per MeV, mean of Q_h, final terms
template <typename T>
__global__ void k_adj_weights(const double* dl_ddose, const T* rho, uint64_t nvox, double vol, double* w) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nvox; v += stride)
    w[v] = dl_ddose[v] * 1e6 / (double(rho[v]) * vol);
}

template <typename T>
__global__ void k_adj_sum(const double* q, uint64_t n, double* out) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  double acc = 0.0;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) acc += q[i];
  acc = wave_sum(acc);
  if (__lane_id() == 0 && acc != 0.0) unsafeAtomicAdd(out, acc);
}

// dL/drho_j = (score and pathwise sums)/N - dL/dD_j * D_j / rho_j
template <typename T>
__global__ void k_adj_finalize(const double* grad_acc, const double* dl_ddose, const double* sum_q, const T* rho,
                               uint64_t nvox, double vol, double nhist, double* out) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nvox; v += stride) {
    const double r = double(rho[v]);
    const double dose = sum_q[v] / nhist * 1e6 / (r * vol);
    out[v] = grad_acc[v] / nhist - dl_ddose[v] * dose / r;
  }
}

// dose (eV/g per history) and its standard error, Eq. (1)-(3)
template <typename T>
__global__ void k_dose(const double* sum_q, const double* sum_q2, const T* rho, uint64_t nvox, double vol,
                       double nhist, double* dose, double* sigma) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < nvox; v += stride) {
    const double mass = double(rho[v]) * vol;
    const double qm = sum_q[v] / nhist, q2 = sum_q2[v] / nhist;
    double var = (q2 - qm * qm) / nhist;
    if (var < 0.0) var = 0.0;
    dose[v] = qm * 1e6 / mass;
    if (sigma) sigma[v] = sqrt(var) * 1e6 / mass;
  }
}

}  // namespace mcx
