// mcx_internal.h -- data layout shared by the host runtime and the HIP
// kernels of libmcx (not part of the public ABI).
//
// Layout in HBM (per context):
//  - table block: n_grid x T_NCH values of the compute type T, channel-major
//    (channel c occupies [c*n, (c+1)*n)), staged into LDS by the kernels;
//  - phantom: rho[nz][ny][nx] in T (FP64 or FP32);
//  - particle queues: Q_NQ structure-of-arrays banks of `cap` records each
//    (positions f64 x3, direction T x3, energy T, uid u64, history u32, draw
//    counter u32, packed voxel u32, type/child-count u32, event hash u64);
//  - tally: open-addressing table of 16-byte slots, a (history, voxel) key
//    and its FP64 score on one line, flushed per chunk into Sum q / Sum q^2
//    (FP64, one per voxel) -- the per-history estimator of Eq. (1)-(3) of
//    the paper.
#pragma once

#include <stdint.h>

namespace mcx {

constexpr double kMc2 = 0.51099895000;       // MeV
constexpr double kRe = 2.8179403262e-13;     // cm
constexpr double kNa = 6.02214076e23;        // 1/mol
constexpr double kAlpha = 1.0 / 137.035999084;
constexpr double kHc = 1.23984198e-2;        // MeV Angstrom
constexpr double kPi = 3.14159265358979323846;

constexpr int kMaxGrid = 512;
// materials per phantom (per-voxel index, one table block each)
constexpr int kMaxMat = 4;
constexpr double kMaxForce = 1.0e5;  // largest interaction-forcing factor
constexpr int kMaxBlock = 256;  // kernels are compiled for blocks of at most 256 threads
constexpr uint64_t kEmptyKey = ~0ull;

enum Particle : uint32_t { PHOTON = 0, ELECTRON = 1, POSITRON = 2 };

// Table channels.  Photon: ln of mass attenuation per process.  Per lepton
// type p (0 = e-, 1 = e+) at T_E + p*T_ES: ln soft stopping power, soft
// stopping power, range, range-segment exponent q = 1 - dlnS/dlnE, ln hard
// elastic, ln hard inelastic, ln hard bremsstrahlung, ln soft transport
// coefficient, node sum of the three hard coefficients, its ln, and its ln
// again but -inf where a channel's threshold falls in the segment above the
// node.  Zero values are stored as ln 0 = -inf.
// Initial guess of the soft angular law parameter: ln A at kSoftN points
// uniform in y = ln(<mu> / (1/2 - <mu>)) over [y(kSoftMLo), y(kSoftMHi)],
// stored after the channel block (offset T_NCH * n).  ln A is close to
// linear in y at both ends (<mu> -> 0 and <mu> -> 1/2).
constexpr int kSoftN = 1024;
constexpr double kSoftMLo = 1e-9;
constexpr double kSoftMHi = 0.49;

enum TabChannel : int {
  T_ENODE = 0,  // node energies
  T_LMU_C = 1, T_LMU_PE = 2, T_LMU_R = 3, T_LMU_PP = 4,
  T_PHOTON_END = 5,  // channels [0, 5) serve the photon kernels
  T_E = 5,
  O_LS = 0, O_S = 1, O_R = 2, O_Q = 3, O_LEL = 4, O_LIN = 5, O_LBR = 6, O_LT1S = 7, O_HSUM = 8,
  O_LH = 9,    // ln of the node sum of the hard cross sections
  O_LHC = 10,  // the same, or -inf where the segment starting at the node holds a threshold
  T_ES = 11,
  T_NCH = T_E + 2 * T_ES
};

// Event queues: photons waiting for a flight (ping-pong pair), electrons and
// positrons waiting for Class II steps (ping-pong pair), photons waiting for
// one interaction type each (Compton, photoelectric, Rayleigh, pair).
enum Queue : int { Q_G0 = 0, Q_G1, Q_E0, Q_E1, Q_KC, Q_KP, Q_KR, Q_KX, Q_NQ };

enum Stat : int {
  S_FLIGHTS = 0, S_COMPTON, S_PHOTO, S_RAYLEIGH, S_PAIR, S_ESTEPS, S_HARD_EL, S_HARD_IN,
  S_HARD_BR, S_DELTA, S_ANNIH, S_CROSSINGS, S_SECONDARIES, S_DEPOSITS, S_ABSORBED,
  S_ESCAPED, S_POSESC,
  S_EVISITS,    // e+- records read by the step kernel
  S_EWRITES,    // records written by the step kernel (survivors + secondaries)
  S_INSERTS,    // tally-table insertions
  S_ANNIH_FLIGHT,  // positrons annihilated in flight (counted in S_ANNIH too)
  S_NSTAT
};

enum Overflow : uint32_t { OVF_QUEUE = 1u, OVF_TALLY = 2u, OVF_SOURCE = 4u, OVF_LOST = 8u };

// bound on rejection-sampling attempts (acceptance is >= 0.3 for every sampler)
constexpr int kMaxTries = 1000;

// a counter alone on its 128-byte cache line: the queue counters take atomics
// from every wavefront of a launch, and counters sharing a line would queue
// behind each other in one L2 channel
struct alignas(128) LineCount {
  uint32_t v;
};

// The photon and e+- ping-pong queues (Q_G0 .. Q_E1) take appends from every
// wavefront of three kernels: each is split into kStripes stripes of cap /
// kStripes records with a counter each (a block appends to stripe
// blockIdx % kStripes), so the atomics spread over as many cache lines.
#ifndef MCX_STRIPES
#define MCX_STRIPES 8
#endif
constexpr int kStripes = MCX_STRIPES;
constexpr int kStripedQueues = 4;

struct Counters {
  LineCount n[Q_NQ];       // occupancy of the interaction queues Q_KC .. Q_KX
  LineCount ns[kStripedQueues][kStripes];  // occupancy of each stripe of Q_G0 .. Q_E1
  LineCount take_e;        // records of the e+- input queue reserved in this iteration
  uint32_t overflow;       // Overflow bits
  uint32_t done;           // chunk finished
  uint32_t adm;            // histories admitted by the next source launch
  uint32_t iter;
  uint64_t cursor;         // next history id to admit
  uint64_t chunk_end;      // end of the current chunk (exclusive)
  uint64_t run_first;      // first history id of the current mcx_run call
  uint64_t stat[S_NSTAT];
  double e_dep, e_esc;
  uint64_t occupied;       // tally pairs seen by the last flush
  uint32_t knock_peak;     // most photons an interaction launch of the chunk took (the photon-chain switch)
};

// A queue record is 4 (FP32 physics) or 5 (FP64) chunks of 16 bytes; chunk k
// of every record of a queue is one array, so a wavefront moves a record with
// one 16-byte access per chunk and lane, each instruction reading or writing
// 1 KiB of contiguous memory.  FP32: {x, y} {z, uid} {u, v, w, E} {meta};
// FP64: {x, y} {z, uid} {u, v} {w, E} {meta}, with meta = {history id, draw
// counter, voxel ix | iy << 10 | iz << 20, type | children << 2}.
struct alignas(16) Chunk {
  uint32_t x, y, z, w;
};
constexpr int kMaxChunks = 5;
template <typename T>
constexpr int rec_chunks() {
  return sizeof(T) == 8 ? 5 : 4;
}

// one slot of the (history, voxel) tally table: the key and its score share
// a 16-byte line segment, so an insertion dirties one cache line
struct alignas(16) TSlot {
  uint64_t key;
  double q;
};

template <typename T>
struct Bank {
  Chunk* c[kMaxChunks];
  uint64_t* hash;  // event hash (test mode)
  double* w;       // statistical weight (interaction forcing)
  T* clk;          // e+- queues only: majorant optical depth left before the next hard event
};

struct SourceDev {
  int particle, kind;
  double energy;
  double pos[3], dir[3], width[2];
  uint64_t end;  // exclusive end of this source's history ids
};

// constants of one material that the kernels need besides its tables
template <typename T>
struct MatConst {
  T k_coef, eta_a, eta_b;  // screened Rutherford elastic (see Tab)
  T ray_a;                 // Rayleigh form factor
  T strag_k, strag_b;      // straggling (see Tab)
  T annih_k;               // annihilation in flight (see Tab)
};

template <typename T>
struct Tab {
  const T* t;        // channel-major block, T_NCH * n
  int n;
  T lemin, inv_dl;   // ln of the first node, 1 / log spacing
  T dl;              // log spacing
  T emin;
  T thr_pp, thr_in[2], thr_br;
  T k_coef;          // n_mol pi r_e^2 sum Z(Z+1): K(E) = k_coef (mc^2 / pv)^2
  T eta_a, eta_b;    // eta(E) = eta_a (mc^2)^2 / p^2c^2 * (1.13 + eta_b / beta^2)
  T ray_a;
  // soft energy-loss straggling: second moment of the soft DCS per unit mass
  // path, strag_k Wc / beta^2 + strag_b Wr^2 / 2, with Wc = min(wcc_soft,
  // W_max) and Wr = min(wcr_soft, E) (the cutoffs are infinite for a
  // switched-off hard channel)
  T strag_k;         // 2 pi r_e^2 mc^2 n_e, MeV cm^2/g
  T strag_b;         // bremsstrahlung DCS constant b, cm^2/g
  T wcc_soft, wcr_soft;
  // two-photon annihilation in flight: pi r_e^2 n_e, cm^2/g
  T annih_k;
  // several materials: their number, their constants, and the offset of
  // material m's channel block in t (material 0 at 0, the soft-law table
  // after it, then materials 1, 2, ...)
  int nmat;
  MatConst<T> mc[kMaxMat];
};

// offset of material m's T_NCH x n channel block in the table block
constexpr uint32_t mat_block(int m, int n) {
  return m == 0 ? 0u : uint32_t(T_NCH * n + kSoftN + (m - 1) * T_NCH * n);
}

template <typename T>
struct KArgs {
  Tab<T> tb;
  // geometry
  int nx, ny, nz;
  double dx, dy, dz, ox, oy, oz;
  double idx, idy, idz;  // 1 / voxel size
  const T* rho;
  // per voxel: half-width (in voxels) of the largest cube around it that lies
  // in the phantom and has its density throughout
  const uint8_t* cube;
  // per-voxel material index (several-material phantoms), else null
  const uint8_t* mat;
  // transport
  T eabs[3];
  T c2, wcc, wcr;
  // run
  uint32_t seed;
  const SourceDev* src;
  int nsrc;
  // tally hash table, key = history id << 32 | voxel index
  TSlot* htab;
  uint64_t hmask;
  double* sum_q;
  double* sum_q2;
  // test mode per-history outputs (indexed by history - cnt->run_first)
  int test_mode;
  uint64_t* hist_hash;
  double* hist_led;      // 3 per history: deposited, escaped, positrons escaped
  // density gradient by replay (0: forward tally; 1: replay A accumulates
  // each history's weighted score Q_h and the local soft-loss derivative;
  // 2: replay B scatters (Q_h - Qbar) times the photon free-flight scores)
  int mode;
  int straggle;          // soft energy-loss straggling on (selects the kernel flavour)
  int grad_e;            // replay B: score the soft deflection's energy dependence (term E)
  int annih;             // positron annihilation in flight on (selects the kernel flavour)
  int mm;                // several materials (selects the kernel flavour)
  int vr;                // interaction forcing: weighted particles (selects the kernel flavour)
  double f_in, f_br;     // forcing factors of hard inelastic collisions and bremsstrahlung
  int split_br;          // bremsstrahlung photons per emission (1 or 2)
  const double* adj_w;   // per voxel: dL/dD_v * 1e6 / (rho_v V)
  double* adj_q;         // per history of the run: Q_h
  double* adj_grad;      // per voxel accumulator
  double adj_qbar;       // mean Q_h (replay B)
  Counters* cnt;
  Bank<T> q[Q_NQ];
  uint32_t cap;          // records per queue
  uint32_t steps;        // Class II steps per visit
};

}  // namespace mcx
