/*
 * mcx.h -- C ABI of the MI355X (gfx950) Monte-Carlo electron-photon dose
 * transport library (libmcx.so).
 *
 * The library runs the independent particle-history loop of PenRed
 * (arXiv:2003.00796): JUMP (distance to the next interaction), STEP (move
 * through the voxel geometry, stopping at interfaces) and KNOCK (simulate the
 * interaction, create secondaries), Sec. 4.1; constant voxel geometry, Sec.
 * 4.2.2 and Sec. 4.3; Class II electron/positron transport with parameters
 * C1, C2, Wcc, Wcr, Eabs (Sec. 5.2, Sec. 6.1); the history-by-history
 * estimators of Sec. 4.3, Eq. (1)-(3), with the square root of Eq. (2)
 * restored; dose in eV/g per history (Fig. 8 caption).  Every step of the
 * path runs in HIP kernels on the device; the host only validates, sizes
 * memory and schedules launches.
 *
 * Conventions
 *  - Every function returns an int status: MCX_OK (0) or a negative MCX_E_*
 *    code.  mcx_last_error() returns a context-owned message describing the
 *    last failure; it stays valid until the next call on that context.
 *  - No exception, exit or abort crosses the ABI.
 *  - Units: MeV, cm, g/cm^3.  Voxel arrays are x-fastest: index
 *    (iz * ny + iy) * nx + ix.
 *  - A context is used by one host thread at a time; contexts are
 *    independent of each other.
 *  - Stream arguments are hipStream_t values passed as void* (NULL = the
 *    context's own stream).
 */
#ifndef MCX_H
#define MCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCX_OK 0
#define MCX_E_INVALID (-1)     /* bad argument value */
#define MCX_E_STATE (-2)       /* call order (e.g. run before phantom) */
#define MCX_E_NOMEM (-3)       /* device or host allocation failed */
#define MCX_E_DEVICE (-4)      /* HIP runtime error or device fault */
#define MCX_E_RANGE (-5)       /* a capacity or energy range exceeded */
#define MCX_E_CANCELLED (-6)   /* run stopped on request (mcx_cancel) */
#define MCX_E_UNSUPPORTED (-7) /* feature not available in this library */

#define MCX_FP64 0   /* all physics and sampling in FP64 */
#define MCX_MIXED 1  /* FP32 physics and sampling; FP64 positions, boundary
                        distances and tallies */

#define MCX_PHOTON 0
#define MCX_ELECTRON 1
#define MCX_POSITRON 2

#define MCX_SRC_PENCIL 0       /* all histories start at pos along dir */
#define MCX_SRC_RECT 1         /* uniform over a width[0] x width[1] rectangle
                                  centred on pos in the x-y plane, along dir */

/* Model channel switches (mcx_transport.flags).  A switched-off hard channel
 * behaves as if its cutoff were infinite (its stopping contribution becomes
 * soft).  Used for analytic checks; production runs use 0. */
#define MCX_NO_COMPTON (1u << 0)
#define MCX_NO_PHOTO (1u << 1)
#define MCX_NO_RAYLEIGH (1u << 2)
#define MCX_NO_PAIR (1u << 3)
#define MCX_NO_HARD_ELASTIC (1u << 4)
#define MCX_NO_HARD_INELASTIC (1u << 5)
#define MCX_NO_HARD_BREMS (1u << 6)
/* Straggling of the soft energy loss of a Class II step: the loss over a
 * path of s g/cm^2 keeps the CSDA value as its mean and gets the variance
 * s * Omega^2(E), the second moment of the soft part of the energy-loss DCS
 * per unit mass path (Bohr's variance from the leading free-electron term of
 * the Moller/Bhabha DCS below Wcc, plus b Wcr^2 / 2 from the b/W
 * bremsstrahlung DCS below Wcr): a Gaussian truncated to (0, 2 x mean) when
 * the mean exceeds 3 standard deviations, a uniform law of the same mean and
 * variance down to sqrt(3) standard deviations, below that a point mass at
 * zero plus a uniform law with the same two moments.  Off by default (the
 * soft loss is then the deterministic CSDA value); not supported by
 * mcx_dose_backward. */
#define MCX_STRAGGLING (1u << 7)
/* Two-photon annihilation of positrons in flight with the material's
 * electrons at rest: a fourth hard channel with Heitler's cross section
 * (bounded over a step by its value at the step's lowest energy, since it
 * falls with energy); the softer photon's share of E + 2mc^2 is drawn from
 * Heitler's DCS and both photon directions follow from energy and momentum
 * conservation.  Off by default (positrons then annihilate at rest only). */
#define MCX_ANNIH_FLIGHT (1u << 8)

typedef struct mcx_ctx mcx_ctx;

/* Parameters of the synthetic analytic material models (one material, scaled
 * per voxel by its mass density).  The library tabulates every cross section
 * from these on the log grid of mcx_transport.  Photon: free-electron Klein-Nishina Compton; photoelectric
 * pe_coef*(E/pe_eref)^-pe_exp; Rayleigh form factor
 * ray_f0*(1+ray_a x^2)^-2; pair pp_coef*ln(E/2mc^2)^2.  Electron/positron:
 * Bethe stopping power with mean excitation energy i_exc, Moller/Bhabha
 * hard collisions, bremsstrahlung DCS brems_b/W, screened Rutherford
 * elastic scattering (Z(Z+1) sum zz1_mol, screening charge z_screen). */
typedef struct {
  double z_mol, a_mol, zz1_mol, z_screen, i_exc;
  double pe_coef, pe_eref, pe_exp;
  double pp_coef;
  double ray_f0, ray_a;
  double brems_b;
} mcx_material_desc;

/* Transport parameters: the table grid (log-spaced, n_grid nodes between
 * e_min and e_max), absorption energies Eabs per particle type, and the
 * Class II parameters C1, C2, Wcc, Wcr of Sec. 5.2.  Validation: 16 <=
 * n_grid <= 512, 0 < e_min < e_max, 0 < c1, c2 <= 0.2, wcc, wcr > 0,
 * eabs[i] >= e_min. */
typedef struct {
  int n_grid;
  double e_min, e_max;
  double eabs[3];
  double c1, c2;
  double wcc, wcr;
  uint32_t flags;
  /* Interaction forcing (the variance reduction of the disc example with
   * forced bremsstrahlung and hard collisions, PENELOPE example tests of
   * the Validation section): the hard inelastic-collision
   * and bremsstrahlung cross sections are multiplied by force_in, force_br;
   * a forced event emits its secondary with the weight w/F and changes the
   * primary (energy loss, deflection) with probability 1/F, so that every
   * expectation is unchanged while F times more secondaries are produced.
   * 0 or 1 = analog; otherwise F in [1, 1e5] (MCX_E_INVALID if not).
   * Each material's tables carry the forced cross sections (several-material
   * phantoms included); mcx_dose_backward weights the deposits and
   * soft-loss terms (the photon-flight scores are the analog ones). */
  double force_in, force_br;
  /* Bremsstrahlung splitting (the same example splits emitted photons by 2):
   * with split_br = 2 each emission yields two photons of the sampled energy,
   * the second with its own polar and azimuthal angle, each with half the
   * weight; the primary loses the energy once.  0 or 1 = no splitting;
   * other values MCX_E_INVALID.  Same restrictions as forcing. */
  int split_br;
} mcx_transport;

/* Voxel phantom.  nx, ny, nz <= 1024; voxel sizes > 0; rho > 0 everywhere
 * (MCX_E_INVALID otherwise).  rho is FP64, x-fastest; if rho_on_device is
 * nonzero it is a device pointer that is copied on the device (the caller
 * may free it after the call returns).  mat (host memory, same layout, may be
 * NULL) gives each voxel a material index < 4 of mcx_load_material: with it
 * the transport runs the several-material kernels (photon flights in
 * optical depth, each interaction and step by its voxel's tables), which
 * need every material up to the largest index loaded before mcx_run. */
typedef struct {
  int nx, ny, nz;
  double voxel_cm[3];
  double origin_cm[3];
  const double* rho;
  int rho_on_device;
  const uint8_t* mat;
} mcx_phantom_desc;

/* One source (a beamlet).  Histories are numbered by concatenating the
 * sources in order: source s owns ids [sum_{r<s} n_hist_r, ... + n_hist_s).
 * energy must lie in (eabs[particle], e_max]; dir must be a unit vector;
 * start points must lie inside the phantom. */
typedef struct {
  int particle;
  int kind;
  double energy;
  double pos[3];
  double dir[3];
  double width[2];
  uint64_t n_hist;
} mcx_source;

/* Counters of the transport since the last mcx_reset_tallies. */
typedef struct {
  uint64_t histories;
  uint64_t flights, compton, photo, rayleigh, pair;
  uint64_t esteps, hard_el, hard_in, hard_br, delta, annih;
  uint64_t crossings, secondaries, deposits;
  uint64_t absorbed, escaped;
  double e_dep, e_esc;
  uint64_t pos_esc;
  uint64_t iterations, chunks, tally_pairs;
  double ms_transport, ms_flush;
  /* work counters of the e+- step kernel: records read, records written,
   * tally-table insertions */
  uint64_t evisits, ewrites, inserts;
  /* per-kernel GPU time (HIP events on the run's stream) when timing is on:
   * source, photon flight, photon interactions, e+- steps; and the number of
   * iterations timed (each iteration launches each kernel once) */
  double ms_source, ms_flight, ms_knock, ms_estep;
  uint64_t timed_iterations;
  /* host wall time of the two density-gradient replays */
  double ms_backward;
  /* first history id the last mcx_run did not complete: first_hist + n_hist
   * after a complete run, the cancellation watermark after MCX_E_CANCELLED */
  uint64_t next_history;
  /* positrons annihilated in flight (MCX_ANNIH_FLIGHT; counted in annih too) */
  uint64_t annih_flight;
} mcx_stats;

/* Create a context on HIP device `hip_device` computing in `precision`
 * (MCX_FP64 or MCX_MIXED).  *out receives the context (NULL on failure). */
int mcx_create(mcx_ctx** out, int hip_device, int precision);
/* Release every device and host resource of the context (NULL is allowed). */
void mcx_destroy(mcx_ctx* ctx);
/* Message of the last failure on ctx (never NULL). */
const char* mcx_last_error(mcx_ctx* ctx);

/* Transport parameters; must precede mcx_load_material.  Copied. */
int mcx_set_transport(mcx_ctx* ctx, const mcx_transport* t);
/* Tabulate material mat_id (0..3) on the transport grid and copy the tables
 * to the device.  Material 0 serves every voxel of a phantom without a
 * material array; the others are selected per voxel by the phantom's
 * material array.  mcx_set_transport discards every loaded material. */
int mcx_load_material(mcx_ctx* ctx, int mat_id, const mcx_material_desc* m);
/* Copy the phantom densities to the device (converted to FP32 in MIXED
 * precision).  Resets the tallies. */
int mcx_load_phantom(mcx_ctx* ctx, const mcx_phantom_desc* p);
/* Copy n >= 1 sources; history ids are their concatenation. */
int mcx_set_sources(mcx_ctx* ctx, const mcx_source* s, int n);

/* Tuning knobs (0 keeps the current value): bank = records per event queue,
 * in [1024, 2^26], default 2^25 (the population target is a quarter of it;
 * the photon and e+- queues are split into 8 stripes of bank/8 records, and
 * a run fails with MCX_E_RANGE if one fills), block = threads per block
 * (multiple of 64, <= 256, default 256), steps = Class II steps per visit of
 * the e+- kernel (default 128).  Device memory of the queues: about
 * 8 x bank x (72 B FP32 physics, 88 B FP64). */
int mcx_set_launch(mcx_ctx* ctx, uint32_t bank, uint32_t block, uint32_t steps);
/* Replay each batch of event-loop iterations as one captured HIP graph
 * (1, default) or launch its kernels one by one (0).  Graphs are used only
 * while per-kernel timing is off. */
int mcx_set_graph(mcx_ctx* ctx, int on);
/* Pick the launch for the sources' histories.  The bank size follows a
 * rule: the smallest power of two whose population target (a quarter of it)
 * holds all the histories, up to 2^24, with the queues in at most a quarter
 * of the device memory.  Block size {128, 256} and steps per visit
 * {32, 128, 512} are chosen by timing a sample of n_sample histories
 * (0: min(total, 2e5)) for each pair.  The choice is applied and the tallies
 * are reset.  With cache_path, a previous result for the same device and
 * workload (a hash of architecture, precision, grid, transport parameters and
 * sources) is reused, and a new one is appended as a JSON line.  chosen (3
 * values: bank, block, steps) may be NULL. */
int mcx_autotune(mcx_ctx* ctx, uint64_t n_sample, const char* cache_path, uint32_t* chosen);
/* Enable (1) or disable (0) per-kernel timing with HIP events recorded on
 * the run's stream around each transport kernel (small overhead). */
int mcx_set_timing(mcx_ctx* ctx, int on);
/* Enable (1) or disable (0) the per-history event hash and energy ledger
 * used by the parity tests (costs extra device traffic). */
int mcx_set_test_mode(mcx_ctx* ctx, int on);

/* Transport histories [first_hist, first_hist + n_hist) with the counter
 * RNG keyed by seed (< 2^32), ACCUMULATING into the tallies.  The run is
 * complete when the call returns (kernels are queued on `stream`, the call
 * waits for them).  Deterministic event content for a given
 * (seed, history range).  first_hist + n_hist must not exceed the total of
 * the sources nor 2^32.  Returns MCX_E_CANCELLED, with the histories before
 * mcx_stats.next_history complete and tallied, when it honours mcx_cancel. */
int mcx_run(mcx_ctx* ctx, uint64_t seed, uint64_t first_hist, uint64_t n_hist, void* stream);

/* Gradient of a dose loss with respect to every voxel density (the density
 * derivative of the estimator of Sec. 4.3, Eq. (1)).  dl_ddose
 * holds dL/dD_v (D in eV/g per history, as from mcx_get_dose); dl_drho
 * receives dL/drho_v (nx*ny*nz doubles each; device arrays if on_device,
 * else host).  The histories of the last mcx_run are replayed twice from
 * their random-number counters (no tracks are stored): the first replay forms
 * each history's weighted score Q_h = sum_v w_v q_hv with
 * w_v = dL/dD_v * 1e6 / (rho_v V); the second adds (Q_h - mean Q) times the
 * likelihood-ratio scores of the history's sampled variables (every photon
 * free flight: -mu l_j per traversed voxel with mu of the voxel's material,
 * +1/rho at the interaction; every e+- step: -smaj s of its hard-event
 * majorant process over its length s, +1/rho where it ends at an event, and
 * the score of its soft deflection), and the pathwise derivative of each
 * e+- step's soft loss at fixed geometric length, s S(E1) times its voxel's
 * weight minus the particle's CSDA energy adjoint after the step.  The
 * explicit mass term -dL/dD_v D_v / rho_v completes the gradient.  Unbiased
 * when electrons are absorbed where they are created; with Class II
 * transport the step control (cap, hinge) is held at its geometric value and
 * the energy dependence of later sampling laws is held fixed, except the soft
 * deflection's under MCX_GRAD_DEFLECTION_ENERGY (mcx_set_gradient).  Requires
 * that the tallies hold exactly one mcx_run since the last reset
 * (MCX_E_STATE otherwise).  Runs with straggling are refused
 * (MCX_E_UNSUPPORTED: the estimator has no term for a straggled loss);
 * annihilation in flight (an unscored e+ hard event like the others),
 * several-material phantoms, forcing and splitting are supported.  The tallies and statistics are unchanged. */
int mcx_dose_backward(mcx_ctx* ctx, const double* dl_ddose, double* dl_drho, int on_device, void* stream);

/* Options of mcx_dose_backward.  MCX_GRAD_DEFLECTION_ENERGY also scores each
 * soft deflection's dependence on the particle's energy (through the soft
 * transport coefficient), chained to the density of every earlier step of
 * the particle through the CSDA energy chain: it removes the estimator's
 * bias on electron tracks (where the energy sets the angular spread) at the
 * price of a larger variance.  Default 0.  Changing it keeps the last run's
 * replays valid.  MCX_E_INVALID for unknown bits. */
#define MCX_GRAD_DEFLECTION_ENERGY (1u << 0)
int mcx_set_gradient(mcx_ctx* ctx, uint32_t flags);

/* Dose (eV/g per history) and its standard error per voxel from the
 * accumulated counters, Eq. (1)-(3).  dose and sigma are caller-owned arrays
 * of nx*ny*nz doubles, on the device if dst_on_device, else on the host;
 * sigma may be NULL. */
int mcx_get_dose(mcx_ctx* ctx, double* dose, double* sigma, int dst_on_device, void* stream);
/* Raw counters Sum q and Sum q^2 (MeV) per voxel, same placement rules. */
int mcx_get_tally(mcx_ctx* ctx, double* sum_q, double* sum_q2, int dst_on_device, void* stream);
/* Zero the tallies, the history count and the statistics. */
int mcx_reset_tallies(mcx_ctx* ctx);
/* Statistics since the last reset. */
int mcx_get_stats(mcx_ctx* ctx, mcx_stats* out);

/* CT calibration, the role of the DICOM import of a transport code without
 * its file I/O: Hounsfield units to mass density by the piecewise-linear
 * curve through (hu[i], rho[i]), i < n_points (hu strictly increasing, rho
 * > 0; constant beyond the end points), and to a material index by
 * thresholds: a voxel takes material k, the number of thresholds mat_hu[j]
 * (strictly increasing, at most 3) at or below its HU. */
typedef struct {
  int n_points;
  const double* hu;
  const double* rho;
  int n_thresholds;
  const double* mat_hu;
} mcx_ct_calibration;
/* Convert nvox HU values (host arrays) into densities (g/cm^3) and material
 * indices (mat may be NULL) for mcx_phantom_desc.  Host code only: needs no
 * context and no device.  MCX_E_INVALID for a malformed calibration. */
int mcx_ct_to_phantom(const mcx_ct_calibration* cal, const int16_t* hu, uint64_t nvox, double* rho, uint8_t* mat);

/* Per-source dose influence (one source = one beamlet): with on != 0, every
 * later run also accumulates, per (source, voxel) pair that received
 * energy, the per-history scores q of that source's histories: Sum q and
 * Sum q^2 (MeV), formed at the chunk flush where each history's score is
 * complete (Eq. (1)-(3)).  The pairs live in a device hash table of
 * 2^log2_slots entries (24 B each; log2_slots in [10, 30]); a run that
 * fills it fails with MCX_E_RANGE.  The dose of source b in voxel v per
 * history of b is Sum q * 1e6 / (rho_v V n_b) eV/g, n_b its histories run.
 * mcx_reset_tallies clears the table; on = 0 frees it.  The table is library
 * memory, and checkpoints do not hold it. */
int mcx_set_influence(mcx_ctx* ctx, int on, uint32_t log2_slots);
/* Read the influence table as n entries (source index, voxel index, Sum q,
 * Sum q^2) in no particular order, into host arrays of `capacity` entries.
 * *n receives the number of entries; with all four arrays NULL only the
 * count is returned; MCX_E_RANGE if capacity < *n.  MCX_E_STATE when the
 * influence output is off. */
int mcx_get_influence(mcx_ctx* ctx, uint32_t* source, uint32_t* voxel, double* sum_q, double* sum_q2,
                      uint64_t capacity, uint64_t* n);

/* Wait for the work queued on the context's own stream and report a device
 * fault or an earlier asynchronous HIP error as MCX_E_DEVICE.  (mcx_run and
 * the result calls already wait for their own work before returning.) */
int mcx_synchronize(mcx_ctx* ctx);

/* Ask the run in progress to stop early; the only call that may come from
 * another host thread while mcx_run executes.  The request stays pending
 * until a forward run honours it at a completion check (after each batch of
 * event-loop iterations; the density-gradient replays ignore it): the run
 * starts no further history, completes the histories already started, adds
 * them to the tallies and returns MCX_E_CANCELLED (or MCX_OK, the request
 * dropped, if every history had started by then).  The completed histories
 * are [first_hist, mcx_stats.next_history); a later mcx_run of the rest with
 * the same seed gives the tallies of the uninterrupted run (histories are
 * independent and their random streams depend only on (seed, history id);
 * Sec. 4.3), up to the order of FP64 summation. */
int mcx_cancel(mcx_ctx* ctx);

/* Checkpoint of the accumulated result, to resume in another context or
 * process: Sum q, Sum q^2, the history count, next_history and the
 * statistics, with a format tag and a checksum.  With buf == NULL, *size
 * receives the size in bytes (16 * nx*ny*nz plus a few hundred); otherwise
 * buf (host memory, *size bytes, MCX_E_RANGE if too small) receives the
 * checkpoint and *size its length. */
int mcx_checkpoint(mcx_ctx* ctx, void* buf, size_t* size);
/* Replace the tallies, history count and statistics of ctx by a checkpoint
 * (host memory, size bytes).  The context must have the checkpoint's
 * precision and phantom grid (MCX_E_INVALID otherwise, and for a buffer that
 * is not an intact checkpoint).  Later runs accumulate onto it; the density
 * gradient needs a run of its own context (MCX_E_STATE until then). */
int mcx_restore(mcx_ctx* ctx, const void* buf, size_t size);

/* Device bytes a run needs besides the tallies, tables, phantom and loop
 * counters: the event queues of the current bank size and the
 * (history, voxel) tally table at its full 2^29 slots (16 B each). */
int mcx_workspace_size(mcx_ctx* ctx, size_t* bytes);
/* Run in caller-owned device memory (e.g. a torch tensor) instead of memory
 * the library allocates: the queues and the tally table are carved
 * from [dev, dev + bytes), dev 256-byte aligned (MCX_E_INVALID otherwise).
 * The table takes the largest power-of-two number of slots, up to 2^29, that
 * fits after the queues; chunks of histories are sized to it.  bytes must
 * leave room for 2^20 slots (MCX_E_RANGE otherwise, and the library's own
 * memory is used again); mcx_workspace_size gives the size for the full
 * table.  The call waits for the device to be idle, so the memory must only
 * hold work queued before it; it must stay valid and unused by others until
 * mcx_set_workspace(ctx, NULL, 0) (back to library memory) or mcx_destroy.
 * A later bank size that does not fit makes mcx_run fail with MCX_E_RANGE.
 * Statistics are kept across the change.  The per-history test outputs and
 * the gradient's buffers are still allocated by the library. */
int mcx_set_workspace(mcx_ctx* ctx, void* dev, size_t bytes);

/* Size of the fixed device array of mcx_run_static (per device). */
#define MCX_STATIC_SCRATCH_BYTES (73ull << 20)
/* mcx_run for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  It
 * transports the same histories into the same tallies as mcx_run (the same
 * events for a given (seed, history range); the sums differ only in the
 * order of FP64 additions), but its event queues and (history, voxel) tally
 * table live in a fixed device array of MCX_STATIC_SCRATCH_BYTES that the
 * library declares statically, one per device, held until the process ends;
 * the call itself allocates nothing (no hipMalloc, no host pinning, no HIP
 * graph: its kernels are launched one by one on `stream`).  The bank is the
 * configured one (mcx_set_launch), at most 2^16 records; the table takes the
 * largest power-of-two number of slots that fits after the queues (2^20 in
 * FP64, 2^21 in MIXED precision at the largest bank), and chunks of
 * histories are sized to it.  Limits: a chunk whose (history, voxel) pairs
 * do not fit the table, or a population that fills the queues, fails with
 * MCX_E_RANGE; test mode is refused with MCX_E_UNSUPPORTED (its per-history
 * outputs are sized by the run).  Every call on a device shares that
 * device's array, which keeps the last call's contents (each call clears the
 * table it uses): calls that overlap on one device race and give wrong
 * tallies, so a caller serialises them (one context on one host thread, or
 * one stream).  Other arguments, results and errors as for mcx_run. */
int mcx_run_static(mcx_ctx* ctx, uint64_t seed, uint64_t first_hist, uint64_t n_hist, void* stream);

/* Per-history results of the LAST mcx_run (test mode only, else
 * MCX_E_STATE): hashes[n_hist] = order-independent hash of the history's
 * events; ledger[n_hist * 3] = {energy deposited, energy escaped, positrons
 * escaped}.  Host arrays; either may be NULL. */
int mcx_get_history_results(mcx_ctx* ctx, uint64_t* hashes, double* ledger);

#ifdef __cplusplus
}
#endif
#endif
