/*
 * oracle.h -- plain single-thread FP64 CPU reference transport.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table generator or
 * constant generator with the HIP path: it builds its own cross-section tables
 * from the analytic model parameters it is given.
 *
 * What it computes (paper arXiv:2003.00796, PenRed):
 *   - the independent particle-history loop of Sec. 4.1 (JUMP = sample the
 *     distance to the next interaction, STEP = move through the geometry and
 *     stop at interfaces, KNOCK = simulate the interaction and create
 *     secondaries);
 *   - voxel geometry with constant STEP/LOCATE (Sec. 4.2.2, Sec. 4.3);
 *   - Class II (mixed) electron/positron transport controlled by the
 *     parameters C1, C2, Wcc, Wcr and Eabs named in Sec. 5.2 and Sec. 6.1;
 *   - the history-by-history tally estimators of Sec. 4.3, Eq. (1)-(3): per
 *     history the score q of each voxel and its square are added to separate
 *     counters;
 *   - dose in eV/g per history (Fig. 8 caption, Sec. 5.4);
 *   - an independent random sequence per history (Sec. 4.3, last paragraphs),
 *     here a counter-based Philox4x32-10 stream per particle.
 * The paper defines the physics only by reference to PENELOPE; the synthetic
 * analytic models and all algorithmic readings are stated in oracle.c next to
 * the code that implements them.
 *
 * Units: MeV, cm, g/cm^3; mass coefficients in cm^2/g; stopping powers in
 * MeV cm^2/g.
 */
#ifndef MCX_ORACLE_H
#define MCX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PHOTON = 0, ORC_ELECTRON = 1, ORC_POSITRON = 2 };
enum { ORC_SRC_PENCIL = 0, ORC_SRC_RECT = 1 };

/* flags: switch model channels off (a switched-off hard channel behaves as if
 * its cutoff were infinite: its stopping contribution becomes soft), or
 * switch the straggling of the soft energy loss on (ORC_STRAGGLING). */
enum {
  ORC_NO_COMPTON = 1u << 0,
  ORC_NO_PHOTO = 1u << 1,
  ORC_NO_RAYLEIGH = 1u << 2,
  ORC_NO_PAIR = 1u << 3,
  ORC_NO_HARD_ELASTIC = 1u << 4,
  ORC_NO_HARD_INELASTIC = 1u << 5,
  ORC_NO_HARD_BREMS = 1u << 6,
  ORC_STRAGGLING = 1u << 7,
  ORC_ANNIH_FLIGHT = 1u << 8, /* two-photon annihilation of positrons in flight */
  /* gradient only (orc_run_gradient): also score each soft deflection's
   * dependence on the particle's energy, chained to the densities of the
   * steps before it (term E) */
  ORC_GRAD_DEFLECTION_ENERGY = 1u << 9
};

typedef struct {
  double z_mol;     /* electrons per molecule */
  double a_mol;     /* molar mass, g/mol */
  double zz1_mol;   /* sum over the atoms of Z(Z+1) */
  double z_screen;  /* effective Z of the Moliere screening parameter */
  double i_exc;     /* mean excitation energy, MeV */
  double pe_coef;   /* photoelectric: mu = pe_coef * (E/pe_eref)^(-pe_exp) */
  double pe_eref;
  double pe_exp;
  double pp_coef;   /* pair: mu = pp_coef * ln(E/2mc^2)^2 above 2mc^2 */
  double ray_f0;    /* Rayleigh form factor F(x) = ray_f0 (1 + ray_a x^2)^-2 */
  double ray_a;     /* Angstrom^2 */
  double brems_b;   /* bremsstrahlung mass DCS b/W, cm^2/g */
} orc_material;

typedef struct {
  int n_grid;
  double e_min, e_max; /* MeV, log-spaced grid */
  double eabs[3];      /* absorption energies: photon, electron, positron */
  double c1, c2;       /* Class II elastic / energy-loss step parameters */
  double wcc, wcr;     /* hard inelastic / hard bremsstrahlung cutoffs */
  uint32_t flags;
  /* interaction forcing (R11): hard inelastic and hard bremsstrahlung cross
   * sections multiplied by these factors (values <= 1: no forcing) */
  double force_in, force_br;
  int split_br; /* bremsstrahlung photons emitted per event, 1 or 2 (R12) */
} orc_transport;

typedef struct {
  int nx, ny, nz;
  double dx, dy, dz;   /* voxel size, cm */
  double ox, oy, oz;   /* corner of voxel (0,0,0), cm */
  const double* rho;   /* g/cm^3, x fastest, length nx*ny*nz */
  const uint8_t* mat;  /* material index per voxel (< the number of tables), or NULL */
  /* test use: a fixed geometric length (cm) of the e+- step cap per voxel,
   * in place of tau_max(E)/rho, so that the derivative checks can hold the
   * step control fixed while densities and energies vary; NULL: tau_max/rho */
  const double* step_cap;
} orc_phantom;

#define ORC_MAX_MAT 4

typedef struct {
  int particle;        /* ORC_PHOTON / ORC_ELECTRON / ORC_POSITRON */
  int kind;            /* ORC_SRC_PENCIL or ORC_SRC_RECT */
  double energy;       /* kinetic energy, MeV */
  double pos[3];       /* pencil position or rectangle centre */
  double dir[3];       /* unit direction */
  double width[2];     /* rectangle full widths along x and y */
  uint64_t n_hist;     /* histories of this source */
} orc_source;

typedef struct {
  uint64_t histories;
  uint64_t flights, compton, photo, rayleigh, pair;
  uint64_t esteps, hard_el, hard_in, hard_br, delta, annih;
  uint64_t crossings, secondaries, deposits;
  uint64_t absorbed, escaped;
  double e_dep, e_esc;
  uint64_t pos_esc;
  uint64_t maj_excess;  /* hard selections whose cross sections exceeded the majorant (must stay 0) */
  uint64_t annih_flight; /* positrons annihilated in flight (counted in annih too) */
} orc_stats;

/* ledger entries written per history when ledger != NULL */
enum { ORC_LED_DEP = 0, ORC_LED_ESC, ORC_LED_POSESC, ORC_LED_PATH, ORC_LED_EABS, ORC_LED_N };

typedef struct orc_tables orc_tables;

/* Build the interpolation tables of one material (returns NULL on bad input). */
orc_tables* orc_tables_create(const orc_material* m, const orc_transport* t);
void orc_tables_destroy(orc_tables* tb);

/* Table channels for orc_eval: 0..3 photon mu (Compton, photo, Rayleigh, pair);
 * 4 + 6*type + c for e-(type 0) / e+(type 1) with c = 0 soft stopping power,
 * 1 range, 2 hard elastic, 3 hard inelastic, 4 hard bremsstrahlung,
 * 5 soft first transport coefficient. */
double orc_eval(const orc_tables* tb, int channel, double e);
double orc_node(const orc_tables* tb, int channel, int i);
double orc_node_energy(const orc_tables* tb, int i);
double orc_range_inverse(const orc_tables* tb, int type, double r);
double orc_sigma_majorant(const orc_tables* tb, int type, double elo, double e);
double orc_screening(const orc_tables* tb, double e);
double orc_elastic_k(const orc_tables* tb, double e);
double orc_mu_cut(const orc_tables* tb, int type, double e);
double orc_soft_a(double mean_mu);
/* d ln p(mu) / d rho of the soft angular law of a Class II step of geometric
 * length len and soft transport coefficient t1s whose mean is mbar and
 * parameter a = orc_soft_a(mbar) (term C of the gradient, see below). */
double orc_soft_score(double a, double mu, double mbar, double len, double t1s);
/* Second moment of the soft energy-loss DCS per unit mass path, MeV^2 cm^2/g,
 * of an electron (type 0) or positron (1) of kinetic energy e: the variance
 * of the soft loss over a path of s g/cm^2 is s times this. */
double orc_soft_omega2(const orc_tables* tb, int type, double e);
/* n soft energy losses of mean m and variance omega2 drawn by the straggling
 * sampler of the Class II step, draw streams (seed, i, uid 1) for i < n. */
int orc_sample_straggle(double m, double omega2, uint32_t seed, int n, double* out);
/* Heitler cross section per gram (cm^2/g) of two-photon annihilation of a
 * positron of kinetic energy e with the material's electrons at rest. */
double orc_sigma_annih(const orc_tables* tb, double e);

/* Raw generators (pinned against published known-answer values). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint64_t orc_splitmix64(uint64_t state);
uint64_t orc_child_uid(uint64_t parent_uid, uint32_t ordinal);
/* n uniforms of the stream (seed, hist, uid) starting at draw 0 */
void orc_uniforms(uint32_t seed, uint32_t hist, uint64_t uid, int n, double* out);

/* Direct sampler access for the distribution tests.  Each sample i uses the
 * stream (seed, hist = i, uid = 1).  Outputs per sample as documented. */
int orc_sample(const orc_tables* tb, int which, double e, uint32_t seed, int n,
               double* out0, double* out1);
enum {
  ORC_SMP_COMPTON = 0,   /* out0 = kappa = E'/E, out1 = cos theta */
  ORC_SMP_RAYLEIGH,      /* out0 = cos theta */
  ORC_SMP_MOLLER,        /* out0 = W/E (electron), out1 = cos theta_primary */
  ORC_SMP_BHABHA,        /* out0 = W/E (positron) */
  ORC_SMP_BREMS,         /* out0 = W, out1 = photon cos theta */
  ORC_SMP_HARD_ELASTIC,  /* out0 = mu = (1 - cos)/2 (electron) */
  ORC_SMP_SOFT,          /* e holds <mu>; out0 = mu */
  ORC_SMP_PAIR,          /* out0 = T-/(E - 2mc^2), out1 = cos theta of e- */
  ORC_SMP_FREE_PATH,     /* out0 = photon mass free path tau (g/cm^2) */
  ORC_SMP_ANNIH,         /* out0 = cos theta of the first photon */
  ORC_SMP_ANNIH_FLIGHT   /* out0 = energy fraction zeta of the softer photon,
                            out1 = its cos theta (the other's follows) */
};

/* Transport histories [first, first + n) of the concatenated sources.
 * sum_q / sum_q2 (length nx*ny*nz, MeV) are ACCUMULATED; stats is
 * accumulated; hashes (n) and ledger (n * ORC_LED_N) are written when non-NULL.
 * Returns 0 or a negative error code. */
/* Several materials (R10): tbs[m] holds the tables of material m, all built
 * on the same grid with the same transport parameters; ph->mat selects one
 * per voxel.  Returns -5 for a material index >= n_mat. */
int orc_run_mm(const orc_tables* const* tbs, int n_mat, const orc_transport* t, const orc_phantom* ph,
               const orc_source* src, int n_src, uint32_t seed, uint64_t first, uint64_t n, double* sum_q,
               double* sum_q2, orc_stats* stats, uint64_t* hashes, double* ledger);
int orc_run(const orc_tables* tb, const orc_transport* t, const orc_phantom* ph,
            const orc_source* src, int n_src, uint32_t seed, uint64_t first,
            uint64_t n, double* sum_q, double* sum_q2, orc_stats* stats,
            uint64_t* hashes, double* ledger);

/* Density gradient of a dose loss, one history at a time (reading A25).
 * w[v] = (dL/dD_v) * 1e6 / (rho_v V) is the loss weight per MeV deposited in
 * voxel v.  Per history h:
 *   Q_h   = sum_v w_v q_hv                       (weighted score of the history)
 *   S_hj  = likelihood-ratio scores d ln p / d rho_j of the history's sampled
 *           variables whose laws depend on rho_j:
 *           photon free flights: -mu l_j per voxel crossed, +1/rho_k where the
 *           flight ends in an interaction (term A, photons);
 *           e+- steps in voxel j: the candidate events of the hard-event
 *           majorant process along the path, -smaj s over the step's length
 *           s, +1/rho_j where the step ends at an event (term A, e+-), and the
 *           soft deflection of the hinge (term C); with
 *           ORC_GRAD_DEFLECTION_ENERGY also -s S(E1) psi for each step (term
 *           E), psi the sum over the particle's later hinges of their
 *           deflection's d ln p / dE times the CSDA chain dE/dE1 back to
 *           this step's end;
 *   P_hj  = pathwise soft-loss terms of the e+- steps in voxel j at fixed
 *           geometric step lengths: l S(E1) (weight w_j - lam), lam the
 *           particle's CSDA energy adjoint after the step (term D);
 * Accumulated: A_j += Q_h S_hj, B_j += S_hj, P_j += P_hj, *sum_q_h += Q_h.
 * The gradient is (A_j - Qbar B_j + P_j)/N - (dL/dD_j) D_j / rho_j (term B),
 * Qbar = sum_q_h / N.  Exact when electrons deposit where they are created;
 * with Class II transport the step cap's geometric length and the majorant
 * are held fixed, and so is the energy dependence of the later sampling laws
 * (hard-event rates and laws, and, without term E, the soft deflection). */
int orc_run_gradient(const orc_tables* tb, const orc_transport* t, const orc_phantom* ph,
                     const orc_source* src, int n_src, uint32_t seed, uint64_t first,
                     uint64_t n, const double* w, double* a_acc, double* b_acc,
                     double* p_acc, double* sum_q_h);
/* The same with several materials (R10): the flight score of voxel j uses
 * its material's mu_m(E), -mu_m l_j, and 1/rho_k where the flight ends;
 * the soft-loss term uses the voxel's material's S_soft. */
int orc_run_gradient_mm(const orc_tables* const* tbs, int n_mat, const orc_transport* t, const orc_phantom* ph,
                        const orc_source* src, int n_src, uint32_t seed, uint64_t first, uint64_t n,
                        const double* w, double* a_acc, double* b_acc, double* p_acc, double* sum_q_h);

/* Dose (eV/g per history) and its standard error from the counters,
 * Eq. (1)-(3) with the square root of Eq. (2) restored. */
void orc_dose(const orc_phantom* ph, uint64_t n_hist, const double* sum_q,
              const double* sum_q2, double* dose, double* sigma);

#ifdef __cplusplus
}
#endif
#endif
