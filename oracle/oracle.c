/*
 * oracle.c -- plain single-thread FP64 CPU reference transport.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written to be read against the
 * paper (arXiv:2003.00796) and the textbook physics it points to, not to be
 * fast: every step is done the direct way, in the order the method states.
 * Compile with -ffp-contract=off so that no multiply-add is fused.
 *
 * Readings (the paper defines physics only by reference to PENELOPE):
 *  R1 one synthetic material, scaled per voxel by its mass density;
 *  R2 photon models: free-electron Klein-Nishina Compton; photoelectric
 *     mu = c (E/Eref)^-p, electron emitted along the photon with T = E;
 *     Rayleigh with F(x) = F0 (1 + a x^2)^-2; pair mu = c ln(E/2mc^2)^2,
 *     uniform energy sharing, leading-term (1 - beta cos)^-2 angles;
 *  R3 electron/positron models: Bethe collision stopping power (no density
 *     effect), Moller / Bhabha hard collisions above Wcc, bremsstrahlung DCS
 *     b/W with hard emission above Wcr, screened-Rutherford elastic DCS with
 *     Moliere screening, PENELOPE-style hard elastic mean free path
 *     lambda_h = max(lambda_el, min(C1 lambda_1, C2 E / S_s));
 *  R4 Class II step: soft energy loss is deterministic (range inversion), or,
 *     with ORC_STRAGGLING, straggled about that value (R8); one hinge per
 *     step at a uniform fraction of the step, soft
 *     angular deflection from a one-parameter (mu + A)^-2 law whose mean
 *     matches the soft transport cross section, hard events by the delta
 *     method with a majorant over the step's energy interval (the log-log
 *     chord of the node sums of the hard cross sections, an upper bound of
 *     their sum); every voxel face ends a step, and the soft loss is charged
 *     where the step ends, over the geometric length travelled (a face
 *     before or after the hinge, or the whole step), so that the energy
 *     along a track is the CSDA energy of the path travelled whatever the
 *     voxel size;
 *  R5 positrons annihilate at rest only;
 *  R6 per-particle counter-based random streams (Philox4x32-10, Salmon et
 *     al. SC'11) keyed by (seed, history) with counter (draw pair, uid), so
 *     the numbers a particle draws do not depend on processing order;
 *  R7 Eq. (2) of the paper lacks the square root: sigma = sqrt((Q2 - Q^2)/N).
 *  R9 two-photon annihilation of positrons in flight (optional): a fourth
 *     hard channel with Heitler's cross section for electrons at rest; the
 *     softer photon's energy fraction drawn from Heitler's DCS, the photon
 *     directions from energy and momentum conservation.
 *  R10 several materials (optional): per-voxel material index, tables per
 *     material on one grid; a photon flight accumulates the optical depth
 *     rho mu_m(E) l voxel by voxel and interacts by the tables of the voxel it
 *     stops in; an e+- step uses the tables of its voxel (every face ends a
 *     step, so a step stays in one material).
 *  R11 interaction forcing (optional variance reduction): the hard inelastic
 *     and bremsstrahlung cross sections are multiplied by F_in, F_br >= 1; a
 *     forced event emits its secondary with weight w/F and changes the
 *     primary (energy loss, deflection) only with probability 1/F, drawn
 *     after the event's azimuth; every particle carries a weight and every
 *     deposit and escape is weighted, so the tallies stay unbiased.
 *  R12 bremsstrahlung splitting (optional variance reduction, S = 1 or 2):
 *     each emission yields S photons of the sampled energy W with weight
 *     w/(F S); the first takes the event's angles, each further one draws
 *     its own polar cosine and azimuth; the primary loses W once.
 *  R8 straggling of the soft energy loss (optional): mean = the CSDA loss over
 *     the step's mass path s, variance = s times the second moment of the
 *     soft part of the energy-loss DCS (Bohr's variance from the leading
 *     free-electron term of the Moller/Bhabha DCS below the collision
 *     cutoff, plus b W^2/2 from the b/W bremsstrahlung DCS below the
 *     radiative cutoff); the distribution is a Gaussian truncated
 *     symmetrically to (0, 2 x mean) when mean > 3 sd, a uniform of the same
 *     mean and variance when sqrt(3) sd < mean <= 3 sd, else a point mass at
 *     0 plus a uniform on (0, w) with the same two moments.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 */
#define MC2 0.51099895000          /* electron rest energy, MeV */
#define R_E 2.8179403262e-13       /* classical electron radius, cm */
#define N_A 6.02214076e23          /* Avogadro constant, 1/mol */
#define ALPHA (1.0 / 137.035999084)/* fine-structure constant */
#define HC 1.23984198e-2           /* h c, MeV Angstrom */
#define PI 3.14159265358979323846
#define INF_D (1.0 / 0.0)

/* ------------------------------------------------------------------------ */
/* Random numbers                                                           */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10: ten rounds of the Philox S-box with the multipliers and
 * Weyl key increments published by Salmon et al. (SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* SplitMix64 (Steele, Lea, Flood, OOPSLA'14): the output for a given state
 * after the golden-gamma increment. */
static uint64_t mix_fin(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
uint64_t orc_splitmix64(uint64_t state) { return mix_fin(state + 0x9E3779B97F4A7C15ull); }

/* uid of the k-th (0-based) secondary a particle creates over its life */
uint64_t orc_child_uid(uint64_t parent_uid, uint32_t ordinal) {
  return orc_splitmix64(parent_uid ^ ((uint64_t)(ordinal + 1u) * 0x9E3779B97F4A7C15ull));
}

typedef struct {
  uint32_t seed, hist;
  uint64_t uid;
  uint32_t ctr; /* index of the next draw */
} stream;

/* Draw d of a particle is 64-bit word (d mod 2) of Philox call d/2 with
 * counter (d/2, uid_lo, uid_hi, 0) and key (seed, hist); the word becomes a
 * double in the open interval (0,1) from its top 53 bits. */
static double draw(stream* s) {
  uint32_t c[4] = {s->ctr >> 1, (uint32_t)s->uid, (uint32_t)(s->uid >> 32), 0u};
  uint32_t k[2] = {s->seed, s->hist};
  uint32_t o[4];
  orc_philox4x32_10(c, k, o);
  uint64_t w = (s->ctr & 1u) ? (((uint64_t)o[3] << 32) | o[2]) : (((uint64_t)o[1] << 32) | o[0]);
  s->ctr++;
  return ((double)(w >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

void orc_uniforms(uint32_t seed, uint32_t hist, uint64_t uid, int n, double* out) {
  stream s = {seed, hist, uid, 0u};
  for (int i = 0; i < n; ++i) out[i] = draw(&s);
}

/* ------------------------------------------------------------------------ */
/* Synthetic analytic cross sections (model formulas, evaluated at nodes)   */
/* ------------------------------------------------------------------------ */

typedef struct {
  double ne;    /* electrons per gram */
  double nmol;  /* molecules per gram */
  orc_material m;
} matc;

/* Klein-Nishina total cross section per free electron (cm^2). */
static double sigma_kn(double e) {
  double k = e / MC2;
  double l = log(1.0 + 2.0 * k);
  double t1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k);
  double t2 = l / (2.0 * k);
  double t3 = (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
  return 2.0 * PI * R_E * R_E * (t1 + t2 - t3);
}

/* Rayleigh: pi r_e^2 n_mol Int_{-1}^{1} (1 + cos^2) F(x)^2 dcos with
 * x^2 = u = U (1 - cos)/2, U = (E/hc)^2, integrated in closed form in u. */
static double mu_rayleigh(const matc* mc, double e) {
  double a = mc->m.ray_a;
  double U = (e / HC) * (e / HC);
  double T = 1.0 + a * U;
  double i0 = -expm1(-3.0 * log1p(a * U)) / (3.0 * a);
  double i1 = (1.0 / 6.0 - 1.0 / (2.0 * T * T) + 1.0 / (3.0 * T * T * T)) / (a * a);
  double i2 = (1.0 / 3.0 - 1.0 / T + 1.0 / (T * T) - 1.0 / (3.0 * T * T * T)) / (a * a * a);
  double integral = 2.0 * i0 - 4.0 * i1 / U + 4.0 * i2 / (U * U);
  return mc->nmol * PI * R_E * R_E * mc->m.ray_f0 * mc->m.ray_f0 * (2.0 / U) * integral;
}

typedef struct {
  double beta2, gamma, pv;
} kin;

static kin kinematics(double t) {
  kin k;
  double etot = t + MC2;
  double p2 = t * (t + 2.0 * MC2);
  k.gamma = etot / MC2;
  k.beta2 = p2 / (etot * etot);
  k.pv = p2 / etot;
  return k;
}

/* Bethe collision stopping power, no density effect; F- (electrons) and F+
 * (positrons) as in ICRU Report 37. */
static double s_col(const matc* mc, int type, double t) {
  kin k = kinematics(t);
  double tau = t / MC2;
  double iratio = mc->m.i_exc / MC2;
  double f;
  if (type == 0) {
    f = 1.0 - k.beta2 + (tau * tau / 8.0 - (2.0 * tau + 1.0) * log(2.0)) / ((tau + 1.0) * (tau + 1.0));
  } else {
    double y = tau + 2.0;
    f = 2.0 * log(2.0) - (k.beta2 / 12.0) * (23.0 + 14.0 / y + 10.0 / (y * y) + 4.0 / (y * y * y));
  }
  double lg = log(tau * tau * (tau + 2.0) / (2.0 * iratio * iratio));
  return 2.0 * PI * R_E * R_E * MC2 * mc->ne / k.beta2 * (lg + f);
}

/* Moller (electron) and Bhabha (positron) DCS brackets, in kappa = W/T:
 *   dsigma/dkappa = 2 pi r_e^2 mc^2 / (beta^2 T) * bracket(kappa).
 * Moller:  1/k^2 + 1/(1-k)^2 + a - (1-a)/(k(1-k)),  a = ((g-1)/g)^2,
 *          kappa in [kc, 1/2];
 * Bhabha:  (1/k^2) (1 - b1 k + b2 k^2 - b3 k^3 + b4 k^4), kappa in [kc, 1],
 *          b1..b4 as in ICRU Report 37 / the PENELOPE manual. */
typedef struct {
  double a, b1, b2, b3, b4;
} inel_coef;

static inel_coef inel_coefficients(double t) {
  inel_coef c;
  double g = 1.0 + t / MC2;
  double a = ((g - 1.0) / g) * ((g - 1.0) / g);
  double gp = g + 1.0;
  c.a = a;
  c.b1 = a * (2.0 * gp * gp - 1.0) / (g * g - 1.0);
  c.b2 = a * (3.0 * gp * gp + 1.0) / (gp * gp);
  c.b3 = a * 2.0 * (g - 1.0) * g / (gp * gp);
  c.b4 = a * (g - 1.0) * (g - 1.0) / (gp * gp);
  return c;
}

/* hard inelastic cross section (cm^2/g) and hard stopping (MeV cm^2/g):
 * closed-form integrals of the brackets above over the hard range. */
static void hard_inelastic(const matc* mc, int type, double t, double wcc, double* sig, double* shard) {
  *sig = 0.0;
  *shard = 0.0;
  kin k = kinematics(t);
  double kc = wcc / t;
  double pref = 2.0 * PI * R_E * R_E * MC2 * mc->ne / k.beta2;
  inel_coef c = inel_coefficients(t);
  if (type == 0) {
    if (!(t > 2.0 * wcc)) return;
    double b = 1.0 - c.a;
    double i0 = 1.0 / kc - 1.0 / (1.0 - kc) + c.a * (0.5 - kc) - b * log((1.0 - kc) / kc);
    double i1 = log(1.0 / (2.0 * kc)) + 2.0 - log(2.0) - 1.0 / (1.0 - kc) - log(1.0 - kc) +
                c.a * (0.125 - 0.5 * kc * kc) - b * log(2.0 * (1.0 - kc));
    *sig = pref / t * i0;
    *shard = pref * i1;
  } else {
    if (!(t > wcc)) return;
    double i0 = (1.0 / kc - 1.0) - c.b1 * log(1.0 / kc) + c.b2 * (1.0 - kc) -
                c.b3 * (1.0 - kc * kc) / 2.0 + c.b4 * (1.0 - kc * kc * kc) / 3.0;
    double i1 = log(1.0 / kc) - c.b1 * (1.0 - kc) + c.b2 * (1.0 - kc * kc) / 2.0 -
                c.b3 * (1.0 - kc * kc * kc) / 3.0 + c.b4 * (1.0 - kc * kc * kc * kc) / 4.0;
    *sig = pref / t * i0;
    *shard = pref * i1;
  }
}

/* Moliere screening parameter eta(T) of the screened Rutherford DCS
 * dsigma/dmu = K / (mu + eta)^2, mu = (1 - cos)/2. */
static double screening(const matc* mc, double t) {
  kin k = kinematics(t);
  double zs = mc->m.z_screen;
  double p2 = t * (t + 2.0 * MC2);
  double c = ALPHA * cbrt(zs) / 0.885;
  double az = ALPHA * zs;
  return 0.25 * c * c * (MC2 * MC2 / p2) * (1.13 + 3.76 * az * az / k.beta2);
}

static double elastic_k(const matc* mc, double t) {
  kin k = kinematics(t);
  double q = R_E * MC2 / k.pv;
  return mc->nmol * PI * q * q * mc->m.zz1_mol;
}

/* ------------------------------------------------------------------------ */
/* Tables                                                                   */
/* ------------------------------------------------------------------------ */

enum { CH_S = 0, CH_R, CH_EL, CH_IN, CH_BR, CH_T1S, N_ECH };

struct orc_tables {
  int n;
  double lemin, dl;
  double* e;           /* node energies */
  double* ph[4];       /* photon mass coefficients */
  double* el[2][N_ECH];/* electron, positron */
  double thr_ph[4];    /* threshold energies (0 = none) */
  double thr_el[2][N_ECH];
  matc mc;
  orc_transport t;
};

void orc_tables_destroy(orc_tables* tb) {
  if (!tb) return;
  free(tb->e);
  for (int c = 0; c < 4; ++c) free(tb->ph[c]);
  for (int p = 0; p < 2; ++p)
    for (int c = 0; c < N_ECH; ++c) free(tb->el[p][c]);
  free(tb);
}

/* node index and fractional log-coordinate of energy e */
static int grid_pos(const orc_tables* tb, double e, double* f) {
  double x = (log(e) - tb->lemin) / tb->dl;
  double fl = floor(x);
  int i;
  if (fl < 0.0) i = 0;
  else if (fl > (double)(tb->n - 2)) i = tb->n - 2;
  else i = (int)fl;
  *f = x - (double)i;
  return i;
}

/* Piecewise power law between positive nodes; on a segment whose lower node
 * is zero (a threshold channel), linear in E from the exact threshold. */
static double interp(const orc_tables* tb, const double* y, double thr, double e) {
  if (thr > 0.0 && !(e > thr)) return 0.0;
  double f;
  int i = grid_pos(tb, e, &f);
  double y0 = y[i], y1 = y[i + 1];
  if (y0 > 0.0 && y1 > 0.0) return y0 * pow(y1 / y0, f);
  if (y1 > 0.0) {
    double lo = thr > tb->e[i] ? thr : tb->e[i];
    return y1 * (e - lo) / (tb->e[i + 1] - lo);
  }
  return 0.0;
}

/* integral of 1/S over [e0, e] on one power-law segment of S */
static double seg_range(double e0, double s0, double b, double e) {
  double q = 1.0 - b;
  if (fabs(q) < 1e-10) return (e0 / s0) * log(e / e0);
  return (e0 / s0) * (pow(e / e0, q) - 1.0) / q;
}

static double seg_slope(const orc_tables* tb, const double* s, int i) {
  return log(s[i + 1] / s[i]) / log(tb->e[i + 1] / tb->e[i]);
}

static double range_of(const orc_tables* tb, int type, double e) {
  const double* s = tb->el[type][CH_S];
  const double* r = tb->el[type][CH_R];
  double f;
  int i = grid_pos(tb, e, &f);
  return r[i] + seg_range(tb->e[i], s[i], seg_slope(tb, s, i), e);
}

double orc_range_inverse(const orc_tables* tb, int type, double rr) {
  const double* s = tb->el[type][CH_S];
  const double* r = tb->el[type][CH_R];
  if (!(rr > 0.0)) return tb->e[0];
  /* the segment i with r[i] <= rr < r[i+1] (last segment extrapolates) */
  int lo = 0, hi = tb->n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (r[mid] <= rr) lo = mid;
    else hi = mid;
  }
  int i = lo;
  double b = seg_slope(tb, s, i);
  double q = 1.0 - b;
  double e0 = tb->e[i];
  double d = rr - r[i];
  if (fabs(q) < 1e-10) return e0 * exp(d * s[i] / e0);
  return e0 * pow(1.0 + d * q * s[i] / e0, 1.0 / q);
}

orc_tables* orc_tables_create(const orc_material* m, const orc_transport* t) {
  if (!m || !t || t->n_grid < 4 || !(t->e_min > 0.0) || !(t->e_max > t->e_min)) return NULL;
  orc_tables* tb = (orc_tables*)calloc(1, sizeof(orc_tables));
  int n = t->n_grid;
  tb->n = n;
  tb->t = *t;
  tb->mc.m = *m;
  tb->mc.ne = N_A * m->z_mol / m->a_mol;
  tb->mc.nmol = N_A / m->a_mol;
  tb->lemin = log(t->e_min);
  tb->dl = (log(t->e_max) - tb->lemin) / (double)(n - 1);
  tb->e = (double*)malloc(sizeof(double) * n);
  for (int c = 0; c < 4; ++c) tb->ph[c] = (double*)calloc(n, sizeof(double));
  for (int p = 0; p < 2; ++p)
    for (int c = 0; c < N_ECH; ++c) tb->el[p][c] = (double*)calloc(n, sizeof(double));
  for (int i = 0; i < n; ++i) tb->e[i] = t->e_min * exp((double)i * tb->dl);

  const matc* mc = &tb->mc;
  uint32_t fl = t->flags;
  tb->thr_ph[3] = 2.0 * MC2;
  for (int i = 0; i < n; ++i) {
    double e = tb->e[i];
    tb->ph[0][i] = (fl & ORC_NO_COMPTON) ? 0.0 : mc->ne * sigma_kn(e);
    tb->ph[1][i] = (fl & ORC_NO_PHOTO) ? 0.0 : m->pe_coef * pow(e / m->pe_eref, -m->pe_exp);
    tb->ph[2][i] = (fl & ORC_NO_RAYLEIGH) ? 0.0 : mu_rayleigh(mc, e);
    if (!(fl & ORC_NO_PAIR) && e > 2.0 * MC2) {
      double l = log(e / (2.0 * MC2));
      tb->ph[3][i] = m->pp_coef * l * l;
    }
  }
  for (int p = 0; p < 2; ++p) {
    tb->thr_el[p][CH_IN] = p == 0 ? 2.0 * t->wcc : t->wcc;
    tb->thr_el[p][CH_BR] = t->wcr;
    for (int i = 0; i < n; ++i) {
      double e = tb->e[i];
      double sc = s_col(mc, p, e);
      double sig_in = 0.0, s_hin = 0.0;
      if (!(fl & ORC_NO_HARD_INELASTIC)) hard_inelastic(mc, p, e, t->wcc, &sig_in, &s_hin);
      double s_rad_soft, sig_br = 0.0;
      if (fl & ORC_NO_HARD_BREMS) {
        s_rad_soft = m->brems_b * e;
      } else {
        s_rad_soft = m->brems_b * (e < t->wcr ? e : t->wcr);
        if (e > t->wcr) sig_br = m->brems_b * log(e / t->wcr);
      }
      double ss = sc - s_hin + s_rad_soft;
      double kk = elastic_k(mc, e);
      double eta = screening(mc, e);
      double sig_el = kk / (eta * (1.0 + eta));
      double sig1 = 2.0 * kk * (log((1.0 + eta) / eta) - 1.0 / (1.0 + eta));
      double sig_h, sig1s;
      if (fl & ORC_NO_HARD_ELASTIC) {
        sig_h = 0.0;
        sig1s = sig1;
      } else {
        double lam_el = 1.0 / sig_el, lam1 = 1.0 / sig1;
        double cap = t->c1 * lam1;
        double lam_s = t->c2 * e / ss;
        if (lam_s < cap) cap = lam_s;
        double lam_h = lam_el > cap ? lam_el : cap;
        sig_h = 1.0 / lam_h;
        double muc = 1.0 / (sig_h / kk + 1.0 / (1.0 + eta)) - eta;
        if (muc < 0.0) muc = 0.0;
        if (muc > 1.0) muc = 1.0;
        sig1s = 2.0 * kk * (log((muc + eta) / eta) - muc / (muc + eta));
      }
      tb->el[p][CH_S][i] = ss;
      tb->el[p][CH_EL][i] = sig_h;
      /* R11: forced channels (the soft stopping power above stays analog) */
      tb->el[p][CH_IN][i] = t->force_in > 1.0 ? sig_in * t->force_in : sig_in;
      tb->el[p][CH_BR][i] = t->force_br > 1.0 ? sig_br * t->force_br : sig_br;
      tb->el[p][CH_T1S][i] = sig1s;
    }
    /* range: exact integral of 1/S over the piecewise power-law S */
    double* s = tb->el[p][CH_S];
    double* r = tb->el[p][CH_R];
    r[0] = 0.0;
    for (int i = 0; i + 1 < n; ++i) r[i + 1] = r[i] + seg_range(tb->e[i], s[i], seg_slope(tb, s, i), tb->e[i + 1]);
  }
  for (int p = 0; p < 2; ++p)
    for (int i = 0; i < n; ++i)
      if (!(tb->el[p][CH_S][i] > 0.0)) { orc_tables_destroy(tb); return NULL; }
  return tb;
}

double orc_eval(const orc_tables* tb, int ch, double e) {
  if (ch < 4) return interp(tb, tb->ph[ch], tb->thr_ph[ch], e);
  int p = (ch - 4) / N_ECH, c = (ch - 4) % N_ECH;
  if (p < 0 || p > 1) return NAN;
  if (c == CH_R) return range_of(tb, p, e);
  return interp(tb, tb->el[p][c], tb->thr_el[p][c], e);
}

double orc_node(const orc_tables* tb, int ch, int i) {
  if (ch < 4) return tb->ph[ch][i];
  return tb->el[(ch - 4) / N_ECH][(ch - 4) % N_ECH][i];
}
double orc_node_energy(const orc_tables* tb, int i) { return tb->e[i]; }
double orc_screening(const orc_tables* tb, double e) { return screening(&tb->mc, e); }
double orc_elastic_k(const orc_tables* tb, double e) { return elastic_k(&tb->mc, e); }

static double sig_hard(const orc_tables* tb, int p, double e) {
  return interp(tb, tb->el[p][CH_EL], 0.0, e) + interp(tb, tb->el[p][CH_IN], tb->thr_el[p][CH_IN], e) +
         interp(tb, tb->el[p][CH_BR], tb->thr_el[p][CH_BR], e);
}

/* ln of the node sum H_j of the three hard cross sections, and the same or
 * -inf where segment j starts a channel's threshold (zero at node j,
 * positive at node j + 1) */
static double lnh(const orc_tables* tb, int p, int j) {
  return log(tb->el[p][CH_EL][j] + tb->el[p][CH_IN][j] + tb->el[p][CH_BR][j]);
}
static double lnh_chord(const orc_tables* tb, int p, int j) {
  const int ch[3] = {CH_EL, CH_IN, CH_BR};
  for (int k = 0; k < 3; ++k)
    if (!(tb->el[p][ch[k]][j] > 0.0) && tb->el[p][ch[k]][j + 1] > 0.0) return -INFINITY;
  return lnh(tb, p, j);
}

/* Upper bound of the hard cross section at e.  On a segment without a
 * threshold every channel is a power law, so ln of their sum is a
 * log-sum-exp of affine functions of ln E, convex, and lies below its chord:
 * exp of the log-log chord of the node sums bounds the sum.  On a threshold
 * segment, the sum itself. */
static double sig_hard_bound(const orc_tables* tb, int p, double e) {
  double f;
  int i = grid_pos(tb, e, &f);
  double l0 = lnh_chord(tb, p, i);
  if (l0 > -INFINITY) return exp(l0 + f * (lnh(tb, p, i + 1) - l0));
  return sig_hard(tb, p, e);
}

/* Majorant of the hard cross section over [elo, e]: the maximum of the bound
 * above, which is monotone on each segment (exp of a linear function of ln E;
 * on a threshold segment a convex function of ln E, as every channel is), so
 * it is attained at elo, e or a node in between. */
double orc_sigma_majorant(const orc_tables* tb, int p, double elo, double e) {
  double m = sig_hard_bound(tb, p, e);
  double a = sig_hard_bound(tb, p, elo);
  if (a > m) m = a;
  for (int j = 0; j < tb->n; ++j) {
    double ej = tb->e[j];
    if (ej > elo && ej < e) {
      double v = tb->el[p][CH_EL][j] + tb->el[p][CH_IN][j] + tb->el[p][CH_BR][j];
      if (v > m) m = v;
    }
  }
  return m;
}

/* cutoff mu_c of the hard elastic events: K (1/(mu_c+eta) - 1/(1+eta)) = sigma_h */
double orc_mu_cut(const orc_tables* tb, int p, double e) {
  double kk = elastic_k(&tb->mc, e);
  double eta = screening(&tb->mc, e);
  double sh = interp(tb, tb->el[p][CH_EL], 0.0, e);
  double muc = 1.0 / (sh / kk + 1.0 / (1.0 + eta)) - eta;
  if (muc < 0.0) muc = 0.0;
  if (muc > 1.0) muc = 1.0;
  return muc;
}

/* Soft angular law p(mu) ~ (mu + A)^-2 on [0,1]; its mean is
 * A (1 + A) ln((1 + A)/A) - A, increasing from 0 to 1/2.  Plain bisection in
 * ln A for the A whose mean equals <mu> (clamped to 0.49). */
static double soft_mean(double a) { return a * ((1.0 + a) * log1p(1.0 / a) - 1.0); }

double orc_soft_a(double mbar) {
  if (!(mbar > 0.0)) return 0.0;
  if (mbar > 0.49) mbar = 0.49;
  double lo = log(1e-300), hi = log(1e6); /* mean(1e6) > 0.49 */
  for (int it = 0; it < 400 && hi - lo > 1e-15 * (fabs(lo) + fabs(hi) + 1.0) * 0.5; ++it) {
    double mid = 0.5 * (lo + hi);
    if (soft_mean(exp(mid)) < mbar) lo = mid;
    else hi = mid;
  }
  return exp(0.5 * (lo + hi));
}

/* Soft energy-loss straggling (R8).  Second moment of the soft DCS per unit
 * mass path: the leading term 2 pi r_e^2 mc^2 n_e / (beta^2 W^2) of the
 * binary-collision DCS times W^2, integrated over (0, Wc], gives
 * 2 pi r_e^2 mc^2 n_e Wc / beta^2 (Bohr); b/W times W^2 over (0, Wr] gives
 * b Wr^2 / 2.  Wc = min(Wcc, W_max), W_max = E/2 (e-) or E (e+), and W_max
 * itself when hard inelastic events are off; Wr = min(Wcr, E), or E when
 * hard bremsstrahlung is off. */
double orc_soft_omega2(const orc_tables* tb, int type, double e) {
  const orc_transport* t = &tb->t;
  double p2 = e * (e + 2.0 * MC2);
  double et = e + MC2;
  double beta2 = p2 / (et * et);
  double wmax = type == 1 ? e : 0.5 * e;
  double wc = wmax;
  if (!(t->flags & ORC_NO_HARD_INELASTIC) && t->wcc < wmax) wc = t->wcc;
  double wr = e;
  if (!(t->flags & ORC_NO_HARD_BREMS) && t->wcr < e) wr = t->wcr;
  double k = 2.0 * PI * R_E * R_E * MC2 * tb->mc.ne;
  return k * wc / beta2 + 0.5 * tb->mc.m.brems_b * wr * wr;
}

/* one soft energy loss of mean m and variance om2 (R8).  Whether and how
 * many numbers are drawn must not hinge on m alone: a zero path can give a
 * CSDA loss of 0 or of a rounding residue, depending on how the range is
 * inverted.  So a zero variance (zero path) draws nothing, and m = 0 with a
 * positive variance falls in the two-mode branch, which returns 0. */
static double straggle(stream* s, double m, double om2) {
  if (!(om2 > 0.0)) return m;
  double m2 = m * m;
  if (m2 > 9.0 * om2) {
    /* Gaussian (Box-Muller, the cosine branch), truncated symmetrically
     * about m to (0, 2m) by rejection: the mean stays m */
    double om = sqrt(om2);
    for (;;) {
      double r = sqrt(-2.0 * log(draw(s)));
      double w = m + om * r * cos(2.0 * PI * draw(s));
      if (w > 0.0 && w < 2.0 * m) return w;
    }
  }
  /* uniform on m -/+ sqrt(3) sd: mean m, variance om2 */
  if (m2 > 3.0 * om2) return m + sqrt(3.0 * om2) * (2.0 * draw(s) - 1.0);
  /* 0 with probability a, else uniform on (0, w): a and w from the mean m
   * and the second moment s2 = om2 + m^2 (mean (1-a) w/2, second moment
   * (1-a) w^2/3) */
  double s2 = om2 + m2;
  double a = 1.0 - 4.0 * m2 / (3.0 * s2);
  double u = draw(s);
  return u < a ? 0.0 : 1.5 * s2 / m * (u - a) / (1.0 - a);
}

/* ------------------------------------------------------------------------ */
/* Geometry: constant LOCATE and STEP on the voxel grid (Sec. 4.2.2)         */
/* ------------------------------------------------------------------------ */

typedef struct {
  int type;
  double x[3], d[3], e;
  int ix[3];
  stream rng;
  uint32_t nchild;
  uint64_t hash;
  double w;  /* statistical weight (R11) */
  /* e+-: the majorant optical depth left before the next hard or delta event
   * (R4); 0 when none is pending (a new particle, or right after an event) */
  double clk;
} part;

typedef struct {
  const orc_tables* tb;
  const orc_tables* tbm[ORC_MAX_MAT];  /* tables per material (R10) */
  const uint8_t* mat;                  /* per-voxel material, NULL: tb everywhere */
  const orc_transport* t;
  const orc_phantom* ph;
  int n[3];
  double dx[3], o[3];
  /* per-history sparse score: tmp[v] valid when mark[v] == current history */
  double* tmp;
  uint64_t* mark;
  int64_t* touched;
  int64_t n_touched;
  uint64_t cur;
  part* stack;
  int sp, cap;
  orc_stats* st;
  double led[ORC_LED_N];
  uint64_t hist_hash;
  /* gradient (score-function) accumulation, NULL when off */
  const double* w;
  double q_h;           /* sum_v w_v q_hv of the current history */
  double* s_tmp;        /* per-history score S_hj, valid where s_mark == cur */
  uint64_t* s_mark;
  int64_t* s_touched;
  int64_t n_s_touched;
  double* p_acc;
  /* the current e+- particle's steps, for the backward sweep of its energy
   * adjoint when it ends (gradient mode) */
  struct elog_rec { int64_t v; double coef, r, d, se; }* elog;
  int n_elog, cap_elog;
} ctx;

static int64_t lin(const ctx* c, const int ix[3]) {
  return ((int64_t)ix[2] * c->n[1] + ix[1]) * c->n[0] + ix[0];
}

/* distance to the exit face of the current voxel; ties go to x, then y, z */
static double face(const ctx* c, const part* p, int* axis) {
  double best = INF_D;
  int a = -1;
  for (int k = 0; k < 3; ++k) {
    double s;
    if (p->d[k] > 0.0) s = (c->o[k] + (double)(p->ix[k] + 1) * c->dx[k] - p->x[k]) / p->d[k];
    else if (p->d[k] < 0.0) s = (c->o[k] + (double)p->ix[k] * c->dx[k] - p->x[k]) / p->d[k];
    else continue;
    if (s < 0.0) s = 0.0;
    if (s < best) { best = s; a = k; }
  }
  *axis = a;
  return best;
}

static void move(part* p, double s) {
  for (int k = 0; k < 3; ++k) p->x[k] = p->x[k] + s * p->d[k];
}

/* move s to the face on axis a, snap onto the face, step the index;
 * returns 1 if the particle left the grid */
static int cross(const ctx* c, part* p, double s, int a) {
  double fv = p->d[a] > 0.0 ? c->o[a] + (double)(p->ix[a] + 1) * c->dx[a] : c->o[a] + (double)p->ix[a] * c->dx[a];
  move(p, s);
  p->x[a] = fv;
  p->ix[a] += p->d[a] > 0.0 ? 1 : -1;
  c->st->crossings++;
  return p->ix[a] < 0 || p->ix[a] >= c->n[a];
}

/* direction after polar deflection cos_t and azimuth phi */
static void rotate(double d[3], double cost, double phi) {
  double s2t = 1.0 - cost * cost;
  double sint = s2t > 0.0 ? sqrt(s2t) : 0.0;
  double cp = cos(phi), sp = sin(phi);
  double u = d[0], v = d[1], w = d[2];
  double s2 = 1.0 - w * w;
  double nu, nv, nw;
  if (s2 > 1e-10) {
    double s = sqrt(s2);
    nu = u * cost + sint * (u * w * cp - v * sp) / s;
    nv = v * cost + sint * (v * w * cp + u * sp) / s;
    nw = w * cost - s * sint * cp;
  } else {
    nu = sint * cp;
    nv = sint * sp;
    nw = w > 0.0 ? cost : -cost;
  }
  double nn = sqrt(nu * nu + nv * nv + nw * nw);
  d[0] = nu / nn;
  d[1] = nv / nn;
  d[2] = nw / nn;
}

/* ------------------------------------------------------------------------ */
/* Tally and event record                                                   */
/* ------------------------------------------------------------------------ */

static void deposit(ctx* c, const part* p, double e) {
  if (e == 0.0) return;
  int64_t v = lin(c, p->ix);
  if (c->mark[v] != c->cur) {
    c->mark[v] = c->cur;
    c->tmp[v] = 0.0;
    c->touched[c->n_touched++] = v;
  }
  e *= p->w;
  c->tmp[v] += e;
  c->led[ORC_LED_DEP] += e;
  c->st->deposits++;
  if (c->w) c->q_h += c->w[v] * e;
}

/* score of voxel v for the current history (gradient mode only) */
static void score(ctx* c, int64_t v, double s) {
  if (c->s_mark[v] != c->cur) {
    c->s_mark[v] = c->cur;
    c->s_tmp[v] = 0.0;
    c->s_touched[c->n_s_touched++] = v;
  }
  c->s_tmp[v] += s;
}

/* ------------------------------------------------------------------------ */
/* Density gradient of the Class II step (reading A25: the terms below, with  */
/* the step control held at its geometric value)                             */
/* ------------------------------------------------------------------------ */

/* Term C: d ln p(mu) / d rho of the soft angular law.  p(mu) = A (1 + A) /
 * (mu + A)^2 on [0, 1] has the mean m(A) = A (1 + A) ln(1 + 1/A) - A, and A is
 * chosen so that m(A) = <mu> = (1 - exp(-x))/2 with x = rho len t1s, the
 * step's soft transport at its geometric length len.  So
 *   d ln p / d rho = [1/A + 1/(1 + A) - 2/(mu + A)] (d<mu>/d rho) / m'(A),
 *   d<mu>/d rho = len t1s exp(-x) / 2 = len t1s (1/2 - <mu>),
 *   m'(A) = (1 + 2A) ln(1 + 1/A) - 2 > 0.
 * Where A is held at its bound (<mu> > 0.49) or vanishes, A does not move
 * with rho and the term is 0. */
double orc_soft_score(double a, double mu, double mbar, double len, double t1s) {
  if (!(a > 0.0) || mbar > 0.49) return 0.0;
  double dmean = len * t1s * (0.5 - mbar); /* = len t1s exp(-x) / 2 */
  double dm_da = (1.0 + 2.0 * a) * log1p(1.0 / a) - 2.0;
  return (1.0 / a + 1.0 / (1.0 + a) - 2.0 / (mu + a)) * dmean / dm_da;
}

/* Pathwise term of the soft energy loss.  A step of the current e+- particle
 * in voxel v loses E - E1 over the mass path rho l (l geometric: the length
 * travelled to the face that ends the step, or the whole step).  At fixed l, d(E - E1)/d rho =
 * l S(E1) (the range is R(E1) = R(E) - rho l, R' = 1/S), and E1 = E - loss
 * moves every later step of the particle: dE1/dE = S(E1)/S(E) = r.  The
 * derivative of the particle's weighted deposits from the start of step k
 * with respect to its energy there, lam_k (the energy adjoint in the CSDA
 * chain: hard events subtract fixed energies, secondaries keep theirs),
 * obeys lam_k = d_k (1 - r_k) + r_k lam_{k+1}, d_k = weight x w_v of step k's
 * voxel, ending at weight x w_v where the particle is absorbed and 0 where it
 * escapes or annihilates in flight.  Each step adds l S(E1) (d_k - lam_{k+1})
 * to voxel v: the loss it deposits there minus what the particle then lacks
 * downstream.  The steps are logged and swept backward at the particle's
 * end.
 *
 * Term E (ORC_GRAD_DEFLECTION_ENERGY): the soft deflection drawn at the hinge
 * of step k has a law that depends on the particle's energy E_k there
 * (through the soft transport coefficient t1s(E_k)), and E_k moves with the
 * density of every earlier step: dE_k/d rho_j = -l_j S(E1_j) times the chain
 * factors r of the steps between.  Its likelihood-ratio score is
 * se_k = d ln p(mu_k)/dE_k = (term C of the step) rho (d ln t1s/dE)(E_k), and
 * psi_j = se_{j+1} + r_{j+1} psi_{j+1} (0 after the last step) collects the
 * later hinges; step j adds -l_j S(E1_j) psi_j to the history's score of its
 * voxel. */
static void elog_push(ctx* c, int64_t v, double coef, double r, double d, double se) {
  if (c->n_elog == c->cap_elog) {
    c->cap_elog = c->cap_elog ? 2 * c->cap_elog : 256;
    c->elog = (struct elog_rec*)realloc(c->elog, sizeof(*c->elog) * (size_t)c->cap_elog);
  }
  c->elog[c->n_elog].v = v;
  c->elog[c->n_elog].coef = coef;
  c->elog[c->n_elog].r = r;
  c->elog[c->n_elog].d = d;
  c->elog[c->n_elog].se = se;
  c->n_elog++;
}

static void elog_close(ctx* c, double lam_end) {
  double lam = lam_end, psi = 0.0;
  for (int k = c->n_elog - 1; k >= 0; --k) {
    const struct elog_rec* e = &c->elog[k];
    c->p_acc[e->v] += e->coef * (e->d - lam);
    if (psi != 0.0) score(c, e->v, -e->coef * psi);
    lam = e->d * (1.0 - e->r) + e->r * lam;
    psi = e->se + e->r * psi;
  }
  c->n_elog = 0;
}

/* event codes folded into the particle hash */
enum {
  EV_COMPTON = 1, EV_PHOTO = 2, EV_RAYLEIGH = 3, EV_PAIR = 4, EV_PH_ESCAPE = 5,
  EV_CROSS = 6, EV_STEP = 7, EV_HARD_EL = 8, EV_HARD_IN = 9, EV_HARD_BR = 10,
  EV_ABSORB = 11, EV_E_ESCAPE = 12, EV_ANNIH_FLIGHT = 13
};

static void event(const ctx* c, part* p, int code, int64_t v) {
  uint64_t word = (uint64_t)code | ((uint64_t)(uint32_t)v << 8) | ((uint64_t)(p->nchild & 0xFFFFFFu) << 40);
  p->hash = mix_fin(p->hash + word);
  (void)c;
}

static void finish(ctx* c, part* p) { c->hist_hash += mix_fin(p->hash ^ p->rng.uid); }

static void push(ctx* c, const part* p) {
  if (c->sp == c->cap) {
    c->cap = c->cap ? 2 * c->cap : 64;
    c->stack = (part*)realloc(c->stack, sizeof(part) * (size_t)c->cap);
  }
  c->stack[c->sp++] = *p;
}

/* A new secondary of parent p: takes the next ordinal; pushed if above its
 * absorption energy (positrons always, so that they annihilate), otherwise
 * its kinetic energy is deposited on the spot. */
static void secondary(ctx* c, part* p, int type, double e, const double d[3]) {
  uint32_t k = p->nchild++;
  c->st->secondaries++;
  if (type != ORC_POSITRON && !(e > c->t->eabs[type])) {
    deposit(c, p, e);
    return;
  }
  part s;
  memset(&s, 0, sizeof(s));
  s.type = type;
  memcpy(s.x, p->x, sizeof(s.x));
  memcpy(s.ix, p->ix, sizeof(s.ix));
  s.d[0] = d[0]; s.d[1] = d[1]; s.d[2] = d[2];
  s.e = e;
  s.rng.seed = p->rng.seed;
  s.rng.hist = p->rng.hist;
  s.rng.uid = orc_child_uid(p->rng.uid, k);
  s.rng.ctr = 0;
  s.w = p->w;
  push(c, &s);
}

/* cos theta from p(cos) ~ (1 - beta cos)^-2 on [-1,1] by inversion */
static double leading_angle(double beta, double xi) {
  return (2.0 * xi - 1.0 + beta) / (2.0 * beta * xi + 1.0 - beta);
}

static double beta_of(double t) {
  return sqrt(t * (t + 2.0 * MC2)) / (t + MC2);
}

/* ------------------------------------------------------------------------ */
/* Photon KNOCK                                                             */
/* ------------------------------------------------------------------------ */

/* Klein-Nishina by composition and rejection (Butcher and Messel 1960):
 * branch 1/kappa with weight ln(1/kmin), branch kappa with weight
 * (1 - kmin^2)/2, accept with 1 - kappa sin^2/(1 + kappa^2). */
static double sample_kn(stream* s, double e, double* cost) {
  double k = e / MC2;
  double kmin = 1.0 / (1.0 + 2.0 * k);
  double a1 = log(1.0 + 2.0 * k);
  double a2 = 0.5 * (1.0 - kmin * kmin);
  double kap, ct;
  for (;;) {
    double ub = draw(s), ux = draw(s), ua = draw(s);
    if (ub * (a1 + a2) < a1) kap = exp(-ux * a1);
    else kap = sqrt(kmin * kmin + ux * (1.0 - kmin * kmin));
    ct = 1.0 - (1.0 - kap) / (k * kap);
    if (ct < -1.0) ct = -1.0;
    if (ct > 1.0) ct = 1.0;
    double g = 1.0 - kap * (1.0 - ct * ct) / (1.0 + kap * kap);
    if (ua <= g) break;
  }
  *cost = ct;
  return kap;
}

/* Rayleigh: u = x^2 from F^2 ~ (1 + a u)^-4 on [0, U] by inversion, then
 * accept with (1 + cos^2)/2. */
static double sample_rayleigh(const orc_tables* tb, stream* s, double e) {
  double a = tb->mc.m.ray_a;
  double U = (e / HC) * (e / HC);
  double c3 = -expm1(-3.0 * log1p(a * U)); /* 1 - (1 + aU)^-3 */
  for (;;) {
    double xi = draw(s), ua = draw(s);
    double u = expm1(-log1p(-xi * c3) / 3.0) / a;
    double ct = 1.0 - 2.0 * u / U;
    if (ct < -1.0) ct = -1.0;
    if (ua <= 0.5 * (1.0 + ct * ct)) return ct;
  }
}

/* tables of voxel v's material */
static const orc_tables* tables_at(const ctx* c, int64_t v) { return c->mat ? c->tbm[c->mat[v]] : c->tb; }

static void photon_knock(ctx* c, part* p, int ch) {
  orc_stats* st = c->st;
  int64_t v = lin(c, p->ix);
  const double* eabs = c->t->eabs;
  if (ch == 0) {
    st->compton++;
    double cost;
    double kap = sample_kn(&p->rng, p->e, &cost);
    double phi = 2.0 * PI * draw(&p->rng);
    double d0[3] = {p->d[0], p->d[1], p->d[2]};
    rotate(p->d, cost, phi);
    double e1 = kap * p->e;
    double te = p->e - e1;
    double pe[3];
    for (int k = 0; k < 3; ++k) pe[k] = p->e * d0[k] - e1 * p->d[k];
    double nn = sqrt(pe[0] * pe[0] + pe[1] * pe[1] + pe[2] * pe[2]);
    if (nn > 0.0) { pe[0] /= nn; pe[1] /= nn; pe[2] /= nn; }
    else { pe[0] = d0[0]; pe[1] = d0[1]; pe[2] = d0[2]; }
    secondary(c, p, ORC_ELECTRON, te, pe);
    if (e1 > eabs[ORC_PHOTON]) {
      p->e = e1;
      event(c, p, EV_COMPTON, v);
    } else {
      deposit(c, p, e1);
      p->e = 0.0;
      event(c, p, EV_COMPTON, v);
    }
  } else if (ch == 1) {
    st->photo++;
    secondary(c, p, ORC_ELECTRON, p->e, p->d);
    p->e = 0.0;
    event(c, p, EV_PHOTO, v);
  } else if (ch == 2) {
    st->rayleigh++;
    double ct = sample_rayleigh(tables_at(c, v), &p->rng, p->e);
    double phi = 2.0 * PI * draw(&p->rng);
    rotate(p->d, ct, phi);
    event(c, p, EV_RAYLEIGH, v);
  } else {
    st->pair++;
    double avail = p->e - 2.0 * MC2;
    double eps = draw(&p->rng);
    double tm = eps * avail, tp = (1.0 - eps) * avail;
    double dm[3] = {p->d[0], p->d[1], p->d[2]};
    double dp[3] = {p->d[0], p->d[1], p->d[2]};
    double cm = leading_angle(beta_of(tm), draw(&p->rng));
    double fm = 2.0 * PI * draw(&p->rng);
    double cp = leading_angle(beta_of(tp), draw(&p->rng));
    double fp = 2.0 * PI * draw(&p->rng);
    rotate(dm, cm, fm);
    rotate(dp, cp, fp);
    secondary(c, p, ORC_ELECTRON, tm, dm);
    secondary(c, p, ORC_POSITRON, tp, dp);
    p->e = 0.0;
    event(c, p, EV_PAIR, v);
  }
}

/* photon: JUMP (free path in mass thickness), STEP (DDA through voxels) and
 * KNOCK until absorbed or escaped */
/* R10: the flight through voxels of several materials in optical depth:
 * tau = -ln u, each voxel takes rho mu_m(E) l of it; the interaction channel
 * is chosen by the tables of the voxel the photon stops in */
static int photon_flight_mm(ctx* c, part* p, double* mu, double* mt_out) {
  orc_stats* st = c->st;
  double mtm[ORC_MAX_MAT];
  for (int m = 0; m < ORC_MAX_MAT; ++m) {
    const orc_tables* tm = c->tbm[m];
    mtm[m] = 0.0;
    if (!tm) continue;
    for (int k = 0; k < 4; ++k) mtm[m] += interp(tm, tm->ph[k], tm->thr_ph[k], p->e);
  }
  st->flights++;
  double tau = -log(draw(&p->rng));
  for (;;) {
    int a;
    double s = face(c, p, &a);
    int64_t v = lin(c, p->ix);
    double att = c->ph->rho[v] * mtm[c->mat[v]];
    if (att * s >= tau) {
      /* the flight ends inside this voxel: d ln p / d rho = -mu_m l + 1/rho */
      if (c->w) score(c, v, -mtm[c->mat[v]] * (tau / att) + 1.0 / c->ph->rho[v]);
      move(p, tau / att);
      break;
    }
    if (c->w) score(c, v, -mtm[c->mat[v]] * s);
    tau -= att * s;
    if (cross(c, p, s, a)) {
      st->escaped++;
      c->led[ORC_LED_ESC] += p->e * p->w;
      event(c, p, EV_PH_ESCAPE, v);
      finish(c, p);
      return 1;
    }
  }
  const orc_tables* tb = tables_at(c, lin(c, p->ix));
  double mt = 0.0;
  for (int k = 0; k < 4; ++k) { mu[k] = interp(tb, tb->ph[k], tb->thr_ph[k], p->e); mt += mu[k]; }
  *mt_out = mt;
  return 0;
}

static void photon_track(ctx* c, part* p) {
  const orc_tables* tb = c->tb;
  orc_stats* st = c->st;
  while (p->e > 0.0 && c->mat) {
    double mu[4], mt;
    if (photon_flight_mm(c, p, mu, &mt)) return;
    double u = draw(&p->rng) * mt;
    int ch = -1;
    double cum = 0.0;
    for (int k = 0; k < 4; ++k) {
      cum += mu[k];
      if (u < cum) { ch = k; break; }
    }
    if (ch < 0)
      for (int k = 3; k >= 0; --k)
        if (mu[k] > 0.0) { ch = k; break; }
    photon_knock(c, p, ch);
  }
  while (p->e > 0.0) {
    double mu[4], mt = 0.0;
    for (int k = 0; k < 4; ++k) { mu[k] = interp(tb, tb->ph[k], tb->thr_ph[k], p->e); mt += mu[k]; }
    st->flights++;
    double tau = -log(draw(&p->rng)) / mt;
    for (;;) {
      int a;
      double s = face(c, p, &a);
      double rho = c->ph->rho[lin(c, p->ix)];
      if (rho * s >= tau) {
        /* the flight ends inside this voxel: d ln p / d rho = -mu l + 1/rho */
        if (c->w) score(c, lin(c, p->ix), -mt * (tau / rho) + 1.0 / rho);
        move(p, tau / rho);
        break;
      }
      if (c->w) score(c, lin(c, p->ix), -mt * s);
      tau -= rho * s;
      int64_t v = lin(c, p->ix);
      if (cross(c, p, s, a)) {
        st->escaped++;
        c->led[ORC_LED_ESC] += p->e * p->w;
        event(c, p, EV_PH_ESCAPE, v);
        finish(c, p);
        return;
      }
    }
    double u = draw(&p->rng) * mt;
    int ch = -1;
    double cum = 0.0;
    for (int k = 0; k < 4; ++k) {
      cum += mu[k];
      if (u < cum) { ch = k; break; }
    }
    if (ch < 0)
      for (int k = 3; k >= 0; --k)
        if (mu[k] > 0.0) { ch = k; break; }
    photon_knock(c, p, ch);
  }
  st->absorbed++;
  finish(c, p);
}

/* ------------------------------------------------------------------------ */
/* Electron / positron Class II transport                                   */
/* ------------------------------------------------------------------------ */

static void e_absorb(ctx* c, part* p) {
  int64_t v = lin(c, p->ix);
  c->led[ORC_LED_EABS] += p->e;
  deposit(c, p, p->e);
  c->st->absorbed++;
  if (p->type == ORC_POSITRON) {
    /* annihilation at rest: two back-to-back photons, isotropic */
    c->st->annih++;
    double ct = 2.0 * draw(&p->rng) - 1.0;
    double phi = 2.0 * PI * draw(&p->rng);
    double st = sqrt(1.0 - ct * ct > 0.0 ? 1.0 - ct * ct : 0.0);
    double d1[3] = {st * cos(phi), st * sin(phi), ct};
    double d2[3] = {-d1[0], -d1[1], -d1[2]};
    secondary(c, p, ORC_PHOTON, MC2, d1);
    secondary(c, p, ORC_PHOTON, MC2, d2);
  }
  p->e = 0.0;
  event(c, p, EV_ABSORB, v);
  finish(c, p);
}

static void e_escape(ctx* c, part* p, int64_t v) {
  c->st->escaped++;
  c->led[ORC_LED_ESC] += p->e * p->w;
  if (p->type == ORC_POSITRON) c->led[ORC_LED_POSESC] += p->w;
  event(c, p, EV_E_ESCAPE, v);
  p->e = 0.0;
  finish(c, p);
}

/* Moller energy transfer k in [kc, 1/2] from the bracket over k^2.  With
 * r = k/(1-k), k^2 times the bracket is f(k) = 1 + r^2 - (1-a) r + a k^2,
 * and f(k) <= 1 + 5 a k^2 on (0, 1/2] (the difference r^2 - r + a (r - 4k^2)
 * is linear in a and <= 0 at a = 0 and a = 1 because r <= 1 and
 * r <= 2k there; equality at k = 1/2).  The proposal is therefore
 * (1 + 5 a k^2)/k^2 = 1/k^2 + 5a, a mixture of 1/k^2 (weight 1/kc - 2,
 * sampled by inversion) and a uniform part (weight 5a (1/2 - kc)); one
 * uniform picks the part and, rescaled, samples it; the acceptance is
 * f(k)/(1 + 5 a k^2), above 0.97 from 1 MeV up */
static double sample_moller(stream* s, double e, double wcc) {
  double kc = wcc / e;
  inel_coef cf = inel_coefficients(e);
  double w1 = 1.0 / kc - 2.0, w2 = 5.0 * cf.a * (0.5 - kc);
  for (;;) {
    double u = draw(s) * (w1 + w2), ua = draw(s);
    double k = u < w1 ? kc / (1.0 - (u / w1) * (1.0 - 2.0 * kc)) : kc + (u - w1) / w2 * (0.5 - kc);
    double r = k / (1.0 - k);
    if (ua * (1.0 + 5.0 * cf.a * k * k) <= 1.0 + r * r + cf.a * k * k - (1.0 - cf.a) * r) return k;
  }
}

static double sample_bhabha(stream* s, double e, double wcc) {
  double kc = wcc / e;
  inel_coef cf = inel_coefficients(e);
  for (;;) {
    double u = draw(s), ua = draw(s);
    double k = kc / (1.0 - u * (1.0 - kc));
    double g = 1.0 - cf.b1 * k + cf.b2 * k * k - cf.b3 * k * k * k + cf.b4 * k * k * k * k;
    if (ua <= g) return k;
  }
}

/* polar cosines of a binary collision with a free electron at rest */
static double binary_cos(double e, double w, int primary) {
  double c2;
  if (primary) c2 = (e - w) * (e + 2.0 * MC2) / (e * (e - w + 2.0 * MC2));
  else c2 = w * (e + 2.0 * MC2) / (e * (w + 2.0 * MC2));
  if (c2 > 1.0) c2 = 1.0;
  return sqrt(c2);
}

/* R9: Heitler's two-photon annihilation of a positron (kinetic energy e,
 * g = 1 + e/mc^2, p = sqrt(g^2 - 1)) with a free electron at rest.  The
 * softer photon takes the fraction z of the total energy e + 2mc^2, with
 * z in [zmin, 1/2], zmin = 1/(g + 1 + p), and DCS per electron
 *   K [S(z) + S(1-z)],  S(x) = -(g+1)^2 + (g^2 + 4g + 1)/x - 1/x^2,
 *   K = pi r_e^2 / ((g+1)(g^2-1));
 * its integral is the total cross section
 *   K [(g^2 + 4g + 1) ln(g + p) - (g + 3) p]. */
double orc_sigma_annih(const orc_tables* tb, double e) {
  double g = 1.0 + e / MC2;
  double p = sqrt(g * g - 1.0);
  double k = PI * R_E * R_E * tb->mc.ne;
  return k * ((g * g + 4.0 * g + 1.0) * log(g + p) - (g + 3.0) * p) / ((g + 1.0) * (g * g - 1.0));
}

/* z from the DCS: proposal 1/z on [zmin, 1/2] (log-uniform), accepted with
 * probability z [S(z) + S(1-z)] / (2 (g^2 + 4g + 1)); z [S(z) + S(1-z)] is
 * at most (g^2 + 4g + 1)(1 + z/(1-z)) <= 2 (g^2 + 4g + 1) for z <= 1/2 */
static double sample_annih(stream* s, double e) {
  double g = 1.0 + e / MC2;
  double p = sqrt(g * g - 1.0);
  double zmin = 1.0 / (g + 1.0 + p);
  double c = g * g + 4.0 * g + 1.0;
  double g1 = (g + 1.0) * (g + 1.0);
  for (;;) {
    double z = zmin * pow(0.5 / zmin, draw(s));
    double y = 1.0 - z;
    double f = -g1 + c / z - 1.0 / (z * z) - g1 + c / y - 1.0 / (y * y);
    if (draw(s) * 2.0 * c <= z * f) return z;
  }
}

/* polar cosine of the photon taking the fraction z (energy-momentum
 * conservation): cos = (g + 1 - 1/z) / p */
static double annih_cos(double e, double z) {
  double g = 1.0 + e / MC2;
  double c = (g + 1.0 - 1.0 / z) / sqrt(g * g - 1.0);
  return c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
}

static void e_hard(ctx* c, part* p, int which) {
  const orc_tables* tb = tables_at(c, lin(c, p->ix));
  int ti = p->type == ORC_POSITRON ? 1 : 0;
  int64_t v = lin(c, p->ix);
  if (which == 0) {
    c->st->hard_el++;
    double muc = orc_mu_cut(tb, ti, p->e);
    double eta = screening(&tb->mc, p->e);
    double a = 1.0 / (muc + eta), b = 1.0 / (1.0 + eta);
    double mu = 1.0 / (a - draw(&p->rng) * (a - b)) - eta;
    if (mu < 0.0) mu = 0.0;
    if (mu > 1.0) mu = 1.0;
    double phi = 2.0 * PI * draw(&p->rng);
    rotate(p->d, 1.0 - 2.0 * mu, phi);
    event(c, p, EV_HARD_EL, v);
  } else if (which == 1) {
    c->st->hard_in++;
    double k = ti == 0 ? sample_moller(&p->rng, p->e, c->t->wcc) : sample_bhabha(&p->rng, p->e, c->t->wcc);
    double phi = 2.0 * PI * draw(&p->rng);
    double e = p->e, w = k * e;
    /* R11: a forced collision changes the primary with probability 1/F and
     * emits the knock-on electron with weight w/F */
    double f = c->t->force_in > 1.0 ? c->t->force_in : 1.0;
    int apply = f > 1.0 ? draw(&p->rng) * f < 1.0 : 1;
    double cp = binary_cos(e, w, 1), cs = binary_cos(e, w, 0);
    double ds[3] = {p->d[0], p->d[1], p->d[2]};
    rotate(ds, cs, phi + PI);
    if (apply) {
      rotate(p->d, cp, phi);
      p->e = e - w;
    }
    double w0 = p->w;
    p->w = w0 / f;
    secondary(c, p, ORC_ELECTRON, w, ds);
    p->w = w0;
    event(c, p, EV_HARD_IN, v);
  } else if (which == 3) {
    /* R9: the positron annihilates with an electron at rest */
    c->st->annih++;
    c->st->annih_flight++;
    double e = p->e;
    double z = sample_annih(&p->rng, e);
    double phi = 2.0 * PI * draw(&p->rng);
    double etot = e + 2.0 * MC2;
    double ka = z * etot, kb = etot - ka;
    double da[3] = {p->d[0], p->d[1], p->d[2]}, dbv[3] = {p->d[0], p->d[1], p->d[2]};
    rotate(da, annih_cos(e, z), phi);
    rotate(dbv, annih_cos(e, 1.0 - z), phi + PI);
    secondary(c, p, ORC_PHOTON, ka, da);
    secondary(c, p, ORC_PHOTON, kb, dbv);
    p->e = 0.0;
    event(c, p, EV_ANNIH_FLIGHT, v);
    finish(c, p);
  } else {
    c->st->hard_br++;
    double wcr = c->t->wcr, e = p->e;
    double w = wcr * pow(e / wcr, draw(&p->rng));
    double ct = leading_angle(beta_of(e), draw(&p->rng));
    double phi = 2.0 * PI * draw(&p->rng);
    /* R11: a forced emission changes the primary with probability 1/F and
     * emits the photon with weight w/F */
    double f = c->t->force_br > 1.0 ? c->t->force_br : 1.0;
    int apply = f > 1.0 ? draw(&p->rng) * f < 1.0 : 1;
    /* R12: split into S photons of energy W, each with its own polar and
     * azimuthal angle (drawn after the above) and weight w/(F S) */
    int ns = c->t->split_br == 2 ? 2 : 1;
    double dg[3] = {p->d[0], p->d[1], p->d[2]};
    double d2[3] = {p->d[0], p->d[1], p->d[2]};
    rotate(dg, ct, phi);
    if (ns == 2) {
      double ct2 = leading_angle(beta_of(e), draw(&p->rng));
      double phi2 = 2.0 * PI * draw(&p->rng);
      rotate(d2, ct2, phi2);
    }
    if (apply) p->e = e - w;
    double w0 = p->w;
    p->w = w0 / (f * ns);
    secondary(c, p, ORC_PHOTON, w, dg);
    if (ns == 2) secondary(c, p, ORC_PHOTON, w, d2);
    p->w = w0;
    event(c, p, EV_HARD_BR, v);
  }
}

/* Class II step loop of one electron or positron.  In gradient mode (c->w)
 * each step also adds its terms of reading A25: the score of the majorant
 * free path (A), the score of the soft deflection (C) and the logged
 * pathwise soft-loss term, swept backward when the particle ends. */
static void electron_track(ctx* c, part* p) {
  const orc_transport* t = c->t;
  int ti = p->type == ORC_POSITRON ? 1 : 0;
  double eabs = t->eabs[p->type];
  for (;;) {
    if (!(p->e > eabs)) {
      if (c->w) elog_close(c, p->w * c->w[lin(c, p->ix)]);
      e_absorb(c, p);
      return;
    }
    c->st->esteps++;
    double e = p->e;
    int64_t v = lin(c, p->ix);
    const orc_tables* tb = tables_at(c, v);  /* the step stays in this voxel's material */
    double rho = c->ph->rho[v];
    /* step control: maximum mass step and the hard-event majorant */
    double ss = interp(tb, tb->el[ti][CH_S], 0.0, e);
    double tau_max = t->c2 * e / ss;
    /* (test use: a fixed geometric cap, whose mass the majorant must cover) */
    const double* cap = c->ph->step_cap;
    double tau_cap = cap ? rho * cap[v] : tau_max;
    double r0 = range_of(tb, ti, e);
    double elo = r0 - tau_cap > 0.0 ? orc_range_inverse(tb, ti, r0 - tau_cap) : tb->e[0];
    if (elo > e) elo = e;
    if (t->flags & ORC_STRAGGLING) {
      /* R14: a straggled loss can exceed the step's CSDA loss: by at most
       * twice the CSDA mean under the Gaussian and uniform laws, and by at
       * most 6 Omega^2(E)/S under the two-mode law (8 here, for the
       * stopping power's change over the step); the hard-event majorant
       * covers every energy the step can end at */
      double dmax = 2.0 * (e - elo);
      double dw = 8.0 * orc_soft_omega2(tb, ti, e) / ss;
      if (dw > dmax) dmax = dw;
      elo = e - dmax > tb->e[0] ? e - dmax : tb->e[0];
    }
    double smaj = orc_sigma_majorant(tb, ti, elo, e);
    /* R9: Heitler's cross section falls with energy: its value at the low
     * end of the step's energy interval bounds it over the step */
    int annih = ti == 1 && (t->flags & ORC_ANNIH_FLIGHT);
    if (annih) smaj += orc_sigma_annih(tb, elo);
    /* the hard-event clock: a pending free path runs on across steps, so
     * where faces cut a track does not change where its hard events fall */
    if (!(p->clk > 0.0)) p->clk = -log(draw(&p->rng));
    double tau_h = smaj > 0.0 ? p->clk / smaj : INF_D;
    int capped;
    double len;
    if (cap) {
      capped = !(tau_h / rho <= cap[v]);
      len = capped ? cap[v] : tau_h / rho;
    } else {
      capped = !(tau_h <= tau_max);
      double tau_s = capped ? tau_max : tau_h;
      len = tau_s / rho;
    }
    double th = draw(&p->rng) * len;
    int a;
    double db = face(c, p, &a);
    /* Reading A6': the step ends at the first face on its path or at its full
     * length; the hinge, if reached, deflects the particle by the soft
     * angular law of the whole step.  The soft loss is charged where the step
     * ends, over the geometric length s actually travelled: the CSDA energy
     * after s is R^-1(R(E) - rho s). */
    int face_end = db <= th;
    double s = db, after = db, hinge_se = 0.0;
    if (!face_end) {
      move(p, th);
      double t1s = interp(tb, tb->el[ti][CH_T1S], 0.0, e);
      double mbar = 0.5 * (1.0 - exp(-rho * len * t1s));
      double aa = orc_soft_a(mbar);
      double u3 = draw(&p->rng);
      double mu = aa * u3 / (1.0 + aa - u3);
      /* A25 term C, and the same law's score with respect to the energy
       * (term E): <mu> moves with E through t1s, a power law between nodes */
      if (c->w) {
        double sc = orc_soft_score(aa, mu, mbar, len, t1s);
        score(c, v, sc);
        if (t->flags & ORC_GRAD_DEFLECTION_ENERGY) {
          double f;
          int gi = grid_pos(tb, e, &f);
          const double* yt = tb->el[ti][CH_T1S];
          if (yt[gi] > 0.0 && yt[gi + 1] > 0.0) hinge_se = sc * rho * log(yt[gi + 1] / yt[gi]) / (tb->dl * e);
        }
      }
      double phi = 2.0 * PI * draw(&p->rng);
      rotate(p->d, 1.0 - 2.0 * mu, phi);
      double rem = len - th;
      double db2 = face(c, p, &a);
      face_end = db2 <= rem;
      after = face_end ? db2 : rem;
      s = face_end ? th + db2 : len;
    }
    /* the clock runs down by the majorant optical depth of the path; a step
     * that ends uncapped at its full length ends at an event (below) */
    int event_end = !face_end && !capped;
    p->clk = event_end ? 0.0 : p->clk - smaj * (rho * s);
    /* A25 term A: the candidate events of the majorant process along the
     * path form a Poisson process of rate rho smaj per unit length:
     * d ln L / d rho = -smaj s over each path segment, +1/rho at an event */
    if (c->w) score(c, v, -smaj * s + (event_end ? 1.0 / rho : 0.0));
    double e1 = orc_range_inverse(tb, ti, r0 - rho * s);
    if (!(e1 < e)) e1 = e;
    if (t->flags & ORC_STRAGGLING) {
      e1 = e - straggle(&p->rng, e - e1, rho * s * orc_soft_omega2(tb, ti, e));
      if (!(e1 > 0.0)) e1 = 0.0;
    }
    deposit(c, p, e - e1);
    c->led[ORC_LED_PATH] += rho * s;
    if (c->w) {
      double s1 = interp(tb, tb->el[ti][CH_S], 0.0, e1);
      elog_push(c, v, s * s1, s1 / ss, p->w * c->w[v], hinge_se);
    }
    p->e = e1;
    if (face_end) {
      /* cross; an energy at or below Eabs is absorbed at the next step's
       * start, in the voxel entered */
      event(c, p, EV_CROSS, v);
      if (cross(c, p, after, a)) {
        if (c->w) elog_close(c, 0.0);
        e_escape(c, p, v);
        return;
      }
      continue;
    }
    move(p, after);
    if (!(e1 > eabs)) {
      if (c->w) elog_close(c, p->w * c->w[v]);
      e_absorb(c, p);
      return;
    }
    if (capped) {
      event(c, p, EV_STEP, v);
      continue;
    }
    /* hard event or delta: channels in the order elastic, inelastic, brems */
    double u = draw(&p->rng) * smaj;
    double s_el = interp(tb, tb->el[ti][CH_EL], 0.0, e1);
    double s_in = interp(tb, tb->el[ti][CH_IN], tb->thr_el[ti][CH_IN], e1);
    double s_br = interp(tb, tb->el[ti][CH_BR], tb->thr_el[ti][CH_BR], e1);
    double s_an = annih ? orc_sigma_annih(tb, e1) : 0.0;
    if (s_el + s_in + s_br + s_an > smaj) c->st->maj_excess++;
    if (u < s_el) e_hard(c, p, 0);
    else if (u < s_el + s_in) e_hard(c, p, 1);
    else if (u < s_el + s_in + s_br) e_hard(c, p, 2);
    else if (u < s_el + s_in + s_br + s_an) {
      /* the photons take the positron's energy away: no adjoint beyond */
      if (c->w) elog_close(c, 0.0);
      e_hard(c, p, 3);
      return;
    } else {
      c->st->delta++;
      event(c, p, EV_STEP, v);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* History loop and estimators                                              */
/* ------------------------------------------------------------------------ */

static int locate(const ctx* c, part* p) {
  for (int k = 0; k < 3; ++k) {
    double f = floor((p->x[k] - c->o[k]) / c->dx[k]);
    if (!(f >= 0.0) || !(f < (double)c->n[k])) return -1;
    p->ix[k] = (int)f;
  }
  return 0;
}

static int run_body(const orc_tables* const* tbs, int n_mat, const orc_transport* t, const orc_phantom* ph,
                    const orc_source* src, int n_src, uint32_t seed, uint64_t first,
                    uint64_t n, double* sum_q, double* sum_q2, orc_stats* stats,
                    uint64_t* hashes, double* ledger, const double* w, double* a_acc,
                    double* b_acc, double* p_acc, double* sum_q_h) {
  if (!tbs || n_mat < 1 || n_mat > ORC_MAX_MAT || !t || !ph || !src || n_src <= 0 || !sum_q || !sum_q2 || !stats)
    return -1;
  for (int m = 0; m < n_mat; ++m)
    if (!tbs[m]) return -1;
  uint64_t total = 0;
  for (int s = 0; s < n_src; ++s) total += src[s].n_hist;
  if (first + n > total || first + n > 0xFFFFFFFFull) return -2;
  int64_t nv = (int64_t)ph->nx * ph->ny * ph->nz;
  if (ph->mat)
    for (int64_t v = 0; v < nv; ++v)
      if (ph->mat[v] >= n_mat) return -5;
  ctx c;
  memset(&c, 0, sizeof(c));
  c.tb = tbs[0];
  for (int m = 0; m < n_mat; ++m) c.tbm[m] = tbs[m];
  c.mat = ph->mat;
  c.t = t;
  c.ph = ph;
  c.n[0] = ph->nx; c.n[1] = ph->ny; c.n[2] = ph->nz;
  c.dx[0] = ph->dx; c.dx[1] = ph->dy; c.dx[2] = ph->dz;
  c.o[0] = ph->ox; c.o[1] = ph->oy; c.o[2] = ph->oz;
  c.tmp = (double*)calloc((size_t)nv, sizeof(double));
  c.mark = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nv);
  c.touched = (int64_t*)malloc(sizeof(int64_t) * (size_t)nv);
  for (int64_t v = 0; v < nv; ++v) c.mark[v] = ~0ull;
  c.st = stats;
  if (w) {
    c.w = w;
    c.p_acc = p_acc;
    c.s_tmp = (double*)calloc((size_t)nv, sizeof(double));
    c.s_mark = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nv);
    c.s_touched = (int64_t*)malloc(sizeof(int64_t) * (size_t)nv);
    for (int64_t v = 0; v < nv; ++v) c.s_mark[v] = ~0ull;
  }
  int rc = 0;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t h = first + i;
    /* the source of history h: concatenation of the sources in order */
    int s = 0;
    uint64_t base = 0;
    while (h >= base + src[s].n_hist) { base += src[s].n_hist; ++s; }
    const orc_source* so = &src[s];
    part p;
    memset(&p, 0, sizeof(p));
    p.type = so->particle;
    p.e = so->energy;
    p.rng.seed = seed;
    p.rng.hist = (uint32_t)h;
    p.rng.uid = 1;
    p.w = 1.0;
    memcpy(p.x, so->pos, sizeof(p.x));
    memcpy(p.d, so->dir, sizeof(p.d));
    if (so->kind == ORC_SRC_RECT) {
      p.x[0] = so->pos[0] + (draw(&p.rng) - 0.5) * so->width[0];
      p.x[1] = so->pos[1] + (draw(&p.rng) - 0.5) * so->width[1];
    }
    if (locate(&c, &p)) { rc = -3; break; }
    c.cur = h;
    c.n_touched = 0;
    c.n_s_touched = 0;
    c.q_h = 0.0;
    memset(c.led, 0, sizeof(c.led));
    c.hist_hash = 0;
    push(&c, &p);
    while (c.sp > 0) {
      part q = c.stack[--c.sp];
      if (q.type == ORC_PHOTON) photon_track(&c, &q);
      else electron_track(&c, &q);
    }
    /* Eq. (1)-(3): per-history score q and q^2 into separate counters */
    for (int64_t j = 0; j < c.n_touched; ++j) {
      int64_t v = c.touched[j];
      double q = c.tmp[v];
      sum_q[v] += q;
      sum_q2[v] += q * q;
    }
    if (w) {
      /* score-function estimator: Q_h times the history's score */
      for (int64_t j = 0; j < c.n_s_touched; ++j) {
        int64_t v = c.s_touched[j];
        a_acc[v] += c.q_h * c.s_tmp[v];
        b_acc[v] += c.s_tmp[v];
      }
      *sum_q_h += c.q_h;
    }
    stats->histories++;
    stats->e_dep += c.led[ORC_LED_DEP];
    stats->e_esc += c.led[ORC_LED_ESC];
    stats->pos_esc += (uint64_t)c.led[ORC_LED_POSESC];
    if (hashes) hashes[i] = c.hist_hash;
    if (ledger) memcpy(ledger + i * ORC_LED_N, c.led, sizeof(c.led));
  }
  free(c.tmp);
  free(c.mark);
  free(c.touched);
  free(c.stack);
  free(c.s_tmp);
  free(c.s_mark);
  free(c.s_touched);
  free(c.elog);
  return rc;
}

int orc_run(const orc_tables* tb, const orc_transport* t, const orc_phantom* ph,
            const orc_source* src, int n_src, uint32_t seed, uint64_t first,
            uint64_t n, double* sum_q, double* sum_q2, orc_stats* stats,
            uint64_t* hashes, double* ledger) {
  return run_body(&tb, 1, t, ph, src, n_src, seed, first, n, sum_q, sum_q2, stats, hashes, ledger,
                  NULL, NULL, NULL, NULL, NULL);
}

int orc_run_mm(const orc_tables* const* tbs, int n_mat, const orc_transport* t, const orc_phantom* ph,
               const orc_source* src, int n_src, uint32_t seed, uint64_t first, uint64_t n, double* sum_q,
               double* sum_q2, orc_stats* stats, uint64_t* hashes, double* ledger) {
  return run_body(tbs, n_mat, t, ph, src, n_src, seed, first, n, sum_q, sum_q2, stats, hashes, ledger,
                  NULL, NULL, NULL, NULL, NULL);
}

int orc_run_gradient(const orc_tables* tb, const orc_transport* t, const orc_phantom* ph,
                     const orc_source* src, int n_src, uint32_t seed, uint64_t first,
                     uint64_t n, const double* w, double* a_acc, double* b_acc,
                     double* p_acc, double* sum_q_h) {
  return orc_run_gradient_mm(&tb, 1, t, ph, src, n_src, seed, first, n, w, a_acc, b_acc, p_acc, sum_q_h);
}

int orc_run_gradient_mm(const orc_tables* const* tbs, int n_mat, const orc_transport* t, const orc_phantom* ph,
                        const orc_source* src, int n_src, uint32_t seed, uint64_t first, uint64_t n,
                        const double* w, double* a_acc, double* b_acc, double* p_acc, double* sum_q_h) {
  if (!w || !a_acc || !b_acc || !p_acc || !sum_q_h) return -1;
  /* the estimator has no term for the score of a straggled soft loss; with
   * forcing or splitting (R11, R12) the scores are those of the sampling
   * laws actually used (the forced majorant), and the deposits and the
   * soft-loss term carry the weights; annihilation in flight (R9) is a
   * hard channel of the majorant like the others */
  if (t->flags & ORC_STRAGGLING) return -4;
  int64_t nv = (int64_t)ph->nx * ph->ny * ph->nz;
  double* q = (double*)calloc((size_t)nv, sizeof(double));
  double* q2 = (double*)calloc((size_t)nv, sizeof(double));
  orc_stats st;
  memset(&st, 0, sizeof(st));
  int rc = run_body(tbs, n_mat, t, ph, src, n_src, seed, first, n, q, q2, &st, NULL, NULL, w, a_acc, b_acc,
                    p_acc, sum_q_h);
  free(q);
  free(q2);
  return rc;
}

void orc_dose(const orc_phantom* ph, uint64_t n_hist, const double* sum_q,
              const double* sum_q2, double* dose, double* sigma) {
  int64_t nv = (int64_t)ph->nx * ph->ny * ph->nz;
  double vol = ph->dx * ph->dy * ph->dz;
  double nn = (double)n_hist;
  for (int64_t v = 0; v < nv; ++v) {
    double mass = ph->rho[v] * vol; /* g */
    double qm = sum_q[v] / nn, q2m = sum_q2[v] / nn;
    double var = (q2m - qm * qm) / nn;
    if (var < 0.0) var = 0.0;
    dose[v] = qm * 1e6 / mass;
    sigma[v] = sqrt(var) * 1e6 / mass;
  }
}

/* ------------------------------------------------------------------------ */
/* Sampler access for the distribution tests                                */
/* ------------------------------------------------------------------------ */

int orc_sample_straggle(double m, double omega2, uint32_t seed, int n, double* out) {
  for (int i = 0; i < n; ++i) {
    stream s = {seed, (uint32_t)i, 1ull, 0u};
    out[i] = straggle(&s, m, omega2);
  }
  return 0;
}

int orc_sample(const orc_tables* tb, int which, double e, uint32_t seed, int n,
               double* out0, double* out1) {
  for (int i = 0; i < n; ++i) {
    stream s = {seed, (uint32_t)i, 1ull, 0u};
    double a = 0.0, b = 0.0;
    switch (which) {
      case ORC_SMP_COMPTON: a = sample_kn(&s, e, &b); break;
      case ORC_SMP_RAYLEIGH: a = sample_rayleigh(tb, &s, e); break;
      case ORC_SMP_MOLLER: a = sample_moller(&s, e, tb->t.wcc); b = binary_cos(e, a * e, 1); break;
      case ORC_SMP_BHABHA: a = sample_bhabha(&s, e, tb->t.wcc); break;
      case ORC_SMP_BREMS: {
        a = tb->t.wcr * pow(e / tb->t.wcr, draw(&s));
        b = leading_angle(beta_of(e), draw(&s));
        break;
      }
      case ORC_SMP_HARD_ELASTIC: {
        double muc = orc_mu_cut(tb, 0, e), eta = screening(&tb->mc, e);
        double aa = 1.0 / (muc + eta), bb = 1.0 / (1.0 + eta);
        a = 1.0 / (aa - draw(&s) * (aa - bb)) - eta;
        break;
      }
      case ORC_SMP_SOFT: {
        double aa = orc_soft_a(e);
        double u = draw(&s);
        a = aa * u / (1.0 + aa - u);
        break;
      }
      case ORC_SMP_PAIR: {
        double avail = e - 2.0 * MC2;
        a = draw(&s);
        b = leading_angle(beta_of(a * avail), draw(&s));
        break;
      }
      case ORC_SMP_FREE_PATH: {
        double mt = 0.0;
        for (int k = 0; k < 4; ++k) mt += interp(tb, tb->ph[k], tb->thr_ph[k], e);
        a = -log(draw(&s)) / mt;
        break;
      }
      case ORC_SMP_ANNIH: a = 2.0 * draw(&s) - 1.0; break;
      case ORC_SMP_ANNIH_FLIGHT: a = sample_annih(&s, e); b = annih_cos(e, a); break;
      default: return -1;
    }
    out0[i] = a;
    if (out1) out1[i] = b;
  }
  return 0;
}
