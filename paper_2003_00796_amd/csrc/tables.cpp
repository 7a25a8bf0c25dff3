// tables.cpp -- host-side tabulation of the synthetic analytic material
// models on the transport's log energy grid (setup, outside the timed
// transport).  The result is the channel-major block described in
// mcx_internal.h, in FP64; the runtime converts it to FP32 for MIXED runs.
//
// Models (the paper defines physics by reference to PENELOPE only, so these
// are synthetic analytic stand-ins with textbook forms):
//  photons   Klein-Nishina Compton on free electrons; photoelectric power law;
//            Rayleigh with form factor F(x) = F0 (1 + a x^2)^-2 integrated in
//            closed form; pair production c ln(E/2mc^2)^2 above 2mc^2.
//  e-/e+     Bethe collision stopping power without density effect (ICRU 37
//            F- / F+ terms); Moller (e-) and Bhabha (e+) hard collisions above
//            Wcc, removed from the soft stopping power; bremsstrahlung
//            dSigma/dW = b/W with emission above Wcr hard; screened Rutherford
//            elastic scattering dsigma/dmu = K/(mu + eta)^2 (Moliere
//            screening), hard elastic mean free path
//            max(lambda_el, min(C1 lambda_1, C2 E/S_soft)) as in PENELOPE's
//            mixed scheme, and the soft first transport coefficient below the
//            resulting cutoff mu_c; range = exact integral of 1/S_soft over
//            the piecewise power-law interpolant of S_soft.
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include <algorithm>

#include "mcx.h"
#include "mcx_internal.h"
#include "tables.h"

namespace mcx {

namespace {

struct Lepton {
  double gamma, beta2, p2, etot;
  explicit Lepton(double t) {
    etot = t + kMc2;
    p2 = t * (t + 2.0 * kMc2);
    gamma = etot / kMc2;
    beta2 = p2 / (etot * etot);
  }
};

double ln_or_inf(double y) { return y > 0.0 ? std::log(y) : -std::numeric_limits<double>::infinity(); }

class Model {
 public:
  Model(const mcx_material_desc& m, const mcx_transport& t) : m_(m), t_(t) {
    ne_ = kNa * m.z_mol / m.a_mol;
    nmol_ = kNa / m.a_mol;
  }

  double compton(double e) const {
    const double k = e / kMc2;
    const double l = std::log(1.0 + 2.0 * k);
    const double a = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k);
    const double b = l / (2.0 * k);
    const double c = (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
    return ne_ * 2.0 * kPi * kRe * kRe * (a + b - c);
  }

  double photo(double e) const { return m_.pe_coef * std::pow(e / m_.pe_eref, -m_.pe_exp); }

  // closed-form integral over u = x^2 in [0, U]: (2/U) Int (2 - 4u/U + 4u^2/U^2) (1+au)^-4 du
  double rayleigh(double e) const {
    const double a = m_.ray_a;
    const double U = (e / kHc) * (e / kHc);
    const double T = 1.0 + a * U;
    const double T2 = T * T, T3 = T2 * T;
    const double j0 = -std::expm1(-3.0 * std::log1p(a * U)) / (3.0 * a);
    const double j1 = (1.0 / 6.0 - 0.5 / T2 + 1.0 / (3.0 * T3)) / (a * a);
    const double j2 = (1.0 / 3.0 - 1.0 / T + 1.0 / T2 - 1.0 / (3.0 * T3)) / (a * a * a);
    const double integral = 2.0 * j0 - 4.0 * j1 / U + 4.0 * j2 / (U * U);
    return nmol_ * kPi * kRe * kRe * m_.ray_f0 * m_.ray_f0 * (2.0 / U) * integral;
  }

  double pair(double e) const {
    if (!(e > 2.0 * kMc2)) return 0.0;
    const double l = std::log(e / (2.0 * kMc2));
    return m_.pp_coef * l * l;
  }

  double s_collision(int lep, double t) const {
    Lepton k(t);
    const double tau = t / kMc2;
    const double ir = m_.i_exc / kMc2;
    double f;
    if (lep == 0) {
      f = 1.0 - k.beta2 + (tau * tau / 8.0 - (2.0 * tau + 1.0) * std::log(2.0)) / ((tau + 1.0) * (tau + 1.0));
    } else {
      const double y = tau + 2.0;
      f = 2.0 * std::log(2.0) - (k.beta2 / 12.0) * (23.0 + 14.0 / y + 10.0 / (y * y) + 4.0 / (y * y * y));
    }
    const double lg = std::log(tau * tau * (tau + 2.0) / (2.0 * ir * ir));
    return 2.0 * kPi * kRe * kRe * kMc2 * ne_ / k.beta2 * (lg + f);
  }

  // hard collision cross section and stopping above Wcc
  void hard_collisions(int lep, double t, double* sig, double* stop) const {
    *sig = 0.0;
    *stop = 0.0;
    const double w = t_.wcc;
    if (lep == 0 ? !(t > 2.0 * w) : !(t > w)) return;
    Lepton k(t);
    const double kc = w / t;
    const double g = k.gamma;
    const double a = ((g - 1.0) / g) * ((g - 1.0) / g);
    const double pref = 2.0 * kPi * kRe * kRe * kMc2 * ne_ / k.beta2;
    if (lep == 0) {
      // Moller: 1/k^2 + 1/(1-k)^2 + a - (1-a)/(k(1-k)) on [kc, 1/2]
      const double b = 1.0 - a;
      const double n0 = 1.0 / kc - 1.0 / (1.0 - kc) + a * (0.5 - kc) - b * std::log((1.0 - kc) / kc);
      const double n1 = std::log(1.0 / (2.0 * kc)) + 2.0 - std::log(2.0) - 1.0 / (1.0 - kc) -
                        std::log(1.0 - kc) + a * (0.125 - 0.5 * kc * kc) - b * std::log(2.0 * (1.0 - kc));
      *sig = pref / t * n0;
      *stop = pref * n1;
    } else {
      // Bhabha: (1 - b1 k + b2 k^2 - b3 k^3 + b4 k^4)/k^2 on [kc, 1]
      const double gp = g + 1.0;
      const double b1 = a * (2.0 * gp * gp - 1.0) / (g * g - 1.0);
      const double b2 = a * (3.0 * gp * gp + 1.0) / (gp * gp);
      const double b3 = a * 2.0 * (g - 1.0) * g / (gp * gp);
      const double b4 = a * (g - 1.0) * (g - 1.0) / (gp * gp);
      const double k2 = kc * kc, k3 = k2 * kc, k4 = k3 * kc;
      const double n0 = (1.0 / kc - 1.0) - b1 * std::log(1.0 / kc) + b2 * (1.0 - kc) -
                        b3 * (1.0 - k2) / 2.0 + b4 * (1.0 - k3) / 3.0;
      const double n1 = std::log(1.0 / kc) - b1 * (1.0 - kc) + b2 * (1.0 - k2) / 2.0 -
                        b3 * (1.0 - k3) / 3.0 + b4 * (1.0 - k4) / 4.0;
      *sig = pref / t * n0;
      *stop = pref * n1;
    }
  }

  double k_elastic(double t) const {
    Lepton k(t);
    const double pv = k.p2 / k.etot;
    const double q = kRe * kMc2 / pv;
    return nmol_ * kPi * q * q * m_.zz1_mol;
  }

  double eta(double t) const {
    Lepton k(t);
    const double c = kAlpha * std::cbrt(m_.z_screen) / 0.885;
    const double az = kAlpha * m_.z_screen;
    return 0.25 * c * c * (kMc2 * kMc2 / k.p2) * (1.13 + 3.76 * az * az / k.beta2);
  }

  double eta_a() const {
    const double c = kAlpha * std::cbrt(m_.z_screen) / 0.885;
    return 0.25 * c * c;
  }
  double eta_b() const {
    const double az = kAlpha * m_.z_screen;
    return 3.76 * az * az;
  }
  double k_coef() const { return nmol_ * kPi * kRe * kRe * m_.zz1_mol; }
  // leading term of the binary-collision DCS, 2 pi r_e^2 mc^2 n_e / (beta^2
  // W^2): times W^2 and integrated over (0, Wc] it gives strag_k Wc / beta^2
  // (Bohr's variance of the soft collision loss per unit mass path)
  double strag_k() const { return 2.0 * kPi * kRe * kRe * kMc2 * ne_; }
  double annih_k() const { return kPi * kRe * kRe * ne_; }

 private:
  mcx_material_desc m_;
  mcx_transport t_;
  double ne_, nmol_;
};

}  // namespace

bool build_tables(const mcx_material_desc& m, const mcx_transport& t, BuiltTables* out, std::string* err) {
  const int n = t.n_grid;
  BuiltTables& b = *out;
  b.n = n;
  b.lemin = std::log(t.e_min);
  b.dl = (std::log(t.e_max) - b.lemin) / double(n - 1);
  b.block.assign(size_t(T_NCH) * n + kSoftN, 0.0);
  auto ch = [&](int c) { return b.block.data() + size_t(c) * n; };
  Model md(m, t);
  const uint32_t fl = t.flags;
  std::vector<double> e(n);
  for (int i = 0; i < n; ++i) e[i] = t.e_min * std::exp(double(i) * b.dl);
  for (int i = 0; i < n; ++i) {
    ch(T_ENODE)[i] = e[i];
    ch(T_LMU_C)[i] = ln_or_inf((fl & MCX_NO_COMPTON) ? 0.0 : md.compton(e[i]));
    ch(T_LMU_PE)[i] = ln_or_inf((fl & MCX_NO_PHOTO) ? 0.0 : md.photo(e[i]));
    ch(T_LMU_R)[i] = ln_or_inf((fl & MCX_NO_RAYLEIGH) ? 0.0 : md.rayleigh(e[i]));
    ch(T_LMU_PP)[i] = ln_or_inf((fl & MCX_NO_PAIR) ? 0.0 : md.pair(e[i]));
  }
  b.thr_pp = 2.0 * kMc2;
  b.thr_br = t.wcr;
  for (int lep = 0; lep < 2; ++lep) {
    b.thr_in[lep] = lep == 0 ? 2.0 * t.wcc : t.wcc;
    const int base = T_E + lep * T_ES;
    std::vector<double> s_soft(n);
    for (int i = 0; i < n; ++i) {
      const double ei = e[i];
      double sig_in = 0.0, s_hard = 0.0;
      if (!(fl & MCX_NO_HARD_INELASTIC)) md.hard_collisions(lep, ei, &sig_in, &s_hard);
      double s_rad, sig_br = 0.0;
      if (fl & MCX_NO_HARD_BREMS) {
        s_rad = m.brems_b * ei;
      } else {
        s_rad = m.brems_b * std::min(ei, t.wcr);
        if (ei > t.wcr) sig_br = m.brems_b * std::log(ei / t.wcr);
      }
      const double ss = md.s_collision(lep, ei) - s_hard + s_rad;
      // interaction forcing: the hard channels' cross sections times F (the
      // soft stopping power above keeps the analog split)
      if (t.force_in > 1.0) sig_in *= t.force_in;
      if (t.force_br > 1.0) sig_br *= t.force_br;
      if (!(ss > 0.0)) {
        *err = "soft stopping power is not positive at E = " + std::to_string(ei) + " MeV";
        return false;
      }
      const double kk = md.k_elastic(ei);
      const double eta = md.eta(ei);
      const double sig_el = kk / (eta * (1.0 + eta));
      const double sig1 = 2.0 * kk * (std::log((1.0 + eta) / eta) - 1.0 / (1.0 + eta));
      double sig_h = 0.0, sig1s = sig1;
      if (!(fl & MCX_NO_HARD_ELASTIC)) {
        const double lam_h = std::max(1.0 / sig_el, std::min(t.c1 / sig1, t.c2 * ei / ss));
        sig_h = 1.0 / lam_h;
        double muc = 1.0 / (sig_h / kk + 1.0 / (1.0 + eta)) - eta;
        muc = std::min(1.0, std::max(0.0, muc));
        sig1s = 2.0 * kk * (std::log((muc + eta) / eta) - muc / (muc + eta));
      }
      s_soft[i] = ss;
      ch(base + O_LS)[i] = std::log(ss);
      ch(base + O_S)[i] = ss;
      ch(base + O_LEL)[i] = ln_or_inf(sig_h);
      ch(base + O_LIN)[i] = ln_or_inf(sig_in);
      ch(base + O_LBR)[i] = ln_or_inf(sig_br);
      ch(base + O_LT1S)[i] = ln_or_inf(sig1s);
      ch(base + O_HSUM)[i] = sig_h + sig_in + sig_br;
      ch(base + O_LH)[i] = std::log(sig_h + sig_in + sig_br);
    }
    // the log-log chord of the node sums bounds the sum on a segment where no
    // channel starts (ln of a sum of power laws is convex in ln E)
    for (int i = 0; i < n; ++i) {
      bool thr = false;
      if (i + 1 < n)
        for (int c : {O_LEL, O_LIN, O_LBR})
          if (!(ch(base + c)[i] > -HUGE_VAL) && ch(base + c)[i + 1] > -HUGE_VAL) thr = true;
      ch(base + O_LHC)[i] = thr ? -HUGE_VAL : ch(base + O_LH)[i];
    }
    // range: Int dE / S over each power-law segment S = S_i (E/E_i)^(1-q)
    double r = 0.0;
    for (int i = 0; i < n; ++i) {
      double q = 0.0;
      if (i + 1 < n) q = 1.0 - std::log(s_soft[i + 1] / s_soft[i]) / std::log(e[i + 1] / e[i]);
      else q = ch(base + O_Q)[i - 1];
      ch(base + O_Q)[i] = q;
      ch(base + O_R)[i] = r;
      if (i + 1 < n) {
        const double x = e[i + 1] / e[i];
        const double seg = std::fabs(q) < 1e-10 ? (e[i] / s_soft[i]) * std::log(x)
                                                : (e[i] / s_soft[i]) * (std::pow(x, q) - 1.0) / q;
        r += seg;
      }
    }
  }
  // ln A(<mu>) of the soft law p(mu) ~ (mu + A)^-2, mean A(1+A)ln(1+1/A) - A,
  // by bisection in ln A (initial guesses for the device's Newton steps)
  {
    double* soft = b.block.data() + size_t(T_NCH) * n;
    const double y0 = std::log(kSoftMLo / (0.5 - kSoftMLo)), y1 = std::log(kSoftMHi / (0.5 - kSoftMHi));
    for (int j = 0; j < kSoftN; ++j) {
      const double y = y0 + (y1 - y0) * j / (kSoftN - 1);
      const double m = 0.5 / (1.0 + std::exp(-y));
      double lo = -700.0, hi = std::log(1e6);
      for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi), a = std::exp(mid);
        const double mean = a * ((1.0 + a) * std::log1p(1.0 / a) - 1.0);
        if (mean < m) lo = mid;
        else hi = mid;
      }
      soft[j] = 0.5 * (lo + hi);
    }
  }
  b.k_coef = md.k_coef();
  b.eta_a = md.eta_a();
  b.eta_b = md.eta_b();
  b.ray_a = m.ray_a;
  b.strag_k = md.strag_k();
  b.strag_b = m.brems_b;
  const double inf = std::numeric_limits<double>::infinity();
  b.wcc_soft = (t.flags & MCX_NO_HARD_INELASTIC) ? inf : t.wcc;
  b.wcr_soft = (t.flags & MCX_NO_HARD_BREMS) ? inf : t.wcr;
  b.annih_k = md.annih_k();
  return true;
}

}  // namespace mcx

// CT calibration (see mcx_ct_to_phantom in mcx.h): piecewise-linear HU ->
// density, thresholds HU -> material index
extern "C" int mcx_ct_to_phantom(const mcx_ct_calibration* cal, const int16_t* hu, uint64_t nvox, double* rho,
                                 uint8_t* mat) {
  if (!cal || !hu || !rho || cal->n_points < 1 || !cal->hu || !cal->rho) return MCX_E_INVALID;
  if (cal->n_thresholds < 0 || cal->n_thresholds > mcx::kMaxMat - 1 || (cal->n_thresholds > 0 && !cal->mat_hu))
    return MCX_E_INVALID;
  const int np = cal->n_points;
  for (int i = 0; i < np; ++i) {
    if (!(cal->rho[i] > 0.0) || !std::isfinite(cal->hu[i])) return MCX_E_INVALID;
    if (i > 0 && !(cal->hu[i] > cal->hu[i - 1])) return MCX_E_INVALID;
  }
  for (int j = 1; j < cal->n_thresholds; ++j)
    if (!(cal->mat_hu[j] > cal->mat_hu[j - 1])) return MCX_E_INVALID;
  for (uint64_t v = 0; v < nvox; ++v) {
    const double x = double(hu[v]);
    double r;
    if (x <= cal->hu[0]) {
      r = cal->rho[0];
    } else if (x >= cal->hu[np - 1]) {
      r = cal->rho[np - 1];
    } else {
      int i = int(std::upper_bound(cal->hu, cal->hu + np, x) - cal->hu) - 1;  // hu[i] <= x < hu[i + 1]
      const double f = (x - cal->hu[i]) / (cal->hu[i + 1] - cal->hu[i]);
      r = cal->rho[i] + f * (cal->rho[i + 1] - cal->rho[i]);
    }
    rho[v] = r;
    if (mat) {
      int k = 0;
      while (k < cal->n_thresholds && x >= cal->mat_hu[k]) ++k;
      mat[v] = uint8_t(k);
    }
  }
  return MCX_OK;
}
