"""Brute-force histogram pins of every sampler the oracle uses.

Each sampler's draws are binned and compared (chi-square) with the analytic
density of the distribution it must produce, written in its textbook form
(not the composition the sampler uses).  The paper's own validation compares
sampled distributions with reference cross sections the same way (Sec. 5.1).
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O
import workloads as W

MC2 = 0.51099895000
HC = 1.23984198e-2
N = 200_000


@pytest.fixture(scope="module")
def tb():
    return O.Tables(W.WATER, W.transport(100.0, 250))


def chi2_pvalue(x, pdf, a, b, bins=60, edges=None):
    if edges is None:
        edges = np.linspace(a, b, bins + 1)
    cnt, _ = np.histogram(x, bins=edges)
    w = np.array([integrate.quad(pdf, lo, hi, epsabs=0, epsrel=1e-10, limit=200)[0]
                  for lo, hi in zip(edges[:-1], edges[1:])])
    exp = w / w.sum() * len(x)
    keep = exp > 5
    chi = ((cnt[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    return stats.chi2.sf(chi, keep.sum() - 1)


@pytest.mark.parametrize("e", [0.05, 1.0, 6.0])
def test_klein_nishina(tb, e):
    kap, cos = tb.sample("compton", e, N)
    k = e / MC2
    kmin = 1 / (1 + 2 * k)
    assert np.allclose(cos, 1 - (1 - kap) / (k * kap), atol=1e-12)

    def pdf(p):  # dsigma/dP from the KN DCS in solid angle, dcos/dP = 1/(k P^2)
        c = 1 - (1 - p) / (k * p)
        return p * p * (p + 1 / p - (1 - c * c)) / (k * p * p)

    assert chi2_pvalue(kap, pdf, kmin, 1.0) > 1e-4


@pytest.mark.parametrize("e", [0.02, 0.1])
def test_rayleigh(tb, e):
    c, _ = tb.sample("rayleigh", e, N)
    q = e / HC

    def pdf(x):
        x2 = q * q * (1 - x) / 2
        return (1 + x * x) * (10.0 / (1 + 4.6 * x2) ** 2) ** 2

    edges = 1 - np.geomspace(2.0, 1e-5, 50)[::-1]
    edges = np.concatenate([[-1.0], np.sort(edges[edges > -1.0])])
    assert chi2_pvalue(c, pdf, -1, 1, edges=np.unique(np.append(edges, 1.0))) > 1e-4


def _moller(k, g):
    a = ((g - 1) / g) ** 2
    return 1 / k**2 + 1 / (1 - k) ** 2 + a - (1 - a) / (k * (1 - k))


def _bhabha(k, g):
    a = ((g - 1) / g) ** 2
    gp = g + 1
    b1 = a * (2 * gp**2 - 1) / (g * g - 1)
    b2 = a * (3 * gp**2 + 1) / gp**2
    b3 = a * 2 * (g - 1) * g / gp**2
    b4 = a * (g - 1) ** 2 / gp**2
    return (1 - b1 * k + b2 * k**2 - b3 * k**3 + b4 * k**4) / k**2


@pytest.mark.parametrize("e", [0.08, 1.0, 15.0])
def test_moller(tb, e):
    k, cp = tb.sample("moller", e, N)
    kc = 0.01 / e
    assert k.min() >= kc and k.max() <= 0.5
    g = 1 + e / MC2
    edges = np.geomspace(kc, 0.5, 61)
    assert chi2_pvalue(k, lambda x: _moller(x, g), kc, 0.5, edges=edges) > 1e-4


@pytest.mark.parametrize("e", [0.3, 15.0])
def test_moller_upper_half(tb, e):
    """The share of Moller transfers with k > 1/4 (where the bracket over k^2
    is largest relative to 1/k^2) against the DCS integrated by quadrature:
    a proposal that dropped or mis-weighted its flat part, or an acceptance
    bound that the bracket exceeds, moves this share by tens of percent."""
    from scipy.integrate import quad
    n = 1_000_000
    k, _ = tb.sample("moller", e, n, seed=11)
    kc = 0.01 / e
    g = 1 + e / MC2
    tot = quad(lambda x: _moller(x, g), kc, 0.5, limit=200, points=[2 * kc, 10 * kc])[0]
    upper = quad(lambda x: _moller(x, g), 0.25, 0.5)[0] / tot
    m = np.count_nonzero(k > 0.25)
    assert abs(m - n * upper) < 5.0 * np.sqrt(n * upper * (1 - upper)) + 1.0


def test_moller_envelope_bound():
    """k^2 times the Moller bracket stays below 1 + 5 a k^2 on (0, 1/2], with
    equality at 1/2, for every a in [0, 1] (the sampler's acceptance bound)."""
    kk = np.linspace(1e-4, 0.5, 20001)
    for a in np.linspace(0.0, 1.0, 41):
        f = kk**2 * (1 / kk**2 + 1 / (1 - kk) ** 2 + a - (1 - a) / (kk * (1 - kk)))
        assert np.all(f <= 1 + 5 * a * kk**2 + 1e-12)
        assert abs(f[-1] - (1 + 1.25 * a)) < 1e-12


@pytest.mark.parametrize("e", [0.08, 1.0, 15.0])
def test_bhabha(tb, e):
    k, _ = tb.sample("bhabha", e, N)
    kc = 0.01 / e
    g = 1 + e / MC2
    edges = np.geomspace(kc, 1.0, 61)
    assert chi2_pvalue(k, lambda x: _bhabha(x, g), kc, 1.0, edges=edges) > 1e-4


@pytest.mark.parametrize("e", [0.5, 12.0])
def test_bremsstrahlung(tb, e):
    w, c = tb.sample("brems", e, N)
    edges = np.geomspace(0.01, e, 41)
    assert chi2_pvalue(w, lambda x: 1 / x, 0.01, e, edges=edges) > 1e-4
    beta = math.sqrt(e * (e + 2 * MC2)) / (e + MC2)
    edges = 1 - np.geomspace(2.0, 1e-4, 40)
    edges = np.unique(np.concatenate([edges, [1.0]]))
    assert chi2_pvalue(c, lambda x: (1 - beta * x) ** -2, -1, 1, edges=edges) > 1e-4


@pytest.mark.parametrize("e", [0.2, 2.0])
def test_hard_elastic(tb, e):
    mu, _ = tb.sample("hard_elastic", e, N)
    muc, eta = tb.mu_cut(0, e), tb.screening(e)
    assert mu.min() >= muc * (1 - 1e-12) and mu.max() <= 1.0
    edges = np.geomspace(max(muc, 1e-12), 1.0, 50)
    assert chi2_pvalue(mu, lambda x: (x + eta) ** -2, muc, 1, edges=edges) > 1e-4


@pytest.mark.parametrize("m", [1e-3, 0.05, 0.3])
def test_soft_deflection(tb, m):
    mu, _ = tb.sample("soft", m, N)
    a = O.soft_a(m)
    assert abs(mu.mean() - m) < 5 * mu.std() / math.sqrt(N)
    edges = np.concatenate([[0.0], np.geomspace(a / 100, 1.0, 50)])
    assert chi2_pvalue(mu, lambda x: (x + a) ** -2, 0, 1, edges=edges) > 1e-4


def test_pair(tb):
    e = 8.0
    eps, c = tb.sample("pair", e, N)
    assert stats.kstest(eps, "uniform").pvalue > 1e-4
    # the electron angle uses the electron's own beta: check on a slice
    sel = (eps > 0.45) & (eps < 0.55)
    t = 0.5 * (e - 2 * MC2)
    beta = math.sqrt(t * (t + 2 * MC2)) / (t + MC2)
    edges = np.unique(np.concatenate([1 - np.geomspace(2.0, 1e-3, 30), [1.0]]))
    # beta varies by +-2% over the slice; compare with the slice-centre law
    assert chi2_pvalue(c[sel], lambda x: (1 - beta * x) ** -2, -1, 1, edges=edges) > 1e-6


@pytest.mark.parametrize("e", [0.05, 1.0, 6.0])
def test_free_path_exponential(tb, e):
    tau, _ = tb.sample("free_path", e, N)
    mu = sum(tb.eval(c, e) for c in range(4))
    assert stats.kstest(tau, "expon", args=(0, 1 / mu)).pvalue > 1e-4


def test_annihilation_isotropic(tb):
    c, _ = tb.sample("annih", 0.0, N)
    assert stats.kstest((c + 1) / 2, "uniform").pvalue > 1e-4
