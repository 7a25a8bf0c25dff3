"""Pins of the oracle's two-photon annihilation of positrons in flight
(reading R9 of the oracle; the "next" extension of the at-rest-only
annihilation of the main path).

- Heitler's total cross section against its two textbook limits: Dirac's
  nonrelativistic pi r_e^2 / beta and the ultra-relativistic
  pi r_e^2 (ln 2 gamma - 1) / gamma, and against a quadrature of the DCS;
- it falls with energy over the whole grid, which the majorant relies on;
- the softer photon's energy fraction against the DCS (Kolmogorov-Smirnov
  with the CDF integrated numerically) and its polar cosine against energy
  and momentum conservation (the other photon must come out massless);
- the transport: with hard channels off and photons absorbed on the spot,
  5 MeV positrons in a large water cube annihilate in flight with
  probability 1 - exp(-int Sigma_an / S dE) (binomial test); the majorant
  bounds every hard selection; energy is conserved per history.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O
import workloads as W

MC2 = 0.51099895000
R_E = 2.8179403262e-13
NE = 6.02214076e23 * W.WATER["z_mol"] / W.WATER["a_mol"]


def tables(flags=O.ANNIH_FLIGHT, **kw):
    return O.Tables(W.WATER, W.transport(100.0, 250, flags=flags, **kw))


def heitler_dcs(e, z):
    """Heitler's DCS per electron (cm^2) in the energy fraction z of one
    photon, over the full range (both photons)."""
    g = 1.0 + e / MC2
    s = lambda x: -(g + 1) ** 2 + (g * g + 4 * g + 1) / x - 1.0 / x ** 2
    return math.pi * R_E ** 2 / ((g + 1) * (g * g - 1)) * (s(z) + s(1 - z)) / 2.0


def zmin(e):
    g = 1.0 + e / MC2
    return 1.0 / (g + 1 + math.sqrt(g * g - 1))


def test_heitler_limits_and_quadrature():
    tb = tables()
    # nonrelativistic limit (Dirac): sigma -> pi r_e^2 / beta per electron
    for e, tol in ((1e-4, 1e-6), (1e-3, 1e-5), (1e-2, 1e-3)):
        g = 1 + e / MC2
        beta = math.sqrt(1 - 1 / g ** 2)
        assert tb.sigma_annih(e) * beta / (math.pi * R_E ** 2 * NE) == pytest.approx(1.0, abs=tol)
    # ultra-relativistic limit: pi r_e^2 (ln 2 gamma - 1) / gamma
    for e, tol in ((1e4, 1e-3), (1e5, 1e-4)):
        g = 1 + e / MC2
        assert tb.sigma_annih(e) * g / (math.pi * R_E ** 2 * NE * (math.log(2 * g) - 1)) == pytest.approx(1.0, abs=tol)
    # the total is the integral of the DCS
    for e in (0.05, 0.5, 5.0, 50.0):
        z0 = zmin(e)
        val, _ = integrate.quad(lambda z: heitler_dcs(e, z), z0, 1 - z0, epsabs=0, epsrel=1e-11, limit=200)
        assert tb.sigma_annih(e) == pytest.approx(NE * val, rel=1e-8)


def test_heitler_falls_with_energy():
    tb = tables()
    e = np.geomspace(1e-3, 100.0, 4001)
    s = np.array([tb.sigma_annih(x) for x in e])
    assert np.all(np.diff(s) < 0)


@pytest.mark.parametrize("e", [0.2, 2.0, 20.0])
def test_annihilation_photon_fraction_and_kinematics(e):
    tb = tables()
    n = 60_000
    z, cos_a = tb.sample("annih_flight", e, n, seed=11)
    z0 = zmin(e)
    assert np.all((z >= z0 * (1 - 1e-12)) & (z <= 0.5))
    # the softer photon's fraction follows S(z) + S(1 - z) on [zmin, 1/2]
    grid = np.linspace(z0, 0.5, 2001)
    pdf = np.array([heitler_dcs(e, x) for x in grid])
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    assert stats.kstest(z, lambda x: np.interp(x, grid, cdf)).pvalue > 1e-3
    # energy and momentum: the second photon, P z - k_a n_a, must be massless
    g = 1 + e / MC2
    pmom = math.sqrt(g * g - 1) * MC2
    etot = e + 2 * MC2
    ka, kb = z * etot, (1 - z) * etot
    pb2 = pmom ** 2 - 2 * pmom * ka * cos_a + ka ** 2
    assert np.allclose(pb2, kb ** 2, rtol=1e-9)


@pytest.mark.parametrize("nvox", [1, 8])
def test_in_flight_fraction_of_slowing_down_positrons(nvox):
    """Hard channels off: the positron loses energy continuously (CSDA) and
    annihilates in flight at the rate Sigma_an(E) per g/cm^2 along its path,
    so it does so before reaching Eabs with probability
    1 - exp(-int_Eabs^E0 Sigma_an(E) / S(E) dE).  Photons are absorbed where
    they are made, so the only charged particles are the positrons: in-flight
    annihilations = annihilations - absorptions.  One 40 cm voxel, and 5 cm
    voxels around a corner start, where faces interrupt many steps: the soft
    loss is charged over the length travelled, so the share is the same
    (charging a whole step's loss at a hinge that a face then cut short
    lowered it by 3% there)."""
    e0, eabs = 5.0, 0.1
    hard_off = O.NO_HARD_ELASTIC | O.NO_HARD_INELASTIC | O.NO_HARD_BREMS
    t = W.transport(100.0, 250, flags=hard_off | O.ANNIH_FLIGHT, eabs=(1e9, eabs, eabs))
    tb = O.Tables(W.WATER, t)
    n = 40_000
    ph = W.water_cube(nvox, 40.0)
    r = O.run(tb, ph, [W.pencil(2, e0, (20.0, 20.0, 20.0), n)], 5, 0, n, ledger=True)
    st = r.stats.as_dict()
    assert st["escaped"] == 0
    flight = st["annih"] - st["absorbed"]
    # S is the piecewise power-law interpolant: a dense trapezoid in ln E
    le = np.linspace(math.log(eabs), math.log(e0), 20001)
    f = np.array([math.exp(x) * tb.sigma_annih(math.exp(x)) / tb.eval(O.ech(1, 0), math.exp(x)) for x in le])
    val = float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(le)))
    p = 1 - math.exp(-val)
    print("in-flight", flight / n, "expected", p)
    assert abs(flight - n * p) < 5 * math.sqrt(n * p * (1 - p))
    bal = r.ledger[:, O.LED_DEP] + r.ledger[:, O.LED_ESC] + 2 * MC2 * r.ledger[:, O.LED_POSESC]
    assert np.max(np.abs(bal - (e0 + 2 * MC2))) <= 1e-12 * (e0 + 2 * MC2)


@pytest.mark.parametrize("flags", [O.ANNIH_FLIGHT, O.ANNIH_FLIGHT | O.STRAGGLING])
def test_annihilation_majorant_and_conservation(flags):
    for wl, n, etot in ((dict(W.workload("water_pencil_32"), phantom=W.water_cube(20, 4.0),
                              sources=[W.pencil(2, 5.0, (2.0, 2.0, 0.0), 400)]), 400, 5.0 + 2 * MC2),
                        (dict(W.workload("water_pencil_32"), phantom=W.water_cube(16, 10.0),
                              sources=[W.pencil(0, 8.0, (5.0, 5.0, 0.0), 400)]), 400, 8.0)):
        t = dict(wl["transport"], flags=flags)
        tb = O.Tables(wl["material"], t)
        r = O.run(tb, wl["phantom"], wl["sources"], 2, 0, n, ledger=True)
        st = r.stats.as_dict()
        assert st["maj_excess"] == 0
        bal = r.ledger[:, O.LED_DEP] + r.ledger[:, O.LED_ESC] + 2 * MC2 * r.ledger[:, O.LED_POSESC]
        assert np.max(np.abs(bal - etot)) <= 1e-12 * etot


def test_gradient_with_annihilation_in_flight():
    """The gradient accepts annihilation in flight (an e+ hard event, which
    the estimator does not score) and refuses straggling.  With e+- absorbed
    where they are created no positron flies, so the flag changes nothing:
    the gradient is the one without it, bit for bit."""
    ph = W.water_cube(8, 8.0)
    ph["rho"] = np.random.default_rng(2).uniform(0.5, 1.8, size=ph["rho"].shape)
    src = [W.pencil(0, 8.0, (4.0, 4.0, 0.0), 2000)]
    c = np.random.default_rng(3).uniform(-1, 1, size=ph["rho"].shape)
    out = []
    for flags in (0, O.ANNIH_FLIGHT):
        tb = O.Tables(W.WATER, W.transport(flags=flags, eabs=(0.01, 1e9, 1e9)))
        r = O.run(tb, ph, src, 1, 0, 2000)
        d, _ = O.dose(ph, r)
        out.append(O.gradient(tb, ph, src, 1, 0, 2000, c, d)[0])
    assert np.array_equal(out[0], out[1])
    tb = O.Tables(W.WATER, W.transport(flags=O.STRAGGLING))
    with pytest.raises(RuntimeError):
        O.gradient(tb, ph, src, 1, 0, 10, c, c)
