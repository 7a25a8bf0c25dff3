"""Pins of the oracle's soft energy-loss straggling (reading R8 of the oracle;
an extension of the Class II step of Sec. 5.2, whose soft loss is otherwise
the deterministic CSDA value).

- the second moment of the soft DCS per unit mass path against a numerical
  integral of W^2 times the full Moller DCS (a textbook formula written out
  here) below the collision cutoff, plus the b/W bremsstrahlung DCS below the
  radiative cutoff;
- the sampler against its target laws in each regime: Kolmogorov-Smirnov
  against scipy's truncated normal and uniform laws, the point mass of the
  two-mode law by a binomial test, and the first two moments;
- the whole step: 10 MeV electrons through one thin slab voxel with the hard
  channels off lose exactly one straggled soft loss, charged over the length
  travelled to the far face (the face distance when the face comes before
  the hinge, a little more when the hinge deflects the track first), so the
  mean and second moment of the deposited energy follow from the range
  tables and the hinge law;
- per-history energy conservation with straggling on.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O
import workloads as W

MC2 = 0.51099895000
R_E = 2.8179403262e-13
N_A = 6.02214076e23


def moller_dcs(e, w):
    """Moller DCS per electron, cm^2/MeV, for an electron of kinetic energy e
    transferring w (e.g. ICRU Report 37, or any text on binary collisions)."""
    g = e / MC2 + 1.0
    beta2 = 1.0 - 1.0 / g ** 2
    pref = 2.0 * math.pi * R_E ** 2 * MC2 / beta2
    return pref * (1.0 / w ** 2 + 1.0 / (e - w) ** 2 + 1.0 / (e + MC2) ** 2
                   - (2.0 * e + MC2) * MC2 / ((e + MC2) ** 2 * w * (e - w)))


def tables(flags=0, **kw):
    return O.Tables(W.WATER, W.transport(flags=flags | O.STRAGGLING, **kw))


@pytest.mark.parametrize("e", [0.5, 1.0, 6.0, 20.0])
def test_soft_second_moment_against_the_moller_and_bremsstrahlung_dcs(e):
    tb = tables()
    wcc = wcr = 0.01
    ne = N_A * W.WATER["z_mol"] / W.WATER["a_mol"]
    col, _ = integrate.quad(lambda w: w * w * moller_dcs(e, w), 0.0, wcc, epsabs=0, epsrel=1e-12)
    rad, _ = integrate.quad(lambda w: w * w * W.WATER["brems_b"] / w, 0.0, wcr, epsabs=0, epsrel=1e-12)
    ref = ne * col + rad
    # the oracle keeps the leading 1/W^2 term of the collision DCS: they
    # differ at order Wcc/E
    assert tb.soft_omega2(0, e) == pytest.approx(ref, rel=wcc / e)
    # positrons: the same leading term below the cutoff
    assert tb.soft_omega2(1, e) == pytest.approx(tb.soft_omega2(0, e), rel=1e-15)


def test_soft_second_moment_with_hard_channels_off():
    e = 6.0
    base = tables()
    nobr = tables(O.NO_HARD_BREMS)
    noin = tables(O.NO_HARD_INELASTIC)
    b = W.WATER["brems_b"]
    extra, _ = integrate.quad(lambda w: w * w * b / w, 0.01, e, epsabs=0, epsrel=1e-12)
    assert nobr.soft_omega2(0, e) - base.soft_omega2(0, e) == pytest.approx(extra, rel=1e-10)
    # no hard collisions: the leading term runs up to the largest transfer,
    # E/2 for electrons and E for positrons
    g = e / MC2 + 1.0
    k = 2 * math.pi * R_E ** 2 * MC2 * N_A * W.WATER["z_mol"] / W.WATER["a_mol"] / (1 - 1 / g ** 2)
    assert noin.soft_omega2(0, e) - base.soft_omega2(0, e) == pytest.approx(k * (e / 2 - 0.01), rel=1e-10)
    assert noin.soft_omega2(1, e) - base.soft_omega2(1, e) == pytest.approx(k * (e - 0.01), rel=1e-10)


def test_straggling_gaussian_regime_is_a_truncated_normal():
    m, om2 = 1.0, 0.04  # mean 5 sd
    x = O.sample_straggle(m, om2, 100_000, seed=3)
    c = m / math.sqrt(om2)
    law = stats.truncnorm(-c, c, loc=m, scale=math.sqrt(om2))
    assert stats.kstest(x, law.cdf).pvalue > 1e-3
    assert x.min() > 0.0 and x.max() < 2 * m
    # edge of the regime: truncation at 3.01 sd removes visible tails
    m, om2 = 0.301, 0.01
    x = O.sample_straggle(m, om2, 100_000, seed=4)
    c = m / 0.1
    law = stats.truncnorm(-c, c, loc=m, scale=0.1)
    assert stats.kstest(x, law.cdf).pvalue > 1e-3
    assert abs(x.var() / law.var() - 1) < 0.02


def test_straggling_uniform_regime():
    m, om2 = 1.0, 0.2  # sqrt(3) sd < m <= 3 sd
    x = O.sample_straggle(m, om2, 100_000, seed=5)
    h = math.sqrt(3 * om2)
    assert stats.kstest(x, stats.uniform(m - h, 2 * h).cdf).pvalue > 1e-3
    n = x.size
    assert abs(x.mean() - m) < 5 * math.sqrt(om2 / n)
    assert abs(x.var() / om2 - 1) < 5 * math.sqrt(0.8 / n)  # var of (x-m)^2 / om2^2 is 4/5


def test_straggling_two_mode_regime():
    m, om2 = 0.5, 1.0  # m < sqrt(3) sd
    n = 100_000
    x = O.sample_straggle(m, om2, n, seed=6)
    s2 = om2 + m * m
    a = 1 - 4 * m * m / (3 * s2)
    w = 1.5 * s2 / m
    zero = x == 0.0
    assert abs(zero.mean() - a) < 5 * math.sqrt(a * (1 - a) / n)
    assert stats.kstest(x[~zero], stats.uniform(0.0, w).cdf).pvalue > 1e-3
    assert abs(x.mean() - m) < 5 * x.std() / math.sqrt(n)
    assert abs((x ** 2).mean() - s2) < 5 * (x ** 2).std() / math.sqrt(n)
    # no mean loss on a positive path: the two-mode branch gives 0
    assert not O.sample_straggle(0.0, 1.0, 10).any()
    # zero variance (a zero path): the loss is the CSDA value, nothing drawn
    assert np.all(O.sample_straggle(0.3, 0.0, 10) == 0.3)


@pytest.mark.parametrize("straggle", [False, True])
def test_thin_slab_loss_is_one_straggled_step(straggle):
    """10 MeV electrons enter a 1 mm water slab (one voxel) with the hard
    channels off: the step is capped at len = C2 E / S_s > d, its hinge lies at
    a uniform fraction u of it, and (but for the rare track that the hinge
    turns back) the electron leaves after one step, charged over the length
    it travelled to the far face: exactly d when u >= d/len (the face comes
    first), else the distance to the hinge plus the deflected path from it to
    the face, a little more than d.  The mass path the history charged tells
    the two apart.  Without straggling the deposited energy is the CSDA loss
    over that path; with straggling a loss of that mean and of variance
    path * Omega^2(E0): the face-first set by its exact two-mode law, the
    hinge-first set (a different path per history) by its first two moments."""
    e0, d = 10.0, 0.1
    flags = O.NO_HARD_ELASTIC | O.NO_HARD_INELASTIC | O.NO_HARD_BREMS | (O.STRAGGLING if straggle else 0)
    t = W.transport(100.0, 250, flags=flags)
    tb = O.Tables(W.WATER, t)
    ph = W.slab_phantom(1, d, [1.0])
    n = 60_000
    r = O.run(tb, ph, [W.pencil(1, e0, (50.0, 50.0, 0.0), n)], 9, 0, n, ledger=True)
    dep = r.ledger[:, O.LED_DEP]
    path = r.ledger[:, O.LED_PATH]
    assert np.allclose(dep + r.ledger[:, O.LED_ESC], e0, rtol=0, atol=1e-12 * e0)
    ss = tb.eval(O.ech(0, 0), e0)
    length = 0.05 * e0 / ss
    assert length > d
    r0 = tb.eval(O.ech(0, 1), e0)
    om2 = tb.soft_omega2(0, e0)
    face = np.isclose(path, d, rtol=1e-12)
    hinge = (path > d * (1 + 1e-12)) & (path < 1.2 * d) & (r.ledger[:, O.LED_ESC] > 0)
    assert (face | hinge).mean() > 0.995
    p_face = 1.0 - d / length
    nf = face.sum() + hinge.sum()
    assert abs(face.sum() / nf - p_face) < 5 * math.sqrt(p_face * (1 - p_face) / nf)
    # the CSDA loss over each history's charged path
    m_path = e0 - np.array([tb.range_inverse(0, r0 - x) for x in path])
    if not straggle:
        assert np.allclose(dep[face | hinge], m_path[face | hinge], rtol=1e-12)
        return
    # face first: one path d, the two-mode regime, whose law has exactly the
    # target mean and variance
    m, v, x = m_path[face][0], d * om2, dep[face]
    assert m * m < 3 * v
    k = x.size
    assert abs(x.mean() - m) < 5 * x.std() / math.sqrt(k)
    assert abs((x ** 2).mean() - (v + m * m)) < 5 * (x ** 2).std() / math.sqrt(k)
    s2 = v + m * m
    a = 1 - 4 * m * m / (3 * s2)
    assert abs((x == 0).mean() - a) < 5 * math.sqrt(a * (1 - a) / k)
    assert stats.kstest(x[x > 0], stats.uniform(0.0, 1.5 * s2 / m).cdf).pvalue > 1e-3
    # hinge first: per history the loss has mean m(path) and second moment
    # path * Omega^2 + m(path)^2
    x, m, v = dep[hinge], m_path[hinge], path[hinge] * om2
    k = x.size
    assert k > 500
    r1, r2 = x - m, x ** 2 - (v + m * m)
    assert abs(r1.mean()) < 5 * r1.std() / math.sqrt(k)
    assert abs(r2.mean()) < 5 * r2.std() / math.sqrt(k)


def test_energy_conservation_with_straggling():
    for ph, src, t, e_tot in (
            (W.water_cube(32, 20.0), [W.pencil(0, 1.0, (10, 10, 0), 300)], W.transport(flags=O.STRAGGLING), 1.0),
            (W.water_cube(20, 20.0), [W.pencil(1, 20.0, (10, 10, 0), 40)],
             W.transport(100.0, 250, flags=O.STRAGGLING), 20.0),
            (W.water_cube(20, 20.0), [W.pencil(2, 5.0, (10, 10, 0), 60)],
             W.transport(100.0, 250, flags=O.STRAGGLING), 5.0 + 2 * MC2)):
        tb = O.Tables(W.WATER, t)
        n = src[0]["n_hist"]
        r = O.run(tb, ph, src, 1, 0, n, ledger=True)
        bal = r.ledger[:, O.LED_DEP] + r.ledger[:, O.LED_ESC] + 2 * MC2 * r.ledger[:, O.LED_POSESC]
        assert np.max(np.abs(bal - e_tot)) <= 1e-12 * e_tot


def test_gradient_refuses_straggling():
    t = W.transport(flags=O.STRAGGLING)
    tb = O.Tables(W.WATER, t)
    ph = W.water_cube(8, 8.0)
    with pytest.raises(Exception):
        O.gradient(tb, ph, [W.pencil(0, 1.0, (4, 4, 0), 10)], 1, 0, 10, np.ones((8, 8, 8)))


@pytest.mark.parametrize("straggle", [False, True])
def test_hard_event_majorant_covers_every_step_end(straggle):
    """The delta method needs the majorant to bound the hard cross sections at
    the energy a step ends at.  A straggled loss can exceed the step's CSDA
    loss, so with straggling the majorant interval is widened (R14): no hard
    selection of a 20 MeV electron or 1 MeV photon run may see cross sections
    above the majorant (without the widening about 3% of the 20 MeV
    electron's selections did)."""
    for wl, n in ((dict(W.workload("electron_200"), phantom=W.water_cube(50, 10.0),
                        sources=[W.pencil(1, 20.0, (5.0, 5.0, 0.0), 200)]), 200),
                  (dict(W.workload("water_pencil_32"), sources=[W.pencil(0, 1.0, (10.0, 10.0, 0.0), 3000)]), 3000),
                  (dict(W.workload("water_pencil_32"), phantom=W.water_cube(20, 4.0),
                        sources=[W.pencil(2, 5.0, (2.0, 2.0, 0.0), 300)]), 300)):
        t = dict(wl["transport"], flags=O.STRAGGLING if straggle else 0)
        tb = O.Tables(wl["material"], t)
        r = O.run(tb, wl["phantom"], wl["sources"], 1, 0, n)
        st = r.stats.as_dict()
        assert st["hard_el"] + st["hard_in"] + st["delta"] > 0
        assert st["maj_excess"] == 0
