"""Pins of the oracle's interaction forcing (reading R11 of the oracle; the
variance-reduction extension of the main path).

- F = 1 is the analog run, history for history;
- forcing multiplies the hard-event rate by F: in a thin slab the number of
  hard bremsstrahlung events per electron is Poisson with mean
  F sigma_br(E0) rho t (E0 barely changes across the slab), while the
  weighted count keeps the analog mean sigma_br rho t; the same in a bone
  slab through the several-material path, with bone's sigma_br;
- forcing leaves every expectation unchanged: the weighted energy balance
  has mean E0 per history, and the depth-dose curve and the escaped energy
  agree with the analog run's within their combined standard errors, at
  step parameters small enough that the Class II result no longer depends
  on the step length (forced events end steps);
- bremsstrahlung splitting (S = 2) doubles the escaping photons of a thin
  slab and keeps the weighted escaped energy's mean;
- the gradient refuses a forced or split transport.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

MC2 = 0.51099895000
EL_IN, EL_BR = 4 + 3, 4 + 4  # electron hard inelastic and bremsstrahlung channels


def test_unit_forcing_is_the_analog_run():
    wl = W.workload("electron_200", 200)
    t1 = dict(wl["transport"], force_in=1.0, force_br=1.0, split_br=1)
    a = O.run(O.Tables(wl["material"], wl["transport"]), wl["phantom"], wl["sources"], 1, 0, 200, hashes=True,
              ledger=True)
    b = O.run(O.Tables(wl["material"], t1), wl["phantom"], wl["sources"], 1, 0, 200, hashes=True, ledger=True)
    assert np.array_equal(a.hashes, b.hashes)
    assert np.array_equal(a.ledger, b.ledger)


@pytest.mark.parametrize("slab", ["water", "bone_several_materials"])
def test_forced_bremsstrahlung_rate_in_a_thin_slab(slab):
    e0, dz, n, f = 10.0, 0.05, 4000, 25.0
    rho = 1.0 if slab == "water" else 1.85
    ph = W.slab_phantom(1, dz, np.array([rho]))
    base = W.transport(100.0, 250, flags=O.NO_HARD_ELASTIC | O.NO_HARD_INELASTIC | O.NO_COMPTON | O.NO_PHOTO
                       | O.NO_RAYLEIGH | O.NO_PAIR)
    src = [W.pencil(1, e0, (50.0, 50.0, 0.0), n)]
    m = W.WATER if slab == "water" else W.BONE
    if slab == "water":
        tables = lambda t: O.Tables(W.WATER, t)
    else:
        ph["mat"] = np.ones(ph["rho"].shape, dtype=np.uint8)
        tables = lambda t: [O.Tables(W.WATER, t), O.Tables(W.BONE, t), O.Tables(W.LUNG, t)]
    sig = O.Tables(m, base).eval(EL_BR, e0)
    mean = sig * rho * dz
    assert 1e-3 < mean < 0.1
    a = O.run(tables(base), ph, src, 2, 0, n, ledger=True)
    tf = dict(base, force_br=f)
    assert O.Tables(m, tf).eval(EL_BR, e0) == pytest.approx(f * sig, rel=1e-14)
    b = O.run(tables(tf), ph, src, 2, 0, n, ledger=True)
    # the step's energy falls by at most a few per cent over 0.05 cm: allow 5 sd plus 3 %
    for st, m in ((a.stats, mean * n), (b.stats, f * mean * n)):
        assert abs(st.hard_br - m) <= 5 * np.sqrt(m) + 0.03 * m, (st.hard_br, m)
    # photons escape: the weighted escaped photon energy has the analog mean
    # (each forced emission carries weight 1/F); the electron's own escape
    # energy is E0 minus its losses, which only a 1/F share of the forced
    # emissions apply
    esc_a, esc_b = a.ledger[:, O.LED_ESC], b.ledger[:, O.LED_ESC]
    bal = b.ledger[:, O.LED_DEP] + esc_b
    assert abs(bal.mean() - e0) <= 5 * bal.std(ddof=1) / np.sqrt(n)
    assert abs(esc_a.mean() - esc_b.mean()) <= 5 * np.hypot(esc_a.std(ddof=1), esc_b.std(ddof=1)) / np.sqrt(n)


def test_forcing_leaves_the_depth_dose_unbiased():
    e0, n = 10.0, 1500
    ph = W.slab_phantom(24, 0.25, np.ones(24))
    # forced events end Class II steps, so forcing shortens the steps; with
    # C1 = C2 = 0.05 the analog depth dose itself moves by ~1 % at the
    # entrance when the steps shorten (C1 = C2 = 0.01 gives the same shift):
    # compare where the step length no longer matters
    base = W.transport(100.0, 250, c1=0.01, c2=0.01)
    src = [W.pencil(1, e0, (50.0, 50.0, 0.0), n)]
    a = O.run(O.Tables(W.WATER, base), ph, src, 3, 0, n, ledger=True)
    b = O.run(O.Tables(W.WATER, dict(base, force_in=4.0, force_br=20.0, split_br=2)), ph, src, 3, 0, n, ledger=True)
    assert b.stats.hard_br > 10 * a.stats.hard_br
    assert b.stats.hard_in > 3 * a.stats.hard_in
    for r in (a, b):
        bal = r.ledger[:, O.LED_DEP] + r.ledger[:, O.LED_ESC] + 2 * MC2 * r.ledger[:, O.LED_POSESC]
        assert abs(bal.mean() - e0) <= 5 * bal.std(ddof=1) / np.sqrt(n) + 1e-12
    da, sa = O.dose(ph, a)
    db, sb = O.dose(ph, b)
    hi = da > 0.05 * da.max()
    z = (da - db)[hi] / np.hypot(sa, sb)[hi]
    assert np.all(np.abs(z) < 4.5), z
    assert abs(np.mean(z)) < 4.0 / np.sqrt(z.size) * 1.5
    ea, eb = a.ledger[:, O.LED_ESC], b.ledger[:, O.LED_ESC]
    assert abs(ea.mean() - eb.mean()) <= 5 * np.hypot(ea.std(ddof=1), eb.std(ddof=1)) / np.sqrt(n)


def test_bremsstrahlung_splitting_in_a_thin_slab():
    e0, dz, n = 10.0, 0.05, 4000
    ph = W.slab_phantom(1, dz, np.array([1.0]))
    base = W.transport(100.0, 250, flags=O.NO_HARD_ELASTIC | O.NO_HARD_INELASTIC | O.NO_COMPTON | O.NO_PHOTO
                       | O.NO_RAYLEIGH | O.NO_PAIR)
    src = [W.pencil(1, e0, (50.0, 50.0, 0.0), n)]
    a = O.run(O.Tables(W.WATER, dict(base, force_br=10.0)), ph, src, 5, 0, n, ledger=True)
    b = O.run(O.Tables(W.WATER, dict(base, force_br=10.0, split_br=2)), ph, src, 5, 0, n, ledger=True)
    # the primaries follow the same law: one escape each; photons escape unscattered
    ga, gb = a.stats.escaped - n, b.stats.escaped - n
    assert gb == 2 * b.stats.hard_br and ga == a.stats.hard_br
    assert abs(b.stats.hard_br - a.stats.hard_br) <= 5 * np.sqrt(a.stats.hard_br)
    esc_a, esc_b = a.ledger[:, O.LED_ESC], b.ledger[:, O.LED_ESC]
    assert abs(esc_a.mean() - esc_b.mean()) <= 5 * np.hypot(esc_a.std(ddof=1), esc_b.std(ddof=1)) / np.sqrt(n)


def test_forced_gradient_agrees_with_the_analog_gradient():
    """The score-function gradient with forcing and splitting (weighted
    deposits and soft-loss terms, analog photon-flight scores) has the
    analog estimator's expectation: 3 MeV electrons through water layers of
    varied density, a linear dose loss, step parameters C = 0.01 (forced
    events end steps, and the soft-loss term is taken on face-ended steps)."""
    import math
    rho = np.array([1.0, 0.5, 1.6, 1.0, 0.3, 1.2])
    ph = W.slab_phantom(rho.size, 0.25, rho)
    base = W.transport(100.0, 250, c1=0.01, c2=0.01)
    c = np.random.default_rng(9).uniform(-1.0, 1.0, size=ph["rho"].shape)
    n, nb = 500, 6
    src = [W.pencil(1, 3.0, (50.0, 50.0, 0.0), n)]

    def batches(t):
        tb = O.Tables(W.WATER, t)
        gs = []
        for b in range(nb):
            r = O.run(tb, ph, src, 40 + b, 0, n)
            d, _ = O.dose(ph, r)
            g, _ = O.gradient(tb, ph, src, 40 + b, 0, n, c, d)
            gs.append(g.ravel())
        gs = np.array(gs)
        return gs.mean(0), gs.std(0, ddof=1) / math.sqrt(nb)

    ma, sa = batches(base)
    mf, sf = batches(dict(base, force_in=4.0, force_br=20.0, split_br=2))
    z = (mf - ma) / np.hypot(sa, sf)
    print("z", np.round(z, 2))
    assert np.all(np.abs(z) < 4.5)
    assert abs(z.mean()) < 2.0
