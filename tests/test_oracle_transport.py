"""Whole-path pins of the oracle transport (FP64, CPU).

- P10/P1 narrow-beam attenuation through a layered absorber (photoelectric
  only, electrons absorbed on the spot): the energy scored per layer and the
  transmitted count follow the exponential law exactly (multinomial test);
- per-history energy conservation to 1e-12;
- P8 CSDA: with hard events off, the mass path charged for soft loss equals
  R(E0) - R(E_final);
- P9 voxelisation invariance: the same homogeneous water seen as 1x1xN or as
  NxNxN voxels gives the same depth profile (photon transport, kerma mode);
- Eq. (1)-(3) estimator: per-history grouping of scores, merging of partial
  runs, determinism.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
import workloads as W

MC2 = 0.51099895000


def test_layered_absorber_exponential_law():
    e0 = 0.03
    rho = np.array([1.0, 0.3, 1.8, 1.0, 0.5, 2.2, 1.0, 1.0, 0.26, 1.3] * 2)
    dz = 0.5
    ph = W.slab_phantom(len(rho), dz, rho)
    t = W.transport(flags=O.NO_COMPTON | O.NO_RAYLEIGH | O.NO_PAIR, eabs=(0.01, 1e9, 1e9))
    tb = O.Tables(W.WATER, t)
    n = 40_000
    src = [W.pencil(0, e0, (50.0, 50.0, 0.0), n)]
    r = O.run(tb, ph, src, 3, 0, n, ledger=True)
    mu = tb.eval(O.MU_PHOTO, e0)
    assert mu == pytest.approx(4.94 * 3.0**-3, rel=1e-12)
    q = r.sum_q.reshape(len(rho)) / e0
    # each history deposits e0 in exactly one layer or escapes: q^2 = e0 * q
    assert np.allclose(r.sum_q2.reshape(len(rho)), e0 * r.sum_q.reshape(len(rho)), rtol=1e-12)
    cnt = np.round(q).astype(int)
    assert np.allclose(q, cnt, atol=1e-9)
    tau = np.concatenate([[0.0], np.cumsum(mu * rho * dz)])
    p = np.exp(-tau[:-1]) - np.exp(-tau[1:])
    p_esc = math.exp(-tau[-1])
    n_esc = int(round(r.ledger[:, O.LED_ESC].sum() / e0))
    obs = np.append(cnt, n_esc)
    exp = np.append(p, p_esc) * n
    assert obs.sum() == n
    chi = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi, len(obs) - 1) > 1e-4
    # narrow-beam transmission alone: binomial, 5 sigma
    assert abs(n_esc - n * p_esc) < 5 * math.sqrt(n * p_esc * (1 - p_esc))


@pytest.mark.parametrize("case", ["photon1", "photon8", "electron20", "positron5"])
def test_per_history_energy_conservation(case):
    if case == "photon1":
        ph, src, t, e_tot = W.water_cube(32, 20.0), [W.pencil(0, 1.0, (10, 10, 0), 300)], W.transport(), 1.0
    elif case == "photon8":
        ph, src, t, e_tot = W.water_cube(16, 10.0), [W.pencil(0, 8.0, (5, 5, 0), 300)], W.transport(), 8.0
    elif case == "electron20":
        ph, src, t, e_tot = W.water_cube(40, 10.0), [W.pencil(1, 20.0, (5, 5, 0), 40)], W.transport(100.0, 250), 20.0
    else:
        ph, src, t, e_tot = W.water_cube(20, 4.0), [W.pencil(2, 5.0, (2, 2, 0), 100)], W.transport(), 5.0 + 2 * MC2
    tb = O.Tables(W.WATER, t)
    n = src[0]["n_hist"]
    r = O.run(tb, ph, src, 9, 0, n, ledger=True)
    led = r.ledger
    bal = led[:, O.LED_DEP] + led[:, O.LED_ESC] + 2 * MC2 * led[:, O.LED_POSESC]
    assert np.max(np.abs(bal - e_tot)) <= 1e-12 * e_tot
    assert r.sum_q.sum() == pytest.approx(led[:, O.LED_DEP].sum(), rel=1e-12)
    if case == "photon8":
        assert r.stats.pair > 0 and r.stats.annih > 0
    if case == "electron20":
        assert r.stats.hard_in > 0 and r.stats.hard_br > 0 and r.stats.hard_el > 0


def test_csda_path_equals_range_difference():
    flags = O.NO_HARD_ELASTIC | O.NO_HARD_INELASTIC | O.NO_HARD_BREMS
    t = W.transport(flags=flags)
    tb = O.Tables(W.WATER, t)
    e0 = 2.0
    ph = W.water_cube(32, 8.0)
    n = 200
    r = O.run(tb, ph, [W.pencil(1, e0, (4.0, 4.0, 2.0), n)], 4, 0, n, ledger=True)
    led = r.ledger
    inside = led[:, O.LED_ESC] == 0
    assert inside.sum() > 0.8 * n
    r0 = tb.eval(O.ech(0, 1), e0)
    for row in led[inside]:
        efin = row[O.LED_EABS]
        assert efin <= 0.1
        assert row[O.LED_PATH] == pytest.approx(r0 - tb.eval(O.ech(0, 1), efin), rel=1e-11)
        # the absorbing step started above Eabs: overshoot below one max step
        tau_max = 0.05 * 0.2 / tb.eval(O.ech(0, 0), 0.2)
        assert 0.0 <= tb.eval(O.ech(0, 1), 0.1) - tb.eval(O.ech(0, 1), efin) <= tau_max


def test_voxelisation_invariance_photons():
    t = W.transport(eabs=(0.01, 1e9, 1e9))
    tb = O.Tables(W.WATER, t)
    n = 3000
    src = [W.pencil(0, 1.0, (10.0, 10.0, 0.0), n)]
    cube = W.water_cube(32, 20.0)
    slab = dict(shape=(32, 1, 1), voxel=(20.0, 20.0, 0.625), origin=(0.0, 0.0, 0.0),
                rho=np.ones((32, 1, 1)))
    a = O.run(tb, cube, src, 2, 0, n)
    b = O.run(tb, slab, src, 2, 0, n)
    da = a.sum_q.reshape(32, 32, 32).sum(axis=(1, 2))
    db = b.sum_q.reshape(32)
    assert np.allclose(da, db, rtol=1e-9, atol=1e-12)
    assert a.stats.compton == b.stats.compton and a.stats.flights == b.stats.flights


def test_voxelisation_invariance_electrons():
    """Depth voxels of 1 mm and of 2 cm must give the same depth dose of a
    10 MeV electron pencil: the soft loss of a Class II step is charged over
    the geometric length travelled up to the face or the step end that ends
    it, so the energy along a track does not depend on where faces interrupt
    steps.  (Charging the whole step's loss at a hinge that a later face cuts
    short moved 14% of the first 2 cm's dose and 76% of the third's.)
    Eight batches of 500 histories per geometry; z-test per 2 cm bin."""
    tb = O.Tables(W.WATER, W.transport(100.0, 250))
    n, nb = 500, 8
    src = [W.pencil(1, 10.0, (10.0, 10.0, 0.0), n * nb)]
    means, ses = [], []
    for dz, nz in ((0.1, 100), (2.0, 5)):
        ph = W.slab_phantom(nz, dz, np.ones(nz), 1, 20.0)
        q = np.array([O.run(tb, ph, src, 3, b * n, n).sum_q.reshape(5, -1).sum(axis=1) / n for b in range(nb)])
        means.append(q.mean(axis=0))
        ses.append(q.std(axis=0, ddof=1) / math.sqrt(nb))
    keep = means[1] > 0.01 * means[1].sum()
    z = (means[0] - means[1])[keep] / np.hypot(ses[0], ses[1])[keep]
    assert keep.sum() >= 3
    assert np.all(np.abs(z) < 4.0), z


def test_voxelisation_invariance_electrons_on_a_voxel_corner():
    """A 20 MeV electron pencil along a line where four columns of 1 mm voxels
    meet (the pencil of the electron workload sits on such a line) must give
    the depth dose of the same beam in 1 mm depth layers of one 2 cm column:
    the first hinge deflection sends the primary across a face at zero
    distance, so faces cut its steps right after their hinges.  The pending
    free path of the majorant process runs on across those cuts; redrawing
    it at each cut (a cut tied to the hinge, a fixed fraction of the sampled
    free path, is not a stopping time of that process) postponed the hard
    collisions and lowered the first layer's dose by 6%.  Sixteen batches of
    400 histories, the same histories in both geometries; z-test of the
    paired batch differences per 1 mm layer over the first 5 mm and per 5 mm
    over the 2 cm."""
    tb = O.Tables(W.WATER, W.transport(100.0, 250))
    n, nb = 400, 16
    src = [W.pencil(1, 20.0, (1.0, 1.0, 0.0), n * nb)]
    out = []
    for ph in (W.water_cube(20, 2.0), W.slab_phantom(20, 0.1, np.ones(20), 1, 2.0)):
        out.append(np.array([O.run(tb, ph, src, 4, b * n, n).sum_q.reshape(20, -1).sum(axis=1) / n
                             for b in range(nb)]))
    for w, m in ((1, 5), (5, 4)):
        a, b = (x.reshape(nb, -1, w).sum(axis=2)[:, :m] for x in out)
        dd = a - b
        z = dd.mean(0) / (dd.std(0, ddof=1) / math.sqrt(nb))
        assert np.all(np.abs(z) < 4.0), (w, z)


def test_estimator_per_history_grouping_single_voxel():
    """With one voxel, the per-history score is the history's total deposit:
    Sum q and Sum q^2 must equal the sums over the independent per-history
    ledger (Eq. (1)-(3))."""
    ph = W.water_cube(1, 20.0)
    src = [W.pencil(0, 1.0, (10.0, 10.0, 0.0), 500)]
    tb = O.Tables(W.WATER, W.transport())
    r = O.run(tb, ph, src, 1, 0, 500, ledger=True)
    q = r.ledger[:, O.LED_DEP]
    assert r.sum_q[0] == pytest.approx(q.sum(), rel=1e-13)
    assert r.sum_q2[0] == pytest.approx((q * q).sum(), rel=1e-13)
    d, s = O.dose(ph, r)
    mass = 20.0**3
    assert d.ravel()[0] == pytest.approx(q.mean() * 1e6 / mass, rel=1e-12)
    assert s.ravel()[0] == pytest.approx(q.std() / math.sqrt(500) * 1e6 / mass, rel=1e-9)


def test_partial_runs_merge_and_determinism():
    wl = W.workload("water_pencil_32", 1000)
    tb = O.Tables(wl["material"], wl["transport"])
    full = O.run(tb, wl["phantom"], wl["sources"], 1, 0, 1000, hashes=True)
    part = O.run(tb, wl["phantom"], wl["sources"], 1, 0, 400, hashes=True)
    h0 = part.hashes.copy()
    part = O.run(tb, wl["phantom"], wl["sources"], 1, 400, 600, result=part, hashes=True)
    assert np.allclose(full.sum_q, part.sum_q, rtol=1e-12, atol=1e-15)
    assert np.allclose(full.sum_q2, part.sum_q2, rtol=1e-12, atol=1e-15)
    assert np.array_equal(full.hashes[:400], h0)
    assert np.array_equal(full.hashes[400:], part.hashes)
    again = O.run(tb, wl["phantom"], wl["sources"], 1, 0, 1000, hashes=True)
    assert np.array_equal(again.sum_q, full.sum_q)
    assert np.array_equal(again.hashes, full.hashes)


def test_source_on_voxel_corner_locates_by_floor():
    """A pencil at (10, 10, 0) on a 0.625 cm grid sits on a voxel corner; floor
    puts it in column (16, 16): with electrons absorbed on the spot and
    photoelectric absorption only, the first-layer deposit lands there."""
    t = W.transport(flags=O.NO_COMPTON | O.NO_RAYLEIGH | O.NO_PAIR, eabs=(0.01, 1e9, 1e9))
    tb = O.Tables(W.WATER, t)
    r = O.run(tb, W.water_cube(32, 20.0), [W.pencil(0, 0.02, (10.0, 10.0, 0.0), 200)], 1, 0, 200)
    q = r.sum_q.reshape(32, 32, 32)
    assert q[:, 16, 16].sum() == pytest.approx(q.sum(), rel=1e-12)
