"""Pins of the oracle's density gradient (score-function estimator).

- Closed form: a layered photoelectric-only absorber with electrons absorbed
  where they are created has E[q_j] = E0 T_j (1 - e^{-mu rho_j dz}),
  T_j = exp(-mu dz sum_{i<j} rho_i); the gradient of a linear dose loss
  sum_j c_j D_j w.r.t. every layer density is known exactly.
- Common-random-number central finite differences of the oracle's own dose
  (full photon physics, electrons absorbed on the spot) on sampled voxels.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _grad_batches(tb, ph, src, c, nb, nper, seed0=100):
    gs = []
    for b in range(nb):
        r = O.run(tb, ph, src, seed0 + b, 0, nper)
        d, _ = O.dose(ph, r)
        g, _ = O.gradient(tb, ph, src, seed0 + b, 0, nper, c, d)
        gs.append(g.ravel())
    gs = np.array(gs)
    return gs.mean(axis=0), gs.std(axis=0, ddof=1) / math.sqrt(nb)


def test_layered_absorber_gradient_closed_form():
    e0, dz = 0.03, 0.5
    rho = np.array([1.0, 0.3, 1.8, 1.0, 0.5, 2.2, 1.0, 1.3, 0.26, 1.1])
    nz = rho.size
    ph = W.slab_phantom(nz, dz, rho)
    t = W.transport(flags=O.NO_COMPTON | O.NO_RAYLEIGH | O.NO_PAIR, eabs=(0.01, 1e9, 1e9))
    tb = O.Tables(W.WATER, t)
    mu = tb.eval(O.MU_PHOTO, e0)
    vol = 100.0 * 100.0 * dz
    rng = np.random.default_rng(5)
    c = rng.uniform(-1.0, 1.0, size=nz).reshape(nz, 1, 1)
    # exact gradient of L = sum_j c_j D_j
    cum = np.concatenate([[0.0], np.cumsum(rho * dz)])
    T = np.exp(-mu * cum[:-1])
    a = 1.0 - np.exp(-mu * rho * dz)
    eq = e0 * T * a
    D = eq * 1e6 / (rho * vol)
    exact = np.zeros(nz)
    for k in range(nz):
        s = 0.0
        for j in range(nz):
            if k < j:
                deq = e0 * (-mu * dz) * T[j] * a[j]
            elif k == j:
                deq = e0 * T[j] * mu * dz * math.exp(-mu * rho[j] * dz)
            else:
                deq = 0.0
            dD = 1e6 / (rho[j] * vol) * deq - (D[j] / rho[j] if k == j else 0.0)
            s += c.ravel()[j] * dD
        exact[k] = s
    src = [W.pencil(0, e0, (50.0, 50.0, 0.0), 20000)]
    mean, sem = _grad_batches(tb, ph, src, c, 10, 20000)
    z = (mean - exact) / sem
    print("z", np.round(z, 2))
    assert np.all(np.abs(z) < 4.5)
    assert abs(z.mean()) < 1.5


def test_kerma_mode_gradient_vs_crn_finite_differences():
    """Photon physics in full, electrons absorbed where created: the
    score-function gradient is unbiased; compare it with central finite
    differences (+-5%, common random numbers) of a linear dose loss."""
    ph = W.water_cube(8, 8.0)
    rng = np.random.default_rng(3)
    ph["rho"] = rng.uniform(0.5, 1.8, size=ph["rho"].shape)
    t = W.transport(eabs=(0.01, 1e9, 1e9))
    tb = O.Tables(W.WATER, t)
    n = 20000
    src = [W.rect_field(0, 2.0, (4.0, 4.0, 0.0), (4.0, 4.0), n)]
    c = rng.uniform(-1.0, 1.0, size=ph["rho"].shape)
    mean, sem = _grad_batches(tb, ph, src, c, 8, n)
    mean = mean.reshape(ph["rho"].shape)
    sem = sem.reshape(ph["rho"].shape)
    voxels = [(1, 4, 4), (3, 3, 4), (5, 4, 3), (2, 5, 5)]
    h = 0.05
    for v in voxels:
        fds = []
        for b in range(8):
            vals = []
            for sgn in (+1, -1):
                p2 = dict(ph, rho=ph["rho"].copy())
                p2["rho"][v] *= 1 + sgn * h
                r = O.run(tb, p2, src, 500 + b, 0, n)
                d, _ = O.dose(p2, r)
                vals.append(float((c * d).sum()))
            fds.append((vals[0] - vals[1]) / (2 * h * ph["rho"][v]))
        fd = np.mean(fds)
        fd_sem = np.std(fds, ddof=1) / math.sqrt(len(fds))
        z = (mean[v] - fd) / math.sqrt(sem[v] ** 2 + fd_sem ** 2)
        print(v, mean[v], sem[v], fd, fd_sem, z)
        assert abs(z) < 4.0


def test_two_material_layered_absorber_gradient_closed_form():
    """Layers of water and bone (photoelectric only, electrons absorbed where
    created): E[q_j] = E0 T_j (1 - e^{-mu_j rho_j dz}), T_j =
    exp(-dz sum_{i<j} mu_i rho_i) with each layer's own mu_m; the gradient of
    a linear dose loss is known exactly and the several-material score must
    reproduce it."""
    e0, dz = 0.03, 0.5
    rho = np.array([1.0, 0.3, 1.8, 1.0, 0.5, 2.2, 1.0, 1.3, 0.26, 1.1])
    mat = np.array([0, 0, 1, 0, 0, 1, 1, 0, 0, 1], dtype=np.uint8)
    nz = rho.size
    ph = W.slab_phantom(nz, dz, rho)
    ph["mat"] = np.broadcast_to(mat[:, None, None], ph["rho"].shape).copy()
    t = W.transport(flags=O.NO_COMPTON | O.NO_RAYLEIGH | O.NO_PAIR, eabs=(0.01, 1e9, 1e9))
    tbs = [O.Tables(W.WATER, t), O.Tables(W.BONE, t)]
    mu = np.array([tb.eval(O.MU_PHOTO, e0) for tb in tbs])[mat]
    vol = 100.0 * 100.0 * dz
    rng = np.random.default_rng(7)
    c = rng.uniform(-1.0, 1.0, size=nz)
    cum = np.concatenate([[0.0], np.cumsum(mu * rho * dz)])
    T = np.exp(-cum[:-1])
    a = 1.0 - np.exp(-mu * rho * dz)
    D = e0 * T * a * 1e6 / (rho * vol)
    exact = np.zeros(nz)
    for k in range(nz):
        for j in range(nz):
            if k < j:
                deq = e0 * (-mu[k] * dz) * T[j] * a[j]
            elif k == j:
                deq = e0 * T[j] * mu[j] * dz * math.exp(-mu[j] * rho[j] * dz)
            else:
                deq = 0.0
            exact[k] += c[j] * (1e6 / (rho[j] * vol) * deq - (D[j] / rho[j] if k == j else 0.0))
    src = [W.pencil(0, e0, (50.0, 50.0, 0.0), 20000)]
    mean, sem = _grad_batches(tbs, ph, src, c.reshape(nz, 1, 1), 10, 20000)
    z = (mean - exact) / sem
    print("z", np.round(z, 2))
    assert np.all(np.abs(z) < 4.5)
    assert abs(z.mean()) < 1.5
    # the one-material score (water's mu everywhere) misses the bone layers
    wrong = O.Tables(W.WATER, t).eval(O.MU_PHOTO, e0)
    assert mu.max() / wrong > 5.0


def test_soft_deflection_score_reproduces_moment_derivatives():
    """Term C of the Class II gradient is the score d ln p(mu)/d rho of the
    soft angular law p(mu) = A(1+A)/(mu+A)^2, A matched to the mean
    <mu> = (1 - exp(-rho len t1s))/2.  A score must average to 0 and turn
    any moment into its derivative: E[mu s] = d<mu>/d rho = len t1s (1/2 -
    <mu>), and E[mu^2 s] = d E[mu^2]/d rho with the closed form
    E[mu^2] = A(1+A)(1 - 2A ln(1 + 1/A)) + A^2, differentiated numerically
    through A(<mu>(rho))."""
    tb = O.Tables(W.WATER, W.transport())
    length, t1s = 0.07, 3.0

    def m2(mbar):
        a = O.soft_a(mbar)
        return a * (1 + a) * (1 - 2 * a * math.log1p(1 / a)) + a * a

    for mbar in (1e-3, 0.02, 0.1, 0.3):
        rho = -math.log(1 - 2 * mbar) / (length * t1s)
        a = O.soft_a(mbar)
        mu = tb.sample("soft", mbar, 300000, seed=3)[0]
        sc = np.array([O.soft_score(a, m, mbar, length, t1s) for m in mu])
        n = sc.size
        assert abs(sc.mean()) < 5 * sc.std() / math.sqrt(n)
        d1 = length * t1s * (0.5 - mbar)
        e1 = mu * sc
        assert abs(e1.mean() - d1) < 5 * e1.std() / math.sqrt(n), (mbar, e1.mean(), d1)
        h = 1e-5 * rho
        mb = lambda r: 0.5 * (1 - math.exp(-r * length * t1s))
        d2 = (m2(mb(rho + h)) - m2(mb(rho - h))) / (2 * h)
        e2 = mu * mu * sc
        assert abs(e2.mean() - d2) < 5 * e2.std() / math.sqrt(n), (mbar, e2.mean(), d2)


def _csda_layers(n):
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 2.0, size=8)
    ph = W.slab_phantom(8, 0.2, rho)
    ph["step_cap"] = np.full(ph["shape"], 0.013)  # a fixed geometric step cap (cm)
    t = dict(W.transport(), flags=O.NO_HARD_ELASTIC | O.NO_HARD_INELASTIC | O.NO_HARD_BREMS)
    mat = dict(W.WATER, zz1_mol=W.WATER["zz1_mol"] * 1e-9)  # no angular deflection to speak of
    tb = O.Tables(mat, t)
    src = [W.pencil(1, 3.0, (50.0, 50.0, 0.0), n)]
    c = rng.uniform(-1.0, 1.0, size=8).reshape(8, 1, 1)
    return ph, tb, src, c


def test_pathwise_soft_loss_and_energy_adjoint_vs_finite_differences():
    """Term D with its energy adjoint, checked where it is the whole
    gradient: 3 MeV electrons through eight layers (densities 0.5-2) with
    every hard channel off and no deflection, the step cap's geometric length
    held fixed (step_cap; with the algorithm's cap tau_max(E)/rho, a change
    of energy upstream moves every later step boundary and the difference
    quotient follows the saw-tooth of the steps that straddle a face).  Every history is then a straight CSDA track
    whose deposits, at fixed random numbers, are smooth functions of the
    densities, so common-random-number central differences of the oracle's
    own dose (h = 1e-4) are the pathwise derivative of the same sample: the
    estimator's pathwise part (each layer's loss l S(E') at fixed l, minus
    what the electron lacks downstream through the chain dE'/dE =
    S(E')/S(E)) plus the mass term must equal them layer by layer.  (The
    likelihood-ratio part is a mean-zero term of another representation of
    the same derivative, not part of this sample's pathwise one.)"""
    n = 50
    ph, tb, src, c = _csda_layers(n)
    r = O.run(tb, ph, src, 1, 0, n)
    d, _ = O.dose(ph, r)
    g, parts = O.gradient(tb, ph, src, 1, 0, n, c, d)
    g = g.ravel() - (parts["a"] - parts["qbar"] * parts["b"]) / n  # pathwise + mass terms
    h = 1e-4
    fd = np.zeros(8)
    for j in range(8):
        vals = []
        for sg in (1, -1):
            p2 = dict(ph, rho=ph["rho"].copy())
            p2["rho"][j] *= 1 + sg * h
            rr = O.run(tb, p2, src, 1, 0, n)
            dd, _ = O.dose(p2, rr)
            vals.append(float((c * dd).sum()))
        fd[j] = (vals[0] - vals[1]) / (2 * h * ph["rho"][j, 0, 0])
    err = np.abs(g - fd) / np.abs(fd).max()
    print("estimator", np.round(g, 3), "fd", np.round(fd, 3), "max rel", err.max())
    assert err.max() < 1e-4
    # the pathwise term is what moves: without its downstream part the
    # estimate would be far off
    assert np.abs(parts["p"]).max() > 0.1 * np.abs(fd).max() * n


def test_class2_gradient_vs_crn_finite_differences():
    """The whole Class II estimator against common-random-number central
    differences (+-5%) of a linear dose loss: 3 MeV electrons through eight
    2 mm layers of densities 0.5-2 with the hard channels off, so that the
    track is CSDA slowing with soft deflections at the hinges and the
    algorithm's own step cap.  The deflection law depends on the particle's
    energy, which moves with every upstream density: with term E
    (GRAD_DEFLECTION_ENERGY) the estimator agrees with the differences
    (|z| < 4 in every layer carrying 5% of the largest derivative); without
    it the same sample shows the omitted part (some layer at |z| > 4).
    Eight batches of 1000 histories; the differences are shared."""
    n, nb, h = 1000, 8, 0.05
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 2.0, size=8)
    c = rng.uniform(-1.0, 1.0, size=8).reshape(8, 1, 1)
    hard_off = O.NO_HARD_ELASTIC | O.NO_HARD_INELASTIC | O.NO_HARD_BREMS
    tb = O.Tables(W.WATER, W.transport(flags=hard_off))
    tbe = O.Tables(W.WATER, W.transport(flags=hard_off | O.GRAD_DEFLECTION_ENERGY))
    src = [W.pencil(1, 3.0, (50.0, 50.0, 0.0), n * nb)]
    cc = np.broadcast_to(c, (8, 1, 1)).copy()
    est = {0: np.zeros((nb, 8)), 1: np.zeros((nb, 8))}
    fd = np.zeros((nb, 8))
    for b in range(nb):
        ph = W.slab_phantom(8, 0.2, rho)
        d, _ = O.dose(ph, O.run(tb, ph, src, 1, b * n, n))
        est[0][b] = O.gradient(tb, ph, src, 1, b * n, n, cc, d)[0].ravel()
        est[1][b] = O.gradient(tbe, ph, src, 1, b * n, n, cc, d)[0].ravel()
        for j in range(8):
            v = []
            for sg in (1, -1):
                r2 = rho.copy()
                r2[j] *= 1 + sg * h
                p2 = W.slab_phantom(8, 0.2, r2)
                dd, _ = O.dose(p2, O.run(tb, p2, src, 1, b * n, n))
                v.append(float((c * dd).sum()))
            fd[b, j] = (v[0] - v[1]) / (2 * h * rho[j])
    f, fse = fd.mean(0), fd.std(0, ddof=1) / math.sqrt(nb)
    keep = np.abs(f) > 0.05 * np.abs(f).max()
    z = {}
    for k, e in est.items():
        m, se = e.mean(0), e.std(0, ddof=1) / math.sqrt(nb)
        z[k] = ((m - f) / np.hypot(se, fse))[keep]
    print("z without term E", np.round(z[0], 2), "with", np.round(z[1], 2))
    assert np.all(np.abs(z[1]) < 4.0), z[1]
    assert np.abs(z[0]).max() > 4.0, z[0]
