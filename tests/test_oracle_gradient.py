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
