"""Pins of the oracle's several-material voxels (reading R10 of the oracle;
the "next" extension of the one-material main path).

- narrow-beam attenuation through layers of three materials (water, bone,
  lung; photoelectric only, electrons absorbed on the spot): the per-layer
  absorptions follow the exponential law with each layer's own rho mu_m
  (multinomial test);
- a phantom made of bone (or of lung) through the several-material path
  gives the one-material run of that material: identical histories for
  electrons (the step uses the voxel's tables), the same histories up to
  rounding for photons (the flight counts optical depth instead of mass
  thickness);
- per-history energy conservation on the heterogeneous phantom with bone
  spheres; material indices beyond the tables are refused.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
import workloads as W

MC2 = 0.51099895000


def test_three_material_layers_follow_the_exponential_law():
    e0 = 0.03
    rho = np.array([1.0, 1.85, 0.3, 1.85, 1.0, 0.26, 1.85, 1.0] * 2)
    mat = np.array([0, 1, 2, 1, 0, 2, 1, 0] * 2, dtype=np.uint8)
    dz = 0.2
    ph = W.slab_phantom(len(rho), dz, rho)
    ph["mat"] = np.broadcast_to(mat[:, None, None], ph["rho"].shape).copy()
    t = W.transport(flags=O.NO_COMPTON | O.NO_RAYLEIGH | O.NO_PAIR, eabs=(0.01, 1e9, 1e9))
    tbs = [O.Tables(W.WATER, t), O.Tables(W.BONE, t), O.Tables(W.LUNG, t)]
    n = 40_000
    r = O.run(tbs, ph, [W.pencil(0, e0, (50.0, 50.0, 0.0), n)], 3, 0, n, ledger=True)
    mu = np.array([tb.eval(O.MU_PHOTO, e0) for tb in tbs])
    assert mu[1] / mu[0] == pytest.approx(28.5 / 4.94, rel=1e-12)
    assert mu[2] / mu[0] == pytest.approx(5.31 / 4.94, rel=1e-12)
    q = r.sum_q.reshape(len(rho)) / e0
    cnt = np.round(q).astype(int)
    assert np.allclose(q, cnt, atol=1e-9)
    tau = np.concatenate([[0.0], np.cumsum(mu[mat] * rho * dz)])
    p = np.exp(-tau[:-1]) - np.exp(-tau[1:])
    n_esc = int(round(r.ledger[:, O.LED_ESC].sum() / e0))
    obs = np.append(cnt, n_esc)
    exp = np.append(p, math.exp(-tau[-1])) * n
    assert obs.sum() == n
    chi = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi, len(obs) - 1) > 1e-4


@pytest.mark.parametrize("which", ["bone", "lung"])
def test_all_bone_phantom_equals_the_one_material_bone_run(which):
    m, k = (W.BONE, 1) if which == "bone" else (W.LUNG, 2)
    ph = W.water_cube(16, 8.0)
    ph_mm = dict(ph, mat=np.full(ph["rho"].shape, k, dtype=np.uint8))
    mats = lambda t: [O.Tables(W.WATER, t), O.Tables(W.BONE, t), O.Tables(W.LUNG, t)]
    # electrons without bremsstrahlung photons: the same steps, bit for bit
    t = W.transport(100.0, 250, flags=O.NO_HARD_BREMS)
    src = [W.pencil(1, 5.0, (4.0, 4.0, 0.0), 300)]
    one = O.run(O.Tables(m, t), ph, src, 4, 0, 300, hashes=True, ledger=True)
    two = O.run(mats(t), ph_mm, src, 4, 0, 300, hashes=True, ledger=True)
    assert np.array_equal(one.hashes, two.hashes)
    assert np.array_equal(one.ledger, two.ledger)
    assert np.array_equal(one.sum_q, two.sum_q)
    # photons: optical depth instead of mass thickness, equal up to rounding
    t = W.transport()
    src = [W.pencil(0, 1.0, (4.0, 4.0, 0.0), 3000)]
    one = O.run(O.Tables(m, t), ph, src, 5, 0, 3000, hashes=True, ledger=True)
    two = O.run(mats(t), ph_mm, src, 5, 0, 3000, hashes=True, ledger=True)
    same = one.hashes == two.hashes
    assert same.mean() >= 0.999
    assert np.allclose(one.ledger[same], two.ledger[same], rtol=0, atol=1e-9)


def test_bone_spheres_conservation_and_index_check():
    wl = W.workload("hetero_mm_64", 1500)
    tbs = [O.Tables(m, wl["transport"]) for m in wl["materials"]]
    r = O.run(tbs, wl["phantom"], wl["sources"], 1, 0, 1500, ledger=True)
    bal = r.ledger[:, O.LED_DEP] + r.ledger[:, O.LED_ESC] + 2 * MC2 * r.ledger[:, O.LED_POSESC]
    assert np.max(np.abs(bal - 6.0)) <= 1e-12 * 6.0
    assert len(tbs) == 3
    bad = dict(wl["phantom"], mat=np.full(wl["phantom"]["rho"].shape, 3, dtype=np.uint8))
    with pytest.raises(RuntimeError):
        O.run(tbs, bad, wl["sources"], 1, 0, 10)
