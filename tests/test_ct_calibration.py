"""CT calibration of the C ABI (mcx_ct_to_phantom, host code: runs without a
GPU): Hounsfield units to density by a piecewise-linear curve, to material
index by thresholds, against numpy's own interpolation and search."""
import os

import numpy as np
import pytest

import paper_2003_00796_amd as mcx

pytestmark = pytest.mark.skipif(not os.path.exists(mcx.LIB_PATH), reason="library not built")

# a typical stoichiometric-style curve: air, lung, water, soft tissue, bone
HU = [-1000.0, -700.0, 0.0, 100.0, 1500.0]
RHO = [0.0012, 0.3, 1.0, 1.07, 1.9]
THRESH = [300.0]  # water-like below 300 HU, bone at and above


def test_density_and_material_against_numpy():
    rng = np.random.default_rng(3)
    hu = rng.integers(-1100, 2000, size=(9, 11, 13)).astype(np.int16)
    hu.flat[:6] = [-1100, -1000, 0, 100, 1500, 2000]
    rho, mat = mcx.ct_to_phantom(hu, HU, RHO, THRESH)
    ref = np.interp(hu.astype(np.float64), HU, RHO)
    assert np.allclose(rho, ref, rtol=1e-14, atol=0)
    assert rho.flat[0] == RHO[0] and rho.flat[5] == RHO[-1]  # clamped beyond the end points
    assert np.array_equal(mat, np.searchsorted(THRESH, hu, side="right").astype(np.uint8))
    assert np.all(rho > 0)


def test_three_thresholds_and_exact_nodes():
    hu = np.array([-1000, -700, -701, 0, 100, 299, 300, 1499, 1500], dtype=np.int16)
    rho, mat = mcx.ct_to_phantom(hu, HU, RHO, [-500.0, 300.0, 1200.0])
    assert rho[0] == 0.0012 and rho[1] == 0.3 and rho[3] == 1.0 and rho[4] == 1.07 and rho[8] == 1.9
    assert list(mat) == [0, 0, 0, 1, 1, 1, 2, 3, 3]


@pytest.mark.parametrize("bad", ["decreasing", "nonpositive", "thresholds"])
def test_malformed_calibrations_are_refused(bad):
    hu = np.zeros(4, dtype=np.int16)
    if bad == "decreasing":
        args = ([0.0, -10.0], [1.0, 1.0], [])
    elif bad == "nonpositive":
        args = ([0.0, 10.0], [1.0, 0.0], [])
    else:
        args = (HU, RHO, [1.0, 2.0, 3.0, 4.0])
    with pytest.raises(mcx.MCXError):
        mcx.ct_to_phantom(hu, *args)
