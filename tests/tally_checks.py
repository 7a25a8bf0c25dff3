"""Shared check of the variance estimator (Sec. 4.3, Eq. (1)-(3) with the
square root of Eq. (2) restored): the GPU's Sum q, Sum q^2 and sigma against
the oracle's on the same seeded histories.

Where (nearly) every history follows the oracle's event sequence, both sides
add the same per-history scores q_hv, so Sum q and Sum q^2 differ only by the
rounding of energies along a track and the order of FP64 additions: the
median relative difference over voxels above `frac` of the maximum is at
rounding level.  (A median, not a maximum: a history whose event sequence
differs changes the voxels it crosses by a statistical amount.)  sigma, a
difference of the two moments, is checked the same way where it is
resolved (above `frac` of its own maximum)."""
import numpy as np


def check_tally_parity(g, o, frac=0.01, tol=1e-9, same=None):
    g = {k: np.ravel(g[k]) for k in ("q", "q2", "sigma")}
    o = {k: np.ravel(o[k]) for k in ("q", "q2", "sigma")}
    hi = o["q"] > frac * o["q"].max()
    assert hi.any()
    out = {}
    for k in ("q", "q2", "sigma"):
        sel = hi if k != "sigma" else hi & (o["sigma"] > frac * o["sigma"].max())
        rel = np.abs(g[k] - o[k])[sel] / np.abs(o[k][sel])
        out[k] = (float(np.median(rel)), float(np.quantile(rel, 0.99)))
    print("tally parity (median, 99th percentile of the relative difference):", out)
    for k, (med, q99) in out.items():
        assert med < tol, (k, med)
        if same is not None and same == 1.0:
            # every history identical: all voxels agree to rounding
            assert q99 < 1e3 * tol, (k, q99)
    return out


def check_gradient_parity(g, go, class2: bool):
    """Replay gradient against the oracle's on histories with identical event
    sequences, relative to the largest component.  Kerma mode (photon scores
    only): every voxel within 1e-9 (summation order and rounding).  Class II:
    the gradient is a large cancelling sum over histories of (Q_h - Qbar)
    times the scores, and the e+- scores carry the majorant and the step
    geometry, so last-bit differences between the two implementations (a
    4e-16 relative change of the oracle's own majorant moves its gradient by
    9e-11) are amplified along a few tracks: 99.9% of the voxels within 1e-9
    (measured: 1e-11 to 3e-11) and every voxel within 1e-6 (measured: up to
    1.1e-7 on one track of 2000 histories of the three-material field).  A
    formula difference moves many voxels and fails the first bound."""
    import numpy as np
    err = np.abs(np.asarray(g) - np.asarray(go)).ravel() / np.abs(go).max()
    if not class2:
        assert err.max() <= 1e-9, err.max()
        return err.max()
    assert np.quantile(err, 0.999) <= 1e-8, np.quantile(err, 0.999)
    assert err.max() <= 1e-6, err.max()
    return err.max()
