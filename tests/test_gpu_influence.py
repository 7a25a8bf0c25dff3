"""GPU tests of the per-source (beamlet) dose-influence output, through the
C ABI.  Each (history, voxel) score lands in exactly one (source, voxel)
entry, so the entries of all sources add up to the voxel tallies Sum q and
Sum q^2 (Eq. (1)-(3)) up to FP64 summation order; and each source's entries
equal the oracle's tallies of that source's histories run alone."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _mcx():
    import paper_2003_00796_amd as mcx
    return mcx


def beamlets_wl():
    """Four 5 x 5 mm beamlets of 2, 4, 6 and 10 MeV photons, uneven counts,
    on the 64^3 heterogeneous phantom."""
    wl = W.workload("hetero_broad_64", 1000)
    srcs = [W.rect_field(0, e, (9.0 + 2.5 * i, 12.8, 0.0), (0.5, 0.5), n)
            for i, (e, n) in enumerate(((2.0, 300), (4.0, 500), (6.0, 700), (10.0, 400)))]
    return dict(wl, sources=srcs)


def per_voxel(src, vox, val, nsrc, nvox):
    m = np.zeros((nsrc, nvox))
    np.add.at(m, (src.astype(np.int64), vox.astype(np.int64)), val)
    return m


@pytest.mark.parametrize("precision", [0, 1])
def test_influence_adds_up_to_the_tallies_and_matches_the_oracle(precision):
    mcx = _mcx()
    wl = beamlets_wl()
    counts = [s["n_hist"] for s in wl["sources"]]
    n = sum(counts)
    sim = mcx.Simulator(precision, 0).setup(wl)
    sim.set_influence(True, 20)
    sim.run(wl["seed"], 0, n)
    src, vox, q, q2 = sim.influence()
    tq, tq2 = sim.tally()
    sim.close()
    nv = tq.size
    assert src.max() == 3 and len(np.unique(src)) == 4
    assert len(np.unique(src.astype(np.int64) << 32 | vox)) == src.size  # one entry per pair
    mq = per_voxel(src, vox, q, 4, nv)
    mq2 = per_voxel(src, vox, q2, 4, nv)
    assert np.allclose(mq.sum(0), tq, rtol=1e-11, atol=1e-14)
    assert np.allclose(mq2.sum(0), tq2, rtol=1e-11, atol=1e-14)
    if precision == 1:
        return
    tb = O.Tables(wl["material"], wl["transport"])
    first = 0
    for b, nb in enumerate(counts):
        r = O.run(tb, wl["phantom"], wl["sources"], wl["seed"], first, nb)
        first += nb
        hi = r.sum_q > 1e-2 * r.sum_q.max()
        rel = np.abs(mq[b] - r.sum_q)[hi] / r.sum_q[hi]
        assert np.median(rel) < 1e-9, b
        assert mq[b].sum() == pytest.approx(r.sum_q.sum(), rel=2e-3)
        # no energy of beamlet b outside the voxels its own histories reached
        # in the oracle, except from the rare histories whose events differ
        assert mq[b][r.sum_q == 0].sum() < 2e-3 * mq[b].sum()


def test_influence_accumulates_resets_and_reports_overflow():
    mcx = _mcx()
    wl = beamlets_wl()
    n = sum(s["n_hist"] for s in wl["sources"])
    sim = mcx.Simulator(0, 0).setup(wl)
    with pytest.raises(mcx.MCXError, match="STATE"):
        sim.influence()
    sim.set_influence(True, 20)
    sim.run(wl["seed"], 0, 800)      # the first two beamlets
    sim.run(wl["seed"], 800, n - 800)  # the rest, accumulating
    src, vox, q, q2 = sim.influence()
    tq, _ = sim.tally()
    assert np.isclose(q.sum(), tq.sum(), rtol=1e-11)
    assert set(np.unique(src)) == {0, 1, 2, 3}
    sim.reset()
    assert sim.influence()[0].size == 0
    sim.set_influence(True, 10)  # 1024 slots: too few for these beamlets
    with pytest.raises(mcx.MCXError, match="RANGE"):
        sim.run(wl["seed"], 0, n)
    sim.set_influence(False)
    sim.close()


def test_influence_of_512_beamlets():
    """The 512-beamlet workload on the 256^3 noise phantom (2e6 histories,
    mixed precision, one run): every beamlet has entries, and they add up to
    the voxel tallies; the count-only call and the unsorted read (the
    device compaction's own order) give the same entries."""
    mcx = _mcx()
    wl = W.workload("beamlets_256", 2_000_000)
    n = sum(s["n_hist"] for s in wl["sources"])
    sim = mcx.Simulator(mcx.MIXED, 0).setup(wl)
    sim.set_influence(True, 27)
    sim.run(wl["seed"], 0, n)
    src, vox, q, q2 = sim.influence()
    count = sim.influence_count()
    raw = sim.influence(sort=False)
    tq, tq2 = sim.tally()
    sim.close()
    assert count == src.size
    order = np.lexsort((raw[1], raw[0]))
    for a, b in zip(raw, (src, vox, q, q2)):
        assert np.array_equal(a[order], b)
    print("influence entries", src.size, "per beamlet", src.size / 512)
    assert len(np.unique(src)) == 512
    tot = np.zeros(tq.size)
    np.add.at(tot, vox.astype(np.int64), q)
    assert np.allclose(tot, tq, rtol=1e-10, atol=1e-14)
