"""GPU parity of interaction forcing and bremsstrahlung splitting (weighted
particles, the forced inelastic-collision and bremsstrahlung channels, two
photons per emission) against the FP64 oracle
with the same forcing factors, through the C ABI: event sequences, weighted
per-history ledgers, doses within 3 combined standard errors; the mixed
precision path against FP64; refusals."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tally_checks import check_tally_parity, check_gradient_parity

pytestmark = pytest.mark.gpu
MC2 = W.MC2


def _mcx():
    import paper_2003_00796_amd as mcx
    return mcx


def gpu_run(wl, n, precision=0, test=True):
    mcx = _mcx()
    sim = mcx.Simulator(precision, 0).setup(wl)
    sim.set_test_mode(test)
    sim.run(wl["seed"], 0, n)
    h, led = sim.history_results(n) if test else (None, None)
    d, s = sim.dose()
    q, q2 = sim.tally()
    st = sim.stats()
    sim.close()
    return dict(hash=h, led=led, dose=d, sigma=s, q=q, q2=q2, stats=st)


def oracle_run(wl, n):
    if wl.get("phantom", {}).get("mat") is not None:
        tbs = [O.Tables(m, wl["transport"]) for m in wl["materials"]]
    else:
        tbs = O.Tables(wl["material"], wl["transport"])
    r = O.run(tbs, wl["phantom"], wl["sources"], wl["seed"], 0, n, hashes=True, ledger=True)
    d, s = O.dose(wl["phantom"], r)
    return dict(hash=r.hashes, led=r.ledger, dose=d, sigma=s, q=r.sum_q, q2=r.sum_q2, stats=r.stats.as_dict())


def check_dose_3sigma(g, o, frac=0.01):
    hi = o["dose"] > frac * o["dose"].max()
    diff = np.abs(g["dose"] - o["dose"])[hi]
    comb = np.sqrt(g["sigma"][hi] ** 2 + o["sigma"][hi] ** 2)
    assert np.all(diff <= 3 * comb + 1e-12 * o["dose"].max()), float(np.max(diff / (comb + 1e-300)))


def layers(particle, energy, n, flags=0, force_in=4.0, force_br=20.0, split_br=0):
    rho = np.array([1.0, 1.85, 0.3, 1.85, 1.0, 0.26, 1.85, 1.0] * 2)
    ph = W.slab_phantom(len(rho), 1.0, rho)
    t = dict(W.transport(100.0, 250, flags=flags), force_in=force_in, force_br=force_br, split_br=split_br)
    return dict(W.workload("electron_200"), phantom=ph, transport=t, material=W.WATER,
                sources=[W.pencil(particle, energy, (50.0, 50.0, 0.0), n)])


CASES = {
    "electrons_10MeV": lambda: layers(1, 10.0, 400),
    "photons_6MeV": lambda: layers(0, 6.0, 3000),
    "positrons_5MeV_brems_only": lambda: layers(2, 5.0, 800, force_in=0.0, force_br=50.0),
    "electrons_straggling_annihilation": lambda: layers(1, 10.0, 300, flags=O.STRAGGLING | O.ANNIH_FLIGHT),
    "electrons_forced_and_split": lambda: layers(1, 10.0, 400, split_br=2),
    "electrons_split_only": lambda: layers(1, 20.0, 300, force_in=0.0, force_br=0.0, split_br=2),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_forcing_parity(case):
    wl = CASES[case]()
    n = wl["sources"][0]["n_hist"]
    g, o = gpu_run(wl, n), oracle_run(wl, n)
    same = g["hash"] == o["hash"]
    print(case, "identical hashes", same.mean(), "hard br", g["stats"]["hard_br"], o["stats"]["hard_br"])
    assert same.mean() >= 0.99
    # weighted deposits, escapes and positron escapes of the same histories
    assert np.allclose(g["led"][same], o["led"][same][:, [0, 1, 2]], rtol=0, atol=1e-8)
    assert abs(g["stats"]["hard_br"] - o["stats"]["hard_br"]) <= 0.01 * o["stats"]["hard_br"] + 5
    check_dose_3sigma(g, o)
    check_tally_parity(g, o, same=same.mean())


def test_forcing_mixed_precision_and_unbiased_balance():
    wl = layers(1, 10.0, 20_000)
    g64 = gpu_run(wl, 20_000, 0)
    g32 = gpu_run(wl, 20_000, 1)
    check_dose_3sigma(g32, g64)
    for g in (g64, g32):
        bal = g["led"][:, 0] + g["led"][:, 1] + 2 * MC2 * g["led"][:, 2]
        assert abs(bal.mean() - 10.0) <= 5 * bal.std(ddof=1) / np.sqrt(bal.size)


def test_forced_bremsstrahlung_rate():
    """Bremsstrahlung forced by F = 20 with analog collisions and photons
    that escape without interacting: the electrons (primaries and knock-ons)
    follow the analog law, so the emissions are F times the analog count in
    expectation."""
    flags = O.NO_COMPTON | O.NO_PHOTO | O.NO_RAYLEIGH | O.NO_PAIR
    wl = layers(1, 10.0, 20_000, flags=flags, force_in=0.0, force_br=20.0)
    f = gpu_run(wl, 20_000, 1, test=False)
    a = gpu_run(dict(wl, transport=dict(wl["transport"], force_br=0.0)), 20_000, 1, test=False)
    ratio = f["stats"]["hard_br"] / a["stats"]["hard_br"]
    print("analog emissions", a["stats"]["hard_br"], "ratio", ratio)
    assert 18.5 < ratio < 21.5, ratio


def test_forcing_reduces_the_variance_behind_a_target():
    """2 MeV electrons stopped in a water target; only bremsstrahlung photons
    reach the detector layers behind the air gap.  Forcing the emissions by
    50 leaves the detector dose unchanged and cuts its variance per history
    by more than 9."""
    n = 1_000_000
    wl = W.workload("target_detector", n)
    a = gpu_run(wl, n, 1, test=False)
    f = gpu_run(dict(wl, transport=dict(wl["transport"], force_br=50.0)), n, 1, test=False)
    det = slice(23, 27)
    da, sa = a["dose"][det].ravel(), a["sigma"][det].ravel()
    df, sf = f["dose"][det].ravel(), f["sigma"][det].ravel()
    print("detector dose", da, df, "sigma", sa, sf)
    assert np.all(da > 0) and np.all(np.abs(da - df) <= 4 * np.hypot(sa, sf))
    assert np.all(sf < sa / 3)
    assert a["dose"][:3].sum() == pytest.approx(f["dose"][:3].sum(), rel=0.01)


def test_forced_gradient_matches_oracle():
    """The density-gradient replays with forcing and splitting (weighted
    deposits and soft-loss terms) against the oracle's gradient on the same
    histories."""
    mcx = _mcx()
    for wl in (layers(1, 10.0, 300, split_br=2), layers(0, 6.0, 3000, split_br=2)):
        n = wl["sources"][0]["n_hist"]
        c = np.random.default_rng(4).uniform(-1.0, 1.0, size=wl["phantom"]["rho"].shape)
        sim = mcx.Simulator(0, 0).setup(wl)
        sim.run(wl["seed"], 0, n)
        g = sim.dose_backward(c)
        sim.close()
        tb = O.Tables(wl["material"], wl["transport"])
        r = O.run(tb, wl["phantom"], wl["sources"], wl["seed"], 0, n)
        do, _ = O.dose(wl["phantom"], r)
        go, _ = O.gradient(tb, wl["phantom"], wl["sources"], wl["seed"], 0, n, c, do)
        rel = np.abs(g - go) / np.abs(go).max()
        print("forced gradient: max deviation", rel.max())
        check_gradient_parity(g, go, class2=True)


def test_forcing_refusals():
    mcx = _mcx()
    wl = layers(1, 10.0, 100)
    sim = mcx.Simulator(0, 0)
    with pytest.raises(mcx.MCXError, match="INVALID"):
        sim.set_transport(dict(wl["transport"], force_br=0.5))
    with pytest.raises(mcx.MCXError, match="INVALID"):
        sim.set_transport(dict(wl["transport"], force_in=1e6))
    with pytest.raises(mcx.MCXError, match="INVALID"):
        sim.set_transport(dict(wl["transport"], split_br=3))
    sim.close()


def _three_material_layers(particle, e0, n, **force):
    """Water, bone and lung layers (1 cm) of the several-material workload's
    materials, with forcing."""
    rho = np.array([1.0, 1.85, 0.26, 1.0, 1.85, 0.3, 1.0, 0.26] * 2)
    mat = np.array([0, 1, 2, 0, 1, 2, 0, 2] * 2, dtype=np.uint8)
    ph = W.slab_phantom(len(rho), 1.0, rho)
    ph["mat"] = np.broadcast_to(mat[:, None, None], ph["rho"].shape).copy()
    base = W.workload("hetero_mm_64")
    t = dict(W.transport(100.0, 250), **force)
    return dict(base, phantom=ph, transport=t, sources=[W.pencil(particle, e0, (50.0, 50.0, 0.0), n)])


@pytest.mark.parametrize("case", ["electrons_forced_split", "photons_forced"])
def test_forcing_on_several_materials_parity(case):
    """Forcing and splitting on a phantom of water, bone and lung: the
    several-material weighted kernels reproduce the oracle's event sequences
    and weighted ledgers, and the doses agree within 3 combined standard
    errors."""
    if case == "electrons_forced_split":
        wl = _three_material_layers(1, 10.0, 800, force_in=4.0, force_br=20.0, split_br=2)
    else:
        wl = _three_material_layers(0, 6.0, 3000, force_in=4.0, force_br=20.0)
    n = wl["sources"][0]["n_hist"]
    g, o = gpu_run(wl, n), oracle_run(wl, n)
    same = g["hash"] == o["hash"]
    print(case, "identical hashes", same.mean())
    assert same.mean() >= 0.99
    assert np.allclose(g["led"][same], o["led"][same][:, [0, 1, 2]], rtol=0, atol=1e-8)
    check_dose_3sigma(g, o)


def test_forced_gradient_on_several_materials_matches_oracle():
    """The replays with weights on a three-material phantom against the
    oracle's several-material gradient on the same histories."""
    mcx = _mcx()
    wl = _three_material_layers(1, 10.0, 400, force_in=4.0, force_br=20.0, split_br=2)
    n = wl["sources"][0]["n_hist"]
    c = np.random.default_rng(8).uniform(-1.0, 1.0, size=wl["phantom"]["rho"].shape)
    sim = mcx.Simulator(0, 0).setup(wl)
    sim.run(wl["seed"], 0, n)
    g = sim.dose_backward(c)
    sim.close()
    tbs = [O.Tables(m, wl["transport"]) for m in wl["materials"]]
    r = O.run(tbs, wl["phantom"], wl["sources"], wl["seed"], 0, n)
    do, _ = O.dose(wl["phantom"], r)
    go, _ = O.gradient(tbs, wl["phantom"], wl["sources"], wl["seed"], 0, n, c, do)
    rel = np.abs(g - go) / np.abs(go).max()
    print("forced several-material gradient: max deviation", rel.max())
    check_gradient_parity(g, go, class2=True)


def test_full_size_sampled_histories_forced_and_split():
    """The forced workload the benchmark times (1e7 histories of the 6 MeV
    field on the 128^3 heterogeneous phantom, hard collisions forced by 4,
    bremsstrahlung by 20 and split by 2; 2^26 records per queue, blocks of
    256, 128 steps per visit), FP64: a sample of histories over the whole
    range re-run one by one by the oracle with the same forcing."""
    mcx = _mcx()
    wl = W.workload("hetero_broad_128")
    wl["transport"] = dict(wl["transport"], force_in=4.0, force_br=20.0, split_br=2)
    n = wl["sources"][0]["n_hist"]
    sim = mcx.Simulator(0, 0).setup(wl)
    sim.set_launch(1 << 26, 256, 128)
    sim.set_test_mode(True)
    sim.run(wl["seed"], 0, n)
    h, led = sim.history_results(n)
    st = sim.stats()
    sim.close()
    assert st["histories"] == n
    tb = O.Tables(wl["material"], wl["transport"])
    sample = np.sort(np.random.default_rng(13).choice(n, size=200, replace=False))
    same = 0
    for k in sample:
        r = O.run(tb, wl["phantom"], wl["sources"], wl["seed"], int(k), 1, hashes=True, ledger=True)
        if r.hashes[0] == h[k]:
            same += 1
            assert np.allclose(led[k], r.ledger[0][[0, 1, 2]], rtol=0, atol=1e-8), int(k)
    print("sampled identical hashes", same, "of", len(sample))
    assert same >= 0.99 * len(sample)
    bal = led[:, 0] + led[:, 1] + 2 * MC2 * led[:, 2]
    assert abs(bal.mean() - 6.0) <= 5 * bal.std(ddof=1) / np.sqrt(n)


def test_forced_runs_split_merge_and_influence():
    """Weighted runs keep the run-control invariants: two partial runs give
    the tallies of one run (FP64 summation order aside), and the
    per-beamlet influence entries add up to the weighted tallies."""
    mcx = _mcx()
    wl = layers(0, 6.0, 6000, split_br=2)
    wl["sources"] = [W.pencil(0, 6.0, (50.0, 50.0, 0.0), 2500), W.pencil(0, 2.0, (50.0, 50.0, 0.0), 3500)]
    one = mcx.Simulator(0, 0).setup(wl)
    one.run(wl["seed"], 0, 6000)
    q1, s1 = one.tally()
    one.close()
    two = mcx.Simulator(0, 0).setup(wl)
    two.set_influence(True, 16)
    two.run(wl["seed"], 0, 2000)
    two.run(wl["seed"], 2000, 4000)
    q2, s2 = two.tally()
    src, vox, iq, iq2 = two.influence()
    two.close()
    assert np.allclose(q1, q2, rtol=1e-11, atol=1e-14) and np.allclose(s1, s2, rtol=1e-11, atol=1e-14)
    tot = np.zeros(q2.size)
    np.add.at(tot, vox.astype(np.int64), iq)
    assert set(np.unique(src)) == {0, 1}
    assert np.allclose(tot, q2, rtol=1e-11, atol=1e-14)
