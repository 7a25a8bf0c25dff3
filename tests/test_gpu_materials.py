"""GPU parity of several-material phantoms (per-voxel material index, the
several-material kernel flavours) against the FP64 oracle with the same
materials, through the C ABI: event sequences, per-history conservation,
doses within 3 combined standard errors; an all-bone phantom through the
several-material kernels against the one-material bone run; refusals."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tally_checks import check_tally_parity

pytestmark = pytest.mark.gpu
MC2 = W.MC2


def _mcx():
    import paper_2003_00796_amd as mcx
    return mcx


def gpu_run(wl, n, precision=0):
    mcx = _mcx()
    sim = mcx.Simulator(precision, 0).setup(wl)
    sim.set_test_mode(True)
    sim.run(wl["seed"], 0, n)
    h, led = sim.history_results(n)
    d, s = sim.dose()
    q, q2 = sim.tally()
    st = sim.stats()
    sim.close()
    return dict(hash=h, led=led, dose=d, sigma=s, q=q, q2=q2, stats=st)


def oracle_run(wl, n):
    tbs = [O.Tables(m, wl["transport"]) for m in wl.get("materials") or [wl["material"]]]
    r = O.run(tbs if "materials" in wl else tbs[0], wl["phantom"], wl["sources"], wl["seed"], 0, n, hashes=True,
              ledger=True)
    d, s = O.dose(wl["phantom"], r)
    return dict(hash=r.hashes, led=r.ledger, dose=d, sigma=s, q=r.sum_q, q2=r.sum_q2, stats=r.stats.as_dict())


def check_balance(led, etot, tol):
    bal = led[:, 0] + led[:, 1] + 2 * MC2 * led[:, 2]
    assert np.max(np.abs(bal - etot)) <= tol * etot, np.max(np.abs(bal - etot))


def check_dose_3sigma(g, o, frac=0.01):
    hi = o["dose"] > frac * o["dose"].max()
    diff = np.abs(g["dose"] - o["dose"])[hi]
    comb = np.sqrt(g["sigma"][hi] ** 2 + o["sigma"][hi] ** 2)
    assert np.all(diff <= 3 * comb + 1e-12 * o["dose"].max()), float(np.max(diff / (comb + 1e-300)))


def layered():
    rho = np.array([1.0, 1.85, 0.3, 1.85, 1.0, 0.26, 1.85, 1.0] * 2)
    mat = np.array([0, 1, 2, 1, 0, 2, 1, 0] * 2, dtype=np.uint8)  # water, bone, lung
    ph = W.slab_phantom(len(rho), 1.0, rho)
    ph["mat"] = np.broadcast_to(mat[:, None, None], ph["rho"].shape).copy()
    return dict(W.workload("hetero_mm_64"), phantom=ph, sources=[W.pencil(0, 1.0, (50.0, 50.0, 0.0), 4000)])


def ct_case():
    """A CT-like volume through a calibration (density by linear
    interpolation, bone at and above 300 HU, lung below -400 HU), converted
    here with numpy so that the oracle's input does not come from the
    library."""
    hu = W.ct_hu_volume(32)
    rho = np.interp(hu.astype(np.float64), [-1000.0, -700.0, 0.0, 100.0, 1500.0], [0.0012, 0.3, 1.0, 1.07, 1.9])
    mat = np.where(hu >= 300, 1, np.where(hu < -400, 2, 0)).astype(np.uint8)
    ph = dict(shape=hu.shape, voxel=(0.5, 0.5, 0.5), origin=(0.0, 0.0, 0.0), rho=rho, mat=mat)
    return dict(W.workload("hetero_mm_64"), phantom=ph, sources=[W.rect_field(0, 6.0, (8.0, 8.0, 0.0), (6.0, 6.0), 3000)])


CASES = {
    "ct_volume": (ct_case, 6.0),
    "bone_spheres": (lambda: W.workload("hetero_mm_64", 3000), 6.0),
    "layers_1MeV": (layered, 1.0),
    "electron_layers": (lambda: dict(layered(), transport=W.transport(100.0, 250),
                                     sources=[W.pencil(1, 10.0, (50.0, 50.0, 0.0), 400)]), 10.0),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_several_materials_parity(case):
    make, etot = CASES[case]
    wl = make()
    n = wl["sources"][0]["n_hist"]
    g, o = gpu_run(wl, n), oracle_run(wl, n)
    same = g["hash"] == o["hash"]
    print(case, "identical hashes", same.mean())
    assert same.mean() >= 0.99
    check_balance(g["led"], etot, 1e-12)
    assert np.allclose(g["led"][same], o["led"][same][:, [0, 1, 2]], rtol=0, atol=1e-8)
    check_dose_3sigma(g, o)
    check_tally_parity(g, o, same=same.mean())


def test_several_materials_with_straggling_and_annihilation():
    wl = dict(layered(), transport=dict(W.transport(100.0, 250), flags=O.STRAGGLING | O.ANNIH_FLIGHT),
              sources=[W.pencil(2, 5.0, (50.0, 50.0, 0.0), 1500)])
    g, o = gpu_run(wl, 1500), oracle_run(wl, 1500)
    assert np.mean(g["hash"] == o["hash"]) >= 0.99
    check_balance(g["led"], 5.0 + 2 * MC2, 1e-12)
    check_dose_3sigma(g, o)


def test_all_bone_phantom_equals_the_one_material_bone_run():
    ph = W.water_cube(16, 8.0)
    base = dict(W.workload("electron_200"), phantom=ph, transport=W.transport(100.0, 250, flags=O.NO_HARD_BREMS),
                sources=[W.pencil(1, 5.0, (4.0, 4.0, 0.0), 500)], material=W.BONE)
    mm = dict(base, phantom=dict(ph, mat=np.ones(ph["rho"].shape, dtype=np.uint8)), materials=[W.WATER, W.BONE])
    one, two = gpu_run(base, 500), gpu_run(mm, 500)
    assert np.array_equal(one["hash"], two["hash"])
    assert np.allclose(one["q"], two["q"], rtol=1e-11, atol=1e-14)
    base = dict(base, transport=W.transport(), sources=[W.pencil(0, 1.0, (4.0, 4.0, 0.0), 3000)])
    mm = dict(mm, transport=base["transport"], sources=base["sources"])
    one, two = gpu_run(base, 3000), gpu_run(mm, 3000)
    assert np.mean(one["hash"] == two["hash"]) >= 0.999


def test_several_materials_mixed_precision_and_refusals():
    mcx = _mcx()
    wl = W.workload("hetero_mm_64", 20_000)
    g64 = gpu_run(wl, 20_000, 0)
    g32 = gpu_run(wl, 20_000, 1)
    check_balance(g32["led"], 6.0, 2e-5)
    check_dose_3sigma(g32, g64)
    sim = mcx.Simulator(0, 0)
    sim.set_transport(wl["transport"])
    sim.load_material(W.WATER, 0)
    sim.load_phantom(wl["phantom"])
    sim.set_sources(wl["sources"])
    with pytest.raises(mcx.MCXError, match="STATE"):
        sim.run(wl["seed"], 0, 100)  # bone (1) not loaded
    sim.load_material(W.BONE, 1)
    with pytest.raises(mcx.MCXError, match="STATE"):
        sim.run(wl["seed"], 0, 100)  # lung (2) not loaded
    sim.load_material(W.LUNG, 2)
    sim.run(wl["seed"], 0, 100)
    g = sim.dose_backward(np.zeros(sim.shape))  # the replays run on several materials too
    assert g.shape == tuple(sim.shape) and np.all(g == 0.0)
    with pytest.raises(mcx.MCXError):
        sim.load_material(W.BONE, 4)
    sim.close()


def test_full_size_sampled_histories_several_materials():
    """The several-material workload the benchmark times (1e7 histories of
    the 6 MeV field on the 128^3 phantom with bone spheres of the second
    material, 2^26 records per queue, blocks of 256, 128 steps per visit),
    FP64: a sample of histories over the whole range re-run one by one by
    the oracle; every history conserves energy."""
    mcx = _mcx()
    wl = W.workload("hetero_mm_128")
    n = wl["sources"][0]["n_hist"]
    sim = mcx.Simulator(0, 0).setup(wl)
    sim.set_launch(1 << 26, 256, 128)
    sim.set_test_mode(True)
    sim.run(wl["seed"], 0, n)
    h, led = sim.history_results(n)
    st = sim.stats()
    sim.close()
    assert st["histories"] == n
    check_balance(led, 6.0, 1e-12)
    tbs = [O.Tables(m, wl["transport"]) for m in wl["materials"]]
    sample = np.sort(np.random.default_rng(12).choice(n, size=200, replace=False))
    same = 0
    for k in sample:
        r = O.run(tbs, wl["phantom"], wl["sources"], wl["seed"], int(k), 1, hashes=True, ledger=True)
        if r.hashes[0] == h[k]:
            same += 1
            assert np.allclose(led[k], r.ledger[0][[0, 1, 2]], rtol=0, atol=1e-8), int(k)
    print("sampled identical hashes", same, "of", len(sample))
    assert same >= 0.99 * len(sample)
