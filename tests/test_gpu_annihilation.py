"""GPU parity of the optional two-photon annihilation of positrons in flight
(MCX_ANNIH_FLIGHT), alone and with straggling, against the FP64 oracle with
the same options, through the C ABI: event sequences (>= 99% of histories),
per-history energy conservation, doses within 3 combined standard errors;
and the in-flight share of slowing-down positrons against
1 - exp(-int Sigma_an / S dE) in both precisions."""
import math

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


def with_flags(wl, flags):
    return dict(wl, transport=dict(wl["transport"], flags=wl["transport"].get("flags", 0) | flags))


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
    tb = O.Tables(wl["material"], wl["transport"])
    r = O.run(tb, wl["phantom"], wl["sources"], wl["seed"], 0, n, hashes=True, ledger=True)
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


CASES = {
    "positron5": (lambda: dict(W.workload("water_pencil_32"), phantom=W.water_cube(20, 4.0),
                               sources=[W.pencil(2, 5.0, (2.0, 2.0, 0.0), 1500)]), 5.0 + 2 * MC2),
    "photon8_pair": (lambda: dict(W.workload("water_pencil_32"), phantom=W.water_cube(16, 10.0),
                                  sources=[W.pencil(0, 8.0, (5.0, 5.0, 0.0), 3000)]), 8.0),
    "rect_hetero": (lambda: W.workload("hetero_broad_64", 3000), 6.0),
}


@pytest.mark.parametrize("flags", ["annih", "annih+strag"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_annihilation_in_flight_parity(case, flags):
    make, etot = CASES[case]
    fl = O.ANNIH_FLIGHT | (O.STRAGGLING if flags == "annih+strag" else 0)
    wl = with_flags(make(), fl)
    n = wl["sources"][0]["n_hist"]
    g, o = gpu_run(wl, n), oracle_run(wl, n)
    same = np.mean(g["hash"] == o["hash"])
    print(case, flags, "identical hashes", same, "annihilations", g["stats"]["annih"], o["stats"]["annih"])
    assert same >= 0.99
    assert g["stats"]["annih"] > 0
    check_balance(g["led"], etot, 1e-12)
    check_dose_3sigma(g, o)
    check_tally_parity(g, o, same=same)


@pytest.mark.parametrize("precision", [0, 1])
def test_in_flight_share_of_slowing_down_positrons(precision):
    """Hard channels off, photons absorbed where they are made, one 40 cm
    voxel: the positrons annihilate in flight with probability
    1 - exp(-int_Eabs^E0 Sigma_an / S dE) (the integral from the oracle's
    tables and Heitler's cross section)."""
    e0, eabs = 5.0, 0.1
    hard_off = O.NO_HARD_ELASTIC | O.NO_HARD_INELASTIC | O.NO_HARD_BREMS
    t = W.transport(100.0, 250, flags=hard_off | O.ANNIH_FLIGHT, eabs=(1e9, eabs, eabs))
    n = 400_000
    wl = dict(W.workload("electron_200"), transport=t, phantom=W.water_cube(1, 40.0),
              sources=[W.pencil(2, e0, (20.0, 20.0, 20.0), n)])
    g = gpu_run(wl, n, precision=precision, test=False)
    st = g["stats"]
    assert st["escaped"] == 0
    flight = st["annih"] - st["absorbed"]
    tb = O.Tables(W.WATER, t)
    le = np.linspace(math.log(eabs), math.log(e0), 20001)
    f = np.array([math.exp(x) * tb.sigma_annih(math.exp(x)) / tb.eval(O.ech(1, 0), math.exp(x)) for x in le])
    p = 1 - math.exp(-float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(le))))
    print("in-flight share", flight / n, "expected", p)
    assert abs(flight - n * p) < 5 * math.sqrt(n * p * (1 - p))


def test_annihilation_mixed_precision_and_gradient():
    mcx = _mcx()
    wl = with_flags(CASES["photon8_pair"][0](), O.ANNIH_FLIGHT)
    n = 3000
    g32 = gpu_run(wl, n, precision=1)
    check_balance(g32["led"], 8.0, 2e-5)
    # the gradient replays with annihilation in flight: the oracle's
    # gradient on the same histories
    c = np.random.default_rng(5).uniform(-1, 1, size=wl["phantom"]["rho"].shape)
    sim = mcx.Simulator(0, 0).setup(wl)
    sim.run(wl["seed"], 0, 1000)
    g = sim.dose_backward(c)
    sim.close()
    tb = O.Tables(wl["material"], wl["transport"])
    r = O.run(tb, wl["phantom"], wl["sources"], wl["seed"], 0, 1000)
    d, _ = O.dose(wl["phantom"], r)
    go, _ = O.gradient(tb, wl["phantom"], wl["sources"], wl["seed"], 0, 1000, c, d)
    rel = np.abs(g - go) / np.abs(go).max()
    print("gradient with annihilation in flight: max deviation", rel.max())
    check_gradient_parity(g, go, class2=True)
