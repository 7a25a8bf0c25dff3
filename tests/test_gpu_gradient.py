"""GPU density gradient (two replays from the random-number counters)
against the oracle's score-function gradient on the same histories, the
closed-form layered absorber, common-random-number finite differences, and
the torch.autograd path."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tally_checks import check_gradient_parity

pytestmark = pytest.mark.gpu


def _mcx():
    import paper_2003_00796_amd as mcx
    return mcx


def gpu_grad(wl, n, c, seed=1, precision=0):
    mcx = _mcx()
    sim = mcx.Simulator(precision, 0).setup(wl)
    sim.run(seed, 0, n)
    d, s = sim.dose()
    g = sim.dose_backward(c)
    st = sim.stats()
    sim.close()
    return g, d, st


def oracle_grad(wl, n, c, seed=1):
    tb = O.Tables(wl["material"], wl["transport"])
    r = O.run(tb, wl["phantom"], wl["sources"], seed, 0, n)
    d, _ = O.dose(wl["phantom"], r)
    g, _ = O.gradient(tb, wl["phantom"], wl["sources"], seed, 0, n, c, d)
    return g, d


def slab_case(n):
    rho = np.array([1.0, 0.3, 1.8, 1.0, 0.5, 2.2, 1.0, 1.3, 0.26, 1.1])
    ph = W.slab_phantom(rho.size, 0.5, rho)
    t = W.transport(flags=O.NO_COMPTON | O.NO_RAYLEIGH | O.NO_PAIR, eabs=(0.01, 1e9, 1e9))
    return dict(name="slab", phantom=ph, transport=t, material=W.WATER,
                sources=[W.pencil(0, 0.03, (50.0, 50.0, 0.0), n)], seed=1), rho


def identical_ranges(wl, tbs, n, seed, precision=0):
    """Maximal sub-ranges of histories [0, n) whose event sequence on the GPU
    is the oracle's (per-history hashes)."""
    mcx = _mcx()
    sim = mcx.Simulator(precision, 0).setup(wl)
    sim.set_test_mode(True)
    sim.run(seed, 0, n)
    h, _ = sim.history_results(n)
    sim.close()
    r = O.run(tbs, wl["phantom"], wl["sources"], seed, 0, n, hashes=True)
    bad = np.nonzero(h != r.hashes)[0].tolist()
    cuts = [-1] + bad + [n]
    rngs = [(a + 1, b) for a, b in zip(cuts[:-1], cuts[1:]) if b - a > 1]
    return rngs, len(bad)


# which parity bound of tally_checks.check_gradient_parity applies
KERMA_TOL, CLASS2_TOL = "kerma", "class2"


def check_against_oracle(wl, tbs, n, c, seed=1, tol=KERMA_TOL, min_frac=0.9):
    """GPU gradient (two replays) = oracle gradient on the same histories, to
    rounding: on the longest run of histories with identical event sequences
    (all of them, unless a history's FP64 rounding took another branch)."""
    rngs, nbad = identical_ranges(wl, tbs, n, seed)
    first, end = max(rngs, key=lambda r: r[1] - r[0])
    assert end - first >= min_frac * n, (nbad, first, end)
    mcx = _mcx()
    sim = mcx.Simulator(0, 0).setup(wl)
    sim.run(seed, first, end - first)
    sim.dose()
    g = sim.dose_backward(c)
    st = sim.stats()
    sim.close()
    r = O.run(tbs, wl["phantom"], wl["sources"], seed, first, end - first)
    do, _ = O.dose(wl["phantom"], r, end - first)
    go, parts = O.gradient(tbs, wl["phantom"], wl["sources"], seed, first, end - first, c, do)
    rel = np.abs(g - go) / np.abs(go).max()
    print(f"histories [{first}, {end}) of {n} ({nbad} differ): max |g - g_oracle| / max |g_oracle| = {rel.max():.2e}, "
          f"99.9th percentile {np.quantile(rel, 0.999):.2e}")
    check_gradient_parity(g, go, class2=tol == CLASS2_TOL)
    return g, go, st, r.stats.as_dict()


def layers_wl(particle, e0, n, flags=0, seed=3, nz=8, dz=0.2):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, size=nz)
    ph = W.slab_phantom(nz, dz, rho)
    t = dict(W.transport(), flags=flags)
    return dict(name="layers", phantom=ph, transport=t, material=W.WATER,
                sources=[W.pencil(particle, e0, (50.0, 50.0, 0.0), n)], seed=1)


def test_gradient_matches_oracle_kerma_and_class2():
    """Kerma mode (exact estimator) and full Class II transport with every
    term of the estimator (free-path and soft-deflection scores, the
    pathwise soft loss with its energy adjoint): the GPU replays equal the
    oracle's estimator on the same histories (bounds above)."""
    rng = np.random.default_rng(7)
    wl = dict(W.workload("hetero_broad_64", 4000))
    wl["transport"] = W.transport(eabs=(0.01, 1e9, 1e9))
    c = rng.uniform(-1, 1, size=wl["phantom"]["shape"])
    tb = O.Tables(wl["material"], wl["transport"])
    check_against_oracle(wl, tb, 4000, c)
    wl = W.workload("hetero_broad_64", 2000)
    tb = O.Tables(wl["material"], wl["transport"])
    check_against_oracle(wl, tb, 2000, c, tol=CLASS2_TOL)


@pytest.mark.parametrize("case", ["electrons_3MeV", "electrons_cube", "positrons_annih_flight"])
def test_class2_gradient_matches_oracle(case):
    """Electron and positron tracks, where the e+- terms carry the gradient:
    3 MeV electrons through eight layers of densities 0.5-2, a 3 MeV
    electron field in a cube of random densities, and 5 MeV positrons with
    annihilation in flight (the run must contain annihilations in flight,
    after which the particle's energy adjoint is 0)."""
    rng = np.random.default_rng(17)
    if case == "electrons_3MeV":
        wl = layers_wl(1, 3.0, 3000)
    elif case == "electrons_cube":
        ph = W.water_cube(8, 4.0)
        ph["rho"] = rng.uniform(0.5, 1.8, size=ph["rho"].shape)
        wl = dict(name="cube", phantom=ph, transport=W.transport(), material=W.WATER,
                  sources=[W.rect_field(1, 3.0, (2.0, 2.0, 0.0), (2.0, 2.0), 2000)], seed=1)
    else:
        wl = layers_wl(2, 5.0, 3000, flags=O.ANNIH_FLIGHT, nz=12, dz=0.4)
    n = wl["sources"][0]["n_hist"]
    c = rng.uniform(-1, 1, size=wl["phantom"]["shape"])
    tb = O.Tables(wl["material"], wl["transport"])
    g, go, st, so = check_against_oracle(wl, tb, n, c, tol=CLASS2_TOL)
    assert np.abs(go).max() > 0
    if case == "positrons_annih_flight":
        print("annihilations in flight", st["annih_flight"], so["annih_flight"])
        assert st["annih_flight"] > 20 and so["annih_flight"] > 20


def test_layered_absorber_closed_form_on_gpu():
    n = 1_000_000
    wl, rho = slab_case(n)
    nz = rho.size
    e0, dz = 0.03, 0.5
    mu = 4.94 * 3.0 ** -3
    vol = 100.0 * 100.0 * dz
    c = np.random.default_rng(5).uniform(-1, 1, size=nz).reshape(nz, 1, 1)
    cum = np.concatenate([[0.0], np.cumsum(rho * dz)])
    T = np.exp(-mu * cum[:-1])
    a = 1.0 - np.exp(-mu * rho * dz)
    D = e0 * T * a * 1e6 / (rho * vol)
    exact = np.zeros(nz)
    for k in range(nz):
        for j in range(nz):
            if k < j:
                deq = e0 * (-mu * dz) * T[j] * a[j]
            elif k == j:
                deq = e0 * T[j] * mu * dz * math.exp(-mu * rho[j] * dz)
            else:
                deq = 0.0
            exact[k] += c.ravel()[j] * (1e6 / (rho[j] * vol) * deq - (D[j] / rho[j] if k == j else 0.0))
    gs = np.array([gpu_grad(wl, n, c, seed=s)[0].ravel() for s in range(1, 9)])
    mean, sem = gs.mean(0), gs.std(0, ddof=1) / math.sqrt(gs.shape[0])
    z = (mean - exact) / sem
    print("z", np.round(z, 2))
    assert np.all(np.abs(z) < 4.5)


def test_kerma_gradient_vs_crn_finite_differences():
    """Exact setting (electrons absorbed where created): the replay gradient
    agrees with central differences (+-10%, common random numbers).  The
    finite differences are heavy-tailed (a density change moves some
    interactions into neighbouring voxels), so they need 2e7 histories per
    evaluation and 12 seeds to reach a useful standard error."""
    rng = np.random.default_rng(3)
    ph = W.water_cube(16, 8.0)
    ph["rho"] = rng.uniform(0.5, 1.8, size=ph["rho"].shape)
    n = 20_000_000
    wl = dict(name="kerma", phantom=ph, transport=W.transport(eabs=(0.01, 1e9, 1e9)), material=W.WATER,
              sources=[W.rect_field(0, 2.0, (4.0, 4.0, 0.0), (6.0, 6.0), n)], seed=1)
    c = rng.uniform(-1, 1, size=ph["shape"])
    mcx = _mcx()
    sim = mcx.Simulator(0, 0).setup(wl)
    gs = []
    for s in range(1, 5):
        sim.reset()
        sim.run(s, 0, n)
        sim.dose()
        gs.append(sim.dose_backward(c))
    sim.close()
    gs = np.array(gs)
    mean, sem = gs.mean(0), gs.std(0, ddof=1) / math.sqrt(gs.shape[0])
    h = 0.1
    for v in [(6, 7, 9), (2, 8, 8)]:
        sims = {}
        for sgn in (+1, -1):
            p2 = dict(ph, rho=ph["rho"].copy())
            p2["rho"][v] *= 1 + sgn * h
            sims[sgn] = mcx.Simulator(0, 0).setup(dict(wl, phantom=p2))
        fds = []
        for s in range(100, 112):
            vals = []
            for sgn in (+1, -1):
                sims[sgn].reset()
                sims[sgn].run(s, 0, n)
                d, _ = sims[sgn].dose()
                vals.append(float((c * d).sum()))
            fds.append((vals[0] - vals[1]) / (2 * h * ph["rho"][v]))
        for sm in sims.values():
            sm.close()
        fd, fd_sem = np.mean(fds), np.std(fds, ddof=1) / math.sqrt(len(fds))
        z = (mean[v] - fd) / math.sqrt(sem[v] ** 2 + fd_sem ** 2)
        print(v, "replay", mean[v], "+-", sem[v], "fd", fd, "+-", fd_sem, "z", z)
        assert abs(z) < 4.0


def test_autograd_function_quadratic_loss():
    import torch
    mcx = _mcx()
    wl = W.workload("hetero_broad_64", 20000)
    model = mcx.DoseModel(wl, 20000, seed=3)
    rho = torch.tensor(wl["phantom"]["rho"], device="cuda", dtype=torch.float64, requires_grad=True)
    dose = mcx.DoseFunction.apply(rho, model)
    target = 0.5 * dose.detach()
    loss = ((dose - target) ** 2).sum()
    loss.backward()
    g = rho.grad.cpu().numpy()
    # the same gradient through the plain ABI call
    sim = mcx.Simulator(0, 0).setup(wl)
    sim.run(3, 0, 20000)
    d, _ = sim.dose()
    assert np.allclose(d, dose.detach().cpu().numpy(), rtol=1e-12, atol=0)
    g2 = sim.dose_backward(2 * (d - 0.5 * d))
    sim.close()
    assert np.allclose(g, g2, rtol=1e-9, atol=1e-12 * np.abs(g2).max())
    assert np.isfinite(g).all() and np.abs(g).max() > 0


def test_several_material_gradient_matches_oracle():
    """The replays on a several-material phantom (the bone-sphere phantom,
    kerma mode with full photon physics, then full Class II transport)
    against the oracle's several-material score-function gradient on the
    same histories; the layered water/bone absorber against its closed
    form."""
    rng = np.random.default_rng(11)
    wl = dict(W.workload("hetero_mm_64", 4000))
    wl["transport"] = W.transport(eabs=(0.01, 1e9, 1e9))
    c = rng.uniform(-1, 1, size=wl["phantom"]["shape"])
    tbs = [O.Tables(m, wl["transport"]) for m in wl["materials"]]
    check_against_oracle(wl, tbs, 4000, c)
    wl = W.workload("hetero_mm_64", 2000)
    tbs = [O.Tables(m, wl["transport"]) for m in wl["materials"]]
    check_against_oracle(wl, tbs, 2000, c, tol=CLASS2_TOL)
    # layered water/bone absorber, photoelectric only: closed form
    e0, dz = 0.03, 0.5
    rho = np.array([1.0, 0.3, 1.8, 1.0, 0.5, 2.2, 1.0, 1.3, 0.26, 1.1])
    mat = np.array([0, 0, 1, 0, 0, 1, 1, 0, 0, 1], dtype=np.uint8)
    nz = rho.size
    ph = W.slab_phantom(nz, dz, rho)
    ph["mat"] = np.broadcast_to(mat[:, None, None], ph["rho"].shape).copy()
    t = W.transport(flags=O.NO_COMPTON | O.NO_RAYLEIGH | O.NO_PAIR, eabs=(0.01, 1e9, 1e9))
    mu = np.array([O.Tables(m, t).eval(O.MU_PHOTO, e0) for m in (W.WATER, W.BONE)])[mat]
    vol = 100.0 * 100.0 * dz
    cz = rng.uniform(-1.0, 1.0, size=nz)
    cum = np.concatenate([[0.0], np.cumsum(mu * rho * dz)])
    T = np.exp(-cum[:-1])
    a = 1.0 - np.exp(-mu * rho * dz)
    D = e0 * T * a * 1e6 / (rho * vol)
    exact = np.zeros(nz)
    for k in range(nz):
        for j in range(nz):
            deq = (e0 * (-mu[k] * dz) * T[j] * a[j] if k < j else
                   (e0 * T[j] * mu[j] * dz * math.exp(-mu[j] * rho[j] * dz) if k == j else 0.0))
            exact[k] += cz[j] * (1e6 / (rho[j] * vol) * deq - (D[j] / rho[j] if k == j else 0.0))
    n = 200_000
    wl = dict(name="slab_mm", phantom=ph, transport=t, material=W.WATER, materials=[W.WATER, W.BONE],
              sources=[W.pencil(0, e0, (50.0, 50.0, 0.0), n)], seed=1)
    gs = np.array([gpu_grad(wl, n, cz.reshape(nz, 1, 1), seed=s)[0].ravel() for s in range(1, 9)])
    mean, sem = gs.mean(0), gs.std(0, ddof=1) / math.sqrt(len(gs))
    z = (mean - exact) / sem
    print("z", np.round(z, 2))
    assert np.all(np.abs(z) < 4.5)


@pytest.mark.parametrize("case", ["electrons_3MeV", "hetero_class2"])
def test_deflection_energy_term_matches_oracle(case):
    """Term E (MCX_GRAD_DEFLECTION_ENERGY: each soft deflection's energy
    score, chained back to every earlier step's density): the replays equal
    the oracle's estimator with the same term on the same histories."""
    mcx = _mcx()
    rng = np.random.default_rng(23)
    if case == "electrons_3MeV":
        wl = layers_wl(1, 3.0, 2000)
    else:
        wl = W.workload("hetero_broad_64", 2000)
    n = wl["sources"][0]["n_hist"]
    c = rng.uniform(-1, 1, size=wl["phantom"]["shape"])
    t_or = dict(wl["transport"], flags=wl["transport"].get("flags", 0) | O.GRAD_DEFLECTION_ENERGY)
    tb = O.Tables(wl["material"], t_or)
    rngs, nbad = identical_ranges(wl, O.Tables(wl["material"], wl["transport"]), n, 1)
    first, end = max(rngs, key=lambda r: r[1] - r[0])
    assert end - first >= 0.9 * n, (nbad, first, end)
    sim = mcx.Simulator(0, 0).setup(wl)
    sim.run(1, first, end - first)
    g0 = sim.dose_backward(c)
    sim.set_gradient(mcx.GRAD_DEFLECTION_ENERGY)
    g = sim.dose_backward(c)  # the same run, the other estimator
    sim.close()
    r = O.run(tb, wl["phantom"], wl["sources"], 1, first, end - first)
    do, _ = O.dose(wl["phantom"], r, end - first)
    go, _ = O.gradient(tb, wl["phantom"], wl["sources"], 1, first, end - first, c, do)
    err = np.abs(g - go).max() / np.abs(go).max()
    print(f"{case}: term E changes the gradient by {np.abs(g - g0).max() / np.abs(go).max():.3f} of its largest "
          f"component; max |g - g_oracle| / max |g_oracle| = {err:.2e}")
    assert np.abs(g - g0).max() > 1e-3 * np.abs(go).max()
    check_gradient_parity(g, go, class2=True)


def _fd_layers(mcx, flags, n, nb, h=0.05):
    """Replay gradients (without and with term E) and CRN central differences
    (+-h) of a linear dose loss for 3 MeV electrons through eight 2 mm layers
    of densities 0.5-2; batches of n histories."""
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 2.0, size=8)
    c = rng.uniform(-1.0, 1.0, size=8).reshape(8, 1, 1)
    wl = layers_wl(1, 3.0, n * nb, flags=flags)
    est = {0: np.zeros((nb, 8)), 1: np.zeros((nb, 8))}
    fd = np.zeros((nb, 8))
    # one context: each run loads its phantom (which resets the tallies)
    sim = mcx.Simulator(0, 0).setup(wl)
    for b in range(nb):
        sim.load_phantom(wl["phantom"])
        sim.run(1, b * n, n)
        sim.dose()
        sim.set_gradient(0)
        est[0][b] = sim.dose_backward(c).ravel()
        sim.set_gradient(mcx.GRAD_DEFLECTION_ENERGY)
        est[1][b] = sim.dose_backward(c).ravel()
        for j in range(8):
            v = []
            for sg in (1, -1):
                r2 = rho.copy()
                r2[j] *= 1 + sg * h
                sim.load_phantom(W.slab_phantom(8, 0.2, r2))
                sim.run(1, b * n, n)
                v.append(float((c * sim.dose()[0]).sum()))
            fd[b, j] = (v[0] - v[1]) / (2 * h * rho[j])
    sim.close()
    f, fse = fd.mean(0), fd.std(0, ddof=1) / np.sqrt(nb)
    keep = np.abs(f) > 0.05 * np.abs(f).max()
    z = {}
    for k, e in est.items():
        m, se = e.mean(0), e.std(0, ddof=1) / np.sqrt(nb)
        z[k] = ((m - f) / np.hypot(se, fse))[keep]
    return z, f, est


def test_deflection_energy_term_vs_crn_finite_differences():
    """The Class II estimator against common-random-number central
    differences (+-5%) on the GPU, 16 batches of 2e4 histories of 3 MeV
    electrons through eight layers.  Hard channels off (CSDA slowing, soft
    deflections, the algorithm's own step cap): with term E every layer
    agrees (|z| < 4), without it the omitted energy dependence of the
    deflection shows (some layer at |z| > 4).  With every channel on, the
    z statistics of both estimators are printed: the laws of the hard events
    (rates, angles, energy transfers) also depend on the energy and stay
    held fixed."""
    mcx = _mcx()
    hard_off = O.NO_HARD_ELASTIC | O.NO_HARD_INELASTIC | O.NO_HARD_BREMS
    z, f, _ = _fd_layers(mcx, hard_off, 20_000, 16)
    print("hard channels off: z without term E", np.round(z[0], 2), "with", np.round(z[1], 2))
    assert np.all(np.abs(z[1]) < 4.0), z[1]
    assert np.abs(z[0]).max() > 4.0, z[0]
    z, f, _ = _fd_layers(mcx, 0, 20_000, 16)
    print("all channels: z without term E", np.round(z[0], 2), "with", np.round(z[1], 2))
